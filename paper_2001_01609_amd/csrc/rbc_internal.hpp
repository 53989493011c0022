// Internal declarations of librbc: grid plans (host-built operator tables and
// band factorisations), their device views, and the kernel launchers.
//
// Discretisation (section 3.2 of the paper): Fourier modes m = 0..Mx-1 in x,
// Chebyshev-T coefficients n = 0..Nz-1 in z; products on the 3/2-padded
// Px x Pz grid.  Equations (section 2.1) in streamfunction form, each written
// in an ultraspherical basis (C^(2) rows for temperature and mean flow,
// C^(4) rows for the streamfunction) so that every operator is banded; the
// last 2 (or 4) rows are replaced by wall conditions (tau method).  Even and
// odd coefficients decouple, so every system is split by parity p: half
// index i stands for coefficient n = 2 i + p.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "rbc.h"

namespace rbc {

constexpr int kMaxStages = 5;     // s + 1 stages of ARS(4,4,3)
constexpr int kDiag = 6;          // diagnostic record: Nu_V, Nu_b, Nu_t, KE, epsilon_U, P
constexpr int kDiagAvg = 9;       // time averages: Nu_V, Nu_b, Nu_t, Nu_int, KE, Re, epsilon_U, P, |P-eps|/P
// Fourier modes per block of the diagnostics kernel (Nz coefficients each).
__host__ __device__ inline int diag_modes(int Nz) { return Nz >= 512 ? 1 : 512 / Nz; }
constexpr int kBlock = 256;       // threads per block of the per-mode kernels
constexpr int kChunkLanes = 32;   // lanes per system of the chunked band solves (more than 64 rows)
constexpr int kXcds = 8;          // XCDs of the device; workgroup b runs on XCD b mod kXcds

// Workgroups to launch for nwork work blocks (GridDev::one_xcd: kXcds per
// work block, of which the one on XCD 0 works and the others exit at once).
inline int xcd_grid(int one_xcd, int nwork) { return one_xcd ? nwork * kXcds : nwork; }

// Per-row entries of the stored bordered band factorisations (rbc_plan.cpp).
constexpr int kFacT = 4;          // lm, 1/u_ii, u_i,i+1, v      (bordered tridiagonal)
constexpr int kFacP = 7;          // lm1, lm2, 1/u_ii, u1, u2, v0, v1 (bordered pentadiagonal)

// IMEX tableau in (s+1)-stage ARS form: stage 0 is the old solution.
struct Tableau {
  int s = 0;
  double ae[kMaxStages][kMaxStages] = {};
  double ai[kMaxStages][kMaxStages] = {};
};
Tableau make_tableau(int scheme);

// Parameters of one run of an ensemble launch (runs of one grid that
// differ in Rayleigh number and step): band factors, diffusivities, and the
// stage coefficients dt a_ij of the tableau, [stage i][j], as the host forms
// them for a single run.
struct RunDev {
  const double* facT;
  const double* facP;
  double nu, kappa, sqrtRaPr;
  double hae[kMaxStages][kMaxStages];
  double hai[kMaxStages][kMaxStages];
};

// Device view of one grid, passed to kernels by value.
struct GridDev {
  int Nx, Nz, Mx, Px, Pz, n;      // n = Nz / 2
  int nrT, nrP;                   // band rows per parity: n - 1 (T, u_bar), n - 2 (psi)
  int MT;                         // modes per block in the per-mode kernel
  int ntile;                      // ceil(Mx / MT): tiles of the per-mode kernel
  int XT, nxt;                    // mode tile of the mixed-space arrays (tile-major) and their count:
                                  // XT = MT in the fused path, kGemmModes in the split path
  int split;                      // 1: split path (transforms as FP32 MFMA GEMMs, see fwd_gemm_kernel)
  int xrows;                      // x-pass rows per block (1, 2, 4), 0: by rule
  int state;                      // doubles per state = 4 Mx Nz
  double kscale;                  // k_m = m * kscale
  double nu, kappa, scale;        // viscosity, diffusivity, dzeta/dz = 2/Lz
  double Lz, sqrtRaPr;
  double T_bot, T_top;
  double bcT[2];                  // m = 0 temperature wall values per parity (wall rows of the plan)
  int fluxT;                      // 1: temperature wall rows are slopes (fixed flux)
  int urgent;                     // 1: waves run at raised SIMD issue priority (coarse grid)
  int one_xcd;                    // 1: x-pass / per-mode launches run on XCD 0 only (coarse grid)
  const double* bS10;             // [2][n][3]  S1S0 rows, half offsets 0..2
  const double* bD2;              // [2][n]     D2 rows, half offset 1
  const double* bA;               // [2][n][3]  S3S2D2 rows, half offsets 1..3
  const double* bB;               // [2][n][5]  S3S2S1S0 rows, half offsets 0..4
  const double* bD4;              // [2][n]     D4 rows, half offset 2
  const double* facT;             // [Mx][2][facT_stride]
  const double* facP;             // [Mx][2][facP_stride]  (m = 0: u_bar eq, T layout)
  int facT_stride, facP_stride;
  const void* Winv;               // Real [4][Pz/2][Nz]: d^q T_n / dz^q at Gauss points
  const void* Wfwd;               // Real [3][Nz][Pz/2]: folded forward maps (psi, T, u_bar rows)
  const void* tw;                 // Real2 [Px]: exp(-2 pi i t / Px)
  // Gather launches of an ensemble (null otherwise): batch position b works
  // on the state at xptrs[b] with the run parameters rptrs[b] (in place of
  // the grid's own factors, diffusivities and stage coefficients); its work
  // arrays are those of slot b.
  const double* const* xptrs;
  const RunDev* const* rptrs;
  const RunDev* run0;             // this grid's own run parameters (device memory)
  const float* Winv2;             // split path: [4 q][2 p][Pz/2 j][Nz/2 i] = Winv[q][j][2 i + p]
  const float* Wfwd2;             // split path: [2 f][2 p][Nz/2 i][Pz/2 j] = Wfwd[f][2 i + p][j]
  int nrad, rad[12];              // FFT radix plan for Px
};

// Host-side plan of one grid.
struct GridPlan {
  int Nx = 0, Nz = 0, Mx = 0, Px = 0, Pz = 0, n = 0;
  double Ra = 0, Pr = 0, Lx = 0, Lz = 0, dt = 0, nu = 0, kappa = 0, scale = 0;
  double T_bot = 1, T_top = 0;
  bool flux = false;              // fixed-flux temperature walls (Eq. 7)
  bool urgent = false;            // coarse grid: the serial sweep is the critical path
  bool one_xcd = false;           // see GridDev::one_xcd
  int scheme = 4;
  Tableau tab;
  int MT = 8;
  bool mixed = false;
  // Split path (mixed precision, Nz >= 64, Nx >= 128): the forward and
  // inverse Chebyshev transforms of a stage run as batched FP32 MFMA GEMMs
  // over every column of the launch (fwd_gemm_kernel, inv_gemm_kernel)
  // around the per-mode solve kernel, instead of inside it.
  bool split = false;
  int xrows = 0;                  // x-pass rows per block (tuned), 0: by rule
  // host tables
  std::vector<double> bS10, bD2, bA, bB, bD4, facT, facP, Winv, Wfwd, tw, Winv2, Wfwd2;

  int facT_stride = 0, facP_stride = 0;
  double max_growth = 0;
  // device copies
  void* d_tables = nullptr;
  GridDev dev{};
};

// Builds every host table of a grid; returns an empty string or an error.
std::string build_plan(GridPlan& g);
// The run parameters of plan g with its band factors at the given device
// addresses (the grid's own, or those of one run of an ensemble).
RunDev make_run_dev(const GridPlan& g, const double* facT_dev, const double* facP_dev);
// Uploads the tables and fills g.dev.  Returns hipSuccess or the error.
hipError_t upload_plan(GridPlan& g);
size_t plan_device_bytes(const GridPlan& g);

// Per-grid work buffers for a batch of `cap` slices.
struct Work {
  int cap = 0;
  void* Q = nullptr;       // Real [cap][6][ntile][Pz][MT][2]
  void* Nh = nullptr;      // Real [cap][2][ntile][Pz][MT][2]
  void* qbar = nullptr;    // Real [cap][Pz]
  void* Ehist = nullptr;   // Real [s][cap][state]
  double* LYhist = nullptr;  // [s-1][cap][state]
  double* dpart = nullptr;   // [cap][mode chunks][4] diagnostic partial sums
  float* Yf = nullptr;       // split path: [cap][field][m][re,im][parity][Nz/2] new stage (FP32)
};
// Modes per column group of the split path's GEMM kernels and the mode tile
// of its mixed-space arrays.
constexpr int kGemmModes = 32;
size_t work_bytes(const GridPlan& g, int cap);
hipError_t alloc_work(const GridPlan& g, int cap, Work& w);
void free_work(Work& w);

// HIP-event timing of one kernel of the fine propagator: on every `every`-th
// step each launch of `kernel` (0 = stage kernel, 1 = x-pass) is bracketed by
// an event pair on the launch stream.
struct KernelTiming {
  int kernel = -1;
  int every = 0;
  std::vector<hipEvent_t> ev;   // pairs: start, stop
  size_t used = 0;              // events in use
  double units = 0;             // states (slices) processed by the timed launches
  static constexpr size_t kMaxPairs = 8192;
};

// ---- launchers (rbc_kernels.hip) -----------------------------------------
// Advance n_slices contiguous states X in place by n_steps IMEX steps.  If
// nu_out is not null, after every nu_stride-th step the diagnostic record of
// each slice goes to nu_out[(s * nu_ld + sample) * kDiag ..].
hipError_t launch_steps(const GridPlan& g, Work& w, double* X, int n_slices, int n_steps,
                        double* nu_out, int nu_stride, int nu_ld, hipStream_t st,
                        KernelTiming* timing = nullptr);

// Steps [step0, step1) of a run of n_total steps on `count` states held in
// ring slots slot0, slot0 + 1, ... (mod w.cap) of X ([w.cap][state]).
// step0 == 0 first transforms the initial states to the padded grid (so
// step0 = step1 = 0 is that transform alone); the last stage of step
// n_total - 1 skips the transform for a following step.  Nu samples as in
// launch_steps, numbered from the start of the run.  Timed steps (see
// KernelTiming) are chosen by timing_index + (step - step0).
struct StepRange {
  int slot0 = 0, count = 0;
  int step0 = 0, step1 = 0, n_total = 0;
  long timing_index = 0;
};
hipError_t launch_step_range(const GridPlan& g, Work& w, double* X, const StepRange& r, double* nu_out,
                             int nu_stride, int nu_ld, hipStream_t st, KernelTiming* timing = nullptr);

// Per-slot record of the pipelined Parareal's fine runs: the run's
// diagnostic samples go to buffer `par` (iteration parity), slice n; it
// started at virtual fine step `start`.
struct SlotMeta {
  int par, n, start, pad;
};
hipError_t launch_set_meta(SlotMeta* meta, int slot, SlotMeta v, hipStream_t st);
// Diagnostic records (kDiag values) of `count` states at batch positions
// slot0, slot0 + 1, ... (mod cap) of X; count <= w.cap (partial sums in
// w.dpart).  Without meta, state i writes out[i * ld .. + kDiag]; with meta
// (the pipelined ring, at virtual fine step t) a run that has completed a
// multiple q+1 of `stride` own steps writes out[((par S + n) nsf + q) kDiag].
hipError_t launch_diag(const GridPlan& g, Work& w, const double* X, int slot0, int count, int cap, double* out,
                       int ld, const SlotMeta* meta, int t, int stride, int nsf, int S, hipStream_t st);
// The same with the partial sums in `part` (diag_partials_per_state doubles
// per state, count states) instead of the work buffers.
hipError_t launch_diag_into(const GridPlan& g, double* part, const double* X, int slot0, int count, int cap,
                            double* out, int ld, const SlotMeta* meta, int t, int stride, int nsf, int S,
                            hipStream_t st);
size_t diag_partials_per_state(const GridDev& d);
// Device scratch of the allocation-free entry points (kScratchBytes per GPU,
// a static device array): scratch_init takes its address on `device` (which
// must be current) once; scratch_ptr returns it, or null before that.
constexpr size_t kScratchBytes = size_t(1) << 20;
hipError_t scratch_init(int device);
double* scratch_ptr(int device);
// Explicit terms of one state (diagnostic): E = state-shaped FP64 array.
hipError_t launch_explicit(const GridPlan& g, Work& w, const double* X, double* E, hipStream_t st);
// Fine -> coarse restriction (truncation).
hipError_t launch_restrict(const GridPlan& f, const GridPlan& c, const double* Xf, double* Xc,
                           hipStream_t st);
// Parareal combination for one slice: mode 0 U = P(gc); 1 U = P(gc) + F - P(gold);
// 2 U = F.  gold <- gc for modes 0 and 1.  Writes (||U_new - U_old||^2,
// ||U_new||^2) block partials to part[kCombineBlocks][2].
constexpr int kCombineBlocks = 64;
hipError_t launch_combine(const GridPlan& f, const GridPlan& c, int mode, double* U,
                          const double* F, const double* gc, double* gold, double* part,
                          hipStream_t st);
// Reduce partials of slices [first, last) (part is [S+1][kCombineBlocks][2]) into
// out[0] = max relative defect, out[1] = non-finite flag (0/1).
hipError_t launch_defect(const double* part, int first, int last, double* out, hipStream_t st);

}  // namespace rbc
