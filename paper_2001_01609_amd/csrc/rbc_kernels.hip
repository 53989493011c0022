// HIP kernels of librbc for gfx950 (CDNA4, 64-wide wavefronts).
//
// One IMEX stage of the fine propagator over a batch of slices is two
// launches (section 3.2 of the paper: transform to grid space, products
// there, transform back, implicit solve per mode):
//
//   xpass_kernel   one block per (slice, z point j of the padded grid):
//                  3 packed inverse complex FFTs of length Px (six real
//                  fields u, w, omega_x, omega_z, T_x, T_z), the products
//                  N_omega = u omega_x + w omega_z, N_T = u T_x + w T_z and the
//                  horizontal mean of u w, one packed forward FFT; keeps m < Mx.
//   stage_kernel   one block per (slice, tile of MT modes): forward Chebyshev
//                  transform of the products folded with the equation bases
//                  (explicit terms E), the stage right-hand side from the
//                  stage history, the bordered banded FP64 solves
//                  (temperature, then streamfunction with the implicit
//                  buoyancy of the new temperature), L Y for later stages,
//                  and the inverse Chebyshev transform of the new stage
//                  (values and z-derivatives at the padded Gauss points) for
//                  the next x-pass.
//
// Data in HBM: states [slice][field][m][re,im][n] (FP64, n contiguous);
// mixed-space arrays [slice][quantity][j][m][re,im] (Real, m contiguous) so
// the x-pass reads whole rows and the stage kernel reads m-tiles.
#include <cmath>
#include <mutex>
#include <vector>

#include "rbc_internal.hpp"

namespace rbc {

template <typename Real>
struct Cx {
  Real x, y;
};

template <typename Real>
__device__ __forceinline__ Cx<Real> cmul(Cx<Real> a, Cx<Real> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename Real>
__device__ __forceinline__ Cx<Real> cadd(Cx<Real> a, Cx<Real> b) { return {a.x + b.x, a.y + b.y}; }

// Work block of this workgroup, or -1: the workgroup exits at once.  With
// one_xcd (GridDev::one_xcd) the launch has kXcds workgroups per work block
// and only those on XCD 0 work.
__device__ __forceinline__ int work_block(int one_xcd) {
  const int b = blockIdx.x;
  if (!one_xcd) return b;
  return (b % kXcds) ? -1 : b / kXcds;
}

// Batch position b -> slot of the state ring (slots slot0, slot0 + 1, ... mod
// cap).  A plain batch is the ring read from slot 0 without wrapping.
__device__ __forceinline__ int ring_slot(int b, int slot0, int cap) {
  const int s = slot0 + b;
  return s >= cap ? s - cap : s;
}

// A pointer that is the same for the whole wavefront, kept in scalar
// registers.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(v)), hi = __builtin_amdgcn_readfirstlane(unsigned(v >> 32));
  return reinterpret_cast<T*>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// Global and constant views of generic pointers.  A pointer the kernels load
// from memory (the grid's tables, the ensemble's pointer tables, the run
// parameters) is generic to the compiler, which then issues flat loads;
// those count against the LDS counter as well, so that every wait for an
// LDS access or a lane shuffle also waits for them.  Loads through a global
// view are global loads, and uniform loads through a constant view (data
// that no kernel writes while it is read) are scalar loads.
template <typename T>
using gview = const __attribute__((address_space(1))) T*;
template <typename T>
using gwview = __attribute__((address_space(1))) T*;
template <typename T>
using cview = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ gview<T> gv(const T* p) { return (gview<T>)p; }
template <typename T>
__device__ __forceinline__ gwview<T> gw(T* p) { return (gwview<T>)p; }
template <typename T>
__device__ __forceinline__ cview<T> cv(const T* p) { return (cview<T>)p; }

// State of batch position b: gathered from the ensemble's pointer table, or
// slot s of the launch's state array X.
__device__ __forceinline__ const double* batch_state(const GridDev& g, const double* X, int b, int s) {
  return g.xptrs ? uniform_ptr(g.xptrs[b]) : X + size_t(s) * g.state;
}

// Run parameters of batch position b: the ensemble's table, or the grid's
// own (always device memory, so that choosing between them never needs the
// address of a kernel argument).
__device__ __forceinline__ const RunDev* batch_run(const GridDev& g, int b) {
  return g.rptrs ? uniform_ptr(g.rptrs[b]) : g.run0;
}
template <typename Real>
__device__ __forceinline__ Cx<Real> csub(Cx<Real> a, Cx<Real> b) { return {a.x - b.x, a.y - b.y}; }

// ------------------------------------------------------------------ x-pass ---

// Radix-4 DFT with sign s (exp(s 2 pi i / 4) = s i).
template <typename Real>
__device__ __forceinline__ void dft4(Cx<Real> a0, Cx<Real> a1, Cx<Real> a2, Cx<Real> a3, Real sign,
                                     Cx<Real>* y) {
  const Cx<Real> s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const Cx<Real> s13 = cadd(a1, a3), d13 = csub(a1, a3);
  const Cx<Real> id13 = {-sign * d13.y, sign * d13.x};   // s i (a1 - a3)
  y[0] = cadd(s02, s13);
  y[1] = cadd(d02, id13);
  y[2] = csub(s02, s13);
  y[3] = csub(d02, id13);
}

// DFT_R of a[0..R-1] with sign s into y[0..R-1], R = 2, 3, 4 or 8.
template <typename Real, int R>
__device__ __forceinline__ void dft_small(const Cx<Real>* a, Real sign, Cx<Real>* y) {
  if constexpr (R == 2) {
    y[0] = cadd(a[0], a[1]);
    y[1] = csub(a[0], a[1]);
  } else if constexpr (R == 3) {
    const Real h = Real(0.86602540378443864676);  // sqrt(3)/2
    const Cx<Real> t = cadd(a[1], a[2]), d = csub(a[1], a[2]);
    const Cx<Real> m = {a[0].x - Real(0.5) * t.x, a[0].y - Real(0.5) * t.y};
    const Cx<Real> id = {-sign * h * d.y, sign * h * d.x};   // s i h d
    y[0] = cadd(a[0], t);
    y[1] = cadd(m, id);
    y[2] = csub(m, id);
  } else if constexpr (R == 4) {
    dft4(a[0], a[1], a[2], a[3], sign, y);
  } else {
    // 8 = 2 x 4: even and odd DFT4s joined with exp(s 2 pi i q / 8)
    Cx<Real> e[4], o[4];
    dft4(a[0], a[2], a[4], a[6], sign, e);
    dft4(a[1], a[3], a[5], a[7], sign, o);
    const Real h = Real(0.70710678118654752440);   // sqrt(2)/2
    const Cx<Real> w1 = {h * (o[1].x - sign * o[1].y), h * (o[1].y + sign * o[1].x)};
    const Cx<Real> w2 = {-sign * o[2].y, sign * o[2].x};
    const Cx<Real> w3 = {h * (-o[3].x - sign * o[3].y), h * (-o[3].y + sign * o[3].x)};
    y[0] = cadd(e[0], o[0]);
    y[4] = csub(e[0], o[0]);
    y[1] = cadd(e[1], w1);
    y[5] = csub(e[1], w1);
    y[2] = cadd(e[2], w2);
    y[6] = csub(e[2], w2);
    y[3] = cadd(e[3], w3);
    y[7] = csub(e[3], w3);
  }
}

// Orders the LDS accesses of one wavefront's lanes around this point.  An
// x-pass row lives in LDS that only its own wavefront touches, and the LDS
// operations of a wavefront complete in issue order, so exchanging values
// between its lanes needs no workgroup barrier, only this compiler fence.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place Stockham radix-R pass (Bainville's autosort form) over CNT
// signals of length N (stride N) by one 64-lane wavefront: every lane first
// gathers the inputs of its butterflies into registers, the wave syncs,
// then writes out[j + q P] = DFT_R over in[i + r N/R] twiddled by
// exp(sign 2 pi i r k / (P R)), k = i mod P, j = (i - k) R + k.  The radix
// plan is 8, ..., 8, (4 or 2), 3, so P is a power of two in every pass and
// r k N/(P R) < N indexes the twiddle table directly; a butterfly's
// twiddles serve all CNT signals.
template <typename Real, int R, int N, int P, int CNT>
__device__ __forceinline__ void stockham_pass(Cx<Real>* x, const Cx<Real>* __restrict__ tw, Real sign) {
  constexpr int T = N / R;
  constexpr int NB = (T + 63) / 64;
  constexpr int TS = N / (P * R);
  const int lane = threadIdx.x & 63;
  Cx<Real> v[NB][CNT][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = lane + 64 * b;
    if (i < T) {
      const int k = i & (P - 1);
      Cx<Real> t[R];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        if (P > 1) {
          t[r] = tw[r * k * TS];
          t[r].y *= -sign;   // table holds exp(-2 pi i t/N); the inverse uses the conjugate
        }
      }
#pragma unroll
      for (int c = 0; c < CNT; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const Cx<Real> u = x[c * N + i + r * T];
          v[b][c][r] = (r > 0 && P > 1) ? cmul(u, t[r]) : u;
        }
    }
  }
  wave_sync();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = lane + 64 * b;
    if (i >= T) continue;
    const int k = i & (P - 1), j = (i - k) * R + k;
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
      Cx<Real> y[R];
      dft_small<Real, R>(v[b][c], sign, y);
#pragma unroll
      for (int q = 0; q < R; ++q) x[c * N + j + q * P] = y[q];
    }
  }
  wave_sync();
}

// Radix plan for N = 3 * 2^q: eights, then a four or a two, then the three.
// CNT signals are transformed together while their butterflies fit in
// registers, otherwise one at a time.
template <typename Real, int N, int P, int CNT>
__device__ __forceinline__ void fft_wave(Cx<Real>* x, const Cx<Real>* tw, Real sign) {
  constexpr int rem = N / P;
  if constexpr (rem > 1) {
    constexpr int p2 = rem / 3;
    constexpr int R = (rem == 3) ? 3 : (p2 >= 8 ? 8 : p2);
    constexpr int regs = CNT * ((N / R + 63) / 64) * R * int(sizeof(Real)) / 2;   // 32-bit registers
    if constexpr (regs <= 96) {
      stockham_pass<Real, R, N, P, CNT>(x, tw, sign);
    } else {
#pragma unroll
      for (int c = 0; c < CNT; ++c) stockham_pass<Real, R, N, P, 1>(x + c * N, tw, sign);
    }
    fft_wave<Real, N, P * R, CNT>(x, tw, sign);
  }
}

template <typename Real>
__device__ __forceinline__ Real wave_sum(Real v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Complex spectra of length PX held in LDS per x-pass row: three (the
// packed pairs (u, w), (omega_x, omega_z), (T_x, T_z) transformed together),
// or two for multi-row FP64 blocks up to PX = 768, where LDS bounds the rows
// per CU: (T_x, T_z) is then transformed after N_omega has gone to registers,
// in the second spectrum's place.  The longest FP32 rows (PX >= 1536) keep
// one: u and w go to registers after the first transform, and the other two
// pairs are transformed in turn in the same place, so that twice as many
// rows fit a compute unit.
template <typename Real, int PX, int RB>
constexpr int xpass_spectra() {
  return (sizeof(Real) == 4 && PX >= 1536) ? 1 : ((sizeof(Real) == 8 && PX <= 768 && RB > 1) ? 2 : 3);
}

// One block of RB wavefronts per (slice, group of RB padded z points); wave w
// transforms row j = RB group + w.  Q holds the six fields of the stage at
// the padded Gauss points and Nh receives N_omega and N_T, both mode-tile
// major ([slice][quantity][tile][j][mode in tile][re, im]) so that a block
// moves RB x MT contiguous values per tile; qbar gets the horizontal mean of
// u w.
template <typename Real, int PX, int RB>
__global__ void __launch_bounds__(64 * RB) xpass_kernel(GridDev g, const Real* __restrict__ Q,
                                                        Real* __restrict__ Nh, Real* __restrict__ qbar,
                                                        int slot0, int cap) {
  if (g.urgent) __builtin_amdgcn_s_setprio(3);
  extern __shared__ __align__(16) unsigned char smem[];
  const int Pz = g.Pz, Mx = g.Mx, MT = g.XT, ntile = g.nxt;   // mixed-space tiles
  const int ngrp = Pz / RB;
  const int bid = work_block(g.one_xcd);
  if (bid < 0) return;
  const int b = bid / ngrp, jg = bid - b * ngrp;
  const int s = ring_slot(b, slot0, cap);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = jg * RB + wv;
  constexpr int NA = xpass_spectra<Real, PX, RB>();
  Cx<Real>* A = reinterpret_cast<Cx<Real>*>(smem) + wv * NA * PX;   // this row's [NA][PX]
  const Cx<Real>* tw = reinterpret_cast<const Cx<Real>*>(g.tw);
  const size_t tq = size_t(Pz) * MT;                 // complex values per (quantity, tile)

  // the zero padding between the retained modes of spectra c0 .. c1-1
  const int nzc = PX - 2 * Mx + 1;
  const Cx<Real>* Qc = reinterpret_cast<const Cx<Real>*>(Q) + size_t(s) * 6 * ntile * tq + size_t(j) * MT;
  // packs the field pairs c0 .. c1-1 of (u, w), (omega_x, omega_z), (T_x,
  // T_z) into spectra at A + (c - d) PX
  auto pack = [&](int c0, int c1, int d) {
    for (int c = c0; c < c1; ++c)
      for (int t = lane; t < nzc; t += 64) A[(c - d) * PX + Mx + t] = {Real(0), Real(0)};
    for (int m = lane; m < Mx; m += 64) {
      const int tile = m / MT, mt = m - tile * MT;
      const Cx<Real>* q0 = Qc + size_t(tile) * tq + mt;
      Cx<Real> q6[6];
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (c >= 2 * c0 && c < 2 * c1) q6[c] = q0[size_t(c) * ntile * tq];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c < c0 || c >= c1) continue;
        const Cx<Real> qa = q6[2 * c], qb = q6[2 * c + 1];
        A[(c - d) * PX + m] = {qa.x - qb.y, qa.y + qb.x};
        if (m > 0) A[(c - d) * PX + PX - m] = {qa.x + qb.y, qb.x - qa.y};
      }
    }
  };
  Real uw = 0;
  if constexpr (NA == 1) {
    constexpr int NT = (PX + 63) / 64;
    Real ur[NT], wr[NT], nw[NT];
    pack(0, 1, 0);   // (u, w)
    wave_sync();
    fft_wave<Real, PX, 1, 1>(A, tw, Real(1));
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int t = lane + 64 * i;
      ur[i] = wr[i] = Real(0);
      if (t < PX) {
        const Cx<Real> v1 = A[t];
        ur[i] = v1.x;
        wr[i] = v1.y;
        uw += v1.x * v1.y;
      }
    }
    wave_sync();
    pack(1, 2, 1);   // (omega_x, omega_z) in the same place
    wave_sync();
    fft_wave<Real, PX, 1, 1>(A, tw, Real(1));
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int t = lane + 64 * i;
      nw[i] = Real(0);
      if (t < PX) {
        const Cx<Real> v2 = A[t];
        nw[i] = ur[i] * v2.x + wr[i] * v2.y;
      }
    }
    wave_sync();
    pack(2, 3, 2);   // (T_x, T_z)
    wave_sync();
    fft_wave<Real, PX, 1, 1>(A, tw, Real(1));
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int t = lane + 64 * i;
      if (t < PX) {
        const Cx<Real> v3 = A[t];
        A[t] = {nw[i], ur[i] * v3.x + wr[i] * v3.y};
      }
    }
  } else if constexpr (NA == 3) {
    pack(0, 3, 0);
    wave_sync();
    fft_wave<Real, PX, 1, 3>(A, tw, Real(1));
    for (int t = lane; t < PX; t += 64) {
      const Cx<Real> v1 = A[t], v2 = A[PX + t], v3 = A[2 * PX + t];
      const Real u = v1.x, w = v1.y;
      A[t] = {u * v2.x + w * v2.y, u * v3.x + w * v3.y};
      uw += u * w;
    }
  } else {
    constexpr int NT = (PX + 63) / 64;
    Real nw[NT];
    pack(0, 2, 0);
    wave_sync();
    fft_wave<Real, PX, 1, 2>(A, tw, Real(1));
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int t = lane + 64 * i;
      nw[i] = Real(0);
      if (t < PX) {
        const Cx<Real> v1 = A[t], v2 = A[PX + t];
        nw[i] = v1.x * v2.x + v1.y * v2.y;
        uw += v1.x * v1.y;
      }
    }
    wave_sync();
    pack(2, 3, 1);   // (T_x, T_z) into the second spectrum
    wave_sync();
    fft_wave<Real, PX, 1, 1>(A + PX, tw, Real(1));
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const int t = lane + 64 * i;
      if (t < PX) {
        const Cx<Real> v1 = A[t], v3 = A[PX + t];
        A[t] = {nw[i], v1.x * v3.x + v1.y * v3.y};
      }
    }
  }
  uw = wave_sum(uw);
  if (lane == 0) qbar[size_t(s) * Pz + j] = uw / Real(PX);
  wave_sync();
  fft_wave<Real, PX, 1, 1>(A, tw, Real(-1));
  const Real inv2 = Real(0.5) / Real(PX);
  Cx<Real>* out = reinterpret_cast<Cx<Real>*>(Nh) + size_t(s) * 2 * ntile * tq + size_t(j) * MT;
  for (int m = lane; m < Mx; m += 64) {
    const int tile = m / MT, mt = m - tile * MT;
    const Cx<Real> a = A[m], b = A[m == 0 ? 0 : PX - m];
    // N_omega = (Z_m + conj Z_-m)/2, N_T = (Z_m - conj Z_-m)/(2i), both / PX
    Cx<Real>* o = out + size_t(tile) * tq + mt;
    o[0] = {(a.x + b.x) * inv2, (a.y - b.y) * inv2};
    o[size_t(ntile) * tq] = {(a.y + b.y) * inv2, (b.x - a.x) * inv2};
  }
}

// ------------------------------------------------------------ stage kernel ---

enum StageMode { kModeStage = 0, kModeZinv = 1, kModeExplicit = 2 };

struct StageArgs {
  int mode;
  int stage;           // i = 1..s
  int s;               // implicit stages
  int cap;             // slices the history arrays are sized for
  int slot0;           // ring slot of the first state of the batch
  int store_E, store_LY, write_X, do_zinv;
  double hae[kMaxStages];   // h a_ij (explicit), j < i
  double hai[kMaxStages];   // h a~_ij (implicit), 1 <= j <= i
  double haii;
};

// LDS stride (in doubles) of one staged factor block: odd, so that lanes
// reading different blocks at the same row fall in different banks.
__host__ __device__ __forceinline__ int lds_fac_stride(int s) { return s | 1; }

// Bordered tridiagonal solve in place on v[2 i + p] (one parity):
// temperature and mean flow.  fac: kFacT entries per row, then the 1 x 1
// Schur inverse.  NR = band rows.  With REG and up to 31 rows the parity
// vector is held in registers for the three sweeps (shorter dependent chain,
// more registers: the latency-bound small-batch variant); otherwise the
// sweeps run in LDS.
// Weight of tail unknown i (coefficient n = 2 (i + 1) + p) in the wall row
// of a bordered tridiagonal system: 1 for wall values, n^2 for wall slopes
// (fixed-flux temperature walls).
__device__ __forceinline__ double wall_w(int i, int p, bool slope) {
  const double n = double(2 * (i + 1) + p);
  return slope ? n * n : 1.0;
}

template <int NR, bool REG>
__device__ __forceinline__ void solve_T_format(double* __restrict__ v, int p, const double* __restrict__ fac,
                                               double gbc, bool slope) {
  if constexpr (REG && NR <= 31) {
    double y[NR + 1];
#pragma unroll
    for (int i = 0; i < NR; ++i) y[i] = v[2 * i + p];
#pragma unroll
    for (int i = 1; i < NR; ++i) y[i] -= fac[i * kFacT + 0] * y[i - 1];
    double sum = 0;
    y[NR - 1] *= fac[(NR - 1) * kFacT + 1];
    sum = wall_w(NR - 1, p, slope) * y[NR - 1];
#pragma unroll
    for (int i = NR - 2; i >= 0; --i) {
      y[i] = (y[i] - fac[i * kFacT + 2] * y[i + 1]) * fac[i * kFacT + 1];
      sum += wall_w(i, p, slope) * y[i];
    }
    const double xh = fac[NR * kFacT] * (gbc - sum);
    v[p] = xh;
#pragma unroll
    for (int i = 0; i < NR; ++i) v[2 * (i + 1) + p] = y[i] - fac[i * kFacT + 3] * xh;
  } else {
    double y = v[p];
#pragma unroll 8
    for (int i = 1; i < NR; ++i) {
      y = v[2 * i + p] - fac[i * kFacT + 0] * y;
      v[2 * i + p] = y;
    }
    double x = y * fac[(NR - 1) * kFacT + 1];
    v[2 * (NR - 1) + p] = x;
    double sum = wall_w(NR - 1, p, slope) * x;
#pragma unroll 8
    for (int i = NR - 2; i >= 0; --i) {
      x = (v[2 * i + p] - fac[i * kFacT + 2] * x) * fac[i * kFacT + 1];
      v[2 * i + p] = x;
      sum += wall_w(i, p, slope) * x;
    }
    const double xh = fac[NR * kFacT] * (gbc - sum);
#pragma unroll 8
    for (int i = NR - 1; i >= 0; --i) v[2 * (i + 1) + p] = v[2 * i + p] - fac[i * kFacT + 3] * xh;
    v[p] = xh;
  }
}

// Bordered pentadiagonal solve in place (streamfunction, two border unknowns).
template <int NR, bool REG>
__device__ __forceinline__ void solve_P_format(double* __restrict__ v, int p, const double* __restrict__ fac) {
  if constexpr (REG && NR <= 31) {
    double y[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) y[i] = v[2 * i + p];
#pragma unroll
    for (int i = 1; i < NR; ++i) {
      y[i] -= fac[i * kFacP + 0] * y[i - 1];
      if (i >= 2) y[i] -= fac[i * kFacP + 1] * y[i - 2];
    }
    double s0 = 0, s1 = 0;
#pragma unroll
    for (int i = NR - 1; i >= 0; --i) {
      double x = y[i];
      if (i + 1 < NR) x -= fac[i * kFacP + 3] * y[i + 1];
      if (i + 2 < NR) x -= fac[i * kFacP + 4] * y[i + 2];
      y[i] = x * fac[i * kFacP + 2];
      const double nn = double(2 * (i + 2) + p);
      s0 += y[i];
      s1 += nn * nn * y[i];
    }
    const double* si = fac + NR * kFacP;
    const double h0 = -(si[0] * s0 + si[1] * s1);
    const double h1 = -(si[2] * s0 + si[3] * s1);
    v[p] = h0;
    v[2 + p] = h1;
#pragma unroll
    for (int i = 0; i < NR; ++i) v[2 * (i + 2) + p] = y[i] - fac[i * kFacP + 5] * h0 - fac[i * kFacP + 6] * h1;
  } else {
    double y2 = 0, y1 = 0;
#pragma unroll 8
    for (int i = 0; i < NR; ++i) {
      const double y = v[2 * i + p] - fac[i * kFacP + 0] * y1 - fac[i * kFacP + 1] * y2;
      v[2 * i + p] = y;
      y2 = y1;
      y1 = y;
    }
    double x1 = 0, x2 = 0, s0 = 0, s1 = 0;
#pragma unroll 8
    for (int i = NR - 1; i >= 0; --i) {
      const double x = (v[2 * i + p] - fac[i * kFacP + 3] * x1 - fac[i * kFacP + 4] * x2) * fac[i * kFacP + 2];
      v[2 * i + p] = x;
      const double nn = double(2 * (i + 2) + p);
      s0 += x;
      s1 += nn * nn * x;
      x2 = x1;
      x1 = x;
    }
    const double* si = fac + NR * kFacP;
    const double h0 = -(si[0] * s0 + si[1] * s1);
    const double h1 = -(si[2] * s0 + si[3] * s1);
#pragma unroll 8
    for (int i = NR - 1; i >= 0; --i)
      v[2 * (i + 2) + p] = v[2 * i + p] - fac[i * kFacP + 5] * h0 - fac[i * kFacP + 6] * h1;
    v[p] = h0;
    v[2 + p] = h1;
  }
}

// Scan form of the same bordered solves: one lane per band row, W lanes per
// system (W = power of two > NR, segments aligned to W).  Each elimination
// sweep is a linear recurrence, i.e. the composition of one affine map per
// row, evaluated as an inclusive Hillis-Steele scan with lane shuffles
// (log2 W steps instead of NR); the wall-row sums are segment reductions.
// li = lane within the segment; every lane of a segment must call.
template <int W>
__device__ __forceinline__ double seg_sum(double x) {
#pragma unroll
  for (int o = 1; o < W; o <<= 1) x += __shfl_xor(x, o, W);
  return x;
}

template <int NR, int W>
__device__ __forceinline__ void solve_T_scan(double* __restrict__ v, int p, const double* __restrict__ fac,
                                             double gbc, bool slope, int li) {
  const bool act = li < NR;
  const double* fr = fac + li * kFacT;
  const double f = act ? v[2 * li + p] : 0.0;
  const double l = act ? fr[0] : 0.0;          // l_0 = 0
  const double d = act ? fr[1] : 0.0;
  const double u = act ? fr[2] : 0.0;          // u_(NR-1) = 0
  const double vc = act ? fr[3] : 0.0;
  // forward: y_i = -l_i y_(i-1) + f_i
  double A = -l, B = f;
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double Ap = __shfl_up(A, o, W), Bp = __shfl_up(B, o, W);
    if (li >= o) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  // backward: x_i = (-u_i d_i) x_(i+1) + d_i y_i   (rows >= NR contribute 0)
  A = -u * d;
  B = d * B;
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double An = __shfl_down(A, o, W), Bn = __shfl_down(B, o, W);
    if (li + o < W) {
      B = A * Bn + B;
      A = A * An;
    }
  }
  const double sum = seg_sum<W>(wall_w(li, p, slope) * B);
  const double xh = fac[NR * kFacT] * (gbc - sum);
  if (act) v[2 * (li + 1) + p] = B - vc * xh;
  if (li == 0) v[p] = xh;
}

template <int NR, int W>
__device__ __forceinline__ void solve_P_scan(double* __restrict__ v, int p, const double* __restrict__ fac, int li) {
  const bool act = li < NR;
  const double* fr = fac + li * kFacP;
  const double f = act ? v[2 * li + p] : 0.0;
  // forward: (y_i, y_(i-1)) = [[-l1, -l2], [1, 0]] (y_(i-1), y_(i-2)) + (f_i, 0)
  double m00 = act ? -fr[0] : 0.0, m01 = act ? -fr[1] : 0.0, m10 = act ? 1.0 : 0.0, m11 = 0.0;
  double c0 = f, c1 = 0.0;
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double p00 = __shfl_up(m00, o, W), p01 = __shfl_up(m01, o, W);
    const double p10 = __shfl_up(m10, o, W), p11 = __shfl_up(m11, o, W);
    const double q0 = __shfl_up(c0, o, W), q1 = __shfl_up(c1, o, W);
    if (li >= o) {   // this composite after the earlier one
      const double n0 = m00 * q0 + m01 * q1 + c0, n1 = m10 * q0 + m11 * q1 + c1;
      const double a00 = m00 * p00 + m01 * p10, a01 = m00 * p01 + m01 * p11;
      const double a10 = m10 * p00 + m11 * p10, a11 = m10 * p01 + m11 * p11;
      m00 = a00; m01 = a01; m10 = a10; m11 = a11;
      c0 = n0; c1 = n1;
    }
  }
  const double y = c0;
  // backward: (x_i, x_(i+1)) = [[-u1 d, -u2 d], [1, 0]] (x_(i+1), x_(i+2)) + (d y_i, 0)
  const double dd = act ? fr[2] : 0.0;
  m00 = act ? -fr[3] * dd : 0.0; m01 = act ? -fr[4] * dd : 0.0; m10 = act ? 1.0 : 0.0; m11 = 0.0;
  c0 = dd * y; c1 = 0.0;
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double p00 = __shfl_down(m00, o, W), p01 = __shfl_down(m01, o, W);
    const double p10 = __shfl_down(m10, o, W), p11 = __shfl_down(m11, o, W);
    const double q0 = __shfl_down(c0, o, W), q1 = __shfl_down(c1, o, W);
    if (li + o < W) {   // this row's map after the later rows' composite
      const double n0 = m00 * q0 + m01 * q1 + c0, n1 = m10 * q0 + m11 * q1 + c1;
      const double a00 = m00 * p00 + m01 * p10, a01 = m00 * p01 + m01 * p11;
      const double a10 = m10 * p00 + m11 * p10, a11 = m10 * p01 + m11 * p11;
      m00 = a00; m01 = a01; m10 = a10; m11 = a11;
      c0 = n0; c1 = n1;
    }
  }
  const double x = c0;
  const double nn = double(2 * (li + 2) + p);
  const double s0 = seg_sum<W>(x), s1 = seg_sum<W>(act ? nn * nn * x : 0.0);
  const double* si = fac + NR * kFacP;
  const double h0 = -(si[0] * s0 + si[1] * s1);
  const double h1 = -(si[2] * s0 + si[3] * s1);
  if (act) v[2 * (li + 2) + p] = x - fr[5] * h0 - fr[6] * h1;
  if (li == 0) {
    v[p] = h0;
    v[2 + p] = h1;
  }
}

// Smallest power of two above n (segment width of the scan solves).
constexpr int seg_width(int n) { return n < 4 ? 4 : (n < 8 ? 8 : (n < 16 ? 16 : (n < 32 ? 32 : 64))); }

// Chunked scan form of the same bordered solves for systems longer than a
// wavefront: W lanes per system, lane li owns the R consecutive band rows
// [li R, li R + R) (R W >= NR).  Each elimination sweep composes the lane's
// R affine maps in registers, combines the lanes' composites by a
// Hillis-Steele scan over the W lanes (log2 W shuffle steps), and re-runs
// its R rows from the incoming value: 2 R + log2 W dependent steps per
// sweep instead of NR.  The re-run uses the sequential recurrences, so
// only the chunk boundaries carry the scan's rounding.
// Factor element i: global memory (GF) or LDS.
template <bool GF>
__device__ __forceinline__ double fac_at(const double* fac, int i) {
  if constexpr (GF)
    return gv(fac)[i];
  else
    return fac[i];
}

template <int NR, int W, int R, bool GF>
__device__ __forceinline__ void solve_T_chunk(double* __restrict__ v, int p, const double* __restrict__ fac,
                                              double gbc, bool slope, int li) {
  static_assert(W * R >= NR && W <= 64, "chunks must cover the system within one wavefront");
  const int i0 = li * R;
  // each sweep loads the factors it uses (fewer registers live at once)
  double f[R], l[R], d[R], u[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = i0 + q;
    const bool act = i < NR;
    const int ic = min(i, NR - 1), fr = ic * kFacT;   // loads at clamped rows, then selects
    const double fv = v[2 * ic + p], lv = fac_at<GF>(fac, fr + 0);
    f[q] = act ? fv : 0.0;
    l[q] = act ? lv : 0.0;   // l_0 = 0
  }
  // forward: y_i = -l_i y_(i-1) + f_i; rows beyond NR give y = 0
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    A = -l[q] * A;
    B = f[q] - l[q] * B;
  }
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double Ap = __shfl_up(A, o, W), Bp = __shfl_up(B, o, W);
    if (li >= o) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  double y = __shfl_up(B, 1, W);
  if (li == 0) y = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    y = f[q] - l[q] * y;
    f[q] = y;   // f now holds y
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = i0 + q;
    const bool act = i < NR;
    const int fr = min(i, NR - 1) * kFacT;
    const double dv = fac_at<GF>(fac, fr + 1), uv = fac_at<GF>(fac, fr + 2);
    d[q] = act ? dv : 0.0;
    u[q] = act ? uv : 0.0;   // u_(NR-1) = 0
  }
  // backward: x_i = (y_i - u_i x_(i+1)) d_i
  A = 1.0;
  B = 0.0;
#pragma unroll
  for (int q = R - 1; q >= 0; --q) {
    B = -u[q] * d[q] * B + d[q] * f[q];
    A = -u[q] * d[q] * A;
  }
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double An = __shfl_down(A, o, W), Bn = __shfl_down(B, o, W);
    if (li + o < W) {
      B = A * Bn + B;
      A = A * An;
    }
  }
  double xn = __shfl_down(B, 1, W);
  if (li == W - 1) xn = 0.0;
  double part = 0.0;
#pragma unroll
  for (int q = R - 1; q >= 0; --q) {
    xn = (f[q] - u[q] * xn) * d[q];
    f[q] = xn;   // f now holds x
    if (i0 + q < NR) part += wall_w(i0 + q, p, slope) * xn;
  }
  const double sum = seg_sum<W>(part);
  const double xh = fac_at<GF>(fac, NR * kFacT) * (gbc - sum);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double vc = fac_at<GF>(fac, min(i0 + q, NR - 1) * kFacT + 3);
    if (i0 + q < NR) v[2 * (i0 + q + 1) + p] = f[q] - vc * xh;
  }
  if (li == 0) v[p] = xh;
}

template <int NR, int W, int R, bool GF>
__device__ __forceinline__ void solve_P_chunk(double* __restrict__ v, int p, const double* __restrict__ fac, int li) {
  static_assert(W * R >= NR && W <= 64, "chunks must cover the system within one wavefront");
  const int i0 = li * R;
  // each sweep loads the factors it uses (fewer registers live at once)
  double f[R], l1[R], l2[R], d[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = i0 + q;
    const bool act = i < NR;
    const int ic = min(i, NR - 1), fr = ic * kFacP;   // loads at clamped rows, then selects
    const double fv = v[2 * ic + p], a1 = fac_at<GF>(fac, fr + 0), a2 = fac_at<GF>(fac, fr + 1);
    f[q] = act ? fv : 0.0;
    l1[q] = act ? a1 : 0.0;
    l2[q] = act ? a2 : 0.0;
  }
  // forward: (y_i, y_(i-1)) = [[-l1, -l2], [1, 0]] (y_(i-1), y_(i-2)) + (f_i, 0);
  // the chunk's composite (M, c), rows beyond NR reset to zero
  double m00 = 1.0, m01 = 0.0, m10 = 0.0, m11 = 1.0, c0 = 0.0, c1 = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const bool act = i0 + q < NR;
    const double a00 = act ? -l1[q] : 0.0, a01 = act ? -l2[q] : 0.0, a10 = act ? 1.0 : 0.0;
    const double n00 = a00 * m00 + a01 * m10, n01 = a00 * m01 + a01 * m11;
    const double n10 = a10 * m00, n11 = a10 * m01;
    const double d0 = a00 * c0 + a01 * c1 + f[q], d1 = a10 * c0;
    m00 = n00; m01 = n01; m10 = n10; m11 = n11;
    c0 = d0; c1 = d1;
  }
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double p00 = __shfl_up(m00, o, W), p01 = __shfl_up(m01, o, W);
    const double p10 = __shfl_up(m10, o, W), p11 = __shfl_up(m11, o, W);
    const double q0 = __shfl_up(c0, o, W), q1 = __shfl_up(c1, o, W);
    if (li >= o) {   // this composite after the earlier one
      const double n0 = m00 * q0 + m01 * q1 + c0, n1 = m10 * q0 + m11 * q1 + c1;
      const double a00 = m00 * p00 + m01 * p10, a01 = m00 * p01 + m01 * p11;
      const double a10 = m10 * p00 + m11 * p10, a11 = m10 * p01 + m11 * p11;
      m00 = a00; m01 = a01; m10 = a10; m11 = a11;
      c0 = n0; c1 = n1;
    }
  }
  double y1 = __shfl_up(c0, 1, W), y2 = __shfl_up(c1, 1, W);
  if (li == 0) y1 = y2 = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double y = f[q] - l1[q] * y1 - l2[q] * y2;
    y2 = y1;
    y1 = y;
    f[q] = y;   // f now holds y
  }
  // the backward sweep's factors, in the forward ones' registers
  double* const u1 = l1;
  double* const u2 = l2;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = i0 + q;
    const bool act = i < NR;
    const int fr = min(i, NR - 1) * kFacP;
    const double dv = fac_at<GF>(fac, fr + 2), b1 = fac_at<GF>(fac, fr + 3), b2 = fac_at<GF>(fac, fr + 4);
    d[q] = act ? dv : 0.0;
    u1[q] = act ? b1 : 0.0;
    u2[q] = act ? b2 : 0.0;
  }
  // backward: (x_i, x_(i+1)) = [[-u1 d, -u2 d], [1, 0]] (x_(i+1), x_(i+2)) + (d y_i, 0)
  m00 = 1.0; m01 = 0.0; m10 = 0.0; m11 = 1.0; c0 = 0.0; c1 = 0.0;
#pragma unroll
  for (int q = R - 1; q >= 0; --q) {
    const bool act = i0 + q < NR;
    const double a00 = act ? -u1[q] * d[q] : 0.0, a01 = act ? -u2[q] * d[q] : 0.0, a10 = act ? 1.0 : 0.0;
    const double n00 = a00 * m00 + a01 * m10, n01 = a00 * m01 + a01 * m11;
    const double n10 = a10 * m00, n11 = a10 * m01;
    const double d0 = a00 * c0 + a01 * c1 + d[q] * f[q], d1 = a10 * c0;
    m00 = n00; m01 = n01; m10 = n10; m11 = n11;
    c0 = d0; c1 = d1;
  }
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const double p00 = __shfl_down(m00, o, W), p01 = __shfl_down(m01, o, W);
    const double p10 = __shfl_down(m10, o, W), p11 = __shfl_down(m11, o, W);
    const double q0 = __shfl_down(c0, o, W), q1 = __shfl_down(c1, o, W);
    if (li + o < W) {   // this chunk's map after the later chunks' composite
      const double n0 = m00 * q0 + m01 * q1 + c0, n1 = m10 * q0 + m11 * q1 + c1;
      const double a00 = m00 * p00 + m01 * p10, a01 = m00 * p01 + m01 * p11;
      const double a10 = m10 * p00 + m11 * p10, a11 = m10 * p01 + m11 * p11;
      m00 = a00; m01 = a01; m10 = a10; m11 = a11;
      c0 = n0; c1 = n1;
    }
  }
  double x1 = __shfl_down(c0, 1, W), x2 = __shfl_down(c1, 1, W);
  if (li == W - 1) x1 = x2 = 0.0;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int q = R - 1; q >= 0; --q) {
    const double xx = (f[q] - u1[q] * x1 - u2[q] * x2) * d[q];
    x2 = x1;
    x1 = xx;
    f[q] = xx;   // f now holds x
    if (i0 + q < NR) {
      const double nn = double(2 * (i0 + q + 2) + p);
      s0 += xx;
      s1 += nn * nn * xx;
    }
  }
  s0 = seg_sum<W>(s0);
  s1 = seg_sum<W>(s1);
  const int si = NR * kFacP;
  const double h0 = -(fac_at<GF>(fac, si) * s0 + fac_at<GF>(fac, si + 1) * s1);
  const double h1 = -(fac_at<GF>(fac, si + 2) * s0 + fac_at<GF>(fac, si + 3) * s1);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = i0 + q, ic = min(i, NR - 1);
    const double w5 = fac_at<GF>(fac, ic * kFacP + 5), w6 = fac_at<GF>(fac, ic * kFacP + 6);
    if (i < NR) v[2 * (i + 2) + p] = f[q] - w5 * h0 - w6 * h1;
  }
  if (li == 0) {
    v[p] = h0;
    v[2 + p] = h1;
  }
}

// Copies the factor blocks of modes m0..m0+MT-1 (both parities) into LDS,
// eight loads in flight per thread.
template <int MT>
__device__ __forceinline__ void stage_factors(double* sF, const double* __restrict__ fac, int stride, int m0,
                                              int Mx) {
  const int ls = lds_fac_stride(stride);
  const int total = min(MT, Mx - m0) * 2 * stride;
  const gview<double> src = gv(fac) + size_t(m0) * 2 * stride;
  constexpr int U = 8;
  for (int base = threadIdx.x; base < total; base += kBlock * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * kBlock;
      v[u] = (e < total) ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * kBlock;
      if (e < total) {
        const int b = e / stride;
        sF[b * ls + (e - b * stride)] = v[u];
      }
    }
  }
}

// Band-table entries of one equation row r (both equations), kept in
// registers by the thread that owns row r.
struct RowTables {
  double s10[3], d2, a[3], b[5], d4;
};
__device__ __forceinline__ RowTables load_row_tables(const GridDev& g, int r) {
  RowTables t;
  const int p = r & 1, i = r >> 1, k = p * g.n + i;
#pragma unroll
  for (int q = 0; q < 3; ++q) t.s10[q] = gv(g.bS10)[k * 3 + q];
  t.d2 = gv(g.bD2)[k];
#pragma unroll
  for (int q = 0; q < 3; ++q) t.a[q] = gv(g.bA)[k * 3 + q];
#pragma unroll
  for (int q = 0; q < 5; ++q) t.b[q] = gv(g.bB)[k * 5 + q];
  t.d4 = gv(g.bD4)[k];
  return t;
}

// Byte offsets of the stage kernel's LDS regions beyond the two FP64 tiles
// and the product region: the staged factor blocks of the temperature (sFT)
// and streamfunction (sFP) equations.  Without `pre` both take turns in the
// union with the products; with `pre` each has its own region, filled at
// kernel entry.  Phase G's scratch starts at the old-state tile.
struct StageLds {
  size_t sFT, sFP, total;
};
template <int NZ, int MT>
__host__ __device__ inline StageLds stage_lds(size_t rb, int fsT, int fsP, bool pre, bool split = false,
                                              bool lean = false) {
  constexpr size_t PZ = 3 * NZ / 2;
  const size_t tile = sizeof(double) * 4 * MT * (NZ + 1);
  if (lean) {   // right-hand sides and the mean of u w only
    StageLds L{};
    L.sFT = L.sFP = 0;
    L.total = tile + rb * PZ;
    return L;
  }
  // products of the tile (fused path) or only the mean of u w (split path)
  const size_t nh = split ? rb * PZ : rb * (4 * PZ * MT + PZ);
  // phase G scratch: only the two-pass inverse transform of two-mode tiles
  const size_t vals = (MT <= 2 && !split) ? rb * PZ * MT * 12 : 0;
  StageLds L{};
  if (!pre) {
    const size_t fac = sizeof(double) * size_t(MT) * 2 * size_t((fsT > fsP ? fsT : fsP) | 1);
    const size_t uni = nh > fac ? nh : fac;
    L.sFT = L.sFP = 2 * tile;
    L.total = tile + (tile + uni > vals ? tile + uni : vals);
    return L;
  }
  size_t o = 2 * tile + ((nh + 15) & ~size_t(15));
  L.sFT = o;
  o += sizeof(double) * size_t(MT) * 2 * size_t(fsT | 1);
  L.sFP = o;
  o += sizeof(double) * size_t(MT) * 2 * size_t(fsP | 1);
  L.total = o > tile + vals ? o : tile + vals;
  return L;
}

// One block per (slice, tile of MT modes).  Each thread owns one row
// r = tid mod NZ of the equations and the columns c = tid / NZ + k (256/NZ)
// of the tile (column c = (field, mode, re/im)).
//
// LDS (doubles first):
//   sY  [2 field][MT][2][NZ+1]   right-hand sides -> new stage values
//   sX  [2 field][MT][2][NZ+1]   old state of the tile
//   U   union { Real sN[2][PZ][2 MT] + sq[PZ];  double sF[2 MT][odd stride] }
//   (latency variant: sN + sq, then the factor blocks of both equations in
//   regions of their own; see stage_lds)
//
// Split path (SPLIT, mixed precision): the forward transform of the products
// (phase B) and the inverse transform of the new stage (phase G) run as
// batched GEMMs in fwd_gemm_kernel and inv_gemm_kernel.  Phase B then only
// reads the explicit terms that fwd_gemm_kernel wrote to this stage's slot
// of Ehist (and forms the mean-flow term of mode 0 from the mean of u w),
// and phase G writes the new stage in FP32, split by parity, to Yf.
// Waves per SIMD the per-mode kernel's register budget is fitted to: five
// for the lean split-path variant of the longest systems (its latency-bound
// solves need blocks in flight more than registers), by need otherwise.
template <int NZ, bool SPLIT>
constexpr int stage_min_waves() { return (SPLIT && NZ >= 256) ? 5 : 1; }

template <typename Real, int NZ, int MT, bool SPLIT = false>
__global__ void __launch_bounds__(kBlock, (stage_min_waves<NZ, SPLIT>()))
stage_kernel(GridDev g, StageArgs a, const Real* __restrict__ Nh, const Real* __restrict__ qbar,
             double* __restrict__ X, Real* __restrict__ Ehist, double* __restrict__ LYhist,
             Real* __restrict__ Q, double* __restrict__ Eout, float* __restrict__ Yf) {
  constexpr int PZ = 3 * NZ / 2, PH = PZ / 2, LD = NZ + 1, NH = NZ / 2;
  constexpr int NRT = NH - 1, NRP = NH - 2;
  constexpr int NC = 4 * MT;                 // columns (field, mode, re/im)
  constexpr int CR = kBlock / NZ;            // columns in parallel
  constexpr int KC = (NC + CR - 1) / CR;     // columns per thread
  // Two-mode tiles serve the latency-bound launches (the single-slice coarse
  // sweep, the largest Nz): more work items per phase and register-held
  // solves.  Wider tiles serve the throughput-bound batched launches.
  constexpr bool kWide = (MT <= 2);
  // Latency variant of the small two-mode launches: the loads that do not
  // depend on this launch's own results (factor blocks, band rows, stage
  // history) are issued at entry beside the product loads instead of at the
  // start of the phases that use them.  (The transform maps stay in global
  // memory: staged in LDS they cost more at entry and in bank conflicts than
  // their cached loads.)
  constexpr bool kPre = kWide && NZ <= 64;
  // Lean variant of the split path for long systems (chunked solves): the
  // old state and the band factors are read from global memory where they
  // are used instead of being staged in LDS, so that four times as many
  // blocks fit a compute unit (the solves are latency-bound).
  constexpr bool kLean = SPLIT && NRT >= 64;
  static_assert(kBlock % NZ == 0, "NZ must divide the block size");
  if (g.urgent) __builtin_amdgcn_s_setprio(3);
  extern __shared__ __align__(16) unsigned char smem[];
  const int Mx = g.Mx;
  const int ntile = g.ntile;   // ceil(Mx / MT)
  const int bid = work_block(g.one_xcd);
  if (bid < 0) return;
  const int b = bid / ntile, tile = bid - b * ntile;
  const int s = ring_slot(b, a.slot0, a.cap);
  const int m0 = tile * MT;
  const int st = g.state;
  // this slot's run (ensemble launches): factors, diffusivities, stage
  // coefficients h a_ij of this stage
  const cview<RunDev> rd = cv(batch_run(g, b));
  const double* facTg = rd->facT;
  const double* facPg = rd->facP;
  const double nu_r = rd->nu, kappa_r = rd->kappa;
  const int si = a.stage;
  auto HAE = [rd, si](int j) { return rd->hae[si][j]; };
  auto HAI = [rd, si](int j) { return rd->hai[si][j]; };
  const double haii = rd->hai[si][si];
  double* sY = reinterpret_cast<double*>(smem);
  double* sX = sY + 4 * MT * LD;   // not used by the lean variant
  unsigned char* uni = reinterpret_cast<unsigned char*>(kLean ? sX : sX + 4 * MT * LD);
  Real* sN = reinterpret_cast<Real*>(uni);
  Real* sq = SPLIT ? sN : sN + 4 * PZ * MT;
  const StageLds Ls = stage_lds<NZ, MT>(sizeof(Real), g.facT_stride, g.facP_stride, kPre, SPLIT, kLean);
  double* sFT = reinterpret_cast<double*>(smem + Ls.sFT);
  double* sFP = reinterpret_cast<double*>(smem + Ls.sFP);
  const int tid = threadIdx.x;
  const int r = tid % NZ, c0 = tid / NZ;     // this thread's row and first column
  // column c -> (field, mode within tile, re/im); LDS and HBM offsets
  auto fld = [](int c) { return c / (2 * MT); };
  auto mtc = [](int c) { return (c >> 1) % MT; };
  auto yoff = [](int c) { return c * LD; };  // == ((f MT + mt) 2 + ri) LD
  auto goff = [&](int c) {
    return size_t((fld(c) * Mx + m0 + mtc(c)) * 2 + (c & 1)) * NZ;
  };
  const double* Xs = batch_state(g, X, b, s);

  // ---- kPre: entry loads into registers (stored to LDS by pre_store)
  constexpr int FTN = (MT * 2 * 2 * NZ + kBlock - 1) / kBlock;        // facT stride 2 Nz
  constexpr int FPN = (MT * 2 * (7 * NZ / 2) + kBlock - 1) / kBlock;  // facP stride <= 3.5 Nz
  double fT[kPre ? FTN : 1], fP[kPre ? FPN : 1];
  double hE[kPre ? KC : 1][3], hL[kPre ? KC : 1][3];
  RowTables tbp{};
  const bool stg = (a.mode == kModeStage);
  const int nmt = min(MT, Mx - m0);
  const int totT = stg ? nmt * 2 * g.facT_stride : 0, totP = stg ? nmt * 2 * g.facP_stride : 0;
  if constexpr (kPre) {
    const double* srcT = facTg + size_t(m0) * 2 * g.facT_stride;
    const double* srcP = facPg + size_t(m0) * 2 * g.facP_stride;
#pragma unroll
    for (int u = 0; u < FTN; ++u) {
      const int e = tid + u * kBlock;
      fT[u] = (e < totT) ? gv(srcT)[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < FPN; ++u) {
      const int e = tid + u * kBlock;
      fP[u] = (e < totP) ? gv(srcP)[e] : 0.0;
    }
    if (stg) tbp = load_row_tables(g, r);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int c = c0 + kc * CR;
      const bool ok = stg && c < NC && m0 + mtc(c) < Mx &&
                      r < ((fld(c) == 0 && m0 + mtc(c) > 0) ? NZ - 4 : NZ - 2);
      const size_t off = ok ? goff(c) + r : 0;
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        hE[kc][jj] = (ok && jj + 1 < a.stage) ? double(Ehist[(size_t(jj) * a.cap + s) * st + off]) : 0.0;
        hL[kc][jj] = (ok && jj + 2 <= a.stage) ? LYhist[(size_t(jj) * a.cap + s) * st + off] : 0.0;
      }
    }
  }
  auto pre_store = [&]() {
    if constexpr (kPre) {
      const int lsT = lds_fac_stride(g.facT_stride), lsP = lds_fac_stride(g.facP_stride);
#pragma unroll
      for (int u = 0; u < FTN; ++u) {
        const int e = tid + u * kBlock;
        if (e < totT) {
          const int bb = e / g.facT_stride;
          sFT[bb * lsT + (e - bb * g.facT_stride)] = fT[u];
        }
      }
#pragma unroll
      for (int u = 0; u < FPN; ++u) {
        const int e = tid + u * kBlock;
        if (e < totP) {
          const int bb = e / g.facP_stride;
          sFP[bb * lsP + (e - bb * g.facP_stride)] = fP[u];
        }
      }
      // factor blocks longer than the register bound (not for the plans built here)
      for (int e = FTN * kBlock + tid; e < totT; e += kBlock) {
        const int bb = e / g.facT_stride;
        sFT[bb * lsT + (e - bb * g.facT_stride)] = gv(facTg)[size_t(m0) * 2 * g.facT_stride + e];
      }
      for (int e = FPN * kBlock + tid; e < totP; e += kBlock) {
        const int bb = e / g.facP_stride;
        sFP[bb * lsP + (e - bb * g.facP_stride)] = gv(facPg)[size_t(m0) * 2 * g.facP_stride + e];
      }
    }
  };

  if (a.mode == kModeZinv) {
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int c = c0 + kc * CR;
      if (c < NC) sY[yoff(c) + r] = (m0 + mtc(c) < Mx) ? gv(Xs)[goff(c) + r] : 0.0;
    }
    pre_store();
    __syncthreads();
  } else {
    // ---- phase A: products of this tile on the padded Gauss points (two
    // contiguous runs of PZ x 2 MT values in the mode-tile-major layout), and
    // the old state; eight loads in flight per thread
    if constexpr (!SPLIT) {
      constexpr int U = 8;
      constexpr int half = PZ * 2 * MT, total = 2 * half;
      const size_t tq = size_t(PZ) * 2 * MT;
      const Real* n0 = Nh + (size_t(s) * 2 * ntile + tile) * tq;
      const Real* n1 = n0 + size_t(ntile) * tq;
      for (int base = tid; base < total; base += kBlock * U) {
        Real v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * kBlock;
          v[u] = (e < half) ? n0[e] : ((e < total) ? n1[e - half] : Real(0));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * kBlock;
          if (e < total) sN[e] = v[u];
        }
      }
    }
    if (m0 == 0)
      for (int j = tid; j < PZ; j += kBlock) sq[j] = qbar[size_t(s) * PZ + j];
    if (a.mode == kModeStage && !kLean) {
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;
        if (c < NC) sX[yoff(c) + r] = (m0 + mtc(c) < Mx) ? gv(Xs)[goff(c) + r] : 0.0;
      }
    }
    pre_store();
    __syncthreads();
    const gview<Real> W = gv(reinterpret_cast<const Real*>(g.Wfwd));
    // writes the explicit terms of item (f, row) to LDS (scaled) and HBM
    auto store_explicit = [&](int f, int rr, const Real* acc) {
      if (f == 2) {
        const double E = double(acc[0]);
        const size_t o0 = size_t(0) * NZ + rr, o1 = size_t(1) * NZ + rr;   // field 0, m 0, re / im
        if (a.mode == kModeExplicit) {
          Eout[o0] = E;
          Eout[o1] = 0.0;
        } else {
          sY[0 * LD + rr] = HAE(a.stage - 1) * E;
          sY[1 * LD + rr] = 0.0;
          if (a.store_E) {
            Real* eh = Ehist + (size_t(a.stage - 1) * a.cap + s) * st;
            eh[o0] = Real(E);
            eh[o1] = Real(0);
          }
        }
        return;
      }
#pragma unroll
      for (int cc = 0; cc < 2 * MT; ++cc) {
        const int mt = cc >> 1, ri = cc & 1, m = m0 + mt;
        if (m >= Mx || (f == 0 && m == 0)) continue;
        const double E = double(acc[cc]);
        const size_t off = size_t((f * Mx + m) * 2 + ri) * NZ + rr;
        if (a.mode == kModeExplicit) {
          Eout[off] = E;
        } else {
          sY[((f * MT + mt) * 2 + ri) * LD + rr] = HAE(a.stage - 1) * E;
          if (a.store_E) Ehist[(size_t(a.stage - 1) * a.cap + s) * st + off] = Real(E);
        }
      }
    };
    // ---- phase B: explicit terms of the previous stage on the band rows.
    // Item (f, row): one row of the folded forward map against every column
    // (mode, re/im) of the field; item f = 2 is the u_bar column of mode 0.
    if constexpr (SPLIT) {
      // the forward GEMM's result for this stage; the u_bar column of mode 0
      // (whose slot holds no streamfunction) from the mean of u w
      // (all loads first, at clamped indices, then the stores)
      const gview<Real> Ein = gv(Ehist) + (size_t(a.stage - 1) * a.cap + s) * st;
      Real ev[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;
        const int f = fld(c), m = m0 + mtc(c);
        const bool ok = c < NC && m < Mx && !(f == 0 && m == 0) && r < ((f == 0) ? NZ - 4 : NZ - 2);
        ev[kc] = Ein[ok ? goff(c) + r : 0];
      }
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;
        const int f = fld(c), m = m0 + mtc(c);
        if (!(c < NC && m < Mx && !(f == 0 && m == 0) && r < ((f == 0) ? NZ - 4 : NZ - 2))) continue;
        const double E = double(ev[kc]);
        if (a.mode == kModeExplicit)
          Eout[goff(c) + r] = E;
        else
          sY[yoff(c) + r] = HAE(a.stage - 1) * E;
      }
      if (m0 == 0)
        for (int rr = tid; rr < NZ - 2; rr += kBlock) {
          const gview<Real> w = W + (size_t(2) * NZ + rr) * PH;
          const Real sg = (rr & 1) ? Real(1) : Real(-1);
          Real acc[2 * MT];
          acc[0] = Real(0);
#pragma unroll 8
          for (int j = 0; j < PH; ++j) acc[0] += w[j] * (sq[j] + sg * sq[PZ - 1 - j]);
          store_explicit(2, rr, acc);
        }
    } else if constexpr (kWide) {
      // two-mode tiles: each item split over JS lanes that take every JS-th
      // Gauss point, summed by shuffles
    constexpr int JS = 4;
    // Gauss points per lane; the latency variant issues all their map loads
    // at once
    constexpr int NJ = (PH + JS - 1) / JS, UB = kPre ? NJ : 4;
    const int nitems = ((m0 == 0) ? 3 : 2) * NZ;
    for (int e = tid; e < nitems * JS; e += kBlock) {
      const int lane = e & (JS - 1), item = e / JS;
      const int rr = item % NZ, f = item / NZ;
      Real acc[2 * MT];
#pragma unroll
      for (int c = 0; c < 2 * MT; ++c) acc[c] = Real(0);
      if (f == 2) {
        if (rr < NZ - 2) {
          const gview<Real> w = W + (size_t(2) * NZ + rr) * PH;
          const Real sg = (rr & 1) ? Real(1) : Real(-1);
#pragma unroll UB
          for (int i = 0; i < NJ; ++i) {
            const int j = lane + i * JS;
            if (j < PH) acc[0] += w[j] * (sq[j] + sg * sq[PZ - 1 - j]);
          }
        }
      } else if (rr < ((f == 0) ? NZ - 4 : NZ - 2)) {
        const gview<Real> w = W + (size_t(f == 0 ? 0 : 1) * NZ + rr) * PH;
        const Real* src = sN + (f == 0 ? 0 : PZ * 2 * MT);
        const Real sg = (rr & 1) ? Real(-1) : Real(1);
#pragma unroll UB
        for (int i = 0; i < NJ; ++i) {
          const int j = lane + i * JS;
          if (j >= PH) break;
          const Real wv = w[j];
          const Real* a0 = src + j * 2 * MT;
          const Real* a1 = src + (PZ - 1 - j) * 2 * MT;
#pragma unroll
          for (int c = 0; c < 2 * MT; ++c) acc[c] += wv * (a0[c] + sg * a1[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < 2 * MT; ++c) {
        acc[c] += __shfl_xor(acc[c], 1, JS);
        acc[c] += __shfl_xor(acc[c], 2, JS);
      }
      if (lane != 0) continue;
      store_explicit(f, rr, acc);
    }
    } else {
      // wider tiles: one item per thread
    const int nitems = ((m0 == 0) ? 3 : 2) * NZ;
    for (int e = tid; e < nitems; e += kBlock) {
      const int rr = e % NZ, f = e / NZ;
      Real acc[2 * MT];
#pragma unroll
      for (int c = 0; c < 2 * MT; ++c) acc[c] = Real(0);
      if (f == 2) {
        if (rr < NZ - 2) {
          const gview<Real> w = W + (size_t(2) * NZ + rr) * PH;
          const Real sg = (rr & 1) ? Real(1) : Real(-1);
#pragma unroll 8
          for (int j = 0; j < PH; ++j) acc[0] += w[j] * (sq[j] + sg * sq[PZ - 1 - j]);
        }
      } else if (rr < ((f == 0) ? NZ - 4 : NZ - 2)) {
        const gview<Real> w = W + (size_t(f == 0 ? 0 : 1) * NZ + rr) * PH;
        const Real* src = sN + (f == 0 ? 0 : PZ * 2 * MT);
        const Real sg = (rr & 1) ? Real(-1) : Real(1);
#pragma unroll 8
        for (int j = 0; j < PH; ++j) {
          const Real wv = w[j];
          const Real* a0 = src + j * 2 * MT;
          const Real* a1 = src + (PZ - 1 - j) * 2 * MT;
#pragma unroll
          for (int c = 0; c < 2 * MT; ++c) acc[c] += wv * (a0[c] + sg * a1[c]);
        }
      }
      store_explicit(f, rr, acc);
    }
    }
    if (a.mode == kModeExplicit) return;
    __syncthreads();
    // temperature factors into the (now free) union region
    if constexpr (!kPre && !kLean) stage_factors<MT>(sFT, facTg, g.facT_stride, m0, Mx);
    // ---- phase C: right-hand side of stage i on this thread's row
    const RowTables tb = kPre ? tbp : load_row_tables(g, r);
    // the lean variant loads the row tables again where they are used after
    // the solves instead of holding them in registers across them (the row
    // index is made opaque so that the loads are not merged)
    auto tables_again = [&]() -> RowTables {
      if constexpr (kLean) {
        int rr = r;
        asm volatile("" : "+v"(rr));
        return load_row_tables(g, rr);
      } else {
        return tb;
      }
    };
    {
      // Every load of this phase is issued for every lane with its index
      // clamped into the arrays (values of rows and stages that do not
      // contribute are selected away afterwards), so that no branch or wait
      // separates them: one round trip to memory for the whole phase.
      double acc[KC];
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;
        const int f = fld(c), m = m0 + mtc(c);
        const bool psi = (f == 0 && m > 0);
        const bool ok = c < NC && m < Mx && r < (psi ? NZ - 4 : NZ - 2);
        const int cs = ok ? c : 0;   // a column of this tile (mode m0 exists)
        // the old state at row r + 2 t (clamped): global memory (lean
        // variant) or its LDS tile
        double xr[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          const int i = min(r + 2 * t, NZ - 1);
          if constexpr (kLean)
            xr[t] = gv(Xs)[goff(cs) + i];
          else
            xr[t] = sX[yoff(cs) + i];
        }
        const size_t off = goff(cs) + r;
        double hE0[3], hL0[3];
        if constexpr (!kPre) {
          // a history term this stage does not use is loaded from an
          // address this kernel reads anyway (this stage's explicit terms,
          // the old state), so that it costs no HBM traffic
#pragma unroll
          for (int jj = 0; jj < 3; ++jj) {
            const bool use = jj + 1 < a.stage;
            hE0[jj] = double(gv(Ehist)[(size_t(use ? jj : a.stage - 1) * a.cap + s) * st + off]);
            const gview<double> lsrc = use ? gv(LYhist) + (size_t(jj) * a.cap + s) * st : gv(Xs);
            hL0[jj] = lsrc[off];
          }
        }
        double MX;
        if (!psi) {
          MX = tb.s10[0] * xr[0] + tb.s10[1] * xr[1] + (r + 4 < NZ ? tb.s10[2] * xr[2] : 0.0);
        } else {
          const double k = m * g.kscale;
          double sa = 0, sb = 0;
#pragma unroll
          for (int t = 0; t < 3; ++t) sa += (r + 2 + 2 * t < NZ) ? tb.a[t] * xr[t + 1] : 0.0;
#pragma unroll
          for (int t = 0; t < 5; ++t) sb += (r + 2 * t < NZ) ? tb.b[t] * xr[t] : 0.0;
          MX = sa - k * k * sb;
        }
        double h = MX + sY[yoff(cs) + r];
        if constexpr (kPre) {
#pragma unroll
          for (int jj = 0; jj < 3; ++jj)
            if (jj + 1 < a.stage) h += HAE(jj) * hE[kc][jj];
#pragma unroll
          for (int jj = 1; jj < 4; ++jj)
            if (jj < a.stage) h += HAI(jj) * hL[kc][jj - 1];
        } else {
#pragma unroll
          for (int jj = 0; jj < 3; ++jj)
            if (jj + 1 < a.stage) h += HAE(jj) * hE0[jj];
#pragma unroll
          for (int jj = 1; jj < 4; ++jj)
            if (jj < a.stage) h += HAI(jj) * hL0[jj - 1];
        }
        acc[kc] = ok ? h : 0.0;
      }
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;
        if (c < NC && m0 + mtc(c) < Mx && r < ((fld(c) == 0 && m0 + mtc(c) > 0) ? NZ - 4 : NZ - 2))
          sY[yoff(c) + r] = acc[kc];
      }
    }
    __syncthreads();
    // ---- phase D: temperature solves of the systems (mode, parity, re/im).
    // Two-mode tiles (latency-bound launches): scans with one lane per band
    // row up to 63 rows.  Wider tiles (throughput-bound batched launches,
    // where the other blocks' phases hide the sweep): one lane per system.
    if constexpr (NRT >= 64) {
      // long systems: chunked scans, 32 lanes of four rows per system
      for (int sys0 = 0; sys0 < 4 * MT; sys0 += kBlock / kChunkLanes) {
        const int sys = sys0 + tid / kChunkLanes, li = tid % kChunkLanes;
        if (sys < 4 * MT) {
          const int mt = sys >> 2, p = (sys >> 1) & 1, ri = sys & 1, m = m0 + mt;
          if (m < Mx) {
            double gbc = 0.0;
            if (m == 0 && ri == 0) gbc = g.bcT[p];
            const double* fac = kLean ? facTg + (size_t(m) * 2 + p) * g.facT_stride
                                      : sFT + (mt * 2 + p) * lds_fac_stride(g.facT_stride);
            solve_T_chunk<NRT, kChunkLanes, (NRT + kChunkLanes - 1) / kChunkLanes, kLean>(
                sY + ((MT + mt) * 2 + ri) * LD, p, fac, gbc, g.fluxT != 0, li);
          }
        }
      }
    } else if constexpr (kWide && NRT < 64) {
      constexpr int WS = seg_width(NRT);
      for (int sys0 = 0; sys0 < 4 * MT; sys0 += kBlock / WS) {
        const int sys = sys0 + tid / WS, li = tid % WS;
        if (sys < 4 * MT) {
          const int mt = sys >> 2, p = (sys >> 1) & 1, ri = sys & 1, m = m0 + mt;
          if (m < Mx) {
            double gbc = 0.0;
            if (m == 0 && ri == 0) gbc = g.bcT[p];
            solve_T_scan<NRT, WS>(sY + ((MT + mt) * 2 + ri) * LD, p,
                                  sFT + (mt * 2 + p) * lds_fac_stride(g.facT_stride), gbc, g.fluxT != 0, li);
          }
        }
      }
    } else if (tid < 4 * MT) {
      const int mt = tid >> 2, p = (tid >> 1) & 1, ri = tid & 1, m = m0 + mt;
      if (m < Mx) {
        double gbc = 0.0;
        if (m == 0 && ri == 0) gbc = g.bcT[p];
        solve_T_format<NRT, kWide>(sY + ((MT + mt) * 2 + ri) * LD, p,
                                   sFT + (mt * 2 + p) * lds_fac_stride(g.facT_stride), gbc, g.fluxT != 0);
      }
    }
    __syncthreads();
    // flow factors; implicit buoyancy of the new temperature into psi
    if constexpr (!kPre && !kLean) stage_factors<MT>(sFP, facPg, g.facP_stride, m0, Mx);
    if (r < NZ - 4) {
      const RowTables tbB = tables_again();
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;          // only field-0 columns (c < 2 MT)
        if (c >= 2 * MT) continue;
        const int mt = c >> 1, ri = c & 1, m = m0 + mt;
        if (m >= Mx || m == 0) continue;
        const double k = m * g.kscale;
        const double* tv = sY + ((MT + mt) * 2 + (ri ^ 1)) * LD;
        double sb = 0;
#pragma unroll
        for (int t = 0; t < 5; ++t)
          if (r + 2 * t < NZ) sb += tbB.b[t] * tv[r + 2 * t];
        sY[yoff(c) + r] += haii * (ri == 0 ? k * sb : -k * sb);
      }
    }
    __syncthreads();
    if constexpr (NRT >= 64) {
      for (int sys0 = 0; sys0 < 4 * MT; sys0 += kBlock / kChunkLanes) {
        const int sys = sys0 + tid / kChunkLanes, li = tid % kChunkLanes;
        if (sys < 4 * MT) {
          const int mt = sys >> 2, p = (sys >> 1) & 1, ri = sys & 1, m = m0 + mt;
          if (m < Mx) {
            const double* fac = kLean ? facPg + (size_t(m) * 2 + p) * g.facP_stride
                                      : sFP + (mt * 2 + p) * lds_fac_stride(g.facP_stride);
            double* v = sY + (mt * 2 + ri) * LD;
            if (m == 0)
              solve_T_chunk<NRT, kChunkLanes, (NRT + kChunkLanes - 1) / kChunkLanes, kLean>(v, p, fac, 0.0, false, li);
            else
              solve_P_chunk<NRP, kChunkLanes, (NRP + kChunkLanes - 1) / kChunkLanes, kLean>(v, p, fac, li);
          }
        }
      }
    } else if constexpr (kWide && NRT < 64) {
      constexpr int WS = seg_width(NRT);   // NRP < NRT: the same segments fit
      for (int sys0 = 0; sys0 < 4 * MT; sys0 += kBlock / WS) {
        const int sys = sys0 + tid / WS, li = tid % WS;
        if (sys < 4 * MT) {
          const int mt = sys >> 2, p = (sys >> 1) & 1, ri = sys & 1, m = m0 + mt;
          if (m < Mx) {
            const double* fac = sFP + (mt * 2 + p) * lds_fac_stride(g.facP_stride);
            double* v = sY + (mt * 2 + ri) * LD;
            if (m == 0)
              solve_T_scan<NRT, WS>(v, p, fac, 0.0, false, li);
            else
              solve_P_scan<NRP, WS>(v, p, fac, li);
          }
        }
      }
    } else if (tid < 4 * MT) {
      const int mt = tid >> 2, p = (tid >> 1) & 1, ri = tid & 1, m = m0 + mt;
      if (m < Mx) {
        const double* fac = sFP + (mt * 2 + p) * lds_fac_stride(g.facP_stride);
        double* v = sY + (mt * 2 + ri) * LD;
        if (m == 0)
          solve_T_format<NRT, kWide>(v, p, fac, 0.0, false);
        else
          solve_P_format<NRP, kWide>(v, p, fac);
      }
    }
    __syncthreads();
    // ---- phase F: L Y_i for later stages; the new state at the last stage
    if (a.store_LY) {
      const RowTables tbF = tables_again();
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;
        if (c >= NC) continue;
        const int f = fld(c), mt = mtc(c), ri = c & 1, m = m0 + mt;
        if (m >= Mx) continue;
        const bool psi = (f == 0 && m > 0);
        if (r >= (psi ? NZ - 4 : NZ - 2)) continue;
        const double* yv = sY + yoff(c);
        const double k = m * g.kscale, k2 = k * k;
        double L;
        if (f == 1) {
          const double sm = tbF.s10[0] * yv[r] + tbF.s10[1] * yv[r + 2] + (r + 4 < NZ ? tbF.s10[2] * yv[r + 4] : 0.0);
          L = kappa_r * (tbF.d2 * yv[r + 2] - k2 * sm);
        } else if (m == 0) {
          L = nu_r * tbF.d2 * yv[r + 2];
        } else {
          const double* tv = sY + ((MT + mt) * 2 + (ri ^ 1)) * LD;
          double sa = 0, sb = 0, st5 = 0;
#pragma unroll
          for (int t = 0; t < 3; ++t)
            if (r + 2 + 2 * t < NZ) sa += tbF.a[t] * yv[r + 2 + 2 * t];
#pragma unroll
          for (int t = 0; t < 5; ++t)
            if (r + 2 * t < NZ) {
              sb += tbF.b[t] * yv[r + 2 * t];
              st5 += tbF.b[t] * tv[r + 2 * t];
            }
          L = nu_r * (tbF.d4 * yv[r + 4] - 2.0 * k2 * sa + k2 * k2 * sb) + (ri == 0 ? k * st5 : -k * st5);
        }
        LYhist[(size_t(a.stage - 1) * a.cap + s) * st + goff(c) + r] = L;
      }
    }
    if (a.write_X) {
      const gwview<double> Xw = gw(const_cast<double*>(Xs));
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        const int c = c0 + kc * CR;
        if (c < NC && m0 + mtc(c) < Mx) Xw[goff(c) + r] = sY[yoff(c) + r];
      }
    }
    if (!a.do_zinv) return;
  }
  if constexpr (SPLIT) {
    // ---- phase G (split path): the new stage in FP32 by parity, for the
    // inverse GEMM
    float* y = Yf + size_t(s) * st;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int c = c0 + kc * CR;
      if (c < NC && m0 + mtc(c) < Mx) y[goff(c) + (r & 1) * (NZ / 2) + (r >> 1)] = float(sY[yoff(c) + r]);
    }
    return;
  }
  // ---- phase G: values and z-derivatives of the new stage at the padded
  // Gauss points, six quantities per mode (m contiguous in HBM).
  // Two-mode tiles: pass 1, item (column, j < PZ/2): the products
  // E D^q c (q = 0..3 for psi / u_bar, 0..1 for T) at j and, by reflection,
  // at PZ-1-j, into sV (the old-state tile and the union are dead here).
  // Pass 2, item (j, mode): the six quantities, written m-contiguous.
  if constexpr (kWide) {
  {
    Real* sV = reinterpret_cast<Real*>(sX);   // [PZ][MT][2 re/im][6]
    const gview<Real> Wi = gv(reinterpret_cast<const Real*>(g.Winv));
    for (int e = tid; e < PH * NC; e += kBlock) {
      // field-major order keeps the four-product (psi) items together
      const int f = e / (PH * 2 * MT), e2 = e - f * (PH * 2 * MT);
      const int cc = e2 % (2 * MT), j = e2 / (2 * MT);
      const int mt = cc >> 1, ri = cc & 1, m = m0 + mt;
      if (m >= Mx) continue;
      const double* yv = sY + ((f * MT + mt) * 2 + ri) * LD;
      Real acc[2][4];
#pragma unroll
      for (int pp = 0; pp < 2; ++pp)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[pp][q] = Real(0);
      const gview<Real> w = Wi + size_t(j) * NZ;
      constexpr size_t QS = size_t(PH) * NZ;
      constexpr int UG = kPre ? 8 : 4;   // coefficient pairs per round of map loads
      if (f == 0) {
#pragma unroll UG
        for (int nn = 0; nn < NZ; nn += 2) {
#pragma unroll
          for (int pp = 0; pp < 2; ++pp) {
            const Real cv = Real(yv[nn + pp]);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[pp][q] += w[q * QS + nn + pp] * cv;
          }
        }
      } else {
#pragma unroll UG
        for (int nn = 0; nn < NZ; nn += 2) {
#pragma unroll
          for (int pp = 0; pp < 2; ++pp) {
            const Real cv = Real(yv[nn + pp]);
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[pp][q] += w[q * QS + nn + pp] * cv;
          }
        }
      }
      const int slot0 = (f == 0) ? 0 : 4, nq = (f == 0) ? 4 : 2;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q >= nq) break;
        // d^q T_n / dz^q at the reflected point is (-1)^(n+q) times that at j
        const Real lo = acc[0][q] + acc[1][q], hi = acc[0][q] - acc[1][q];
        sV[((j * MT + mt) * 2 + ri) * 6 + slot0 + q] = lo;
        sV[(((PZ - 1 - j) * MT + mt) * 2 + ri) * 6 + slot0 + q] = (q & 1) ? -hi : hi;
      }
    }
    __syncthreads();
    for (int e = tid; e < PZ * MT; e += kBlock) {
      const int mt = e % MT, jj = e / MT, m = m0 + mt;
      if (m >= Mx) continue;
      const Real* vr = sV + (jj * MT + mt) * 12;       // re: [0..5], im: [6..11]
      const Real* vi = vr + 6;
      const Real k = Real(m * g.kscale), k2 = k * k;
      Real out[6][2];
      if (m > 0) {
        out[0][0] = vr[1]; out[0][1] = vi[1];                            // u = psi_z
        out[1][0] = k * vi[0]; out[1][1] = -k * vr[0];                   // w = -i k psi
        const Real omr = vr[2] - k2 * vr[0], omi = vi[2] - k2 * vi[0];
        out[2][0] = -k * omi; out[2][1] = k * omr;                       // omega_x = i k omega
        out[3][0] = vr[3] - k2 * vr[1]; out[3][1] = vi[3] - k2 * vi[1];  // omega_z
        out[4][0] = -k * vi[4]; out[4][1] = k * vr[4];                   // T_x = i k T
        out[5][0] = vr[5]; out[5][1] = vi[5];                            // T_z
      } else {
        out[0][0] = vr[0]; out[0][1] = 0;                                // u = u_bar
        out[1][0] = 0; out[1][1] = 0;
        out[2][0] = 0; out[2][1] = 0;
        out[3][0] = vr[2]; out[3][1] = 0;                                // omega_z = u_bar_zz
        out[4][0] = 0; out[4][1] = 0;
        out[5][0] = vr[5]; out[5][1] = 0;
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        Cx<Real>* d = reinterpret_cast<Cx<Real>*>(Q) + ((size_t(s) * 6 + q) * ntile + tile) * (PZ * MT) +
                      jj * MT + mt;
        *d = {out[q][0], out[q][1]};
      }
    }
  }
  } else {
  // wider tiles: item (j < PZ/2, mode) computes all six products and
  // quantities at j and PZ-1-j directly (fewer map loads per column)
  const gview<Real> Wi = gv(reinterpret_cast<const Real*>(g.Winv));
  for (int e = tid; e < PH * MT; e += kBlock) {
    const int mt = e % MT, j = e / MT, m = m0 + mt;
    if (m >= Mx) continue;
    // acc[parity][q][re/im]: q = 0..3 on psi (E D^q psi), 4..5 on T (E, E D)
    Real acc[2][6][2];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[pp][q][0] = acc[pp][q][1] = Real(0);
    const double* pr = sY + (mt * 2 + 0) * LD;
    const double* pi = sY + (mt * 2 + 1) * LD;
    const double* tr = sY + ((MT + mt) * 2 + 0) * LD;
    const double* ti = sY + ((MT + mt) * 2 + 1) * LD;
    const gview<Real> w0 = Wi + (size_t(0) * PH + j) * NZ;
    const gview<Real> w1 = Wi + (size_t(1) * PH + j) * NZ;
    const gview<Real> w2 = Wi + (size_t(2) * PH + j) * NZ;
    const gview<Real> w3 = Wi + (size_t(3) * PH + j) * NZ;
#pragma unroll 4
    for (int nn = 0; nn < NZ; nn += 2) {
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) {
        const int c = nn + pp;
        const Real a0 = Real(pr[c]), a1 = Real(pi[c]), b0 = Real(tr[c]), b1 = Real(ti[c]);
        const Real e0 = w0[c], e1 = w1[c], e2 = w2[c], e3 = w3[c];
        acc[pp][0][0] += e0 * a0; acc[pp][0][1] += e0 * a1;
        acc[pp][1][0] += e1 * a0; acc[pp][1][1] += e1 * a1;
        acc[pp][2][0] += e2 * a0; acc[pp][2][1] += e2 * a1;
        acc[pp][3][0] += e3 * a0; acc[pp][3][1] += e3 * a1;
        acc[pp][4][0] += e0 * b0; acc[pp][4][1] += e0 * b1;
        acc[pp][5][0] += e1 * b0; acc[pp][5][1] += e1 * b1;
      }
    }
    const Real k = Real(m * g.kscale), k2 = k * k;
    // derivative order of each product (for the reflection sign)
    const int qord[6] = {0, 1, 2, 3, 0, 1};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int jj = side ? PZ - 1 - j : j;
      Real v[6][2];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const Real sg = (side && (qord[q] & 1)) ? Real(-1) : Real(1);
        const Real od = side ? Real(-1) : Real(1);
        v[q][0] = sg * (acc[0][q][0] + od * acc[1][q][0]);
        v[q][1] = sg * (acc[0][q][1] + od * acc[1][q][1]);
      }
      Real out[6][2];
      if (m > 0) {
        out[0][0] = v[1][0]; out[0][1] = v[1][1];                      // u = psi_z
        out[1][0] = k * v[0][1]; out[1][1] = -k * v[0][0];              // w = -i k psi
        const Real omr = v[2][0] - k2 * v[0][0], omi = v[2][1] - k2 * v[0][1];
        out[2][0] = -k * omi; out[2][1] = k * omr;                      // omega_x = i k omega
        out[3][0] = v[3][0] - k2 * v[1][0]; out[3][1] = v[3][1] - k2 * v[1][1];  // omega_z
        out[4][0] = -k * v[4][1]; out[4][1] = k * v[4][0];              // T_x = i k T
        out[5][0] = v[5][0]; out[5][1] = v[5][1];                       // T_z
      } else {
        out[0][0] = v[0][0]; out[0][1] = 0;                             // u = u_bar
        out[1][0] = 0; out[1][1] = 0;
        out[2][0] = 0; out[2][1] = 0;
        out[3][0] = v[2][0]; out[3][1] = 0;                             // omega_z = u_bar_zz
        out[4][0] = 0; out[4][1] = 0;
        out[5][0] = v[5][0]; out[5][1] = 0;
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        Cx<Real>* d = reinterpret_cast<Cx<Real>*>(Q) + ((size_t(s) * 6 + q) * ntile + tile) * (PZ * MT) +
                      jj * MT + mt;
        *d = {out[q][0], out[q][1]};
      }
    }
  }
  }
}

// ------------------------------------------------ split path: GEMM kernels ---
//
// The Chebyshev transforms of a stage as batched FP32 MFMA GEMMs over every
// column (slice, mode, re/im) of the launch, so that each element of a
// transform map, held in LDS, serves every column a block visits instead of
// being streamed from L2 once per two-mode block.  Both kernels are
// persistent over columns: a block loads its slab of the map once and loops
// over column groups.  Even and odd Chebyshev coefficients are separate
// reductions (the Gauss-point reflection halves every map).
//
// MFMA v_mfma_f32_16x16x4f32 (one 64-lane wavefront): lane l supplies
// A[l % 16][k] and B[k][l % 16] for k = l / 16, and holds D[4 (l / 16) + r]
// [l % 16], r = 0..3.  The reduction index of the four lane groups is
// permuted consistently on both operands (group g takes k = 4 g + t at
// instruction t of four), so that each lane's four operands of four
// consecutive instructions are contiguous: one 16-byte load.

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Block -> (map slab `part`, column sequence bi of nb) of a persistent GEMM
// grid of parts x nb blocks (nb a multiple of kXcds).  The `parts` blocks
// that walk one column sequence sit on one XCD (workgroup b runs on XCD
// b mod kXcds), so each column operand they all read is fetched once into
// that XCD's L2.
__device__ __forceinline__ void gemm_block(int parts, int* part, int* bi, int* nb) {
  const int x = blockIdx.x % kXcds, w = blockIdx.x / kXcds;
  *part = w % parts;
  *bi = (w / parts) * kXcds + x;
  *nb = gridDim.x / parts;
}

__device__ __forceinline__ f32x4 mfma_16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NZ>
struct InvGemmShape {
  static constexpr int NH = NZ / 2, PH = 3 * NZ / 4, PZ = 3 * NZ / 2;
  static constexpr int JT = 16;                         // Gauss points per block (two blocks per CU)
  static constexpr int RT = JT / 16;                    // 16-row tiles per (q, parity)
  static constexpr int LDA = NH + 4;                    // LDS row stride (floats): 4-bank shift per row
  static constexpr int NJT = PH / JT;
  static constexpr size_t lds = sizeof(float) * 4 * 2 * JT * LDA;
};

template <int NZ>
struct FwdGemmShape {
  static constexpr int NH = NZ / 2, PH = 3 * NZ / 4, PZ = 3 * NZ / 2;
  static constexpr int RH = NH < 64 ? NH : 64;          // half-index rows per block (both parities)
  static constexpr int NRH = NH / RH;
  static constexpr int RT = RH / 16;
  static constexpr int LDA = PH + 4;
  static constexpr int CT = 2;                          // column tiles (8 modes x re/im) per wavefront
  static constexpr int GM = 4 * 8 * CT;                 // modes per block and column group
  static constexpr size_t lds = sizeof(float) * 2 * RH * LDA;
};

// Inverse transform of the new stage: for every column of Yf, values and
// z-derivatives d^q/dz^q (q = 0..3 for psi / u_bar, 0..1 for T) at the
// padded Gauss points, combined into the six mixed-space quantities u, w,
// omega_x, omega_z, T_x, T_z of each mode and written to Q.  Block: one tile
// of JT Gauss points j < Pz/2 (and, by reflection, Pz-1-j) and column groups
// of kGemmModes modes of one state (each wavefront eight modes, re and im,
// of both fields).
template <int NZ>
__global__ void __launch_bounds__(256)
inv_gemm_kernel(GridDev g, const float* __restrict__ Yf, float* __restrict__ Q, int slot0, int cap, int count) {
  using S = InvGemmShape<NZ>;
  constexpr int NH = S::NH, PH = S::PH, PZ = S::PZ, JT = S::JT, RT = S::RT, LDA = S::LDA, NJT = S::NJT;
  extern __shared__ __align__(16) unsigned char smem[];
  float* sA = reinterpret_cast<float*>(smem);   // [q][parity][JT][LDA]
  int jt, bi, nb;
  gemm_block(NJT, &jt, &bi, &nb);
  const int j0 = jt * JT;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4 * 2 * JT * (NH / 4); e += 256) {
    const int i4 = e % (NH / 4), row = e / (NH / 4);   // row = (q 2 + p) JT + jj
    const int jj = row % JT, qp = row / JT;
    const f32x4 v = *reinterpret_cast<const f32x4*>(g.Winv2 + (size_t(qp) * PH + j0 + jj) * NH + 4 * i4);
    *reinterpret_cast<f32x4*>(sA + size_t(row) * LDA + 4 * i4) = v;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, lc = lane & 15, lg = lane >> 4;
  const int Mx = g.Mx, st = g.state, XT = g.XT, nxt = g.nxt;
  const int gps = Mx / kGemmModes;
  const int ngroups = count * gps;
  const size_t qs = size_t(nxt) * PZ * XT * 2;   // floats between quantities of one state
  for (int cg = bi; cg < ngroups; cg += nb) {
    const int b = cg / gps, mg = cg - b * gps;
    const int s = ring_slot(b, slot0, cap);
    const int m = mg * kGemmModes + wave * 8 + (lc >> 1), ri = lc & 1;
    const float* yp = Yf + size_t(s) * st + size_t((0 * Mx + m) * 2 + ri) * NZ;
    const float* yt = Yf + size_t(s) * st + size_t((1 * Mx + m) * 2 + ri) * NZ;
    f32x4 aP[4][2][RT], aT[2][2][RT];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) aP[q][p][rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 2; ++q) aT[q][p][rt] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    // the column operands of the next 16-coefficient chunk are loaded while
    // the current one is multiplied (one wavefront per SIMD: nothing else
    // hides the load latency)
    f32x4 bpn = *reinterpret_cast<const f32x4*>(yp + 4 * lg);
    f32x4 btn = *reinterpret_cast<const f32x4*>(yt + 4 * lg);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll 1
      for (int kc = 0; kc < NH; kc += 16) {
        const f32x4 bp = bpn, bt = btn;
        const int nxt_off = (kc + 16 < NH) ? p * NH + kc + 16 : (p == 0 ? NH : p * NH + kc);
        bpn = *reinterpret_cast<const f32x4*>(yp + nxt_off + 4 * lg);
        btn = *reinterpret_cast<const f32x4*>(yt + nxt_off + 4 * lg);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f32x4 a =
                *reinterpret_cast<const f32x4*>(sA + size_t((q * 2 + p) * JT + rt * 16 + lc) * LDA + kc + 4 * lg);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              aP[q][p][rt] = mfma_16x16x4(a[t], bp[t], aP[q][p][rt]);
              if (q < 2) aT[q][p][rt] = mfma_16x16x4(a[t], bt[t], aT[q][p][rt]);
            }
          }
      }
    }
    // six quantities of this lane's (mode, re/im) at j and Pz-1-j; the other
    // half of the complex pair sits in the neighbouring lane
    const float k = float(m * g.kscale), k2 = k * k;
    const float sre = ri ? -1.f : 1.f;
    const int tile = m / XT, mt = m - tile * XT;
    float* qb = Q + size_t(s) * 6 * qs + size_t(tile) * PZ * XT * 2 + size_t(mt) * 2 + ri;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + rt * 16 + 4 * lg + r;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          // d^q T_n / dz^q at the reflected point is (-1)^(n+q) times that at j
          float vP[4], vT[2];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float e0 = aP[q][0][rt][r], e1 = aP[q][1][rt][r];
            vP[q] = side ? ((q & 1) ? e1 - e0 : e0 - e1) : e0 + e1;
          }
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const float e0 = aT[q][0][rt][r], e1 = aT[q][1][rt][r];
            vT[q] = side ? ((q & 1) ? e1 - e0 : e0 - e1) : e0 + e1;
          }
          const float om = vP[2] - k2 * vP[0];
          const float xP0 = __shfl_xor(vP[0], 1, 64), xom = __shfl_xor(om, 1, 64), xT0 = __shfl_xor(vT[0], 1, 64);
          float out[6];
          if (m > 0) {
            out[0] = vP[1];                    // u = psi_z
            out[1] = sre * k * xP0;            // w = -i k psi
            out[2] = -sre * k * xom;           // omega_x = i k omega
            out[3] = vP[3] - k2 * vP[1];       // omega_z
            out[4] = -sre * k * xT0;           // T_x = i k T
            out[5] = vT[1];                    // T_z
          } else {
            out[0] = ri ? 0.f : vP[0];         // u = u_bar
            out[1] = 0.f;
            out[2] = 0.f;
            out[3] = ri ? 0.f : vP[2];         // omega_z = u_bar_zz
            out[4] = 0.f;
            out[5] = ri ? 0.f : vT[1];
          }
          const int jj = side ? PZ - 1 - j : j;
#pragma unroll
          for (int qq = 0; qq < 6; ++qq) qb[qq * qs + size_t(jj) * XT * 2] = out[qq];
        }
      }
  }
}

// Forward transform of the products: for every column (mode, re/im) of the
// field f of each state, the explicit term -S F N on all rows n (the
// equation basis folded into the map; rows beyond the band are not read),
// written to this stage's slot of Ehist.  Block: field f, rows 2 i + p
// for i in one RH-row half and both parities (so that a lane writes eight
// consecutive coefficients), column groups of GM modes of one state.
template <int NZ>
__global__ void __launch_bounds__(256)
fwd_gemm_kernel(GridDev g, const float* __restrict__ Nh, float* __restrict__ E, int slot0, int cap, int count) {
  using S = FwdGemmShape<NZ>;
  constexpr int NH = S::NH, PH = S::PH, PZ = S::PZ, RH = S::RH, NRH = S::NRH, RT = S::RT, LDA = S::LDA,
                CT = S::CT, GM = S::GM;
  extern __shared__ __align__(16) unsigned char smem[];
  float* sA = reinterpret_cast<float*>(smem);   // [parity][RH][LDA]
  int fh, bi, nb;
  gemm_block(2 * NRH, &fh, &bi, &nb);
  const int f = fh / NRH, h = fh - f * NRH;
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * RH * (PH / 4); e += 256) {
    const int j4 = e % (PH / 4), row = e / (PH / 4);   // row = p RH + ii
    const int ii = row % RH, p = row / RH;
    const f32x4 v = *reinterpret_cast<const f32x4*>(g.Wfwd2 + ((size_t(f) * 2 + p) * NH + h * RH + ii) * PH + 4 * j4);
    *reinterpret_cast<f32x4*>(sA + size_t(row) * LDA + 4 * j4) = v;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, lc = lane & 15, lg = lane >> 4;
  const int Mx = g.Mx, st = g.state, XT = g.XT, nxt = g.nxt;
  const int gps = Mx / GM;
  const int ngroups = count * gps;
  const int rs = XT * 2;   // floats between Gauss points in a mixed-space tile
  for (int cg = bi; cg < ngroups; cg += nb) {
    const int b = cg / gps, mg = cg - b * gps;
    const int s = ring_slot(b, slot0, cap);
    const float* nc[CT];
    int mm[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int m = mg * GM + wave * (8 * CT) + ct * 8 + (lc >> 1);
      const int tile = m / XT, mt = m - tile * XT;
      mm[ct] = m;
      nc[ct] = Nh + ((size_t(s) * 2 + f) * nxt + tile) * PZ * XT * 2 + mt * 2 + (lc & 1);
    }
    f32x4 acc[2][RT][CT];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[p][rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    // products of the next 16 Gauss points are loaded while the current
    // ones are multiplied
    float n0n[CT][4], n1n[CT][4];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = 4 * lg + t;
        n0n[ct][t] = nc[ct][size_t(j) * rs];
        n1n[ct][t] = nc[ct][size_t(PZ - 1 - j) * rs];
      }
#pragma unroll 1
    for (int kc = 0; kc < PH; kc += 16) {
      float bs[CT][4], bd[CT][4];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          bs[ct][t] = n0n[ct][t] + n1n[ct][t];   // even rows: the value at Pz-1-j enters with +1
          bd[ct][t] = n0n[ct][t] - n1n[ct][t];   // odd rows: with -1
        }
      const int kn = (kc + 16 < PH) ? kc + 16 : kc;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int j = kn + 4 * lg + t;
          n0n[ct][t] = nc[ct][size_t(j) * rs];
          n1n[ct][t] = nc[ct][size_t(PZ - 1 - j) * rs];
        }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const f32x4 a = *reinterpret_cast<const f32x4*>(sA + size_t(p * RH + rt * 16 + lc) * LDA + kc + 4 * lg);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int t = 0; t < 4; ++t)
              acc[p][rt][ct] = mfma_16x16x4(a[t], p ? bd[ct][t] : bs[ct][t], acc[p][rt][ct]);
        }
    }
    // lane: rows i = h RH + 16 rt + 4 lg + r of both parities = coefficients
    // n = 2 i + p, eight consecutive ones per (rt, ct)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      float* eo = E + size_t(s) * st + size_t((f * Mx + mm[ct]) * 2 + (lc & 1)) * NZ;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int n0 = 2 * (h * RH + rt * 16 + 4 * lg);
        const f32x4 lo = {acc[0][rt][ct][0], acc[1][rt][ct][0], acc[0][rt][ct][1], acc[1][rt][ct][1]};
        const f32x4 hi = {acc[0][rt][ct][2], acc[1][rt][ct][2], acc[0][rt][ct][3], acc[1][rt][ct][3]};
        *reinterpret_cast<f32x4*>(eo + n0) = lo;
        *reinterpret_cast<f32x4*>(eo + n0 + 4) = hi;
      }
    }
  }
}

// ------------------------------------------------------------- diagnostics ---
//
// The per-state record of section 2.2 (Nu_V, Nu_b, Nu_t, KE, epsilon_U, P)
// from exact volume means of products of the discrete fields.  For real
// fields f, g with modes f_m, g_m (m >= 0), the horizontal mean of f g is
// f_0 g_0 + 2 sum_{m>=1} Re(f_m conj g_m); the vertical mean over z in
// [0, Lz] of two Chebyshev series a, b is (1/2) sum_ab a_a b_b J_ab with
// J_ab = int_{-1}^{1} T_a T_b = 1/(1-(a+b)^2) + 1/(1-(a-b)^2) for a + b even
// (zero otherwise).  u = psi_z (u_bar for m = 0), w = -i k psi,
// omega = psi_zz - k^2 psi (u_bar_z for m = 0); <|grad u|^2> = <omega^2> for
// these no-slip, periodic fields.  Two kernels: partial sums per (state,
// chunk of modes), then a fixed-order sum per state.

// Chebyshev-T coefficients of d/dzeta of c[0..N) into d[0..N):
// d_n = d_(n+2) + 2 (n+1) c_(n+1), then d_0 / 2.
__device__ void cheb_deriv_col(const double* c, double* d, int N, double scale) {
  double a = 0.0, b = 0.0;   // d_(n+1), d_(n+2)
  d[N - 1] = 0.0;
  for (int n = N - 2; n >= 0; --n) {
    const double v = b + 2.0 * (n + 1) * c[n + 1];
    d[n] = v;
    b = a;
    a = v;
  }
  d[0] *= 0.5;
  for (int n = 0; n < N; ++n) d[n] *= scale;
}

// Block-wide sum of four values; thread 0 receives the totals.
__device__ void block_sum4(double v[4], double* red) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wv * 4 + q] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[w * 4 + q];
      v[q] = t;
    }
}

// Partial sums (<w T>, <u^2>, <w^2>, <omega^2>) of modes [chunk * MC, ...)
// of the state at batch position blockIdx.x / nchunk.
__global__ void __launch_bounds__(kBlock)
diag_partial_kernel(GridDev g, const double* __restrict__ X, int slot0, int cap, int nchunk,
                    double* __restrict__ part) {
  extern __shared__ double sd[];
  __shared__ double red[(kBlock / 64) * 4];
  const int Nz = g.Nz, Mx = g.Mx, MC = diag_modes(Nz);
  const int bpos = blockIdx.x / nchunk, chunk = blockIdx.x - bpos * nchunk;
  const double* x = batch_state(g, X, bpos, ring_slot(bpos, slot0, cap));
  const int m0 = chunk * MC, nm = min(MC, Mx - m0);
  double* sP = sd;                      // [MC][re, im][Nz] psi (u_bar at m = 0)
  double* sT = sP + MC * 2 * Nz;        // T
  double* sU = sT + MC * 2 * Nz;        // u
  double* sO = sU + MC * 2 * Nz;        // omega
  for (int e = threadIdx.x; e < nm * 2 * Nz; e += blockDim.x) {
    const int mm = e / (2 * Nz), rest = e - mm * 2 * Nz;
    sP[e] = x[size_t(0 * Mx + m0 + mm) * 2 * Nz + rest];
    sT[e] = x[size_t(1 * Mx + m0 + mm) * 2 * Nz + rest];
  }
  __syncthreads();
  for (int col = threadIdx.x; col < nm * 2; col += blockDim.x) {
    const int m = m0 + (col >> 1);
    const double* c = sP + col * Nz;
    double* u = sU + col * Nz;
    double* om = sO + col * Nz;
    if (m == 0) {
      for (int n = 0; n < Nz; ++n) u[n] = c[n];
      cheb_deriv_col(c, om, Nz, g.scale);
    } else {
      const double k = m * g.kscale;
      cheb_deriv_col(c, u, Nz, g.scale);
      cheb_deriv_col(u, om, Nz, g.scale);
      for (int n = 0; n < Nz; ++n) om[n] -= k * k * c[n];
    }
  }
  __syncthreads();
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e = threadIdx.x; e < nm * Nz; e += blockDim.x) {
    const int mm = e / Nz, a = e - mm * Nz, m = m0 + mm;
    const double k = m * g.kscale, wgt = (m == 0) ? 0.5 : 1.0;
    const double* pr = sP + mm * 2 * Nz; const double* pi = pr + Nz;
    const double* tr = sT + mm * 2 * Nz; const double* ti = tr + Nz;
    const double* ur = sU + mm * 2 * Nz; const double* ui = ur + Nz;
    const double* orr = sO + mm * 2 * Nz; const double* oi = orr + Nz;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = a & 1; b < Nz; b += 2) {
      const int sp = a + b, df = a > b ? a - b : b - a;
      const double J = 1.0 / (1.0 - double(sp) * sp) + 1.0 / (1.0 - double(df) * df);
      s[0] += J * tr[b]; s[1] += J * ti[b];
      s[2] += J * ur[b]; s[3] += J * ui[b];
      s[4] += J * pr[b]; s[5] += J * pi[b];
      s[6] += J * orr[b]; s[7] += J * oi[b];
    }
    if (m > 0) {
      acc[0] += wgt * k * (pi[a] * s[0] - pr[a] * s[1]);            // w = -i k psi against T
      acc[2] += wgt * k * k * (pr[a] * s[4] + pi[a] * s[5]);        // |w|^2
    }
    acc[1] += wgt * (ur[a] * s[2] + ui[a] * s[3]);                  // |u|^2
    acc[3] += wgt * (orr[a] * s[6] + oi[a] * s[7]);                 // omega^2
  }
  block_sum4(acc, red);
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) part[size_t(blockIdx.x) * 4 + q] = acc[q];
}

// Per state: the chunk partials in order, the wall gradients of the mean
// temperature, and the record.  Plain batches write out + bpos * ld; with
// meta (the pipelined ring) a run that has completed a multiple q+1 of
// `stride` own steps at virtual step t writes out[(par S + n) nsf + q][6].
__global__ void diag_final_kernel(GridDev g, const double* __restrict__ X, int slot0, int cap, int nchunk,
                                  const double* __restrict__ part, double* __restrict__ out, int ld,
                                  const SlotMeta* __restrict__ meta, int t, int stride, int nsf, int S) {
  if (threadIdx.x != 0) return;
  const int bpos = blockIdx.x, slot = ring_slot(bpos, slot0, cap);
  const RunDev* rd = batch_run(g, bpos);
  double* o;
  if (meta) {
    const SlotMeta mt = meta[slot];
    const int d = t - mt.start;
    if (d <= 0 || d % stride != 0 || d / stride > nsf) return;
    o = out + ((size_t(mt.par) * S + mt.n) * nsf + (d / stride - 1)) * kDiag;
  } else {
    o = out + size_t(bpos) * ld;
  }
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nchunk; ++c)
    for (int q = 0; q < 4; ++q) v[q] += part[(size_t(bpos) * nchunk + c) * 4 + q];
  const int Nz = g.Nz;
  const double* tm = batch_state(g, X, bpos, slot) + size_t(1 * g.Mx + 0) * 2 * Nz;
  double nb = 0, nt = 0, t0 = 0, t1 = 0;
  for (int n = 0; n < Nz; ++n) {
    const double sgn = (n & 1) ? -1.0 : 1.0, n2 = double(n) * n;
    nb += tm[n] * (-sgn) * n2;   // T_n'(-1) = (-1)^(n+1) n^2
    nt += tm[n] * n2;            // T_n'(1) = n^2
    t0 += tm[n] * sgn;
    t1 += tm[n];
  }
  const double ref = (t0 - t1) / g.Lz;           // conductive flux of the mean temperature drop
  o[0] = ((t0 - t1) / g.Lz + rd->sqrtRaPr * v[0]) / ref;   // Nu_V
  o[1] = -g.scale * nb / ref;                            // Nu_b
  o[2] = -g.scale * nt / ref;                            // Nu_t
  o[3] = 0.5 * (v[1] + v[2]);                    // KE
  o[4] = rd->nu * v[3];                          // epsilon_U
  o[5] = v[0];                                   // P = <w T>
}

__global__ void set_meta_kernel(SlotMeta* meta, int slot, SlotMeta v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) meta[slot] = v;
}

// ----------------------------------------------------- transfer / correction ---

__global__ void restrict_kernel(GridDev f, GridDev c, const double* __restrict__ Xf, double* __restrict__ Xc) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c.state; e += gridDim.x * blockDim.x) {
    const int nn = e % c.Nz, col = e / c.Nz, ri = col & 1, m = (col >> 1) % c.Mx, fl = col / (2 * c.Mx);
    Xc[e] = Xf[size_t(((fl * f.Mx + m) * 2 + ri)) * f.Nz + nn];
  }
}

__global__ void __launch_bounds__(kBlock)
combine_kernel(GridDev f, GridDev c, int mode, double* __restrict__ U, const double* __restrict__ F,
               const double* __restrict__ gc, double* __restrict__ gold, double* __restrict__ part) {
  __shared__ double r1[kBlock], r2[kBlock];
  double d2 = 0, n2 = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < f.state; e += gridDim.x * blockDim.x) {
    const int nn = e % f.Nz, col = e / f.Nz, ri = col & 1, m = (col >> 1) % f.Mx, fl = col / (2 * f.Mx);
    const bool inc = (m < c.Mx) && (nn < c.Nz);
    const size_t ce = size_t(((fl * c.Mx + m) * 2 + ri)) * c.Nz + nn;
    double un;
    if (mode == 2) {
      un = F[e];
    } else {
      const double gv = inc ? gc[ce] : 0.0;
      if (mode == 0) {
        un = gv;
      } else {
        const double go = inc ? gold[ce] : 0.0;
        un = gv + F[e] - go;
      }
      if (inc) gold[ce] = gv;
    }
    const double uo = U[e];
    U[e] = un;
    const double d = un - uo;
    d2 += d * d;
    n2 += un * un;
  }
  r1[threadIdx.x] = d2;
  r2[threadIdx.x] = n2;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

__global__ void defect_kernel(const double* __restrict__ part, int first, int last, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double dmax = 0;
  int bad = 0;
  for (int sl = first; sl < last; ++sl) {
    double d2 = 0, n2 = 0;
    for (int b = 0; b < kCombineBlocks; ++b) {
      d2 += part[(size_t(sl) * kCombineBlocks + b) * 2];
      n2 += part[(size_t(sl) * kCombineBlocks + b) * 2 + 1];
    }
    if (!isfinite(d2) || !isfinite(n2)) {
      bad = 1;
      continue;
    }
    const double r = sqrt(d2 / (n2 > 0 ? n2 : 1.0));
    dmax = fmax(dmax, r);
  }
  out[0] = dmax;
  out[1] = bad;
}

// ---------------------------------------------------------------- launchers ---

namespace {

template <typename Real, int NZ, int MT, bool SPLIT = false>
hipError_t run_stage_t(const GridPlan& g, Work& w, const StageArgs& a, double* X, int n_slices, double* Eout,
                       hipStream_t st) {
  const GridDev& d = g.dev;
  const int ntile = (d.Mx + MT - 1) / MT;
  constexpr bool pre = MT <= 2 && NZ <= 64;   // as in the kernel
  constexpr bool lean = SPLIT && NZ / 2 - 1 >= 64;
  const size_t lds = stage_lds<NZ, MT>(sizeof(Real), d.facT_stride, d.facP_stride, pre, SPLIT, lean).total;
  hipLaunchKernelGGL((stage_kernel<Real, NZ, MT, SPLIT>), dim3(xcd_grid(d.one_xcd, n_slices * ntile)), dim3(kBlock),
                     lds, st, d, a, (const Real*)w.Nh, (const Real*)w.qbar, X, (Real*)w.Ehist, w.LYhist, (Real*)w.Q,
                     Eout, w.Yf);
  return hipGetLastError();
}

template <typename Real, int NZ>
hipError_t run_stage_nz(const GridPlan& g, Work& w, const StageArgs& a, double* X, int n_slices, double* Eout,
                        hipStream_t st) {
  if constexpr (sizeof(Real) == 4 && NZ >= 64) {
    if (g.split) {
      switch (g.dev.MT) {
        case 2: return run_stage_t<Real, NZ, 2, true>(g, w, a, X, n_slices, Eout, st);
        case 4: return run_stage_t<Real, NZ, 4, true>(g, w, a, X, n_slices, Eout, st);
        default: return hipErrorInvalidValue;
      }
    }
  }
  if (g.split) return hipErrorInvalidValue;
  switch (g.dev.MT) {
    case 2: return run_stage_t<Real, NZ, 2>(g, w, a, X, n_slices, Eout, st);
    case 4: return run_stage_t<Real, NZ, 4>(g, w, a, X, n_slices, Eout, st);
    case 6: return run_stage_t<Real, NZ, 6>(g, w, a, X, n_slices, Eout, st);
    case 8: return run_stage_t<Real, NZ, 8>(g, w, a, X, n_slices, Eout, st);
    default: return hipErrorInvalidValue;
  }
}

// Persistent grid of a GEMM kernel: `parts` map slabs, each with as many
// blocks as fit on the device next to the others (by LDS), a multiple of
// kXcds (see gemm_block), no more than the column groups need.
inline int gemm_blocks(int parts, size_t lds, int ngroups) {
  int per_cu = int((160 * 1024) / (lds ? lds : 1));
  per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
  int nb = (256 * per_cu) / parts;
  const int need = (ngroups + kXcds - 1) / kXcds * kXcds;
  if (nb > need) nb = need;
  nb = nb / kXcds * kXcds;
  if (nb < kXcds) nb = kXcds;
  return parts * nb;
}

template <int NZ>
hipError_t run_fwd_gemm_t(const GridPlan& g, Work& w, int stage, int slot0, int count, hipStream_t st) {
  using S = FwdGemmShape<NZ>;
  const int ngroups = count * (g.dev.Mx / S::GM);
  float* E = static_cast<float*>(w.Ehist) + size_t(stage - 1) * w.cap * g.dev.state;
  hipLaunchKernelGGL((fwd_gemm_kernel<NZ>), dim3(gemm_blocks(2 * S::NRH, S::lds, ngroups)), dim3(256), S::lds, st,
                     g.dev, (const float*)w.Nh, E, slot0, w.cap, count);
  return hipGetLastError();
}

template <int NZ>
hipError_t run_inv_gemm_t(const GridPlan& g, Work& w, int slot0, int count, hipStream_t st) {
  using S = InvGemmShape<NZ>;
  const int ngroups = count * (g.dev.Mx / kGemmModes);
  hipLaunchKernelGGL((inv_gemm_kernel<NZ>), dim3(gemm_blocks(S::NJT, S::lds, ngroups)), dim3(256), S::lds, st,
                     g.dev, (const float*)w.Yf, (float*)w.Q, slot0, w.cap, count);
  return hipGetLastError();
}

// The split path's transforms: forward (products of `stage` into its Ehist
// slot) or inverse (Yf to the mixed-space quantities).
hipError_t run_gemm(const GridPlan& g, Work& w, bool forward, int stage, int slot0, int count, hipStream_t st) {
  if (!g.split) return hipErrorInvalidValue;
  switch (g.dev.Nz) {
    case 64: return forward ? run_fwd_gemm_t<64>(g, w, stage, slot0, count, st) : run_inv_gemm_t<64>(g, w, slot0, count, st);
    case 128: return forward ? run_fwd_gemm_t<128>(g, w, stage, slot0, count, st) : run_inv_gemm_t<128>(g, w, slot0, count, st);
    case 256: return forward ? run_fwd_gemm_t<256>(g, w, stage, slot0, count, st) : run_inv_gemm_t<256>(g, w, slot0, count, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t run_stage(const GridPlan& g, Work& w, const StageArgs& a, double* X, int n_slices, double* Eout,
                     hipStream_t st) {
  switch (g.dev.Nz) {
    case 8: return run_stage_nz<Real, 8>(g, w, a, X, n_slices, Eout, st);
    case 16: return run_stage_nz<Real, 16>(g, w, a, X, n_slices, Eout, st);
    case 32: return run_stage_nz<Real, 32>(g, w, a, X, n_slices, Eout, st);
    case 64: return run_stage_nz<Real, 64>(g, w, a, X, n_slices, Eout, st);
    case 128: return run_stage_nz<Real, 128>(g, w, a, X, n_slices, Eout, st);
    case 256: return run_stage_nz<Real, 256>(g, w, a, X, n_slices, Eout, st);
    default: return hipErrorInvalidValue;
  }
}

// Rows per x-pass block: as many (up to four) as fit in 80 KiB of LDS.
template <typename Real, int PX>
constexpr int xpass_rows() {
  constexpr size_t row = sizeof(Real) * 2 * xpass_spectra<Real, PX, 4>() * size_t(PX);
  return (4 * row <= 80 * 1024) ? 4 : ((2 * row <= 80 * 1024) ? 2 : 1);
}

template <typename Real, int PX, int RB>
hipError_t launch_xpass_rb(const GridDev& d, Work& w, int slot0, int n_slices, hipStream_t st) {
  const size_t lds = sizeof(Real) * 2 * xpass_spectra<Real, PX, RB>() * size_t(PX) * RB;
  hipLaunchKernelGGL((xpass_kernel<Real, PX, RB>), dim3(xcd_grid(d.one_xcd, n_slices * (d.Pz / RB))), dim3(64 * RB),
                     lds, st, d, (const Real*)w.Q, (Real*)w.Nh, (Real*)w.qbar, slot0, w.cap);
  return hipGetLastError();
}

template <typename Real, int PX, int RB>
constexpr bool xpass_rows_fit() {
  return sizeof(Real) * 2 * xpass_spectra<Real, PX, RB>() * size_t(PX) * RB <= 160 * 1024;
}

template <typename Real, int PX>
hipError_t run_xpass_t(const GridPlan& g, Work& w, int slot0, int n_slices, hipStream_t st) {
  const GridDev& d = g.dev;
  int rb = d.xrows;   // tuned rows per block, 0: by rule
  if (rb != 1 && rb != 2 && rb != 4) {
    rb = xpass_rows<Real, PX>();
    // a small batch (the single-slice coarse sweep) would leave most CUs
    // idle with several rows per block: one row per block there
    if (rb > 1 && n_slices * (d.Pz / rb) < 256) rb = 1;
  }
  if (rb == 4 && !xpass_rows_fit<Real, PX, 4>()) rb = 2;
  if (rb == 2 && !xpass_rows_fit<Real, PX, 2>()) rb = 1;
  if constexpr (xpass_rows_fit<Real, PX, 4>())
    if (rb == 4) return launch_xpass_rb<Real, PX, 4>(d, w, slot0, n_slices, st);
  if constexpr (xpass_rows_fit<Real, PX, 2>())
    if (rb == 2) return launch_xpass_rb<Real, PX, 2>(d, w, slot0, n_slices, st);
  return launch_xpass_rb<Real, PX, 1>(d, w, slot0, n_slices, st);
}

template <typename Real>
hipError_t run_xpass(const GridPlan& g, Work& w, int slot0, int n_slices, hipStream_t st) {
  switch (g.dev.Px) {
    case 6: return run_xpass_t<Real, 6>(g, w, slot0, n_slices, st);
    case 12: return run_xpass_t<Real, 12>(g, w, slot0, n_slices, st);
    case 24: return run_xpass_t<Real, 24>(g, w, slot0, n_slices, st);
    case 48: return run_xpass_t<Real, 48>(g, w, slot0, n_slices, st);
    case 96: return run_xpass_t<Real, 96>(g, w, slot0, n_slices, st);
    case 192: return run_xpass_t<Real, 192>(g, w, slot0, n_slices, st);
    case 384: return run_xpass_t<Real, 384>(g, w, slot0, n_slices, st);
    case 768: return run_xpass_t<Real, 768>(g, w, slot0, n_slices, st);
    case 1536: return run_xpass_t<Real, 1536>(g, w, slot0, n_slices, st);
    case 3072: return run_xpass_t<Real, 3072>(g, w, slot0, n_slices, st);
    default: return hipErrorInvalidValue;
  }
}

// Records an event of the timing pool (start or stop of one launch).
hipError_t timing_mark(KernelTiming* t, hipStream_t st) {
  if (t->used >= t->ev.size()) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    t->ev.push_back(e);
  }
  return hipEventRecord(t->ev[t->used++], st);
}

template <typename Real>
hipError_t steps_impl(const GridPlan& g, Work& w, double* X, const StepRange& r, double* nu_out, int nu_stride,
                      int nu_ld, hipStream_t st, KernelTiming* tm) {
  const Tableau& tb = g.tab;
  hipError_t e;
  const bool split = g.split;
  if (r.step0 == 0) {
    StageArgs a{};
    a.mode = kModeZinv;
    a.do_zinv = 1;
    a.cap = w.cap;
    a.slot0 = r.slot0;
    a.s = tb.s;
    if ((e = run_stage<Real>(g, w, a, X, r.count, nullptr, st)) != hipSuccess) return e;
    if (split && (e = run_gemm(g, w, false, 0, r.slot0, r.count, st)) != hipSuccess) return e;
  }
  for (int step = r.step0; step < r.step1; ++step) {
    const bool last = (step == r.n_total - 1);
    const long ti = r.timing_index + (step - r.step0);
    const bool timed = tm && tm->every > 0 && ti % tm->every == 0 &&
                       tm->used + 2 * tb.s <= 2 * KernelTiming::kMaxPairs;
    for (int i = 1; i <= tb.s; ++i) {
      if (timed && tm->kernel == 1 && (e = timing_mark(tm, st)) != hipSuccess) return e;
      if ((e = run_xpass<Real>(g, w, r.slot0, r.count, st)) != hipSuccess) return e;
      if (timed && tm->kernel == 1 && (e = timing_mark(tm, st)) != hipSuccess) return e;
      StageArgs b{};
      b.mode = kModeStage;
      b.stage = i;
      b.s = tb.s;
      b.cap = w.cap;
      b.slot0 = r.slot0;
      b.store_E = (i < tb.s);
      b.store_LY = (i < tb.s);
      b.write_X = (i == tb.s);
      b.do_zinv = !(last && i == tb.s);
      for (int j = 0; j < i; ++j) b.hae[j] = g.dt * tb.ae[i][j];
      for (int j = 1; j <= i; ++j) b.hai[j] = g.dt * tb.ai[i][j];
      b.haii = g.dt * tb.ai[i][i];
      // split path: the forward GEMM, the per-mode solve kernel and (unless
      // this is the run's last stage) the inverse GEMM; kernel 0 of the
      // timing brackets all three
      if (timed && tm->kernel == 0 && (e = timing_mark(tm, st)) != hipSuccess) return e;
      if (timed) tm->units += r.count;
      if (split && (e = run_gemm(g, w, true, i, r.slot0, r.count, st)) != hipSuccess) return e;
      if ((e = run_stage<Real>(g, w, b, X, r.count, nullptr, st)) != hipSuccess) return e;
      if (split && b.do_zinv && (e = run_gemm(g, w, false, i, r.slot0, r.count, st)) != hipSuccess) return e;
      if (timed && tm->kernel == 0 && (e = timing_mark(tm, st)) != hipSuccess) return e;
    }
    if (nu_out && nu_stride > 0 && (step + 1) % nu_stride == 0) {
      const int sample = (step + 1) / nu_stride - 1;
      if (sample < nu_ld &&
          (e = launch_diag(g, w, X, 0, r.count, w.cap, nu_out + size_t(sample) * kDiag, nu_ld * kDiag, nullptr, 0,
                           1, 0, 0, st)) != hipSuccess)
        return e;
    }
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_step_range(const GridPlan& g, Work& w, double* X, const StepRange& r, double* nu_out,
                             int nu_stride, int nu_ld, hipStream_t st, KernelTiming* tm) {
  if (r.count < 1 || r.count > w.cap || r.slot0 < 0 || r.slot0 >= w.cap) return hipErrorInvalidValue;
  // the Nu launch indexes X by batch position: plain batches only
  if (nu_out && nu_stride > 0 && r.slot0 != 0) return hipErrorInvalidValue;
  if (g.mixed) return steps_impl<float>(g, w, X, r, nu_out, nu_stride, nu_ld, st, tm);
  return steps_impl<double>(g, w, X, r, nu_out, nu_stride, nu_ld, st, tm);
}

hipError_t launch_steps(const GridPlan& g, Work& w, double* X, int n_slices, int n_steps, double* nu_out,
                        int nu_stride, int nu_ld, hipStream_t st, KernelTiming* tm) {
  if (n_steps <= 0) return hipSuccess;
  StepRange r;
  r.slot0 = 0;
  r.count = n_slices;
  r.step0 = 0;
  r.step1 = n_steps;
  r.n_total = n_steps;
  return launch_step_range(g, w, X, r, nu_out, nu_stride, nu_ld, st, tm);
}

hipError_t launch_explicit(const GridPlan& g, Work& w, const double* X, double* E, hipStream_t st) {
  StageArgs a{};
  a.mode = kModeZinv;
  a.do_zinv = 1;
  a.cap = w.cap;
  a.s = g.tab.s;
  a.stage = 1;   // the split path's forward GEMM writes the first Ehist slot
  hipError_t e;
  double* Xm = const_cast<double*>(X);
  if (g.mixed) {
    if ((e = run_stage<float>(g, w, a, Xm, 1, nullptr, st)) != hipSuccess) return e;
    if (g.split && (e = run_gemm(g, w, false, 0, 0, 1, st)) != hipSuccess) return e;
    if ((e = run_xpass<float>(g, w, 0, 1, st)) != hipSuccess) return e;
    if (g.split && (e = run_gemm(g, w, true, 1, 0, 1, st)) != hipSuccess) return e;
    a.mode = kModeExplicit;
    return run_stage<float>(g, w, a, Xm, 1, E, st);
  }
  if ((e = run_stage<double>(g, w, a, Xm, 1, nullptr, st)) != hipSuccess) return e;
  if ((e = run_xpass<double>(g, w, 0, 1, st)) != hipSuccess) return e;
  a.mode = kModeExplicit;
  return run_stage<double>(g, w, a, Xm, 1, E, st);
}

hipError_t launch_set_meta(SlotMeta* meta, int slot, SlotMeta v, hipStream_t st) {
  hipLaunchKernelGGL(set_meta_kernel, dim3(1), dim3(64), 0, st, meta, slot, v);
  return hipGetLastError();
}

size_t diag_partials_per_state(const GridDev& d) {
  const int MC = diag_modes(d.Nz);
  return size_t(4) * ((d.Mx + MC - 1) / MC);
}

hipError_t launch_diag_into(const GridPlan& g, double* part, const double* X, int slot0, int count, int cap,
                            double* out, int ld, const SlotMeta* meta, int t, int stride, int nsf, int S,
                            hipStream_t st) {
  if (count < 1 || slot0 < 0 || slot0 >= cap || (meta && stride < 1)) return hipErrorInvalidValue;
  const int MC = diag_modes(g.dev.Nz), nchunk = (g.dev.Mx + MC - 1) / MC;
  const size_t lds = sizeof(double) * 8 * size_t(MC) * g.dev.Nz;
  hipLaunchKernelGGL(diag_partial_kernel, dim3(count * nchunk), dim3(kBlock), lds, st, g.dev, X, slot0, cap, nchunk,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(count), dim3(64), 0, st, g.dev, X, slot0, cap, nchunk,
                     (const double*)part, out, ld, meta, t, stride, nsf, S);
  return hipGetLastError();
}

hipError_t launch_diag(const GridPlan& g, Work& w, const double* X, int slot0, int count, int cap, double* out,
                       int ld, const SlotMeta* meta, int t, int stride, int nsf, int S, hipStream_t st) {
  if (count > w.cap) return hipErrorInvalidValue;   // w.dpart holds w.cap states' partials
  return launch_diag_into(g, w.dpart, X, slot0, count, cap, out, ld, meta, t, stride, nsf, S, st);
}

// ---------------------------------------------------- allocation-free scratch ---
//
// Device scratch of the allocation-free entry points: one array per GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address hipGetSymbolAddress returns, taken
// once per device with that device current (at handle creation).
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;   // per device id
}  // namespace

hipError_t scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if (int(g_scratch_dev.size()) <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (g_scratch_dev[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < int(g_scratch_dev.size())) ? g_scratch_dev[device] : nullptr;
}

hipError_t launch_restrict(const GridPlan& f, const GridPlan& c, const double* Xf, double* Xc, hipStream_t st) {
  const int blocks = (c.dev.state + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(restrict_kernel, dim3(blocks < 1024 ? blocks : 1024), dim3(kBlock), 0, st, f.dev, c.dev, Xf,
                     Xc);
  return hipGetLastError();
}

hipError_t launch_combine(const GridPlan& f, const GridPlan& c, int mode, double* U, const double* F,
                          const double* gc, double* gold, double* part, hipStream_t st) {
  hipLaunchKernelGGL(combine_kernel, dim3(kCombineBlocks), dim3(kBlock), 0, st, f.dev, c.dev, mode, U, F, gc,
                     gold, part);
  return hipGetLastError();
}

hipError_t launch_defect(const double* part, int first, int last, double* out, hipStream_t st) {
  hipLaunchKernelGGL(defect_kernel, dim3(1), dim3(64), 0, st, part, first, last, out);
  return hipGetLastError();
}

}  // namespace rbc
