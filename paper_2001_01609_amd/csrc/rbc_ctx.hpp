// The library handle (rbc_handle) shared by the ABI sources: plans, work
// buffers, Parareal buffers and the two streams of the pipelined iteration.
#pragma once

#include <string>
#include <vector>

#include "rbc_internal.hpp"

struct rbc_ctx {
  rbc_params p{};
  hipStream_t stream = nullptr;     // the caller's stream
  hipStream_t fstream = nullptr;    // pipelined Parareal: batched fine runs
  hipStream_t gstream = nullptr;    // pipelined Parareal: serial coarse sweep
  hipStream_t f64stream = nullptr;  // pipelined Parareal: FP64 fine runs (with the FP64 switch only)
  int device = 0;
  rbc::GridPlan fine, coarse;
  rbc::GridPlan fine64, coarse64;   // all-FP64 plans for promoted sweeps (mixed + promote_fp64)
  bool has64 = false;
  int k_fp64 = 0;              // first iteration the last parareal_iterate ran F in FP64 (0: never)
  int stop_reason = -1;        // of the last parareal_iterate (rbc_stop_reason)
  double* U_hist = nullptr;    // iterate history (rbc_set_iterate_history)
  int hist_cap = -1;
  rbc::Work wf, wc, wf64, wc64;  // fine work for ring_cap slices, coarse work for one
  int nf = 0, nc = 0;          // steps per slice
  int ring_cap = 0;            // fine state slots: n_slices + 2
  double* Xc = nullptr;        // coarse state being advanced
  double* Fbuf = nullptr;      // [S][state]   F(U_n^(k-1)) (sequential iteration)
  double* Xring = nullptr;     // [ring_cap][state] fine runs of the pipelined iteration
  rbc::SlotMeta* meta = nullptr;  // [ring_cap]
  double* Gbuf = nullptr;      // [S][cstate]  coarse part of G(U_n^k)
  double* part = nullptr;      // [S+1][kCombineBlocks][2]
  double* dscal = nullptr;     // [2] defect, non-finite flag
  double* nu_f = nullptr;      // [2][S][nsf][kDiag]  diagnostic samples (sequential: first half)
  double* nu_c = nullptr;      // [S][nsc][kDiag]
  double* host_pin = nullptr;  // pinned: [2] defect + [2][S][nsf][kDiag] + [S][nsc][kDiag]
  int nsf = 0, nsc = 0, stride_c = 0;
  std::vector<hipEvent_t> evpool;  // events of the pipelined iteration, reused across calls
  // graphs of kCoarseGraphSteps coarse steps on Xc (mixed / FP64 coarse plan),
  // built at the first pipelined iteration that needs them
  hipGraphExec_t cgraph = nullptr, cgraph64 = nullptr;
  rbc_pipeline_stats pstats{};  // statistics of the last pipelined iteration
  // Where the last parareal_iterate ended (rbc_get_state): iterations done,
  // the last two defects, the precision-switch iterations as they stood
  // before the switch test of that last iteration, and its time averages.
  // `resume` (rbc_set_state) is the same record, consumed by the next
  // parareal_iterate, which then continues at iteration k + 1.
  struct IterState {
    int k = -1;
    int kG64 = 0, kF64 = 0;     // INT_MAX: not switched
    double defect = 0, prev = 0;
    int has_avg = 0;
    double avg[rbc::kDiagAvg] = {};
  };
  IterState last, resume;
  rbc::KernelTiming timing;    // fine-grid kernel timing (rbc_kernel_timing_*)
  std::string err;
};

namespace rbc {

constexpr int kCoarseGraphSteps = 8;

// Plans of one run as rbc_create builds them (rbc_api.cpp): "" or the error.
std::string make_run_plans(const rbc_params* p, GridPlan& fine, GridPlan& coarse, int* nf, int* nc);
// Device bytes of those plans' tables; fills the grid shapes and step counts.
size_t run_plan_bytes(const rbc_params* p, int* nf, int* nc, GridPlan* fine_shape, GridPlan* coarse_shape);
// Parameter validation of rbc_create: "" or the error.
std::string params_error(const rbc_params* p);

rbc_status fail(rbc_handle h, rbc_status s, const std::string& msg);

}  // namespace rbc

#define RBC_HIPCHK(h, call)                                                                      \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return rbc::fail((h), RBC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)
