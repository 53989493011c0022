// Parareal (section 3.1, Eq. 19) around the batched fine propagator: the
// serial coarse sweep, the sweep-then-batch iteration, and the pipelined
// iteration, a host scheduler that overlaps the two propagators on two
// streams.
//
// Pipelined iteration.  The fine run F(U_n^(k-1)) of iteration k needs only
// U_n^(k-1), which the coarse sweep of iteration k-1 corrects slice by
// slice, and the sweep of iteration k needs F(U_n^(k-1)) only when it reaches
// slice n.  So each fine run (a "job") is admitted as soon as its initial
// state exists, into a ring of state slots; every fine launch advances all
// jobs in flight by one step, whatever their slice and iteration (the
// kernels are batch-invariant, so a job's result does not depend on its
// batch); a job leaves after its n_f steps, and the coarse stream, which
// waits for it with an event, corrects the next slice.  Jobs enter and leave
// in one order, so those in flight always fill a contiguous range of the
// ring and one launch covers them.  The host never blocks the fine stream on
// the coarse one: it admits a job only after polling that the producing
// coarse task has completed.  Stream-order constraints:
//   - job (k, n) reads U_n^(k-1) (copied into its slot at admission): after
//     the coarse task that wrote it (polled);
//   - the coarse task that overwrites U_n^(k-1) with U_n^k waits for that
//     copy (event);
//   - a slot is reused only after the coarse task that read the previous
//     job's result has completed (polled);
//   - the sweep of iteration k starts after the host has read the defect of
//     iteration k-1 (stop test, precision switch).
// The jobs of iteration k+1 start before the defect of iteration k is known:
// after convergence they are abandoned.
// Two host threads enqueue the work (a kernel launch costs the host
// microseconds, and one thread could not keep both streams fed): the fine
// thread admits jobs and enqueues batched steps, the calling thread enqueues
// coarse work and reads the reports.  With the FP64 switch, FP64 jobs live on
// a third stream: each batched step then advances the mixed and the FP64
// jobs in flight concurrently (disjoint slots and work buffers), and a job's
// events are recorded on its own stream.  They share the admission and
// completion counters and the coarse task counter (atomics, release on
// write after the matching event is recorded, acquire on read).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <climits>
#include <cmath>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "rbc_ctx.hpp"

using rbc::fail;

namespace {

// Coarse sweep over slices [first, S): see rbc_coarse_sweep.  Coarse Nu
// samples of slice n go to nu_c[n] when requested.
rbc_status sweep(rbc_handle h, int mode, int first, double* U, const double* F, double* G, bool with_nu,
                 bool use64 = false) {
  const int S = h->p.n_slices;
  const size_t fs = h->fine.dev.state, cs = h->coarse.dev.state;
  rbc::GridPlan& cp = use64 ? h->coarse64 : h->coarse;
  rbc::Work& cw = use64 ? h->wc64 : h->wc;
  for (int n = first; n < S; ++n) {
    RBC_HIPCHK(h, rbc::launch_restrict(h->fine, cp, U + n * fs, h->Xc, h->stream));
    double* nu = (with_nu && h->nu_c) ? h->nu_c + size_t(n) * h->nsc * rbc::kDiag : nullptr;
    RBC_HIPCHK(h, rbc::launch_steps(cp, cw, h->Xc, 1, h->nc, nu, h->stride_c, h->nsc, h->stream));
    RBC_HIPCHK(h, rbc::launch_combine(h->fine, h->coarse, mode, U + (n + 1) * fs, mode == 1 ? F + n * fs : nullptr,
                                      h->Xc, G + n * cs, h->part + size_t(n + 1) * rbc::kCombineBlocks * 2,
                                      h->stream));
  }
  return RBC_OK;
}

rbc_status read_defect(rbc_handle h, int first, int last, double* defect, bool* bad) {
  RBC_HIPCHK(h, rbc::launch_defect(h->part, first, last, h->dscal, h->stream));
  double v[2];
  RBC_HIPCHK(h, hipMemcpyAsync(v, h->dscal, 16, hipMemcpyDeviceToHost, h->stream));
  RBC_HIPCHK(h, hipStreamSynchronize(h->stream));
  *defect = v[0];
  *bad = v[1] != 0.0;
  return RBC_OK;
}

// Time averages over [nu_t_start, t_end] of the diagnostic samples of slices
// [0, S) (slice(n) points at slice n's [ns][kDiag] records), the consistency
// checks of section 2.2: out = (Nu_V, Nu_b, Nu_t, Nu_int (Eq. 13), KE, Re,
// epsilon_U, P, |P - epsilon_U| / P (Eq. 15)); Re is the mean RMS velocity
// <u^2 + w^2>^(1/2) = (2 KE)^(1/2) over the viscosity.  Fixed summation
// order.
template <typename SliceFn>
void diag_average_host(rbc_handle h, int ns, int stride, double dt, double nu, SliceFn slice, double* out) {
  const int S = h->p.n_slices;
  const double dT = (h->p.t_end - h->p.t0) / S;
  double acc[rbc::kDiag] = {0, 0, 0, 0, 0, 0}, urms = 0;
  long cnt = 0;
  for (int n = 0; n < S; ++n) {
    const double* b = slice(n);
    for (int q = 0; q < ns; ++q) {
      const double t = h->p.t0 + n * dT + (q + 1) * stride * dt;
      if (t < h->p.nu_t_start) continue;
      const double* r = b + size_t(q) * rbc::kDiag;
      for (int c = 0; c < rbc::kDiag; ++c) acc[c] += r[c];
      urms += std::sqrt(2.0 * r[3]);
      ++cnt;
    }
  }
  if (!cnt) {
    for (int c = 0; c < rbc::kDiagAvg; ++c) out[c] = NAN;
    return;
  }
  const double nv = acc[0] / cnt, nb = acc[1] / cnt, nt = acc[2] / cnt;
  const double P = acc[5] / cnt, eps = acc[4] / cnt;
  out[0] = nv;
  out[1] = nb;
  out[2] = nt;
  out[3] = std::max(std::max(std::fabs(nb - nv), std::fabs(nb - nt)), std::fabs(nv - nt)) / nv;
  out[4] = acc[3] / cnt;
  out[5] = urms / cnt / nu;
  out[6] = eps;
  out[7] = P;
  out[8] = std::fabs(P - eps) / P;
}

rbc_status diag_average(rbc_handle h, const double* dev, int ns, int stride, double dt, double nu, double* out) {
  const int S = h->p.n_slices;
  std::vector<double> buf(size_t(S) * ns * rbc::kDiag);
  RBC_HIPCHK(h, hipMemcpyAsync(buf.data(), dev, buf.size() * 8, hipMemcpyDeviceToHost, h->stream));
  RBC_HIPCHK(h, hipStreamSynchronize(h->stream));
  diag_average_host(h, ns, stride, dt, nu, [&](int n) { return buf.data() + size_t(n) * ns * rbc::kDiag; }, out);
  return RBC_OK;
}

// Statistics-based stop (section 5): the time-averaged Nusselt numbers of
// iteration k moved by at most stat_tol (relative) from those of k - 1.
bool stats_converged(rbc_handle h, const double* cur, const double* prev) {
  if (!(h->p.stat_tol > 0)) return false;
  for (int c = 0; c < 3; ++c)
    if (!(std::fabs(cur[c] - prev[c]) <= h->p.stat_tol * std::fabs(cur[c]))) return false;
  return true;
}

// Copies U after iteration k into the iterate history when one is set.
rbc_status save_iterate(rbc_handle h, const double* U, int k, hipStream_t st) {
  if (!h->U_hist || k > h->hist_cap) return RBC_OK;
  const size_t n = size_t(h->p.n_slices + 1) * h->fine.dev.state;
  RBC_HIPCHK(h, hipMemcpyAsync(h->U_hist + size_t(k) * n, U, n * 8, hipMemcpyDeviceToDevice, st));
  return RBC_OK;
}

// The precision switch of promote_fp64, decided after iteration k (defect
// d, previous defect prev): the coarse sweeps switch from k + 1, the fine
// runs from k + 2.
bool promote_now(rbc_handle h, int k, double d, double prev, double tol) {
  return h->has64 && k >= 2 && ((tol < 1e-6 && d <= 1e-3) || (d <= 1e-4 && d > 0.5 * prev));
}

// Records where an iteration ended (rbc_get_state): before the precision
// switch test of iteration k, which a resumed run makes first.
void record_iteration(rbc_handle h, int k, int kG64, int kF64, double defect, double prev, const double* avg) {
  rbc_ctx::IterState& r = h->last;
  r.k = k;
  r.kG64 = kG64;
  r.kF64 = kF64;
  r.defect = defect;
  r.prev = prev;
  r.has_avg = avg ? 1 : 0;
  for (int c = 0; c < rbc::kDiagAvg; ++c) r.avg[c] = avg ? avg[c] : 0.0;
}

// Start of a resumed iteration: the record's switch test of iteration k (as
// the uninterrupted run makes it after reading k's defect), its averages in
// nu_hist[k].
void resume_start(rbc_handle h, const rbc_ctx::IterState& r, double tol, bool want_nu, double* nu_hist, int* kG64,
                  int* kF64, double* defect, double* prev) {
  *kG64 = r.kG64;
  *kF64 = r.kF64;
  *defect = r.defect;
  *prev = r.prev;
  if (*kG64 == INT_MAX && r.k >= 1 && promote_now(h, r.k, r.defect, r.prev, tol)) {
    *kG64 = r.k + 1;
    *kF64 = r.k + 2;
  }
  *prev = r.defect;
  if (want_nu)
    for (int c = 0; c < rbc::kDiagAvg; ++c) nu_hist[size_t(rbc::kDiagAvg) * r.k + c] = r.has_avg ? r.avg[c] : NAN;
}

// ---------------------------------------------------------------- sweep-then-batch ---

rbc_status parareal_sequential(rbc_handle h, double* U, int k_max, double tol, int* k_done, double* defect_hist,
                               double* nu_hist, const rbc_ctx::IterState* from) {
  const int S = h->p.n_slices;
  const size_t fs = h->fine.dev.state;
  const bool want_nu = nu_hist && h->p.nu_stride > 0 && h->nsf > 0;
  rbc_status s;
  *k_done = 0;
  double defect = INFINITY, prev = INFINITY;
  int k = 0, kG64 = INT_MAX, kF64 = INT_MAX;
  if (from) {
    k = from->k;
    *k_done = k;
    resume_start(h, *from, tol, want_nu, nu_hist, &kG64, &kF64, &defect, &prev);
  } else {
    if ((s = sweep(h, 0, 0, U, nullptr, h->Gbuf, want_nu && h->nsc > 0)) != RBC_OK) return s;
    if ((s = save_iterate(h, U, 0, h->stream)) != RBC_OK) return s;
    if (want_nu) {
      if (h->nsc > 0) {
        if ((s = diag_average(h, h->nu_c, h->nsc, h->stride_c, h->coarse.dt, h->coarse.dev.nu, nu_hist)) != RBC_OK)
          return s;
      } else {
        for (int c = 0; c < rbc::kDiagAvg; ++c) nu_hist[c] = NAN;
      }
    }
    RBC_HIPCHK(h, hipStreamSynchronize(h->stream));
    record_iteration(h, 0, kG64, kF64, defect, prev, want_nu ? nu_hist : nullptr);
  }
  h->stop_reason = RBC_STOP_KMAX;
  while (k < k_max && k < S) {
    ++k;
    // F on slices k-1..S-1 from U^(k-1)
    const int na = S - (k - 1);
    double* nu = want_nu ? h->nu_f + size_t(k - 1) * h->nsf * rbc::kDiag : nullptr;
    RBC_HIPCHK(h, hipMemcpyAsync(h->Fbuf + (k - 1) * fs, U + (k - 1) * fs, size_t(na) * fs * 8,
                                 hipMemcpyDeviceToDevice, h->stream));
    const bool f64 = k >= kF64;
    rbc::GridPlan& fp = f64 ? h->fine64 : h->fine;
    rbc::Work& fw = f64 ? h->wf64 : h->wf;
    RBC_HIPCHK(h, rbc::launch_steps(fp, fw, h->Fbuf + (k - 1) * fs, na, h->nf, nu, h->p.nu_stride, h->nsf,
                                    h->stream, f64 ? nullptr : &h->timing));
    // U_k^k = F(U_(k-1)^(k-1)) exactly; then the correction sweep
    RBC_HIPCHK(h, rbc::launch_combine(h->fine, h->coarse, 2, U + k * fs, h->Fbuf + (k - 1) * fs, nullptr, nullptr,
                                      h->part + size_t(k) * rbc::kCombineBlocks * 2, h->stream));
    if ((s = sweep(h, 1, k, U, h->Fbuf, h->Gbuf, false, k >= kG64)) != RBC_OK) return s;
    if ((s = save_iterate(h, U, k, h->stream)) != RBC_OK) return s;
    bool bad = false;
    if ((s = read_defect(h, k, S + 1, &defect, &bad)) != RBC_OK) return s;
    defect_hist[k - 1] = defect;
    *k_done = k;
    if (want_nu && (s = diag_average(h, h->nu_f, h->nsf, h->p.nu_stride, h->fine.dt, h->fine.dev.nu,
                                     nu_hist + rbc::kDiagAvg * k)) != RBC_OK)
      return s;
    record_iteration(h, k, kG64, kF64, defect, prev, want_nu ? nu_hist + rbc::kDiagAvg * k : nullptr);
    if (bad) return fail(h, RBC_ERR_NONFINITE, "non-finite value in Parareal iteration " + std::to_string(k));
    if (defect <= tol) {
      h->stop_reason = RBC_STOP_DEFECT;
      break;
    }
    if (want_nu && stats_converged(h, nu_hist + rbc::kDiagAvg * k, nu_hist + rbc::kDiagAvg * (k - 1))) {
      h->stop_reason = RBC_STOP_STATISTICS;
      break;
    }
    if (kG64 == INT_MAX && promote_now(h, k, defect, prev, tol)) {
      kG64 = k + 1;
      kF64 = k + 2;
    }
    prev = defect;
  }
  h->k_fp64 = (kF64 <= k) ? kF64 : 0;
  if (h->stop_reason == RBC_STOP_KMAX && k == S) h->stop_reason = RBC_STOP_EXACT;
  if (h->stop_reason == RBC_STOP_KMAX && tol > 0) return RBC_NOT_CONVERGED;
  return RBC_OK;
}

// ---------------------------------------------------------------- pipelined ---

constexpr int kFDepth = 6;    // batched fine steps in flight on the fine stream
constexpr int kGDepth = 16;   // coarse chunks (kCoarseGraphSteps steps each) in flight on the coarse stream

enum TaskKind { kPredict, kCopy, kCorrect, kReport };
struct Task {
  TaskKind kind;
  int k, n;
};
struct Job {
  int k, n, slot, start;   // iteration, slice (input U_n^(k-1)), ring slot, first virtual step
  bool f64;
};

class Pipeline {
 public:
  // from: a checkpoint (rbc_set_state) to continue at iteration from->k + 1,
  // or null to start with the coarse prediction.
  Pipeline(rbc_handle h, double* U, int K, double tol, bool want_nu, int* k_done, double* defect_hist,
           double* nu_hist, const rbc_ctx::IterState* from)
      : h_(h), U_(U), S_(h->p.n_slices), K_(K), k0_(from ? from->k : 0), resumed_(from != nullptr),
        nf_(h->nf), nc_(h->nc), cap_(h->ring_cap),
        stride_(h->p.nu_stride), tol_(tol), want_nu_(want_nu), k_done_(k_done), defect_hist_(defect_hist),
        nu_hist_(nu_hist), fs_(h->fine.dev.state), cs_(h->coarse.dev.state), F_(h->fstream), G_(h->gstream),
        F64_(h->f64stream ? h->f64stream : h->fstream) {
    if (from) {
      int g64 = INT_MAX, f64 = INT_MAX;
      resume_start(h, *from, tol, want_nu, nu_hist, &g64, &f64, &defect_, &prev_);
      kG64_ = g64;
      kF64_ = f64;
      processed_ = k0_;
      *k_done = k0_;
    }
  }

  rbc_status run();

 private:
  rbc_handle h_;
  double* U_;
  const int S_, K_, k0_;      // k0_: iterations done before this call (resumed) or 0
  const bool resumed_;
  const int nf_, nc_, cap_, stride_;
  const double tol_;
  const bool want_nu_;
  int* k_done_;
  double* defect_hist_;
  double* nu_hist_;
  const size_t fs_, cs_;
  hipStream_t F_, G_, F64_;   // F64_: FP64 fine jobs (F_ when there is no FP64 stream)

  std::vector<Job> jobs_;
  std::vector<int> job_base_;    // [K+1]: index of job (k, k-1)
  std::vector<Task> tasks_;
  std::vector<int> task_base_;   // [K+1]: index of Copy(k), k >= 1
  hipEvent_t *ev_admit_ = nullptr, *ev_done_ = nullptr, *ev_task_ = nullptr;
  hipEvent_t *ev_step_ = nullptr, *ev_step64_ = nullptr, *ev_chunk_ = nullptr, ev_entry_ = nullptr;

  // fine thread: writes jn_, ja_ (shared), owns t_, freal_
  std::atomic<int> jn_{0}, ja_{0};   // next job to admit, first unfinished job
  int t_ = 0;                        // virtual fine step
  long freal_ = 0;                   // batched fine steps enqueued
  long f64real_ = 0;                 // of those, steps with FP64 jobs on F64_
  // coarse thread: writes gi_, kF64_ (shared), owns the rest
  std::atomic<int> gi_{0};           // next coarse task
  int gstep_ = -1;                   // coarse steps enqueued of task gi_ (-1: not started)
  long gchunks_ = 0;
  int kG64_ = INT_MAX;
  std::atomic<int> kF64_{INT_MAX};
  int processed_ = -1, pending_ = -1;   // last report read, report in flight
  double defect_ = INFINITY, prev_ = INFINITY;
  // both
  std::atomic<bool> stop_{false};
  std::atomic<long> progress_{0};
  std::mutex err_mu_;
  rbc_status status_ = RBC_OK;       // first error (under err_mu_)
  // statistics (per thread, merged at the end)
  double f_admit_s_ = 0, f_fine_s_ = 0, f_wait_s_ = 0, runs_ = 0;
  long f_steps_ = 0;

  int job_index(int k, int n) const { return job_base_[k] + (n - (k - 1)); }
  int producer(const Job& J) const {
    if (J.n == 0) return -1;                                          // U_0
    if (J.k == k0_ + 1 && resumed_) return -1;                        // U^(k0) of the checkpoint
    if (J.k == 1) return J.n - 1;                                     // Predict(0, n-1)
    if (J.n == J.k - 1) return task_base_[J.k - 1];                   // Copy(k-1)
    return task_base_[J.k - 1] + 1 + (J.n - 1 - (J.k - 1));           // Correct(k-1, n-1)
  }
  int consumer(const Job& J) const {
    if (J.n == J.k - 1) return task_base_[J.k];                       // Copy(k)
    return task_base_[J.k] + 1 + (J.n - J.k);                         // Correct(k, n)
  }
  int report_task(int k) const { return k == 0 ? S_ : task_base_[k] + 1 + (S_ - k); }

  // 1 complete, 0 pending, -1 error (status_ set)
  int query(hipEvent_t e) {
    const hipError_t r = hipEventQuery(e);
    if (r == hipSuccess) return 1;
    if (r == hipErrorNotReady) return 0;
    herr(r, "hipEventQuery");
    return -1;
  }
  int task_done(int ti) { return ti < gi_.load(std::memory_order_acquire) ? query(ev_task_[ti]) : 0; }
  void seterr(rbc_status st, const std::string& msg) {
    std::lock_guard<std::mutex> lk(err_mu_);
    if (status_ == RBC_OK) status_ = fail(h_, st, msg);
    stop_.store(true);
  }
  rbc_status status() {
    std::lock_guard<std::mutex> lk(err_mu_);
    return status_;
  }
  void herr(hipError_t e, const char* what) { seterr(RBC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e)); }
  bool ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    herr(e, what);
    return false;
  }

  rbc_status setup();
  rbc_status build_graph(rbc::GridPlan& cp, rbc::Work& cw, hipGraphExec_t* ex);
  int admit();
  int fine_step();
  int coarse_work();
  int poll_report();
  void fine_loop();
};

// Captures kCoarseGraphSteps coarse steps on Xc (the steps inside a coarse
// run: no first transform, no Nu samples, never the last step) as a graph;
// every coarse run replays it.  Kernel arguments are fixed per plan.
rbc_status Pipeline::build_graph(rbc::GridPlan& cp, rbc::Work& cw, hipGraphExec_t* ex) {
  if (*ex) return RBC_OK;
  hipStream_t cs = nullptr;
  RBC_HIPCHK(h_, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rbc::StepRange r;
    r.slot0 = 0;
    r.count = 1;
    r.step0 = 1;
    r.step1 = 1 + rbc::kCoarseGraphSteps;
    r.n_total = INT_MAX;
    const hipError_t e1 = rbc::launch_step_range(cp, cw, h_->Xc, r, nullptr, 0, 0, cs, nullptr);
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    e = (e1 != hipSuccess) ? e1 : e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    *ex = nullptr;
    return fail(h_, RBC_ERR_HIP, std::string("coarse step graph: ") + hipGetErrorString(e));
  }
  return RBC_OK;
}

rbc_status Pipeline::setup() {
  rbc_status s_;
  for (int k = 0; k <= K_; ++k) job_base_.push_back(0);
  for (int k = k0_ + 1; k <= K_; ++k) {
    job_base_[k] = int(jobs_.size());
    for (int n = k - 1; n < S_; ++n) jobs_.push_back({k, n, int(jobs_.size() % cap_), -1, false});
  }
  task_base_.assign(K_ + 1, 0);
  if (!resumed_) {
    for (int n = 0; n < S_; ++n) tasks_.push_back({kPredict, 0, n});
    tasks_.push_back({kReport, 0, -1});
  }
  for (int k = k0_ + 1; k <= K_; ++k) {
    task_base_[k] = int(tasks_.size());
    tasks_.push_back({kCopy, k, k - 1});
    for (int n = k; n < S_; ++n) tasks_.push_back({kCorrect, k, n});
    tasks_.push_back({kReport, k, -1});
  }
  const size_t need = 2 * jobs_.size() + tasks_.size() + 2 * kFDepth + kGDepth + 1;
  while (h_->evpool.size() < need) {
    hipEvent_t e;
    RBC_HIPCHK(h_, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h_->evpool.push_back(e);
  }
  if ((s_ = build_graph(h_->coarse, h_->wc, &h_->cgraph)) != RBC_OK) return s_;
  if (h_->has64 && (s_ = build_graph(h_->coarse64, h_->wc64, &h_->cgraph64)) != RBC_OK) return s_;
  hipEvent_t* p = h_->evpool.data();
  ev_admit_ = p; p += jobs_.size();
  ev_done_ = p; p += jobs_.size();
  ev_task_ = p; p += tasks_.size();
  ev_step_ = p; p += kFDepth;
  ev_step64_ = p; p += kFDepth;
  ev_chunk_ = p; p += kGDepth;
  ev_entry_ = *p;
  return RBC_OK;
}

// Admits jobs in order while their input exists and a slot is free.
int Pipeline::admit() {
  int did = 0;
  while (jn_ < int(jobs_.size())) {
    Job& J = jobs_[jn_];
    const int p = producer(J);
    if (p >= 0) {
      const int q = task_done(p);
      if (q <= 0) return q < 0 ? -1 : did;
    }
    if (jn_ >= cap_) {
      const int q = task_done(consumer(jobs_[jn_ - cap_]));
      if (q <= 0) return q < 0 ? -1 : did;
    }
    if (want_nu_) {   // runs start on multiples of the sampling stride
      if (ja_ < jn_) {
        if (t_ % stride_ != 0) return did;
      } else {
        t_ = (t_ + stride_ - 1) / stride_ * stride_;
      }
    }
    J.f64 = J.k >= kF64_;   // final: the report of iteration k-2 has been read
    J.start = t_;
    rbc::GridPlan& fp = J.f64 ? h_->fine64 : h_->fine;
    rbc::Work& fw = J.f64 ? h_->wf64 : h_->wf;
    hipStream_t js = J.f64 ? F64_ : F_;
    if (want_nu_ && !ok(rbc::launch_set_meta(h_->meta, J.slot, {J.k & 1, J.n, J.start, 0}, js), "set_meta"))
      return -1;
    if (!ok(hipMemcpyAsync(h_->Xring + J.slot * fs_, U_ + J.n * fs_, fs_ * 8, hipMemcpyDeviceToDevice, js),
            "hipMemcpyAsync"))
      return -1;
    rbc::StepRange r;
    r.slot0 = J.slot;
    r.count = 1;
    r.step0 = r.step1 = 0;   // the inverse transform of the initial state only
    r.n_total = 1;
    if (!ok(rbc::launch_step_range(fp, fw, h_->Xring, r, nullptr, 0, 0, js), "zinv")) return -1;
    if (!ok(hipEventRecord(ev_admit_[jn_], js), "hipEventRecord")) return -1;
    ++jn_;
    did = 1;
  }
  return did;
}

// One batched step of every job in flight (mixed jobs on F_, FP64 jobs on
// F64_).
int Pipeline::fine_step() {
  if (ja_ == jn_) return 0;
  if (freal_ >= kFDepth) {
    const int q = query(ev_step_[freal_ % kFDepth]);
    if (q <= 0) return q;
  }
  int jm = ja_;
  while (jm < jn_ && !jobs_[jm].f64) ++jm;
  const bool sep = F64_ != F_ && jn_ > jm;   // FP64 jobs on their own stream this step
  if (sep && f64real_ >= kFDepth) {
    const int q = query(ev_step64_[f64real_ % kFDepth]);
    if (q <= 0) return q;
  }
  rbc::StepRange r;
  r.step0 = 1;
  r.step1 = 2;
  r.n_total = INT_MAX;   // never the last step: the next step's transform is always made
  r.timing_index = freal_;
  if (jm > ja_) {
    r.slot0 = jobs_[ja_].slot;
    r.count = jm - ja_;
    if (!ok(rbc::launch_step_range(h_->fine, h_->wf, h_->Xring, r, nullptr, 0, 0, F_, &h_->timing), "fine step"))
      return -1;
  }
  if (jn_ > jm) {
    r.slot0 = jobs_[jm].slot;
    r.count = jn_ - jm;
    if (!ok(rbc::launch_step_range(h_->fine64, h_->wf64, h_->Xring, r, nullptr, 0, 0, F64_), "fine step")) return -1;
  }
  ++t_;
  if (want_nu_ && t_ % stride_ == 0) {
    // the samples of each range on its stream, each with its own partials
    if (!sep && !ok(rbc::launch_diag(h_->fine, h_->wf, h_->Xring, jobs_[ja_].slot, jn_ - ja_, cap_, h_->nu_f, 0,
                                     h_->meta, t_, stride_, h_->nsf, S_, F_),
                    "diagnostics"))
      return -1;
    if (sep && jm > ja_ &&
        !ok(rbc::launch_diag(h_->fine, h_->wf, h_->Xring, jobs_[ja_].slot, jm - ja_, cap_, h_->nu_f, 0, h_->meta, t_,
                             stride_, h_->nsf, S_, F_),
            "diagnostics"))
      return -1;
    if (sep && !ok(rbc::launch_diag(h_->fine64, h_->wf64, h_->Xring, jobs_[jm].slot, jn_ - jm, cap_, h_->nu_f, 0,
                                    h_->meta, t_, stride_, h_->nsf, S_, F64_),
                   "diagnostics"))
      return -1;
  }
  while (ja_ < jn_ && jobs_[ja_].start + nf_ == t_) {
    if (!ok(hipEventRecord(ev_done_[ja_], jobs_[ja_].f64 ? F64_ : F_), "hipEventRecord")) return -1;
    ++ja_;
  }
  if (!ok(hipEventRecord(ev_step_[freal_ % kFDepth], F_), "hipEventRecord")) return -1;
  ++freal_;
  if (sep) {
    if (!ok(hipEventRecord(ev_step64_[f64real_ % kFDepth], F64_), "hipEventRecord")) return -1;
    ++f64real_;
  }
  return 1;
}

// Enqueues the next piece of the coarse stream: a whole copy or report
// task, or the start or a chunk of coarse steps of a predict / correct task.
int Pipeline::coarse_work() {
  if (gi_ == int(tasks_.size())) return 0;
  if (gchunks_ >= kGDepth) {
    const int q = query(ev_chunk_[gchunks_ % kGDepth]);
    if (q <= 0) return q;
  }
  const Task T = tasks_[gi_];
  const bool g64 = T.k >= kG64_;
  rbc::GridPlan& cp = g64 ? h_->coarse64 : h_->coarse;
  rbc::Work& cw = g64 ? h_->wc64 : h_->wc;
  if (gstep_ < 0) {
    if (T.kind == kCopy) {
      if (processed_ < T.k - 1) return 0;
      const int j0 = job_index(T.k, T.k - 1);
      const int j1 = (T.k <= S_ - 1) ? job_index(T.k, T.k) : -1;
      if (ja_ <= j0 || (j1 >= 0 && jn_ <= j1)) return 0;
      if (!ok(hipStreamWaitEvent(G_, ev_done_[j0], 0), "hipStreamWaitEvent")) return -1;
      if (j1 >= 0 && !ok(hipStreamWaitEvent(G_, ev_admit_[j1], 0), "hipStreamWaitEvent")) return -1;
      if (!ok(rbc::launch_combine(h_->fine, h_->coarse, 2, U_ + T.k * fs_, h_->Xring + jobs_[j0].slot * fs_, nullptr,
                                  nullptr, h_->part + size_t(T.k) * rbc::kCombineBlocks * 2, G_),
              "combine"))
        return -1;
      if (!ok(hipEventRecord(ev_task_[gi_], G_), "hipEventRecord")) return -1;
      ++gi_;
      return 1;
    }
    if (T.kind == kReport) {
      double* pin = h_->host_pin;
      if (h_->U_hist && T.k <= h_->hist_cap) {
        const size_t n = size_t(S_ + 1) * fs_;
        if (!ok(hipMemcpyAsync(h_->U_hist + size_t(T.k) * n, U_, n * 8, hipMemcpyDeviceToDevice, G_),
                "hipMemcpyAsync"))
          return -1;
      }
      if (T.k >= 1) {
        if (!ok(rbc::launch_defect(h_->part, T.k, S_ + 1, h_->dscal, G_), "defect")) return -1;
        if (!ok(hipMemcpyAsync(pin, h_->dscal, 16, hipMemcpyDeviceToHost, G_), "hipMemcpyAsync")) return -1;
      }
      if (want_nu_) {
        double* nuF = pin + 2;
        double* nuC = nuF + size_t(2) * S_ * h_->nsf * rbc::kDiag;
        if (T.k == 0 && h_->nsc > 0 &&
            !ok(hipMemcpyAsync(nuC, h_->nu_c, size_t(S_) * h_->nsc * rbc::kDiag * 8, hipMemcpyDeviceToHost, G_),
                "hipMemcpyAsync"))
          return -1;
        if (T.k >= 1 &&
            !ok(hipMemcpyAsync(nuF, h_->nu_f, size_t(2) * S_ * h_->nsf * rbc::kDiag * 8, hipMemcpyDeviceToHost, G_),
                "hipMemcpyAsync"))
          return -1;
      }
      if (!ok(hipEventRecord(ev_task_[gi_], G_), "hipEventRecord")) return -1;
      pending_ = T.k;
      ++gi_;
      return 1;
    }
    if (T.kind == kCorrect) {
      const int j = job_index(T.k, T.n);
      const int j1 = (T.n + 1 <= S_ - 1) ? job_index(T.k, T.n + 1) : -1;
      if (ja_ <= j || (j1 >= 0 && jn_ <= j1)) return 0;
      if (!ok(hipStreamWaitEvent(G_, ev_done_[j], 0), "hipStreamWaitEvent")) return -1;
      if (j1 >= 0 && !ok(hipStreamWaitEvent(G_, ev_admit_[j1], 0), "hipStreamWaitEvent")) return -1;
    }
    if (!ok(rbc::launch_restrict(h_->fine, cp, U_ + T.n * fs_, h_->Xc, G_), "restrict")) return -1;
    gstep_ = 0;
  }
  // the first chunk (with the first transform), the chunk holding the last
  // step and runs with Nu samples are launched directly; the rest replay
  // the graph
  const int C = rbc::kCoarseGraphSteps;
  double* nu =
      (T.kind == kPredict && want_nu_ && h_->nu_c) ? h_->nu_c + size_t(T.n) * h_->nsc * rbc::kDiag : nullptr;
  hipGraphExec_t gx = g64 ? h_->cgraph64 : h_->cgraph;
  if (gstep_ > 0 && !nu && gx && gstep_ + C <= nc_ - 1) {
    if (!ok(hipGraphLaunch(gx, G_), "hipGraphLaunch")) return -1;
    gstep_ += C;
  } else {
    const int c = std::min(C, nc_ - gstep_);
    rbc::StepRange r;
    r.slot0 = 0;
    r.count = 1;
    r.step0 = gstep_;
    r.step1 = gstep_ + c;
    r.n_total = nc_;
    if (!ok(rbc::launch_step_range(cp, cw, h_->Xc, r, nu, h_->stride_c, h_->nsc, G_), "coarse steps")) return -1;
    gstep_ += c;
  }
  if (gstep_ == nc_) {
    const int mode = (T.kind == kPredict) ? 0 : 1;
    const double* F = (mode == 1) ? h_->Xring + jobs_[job_index(T.k, T.n)].slot * fs_ : nullptr;
    if (!ok(rbc::launch_combine(h_->fine, h_->coarse, mode, U_ + (T.n + 1) * fs_, F, h_->Xc, h_->Gbuf + T.n * cs_,
                                h_->part + size_t(T.n + 1) * rbc::kCombineBlocks * 2, G_),
            "combine"))
      return -1;
    if (!ok(hipEventRecord(ev_task_[gi_], G_), "hipEventRecord")) return -1;
    ++gi_;
    gstep_ = -1;
  }
  if (!ok(hipEventRecord(ev_chunk_[gchunks_ % kGDepth], G_), "hipEventRecord")) return -1;
  ++gchunks_;
  return 1;
}

// Reads a completed report: defect, Nu averages, the stop test and the
// precision switch (the same rules, in the same order, as the
// sweep-then-batch iteration).
int Pipeline::poll_report() {
  if (pending_ < 0) return 0;
  const int q = query(ev_task_[report_task(pending_)]);
  if (q <= 0) return q;
  const int k = pending_;
  pending_ = -1;
  processed_ = k;
  const double* pin = h_->host_pin;
  const double* nuF = pin + 2;
  const double* nuC = nuF + size_t(2) * S_ * h_->nsf * rbc::kDiag;
  if (k == 0) {
    if (want_nu_) {
      if (h_->nsc > 0)
        diag_average_host(h_, h_->nsc, h_->stride_c, h_->coarse.dt, h_->coarse.dev.nu,
                          [&](int n) { return nuC + size_t(n) * h_->nsc * rbc::kDiag; }, nu_hist_);
      else
        for (int c = 0; c < rbc::kDiagAvg; ++c) nu_hist_[c] = NAN;
    }
    record_iteration(h_, 0, kG64_, kF64_, defect_, prev_, want_nu_ ? nu_hist_ : nullptr);
    if (K_ == 0) stop_ = true;
    return 1;
  }
  defect_ = pin[0];
  const bool bad = pin[1] != 0.0;
  defect_hist_[k - 1] = defect_;
  *k_done_ = k;
  if (want_nu_) {
    // slice n's latest run: iteration k for n >= k-1, else iteration n+1
    const int nsf = h_->nsf;
    diag_average_host(h_, nsf, stride_, h_->fine.dt, h_->fine.dev.nu,
                      [&](int n) {
                        const int par = (n >= k - 1) ? (k & 1) : ((n + 1) & 1);
                        return nuF + (size_t(par) * S_ + n) * nsf * rbc::kDiag;
                      },
                      nu_hist_ + rbc::kDiagAvg * k);
  }
  record_iteration(h_, k, kG64_, kF64_.load(), defect_, prev_, want_nu_ ? nu_hist_ + rbc::kDiagAvg * k : nullptr);
  if (bad) {
    seterr(RBC_ERR_NONFINITE, "non-finite value in Parareal iteration " + std::to_string(k));
    return 1;
  }
  if (defect_ <= tol_) {
    h_->stop_reason = RBC_STOP_DEFECT;
    stop_ = true;
    return 1;
  }
  if (want_nu_ && stats_converged(h_, nu_hist_ + rbc::kDiagAvg * k, nu_hist_ + rbc::kDiagAvg * (k - 1))) {
    h_->stop_reason = RBC_STOP_STATISTICS;
    stop_ = true;
    return 1;
  }
  if (k == K_) {
    stop_ = true;
    return 1;
  }
  if (kG64_ == INT_MAX && promote_now(h_, k, defect_, prev_, tol_)) {
    kG64_ = k + 1;
    kF64_ = k + 2;
  }
  prev_ = defect_;
  return 1;
}

// The fine thread: admissions and batched steps until the iteration stops.
void Pipeline::fine_loop() {
  using clk = std::chrono::steady_clock;
  const hipError_t e = hipSetDevice(h_->device);
  if (e != hipSuccess) {
    herr(e, "hipSetDevice");
    return;
  }
  while (!stop_.load()) {
    auto tp = clk::now();
    const int a = admit();
    const auto t1 = clk::now();
    f_admit_s_ += std::chrono::duration<double>(t1 - tp).count();
    if (a < 0) break;
    const int inflight = jn_ - ja_;
    const int b = fine_step();
    const auto t2 = clk::now();
    f_fine_s_ += std::chrono::duration<double>(t2 - t1).count();
    if (b < 0) break;
    if (b > 0) {
      ++f_steps_;
      runs_ += inflight;
    }
    if (a | b) {
      progress_.fetch_add(1);
      continue;
    }
    std::this_thread::yield();
    f_wait_s_ += std::chrono::duration<double>(clk::now() - t2).count();
  }
}

rbc_status Pipeline::run() {
  using clk = std::chrono::steady_clock;
  *k_done_ = k0_;
  h_->stop_reason = RBC_STOP_KMAX;
  rbc_status s = setup();
  if (s != RBC_OK) return s;
  // the streams start after the caller's work
  RBC_HIPCHK(h_, hipEventRecord(ev_entry_, h_->stream));
  RBC_HIPCHK(h_, hipStreamWaitEvent(F_, ev_entry_, 0));
  RBC_HIPCHK(h_, hipStreamWaitEvent(G_, ev_entry_, 0));
  if (F64_ != F_) RBC_HIPCHK(h_, hipStreamWaitEvent(F64_, ev_entry_, 0));
  rbc_pipeline_stats& ps = h_->pstats;
  ps = rbc_pipeline_stats{};
  const auto t_start = clk::now();
  std::thread fine;
  try {
    fine = std::thread(&Pipeline::fine_loop, this);
  } catch (const std::exception& ex) {
    return fail(h_, RBC_ERR_STATE, std::string("cannot start the fine-run thread: ") + ex.what());
  }
  // the coarse work and the reports on this thread; a watchdog ends a
  // schedule in which neither thread has enqueued anything for a minute
  long seen = -1;
  auto last = t_start;
  while (!stop_.load()) {
    auto tp = clk::now();
    const int processed_before = processed_;
    const int r = poll_report();
    const auto t1 = clk::now();
    ps.host_report_s += std::chrono::duration<double>(t1 - tp).count();
    if (r < 0) break;
    if (processed_ != processed_before && processed_ >= 0 && processed_ < 64)
      ps.report_at_s[processed_] = std::chrono::duration<double>(t1 - t_start).count();
    if (stop_.load()) break;
    const int c = coarse_work();
    const auto t2 = clk::now();
    ps.host_coarse_s += std::chrono::duration<double>(t2 - t1).count();
    if (c < 0) break;
    if (c > 0) ++ps.coarse_chunks;
    if (r | c) progress_.fetch_add(1);
    const long pg = progress_.load();
    if (pg != seen) {
      seen = pg;
      last = t2;
    } else if (t2 - last > std::chrono::seconds(60)) {
      seterr(RBC_ERR_STATE, "pipelined Parareal: nothing enqueued for 60 s");
      break;
    }
    if (!(r | c)) {
      std::this_thread::yield();
      ps.host_wait_s += std::chrono::duration<double>(clk::now() - t2).count();
    }
  }
  stop_.store(true);
  fine.join();
  // abandoned speculative work and everything enqueued finishes here
  hipError_t e1 = hipStreamSynchronize(F_);
  const hipError_t e2 = hipStreamSynchronize(G_);
  if (F64_ != F_) {
    const hipError_t e3 = hipStreamSynchronize(F64_);
    if (e1 == hipSuccess) e1 = e3;
  }
  ps.wall_s = std::chrono::duration<double>(clk::now() - t_start).count();
  ps.host_admit_s = f_admit_s_;
  ps.host_fine_s = f_fine_s_;
  ps.host_wait_s += f_wait_s_;
  ps.fine_steps = f_steps_;
  ps.mean_runs_per_step = f_steps_ ? runs_ / f_steps_ : 0.0;
  const rbc_status st = status();
  if (st != RBC_OK) return st;
  if (e1 != hipSuccess || e2 != hipSuccess)
    return fail(h_, RBC_ERR_HIP, std::string("pipelined Parareal: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  h_->k_fp64 = (kF64_ <= *k_done_) ? kF64_.load() : 0;
  if (h_->stop_reason == RBC_STOP_KMAX && *k_done_ == S_) h_->stop_reason = RBC_STOP_EXACT;
  if (h_->stop_reason == RBC_STOP_KMAX && tol_ > 0) return RBC_NOT_CONVERGED;
  return RBC_OK;
}

}  // namespace

extern "C" {

rbc_status rbc_coarse_sweep(rbc_handle h, int32_t mode, int32_t first, double* U, const double* F, double* G,
                            double* defect_host) {
  if (!h || !U || !G) return fail(h, RBC_ERR_ARG, "null argument");
  if (mode != 0 && mode != 1) return fail(h, RBC_ERR_ARG, "mode must be 0 (predict) or 1 (correct)");
  if (mode == 1 && !F) return fail(h, RBC_ERR_ARG, "F is NULL in correct mode");
  if (first < 0 || first > h->p.n_slices) return fail(h, RBC_ERR_ARG, "first_slice out of range");
  rbc_status s = sweep(h, mode, first, U, F, G, false);
  if (s != RBC_OK) return s;
  if (defect_host) {
    bool bad = false;
    if ((s = read_defect(h, first + 1, h->p.n_slices + 1, defect_host, &bad)) != RBC_OK) return s;
    if (bad) return fail(h, RBC_ERR_NONFINITE, "non-finite value in the coarse sweep");
  }
  return RBC_OK;
}

rbc_status parareal_iterate(rbc_handle h, double* U, int32_t k_max, double tol, int32_t* k_done,
                            double* defect_hist, double* nu_hist) {
  if (!h || !U || !k_done || !defect_hist) return fail(h, RBC_ERR_ARG, "null argument");
  if (k_max < 0) return fail(h, RBC_ERR_ARG, "k_max < 0");
  h->k_fp64 = 0;
  h->stop_reason = -1;
  // a checkpoint set by rbc_set_state is consumed by this call
  const rbc_ctx::IterState from = h->resume;
  h->resume = rbc_ctx::IterState{};
  const rbc_ctx::IterState* fp = from.k >= 0 ? &from : nullptr;
  const int K = std::min<int>(k_max, h->p.n_slices);
  if (fp && fp->k >= K) {
    // nothing left to do: the checkpoint already holds iteration K
    *k_done = fp->k;
    h->last = from;
    h->stop_reason = (fp->k == h->p.n_slices) ? RBC_STOP_EXACT : RBC_STOP_KMAX;
    return RBC_OK;
  }
  if (!h->p.pipelined) return parareal_sequential(h, U, k_max, tol, k_done, defect_hist, nu_hist, fp);
  const bool want_nu = nu_hist && h->p.nu_stride > 0 && h->nsf > 0;
  Pipeline pl(h, U, K, tol, want_nu, k_done, defect_hist, nu_hist, fp);
  return pl.run();
}

// ------------------------------------------------------------ checkpoints ---
//
// Layout of a checkpoint (host memory, native byte order):
//   char[8] "RBCCKPT1";
//   int64 n_slices, fine state doubles, coarse state doubles, samples per
//         slice (nsf), k, kG64, kF64, has_avg;
//   double defect, prev, avg[RBC_DIAG_AVG];
//   double G[n_slices][coarse state]        the coarse part of G(U_n^k);
//   double samples[n_slices][nsf][RBC_DIAG]  slice n's diagnostic samples
//         from its latest fine run (read by the time averages of later
//         iterations for the slices that no longer run).
namespace {
constexpr char kCkptMagic[8] = {'R', 'B', 'C', 'C', 'K', 'P', 'T', '1'};
constexpr size_t kCkptHead = 8 + 8 * 8 + (2 + rbc::kDiagAvg) * 8;

size_t ckpt_bytes(rbc_handle h) {
  const size_t S = h->p.n_slices;
  return kCkptHead + S * h->coarse.dev.state * 8 + S * size_t(h->nsf) * rbc::kDiag * 8;
}

// Slot of slice n's latest samples in the handle's sample buffer after
// iteration k (the pipelined schedule alternates two buffers by iteration
// parity; the sweep-then-batch schedule keeps one).
size_t sample_block(rbc_handle h, int k, int n) {
  const size_t blk = size_t(h->nsf) * rbc::kDiag;
  if (!h->p.pipelined) return size_t(n) * blk;
  const int par = (n >= k - 1) ? (k & 1) : ((n + 1) & 1);
  return (size_t(par) * h->p.n_slices + n) * blk;
}
}  // namespace

extern "C" rbc_status rbc_get_state(rbc_handle h, void* buf, size_t* bytes) {
  if (!h || !bytes) return fail(h, RBC_ERR_ARG, "null argument");
  const size_t need = ckpt_bytes(h);
  if (!buf) {
    *bytes = need;
    return RBC_OK;
  }
  if (*bytes < need) return fail(h, RBC_ERR_ARG, "checkpoint buffer too small: " + std::to_string(need) + " bytes");
  if (h->last.k < 0) return fail(h, RBC_ERR_STATE, "no Parareal iteration to checkpoint");
  const rbc_ctx::IterState& r = h->last;
  const int S = h->p.n_slices;
  unsigned char* o = static_cast<unsigned char*>(buf);
  std::memcpy(o, kCkptMagic, 8);
  const int64_t hi[8] = {S, int64_t(h->fine.dev.state), int64_t(h->coarse.dev.state), h->nsf,
                         r.k, r.kG64, r.kF64, r.has_avg};
  std::memcpy(o + 8, hi, sizeof(hi));
  double hd[2 + rbc::kDiagAvg];
  hd[0] = r.defect;
  hd[1] = r.prev;
  for (int c = 0; c < rbc::kDiagAvg; ++c) hd[2 + c] = r.avg[c];
  std::memcpy(o + 8 + sizeof(hi), hd, sizeof(hd));
  double* G = reinterpret_cast<double*>(o + kCkptHead);
  const size_t cs = h->coarse.dev.state;
  RBC_HIPCHK(h, hipMemcpyAsync(G, h->Gbuf, size_t(S) * cs * 8, hipMemcpyDeviceToHost, h->stream));
  const size_t blk = size_t(h->nsf) * rbc::kDiag;
  double* smp = G + size_t(S) * cs;
  if (blk > 0 && h->nu_f)
    for (int n = 0; n < S; ++n)
      RBC_HIPCHK(h, hipMemcpyAsync(smp + n * blk, h->nu_f + sample_block(h, r.k, n), blk * 8, hipMemcpyDeviceToHost,
                                   h->stream));
  RBC_HIPCHK(h, hipStreamSynchronize(h->stream));
  *bytes = need;
  return RBC_OK;
}

extern "C" rbc_status rbc_set_state(rbc_handle h, const void* buf, size_t bytes) {
  if (!h || !buf) return fail(h, RBC_ERR_ARG, "null argument");
  if (bytes < kCkptHead) return fail(h, RBC_ERR_ARG, "checkpoint too short");
  const unsigned char* in = static_cast<const unsigned char*>(buf);
  if (std::memcmp(in, kCkptMagic, 8) != 0) return fail(h, RBC_ERR_ARG, "not a checkpoint (bad magic)");
  int64_t hi[8];
  std::memcpy(hi, in + 8, sizeof(hi));
  const int S = h->p.n_slices;
  if (hi[0] != S || hi[1] != int64_t(h->fine.dev.state) || hi[2] != int64_t(h->coarse.dev.state) ||
      hi[3] != h->nsf)
    return fail(h, RBC_ERR_ARG, "checkpoint of another configuration (slices, grids or sampling differ)");
  if (bytes < ckpt_bytes(h)) return fail(h, RBC_ERR_ARG, "checkpoint too short");
  if (hi[4] < 0 || hi[4] > S) return fail(h, RBC_ERR_ARG, "checkpoint iteration out of range");
  double hd[2 + rbc::kDiagAvg];
  std::memcpy(hd, in + 8 + sizeof(hi), sizeof(hd));
  rbc_ctx::IterState r;
  r.k = int(hi[4]);
  r.kG64 = hi[5] >= INT_MAX ? INT_MAX : int(hi[5]);
  r.kF64 = hi[6] >= INT_MAX ? INT_MAX : int(hi[6]);
  r.has_avg = int(hi[7]);
  r.defect = hd[0];
  r.prev = hd[1];
  for (int c = 0; c < rbc::kDiagAvg; ++c) r.avg[c] = hd[2 + c];
  if (!h->has64) r.kG64 = r.kF64 = INT_MAX;   // this handle has no FP64 propagators
  const double* G = reinterpret_cast<const double*>(in + kCkptHead);
  const size_t cs = h->coarse.dev.state;
  RBC_HIPCHK(h, hipMemcpyAsync(h->Gbuf, G, size_t(S) * cs * 8, hipMemcpyHostToDevice, h->stream));
  const size_t blk = size_t(h->nsf) * rbc::kDiag;
  const double* smp = G + size_t(S) * cs;
  // each slice's samples where the next iteration reads those of slices that
  // no longer run: the one buffer, or the parity buffer of iteration n + 1
  if (blk > 0 && h->nu_f)
    for (int n = 0; n < S; ++n) {
      const size_t at = h->p.pipelined ? (size_t((n + 1) & 1) * S + n) * blk : size_t(n) * blk;
      RBC_HIPCHK(h, hipMemcpyAsync(h->nu_f + at, smp + n * blk, blk * 8, hipMemcpyHostToDevice, h->stream));
    }
  RBC_HIPCHK(h, hipStreamSynchronize(h->stream));
  h->resume = r;
  h->last = r;
  return RBC_OK;
}

rbc_status rbc_get_pipeline_stats(rbc_handle h, rbc_pipeline_stats* out) {
  if (!h || !out) return fail(h, RBC_ERR_ARG, "null argument");
  *out = h->pstats;
  return RBC_OK;
}

rbc_status rbc_set_iterate_history(rbc_handle h, double* U_hist, int32_t k_cap) {
  if (!h) return RBC_ERR_ARG;
  if (U_hist && k_cap < 0) return fail(h, RBC_ERR_ARG, "k_cap < 0");
  h->U_hist = U_hist;
  h->hist_cap = U_hist ? k_cap : -1;
  return RBC_OK;
}

rbc_status rbc_stop_reason(rbc_handle h, int32_t* reason) {
  if (!h || !reason) return fail(h, RBC_ERR_ARG, "null argument");
  *reason = h->stop_reason;
  return RBC_OK;
}

rbc_status rbc_fine_fp64_from(rbc_handle h, int32_t* k) {
  if (!h || !k) return fail(h, RBC_ERR_ARG, "null argument");
  *k = h->k_fp64;
  return RBC_OK;
}

}  // extern "C"
