// Ensembles of independent Parareal runs advanced together (rbc_ensemble_*
// in include/rbc.h): many runs of different Rayleigh numbers, grids, steps
// and horizons share the device, and every launch of a stage covers the
// work of all runs of one grid shape.
//
// Each run is the Parareal iteration of section 3.1 (Eq. 19) in the
// sweep-then-batch order, exactly as parareal_iterate runs it on a handle
// without the pipelined schedule: iteration k runs F on slices k-1..S-1
// from U^(k-1), sets U_k^k = F(U_(k-1)^(k-1)), corrects slices k..S-1 with
// the serial coarse sweep and takes the defect of section 3.7.  The engine
// advances every active run by one iteration per rbc_ensemble_step:
//   - fine work: the (run, slice) pairs of all runs of one fine grid shape
//     form one batch, ordered by the run's fine steps per slice (most
//     first), so the pairs still stepping at fine step t are a prefix and
//     each launch covers that prefix (a cost-ordered work list);
//   - coarse sweeps: the runs' serial sweeps go in lock step, position by
//     position; at each position the coarse steps of all runs of one coarse
//     grid shape are one batch, ordered by coarse steps per slice;
//   - restriction, correction and defect stay per run (they are small).
// A batch gathers its states through a pointer table and each state's run
// parameters (band factors, diffusivities, stage coefficients) through a
// second one (GridDev::xptrs, rptrs), so runs keep their own buffers and a
// run computes the same bits alone or in any batch.  Runs may be added
// between steps (continuous batching): a new run starts with its coarse
// prediction in the next step.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "rbc_ctx.hpp"

namespace {

using rbc::GridPlan;

enum RunState { kActive = 0, kDone = 1, kFailed = 2, kReleased = 3 };

struct Run {
  rbc_params p{};
  GridPlan fine, coarse;
  int nf = 0, nc = 0, S = 0;
  double* U = nullptr;      // [S+1][fine state]  iterates
  double* F = nullptr;      // [S][fine state]    fine runs of the current iteration
  double* G = nullptr;      // [S][coarse state]  coarse part of G(U_n^k)
  double* Xc = nullptr;     // [coarse state]     coarse state being advanced
  double* part = nullptr;   // [S+1][kCombineBlocks][2]
  double* dscal = nullptr;  // [2] defect, non-finite flag
  int k = -1;               // iterations done (-1: coarse prediction pending)
  int k_max = 0;
  double tol = 0;
  int state = kActive;
  int stop = -1;            // rbc_stop of a finished run
  std::vector<double> defects;
  size_t bytes = 0;
  std::string fkey, ckey;
  int first = 0;            // first sweep position of this step
};

// Runs that share a grid shape: the class's own plan holds the shared
// tables (band operators, transform maps, twiddles); batches of it gather
// states and run parameters through pointer tables.
struct Class {
  std::unique_ptr<GridPlan> plan;
  rbc::Work w;
  int wcap = 0;
  const double** hx = nullptr;        // pinned host tables, tcap entries
  const rbc::RunDev** hr = nullptr;
  const double** dx = nullptr;        // device tables
  const rbc::RunDev** dr = nullptr;
  size_t tcap = 0, tused = 0;         // entries used in the current step
};

std::string shape_key(const GridPlan& g, char role) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%c:%dx%d:L%.17g,%.17g:s%d:m%d:MT%d:sp%d:bc%d:%.17g,%.17g", role, g.Nx, g.Nz,
                g.Lx, g.Lz, g.scheme, g.mixed ? 1 : 0, g.MT, g.split ? 1 : 0, g.flux ? 1 : 0, g.T_bot, g.T_top);
  return buf;
}

void free_run_buffers(Run& r) {
  for (void* q : {(void*)r.U, (void*)r.F, (void*)r.G, (void*)r.Xc, (void*)r.part, (void*)r.dscal})
    if (q) (void)hipFree(q);
  r.U = r.F = r.G = r.Xc = r.part = r.dscal = nullptr;
  if (r.fine.d_tables) (void)hipFree(r.fine.d_tables);
  if (r.coarse.d_tables) (void)hipFree(r.coarse.d_tables);
  r.fine.d_tables = r.coarse.d_tables = nullptr;
}

size_t run_buffer_bytes(const rbc_params* p, const GridPlan& f, const GridPlan& c) {
  const size_t S = p->n_slices, fs = size_t(4) * f.Mx * f.Nz, cs = size_t(4) * c.Mx * c.Nz;
  return ((2 * S + 1) * fs + (S + 1) * cs + (S + 1) * rbc::kCombineBlocks * 2 + 8) * 8;
}

}  // namespace

struct rbc_ensemble_s {
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<std::unique_ptr<Run>> runs;
  std::map<std::string, Class> classes;
  double* pin = nullptr;        // pinned: defect readback, 2 per run
  size_t pin_cap = 0;
  std::string err;
};

namespace {

rbc_status efail(rbc_ensemble e, rbc_status s, const std::string& m) {
  if (e) e->err = m;
  return s;
}

#define EHIP(e, call)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return efail((e), RBC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The class of a run's fine or coarse grid, created from that run's
// parameters when it is the first of its shape.
rbc_status get_class(rbc_ensemble e, const std::string& key, const rbc_params* p, bool coarse, Class** out) {
  auto it = e->classes.find(key);
  if (it == e->classes.end()) {
    Class c;
    c.plan = std::make_unique<GridPlan>();
    GridPlan other;
    int nf, nc;
    std::string s = rbc::make_run_plans(p, coarse ? other : *c.plan, coarse ? *c.plan : other, &nf, &nc);
    if (other.d_tables) (void)hipFree(other.d_tables);
    if (!s.empty()) {
      if (c.plan->d_tables) (void)hipFree(c.plan->d_tables);
      return efail(e, RBC_ERR_STATE, s);
    }
    // batches of many runs: spread over every XCD, default wave priority
    c.plan->one_xcd = false;
    c.plan->dev.one_xcd = 0;
    c.plan->urgent = false;
    c.plan->dev.urgent = 0;
    it = e->classes.emplace(key, std::move(c)).first;
  }
  *out = &it->second;
  return RBC_OK;
}

// Makes room for n batch entries in the class's work arrays and for `t`
// more pointer-table entries in this step.
rbc_status reserve(rbc_ensemble e, Class& c, int n, size_t t) {
  if (n > c.wcap) {
    EHIP(e, hipStreamSynchronize(e->stream));
    rbc::free_work(c.w);
    const int cap = std::max(n, c.wcap + c.wcap / 2);
    EHIP(e, rbc::alloc_work(*c.plan, cap, c.w));
    c.wcap = cap;
  }
  if (c.tused + t > c.tcap) {
    // tables are only grown at the start of a step (the stream has drained)
    if (c.tused > 0) return efail(e, RBC_ERR_STATE, "pointer tables grown within a step");
    EHIP(e, hipStreamSynchronize(e->stream));
    if (c.hx) (void)hipHostFree(c.hx);
    if (c.hr) (void)hipHostFree(c.hr);
    if (c.dx) (void)hipFree(c.dx);
    if (c.dr) (void)hipFree(c.dr);
    c.hx = nullptr;
    c.hr = nullptr;
    c.dx = nullptr;
    c.dr = nullptr;
    const size_t cap = std::max(t, 2 * c.tcap);
    EHIP(e, hipHostMalloc((void**)&c.hx, cap * sizeof(void*), hipHostMallocDefault));
    EHIP(e, hipHostMalloc((void**)&c.hr, cap * sizeof(void*), hipHostMallocDefault));
    EHIP(e, hipMalloc((void**)&c.dx, cap * sizeof(void*)));
    EHIP(e, hipMalloc((void**)&c.dr, cap * sizeof(void*)));
    c.tcap = cap;
  }
  return RBC_OK;
}

// One gathered batch of `items` (state, run parameters, steps), ordered by
// steps, most first: the launches step the prefix still running.
struct Item {
  double* x;
  const rbc::RunDev* r;
  int steps;
};

rbc_status run_batch(rbc_ensemble e, Class& c, std::vector<Item>& items) {
  if (items.empty()) return RBC_OK;
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.steps > b.steps; });
  const int n = int(items.size());
  rbc_status s = reserve(e, c, n, items.size());
  if (s != RBC_OK) return s;
  const size_t off = c.tused;
  for (int i = 0; i < n; ++i) {
    c.hx[off + i] = items[i].x;
    c.hr[off + i] = items[i].r;
  }
  EHIP(e, hipMemcpyAsync(c.dx + off, c.hx + off, n * sizeof(void*), hipMemcpyHostToDevice, e->stream));
  EHIP(e, hipMemcpyAsync(c.dr + off, c.hr + off, n * sizeof(void*), hipMemcpyHostToDevice, e->stream));
  c.tused += n;
  GridPlan& g = *c.plan;
  g.dev.xptrs = c.dx + off;
  g.dev.rptrs = c.dr + off;
  // steps [t0, t1) in which the same prefix steps
  int t0 = 0;
  int cnt = n;
  hipError_t he = hipSuccess;
  while (cnt > 0 && he == hipSuccess) {
    const int t1 = items[cnt - 1].steps;
    rbc::StepRange r;
    r.slot0 = 0;
    r.count = cnt;
    r.step0 = t0;
    r.step1 = t1;
    r.n_total = INT_MAX;   // every step ends with the next step's transform
    if (t1 > t0) he = rbc::launch_step_range(g, c.w, nullptr, r, nullptr, 0, 0, e->stream, nullptr);
    t0 = t1;
    while (cnt > 0 && items[cnt - 1].steps <= t0) --cnt;
  }
  g.dev.xptrs = nullptr;
  g.dev.rptrs = nullptr;
  if (he != hipSuccess) return efail(e, RBC_ERR_HIP, std::string("batched steps: ") + hipGetErrorString(he));
  return RBC_OK;
}

rbc_status step(rbc_ensemble e, int* n_active) {
  std::vector<Run*> act;
  for (auto& r : e->runs)
    if (r && r->state == kActive) act.push_back(r.get());
  for (auto& kv : e->classes) kv.second.tused = 0;
  if (act.empty()) {
    *n_active = 0;
    return RBC_OK;
  }
  // pointer-table entries of this step per class (tables only grow here)
  {
    std::map<std::string, size_t> need;
    for (Run* r : act) {
      if (r->k >= 0) need[r->fkey] += size_t(r->S - r->k);
      need[r->ckey] += size_t(r->S - (r->k < 0 ? 0 : r->k + 1));
    }
    for (auto& kv : need) {
      rbc_status s = reserve(e, e->classes.at(kv.first), 0, kv.second);
      if (s != RBC_OK) return s;
    }
  }
  // fine runs of the next iteration: slices k..S-1 of every predicted run
  std::map<std::string, std::vector<Item>> fine;
  for (Run* r : act) {
    if (r->k < 0) continue;
    const size_t fs = r->fine.dev.state;
    const int na = r->S - r->k;
    EHIP(e, hipMemcpyAsync(r->F + r->k * fs, r->U + r->k * fs, size_t(na) * fs * 8, hipMemcpyDeviceToDevice,
                           e->stream));
    for (int n = r->k; n < r->S; ++n) fine[r->fkey].push_back({r->F + n * fs, r->fine.dev.run0, r->nf});
  }
  for (auto& kv : fine) {
    rbc_status s = run_batch(e, e->classes.at(kv.first), kv.second);
    if (s != RBC_OK) return s;
  }
  // the sweeps in lock step: prediction (positions 0..S-1) for new runs;
  // U_(k+1) = F(U_k^k) and positions k+1..S-1 for the others
  int jmax = 0;
  for (Run* r : act) {
    if (r->k < 0) {
      r->first = 0;
    } else {
      const int K = r->k + 1;
      EHIP(e, rbc::launch_combine(r->fine, r->coarse, 2, r->U + size_t(K) * r->fine.dev.state,
                                  r->F + size_t(K - 1) * r->fine.dev.state, nullptr, nullptr,
                                  r->part + size_t(K) * rbc::kCombineBlocks * 2, e->stream));
      r->first = K;
    }
    jmax = std::max(jmax, r->S - r->first);
  }
  for (int j = 0; j < jmax; ++j) {
    std::map<std::string, std::vector<Item>> crs;
    for (Run* r : act) {
      const int n = r->first + j;
      if (n >= r->S) continue;
      EHIP(e, rbc::launch_restrict(r->fine, r->coarse, r->U + size_t(n) * r->fine.dev.state, r->Xc, e->stream));
      crs[r->ckey].push_back({r->Xc, r->coarse.dev.run0, r->nc});
    }
    for (auto& kv : crs) {
      rbc_status s = run_batch(e, e->classes.at(kv.first), kv.second);
      if (s != RBC_OK) return s;
    }
    for (Run* r : act) {
      const int n = r->first + j;
      if (n >= r->S) continue;
      const int mode = r->k < 0 ? 0 : 1;
      const size_t fs = r->fine.dev.state, cs = r->coarse.dev.state;
      EHIP(e, rbc::launch_combine(r->fine, r->coarse, mode, r->U + size_t(n + 1) * fs,
                                  mode == 1 ? r->F + size_t(n) * fs : nullptr, r->Xc, r->G + size_t(n) * cs,
                                  r->part + size_t(n + 1) * rbc::kCombineBlocks * 2, e->stream));
    }
  }
  // defects (section 3.7) of the corrected runs, read in one synchronisation
  if (e->pin_cap < 2 * act.size()) {
    EHIP(e, hipStreamSynchronize(e->stream));
    if (e->pin) (void)hipHostFree(e->pin);
    e->pin = nullptr;
    EHIP(e, hipHostMalloc((void**)&e->pin, 2 * act.size() * 2 * sizeof(double), hipHostMallocDefault));
    e->pin_cap = 2 * act.size() * 2;
  }
  for (size_t i = 0; i < act.size(); ++i) {
    Run* r = act[i];
    if (r->k < 0) continue;
    EHIP(e, rbc::launch_defect(r->part, r->k + 1, r->S + 1, r->dscal, e->stream));
    EHIP(e, hipMemcpyAsync(e->pin + 2 * i, r->dscal, 16, hipMemcpyDeviceToHost, e->stream));
  }
  EHIP(e, hipStreamSynchronize(e->stream));
  int left = 0;
  for (size_t i = 0; i < act.size(); ++i) {
    Run* r = act[i];
    if (r->k < 0) {
      r->k = 0;
      if (r->k_max == 0) {
        r->state = kDone;
        r->stop = RBC_STOP_KMAX;
      }
    } else {
      ++r->k;
      const double d = e->pin[2 * i];
      r->defects.push_back(d);
      if (e->pin[2 * i + 1] != 0.0) {
        r->state = kFailed;
      } else if (d <= r->tol) {
        r->state = kDone;
        r->stop = RBC_STOP_DEFECT;
      } else if (r->k >= r->S) {
        r->state = kDone;
        r->stop = RBC_STOP_EXACT;
      } else if (r->k >= r->k_max) {
        r->state = kDone;
        r->stop = RBC_STOP_KMAX;
      }
    }
    if (r->state == kActive) ++left;
  }
  *n_active = left;
  return RBC_OK;
}

Run* get_run(rbc_ensemble e, int32_t id) {
  if (!e || id < 0 || id >= int32_t(e->runs.size()) || !e->runs[id]) return nullptr;
  return e->runs[id].get();
}

}  // namespace

extern "C" {

rbc_status rbc_ensemble_create(void* hip_stream, rbc_ensemble* out) {
  if (!out) return RBC_ERR_ARG;
  *out = nullptr;
  rbc_ensemble e = new (std::nothrow) rbc_ensemble_s();
  if (!e) return RBC_ERR_OOM;
  e->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&e->device) != hipSuccess) {
    delete e;
    return RBC_ERR_HIP;
  }
  *out = e;
  return RBC_OK;
}

rbc_status rbc_ensemble_destroy(rbc_ensemble e) {
  if (!e) return RBC_ERR_ARG;
  (void)hipStreamSynchronize(e->stream);
  for (auto& r : e->runs)
    if (r) free_run_buffers(*r);
  for (auto& kv : e->classes) {
    Class& c = kv.second;
    rbc::free_work(c.w);
    if (c.plan && c.plan->d_tables) (void)hipFree(c.plan->d_tables);
    if (c.hx) (void)hipHostFree(c.hx);
    if (c.hr) (void)hipHostFree(c.hr);
    if (c.dx) (void)hipFree(c.dx);
    if (c.dr) (void)hipFree(c.dr);
  }
  if (e->pin) (void)hipHostFree(e->pin);
  delete e;
  return RBC_OK;
}

const char* rbc_ensemble_last_error(rbc_ensemble e) { return e ? e->err.c_str() : ""; }

rbc_status rbc_ensemble_footprint(const rbc_params* p, size_t* bytes) {
  if (!p || !bytes) return RBC_ERR_ARG;
  if (!rbc::params_error(p).empty()) return RBC_ERR_ARG;
  GridPlan f, c;
  int nf, nc;
  const size_t tables = rbc::run_plan_bytes(p, &nf, &nc, &f, &c);
  *bytes = tables + run_buffer_bytes(p, f, c) + rbc::work_bytes(f, p->n_slices) + rbc::work_bytes(c, 1);
  return RBC_OK;
}

rbc_status rbc_ensemble_add(rbc_ensemble e, const rbc_params* p, const double* U0, int32_t k_max, double tol,
                            int32_t* run_id) {
  if (!e || !p || !U0 || !run_id || k_max < 0) return efail(e, RBC_ERR_ARG, "bad argument");
  std::string msg = rbc::params_error(p);
  if (!msg.empty()) return efail(e, RBC_ERR_ARG, msg);
  auto run = std::make_unique<Run>();
  Run& r = *run;
  r.p = *p;
  r.S = p->n_slices;
  r.k_max = std::min<int>(k_max, p->n_slices);
  r.tol = tol;
  msg = rbc::make_run_plans(p, r.fine, r.coarse, &r.nf, &r.nc);
  if (!msg.empty()) {
    free_run_buffers(r);
    return efail(e, RBC_ERR_STATE, msg);
  }
  r.fkey = shape_key(r.fine, 'F');
  r.ckey = shape_key(r.coarse, 'C');
  const size_t fs = r.fine.dev.state, cs = r.coarse.dev.state, S = r.S;
  if (hipMalloc((void**)&r.U, (S + 1) * fs * 8) != hipSuccess || hipMalloc((void**)&r.F, S * fs * 8) != hipSuccess ||
      hipMalloc((void**)&r.G, S * cs * 8) != hipSuccess || hipMalloc((void**)&r.Xc, cs * 8) != hipSuccess ||
      hipMalloc((void**)&r.part, (S + 1) * rbc::kCombineBlocks * 2 * 8) != hipSuccess ||
      hipMalloc((void**)&r.dscal, 64) != hipSuccess) {
    free_run_buffers(r);
    return efail(e, RBC_ERR_OOM, "run buffers");
  }
  r.bytes = rbc::plan_device_bytes(r.fine) + rbc::plan_device_bytes(r.coarse) + run_buffer_bytes(p, r.fine, r.coarse);
  Class* c;
  rbc_status s = get_class(e, r.fkey, p, false, &c);
  if (s == RBC_OK) s = get_class(e, r.ckey, p, true, &c);
  if (s != RBC_OK) {
    free_run_buffers(r);
    return s;
  }
  if (hipMemcpyAsync(r.U, U0, fs * 8, hipMemcpyDeviceToDevice, e->stream) != hipSuccess) {
    free_run_buffers(r);
    return efail(e, RBC_ERR_HIP, "initial state copy");
  }
  *run_id = int32_t(e->runs.size());
  e->runs.push_back(std::move(run));
  return RBC_OK;
}

rbc_status rbc_ensemble_step(rbc_ensemble e, int32_t* n_active) {
  if (!e || !n_active) return efail(e, RBC_ERR_ARG, "bad argument");
  return step(e, n_active);
}

rbc_status rbc_ensemble_run_info(rbc_ensemble e, int32_t id, int32_t* state, int32_t* k_done, int32_t* stop,
                                 double* defect_hist, int32_t hist_len) {
  Run* r = get_run(e, id);
  if (!r || !state || !k_done) return efail(e, RBC_ERR_ARG, "bad run id or argument");
  *state = r->state;
  *k_done = std::max(r->k, 0);
  if (stop) *stop = r->stop;
  if (defect_hist)
    for (int i = 0; i < hist_len && i < int(r->defects.size()); ++i) defect_hist[i] = r->defects[i];
  return RBC_OK;
}

rbc_status rbc_ensemble_result(rbc_ensemble e, int32_t id, double* U_dev) {
  Run* r = get_run(e, id);
  if (!r || !U_dev || r->state == kReleased) return efail(e, RBC_ERR_ARG, "bad run id or argument");
  EHIP(e, hipMemcpyAsync(U_dev, r->U, size_t(r->S + 1) * r->fine.dev.state * 8, hipMemcpyDeviceToDevice,
                         e->stream));
  return RBC_OK;
}

rbc_status rbc_ensemble_release(rbc_ensemble e, int32_t id) {
  Run* r = get_run(e, id);
  if (!r) return efail(e, RBC_ERR_ARG, "bad run id");
  if (r->state == kActive) return efail(e, RBC_ERR_STATE, "run still active");
  EHIP(e, hipStreamSynchronize(e->stream));
  free_run_buffers(*r);
  r->state = kReleased;
  return RBC_OK;
}

rbc_status rbc_ensemble_run_bytes(rbc_ensemble e, int32_t id, size_t* bytes) {
  Run* r = get_run(e, id);
  if (!r || !bytes) return efail(e, RBC_ERR_ARG, "bad run id or argument");
  *bytes = r->bytes;
  return RBC_OK;
}

}  // extern "C"
