// C ABI of librbc (include/rbc.h): handle management, the seeded initial
// state, the fine propagator over a batch of slices and the diagnostics; the
// coarse sweep and the Parareal iteration are in rbc_parareal.cpp.  Every
// arithmetic step runs in the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "rbc_ctx.hpp"

namespace {
thread_local std::string g_create_err;
}  // namespace

namespace rbc {
rbc_status fail(rbc_handle h, rbc_status s, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_create_err = msg;
  return s;
}
}  // namespace rbc

namespace {

using rbc::fail;
#define HIPCHK RBC_HIPCHK

// Tuning table (rbc_tuning_load): measured launch shapes per role (fine or
// coarse plan), precision, grid and batch size.
struct TuneEntry {
  int coarse, mixed, Nx, Nz, slices;
  int MT, split, xrows;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

// The entry for this role, precision and grid whose batch is nearest (in
// ratio) to `slices`, or null.
const TuneEntry* tune_lookup(bool coarse, bool mixed, int Nx, int Nz, int slices) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const TuneEntry* best = nullptr;
  double bd = 0;
  for (const TuneEntry& t : g_tune) {
    if (t.coarse != int(coarse) || t.mixed != int(mixed) || t.Nx != Nx || t.Nz != Nz) continue;
    const double d = std::fabs(std::log(double(std::max(t.slices, 1)) / std::max(slices, 1)));
    if (!best || d < bd) {
      best = &t;
      bd = d;
    }
  }
  return best;
}

int steps_for(double t0, double t1, int S, double dt, double* dt_used) {
  const double dT = (t1 - t0) / S;
  int n = int(std::ceil(dT / dt - 1e-9));
  if (n < 1) n = 1;
  *dt_used = dT / n;
  return n;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

std::string check_params(const rbc_params* p) {
  if (!p) return "params is NULL";
  if (!(p->Ra > 0) || !(p->Pr > 0) || !(p->Lx > 0) || !(p->Lz > 0)) return "Ra, Pr, Lx, Lz must be > 0";
  if (!pow2(p->Nx) || p->Nx < 4 || !pow2(p->Nx_c) || p->Nx_c < 4)
    return "Nx and Nx_c must be powers of two >= 4 (padded grid 3 Nx / 2)";
  if (!pow2(p->Nz) || p->Nz < 8 || p->Nz > 256 || !pow2(p->Nz_c) || p->Nz_c < 8)
    return "Nz and Nz_c must be powers of two in [8, 256]";
  // the x-pass keeps three padded rows of complex values in LDS
  if (p->Nx > 2048) return "Nx must be <= 2048";
  if (p->Nx_c > p->Nx || p->Nz_c > p->Nz) return "coarse grid must not exceed the fine grid";
  if (p->n_slices < 1) return "n_slices must be >= 1";
  if (!(p->t_end > p->t0)) return "t_end must exceed t0";
  if (!(p->dt_f > 0) || !(p->dt_c > 0)) return "dt_f, dt_c must be > 0";
  for (int s : {p->scheme_f, p->scheme_c})
    if (s != RBC_ARS222 && s != RBC_ARS443) return "scheme must be RBC_ARS222 or RBC_ARS443";
  if (p->precision != RBC_FP64 && p->precision != RBC_MIXED) return "precision must be RBC_FP64 or RBC_MIXED";
  if (p->nu_stride < 0) return "nu_stride must be >= 0";
  if (!(p->stat_tol >= 0)) return "stat_tol must be >= 0";
  if (p->bc_T != RBC_BC_TEMPERATURE && p->bc_T != RBC_BC_FLUX) return "bc_T must be RBC_BC_TEMPERATURE or RBC_BC_FLUX";
  return "";
}

void setup_grid(rbc::GridPlan& g, const rbc_params* p, bool coarse, double dt) {
  g.Nx = coarse ? p->Nx_c : p->Nx;
  g.Nz = coarse ? p->Nz_c : p->Nz;
  g.Mx = g.Nx / 2;
  g.Px = 3 * g.Nx / 2;
  g.Pz = 3 * g.Nz / 2;
  g.n = g.Nz / 2;
  g.Ra = p->Ra; g.Pr = p->Pr; g.Lx = p->Lx; g.Lz = p->Lz;
  g.dt = dt;
  g.T_bot = p->T_bot; g.T_top = p->T_top;
  g.flux = (p->bc_T == RBC_BC_FLUX);
  g.scheme = coarse ? p->scheme_c : p->scheme_f;
  g.mixed = (p->precision == RBC_MIXED);
  // The coarse sweep is serial and runs beside the batched fine launches on
  // the same compute units: its waves take the SIMD issue slots first, and
  // the launches of a mixed coarse plan stay on one XCD, so that what one
  // launch writes and the next reads (and the grid's tables) stay in that
  // XCD's L2.  (FP64 coarse blocks beside FP64 fine blocks lose more to the
  // fewer compute units than they gain.)  RBC_COARSE_PRIO=0 and
  // RBC_COARSE_ONE_XCD=0 turn these off (for measurement).
  g.urgent = coarse;
  if (const char* e = std::getenv("RBC_COARSE_PRIO")) g.urgent = coarse && std::atoi(e) != 0;
  g.one_xcd = coarse && g.mixed;
  if (const char* e = std::getenv("RBC_COARSE_ONE_XCD")) g.one_xcd = g.one_xcd && std::atoi(e) != 0;
  // modes per block of the per-mode kernel (2, 4, 6 or 8); RBC_MODE_TILE overrides
  // (the single-slice coarse grid and single-run fine batches are latency-bound:
  // small tiles, more blocks)
  g.MT = (coarse || g.Nz >= 128 || p->n_slices <= 2) ? 2 : 4;
  // split path (the Chebyshev transforms as FP32 MFMA GEMMs over the whole
  // batch): by rule for mixed-precision fine grids with Nz >= 128
  const bool split_grid = g.mixed && !coarse && g.Nz >= 64 && g.Mx % 64 == 0;
  g.split = split_grid && g.Nz >= 128 && g.MT <= 4;
  g.xrows = 0;
  // a measured choice for this role, precision, grid and batch (rbc_tuning_load)
  // (an entry with MT = 0 was measured and keeps the rules)
  const TuneEntry* t = tune_lookup(coarse, g.mixed, g.Nx, g.Nz, coarse ? 1 : p->n_slices);
  if (t && t->MT != 0) {
    g.MT = t->MT;
    g.split = split_grid && t->split && t->MT <= 4;
    g.xrows = t->xrows;
  }
  // measurement overrides: RBC_MODE_TILE, RBC_SPLIT, RBC_XPASS_ROWS
  if (const char* e = std::getenv("RBC_MODE_TILE")) {
    const int v = std::atoi(e);
    if (v == 2 || v == 4 || v == 6 || v == 8) g.MT = v;
  }
  if (const char* e = std::getenv("RBC_SPLIT")) g.split = split_grid && std::atoi(e) != 0;
  if (const char* e = std::getenv("RBC_XPASS_ROWS")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) g.xrows = v;
  }
  if (g.MT > g.Mx) g.MT = g.Mx;   // Mx is a power of two >= 2
  // keep the per-mode kernel's LDS (two FP64 tiles + staged factors) < 150 KiB
  const size_t rb = g.mixed ? 4 : 8;
  auto lds = [&](int mt) {
    const size_t y = size_t(8) * 4 * mt * (g.Nz + 1);
    const size_t n = rb * (4 * size_t(g.Pz) * mt + g.Pz);
    const size_t f = size_t(8) * mt * 2 * ((rbc::kFacP * (g.Nz / 2 - 2) + 4) | 1);
    const size_t u = n > f ? n : f, v = (mt <= 2) ? rb * size_t(g.Pz) * mt * 12 : 0;
    return y + (y + u > v ? y + u : v);
  };
  while (g.MT > 2 && lds(g.MT) > 150 * 1024) g.MT = (g.MT == 6) ? 4 : g.MT / 2;
  if (g.MT > 4) g.split = false;   // the split path's per-mode kernel takes tiles of 2 or 4
}

size_t pararea_bytes(const rbc_params* p, const rbc::GridPlan& f, const rbc::GridPlan& c, int nsf, int nsc) {
  const size_t S = p->n_slices;
  size_t b = 0;
  b += size_t(4) * c.Mx * c.Nz * 8;                 // Xc
  b += S * 4 * f.Mx * f.Nz * 8;                     // F
  b += (S + 2) * 4 * f.Mx * f.Nz * 8 + (S + 2) * 16; // state ring, slot records
  b += S * 4 * c.Mx * c.Nz * 8;                     // G
  b += (S + 1) * rbc::kCombineBlocks * 2 * 8 + 64;  // partials, scalars
  b += 2 * S * size_t(nsf) * rbc::kDiag * 8 + S * size_t(nsc) * rbc::kDiag * 8;
  return b;
}

void release(rbc_handle h) {
  if (!h) return;
  for (hipEvent_t e : h->timing.ev) (void)hipEventDestroy(e);
  h->timing.ev.clear();
  for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
  h->evpool.clear();
  if (h->cgraph) (void)hipGraphExecDestroy(h->cgraph);
  if (h->cgraph64) (void)hipGraphExecDestroy(h->cgraph64);
  if (h->fstream) (void)hipStreamDestroy(h->fstream);
  if (h->gstream) (void)hipStreamDestroy(h->gstream);
  if (h->f64stream) (void)hipStreamDestroy(h->f64stream);
  if (h->host_pin) (void)hipHostFree(h->host_pin);
  rbc::free_work(h->wf);
  rbc::free_work(h->wc);
  rbc::free_work(h->wf64);
  rbc::free_work(h->wc64);
  if (h->fine64.d_tables) (void)hipFree(h->fine64.d_tables);
  if (h->coarse64.d_tables) (void)hipFree(h->coarse64.d_tables);
  for (void* q : {(void*)h->Xc, (void*)h->Fbuf, (void*)h->Xring, (void*)h->meta, (void*)h->Gbuf, (void*)h->part,
                  (void*)h->dscal,
                  (void*)h->nu_f, (void*)h->nu_c, h->fine.d_tables, h->coarse.d_tables})
    if (q) (void)hipFree(q);
}

// Sample counts and the coarse sampling stride.
void sampling(const rbc_params* p, int nf, int nc, double dtf, double dtc, int* nsf, int* nsc, int* sc) {
  if (p->nu_stride <= 0) {
    *nsf = *nsc = *sc = 0;
    return;
  }
  *nsf = nf / p->nu_stride;
  int s = int(std::lround(p->nu_stride * dtf / dtc));
  if (s < 1) s = 1;
  *sc = s;
  *nsc = nc / s;
}

}  // namespace

// The seeded initial state of grid g into host memory U (one fine state).
static void initial_state_host(const rbc::GridPlan& g, uint64_t seed, double amp, std::vector<double>& U_out) {
  const int Nx = g.Nx, Nz = g.Nz, Mx = g.Mx;
  // seeded noise: SplitMix64 outputs 2p, 2p+1 -> Box-Muller (cosine branch)
  auto mix = [seed](uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto unif = [&](uint64_t c) { return double(mix(c) >> 11) * (1.0 / 9007199254740992.0); };
  std::vector<double> Tg(size_t(Nx) * Nz), zj(Nz);
  for (int j = 0; j < Nz; ++j) zj[j] = (std::cos(M_PI * (j + 0.5) / Nz) + 1.0) * 0.5;   // z / Lz
  for (int ix = 0; ix < Nx; ++ix)
    for (int iz = 0; iz < Nz; ++iz) {
      const uint64_t pidx = uint64_t(ix) * Nz + iz;
      const double u1 = unif(2 * pidx), u2 = unif(2 * pidx + 1);
      const double xi = std::sqrt(-2.0 * std::log(1.0 - u1)) * std::cos(2.0 * M_PI * u2);
      const double z = zj[iz];
      const double base = g.flux ? g.T_bot - z * g.Lz : g.T_bot + (g.T_top - g.T_bot) * z;
      Tg[size_t(ix) * Nz + iz] = base + amp * xi * z * (1.0 - z);
    }
  // Fourier in x (modes m < Mx, 1/Nx normalisation), Chebyshev in z
  std::vector<double> cs(Nx), sn(Nx);
  for (int t = 0; t < Nx; ++t) {
    cs[t] = std::cos(2.0 * M_PI * t / Nx);
    sn[t] = std::sin(2.0 * M_PI * t / Nx);
  }
  std::vector<double> U(size_t(4) * Mx * Nz, 0.0), fr(Nz), fi(Nz);
  std::vector<double> Tc(size_t(Nz) * Nz);
  for (int n = 0; n < Nz; ++n)
    for (int j = 0; j < Nz; ++j) Tc[size_t(n) * Nz + j] = (n == 0 ? 1.0 : 2.0) / Nz * std::cos(n * M_PI * (j + 0.5) / Nz);
  for (int m = 0; m < Mx; ++m) {
    for (int j = 0; j < Nz; ++j) {
      double ar = 0, ai = 0;
      for (int ix = 0; ix < Nx; ++ix) {
        const int t = int((int64_t(m) * ix) % Nx);
        ar += Tg[size_t(ix) * Nz + j] * cs[t];
        ai -= Tg[size_t(ix) * Nz + j] * sn[t];
      }
      fr[j] = ar / Nx;
      fi[j] = (m == 0) ? 0.0 : ai / Nx;
    }
    for (int n = 0; n < Nz; ++n) {
      double cr = 0, ci = 0;
      for (int j = 0; j < Nz; ++j) {
        cr += Tc[size_t(n) * Nz + j] * fr[j];
        ci += Tc[size_t(n) * Nz + j] * fi[j];
      }
      U[((size_t(1) * Mx + m) * 2 + 0) * Nz + n] = cr;
      U[((size_t(1) * Mx + m) * 2 + 1) * Nz + n] = ci;
    }
  }
  U_out.swap(U);
}

namespace rbc {

// The fine and coarse plans of one run, built and uploaded as rbc_create
// builds them (without the FP64 promotion plans); returns "" or the error.
std::string make_run_plans(const rbc_params* p, GridPlan& fine, GridPlan& coarse, int* nf, int* nc) {
  std::string e = check_params(p);
  if (!e.empty()) return e;
  double dtf, dtc;
  *nf = steps_for(p->t0, p->t_end, p->n_slices, p->dt_f, &dtf);
  *nc = steps_for(p->t0, p->t_end, p->n_slices, p->dt_c, &dtc);
  setup_grid(fine, p, false, dtf);
  setup_grid(coarse, p, true, dtc);
  e = build_plan(fine);
  if (e.empty()) e = build_plan(coarse);
  if (!e.empty()) return e;
  hipError_t he;
  if ((he = upload_plan(fine)) != hipSuccess || (he = upload_plan(coarse)) != hipSuccess)
    return std::string("table upload: ") + hipGetErrorString(he);
  return "";
}

size_t run_plan_bytes(const rbc_params* p, int* nf, int* nc, GridPlan* fine_shape, GridPlan* coarse_shape) {
  double dtf, dtc;
  *nf = steps_for(p->t0, p->t_end, p->n_slices, p->dt_f, &dtf);
  *nc = steps_for(p->t0, p->t_end, p->n_slices, p->dt_c, &dtc);
  setup_grid(*fine_shape, p, false, dtf);
  setup_grid(*coarse_shape, p, true, dtc);
  fine_shape->tab = make_tableau(fine_shape->scheme);
  coarse_shape->tab = make_tableau(coarse_shape->scheme);
  auto tables = [](const GridPlan& g) {
    size_t n = g.Nz / 2, rb = g.mixed ? 4 : 8;
    size_t d = 2 * n * 14 + size_t(g.Mx) * 2 * (kFacT * n + 4) + size_t(g.Mx) * 2 * (kFacP * n + 4);
    size_t r = size_t(4) * (g.Pz / 2) * g.Nz + size_t(3) * g.Nz * (g.Pz / 2) + 2 * size_t(g.Px);
    if (g.split) r += size_t(4) * (g.Pz / 2) * g.Nz + size_t(2) * g.Nz * (g.Pz / 2);
    return d * 8 + r * rb + 16 * 256 + sizeof(RunDev);
  };
  return tables(*fine_shape) + tables(*coarse_shape);
}

std::string params_error(const rbc_params* p) { return check_params(p); }

}  // namespace rbc

extern "C" {

rbc_status rbc_default_params(rbc_params* p) {
  if (!p) return RBC_ERR_ARG;
  std::memset(p, 0, sizeof(*p));
  p->Ra = 1e4; p->Pr = 1; p->Lx = 2; p->Lz = 1;
  p->Nx = 64; p->Nz = 32; p->Nx_c = 64; p->Nz_c = 32;
  p->t0 = 0; p->t_end = 1; p->n_slices = 1;
  p->dt_f = 1e-3; p->dt_c = 1e-2;
  p->scheme_f = RBC_ARS443; p->scheme_c = RBC_ARS443;
  p->precision = RBC_FP64;
  p->nu_stride = 0; p->nu_t_start = 0;
  p->T_bot = 1; p->T_top = 0;
  p->promote_fp64 = 1;
  p->pipelined = 1;
  p->stat_tol = 0;
  return RBC_OK;
}

rbc_status rbc_tuning_load(const char* path) {
  std::vector<TuneEntry> tab;
  if (path) {
    std::ifstream in(path);
    if (!in) return fail(nullptr, RBC_ERR_ARG, std::string("cannot open tuning table ") + path);
    std::string line;
    int ln = 0;
    while (std::getline(in, line)) {
      ++ln;
      const size_t hash = line.find('#');
      if (hash != std::string::npos) line.resize(hash);
      std::istringstream ss(line);
      std::string role, prec;
      TuneEntry t{};
      if (!(ss >> role)) continue;
      if (!(ss >> prec >> t.Nx >> t.Nz >> t.slices >> t.MT >> t.split >> t.xrows) ||
          (role != "fine" && role != "coarse") || (prec != "mixed" && prec != "fp64") ||
          (t.MT != 0 && t.MT != 2 && t.MT != 4 && t.MT != 6 && t.MT != 8) ||
          (t.xrows != 0 && t.xrows != 1 && t.xrows != 2 && t.xrows != 4) || (t.MT == 0 && (t.split || t.xrows)))
        return fail(nullptr, RBC_ERR_ARG, std::string(path) + ":" + std::to_string(ln) + ": bad tuning entry");
      t.coarse = role == "coarse";
      t.mixed = prec == "mixed";
      tab.push_back(t);
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.swap(tab);
  return RBC_OK;
}

rbc_status rbc_tuning_entries(int32_t* n) {
  if (!n) return RBC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  *n = int32_t(g_tune.size());
  return RBC_OK;
}

rbc_status rbc_query_footprint(const rbc_params* p, size_t* device_bytes) {
  std::string e = check_params(p);
  if (!e.empty()) return fail(nullptr, RBC_ERR_ARG, e);
  if (!device_bytes) return fail(nullptr, RBC_ERR_ARG, "device_bytes is NULL");
  rbc::GridPlan f, c;
  double dtf, dtc;
  int nf = steps_for(p->t0, p->t_end, p->n_slices, p->dt_f, &dtf);
  int nc = steps_for(p->t0, p->t_end, p->n_slices, p->dt_c, &dtc);
  setup_grid(f, p, false, dtf);
  setup_grid(c, p, true, dtc);
  f.tab = rbc::make_tableau(f.scheme);
  c.tab = rbc::make_tableau(c.scheme);
  // plan sizes without building the factorisations
  auto tables = [](const rbc::GridPlan& g) {
    size_t n = g.Nz / 2, rb = g.mixed ? 4 : 8;
    size_t d = 2 * n * 14 + size_t(g.Mx) * 2 * (rbc::kFacT * n + 4) + size_t(g.Mx) * 2 * (rbc::kFacP * n + 4);
    size_t r = size_t(4) * (g.Pz / 2) * g.Nz + size_t(3) * g.Nz * (g.Pz / 2) + 2 * size_t(g.Px);
    if (g.split) r += size_t(4) * (g.Pz / 2) * g.Nz + size_t(2) * g.Nz * (g.Pz / 2);   // maps by parity
    return d * 8 + r * rb + 16 * 256;
  };
  int nsf, nsc, sc;
  sampling(p, nf, nc, dtf, dtc, &nsf, &nsc, &sc);
  const int cap = p->n_slices + 2;
  *device_bytes = tables(f) + tables(c) + rbc::work_bytes(f, cap) + rbc::work_bytes(c, 1) +
                  pararea_bytes(p, f, c, nsf, nsc);
  if (p->precision == RBC_MIXED && p->promote_fp64) {
    rbc::GridPlan f64 = f, c64 = c;
    f64.mixed = c64.mixed = false;
    f64.split = c64.split = false;
    *device_bytes += tables(f64) + rbc::work_bytes(f64, cap) + tables(c64) + rbc::work_bytes(c64, 1);
  }
  return RBC_OK;
}

rbc_status rbc_create(const rbc_params* p, void* hip_stream, rbc_handle* out) {
  if (!out) return fail(nullptr, RBC_ERR_ARG, "out is NULL");
  *out = nullptr;
  std::string e = check_params(p);
  if (!e.empty()) return fail(nullptr, RBC_ERR_ARG, e);
  rbc_handle h = new (std::nothrow) rbc_ctx();
  if (!h) return fail(nullptr, RBC_ERR_OOM, "host allocation failed");
  h->p = *p;
  h->stream = static_cast<hipStream_t>(hip_stream);
  double dtf, dtc;
  h->nf = steps_for(p->t0, p->t_end, p->n_slices, p->dt_f, &dtf);
  h->nc = steps_for(p->t0, p->t_end, p->n_slices, p->dt_c, &dtc);
  setup_grid(h->fine, p, false, dtf);
  setup_grid(h->coarse, p, true, dtc);
  e = rbc::build_plan(h->fine);
  if (e.empty()) e = rbc::build_plan(h->coarse);
  h->has64 = (p->precision == RBC_MIXED && p->promote_fp64 != 0);
  if (e.empty() && h->has64) {
    setup_grid(h->fine64, p, false, dtf);
    setup_grid(h->coarse64, p, true, dtc);
    h->fine64.mixed = h->coarse64.mixed = false;
    h->fine64.split = h->coarse64.split = false;
    h->coarse64.one_xcd = false;
    e = rbc::build_plan(h->fine64);
    if (e.empty()) e = rbc::build_plan(h->coarse64);
  }
  if (!e.empty()) {
    delete h;
    return fail(nullptr, RBC_ERR_STATE, e);
  }
  sampling(p, h->nf, h->nc, dtf, dtc, &h->nsf, &h->nsc, &h->stride_c);
  hipError_t he = hipGetDevice(&h->device);
  auto bail = [&](rbc_status st, const std::string& m) {
    release(h);
    delete h;
    return fail(nullptr, st, m);
  };
  if (he != hipSuccess) return bail(RBC_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
  // the allocation-free entry points' scratch on this device (once per device)
  if ((he = rbc::scratch_init(h->device)) != hipSuccess)
    return bail(RBC_ERR_HIP, std::string("device scratch address: ") + hipGetErrorString(he));
  if ((he = rbc::upload_plan(h->fine)) != hipSuccess || (he = rbc::upload_plan(h->coarse)) != hipSuccess ||
      (h->has64 && ((he = rbc::upload_plan(h->fine64)) != hipSuccess ||
                    (he = rbc::upload_plan(h->coarse64)) != hipSuccess)))
    return bail(RBC_ERR_OOM, std::string("table upload: ") + hipGetErrorString(he));
  h->ring_cap = p->n_slices + 2;
  if (h->has64 && ((he = rbc::alloc_work(h->fine64, h->ring_cap, h->wf64)) != hipSuccess ||
                   (he = rbc::alloc_work(h->coarse64, 1, h->wc64)) != hipSuccess))
    return bail(RBC_ERR_OOM, std::string("workspace: ") + hipGetErrorString(he));
  if ((he = rbc::alloc_work(h->fine, h->ring_cap, h->wf)) != hipSuccess ||
      (he = rbc::alloc_work(h->coarse, 1, h->wc)) != hipSuccess)
    return bail(RBC_ERR_OOM, std::string("workspace: ") + hipGetErrorString(he));
  const size_t S = p->n_slices;
  const size_t fs = h->fine.dev.state, cs = h->coarse.dev.state;
  if (hipMalloc((void**)&h->Xc, cs * 8) != hipSuccess || hipMalloc((void**)&h->Fbuf, S * fs * 8) != hipSuccess ||
      hipMalloc((void**)&h->Xring, size_t(h->ring_cap) * fs * 8) != hipSuccess ||
      hipMalloc((void**)&h->meta, size_t(h->ring_cap) * sizeof(rbc::SlotMeta)) != hipSuccess ||
      hipMalloc((void**)&h->Gbuf, S * cs * 8) != hipSuccess ||
      hipMalloc((void**)&h->part, (S + 1) * rbc::kCombineBlocks * 2 * 8) != hipSuccess ||
      hipMalloc((void**)&h->dscal, 64) != hipSuccess)
    return bail(RBC_ERR_OOM, "parareal buffers");
  if (h->nsf > 0 && hipMalloc((void**)&h->nu_f, 2 * S * h->nsf * rbc::kDiag * 8) != hipSuccess)
    return bail(RBC_ERR_OOM, "nu sample buffer");
  if (h->nsc > 0 && hipMalloc((void**)&h->nu_c, S * h->nsc * rbc::kDiag * 8) != hipSuccess)
    return bail(RBC_ERR_OOM, "nu sample buffer");
  if (hipHostMalloc((void**)&h->host_pin, (2 + (2 * S * h->nsf + S * h->nsc) * rbc::kDiag) * 8, hipHostMallocDefault) !=
      hipSuccess)
    return bail(RBC_ERR_OOM, "pinned host buffer");
  // the pipelined iteration's streams (default priority): fine runs, coarse
  // sweep, and with the FP64 switch the FP64 fine runs, which then step
  // beside the mixed runs still in flight instead of after them
  if ((he = hipStreamCreateWithFlags(&h->fstream, hipStreamNonBlocking)) != hipSuccess ||
      (he = hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking)) != hipSuccess ||
      (h->has64 && (he = hipStreamCreateWithFlags(&h->f64stream, hipStreamNonBlocking)) != hipSuccess))
    return bail(RBC_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(he));
  *out = h;
  return RBC_OK;
}

rbc_status rbc_destroy(rbc_handle h) {
  if (!h) return RBC_ERR_ARG;
  (void)hipStreamSynchronize(h->stream);
  release(h);
  delete h;
  return RBC_OK;
}

const char* rbc_last_error(rbc_handle h) { return h ? h->err.c_str() : g_create_err.c_str(); }

rbc_status rbc_state_size(rbc_handle h, int32_t coarse, size_t* n) {
  if (!h || !n) return fail(h, RBC_ERR_ARG, "null argument");
  *n = coarse ? h->coarse.dev.state : h->fine.dev.state;
  return RBC_OK;
}

rbc_status rbc_steps_per_slice(rbc_handle h, int32_t coarse, int32_t* n_steps, double* dt) {
  if (!h || !n_steps || !dt) return fail(h, RBC_ERR_ARG, "null argument");
  *n_steps = coarse ? h->nc : h->nf;
  *dt = coarse ? h->coarse.dt : h->fine.dt;
  return RBC_OK;
}

rbc_status rbc_init_state(rbc_handle h, uint64_t seed, double amp, double* U0) {
  if (!h || !U0) return fail(h, RBC_ERR_ARG, "null argument");
  std::vector<double> U;
  initial_state_host(h->fine, seed, amp, U);
  HIPCHK(h, hipMemcpyAsync(U0, U.data(), U.size() * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RBC_OK;
}

rbc_status rbc_initial_state(const rbc_params* p, uint64_t seed, double amp, double* U0, void* hip_stream) {
  if (!p || !U0) return fail(nullptr, RBC_ERR_ARG, "null argument");
  std::string e = check_params(p);
  if (!e.empty()) return fail(nullptr, RBC_ERR_ARG, e);
  rbc::GridPlan g;
  double dtf;
  steps_for(p->t0, p->t_end, p->n_slices, p->dt_f, &dtf);
  setup_grid(g, p, false, dtf);
  std::vector<double> U;
  initial_state_host(g, seed, amp, U);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipError_t he = hipMemcpyAsync(U0, U.data(), U.size() * 8, hipMemcpyHostToDevice, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return fail(nullptr, RBC_ERR_HIP, std::string("rbc_initial_state: ") + hipGetErrorString(he));
  return RBC_OK;
}

rbc_status rbc_fine_step_batch(rbc_handle h, const double* U_in, double* U_out, int32_t n_slices, int32_t n_steps,
                               double* nu_samples) {
  if (!h || !U_in || !U_out) return fail(h, RBC_ERR_ARG, "null argument");
  if (n_slices < 1 || n_slices > h->p.n_slices) return fail(h, RBC_ERR_ARG, "n_slices out of range");
  if (n_steps < 0) return fail(h, RBC_ERR_ARG, "n_steps < 0");
  const size_t bytes = size_t(n_slices) * h->fine.dev.state * 8;
  if (U_in != U_out) HIPCHK(h, hipMemcpyAsync(U_out, U_in, bytes, hipMemcpyDeviceToDevice, h->stream));
  const int stride = h->p.nu_stride;
  const int ld = (nu_samples && stride > 0) ? n_steps / stride : 0;
  HIPCHK(h, rbc::launch_steps(h->fine, h->wf, U_out, n_slices, n_steps, ld > 0 ? nu_samples : nullptr, stride,
                              ld, h->stream, &h->timing));
  return RBC_OK;
}

// Diagnostic records of n fine states into host memory (batches of at most
// the work buffers' capacity).
static rbc_status diag_states(rbc_handle h, const double* U, int n, double* host, const char* what) {
  double* d = nullptr;
  HIPCHK(h, hipMallocAsync((void**)&d, size_t(n) * rbc::kDiag * 8, h->stream));
  hipError_t e = hipSuccess;
  for (int i0 = 0; i0 < n && e == hipSuccess; i0 += h->wf.cap) {
    const int cnt = std::min(h->wf.cap, n - i0);
    e = rbc::launch_diag(h->fine, h->wf, U + size_t(i0) * h->fine.dev.state, 0, cnt, cnt, d + size_t(i0) * rbc::kDiag,
                         rbc::kDiag, nullptr, 0, 1, 0, 0, h->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(host, d, size_t(n) * rbc::kDiag * 8, hipMemcpyDeviceToHost, h->stream);
  hipError_t e2 = hipFreeAsync(d, h->stream);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, RBC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return RBC_OK;
}

rbc_status rbc_nusselt(rbc_handle h, const double* U, int32_t n, double* nu_host) {
  if (!h || !U || !nu_host || n < 0) return fail(h, RBC_ERR_ARG, "bad argument");
  if (n == 0) return RBC_OK;
  std::vector<double> rec(size_t(n) * rbc::kDiag);
  rbc_status s = diag_states(h, U, n, rec.data(), "rbc_nusselt");
  if (s != RBC_OK) return s;
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) nu_host[size_t(i) * 3 + c] = rec[size_t(i) * rbc::kDiag + c];
  return RBC_OK;
}

rbc_status rbc_diagnostics(rbc_handle h, const double* U, int32_t n, double* out_host) {
  if (!h || !U || !out_host || n < 0) return fail(h, RBC_ERR_ARG, "bad argument");
  if (n == 0) return RBC_OK;
  return diag_states(h, U, n, out_host, "rbc_diagnostics");
}

rbc_status rbc_diagnostics_noalloc(rbc_handle h, const double* U, int32_t n, double* out_dev) {
  if (!h || !U || !out_dev || n < 0) return fail(h, RBC_ERR_ARG, "bad argument");
  if (n == 0) return RBC_OK;
  const size_t per = rbc::diag_partials_per_state(h->fine.dev);
  const size_t cap = rbc::kScratchBytes / sizeof(double) / per;
  if (size_t(n) > cap)
    return fail(h, RBC_ERR_ARG, "rbc_diagnostics_noalloc: " + std::to_string(n) + " states exceed the maximum of " +
                                    std::to_string(cap) + " for this grid (" + std::to_string(rbc::kScratchBytes) +
                                    " bytes of device scratch)");
  double* part = rbc::scratch_ptr(h->device);
  if (!part) return fail(h, RBC_ERR_STATE, "rbc_diagnostics_noalloc: device scratch not set up");
  HIPCHK(h, rbc::launch_diag_into(h->fine, part, U, 0, n, n, out_dev, rbc::kDiag, nullptr, 0, 1, 0, 0, h->stream));
  return RBC_OK;
}

rbc_status rbc_explicit_terms(rbc_handle h, const double* U, double* E) {
  if (!h || !U || !E) return fail(h, RBC_ERR_ARG, "null argument");
  HIPCHK(h, hipMemsetAsync(E, 0, size_t(h->fine.dev.state) * 8, h->stream));
  HIPCHK(h, rbc::launch_explicit(h->fine, h->wf, U, E, h->stream));
  return RBC_OK;
}

rbc_status rbc_kernel_timing_enable(rbc_handle h, int32_t kernel, int32_t every) {
  if (!h) return RBC_ERR_ARG;
  if (kernel < -1 || kernel > 1 || every < 0) return fail(h, RBC_ERR_ARG, "kernel must be -1, 0 or 1; every >= 0");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->timing.kernel = kernel;
  h->timing.every = (kernel < 0) ? 0 : every;
  h->timing.used = 0;
  h->timing.units = 0;
  return RBC_OK;
}

rbc_status rbc_kernel_timing(rbc_handle h, double* mean_ms, int64_t* count, double* mean_batch) {
  if (!h || !mean_ms || !count) return fail(h, RBC_ERR_ARG, "null argument");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double tot = 0;
  int64_t n = 0;
  for (size_t i = 0; i + 1 < h->timing.used; i += 2) {
    float ms = 0;
    HIPCHK(h, hipEventElapsedTime(&ms, h->timing.ev[i], h->timing.ev[i + 1]));
    tot += ms;
    ++n;
  }
  *mean_ms = n ? tot / n : 0.0;
  *count = n;
  if (mean_batch) *mean_batch = n ? h->timing.units / n : 0.0;
  h->timing.used = 0;
  h->timing.units = 0;
  return RBC_OK;
}

rbc_status rbc_synchronize(rbc_handle h) {
  if (!h) return RBC_ERR_ARG;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RBC_OK;
}

}  // extern "C"
