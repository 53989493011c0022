// Host-side construction of the per-grid tables of librbc.
//
// Operators (ultraspherical spectral method, Olver & Townsend 2013) on
// Chebyshev-T coefficient vectors in zeta = 2z/Lz - 1:
//   D_l : T_n -> 2^(l-1) (l-1)! n C^(l)_(n-l)   (times (2/Lz)^l)
//   S_0 : T_0 = C^(1)_0, T_n = (C^(1)_n - C^(1)_(n-2)) / 2
//   S_l : C^(l)_n = l/(n+l) (C^(l+1)_n - C^(l+1)_(n-2))
// Equations per Fourier mode k (section 2.1 in streamfunction form):
//   temperature  M = S1S0,                  L = kappa (D2 - k^2 S1S0)
//   psi (m >= 1) M = S3S2 (D2 - k^2 S1S0),  L = nu (D4 - 2k^2 S3S2D2 + k^4 S3S2S1S0),
//                buoyancy B = -i k S3S2S1S0 on T
//   u_bar (m=0)  M = S1S0,                  L = nu D2
// Every stage of the ARS schemes solves (M - h a_ii L) y = r with the last
// rows replaced by wall conditions.  Split by parity, each system is
//   [ C ]        C: 1 or 2 dense wall rows  (sum of coefficients, sum of n^2 c_n;
//                fixed-flux temperature walls: sum of n^2 c_n alone)
//   [ R ] y = f  R: banded rows, half-column offsets 0..w (w = 2 or 4)
// It is solved by bordering: with the first b unknowns as the border,
// R = [R1 | R2] and R2 square banded (b sub-, w-b super-diagonals),
//   x = R2^-1 f,  V = R2^-1 R1,  y_head = (C1 - C2 V)^-1 (g - C2 x),
//   y_tail = x - V y_head.
// R2 is factored without pivoting; factor_bordered() reports the growth.
#include <cmath>
#include <cstring>
#include <sstream>

#include "rbc_internal.hpp"

namespace rbc {

namespace {

using Mat = std::vector<double>;   // dense row-major N x N

Mat zeros(int N) { return Mat(size_t(N) * N, 0.0); }

Mat matmul(const Mat& A, const Mat& B, int N) {
  Mat C = zeros(N);
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k) {
      double a = A[size_t(i) * N + k];
      if (a == 0.0) continue;
      for (int j = 0; j < N; ++j) C[size_t(i) * N + j] += a * B[size_t(k) * N + j];
    }
  return C;
}

Mat opD(int lam, int N, double scale) {
  Mat A = zeros(N);
  double f = std::pow(2.0, lam - 1);
  for (int t = 2; t < lam; ++t) f *= t;
  f *= std::pow(scale, lam);
  for (int n = lam; n < N; ++n) A[size_t(n - lam) * N + n] = f * n;
  return A;
}

Mat opS0(int N) {
  Mat A = zeros(N);
  A[0] = 1.0;
  for (int n = 1; n < N; ++n) A[size_t(n) * N + n] = 0.5;
  for (int n = 2; n < N; ++n) A[size_t(n - 2) * N + n] = -0.5;
  return A;
}

Mat opS(int lam, int N) {
  Mat A = zeros(N);
  for (int n = 0; n < N; ++n) {
    A[size_t(n) * N + n] = double(lam) / (n + lam);
    if (n >= 2) A[size_t(n - 2) * N + n] = -double(lam) / (n + lam);
  }
  return A;
}

// Chebyshev-T derivative matrix (T basis -> T basis) times scale.
Mat derivT(int N, double scale) {
  Mat A = zeros(N);
  for (int n = 1; n < N; ++n)
    for (int a = n - 1; a >= 0; a -= 2) A[size_t(a) * N + n] = (a == 0 ? 1.0 : 2.0) * n * scale;
  return A;
}

struct Ops {
  int N;
  Mat S10, D2, S32D2, S3210, D4, S1D1;
};

Ops make_ops(int N, double scale) {
  Ops o;
  o.N = N;
  Mat S0 = opS0(N), S1 = opS(1, N), S2 = opS(2, N), S3 = opS(3, N);
  o.S10 = matmul(S1, S0, N);
  Mat S32 = matmul(S3, S2, N);
  o.D2 = opD(2, N, scale);
  o.S32D2 = matmul(S32, o.D2, N);
  o.S3210 = matmul(S32, o.S10, N);
  o.D4 = opD(4, N, scale);
  o.S1D1 = matmul(S1, opD(1, N, scale), N);
  return o;
}

// Bordered, no-pivot banded factorisation of one parity system.
// R: nr x n dense (band rows of parity p in half indices), b border columns,
// ku super-diagonals of R2.  C: b x n wall rows.  Writes kFac* entries per
// row followed by the b x b Schur inverse.  Returns the growth factor.
double factor_bordered(const std::vector<double>& R, int nr, int n, int b, int ku,
                       const std::vector<double>& C, double* out, int per_row, std::string& err) {
  const int m = n - b;  // == nr
  if (m != nr) { err = "internal: band row count"; return 0; }
  std::vector<double> A(size_t(m) * m), R1(size_t(m) * b);
  double amax = 0;
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) {
      A[size_t(i) * m + j] = R[size_t(i) * n + b + j];
      amax = std::fmax(amax, std::fabs(A[size_t(i) * m + j]));
    }
    for (int t = 0; t < b; ++t) R1[size_t(i) * b + t] = R[size_t(i) * n + t];
  }
  // the band: sub-diagonals 1..b, super-diagonals 1..ku
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      if ((j < i - b || j > i + ku) && A[size_t(i) * m + j] != 0.0) {
        err = "internal: entry outside the band";
        return 0;
      }
  std::vector<double> L(size_t(m) * (b + 1), 0.0);
  for (int j = 0; j < m; ++j) {
    double piv = A[size_t(j) * m + j];
    if (piv == 0.0 || !std::isfinite(piv)) { err = "zero pivot in band factorisation"; return 0; }
    for (int i = j + 1; i <= std::min(m - 1, j + b); ++i) {
      double l = A[size_t(i) * m + j] / piv;
      L[size_t(i) * (b + 1) + (i - j)] = l;
      for (int c = j; c <= std::min(m - 1, j + ku); ++c) A[size_t(i) * m + c] -= l * A[size_t(j) * m + c];
      A[size_t(i) * m + j] = 0.0;
    }
  }
  double umax = 0;
  for (int i = 0; i < m; ++i)
    for (int c = i; c <= std::min(m - 1, i + ku); ++c) umax = std::fmax(umax, std::fabs(A[size_t(i) * m + c]));
  // V = R2^-1 R1
  std::vector<double> V(size_t(m) * b);
  for (int t = 0; t < b; ++t) {
    std::vector<double> y(m);
    for (int i = 0; i < m; ++i) {
      double v = R1[size_t(i) * b + t];
      for (int d = 1; d <= b && i - d >= 0; ++d) v -= L[size_t(i) * (b + 1) + d] * y[i - d];
      y[i] = v;
    }
    for (int i = m - 1; i >= 0; --i) {
      double v = y[i];
      for (int d = 1; d <= ku && i + d < m; ++d) v -= A[size_t(i) * m + i + d] * y[i + d];
      y[i] = v / A[size_t(i) * m + i];
    }
    for (int i = 0; i < m; ++i) V[size_t(i) * b + t] = y[i];
  }
  // Schur complement
  double Sc[4] = {0, 0, 0, 0};
  for (int r = 0; r < b; ++r)
    for (int t = 0; t < b; ++t) {
      double v = C[size_t(r) * n + t];
      for (int i = 0; i < m; ++i) v -= C[size_t(r) * n + b + i] * V[size_t(i) * b + t];
      Sc[r * b + t] = v;
    }
  double Si[4];
  if (b == 1) {
    if (Sc[0] == 0.0) { err = "singular wall-condition Schur complement"; return 0; }
    Si[0] = 1.0 / Sc[0];
  } else {
    double det = Sc[0] * Sc[3] - Sc[1] * Sc[2];
    if (det == 0.0 || !std::isfinite(det)) { err = "singular wall-condition Schur complement"; return 0; }
    Si[0] = Sc[3] / det; Si[1] = -Sc[1] / det; Si[2] = -Sc[2] / det; Si[3] = Sc[0] / det;
  }
  for (int i = 0; i < m; ++i) {
    double* o = out + size_t(i) * per_row;
    if (b == 1) {
      o[0] = L[size_t(i) * 2 + 1];
      o[1] = 1.0 / A[size_t(i) * m + i];
      o[2] = (i + 1 < m) ? A[size_t(i) * m + i + 1] : 0.0;
      o[3] = V[i];
    } else {
      o[0] = L[size_t(i) * 3 + 1];
      o[1] = L[size_t(i) * 3 + 2];
      o[2] = 1.0 / A[size_t(i) * m + i];
      o[3] = (i + 1 < m) ? A[size_t(i) * m + i + 1] : 0.0;
      o[4] = (i + 2 < m) ? A[size_t(i) * m + i + 2] : 0.0;
      o[5] = V[size_t(i) * 2];
      o[6] = V[size_t(i) * 2 + 1];
    }
  }
  double* s = out + size_t(m) * per_row;
  for (int t = 0; t < b * b; ++t) s[t] = Si[t];
  return umax / amax;
}

// Parity rows r = 2 i + p (r < rmax) of a dense N x N operator, in half columns.
std::vector<double> parity_rows(const Mat& A, int N, int p, int nr) {
  int n = N / 2;
  std::vector<double> R(size_t(nr) * n, 0.0);
  for (int i = 0; i < nr; ++i) {
    int r = 2 * i + p;
    for (int c = 0; c < n; ++c) R[size_t(i) * n + c] = A[size_t(r) * N + 2 * c + p];
  }
  return R;
}

}  // namespace

Tableau make_tableau(int scheme) {
  Tableau t;
  if (scheme == 2) {
    double g = 1.0 - 1.0 / std::sqrt(2.0), d = 1.0 - 1.0 / (2.0 * g);
    t.s = 2;
    t.ae[1][0] = g;
    t.ae[2][0] = d; t.ae[2][1] = 1.0 - d;
    t.ai[1][1] = g;
    t.ai[2][1] = 1.0 - g; t.ai[2][2] = g;
  } else {
    t.s = 4;
    t.ae[1][0] = 0.5;
    t.ae[2][0] = 11.0 / 18.0; t.ae[2][1] = 1.0 / 18.0;
    t.ae[3][0] = 5.0 / 6.0; t.ae[3][1] = -5.0 / 6.0; t.ae[3][2] = 0.5;
    t.ae[4][0] = 0.25; t.ae[4][1] = 1.75; t.ae[4][2] = 0.75; t.ae[4][3] = -1.75;
    t.ai[1][1] = 0.5;
    t.ai[2][1] = 1.0 / 6.0; t.ai[2][2] = 0.5;
    t.ai[3][1] = -0.5; t.ai[3][2] = 0.5; t.ai[3][3] = 0.5;
    t.ai[4][1] = 1.5; t.ai[4][2] = -1.5; t.ai[4][3] = 0.5; t.ai[4][4] = 0.5;
  }
  return t;
}

std::string build_plan(GridPlan& g) {
  const int N = g.Nz, n = N / 2, Mx = g.Mx, Pz = g.Pz, Ph = Pz / 2;
  g.nu = std::sqrt(g.Pr / g.Ra);
  g.kappa = 1.0 / std::sqrt(g.Ra * g.Pr);
  g.scale = 2.0 / g.Lz;
  g.tab = make_tableau(g.scheme);
  const double haii = g.dt * g.tab.ai[1][1];
  Ops o = make_ops(N, g.scale);

  // mode-independent band tables
  g.bS10.assign(size_t(2) * n * 3, 0.0);
  g.bD2.assign(size_t(2) * n, 0.0);
  g.bA.assign(size_t(2) * n * 3, 0.0);
  g.bB.assign(size_t(2) * n * 5, 0.0);
  g.bD4.assign(size_t(2) * n, 0.0);
  auto at = [N](const Mat& A, int r, int c) { return (c < N) ? A[size_t(r) * N + c] : 0.0; };
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i < n; ++i) {
      int r = 2 * i + p;
      for (int t = 0; t < 3; ++t) g.bS10[(size_t(p) * n + i) * 3 + t] = at(o.S10, r, r + 2 * t);
      g.bD2[size_t(p) * n + i] = at(o.D2, r, r + 2);
      for (int t = 0; t < 3; ++t) g.bA[(size_t(p) * n + i) * 3 + t] = at(o.S32D2, r, r + 2 + 2 * t);
      for (int t = 0; t < 5; ++t) g.bB[(size_t(p) * n + i) * 5 + t] = at(o.S3210, r, r + 2 * t);
      g.bD4[size_t(p) * n + i] = at(o.D4, r, r + 4);
    }

  // factorisations per mode and parity
  const int nrT = n - 1, nrP = n - 2;
  g.facT_stride = kFacT * nrT + 4;
  g.facP_stride = kFacP * nrP + 4;
  if (g.facP_stride < g.facT_stride) g.facP_stride = g.facT_stride;
  g.facT.assign(size_t(Mx) * 2 * g.facT_stride, 0.0);
  g.facP.assign(size_t(Mx) * 2 * g.facP_stride, 0.0);
  g.max_growth = 0;
  std::string err;
  const double dx = 2.0 * M_PI / g.Lx;
  for (int m = 0; m < Mx; ++m) {
    const double k = m * dx, k2 = k * k;
    Mat AT = zeros(N), AP = zeros(N);
    for (size_t e = 0; e < AT.size(); ++e) {
      AT[e] = (1.0 + haii * g.kappa * k2) * o.S10[e] - haii * g.kappa * o.D2[e];
      if (m == 0)
        AP[e] = o.S10[e] - haii * g.nu * o.D2[e];
      else
        AP[e] = (1.0 + 2.0 * haii * g.nu * k2) * o.S32D2[e] -
                k2 * (1.0 + haii * g.nu * k2) * o.S3210[e] - haii * g.nu * o.D4[e];
    }
    for (int p = 0; p < 2; ++p) {
      // wall row of one parity: values (T(1) +- T(-1))/2 = sum c_n, or for
      // fixed flux slopes (T'(1) -+ T'(-1))/2 = sum n^2 c_n
      std::vector<double> C1(n, 1.0), CT(n, 1.0);
      if (g.flux)
        for (int c = 0; c < n; ++c) CT[c] = double(2 * c + p) * double(2 * c + p);
      double gr = factor_bordered(parity_rows(AT, N, p, nrT), nrT, n, 1, 1, CT,
                                  &g.facT[(size_t(m) * 2 + p) * g.facT_stride], kFacT, err);
      if (!err.empty()) return err + " (temperature, mode " + std::to_string(m) + ")";
      g.max_growth = std::fmax(g.max_growth, gr);
      if (m == 0) {
        gr = factor_bordered(parity_rows(AP, N, p, nrT), nrT, n, 1, 1, C1,
                             &g.facP[(size_t(m) * 2 + p) * g.facP_stride], kFacT, err);
      } else {
        std::vector<double> C2(size_t(2) * n);
        for (int c = 0; c < n; ++c) {
          C2[c] = 1.0;
          double nn = 2 * c + p;
          C2[n + c] = nn * nn;
        }
        gr = factor_bordered(parity_rows(AP, N, p, nrP), nrP, n, 2, 2, C2,
                             &g.facP[(size_t(m) * 2 + p) * g.facP_stride], kFacP, err);
      }
      if (!err.empty()) return err + " (flow, mode " + std::to_string(m) + ")";
      g.max_growth = std::fmax(g.max_growth, gr);
    }
  }
  if (!(g.max_growth < 1e8)) return "band factorisation growth too large";

  // Inverse transform: Winv[q][j][n] = d^q/dz^q T_n at Gauss point j < Pz/2.
  g.Winv.assign(size_t(4) * Ph * N, 0.0);
  {
    Mat E(size_t(Pz) * N);
    for (int j = 0; j < Pz; ++j) {
      double th = M_PI * (j + 0.5) / Pz;
      for (int c = 0; c < N; ++c) E[size_t(j) * N + c] = std::cos(c * th);
    }
    Mat D = derivT(N, g.scale);
    Mat Dq = zeros(N);
    for (int c = 0; c < N; ++c) Dq[size_t(c) * N + c] = 1.0;
    for (int q = 0; q < 4; ++q) {
      for (int j = 0; j < Ph; ++j)
        for (int c = 0; c < N; ++c) {
          double v = 0;
          for (int a = 0; a <= c; ++a) v += E[size_t(j) * N + a] * Dq[size_t(a) * N + c];
          g.Winv[(size_t(q) * Ph + j) * N + c] = v;
        }
      Dq = matmul(D, Dq, N);
    }
  }
  // Forward transform folded with the equation bases:
  // Wfwd[e][r][j] (j < Pz/2), e = 0: -S3S2S1S0 F, 1: -S1S0 F, 2: -S1D1 F,
  // F[c][j] = (2 - delta_c0)/Pz T_c(zeta_j).  Row r of e = 0, 1 uses F rows
  // of parity r, of e = 2 parity r + 1; the value at Pz-1-j is the value at j
  // times (-1)^(that parity).
  g.Wfwd.assign(size_t(3) * N * Ph, 0.0);
  {
    std::vector<double> F(size_t(N) * Pz);
    for (int c = 0; c < N; ++c)
      for (int j = 0; j < Pz; ++j)
        F[size_t(c) * Pz + j] = (c == 0 ? 1.0 : 2.0) / Pz * std::cos(c * M_PI * (j + 0.5) / Pz);
    const Mat* ops[3] = {&o.S3210, &o.S10, &o.S1D1};
    for (int e = 0; e < 3; ++e)
      for (int r = 0; r < N; ++r)
        for (int j = 0; j < Ph; ++j) {
          double v = 0;
          for (int c = 0; c < N; ++c) v += (*ops[e])[size_t(r) * N + c] * F[size_t(c) * Pz + j];
          g.Wfwd[(size_t(e) * N + r) * Ph + j] = -v;
        }
  }
  // Split path: the same maps by parity for the GEMM kernels (FP32 rows of
  // contiguous reduction index).
  g.Winv2.clear();
  g.Wfwd2.clear();
  if (g.split) {
    const int Nh = N / 2;
    g.Winv2.assign(size_t(4) * 2 * Ph * Nh, 0.0);
    for (int q = 0; q < 4; ++q)
      for (int p = 0; p < 2; ++p)
        for (int j = 0; j < Ph; ++j)
          for (int i = 0; i < Nh; ++i)
            g.Winv2[((size_t(q) * 2 + p) * Ph + j) * Nh + i] = g.Winv[(size_t(q) * Ph + j) * N + 2 * i + p];
    g.Wfwd2.assign(size_t(2) * 2 * Nh * Ph, 0.0);
    for (int f = 0; f < 2; ++f)
      for (int p = 0; p < 2; ++p)
        for (int i = 0; i < Nh; ++i)
          for (int j = 0; j < Ph; ++j)
            g.Wfwd2[((size_t(f) * 2 + p) * Nh + i) * Ph + j] = g.Wfwd[(size_t(f) * N + 2 * i + p) * Ph + j];
  }
  // FFT twiddles and radix plan for Px = 3 * 2^q
  g.tw.assign(size_t(2) * g.Px, 0.0);
  for (int t = 0; t < g.Px; ++t) {
    g.tw[2 * t] = std::cos(2.0 * M_PI * t / g.Px);
    g.tw[2 * t + 1] = -std::sin(2.0 * M_PI * t / g.Px);
  }
  {
    int rem = g.Px, nr = 0;
    if (rem % 3 != 0) return "Px must be 3 * 2^q";
    g.dev.rad[nr++] = 3;
    rem /= 3;
    while (rem % 4 == 0) { g.dev.rad[nr++] = 4; rem /= 4; }
    if (rem == 2) { g.dev.rad[nr++] = 2; rem = 1; }
    if (rem != 1) return "Nx must be 2^q with q >= 2 (Px = 3 Nx / 2)";
    g.dev.nrad = nr;
  }
  return "";
}

size_t plan_device_bytes(const GridPlan& g) {
  size_t rb = g.mixed ? 4 : 8;
  size_t d = g.bS10.size() + g.bD2.size() + g.bA.size() + g.bB.size() + g.bD4.size() +
             g.facT.size() + g.facP.size() + sizeof(RunDev) / 8 + 1;
  size_t r = g.Winv.size() + g.Wfwd.size() + g.tw.size() + g.Winv2.size() + g.Wfwd2.size();
  return d * 8 + r * rb + 64 * 16;
}

RunDev make_run_dev(const GridPlan& g, const double* facT_dev, const double* facP_dev) {
  RunDev r{};
  r.facT = facT_dev;
  r.facP = facP_dev;
  r.nu = g.nu;
  r.kappa = g.kappa;
  r.sqrtRaPr = std::sqrt(g.Ra * g.Pr);
  // the stage coefficients as the launchers form them for StageArgs
  for (int i = 0; i < kMaxStages; ++i)
    for (int j = 0; j < kMaxStages; ++j) {
      r.hae[i][j] = g.dt * g.tab.ae[i][j];
      r.hai[i][j] = g.dt * g.tab.ai[i][j];
    }
  return r;
}

hipError_t upload_plan(GridPlan& g) {
  const bool mx = g.mixed;
  const size_t rb = mx ? 4 : 8;
  std::vector<const std::vector<double>*> dbl = {&g.bS10, &g.bD2, &g.bA, &g.bB, &g.bD4, &g.facT, &g.facP};
  std::vector<const std::vector<double>*> rl = {&g.Winv, &g.Wfwd, &g.tw, &g.Winv2, &g.Wfwd2};
  size_t off = 0;
  std::vector<size_t> offs;
  auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
  for (auto* v : dbl) { offs.push_back(off); off = align(off + v->size() * 8); }
  for (auto* v : rl) { offs.push_back(off); off = align(off + v->size() * rb); }
  const size_t run_off = off;   // the grid's own RunDev
  off = align(off + sizeof(RunDev));
  std::vector<unsigned char> host(off, 0);
  size_t k = 0;
  for (auto* v : dbl) { std::memcpy(host.data() + offs[k++], v->data(), v->size() * 8); }
  for (auto* v : rl) {
    if (mx) {
      std::vector<float> f(v->begin(), v->end());
      std::memcpy(host.data() + offs[k++], f.data(), f.size() * 4);
    } else {
      std::memcpy(host.data() + offs[k++], v->data(), v->size() * 8);
    }
  }
  hipError_t e = hipMalloc(&g.d_tables, off);
  if (e != hipSuccess) return e;
  auto* base = static_cast<unsigned char*>(g.d_tables);
  const RunDev r0 = make_run_dev(g, reinterpret_cast<const double*>(base + offs[5]),
                                 reinterpret_cast<const double*>(base + offs[6]));
  std::memcpy(host.data() + run_off, &r0, sizeof(RunDev));
  e = hipMemcpy(g.d_tables, host.data(), off, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  GridDev& d = g.dev;
  d.Nx = g.Nx; d.Nz = g.Nz; d.Mx = g.Mx; d.Px = g.Px; d.Pz = g.Pz; d.n = g.Nz / 2;
  d.nrT = d.n - 1; d.nrP = d.n - 2; d.MT = g.MT;
  d.ntile = (g.Mx + g.MT - 1) / g.MT;
  d.split = g.split ? 1 : 0;
  d.xrows = g.xrows;
  d.XT = g.split ? kGemmModes : g.MT;
  d.nxt = (g.Mx + d.XT - 1) / d.XT;
  d.state = 4 * g.Mx * g.Nz;
  d.kscale = 2.0 * M_PI / g.Lx;
  d.nu = g.nu; d.kappa = g.kappa; d.scale = g.scale; d.Lz = g.Lz;
  d.sqrtRaPr = std::sqrt(g.Ra * g.Pr);
  d.T_bot = g.T_bot; d.T_top = g.T_top;
  // right-hand sides of the m = 0 temperature wall rows per parity: values
  // (T_top +- T_bot)/2, or for fixed flux the zeta-slopes (0, -Lz/2) of
  // dT/dz = -1 at both walls
  d.bcT[0] = g.flux ? 0.0 : 0.5 * (g.T_top + g.T_bot);
  d.bcT[1] = g.flux ? -0.5 * g.Lz : 0.5 * (g.T_top - g.T_bot);
  d.fluxT = g.flux ? 1 : 0;
  d.urgent = g.urgent ? 1 : 0;
  d.one_xcd = g.one_xcd ? 1 : 0;
  d.bS10 = reinterpret_cast<const double*>(base + offs[0]);
  d.bD2 = reinterpret_cast<const double*>(base + offs[1]);
  d.bA = reinterpret_cast<const double*>(base + offs[2]);
  d.bB = reinterpret_cast<const double*>(base + offs[3]);
  d.bD4 = reinterpret_cast<const double*>(base + offs[4]);
  d.facT = reinterpret_cast<const double*>(base + offs[5]);
  d.facP = reinterpret_cast<const double*>(base + offs[6]);
  d.facT_stride = g.facT_stride; d.facP_stride = g.facP_stride;
  d.Winv = base + offs[7];
  d.Wfwd = base + offs[8];
  d.tw = base + offs[9];
  d.Winv2 = g.split ? reinterpret_cast<const float*>(base + offs[10]) : nullptr;
  d.Wfwd2 = g.split ? reinterpret_cast<const float*>(base + offs[11]) : nullptr;
  d.run0 = reinterpret_cast<const RunDev*>(base + run_off);
  d.xptrs = nullptr;
  d.rptrs = nullptr;
  return hipSuccess;
}

// Modes rounded up to whole tiles of the mixed-space arrays (tile-major).
static size_t padded_modes(const GridPlan& g) {
  const int xt = g.split ? kGemmModes : g.MT;
  return size_t((g.Mx + xt - 1) / xt) * xt;
}

size_t work_bytes(const GridPlan& g, int cap) {
  size_t rb = g.mixed ? 4 : 8;
  size_t st = size_t(4) * g.Mx * g.Nz;
  size_t q = size_t(cap) * 6 * g.Pz * padded_modes(g) * 2 * rb;
  size_t nh = size_t(cap) * 2 * g.Pz * padded_modes(g) * 2 * rb + size_t(cap) * g.Pz * rb;
  size_t eh = size_t(g.tab.s) * cap * st * rb;
  size_t ly = size_t(g.tab.s - 1) * cap * st * 8;
  size_t dp = size_t(cap) * ((g.Mx + diag_modes(g.Nz) - 1) / diag_modes(g.Nz)) * 4 * 8;
  size_t yf = g.split ? size_t(cap) * st * 4 : 0;
  return q + nh + eh + ly + dp + yf + 6 * 256;
}

hipError_t alloc_work(const GridPlan& g, int cap, Work& w) {
  size_t rb = g.mixed ? 4 : 8;
  size_t st = size_t(4) * g.Mx * g.Nz;
  w.cap = cap;
  hipError_t e;
  if ((e = hipMalloc(&w.Q, size_t(cap) * 6 * g.Pz * padded_modes(g) * 2 * rb)) != hipSuccess) return e;
  if ((e = hipMalloc(&w.Nh, size_t(cap) * 2 * g.Pz * padded_modes(g) * 2 * rb)) != hipSuccess) return e;
  if ((e = hipMalloc(&w.qbar, size_t(cap) * g.Pz * rb)) != hipSuccess) return e;
  if ((e = hipMalloc(&w.Ehist, size_t(g.tab.s) * cap * st * rb)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.LYhist, size_t(g.tab.s - 1) * cap * st * 8)) != hipSuccess) return e;
  const size_t nchunk = (g.Mx + diag_modes(g.Nz) - 1) / diag_modes(g.Nz);
  if ((e = hipMalloc((void**)&w.dpart, size_t(cap) * nchunk * 4 * 8)) != hipSuccess) return e;
  if (g.split && (e = hipMalloc((void**)&w.Yf, size_t(cap) * st * 4)) != hipSuccess) return e;
  return hipSuccess;
}

void free_work(Work& w) {
  if (w.Q) (void)hipFree(w.Q);
  if (w.Nh) (void)hipFree(w.Nh);
  if (w.qbar) (void)hipFree(w.qbar);
  if (w.Ehist) (void)hipFree(w.Ehist);
  if (w.LYhist) (void)hipFree(w.LYhist);
  if (w.dpart) (void)hipFree(w.dpart);
  if (w.Yf) (void)hipFree(w.Yf);
  w = Work{};
}

}  // namespace rbc
