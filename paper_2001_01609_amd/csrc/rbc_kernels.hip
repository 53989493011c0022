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
template <typename Real>
__device__ __forceinline__ Cx<Real> csub(Cx<Real> a, Cx<Real> b) { return {a.x - b.x, a.y - b.y}; }

// ------------------------------------------------------------------ x-pass ---

// One Stockham radix-R pass over `cnt` signals of length N stored with
// stride N: out[j + q p] = DFT_R over the twiddled in[i + r N/R] (Bainville's
// autosort form).  sign = -1 forward, +1 inverse.
template <typename Real, int R>
__device__ void stockham_pass(const Cx<Real>* __restrict__ in, Cx<Real>* __restrict__ out,
                              const Cx<Real>* __restrict__ tw, int N, int p, int cnt, Real sign) {
  const int T = N / R;
  const int stride_t = N / (p * R);
  for (int w = threadIdx.x; w < cnt * T; w += blockDim.x) {
    const int c = w / T, i = w - c * T;
    const Cx<Real>* x = in + c * N;
    Cx<Real>* y = out + c * N;
    const int k = i % p;
    Cx<Real> a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Cx<Real> v = x[i + r * T];
      if (r > 0 && k > 0) {
        Cx<Real> t = tw[(r * k * stride_t) % N];
        t.y *= -sign;   // table holds exp(-2 pi i t/N); inverse uses the conjugate
        v = cmul(v, t);
      }
      a[r] = v;
    }
    const int j = (i - k) * R + k;
    if constexpr (R == 2) {
      y[j] = cadd(a[0], a[1]);
      y[j + p] = csub(a[0], a[1]);
    } else if constexpr (R == 3) {
      const Real h = Real(0.86602540378443864676);  // sqrt(3)/2
      Cx<Real> t = cadd(a[1], a[2]), d = csub(a[1], a[2]);
      Cx<Real> m = {a[0].x - Real(0.5) * t.x, a[0].y - Real(0.5) * t.y};
      Cx<Real> id = {-sign * h * d.y, sign * h * d.x};   // sign * i * h * d
      y[j] = cadd(a[0], t);
      y[j + p] = cadd(m, id);
      y[j + 2 * p] = csub(m, id);
    } else {
      Cx<Real> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
      Cx<Real> s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
      Cx<Real> id13 = {-sign * d13.y, sign * d13.x};      // sign * i * (a1 - a3)
      y[j] = cadd(s02, s13);
      y[j + p] = cadd(d02, id13);
      y[j + 2 * p] = csub(s02, s13);
      y[j + 3 * p] = csub(d02, id13);
    }
  }
}

// Runs the radix plan on cnt signals; returns the buffer holding the result.
template <typename Real>
__device__ Cx<Real>* fft_lds(Cx<Real>* a, Cx<Real>* b, const Cx<Real>* tw, const GridDev& g, int cnt,
                             Real sign) {
  int p = 1;
  for (int st = 0; st < g.nrad; ++st) {
    const int R = g.rad[st];
    if (R == 3)
      stockham_pass<Real, 3>(a, b, tw, g.Px, p, cnt, sign);
    else if (R == 4)
      stockham_pass<Real, 4>(a, b, tw, g.Px, p, cnt, sign);
    else
      stockham_pass<Real, 2>(a, b, tw, g.Px, p, cnt, sign);
    __syncthreads();
    p *= R;
    Cx<Real>* t = a;
    a = b;
    b = t;
  }
  return a;
}

template <typename Real>
__global__ void __launch_bounds__(kBlock) xpass_kernel(GridDev g, const Real* __restrict__ Q,
                                                       Real* __restrict__ Nh, Real* __restrict__ qbar) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Px = g.Px, Pz = g.Pz, Mx = g.Mx;
  const int s = blockIdx.x / Pz, j = blockIdx.x - s * Pz;
  Cx<Real>* A = reinterpret_cast<Cx<Real>*>(smem);   // [3][Px]
  Cx<Real>* B = A + 3 * Px;                           // [3][Px]
  Cx<Real>* tw = B + 3 * Px;                          // [Px] twiddles
  Real* red = reinterpret_cast<Real*>(tw + Px);       // [blockDim]
  const Cx<Real>* gtw = reinterpret_cast<const Cx<Real>*>(g.tw);

  for (int t = threadIdx.x; t < Px; t += blockDim.x) tw[t] = gtw[t];
  for (int t = threadIdx.x; t < 3 * Px; t += blockDim.x) A[t] = {Real(0), Real(0)};
  __syncthreads();
  // pack (u, w), (omega_x, omega_z), (T_x, T_z) into three complex spectra
  const size_t rowQ = size_t(Mx) * 2;
  for (int t = threadIdx.x; t < 3 * Mx; t += blockDim.x) {
    const int c = t / Mx, m = t - c * Mx;
    const Real* qa = Q + ((size_t(s) * 6 + 2 * c) * Pz + j) * rowQ + 2 * m;
    const Real* qb = Q + ((size_t(s) * 6 + 2 * c + 1) * Pz + j) * rowQ + 2 * m;
    const Real ar = qa[0], ai = qa[1], br = qb[0], bi = qb[1];
    A[c * Px + m] = {ar - bi, ai + br};
    if (m > 0) A[c * Px + Px - m] = {ar + bi, br - ai};
  }
  __syncthreads();
  Cx<Real>* z = fft_lds<Real>(A, B, tw, g, 3, Real(1));
  Cx<Real>* o = (z == A) ? B : A;
  Real uw = 0;
  for (int t = threadIdx.x; t < Px; t += blockDim.x) {
    const Cx<Real> v1 = z[t], v2 = z[Px + t], v3 = z[2 * Px + t];
    const Real u = v1.x, w = v1.y;
    o[t] = {u * v2.x + w * v2.y, u * v3.x + w * v3.y};
    uw += u * w;
  }
  red[threadIdx.x] = uw;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) qbar[size_t(s) * Pz + j] = red[0] / Real(Px);
  Cx<Real>* Z = fft_lds<Real>(o, z, tw, g, 1, Real(-1));
  const Real inv2 = Real(0.5) / Real(Px);
  Real* out0 = Nh + ((size_t(s) * 2 + 0) * Pz + j) * rowQ;
  Real* out1 = Nh + ((size_t(s) * 2 + 1) * Pz + j) * rowQ;
  for (int m = threadIdx.x; m < Mx; m += blockDim.x) {
    const Cx<Real> a = Z[m], b = Z[m == 0 ? 0 : Px - m];
    // N_omega = (Z_m + conj Z_-m)/2, N_T = (Z_m - conj Z_-m)/(2i), both / Px
    out0[2 * m] = (a.x + b.x) * inv2;
    out0[2 * m + 1] = (a.y - b.y) * inv2;
    out1[2 * m] = (a.y + b.y) * inv2;
    out1[2 * m + 1] = (b.x - a.x) * inv2;
  }
}

// ------------------------------------------------------------ stage kernel ---

enum StageMode { kModeStage = 0, kModeZinv = 1, kModeExplicit = 2 };

struct StageArgs {
  int mode;
  int stage;           // i = 1..s
  int s;               // implicit stages
  int cap;             // slices the history arrays are sized for
  int store_E, store_LY, write_X, do_zinv;
  double hae[kMaxStages];   // h a_ij (explicit), j < i
  double hai[kMaxStages];   // h a~_ij (implicit), 1 <= j <= i
  double haii;
};

// LDS strides (in doubles) of one staged factor block: odd, so that lanes
// reading different blocks at the same row fall in different banks.
__host__ __device__ __forceinline__ int lds_fac_stride(int s) { return s | 1; }

// Bordered tridiagonal solve in place on v[2 i + p] (stride-2 view of one
// parity): temperature and mean-flow systems.  fac: kFacT per row, then the
// 1 x 1 Schur inverse.
__device__ __forceinline__ void solve_T_format(double* v, int p, const double* fac, int nr, double gbc) {
  double y = v[p];
#pragma unroll 4
  for (int i = 1; i < nr; ++i) {
    y = v[2 * i + p] - fac[i * kFacT + 0] * y;
    v[2 * i + p] = y;
  }
  double x = v[2 * (nr - 1) + p] * fac[(nr - 1) * kFacT + 1];
  v[2 * (nr - 1) + p] = x;
  double sum = x;
#pragma unroll 4
  for (int i = nr - 2; i >= 0; --i) {
    x = (v[2 * i + p] - fac[i * kFacT + 2] * x) * fac[i * kFacT + 1];
    v[2 * i + p] = x;
    sum += x;
  }
  const double xh = fac[nr * kFacT] * (gbc - sum);
#pragma unroll 4
  for (int i = nr - 1; i >= 0; --i) v[2 * (i + 1) + p] = v[2 * i + p] - fac[i * kFacT + 3] * xh;
  v[p] = xh;
}

// Bordered pentadiagonal solve in place (streamfunction, two border unknowns).
__device__ __forceinline__ void solve_P_format(double* v, int p, const double* fac, int nr) {
  double y2 = 0, y1 = 0;
#pragma unroll 4
  for (int i = 0; i < nr; ++i) {
    const double y = v[2 * i + p] - fac[i * kFacP + 0] * y1 - fac[i * kFacP + 1] * y2;
    v[2 * i + p] = y;
    y2 = y1;
    y1 = y;
  }
  double x1 = 0, x2 = 0, s0 = 0, s1 = 0;
#pragma unroll 4
  for (int i = nr - 1; i >= 0; --i) {
    const double* f = fac + i * kFacP;
    const double x = (v[2 * i + p] - f[3] * x1 - f[4] * x2) * f[2];
    v[2 * i + p] = x;
    const double nn = double(2 * (i + 2) + p);
    s0 += x;
    s1 += nn * nn * x;
    x2 = x1;
    x1 = x;
  }
  const double* si = fac + nr * kFacP;
  const double h0 = -(si[0] * s0 + si[1] * s1);
  const double h1 = -(si[2] * s0 + si[3] * s1);
#pragma unroll 4
  for (int i = nr - 1; i >= 0; --i)
    v[2 * (i + 2) + p] = v[2 * i + p] - fac[i * kFacP + 5] * h0 - fac[i * kFacP + 6] * h1;
  v[p] = h0;
  v[2 + p] = h1;
}

// Copies the factor blocks of modes m0..m0+MT-1 (both parities) into LDS.
template <int MT>
__device__ __forceinline__ void stage_factors(double* sF, const double* __restrict__ fac, int stride, int m0,
                                              int Mx) {
  const int ls = lds_fac_stride(stride);
  const int nm = min(MT, Mx - m0);
  const double* src = fac + size_t(m0) * 2 * stride;
  for (int e = threadIdx.x; e < nm * 2 * stride; e += blockDim.x) {
    const int b = e / stride, o = e - b * stride;
    sF[b * ls + o] = src[e];
  }
}

// LDS layout of a block (doubles first, then Real):
//   sY  double [2 field][MT][2 re/im][Nz+1]     right-hand sides -> new stage
//   U   union { Real sN[2][Pz][MT][2] + sq[Pz];  double sF[MT*2][odd stride] }
template <typename Real, int MT>
__global__ void __launch_bounds__(kBlock)
stage_kernel(GridDev g, StageArgs a, const Real* __restrict__ Nh, const Real* __restrict__ qbar,
             double* __restrict__ X, Real* __restrict__ Ehist, double* __restrict__ LYhist,
             Real* __restrict__ Q, double* __restrict__ Eout) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Nz = g.Nz, Mx = g.Mx, Pz = g.Pz, Ph = Pz / 2, LD = Nz + 1;
  const int ntile = (Mx + MT - 1) / MT;
  const int s = blockIdx.x / ntile, tile = blockIdx.x - s * ntile;
  const int m0 = tile * MT;
  const int st = g.state;
  double* sY = reinterpret_cast<double*>(smem);
  unsigned char* uni = smem + sizeof(double) * 4 * MT * LD;
  Real* sN = reinterpret_cast<Real*>(uni);
  Real* sq = sN + 4 * Pz * MT;
  double* sF = reinterpret_cast<double*>(uni);
  auto yi = [&](int f, int mt, int ri) { return ((f * MT + mt) * 2 + ri) * LD; };
  auto gidx = [&](int f, int m, int ri) { return size_t(((f * Mx + m) * 2 + ri)) * Nz; };
  const double* Xs = X + size_t(s) * st;
  const int tid = threadIdx.x, nth = blockDim.x;

  if (a.mode == kModeZinv) {
    for (int e = tid; e < 4 * MT * Nz; e += nth) {
      const int nn = e % Nz, c = e / Nz, ri = c & 1, mt = (c >> 1) % MT, f = c / (2 * MT);
      const int m = m0 + mt;
      sY[yi(f, mt, ri) + nn] = (m < Mx) ? Xs[gidx(f, m, ri) + nn] : 0.0;
    }
    __syncthreads();
  } else {
    // ---- phase A: products of this tile on the padded Gauss points
    // (8 loads in flight per thread before the LDS stores)
    const size_t rowQ = size_t(Mx) * 2;
    {
      constexpr int U = 8;
      const int total = 4 * Pz * MT;
      for (int base = tid; base < total; base += nth * U) {
        Real v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * nth;
          v[u] = Real(0);
          if (e < total) {
            const int c = e % (2 * MT), j = (e / (2 * MT)) % Pz, qq = e / (2 * MT * Pz);
            if (m0 + (c >> 1) < Mx) v[u] = Nh[((size_t(s) * 2 + qq) * Pz + j) * rowQ + 2 * m0 + c];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * nth;
          if (e < total) sN[e] = v[u];
        }
      }
    }
    if (m0 == 0)
      for (int j = tid; j < Pz; j += nth) sq[j] = qbar[size_t(s) * Pz + j];
    __syncthreads();
    // ---- phase B: explicit terms of the previous stage on the band rows.
    // Item (f, r): one row of the folded forward map against every column
    // (mode, re/im) of the tile; the u_bar column of mode 0 separately.
    const Real* W = reinterpret_cast<const Real*>(g.Wfwd);
    const int nitems = 2 * Nz + (m0 == 0 ? Nz : 0);
    for (int e = tid; e < nitems; e += nth) {
      const int r = e % Nz, f = e / Nz;   // f = 2: the u_bar column
      const int rows = (f == 0) ? Nz - 4 : Nz - 2;
      if (f == 2) {
        double E = 0.0;
        if (r < Nz - 2) {
          const Real* w = W + (size_t(2) * Nz + r) * Ph;
          const Real sg = (r & 1) ? Real(1) : Real(-1);
          Real acc = 0;
#pragma unroll 8
          for (int j = 0; j < Ph; ++j) acc += w[j] * (sq[j] + sg * sq[Pz - 1 - j]);
          E = double(acc);
        }
        if (a.mode == kModeExplicit) {
          Eout[gidx(0, 0, 0) + r] = E;
          Eout[gidx(0, 0, 1) + r] = 0.0;
        } else {
          sY[yi(0, 0, 0) + r] = a.hae[a.stage - 1] * E;
          sY[yi(0, 0, 1) + r] = 0.0;
          if (a.store_E) {
            Real* eh = Ehist + (size_t(a.stage - 1) * a.cap + s) * st;
            eh[gidx(0, 0, 0) + r] = Real(E);
            eh[gidx(0, 0, 1) + r] = Real(0);
          }
        }
        continue;
      }
      Real acc[2 * MT];
#pragma unroll
      for (int c = 0; c < 2 * MT; ++c) acc[c] = Real(0);
      if (r < rows) {
        const Real* w = W + (size_t(f == 0 ? 0 : 1) * Nz + r) * Ph;
        const Real* src = sN + (f == 0 ? 0 : Pz * 2 * MT);
        const Real sg = (r & 1) ? Real(-1) : Real(1);
#pragma unroll 8
        for (int j = 0; j < Ph; ++j) {
          const Real wv = w[j];
          const Real* a0 = src + j * 2 * MT;
          const Real* a1 = src + (Pz - 1 - j) * 2 * MT;
#pragma unroll
          for (int c = 0; c < 2 * MT; ++c) acc[c] += wv * (a0[c] + sg * a1[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < 2 * MT; ++c) {
        const int mt = c >> 1, ri = c & 1, m = m0 + mt;
        if (m >= Mx || (f == 0 && m == 0)) continue;
        const double E = double(acc[c]);
        if (a.mode == kModeExplicit) {
          Eout[gidx(f, m, ri) + r] = E;
        } else {
          sY[yi(f, mt, ri) + r] = a.hae[a.stage - 1] * E;
          if (a.store_E) Ehist[(size_t(a.stage - 1) * a.cap + s) * st + gidx(f, m, ri) + r] = Real(E);
        }
      }
    }
    if (a.mode == kModeExplicit) return;
    __syncthreads();
    // temperature factors into the (now free) union region
    stage_factors<MT>(sF, g.facT, g.facT_stride, m0, Mx);
    // ---- phase C: right-hand side of stage i on the band rows
#pragma unroll 4
    for (int e = tid; e < 4 * MT * Nz; e += nth) {
      const int r = e % Nz, c = e / Nz, ri = c & 1, mt = (c >> 1) % MT, f = c / (2 * MT);
      const int m = m0 + mt;
      if (m >= Mx) continue;
      const bool psi = (f == 0 && m > 0);
      const int rows = psi ? Nz - 4 : Nz - 2;
      if (r >= rows) continue;
      const int p = r & 1, i = r >> 1;
      const double* xv = Xs + gidx(f, m, ri);
      double MX = 0;
      if (!psi) {
        const double* b = g.bS10 + (p * g.n + i) * 3;
        for (int t = 0; t < 3; ++t)
          if (r + 2 * t < Nz) MX += b[t] * xv[r + 2 * t];
      } else {
        const double k = m * g.kscale;
        const double* bA = g.bA + (p * g.n + i) * 3;
        const double* bB = g.bB + (p * g.n + i) * 5;
        double sa = 0, sb = 0;
        for (int t = 0; t < 3; ++t)
          if (r + 2 + 2 * t < Nz) sa += bA[t] * xv[r + 2 + 2 * t];
        for (int t = 0; t < 5; ++t)
          if (r + 2 * t < Nz) sb += bB[t] * xv[r + 2 * t];
        MX = sa - k * k * sb;
      }
      double acc = MX + sY[yi(f, mt, ri) + r];
      const size_t off = gidx(f, m, ri) + r;
      for (int jj = 0; jj + 1 < a.stage; ++jj)
        acc += a.hae[jj] * double(Ehist[(size_t(jj) * a.cap + s) * st + off]);
      for (int jj = 1; jj < a.stage; ++jj)
        acc += a.hai[jj] * LYhist[(size_t(jj - 1) * a.cap + s) * st + off];
      sY[yi(f, mt, ri) + r] = acc;
    }
    __syncthreads();
    // ---- phase D: temperature solves, lanes (mode, parity, re/im)
    if (tid < 4 * MT) {
      const int mt = tid >> 2, p = (tid >> 1) & 1, ri = tid & 1, m = m0 + mt;
      if (m < Mx) {
        double gbc = 0.0;
        if (m == 0 && ri == 0) gbc = (p == 0) ? 0.5 * (g.T_top + g.T_bot) : 0.5 * (g.T_top - g.T_bot);
        solve_T_format(sY + yi(1, mt, ri), p, sF + (mt * 2 + p) * lds_fac_stride(g.facT_stride), g.nrT, gbc);
      }
    }
    __syncthreads();
    // flow factors; implicit buoyancy of the new temperature into psi
    stage_factors<MT>(sF, g.facP, g.facP_stride, m0, Mx);
    for (int e = tid; e < 2 * MT * Nz; e += nth) {
      const int r = e % Nz, c = e / Nz, ri = c & 1, mt = c >> 1, m = m0 + mt;
      if (m >= Mx || m == 0 || r >= Nz - 4) continue;
      const int p = r & 1, i = r >> 1;
      const double k = m * g.kscale;
      const double* bB = g.bB + (p * g.n + i) * 5;
      const double* tv = sY + yi(1, mt, ri ^ 1);
      double sb = 0;
      for (int t = 0; t < 5; ++t)
        if (r + 2 * t < Nz) sb += bB[t] * tv[r + 2 * t];
      sY[yi(0, mt, ri) + r] += a.haii * (ri == 0 ? k * sb : -k * sb);
    }
    __syncthreads();
    if (tid < 4 * MT) {
      const int mt = tid >> 2, p = (tid >> 1) & 1, ri = tid & 1, m = m0 + mt;
      if (m < Mx) {
        const double* fac = sF + (mt * 2 + p) * lds_fac_stride(g.facP_stride);
        if (m == 0)
          solve_T_format(sY + yi(0, mt, ri), p, fac, g.nrT, 0.0);
        else
          solve_P_format(sY + yi(0, mt, ri), p, fac, g.nrP);
      }
    }
    __syncthreads();
    // ---- phase F: L Y_i for later stages; the new state at the last stage
    if (a.store_LY) {
      for (int e = tid; e < 4 * MT * Nz; e += nth) {
        const int r = e % Nz, c = e / Nz, ri = c & 1, mt = (c >> 1) % MT, f = c / (2 * MT);
        const int m = m0 + mt;
        if (m >= Mx) continue;
        const bool psi = (f == 0 && m > 0);
        if (r >= (psi ? Nz - 4 : Nz - 2)) continue;
        const int p = r & 1, i = r >> 1;
        const double* yv = sY + yi(f, mt, ri);
        const double k = m * g.kscale, k2 = k * k;
        double L;
        if (f == 1) {
          const double* b = g.bS10 + (p * g.n + i) * 3;
          double sm = 0;
          for (int t = 0; t < 3; ++t)
            if (r + 2 * t < Nz) sm += b[t] * yv[r + 2 * t];
          L = g.kappa * (g.bD2[p * g.n + i] * yv[r + 2] - k2 * sm);
        } else if (m == 0) {
          L = g.nu * g.bD2[p * g.n + i] * yv[r + 2];
        } else {
          const double* bA = g.bA + (p * g.n + i) * 3;
          const double* bB = g.bB + (p * g.n + i) * 5;
          const double* tv = sY + yi(1, mt, ri ^ 1);
          double sa = 0, sb = 0, st5 = 0;
          for (int t = 0; t < 3; ++t)
            if (r + 2 + 2 * t < Nz) sa += bA[t] * yv[r + 2 + 2 * t];
          for (int t = 0; t < 5; ++t)
            if (r + 2 * t < Nz) {
              sb += bB[t] * yv[r + 2 * t];
              st5 += bB[t] * tv[r + 2 * t];
            }
          L = g.nu * (g.bD4[p * g.n + i] * yv[r + 4] - 2.0 * k2 * sa + k2 * k2 * sb) +
              (ri == 0 ? k * st5 : -k * st5);
        }
        LYhist[(size_t(a.stage - 1) * a.cap + s) * st + gidx(f, m, ri) + r] = L;
      }
    }
    if (a.write_X) {
      double* Xw = X + size_t(s) * st;
      for (int e = tid; e < 4 * MT * Nz; e += nth) {
        const int nn = e % Nz, c = e / Nz, ri = c & 1, mt = (c >> 1) % MT, f = c / (2 * MT);
        const int m = m0 + mt;
        if (m < Mx) Xw[gidx(f, m, ri) + nn] = sY[yi(f, mt, ri) + nn];
      }
    }
    if (!a.do_zinv) return;
  }
  // ---- phase G: values and z-derivatives of the new stage at the padded
  // Gauss points j and Pz-1-j, six quantities per mode (m contiguous in HBM)
  const Real* Wi = reinterpret_cast<const Real*>(g.Winv);
  const size_t rowQ = size_t(Mx) * 2;
  for (int e = tid; e < Ph * MT; e += nth) {
    const int mt = e % MT, j = e / MT, m = m0 + mt;
    if (m >= Mx) continue;
    // acc[parity][q][re/im]: q = 0..3 on psi (E D^q psi), 4..5 on T (E, E D)
    Real acc[2][6][2];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[pp][q][0] = acc[pp][q][1] = Real(0);
    const double* pr = sY + yi(0, mt, 0);
    const double* pi = sY + yi(0, mt, 1);
    const double* tr = sY + yi(1, mt, 0);
    const double* ti = sY + yi(1, mt, 1);
    const Real* w0 = Wi + (size_t(0) * Ph + j) * Nz;
    const Real* w1 = Wi + (size_t(1) * Ph + j) * Nz;
    const Real* w2 = Wi + (size_t(2) * Ph + j) * Nz;
    const Real* w3 = Wi + (size_t(3) * Ph + j) * Nz;
#pragma unroll 4
    for (int nn = 0; nn < Nz; nn += 2) {
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
      const int jj = side ? Pz - 1 - j : j;
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
        Real* d = Q + ((size_t(s) * 6 + q) * Pz + jj) * rowQ + 2 * m;
        d[0] = out[q][0];
        d[1] = out[q][1];
      }
    }
  }
}

// ------------------------------------------------------------------ Nusselt ---

// One block per state.  <w T> = sum_{m>=1} Re(w_m^T J conj(T_m)) with
// J_ab = int_{-1}^{1} T_a T_b = (I(a+b) + I(|a-b|))/2, I(n) = 2/(1-n^2) for
// even n; w_m = -i k psi_m.  Fixed-order partial sums and tree reduction.
__global__ void __launch_bounds__(kBlock)
nusselt_kernel(GridDev g, const double* __restrict__ X, double* __restrict__ out, int ld3) {
  __shared__ double red[kBlock];
  const int Nz = g.Nz, Mx = g.Mx;
  const double* x = X + size_t(blockIdx.x) * g.state;
  double acc = 0;
  for (int e = threadIdx.x; e < (Mx - 1) * Nz; e += blockDim.x) {
    const int m = 1 + e / Nz, aa = e % Nz;
    const double k = m * g.kscale;
    const double pr = x[((0 * Mx + m) * 2 + 0) * Nz + aa], pim = x[((0 * Mx + m) * 2 + 1) * Nz + aa];
    const double wr = k * pim, wi = -k * pr;
    const double* tr = x + size_t((1 * Mx + m) * 2 + 0) * Nz;
    const double* ti = x + size_t((1 * Mx + m) * 2 + 1) * Nz;
    double sr = 0, si = 0;
    for (int b = aa & 1; b < Nz; b += 2) {
      const int sp = aa + b, df = aa > b ? aa - b : b - aa;
      const double J = 1.0 / (1.0 - double(sp) * sp) + 1.0 / (1.0 - double(df) * df);
      sr += J * tr[b];
      si += J * ti[b];
    }
    acc += wr * sr + wi * si;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double* tm = x + size_t((1 * Mx + 0) * 2 + 0) * Nz;
    double nb = 0, nt = 0, t0 = 0, t1 = 0;
    for (int n = 0; n < Nz; ++n) {
      const double sgn = (n & 1) ? -1.0 : 1.0, n2 = double(n) * n;
      nb += tm[n] * (-sgn) * n2;   // T_n'(-1) = (-1)^(n+1) n^2
      nt += tm[n] * n2;            // T_n'(1) = n^2
      t0 += tm[n] * sgn;
      t1 += tm[n];
    }
    double* o = out + size_t(blockIdx.x) * ld3;
    o[0] = (t0 - t1) / g.Lz + g.sqrtRaPr * red[0];
    o[1] = -g.scale * nb;
    o[2] = -g.scale * nt;
  }
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

size_t stage_lds(const GridDev& d, size_t rb) {
  const size_t y = sizeof(double) * 4 * d.MT * (d.Nz + 1);
  const size_t n = rb * (4 * size_t(d.Pz) * d.MT + d.Pz);
  const int fs = d.facT_stride > d.facP_stride ? d.facT_stride : d.facP_stride;
  const size_t f = sizeof(double) * size_t(d.MT) * 2 * lds_fac_stride(fs);
  return y + (n > f ? n : f);
}
size_t xpass_lds(const GridDev& d, size_t rb) {
  return rb * 2 * (7 * size_t(d.Px)) + rb * kBlock;
}

template <typename Real, int MT>
hipError_t run_stage_mt(const GridPlan& g, Work& w, const StageArgs& a, double* X, int n_slices, double* Eout,
                        hipStream_t st) {
  const GridDev& d = g.dev;
  const int ntile = (d.Mx + MT - 1) / MT;
  hipLaunchKernelGGL((stage_kernel<Real, MT>), dim3(n_slices * ntile), dim3(kBlock), stage_lds(d, sizeof(Real)),
                     st, d, a, (const Real*)w.Nh, (const Real*)w.qbar, X, (Real*)w.Ehist, w.LYhist, (Real*)w.Q,
                     Eout);
  return hipGetLastError();
}

template <typename Real>
hipError_t run_stage(const GridPlan& g, Work& w, const StageArgs& a, double* X, int n_slices, double* Eout,
                     hipStream_t st) {
  switch (g.dev.MT) {
    case 2: return run_stage_mt<Real, 2>(g, w, a, X, n_slices, Eout, st);
    case 4: return run_stage_mt<Real, 4>(g, w, a, X, n_slices, Eout, st);
    case 6: return run_stage_mt<Real, 6>(g, w, a, X, n_slices, Eout, st);
    case 8: return run_stage_mt<Real, 8>(g, w, a, X, n_slices, Eout, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t run_xpass(const GridPlan& g, Work& w, int n_slices, hipStream_t st) {
  const GridDev& d = g.dev;
  hipLaunchKernelGGL(xpass_kernel<Real>, dim3(n_slices * d.Pz), dim3(kBlock), xpass_lds(d, sizeof(Real)), st,
                     d, (const Real*)w.Q, (Real*)w.Nh, (Real*)w.qbar);
  return hipGetLastError();
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
hipError_t steps_impl(const GridPlan& g, Work& w, double* X, int n_slices, int n_steps, double* nu_out,
                      int nu_stride, int nu_ld, hipStream_t st, KernelTiming* tm) {
  if (n_steps <= 0) return hipSuccess;
  const Tableau& tb = g.tab;
  StageArgs a{};
  a.mode = kModeZinv;
  a.do_zinv = 1;
  a.cap = w.cap;
  a.s = tb.s;
  hipError_t e = run_stage<Real>(g, w, a, X, n_slices, nullptr, st);
  if (e != hipSuccess) return e;
  int sample = 0;
  for (int step = 0; step < n_steps; ++step) {
    const bool last = (step == n_steps - 1);
    const bool timed = tm && tm->every > 0 && step % tm->every == 0 &&
                       tm->used + 2 * tb.s <= 2 * KernelTiming::kMaxPairs;
    for (int i = 1; i <= tb.s; ++i) {
      if (timed && tm->kernel == 1 && (e = timing_mark(tm, st)) != hipSuccess) return e;
      if ((e = run_xpass<Real>(g, w, n_slices, st)) != hipSuccess) return e;
      if (timed && tm->kernel == 1 && (e = timing_mark(tm, st)) != hipSuccess) return e;
      StageArgs b{};
      b.mode = kModeStage;
      b.stage = i;
      b.s = tb.s;
      b.cap = w.cap;
      b.store_E = (i < tb.s);
      b.store_LY = (i < tb.s);
      b.write_X = (i == tb.s);
      b.do_zinv = !(last && i == tb.s);
      for (int j = 0; j < i; ++j) b.hae[j] = g.dt * tb.ae[i][j];
      for (int j = 1; j <= i; ++j) b.hai[j] = g.dt * tb.ai[i][j];
      b.haii = g.dt * tb.ai[i][i];
      if (timed && tm->kernel == 0 && (e = timing_mark(tm, st)) != hipSuccess) return e;
      if ((e = run_stage<Real>(g, w, b, X, n_slices, nullptr, st)) != hipSuccess) return e;
      if (timed && tm->kernel == 0 && (e = timing_mark(tm, st)) != hipSuccess) return e;
    }
    if (nu_out && nu_stride > 0 && (step + 1) % nu_stride == 0) {
      hipLaunchKernelGGL(nusselt_kernel, dim3(n_slices), dim3(kBlock), 0, st, g.dev, X,
                         nu_out + size_t(sample) * 3, nu_ld * 3);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      ++sample;
    }
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_steps(const GridPlan& g, Work& w, double* X, int n_slices, int n_steps, double* nu_out,
                        int nu_stride, int nu_ld, hipStream_t st, KernelTiming* tm) {
  if (g.mixed) return steps_impl<float>(g, w, X, n_slices, n_steps, nu_out, nu_stride, nu_ld, st, tm);
  return steps_impl<double>(g, w, X, n_slices, n_steps, nu_out, nu_stride, nu_ld, st, tm);
}

hipError_t launch_explicit(const GridPlan& g, Work& w, const double* X, double* E, hipStream_t st) {
  StageArgs a{};
  a.mode = kModeZinv;
  a.do_zinv = 1;
  a.cap = w.cap;
  a.s = g.tab.s;
  hipError_t e;
  double* Xm = const_cast<double*>(X);
  if (g.mixed) {
    if ((e = run_stage<float>(g, w, a, Xm, 1, nullptr, st)) != hipSuccess) return e;
    if ((e = run_xpass<float>(g, w, 1, st)) != hipSuccess) return e;
    a.mode = kModeExplicit;
    return run_stage<float>(g, w, a, Xm, 1, E, st);
  }
  if ((e = run_stage<double>(g, w, a, Xm, 1, nullptr, st)) != hipSuccess) return e;
  if ((e = run_xpass<double>(g, w, 1, st)) != hipSuccess) return e;
  a.mode = kModeExplicit;
  return run_stage<double>(g, w, a, Xm, 1, E, st);
}

hipError_t launch_nusselt(const GridPlan& g, const double* X, int n, double* out, int ld3, hipStream_t st) {
  hipLaunchKernelGGL(nusselt_kernel, dim3(n), dim3(kBlock), 0, st, g.dev, X, out, ld3);
  return hipGetLastError();
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
