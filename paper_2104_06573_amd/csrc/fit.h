// Broken-line helix fit of one n-tuplet per thread.
//
// The paper's Tracks module fits each hit n-tuplet to obtain the track
// parameters (Sec. 2) with small dense matrices (Eigen in the original code,
// the track covariance being its only multi-dimensional array, Sec. 4.2).
// This library's reading is a one-pass linearised broken-line fit (Blobel,
// NIM A 566 (2006) 14) about a reference circle through the first, middle
// and last hits:
//
//  transverse  unknowns u_0..u_{n-1} (offsets from the reference circle,
//              positive to the left) and dk (curvature correction);
//              chi2 = sum (m_i - u_i)^2 / su^2 + sum beta_j^2 / sb_j^2 with
//              the kink beta_j = (u_{j+1}-u_j)/ds_j - (u_j-u_{j-1})/ds_{j-1}
//              - dk (ds_{j-1} + ds_j) / 2 and sb_j = theta0_j / sin(theta);
//  longitudinal unknowns w_0..w_{n-1} in arc length vs z, kinks without the
//              curvature term and sb_j = theta0_j / sin^2(theta);
//  theta0      Highland with beta = 1 and x = X/X0 / sin(theta) (barrel)
//              or / |cos(theta)| (disk); p from the reference curvature.
//
// Precision split for gfx950: the geometry that differences coordinates
// (reference circle, local frame, residuals, arc lengths, and the final
// parameters) runs in FP64, where it costs a few dozen operations per hit;
// the small-matrix work (normal equations, Cholesky, inversion, covariance
// propagation) runs in FP32 registers, Jacobi-scaled.  Tuples whose
// reference pT exceeds pt_fp64, whose Cholesky pivot ratio falls below 2^-12,
// or whose FP32 result is not finite are refitted with the same code in FP64.
// The covariance Jacobian of (phi0, d0, q/pT) w.r.t. (u0, u1, dk) is exact,
// by forward-mode dual numbers; that of (cot theta, z0) w.r.t. (w0, w1) is
// written out.
#pragma once

#include "common.h"

namespace pxt {

// ------------------------------------------------------------ geometry --

struct FitGeo {
  int n;
  double x0, y0, z0;
  double tx, ty, nx, ny;
  double kref, tref, sinT, cosT;
  double m[kMaxHits], s[kMaxHits], mz[kMaxHits], th0[kMaxHits], sz[kMaxHits];
  double ds[kMaxHits];
};

// Signed distance of local (a, b) from the circle of curvature k through the
// local origin with tangent +a (positive to the left); exact as k -> 0.
__device__ __forceinline__ double circ_dist(double a, double b, double k) {
  const double q = a * a + b * b;
  return (2.0 * b - k * q) / (1.0 + sqrt(1.0 - 2.0 * k * b + k * k * q));
}

__device__ __forceinline__ double circ_arc(double a, double b, double k) {
  return k == 0.0 ? a : atan2(k * a, 1.0 - k * b) / k;
}

// N is the number of hits, a compile-time constant so that every array index
// is static and the arrays stay in registers.
template <int N>
__device__ inline void fit_geometry(const DevCfg& c, const double (&X)[kMaxHits],
                                    const double (&Y)[kMaxHits], const double (&Z)[kMaxHits],
                                    const int (&kind)[kMaxHits], FitGeo& g) {
  constexpr int m = N / 2;
  g.n = N;
  const double d1x = X[m] - X[0], d1y = Y[m] - Y[0];
  const double d2x = X[N - 1] - X[0], d2y = Y[N - 1] - Y[0];
  const double d3x = X[N - 1] - X[m], d3y = Y[N - 1] - Y[m];
  const double cr = d1x * d2y - d1y * d2x;
  const double l1 = sqrt(d1x * d1x + d1y * d1y);
  const double l2 = sqrt(d2x * d2x + d2y * d2y);
  const double l3 = sqrt(d3x * d3x + d3y * d3y);
  const double k = 2.0 * cr / (l1 * l2 * l3);
  const double chx = d2x / l2, chy = d2y / l2;
  double sa = k * l2 / 2.0;
  sa = fmin(1.0, fmax(-1.0, sa));
  const double al = asin(sa);
  const double ca = cos(al), sn = sin(al);
  g.tx = chx * ca + chy * sn;
  g.ty = -chx * sn + chy * ca;
  g.nx = -g.ty;
  g.ny = g.tx;
  g.x0 = X[0]; g.y0 = Y[0]; g.z0 = Z[0];
  g.kref = k;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double ex = X[i] - X[0], ey = Y[i] - Y[0];
    const double a = ex * g.tx + ey * g.ty;
    const double b = ex * g.nx + ey * g.ny;
    g.m[i] = circ_dist(a, b, k);
    g.s[i] = circ_arc(a, b, k);
  }
  g.tref = (Z[N - 1] - Z[0]) / (g.s[N - 1] - g.s[0]);
  g.sinT = 1.0 / sqrt(1.0 + g.tref * g.tref);
  g.cosT = g.tref * g.sinT;
  const double kabs = fmax(fabs(k), c.c_kappa / c.pt_max);
  const double p = c.c_kappa / (kabs * g.sinT);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double x = c.x_over_x0 / (kind[i] == PXT_LAYER_BARREL ? g.sinT : fabs(g.cosT));
    g.th0[i] = 0.0136 / p * sqrt(x) * (1.0 + 0.038 * log(x));
    g.sz[i] = kind[i] == PXT_LAYER_BARREL ? c.sigma_z : c.sigma_r * fabs(g.tref);
    g.mz[i] = Z[i] - Z[0] - g.tref * (g.s[i] - g.s[0]);
  }
#pragma unroll
  for (int i = 0; i + 1 < N; ++i) g.ds[i] = g.s[i + 1] - g.s[i];
}

// ------------------------------------------------------- linear algebra --

// Solve the Jacobi-scaled SPD system As y = b in place of b by Cholesky in T.
// Returns the pivot ratio min/max (0 if not positive definite).
template <int K, typename T>
__device__ __forceinline__ T cholesky(T (&A)[K][K]) {
  T pmin = (T)1e30, pmax = (T)0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    T s = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= A[j][k] * A[j][k];
    pmin = s < pmin ? s : pmin;
    pmax = s > pmax ? s : pmax;
    const T d = s > (T)0 ? sqrt(s) : (T)1;
    A[j][j] = d;
    const T inv = (T)1 / d;
#pragma unroll
    for (int i = j + 1; i < K; ++i) {
      T t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= A[i][k] * A[j][k];
      A[i][j] = t * inv;
    }
  }
  return pmin > (T)0 ? pmin / pmax : (T)0;
}

template <int K, typename T>
__device__ __forceinline__ void chol_solve(const T (&L)[K][K], T (&b)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    T t = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[i][k] * b[k];
    b[i] = t / L[i][i];
  }
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
    T t = b[i];
#pragma unroll
    for (int k = i + 1; k < K; ++k) t -= L[k][i] * b[k];
    b[i] = t / L[i][i];
  }
}

// ---------------------------------------------------------- dual numbers --

struct Dual3 {
  double v, d[3];
};
__device__ __forceinline__ Dual3 dconst(double v) { return {v, {0.0, 0.0, 0.0}}; }
__device__ __forceinline__ Dual3 dvar(double v, int i) {
  Dual3 r = dconst(v);
  r.d[i] = 1.0;
  return r;
}
__device__ __forceinline__ Dual3 operator+(Dual3 a, Dual3 b) {
  return {a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
__device__ __forceinline__ Dual3 operator-(Dual3 a, Dual3 b) {
  return {a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
__device__ __forceinline__ Dual3 operator-(Dual3 a) { return {-a.v, {-a.d[0], -a.d[1], -a.d[2]}}; }
__device__ __forceinline__ Dual3 operator*(Dual3 a, Dual3 b) {
  return {a.v * b.v,
          {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1], a.d[2] * b.v + a.v * b.d[2]}};
}
__device__ __forceinline__ Dual3 operator*(double s, Dual3 a) {
  return {s * a.v, {s * a.d[0], s * a.d[1], s * a.d[2]}};
}
__device__ __forceinline__ Dual3 operator/(Dual3 a, Dual3 b) {
  const double iv = 1.0 / b.v;
  const double q = a.v * iv;
  return {q, {(a.d[0] - q * b.d[0]) * iv, (a.d[1] - q * b.d[1]) * iv, (a.d[2] - q * b.d[2]) * iv}};
}
__device__ __forceinline__ Dual3 dscale(Dual3 a, double s) { return s * a; }
__device__ __forceinline__ Dual3 dsqrt(Dual3 a) {
  const double r = sqrt(a.v);
  const double f = 0.5 / r;
  return {r, {f * a.d[0], f * a.d[1], f * a.d[2]}};
}
__device__ __forceinline__ Dual3 dsin(Dual3 a) {
  const double c = cos(a.v);
  return {sin(a.v), {c * a.d[0], c * a.d[1], c * a.d[2]}};
}
__device__ __forceinline__ Dual3 dcos(Dual3 a) {
  const double s = -sin(a.v);
  return {cos(a.v), {s * a.d[0], s * a.d[1], s * a.d[2]}};
}
__device__ __forceinline__ Dual3 datan2(Dual3 y, Dual3 x) {
  const double r2 = x.v * x.v + y.v * y.v;
  const double fy = x.v / r2, fx = -y.v / r2;
  return {atan2(y.v, x.v),
          {fy * y.d[0] + fx * x.d[0], fy * y.d[1] + fx * x.d[1], fy * y.d[2] + fx * x.d[2]}};
}

// Transverse parameters (phi0, d0, q/pT) at the point of closest approach,
// with derivatives w.r.t. (u0, u1, dk); spca = arc length to it.
__device__ inline void pca_transverse(const DevCfg& c, const FitGeo& g, double u0v,
                                      double u1v, double dkv, Dual3 out[3],
                                      double& spca) {
  const Dual3 u0 = dvar(u0v, 0), u1 = dvar(u1v, 1), dk = dvar(dkv, 2);
  const Dual3 kap = dconst(g.kref) + dk;
  const Dual3 Px = dconst(g.x0) + dscale(u0, g.nx);
  const Dual3 Py = dconst(g.y0) + dscale(u0, g.ny);
  const Dual3 slope = dscale(u1 - u0, 1.0 / g.ds[0]) - dscale(dk, g.ds[0] / 2.0);
  const Dual3 phis = dconst(atan2(g.ty, g.tx)) + slope;
  const Dual3 ctx = dcos(phis), cty = dsin(phis);
  const Dual3 aO = -(Px * ctx) - Py * cty;
  const Dual3 bO = Px * cty - Py * ctx;
  const Dual3 q = aO * aO + bO * bO;
  const Dual3 d0 = (dscale(bO, 2.0) - kap * q) /
                   (dconst(1.0) + dsqrt(dconst(1.0) - dscale(kap * bO, 2.0) + kap * kap * q));
  Dual3 sp;
  if (kap.v == 0.0) sp = aO;
  else sp = datan2(kap * aO, dconst(1.0) - kap * bO) / kap;
  Dual3 phi0 = phis + kap * sp;
  phi0.v = atan2(sin(phi0.v), cos(phi0.v));
  out[0] = phi0;
  out[1] = d0;
  out[2] = dscale(kap, -1.0 / c.c_kappa);
  spca = sp.v;
}

__device__ __forceinline__ int tri(int a, int b) { return a * (a + 1) / 2 + b; }

struct FitOut {
  float params[5];
  float cov[15];
  float chi2[2];
  bool need64;
};

// Fit with the linear algebra in T for a tuple of exactly N hits.
//
// The normal matrices are built directly in their Jacobi-scaled form
// As = D A D with D = diag(A)^-1/2 (the scaled diagonal is exactly 1): the
// diagonal of A is accumulated in FP64 first, then every kink adds its
// rank-one term, scaled, to the working-precision matrix.  The kink
// coefficients are recomputed rather than stored, to keep registers low.
template <int N, typename T>
__device__ inline void fit_linear(const DevCfg& c, const FitGeo& g, FitOut& o) {
  constexpr int K = N + 1;
  // ---- transverse: unknowns u_0..u_{N-1}, dk
  const double wu = 1.0 / (c.sigma_u * c.sigma_u);
  double inv_ds[N - 1];
#pragma unroll
  for (int i = 0; i + 1 < N; ++i) inv_ds[i] = 1.0 / g.ds[i];
  double Dg[K];
#pragma unroll
  for (int i = 0; i < N; ++i) Dg[i] = wu;
  Dg[N] = 0.0;
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT / g.th0[j];
    const double v = w * w;
    const double c0 = inv_ds[j - 1], c1 = -(inv_ds[j - 1] + inv_ds[j]), c2 = inv_ds[j];
    const double c3 = -(g.ds[j - 1] + g.ds[j]) / 2.0;
    Dg[j - 1] += v * c0 * c0;
    Dg[j] += v * c1 * c1;
    Dg[j + 1] += v * c2 * c2;
    Dg[N] += v * c3 * c3;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) Dg[i] = 1.0 / sqrt(Dg[i]);
  T As[K][K];
  T y[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
#pragma unroll
    for (int j = 0; j < K; ++j) As[i][j] = (T)0;
    As[i][i] = (T)1;
    y[i] = i < N ? (T)(wu * g.m[i] * Dg[i]) : (T)0;
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT / g.th0[j];
    const double v = w * w;
    const int idx[4] = {j - 1, j, j + 1, N};
    const double cf[4] = {inv_ds[j - 1] * Dg[j - 1], -(inv_ds[j - 1] + inv_ds[j]) * Dg[j],
                          inv_ds[j] * Dg[j + 1], -(g.ds[j - 1] + g.ds[j]) / 2.0 * Dg[N]};
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (p != q) As[idx[p]][idx[q]] += (T)(v * cf[p] * cf[q]);
  }
  const T pr = cholesky<K, T>(As);
  chol_solve<K, T>(As, y);
  double x[K];
#pragma unroll
  for (int i = 0; i < K; ++i) x[i] = (double)y[i] * Dg[i];
  // inverse-matrix block on (u0, u1, dk)
  const int vi[3] = {0, 1, N};
  double C3[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T e[K];
#pragma unroll
    for (int i = 0; i < K; ++i) e[i] = (T)0;
    e[vi[a]] = (T)1;
    chol_solve<K, T>(As, e);
#pragma unroll
    for (int b = 0; b < 3; ++b) C3[b][a] = Dg[vi[b]] * (double)e[vi[b]] * Dg[vi[a]];
  }
  // chi2 at the solution (FP64 accumulation)
  double chic = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) chic += wu * (g.m[i] - x[i]) * (g.m[i] - x[i]);
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT / g.th0[j];
    const double beta = (x[j + 1] - x[j]) * inv_ds[j] - (x[j] - x[j - 1]) * inv_ds[j - 1] -
                        x[N] * (g.ds[j - 1] + g.ds[j]) / 2.0;
    chic += w * w * beta * beta;
  }
  // ---- longitudinal: unknowns w_0..w_{N-1}
  double Dz[N];
#pragma unroll
  for (int i = 0; i < N; ++i) Dz[i] = 1.0 / (g.sz[i] * g.sz[i]);
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT * g.sinT / g.th0[j];
    const double v = w * w;
    const double c0 = inv_ds[j - 1], c1 = -(inv_ds[j - 1] + inv_ds[j]), c2 = inv_ds[j];
    Dz[j - 1] += v * c0 * c0;
    Dz[j] += v * c1 * c1;
    Dz[j + 1] += v * c2 * c2;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) Dz[i] = 1.0 / sqrt(Dz[i]);
  T Bs[N][N];
  T yz[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) Bs[i][j] = (T)0;
    Bs[i][i] = (T)1;
    yz[i] = (T)(g.mz[i] / (g.sz[i] * g.sz[i]) * Dz[i]);
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT * g.sinT / g.th0[j];
    const double v = w * w;
    const int idx[3] = {j - 1, j, j + 1};
    const double cf[3] = {inv_ds[j - 1] * Dz[j - 1], -(inv_ds[j - 1] + inv_ds[j]) * Dz[j],
                          inv_ds[j] * Dz[j + 1]};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (p != q) Bs[idx[p]][idx[q]] += (T)(v * cf[p] * cf[q]);
  }
  const T prz = cholesky<N, T>(Bs);
  chol_solve<N, T>(Bs, yz);
  double wv[N];
#pragma unroll
  for (int i = 0; i < N; ++i) wv[i] = (double)yz[i] * Dz[i];
  double CL[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    T e[N];
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = (T)0;
    e[a] = (T)1;
    chol_solve<N, T>(Bs, e);
#pragma unroll
    for (int b = 0; b < 2; ++b) CL[b][a] = Dz[b] * (double)e[b] * Dz[a];
  }
  double chiz = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double e = g.mz[i] - wv[i];
    chiz += e * e / (g.sz[i] * g.sz[i]);
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT * g.sinT / g.th0[j];
    const double gam = (wv[j + 1] - wv[j]) * inv_ds[j] - (wv[j] - wv[j - 1]) * inv_ds[j - 1];
    chiz += w * w * gam * gam;
  }
  // ---- parameters at the point of closest approach (FP64)
  Dual3 tp[3];
  double spca;
  pca_transverse(c, g, x[0], x[1], x[N], tp, spca);
  const double cot = g.tref + (wv[1] - wv[0]) / g.ds[0];
  const double z0 = g.z0 + wv[0] + cot * spca;
  // ---- covariance: transverse block J C3 J^T, longitudinal JL CL JL^T
  double cv[5][5];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) cv[a][b] = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) s += tp[a].d[p] * C3[p][q] * tp[b].d[q];
      cv[a][b] = s;
    }
  const double JL[2][2] = {{-1.0 / g.ds[0], 1.0 / g.ds[0]},
                           {1.0 - spca / g.ds[0], spca / g.ds[0]}};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) s += JL[a][p] * CL[p][q] * JL[b][q];
      cv[3 + a][3 + b] = s;
    }
  o.params[0] = (float)tp[0].v;
  o.params[1] = (float)tp[1].v;
  o.params[2] = (float)tp[2].v;
  o.params[3] = (float)cot;
  o.params[4] = (float)z0;
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) o.cov[tri(a, b)] = (float)cv[a][b];
  o.chi2[0] = (float)chic;
  o.chi2[1] = (float)chiz;
  const double pmin = 1.0 / 4096.0;  // 2^-12
  bool bad = !((double)pr >= pmin) || !((double)prz >= pmin);
#pragma unroll
  for (int i = 0; i < 5; ++i) bad |= !isfinite(o.params[i]);
  bad |= fabs(g.kref) < c.c_kappa / c.pt_fp64;
  o.need64 = bad;
}

template <int N, typename T>
__device__ inline void fit_n(const DevCfg& c, const double (&X)[kMaxHits],
                             const double (&Y)[kMaxHits], const double (&Z)[kMaxHits],
                             const int (&kind)[kMaxHits], FitOut& o) {
  FitGeo g;
  fit_geometry<N>(c, X, Y, Z, kind, g);
  fit_linear<N, T>(c, g, o);
}

// Fit a tuple of n hits (3..8) given in path order.
template <typename T>
__device__ inline void fit_tuple(const DevCfg& c, int n, const double (&X)[kMaxHits],
                                 const double (&Y)[kMaxHits], const double (&Z)[kMaxHits],
                                 const int (&kind)[kMaxHits], FitOut& o) {
  switch (n) {
    case 3: fit_n<3, T>(c, X, Y, Z, kind, o); break;
    case 4: fit_n<4, T>(c, X, Y, Z, kind, o); break;
    case 5: fit_n<5, T>(c, X, Y, Z, kind, o); break;
    case 6: fit_n<6, T>(c, X, Y, Z, kind, o); break;
    case 7: fit_n<7, T>(c, X, Y, Z, kind, o); break;
    default: fit_n<8, T>(c, X, Y, Z, kind, o); break;
  }
}

}  // namespace pxt
