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
// (reference circle, local frame, arc lengths, and the final parameters)
// runs in FP64, where it costs a few dozen operations per hit; the
// residuals, hit errors and multiple-scattering widths are stored in the
// working precision.  The transverse system (N + 1 unknowns) is factorised
// and solved in FP32, Jacobi-scaled, and refined once against its residual
// computed in FP64, which restores FP64-level parameters at any pT for
// systems that are not ill-conditioned; the small longitudinal system is
// solved in FP64.  Tuples whose transverse Cholesky pivot ratio falls below
// 2^-12, whose result is not finite, or whose reference pT exceeds pt_fp64
// (a configuration option, off by default) are refitted with the same code
// in FP64 throughout.  The covariance Jacobian of (phi0, d0, q/pT) w.r.t.
// (u0, u1, dk) and that of (cot theta, z0) w.r.t. (w0, w1) are written out
// by the chain rule.
#pragma once

#include "common.h"

namespace pxt {

// ------------------------------------------------------------ geometry --

// T is the fit's working precision: the residuals, hit errors and
// multiple-scattering widths enter only its systems and are stored in T.
template <typename T>
struct FitGeo {
  int n;
  double x0, y0, z0;
  double tx, ty, nx, ny;
  double kref, tref, sinT, cosT;
  double s[kMaxHits], ds[kMaxHits];
  T m[kMaxHits], mz[kMaxHits], sz[kMaxHits], th0[kMaxHits];
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
template <int N, typename T>
__device__ inline void fit_geometry(const DevCfg& c, const float (&Xf)[kMaxHits],
                                    const float (&Yf)[kMaxHits], const float (&Zf)[kMaxHits],
                                    const int (&kind)[kMaxHits], FitGeo<T>& g) {
  constexpr int m = N / 2;
  g.n = N;
  double X[N], Y[N], Z[N];  // the hit coordinates are FP32; differences in FP64 are exact
#pragma unroll
  for (int i = 0; i < N; ++i) {
    X[i] = (double)Xf[i];
    Y[i] = (double)Yf[i];
    Z[i] = (double)Zf[i];
  }
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
  // rotation by asin(sa): cosine sqrt(1 - sa^2) >= 0, sine sa
  const double ca = sqrt(1.0 - sa * sa), sn = sa;
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
    g.m[i] = (T)circ_dist(a, b, k);
    g.s[i] = circ_arc(a, b, k);
  }
  g.tref = (Z[N - 1] - Z[0]) / (g.s[N - 1] - g.s[0]);
  g.sinT = 1.0 / sqrt(1.0 + g.tref * g.tref);
  g.cosT = g.tref * g.sinT;
  const double kabs = fmax(fabs(k), c.c_kappa / c.pt_max);
  const double p = c.c_kappa / (kabs * g.sinT);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const T x = (T)(c.x_over_x0 / (kind[i] == PXT_LAYER_BARREL ? g.sinT : fabs(g.cosT)));
    g.th0[i] = (T)(0.0136 / p) * sqrt(x) * ((T)1 + (T)0.038 * log(x));
    g.sz[i] = (T)(kind[i] == PXT_LAYER_BARREL ? c.sigma_z : c.sigma_r * fabs(g.tref));
    g.mz[i] = (T)(Z[i] - Z[0] - g.tref * (g.s[i] - g.s[0]));
  }
#pragma unroll
  for (int i = 0; i + 1 < N; ++i) g.ds[i] = g.s[i + 1] - g.s[i];
}

// ------------------------------------------------------- linear algebra --

// Cholesky factorisation A = L L^T of the Jacobi-scaled SPD matrix in place,
// in T: the lower triangle receives L, with the reciprocal 1/L_jj stored on
// the diagonal.  Returns the pivot ratio min/max (0 if not positive
// definite).
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
    const T inv = (T)1 / d;
    A[j][j] = inv;
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
    b[i] = t * L[i][i];
  }
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
    T t = b[i];
#pragma unroll
    for (int k = i + 1; k < K; ++k) t -= L[k][i] * b[k];
    b[i] = t * L[i][i];
  }
}

// ------------------------------------------- point of closest approach --

// sin and cos of an angle that is almost always small (the fitted slope
// against the reference tangent): Taylor series to the 8th order below 1/32
// (truncation below 2^-60 relative), the library otherwise.
__device__ __forceinline__ void small_sincos(double x, double& s, double& c) {
  if (fabs(x) < 0.03125) {
    const double x2 = x * x;
    s = x * (1.0 - x2 / 6.0 * (1.0 - x2 / 20.0 * (1.0 - x2 / 42.0 * (1.0 - x2 / 72.0))));
    c = 1.0 - x2 / 2.0 * (1.0 - x2 / 12.0 * (1.0 - x2 / 30.0 * (1.0 - x2 / 56.0)));
  } else {
    sincos(x, &s, &c);
  }
}

// atan2 in the precision of the fit: the angles it gives (the direction and
// turning angle at the point of closest approach) need 1e-7 absolute only.
template <typename D>
__device__ __forceinline__ double atan2_in(double y, double x) {
  if constexpr (sizeof(D) == sizeof(float))
    return (double)atan2f((float)y, (float)x);
  else
    return atan2(y, x);
}

// Transverse parameters (phi0, d0, q/pT) at the point of closest approach to
// the beam line, from the fitted offsets u0, u1 of the first two hits and the
// curvature correction dk, in FP64; their Jacobian J[a][p] with respect to
// (u0, u1, dk) in D (FP32 for the single-precision fits: it only feeds the
// covariance, which is output in FP32), written out by the chain rule;
// spca = arc length from the first hit to that point.
//
// The track leaves the first hit P (on the reference circle's normal at u0)
// in direction c, the reference tangent turned by the fitted slope.  In the
// frame of P and c the origin sits at (aO, bO); d0 is its signed distance
// from the circle of curvature kap, and th = kap * spca the angle the track
// turns through between the two points.
template <typename D>
__device__ inline void pca_transverse(const DevCfg& c, const FitGeo<D>& g, double u0, double u1,
                                      double dk, double (&val)[3], D (&J)[3][3],
                                      double& spca) {
  const double kap = g.kref + dk;
  const double Px = g.x0 + u0 * g.nx, Py = g.y0 + u0 * g.ny;
  const double slope = (u1 - u0) * (1.0 / g.ds[0]) - dk * (g.ds[0] / 2.0);
  double ss, cs;
  small_sincos(slope, ss, cs);
  const double cx = g.tx * cs - g.ty * ss, cy = g.ty * cs + g.tx * ss;
  const double aO = -(Px * cx) - Py * cy;
  const double bO = Px * cy - Py * cx;
  const double q = aO * aO + bO * bO;
  const double r = sqrt(1.0 - 2.0 * (kap * bO) + kap * kap * q);
  const double den = 1.0 + r;
  const double d0 = (2.0 * bO - kap * q) / den;
  const double Yv = kap * aO, Xv = 1.0 - kap * bO;
  const double th = atan2_in<D>(Yv, Xv);
  spca = kap == 0.0 ? aO : th / kap;
  double phi0 = atan2_in<D>(cy, cx) + th;
  const double pi = 3.141592653589793;
  if (phi0 > pi) phi0 -= 2.0 * pi;
  else if (phi0 <= -pi) phi0 += 2.0 * pi;
  val[0] = phi0;
  val[1] = d0;
  val[2] = -kap / c.c_kappa;
  // Jacobian: d slope / d(u0, u1, dk), dP / du0 = (nx, ny), dc = (-cy, cx) d slope
  const D dsl[3] = {(D)(-1.0 / g.ds[0]), (D)(1.0 / g.ds[0]), (D)(-g.ds[0] / 2.0)};
  const D fa = (D)aO, fb = (D)bO, fcx = (D)cx, fcy = (D)cy, fk = (D)kap, fq = (D)q;
  const D fd0 = (D)d0, i2r = (D)(0.5 / r), iden = (D)(1.0 / den);
  const D fX = (D)Xv, fY = (D)Yv, iR2 = (D)(1.0 / (Xv * Xv + Yv * Yv));
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const D dPx = p == 0 ? (D)g.nx : (D)0, dPy = p == 0 ? (D)g.ny : (D)0;
    const D dkap = p == 2 ? (D)1 : (D)0;
    const D daO = -(dPx * fcx + dPy * fcy) + fb * dsl[p];
    const D dbO = (dPx * fcy - dPy * fcx) - fa * dsl[p];
    const D dq = (D)2 * (fa * daO + fb * dbO);
    const D dnum = (D)2 * dbO - dkap * fq - fk * dq;
    const D dr = ((D)-2 * (dkap * fb + fk * dbO) + (D)2 * fk * dkap * fq + fk * fk * dq) * i2r;
    J[1][p] = (dnum - fd0 * dr) * iden;
    const D dY = dkap * fa + fk * daO, dX = -(dkap * fb + fk * dbO);
    J[0][p] = dsl[p] + (fX * dY - fY * dX) * iR2;
    J[2][p] = p == 2 ? (D)(-1.0 / c.c_kappa) : (D)0;
  }
}

__device__ __forceinline__ int tri(int a, int b) { return a * (a + 1) / 2 + b; }

// Results of one fit: the parameters and chi2 are kept (the quality flags
// are derived from them); the 15 covariance terms go straight to `cov`
// (lower triangle, row by row) as they are computed.
struct FitOut {
  float params[5];
  float* cov;
  float chi2[2];
  bool need64;
};

// Lower triangle of the trailing M x M block of (L L^T)^-1 for a Cholesky
// factor L: with L = [[L11, 0], [L21, L22]] that block is (L22 L22^T)^-1 =
// L22^-T L22^-1, so only the trailing block of L is inverted.
template <int K, int M, typename T>
__device__ __forceinline__ void tail_inverse(const T (&L)[K][K], T (&C)[M * (M + 1) / 2]) {
  constexpr int B = K - M;
  T Mi[M][M];  // L22^-1, lower triangular
#pragma unroll
  for (int j = 0; j < M; ++j) {
    Mi[j][j] = L[B + j][B + j];
#pragma unroll
    for (int i = j + 1; i < M; ++i) {
      T t = (T)0;
#pragma unroll
      for (int k = j; k < i; ++k) t -= L[B + i][B + k] * Mi[k][j];
      Mi[i][j] = t * L[B + i][B + i];
    }
  }
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T t = (T)0;
#pragma unroll
      for (int k = i; k < M; ++k) t += Mi[k][i] * Mi[k][j];
      C[tri(i, j)] = t;
    }
}

// Place of unknown i (0..N-1) in the elimination order of a fit of N hits:
// the unknowns of the hits from the third on come first, those of the first
// two hits last (followed only by the curvature correction, place N), so that
// the covariance of the first two is the trailing block of the inverse.
template <int N>
__device__ constexpr int elim_pos(int i) {
  return i >= 2 ? i - 2 : N - 2 + i;
}

// Fit with the linear algebra in T for a tuple of exactly N hits.
//
// Both systems are solved with the unknowns in elimination order (elim_pos),
// so that the covariance of the parameters at the first two hits, which the
// track covariance needs, is the trailing block of the inverse.
// The normal matrices are built directly in their Jacobi-scaled form
// As = D A D with D = diag(A)^-1/2 (the scaled diagonal is exactly 1): the
// diagonal of A is accumulated in FP64 first, then every kink adds its
// rank-one term, scaled, to the working-precision matrix.  The kink
// coefficients are recomputed rather than stored, to keep registers low.
template <int N, typename T>
__device__ inline void fit_linear(const DevCfg& c, const FitGeo<T>& g, FitOut& o) {
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
  }
#pragma unroll
  for (int i = 0; i < N; ++i) y[elim_pos<N>(i)] = (T)(wu * g.m[i] * Dg[i]);
  y[N] = (T)0;
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT / g.th0[j];
    const double v = w * w;
    const int idx[4] = {elim_pos<N>(j - 1), elim_pos<N>(j), elim_pos<N>(j + 1), N};
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
  double yd[K];
#pragma unroll
  for (int i = 0; i < K; ++i) yd[i] = (double)y[i];
  if constexpr (sizeof(T) < sizeof(double)) {
    // one step of iterative refinement: the residual of the scaled system
    // in FP64 (its off-diagonal entries recomputed from the kinks, unrounded),
    // corrected with the FP32 factor
    double r[K];
#pragma unroll
    for (int i = 0; i < N; ++i) r[elim_pos<N>(i)] = wu * (double)g.m[i] * Dg[i];
    r[N] = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) r[i] -= yd[i];
#pragma unroll
    for (int j = 1; j + 1 < N; ++j) {
      const double w = g.sinT / g.th0[j];
      const double v = w * w;
      const int idx[4] = {elim_pos<N>(j - 1), elim_pos<N>(j), elim_pos<N>(j + 1), N};
      const double cf[4] = {inv_ds[j - 1] * Dg[j - 1], -(inv_ds[j - 1] + inv_ds[j]) * Dg[j],
                            inv_ds[j] * Dg[j + 1], -(g.ds[j - 1] + g.ds[j]) / 2.0 * Dg[N]};
      double sk = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) sk += cf[q] * yd[idx[q]];
#pragma unroll
      for (int p = 0; p < 4; ++p) r[idx[p]] -= v * cf[p] * (sk - cf[p] * yd[idx[p]]);
    }
    T rr[K];
#pragma unroll
    for (int i = 0; i < K; ++i) rr[i] = (T)r[i];
    chol_solve<K, T>(As, rr);
#pragma unroll
    for (int i = 0; i < K; ++i) yd[i] += (double)rr[i];
  }
  double x[K];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = yd[elim_pos<N>(i)] * Dg[i];
  x[N] = yd[N] * Dg[N];
  // (u0, u1, dk) covariance, lower triangle
  T C3[6];
  {
    T Cs[6];
    tail_inverse<K, 3, T>(As, Cs);
    const int vi[3] = {0, 1, N};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b)
        C3[tri(a, b)] = (T)(Dg[vi[a]] * (double)Cs[tri(a, b)] * Dg[vi[b]]);
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
  // transverse parameters at the point of closest approach (FP64 values)
  // and their covariance block J C3 J^T (in T)
  double tv[3];
  T J[3][3];
  double spca;
  pca_transverse<T>(c, g, x[0], x[1], x[N], tv, J, spca);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T jc[3];  // row a of J C3
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      T s = (T)0;
#pragma unroll
      for (int p = 0; p < 3; ++p) s += J[a][p] * C3[p >= q ? tri(p, q) : tri(q, p)];
      jc[q] = s;
    }
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      T s = (T)0;
#pragma unroll
      for (int q = 0; q < 3; ++q) s += jc[q] * J[b][q];
      o.cov[tri(a, b)] = (float)s;
    }
  }
  o.params[0] = (float)tv[0];
  o.params[1] = (float)tv[1];
  o.params[2] = (float)tv[2];
  o.chi2[0] = (float)chic;
  bool bad = !((double)pr >= 1.0 / 4096.0);  // pivot ratio below 2^-12
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
  double Bs[N][N];  // the longitudinal system is small: FP64
  double yz[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) Bs[i][j] = 0.0;
    Bs[i][i] = 1.0;
    yz[elim_pos<N>(i)] = (double)g.mz[i] / ((double)g.sz[i] * (double)g.sz[i]) * Dz[i];
  }
#pragma unroll
  for (int j = 1; j + 1 < N; ++j) {
    const double w = g.sinT * g.sinT / g.th0[j];
    const double v = w * w;
    const int idx[3] = {elim_pos<N>(j - 1), elim_pos<N>(j), elim_pos<N>(j + 1)};
    const double cf[3] = {inv_ds[j - 1] * Dz[j - 1], -(inv_ds[j - 1] + inv_ds[j]) * Dz[j],
                          inv_ds[j] * Dz[j + 1]};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (p != q) Bs[idx[p]][idx[q]] += v * cf[p] * cf[q];
  }
  cholesky<N, double>(Bs);
  chol_solve<N, double>(Bs, yz);
  double wv[N];
#pragma unroll
  for (int i = 0; i < N; ++i) wv[i] = yz[elim_pos<N>(i)] * Dz[i];
  // (w0, w1) covariance, lower triangle
  T CL[3];
  {
    double Cs[3];
    tail_inverse<N, 2, double>(Bs, Cs);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) CL[tri(a, b)] = (T)(Dz[a] * Cs[tri(a, b)] * Dz[b]);
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
  const double cot = g.tref + (wv[1] - wv[0]) / g.ds[0];
  const double z0 = g.z0 + wv[0] + cot * spca;
  // longitudinal block JL CL JL^T; the blocks do not correlate
  const T JL[2][2] = {{(T)(-1.0 / g.ds[0]), (T)(1.0 / g.ds[0])},
                      {(T)(1.0 - spca / g.ds[0]), (T)(spca / g.ds[0])}};
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b) o.cov[tri(3 + a, b)] = 0.0f;
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      T s = (T)0;
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) s += JL[a][p] * CL[p >= q ? tri(p, q) : tri(q, p)] * JL[b][q];
      o.cov[tri(3 + a, 3 + b)] = (float)s;
    }
  }
  o.params[3] = (float)cot;
  o.params[4] = (float)z0;
  o.chi2[1] = (float)chiz;
#pragma unroll
  for (int i = 0; i < 5; ++i) bad |= !isfinite(o.params[i]);
  bad |= fabs(g.kref) < c.c_kappa / c.pt_fp64;
  o.need64 = bad;
}

template <int N, typename T>
__device__ inline void fit_n(const DevCfg& c, const float (&X)[kMaxHits],
                             const float (&Y)[kMaxHits], const float (&Z)[kMaxHits],
                             const int (&kind)[kMaxHits], FitOut& o) {
  FitGeo<T> g;
  fit_geometry<N, T>(c, X, Y, Z, kind, g);
  fit_linear<N, T>(c, g, o);
}

// Fit a tuple of n hits (3..8) given in path order.
template <typename T>
__device__ inline void fit_tuple(const DevCfg& c, int n, const float (&X)[kMaxHits],
                                 const float (&Y)[kMaxHits], const float (&Z)[kMaxHits],
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
