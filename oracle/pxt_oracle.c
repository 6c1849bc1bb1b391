/*
 * CPU oracle for the pixel-track reconstruction path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the HIP
 * library: the two are written independently from the same definitions.
 *
 * What it computes is the Tracks module of the paper (Sec. 2: n-tuplets are
 * formed from the hits and fitted to obtain track parameters), split into
 * the steps doublets -> cellular-automaton links -> n-tuplets -> duplicate
 * cleaning -> broken-line fit.  The paper gives no formula for any step, so
 * each step follows an explicit reading, stated beside the code:
 *
 *   doublets  every ordered hit pair on an allowed layer pair that passes
 *             the four geometric cuts D1-D4 (brute force over all pairs);
 *   links     every pair of doublets (a,b),(b,c) sharing hit b that passes
 *             the alignment cuts L1-L3;
 *   tuples    every root-to-leaf path of the link graph with 3..8 hits
 *             (root: a doublet with no inner neighbour; leaf: none outer);
 *   cleaning  per doublet keep only its best tuple under the total order
 *             (more hits, then lower score, then lexicographically smaller
 *             hit tuple); all doublets decide at once;
 *   fit       a one-pass linearised broken-line fit (Blobel, NIM A 566
 *             (2006) 14) about a reference circle through three hits,
 *             separately in the transverse plane and in arc length vs z.
 *
 * Every predicate is evaluated in double precision on single-precision
 * inputs promoted exactly, with the operations in the written order and no
 * contraction into fused multiply-adds (build with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LAYERS 16
#define ORC_MAX_PAIRS 64
#define ORC_MAX_HITS_PER_TUPLE 8
#define ORC_PAD 0xffffffffu

typedef struct {
  double c_kappa;       /* kappa [1/cm] = c_kappa / pT [GeV] */
  int n_layers;
  int layer_kind[ORC_MAX_LAYERS]; /* 0 barrel, 1 disk */
  int n_pairs;
  int pair_inner[ORC_MAX_PAIRS];
  int pair_outer[ORC_MAX_PAIRS];
  double kmax, z0max, arz, d0max;
  double sigma_u, sigma_z, sigma_r, x_over_x0, pt_max;
} orc_config;

enum {
  ORC_OK = 0,
  ORC_ERR_PATH_TOO_LONG = 1,
  ORC_ERR_ALLOC = 2,
};

enum {
  ORC_DOUBLETS = 0,   /* uint32 [n][2]  (inner hit, outer hit)           */
  ORC_LINKS = 1,      /* uint32 [n][3]  (a, b, c)                        */
  ORC_RAW = 2,        /* uint32 [n][8]  hits in path order, padded       */
  ORC_RAW_SCORE = 3,  /* double [n]                                      */
  ORC_KEEP = 4,       /* uint8  [n]     survives cleaning                */
  ORC_TRACKS = 5,     /* uint32 [n][8]  surviving tuples                 */
  ORC_PARAMS = 6,     /* double [n][5]  phi0, d0, q/pT, cot(theta), z0   */
  ORC_COV = 7,        /* double [n][15] packed lower triangle            */
  ORC_CHI2 = 8,       /* double [n][2]  transverse, longitudinal         */
  ORC_KREF = 9,       /* double [n]     reference-circle curvature       */
  ORC_NITEMS = 10,
};

/* ------------------------------------------------------------------ */
/* growable arrays                                                     */

typedef struct {
  void* p;
  uint64_t n, cap;
  size_t esz;
} vec_t;

static int vec_push(vec_t* v, const void* e) {
  if (v->n == v->cap) {
    uint64_t nc = v->cap ? v->cap * 2 : 1024;
    void* np = realloc(v->p, nc * v->esz);
    if (!np) return -1;
    v->p = np;
    v->cap = nc;
  }
  memcpy((char*)v->p + v->n * v->esz, e, v->esz);
  v->n++;
  return 0;
}

struct orc_result {
  int status;
  vec_t item[ORC_NITEMS];
};
typedef struct orc_result orc_result;

/* ------------------------------------------------------------------ */
/* geometric predicates (reading of the doublet and link cuts)         */

static double rad(double x, double y) { return sqrt(x * x + y * y); }

/* D1..D4 for inner hit i and outer hit o. */
int orc_doublet_ok(const orc_config* c, double xi, double yi, double zi,
                   double xo, double yo, double zo) {
  double ri = rad(xi, yi), ro = rad(xo, yo);
  /* D1: the outer hit lies at larger radius */
  if (!(ro > ri)) return 0;
  /* D2: the r-z line through the two hits meets r = 0 within |z| <= z0max */
  double dr = ro - ri;
  double lhs2 = fabs(zi * dr - ri * (zo - zi));
  if (!(lhs2 <= c->z0max * dr)) return 0;
  /* D3: the circle through the origin and both hits has curvature <= kmax */
  double cr = xi * yo - yi * xo;
  double dx = xo - xi, dy = yo - yi;
  double chord = sqrt(dx * dx + dy * dy);
  if (!(2.0 * fabs(cr) <= c->kmax * ri * ro * chord)) return 0;
  /* D4: the two hits lie in the same transverse half plane */
  if (!(xi * xo + yi * yo > 0.0)) return 0;
  return 1;
}

/* Terms of the link cuts for hits a, b, c (in path order).
 * out[0] = |r-z cross|, out[1] = arz * l_ab * l_bc,
 * out[2] = 2 |transverse cross|, out[3] = kmax * |ab| |bc| |ac|,
 * out[4] = transverse impact d0 of the circle through a, b, c. */
void orc_link_terms(const orc_config* c, double xa, double ya, double za,
                    double xb, double yb, double zb, double xc, double yc,
                    double zc, double* out) {
  double ra = rad(xa, ya), rb = rad(xb, yb), rc = rad(xc, yc);
  /* L1: alignment of the two segments in the r-z plane */
  double dra = rb - ra, dza = zb - za, drb = rc - rb, dzb = zc - zb;
  out[0] = fabs(dra * dzb - dza * drb);
  double lab = sqrt(dra * dra + dza * dza);
  double lbc = sqrt(drb * drb + dzb * dzb);
  out[1] = c->arz * lab * lbc;
  /* L2: transverse three-point (Menger) curvature */
  double ux = xb - xa, uy = yb - ya, vx = xc - xa, vy = yc - ya;
  double wx = xc - xb, wy = yc - yb;
  double cr = ux * vy - uy * vx;
  double nab = sqrt(ux * ux + uy * uy);
  double nac = sqrt(vx * vx + vy * vy);
  double nbc = sqrt(wx * wx + wy * wy);
  out[2] = 2.0 * fabs(cr);
  out[3] = c->kmax * nab * nbc * nac;
  /* L3: distance of the origin from the circle through a, b, c; for exactly
   * collinear transverse points, the distance from their line */
  double D = 2.0 * cr;
  if (D == 0.0) {
    out[4] = fabs(xa * vy - ya * vx) / nac;
  } else {
    double uu = ux * ux + uy * uy, vv = vx * vx + vy * vy;
    double ox = (vy * uu - uy * vv) / D;
    double oy = (ux * vv - vx * uu) / D;
    double R = sqrt(ox * ox + oy * oy);
    double cx = xa + ox, cy = ya + oy;
    double dc = sqrt(cx * cx + cy * cy);
    /* |C| - R = (|C|^2 - R^2) / (|C| + R) and |C|^2 - R^2 = |a|^2 + 2 a.o:
     * the same distance without the cancellation of two large radii */
    double aa = xa * xa + ya * ya;
    double ao = xa * ox + ya * oy;
    out[4] = fabs(aa + 2.0 * ao) / (dc + R);
  }
}

int orc_link_ok(const orc_config* c, double xa, double ya, double za,
                double xb, double yb, double zb, double xc, double yc,
                double zc) {
  double t[5];
  orc_link_terms(c, xa, ya, za, xb, yb, zb, xc, yc, zc, t);
  if (!(t[0] <= t[1])) return 0;
  if (!(t[2] <= t[3])) return 0;
  if (!(t[4] <= c->d0max)) return 0;
  return 1;
}

/* Cleaning score of one consecutive hit triple. */
static double triple_score(const orc_config* c, double xa, double ya,
                           double za, double xb, double yb, double zb,
                           double xc, double yc, double zc) {
  double t[5];
  orc_link_terms(c, xa, ya, za, xb, yb, zb, xc, yc, zc, t);
  double q1 = t[0] / t[1];
  double q2 = t[4] / c->d0max;
  return q1 * q1 + q2 * q2;
}

/* ------------------------------------------------------------------ */
/* broken-line fit                                                     */

/* Signed distance of local point (a,b) from the circle of signed curvature
 * k that passes through the local origin with tangent along +a; positive
 * on the left.  The form stays exact as k -> 0. */
static double circ_dist(double a, double b, double k) {
  double q = a * a + b * b;
  return (2.0 * b - k * q) / (1.0 + sqrt(1.0 - 2.0 * k * b + k * k * q));
}

/* Arc length along that circle to the foot of the perpendicular from (a,b). */
static double circ_arc(double a, double b, double k) {
  if (k == 0.0) return a;
  return atan2(k * a, 1.0 - k * b) / k;
}

/* Highland width of the projected scattering angle (beta = 1). */
static double highland(double p, double x) {
  return 0.0136 / p * sqrt(x) * (1.0 + 0.038 * log(x));
}

/* Dense least squares min |A x - y|^2 by Householder QR.  A is m x k
 * (row-major, m <= 32, k <= 16), overwritten.  Writes the solution and
 * the inverse normal matrix (A^T A)^-1. Returns 0 on success. */
static int lsq_qr(int m, int k, double* A, double* y, double* x, double* cov) {
  for (int j = 0; j < k; ++j) {
    double nrm = 0.0;
    for (int i = j; i < m; ++i) nrm += A[i * k + j] * A[i * k + j];
    nrm = sqrt(nrm);
    if (nrm == 0.0) return -1;
    double alpha = A[j * k + j] > 0 ? -nrm : nrm;
    double v[32];
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int i = j; i < m; ++i) v[i] = A[i * k + j];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int c2 = j; c2 < k; ++c2) {
      double s = 0.0;
      for (int i = j; i < m; ++i) s += v[i] * A[i * k + c2];
      s = 2.0 * s / vv;
      for (int i = j; i < m; ++i) A[i * k + c2] -= s * v[i];
    }
    double s = 0.0;
    for (int i = j; i < m; ++i) s += v[i] * y[i];
    s = 2.0 * s / vv;
    for (int i = j; i < m; ++i) y[i] -= s * v[i];
  }
  /* back substitution R x = Q^T y */
  for (int j = k - 1; j >= 0; --j) {
    double s = y[j];
    for (int c2 = j + 1; c2 < k; ++c2) s -= A[j * k + c2] * x[c2];
    if (A[j * k + j] == 0.0) return -1;
    x[j] = s / A[j * k + j];
  }
  /* (A^T A)^-1 = R^-1 R^-T */
  double Ri[16 * 16];
  memset(Ri, 0, sizeof(Ri));
  for (int j = 0; j < k; ++j) {
    Ri[j * k + j] = 1.0 / A[j * k + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += A[i * k + l] * Ri[l * k + j];
      Ri[i * k + j] = -s / A[i * k + i];
    }
  }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += Ri[i * k + l] * Ri[j * k + l];
      cov[i * k + j] = s;
    }
  return 0;
}

/* Helix parameters at the point of closest approach to the transverse
 * origin, from the fitted offsets (u0, u1, dk) about the reference circle
 * and the longitudinal offsets (w0, w1). */
typedef struct {
  double x0, y0, z0;      /* first hit */
  double tx, ty, nx, ny;  /* tangent and left normal at the first hit */
  double kref, ds0, tref, c_kappa;
} fit_frame;

static void pca_params(const fit_frame* f, double u0, double u1, double dk,
                       double w0, double w1, double* out) {
  double kap = f->kref + dk;
  double Px = f->x0 + u0 * f->nx, Py = f->y0 + u0 * f->ny;
  double slope = (u1 - u0) / f->ds0 - dk * f->ds0 / 2.0;
  double phis = atan2(f->ty, f->tx) + slope;
  double ctx = cos(phis), cty = sin(phis);
  double aO = (0.0 - Px) * ctx + (0.0 - Py) * cty;
  double bO = (0.0 - Px) * (-cty) + (0.0 - Py) * ctx;
  double d0 = circ_dist(aO, bO, kap);
  double spca = circ_arc(aO, bO, kap);
  double phi0 = phis + kap * spca;
  /* wrap phi0 into (-pi, pi] */
  phi0 = atan2(sin(phi0), cos(phi0));
  double cot = f->tref + (w1 - w0) / f->ds0;
  double z0 = f->z0 + w0 + cot * spca;
  out[0] = phi0;
  out[1] = d0;
  out[2] = -kap / f->c_kappa;
  out[3] = cot;
  out[4] = z0;
}

/* Fit one tuple of n hits (3 <= n <= 8) given in path order.
 * kind[i] is 0 for a barrel hit, 1 for a disk hit.
 * params[5], cov[15] (packed lower triangle), chi2[2], kref_out (may be 0).
 * Returns 0 on success. */
int orc_fit(const orc_config* c, int n, const double* X, const double* Y,
            const double* Z, const int* kind, double* params, double* cov,
            double* chi2, double* kref_out) {
  if (n < 3 || n > ORC_MAX_HITS_PER_TUPLE) return -1;
  int m = n / 2;
  /* 1. reference circle through the first, middle and last hits */
  double d1x = X[m] - X[0], d1y = Y[m] - Y[0];
  double d2x = X[n - 1] - X[0], d2y = Y[n - 1] - Y[0];
  double d3x = X[n - 1] - X[m], d3y = Y[n - 1] - Y[m];
  double cr = d1x * d2y - d1y * d2x;
  double l1 = rad(d1x, d1y), l2 = rad(d2x, d2y), l3 = rad(d3x, d3y);
  double kref = 2.0 * cr / (l1 * l2 * l3);
  double chx = d2x / l2, chy = d2y / l2;
  double sa = kref * l2 / 2.0;
  if (sa > 1.0) sa = 1.0;
  if (sa < -1.0) sa = -1.0;
  double al = asin(sa);
  double tx = chx * cos(al) + chy * sin(al);
  double ty = -chx * sin(al) + chy * cos(al);
  double nx = -ty, ny = tx;
  /* 2. local frame, residuals about the reference circle, arc lengths */
  double mres[ORC_MAX_HITS_PER_TUPLE], s[ORC_MAX_HITS_PER_TUPLE];
  for (int i = 0; i < n; ++i) {
    double ex = X[i] - X[0], ey = Y[i] - Y[0];
    double a = ex * tx + ey * ty;
    double b = ex * nx + ey * ny;
    mres[i] = circ_dist(a, b, kref);
    s[i] = circ_arc(a, b, kref);
  }
  double tref = (Z[n - 1] - Z[0]) / (s[n - 1] - s[0]);
  double sinT = 1.0 / sqrt(1.0 + tref * tref);
  double cosT = tref * sinT;
  double kabs = fabs(kref);
  if (kabs < c->c_kappa / c->pt_max) kabs = c->c_kappa / c->pt_max;
  double pmom = c->c_kappa / (kabs * sinT);
  double th0[ORC_MAX_HITS_PER_TUPLE], ds[ORC_MAX_HITS_PER_TUPLE];
  for (int i = 0; i + 1 < n; ++i) ds[i] = s[i + 1] - s[i];
  for (int j = 0; j < n; ++j) {
    double x = c->x_over_x0 / (kind[j] == 0 ? sinT : fabs(cosT));
    th0[j] = highland(pmom, x);
  }
  /* 3. transverse system: unknowns u_0..u_{n-1}, dk */
  {
    int k = n + 1, rows = n + (n - 2);
    double A[32 * 16], yv[32], xs[16], C[16 * 16];
    memset(A, 0, sizeof(A));
    for (int i = 0; i < n; ++i) {
      A[i * k + i] = 1.0 / c->sigma_u;
      yv[i] = mres[i] / c->sigma_u;
    }
    for (int j = 1; j <= n - 2; ++j) {
      int r = n + j - 1;
      double w = sinT / th0[j];
      A[r * k + (j + 1)] += w / ds[j];
      A[r * k + j] += w * (-1.0 / ds[j] - 1.0 / ds[j - 1]);
      A[r * k + (j - 1)] += w / ds[j - 1];
      A[r * k + n] += -w * (ds[j - 1] + ds[j]) / 2.0;
      yv[r] = 0.0;
    }
    double Acopy[32 * 16];
    memcpy(Acopy, A, sizeof(A));
    double ycopy[32];
    memcpy(ycopy, yv, sizeof(yv));
    if (lsq_qr(rows, k, A, yv, xs, C)) return -2;
    double chi = 0.0;
    for (int r = 0; r < rows; ++r) {
      double e = -ycopy[r];
      for (int q = 0; q < k; ++q) e += Acopy[r * k + q] * xs[q];
      chi += e * e;
    }
    chi2[0] = chi;
    /* 4. longitudinal system: unknowns w_0..w_{n-1} */
    double mz[ORC_MAX_HITS_PER_TUPLE];
    for (int i = 0; i < n; ++i) mz[i] = Z[i] - Z[0] - tref * (s[i] - s[0]);
    int kz = n, rz = n + (n - 2);
    double B[32 * 16], yz[32], wz[16], Cz[16 * 16];
    memset(B, 0, sizeof(B));
    for (int i = 0; i < n; ++i) {
      double sz = kind[i] == 0 ? c->sigma_z : c->sigma_r * fabs(tref);
      B[i * kz + i] = 1.0 / sz;
      yz[i] = mz[i] / sz;
    }
    for (int j = 1; j <= n - 2; ++j) {
      int r = n + j - 1;
      double w = sinT * sinT / th0[j];
      B[r * kz + (j + 1)] += w / ds[j];
      B[r * kz + j] += w * (-1.0 / ds[j] - 1.0 / ds[j - 1]);
      B[r * kz + (j - 1)] += w / ds[j - 1];
      yz[r] = 0.0;
    }
    double Bcopy[32 * 16], yzc[32];
    memcpy(Bcopy, B, sizeof(B));
    memcpy(yzc, yz, sizeof(yz));
    if (lsq_qr(rz, kz, B, yz, wz, Cz)) return -3;
    chi = 0.0;
    for (int r = 0; r < rz; ++r) {
      double e = -yzc[r];
      for (int q = 0; q < kz; ++q) e += Bcopy[r * kz + q] * wz[q];
      chi += e * e;
    }
    chi2[1] = chi;
    /* 5. parameters at the point of closest approach */
    fit_frame f = {X[0], Y[0], Z[0], tx, ty, nx, ny, kref, ds[0], tref,
                   c->c_kappa};
    double u0 = xs[0], u1 = xs[1], dk = xs[n], w0 = wz[0], w1 = wz[1];
    pca_params(&f, u0, u1, dk, w0, w1, params);
    /* covariance: central differences of the parameters with respect to
     * (u0, u1, dk) and (w0, w1), propagated from the inverse normal
     * matrices; the transverse and longitudinal blocks are independent */
    double hstep[5] = {1e-6, 1e-6, 1e-8, 1e-6, 1e-6};
    double J[5][5];
    for (int q = 0; q < 5; ++q) {
      double vp[5] = {u0, u1, dk, w0, w1}, vm[5] = {u0, u1, dk, w0, w1};
      vp[q] += hstep[q];
      vm[q] -= hstep[q];
      double pp[5], pm[5];
      pca_params(&f, vp[0], vp[1], vp[2], vp[3], vp[4], pp);
      pca_params(&f, vm[0], vm[1], vm[2], vm[3], vm[4], pm);
      for (int o = 0; o < 5; ++o) {
        double d = pp[o] - pm[o];
        if (o == 0) d = atan2(sin(d), cos(d));
        J[o][q] = d / (2.0 * hstep[q]);
      }
    }
    /* transverse block: variables (u0, u1, dk) = indices (0, 1, n) */
    int tv[3] = {0, 1, n};
    double full[5][5];
    memset(full, 0, sizeof(full));
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double sum = 0.0;
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q)
            sum += J[a][p] * C[tv[p] * k + tv[q]] * J[b][q];
        full[a][b] = sum;
      }
    /* longitudinal block: variables (w0, w1) = indices (0, 1) */
    for (int a = 3; a < 5; ++a)
      for (int b = 3; b < 5; ++b) {
        double sum = 0.0;
        for (int p = 0; p < 2; ++p)
          for (int q = 0; q < 2; ++q)
            sum += J[a][3 + p] * Cz[p * kz + q] * J[b][3 + q];
        full[a][b] = sum;
      }
    int o = 0;
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b <= a; ++b) cov[o++] = full[a][b];
  }
  if (kref_out) *kref_out = kref;
  return 0;
}

/* ------------------------------------------------------------------ */
/* the whole path for one event                                        */

typedef struct {
  const orc_config* c;
  const double *X, *Y, *Z;
  const uint32_t* cin;     /* doublet inner hit */
  const uint32_t* cout;    /* doublet outer hit */
  const uint64_t* loff;    /* outer links of doublet d: lst[loff[d]..loff[d+1]) */
  const uint32_t* lst;
  uint32_t path[ORC_MAX_HITS_PER_TUPLE + 2];  /* doublet ids */
  vec_t* raw;
  vec_t* rawcells;
  int status;
} dfs_ctx;

static void dfs(dfs_ctx* d, int depth) {
  uint32_t cell = d->path[depth];
  uint64_t b = d->loff[cell], e = d->loff[cell + 1];
  int hits = depth + 2;
  if (b == e) {
    if (hits >= 3) {
      uint32_t t[ORC_MAX_HITS_PER_TUPLE], cl[ORC_MAX_HITS_PER_TUPLE];
      for (int i = 0; i < ORC_MAX_HITS_PER_TUPLE; ++i) t[i] = cl[i] = ORC_PAD;
      t[0] = d->cin[d->path[0]];
      for (int i = 0; i <= depth; ++i) {
        t[i + 1] = d->cout[d->path[i]];
        cl[i] = d->path[i];
      }
      if (vec_push(d->raw, t) || vec_push(d->rawcells, cl)) d->status = ORC_ERR_ALLOC;
    }
    return;
  }
  if (hits + 1 > ORC_MAX_HITS_PER_TUPLE) {
    d->status = ORC_ERR_PATH_TOO_LONG;
    return;
  }
  for (uint64_t l = b; l < e; ++l) {
    d->path[depth + 1] = d->lst[l];
    dfs(d, depth + 1);
  }
}

/* Total order of the cleaning step: returns <0 if tuple a ranks before b.
 * A NaN score (only non-finite hits produce one) ranks after every number
 * and NaN scores tie, so the order stays total and the best tuple of a
 * doublet does not depend on the order the tuples are visited in. */
static int rank_cmp(const uint32_t* ta, int na, double sa, const uint32_t* tb,
                    int nb, double sb) {
  if (na != nb) return na > nb ? -1 : 1;
  const int an = sa != sa, bn = sb != sb;
  if (an != bn) return an ? 1 : -1;
  if (!an && sa != sb) return sa < sb ? -1 : 1;
  for (int i = 0; i < ORC_MAX_HITS_PER_TUPLE; ++i)
    if (ta[i] != tb[i]) return ta[i] < tb[i] ? -1 : 1;
  return 0;
}

static int tuple_len(const uint32_t* t) {
  int n = 0;
  while (n < ORC_MAX_HITS_PER_TUPLE && t[n] != ORC_PAD) ++n;
  return n;
}

orc_result* orc_run(const orc_config* c, uint32_t nh, const float* x,
                    const float* y, const float* z, const int16_t* layer) {
  orc_result* R = (orc_result*)calloc(1, sizeof(orc_result));
  if (!R) return 0;
  size_t esz[ORC_NITEMS] = {8, 12, 32, 8, 1, 32, 40, 120, 16, 8};
  for (int i = 0; i < ORC_NITEMS; ++i) R->item[i].esz = esz[i];
  double* X = (double*)malloc(sizeof(double) * (nh + 1));
  double* Y = (double*)malloc(sizeof(double) * (nh + 1));
  double* Z = (double*)malloc(sizeof(double) * (nh + 1));
  for (uint32_t i = 0; i < nh; ++i) {
    X[i] = (double)x[i];
    Y[i] = (double)y[i];
    Z[i] = (double)z[i];
  }
  /* doublets: all ordered pairs over the layer-pair table */
  vec_t* D = &R->item[ORC_DOUBLETS];
  for (int p = 0; p < c->n_pairs; ++p)
    for (uint32_t i = 0; i < nh; ++i) {
      if (layer[i] != c->pair_inner[p]) continue;
      for (uint32_t o = 0; o < nh; ++o) {
        if (layer[o] != c->pair_outer[p]) continue;
        if (orc_doublet_ok(c, X[i], Y[i], Z[i], X[o], Y[o], Z[o])) {
          uint32_t e[2] = {i, o};
          vec_push(D, e);
        }
      }
    }
  uint64_t nd = D->n;
  uint32_t* cin = (uint32_t*)malloc(sizeof(uint32_t) * (nd + 1));
  uint32_t* cout = (uint32_t*)malloc(sizeof(uint32_t) * (nd + 1));
  for (uint64_t d = 0; d < nd; ++d) {
    cin[d] = ((uint32_t*)D->p)[2 * d];
    cout[d] = ((uint32_t*)D->p)[2 * d + 1];
  }
  /* doublets leaving each hit */
  uint64_t* hoff = (uint64_t*)calloc(nh + 2, sizeof(uint64_t));
  uint32_t* hlst = (uint32_t*)malloc(sizeof(uint32_t) * (nd + 1));
  for (uint64_t d = 0; d < nd; ++d) hoff[cin[d] + 1]++;
  for (uint32_t i = 0; i < nh; ++i) hoff[i + 1] += hoff[i];
  {
    uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * (nh + 1));
    memcpy(fill, hoff, sizeof(uint64_t) * (nh + 1));
    for (uint64_t d = 0; d < nd; ++d) hlst[fill[cin[d]]++] = (uint32_t)d;
    free(fill);
  }
  /* links: every (a,b),(b,c) sharing hit b that passes L1..L3 */
  vec_t L = {0, 0, 0, 8};      /* (inner doublet, outer doublet) */
  uint8_t* has_inner = (uint8_t*)calloc(nd + 1, 1);
  for (uint64_t d = 0; d < nd; ++d) {
    uint32_t a = cin[d], b = cout[d];
    for (uint64_t q = hoff[b]; q < hoff[b + 1]; ++q) {
      uint32_t e = hlst[q];
      uint32_t cc = cout[e];
      if (orc_link_ok(c, X[a], Y[a], Z[a], X[b], Y[b], Z[b], X[cc], Y[cc], Z[cc])) {
        uint32_t pr[2] = {(uint32_t)d, e};
        vec_push(&L, pr);
        uint32_t t3[3] = {a, b, cc};
        vec_push(&R->item[ORC_LINKS], t3);
        has_inner[e] = 1;
      }
    }
  }
  /* outer-neighbour lists per doublet (links were produced in doublet order) */
  uint64_t nl = L.n;
  uint64_t* loff = (uint64_t*)calloc(nd + 2, sizeof(uint64_t));
  uint32_t* lst = (uint32_t*)malloc(sizeof(uint32_t) * (nl + 1));
  for (uint64_t l = 0; l < nl; ++l) loff[((uint32_t*)L.p)[2 * l] + 1]++;
  for (uint64_t d = 0; d < nd; ++d) loff[d + 1] += loff[d];
  for (uint64_t l = 0; l < nl; ++l) lst[l] = ((uint32_t*)L.p)[2 * l + 1];
  /* tuples: depth-first from every root */
  vec_t rawcells = {0, 0, 0, 32};
  dfs_ctx dc;
  memset(&dc, 0, sizeof(dc));
  dc.c = c; dc.X = X; dc.Y = Y; dc.Z = Z; dc.cin = cin; dc.cout = cout;
  dc.loff = loff; dc.lst = lst; dc.raw = &R->item[ORC_RAW]; dc.rawcells = &rawcells;
  for (uint64_t d = 0; d < nd && dc.status == ORC_OK; ++d) {
    if (has_inner[d]) continue;
    dc.path[0] = (uint32_t)d;
    dfs(&dc, 0);
  }
  R->status = dc.status;
  uint64_t nt = R->item[ORC_RAW].n;
  const uint32_t* raw = (const uint32_t*)R->item[ORC_RAW].p;
  const uint32_t* rc = (const uint32_t*)rawcells.p;
  /* cleaning: score, per-doublet best tuple, survivors */
  double* score = (double*)malloc(sizeof(double) * (nt + 1));
  int* tn = (int*)malloc(sizeof(int) * (nt + 1));
  for (uint64_t t = 0; t < nt; ++t) {
    const uint32_t* h = raw + 8 * t;
    int n = tuple_len(h);
    tn[t] = n;
    double s = 0.0;
    for (int j = 1; j + 1 < n; ++j)
      s += triple_score(c, X[h[j - 1]], Y[h[j - 1]], Z[h[j - 1]], X[h[j]],
                        Y[h[j]], Z[h[j]], X[h[j + 1]], Y[h[j + 1]], Z[h[j + 1]]);
    score[t] = s;
    vec_push(&R->item[ORC_RAW_SCORE], &s);
  }
  int64_t* best = (int64_t*)malloc(sizeof(int64_t) * (nd + 1));
  for (uint64_t d = 0; d < nd; ++d) best[d] = -1;
  for (uint64_t t = 0; t < nt; ++t)
    for (int j = 0; j + 1 < tn[t]; ++j) {
      uint32_t d = rc[8 * t + j];
      int64_t bt = best[d];
      if (bt < 0 || rank_cmp(raw + 8 * t, tn[t], score[t], raw + 8 * bt, tn[bt], score[bt]) < 0)
        best[d] = (int64_t)t;
    }
  for (uint64_t t = 0; t < nt; ++t) {
    uint8_t keep = 1;
    for (int j = 0; j + 1 < tn[t]; ++j)
      if (best[rc[8 * t + j]] != (int64_t)t) keep = 0;
    vec_push(&R->item[ORC_KEEP], &keep);
    if (!keep) continue;
    vec_push(&R->item[ORC_TRACKS], raw + 8 * t);
    /* fit */
    const uint32_t* h = raw + 8 * t;
    int n = tn[t];
    double hx[8], hy[8], hz[8];
    int kd[8];
    for (int i = 0; i < n; ++i) {
      hx[i] = X[h[i]]; hy[i] = Y[h[i]]; hz[i] = Z[h[i]];
      int l = layer[h[i]];
      kd[i] = (l >= 0 && l < c->n_layers) ? c->layer_kind[l] : 0;
    }
    double prm[5] = {0}, cv[15] = {0}, ch[2] = {0}, kr = 0.0;
    if (orc_fit(c, n, hx, hy, hz, kd, prm, cv, ch, &kr)) {
      for (int i = 0; i < 5; ++i) prm[i] = NAN;
    }
    vec_push(&R->item[ORC_PARAMS], prm);
    vec_push(&R->item[ORC_COV], cv);
    vec_push(&R->item[ORC_CHI2], ch);
    vec_push(&R->item[ORC_KREF], &kr);
  }
  free(score); free(tn); free(best); free(rawcells.p);
  free(loff); free(lst); free(L.p); free(has_inner); free(hoff); free(hlst);
  free(cin); free(cout); free(X); free(Y); free(Z);
  return R;
}

int orc_status(const orc_result* R) { return R->status; }
uint64_t orc_count(const orc_result* R, int what) {
  return (what >= 0 && what < ORC_NITEMS) ? R->item[what].n : 0;
}
const void* orc_data(const orc_result* R, int what) {
  return (what >= 0 && what < ORC_NITEMS) ? R->item[what].p : 0;
}
void orc_free(orc_result* R) {
  if (!R) return;
  for (int i = 0; i < ORC_NITEMS; ++i) free(R->item[i].p);
  free(R);
}

/* ------------------------------------------------------------------ */
/* Vertices (the paper's Vertices module, Sec. 2 and Fig. 1: vertices are
 * formed from the pixel tracks).  The paper gives no algorithm; the reading
 * here is one-dimensional density-based clustering (DBSCAN, Ester et al.,
 * KDD 1996) of the tracks' longitudinal impact parameters z0:
 *
 *   selection  tracks with at least min_hits hits, |q/pT| <= qopt_max
 *              (single precision, as the values are given), finite z0 and
 *              a finite positive variance of z0;
 *   neighbours tracks i, j with |z0_j - z0_i| <= eps (the difference of the
 *              single-precision values taken in double precision, which is
 *              exact), each track its own neighbour;
 *   core       a track with at least min_pts neighbours;
 *   clusters   connected components of the cores under the neighbour
 *              relation;
 *   border     a non-core track with a core neighbour joins the cluster of
 *              its nearest core neighbour (on a tie, the core with the
 *              smaller z0, then the smaller index); other tracks are noise;
 *   vertex     per cluster, over its members in increasing (z0, index):
 *              w = 1/var, z = sum(w z0)/sum(w), sigma_z = sqrt(1/sum(w)),
 *              chi2 = sum(w (z0 - z)^2), summed in that order.
 *
 * Vertices come out in increasing z (clusters are disjoint intervals of the
 * sorted track list).  assign[i] = the vertex of track i, or -1. */

typedef struct {
  double eps;
  int min_pts;
  int min_hits;
  float qopt_max;
} orc_vtx_config;

typedef struct {
  float z;
  uint32_t i;
} orc_zi;

static int zi_cmp(const void* a, const void* b) {
  const orc_zi* p = (const orc_zi*)a;
  const orc_zi* q = (const orc_zi*)b;
  if (p->z != q->z) return p->z < q->z ? -1 : 1;
  return p->i < q->i ? -1 : (p->i > q->i ? 1 : 0);
}

static uint32_t uf_find(uint32_t* par, uint32_t a) {
  while (par[a] != a) {
    par[a] = par[par[a]];
    a = par[a];
  }
  return a;
}

int orc_vertices(const orc_vtx_config* c, uint32_t n, const float* z0, const float* var,
                 const float* qopt, const uint8_t* nhits, int32_t* assign, double* vz,
                 double* verr, double* vchi2, uint32_t* vn, uint32_t cap) {
  orc_zi* s = (orc_zi*)malloc(sizeof(orc_zi) * (n + 1));
  uint32_t m = 0;
  for (uint32_t i = 0; i < n; ++i) {
    assign[i] = -1;
    const int ok = nhits[i] >= c->min_hits && fabsf(qopt[i]) <= c->qopt_max &&
                   isfinite(z0[i]) && isfinite(var[i]) && var[i] > 0.0f;
    if (ok) {
      s[m].z = z0[i];
      s[m].i = i;
      ++m;
    }
  }
  qsort(s, m, sizeof(orc_zi), zi_cmp);
  /* cores: neighbours counted over all selected tracks */
  uint8_t* core = (uint8_t*)calloc(m + 1, 1);
  for (uint32_t a = 0; a < m; ++a) {
    int cnt = 0;
    for (uint32_t b = 0; b < m; ++b)
      if (fabs((double)s[b].z - (double)s[a].z) <= c->eps) ++cnt;
    core[a] = cnt >= c->min_pts;
  }
  /* clusters: union of every pair of neighbouring cores */
  uint32_t* par = (uint32_t*)malloc(sizeof(uint32_t) * (m + 1));
  for (uint32_t a = 0; a < m; ++a) par[a] = a;
  for (uint32_t a = 0; a < m; ++a)
    for (uint32_t b = a + 1; b < m; ++b)
      if (core[a] && core[b] && fabs((double)s[b].z - (double)s[a].z) <= c->eps) {
        const uint32_t ra = uf_find(par, a), rb = uf_find(par, b);
        if (ra != rb) par[ra > rb ? ra : rb] = ra < rb ? ra : rb;
      }
  /* label of each sorted track: the root of its core (cores), or of its
   * nearest core neighbour (borders); UINT32_MAX for noise */
  uint32_t* lab = (uint32_t*)malloc(sizeof(uint32_t) * (m + 1));
  for (uint32_t a = 0; a < m; ++a) {
    lab[a] = 0xffffffffu;
    if (core[a]) {
      lab[a] = uf_find(par, a);
      continue;
    }
    double bd = 0.0;
    int64_t bb = -1;
    for (uint32_t b = 0; b < m; ++b) {
      if (!core[b]) continue;
      const double d = fabs((double)s[b].z - (double)s[a].z);
      if (d > c->eps) continue;
      /* b runs in increasing (z0, index): a later core wins only if nearer */
      if (bb < 0 || d < bd) {
        bd = d;
        bb = b;
      }
    }
    if (bb >= 0) lab[a] = uf_find(par, (uint32_t)bb);
  }
  /* vertices in increasing z: a cluster's number is fixed by its first
   * member in sorted order */
  int32_t* vid = (int32_t*)malloc(sizeof(int32_t) * (m + 1));
  for (uint32_t a = 0; a < m; ++a) vid[a] = -1;
  uint32_t nv = 0;
  for (uint32_t a = 0; a < m; ++a) {
    if (lab[a] == 0xffffffffu) continue;
    if (vid[lab[a]] < 0) vid[lab[a]] = (int32_t)nv++;
  }
  for (uint32_t v = 0; v < nv && v < cap; ++v) {
    double sw = 0.0, swz = 0.0;
    uint32_t k = 0;
    for (uint32_t a = 0; a < m; ++a) {
      if (lab[a] == 0xffffffffu || vid[lab[a]] != (int32_t)v) continue;
      const double w = 1.0 / (double)var[s[a].i];
      sw += w;
      swz += w * (double)s[a].z;
      ++k;
    }
    const double zv = swz / sw;
    double chi2 = 0.0;
    for (uint32_t a = 0; a < m; ++a) {
      if (lab[a] == 0xffffffffu || vid[lab[a]] != (int32_t)v) continue;
      const double w = 1.0 / (double)var[s[a].i];
      const double r = (double)s[a].z - zv;
      chi2 += w * r * r;
    }
    vz[v] = zv;
    verr[v] = sqrt(1.0 / sw);
    vchi2[v] = chi2;
    vn[v] = k;
  }
  for (uint32_t a = 0; a < m; ++a)
    if (lab[a] != 0xffffffffu) assign[s[a].i] = vid[lab[a]];
  free(s); free(core); free(par); free(lab); free(vid);
  return (int)nv;
}

/* ------------------------------------------------------------------ */
/* RecHits (the paper's RecHits module, Sec. 2: it estimates the 3-D
 * position of each cluster, forming hits; its Fig. 3 shows the per-module
 * step that limits each module's cluster count and turns the counts into
 * the modules' first-hit offsets).  Reading, for one event:
 *
 *   counts     c[m] = clusters of module m, limited to max_per_module;
 *   offsets    module_start[0] = 0, module_start[m+1] = module_start[m] + c[m];
 *   rank       of cluster i: the number of earlier clusters (lower index)
 *              of its module; clusters ranked max_per_module or beyond make
 *              no hit, cluster i otherwise makes hit module_start[m] + rank;
 *   centroid   Q = sum q, SU = sum q (iu + 1/2), SV = sum q (iv + 1/2) over
 *              its pixels in order (double precision), local
 *              u = u0 + pitch_u (SU / Q), v = v0 + pitch_v (SV / Q);
 *   3-D        barrel module (direction c, s; radius r; centre z_c): the
 *              point r n + u t of the tangent plane projected radially
 *              onto the cylinder, p = (r c - u s, r s + u c) r / sqrt(r r +
 *              u u), z = z_c + v; disk module (ring centre r, disk z): x =
 *              (r + u) c - v s, y = (r + u) s + v c, z = z_disk;
 *   output     single precision x, y, z, the module's layer, the module id
 *              and the cluster index; a cluster with no charge makes a hit
 *              with layer -1 at the origin (it takes part in nothing).
 *
 * The module table is float64 rows (layer, kind, cos phi_c, sin phi_c, r,
 * z, u0, v0, pitch_u, pitch_v).  Returns the number of hits. */
uint32_t orc_rechits(const double* table, uint32_t n_modules, uint32_t max_per_module,
                     uint32_t nc, const uint16_t* module, const uint32_t* pixel_offsets,
                     const uint16_t* pix_u, const uint16_t* pix_v, const uint16_t* charge,
                     uint32_t* module_start, float* x, float* y, float* z, int16_t* layer,
                     uint16_t* hit_module, uint32_t* cluster_of_hit) {
  uint32_t* cnt = (uint32_t*)calloc(n_modules + 1, sizeof(uint32_t));
  for (uint32_t i = 0; i < nc; ++i) cnt[module[i]]++;
  module_start[0] = 0;
  for (uint32_t m = 0; m < n_modules; ++m) {
    const uint32_t c = cnt[m] < max_per_module ? cnt[m] : max_per_module;
    module_start[m + 1] = module_start[m] + c;
  }
  uint32_t* seen = (uint32_t*)calloc(n_modules + 1, sizeof(uint32_t));
  for (uint32_t i = 0; i < nc; ++i) {
    const uint32_t m = module[i];
    const uint32_t rank = seen[m]++;
    if (rank >= max_per_module) continue;
    const uint32_t h = module_start[m] + rank;
    const double* T = table + 10 * (size_t)m;
    double Q = 0.0, SU = 0.0, SV = 0.0;
    for (uint32_t p = pixel_offsets[i]; p < pixel_offsets[i + 1]; ++p) {
      const double q = (double)charge[p];
      Q += q;
      SU += q * ((double)pix_u[p] + 0.5);
      SV += q * ((double)pix_v[p] + 0.5);
    }
    hit_module[h] = (uint16_t)m;
    cluster_of_hit[h] = i;
    if (!(Q > 0.0)) {
      x[h] = 0.0f;
      y[h] = 0.0f;
      z[h] = 0.0f;
      layer[h] = -1;
      continue;
    }
    const double c = T[2], s = T[3], r = T[4], zc = T[5];
    const double u = T[6] + T[8] * (SU / Q);
    const double v = T[7] + T[9] * (SV / Q);
    double gx, gy, gz;
    if (T[1] == 0.0) {
      const double f = r / sqrt(r * r + u * u);
      gx = (r * c - u * s) * f;
      gy = (r * s + u * c) * f;
      gz = zc + v;
    } else {
      gx = (r + u) * c - v * s;
      gy = (r + u) * s + v * c;
      gz = zc;
    }
    x[h] = (float)gx;
    y[h] = (float)gy;
    z[h] = (float)gz;
    layer[h] = (int16_t)T[0];
  }
  const uint32_t nh = module_start[n_modules];
  free(cnt);
  free(seen);
  return nh;
}
