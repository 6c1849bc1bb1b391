// Geometric cuts of the doublet and link steps, in FP64 on FP32 hits.
//
// The paper names the steps (hit doublets, cellular-automaton linking into
// n-tuplets, Sec. 2) but no cut; the cuts below are this library's reading:
//
//  doublet (inner i, outer o):
//   D1  r_o > r_i
//   D2  the r-z line through both hits meets r = 0 within |z| <= z0max:
//       |z_i (r_o - r_i) - r_i (z_o - z_i)| <= z0max (r_o - r_i)
//   D3  the circle through the origin and both hits has curvature <= kmax:
//       2 |x_i y_o - y_i x_o| <= kmax r_i r_o |p_o - p_i|
//   D4  x_i x_o + y_i y_o > 0
//  link (hits a, b, c of doublets (a,b), (b,c)):
//   L1  r-z alignment: |dr_ab dz_bc - dz_ab dr_bc| <= arz l_ab l_bc
//   L2  Menger curvature: 2 |(b-a) x (c-a)| <= kmax |ab| |bc| |ac|
//   L3  distance of the origin from the circle through a, b, c <= d0max,
//       evaluated as | |a|^2 + 2 a.o | / (|C| + R) with o = C - a (the same
//       quantity as ||C| - R|, free of the cancellation of two large radii);
//       for exactly collinear points, the distance from their line.
//
// Every operation is written in the order the decision is defined in, and
// the library is built without FP contraction, so each comparison sees the
// correctly rounded IEEE double of the written expression.
#pragma once

#include "common.h"

namespace pxt {

struct HitD {
  double x, y, z, r;
};

// A hit from its FP32 coordinates; r is the same FP64 expression the
// binned arrays hold, so it is bit-identical to the stored radius.
__device__ __forceinline__ HitD hit_xyz(float x, float y, float z) {
  HitD h;
  h.x = (double)x;
  h.y = (double)y;
  h.z = (double)z;
  h.r = sqrt(h.x * h.x + h.y * h.y);
  return h;
}

__device__ __forceinline__ HitD load_hit(const Ws& w, uint32_t i) {
  HitD h;
  const float4 v = w.bh[i];
  h.x = (double)v.x;
  h.y = (double)v.y;
  h.z = (double)v.z;
  h.r = w.br[i];
  return h;
}

__device__ __forceinline__ bool doublet_ok(const DevCfg& c, const HitD& i,
                                           const HitD& o) {
  if (!(o.r > i.r)) return false;
  const double dr = o.r - i.r;
  const double l2 = fabs(i.z * dr - i.r * (o.z - i.z));
  if (!(l2 <= c.z0max * dr)) return false;
  const double cr = i.x * o.y - i.y * o.x;
  const double dx = o.x - i.x, dy = o.y - i.y;
  const double chord = sqrt(dx * dx + dy * dy);
  if (!(2.0 * fabs(cr) <= c.kmax * i.r * o.r * chord)) return false;
  return i.x * o.x + i.y * o.y > 0.0;
}

// Terms of the link cuts: t0 = |r-z cross|, t1 = arz l_ab l_bc,
// t2 = 2 |cross|, t3 = kmax |ab||bc||ac|, d0 = transverse impact.
struct LinkTerms {
  double t0, t1, t2, t3, d0;
};

__device__ __forceinline__ LinkTerms link_terms(const DevCfg& c, const HitD& a,
                                                const HitD& b, const HitD& h) {
  LinkTerms t;
  const double dra = b.r - a.r, dza = b.z - a.z;
  const double drb = h.r - b.r, dzb = h.z - b.z;
  t.t0 = fabs(dra * dzb - dza * drb);
  const double lab = sqrt(dra * dra + dza * dza);
  const double lbc = sqrt(drb * drb + dzb * dzb);
  t.t1 = c.arz * lab * lbc;
  const double ux = b.x - a.x, uy = b.y - a.y;
  const double vx = h.x - a.x, vy = h.y - a.y;
  const double wx = h.x - b.x, wy = h.y - b.y;
  const double cr = ux * vy - uy * vx;
  const double nab = sqrt(ux * ux + uy * uy);
  const double nac = sqrt(vx * vx + vy * vy);
  const double nbc = sqrt(wx * wx + wy * wy);
  t.t2 = 2.0 * fabs(cr);
  t.t3 = c.kmax * nab * nbc * nac;
  const double D = 2.0 * cr;
  if (D == 0.0) {
    t.d0 = fabs(a.x * vy - a.y * vx) / nac;
  } else {
    const double uu = ux * ux + uy * uy, vv = vx * vx + vy * vy;
    const double ox = (vy * uu - uy * vv) / D;
    const double oy = (ux * vv - vx * uu) / D;
    const double R = sqrt(ox * ox + oy * oy);
    const double cx = a.x + ox, cy = a.y + oy;
    const double dc = sqrt(cx * cx + cy * cy);
    const double aa = a.x * a.x + a.y * a.y;
    const double ao = a.x * ox + a.y * oy;
    t.d0 = fabs(aa + 2.0 * ao) / (dc + R);
  }
  return t;
}

__device__ __forceinline__ bool link_ok(const DevCfg& c, const HitD& a,
                                        const HitD& b, const HitD& h) {
  // L1 first: the terms are the same expressions as in link_terms, only
  // evaluated lazily, so every decision is unchanged
  const double dra = b.r - a.r, dza = b.z - a.z;
  const double drb = h.r - b.r, dzb = h.z - b.z;
  const double t0 = fabs(dra * dzb - dza * drb);
  const double lab = sqrt(dra * dra + dza * dza);
  const double lbc = sqrt(drb * drb + dzb * dzb);
  if (!(t0 <= c.arz * lab * lbc)) return false;
  const double ux = b.x - a.x, uy = b.y - a.y;
  const double vx = h.x - a.x, vy = h.y - a.y;
  const double wx = h.x - b.x, wy = h.y - b.y;
  const double cr = ux * vy - uy * vx;
  const double nab = sqrt(ux * ux + uy * uy);
  const double nac = sqrt(vx * vx + vy * vy);
  const double nbc = sqrt(wx * wx + wy * wy);
  if (!(2.0 * fabs(cr) <= c.kmax * nab * nbc * nac)) return false;
  const double D = 2.0 * cr;
  double d0;
  if (D == 0.0) {
    d0 = fabs(a.x * vy - a.y * vx) / nac;
  } else {
    const double uu = ux * ux + uy * uy, vv = vx * vx + vy * vy;
    const double ox = (vy * uu - uy * vv) / D;
    const double oy = (ux * vv - vx * uu) / D;
    const double R = sqrt(ox * ox + oy * oy);
    const double cx = a.x + ox, cy = a.y + oy;
    const double dc = sqrt(cx * cx + cy * cy);
    const double aa = a.x * a.x + a.y * a.y;
    const double ao = a.x * ox + a.y * oy;
    d0 = fabs(aa + 2.0 * ao) / (dc + R);
  }
  return d0 <= c.d0max;
}

// ---------------------------------------------------------------------
// Decision-identical fast forms.  A comparison lhs <= k * sqrt(p) * ...
// between non-negative doubles is first made on squares, lhs^2 against
// k^2 * p * ..., which needs no square root.  Both sides of the squared
// comparison are within a few ulps (relative 1e-15) of the exact squares of
// the rounded quantities the defining expression compares, so outside a
// relative band of 1e-9 around equality the squared comparison returns the
// same answer; inside the band the defining expression itself is evaluated.

constexpr double kBandHi = 1.0 + 1e-9;
constexpr double kBandLo = 1.0 - 1e-9;

__device__ __forceinline__ bool doublet_ok_fast(const DevCfg& c, const HitD& i,
                                                const HitD& o) {
  if (!(o.r > i.r)) return false;
  const double dr = o.r - i.r;
  const double l2 = fabs(i.z * dr - i.r * (o.z - i.z));
  if (!(l2 <= c.z0max * dr)) return false;
  if (!(i.x * o.x + i.y * o.y > 0.0)) return false;
  const double cr = i.x * o.y - i.y * o.x;
  const double dx = o.x - i.x, dy = o.y - i.y;
  const double ch2 = dx * dx + dy * dy;
  const double lhs = 2.0 * fabs(cr);
  const double L = lhs * lhs;
  const double R = c.kmax2 * (i.r * i.r) * (o.r * o.r) * ch2;
  if (L > R * kBandHi) return false;
  if (L < R * kBandLo) return true;
  return lhs <= c.kmax * i.r * o.r * sqrt(ch2);
}

// Link cut split in two: the r-z cut L1 needs only (r, z) of the third hit;
// the transverse cuts L2, L3 need its (x, y).
__device__ __forceinline__ bool link_rz_pass(const DevCfg& c, const HitD& a, const HitD& b,
                                             double rc, double zc) {
  const double dra = b.r - a.r, dza = b.z - a.z;
  const double drb = rc - b.r, dzb = zc - b.z;
  const double t0 = fabs(dra * dzb - dza * drb);
  const double lab2 = dra * dra + dza * dza;
  const double lbc2 = drb * drb + dzb * dzb;
  const double L = t0 * t0, R = c.arz2 * lab2 * lbc2;
  if (L > R * kBandHi) return false;
  if (L < R * kBandLo) return true;
  return t0 <= c.arz * sqrt(lab2) * sqrt(lbc2);
}

__device__ __forceinline__ bool link_xy_pass(const DevCfg& c, const HitD& a, const HitD& b,
                                             const HitD& h) {
  const double ux = b.x - a.x, uy = b.y - a.y;
  const double vx = h.x - a.x, vy = h.y - a.y;
  const double wx = h.x - b.x, wy = h.y - b.y;
  const double cr = ux * vy - uy * vx;
  const double ab2 = ux * ux + uy * uy;
  const double ac2 = vx * vx + vy * vy;
  const double bc2 = wx * wx + wy * wy;
  const double t2 = 2.0 * fabs(cr);
  {
    const double L = t2 * t2, R = c.kmax2 * ab2 * bc2 * ac2;
    if (L > R * kBandHi) return false;
    if (!(L < R * kBandLo) && !(t2 <= c.kmax * sqrt(ab2) * sqrt(bc2) * sqrt(ac2)))
      return false;
  }
  const double D = 2.0 * cr;
  // L3 first in a form without divisions: with N = D * (centre - a) =
  // (vy ab2 - uy ac2, ux ac2 - vx ab2), the defining expression below is
  // d0 = |aa D + 2 a.N| / (|a D + N| + |N|) (also for D = 0, where it is the
  // distance from the origin to the line), compared with d0max; outside the
  // relative band its answer is that of the defining expression
  {
    const double Nx = vy * ab2 - uy * ac2, Ny = ux * ac2 - vx * ab2;
    const double px = a.x * D + Nx, py = a.y * D + Ny;
    const double num = fabs((a.x * a.x + a.y * a.y) * D + 2.0 * (a.x * Nx + a.y * Ny));
    const double den = c.d0max * (sqrt(px * px + py * py) + sqrt(Nx * Nx + Ny * Ny));
    if (num > den * kBandHi) return false;
    if (num < den * kBandLo) return true;
  }
  double d0;
  if (D == 0.0) {
    d0 = fabs(a.x * vy - a.y * vx) / sqrt(ac2);
  } else {
    const double ox = (vy * ab2 - uy * ac2) / D;
    const double oy = (ux * ac2 - vx * ab2) / D;
    const double R = sqrt(ox * ox + oy * oy);
    const double cx = a.x + ox, cy = a.y + oy;
    const double dc = sqrt(cx * cx + cy * cy);
    const double aa = a.x * a.x + a.y * a.y;
    const double ao = a.x * ox + a.y * oy;
    d0 = fabs(aa + 2.0 * ao) / (dc + R);
  }
  return d0 <= c.d0max;
}

// Direction of a doublet in the r-z plane, in FP32: the angle of
// (r_o - r_i, z_o - z_i).  For two doublets (a,b), (b,c) the r-z cross
// product of L1 is l_ab l_bc sin(angle_bc - angle_ab), so L1 can hold only
// where the angles differ by at most asin(arz), or by at least
// pi - asin(arz); rz_prefilter tests that on the angles stored in 16-bit
// units, with windows (q_win, q_far) widened to cover the FP32 error and
// the rounding to units of both angles.  Candidates it rejects fail L1;
// the ones it keeps go on to the exact cuts.
__device__ __forceinline__ float rz_angle(const HitD& i, const HitD& o) {
  return atan2f((float)(o.z - i.z), (float)(o.r - i.r));
}

// The r-z angle of a doublet in angle units of (pi/2) / 32767 rad, rounded
// to nearest: doublets point outward (r grows), so the FP32 angle lies in
// [-pi/2, pi/2] (pi/2 rounded up, hence the clamp), and the stored value is
// within one unit of it (half a unit from the rounding, ~0.005 from the
// FP32 product and scale).
constexpr float kAngleUnits = 32767.0f / 1.57079632679f;
__device__ __forceinline__ int16_t angle_units(float th) {
  const float q = rintf(th * kAngleUnits);
  return (int16_t)fminf(32767.0f, fmaxf(-32767.0f, q));
}

__device__ __forceinline__ bool rz_prefilter(const DevCfg& c, int ta, int tc) {
  const int dd = abs(tc - ta);
  return dd <= c.q_win || dd >= c.q_far;
}

// Cleaning score of one consecutive hit triple.
__device__ __forceinline__ double triple_score(const DevCfg& c, const HitD& a,
                                               const HitD& b, const HitD& h) {
  const LinkTerms t = link_terms(c, a, b, h);
  const double q1 = t.t0 / t.t1;
  const double q2 = t.d0 / c.d0max;
  return q1 * q1 + q2 * q2;
}

}  // namespace pxt
