// physics.hpp -- device-side physics of one GRMHD stage for gfx950, FP64.
//
//   EOS                 ideal gas; hybrid cold piecewise polytrope + thermal
//                       Gamma_th part (Sec. III-D)
//   3-metric            determinant, inverse, sqrt(gamma) (Eq. 5)
//   cell state          Eq. 7 (densitized), Eq. 8 for b^mu, Eq. 9 fluxes,
//                       fast magnetosonic characteristic speeds
//   Riemann             HLLE / LLF (Sec. III-B)
//   WENOZ               Borges et al. 2008 (p = 2, eps = 1e-40)
//   C2P                 Kastaun et al. master function in mu = 1/(hW),
//                       bracketed root by Brent's method, atmosphere rules
//                       of Sec. III-C
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grmhd.h"

namespace gk {

constexpr double kEps = 2.220446049250313e-16;
// tau and T floors fire only below (1 - margin) x the floor: a state at the
// atmosphere values, recovered within rounding of T_atm, does not need it
constexpr double kFloorMargin = 1e-10;

// ---------------------------------------------------------------------------
// EOS: derived piece constants are computed once on the host
// ---------------------------------------------------------------------------
// 1/x for a normal, finite, nonzero x (every use below has x > 0 or a
// guard): the hardware reciprocal refined by one Newton
// step (error within an ulp or so of the correctly rounded quotient)
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

struct Eos {
  int type, n;
  double gam, gth;
  double rb[3], K[4], G[4], a[4];
};

// The EOS type as a compile-time constant inside a kernel: every eos_*
// branch on e.type folds away, so an ideal-gas kernel carries none of the
// piecewise-polytrope code (nor its registers).
template <int ET>
__device__ __forceinline__ Eos eos_fixed(const Eos& e) {
  Eos r = e;
  r.type = ET;
  return r;
}

// host side: call f(std::integral_constant<int, type>) for type 0 or 1
template <class F>
inline void eos_dispatch(int type, F&& f) {
  if (type == 0) f(std::integral_constant<int, 0>{});
  else f(std::integral_constant<int, 1>{});
}

struct Cold { double p, e, g; };   // P_cold, eps_cold, Gamma of the piece

// The piece's constants are picked by selection, not by indexing the arrays
// with a runtime piece number: an indexed struct member cannot live in
// registers and would put the whole Eos in private (scratch) memory.
__device__ __forceinline__ Cold eos_cold(const Eos& e, double rho) {
  Cold c{0.0, 0.0, 1.0};
  if (e.type == 1) {
    double gi = e.G[0], ki = e.K[0], ai = e.a[0];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (t + 1 < e.n && rho >= e.rb[t]) {
        gi = e.G[t + 1];
        ki = e.K[t + 1];
        ai = e.a[t + 1];
      }
    }
    const double pr = ki * pow(rho, gi);
    c.p = pr;
    c.e = ai + pr / (rho * (gi - 1.0));
    c.g = gi;
  }
  return c;
}

__device__ __forceinline__ double eos_P_from_eps(const Eos& e, double rho, double eps) {
  if (e.type == 0) return (e.gam - 1.0) * rho * eps;
  Cold c = eos_cold(e, rho);
  return c.p + (e.gth - 1.0) * rho * (eps - c.e);
}
__device__ __forceinline__ double eos_eps_from_P(const Eos& e, double rho, double P) {
  if (e.type == 0) return P / ((e.gam - 1.0) * rho);
  Cold c = eos_cold(e, rho);
  return c.e + (P - c.p) / ((e.gth - 1.0) * rho);
}
__device__ __forceinline__ double eos_T_from_P(const Eos& e, double rho, double P) {
  if (e.type == 0) return P / rho;
  return (P - eos_cold(e, rho).p) / rho;
}
__device__ __forceinline__ double eos_P_from_T(const Eos& e, double rho, double T) {
  if (e.type == 0) return rho * T;
  return eos_cold(e, rho).p + rho * T;
}
__device__ __forceinline__ double eos_eps_from_T(const Eos& e, double rho, double T) {
  if (e.type == 0) return T / (e.gam - 1.0);
  return eos_cold(e, rho).e + T / (e.gth - 1.0);
}
__device__ __forceinline__ double eos_eps_min(const Eos& e, double rho) {
  return e.type == 0 ? 0.0 : eos_cold(e, rho).e;
}
// c_s^2 h = dP/drho|_eps + (P/rho^2) dP/deps|_rho
__device__ __forceinline__ double eos_cs2(const Eos& e, double rho, double eps, double P, double h) {
  if (e.type == 0) return e.gam * P / (rho * h);
  Cold c = eos_cold(e, rho);
  double gm1 = e.gth - 1.0;
  double chi = c.g * c.p / rho + gm1 * (eps - c.e) - gm1 * c.p / rho;
  return (chi + gm1 * P / rho) / h;
}

// ---------------------------------------------------------------------------
// 3-metric (symmetric: xx xy xz yy yz zz)
// ---------------------------------------------------------------------------
struct M3 {
  double g[6];   // lower
  double u[6];   // inverse
  double sg;     // sqrt(det)
};

__device__ __forceinline__ void metric_build(M3& m, double xx, double xy, double xz, double yy,
                                             double yz, double zz) {
  m.g[0] = xx; m.g[1] = xy; m.g[2] = xz; m.g[3] = yy; m.g[4] = yz; m.g[5] = zz;
  double cxx = yy * zz - yz * yz;
  double cxy = yz * xz - xy * zz;
  double cxz = xy * yz - yy * xz;
  double det = xx * cxx + xy * cxy + xz * cxz;
  double id = 1.0 / det;
  m.u[0] = cxx * id;
  m.u[1] = cxy * id;
  m.u[2] = cxz * id;
  m.u[3] = (xx * zz - xz * xz) * id;
  m.u[4] = (xz * xy - xx * yz) * id;
  m.u[5] = (xx * yy - xy * xy) * id;
  m.sg = sqrt(det);
}

__device__ __forceinline__ void lower(const double* g, double ax, double ay, double az, double& lx,
                                      double& ly, double& lz) {
  lx = g[0] * ax + g[1] * ay + g[2] * az;
  ly = g[1] * ax + g[3] * ay + g[4] * az;
  lz = g[2] * ax + g[4] * ay + g[5] * az;
}

// component (a, b) of a symmetric 3x3 stored as 6
__device__ __forceinline__ constexpr int sym(int a, int b) {
  return a == b ? (a == 0 ? 0 : a == 1 ? 3 : 5) : ((a + b) == 1 ? 1 : (a + b) == 2 ? 2 : 4);
}

// ---------------------------------------------------------------------------
// Cell/face state: Eq. 7 (densitized), Eq. 8, Eq. 9 fluxes, wave speeds
// q = (rho, W v^x, W v^y, W v^z, P); B = Eulerian B^i (un-densitized)
// U, F: D~, S~_x, S~_y, S~_z, tau~, B~^{t1}, B~^{t2}  (t1 = (D+1)%3, t2 = (D+2)%3)
// ---------------------------------------------------------------------------
struct Side {
  double U[7], F[7];
  double lm, lp;
};

// rho h W^2 - P - D without cancellation:
//   D (W^2 - 1)/(W + 1) + rho eps W^2 + P (W^2 - 1), with W^2 - 1 = u.u
__device__ __forceinline__ double tau_hydro(double D, double usq, double W, double rho, double eps,
                                            double P) {
  return D * usq / (W + 1.0) + rho * eps * (W * W) + P * usq;
}

template <int DIR>
__device__ __forceinline__ void side_state(const Eos& e, const M3& m, double alpha, const double beta[3],
                                           const double q[5], const double B[3], Side& s) {
  constexpr int T1 = (DIR + 1) % 3, T2 = (DIR + 2) % 3;
  const double rho = q[0], P = q[4];
  double ul[3];
  lower(m.g, q[1], q[2], q[3], ul[0], ul[1], ul[2]);
  const double usq = q[1] * ul[0] + q[2] * ul[1] + q[3] * ul[2];
  const double W = sqrt(1.0 + usq);
  const double iW = rcp_nr(W);
  const double iW2 = iW * iW;
  double v[3] = {q[1] * iW, q[2] * iW, q[3] * iW};
  double vl[3] = {ul[0] * iW, ul[1] * iW, ul[2] * iW};
  double Bl[3];
  lower(m.g, B[0], B[1], B[2], Bl[0], Bl[1], Bl[2]);
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  const double Bv = B[0] * vl[0] + B[1] * vl[1] + B[2] * vl[2];
  const double eps = eos_eps_from_P(e, rho, P);
  const double h = 1.0 + eps + P * rcp_nr(rho);
  const double ia = rcp_nr(alpha);
  const double b0 = W * Bv * ia;
  const double W2 = W * W;
  const double bsq = B2 * iW2 + Bv * Bv;
  const double sg = m.sg;
  const double Ptt = sg * (P + 0.5 * bsq);
  const double D = rho * W;
  const double ehw = rho * h * W2 + B2;
  const double tau = D * usq * rcp_nr(W + 1.0) + rho * eps * W2 + P * usq + B2 -
                     0.5 * (Bv * Bv + B2 * iW2);
  double vh[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) vh[a] = v[a] - beta[a] * ia;
  const double Btd = sg * B[DIR];
  s.U[0] = sg * D;
#pragma unroll
  for (int a = 0; a < 3; ++a) s.U[1 + a] = sg * (ehw * vl[a] - Bv * Bl[a]);
  s.U[4] = sg * tau;
  s.U[5] = sg * B[T1];
  s.U[6] = sg * B[T2];
  const double avd = alpha * vh[DIR];
  s.F[0] = avd * s.U[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double bl = Bl[a] * iW + W * Bv * vl[a];     // b_i
    s.F[1 + a] = avd * s.U[1 + a] - alpha * bl * Btd * iW + (a == DIR ? alpha * Ptt : 0.0);
  }
  s.F[4] = avd * s.U[4] - alpha * alpha * b0 * Btd * iW + alpha * Ptt * v[DIR];
  s.F[5] = alpha * (s.U[5] * vh[DIR] - Btd * vh[T1]);
  s.F[6] = alpha * (s.U[6] * vh[DIR] - Btd * vh[T2]);
  // fast magnetosonic estimate c^2 = cs^2 + ca^2 - cs^2 ca^2
  const double cs2 = eos_cs2(e, rho, eps, P, h);
  const double ca2 = bsq * rcp_nr(rho * h + bsq);
  const double c2 = cs2 + ca2 - cs2 * ca2;
  const double v2 = usq * iW2;
  const double gdd = m.u[sym(DIR, DIR)];
  const double vd = v[DIR];
  double disc = c2 * (1.0 - v2) * (gdd * (1.0 - v2 * c2) - vd * vd * (1.0 - c2));
  disc = disc > 0.0 ? disc : 0.0;
  const double sq = sqrt(disc);
  const double iden = rcp_nr(1.0 - v2 * c2);
  const double base = vd * (1.0 - c2);
  s.lp = alpha * (base + sq) * iden - beta[DIR];
  s.lm = alpha * (base - sq) * iden - beta[DIR];
}

// A mass flux below this fraction of the magnitude scale of its Riemann
// formula is rounding noise of a flux that vanishes exactly (e.g. atmosphere
// at rest); it is set to zero so that the upwind CT averages there instead of
// following the noise's sign.
constexpr double kMassFluxZero = 1e-12;

// No contraction to FMA in this function (elsewhere the library fuses
// products within an expression): the two sides enter the flux formula as
// mirror images (L <-> R with the normal components negated), and a fused
// product keeps one side's product exact while the other's is rounded, so a
// mirror-symmetric state would get fluxes that are not mirror images bit for
// bit.  With every product rounded, the flux of the mirrored state is the
// mirrored flux exactly.
__device__ __forceinline__ void riemann(int kind, const Side& L, const Side& R, double F[7]) {
#pragma clang fp contract(off)
  double scale;
  if (kind == 0) {
    double a = fmax(fmax(fabs(L.lm), fabs(L.lp)), fmax(fabs(R.lm), fabs(R.lp)));
#pragma unroll
    for (int c = 0; c < 7; ++c) F[c] = 0.5 * (L.F[c] + R.F[c]) - 0.5 * a * (R.U[c] - L.U[c]);
    scale = 0.5 * (fabs(L.F[0]) + fabs(R.F[0])) + 0.5 * a * (fabs(R.U[0]) + fabs(L.U[0]));
  } else {
    const double ar = fmax(0.0, fmax(L.lp, R.lp));
    const double al = fmin(0.0, fmin(L.lm, R.lm));
    const double den = ar - al;
    if (den == 0.0) {
#pragma unroll
      for (int c = 0; c < 7; ++c) F[c] = 0.5 * (L.F[c] + R.F[c]);
      scale = 0.5 * (fabs(L.F[0]) + fabs(R.F[0]));
    } else {
      const double id = 1.0 / den;
      const double arl = ar * al;
#pragma unroll
      for (int c = 0; c < 7; ++c)
        F[c] = (ar * L.F[c] - al * R.F[c] + arl * (R.U[c] - L.U[c])) * id;
      scale = (ar * fabs(L.F[0]) - al * fabs(R.F[0]) - arl * (fabs(R.U[0]) + fabs(L.U[0]))) * id;
    }
  }
  if (fabs(F[0]) <= kMassFluxZero * scale) F[0] = 0.0;
}

// WENOZ (reading R3).  The smoothness indicators are written so that the
// mirror image of a stencil gives the same bits: the side stencils as
// (near + far) - 2 mid and (3 near - 4 mid) + far, the centre one from the
// sum and the difference of its outer cells.  (The value at the lower edge
// of a cell is then the value at the upper edge of its mirror image.)

// indicator of a side stencil: the cell itself (near), its neighbour (mid)
// and the next cell (far)
__device__ __forceinline__ double wz_beta_side(double near, double mid, double far) {
  const double sa = (near + far) - 2.0 * mid;
  const double sb = (3.0 * near - 4.0 * mid) + far;
  return (13.0 / 12.0) * sa * sa + 0.25 * sb * sb;
}

// indicator of the centre stencil (l, c, r)
__device__ __forceinline__ double wz_beta_mid(double l, double c, double r) {
  const double sa = (l + r) - 2.0 * c;
  const double sb = l - r;
  return (13.0 / 12.0) * sa * sa + 0.25 * sb * sb;
}

// value at the edge of cell c on the side of f, from the cells a, b, c, d, f
// in that order and the ratios r_k = tau5 / (beta_k + eps) of the stencils
// (a, b, c), (b, c, d), (c, d, f)
__device__ __forceinline__ double wz_edge(double r0, double r1, double r2, double a, double b,
                                          double c, double d, double f) {
  const double w0 = 0.1 * (1.0 + r0 * r0);
  const double w1 = 0.6 * (1.0 + r1 * r1);
  const double w2 = 0.3 * (1.0 + r2 * r2);
  const double p0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
  const double p1 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
  const double p2 = (2.0 * c + 5.0 * d - f) * (1.0 / 6.0);
  return (w0 * p0 + w1 * p1 + w2 * p2) * rcp_nr(w0 + w1 + w2);
}

// the ratios t5 / (beta_k + eps), each from a refined reciprocal of its own
// denominator (at least 1e-40, so no reciprocal overflows; one reciprocal of
// the product of the three would overflow for indicators beyond ~1e100)
__device__ __forceinline__ void wz_ratios(double a, double b, double c, double d, double f,
                                          double& r0, double& r1, double& r2) {
  const double be0 = wz_beta_side(c, b, a);
  const double be1 = wz_beta_mid(b, c, d);
  const double be2 = wz_beta_side(c, d, f);
  const double t5 = fabs(be0 - be2);
  r0 = t5 * rcp_nr(be0 + 1e-40);
  r1 = t5 * rcp_nr(be1 + 1e-40);
  r2 = t5 * rcp_nr(be2 + 1e-40);
}

// value at the upper edge of cell c from cells c-2..c+2
__device__ __forceinline__ double wenoz(double a, double b, double c, double d, double f) {
  double r0, r1, r2;
  wz_ratios(a, b, c, d, f, r0, r1, r2);
  return wz_edge(r0, r1, r2, a, b, c, d, f);
}

// ---------------------------------------------------------------------------
// Reconstruction at one face (Sec. III-B).  The six cells m3, m2, m1 | p0, p1,
// p2 straddle the face; qL is the upper edge value of cell m1 and qR the
// lower edge value of cell p0.  RC: 0 donor cell, 1 PLM, 2 WENOZ, 3 PPM4,
// 4 PPMX.  Every interface value and second difference is computed once per
// face and shared by the two cells that use it.
// ---------------------------------------------------------------------------

// PLM: half of van Leer's (1974) harmonic-mean slope, 0 across an extremum.
// A correctly rounded quotient (not a refined reciprocal): where the slope
// nearly cancels the cell value at an edge (an edge next to a near-zero
// neighbour), an ulp of the slope is a large part of the edge value.
__device__ __forceinline__ double vl_half_slope(double l, double c, double r) {
  const double dl = c - l, dr = r - c, pr = dl * dr;
  return pr > 0.0 ? pr / (dl + dr) : 0.0;
}

// Colella & Woodward (1984): the centred slope bounded by twice each
// one-sided difference, 0 at an extremum
__device__ __forceinline__ double cw_dm(double l, double c, double r) {
  const double dl = c - l, dr = r - c;
  const double dc = 0.5 * (r - l);
  const double m = fmin(fabs(dc), 2.0 * fmin(fabs(dl), fabs(dr)));
  return dl * dr > 0.0 ? copysign(m, dc) : 0.0;
}

// their monotonicity constraints on the edges (lo, hi) of a cell of mean a
__device__ __forceinline__ void cw_constrain(double a, double& lo, double& hi) {
  if ((hi - a) * (a - lo) <= 0.0) {
    lo = a;
    hi = a;
    return;
  }
  const double da = hi - lo;
  const double a6 = 6.0 * (a - 0.5 * (lo + hi));
  const double da2 = da * da;
  if (da * a6 > da2) lo = 3.0 * a - 2.0 * hi;
  else if (-da2 > da * a6) hi = 3.0 * a - 2.0 * lo;
}

// Colella & Sekora (2008): smallest magnitude of x and C y, C z (C = 1.25)
// when all three share a sign, else 0
__device__ __forceinline__ double cs_lim3(double x, double y, double z) {
  constexpr double C = 1.25;
  const bool pos = x > 0.0 && y > 0.0 && z > 0.0;
  const bool neg = x < 0.0 && y < 0.0 && z < 0.0;
  const double m = fmin(fabs(x), C * fmin(fabs(y), fabs(z)));
  return pos ? m : (neg ? -m : 0.0);
}

// fourth-order interface value between cells c0 and c1 (second differences
// d0, d1 of those cells); limited where it leaves their range
__device__ __forceinline__ double cs_iface(double cm, double c0, double c1, double cp, double d0,
                                           double d1) {
  double a = (7.0 / 12.0) * (c0 + c1) - (1.0 / 12.0) * (cm + cp);
  if ((a - c0) * (c1 - a) < 0.0) {
    const double d = 3.0 * ((c0 + c1) - 2.0 * a);
    a = 0.5 * (c0 + c1) - (1.0 / 6.0) * cs_lim3(d, d0, d1);
  }
  return a;
}

// their cell limiter: mean a, neighbour means l and r, second differences
// dl, dc, dr of the left, own and right cells
__device__ __forceinline__ void cs_constrain(double a, double l, double r, double dl, double dc,
                                             double dr, double& lo, double& hi) {
  if ((hi - a) * (a - lo) <= 0.0 || (r - a) * (a - l) <= 0.0) {
    const double d = -2.0 * (6.0 * a - 3.0 * (lo + hi));
    constexpr double C = 1.25;
    const bool pos = d > 0.0 && dl > 0.0 && dc > 0.0 && dr > 0.0;
    const bool neg = d < 0.0 && dl < 0.0 && dc < 0.0 && dr < 0.0;
    if (d != 0.0 && (pos || neg)) {
      const double m = fmin(fabs(d), C * fmin(fabs(dc), fmin(fabs(dl), fabs(dr))));
      const double s = (pos ? m : -m) / d;
      lo = a + (lo - a) * s;
      hi = a + (hi - a) * s;
    } else {
      lo = a;
      hi = a;
    }
    return;
  }
  if (fabs(hi - a) >= 2.0 * fabs(lo - a)) hi = a - 2.0 * (lo - a);
  if (fabs(lo - a) >= 2.0 * fabs(hi - a)) lo = a - 2.0 * (hi - a);
}

template <int RC>
__device__ __forceinline__ void recon_face(double m3, double m2, double m1, double p0, double p1,
                                           double p2, double& qL, double& qR) {
  if constexpr (RC == 0) {
    qL = m1;
    qR = p0;
  } else if constexpr (RC == 1) {
    qL = m1 + vl_half_slope(m2, m1, p0);
    qR = p0 - vl_half_slope(m1, p0, p1);
  } else if constexpr (RC == 2) {
    qL = wenoz(m3, m2, m1, p0, p1);
    qR = wenoz(p2, p1, p0, m1, m2);
  } else if constexpr (RC == 3) {
    const double s_m2 = cw_dm(m3, m2, m1), s_m1 = cw_dm(m2, m1, p0);
    const double s_p0 = cw_dm(m1, p0, p1), s_p1 = cw_dm(p0, p1, p2);
    const double ia = 0.5 * (m2 + m1) - (s_m1 - s_m2) * (1.0 / 6.0);
    double ib = 0.5 * (m1 + p0) - (s_p0 - s_m1) * (1.0 / 6.0);
    const double ic = 0.5 * (p0 + p1) - (s_p1 - s_p0) * (1.0 / 6.0);
    double lo = ia, hi = ib;
    cw_constrain(m1, lo, hi);
    qL = hi;
    lo = ib;
    hi = ic;
    cw_constrain(p0, lo, hi);
    qR = lo;
  } else {
    const double d_m2 = (m3 + m1) - 2.0 * m2, d_m1 = (m2 + p0) - 2.0 * m1;
    const double d_p0 = (m1 + p1) - 2.0 * p0, d_p1 = (p0 + p2) - 2.0 * p1;
    const double ia = cs_iface(m3, m2, m1, p0, d_m2, d_m1);
    const double ib = cs_iface(m2, m1, p0, p1, d_m1, d_p0);
    const double ic = cs_iface(m1, p0, p1, p2, d_p0, d_p1);
    double lo = ia, hi = ib;
    cs_constrain(m1, m2, p0, d_m2, d_m1, d_p0, lo, hi);
    qL = hi;
    lo = ib;
    hi = ic;
    cs_constrain(p0, m1, p1, d_m1, d_p0, d_p1, lo, hi);
    qR = lo;
  }
}

template <typename F>
inline void recon_dispatch(int rc, F&& f) {
  switch (rc) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: f(std::integral_constant<int, 4>{}); break;
  }
}

// ADM matter sources for the spacetime coupling (Sec. III-A): the
// stress-energy tensor of Eq. 2 projected on the slice, from the primitives
// and the densitized cell-centred field.  out = (E, S_x, S_y, S_z, S_xx,
// S_xy, S_xz, S_yy, S_yz, S_zz), lower indices, not densitized; with the
// slice projection of b^mu, b_i = B_i / W + W (B.v) v_i:
//   E = (rho h + b^2) W^2 - (P + b^2/2) - W^2 (B.v)^2,
//   S_i = (rho h + b^2) W^2 v_i - W (B.v) b_i,
//   S_ij = (rho h + b^2) W^2 v_i v_j + (P + b^2/2) gamma_ij - b_i b_j.
__device__ __forceinline__ void matter_sources(const Eos& e, const M3& m, const double w[5],
                                               const double Bt[3], double out[10]) {
  const double is = 1.0 / m.sg;
  const double B[3] = {Bt[0] * is, Bt[1] * is, Bt[2] * is};
  double ul[3], Bl[3];
  lower(m.g, w[1], w[2], w[3], ul[0], ul[1], ul[2]);
  lower(m.g, B[0], B[1], B[2], Bl[0], Bl[1], Bl[2]);
  const double W = sqrt(1.0 + w[1] * ul[0] + w[2] * ul[1] + w[3] * ul[2]);
  const double iW = 1.0 / W;
  const double vl[3] = {ul[0] * iW, ul[1] * iW, ul[2] * iW};
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  const double Bv = B[0] * vl[0] + B[1] * vl[1] + B[2] * vl[2];
  const double rho = w[0], P = w[4];
  const double h = 1.0 + eos_eps_from_P(e, rho, P) + P / rho;
  const double b2 = B2 * iW * iW + Bv * Bv;
  const double ew = (rho * h + b2) * W * W;
  const double pt = P + 0.5 * b2;
  const double wbv = W * Bv;
  double bl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) bl[a] = Bl[a] * iW + wbv * vl[a];
  out[0] = ew - pt - wbv * wbv;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[1 + a] = ew * vl[a] - wbv * bl[a];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = a; c < 3; ++c)
      out[4 + sym(a, c)] = ew * vl[a] * vl[c] + pt * m.g[sym(a, c)] - bl[a] * bl[c];
}

// atmosphere rules on a reconstructed face state (Sec. III-C)
__device__ __forceinline__ void floor_face(const Eos& e, const grmhd_params& p, double q[5]) {
  if (q[0] < p.f_thr * p.rho_atm) {
    q[0] = p.rho_atm;
    q[1] = q[2] = q[3] = 0.0;
    q[4] = eos_P_from_T(e, p.rho_atm, p.T_atm);
  } else if (eos_T_from_P(e, q[0], q[4]) < p.T_atm) {
    q[4] = eos_P_from_T(e, q[0], p.T_atm);
  }
}

// Eq. 7 at a point (densitized), used by the inversion and prim2con
__device__ __forceinline__ void prim_to_cons(const Eos& e, const M3& m, const double w[5],
                                             const double Bt[3], double U[5]) {
  const double is = 1.0 / m.sg;
  const double B[3] = {Bt[0] * is, Bt[1] * is, Bt[2] * is};
  double ul[3], Bl[3];
  lower(m.g, w[1], w[2], w[3], ul[0], ul[1], ul[2]);
  lower(m.g, B[0], B[1], B[2], Bl[0], Bl[1], Bl[2]);
  const double usq = w[1] * ul[0] + w[2] * ul[1] + w[3] * ul[2];
  const double W = sqrt(1.0 + usq);
  const double iW = 1.0 / W;
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  const double Bv = (B[0] * ul[0] + B[1] * ul[1] + B[2] * ul[2]) * iW;
  const double rho = w[0], P = w[4];
  const double eps = eos_eps_from_P(e, rho, P);
  const double h = 1.0 + eps + P / rho;
  const double D = rho * W;
  const double ehw = rho * h * W * W + B2;
  U[0] = m.sg * D;
#pragma unroll
  for (int a = 0; a < 3; ++a) U[1 + a] = m.sg * (ehw * ul[a] * iW - Bv * Bl[a]);
  U[4] = m.sg * (tau_hydro(D, usq, W, rho, eps, P) + B2 - 0.5 * (Bv * Bv + B2 / (W * W)));
}

// ---------------------------------------------------------------------------
// C2P: Kastaun master function in mu = 1/(hW)
// ---------------------------------------------------------------------------
struct KState {
  double D, q, r2, b2, s, v0sq;
};

struct KEval { double chi, rb2, qb, vsq, W, rho, eps, P; };

__device__ __forceinline__ KEval k_eval(const Eos& e, const KState& k, double mu) {
  KEval o;
  const double chi = rcp_nr(1.0 + mu * k.b2);
  const double rb2 = chi * chi * k.r2 + mu * chi * (1.0 + chi) * (k.s * k.s);
  const double qb = k.q - 0.5 * k.b2 - 0.5 * (mu * mu) * (chi * chi) * (k.b2 * k.r2 - k.s * k.s);
  const double vsq = fmin(mu * mu * rb2, k.v0sq);
  const double sw = sqrt(1.0 - vsq);      // 1 / W
  const double W = rcp_nr(sw);
  const double rho = k.D * sw;
  double eps = W * (qb - mu * rb2) + vsq * (W * W) / (1.0 + W);
  eps = fmax(eps, eos_eps_min(e, rho));
  o.chi = chi; o.rb2 = rb2; o.qb = qb; o.vsq = vsq; o.W = W; o.rho = rho; o.eps = eps;
  o.P = eos_P_from_eps(e, rho, eps);
  return o;
}

__device__ __forceinline__ double k_master(const Eos& e, const KState& k, double mu) {
  const KEval s = k_eval(e, k, mu);
  const double a = s.P * rcp_nr(s.rho * (1.0 + s.eps));
  const double nu = fmax((1.0 + a) * (1.0 + s.eps) * rcp_nr(s.W), (1.0 + a) * (1.0 + s.qb - mu * s.rb2));
  return mu - rcp_nr(nu + mu * s.rb2);
}

__device__ __forceinline__ double k_aux(const KState& k, double mu) {
  const double chi = 1.0 / (1.0 + mu * k.b2);
  const double rb2 = chi * chi * k.r2 + mu * chi * (1.0 + chi) * (k.s * k.s);
  return mu * sqrt(1.0 + rb2) - 1.0;     // minimum enthalpy h0 = 1
}

// Brent (1973): bracketing root finder; f(a) <= 0 <= f(b) or the reverse.
// Returns the root; ok = false on the iteration cap or a non-finite value.
template <class Fn>
__device__ __forceinline__ double brent_root(Fn f, double a, double b, double fa, double fb,
                                             double rtol, int maxit, int& nev, bool& ok) {
  ok = true;
  if (fa == 0.0) return a;
  if (fb == 0.0) return b;
  double c = a, fc = fa, d = b - a, e = d;
  for (int it = 0; it < maxit; ++it) {
    if ((fb > 0.0) == (fc > 0.0)) {
      c = a; fc = fa; d = b - a; e = d;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b; b = c; c = a;
      fa = fb; fb = fc; fc = fa;
    }
    const double tol1 = (2.0 * kEps + 0.5 * rtol) * fabs(b) + 1e-300;
    const double xm = 0.5 * (c - b);
    if (fabs(xm) <= tol1 || fb == 0.0) return b;
    bool bisect = true;
    if (fabs(e) >= tol1 && fabs(fa) > fabs(fb)) {
      const double s = fb / fa;
      double p, q;
      if (a == c) {
        p = 2.0 * xm * s;
        q = 1.0 - s;
      } else {
        const double qq = fa / fc, r = fb / fc;
        p = s * (2.0 * xm * qq * (qq - r) - (b - a) * (r - 1.0));
        q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
      }
      if (p > 0.0) q = -q; else p = -p;
      if (2.0 * p < fmin(3.0 * xm * q - fabs(tol1 * q), fabs(e * q))) {
        e = d;
        d = p / q;
        bisect = false;
      }
    }
    if (bisect) { d = xm; e = d; }
    a = b;
    fa = fb;
    b += fabs(d) > tol1 ? d : (xm > 0.0 ? tol1 : -tol1);
    fb = f(b);
    ++nev;
    if (!__builtin_isfinite(fb)) { ok = false; return b; }
  }
  ok = false;
  return b;
}

__device__ __forceinline__ void atmosphere(const Eos& e, const grmhd_params& p, double w[5]) {
  w[0] = p.rho_atm;
  w[1] = 0.0; w[2] = 0.0; w[3] = 0.0;
  w[4] = eos_P_from_T(e, p.rho_atm, p.T_atm);
}

constexpr uint32_t kFloorBits = GRMHD_F_C2P_FAIL | GRMHD_F_DFLOOR | GRMHD_F_TAUFLOOR |
                                GRMHD_F_MAGCAP | GRMHD_F_TFLOOR | GRMHD_F_RHOFLOOR | GRMHD_F_MAXIT;

// Inversion state between the conserved-floor rules and the root solve.
struct C2PWork {
  KState k;
  double ru[3], bu[3];
  uint32_t fl;
  bool done;      // an atmosphere rule already produced w and U
};

// Conserved-variable rules of Sec. III-C (non-finite input, D floor,
// magnetisation cap, tau floor) and the scaled variables of the master
// function.  When done is set, w and U are final.
__device__ __forceinline__ C2PWork c2p_prepare(const Eos& e, const grmhd_params& p, const M3& m,
                                               double U[5], const double Bt[3], double w[5]) {
  C2PWork cw;
  cw.fl = 0;
  cw.done = false;
  const double is = 1.0 / m.sg;
  double D = U[0] * is;
  const double Sx = U[1] * is, Sy = U[2] * is, Sz = U[3] * is;
  double tau = U[4] * is;
  const double B[3] = {Bt[0] * is, Bt[1] * is, Bt[2] * is};
  double Bl[3];
  lower(m.g, B[0], B[1], B[2], Bl[0], Bl[1], Bl[2]);
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  const bool finite = __builtin_isfinite(D) && __builtin_isfinite(Sx) && __builtin_isfinite(Sy) &&
                      __builtin_isfinite(Sz) && __builtin_isfinite(tau);
  if (!finite || D < p.f_thr * p.rho_atm) {
    atmosphere(e, p, w);
    prim_to_cons(e, m, w, Bt, U);
    cw.fl = finite ? GRMHD_F_DFLOOR : GRMHD_F_C2P_FAIL;
    cw.done = true;
    cw.k.D = 1.0; cw.k.q = 0.0; cw.k.r2 = 0.0; cw.k.b2 = 0.0; cw.k.s = 0.0; cw.k.v0sq = 0.0;
    cw.ru[0] = cw.ru[1] = cw.ru[2] = 0.0;   // defined on every path: in a loop over
    cw.bu[0] = cw.bu[1] = cw.bu[2] = 0.0;   // states, undefined ones get carried across passes
    return cw;
  }
  if (B2 / D > p.M_max) {
    D = B2 / p.M_max;
    cw.fl |= GRMHD_F_MAGCAP;
  }
  const double tau_atm = D * eos_eps_from_T(e, D, p.T_atm) + 0.5 * B2;
  if (tau < tau_atm * (1.0 - kFloorMargin)) {
    tau = tau_atm;
    cw.fl |= GRMHD_F_TAUFLOOR;
  }
  KState& k = cw.k;
  k.D = D;
  const double iD = 1.0 / D;
  k.q = tau * iD;
  const double rl[3] = {Sx * iD, Sy * iD, Sz * iD};
  cw.ru[0] = m.u[0] * rl[0] + m.u[1] * rl[1] + m.u[2] * rl[2];
  cw.ru[1] = m.u[1] * rl[0] + m.u[3] * rl[1] + m.u[4] * rl[2];
  cw.ru[2] = m.u[2] * rl[0] + m.u[4] * rl[1] + m.u[5] * rl[2];
  k.r2 = rl[0] * cw.ru[0] + rl[1] * cw.ru[1] + rl[2] * cw.ru[2];
  const double isD = 1.0 / sqrt(D);
  cw.bu[0] = B[0] * isD; cw.bu[1] = B[1] * isD; cw.bu[2] = B[2] * isD;
  k.b2 = B2 * iD;
  k.s = rl[0] * cw.bu[0] + rl[1] * cw.bu[1] + rl[2] * cw.bu[2];
  const double z2 = k.r2;      // z0 = r/h0 with h0 = 1
  k.v0sq = z2 / (1.0 + z2);
  return cw;
}

// For a loop over states: the EOS and parameter fields that the ideal-gas
// inversion reads, marked as redefined at the top of every pass (an empty
// asm on their scalar registers).  Otherwise the compiler hoists the FP64
// constants derived from them out of the loop into vector registers that
// stay live across the root solve (about 24 VGPRs: one wave per SIMD less).
__device__ __forceinline__ void consts_per_pass(Eos& e, grmhd_params& p) {
  __asm__ volatile("" : "+s"(e.gam), "+s"(e.gth), "+s"(p.rho_atm), "+s"(p.T_atm), "+s"(p.f_thr),
                   "+s"(p.M_max), "+s"(p.c2p_tol), "+s"(p.c2p_maxit));
}

// Root solve, recovery, primitive floors and the failure policy.  With
// use_br, [blo, bhi] is tried first (learned bracket).
// Root solve and primitive rules of one prepared cell.  Needs neither the
// metric nor the field: when the result has a kFloorBits rule set, the
// caller rebuilds U from w (prim_to_cons) with the metric and field it
// reloads, so that they need not stay live across the root solve.
__device__ __forceinline__ uint32_t c2p_lean(const Eos& e, const grmhd_params& p, C2PWork& cw,
                                             double w[5], bool use_br, double blo, double bhi,
                                             int& nev, double& mu_out) {
  uint32_t fl = cw.fl;
  const KState& k = cw.k;
  const double* ru = cw.ru;
  const double* bu = cw.bu;
  auto fm = [&](double x) { return k_master(e, k, x); };
  nev = 0;
  mu_out = 0.0;
  // Bracket: the given one when f changes sign over it, else (0, 1] cut at
  // mu_+.  One Brent loop serves both, so that lanes of a wave that fall
  // back do not run a second, serialised root loop.
  double lo = 0.0, hi = 1.0, flo = 0.0, fhi = 0.0;
  bool have = false;
  if (use_br) {
    double l0 = fmax(blo, 0.0), h0 = fmin(bhi, 1.0);
    if (l0 < h0 && __builtin_isfinite(l0) && __builtin_isfinite(h0)) {
      flo = fm(l0);
      fhi = fm(h0);
      nev += 2;
      have = flo <= 0.0 && fhi >= 0.0;
      if (!have) fl |= GRMHD_F_BRACKET_FALLBACK;
      // A bracket that misses the root (mostly by little) is first moved
      // towards it, 4 and then 16 times its width, one evaluation each; only
      // then the full bracket.  f(0) < 0, so moving down stays valid.
      for (int x = 0; x < 2 && !have && __builtin_isfinite(flo) && __builtin_isfinite(fhi); ++x) {
        const double wdt = 4.0 * (h0 - l0);
        if (flo > 0.0 && fhi > 0.0) {         // root below the bracket
          h0 = l0; fhi = flo;
          l0 = fmax(l0 - wdt, 0.0);
          flo = fm(l0);
          ++nev;
        } else if (flo < 0.0 && fhi < 0.0 && h0 < 1.0) {   // root above it
          l0 = h0; flo = fhi;
          h0 = fmin(h0 + wdt, 1.0);
          fhi = fm(h0);
          ++nev;
        } else {
          break;
        }
        have = flo <= 0.0 && fhi >= 0.0;
      }
      if (have) {
        lo = l0;
        hi = h0;
      }
    } else {
      fl |= GRMHD_F_BRACKET_FALLBACK;
    }
  }
  bool valid = true;
  if (!have) {
    lo = 0.0;
    hi = 1.0;
    flo = fm(0.0);
    fhi = fm(hi);
    nev += 2;
    if (fhi < 0.0) {
      // bound from above by the root mu_+ of the auxiliary function
      auto fa = [&](double x) { return k_aux(k, x); };
      bool oka;
      const double mp = brent_root(fa, 0.0, 1.0, fa(0.0), fa(1.0), 1e-15, p.c2p_maxit, nev, oka);
      hi = fmin(mp * (1.0 + 4.0 * kEps), 1.0);
      fhi = fm(hi);
      nev += 1;
    }
    valid = !(flo > 0.0 || fhi < 0.0 || !__builtin_isfinite(flo) || !__builtin_isfinite(fhi));
  }
  bool ok = false;
  double mu = 0.0;
  if (valid) mu = brent_root(fm, lo, hi, flo, fhi, p.c2p_tol, p.c2p_maxit, nev, ok);
  mu_out = mu;
  bool good = ok && __builtin_isfinite(mu);
  if (good) {
    const KEval s = k_eval(e, k, mu);
    const double f1 = mu * s.chi, f2 = mu * k.s;
    w[0] = s.rho;
    w[1] = s.W * (f1 * (ru[0] + f2 * bu[0]));
    w[2] = s.W * (f1 * (ru[1] + f2 * bu[1]));
    w[3] = s.W * (f1 * (ru[2] + f2 * bu[2]));
    w[4] = s.P;
    good = __builtin_isfinite(w[0]) && __builtin_isfinite(w[1]) && __builtin_isfinite(w[2]) &&
           __builtin_isfinite(w[3]) && __builtin_isfinite(w[4]);
    if (good) {
      if (w[0] < p.f_thr * p.rho_atm) {
        atmosphere(e, p, w);
        fl |= GRMHD_F_RHOFLOOR;
      } else if (eos_T_from_P(e, w[0], w[4]) < p.T_atm * (1.0 - kFloorMargin)) {
        w[4] = eos_P_from_T(e, w[0], p.T_atm);
        fl |= GRMHD_F_TFLOOR;
      }
    }
  } else {
    fl |= ok ? 0u : GRMHD_F_MAXIT;
  }
  if (!good) {
    atmosphere(e, p, w);
    fl |= GRMHD_F_C2P_FAIL;
  }
  return fl;
}

__device__ __forceinline__ uint32_t c2p_solve(const Eos& e, const grmhd_params& p, const M3& m,
                                              C2PWork& cw, double U[5], const double Bt[3],
                                              double w[5], bool use_br, double blo, double bhi,
                                              int& nev, double& mu_out) {
  const uint32_t fl = c2p_lean(e, p, cw, w, use_br, blo, bhi, nev, mu_out);
  if (fl & kFloorBits) prim_to_cons(e, m, w, Bt, U);
  return fl;
}

// Inversion of one cell with the atmosphere rules of Sec. III-C.  U
// (densitized) is rewritten from the final primitives whenever a rule fires.
__device__ __forceinline__ uint32_t c2p_cell(const Eos& e, const grmhd_params& p, const M3& m,
                                             double U[5], const double Bt[3], double w[5],
                                             bool use_br, double blo, double bhi, int& nev,
                                             double& mu_out) {
  C2PWork cw = c2p_prepare(e, p, m, U, Bt, w);
  if (cw.done) {
    nev = 0;
    mu_out = 0.0;
    return cw.fl;
  }
  return c2p_solve(e, p, m, cw, U, Bt, w, use_br, blo, bhi, nev, mu_out);
}

}  // namespace gk
