/*
 * grmhd_oracle.c -- plain, slow FP64 CPU oracle of one Runge-Kutta stage of
 * the 3+1 Valencia GRMHD finite-volume update (arXiv 2409.10384, Sec. II-III).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code, header,
 * table or helper with the HIP library; the two are written independently from
 * the paper and must agree to rounding.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off so every operation is an
 * IEEE-rounded double operation in source order.
 *
 * What each part follows (section / equation of the paper):
 *   EOS                ideal gas P=(Gamma-1) rho eps; hybrid piecewise polytrope
 *                      with a thermal Gamma_th part (Sec. III-D, "PrimitiveSolver")
 *   prim -> cons       Eq. 7 (densitized by sqrt(gamma), Sec. II); tau uses an
 *                      exact algebraic rearrangement of Eq. 7c that avoids the
 *                      rho h W^2 - P - D cancellation
 *   b^mu               Eq. 8
 *   fluxes             Eq. 9
 *   sources            Eq. 10
 *   reconstruction     of rho, W v^i, P (Sec. III-B): donor cell; PLM with van
 *                      Leer's (1974) limiter; PPM4, the piecewise-parabolic method
 *                      of Colella & Woodward (1984); PPMX, the extremum-preserving
 *                      limiter of Colella & Sekora (2008); WENOZ (Borges et al. 2008)
 *   Riemann solver     HLLE / LLF (Sec. III-B)
 *   CT                 upwind constrained transport (Sec. III-B; Gardiner & Stone)
 *   floors             atmosphere rules for primitive and conserved variables
 *                      (Sec. III-C)
 *   FOFC, FOFC+DMP     first-order flux correction and the relaxed discrete
 *                      maximum principle, Eq. 12 (Sec. III-C)
 *   C2P                master function of Kastaun et al. 2021 in mu = 1/(hW),
 *                      bracketed with Brent's method (Sec. III-D)
 *   matter sources     E, S_i, S_ij of the stress-energy tensor for the
 *                      spacetime coupling (Sec. III-A, Eq. 2, 5, 8)
 *   excision           atmosphere where alpha < alpha_min (Sec. IV)
 *
 * Readings where the paper is silent are listed in the design notes of the
 * repository (face metric by 4th-order Lagrange interpolation, 4th-order
 * centred metric derivatives, WENOZ p=2 eps=1e-40, fast-magnetosonic wave
 * speeds, SSP-RK2 in Shu-Osher form, DMP on the stage-input state, ...).
 *
 * Parity status of each function is stated beside it: every function below
 * is pinned by a CPU test against the paper or the mathematics.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* parameters (Sec. III-B..III-D)                                             */
/* ------------------------------------------------------------------------- */
typedef struct {
  double gamma;       /* ideal-gas adiabatic index */
  double rho_b[3];    /* hybrid: dividing densities between cold pieces */
  double K0;          /* hybrid: polytropic constant of the first piece */
  double Gam[4];      /* hybrid: adiabatic index of each cold piece */
  double gamma_th;    /* hybrid: thermal index */
  double rho_atm, T_atm, f_thr, M_max;   /* atmosphere (Sec. III-C) */
  double dmp_M;       /* <=0: no DMP; else relaxed DMP factor M of Eq. 12 */
  double c2p_tol;     /* relative tolerance of the root bracket */
  int32_t eos;        /* 0 ideal gas, 1 hybrid piecewise polytrope */
  int32_t npieces;    /* hybrid: number of cold pieces (1..4) */
  int32_t recon;      /* 0 donor cell, 1 PLM, 2 WENOZ, 3 PPM4, 4 PPMX */
  int32_t riemann;    /* 0 LLF, 1 HLLE */
  int32_t fofc;       /* 0 off, 1 on */
  int32_t c2p_maxit;  /* iteration cap of the root solve */
} or_params;

enum {
  F_C2P_FAIL = 1 << 0, F_DFLOOR = 1 << 1, F_TAUFLOOR = 1 << 2, F_MAGCAP = 1 << 3,
  F_TFLOOR = 1 << 4, F_RHOFLOOR = 1 << 5, F_FOFC = 1 << 6, F_DMP = 1 << 7,
  F_BRACKET_FALLBACK = 1 << 8, F_MAXIT = 1 << 9, F_EXCISED = 1 << 10
};
#define F_FLOORS (F_C2P_FAIL | F_DFLOOR | F_TAUFLOOR | F_MAGCAP | F_TFLOOR | F_RHOFLOOR | F_MAXIT)

/* Reading of "a state requires a floor" (Sec. III-C): the tau and T floors
   fire only when the value lies below the floor by more than a rounding
   margin.  A cell sitting at the atmosphere values is recovered at
   T_atm (1 +- a few ulp); without the margin such a cell would randomly
   count as needing the floor (and be FOFC-flagged) on rounding alone. */
#define FLOOR_MARGIN 1e-10

/* Decision margin (test instrument, 0 in every ordinary run): each threshold
   test of the method -- the face and inversion floors, the magnetisation cap,
   the relaxed DMP bounds of Eq. 12 and the vanishing-mass-flux test of the
   Riemann flux -- is taken against its threshold moved by the relative amount
   g_margin (floors and the cap: thr (1 + m); DMP: [lo - m|lo|, hi + m|hi|];
   mass flux: 1e-12 scale (1 + m)).  With m = 0 each moved threshold is the
   threshold itself, bit for bit.  Runs at m = +delta and m = -delta differ
   exactly where some decision lies within a relative delta of its threshold,
   which is how the parity tests find the cells a rounding-level difference
   could send the other way. */
static double g_margin = 0.0;
void or_set_decision_margin(double m) { g_margin = m; }

/* OpenMP threads of the oracle's loops (timing of the CPU baseline) */
#ifdef _OPENMP
#include <omp.h>
int or_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}
#else
int or_set_threads(int n) {
  (void)n;
  return 1;
}
#endif
#define THR(x) ((x) * (1.0 + g_margin))

/* Term magnitudes (test instrument, off unless set).  When set, the update
   writes for every interior cell and component the sum of the magnitudes of
   the terms it adds up, |a0 U^n| + |a1 U^(s)| + |b| dt (sum_d (|F_hi| +
   |F_lo|) / dx_d + the magnitudes of the source terms), and CT does the same
   for every interior face, with the magnitudes of the terms of the corner
   EMFs and of the cell-centre EMFs they use.  Those are the scales of the
   rounding errors of the two sums: a value formed by cancellation (momentum
   near hydrostatic balance, a face field under a nearly vanishing curl) is
   rounded relative to them, not to itself.  u: nblk x 5 padded cell arrays,
   bf: nblk x 3 face arrays (interiors written). */
static double **g_tscale_u = NULL;
static double **g_tscale_b = NULL;
static double **g_tscale_f = NULL;   /* flux-term magnitudes, nblk x 21, set by or_stage */
void or_set_term_scales(double **u, double **bf) {
  g_tscale_u = u;
  g_tscale_b = bf;
}
/* the flux-term magnitudes alone (nblk x 21 face arrays, as the flux
   workspace of or_stage_steps), for tests of the face fluxes */
void or_set_flux_term_scales(double **f) { g_tscale_f = f; }

/* ------------------------------------------------------------------------- */
/* equation of state                                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
  int type, n;
  double gam;
  double rb[3], K[4], G[4], a[4];
  double gth;
} eos_t;

static void eos_setup(const or_params *p, eos_t *e) {
  memset(e, 0, sizeof(*e));
  e->type = p->eos;
  e->gam = p->gamma;
  e->gth = p->gamma_th;
  e->n = p->eos == 1 ? p->npieces : 1;
  if (p->eos == 1) {
    /* continuity of P_cold and eps_cold at each dividing density fixes
       K_{i+1} and the additive constant a_{i+1}; a_0 = 0 so eps_cold(0)=0 */
    e->K[0] = p->K0;
    e->a[0] = 0.0;
    for (int i = 0; i < e->n; ++i) e->G[i] = p->Gam[i];
    for (int i = 0; i + 1 < e->n; ++i) {
      double r = p->rho_b[i];
      e->rb[i] = r;
      e->K[i + 1] = e->K[i] * pow(r, e->G[i] - e->G[i + 1]);
      double eps_lo = e->a[i] + e->K[i] * pow(r, e->G[i] - 1.0) / (e->G[i] - 1.0);
      double eps_hi_noa = e->K[i + 1] * pow(r, e->G[i + 1] - 1.0) / (e->G[i + 1] - 1.0);
      e->a[i + 1] = eps_lo - eps_hi_noa;
    }
  }
}

static int eos_piece(const eos_t *e, double rho) {
  int i = 0;
  while (i + 1 < e->n && rho >= e->rb[i]) ++i;
  return i;
}
static double eos_pcold(const eos_t *e, double rho) {
  if (e->type == 0) return 0.0;
  int i = eos_piece(e, rho);
  return e->K[i] * pow(rho, e->G[i]);
}
static double eos_ecold(const eos_t *e, double rho) {
  if (e->type == 0) return 0.0;
  int i = eos_piece(e, rho);
  return e->a[i] + e->K[i] * pow(rho, e->G[i] - 1.0) / (e->G[i] - 1.0);
}
/* P(rho, eps) */
static double eos_press(const eos_t *e, double rho, double eps) {
  if (e->type == 0) return (e->gam - 1.0) * rho * eps;
  return eos_pcold(e, rho) + (e->gth - 1.0) * rho * (eps - eos_ecold(e, rho));
}
/* eps(rho, P) */
static double eos_eps_P(const eos_t *e, double rho, double P) {
  if (e->type == 0) return P / ((e->gam - 1.0) * rho);
  return eos_ecold(e, rho) + (P - eos_pcold(e, rho)) / ((e->gth - 1.0) * rho);
}
/* temperature (k_B = m_b = 1): ideal T = P/rho; hybrid T = P_th/rho */
static double eos_T(const eos_t *e, double rho, double P) {
  if (e->type == 0) return P / rho;
  return (P - eos_pcold(e, rho)) / rho;
}
static double eos_P_T(const eos_t *e, double rho, double T) {
  return eos_pcold(e, rho) + rho * T;
}
static double eos_eps_T(const eos_t *e, double rho, double T) {
  if (e->type == 0) return T / (e->gam - 1.0);
  return eos_ecold(e, rho) + T / (e->gth - 1.0);
}
static double eos_eps_min(const eos_t *e, double rho) { return eos_ecold(e, rho); }
/* minimum enthalpy over the EOS: 1 for both EOSs (eps_cold(0)=0, P/rho>=0) */
static double eos_h0(const eos_t *e) { (void)e; return 1.0; }
/* squared sound speed c_s^2 = (dP/drho|_eps + P/rho^2 dP/deps|_rho) / h */
static double eos_cs2(const eos_t *e, double rho, double eps, double P) {
  double h = 1.0 + eps + P / rho;
  if (e->type == 0) return e->gam * P / (rho * h);
  int i = eos_piece(e, rho);
  double pc = e->K[i] * pow(rho, e->G[i]);
  double ec = e->a[i] + e->K[i] * pow(rho, e->G[i] - 1.0) / (e->G[i] - 1.0);
  double dPdrho = e->G[i] * pc / rho + (e->gth - 1.0) * (eps - ec) - (e->gth - 1.0) * pc / rho;
  double dPdeps = (e->gth - 1.0) * rho;
  return (dPdrho + P / (rho * rho) * dPdeps) / h;
}

/* ------------------------------------------------------------------------- */
/* 3-metric (Eq. 5).  Symmetric storage xx, xy, xz, yy, yz, zz               */
/* ------------------------------------------------------------------------- */
typedef struct { double g[3][3], gu[3][3], det, sg; } met3;

static void met_set(met3 *m, const double s[6]) {
  m->g[0][0] = s[0]; m->g[0][1] = m->g[1][0] = s[1]; m->g[0][2] = m->g[2][0] = s[2];
  m->g[1][1] = s[3]; m->g[1][2] = m->g[2][1] = s[4]; m->g[2][2] = s[5];
  double (*g)[3] = m->g;
  double c00 = g[1][1] * g[2][2] - g[1][2] * g[2][1];
  double c01 = g[1][2] * g[2][0] - g[1][0] * g[2][2];
  double c02 = g[1][0] * g[2][1] - g[1][1] * g[2][0];
  m->det = g[0][0] * c00 + g[0][1] * c01 + g[0][2] * c02;
  double id = 1.0 / m->det;
  m->gu[0][0] = c00 * id;
  m->gu[0][1] = m->gu[1][0] = c01 * id;
  m->gu[0][2] = m->gu[2][0] = c02 * id;
  m->gu[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[2][0]) * id;
  m->gu[1][2] = m->gu[2][1] = (g[0][2] * g[1][0] - g[0][0] * g[1][2]) * id;
  m->gu[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[1][0]) * id;
  m->sg = sqrt(m->det);
}
static void lower3(const met3 *m, const double a[3], double out[3]) {
  for (int i = 0; i < 3; ++i) {
    out[i] = 0.0;
    for (int j = 0; j < 3; ++j) out[i] += m->g[i][j] * a[j];
  }
}
static void raise3(const met3 *m, const double a[3], double out[3]) {
  for (int i = 0; i < 3; ++i) {
    out[i] = 0.0;
    for (int j = 0; j < 3; ++j) out[i] += m->gu[i][j] * a[j];
  }
}
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ------------------------------------------------------------------------- */
/* Eq. 7: primitive -> conserved at a point.                                  */
/*  w = (rho, W v^x, W v^y, W v^z, P); Bt = densitized B~^i; out densitized.  */
/* ------------------------------------------------------------------------- */
static void p2c_point(const eos_t *e, const met3 *m, const double w[5], const double Bt[3],
                      double U[5]) {
  double rho = w[0], P = w[4];
  double u[3] = {w[1], w[2], w[3]};
  double B[3] = {Bt[0] / m->sg, Bt[1] / m->sg, Bt[2] / m->sg};
  double ul[3];
  lower3(m, u, ul);
  double usq = dot3(u, ul);
  double W = sqrt(1.0 + usq);
  double v[3] = {u[0] / W, u[1] / W, u[2] / W};
  double vl[3] = {ul[0] / W, ul[1] / W, ul[2] / W};
  double Bl[3];
  lower3(m, B, Bl);
  double B2 = dot3(B, Bl), Bv = dot3(B, vl);
  double eps = eos_eps_P(e, rho, P);
  double h = 1.0 + eps + P / rho;
  double D = rho * W;
  double rhohW2 = rho * h * W * W;
  double S[3];
  for (int i = 0; i < 3; ++i) S[i] = (rhohW2 + B2) * vl[i] - Bv * Bl[i];
  /* rho h W^2 - P - D written without cancellation:
     = D (W^2-1)/(W+1) + rho eps W^2 + P (W^2-1),  W^2-1 = usq            */
  double hydro = D * usq / (W + 1.0) + rho * eps * W * W + P * usq;
  double tau = hydro + B2 - 0.5 * (Bv * Bv + B2 / (W * W));
  (void)v;
  U[0] = m->sg * D;
  U[1] = m->sg * S[0];
  U[2] = m->sg * S[1];
  U[3] = m->sg * S[2];
  U[4] = m->sg * tau;
}

/* ------------------------------------------------------------------------- */
/* ADM matter sources of the spacetime coupling (Sec. III-A: the Z4c          */
/* equations are driven by the fluid's stress-energy tensor, Eq. 2 with the   */
/* metric of Eq. 5 and b^mu of Eq. 8, projected on the slice with the unit    */
/* normal n):                                                                 */
/*   E    = n_mu n_nu T^{mu nu}            energy density of the normal frame */
/*   S_i  = -gamma_i^mu n^nu T_{mu nu}     momentum density                   */
/*   S_ij = gamma_i^mu gamma_j^nu T_{mu nu} stress                            */
/* With n_mu u^mu = -W, n_mu b^mu = -W (B.v) and the projection of b on the   */
/* slice b_i = B_i / W + W (B.v) v_i:                                         */
/*   E    = (rho h + b^2) W^2 - (P + b^2/2) - W^2 (B.v)^2                     */
/*   S_i  = (rho h + b^2) W^2 v_i - W (B.v) b_i                               */
/*   S_ij = (rho h + b^2) W^2 v_i v_j + (P + b^2/2) gamma_ij - b_i b_j        */
/* out = (E, S_x, S_y, S_z, S_xx, S_xy, S_xz, S_yy, S_yz, S_zz), not          */
/* densitized.                                                                */
/* ------------------------------------------------------------------------- */
static void matter_point(const eos_t *e, const met3 *m, const double w[5], const double Bt[3],
                         double out[10]) {
  double rho = w[0], P = w[4];
  double u[3] = {w[1], w[2], w[3]};
  double B[3] = {Bt[0] / m->sg, Bt[1] / m->sg, Bt[2] / m->sg};
  double ul[3];
  lower3(m, u, ul);
  double W = sqrt(1.0 + dot3(u, ul));
  double vl[3] = {ul[0] / W, ul[1] / W, ul[2] / W};
  double Bl[3];
  lower3(m, B, Bl);
  double B2 = dot3(B, Bl), Bv = dot3(B, vl);
  double h = 1.0 + eos_eps_P(e, rho, P) + P / rho;
  double b2 = B2 / (W * W) + Bv * Bv;
  double ew = (rho * h + b2) * W * W;
  double pt = P + 0.5 * b2;
  double bl[3];
  for (int i = 0; i < 3; ++i) bl[i] = Bl[i] / W + W * Bv * vl[i];
  out[0] = ew - pt - W * W * Bv * Bv;
  for (int i = 0; i < 3; ++i) out[1 + i] = ew * vl[i] - W * Bv * bl[i];
  static const int sym[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  for (int s6 = 0; s6 < 6; ++s6) {
    int i = sym[s6][0], j = sym[s6][1];
    out[4 + s6] = ew * vl[i] * vl[j] + pt * m->g[i][j] - bl[i] * bl[j];
  }
}

/* ------------------------------------------------------------------------- */
/* Brent's method (Brent 1973) on a bracketing interval [a,b] with            */
/* f(a) f(b) <= 0.  Stops when the half-width of the bracket is below         */
/* tol*|b| + tiny, or f(b) == 0.  Returns the number of f evaluations in      */
/* *nev; *ok = 0 on iteration cap or a bad bracket.                           */
/* ------------------------------------------------------------------------- */
typedef double (*or_fun)(double x, void *ctx);

static double brent(or_fun f, void *ctx, double a, double b, double fa, double fb, double tol,
                    int maxit, int *nev, int *ok) {
  const double eps = 2.220446049250313e-16;
  *ok = 1;
  if ((fa > 0 && fb > 0) || (fa < 0 && fb < 0) || !isfinite(fa) || !isfinite(fb)) {
    *ok = 0;
    return b;
  }
  if (fa == 0.0) return a;
  if (fb == 0.0) return b;
  double c = a, fc = fa, d = b - a, e = d;
  for (int it = 0; it < maxit; ++it) {
    if ((fb > 0 && fc > 0) || (fb < 0 && fc < 0)) {
      c = a; fc = fa; d = b - a; e = d;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b; b = c; c = a;
      fa = fb; fb = fc; fc = fa;
    }
    double tol1 = 2.0 * eps * fabs(b) + 0.5 * tol * fabs(b) + 1e-300;
    double xm = 0.5 * (c - b);
    if (fabs(xm) <= tol1 || fb == 0.0) return b;
    if (fabs(e) >= tol1 && fabs(fa) > fabs(fb)) {
      double s = fb / fa, p, q;
      if (a == c) {            /* secant step */
        p = 2.0 * xm * s;
        q = 1.0 - s;
      } else {                 /* inverse quadratic interpolation */
        double qq = fa / fc, r = fb / fc;
        p = s * (2.0 * xm * qq * (qq - r) - (b - a) * (r - 1.0));
        q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
      }
      if (p > 0) q = -q; else p = -p;
      double m1 = 3.0 * xm * q - fabs(tol1 * q), m2 = fabs(e * q);
      if (2.0 * p < (m1 < m2 ? m1 : m2)) {
        e = d; d = p / q;
      } else {
        d = xm; e = d;
      }
    } else {
      d = xm; e = d;
    }
    a = b; fa = fb;
    if (fabs(d) > tol1) b += d;
    else b += (xm > 0 ? tol1 : -tol1);
    fb = f(b, ctx);
    ++*nev;
    if (!isfinite(fb)) { *ok = 0; return b; }
  }
  *ok = 0;
  return b;
}

/* ------------------------------------------------------------------------- */
/* Kastaun et al. 2021 master function (Sec. III-D).                          */
/* Scaled variables: q = tau/D, r_i = S_i/D, B^i/sqrt(D); unknown mu = 1/(hW) */
/* ------------------------------------------------------------------------- */
typedef struct {
  const eos_t *e;
  double D, q, r2, b2, s, h0, v0sq;
} kctx;

typedef struct { double chi, rb2, qb, vsq, W, rho, eps, P; } kstate;

static void kastaun_eval(const kctx *k, double mu, kstate *o) {
  double chi = 1.0 / (1.0 + mu * k->b2);
  double rb2 = chi * chi * k->r2 + mu * chi * (1.0 + chi) * k->s * k->s;
  double qb = k->q - 0.5 * k->b2 - 0.5 * mu * mu * chi * chi * (k->b2 * k->r2 - k->s * k->s);
  double vsq = mu * mu * rb2;
  if (vsq > k->v0sq) vsq = k->v0sq;
  double W = 1.0 / sqrt(1.0 - vsq);
  double rho = k->D / W;
  double eps = W * (qb - mu * rb2) + vsq * W * W / (1.0 + W);
  double emin = eos_eps_min(k->e, rho);
  if (eps < emin) eps = emin;
  o->chi = chi; o->rb2 = rb2; o->qb = qb; o->vsq = vsq; o->W = W; o->rho = rho; o->eps = eps;
  o->P = eos_press(k->e, rho, eps);
}

static double kastaun_f(double mu, void *ctx) {
  const kctx *k = (const kctx *)ctx;
  kstate s;
  kastaun_eval(k, mu, &s);
  double a = s.P / (s.rho * (1.0 + s.eps));
  double nu1 = (1.0 + a) * (1.0 + s.eps) / s.W;
  double nu2 = (1.0 + a) * (1.0 + s.qb - mu * s.rb2);
  double nu = nu1 > nu2 ? nu1 : nu2;
  return mu - 1.0 / (nu + mu * s.rb2);
}

/* auxiliary function whose root mu_+ bounds the physical root from above */
static double kastaun_fa(double mu, void *ctx) {
  const kctx *k = (const kctx *)ctx;
  double chi = 1.0 / (1.0 + mu * k->b2);
  double rb2 = chi * chi * k->r2 + mu * chi * (1.0 + chi) * k->s * k->s;
  return mu * sqrt(k->h0 * k->h0 + rb2) - 1.0;
}

/* ------------------------------------------------------------------------- */
/* C2P with the atmosphere rules of Sec. III-C, at one point.                  */
/*  U (densitized) in/out: rewritten from the final primitives whenever a     */
/*  rule fires.  Optional bracket [blo, bhi] (learned guess); if it does not  */
/*  bracket a sign change the full bracket is used and F_BRACKET_FALLBACK set. */
/*  Returns flags; *nev the number of master-function evaluations; *mu_out.   */
/* ------------------------------------------------------------------------- */
static void atmosphere_prims(const eos_t *e, const or_params *p, double w[5]) {
  w[0] = p->rho_atm;
  w[1] = w[2] = w[3] = 0.0;
  w[4] = eos_P_T(e, p->rho_atm, p->T_atm);
}

static int c2p_point(const eos_t *e, const or_params *p, const met3 *m, double U[5],
                     const double Bt[3], double w[5], int use_bracket, double blo, double bhi,
                     int *nev, double *mu_out) {
  int flags = 0;
  *nev = 0;
  *mu_out = 0.0;
  double sg = m->sg;
  double D = U[0] / sg;
  double Sl[3] = {U[1] / sg, U[2] / sg, U[3] / sg};
  double tau = U[4] / sg;
  double B[3] = {Bt[0] / sg, Bt[1] / sg, Bt[2] / sg};
  double Bl[3];
  lower3(m, B, Bl);
  double B2 = dot3(B, Bl);

  if (!(isfinite(D) && isfinite(Sl[0]) && isfinite(Sl[1]) && isfinite(Sl[2]) && isfinite(tau))) {
    atmosphere_prims(e, p, w);
    p2c_point(e, m, w, Bt, U);
    return F_C2P_FAIL;
  }
  /* rule: D below the threshold -> atmosphere */
  if (D < THR(p->f_thr * p->rho_atm)) {
    atmosphere_prims(e, p, w);
    p2c_point(e, m, w, Bt, U);
    return F_DFLOOR;
  }
  /* rule: magnetisation cap B^2/D <= M_max by raising D */
  if (B2 / D > THR(p->M_max)) {
    D = B2 / p->M_max;
    flags |= F_MAGCAP;
  }
  /* rule: tau floor for a fluid at rest at T_atm:  tau_atm = D eps(D,T_atm) + B^2/2 */
  double tau_atm = D * eos_eps_T(e, D, p->T_atm) + 0.5 * B2;
  if (tau < THR(tau_atm * (1.0 - FLOOR_MARGIN))) {
    tau = tau_atm;
    flags |= F_TAUFLOOR;
  }

  kctx k;
  k.e = e;
  k.D = D;
  k.q = tau / D;
  double rl[3] = {Sl[0] / D, Sl[1] / D, Sl[2] / D};
  double ru[3];
  raise3(m, rl, ru);
  k.r2 = dot3(rl, ru);
  double sD = sqrt(D);
  double bu[3] = {B[0] / sD, B[1] / sD, B[2] / sD};
  k.b2 = B2 / D;
  k.s = dot3(rl, bu);
  k.h0 = eos_h0(e);
  double z0 = sqrt(k.r2) / k.h0;
  k.v0sq = z0 * z0 / (1.0 + z0 * z0);

  double tol = p->c2p_tol;
  int maxit = p->c2p_maxit;
  int ok = 0, n = 0;
  double mu = 0.0;
  int have = 0;
  if (use_bracket) {
    double lo = blo, hi = bhi;
    double mhi = 1.0 / k.h0;
    if (lo < 0.0) lo = 0.0;
    if (hi > mhi) hi = mhi;
    if (lo < hi && isfinite(lo) && isfinite(hi)) {
      double flo = kastaun_f(lo, &k), fhi = kastaun_f(hi, &k);
      n += 2;
      if (flo <= 0.0 && fhi >= 0.0) {
        int nn = 0;
        mu = brent(kastaun_f, &k, lo, hi, flo, fhi, tol, maxit, &nn, &ok);
        n += nn;
        have = 1;
      }
    }
    if (!have) flags |= F_BRACKET_FALLBACK;
  }
  if (!have) {
    /* full bracket (0, mu_hi]: mu_hi = 1/h0 if f changes sign there, else the
       root mu_+ of the auxiliary function */
    double lo = 0.0, hi = 1.0 / k.h0;
    double flo = kastaun_f(lo, &k), fhi = kastaun_f(hi, &k);
    n += 2;
    if (fhi < 0.0) {
      int nn = 0, oka = 0;
      double fa0 = kastaun_fa(0.0, &k), fa1 = kastaun_fa(hi, &k);
      double mp = brent(kastaun_fa, &k, 0.0, hi, fa0, fa1, 1e-15, maxit, &nn, &oka);
      n += nn;
      /* step just above mu_+ so the bracket end is on the f>=0 side */
      hi = mp * (1.0 + 4.0 * 2.220446049250313e-16);
      if (hi > 1.0 / k.h0) hi = 1.0 / k.h0;
      fhi = kastaun_f(hi, &k);
      n += 1;
    }
    int nn = 0;
    mu = brent(kastaun_f, &k, lo, hi, flo, fhi, tol, maxit, &nn, &ok);
    n += nn;
  }
  *nev = n;
  *mu_out = mu;
  if (!ok || !isfinite(mu)) {
    atmosphere_prims(e, p, w);
    p2c_point(e, m, w, Bt, U);
    return flags | F_C2P_FAIL | (ok ? 0 : F_MAXIT);
  }

  /* recovery at the root */
  kstate st;
  kastaun_eval(&k, mu, &st);
  double vu[3];
  for (int i = 0; i < 3; ++i) vu[i] = mu * st.chi * (ru[i] + mu * k.s * bu[i]);
  w[0] = st.rho;
  w[1] = st.W * vu[0];
  w[2] = st.W * vu[1];
  w[3] = st.W * vu[2];
  w[4] = st.P;
  if (!(isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2]) && isfinite(w[3]) && isfinite(w[4]))) {
    atmosphere_prims(e, p, w);
    p2c_point(e, m, w, Bt, U);
    return flags | F_C2P_FAIL;
  }
  /* primitive floors (Sec. III-C): rho below threshold -> atmosphere;
     T below T_atm -> reset T, keep rho and W v^i */
  if (w[0] < THR(p->f_thr * p->rho_atm)) {
    atmosphere_prims(e, p, w);
    flags |= F_RHOFLOOR;
  } else if (eos_T(e, w[0], w[4]) < THR(p->T_atm * (1.0 - FLOOR_MARGIN))) {
    w[4] = eos_P_T(e, w[0], p->T_atm);
    flags |= F_TFLOOR;
  }
  if (flags & F_FLOORS) p2c_point(e, m, w, Bt, U);
  return flags;
}

/* ------------------------------------------------------------------------- */
/* Face physics: Eq. 7-9 for one side of a face in direction d; wave speeds.  */
/*  q = (rho, W v^i, P); B = un-densitized B^i (all three); metric at face.   */
/*  U, F: 7 components D~, S~_x, S~_y, S~_z, tau~, B~^{t1}, B~^{t2} with      */
/*  t1 = (d+1)%3, t2 = (d+2)%3.                                               */
/* ------------------------------------------------------------------------- */
static void face_physics(const eos_t *e, const met3 *m, double alpha, const double beta[3], int d,
                         const double q[5], const double B[3], double U[7], double F[7],
                         double *lm, double *lp, double *Fs) {
  double rho = q[0], P = q[4];
  double u[3] = {q[1], q[2], q[3]};
  double ul[3];
  lower3(m, u, ul);
  double usq = dot3(u, ul);
  double W = sqrt(1.0 + usq);
  double v[3] = {u[0] / W, u[1] / W, u[2] / W};
  double vl[3] = {ul[0] / W, ul[1] / W, ul[2] / W};
  double Bl[3];
  lower3(m, B, Bl);
  double B2 = dot3(B, Bl), Bv = dot3(B, vl);
  double eps = eos_eps_P(e, rho, P);
  double h = 1.0 + eps + P / rho;
  double b0 = W * Bv / alpha;                              /* Eq. 8 */
  double vh[3];
  for (int i = 0; i < 3; ++i) vh[i] = v[i] - beta[i] / alpha;
  double bl[3];                                            /* b_i = B_i/W + W (B.v) v_i */
  for (int i = 0; i < 3; ++i) bl[i] = Bl[i] / W + W * Bv * vl[i];
  double bsq = B2 / (W * W) + Bv * Bv;
  double Ptot = P + 0.5 * bsq;
  double sg = m->sg;
  /* conserved (Eq. 7, densitized) */
  double D = rho * W;
  double rhohW2 = rho * h * W * W;
  double Dt = sg * D;
  double St[3];
  for (int i = 0; i < 3; ++i) St[i] = sg * ((rhohW2 + B2) * vl[i] - Bv * Bl[i]);
  double hydro = D * usq / (W + 1.0) + rho * eps * W * W + P * usq;
  double taut = sg * (hydro + B2 - 0.5 * (Bv * Bv + B2 / (W * W)));
  double Bt[3] = {sg * B[0], sg * B[1], sg * B[2]};
  double Ptt = sg * Ptot;
  /* fluxes (Eq. 9) */
  F[0] = alpha * Dt * vh[d];
  for (int i = 0; i < 3; ++i)
    F[1 + i] = alpha * St[i] * vh[d] - alpha * bl[i] * Bt[d] / W + (i == d ? alpha * Ptt : 0.0);
  F[4] = alpha * taut * vh[d] - alpha * alpha * b0 * Bt[d] / W + alpha * Ptt * v[d];
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  F[5] = alpha * (Bt[t1] * vh[d] - Bt[d] * vh[t1]);
  F[6] = alpha * (Bt[t2] * vh[d] - Bt[d] * vh[t2]);
  if (Fs) {
    /* magnitudes of the terms of each flux (term-scale instrument) */
    double aa = fabs(alpha);
    Fs[0] = fabs(F[0]);
    for (int i = 0; i < 3; ++i)
      Fs[1 + i] = aa * (fabs(St[i] * vh[d]) + fabs(bl[i] * Bt[d] / W)) + (i == d ? aa * fabs(Ptt) : 0.0);
    Fs[4] = aa * (fabs(taut * vh[d]) + aa * fabs(b0 * Bt[d] / W) + fabs(Ptt * v[d]));
    Fs[5] = aa * (fabs(Bt[t1] * vh[d]) + fabs(Bt[d] * vh[t1]));
    Fs[6] = aa * (fabs(Bt[t2] * vh[d]) + fabs(Bt[d] * vh[t2]));
  }
  U[0] = Dt; U[1] = St[0]; U[2] = St[1]; U[3] = St[2]; U[4] = taut;
  U[5] = Bt[t1]; U[6] = Bt[t2];
  /* fast magnetosonic speeds: c^2 = cs^2 + ca^2 - cs^2 ca^2 */
  double cs2 = eos_cs2(e, rho, eps, P);
  double ca2 = bsq / (rho * h + bsq);
  double c2 = cs2 + ca2 - cs2 * ca2;
  double v2 = usq / (W * W);
  double gdd = m->gu[d][d];
  double disc = c2 * (1.0 - v2) * (gdd * (1.0 - v2 * c2) - v[d] * v[d] * (1.0 - c2));
  if (disc < 0.0) disc = 0.0;
  double sq = sqrt(disc);
  double den = 1.0 - v2 * c2;
  *lp = alpha * (v[d] * (1.0 - c2) + sq) / den - beta[d];
  *lm = alpha * (v[d] * (1.0 - c2) - sq) / den - beta[d];
}

/* Mass-flux dead band.  The upwind CT (Sec. III-B) picks the upwind cell by
   the sign of the face mass flux.  Where that flux vanishes in exact
   arithmetic (e.g. atmosphere at rest on both sides) the computed value is
   rounding noise of either sign, so the pick would be arbitrary.  A mass flux
   whose magnitude is at most MASS_FLUX_ZERO times the magnitude scale of the
   Riemann formula that produced it is taken to be exactly zero. */
#define MASS_FLUX_ZERO 1e-12

/* HLLE (Harten 1983, Einfeldt 1991); LLF when riemann == 0 */
static void riemann_solve(int riemann, const double UL[7], const double FL[7], double lmL,
                          double lpL, const double UR[7], const double FR[7], double lmR,
                          double lpR, double F[7]) {
  double scale;
  if (riemann == 0) {
    double a = fabs(lmL);
    if (fabs(lpL) > a) a = fabs(lpL);
    if (fabs(lmR) > a) a = fabs(lmR);
    if (fabs(lpR) > a) a = fabs(lpR);
    for (int c = 0; c < 7; ++c) F[c] = 0.5 * (FL[c] + FR[c]) - 0.5 * a * (UR[c] - UL[c]);
    scale = 0.5 * (fabs(FL[0]) + fabs(FR[0])) + 0.5 * a * (fabs(UR[0]) + fabs(UL[0]));
  } else {
    double lr = 0.0, ll = 0.0;
    if (lpL > lr) lr = lpL;
    if (lpR > lr) lr = lpR;
    if (lmL < ll) ll = lmL;
    if (lmR < ll) ll = lmR;
    if (lr - ll == 0.0) {
      for (int c = 0; c < 7; ++c) F[c] = 0.5 * (FL[c] + FR[c]);
      scale = 0.5 * (fabs(FL[0]) + fabs(FR[0]));
    } else {
      for (int c = 0; c < 7; ++c)
        F[c] = (lr * FL[c] - ll * FR[c] + lr * ll * (UR[c] - UL[c])) / (lr - ll);
      scale = (lr * fabs(FL[0]) - ll * fabs(FR[0]) - lr * ll * (fabs(UR[0]) + fabs(UL[0]))) /
              (lr - ll);
    }
  }
  if (fabs(F[0]) <= THR(MASS_FLUX_ZERO * scale)) F[0] = 0.0;
}

/* the magnitudes of the terms of the Riemann flux (term-scale instrument):
   the same combination over the sides' flux-term magnitudes and |U| */
static void riemann_scale(int riemann, const double UL[7], const double FLs[7], double lmL,
                          double lpL, const double UR[7], const double FRs[7], double lmR,
                          double lpR, double Fs[7]) {
  if (riemann == 0) {
    double a = fabs(lmL);
    if (fabs(lpL) > a) a = fabs(lpL);
    if (fabs(lmR) > a) a = fabs(lmR);
    if (fabs(lpR) > a) a = fabs(lpR);
    for (int c = 0; c < 7; ++c) Fs[c] = 0.5 * (FLs[c] + FRs[c]) + 0.5 * a * (fabs(UR[c]) + fabs(UL[c]));
    return;
  }
  double lr = 0.0, ll = 0.0;
  if (lpL > lr) lr = lpL;
  if (lpR > lr) lr = lpR;
  if (lmL < ll) ll = lmL;
  if (lmR < ll) ll = lmR;
  if (lr - ll == 0.0) {
    for (int c = 0; c < 7; ++c) Fs[c] = 0.5 * (FLs[c] + FRs[c]);
    return;
  }
  for (int c = 0; c < 7; ++c)
    Fs[c] = (lr * FLs[c] - ll * FRs[c] - lr * ll * (fabs(UR[c]) + fabs(UL[c]))) / (lr - ll);
}

/* WENOZ (Borges et al. 2008), value at the right interface of cell 0 from
   the five cell averages q[-2..2]; p = 2, eps = 1e-40 */
static double wenoz_right(double qm2, double qm1, double q0, double qp1, double qp2) {
  double b0 = 13.0 / 12.0 * (qm2 - 2.0 * qm1 + q0) * (qm2 - 2.0 * qm1 + q0) +
              0.25 * (qm2 - 4.0 * qm1 + 3.0 * q0) * (qm2 - 4.0 * qm1 + 3.0 * q0);
  double b1 = 13.0 / 12.0 * (qm1 - 2.0 * q0 + qp1) * (qm1 - 2.0 * q0 + qp1) +
              0.25 * (qm1 - qp1) * (qm1 - qp1);
  double b2 = 13.0 / 12.0 * (q0 - 2.0 * qp1 + qp2) * (q0 - 2.0 * qp1 + qp2) +
              0.25 * (3.0 * q0 - 4.0 * qp1 + qp2) * (3.0 * q0 - 4.0 * qp1 + qp2);
  double t5 = fabs(b0 - b2);
  const double eps = 1e-40;
  double r0 = t5 / (b0 + eps), r1 = t5 / (b1 + eps), r2 = t5 / (b2 + eps);
  double a0 = 0.1 * (1.0 + r0 * r0);
  double a1 = 0.6 * (1.0 + r1 * r1);
  double a2 = 0.3 * (1.0 + r2 * r2);
  double p0 = (2.0 * qm2 - 7.0 * qm1 + 11.0 * q0) / 6.0;
  double p1 = (-qm1 + 5.0 * q0 + 2.0 * qp1) / 6.0;
  double p2 = (2.0 * q0 + 5.0 * qp1 - qp2) / 6.0;
  return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

/* PLM: cell 0 is linear with van Leer's (1974) harmonic-mean slope of the
   two one-sided differences, zero where they differ in sign. */
static void plm_edges(double qm1, double q0, double qp1, double *lo, double *hi) {
  double dl = q0 - qm1, dr = qp1 - q0;
  double slope = 0.0;
  if (dl * dr > 0.0) slope = 2.0 * dl * dr / (dl + dr);
  *lo = q0 - 0.5 * slope;
  *hi = q0 + 0.5 * slope;
}

/* PPM4 = the piecewise-parabolic method of Colella & Woodward (1984) on a
   uniform grid.  Limited average slope of cell 0 (their Eq. 1.8): the
   centred difference, bounded by twice each one-sided difference, zero at a
   local extremum. */
static double cw_slope(double qm1, double q0, double qp1) {
  double dl = q0 - qm1, dr = qp1 - q0, dc = 0.5 * (qp1 - qm1);
  if (dl * dr <= 0.0) return 0.0;
  double m = fabs(dc);
  if (2.0 * fabs(dl) < m) m = 2.0 * fabs(dl);
  if (2.0 * fabs(dr) < m) m = 2.0 * fabs(dr);
  return dc > 0.0 ? m : -m;
}

/* interface value between cells 0 and 1 (their Eqs. 1.6-1.7 with equal
   widths): the mean of the two cells less a sixth of the change of slope */
static double cw_interface(double qm1, double q0, double qp1, double qp2) {
  return 0.5 * (q0 + qp1) - (cw_slope(q0, qp1, qp2) - cw_slope(qm1, q0, qp1)) / 6.0;
}

/* edge values of cell 0 from cells -2..2, after the monotonicity constraints
   (their Eq. 1.10): flat at a local extremum; otherwise the edge on the side
   of an overshooting parabola is moved until the parabola is monotone */
static void ppm4_edges(const double q[5], double *lo, double *hi) {
  double a = q[2];
  double aL = cw_interface(q[0], q[1], q[2], q[3]);
  double aR = cw_interface(q[1], q[2], q[3], q[4]);
  if ((aR - a) * (a - aL) <= 0.0) {
    aL = a;
    aR = a;
  } else {
    double da = aR - aL;
    double a6 = 6.0 * (a - 0.5 * (aL + aR));
    if (da * a6 > da * da) aL = 3.0 * a - 2.0 * aR;
    else if (-da * da > da * a6) aR = 3.0 * a - 2.0 * aL;
  }
  *lo = aL;
  *hi = aR;
}

/* PPMX = PPM with the extremum-preserving limiter of Colella & Sekora (2008).
   Limited second derivative: the smallest magnitude of its arguments (the
   first unscaled, the rest scaled by C = 1.25) when all have one sign, else 0. */
#define CS_C 1.25
static double cs_d2lim(int n, const double *d2) {
  int pos = 1, neg = 1;
  for (int k = 0; k < n; ++k) {
    if (!(d2[k] > 0.0)) pos = 0;
    if (!(d2[k] < 0.0)) neg = 0;
  }
  if (!pos && !neg) return 0.0;
  double m = fabs(d2[0]);
  for (int k = 1; k < n; ++k)
    if (CS_C * fabs(d2[k]) < m) m = CS_C * fabs(d2[k]);
  return pos ? m : -m;
}

/* interface value between cells 0 and 1: the fourth-order value, and where
   it leaves the range of the two cells, the mean of the two cells corrected
   by a limited second derivative (an unlimited one, 3 (q0 - 2a + q1),
   returns the fourth-order value itself) */
static double cs_interface(double qm1, double q0, double qp1, double qp2) {
  double a = 7.0 / 12.0 * (q0 + qp1) - 1.0 / 12.0 * (qm1 + qp2);
  if ((a - q0) * (qp1 - a) < 0.0) {
    double d2[3];
    d2[0] = 3.0 * ((q0 + qp1) - 2.0 * a);
    d2[1] = (qm1 + qp1) - 2.0 * q0;
    d2[2] = (q0 + qp2) - 2.0 * qp1;
    a = 0.5 * (q0 + qp1) - cs_d2lim(3, d2) / 6.0;
  }
  return a;
}

/* edge values of cell 0 from cells -2..2.  At a local extremum (of the
   parabola or of the cell averages) the parabola's curvature is scaled by
   the limited second derivative over its own; elsewhere an overshooting
   edge is moved as in PPM.  Second differences are written as (sum of the
   outer values) - 2 (centre), so mirrored data give mirrored edges exactly. */
static void ppmx_edges(const double q[5], double *lo, double *hi) {
  double a = q[2];
  double aL = cs_interface(q[0], q[1], q[2], q[3]);
  double aR = cs_interface(q[1], q[2], q[3], q[4]);
  if ((aR - a) * (a - aL) <= 0.0 || (q[3] - a) * (a - q[1]) <= 0.0) {
    double d2[4];
    d2[0] = -2.0 * (6.0 * a - 3.0 * (aL + aR));
    d2[1] = (q[0] + a) - 2.0 * q[1];
    d2[2] = (q[1] + q[3]) - 2.0 * a;
    d2[3] = (a + q[4]) - 2.0 * q[3];
    double lim = cs_d2lim(4, d2);
    if (d2[0] != 0.0) {
      aL = a + (aL - a) * lim / d2[0];
      aR = a + (aR - a) * lim / d2[0];
    } else {
      aL = a;
      aR = a;
    }
  } else {
    if (fabs(aR - a) >= 2.0 * fabs(aL - a)) aR = a - 2.0 * (aL - a);
    if (fabs(aL - a) >= 2.0 * fabs(aR - a)) aL = a - 2.0 * (aR - a);
  }
  *lo = aL;
  *hi = aR;
}

/* lower and upper edge values of cell 0 from the cells -2..2 around it */
static void recon_edges(int kind, const double q[5], double *lo, double *hi) {
  switch (kind) {
    case 0: *lo = q[2]; *hi = q[2]; break;
    case 1: plm_edges(q[1], q[2], q[3], lo, hi); break;
    case 2:
      *lo = wenoz_right(q[4], q[3], q[2], q[1], q[0]);
      *hi = wenoz_right(q[0], q[1], q[2], q[3], q[4]);
      break;
    case 3: ppm4_edges(q, lo, hi); break;
    default: ppmx_edges(q, lo, hi); break;
  }
}

/* ------------------------------------------------------------------------- */
/* Block storage                                                              */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz, ng;
  double dx[3];
  double *w[5];      /* stage-input primitives rho, W v^x, W v^y, W v^z, P (padded) */
  double *un[5];     /* U^n  (padded; interior read)                          */
  double *us[5];     /* U^(s) (padded; ghosts used by the DMP)                 */
  double *bn[3];     /* B~^n on faces                                          */
  double *bs[3];     /* B~^(s) on faces                                        */
  double *adm[16];   /* alpha, beta^{x,y,z}, g_{xx,xy,xz,yy,yz,zz}, K_{xx..zz} */
  double *uo[5];     /* output U (may alias un)                               */
  double *bo[3];     /* output faces (may alias bn)                           */
  double *wo[5];     /* output primitives                                     */
  uint16_t *flags;   /* padded cell flags                                     */
  int32_t nbr[27];   /* neighbour block per offset (ox+1)+3(oy+1)+9(oz+1); -1 outflow */
  int32_t bc;        /* 0: ghosts frozen, 1: filled from nbr / outflow        */
} or_block;

static inline int64_t cidx(const or_block *b, int i, int j, int k) {
  int sx = b->nx + 2 * b->ng, sy = b->ny + 2 * b->ng;
  return ((int64_t)k * sy + j) * sx + i;
}
/* face arrays: direction d has one more entry along d */
static inline int64_t fidx(const or_block *b, int d, int i, int j, int k) {
  int sx = b->nx + 2 * b->ng, sy = b->ny + 2 * b->ng;
  if (d == 0) return ((int64_t)k * sy + j) * (sx + 1) + i;
  if (d == 1) return ((int64_t)k * (sy + 1) + j) * sx + i;
  return ((int64_t)k * sy + j) * sx + i;
}
static int64_t ncell(const or_block *b) {
  return (int64_t)(b->nx + 2 * b->ng) * (b->ny + 2 * b->ng) * (b->nz + 2 * b->ng);
}
static int64_t nface(const or_block *b, int d) {
  int64_t sx = b->nx + 2 * b->ng, sy = b->ny + 2 * b->ng, sz = b->nz + 2 * b->ng;
  return d == 0 ? (sx + 1) * sy * sz : d == 1 ? sx * (sy + 1) * sz : sx * sy * (sz + 1);
}
static int64_t nedge(const or_block *b) {
  return (int64_t)(b->nx + 2 * b->ng + 1) * (b->ny + 2 * b->ng + 1) * (b->nz + 2 * b->ng + 1);
}
static inline int64_t eidx(const or_block *b, int i, int j, int k) {
  int ex = b->nx + 2 * b->ng + 1, ey = b->ny + 2 * b->ng + 1;
  return ((int64_t)k * ey + j) * ex + i;
}

static void cell_metric(const or_block *b, int64_t c, met3 *m) {
  double s[6];
  for (int n = 0; n < 6; ++n) s[n] = b->adm[4 + n][c];
  met_set(m, s);
}

/* densitized cell-centred field: average of the two faces per direction */
static void cell_bt(const or_block *b, double *const f[3], int i, int j, int k, double Bt[3]) {
  Bt[0] = 0.5 * (f[0][fidx(b, 0, i, j, k)] + f[0][fidx(b, 0, i + 1, j, k)]);
  Bt[1] = 0.5 * (f[1][fidx(b, 1, i, j, k)] + f[1][fidx(b, 1, i, j + 1, k)]);
  Bt[2] = 0.5 * (f[2][fidx(b, 2, i, j, k)] + f[2][fidx(b, 2, i, j, k + 1)]);
}

/* primitive floors on a reconstructed face state (Sec. III-C) */
static void face_floor(const eos_t *e, const or_params *p, double q[5]) {
  if (q[0] < THR(p->f_thr * p->rho_atm)) {
    q[0] = p->rho_atm;
    q[1] = q[2] = q[3] = 0.0;
    q[4] = eos_P_T(e, p->rho_atm, p->T_atm);
  } else if (eos_T(e, q[0], q[4]) < THR(p->T_atm)) {
    q[4] = eos_P_T(e, q[0], p->T_atm);
  }
}

/* ------------------------------------------------------------------------- */
/* Flux at one face (i,j,k) in direction d (face i = left face of cell i):    */
/* reconstruction (order = recon kind, 0 DC), face metric, floors, physics,  */
/* Riemann solver.  Uses stage-input w and B~^(s).                            */
/* ------------------------------------------------------------------------- */
static void face_flux(const eos_t *e, const or_params *p, const or_block *b, int d, int i, int j,
                      int k, int order, double F[7], double *Fs) {
  int off[3] = {0, 0, 0};
  off[d] = 1;
  /* cell index of the cell n steps along d from cell (i,j,k), n in -3..2 */
#define CELL(n) cidx(b, i + (n)*off[0], j + (n)*off[1], k + (n)*off[2])
  /* metric at the face: 4th-order Lagrange (-1, 9, 9, -1)/16 */
  double gf[10];
  for (int n = 0; n < 10; ++n) {
    const double *a = b->adm[n];
    gf[n] = (9.0 * (a[CELL(-1)] + a[CELL(0)]) - (a[CELL(-2)] + a[CELL(1)])) / 16.0;
  }
  met3 m;
  met_set(&m, gf + 4);
  double alpha = gf[0];
  double beta[3] = {gf[1], gf[2], gf[3]};
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  /* stencil values of the 7 reconstructed quantities at cells -3..2 */
  double st[7][6];
  int lo = order == 0 ? -1 : -3, hi = order == 0 ? 0 : 2;
  for (int n = lo; n <= hi; ++n) {
    int ii = i + n * off[0], jj = j + n * off[1], kk = k + n * off[2];
    int64_t c = cidx(b, ii, jj, kk);
    for (int v = 0; v < 5; ++v) st[v][n + 3] = b->w[v][c];
    met3 mc;
    cell_metric(b, c, &mc);
    double Bt[3];
    cell_bt(b, b->bs, ii, jj, kk, Bt);
    st[5][n + 3] = Bt[t1] / mc.sg;
    st[6][n + 3] = Bt[t2] / mc.sg;
  }
#undef CELL
  double qL[7], qR[7];
  for (int v = 0; v < 7; ++v) {
    if (order == 0) {
      qL[v] = st[v][2];
      qR[v] = st[v][3];
    } else {
      /* st[v][0..5] = cells -3..2; left state = upper edge of cell -1,
         right state = lower edge of cell 0 */
      double e_lo, e_hi;
      recon_edges(order, st[v], &e_lo, &e_hi);
      qL[v] = e_hi;
      recon_edges(order, st[v] + 1, &e_lo, &e_hi);
      qR[v] = e_lo;
    }
  }
  face_floor(e, p, qL);
  face_floor(e, p, qR);
  double Bn = b->bs[d][fidx(b, d, i, j, k)] / m.sg;
  double BL[3], BR[3];
  BL[d] = Bn; BR[d] = Bn;
  BL[t1] = qL[5]; BL[t2] = qL[6];
  BR[t1] = qR[5]; BR[t2] = qR[6];
  double UL[7], FL[7], UR[7], FR[7], lmL, lpL, lmR, lpR;
  double FLs[7], FRs[7];
  face_physics(e, &m, alpha, beta, d, qL, BL, UL, FL, &lmL, &lpL, Fs ? FLs : NULL);
  face_physics(e, &m, alpha, beta, d, qR, BR, UR, FR, &lmR, &lpR, Fs ? FRs : NULL);
  riemann_solve(p->riemann, UL, FL, lmL, lpL, UR, FR, lmR, lpR, F);
  if (Fs) riemann_scale(p->riemann, UL, FLs, lmL, lpL, UR, FRs, lmR, lpR, Fs);
}

/* extended face range of direction d: faces [g, g+n_d] along d, cells
   [g-1, g+n_t] across (one ghost column each side, needed by the corner EMFs) */
static void face_range(const or_block *b, int d, int lo[3], int hi[3]) {
  int n[3] = {b->nx, b->ny, b->nz}, g = b->ng;
  for (int a = 0; a < 3; ++a) {
    if (a == d) { lo[a] = g; hi[a] = g + n[a]; }
    else { lo[a] = g - 1; hi[a] = g + n[a]; }
  }
}

/* a2+a3: high-order fluxes on the extended face ranges.  F[d][c] are face
   arrays of direction d (same indexing as the face fields). */
int or_fluxes(or_block *blks, int nblk, const or_params *p, double **Fall) {
  eos_t e;
  eos_setup(p, &e);
  for (int ib = 0; ib < nblk; ++ib) {
    const or_block *b = &blks[ib];
    for (int d = 0; d < 3; ++d) {
      double **F = Fall + (int64_t)ib * 21 + d * 7;
      int lo[3], hi[3];
      face_range(b, d, lo, hi);
#pragma omp parallel for schedule(static)
      for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
          for (int i = lo[0]; i <= hi[0]; ++i) {
            double f[7], fs[7];
            face_flux(&e, p, b, d, i, j, k, p->recon, f, g_tscale_f ? fs : NULL);
            int64_t x = fidx(b, d, i, j, k);
            for (int c = 0; c < 7; ++c) F[c][x] = f[c];
            if (g_tscale_f)
              for (int c = 0; c < 7; ++c) g_tscale_f[(int64_t)ib * 21 + d * 7 + c][x] = fs[c];
          }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Ghost fill of padded cell arrays, face arrays and flags.                   */
/*  For each ghost entry, every coordinate outside the interior on a side     */
/*  with no neighbour (nbr == -1 along that axis) is clamped to the nearest   */
/*  interior value (outflow); the remaining offset selects the neighbour      */
/*  block, whose interior supplies the value (same-level copy / periodic).    */
/* ------------------------------------------------------------------------- */
enum { GF_W = 1, GF_US = 2, GF_BS = 4, GF_FLAGS = 8 };

/* map coordinate x of extent n (interior [g, g+n)) : returns offset -1/0/1 */
static int side_of(int x, int g, int n) { return x < g ? -1 : (x >= g + n ? 1 : 0); }

/* source location of ghost cell (or face) (i,j,k) in block b; face_dir = -1
   for cells, else the face direction (faces g and g+n along it are interior) */
static int ghost_source(const or_block *blks, int ib, int face_dir, int i, int j, int k, int *src_b,
                        int *si, int *sj, int *sk) {
  const or_block *b = &blks[ib];
  int g = b->ng;
  int n[3] = {b->nx, b->ny, b->nz};
  int x[3] = {i, j, k};
  int o[3];
  for (int a = 0; a < 3; ++a) {
    if (a == face_dir) {
      /* faces along their own direction: interior is [g, g+n] */
      o[a] = x[a] < g ? -1 : (x[a] > g + n[a] ? 1 : 0);
    } else {
      o[a] = side_of(x[a], g, n[a]);
    }
  }
  if (o[0] == 0 && o[1] == 0 && o[2] == 0) return 0; /* interior: not a ghost */
  /* axes without a neighbour -> clamp (outflow) */
  for (int a = 0; a < 3; ++a) {
    if (o[a] == 0) continue;
    int oo[3] = {0, 0, 0};
    oo[a] = o[a];
    int nb = b->nbr[(oo[0] + 1) + 3 * (oo[1] + 1) + 9 * (oo[2] + 1)];
    if (nb < 0) {
      if (a == face_dir) x[a] = o[a] < 0 ? g : g + n[a];
      else x[a] = o[a] < 0 ? g : g + n[a] - 1;
      o[a] = 0;
    }
  }
  int nb = ib;
  if (o[0] || o[1] || o[2]) {
    nb = b->nbr[(o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
    if (nb < 0) {
      /* diagonal neighbour missing although each axis has one: clamp all */
      for (int a = 0; a < 3; ++a) {
        if (o[a] == 0) continue;
        if (a == face_dir) x[a] = o[a] < 0 ? g : g + n[a];
        else x[a] = o[a] < 0 ? g : g + n[a] - 1;
      }
      nb = ib;
    } else if (nb == ib) {
      /* periodic self-neighbour: wrap modulo the extent (a block thinner
         than the ghost depth wraps more than once) */
      for (int a = 0; a < 3; ++a) {
        if (o[a] == 0) continue;
        int r = (x[a] - g) % n[a];
        if (r < 0) r += n[a];
        x[a] = g + r;
      }
    } else {
      for (int a = 0; a < 3; ++a) x[a] -= o[a] * n[a];
    }
  }
  *src_b = nb;
  *si = x[0]; *sj = x[1]; *sk = x[2];
  return 1;
}

int or_ghost_fill(or_block *blks, int nblk, int mask) {
  for (int ib = 0; ib < nblk; ++ib) {
    or_block *b = &blks[ib];
    if (b->bc == 0) continue;
    int sx = b->nx + 2 * b->ng, sy = b->ny + 2 * b->ng, sz = b->nz + 2 * b->ng;
    if (mask & (GF_W | GF_US | GF_FLAGS)) {
      for (int k = 0; k < sz; ++k)
        for (int j = 0; j < sy; ++j)
          for (int i = 0; i < sx; ++i) {
            int sb, si, sj, sk;
            if (!ghost_source(blks, ib, -1, i, j, k, &sb, &si, &sj, &sk)) continue;
            const or_block *s = &blks[sb];
            int64_t dst = cidx(b, i, j, k), src = cidx(s, si, sj, sk);
            if (mask & GF_W)
              for (int v = 0; v < 5; ++v) b->w[v][dst] = s->w[v][src];
            if (mask & GF_US)
              for (int v = 0; v < 5; ++v) b->us[v][dst] = s->us[v][src];
            if (mask & GF_FLAGS) b->flags[dst] = s->flags[src];
          }
    }
    if (mask & GF_BS) {
      for (int d = 0; d < 3; ++d) {
        int ex = sx + (d == 0), ey = sy + (d == 1), ez = sz + (d == 2);
        for (int k = 0; k < ez; ++k)
          for (int j = 0; j < ey; ++j)
            for (int i = 0; i < ex; ++i) {
              int sb, si, sj, sk;
              if (!ghost_source(blks, ib, d, i, j, k, &sb, &si, &sj, &sk)) continue;
              const or_block *s = &blks[sb];
              b->bs[d][fidx(b, d, i, j, k)] = s->bs[d][fidx(s, d, si, sj, sk)];
            }
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Inter-level transfer on a refined mesh (the block-based mesh refinement   */
/* of Sec. I; the prolongation and restriction that Sec. V-A counts among    */
/* the costs).  Refinement by a factor 2; every block is a leaf; leaves that */
/* touch (across a face, an edge or a corner) differ by at most one level.   */
/* A ghost cell or face takes its value from the leaf covering its position: */
/*  - a leaf of the same level: a copy;                                       */
/*  - a finer leaf: restriction -- the mean of the 8 child cells (flags: OR), */
/*    of the 4 child faces in the face's plane;                               */
/*  - a coarser leaf: prolongation -- a cell: the parent's value plus, per    */
/*    axis, a quarter of the parent's minmod-limited slope, signed towards   */
/*    the child (the 8 children average to the parent); flags: the parent's; */
/*    a face on a parent face: that face's value; a face inside a parent     */
/*    cell: the mean of the parent's two faces along its normal (each child  */
/*    cell then has its parent's divergence).                                 */
/* Copies and restrictions read interiors only and go first; prolongations   */
/* go level by level upwards, since the parent's slope may read the parent   */
/* leaf's ghosts.  In a stage, every face flux a block holds on its boundary */
/* next to a finer leaf becomes the mean of the 4 fine fluxes there          */
/* (conservation across the level boundary), and every boundary edge EMF     */
/* next to a finer leaf the mean of the 2 fine EMFs along it (the coarse     */
/* face then changes by the mean of the fine faces' changes: div B~ stays at */
/* round-off).  One dt for every level.  Outflow boundaries take the         */
/* nearest cell of the domain, periodic ones wrap.                           */
/* ------------------------------------------------------------------------- */
/* test instrument: switch the flux / EMF correction off (1, 1 = the method) */
static int g_amr_flux_fix = 1, g_amr_emf_fix = 1;
void or_set_amr_corrections(int flux, int emf) {
  g_amr_flux_fix = flux;
  g_amr_emf_fix = emf;
}

typedef struct {
  int32_t n0[3];        /* the domain in level-0 cells                          */
  int32_t periodic[3];  /* per axis: 1 periodic, 0 outflow                      */
  const int32_t *level; /* per block: its refinement level (dx = dx0 / 2^level) */
  const int32_t *org;   /* per block, 3 each: global index at its level of its first interior cell */
} or_amr;

static int amr_cell_axis(const or_amr *amr, int lvl, int a, int I) {
  const int N = amr->n0[a] << lvl;
  if (I >= 0 && I < N) return I;
  if (amr->periodic[a]) return ((I % N) + N) % N;
  return I < 0 ? 0 : N - 1;
}

/* Lookup of the leaf that covers a cell.  The definition is a search over
   all leaves (find_leaf_search); where every leaf has one size nb, a table
   per level of the leaves on that level's lattice of nb-blocks answers the
   same question in a few probes (a cell is covered by at most one leaf).
   The table is built by each public entry point of the refined mesh and
   released on return. */
static struct {
  int on, nb, maxlvl;
  int32_t nbk[32][3];
  int32_t *tab[32];
} g_leafidx;
static int g_leafidx_use = 1;   /* test instrument: 0 searches every time */
void or_set_leaf_index(int on) { g_leafidx_use = on; }

static int leaf_contains(const or_block *blks, const or_amr *amr, int ib, int lvl, const int I[3]) {
  const int L = amr->level[ib];
  const int n[3] = {blks[ib].nx, blks[ib].ny, blks[ib].nz};
  for (int a = 0; a < 3; ++a) {
    const int64_t lo = (int64_t)amr->org[3 * ib + a], hi = lo + n[a];
    /* the cell's extent in leaf-level indices: [c0, c1) */
    int64_t c0, c1;
    if (L >= lvl) {
      c0 = (int64_t)I[a] << (L - lvl);
      c1 = c0 + ((int64_t)1 << (L - lvl));
    } else {
      c0 = (int64_t)I[a] >> (lvl - L);
      c1 = c0 + 1;
    }
    if (!(c0 >= lo && c1 <= hi)) return 0;
  }
  return 1;
}

static int find_leaf_search(const or_block *blks, int nblk, const or_amr *amr, int lvl, const int I[3]) {
  for (int ib = 0; ib < nblk; ++ib)
    if (leaf_contains(blks, amr, ib, lvl, I)) return ib;
  return -1;
}

static void leaf_index_build(const or_block *blks, int nblk, const or_amr *amr) {
  g_leafidx.on = 0;
  if (!g_leafidx_use) return;
  const int nb = blks[0].nx;
  int maxlvl = 0;
  for (int ib = 0; ib < nblk; ++ib) {
    if (blks[ib].nx != nb || blks[ib].ny != nb || blks[ib].nz != nb) return;
    if (amr->level[ib] > maxlvl) maxlvl = amr->level[ib];
    for (int a = 0; a < 3; ++a)
      if (amr->org[3 * ib + a] % nb) return;
  }
  if (maxlvl >= 32) return;
  for (int a = 0; a < 3; ++a)
    if (amr->n0[a] % nb) return;
  g_leafidx.nb = nb;
  g_leafidx.maxlvl = maxlvl;
  for (int L = 0; L <= maxlvl; ++L) {
    int64_t cnt = 1;
    for (int a = 0; a < 3; ++a) {
      g_leafidx.nbk[L][a] = (amr->n0[a] << L) / nb;
      cnt *= g_leafidx.nbk[L][a];
    }
    g_leafidx.tab[L] = (int32_t *)malloc((size_t)cnt * sizeof(int32_t));
    for (int64_t x = 0; x < cnt; ++x) g_leafidx.tab[L][x] = -1;
  }
  for (int ib = 0; ib < nblk; ++ib) {
    const int L = amr->level[ib];
    const int32_t *nk = g_leafidx.nbk[L];
    const int bx = amr->org[3 * ib] / nb, by = amr->org[3 * ib + 1] / nb, bz = amr->org[3 * ib + 2] / nb;
    g_leafidx.tab[L][((int64_t)bz * nk[1] + by) * nk[0] + bx] = ib;
  }
  g_leafidx.on = 1;
}

static void leaf_index_free(void) {
  if (!g_leafidx.on) return;
  for (int L = 0; L <= g_leafidx.maxlvl; ++L) free(g_leafidx.tab[L]);
  g_leafidx.on = 0;
}

/* the leaf that covers global cell I (inside the domain) of level lvl */
static int find_leaf(const or_block *blks, int nblk, const or_amr *amr, int lvl, const int I[3]) {
  if (!g_leafidx.on) return find_leaf_search(blks, nblk, amr, lvl, I);
  const int nb = g_leafidx.nb;
  for (int L = 0; L <= g_leafidx.maxlvl; ++L) {
    int c[3];
    for (int a = 0; a < 3; ++a) {
      const int64_t J = L >= lvl ? ((int64_t)I[a] << (L - lvl)) : ((int64_t)I[a] >> (lvl - L));
      c[a] = (int)(J / nb);
    }
    const int32_t *nk = g_leafidx.nbk[L];
    if (c[0] >= nk[0] || c[1] >= nk[1] || c[2] >= nk[2]) continue;
    const int ib = g_leafidx.tab[L][((int64_t)c[2] * nk[1] + c[1]) * nk[0] + c[0]];
    if (ib >= 0 && leaf_contains(blks, amr, ib, lvl, I)) return ib;
  }
  return -1;
}

static double minmod2(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

/* padded index in leaf L (at level lvl(L)) of global cell J of that level */
static int64_t leaf_cell(const or_block *L, const int32_t *org, const int J[3]) {
  return cidx(L, J[0] - org[0] + L->ng, J[1] - org[1] + L->ng, J[2] - org[2] + L->ng);
}

/* prolongation of padded cell array f of leaf L to the child Ic (a global
   index one level finer than L) */
static double prolong_cell(const or_block *L, const int32_t *org, const double *f, const int Ic[3]) {
  const int P[3] = {Ic[0] >> 1, Ic[1] >> 1, Ic[2] >> 1};
  const int64_t c = leaf_cell(L, org, P);
  const double v = f[c];
  double out = v;
  for (int a = 0; a < 3; ++a) {
    int lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    lo[a] -= 1;
    hi[a] += 1;
    const double s = minmod2(f[leaf_cell(L, org, hi)] - v, v - f[leaf_cell(L, org, lo)]);
    out += (Ic[a] & 1) ? 0.25 * s : -0.25 * s;
  }
  return out;
}

/* ghost cells of block ib: pass 0 copies and restrictions, pass > 0 the
   prolongations of a block at level == pass */
static void amr_fill_cells(or_block *blks, int nblk, const or_amr *amr, int ib, int mask, int pass) {
  or_block *b = &blks[ib];
  const int lv = amr->level[ib], g = b->ng;
  const int n[3] = {b->nx, b->ny, b->nz};
  const int s[3] = {n[0] + 2 * g, n[1] + 2 * g, n[2] + 2 * g};
  for (int k = 0; k < s[2]; ++k)
    for (int j = 0; j < s[1]; ++j)
      for (int i = 0; i < s[0]; ++i) {
        const int x[3] = {i, j, k};
        int inner = 1;
        for (int a = 0; a < 3; ++a) inner = inner && x[a] >= g && x[a] < g + n[a];
        if (inner) continue;
        int I[3];
        for (int a = 0; a < 3; ++a) I[a] = amr_cell_axis(amr, lv, a, amr->org[3 * ib + a] + x[a] - g);
        const int il = find_leaf(blks, nblk, amr, lv, I);
        if (il < 0) continue;
        const or_block *L = &blks[il];
        const int32_t *lorg = amr->org + 3 * il;
        const int ll = amr->level[il];
        const int64_t dst = cidx(b, i, j, k);
        if (pass == 0 && ll == lv) {
          const int64_t src = leaf_cell(L, lorg, I);
          if (mask & GF_W)
            for (int v = 0; v < 5; ++v) b->w[v][dst] = L->w[v][src];
          if (mask & GF_US)
            for (int v = 0; v < 5; ++v) b->us[v][dst] = L->us[v][src];
          if (mask & GF_FLAGS) b->flags[dst] = L->flags[src];
        } else if (pass == 0 && ll == lv + 1) {
          double sw[5] = {0, 0, 0, 0, 0}, su[5] = {0, 0, 0, 0, 0};
          uint16_t fl = 0;
          for (int c = 0; c < 8; ++c) {
            const int C[3] = {2 * I[0] + (c & 1), 2 * I[1] + ((c >> 1) & 1), 2 * I[2] + (c >> 2)};
            const int64_t src = leaf_cell(L, lorg, C);
            for (int v = 0; v < 5; ++v) {
              if (mask & GF_W) sw[v] += L->w[v][src];
              if (mask & GF_US) su[v] += L->us[v][src];
            }
            fl |= L->flags[src];
          }
          if (mask & GF_W)
            for (int v = 0; v < 5; ++v) b->w[v][dst] = 0.125 * sw[v];
          if (mask & GF_US)
            for (int v = 0; v < 5; ++v) b->us[v][dst] = 0.125 * su[v];
          if (mask & GF_FLAGS) b->flags[dst] = fl;
        } else if (pass == lv && ll == lv - 1) {
          if (mask & GF_W)
            for (int v = 0; v < 5; ++v) b->w[v][dst] = prolong_cell(L, lorg, L->w[v], I);
          if (mask & GF_US)
            for (int v = 0; v < 5; ++v) b->us[v][dst] = prolong_cell(L, lorg, L->us[v], I);
          if (mask & GF_FLAGS) {
            const int P[3] = {I[0] >> 1, I[1] >> 1, I[2] >> 1};
            b->flags[dst] = L->flags[leaf_cell(L, lorg, P)];
          }
        }
      }
}

/* value of the face of direction d whose lower corner, in global indices of
   leaf L's level, is J (J[d] the face index), read from L's face array */
static double leaf_face(const or_block *L, const int32_t *org, int d, const int J[3]) {
  return L->bs[d][fidx(L, d, J[0] - org[0] + L->ng, J[1] - org[1] + L->ng, J[2] - org[2] + L->ng)];
}

/* ghost faces of direction d of block ib (passes as for the cells) */
static void amr_fill_faces(or_block *blks, int nblk, const or_amr *amr, int ib, int d, int pass) {
  or_block *b = &blks[ib];
  const int lv = amr->level[ib], g = b->ng;
  const int n[3] = {b->nx, b->ny, b->nz};
  const int e[3] = {n[0] + 2 * g + (d == 0), n[1] + 2 * g + (d == 1), n[2] + 2 * g + (d == 2)};
  const int N = amr->n0[d] << lv;
  for (int k = 0; k < e[2]; ++k)
    for (int j = 0; j < e[1]; ++j)
      for (int i = 0; i < e[0]; ++i) {
        const int x[3] = {i, j, k};
        int inner = 1;
        for (int a = 0; a < 3; ++a) inner = inner && x[a] >= g && x[a] <= g + n[a] - (a != d);
        if (inner) continue;
        /* the face in global indices of level lv: along d a face index
           (periodic: mod N; outflow: clamped to the boundary faces 0 and N),
           across d the cell indices */
        int F[3];
        for (int a = 0; a < 3; ++a) {
          const int G = amr->org[3 * ib + a] + x[a] - g;
          if (a != d) {
            F[a] = amr_cell_axis(amr, lv, a, G);
          } else if (amr->periodic[a]) {
            F[a] = ((G % N) + N) % N;
          } else {
            F[a] = G < 0 ? 0 : (G > N ? N : G);
          }
        }
        /* the cells above (F) and below (F - e_d) the face, where inside the domain */
        int Ip[3] = {F[0], F[1], F[2]}, Im[3] = {F[0], F[1], F[2]};
        Im[d] = F[d] - 1;
        if (amr->periodic[d] && Im[d] < 0) Im[d] += N;
        const int lp = Ip[d] < N ? find_leaf(blks, nblk, amr, lv, Ip) : -1;
        const int lm = Im[d] >= 0 ? find_leaf(blks, nblk, amr, lv, Im) : -1;
        /* the two sides: leaf, its level, and the face's index along d in that
           side's numbering (the upper face of M's cell is Im + 1, N across a
           periodic boundary); the side within the block's own range along d
           first (the upper side except on the block's upper boundary plane) */
        const int first_m = x[d] == g + n[d];
        const int sl[2] = {first_m ? lm : lp, first_m ? lp : lm};
        const int sf[2] = {first_m ? Im[d] + 1 : F[d], first_m ? F[d] : Im[d] + 1};
        int sv[2];
        for (int q = 0; q < 2; ++q) sv[q] = sl[q] >= 0 ? amr->level[sl[q]] : -100;
        int pick = -1, kind = -1;   /* kind 0 copy, 1 restriction, 2 prolongation */
        for (int want = 0; want < 3 && pick < 0; ++want) {
          const int lw = want == 0 ? lv : want == 1 ? lv + 1 : lv - 1;
          for (int q = 0; q < 2 && pick < 0; ++q)
            if (sv[q] == lw) {
              pick = q;
              kind = want;
            }
        }
        if (pick < 0) continue;
        if ((kind < 2 && pass != 0) || (kind == 2 && pass != lv)) continue;
        const int il = sl[pick];
        const int32_t *lorg = amr->org + 3 * il;
        const int Fd = sf[pick];
        const int64_t dst = fidx(b, d, i, j, k);
        if (kind == 0) {
          int J[3] = {F[0], F[1], F[2]};
          J[d] = Fd;
          b->bs[d][dst] = leaf_face(&blks[il], lorg, d, J);
        } else if (kind == 1) {
          double sum = 0.0;
          for (int c = 0; c < 4; ++c) {
            int J[3];
            int t = 0;
            for (int a = 0; a < 3; ++a) {
              if (a == d) {
                J[a] = 2 * Fd;
              } else {
                J[a] = 2 * F[a] + ((c >> t) & 1);
                ++t;
              }
            }
            sum += leaf_face(&blks[il], lorg, d, J);
          }
          b->bs[d][dst] = 0.25 * sum;
        } else {
          /* on a parent face (even index) its value; inside a parent cell
             (odd index) the mean of that cell's two faces along d */
          int J[3] = {F[0] >> 1, F[1] >> 1, F[2] >> 1};
          J[d] = Fd >> 1;
          if ((Fd & 1) == 0) {
            b->bs[d][dst] = leaf_face(&blks[il], lorg, d, J);
          } else {
            int J1[3] = {J[0], J[1], J[2]};
            J1[d] += 1;
            b->bs[d][dst] = 0.5 * (leaf_face(&blks[il], lorg, d, J) + leaf_face(&blks[il], lorg, d, J1));
          }
        }
      }
}

static int ghost_fill_amr_body(or_block *blks, int nblk, int mask, const or_amr *amr);
int or_ghost_fill_amr(or_block *blks, int nblk, int mask, const or_amr *amr) {
  const int own = !g_leafidx.on;
  if (own) leaf_index_build(blks, nblk, amr);
  const int r = ghost_fill_amr_body(blks, nblk, mask, amr);
  if (own) leaf_index_free();
  return r;
}

static int ghost_fill_amr_body(or_block *blks, int nblk, int mask, const or_amr *amr) {
  int maxlvl = 0;
  for (int ib = 0; ib < nblk; ++ib)
    if (amr->level[ib] > maxlvl) maxlvl = amr->level[ib];
  /* within a pass each block writes its own ghosts and reads only what an
     earlier pass (or no pass) wrote: the blocks of a pass are independent */
  for (int pass = 0; pass <= maxlvl; ++pass)
#pragma omp parallel for schedule(dynamic)
    for (int ib = 0; ib < nblk; ++ib) {
      if (blks[ib].bc == 0) continue;
      if (pass > 0 && amr->level[ib] != pass) continue;
      if (mask & (GF_W | GF_US | GF_FLAGS)) amr_fill_cells(blks, nblk, amr, ib, mask, pass);
      if (mask & GF_BS)
        for (int d = 0; d < 3; ++d) amr_fill_faces(blks, nblk, amr, ib, d, pass);
    }
  return 0;
}

/* flux correction: each boundary face of a block next to a finer leaf takes
   the mean of that leaf's 4 fluxes there (all 7 components) */
static void amr_flux_correct(or_block *blks, int nblk, const or_amr *amr, double **Fall) {
  /* each block writes its own boundary values; the finer leaves' values it
     reads are never written here (a leaf next to a finer one is not next to
     a coarser one across the same face or edge) */
#pragma omp parallel for schedule(dynamic)
  for (int ib = 0; ib < nblk; ++ib) {
    or_block *b = &blks[ib];
    const int lv = amr->level[ib], g = b->ng;
    const int n[3] = {b->nx, b->ny, b->nz};
    double **Fb = Fall + (int64_t)ib * 21;
    for (int d = 0; d < 3; ++d)
      for (int side = 0; side < 2; ++side) {
        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        const int N = amr->n0[d] << lv;
        /* the cell across the face, at level lv */
        const int Gd = amr->org[3 * ib + d] + (side ? n[d] : -1);
        if (!amr->periodic[d] && (Gd < 0 || Gd >= N)) continue;   /* domain boundary */
        for (int q2 = 0; q2 < n[t2]; ++q2)
          for (int q1 = 0; q1 < n[t1]; ++q1) {
            int I[3];
            I[d] = ((Gd % N) + N) % N;
            I[t1] = amr->org[3 * ib + t1] + q1;
            I[t2] = amr->org[3 * ib + t2] + q2;
            const int il = find_leaf(blks, nblk, amr, lv, I);
            if (il < 0 || amr->level[il] != lv + 1) continue;
            const or_block *L = &blks[il];
            double **FL = Fall + (int64_t)il * 21;
            double sum[7] = {0, 0, 0, 0, 0, 0, 0};
            for (int c = 0; c < 4; ++c) {
              int J[3];
              /* across the lower face: the upper faces of children 2I+1; across
                 the upper face: the lower faces of children 2I */
              J[d] = side ? 2 * I[d] : 2 * I[d] + 2;
              J[t1] = 2 * I[t1] + (c & 1);
              J[t2] = 2 * I[t2] + (c >> 1);
              const int64_t f = fidx(L, d, J[0] - amr->org[3 * il] + L->ng, J[1] - amr->org[3 * il + 1] + L->ng,
                                     J[2] - amr->org[3 * il + 2] + L->ng);
              for (int v = 0; v < 7; ++v) sum[v] += FL[d * 7 + v][f];
            }
            int x[3];
            x[d] = side ? g + n[d] : g;
            x[t1] = g + q1;
            x[t2] = g + q2;
            const int64_t f0 = fidx(b, d, x[0], x[1], x[2]);
            for (int v = 0; v < 7; ++v) Fb[d * 7 + v][f0] = 0.25 * sum[v];
          }
      }
  }
}

/* EMF correction: each boundary edge EMF of a block where one of the 4 cells
   around the edge lies in a finer leaf takes the mean of that leaf's 2 EMFs
   along the edge.  Eall[3 * ib + c]: block ib's edge array of component c. */
static void amr_emf_correct(or_block *blks, int nblk, const or_amr *amr, double **Eall) {
  /* each block writes its own boundary values; the finer leaves' values it
     reads are never written here (a leaf next to a finer one is not next to
     a coarser one across the same face or edge) */
#pragma omp parallel for schedule(dynamic)
  for (int ib = 0; ib < nblk; ++ib) {
    or_block *b = &blks[ib];
    const int lv = amr->level[ib], g = b->ng;
    const int n[3] = {b->nx, b->ny, b->nz};
    for (int comp = 0; comp < 3; ++comp) {
      const int A = (comp + 1) % 3, Bx = (comp + 2) % 3;
      for (int k = g; k <= g + n[2] - (comp == 2); ++k)
        for (int j = g; j <= g + n[1] - (comp == 1); ++j)
          for (int i = g; i <= g + n[0] - (comp == 0); ++i) {
            const int x[3] = {i, j, k};
            if (x[A] != g && x[A] != g + n[A] && x[Bx] != g && x[Bx] != g + n[Bx]) continue;
            for (int cell = 0; cell < 4; ++cell) {
              const int oa = cell & 1, ob = cell >> 1;   /* the cell (a - oa, b - ob) */
              int I[3], outside = 0;
              for (int a = 0; a < 3; ++a) {
                int G = amr->org[3 * ib + a] + x[a] - g;
                if (a == A) G -= oa;
                if (a == Bx) G -= ob;
                const int N = amr->n0[a] << lv;
                if (!amr->periodic[a] && (G < 0 || G >= N)) outside = 1;
                I[a] = ((G % N) + N) % N;
              }
              if (outside) continue;
              const int il = find_leaf(blks, nblk, amr, lv, I);
              if (il < 0 || amr->level[il] != lv + 1) continue;
              const or_block *L = &blks[il];
              const double *EL = Eall[3 * il + comp];
              double sum = 0.0;
              for (int h = 0; h < 2; ++h) {
                int J[3];
                J[comp] = 2 * I[comp] + h;
                J[A] = 2 * (I[A] + oa);
                J[Bx] = 2 * (I[Bx] + ob);
                sum += EL[eidx(L, J[0] - amr->org[3 * il] + L->ng, J[1] - amr->org[3 * il + 1] + L->ng,
                               J[2] - amr->org[3 * il + 2] + L->ng)];
              }
              Eall[3 * ib + comp][eidx(b, i, j, k)] = 0.5 * sum;
              break;
            }
          }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* a4: FOFC (+DMP).  Trial state without sources or CT, trial C2P with the   */
/* stage-input cell-centred field; flag cells whose trial needs a floor or    */
/* fails, or (DMP) whose D~ or tau~ leaves [lo(min), hi(max)] of Eq. 12 over   */
/* the 27-cell neighbourhood of U^(s).  Then redo every face of a flagged     */
/* cell with donor cell + the Riemann solver.                                 */
/* ------------------------------------------------------------------------- */
static void dmp_bounds(double mn, double mx, double M, double *lo, double *hi) {
  *lo = mn >= 0.0 ? mn / M : mn * M;
  *hi = mx >= 0.0 ? mx * M : mx / M;
}

int or_fofc_flags(or_block *blks, int nblk, const or_params *p, double dt, double a0, double a1,
                  double bb, double **Fall) {
  eos_t e;
  eos_setup(p, &e);
  for (int ib = 0; ib < nblk; ++ib) {
    or_block *b = &blks[ib];
    int64_t nc = ncell(b);
    for (int64_t c = 0; c < nc; ++c) b->flags[c] = 0;
    int g = b->ng;
    double **F = Fall + (int64_t)ib * 21;
#pragma omp parallel for schedule(static)
    for (int k = g; k < g + b->nz; ++k)
      for (int j = g; j < g + b->ny; ++j)
        for (int i = g; i < g + b->nx; ++i) {
          int64_t c = cidx(b, i, j, k);
          double U[5];
          for (int v = 0; v < 5; ++v) {
            double div = (F[0 * 7 + v][fidx(b, 0, i + 1, j, k)] - F[0 * 7 + v][fidx(b, 0, i, j, k)]) / b->dx[0] +
                         (F[1 * 7 + v][fidx(b, 1, i, j + 1, k)] - F[1 * 7 + v][fidx(b, 1, i, j, k)]) / b->dx[1] +
                         (F[2 * 7 + v][fidx(b, 2, i, j, k + 1)] - F[2 * 7 + v][fidx(b, 2, i, j, k)]) / b->dx[2];
            U[v] = a0 * b->un[v][c] + a1 * b->us[v][c] - bb * dt * div;
          }
          uint16_t fl = 0;
          if (p->dmp_M > 0.0) {
            const int vv[2] = {0, 4};
            for (int t = 0; t < 2; ++t) {
              int v = vv[t];
              double mn = b->us[v][c], mx = mn;
              for (int dk = -1; dk <= 1; ++dk)
                for (int dj = -1; dj <= 1; ++dj)
                  for (int di = -1; di <= 1; ++di) {
                    double x = b->us[v][cidx(b, i + di, j + dj, k + dk)];
                    if (x < mn) mn = x;
                    if (x > mx) mx = x;
                  }
              double lo, hi;
              dmp_bounds(mn, mx, p->dmp_M, &lo, &hi);
              lo -= g_margin * fabs(lo);
              hi += g_margin * fabs(hi);
              if (!(U[v] >= lo && U[v] <= hi)) fl |= F_DMP;
            }
          }
          met3 m;
          cell_metric(b, c, &m);
          double Bt[3];
          cell_bt(b, b->bs, i, j, k, Bt);
          double w[5];
          int nev;
          double mu;
          int r = c2p_point(&e, p, &m, U, Bt, w, 0, 0.0, 0.0, &nev, &mu);
          if (r & F_FLOORS) fl |= F_FOFC;
          b->flags[c] = fl;
        }
  }
  return 0;
}

int or_fofc_fix(or_block *blks, int nblk, const or_params *p, double **Fall) {
  eos_t e;
  eos_setup(p, &e);
  for (int ib = 0; ib < nblk; ++ib) {
    const or_block *b = &blks[ib];
    for (int d = 0; d < 3; ++d) {
      double **F = Fall + (int64_t)ib * 21 + d * 7;
      int lo[3], hi[3];
      face_range(b, d, lo, hi);
      int off[3] = {0, 0, 0};
      off[d] = 1;
#pragma omp parallel for schedule(static)
      for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
          for (int i = lo[0]; i <= hi[0]; ++i) {
            uint16_t fl = b->flags[cidx(b, i, j, k)] |
                          b->flags[cidx(b, i - off[0], j - off[1], k - off[2])];
            if (!(fl & (F_FOFC | F_DMP))) continue;
            double f[7], fs[7];
            face_flux(&e, p, b, d, i, j, k, 0, f, g_tscale_f ? fs : NULL);
            int64_t x = fidx(b, d, i, j, k);
            for (int c = 0; c < 7; ++c) F[c][x] = f[c];
            if (g_tscale_f)
              for (int c = 0; c < 7; ++c) g_tscale_f[(int64_t)ib * 21 + d * 7 + c][x] = fs[c];
          }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* a5: upwind constrained transport.                                           */
/* Face EMFs from the fluxes of the transverse field:                          */
/*   on d-faces   E_{t2} = -F(B~^{t1}),  E_{t1} = +F(B~^{t2})                  */
/* Cell-centre reference EMF E = -alpha (vhat x B~) from stage-input prims.    */
/* Corner EMF of E_c on the (a,b) plane, (a,b,c) cyclic: average of the four  */
/* adjacent face EMFs plus upwinded gradient corrections toward the cell-     */
/* centre EMF, the upwind side chosen by the sign of the face mass flux       */
/* (average of both sides when it is zero).                                   */
/* Face update: B~ = a0 B~^n + a1 B~^(s) - b dt curl(E) (discrete Stokes).     */
/* ------------------------------------------------------------------------- */
static double face_emf(const or_block *b, double **Fb, int face_d, int comp, int i, int j, int k) {
  /* EMF component comp on a face of direction face_d */
  int t1 = (face_d + 1) % 3, t2 = (face_d + 2) % 3;
  int64_t x = fidx(b, face_d, i, j, k);
  double **F = Fb + face_d * 7;
  if (comp == t2) return -F[5][x];
  if (comp == t1) return F[6][x];
  return 0.0;
}

static double upwind_pick(double mflux, double up_neg_side, double up_pos_side) {
  /* mflux > 0: flow toward +; the upwind cell is on the negative side */
  if (mflux > 0.0) return up_neg_side;
  if (mflux < 0.0) return up_pos_side;
  return 0.5 * (up_neg_side + up_pos_side);
}

/* Corner EMF of component c at the edge shared by the cells (a-1, b-1),
   (a, b-1), (a-1, b), (a, b) of the (a, b) plane ((a, b, c) cyclic).
   Face EMFs: EA_b, EA_bm on the a-faces at (a-1/2, b) and (a-1/2, b-1);
   EB_a, EB_am on the b-faces at (a, b-1/2) and (a-1, b-1/2); mA_*, mB_*
   the mass fluxes through those faces.  Cell-centre EMFs E00 (a, b),
   E10 (a-1, b), E01 (a, b-1), E11 (a-1, b-1). */
static double corner_emf(double EA_b, double EA_bm, double EB_a, double EB_am, double mA_b,
                         double mA_bm, double mB_a, double mB_am, double E00, double E10,
                         double E01, double E11) {
  /* half-cell gradients of E along b at the a-faces, from the upwind cell */
  double db_hi = upwind_pick(mA_b, E10 - EB_am, E00 - EB_a);     /* between b-1/2 and b */
  double db_lo = upwind_pick(mA_bm, EB_am - E11, EB_a - E01);    /* between b-1 and b-1/2 */
  /* half-cell gradients of E along a at the b-faces */
  double da_hi = upwind_pick(mB_a, E01 - EA_bm, E00 - EA_b);     /* between a-1/2 and a */
  double da_lo = upwind_pick(mB_am, EA_bm - E11, EA_b - E10);    /* between a-1 and a-1/2 */
  return 0.25 * (EA_b + EA_bm + EB_a + EB_am) + 0.25 * (db_lo - db_hi + da_lo - da_hi);
}

/* the magnitudes of the terms of corner_emf (term-scale instrument): the
   same upwind picks over |E_cc| + |E_face| in place of their differences */
static double corner_emf_scale(double EA_b, double EA_bm, double EB_a, double EB_am, double mA_b,
                               double mA_bm, double mB_a, double mB_am, double E00, double E10,
                               double E01, double E11) {
  double db_hi = upwind_pick(mA_b, fabs(E10) + fabs(EB_am), fabs(E00) + fabs(EB_a));
  double db_lo = upwind_pick(mA_bm, fabs(EB_am) + fabs(E11), fabs(EB_a) + fabs(E01));
  double da_hi = upwind_pick(mB_a, fabs(E01) + fabs(EA_bm), fabs(E00) + fabs(EA_b));
  double da_lo = upwind_pick(mB_am, fabs(EA_bm) + fabs(E11), fabs(EA_b) + fabs(E10));
  return 0.25 * (fabs(EA_b) + fabs(EA_bm) + fabs(EB_a) + fabs(EB_am)) +
         0.25 * (db_lo + db_hi + da_lo + da_hi);
}

/* corner EMFs of block ib into Ec[3] (edge arrays; with the term-scale
   instrument also their term magnitudes into Ecs[3]) */
static void ct_emfs(or_block *blks, int ib, double **Fall, double *Ec[3], double *Ecs[3]) {
  or_block *b = &blks[ib];
  double **Fb = Fall + (int64_t)ib * 21;
  int g = b->ng;
  int n[3] = {b->nx, b->ny, b->nz};
  int64_t nc = ncell(b);
  double *Ecc[3], *Eccs[3] = {NULL, NULL, NULL};
  for (int a = 0; a < 3; ++a) {
    Ecc[a] = (double *)calloc((size_t)nc, sizeof(double));
    if (g_tscale_b) Eccs[a] = (double *)calloc((size_t)nc, sizeof(double));
  }
  /* cell-centre EMF on cells [g-1, g+n] */
  for (int k = g - 1; k <= g + n[2]; ++k)
    for (int j = g - 1; j <= g + n[1]; ++j)
      for (int i = g - 1; i <= g + n[0]; ++i) {
        int64_t c = cidx(b, i, j, k);
        met3 m;
        cell_metric(b, c, &m);
        double al = b->adm[0][c];
        double u[3] = {b->w[1][c], b->w[2][c], b->w[3][c]};
        double ul[3];
        lower3(&m, u, ul);
        double W = sqrt(1.0 + dot3(u, ul));
        double vh[3];
        for (int a = 0; a < 3; ++a) vh[a] = u[a] / W - b->adm[1 + a][c] / al;
        double Bt[3];
        cell_bt(b, b->bs, i, j, k, Bt);
        Ecc[0][c] = -al * (vh[1] * Bt[2] - vh[2] * Bt[1]);
        Ecc[1][c] = -al * (vh[2] * Bt[0] - vh[0] * Bt[2]);
        Ecc[2][c] = -al * (vh[0] * Bt[1] - vh[1] * Bt[0]);
        if (g_tscale_b) {
          Eccs[0][c] = fabs(al) * (fabs(vh[1] * Bt[2]) + fabs(vh[2] * Bt[1]));
          Eccs[1][c] = fabs(al) * (fabs(vh[2] * Bt[0]) + fabs(vh[0] * Bt[2]));
          Eccs[2][c] = fabs(al) * (fabs(vh[0] * Bt[1]) + fabs(vh[1] * Bt[0]));
        }
      }
  /* corner EMFs.  For component c with plane axes (a, bx) cyclic, the edge
     (ia-1/2, ib-1/2) is stored at edge index with face indices on a and bx */
  for (int comp = 0; comp < 3; ++comp) {
    int A = (comp + 1) % 3, Bx = (comp + 2) % 3;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (a == comp) { lo[a] = g; hi[a] = g + n[a] - 1; }
      else { lo[a] = g; hi[a] = g + n[a]; }
    }
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          int x[3] = {i, j, k};
          /* helpers: position shifted by -1 along A and/or Bx */
#define AT(da, db, out) do { int y_[3] = {x[0], x[1], x[2]}; y_[A] += (da); y_[Bx] += (db); \
                           out[0] = y_[0]; out[1] = y_[1]; out[2] = y_[2]; } while (0)
          int p00[3], p10[3], p01[3], p11[3];
          AT(0, 0, p00);    /* cell (a, b)       */
          AT(-1, 0, p10);   /* cell (a-1, b)     */
          AT(0, -1, p01);   /* cell (a, b-1)     */
          AT(-1, -1, p11);  /* cell (a-1, b-1)   */
#undef AT
          /* a-faces at (a-1/2, b) and (a-1/2, b-1): face index = p00 / p01 along A */
          double EA_b = face_emf(b, Fb, A, comp, p00[0], p00[1], p00[2]);
          double EA_bm = face_emf(b, Fb, A, comp, p01[0], p01[1], p01[2]);
          /* b-faces at (a, b-1/2) and (a-1, b-1/2): face index = p00 / p10 along Bx */
          double EB_a = face_emf(b, Fb, Bx, comp, p00[0], p00[1], p00[2]);
          double EB_am = face_emf(b, Fb, Bx, comp, p10[0], p10[1], p10[2]);
          double mA_b = Fb[A * 7 + 0][fidx(b, A, p00[0], p00[1], p00[2])];
          double mA_bm = Fb[A * 7 + 0][fidx(b, A, p01[0], p01[1], p01[2])];
          double mB_a = Fb[Bx * 7 + 0][fidx(b, Bx, p00[0], p00[1], p00[2])];
          double mB_am = Fb[Bx * 7 + 0][fidx(b, Bx, p10[0], p10[1], p10[2])];
          double *E = Ecc[comp];
          double Ec00 = E[cidx(b, p00[0], p00[1], p00[2])];
          double Ec10 = E[cidx(b, p10[0], p10[1], p10[2])];
          double Ec01 = E[cidx(b, p01[0], p01[1], p01[2])];
          double Ec11 = E[cidx(b, p11[0], p11[1], p11[2])];
          Ec[comp][eidx(b, i, j, k)] = corner_emf(EA_b, EA_bm, EB_a, EB_am, mA_b, mA_bm, mB_a,
                                                  mB_am, Ec00, Ec10, Ec01, Ec11);
          if (g_tscale_b && g_tscale_f) {
            double *Es = Eccs[comp];
            double **Sb = g_tscale_f + (int64_t)ib * 21;
            Ecs[comp][eidx(b, i, j, k)] = corner_emf_scale(
                face_emf(b, Sb, A, comp, p00[0], p00[1], p00[2]),
                face_emf(b, Sb, A, comp, p01[0], p01[1], p01[2]),
                face_emf(b, Sb, Bx, comp, p00[0], p00[1], p00[2]),
                face_emf(b, Sb, Bx, comp, p10[0], p10[1], p10[2]), mA_b, mA_bm, mB_a, mB_am,
                Es[cidx(b, p00[0], p00[1], p00[2])], Es[cidx(b, p10[0], p10[1], p10[2])],
                Es[cidx(b, p01[0], p01[1], p01[2])], Es[cidx(b, p11[0], p11[1], p11[2])]);
          }
        }
  }
  for (int a = 0; a < 3; ++a) {
    free(Ecc[a]);
    free(Eccs[a]);
  }
}

/* face update of block ib's interior faces from its corner EMFs */
static void ct_faces(or_block *blks, int ib, double dt, double a0, double a1, double bb,
                     double *Ec[3], double *Ecs[3]) {
  or_block *b = &blks[ib];
  int g = b->ng;
  int n[3] = {b->nx, b->ny, b->nz};
  /* face update on interior faces */
  for (int d = 0; d < 3; ++d) {
    int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = g;
      hi[a] = a == d ? g + n[a] : g + n[a] - 1;
    }
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          int x1[3] = {i, j, k}, x2[3] = {i, j, k};
          x1[d1] += 1;
          x2[d2] += 1;
          /* (curl E)^d = d_{d1} E_{d2} - d_{d2} E_{d1} */
          double c1 = (Ec[d2][eidx(b, x1[0], x1[1], x1[2])] - Ec[d2][eidx(b, i, j, k)]) / b->dx[d1];
          double c2 = (Ec[d1][eidx(b, x2[0], x2[1], x2[2])] - Ec[d1][eidx(b, i, j, k)]) / b->dx[d2];
          int64_t f = fidx(b, d, i, j, k);
          b->bo[d][f] = a0 * b->bn[d][f] + a1 * b->bs[d][f] - bb * dt * (c1 - c2);
          if (g_tscale_b && g_tscale_f) {
            double s1 = (Ecs[d2][eidx(b, x1[0], x1[1], x1[2])] + Ecs[d2][eidx(b, i, j, k)]) / b->dx[d1];
            double s2 = (Ecs[d1][eidx(b, x2[0], x2[1], x2[2])] + Ecs[d1][eidx(b, i, j, k)]) / b->dx[d2];
            g_tscale_b[ib * 3 + d][f] = fabs(a0 * b->bn[d][f]) + fabs(a1 * b->bs[d][f]) +
                                        fabs(bb) * dt * (s1 + s2);
          }
        }
  }
}

static void alloc_emfs(const or_block *b, double *Ec[3], double *Ecs[3]) {
  int64_t ne = nedge(b);
  for (int a = 0; a < 3; ++a) {
    Ec[a] = (double *)calloc((size_t)ne, sizeof(double));
    Ecs[a] = g_tscale_b ? (double *)calloc((size_t)ne, sizeof(double)) : NULL;
  }
}
static void free_emfs(double *Ec[3], double *Ecs[3]) {
  for (int a = 0; a < 3; ++a) {
    free(Ec[a]);
    free(Ecs[a]);
  }
}

int or_ct(or_block *blks, int nblk, const or_params *p, double dt, double a0, double a1, double bb,
          double **Fall) {
  (void)p;
  for (int ib = 0; ib < nblk; ++ib) {
    double *Ec[3], *Ecs[3];
    alloc_emfs(&blks[ib], Ec, Ecs);
    ct_emfs(blks, ib, Fall, Ec, Ecs);
    ct_faces(blks, ib, dt, a0, a1, bb, Ec, Ecs);
    free_emfs(Ec, Ecs);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* a6: update with the flux divergence and the Eq. 10 sources evaluated from  */
/* the stage input (w^(s), U^(s), B~^(s)) and the ADM fields.  Metric          */
/* derivatives: 4th-order centred differences.                                */
/* ------------------------------------------------------------------------- */
static double dcen(const double *a, const or_block *b, int d, int i, int j, int k) {
  int o[3] = {0, 0, 0};
  o[d] = 1;
  double qm2 = a[cidx(b, i - 2 * o[0], j - 2 * o[1], k - 2 * o[2])];
  double qm1 = a[cidx(b, i - o[0], j - o[1], k - o[2])];
  double qp1 = a[cidx(b, i + o[0], j + o[1], k + o[2])];
  double qp2 = a[cidx(b, i + 2 * o[0], j + 2 * o[1], k + 2 * o[2])];
  return ((qm2 - qp2) - 8.0 * (qm1 - qp1)) / (12.0 * b->dx[d]);
}

/* Eq. 10 at one cell; w prims, Bt densitized, U densitized conserved of the
   same cell, dal[3], dbe[3][3] (d_i beta^j as [i][j]), dg[3][6] (d_i gamma_jk),
   K6 extrinsic curvature.  Output G[5] (0 for D~). */
static void sources_point(const eos_t *e, const met3 *m, double alpha, const double w[5],
                          const double Bt[3], const double U[5], const double dal[3],
                          double dbe[3][3], double dg[3][6], const double K6[6], double G[5],
                          double *Gs) {
  double rho = w[0], P = w[4];
  double u[3] = {w[1], w[2], w[3]};
  double ul[3];
  lower3(m, u, ul);
  double W = sqrt(1.0 + dot3(u, ul));
  double v[3] = {u[0] / W, u[1] / W, u[2] / W};
  double vl[3] = {ul[0] / W, ul[1] / W, ul[2] / W};
  double B[3] = {Bt[0] / m->sg, Bt[1] / m->sg, Bt[2] / m->sg};
  double Bl[3];
  lower3(m, B, Bl);
  double B2 = dot3(B, Bl), Bv = dot3(B, vl);
  double eps = eos_eps_P(e, rho, P);
  double h = 1.0 + eps + P / rho;
  double bsq = B2 / (W * W) + Bv * Bv;
  double Ptot = P + 0.5 * bsq;
  double bs[3];                           /* spatial projection of b^mu */
  for (int i = 0; i < 3; ++i) bs[i] = B[i] / W + W * Bv * v[i];
  double Sij[3][3];                        /* densitized S~^{ij} */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Sij[i][j] = m->sg * ((rho * h + bsq) * W * W * v[i] * v[j] + Ptot * m->gu[i][j] - bs[i] * bs[j]);
  double Sl[3] = {U[1], U[2], U[3]};
  double Su[3];
  raise3(m, Sl, Su);
  double Et = U[4] + U[0];
  static const int sidx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  G[0] = 0.0;
  for (int i = 0; i < 3; ++i) {
    double t1 = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) t1 += Sij[j][k] * dg[i][sidx[j][k]];
    double t2 = 0.0;
    for (int j = 0; j < 3; ++j) t2 += Sl[j] * dbe[i][j];
    G[1 + i] = 0.5 * alpha * t1 + t2 - Et * dal[i];
  }
  double kS = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) kS += K6[sidx[i][j]] * Sij[i][j];
  G[4] = alpha * kS - dot3(Su, dal);
  if (Gs) {
    /* the same sums over the magnitudes of their terms (instrument) */
    Gs[0] = 0.0;
    for (int i = 0; i < 3; ++i) {
      double a1 = 0.0, a2 = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) a1 += fabs(Sij[j][k] * dg[i][sidx[j][k]]);
      for (int j = 0; j < 3; ++j) a2 += fabs(Sl[j] * dbe[i][j]);
      Gs[1 + i] = 0.5 * fabs(alpha) * a1 + a2 + fabs(Et * dal[i]);
    }
    double ak = 0.0, ad = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) ak += fabs(K6[sidx[i][j]] * Sij[i][j]);
    for (int i = 0; i < 3; ++i) ad += fabs(Su[i] * dal[i]);
    Gs[4] = fabs(alpha) * ak + ad;
  }
}

int or_update(or_block *blks, int nblk, const or_params *p, double dt, double a0, double a1,
              double bb, double **Fall) {
  eos_t e;
  eos_setup(p, &e);
  for (int ib = 0; ib < nblk; ++ib) {
    or_block *b = &blks[ib];
    double **F = Fall + (int64_t)ib * 21;
    int g = b->ng;
#pragma omp parallel for schedule(static)
    for (int k = g; k < g + b->nz; ++k)
      for (int j = g; j < g + b->ny; ++j)
        for (int i = g; i < g + b->nx; ++i) {
          int64_t c = cidx(b, i, j, k);
          met3 m;
          cell_metric(b, c, &m);
          double dal[3], dbe[3][3], dg[3][6];
          for (int d = 0; d < 3; ++d) {
            dal[d] = dcen(b->adm[0], b, d, i, j, k);
            for (int q = 0; q < 3; ++q) dbe[d][q] = dcen(b->adm[1 + q], b, d, i, j, k);
            for (int q = 0; q < 6; ++q) dg[d][q] = dcen(b->adm[4 + q], b, d, i, j, k);
          }
          double K6[6];
          for (int q = 0; q < 6; ++q) K6[q] = b->adm[10 + q][c];
          double w[5], Us[5], Bt[3], G[5];
          for (int v = 0; v < 5; ++v) { w[v] = b->w[v][c]; Us[v] = b->us[v][c]; }
          cell_bt(b, b->bs, i, j, k, Bt);
          double Gs[5];
          sources_point(&e, &m, b->adm[0][c], w, Bt, Us, dal, dbe, dg, K6, G,
                        g_tscale_u ? Gs : NULL);
          for (int v = 0; v < 5; ++v) {
            double div = (F[0 * 7 + v][fidx(b, 0, i + 1, j, k)] - F[0 * 7 + v][fidx(b, 0, i, j, k)]) / b->dx[0] +
                         (F[1 * 7 + v][fidx(b, 1, i, j + 1, k)] - F[1 * 7 + v][fidx(b, 1, i, j, k)]) / b->dx[1] +
                         (F[2 * 7 + v][fidx(b, 2, i, j, k + 1)] - F[2 * 7 + v][fidx(b, 2, i, j, k)]) / b->dx[2];
            b->uo[v][c] = a0 * b->un[v][c] + a1 * Us[v] + bb * dt * (-div + G[v]);
            if (g_tscale_u && g_tscale_f) {
              double **S = g_tscale_f + (int64_t)ib * 21;
              double fs = (S[0 * 7 + v][fidx(b, 0, i + 1, j, k)] + S[0 * 7 + v][fidx(b, 0, i, j, k)]) / b->dx[0] +
                          (S[1 * 7 + v][fidx(b, 1, i, j + 1, k)] + S[1 * 7 + v][fidx(b, 1, i, j, k)]) / b->dx[1] +
                          (S[2 * 7 + v][fidx(b, 2, i, j, k + 1)] + S[2 * 7 + v][fidx(b, 2, i, j, k)]) / b->dx[2];
              g_tscale_u[ib * 5 + v][c] = fabs(a0 * b->un[v][c]) + fabs(a1 * Us[v]) +
                                          fabs(bb) * dt * (fs + Gs[v]);
            }
          }
        }
  }
  return 0;
}

/* a8 over the interior of each block: U^out -> w^out with the updated field */
int or_stage_c2p(or_block *blks, int nblk, const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  for (int ib = 0; ib < nblk; ++ib) {
    or_block *b = &blks[ib];
    int g = b->ng;
#pragma omp parallel for schedule(static)
    for (int k = g; k < g + b->nz; ++k)
      for (int j = g; j < g + b->ny; ++j)
        for (int i = g; i < g + b->nx; ++i) {
          int64_t c = cidx(b, i, j, k);
          met3 m;
          cell_metric(b, c, &m);
          double U[5], Bt[3], w[5];
          for (int v = 0; v < 5; ++v) U[v] = b->uo[v][c];
          cell_bt(b, b->bo, i, j, k, Bt);
          int nev;
          double mu;
          int r = c2p_point(&e, p, &m, U, Bt, w, 0, 0.0, 0.0, &nev, &mu);
          for (int v = 0; v < 5; ++v) { b->uo[v][c] = U[v]; b->wo[v][c] = w[v]; }
          b->flags[c] = (uint16_t)(b->flags[c] | r);
        }
  }
  return 0;
}

/* Lapse excision (Sec. IV, the collapse runs): interior cells of the stage
   output with alpha < alpha_min get the atmosphere primitives (rho_atm, v = 0,
   T_atm) and the conserved state of those primitives with the unchanged
   field; flagged F_EXCISED. */
int or_excise(or_block *blks, int nblk, const or_params *p, double alpha_min) {
  eos_t e;
  eos_setup(p, &e);
  for (int ib = 0; ib < nblk; ++ib) {
    or_block *b = &blks[ib];
    int g = b->ng;
    for (int k = g; k < g + b->nz; ++k)
      for (int j = g; j < g + b->ny; ++j)
        for (int i = g; i < g + b->nx; ++i) {
          int64_t c = cidx(b, i, j, k);
          if (!(b->adm[0][c] < alpha_min)) continue;
          met3 m;
          cell_metric(b, c, &m);
          double w[5], Bt[3], U[5];
          atmosphere_prims(&e, p, w);
          cell_bt(b, b->bo, i, j, k, Bt);
          p2c_point(&e, &m, w, Bt, U);
          for (int v = 0; v < 5; ++v) { b->uo[v][c] = U[v]; b->wo[v][c] = w[v]; }
          b->flags[c] = (uint16_t)(b->flags[c] | F_EXCISED);
        }
  }
  return 0;
}

/* flux workspace of a block list: 21 face arrays per block */
static double **alloc_fluxes(const or_block *blks, int nblk) {
  double **F = (double **)calloc((size_t)nblk * 21, sizeof(double *));
  for (int ib = 0; ib < nblk; ++ib)
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 7; ++c)
        F[ib * 21 + d * 7 + c] = (double *)calloc((size_t)nface(&blks[ib], d), sizeof(double));
  return F;
}
static void free_fluxes(double **F, int nblk) {
  for (int x = 0; x < nblk * 21; ++x) free(F[x]);
  free(F);
}

/* One stage with RK coefficients (a0, a1, b):
   U^out = a0 U^n + a1 U^(s) + b dt L(U^(s)).  Order of the steps: fluxes,
   FOFC flags, flag exchange between blocks, FOFC refluxing, CT, update with
   sources, C2P with floors. */
int or_stage(or_block *blks, int nblk, const or_params *p, double dt, double a0, double a1,
             double bb) {
  double **F = alloc_fluxes(blks, nblk);
  if (g_tscale_u || g_tscale_b) g_tscale_f = alloc_fluxes(blks, nblk);
  or_fluxes(blks, nblk, p, F);
  if (p->fofc) {
    or_fofc_flags(blks, nblk, p, dt, a0, a1, bb, F);
    or_ghost_fill(blks, nblk, GF_FLAGS);
    or_fofc_fix(blks, nblk, p, F);
  } else {
    for (int ib = 0; ib < nblk; ++ib) {
      int64_t nc = ncell(&blks[ib]);
      for (int64_t c = 0; c < nc; ++c) blks[ib].flags[c] = 0;
    }
  }
  or_ct(blks, nblk, p, dt, a0, a1, bb, F);
  or_update(blks, nblk, p, dt, a0, a1, bb, F);
  or_stage_c2p(blks, nblk, p);
  free_fluxes(F, nblk);
  if (g_tscale_f) {
    free_fluxes(g_tscale_f, nblk);
    g_tscale_f = NULL;
  }
  return 0;
}

/* One stage on a refined mesh (leaves of several levels, amr): the steps of
   or_stage, with the flag exchange across levels, and the flux correction
   (after the FOFC refluxing) and EMF correction (between the corner EMFs and
   the face update) at level boundaries. */
int or_stage_amr(or_block *blks, int nblk, const or_params *p, double dt, double a0, double a1,
                 double bb, const or_amr *amr) {
  leaf_index_build(blks, nblk, amr);
  double **F = alloc_fluxes(blks, nblk);
  if (g_tscale_u || g_tscale_b) g_tscale_f = alloc_fluxes(blks, nblk);
  or_fluxes(blks, nblk, p, F);
  if (p->fofc) {
    or_fofc_flags(blks, nblk, p, dt, a0, a1, bb, F);
    or_ghost_fill_amr(blks, nblk, GF_FLAGS, amr);
    or_fofc_fix(blks, nblk, p, F);
  } else {
    for (int ib = 0; ib < nblk; ++ib) {
      int64_t nc = ncell(&blks[ib]);
      for (int64_t c = 0; c < nc; ++c) blks[ib].flags[c] = 0;
    }
  }
  if (g_amr_flux_fix) {
    amr_flux_correct(blks, nblk, amr, F);
    if (g_tscale_f) amr_flux_correct(blks, nblk, amr, g_tscale_f);
  }
  double **E = (double **)calloc((size_t)nblk * 3, sizeof(double *));
  double **Es = (double **)calloc((size_t)nblk * 3, sizeof(double *));
  for (int ib = 0; ib < nblk; ++ib) {
    alloc_emfs(&blks[ib], E + 3 * ib, Es + 3 * ib);
    ct_emfs(blks, ib, F, E + 3 * ib, Es + 3 * ib);
  }
  if (g_amr_emf_fix) {
    amr_emf_correct(blks, nblk, amr, E);
    if (g_tscale_b) amr_emf_correct(blks, nblk, amr, Es);
  }
  for (int ib = 0; ib < nblk; ++ib) {
    ct_faces(blks, ib, dt, a0, a1, bb, E + 3 * ib, Es + 3 * ib);
    free_emfs(E + 3 * ib, Es + 3 * ib);
  }
  free(E);
  free(Es);
  or_update(blks, nblk, p, dt, a0, a1, bb, F);
  or_stage_c2p(blks, nblk, p);
  free_fluxes(F, nblk);
  if (g_tscale_f) {
    free_fluxes(g_tscale_f, nblk);
    g_tscale_f = NULL;
  }
  leaf_index_free();
  return 0;
}

/* granular entry: the same stage with a caller-provided flux workspace, so a
   test can inspect the fluxes after each step (mode bit 1 fluxes, 2 FOFC,
   4 CT, 8 update, 16 C2P) */
int or_stage_steps(or_block *blks, int nblk, const or_params *p, double dt, double a0, double a1,
                   double bb, double **F, int mode) {
  if (mode & 1) or_fluxes(blks, nblk, p, F);
  if (mode & 2) {
    or_fofc_flags(blks, nblk, p, dt, a0, a1, bb, F);
    or_ghost_fill(blks, nblk, GF_FLAGS);
    or_fofc_fix(blks, nblk, p, F);
  }
  if (mode & 4) or_ct(blks, nblk, p, dt, a0, a1, bb, F);
  if (mode & 8) or_update(blks, nblk, p, dt, a0, a1, bb, F);
  if (mode & 16) or_stage_c2p(blks, nblk, p);
  return 0;
}

/* a9: dt = cfl / max over interior cells and directions of |lambda|/dx */
double or_dt(or_block *blks, int nblk, const or_params *p, double cfl) {
  eos_t e;
  eos_setup(p, &e);
  double mx = 0.0;
  for (int ib = 0; ib < nblk; ++ib) {
    const or_block *b = &blks[ib];
    int g = b->ng;
    for (int k = g; k < g + b->nz; ++k)
      for (int j = g; j < g + b->ny; ++j)
        for (int i = g; i < g + b->nx; ++i) {
          int64_t c = cidx(b, i, j, k);
          met3 m;
          cell_metric(b, c, &m);
          double beta[3] = {b->adm[1][c], b->adm[2][c], b->adm[3][c]};
          double q[5], Bt[3], B[3];
          for (int v = 0; v < 5; ++v) q[v] = b->w[v][c];
          cell_bt(b, b->bs, i, j, k, Bt);
          for (int a = 0; a < 3; ++a) B[a] = Bt[a] / m.sg;
          for (int d = 0; d < 3; ++d) {
            double U[7], F[7], lm, lp;
            face_physics(&e, &m, b->adm[0][c], beta, d, q, B, U, F, &lm, &lp, NULL);
            double s = fabs(lm) > fabs(lp) ? fabs(lm) : fabs(lp);
            s /= b->dx[d];
            if (s > mx) mx = s;
          }
        }
  }
  return cfl / mx;
}

/* baryon mass sum D~ dV over the interior of the given conserved array */
double or_mass(or_block *blks, int nblk, int which) {
  double tot = 0.0;
  for (int ib = 0; ib < nblk; ++ib) {
    const or_block *b = &blks[ib];
    const double *D = which == 0 ? b->us[0] : which == 1 ? b->uo[0] : b->un[0];
    int g = b->ng;
    double dv = b->dx[0] * b->dx[1] * b->dx[2];
    for (int k = g; k < g + b->nz; ++k)
      for (int j = g; j < g + b->ny; ++j)
        for (int i = g; i < g + b->nx; ++i) tot += D[cidx(b, i, j, k)] * dv;
  }
  return tot;
}

/* ------------------------------------------------------------------------- */
/* Pointwise entry points (arrays of n points, SoA)                           */
/* ------------------------------------------------------------------------- */
int or_prim2con(int64_t n, double *const w[5], double *const bt[3], double *const gam[6],
                double *u[5], const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  for (int64_t x = 0; x < n; ++x) {
    double s[6], ww[5], B[3], U[5];
    for (int q = 0; q < 6; ++q) s[q] = gam[q][x];
    for (int q = 0; q < 5; ++q) ww[q] = w[q][x];
    for (int q = 0; q < 3; ++q) B[q] = bt[q][x];
    met3 m;
    met_set(&m, s);
    p2c_point(&e, &m, ww, B, U);
    for (int q = 0; q < 5; ++q) u[q][x] = U[q];
  }
  return 0;
}

/* ADM matter sources of n points (see matter_point); out[10] arrays */
int or_matter_sources(int64_t n, double *const w[5], double *const bt[3], double *const gam[6],
                      double *out[10], const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  for (int64_t x = 0; x < n; ++x) {
    double s[6], ww[5], B[3], o[10];
    for (int q = 0; q < 6; ++q) s[q] = gam[q][x];
    for (int q = 0; q < 5; ++q) ww[q] = w[q][x];
    for (int q = 0; q < 3; ++q) B[q] = bt[q][x];
    met3 m;
    met_set(&m, s);
    matter_point(&e, &m, ww, B, o);
    for (int q = 0; q < 10; ++q) out[q][x] = o[q];
  }
  return 0;
}

/* C2P of n points.  u in/out (rewritten when a rule fires); optional bracket
   arrays (NULL = plain full bracket); optional per-point evaluation counts and
   roots. */
int or_c2p(int64_t n, double *u[5], double *const bt[3], double *const gam[6], double *w[5],
           uint16_t *flags, const or_params *p, const double *blo, const double *bhi,
           int32_t *nev, double *mu) {
  eos_t e;
  eos_setup(p, &e);
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < n; ++x) {
    double s[6], U[5], B[3], ww[5];
    for (int q = 0; q < 6; ++q) s[q] = gam[q][x];
    for (int q = 0; q < 5; ++q) U[q] = u[q][x];
    for (int q = 0; q < 3; ++q) B[q] = bt[q][x];
    met3 m;
    met_set(&m, s);
    int ne;
    double mm;
    int r = c2p_point(&e, p, &m, U, B, ww, blo != NULL, blo ? blo[x] : 0.0, bhi ? bhi[x] : 0.0,
                      &ne, &mm);
    for (int q = 0; q < 5; ++q) { u[q][x] = U[q]; w[q][x] = ww[q]; }
    flags[x] = (uint16_t)r;
    if (nev) nev[x] = ne;
    if (mu) mu[x] = mm;
  }
  return 0;
}

/* master function f(mu) of n points at the given mu (for pins) */
int or_master(int64_t n, double *const u[5], double *const bt[3], double *const gam[6],
              const double *mu, double *f, double *fa, const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  for (int64_t x = 0; x < n; ++x) {
    double s[6];
    for (int q = 0; q < 6; ++q) s[q] = gam[q][x];
    met3 m;
    met_set(&m, s);
    double D = u[0][x] / m.sg, Sl[3] = {u[1][x] / m.sg, u[2][x] / m.sg, u[3][x] / m.sg};
    double tau = u[4][x] / m.sg;
    double B[3] = {bt[0][x] / m.sg, bt[1][x] / m.sg, bt[2][x] / m.sg}, Bl[3];
    lower3(&m, B, Bl);
    kctx k;
    k.e = &e;
    k.D = D;
    k.q = tau / D;
    double rl[3] = {Sl[0] / D, Sl[1] / D, Sl[2] / D}, ru[3];
    raise3(&m, rl, ru);
    k.r2 = dot3(rl, ru);
    double sD = sqrt(D);
    double bu[3] = {B[0] / sD, B[1] / sD, B[2] / sD};
    k.b2 = dot3(B, Bl) / D;
    k.s = dot3(rl, bu);
    k.h0 = eos_h0(&e);
    double z0 = sqrt(k.r2) / k.h0;
    k.v0sq = z0 * z0 / (1.0 + z0 * z0);
    f[x] = kastaun_f(mu[x], &k);
    if (fa) fa[x] = kastaun_fa(mu[x], &k);
  }
  return 0;
}

/* test entry: the primitives the inversion recovers at a given root mu
   (no floors), n points; the recovery of c2p_point at mu */
int or_recover(int64_t n, double *const u[5], double *const bt[3], double *const gam[6],
               const double *mu, double *w[5], double *teps, const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  for (int64_t x = 0; x < n; ++x) {
    double s[6];
    for (int q = 0; q < 6; ++q) s[q] = gam[q][x];
    met3 m;
    met_set(&m, s);
    double D = u[0][x] / m.sg, Sl[3] = {u[1][x] / m.sg, u[2][x] / m.sg, u[3][x] / m.sg};
    double tau = u[4][x] / m.sg;
    double B[3] = {bt[0][x] / m.sg, bt[1][x] / m.sg, bt[2][x] / m.sg}, Bl[3];
    lower3(&m, B, Bl);
    kctx k;
    k.e = &e;
    k.D = D;
    k.q = tau / D;
    double rl[3] = {Sl[0] / D, Sl[1] / D, Sl[2] / D}, ru[3];
    raise3(&m, rl, ru);
    k.r2 = dot3(rl, ru);
    double sD = sqrt(D);
    double bu[3] = {B[0] / sD, B[1] / sD, B[2] / sD};
    k.b2 = dot3(B, Bl) / D;
    k.s = dot3(rl, bu);
    k.h0 = eos_h0(&e);
    double z0 = sqrt(k.r2) / k.h0;
    k.v0sq = z0 * z0 / (1.0 + z0 * z0);
    kstate st;
    kastaun_eval(&k, mu[x], &st);
    double vu[3];
    for (int i = 0; i < 3; ++i) vu[i] = mu[x] * st.chi * (ru[i] + mu[x] * k.s * bu[i]);
    w[0][x] = st.rho;
    w[1][x] = st.W * vu[0];
    w[2][x] = st.W * vu[1];
    w[3][x] = st.W * vu[2];
    w[4][x] = st.P;
    if (teps) {
      /* magnitude of the terms eps is summed from (its rounding scale) */
      double m2c2 = mu[x] * mu[x] * st.chi * st.chi;
      double qbs = fabs(k.q) + 0.5 * k.b2 + 0.5 * m2c2 * (k.b2 * k.r2 + k.s * k.s);
      teps[x] = st.W * (qbs + mu[x] * st.rb2) + st.vsq * st.W * st.W / (1.0 + st.W);
    }
  }
  return 0;
}

/* Eq. 9 + wave speeds at n points for direction d (for pins).  q prims,
   B un-densitized, metric fields al, be[3], gam[6].  U[7], F[7], lm, lp out. */
int or_face_physics(int64_t n, int d, double *const q[5], double *const B[3],
                    const double *al, double *const be[3], double *const gam[6], double *U[7],
                    double *F[7], double *lm, double *lp, const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  for (int64_t x = 0; x < n; ++x) {
    double s[6], qq[5], BB[3], beta[3], UU[7], FF[7];
    for (int c = 0; c < 6; ++c) s[c] = gam[c][x];
    for (int c = 0; c < 5; ++c) qq[c] = q[c][x];
    for (int c = 0; c < 3; ++c) { BB[c] = B[c][x]; beta[c] = be[c][x]; }
    met3 m;
    met_set(&m, s);
    face_physics(&e, &m, al[x], beta, d, qq, BB, UU, FF, &lm[x], &lp[x], NULL);
    for (int c = 0; c < 7; ++c) { U[c][x] = UU[c]; F[c][x] = FF[c]; }
  }
  return 0;
}

/* Eq. 10 at one point with explicit derivative input (for pins).
   dal[3], dbe[9] ([i][j] = d_i beta^j), dg[18] ([i][jk]), K6[6] */
int or_sources_point(const double *w, const double *bt, const double *u, const double *gam6,
                     double alpha, const double *dal, const double *dbe, const double *dg,
                     const double *K6, double *G, const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  met3 m;
  met_set(&m, gam6);
  double dbe3[3][3], dg3[3][6];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) dbe3[i][j] = dbe[3 * i + j];
    for (int j = 0; j < 6; ++j) dg3[i][j] = dg[6 * i + j];
  }
  sources_point(&e, &m, alpha, w, bt, u, dal, dbe3, dg3, K6, G, NULL);
  return 0;
}

/* lower and upper edge values of the middle cell of n five-point stencils
   for reconstruction kind 0..4 (for pins) */
int or_recon_edges(int kind, int64_t n, const double *q5, double *lo, double *hi) {
  if (kind < 0 || kind > 4) return -1;
  for (int64_t x = 0; x < n; ++x) recon_edges(kind, q5 + 5 * x, lo + x, hi + x);
  return 0;
}

/* WENOZ right-interface value for n five-point stencils (for pins) */
int or_wenoz(int64_t n, const double *q5, double *out) {
  for (int64_t x = 0; x < n; ++x) {
    const double *s = q5 + 5 * x;
    out[x] = wenoz_right(s[0], s[1], s[2], s[3], s[4]);
  }
  return 0;
}

/* Riemann solver on n faces (for pins): UL,FL,UR,FR as [7][n]; speeds [n] */
int or_riemann(int64_t n, int riemann, double *const UL[7], double *const FL[7],
               const double *lmL, const double *lpL, double *const UR[7], double *const FR[7],
               const double *lmR, const double *lpR, double *F[7]) {
  for (int64_t x = 0; x < n; ++x) {
    double a[7], b[7], c[7], d[7], o[7];
    for (int q = 0; q < 7; ++q) { a[q] = UL[q][x]; b[q] = FL[q][x]; c[q] = UR[q][x]; d[q] = FR[q][x]; }
    riemann_solve(riemann, a, b, lmL[x], lpL[x], c, d, lmR[x], lpR[x], o);
    for (int q = 0; q < 7; ++q) F[q][x] = o[q];
  }
  return 0;
}

/* EOS evaluations for pins: mode 0 P(rho,eps), 1 eps(rho,P), 2 T(rho,P),
   3 cs2(rho,eps,P), 4 eps_cold(rho), 5 P_cold(rho) */
int or_eos(int64_t n, int mode, const double *rho, const double *x, const double *y, double *out,
           const or_params *p) {
  eos_t e;
  eos_setup(p, &e);
  for (int64_t i = 0; i < n; ++i) {
    switch (mode) {
      case 0: out[i] = eos_press(&e, rho[i], x[i]); break;
      case 1: out[i] = eos_eps_P(&e, rho[i], x[i]); break;
      case 2: out[i] = eos_T(&e, rho[i], x[i]); break;
      case 3: out[i] = eos_cs2(&e, rho[i], x[i], y[i]); break;
      case 4: out[i] = eos_ecold(&e, rho[i]); break;
      default: out[i] = eos_pcold(&e, rho[i]); break;
    }
  }
  return 0;
}

/* size of the structs, for the Python side to check its layout */
/* test entry: corner_emf at n points; in[12][n] in the argument order of
   corner_emf */
int or_corner_emf(int64_t n, double *const in[12], double *out) {
  for (int64_t t = 0; t < n; ++t)
    out[t] = corner_emf(in[0][t], in[1][t], in[2][t], in[3][t], in[4][t], in[5][t], in[6][t],
                        in[7][t], in[8][t], in[9][t], in[10][t], in[11][t]);
  return 0;
}

int or_sizeof_params(void) { return (int)sizeof(or_params); }
int or_sizeof_block(void) { return (int)sizeof(or_block); }
