// grmhd.hip -- kernels and C-ABI entry points of libgrmhd.so (gfx950, FP64).
//
// One workgroup-grid per step of the stage; every grid spans all blocks
// (blockIdx.y = block index) so a stage over many MeshBlocks costs a fixed
// number of launches.  Thread index runs fastest along x so that every
// stencil load of a wavefront is a contiguous row of the SoA arrays.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "grmhd.h"
#include "physics.hpp"
#include "timing.hpp"
#include "blocks.hpp"

using namespace gk;

namespace gk {
// inter-level transfer (amr.hip)
int amr_max_level(const grmhd_amr_link* h, int nblk);
int amr_check(const grmhd_block* h, const grmhd_amr_link* lh, int nblk);
void launch_ghost_cells_amr(const grmhd_block* h, const grmhd_block* d, int nblk,
                            const grmhd_amr_link* lh, const grmhd_amr_link* ld, int mask, int list,
                            int pass, int threads, hipStream_t s);
void launch_ghost_faces_amr(const grmhd_block* h, const grmhd_block* d, int nblk,
                            const grmhd_amr_link* lh, const grmhd_amr_link* ld, int dir, int pass,
                            int threads, hipStream_t s);
void launch_amr_flux_fix(const grmhd_block* d, const grmhd_amr_link* ld, int nblk, int nb,
                         hipStream_t s);
void launch_amr_emf_fix(const grmhd_block* d, const grmhd_amr_link* ld, int nblk, int nb,
                        hipStream_t s);
}  // namespace gk

namespace {

constexpr int kThreads = 256;      // fixed-size kernels (pointwise, reductions)
constexpr int kMaxThreads = 512;   // stage kernels: runtime workgroup size up to this


// ---------------------------------------------------------------------------
// a9 pieces: the CFL speed of one interior cell (the largest |lambda_+-|/dx
// over the three directions, Eq. 7-9 fast speeds of the slot w and the face
// average of bs), the wave maximum, and the workgroup maximum folded into
// *red (non-negative doubles order like their bit patterns: exact, order-
// independent)
// ---------------------------------------------------------------------------
__global__ void k_zero1(double* x) {
  if (threadIdx.x == 0 && blockIdx.x == 0) x[0] = 0.0;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double cfl_speed_of(const Eos& e, const M3& m, double al,
                                               const double beta[3], const double w[5],
                                               const double B[3], const double dx[3]) {
  Side sd;
  double s = 0.0;
  side_state<0>(e, m, al, beta, w, B, sd);
  s = fmax(s, fmax(fabs(sd.lm), fabs(sd.lp)) / dx[0]);
  side_state<1>(e, m, al, beta, w, B, sd);
  s = fmax(s, fmax(fabs(sd.lm), fabs(sd.lp)) / dx[1]);
  side_state<2>(e, m, al, beta, w, B, sd);
  s = fmax(s, fmax(fabs(sd.lm), fabs(sd.lp)) / dx[2]);
  return s;
}

__device__ __forceinline__ double cfl_speed(const Eos& e, const GB& b, const Geo& q, int i, int j,
                                            int k) {
  const int64_t c = cell(q, i, j, k);
  M3 m;
  cell_metric(b, c, m);
  const double beta[3] = {b.adm[1][c], b.adm[2][c], b.adm[3][c]};
  double w[5], Bt[3];
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = b.w[v][c];
  cell_bt(q, b.bs, i, j, k, Bt);
  const double is = 1.0 / m.sg;
  const double B[3] = {Bt[0] * is, Bt[1] * is, Bt[2] * is};
  return cfl_speed_of(e, m, b.adm[0][c], beta, w, B, b.dx);
}

// every thread of the workgroup calls this (it holds a barrier)
__device__ __forceinline__ void workgroup_max_into(double s, double* red) {
  s = wave_max(s);
  __shared__ double part[kMaxThreads / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = part[0];
    for (int x = 1; x < (int)(blockDim.x >> 6); ++x) r = fmax(r, part[x]);
    atomicMax((unsigned long long*)red, (unsigned long long)__double_as_longlong(r));
  }
}

// ---------------------------------------------------------------------------
// a1: cell-centred un-densitized field B^i = B~_cc / sqrt(gamma), all cells
// ---------------------------------------------------------------------------
// and, on cells [g-1, g+n]^3, the cell-centre EMF E = -alpha (vhat x B~) of
// the stage input (the reference value of the upwind corner EMFs of a5)
// With DT (the first stage of a step with device dt), the same pass also
// folds the CFL speed of every interior cell into *red (a9): the stage input
// it reads is the state the step's dt is taken from.  With CLR (a whole
// stage) it also clears the cell flags and the FOFC list of the stage.
template <int ET, bool DT, bool CLR>
__global__ __launch_bounds__(kMaxThreads) void k_bcc(const grmhd_block* __restrict__ blks, Eos e_in,
                                                    double* red) {
  int bi;
  int64_t t;
  // no early return before the workgroup reduction of DT
  const bool live = locate(blks, S_CELLS, bi, t);
  double sp = 0.0;
  if (live) {
    const GB b = gview(blks[bi]);
    const Geo q = geo_of(b);
    if (CLR) {
      b.flags[t] = 0;
      if (t == 0) *fofc_count(b, q) = 0u;
    }
    const int i = (int)(t % q.sx), j = (int)((t / q.sx) % q.sy), k = (int)(t / ((int64_t)q.sx * q.sy));
    // face i+1 exists for every cell of the padded block
    M3 m;
    cell_metric(b, t, m);
    double Bt[3];
    cell_bt(q, b.bs, i, j, k, Bt);
    gptr<double> out = b.scratch + off_bcc(q);
    const int64_t nc = n_cells(q);
    const double is = 1.0 / m.sg;
    out[t] = Bt[0] * is;
    out[nc + t] = Bt[1] * is;
    out[2 * nc + t] = Bt[2] * is;
    const int g1 = q.g - 1;
    if (i >= g1 && j >= g1 && k >= g1 && i <= q.g + q.nx && j <= q.g + q.ny && k <= q.g + q.nz) {
      const double al = b.adm[0][t];
      const double beta[3] = {b.adm[1][t], b.adm[2][t], b.adm[3][t]};
      const double ux = b.w[1][t], uy = b.w[2][t], uz = b.w[3][t];
      double lx, ly, lz;
      lower(m.g, ux, uy, uz, lx, ly, lz);
      const double iW = 1.0 / sqrt(1.0 + ux * lx + uy * ly + uz * lz);
      const double ia = 1.0 / al;
      const double vx = ux * iW - beta[0] * ia;
      const double vy = uy * iW - beta[1] * ia;
      const double vz = uz * iW - beta[2] * ia;
      gptr<double> E = b.scratch + off_ecc(q);
      E[t] = -al * (vy * Bt[2] - vz * Bt[1]);
      E[nc + t] = -al * (vz * Bt[0] - vx * Bt[2]);
      E[2 * nc + t] = -al * (vx * Bt[1] - vy * Bt[0]);
      if (DT && i >= q.g && j >= q.g && k >= q.g && i < q.g + q.nx && j < q.g + q.ny &&
          k < q.g + q.nz) {
        const double w[5] = {b.w[0][t], ux, uy, uz, b.w[4][t]};
        const double B[3] = {Bt[0] * is, Bt[1] * is, Bt[2] * is};
        sp = cfl_speed_of(eos_fixed<ET>(e_in), m, al, beta, w, B, b.dx);
      }
    }
  }
  if (DT) workgroup_max_into(sp, red);
}

// ---------------------------------------------------------------------------
// a2 + a3: flux through one face of direction D
// ---------------------------------------------------------------------------
// a3 at the face of direction D below cell c0 (face index fi) from the
// reconstructed states qL, qR (rho, W v^i, P, B^{t1}, B^{t2}; floored here,
// so the caller's copies may be reused): face metric, Eq. 7-9 on both sides,
// Riemann flux
template <int D>
__device__ __forceinline__ void face_solve(const Eos& e, const grmhd_params& p, const GB& b,
                                           const Geo& q, int64_t c0, int64_t fi, double qL[7],
                                           double qR[7], double F[7]) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const int64_t st = D == 0 ? 1 : D == 1 ? (int64_t)q.sx : (int64_t)q.sx * q.sy;
  // metric at the face: 4th-order Lagrange (-1, 9, 9, -1)/16
  double gf[10];
#pragma unroll
  for (int n = 0; n < 10; ++n) {
    gptr<const double> a = b.adm[n];
    gf[n] = (9.0 * (a[c0 - st] + a[c0]) - (a[c0 - 2 * st] + a[c0 + st])) * (1.0 / 16.0);
  }
  M3 m;
  metric_build(m, gf[4], gf[5], gf[6], gf[7], gf[8], gf[9]);
  floor_face(e, p, qL);
  floor_face(e, p, qR);
  const double Bn = b.bs[D][fi] / m.sg;
  double BL[3], BR[3];
  BL[D] = Bn; BR[D] = Bn;
  BL[T1] = qL[5]; BL[T2] = qL[6];
  BR[T1] = qR[5]; BR[T2] = qR[6];
  const double beta[3] = {gf[1], gf[2], gf[3]};
  Side L, R;
  side_state<D>(e, m, gf[0], beta, qL, BL, L);
  side_state<D>(e, m, gf[0], beta, qR, BR, R);
  riemann(p.riemann, L, R, F);
}

// the seven reconstructed fields of direction D: rho, W v^i, P, and the
// cell-centred B^{t1}, B^{t2} of the field kernel
template <int D>
__device__ __forceinline__ void recon_sources(const GB& b, const Geo& q,
                                              gptr<const double> src[7]) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  gptr<const double> bcc = b.scratch + off_bcc(q);
  const int64_t nc = n_cells(q);
#pragma unroll
  for (int v = 0; v < 5; ++v) src[v] = b.w[v];
  src[5] = bcc + T1 * nc;
  src[6] = bcc + T2 * nc;
}

template <int D, int RC>
__device__ __forceinline__ void face_flux(const Eos& e, const grmhd_params& p,
                                          const GB& b, const Geo& q, int i, int j, int k,
                                          double F[7]) {
  const int64_t st = D == 0 ? 1 : D == 1 ? (int64_t)q.sx : (int64_t)q.sx * q.sy;
  const int64_t c0 = cell(q, i, j, k);
  gptr<const double> src[7];
  recon_sources<D>(b, q, src);
  double qL[7], qR[7];
  // Donor cell is also reached at run time in the high-order variants (where
  // p.recon == RC, so it is never taken): with the reconstruction in a basic
  // block of its own, ahead of the face metric's loads, the compiler keeps
  // every ideal-gas variant at 122-124 VGPRs (4 waves per SIMD); scheduled
  // in one block with the face solve it holds both at once (240 VGPRs).
  if (RC == 0 || p.recon == 0) {
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      qL[v] = src[v][c0 - st];
      qR[v] = src[v][c0];
    }
  } else {
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const gptr<const double> a = src[v];
      recon_face<RC>(a[c0 - 3 * st], a[c0 - 2 * st], a[c0 - st], a[c0], a[c0 + st],
                     a[c0 + 2 * st], qL[v], qR[v]);
    }
  }
  face_solve<D>(e, p, b, q, c0, face<D>(q, i, j, k), qL, qR, F);
}

template <int D, int ET, int RC>
__global__ __launch_bounds__(kMaxThreads) void k_flux(const grmhd_block* __restrict__ blks, Eos e_in,
                                                   grmhd_params p) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int64_t t;
  if (!locate(blks, S_XFACE + D, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  const Box bx = face_box<D>(q);
  int i, j, k;
  if (D == 2) {
    // z faces run x fastest, then z, then y: a face's z stencil (three
    // planes each way) then lies in the waves just before and after it,
    // whose loads are still in L2, instead of planes apart
    i = bx.lo[0] + (int)(t % bx.cnt[0]);
    const int64_t r = t / bx.cnt[0];
    k = bx.lo[2] + (int)(r % bx.cnt[2]);
    j = bx.lo[1] + (int)(r / bx.cnt[2]);
  } else {
    bx.at(t, i, j, k);
  }
  double F[7];
  face_flux<D, RC>(e, p, b, q, i, j, k, F);
  const int64_t f = face<D>(q, i, j, k);
  const int64_t nf = n_faces(q, D);
  gptr<double> out = b.scratch + off_flux(q, D, 0);
#pragma unroll
  for (int c = 0; c < 7; ++c) out[c * nf + f] = F[c];
}

// ---------------------------------------------------------------------------
// a4: FOFC flags (trial state, trial inversion, relaxed DMP of Eq. 12)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxThreads) void k_clear_flags(const grmhd_block* __restrict__ blks) {
  int bi;
  int64_t t;
  if (!locate(blks, S_CELLS, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  if (t < n_cells(q)) b.flags[t] = 0;
  if (t == 0) *fofc_count(b, q) = 0u;
}

__device__ __forceinline__ void dmp_range(double mn, double mx, double M, double& lo, double& hi) {
  lo = mn >= 0.0 ? mn / M : mn * M;
  hi = mx >= 0.0 ? mx * M : mx / M;
}

__device__ __forceinline__ double flux_div(const GB& b, const Geo& q, int v, int i, int j,
                                           int k) {
  gptr<const double> fx = b.scratch + off_flux(q, 0, v);
  gptr<const double> fy = b.scratch + off_flux(q, 1, v);
  gptr<const double> fz = b.scratch + off_flux(q, 2, v);
  return (fx[face<0>(q, i + 1, j, k)] - fx[face<0>(q, i, j, k)]) / b.dx[0] +
         (fy[face<1>(q, i, j + 1, k)] - fy[face<1>(q, i, j, k)]) / b.dx[1] +
         (fz[face<2>(q, i, j, k + 1)] - fz[face<2>(q, i, j, k)]) / b.dx[2];
}

template <int ET>
__global__ __launch_bounds__(kMaxThreads) void k_fofc_flags(const grmhd_block* __restrict__ blks,
                                                         Eos e_in, grmhd_params p,
                                                         const double* dt_d, double dt_h,
                                                         double a0, double a1, double bb) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int64_t t;
  if (!locate(blks, S_INTERIOR, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  const Box bx = interior_box(q);
  int i, j, k;
  bx.at(t, i, j, k);
  const double dt = dt_of(dt_d, dt_h);
  const int64_t c = cell(q, i, j, k);
  double U[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) U[v] = a0 * b.un[v][c] + a1 * b.us[v][c] - bb * dt * flux_div(b, q, v, i, j, k);
  uint32_t fl = 0;
  if (p.dmp_M > 0.0) {
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
      const int v = t2 == 0 ? 0 : 4;
      gptr<const double> a = b.us[v];
      double mn = a[c], mx = a[c];
      for (int dk = -1; dk <= 1; ++dk)
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const double x = a[cell(q, i + di, j + dj, k + dk)];
            mn = fmin(mn, x);
            mx = fmax(mx, x);
          }
      double lo, hi;
      dmp_range(mn, mx, p.dmp_M, lo, hi);
      if (!(U[v] >= lo && U[v] <= hi)) fl |= GRMHD_F_DMP;
    }
  }
  // trial inversion: only whether a rule fires matters (U is not rebuilt)
  double w[5];
  C2PWork cw;
  {
    M3 m;
    cell_metric(b, c, m);
    double Bt[3];
    cell_bt(q, b.bs, i, j, k, Bt);
    cw = c2p_prepare(e, p, m, U, Bt, w);
  }
  uint32_t r = cw.fl;
  if (!cw.done) {
    int nev;
    double mu;
    r = c2p_lean(e, p, cw, w, false, 0.0, 0.0, nev, mu);
  }
  if (r & kFloorBits) fl |= GRMHD_F_FOFC;
  b.flags[c] = (uint16_t)fl;
  fofc_append(b, q, fl != 0u, c);
}

// donor-cell refluxing of the faces of one listed (flagged) cell along D:
// the lower face always, the upper face unless the upper neighbour is listed
// too (it owns that face as its lower one), so each face is written once
template <int D>
__device__ __forceinline__ void fofc_cell_faces(const Eos& e, const grmhd_params& p,
                                                const GB& b, const Geo& q, int x[3]) {
  const int n[3] = {q.nx, q.ny, q.nz};
  const int64_t st = D == 0 ? 1 : D == 1 ? (int64_t)q.sx : (int64_t)q.sx * q.sy;
  const int64_t nf = n_faces(q, D);
  gptr<double> out = b.scratch + off_flux(q, D, 0);
  double F[7];
  if (x[D] >= q.g) {
    face_flux<D, 0>(e, p, b, q, x[0], x[1], x[2], F);
    const int64_t f = face<D>(q, x[0], x[1], x[2]);
#pragma unroll
    for (int cc = 0; cc < 7; ++cc) out[cc * nf + f] = F[cc];
  }
  if (x[D] + 1 <= q.g + n[D]) {
    const int64_t cu = cell(q, x[0], x[1], x[2]) + st;
    if (!(b.flags[cu] & (GRMHD_F_FOFC | GRMHD_F_DMP))) {
      int y[3] = {x[0], x[1], x[2]};
      y[D] += 1;
      face_flux<D, 0>(e, p, b, q, y[0], y[1], y[2], F);
      const int64_t f = face<D>(q, y[0], y[1], y[2]);
#pragma unroll
      for (int cc = 0; cc < 7; ++cc) out[cc * nf + f] = F[cc];
    }
  }
}

// a4 refluxing: workgroup (block bi, chunk r) of a grid of nblk * chunks
// walks entries r * blockDim + tid, stride chunks * blockDim, of block bi's
// list of flagged cells; every face of the extended ranges with a flagged
// cell on either side gets the donor-cell flux
template <int ET>
__global__ __launch_bounds__(kMaxThreads) void k_fofc_fix(const grmhd_block* __restrict__ blks, Eos e_in,
                                                       grmhd_params p, int chunks) {
  const Eos e = eos_fixed<ET>(e_in);
  const int bi = blockIdx.x / chunks, r = blockIdx.x % chunks;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  const int64_t cnt_raw = (int64_t)*fofc_count(b, q);
  const int64_t cnt = cnt_raw < fofc_cap(q) ? cnt_raw : fofc_cap(q);
  gptr<const int> list = fofc_list(b, q);
  for (int64_t ei = (int64_t)r * blockDim.x + threadIdx.x; ei < cnt;
       ei += (int64_t)chunks * blockDim.x) {
    const int64_t c = list[ei];
    int x[3];
    x[0] = (int)(c % q.sx);
    x[1] = (int)((c / q.sx) % q.sy);
    x[2] = (int)(c / ((int64_t)q.sx * q.sy));
    fofc_cell_faces<0>(e, p, b, q, x);
    fofc_cell_faces<1>(e, p, b, q, x);
    fofc_cell_faces<2>(e, p, b, q, x);
  }
}

// ---------------------------------------------------------------------------
// a5: upwind constrained transport
// ---------------------------------------------------------------------------
__device__ __forceinline__ double upwind(double mflux, double from_neg, double from_pos) {
  return mflux > 0.0 ? from_neg : (mflux < 0.0 ? from_pos : 0.5 * (from_neg + from_pos));
}

// EMF component C on a face of direction FD (from the stored transverse-field fluxes)
template <int FD, int C>
__device__ __forceinline__ double face_emf(gptr<const double> sc, const Geo& q, int64_t f) {
  constexpr int T1 = (FD + 1) % 3, T2 = (FD + 2) % 3;
  static_assert(C == T1 || C == T2, "EMF component must be transverse to the face");
  const int64_t nf = n_faces(q, FD);
  const gptr<const double> F = sc + off_flux(q, FD, 0);
  if (C == T2) return -F[5 * nf + f];
  return F[6 * nf + f];
}

// corner EMF of component C on the plane (A, Bx) = ((C+1)%3, (C+2)%3) at the
// edge whose lower corner is cell x (edge along C through the corner of the
// cells x, x - e_A, x - e_Bx, x - e_A - e_Bx)
template <int C>
__device__ __forceinline__ double corner_emf(const GB& b, const Geo& q, const int x[3]) {
  // no contraction to FMA: mirrored neighbourhoods exchange the roles of the
  // terms, and every product and sum rounded as written keeps the corner
  // EMF of a mirrored state the mirrored EMF bit for bit
#pragma clang fp contract(off)
  constexpr int A = (C + 1) % 3, BX = (C + 2) % 3;
  gptr<const double> sc = b.scratch;
  // cells (a,b), (a-1,b), (a,b-1), (a-1,b-1)
  int p10[3] = {x[0], x[1], x[2]};
  int p01[3] = {x[0], x[1], x[2]};
  int p11[3] = {x[0], x[1], x[2]};
  p10[A] -= 1;
  p01[BX] -= 1;
  p11[A] -= 1;
  p11[BX] -= 1;
  const int64_t fa_b = face<A>(q, x[0], x[1], x[2]);
  const int64_t fa_bm = face<A>(q, p01[0], p01[1], p01[2]);
  const int64_t fb_a = face<BX>(q, x[0], x[1], x[2]);
  const int64_t fb_am = face<BX>(q, p10[0], p10[1], p10[2]);
  const double EA_b = face_emf<A, C>(sc, q, fa_b);
  const double EA_bm = face_emf<A, C>(sc, q, fa_bm);
  const double EB_a = face_emf<BX, C>(sc, q, fb_a);
  const double EB_am = face_emf<BX, C>(sc, q, fb_am);
  gptr<const double> mA = sc + off_flux(q, A, 0);
  gptr<const double> mB = sc + off_flux(q, BX, 0);
  const double mA_b = mA[fa_b], mA_bm = mA[fa_bm], mB_a = mB[fb_a], mB_am = mB[fb_am];
  gptr<const double> Ec = sc + off_ecc(q) + C * n_cells(q);
  const double E00 = Ec[cell(q, x[0], x[1], x[2])];
  const double E10 = Ec[cell(q, p10[0], p10[1], p10[2])];
  const double E01 = Ec[cell(q, p01[0], p01[1], p01[2])];
  const double E11 = Ec[cell(q, p11[0], p11[1], p11[2])];
  const double db_hi = upwind(mA_b, E10 - EB_am, E00 - EB_a);
  const double db_lo = upwind(mA_bm, EB_am - E11, EB_a - E01);
  const double da_hi = upwind(mB_a, E01 - EA_bm, E00 - EA_b);
  const double da_lo = upwind(mB_am, EA_bm - E11, EA_b - E10);
  return 0.25 * (EA_b + EA_bm + EB_a + EB_am) + 0.25 * (db_lo - db_hi + da_lo - da_hi);
}

// the corner EMFs of all three components at the corners [g, g+n]^3: the
// corner item x owns the edges of each component C whose lower end is x
// (those with x_C < g + n_C)
__global__ __launch_bounds__(kMaxThreads) void k_emf_corners(const grmhd_block* __restrict__ blks) {
  int bi;
  int64_t t;
  if (!locate(blks, S_CORNER, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  const int ex = q.nx + 1, ey = q.ny + 1;
  int x[3];
  x[2] = (int)(t / ((int64_t)ex * ey));
  const int64_t r = t - (int64_t)x[2] * ex * ey;
  x[1] = (int)(r / ex);
  x[0] = (int)(r - (int64_t)x[1] * ex);
  x[0] += q.g; x[1] += q.g; x[2] += q.g;
  gptr<double> Ee = b.scratch + off_edge(q);
  const int64_t ne = n_edges(q), e = edge(q, x[0], x[1], x[2]);
  if (x[0] < q.g + q.nx) Ee[e] = corner_emf<0>(b, q, x);
  if (x[1] < q.g + q.ny) Ee[ne + e] = corner_emf<1>(b, q, x);
  if (x[2] < q.g + q.nz) Ee[2 * ne + e] = corner_emf<2>(b, q, x);
}

// bo = a0 bn + a1 bs - b dt (curl E)^D on the interior face of direction D at x
template <int D>
__device__ __forceinline__ void ct_face(const GB& b, const Geo& q, const int x[3], double dt,
                                        double a0, double a1, double bb) {
#pragma clang fp contract(off)
  constexpr int D1 = (D + 1) % 3, D2 = (D + 2) % 3;
  gptr<const double> Ee = b.scratch + off_edge(q);
  const int64_t ne = n_edges(q);
  int x1[3] = {x[0], x[1], x[2]}, x2[3] = {x[0], x[1], x[2]};
  x1[D1] += 1;
  x2[D2] += 1;
  const int64_t e0 = edge(q, x[0], x[1], x[2]);
  const double c1 = (Ee[D2 * ne + edge(q, x1[0], x1[1], x1[2])] - Ee[D2 * ne + e0]) / b.dx[D1];
  const double c2 = (Ee[D1 * ne + edge(q, x2[0], x2[1], x2[2])] - Ee[D1 * ne + e0]) / b.dx[D2];
  const int64_t f = face<D>(q, x[0], x[1], x[2]);
  b.bo[D][f] = a0 * b.bn[D][f] + a1 * b.bs[D][f] - bb * dt * (c1 - c2);
}

// the face update of all three directions at the corners [g, g+n]^3: item x
// owns the lower face of direction D of cell x when x is inside along the
// other two directions
__global__ __launch_bounds__(kMaxThreads) void k_ct_faces(const grmhd_block* __restrict__ blks,
                                                       const double* dt_d, double dt_h, double a0,
                                                       double a1, double bb) {
  int bi;
  int64_t t;
  if (!locate(blks, S_CORNER, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  const int ex = q.nx + 1, ey = q.ny + 1;
  int x[3];
  x[2] = (int)(t / ((int64_t)ex * ey));
  const int64_t r = t - (int64_t)x[2] * ex * ey;
  x[1] = (int)(r / ex);
  x[0] = (int)(r - (int64_t)x[1] * ex);
  x[0] += q.g; x[1] += q.g; x[2] += q.g;
  const double dt = dt_of(dt_d, dt_h);
  const bool in0 = x[0] < q.g + q.nx, in1 = x[1] < q.g + q.ny, in2 = x[2] < q.g + q.nz;
  if (in1 && in2) ct_face<0>(b, q, x, dt, a0, a1, bb);
  if (in0 && in2) ct_face<1>(b, q, x, dt, a0, a1, bb);
  if (in0 && in1) ct_face<2>(b, q, x, dt, a0, a1, bb);
}

// ---------------------------------------------------------------------------
// a6: update with the Eq. 10 sources of the stage input
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dcen(gptr<const double> a, int64_t c, int64_t st, double idx12) {
  return ((a[c - 2 * st] - a[c + 2 * st]) - 8.0 * (a[c - st] - a[c + st])) * idx12;
}

// Brick layout of the update, for block lists whose blocks are all kBrickW
// cells wide with ny a multiple of kBrickY and nz a multiple of kBrickZ,
// launched with kMaxThreads-thread workgroups: a workgroup is a brick of
// kBrickY x kBrickZ x rows (wave w on row j0 + w % kBrickY of plane
// k0 + w / kBrickY, lane = x), bricks ordered y fastest, then z.  The metric
// fields pass through LDS one at a time: each wave stores its own row with
// its four x ghosts and three of the brick's 24 halo rows (two rows beyond it
// in y on each of its planes, two planes beyond it in z on each of its rows),
// so every neighbour of the gradient stencil is read from LDS: the stencils
// take 5 vector-memory loads per field and wave instead of 10.
constexpr int kBrickW = 64;
constexpr int kBrickY = 2;
constexpr int kBrickZ = kMaxThreads / 64 / kBrickY;
constexpr int kBrickPitch = kBrickW + 4;
constexpr int kBrickPlane = (kBrickY + 4) * kBrickPitch;
constexpr int kBrickHalo = 4 * kBrickZ + 4 * kBrickY;   // y halo rows + z halo rows
static_assert(kBrickHalo == 3 * (kMaxThreads / 64), "three halo rows per wave");

// block and brick of this workgroup in the brick layout (uniform over it)
__device__ __forceinline__ void locate_brick(const grmhd_block* __restrict__ blks, int& bi,
                                             int& brick) {
  const int w = __builtin_amdgcn_readfirstlane(xcd_linear() * (kMaxThreads / 64));
  const int nb = blks[0].nblk;
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blks[mid].wave0[S_INTERIOR] <= w) lo = mid; else hi = mid - 1;
  }
  bi = lo;
  brick = (w - blks[bi].wave0[S_INTERIOR]) / (kMaxThreads / 64);
}

// C2P: the inversion of a8 follows in the same thread (the updated U and the
// faces bo of the CT step are final by then), so U is written once, after
// the floors, and never read back; the granular update entry point runs
// without it.
template <int ET, bool BRICK, bool C2P>
__global__ __launch_bounds__(kMaxThreads) void k_update(const grmhd_block* __restrict__ blks, Eos e_in,
                                                     const double* dt_d, double dt_h, double a0,
                                                     double a1, double bb, grmhd_params p) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int i, j, k;
  if constexpr (BRICK) {
    int brick;
    locate_brick(blks, bi, brick);
    const int by = blks[bi].ny / kBrickY, g0 = blks[bi].ng;
    // uniform over the workgroup: a launch that does not match the layout
    // returns before any memory access or barrier
    if (blockDim.x != kMaxThreads || brick < 0 || brick >= by * (blks[bi].nz / kBrickZ)) return;
    const int w = (int)(threadIdx.x >> 6);
    i = g0 + (int)(threadIdx.x & 63);
    j = g0 + (brick % by) * kBrickY + w % kBrickY;
    k = g0 + (brick / by) * kBrickZ + w / kBrickY;
  } else {
    int64_t t;
    if (!locate(blks, S_INTERIOR, bi, t)) return;
    interior_box(geo_of(blks[bi])).at(t, i, j, k);
  }
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  const int64_t c = cell(q, i, j, k);
  const double dt = dt_of(dt_d, dt_h);
  const int64_t strides[3] = {1, (int64_t)q.sx, (int64_t)q.sx * q.sy};
  M3 m;
  cell_metric(b, c, m);
  const double alpha = b.adm[0][c];
  // primitive-derived quantities of the stage input
  const double rho = b.w[0][c], P = b.w[4][c];
  const double u[3] = {b.w[1][c], b.w[2][c], b.w[3][c]};
  double ul[3];
  lower(m.g, u[0], u[1], u[2], ul[0], ul[1], ul[2]);
  const double W = sqrt(1.0 + u[0] * ul[0] + u[1] * ul[1] + u[2] * ul[2]);
  const double iW = 1.0 / W;
  const double v[3] = {u[0] * iW, u[1] * iW, u[2] * iW};
  double Bt[3];
  cell_bt(q, b.bs, i, j, k, Bt);
  const double is = 1.0 / m.sg;
  const double B[3] = {Bt[0] * is, Bt[1] * is, Bt[2] * is};
  double Bl[3];
  lower(m.g, B[0], B[1], B[2], Bl[0], Bl[1], Bl[2]);
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  const double Bv = (B[0] * ul[0] + B[1] * ul[1] + B[2] * ul[2]) * iW;
  const double eps = eos_eps_from_P(e, rho, P);
  const double h = 1.0 + eps + P / rho;
  const double bsq = B2 * iW * iW + Bv * Bv;
  const double Ptot = P + 0.5 * bsq;
  const double ew = (rho * h + bsq) * W * W;
  double bsp[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) bsp[a] = B[a] * iW + W * Bv * v[a];
  // densitized S~^{ij} (symmetric)
  double S[6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c2 = a; c2 < 3; ++c2)
      S[sym(a, c2)] = m.sg * (ew * v[a] * v[c2] + Ptot * m.u[sym(a, c2)] - bsp[a] * bsp[c2]);
  double Us[5];
#pragma unroll
  for (int v2 = 0; v2 < 5; ++v2) Us[v2] = b.us[v2][c];
  const double Su[3] = {m.u[0] * Us[1] + m.u[1] * Us[2] + m.u[2] * Us[3],
                        m.u[1] * Us[1] + m.u[3] * Us[2] + m.u[4] * Us[3],
                        m.u[2] * Us[1] + m.u[4] * Us[2] + m.u[5] * Us[3]};
  const double Et = Us[4] + Us[0];
  double G[5];
  G[0] = 0.0;
  G[1] = G[2] = G[3] = 0.0;
  double gt = 0.0;
  const double idx12[3] = {1.0 / (12.0 * b.dx[0]), 1.0 / (12.0 * b.dx[1]), 1.0 / (12.0 * b.dx[2])};
  // One metric field at a time, in a loop that is not unrolled: unrolled, the
  // compiler issues the 120 stencil loads of the ten fields together and
  // holds them in registers (two waves per SIMD instead of four).  Field f's
  // gradient enters G[1..3] with coefficient -E (alpha), S~_a (beta^a) or
  // alpha S~^{jk}/2 (gamma_jk, the off-diagonal ones twice); the alpha
  // gradient also enters the tau source.
#pragma unroll 1
  for (int f = 0; f < 10; ++f) {
    double cf;
    if (f == 0) {
      cf = -Et;
    } else if (f < 4) {
      cf = f == 1 ? Us[1] : (f == 2 ? Us[2] : Us[3]);
    } else {
      const int s6 = f - 4;
      const double Sv = s6 == 0 ? S[0] : s6 == 1 ? S[1] : s6 == 2 ? S[2] : s6 == 3 ? S[3]
                                                                        : s6 == 4 ? S[4] : S[5];
      cf = 0.5 * alpha * ((s6 == 1 || s6 == 2 || s6 == 4) ? 2.0 : 1.0) * Sv;
    }
    const gptr<const double> a = (gptr<const double>)blks[bi].adm[f];
    double gr[3];
    if constexpr (BRICK) {
      // tile[z][y][x] over planes k0-2..k0+kBrickZ+1, rows j0-2..j0+kBrickY+1
      __shared__ double tile[(kBrickZ + 4) * kBrickPlane];
      const int lane = threadIdx.x & 63;
      const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
      const int wy = w % kBrickY, wz = w / kBrickY;
      const int64_t py = strides[1], pz = strides[2];
      const int64_t c0 = c - wy * py - wz * pz;   // the brick's first row, this lane's x
      const double v0 = a[c];
      double vx = 0.0;
      // lanes 0..3 fetch the row's x ghosts -2, -1, 64, 65
      const int xo = lane < 2 ? lane - 2 : kBrickW - 2 + lane;
      if (lane < 4) vx = a[c - lane + xo];
      // three halo rows: h < 4 kBrickZ are the y halo (plane h / 4, rows
      // -2, -1, kBrickY, kBrickY + 1), the rest the z halo (row (h - 4 kBrickZ)
      // % kBrickY, planes -2, -1, kBrickZ, kBrickZ + 1)
      double vh[3];
      int th[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int h = w + r * (kMaxThreads / 64);
        int hy, hz;
        if (h < 4 * kBrickZ) {
          const int m = h % 4;
          hz = h / 4;
          hy = m < 2 ? m - 2 : kBrickY - 2 + m;
        } else {
          const int m = (h - 4 * kBrickZ) / kBrickY;
          hy = (h - 4 * kBrickZ) % kBrickY;
          hz = m < 2 ? m - 2 : kBrickZ - 2 + m;
        }
        vh[r] = a[c0 + hz * pz + hy * py];
        th[r] = (hz + 2) * kBrickPlane + (hy + 2) * kBrickPitch + lane + 2;
      }
      __syncthreads();  // the previous field's reads of the tile are done
      double* row = tile + (wz + 2) * kBrickPlane + (wy + 2) * kBrickPitch;
      row[lane + 2] = v0;
      if (lane < 4) row[xo + 2] = vx;
#pragma unroll
      for (int r = 0; r < 3; ++r) tile[th[r]] = vh[r];
      __syncthreads();
      const double* p = row + lane + 2;
      gr[0] = ((p[-2] - p[2]) - 8.0 * (p[-1] - p[1])) * idx12[0];
      gr[1] = ((p[-2 * kBrickPitch] - p[2 * kBrickPitch]) -
               8.0 * (p[-kBrickPitch] - p[kBrickPitch])) * idx12[1];
      gr[2] = ((p[-2 * kBrickPlane] - p[2 * kBrickPlane]) -
               8.0 * (p[-kBrickPlane] - p[kBrickPlane])) * idx12[2];
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) gr[d] = dcen(a, c, strides[d], idx12[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      G[1 + d] += cf * gr[d];
      if (f == 0) gt -= Su[d] * gr[d];
    }
  }
  double kS = 0.0;
#pragma unroll
  for (int s6 = 0; s6 < 6; ++s6) {
    const double w6 = (s6 == 1 || s6 == 2 || s6 == 4) ? 2.0 : 1.0;
    kS += w6 * b.adm[10 + s6][c] * S[s6];
  }
  G[4] = alpha * kS + gt;
  double Uo[5];
#pragma unroll
  for (int v2 = 0; v2 < 5; ++v2)
    Uo[v2] = a0 * b.un[v2][c] + a1 * Us[v2] + bb * dt * (G[v2] - flux_div(b, q, v2, i, j, k));
  if constexpr (!C2P) {
#pragma unroll
    for (int v2 = 0; v2 < 5; ++v2) b.uo[v2][c] = Uo[v2];
  } else {
    // a8 on the updated state with the updated faces (as k_stage_c2p); the
    // metric is loaded again (the barrier keeps the update's copy from
    // living on into the root solve)
    __asm__ volatile("" ::: "memory");
    double w[5];
    C2PWork cw;
    {
      M3 m1;
      cell_metric(b, c, m1);
      double Bt[3];
      cell_bt(q, b.bo, i, j, k, Bt);
      cw = c2p_prepare(e, p, m1, Uo, Bt, w);
    }
    uint32_t r = cw.fl;
    bool rebuilt = cw.done;
    if (!cw.done) {
      int nev;
      double mu;
      r = c2p_lean(e, p, cw, w, false, 0.0, 0.0, nev, mu);
      if (r & kFloorBits) {
        // U from the final primitives; metric and field loaded again (the
        // barrier keeps them from living across the root solve)
        __asm__ volatile("" ::: "memory");
        M3 m2;
        cell_metric(b, c, m2);
        double Bt[3];
        cell_bt(q, b.bo, i, j, k, Bt);
        prim_to_cons(e, m2, w, Bt, Uo);
        rebuilt = true;
      }
    }
    (void)rebuilt;
#pragma unroll
    for (int v2 = 0; v2 < 5; ++v2) b.uo[v2][c] = Uo[v2];
#pragma unroll
    for (int v2 = 0; v2 < 5; ++v2) b.wo[v2][c] = w[v2];
    b.flags[c] = (uint16_t)(b.flags[c] | r);
  }
}

// ---------------------------------------------------------------------------
// a8: inversion of the updated state with the updated field
// ---------------------------------------------------------------------------
template <int ET>
__global__ __launch_bounds__(kMaxThreads) void k_stage_c2p(const grmhd_block* __restrict__ blks, Eos e_in,
                                                        grmhd_params p, c2p_stats* stats) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int64_t t;
  const bool live = locate(blks, S_INTERIOR, bi, t);   // no early return: wave sums below
  unsigned long long c_n = 0, c_ev = 0, c_fail = 0;
  if (live) {
    const GB b = gview(blks[bi]);
    const Geo q = geo_of(b);
    const Box bx = interior_box(q);
    int i, j, k;
    bx.at(t, i, j, k);
    const int64_t c = cell(q, i, j, k);
    double w[5];
    C2PWork cw;
    {
      M3 m;
      cell_metric(b, c, m);
      double U[5], Bt[3];
#pragma unroll
      for (int v = 0; v < 5; ++v) U[v] = b.uo[v][c];
      cell_bt(q, b.bo, i, j, k, Bt);
      cw = c2p_prepare(e, p, m, U, Bt, w);
      if (cw.done) {
#pragma unroll
        for (int v = 0; v < 5; ++v) b.uo[v][c] = U[v];
      }
    }
    uint32_t r = cw.fl;
    int nev = 0;
    if (!cw.done) {
      double mu;
      r = c2p_lean(e, p, cw, w, false, 0.0, 0.0, nev, mu);
      if (r & kFloorBits) {
        // U from the final primitives; metric and field loaded again (the
        // barrier keeps them from living across the root solve)
        __asm__ volatile("" ::: "memory");
        M3 m;
        cell_metric(b, c, m);
        double U[5], Bt[3];
        cell_bt(q, b.bo, i, j, k, Bt);
        prim_to_cons(e, m, w, Bt, U);
#pragma unroll
        for (int v = 0; v < 5; ++v) b.uo[v][c] = U[v];
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) b.wo[v][c] = w[v];
    b.flags[c] = (uint16_t)(b.flags[c] | r);
    c_n = 1;
    c_ev = (unsigned long long)nev;
    c_fail = (r & GRMHD_F_C2P_FAIL) ? 1 : 0;
  }
  // per-wave sums into the block's scratch (summed by k_stats_sum): no
  // global atomics per wave
  if (stats && __shfl((int)live, 0, 64)) {
    const GB b = gview(blks[bi]);
    wave_stats_store(b, geo_of(b), t, c_n, c_ev, 0ull, c_fail);
  }
}

// sum of the per-wave inversion statistics of every block into stats
// (one workgroup per block, four atomics per block)
__global__ __launch_bounds__(kThreads) void k_stats_sum(const grmhd_block* __restrict__ blks,
                                                        c2p_stats* stats) {
  const grmhd_block& b = blks[blockIdx.x];
  const Geo q = geo_of(b);
  const int64_t nw = (shape_items(q, S_INTERIOR) + 63) / 64;
  const unsigned long long* ws = (const unsigned long long*)(b.scratch + off_wstat(q));
  unsigned long long a[4] = {0ull, 0ull, 0ull, 0ull};
  for (int64_t i = threadIdx.x; i < nw; i += blockDim.x)
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] += ws[4 * i + c];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) a[c] += __shfl_xor(a[c], o, 64);
  __shared__ unsigned long long part[kThreads / 64][4];
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) part[threadIdx.x >> 6][c] = a[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv)
      for (int c = 0; c < 4; ++c) part[0][c] += part[wv][c];
    atomicAdd(&stats->solves, part[0][0]);
    atomicAdd(&stats->evaluations, part[0][1]);
    atomicAdd(&stats->fallbacks, part[0][2]);
    atomicAdd(&stats->failures, part[0][3]);
  }
}

// ---------------------------------------------------------------------------
// ADM matter sources of the interior cells (stage-input w and faces bs) into
// out[10 * block + n], padded cell arrays
// ---------------------------------------------------------------------------
template <int ET>
__global__ __launch_bounds__(kMaxThreads) void k_matter(const grmhd_block* __restrict__ blks, Eos e_in,
                                                     double* const* __restrict__ out) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int64_t t;
  if (!locate(blks, S_INTERIOR, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  int i, j, k;
  interior_box(q).at(t, i, j, k);
  const int64_t c = cell(q, i, j, k);
  M3 m;
  cell_metric(b, c, m);
  double w[5], Bt[3], o[10];
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = b.w[v][c];
  cell_bt(q, b.bs, i, j, k, Bt);
  matter_sources(e, m, w, Bt, o);
#pragma unroll
  for (int n = 0; n < 10; ++n) ((gptr<double>)out[10 * bi + n])[c] = o[n];
}

// lapse excision of the stage output: atmosphere where alpha < alpha_min,
// conserved state rebuilt with the unchanged field (Sec. IV)
template <int ET>
__global__ __launch_bounds__(kMaxThreads) void k_excise(const grmhd_block* __restrict__ blks, Eos e_in,
                                                     grmhd_params p, double alpha_min) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int64_t t;
  if (!locate(blks, S_INTERIOR, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  int i, j, k;
  interior_box(q).at(t, i, j, k);
  const int64_t c = cell(q, i, j, k);
  if (!(b.adm[0][c] < alpha_min)) return;
  M3 m;
  cell_metric(b, c, m);
  double w[5], Bt[3], U[5];
  atmosphere(e, p, w);
  cell_bt(q, b.bo, i, j, k, Bt);
  prim_to_cons(e, m, w, Bt, U);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    b.uo[v][c] = U[v];
    b.wo[v][c] = w[v];
  }
  b.flags[c] = (uint16_t)(b.flags[c] | GRMHD_F_EXCISED);
}

// ---------------------------------------------------------------------------
// ghost fill (same-level copy, periodic self-neighbour, outflow)
// ---------------------------------------------------------------------------
// source of ghost entry x[] of block ib; fd = -1 for cells, else the face
// direction (faces g and g+n along it are interior).  Returns false if x is
// interior.
__device__ __forceinline__ bool ghost_src(const grmhd_block* blks, int ib, int fd, int x[3],
                                          int& sb) {
  const grmhd_block& b = blks[ib];
  const int g = b.ng;
  const int n[3] = {b.nx, b.ny, b.nz};
  int o[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int hi = a == fd ? g + n[a] : g + n[a] - 1;   // last interior index
    o[a] = x[a] < g ? -1 : (x[a] > hi ? 1 : 0);
  }
  if (!o[0] && !o[1] && !o[2]) return false;
  // axes with no neighbour: clamp (outflow)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!o[a]) continue;
    const int idx = (a == 0 ? o[a] + 1 : 1) + 3 * (a == 1 ? o[a] + 1 : 1) + 9 * (a == 2 ? o[a] + 1 : 1);
    if (b.nbr[idx] < 0) {
      const int hi = a == fd ? g + n[a] : g + n[a] - 1;
      x[a] = o[a] < 0 ? g : hi;
      o[a] = 0;
    }
  }
  sb = ib;
  if (o[0] || o[1] || o[2]) {
    const int nb = b.nbr[(o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
    if (nb < 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (!o[a]) continue;
        const int hi = a == fd ? g + n[a] : g + n[a] - 1;
        x[a] = o[a] < 0 ? g : hi;
      }
    } else if (nb == ib) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (!o[a]) continue;
        int r = (x[a] - g) % n[a];
        if (r < 0) r += n[a];
        x[a] = g + r;
      }
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] -= o[a] * n[a];
      sb = nb;
    }
  }
  return true;
}

// list != 0 (flags exchange of a stage): flagged cells of the first ghost
// shell [g-1, g+n]^3 are appended to the block's FOFC list
// Items are the ghost cells only (launch shape S_GCELLS), or, for the flag
// exchange of a stage (list != 0, flags only), the first ghost shell
// [g-1, g+n]^3 (S_GSHELL), whose flagged cells are appended to the block's
// FOFC list; the refluxing reads no flag farther out.
__global__ __launch_bounds__(kMaxThreads) void k_ghost_cells(const grmhd_block* __restrict__ blks,
                                                          int mask, int list) {
  int ib;
  int64_t t;
  const int cls = list ? S_GSHELL : S_GCELLS;
  if (!locate(blks, cls, ib, t)) return;
  if (blks[ib].bc == 0) return;
  const GB b = gview(blks[ib]);
  const Geo q = geo_of(b);
  int x[3];
  ghost_ring(q, cls).at(t, x[0], x[1], x[2]);
  if (list) {
    x[0] += q.g - 1; x[1] += q.g - 1; x[2] += q.g - 1;
  }
  const int64_t c = cell(q, x[0], x[1], x[2]);
  int sb;
  if (!ghost_src(blks, ib, -1, x, sb)) return;   // never taken: every item is a ghost
  const GB s = gview(blks[sb]);
  const Geo qs = geo_of(s);
  const int64_t src = cell(qs, x[0], x[1], x[2]);
  if (mask & 1)
#pragma unroll
    for (int v = 0; v < 5; ++v) b.w[v][c] = s.w[v][src];
  if (mask & 2)
#pragma unroll
    for (int v = 0; v < 5; ++v) b.us[v][c] = s.us[v][src];
  if (mask & 8) {
    const uint16_t f = s.flags[src];
    b.flags[c] = f;
    if (list) fofc_append(b, q, (f & (GRMHD_F_FOFC | GRMHD_F_DMP)) != 0, c);
  }
}

// ghost faces of direction d (launch shape S_GXFACE + d)
__global__ __launch_bounds__(kMaxThreads) void k_ghost_faces(const grmhd_block* __restrict__ blks,
                                                          int d) {
  int ib;
  int64_t t;
  if (!locate(blks, S_GXFACE + d, ib, t)) return;
  if (blks[ib].bc == 0) return;
  const Geo q = geo_of(blks[ib]);
  int x[3];
  ghost_ring(q, S_GXFACE + d).at(t, x[0], x[1], x[2]);
  const int64_t f = face_rt(q, d, x[0], x[1], x[2]);
  int sb;
  if (!ghost_src(blks, ib, d, x, sb)) return;   // never taken: every item is a ghost
  // the face direction is a runtime value: index the C struct's arrays
  // (an indexed copy of the view would live in scratch memory)
  const Geo qs = geo_of(blks[sb]);
  const gptr<const double> src = (gptr<const double>)blks[sb].bs[d];
  ((gptr<double>)blks[ib].bs[d])[f] = src[face_rt(qs, d, x[0], x[1], x[2])];
}

// pointer arrays of the pointwise kernels (passed by value)
struct Ptrs5 { double* p[5]; };
struct Ptrs3 { double* p[3]; };
struct Ptrs6 { double* p[6]; };

// ---------------------------------------------------------------------------
// training pairs of the learned inversion: the interior cells of every block
// (every stride-th along x), flattened block by block from base[block]: the
// conserved state of the us slot, the densitized cell-centred field of the
// bs faces (reading R1: the face average per direction), gamma_ij and the
// primitives of the w slot
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_c2p_pairs(const grmhd_block* __restrict__ blks,
                                                        int stride, const int64_t* __restrict__ base,
                                                        Ptrs5 u, Ptrs3 bt, Ptrs6 gm, Ptrs5 w) {
  int bi;
  int64_t t;
  if (!locate(blks, S_INTERIOR, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  int i, j, k;
  interior_box(q).at(t, i, j, k);
  const int li = i - q.g;
  if (li % stride) return;
  const int64_t row = (q.nx + stride - 1) / stride;
  const int64_t o = base[bi] + ((int64_t)(k - q.g) * q.ny + (j - q.g)) * row + li / stride;
  const int64_t c = cell(q, i, j, k);
  double Bt[3];
  cell_bt(q, b.bs, i, j, k, Bt);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    u.p[v][o] = b.us[v][c];
    w.p[v][o] = b.w[v][c];
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) bt.p[v][o] = Bt[v];
#pragma unroll
  for (int v = 0; v < 6; ++v) gm.p[v][o] = b.adm[4 + v][c];
}

// ---------------------------------------------------------------------------
// a9: dt reduction (max of |lambda|/dx; order-independent, exact), alone
// ---------------------------------------------------------------------------

template <int ET>
__global__ __launch_bounds__(kMaxThreads) void k_dt(const grmhd_block* __restrict__ blks, Eos e_in,
                                                 double* red) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int64_t t;
  const bool live = locate(blks, S_INTERIOR, bi, t);   // no early return: barrier below
  double s = 0.0;
  if (live) {
    const GB b = gview(blks[bi]);
    const Geo q = geo_of(b);
    const Box bx = interior_box(q);
    int i, j, k;
    bx.at(t, i, j, k);
    s = cfl_speed(e, b, q, i, j, k);
  }
  workgroup_max_into(s, red);
}

__global__ void k_dt_final(const double* red, double cfl, double* dt_out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dt_out[0] = cfl / red[0];
}

// ---------------------------------------------------------------------------
// mass: deterministic two-level sum
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_mass_block(const grmhd_block* __restrict__ blks,
                                                         double* partial) {
  const grmhd_block& b = blks[blockIdx.x];
  const Geo q = geo_of(b);
  const Box bx = interior_box(q);
  const int64_t n = bx.size();
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
    int i, j, k;
    bx.at(t, i, j, k);
    s += b.us[0][cell(q, i, j, k)];
  }
  __shared__ double sh[kThreads];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] * (b.dx[0] * b.dx[1] * b.dx[2]);
}

__global__ void k_mass_final(const double* partial, int nblk, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int x = 0; x < nblk; ++x) s += partial[x];
    out[0] = s;
  }
}

// Eq. 7 over every padded cell of a block: us <- prim2con(w, B~_cc(bs))
template <int ET>
__global__ __launch_bounds__(kMaxThreads) void k_p2c_block(const grmhd_block* __restrict__ blks, Eos e_in) {
  const Eos e = eos_fixed<ET>(e_in);
  int bi;
  int64_t t;
  if (!locate(blks, S_CELLS, bi, t)) return;
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  const int i = (int)(t % q.sx), j = (int)((t / q.sx) % q.sy), k = (int)(t / ((int64_t)q.sx * q.sy));
  M3 m;
  cell_metric(b, t, m);
  double Bt[3], w[5], U[5];
  cell_bt(q, b.bs, i, j, k, Bt);
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = b.w[v][t];
  prim_to_cons(e, m, w, Bt, U);
#pragma unroll
  for (int v = 0; v < 5; ++v) b.us[v][t] = U[v];
}

// ---------------------------------------------------------------------------
// pointwise kernels
// ---------------------------------------------------------------------------

template <int ET>
__global__ __launch_bounds__(kThreads) void k_prim2con(int64_t n, Ptrs5 w, Ptrs3 bt, Ptrs6 gm,
                                                       Ptrs5 u, Eos e_in) {
  const Eos e = eos_fixed<ET>(e_in);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  M3 m;
  metric_build(m, gm.p[0][t], gm.p[1][t], gm.p[2][t], gm.p[3][t], gm.p[4][t], gm.p[5][t]);
  const double ww[5] = {w.p[0][t], w.p[1][t], w.p[2][t], w.p[3][t], w.p[4][t]};
  const double B[3] = {bt.p[0][t], bt.p[1][t], bt.p[2][t]};
  double U[5];
  prim_to_cons(e, m, ww, B, U);
#pragma unroll
  for (int v = 0; v < 5; ++v) u.p[v][t] = U[v];
}

// inversion of n states; optional per-state bracket [blo, bhi] (learned
// guess, computed by a separate kernel); statistics reduced per wave first
template <int ET>
__global__ __launch_bounds__(kThreads) void k_c2p_batch(int64_t n, Ptrs5 u, Ptrs3 bt, Ptrs6 gm,
                                                        Ptrs5 w, uint16_t* flags, Eos e_in,
                                                        grmhd_params p_in, const double* blo,
                                                        const double* bhi, double* mu_out,
                                                        int32_t* nev_out, c2p_stats* stats) {
  const Eos e0 = eos_fixed<ET>(e_in);
  const grmhd_params p0 = p_in;
  unsigned long long c_n = 0, c_ev = 0, c_fb = 0, c_fail = 0;
  // grid-stride loop: each lane keeps its statistics until the end, so the
  // atomics are per wave of a bounded grid, not per 64 states
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    Eos e = e0;
    grmhd_params p = p0;
    consts_per_pass(e, p);
    C2PWork cw;
    double ww[5];
    {
      M3 m;
      metric_build(m, gm.p[0][t], gm.p[1][t], gm.p[2][t], gm.p[3][t], gm.p[4][t], gm.p[5][t]);
      double U[5] = {u.p[0][t], u.p[1][t], u.p[2][t], u.p[3][t], u.p[4][t]};
      const double B[3] = {bt.p[0][t], bt.p[1][t], bt.p[2][t]};
      cw = c2p_prepare(e, p, m, U, B, ww);
      if (cw.done) {
#pragma unroll
        for (int v = 0; v < 5; ++v) u.p[v][t] = U[v];
      }
    }
    int nev = 0;
    double mu = 0.0;
    uint32_t r = cw.fl;
    if (!cw.done) {
      const bool br = blo != nullptr;
      r = c2p_lean(e, p, cw, ww, br, br ? blo[t] : 0.0, br ? bhi[t] : 0.0, nev, mu);
      if (r & kFloorBits) {
        // a rule fired: U from the final primitives, with the metric and field
        // loaded again (the barrier keeps them from living across the solve)
        __asm__ volatile("" ::: "memory");
        M3 m;
        metric_build(m, gm.p[0][t], gm.p[1][t], gm.p[2][t], gm.p[3][t], gm.p[4][t], gm.p[5][t]);
        const double B[3] = {bt.p[0][t], bt.p[1][t], bt.p[2][t]};
        double U[5];
        prim_to_cons(e, m, ww, B, U);
#pragma unroll
        for (int v = 0; v < 5; ++v) u.p[v][t] = U[v];
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) w.p[v][t] = ww[v];
    flags[t] = (uint16_t)r;
    if (mu_out) mu_out[t] = mu;
    if (nev_out) nev_out[t] = nev;
    c_n += 1;
    c_ev += (unsigned long long)nev;
    c_fb += (r & GRMHD_F_BRACKET_FALLBACK) ? 1 : 0;
    c_fail += (r & GRMHD_F_C2P_FAIL) ? 1 : 0;
  }
  if (stats) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      c_n += __shfl_xor(c_n, o, 64);
      c_ev += __shfl_xor(c_ev, o, 64);
      c_fb += __shfl_xor(c_fb, o, 64);
      c_fail += __shfl_xor(c_fail, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && c_n) {
      atomicAdd(&stats->solves, c_n);
      atomicAdd(&stats->evaluations, c_ev);
      if (c_fb) atomicAdd(&stats->fallbacks, c_fb);
      if (c_fail) atomicAdd(&stats->failures, c_fail);
    }
  }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
Eos make_eos(const grmhd_params& p) {
  Eos e;
  memset(&e, 0, sizeof(e));
  e.type = p.eos;
  e.gam = p.gamma;
  e.gth = p.gamma_th;
  e.n = p.eos == 1 ? p.npieces : 1;
  if (p.eos == 1) {
    for (int i = 0; i < e.n; ++i) e.G[i] = p.Gam[i];
    e.K[0] = p.K0;
    e.a[0] = 0.0;
    for (int i = 1; i < e.n; ++i) {
      const double r = p.rho_b[i - 1];
      e.rb[i - 1] = r;
      // P_cold and eps_cold continuous at r
      e.K[i] = e.K[i - 1] * pow(r, e.G[i - 1]) / pow(r, e.G[i]);
      const double pr = e.K[i - 1] * pow(r, e.G[i - 1]);
      e.a[i] = e.a[i - 1] + pr / (r * (e.G[i - 1] - 1.0)) - pr / (r * (e.G[i] - 1.0));
    }
  }
  return e;
}

int check_params(const grmhd_params* p) {
  if (!p) return GRMHD_EINVAL;
  if (p->eos != 0 && p->eos != 1) return GRMHD_EINVAL;
  if (p->eos == 1 && (p->npieces < 1 || p->npieces > 4)) return GRMHD_EINVAL;
  if (p->recon < 0 || p->recon > 4) return GRMHD_EUNSUPPORTED;
  if (p->riemann != 0 && p->riemann != 1) return GRMHD_EINVAL;
  if (p->c2p_maxit < 1) return GRMHD_EINVAL;
  return GRMHD_OK;
}

int64_t prepare_layout(grmhd_block* h, int nblk, bool write);

int check_blocks(const grmhd_block* h, const grmhd_block* d, int nblk) {
  if (!h || !d || nblk < 1) return GRMHD_EINVAL;
  if (prepare_layout(const_cast<grmhd_block*>(h), nblk, false) != 0) return GRMHD_EINVAL;
  for (int i = 0; i < nblk; ++i) {
    const grmhd_block& b = h[i];
    if (b.ng < 3 || b.nx < 1 || b.ny < 1 || b.nz < 1) return GRMHD_EINVAL;
    if (!b.scratch || !b.flags) return GRMHD_EINVAL;
    for (int v = 0; v < 5; ++v)
      if (!b.w[v] || !b.un[v] || !b.us[v] || !b.uo[v] || !b.wo[v]) return GRMHD_EINVAL;
    for (int v = 0; v < 3; ++v)
      if (!b.bn[v] || !b.bs[v] || !b.bo[v]) return GRMHD_EINVAL;
    for (int v = 0; v < 16; ++v)
      if (!b.adm[v]) return GRMHD_EINVAL;
    for (int v = 0; v < 27; ++v)
      if (b.nbr[v] < -1 || b.nbr[v] >= nblk) return GRMHD_EINVAL;
    if (b.bc == 1) {
      // a neighbour supplies ng layers: its extent must cover them
      for (int v = 0; v < 27; ++v) {
        const int nb = b.nbr[v];
        if (nb < 0 || nb == i) continue;
        const grmhd_block& s = h[nb];
        if (s.nx != b.nx || s.ny != b.ny || s.nz != b.nz || s.ng != b.ng) return GRMHD_EINVAL;
        if (s.nx < b.ng || s.ny < b.ng || s.nz < b.ng) return GRMHD_EINVAL;
      }
    }
  }
  return GRMHD_OK;
}


// Arrays a pointwise block-list call reads: the layout must be current and
// every block at least one cell wide with the arrays in `need` set
// (bits: 1 w, 2 us[0] only, 4 bs, 8 metric adm[0..9], 16 all of us).
enum { NEED_W = 1, NEED_D = 2, NEED_BS = 4, NEED_ADM = 8, NEED_US = 16 };
int check_reads(const grmhd_block* h, const grmhd_block* d, int nblk, int need) {
  if (!h || !d || nblk < 1) return GRMHD_EINVAL;
  if (prepare_layout(const_cast<grmhd_block*>(h), nblk, false) != 0) return GRMHD_EINVAL;
  for (int i = 0; i < nblk; ++i) {
    const grmhd_block& b = h[i];
    if (b.nx < 1 || b.ny < 1 || b.nz < 1 || b.ng < 0) return GRMHD_EINVAL;
    for (int v = 0; v < 5; ++v) {
      if ((need & NEED_W) && !b.w[v]) return GRMHD_EINVAL;
      if ((need & NEED_US) && !b.us[v]) return GRMHD_EINVAL;
    }
    if ((need & NEED_D) && !b.us[0]) return GRMHD_EINVAL;
    for (int v = 0; v < 3; ++v)
      if ((need & NEED_BS) && !b.bs[v]) return GRMHD_EINVAL;
    for (int v = 0; v < 10; ++v)
      if ((need & NEED_ADM) && !b.adm[v]) return GRMHD_EINVAL;
  }
  return GRMHD_OK;
}

// 1-D grid over all 64-item waves of launch shape cls in the block list
dim3 grid_cls(const grmhd_block* h, int nblk, int cls, int threads) {
  const int64_t waves = (int64_t)h[nblk - 1].wave0[cls] + (shape_items(geo_of(h[nblk - 1]), cls) + 63) / 64;
  return dim3((unsigned)((waves * 64 + threads - 1) / threads), 1, 1);
}

// workgroup size per kernel family (64..512, multiple of 64), set by the
// autotuner through grmhd_set_threads
int g_threads[kFamilies] = {256, 256, 256, 256, 256, 256, 256, 256, 256,
                             256, 256, 256, 256, 256, 256, 256, 256, 256};
inline int tpb(int fam) { return g_threads[fam]; }

// launch layout of a block table: first wave of each block per shape
constexpr int kWaveSlots = (int)(sizeof(((grmhd_block*)0)->wave0) / sizeof(int32_t));
int64_t prepare_layout(grmhd_block* h, int nblk, bool write) {
  int64_t wave[S_COUNT] = {0};
  for (int i = 0; i < nblk; ++i) {
    const Geo q = geo_of(h[i]);
    for (int c = 0; c < S_COUNT; ++c) {
      if (write) h[i].wave0[c] = (int32_t)wave[c];
      else if (h[i].wave0[c] != (int32_t)wave[c]) return -1;
      wave[c] += (shape_items(q, c) + 63) / 64;
      if (wave[c] > 0x3fffffff) return -1;
    }
    if (write) {
      for (int c = S_COUNT; c < kWaveSlots; ++c) h[i].wave0[c] = 0;
      h[i].nblk = nblk;
      h[i].reserved = 0;
    } else if (h[i].nblk != nblk) {
      return -1;
    }
  }
  return 0;
}


int last_err() { return hipGetLastError() == hipSuccess ? GRMHD_OK : GRMHD_EHIP; }

// grid of a grid-stride point kernel: enough workgroups to fill every CU at
// any occupancy (8 per CU), no more than the work needs
unsigned batch_grid(int64_t n) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t pr;
    cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&pr, dev) == hipSuccess)
              ? pr.multiProcessorCount
              : 256;
  }
  const int64_t tiles = (n + kThreads - 1) / kThreads;
  const int64_t g = (int64_t)cus * 8;
  return (unsigned)(tiles < g ? tiles : g);
}

// the steps; validation is done by the public entry points
// red, dt_out (device): the first stage of a step with device dt, whose CFL
// reduction rides on the field kernel; dt_out = cfl / max speed before the
// fluxes (the stage reads it from the FOFC trial state on)
// clear: a whole stage (the field kernel also clears the flags and the FOFC
// list; run_fofc is then told so)
void run_fluxes(const grmhd_block* h, const grmhd_block* d, int nblk, const grmhd_params& p,
                const Eos& e, hipStream_t s, double* red = nullptr, double cfl = 0.0,
                double* dt_out = nullptr, bool clear = false) {
  const dim3 gb = grid_cls(h, nblk, S_CELLS, tpb(T_BCC));
  if (red) {
    k_zero1<<<1, 64, 0, s>>>(red);
    TIMED(T_BCC, s);
    eos_dispatch(e.type, [&](auto et) {
      if (clear)
        k_bcc<decltype(et)::value, true, true><<<gb, tpb(T_BCC), 0, s>>>(d, e, red);
      else
        k_bcc<decltype(et)::value, true, false><<<gb, tpb(T_BCC), 0, s>>>(d, e, red);
    });
  } else {
    TIMED(T_BCC, s);
    if (clear)
      k_bcc<0, false, true><<<gb, tpb(T_BCC), 0, s>>>(d, e, nullptr);
    else
      k_bcc<0, false, false><<<gb, tpb(T_BCC), 0, s>>>(d, e, nullptr);
  }
  if (red) k_dt_final<<<1, 64, 0, s>>>(red, cfl, dt_out);
  {
    TIMED(T_FLUX_X, s);
    eos_dispatch(e.type, [&](auto et) {
      recon_dispatch(p.recon, [&](auto rc) {
        k_flux<0, decltype(et)::value, decltype(rc)::value>
            <<<grid_cls(h, nblk, S_XFACE + 0, tpb(T_FLUX_X)), tpb(T_FLUX_X), 0, s>>>(d, e, p);
      });
    });
  }
  {
    TIMED(T_FLUX_Y, s);
    eos_dispatch(e.type, [&](auto et) {
      recon_dispatch(p.recon, [&](auto rc) {
        k_flux<1, decltype(et)::value, decltype(rc)::value>
            <<<grid_cls(h, nblk, S_XFACE + 1, tpb(T_FLUX_Y)), tpb(T_FLUX_Y), 0, s>>>(d, e, p);
      });
    });
  }
  TIMED(T_FLUX_Z, s);
  eos_dispatch(e.type, [&](auto et) {
    recon_dispatch(p.recon, [&](auto rc) {
      k_flux<2, decltype(et)::value, decltype(rc)::value>
          <<<grid_cls(h, nblk, S_XFACE + 2, tpb(T_FLUX_Z)), tpb(T_FLUX_Z), 0, s>>>(d, e, p);
    });
  });
}

// links / links_h (device / host): a refined mesh, whose flag exchange
// crosses levels
// cleared: the flags and the FOFC list were cleared by the field kernel
void run_fofc(const grmhd_block* h, const grmhd_block* d, int nblk, const grmhd_params& p,
              const Eos& e, const double* dt_d, double dt, double a0, double a1, double b,
              hipStream_t s, const grmhd_amr_link* links = nullptr,
              const grmhd_amr_link* links_h = nullptr, bool cleared = false) {
  if (!cleared)
    k_clear_flags<<<grid_cls(h, nblk, S_CELLS, tpb(T_FOFC_FLAGS)), tpb(T_FOFC_FLAGS), 0, s>>>(d);
  if (!p.fofc) return;
  {
    TIMED(T_FOFC_FLAGS, s);
    eos_dispatch(e.type, [&](auto et) {
      k_fofc_flags<decltype(et)::value><<<grid_cls(h, nblk, S_INTERIOR, tpb(T_FOFC_FLAGS)), tpb(T_FOFC_FLAGS), 0, s>>>(d, e, p, dt_d, dt, a0, a1, b);
    });
  }
  bool exchange = false;
  for (int i = 0; i < nblk; ++i) exchange = exchange || h[i].bc == 1;
  if (links) {
    TIMED(T_GHOST, s);
    launch_ghost_cells_amr(h, d, nblk, links_h, links, 8, 1, -1, tpb(T_GHOST), s);
  } else if (exchange) {
    TIMED(T_GHOST, s);
    k_ghost_cells<<<grid_cls(h, nblk, S_GSHELL, tpb(T_GHOST)), tpb(T_GHOST), 0, s>>>(d, 8, 1);
  }
  TIMED(T_FOFC_FIX, s);
  const int chunks = nblk >= 4096 ? 1 : (4096 + nblk - 1) / nblk;
  eos_dispatch(e.type, [&](auto et) {
    k_fofc_fix<decltype(et)::value><<<(unsigned)(nblk * chunks), tpb(T_FOFC_FIX), 0, s>>>(d, e, p,
                                                                                        chunks);
  });
}

// links (device): a refined mesh, whose boundary EMFs next to finer leaves
// are corrected between the corner EMFs and the face update
void run_ct(const grmhd_block* h, const grmhd_block* d, int nblk, const double* dt_d, double dt,
            double a0, double a1, double b, hipStream_t s, const grmhd_amr_link* links = nullptr) {
  TIMED(T_CT, s);
  k_emf_corners<<<grid_cls(h, nblk, S_CORNER, tpb(T_CT)), tpb(T_CT), 0, s>>>(d);
  if (links) launch_amr_emf_fix(d, links, nblk, h[0].nx, s);
  k_ct_faces<<<grid_cls(h, nblk, S_CORNER, tpb(T_CT)), tpb(T_CT), 0, s>>>(d, dt_d, dt, a0, a1, b);
}

// every block kBrickW cells wide with ny a multiple of kBrickY and nz of
// kBrickZ (then every block's interior waves, and so every block's first
// wave, are multiples of the waves per workgroup, and the bricks tile the
// launch exactly)
bool brick_layout_fits(const grmhd_block* h, int nblk) {
  for (int i = 0; i < nblk; ++i)
    if (h[i].nx != kBrickW || h[i].ny % kBrickY != 0 || h[i].nz % kBrickZ != 0 || h[i].ny < 1 ||
        h[i].ng < 2)
      return false;
  return true;
}

// a6 alone (c2p false) or a6 + a8 in one pass (c2p true: the stage's
// inversion fused into the update, timed as the update family)
void run_update(const grmhd_block* h, const grmhd_block* d, int nblk, const Eos& e,
                const grmhd_params& p, const double* dt_d, double dt, double a0, double a1,
                double b, hipStream_t s, bool c2p = false) {
  TIMED(T_UPDATE, s);
  const bool brick = tpb(T_UPDATE) == kMaxThreads && brick_layout_fits(h, nblk);
  auto go = [&](auto et, auto fused) {
    constexpr int ET = decltype(et)::value;
    constexpr bool F = decltype(fused)::value;
    if (brick) {
      const int64_t waves = (int64_t)h[nblk - 1].wave0[S_INTERIOR] +
                            shape_items(geo_of(h[nblk - 1]), S_INTERIOR) / 64;
      k_update<ET, true, F><<<(unsigned)(waves / (kMaxThreads / 64)), kMaxThreads, 0, s>>>(
          d, e, dt_d, dt, a0, a1, b, p);
    } else {
      k_update<ET, false, F><<<grid_cls(h, nblk, S_INTERIOR, tpb(T_UPDATE)), tpb(T_UPDATE), 0, s>>>(
          d, e, dt_d, dt, a0, a1, b, p);
    }
  };
  eos_dispatch(e.type, [&](auto et) {
    if (c2p) go(et, std::true_type{});
    else go(et, std::false_type{});
  });
}

void run_c2p(const grmhd_block* h, const grmhd_block* d, int nblk, const grmhd_params& p,
             const Eos& e, hipStream_t s, c2p_stats* stats = nullptr) {
  TIMED(T_C2P, s);
  eos_dispatch(e.type, [&](auto et) {
    k_stage_c2p<decltype(et)::value><<<grid_cls(h, nblk, S_INTERIOR, tpb(T_C2P)), tpb(T_C2P), 0, s>>>(
        d, e, p, stats);
  });
  if (stats) k_stats_sum<<<nblk, kThreads, 0, s>>>(d, stats);
}

// plain streaming copy (counter calibration)
__global__ __launch_bounds__(kThreads) void k_copy(const double* __restrict__ a, double* __restrict__ b,
                                                   int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    b[t] = a[t];
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free baryon-mass sum (grmhd_mass_noalloc): the per-block partial
// sums live in this file-scope device array instead of a caller workspace.
// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is taken once per device with hipGetSymbolAddress and
// only that address is passed to kernels.
// ---------------------------------------------------------------------------
constexpr int kMassNoAllocBlocks = 65536;   // 512 KiB of partial sums
static __device__ __align__(256) double scratch[kMassNoAllocBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call per device, with that device current)
int scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GRMHD_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GRMHD_EHIP;
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return GRMHD_OK;
}
}  // namespace

namespace gk {
Timing g_tm;
// plain or bracketed inversion of n states (pointer arrays already checked)
void launch_c2p_batch(int64_t n, double* const* u, double* const* bt, double* const* gam, double* const* w,
                      uint16_t* flags, const grmhd_params& p, const double* blo, const double* bhi,
                      double* mu_out, int32_t* nev_out, c2p_stats* stats, hipStream_t s) {
  Ptrs5 pw, pu;
  Ptrs3 pb;
  Ptrs6 pg;
  for (int v = 0; v < 5; ++v) { pw.p[v] = w[v]; pu.p[v] = u[v]; }
  for (int v = 0; v < 3; ++v) pb.p[v] = bt[v];
  for (int v = 0; v < 6; ++v) pg.p[v] = gam[v];
  TIMED(blo ? T_C2P_LEARNED : T_C2P_BATCH, s);
  const Eos e = make_eos(p);
  eos_dispatch(e.type, [&](auto et) {
    k_c2p_batch<decltype(et)::value><<<batch_grid(n), kThreads, 0, s>>>(
        n, pu, pb, pg, pw, flags, e, p, blo, bhi, mu_out, nev_out, stats);
  });
}
Eos make_eos_host(const grmhd_params& p) { return make_eos(p); }
unsigned stage_grid(const grmhd_block* h, int nblk, int cls, int threads) {
  return grid_cls(h, nblk, cls, threads).x;
}
void launch_stats_sum(const grmhd_block* d, int nblk, c2p_stats* stats, hipStream_t s) {
  k_stats_sum<<<nblk, kThreads, 0, s>>>(d, stats);
}
int launch_stage_c2p_learned(const grmhd_block* h, const grmhd_block* d, int nblk,
                             const grmhd_params& p, const c2p_mlp* mlp, c2p_stats* stats,
                             hipStream_t s);
int check_params_host(const grmhd_params* p) { return check_params(p); }
}  // namespace gk

extern "C" int c2p_batch_learned(int64_t n, double* u[5], double* const bt[3], double* const gam[6],
                                 double* w[5], uint16_t* flags, const grmhd_params* p,
                                 const c2p_mlp* mlp, c2p_stats* stats, double* mu_out,
                                 int32_t* nev_out, void* stream);

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int grmhd_blocks_prepare(grmhd_block* blk_h, int32_t nblk) {
  if (!blk_h || nblk < 1) return GRMHD_EINVAL;
  for (int i = 0; i < nblk; ++i)
    if (blk_h[i].nx < 1 || blk_h[i].ny < 1 || blk_h[i].nz < 1 || blk_h[i].ng < 0) return GRMHD_EINVAL;
  return prepare_layout(blk_h, nblk, true) == 0 ? GRMHD_OK : GRMHD_EINVAL;
}

int64_t grmhd_scratch_doubles(int32_t nx, int32_t ny, int32_t nz, int32_t ng) {
  if (nx < 1 || ny < 1 || nz < 1 || ng < 0) return -1;
  Geo q;
  q.nx = nx; q.ny = ny; q.nz = nz; q.g = ng;
  q.sx = nx + 2 * ng; q.sy = ny + 2 * ng; q.sz = nz + 2 * ng;
  return scratch_total(q);
}

int64_t grmhd_flux_offset(int32_t nx, int32_t ny, int32_t nz, int32_t ng, int32_t d, int32_t c) {
  if (nx < 1 || ny < 1 || nz < 1 || ng < 0 || d < 0 || d > 2 || c < 0 || c > 6) return -1;
  Geo q;
  q.nx = nx; q.ny = ny; q.nz = nz; q.g = ng;
  q.sx = nx + 2 * ng; q.sy = ny + 2 * ng; q.sz = nz + 2 * ng;
  return off_flux(q, d, c);
}

int grmhd_fluxes(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                 const grmhd_params* p, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  run_fluxes(blk_h, blk_d, nblk, *p, make_eos(*p), (hipStream_t)stream);
  return last_err();
}

int fofc_correct(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                 const grmhd_params* p, const double* dt_d, double dt, double a0, double a1,
                 double b, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  run_fofc(blk_h, blk_d, nblk, *p, make_eos(*p), dt_d, dt, a0, a1, b, (hipStream_t)stream);
  return last_err();
}

int ct_update(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
              const grmhd_params* p, const double* dt_d, double dt, double a0, double a1, double b,
              void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  run_ct(blk_h, blk_d, nblk, dt_d, dt, a0, a1, b, (hipStream_t)stream);
  return last_err();
}

int grmhd_update(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                 const grmhd_params* p, const double* dt_d, double dt, double a0, double a1,
                 double b, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  run_update(blk_h, blk_d, nblk, make_eos(*p), *p, dt_d, dt, a0, a1, b, (hipStream_t)stream);
  return last_err();
}

int grmhd_stage_c2p(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                    const grmhd_params* p, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  run_c2p(blk_h, blk_d, nblk, *p, make_eos(*p), (hipStream_t)stream);
  return last_err();
}

int grmhd_matter_sources(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                         const grmhd_params* p, double* const* out_d, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if (!out_d) return GRMHD_EINVAL;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  const Eos e = make_eos(*p);
  hipStream_t s = (hipStream_t)stream;
  TIMED(T_MATTER, s);
  eos_dispatch(e.type, [&](auto et) {
    k_matter<decltype(et)::value>
        <<<grid_cls(blk_h, nblk, S_INTERIOR, tpb(T_MATTER)), tpb(T_MATTER), 0, s>>>(blk_d, e, out_d);
  });
  return last_err();
}

int grmhd_excise(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                 const grmhd_params* p, double alpha_min, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  if (!(alpha_min > 0.0)) return GRMHD_OK;
  const Eos e = make_eos(*p);
  hipStream_t s = (hipStream_t)stream;
  TIMED(T_EXCISE, s);
  eos_dispatch(e.type, [&](auto et) {
    k_excise<decltype(et)::value>
        <<<grid_cls(blk_h, nblk, S_INTERIOR, tpb(T_EXCISE)), tpb(T_EXCISE), 0, s>>>(blk_d, e, *p,
                                                                                    alpha_min);
  });
  return last_err();
}

int grmhd_stage(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                const grmhd_params* p, const double* dt_d, double dt, double a0, double a1,
                double b, void* stream) {
  return grmhd_stage_learned(blk_h, blk_d, nblk, p, dt_d, dt, a0, a1, b, nullptr, nullptr, stream);
}

int grmhd_stage_cfl(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                    const grmhd_params* p, double cfl, double* red, double* dt_out, double a0,
                    double a1, double b, void* stream) {
  if (!red || !dt_out || !(cfl > 0.0)) return GRMHD_EINVAL;
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  const Eos e = make_eos(*p);
  hipStream_t s = (hipStream_t)stream;
  run_fluxes(blk_h, blk_d, nblk, *p, e, s, red, cfl, dt_out, true);
  run_fofc(blk_h, blk_d, nblk, *p, e, dt_out, 0.0, a0, a1, b, s, nullptr, nullptr, true);
  run_ct(blk_h, blk_d, nblk, dt_out, 0.0, a0, a1, b, s);
  run_update(blk_h, blk_d, nblk, e, *p, dt_out, 0.0, a0, a1, b, s, true);
  return last_err();
}

int grmhd_stage_learned(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                        const grmhd_params* p, const double* dt_d, double dt, double a0,
                        double a1, double b, const c2p_mlp* mlp, c2p_stats* stats, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  if (mlp && (!mlp->w_bf16 || !mlp->w_f32)) return GRMHD_EINVAL;
  const Eos e = make_eos(*p);
  hipStream_t s = (hipStream_t)stream;
  run_fluxes(blk_h, blk_d, nblk, *p, e, s, nullptr, 0.0, nullptr, true);
  run_fofc(blk_h, blk_d, nblk, *p, e, dt_d, dt, a0, a1, b, s, nullptr, nullptr, true);
  run_ct(blk_h, blk_d, nblk, dt_d, dt, a0, a1, b, s);
  if (mlp) {
    run_update(blk_h, blk_d, nblk, e, *p, dt_d, dt, a0, a1, b, s);
    if ((r = launch_stage_c2p_learned(blk_h, blk_d, nblk, *p, mlp, stats, s))) return r;
  } else if (stats) {
    // inversion statistics are summed per wave by the inversion kernel
    run_update(blk_h, blk_d, nblk, e, *p, dt_d, dt, a0, a1, b, s);
    run_c2p(blk_h, blk_d, nblk, *p, e, s, stats);
  } else {
    run_update(blk_h, blk_d, nblk, e, *p, dt_d, dt, a0, a1, b, s, true);
  }
  return last_err();
}

int grmhd_stage_c2p_learned(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                            const grmhd_params* p, const c2p_mlp* mlp, c2p_stats* stats,
                            void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  if (!mlp) return GRMHD_EINVAL;
  if ((r = launch_stage_c2p_learned(blk_h, blk_d, nblk, *p, mlp, stats, (hipStream_t)stream)))
    return r;
  return last_err();
}

int grmhd_ghost_fill(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                     int32_t mask, void* stream) {
  if (!blk_h || !blk_d || nblk < 1 || (mask & ~15)) return GRMHD_EINVAL;
  if (prepare_layout(const_cast<grmhd_block*>(blk_h), nblk, false) != 0) return GRMHD_EINVAL;
  bool any = false;
  for (int i = 0; i < nblk; ++i) {
    const grmhd_block& b = blk_h[i];
    if (b.ng < 1 || b.nx < 1 || b.ny < 1 || b.nz < 1) return GRMHD_EINVAL;
    if (b.bc != 1) continue;
    any = true;
    if (((mask & 1) && !b.w[4]) || ((mask & 2) && !b.us[4]) || ((mask & 4) && !b.bs[2]) ||
        ((mask & 8) && !b.flags))
      return GRMHD_EINVAL;
    for (int v = 0; v < 27; ++v) {
      const int nb = b.nbr[v];
      if (nb < -1 || nb >= nblk) return GRMHD_EINVAL;
      if (nb < 0 || nb == i) continue;
      const grmhd_block& o = blk_h[nb];
      if (o.nx != b.nx || o.ny != b.ny || o.nz != b.nz || o.ng != b.ng) return GRMHD_EINVAL;
      if (b.nx < b.ng || b.ny < b.ng || b.nz < b.ng) return GRMHD_EINVAL;
    }
  }
  if (!any) return GRMHD_OK;   // every block's ghosts are frozen: nothing to launch
  hipStream_t s = (hipStream_t)stream;
  TIMED(T_GHOST, s);
  if (mask & 11) k_ghost_cells<<<grid_cls(blk_h, nblk, S_GCELLS, tpb(T_GHOST)), tpb(T_GHOST), 0, s>>>(blk_d, mask & 11, 0);
  if (mask & 4) {
    for (int d = 0; d < 3; ++d) k_ghost_faces<<<grid_cls(blk_h, nblk, S_GXFACE + d, tpb(T_GHOST)), tpb(T_GHOST), 0, s>>>(blk_d, d);
  }
  return last_err();
}

int grmhd_ghost_fill_amr(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                         const grmhd_amr_link* links_h, const grmhd_amr_link* links_d,
                         int32_t mask, void* stream) {
  if (!blk_h || !blk_d || !links_d || nblk < 1 || (mask & ~15)) return GRMHD_EINVAL;
  if (prepare_layout(const_cast<grmhd_block*>(blk_h), nblk, false) != 0) return GRMHD_EINVAL;
  int r = amr_check(blk_h, links_h, nblk);
  if (r) return r;
  for (int i = 0; i < nblk; ++i) {
    const grmhd_block& b = blk_h[i];
    if (((mask & 1) && !b.w[4]) || ((mask & 2) && !b.us[4]) || ((mask & 4) && !b.bs[2]) ||
        ((mask & 8) && !b.flags))
      return GRMHD_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  TIMED(T_GHOST, s);
  const int top = amr_max_level(links_h, nblk);
  // copies and restrictions (pass 0), then the prolongations level by level
  for (int pass = 0; pass <= top; ++pass) {
    if (mask & 11)
      launch_ghost_cells_amr(blk_h, blk_d, nblk, links_h, links_d, mask & 11, 0, pass, tpb(T_GHOST), s);
    if (mask & 4)
      for (int d = 0; d < 3; ++d)
        launch_ghost_faces_amr(blk_h, blk_d, nblk, links_h, links_d, d, pass, tpb(T_GHOST), s);
  }
  return last_err();
}

int grmhd_stage_amr(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                    const grmhd_amr_link* links_h, const grmhd_amr_link* links_d,
                    const grmhd_params* p, const double* dt_d, double dt, double a0, double a1,
                    double b, const c2p_mlp* mlp, c2p_stats* stats, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(blk_h, blk_d, nblk))) return r;
  if (!links_d) return GRMHD_EINVAL;
  if ((r = amr_check(blk_h, links_h, nblk))) return r;
  if (mlp && (!mlp->w_bf16 || !mlp->w_f32)) return GRMHD_EINVAL;
  const Eos e = make_eos(*p);
  hipStream_t s = (hipStream_t)stream;
  run_fluxes(blk_h, blk_d, nblk, *p, e, s, nullptr, 0.0, nullptr, true);
  run_fofc(blk_h, blk_d, nblk, *p, e, dt_d, dt, a0, a1, b, s, links_d, links_h, true);
  launch_amr_flux_fix(blk_d, links_d, nblk, blk_h[0].nx, s);
  run_ct(blk_h, blk_d, nblk, dt_d, dt, a0, a1, b, s, links_d);
  if (mlp) {
    run_update(blk_h, blk_d, nblk, e, *p, dt_d, dt, a0, a1, b, s);
    if ((r = launch_stage_c2p_learned(blk_h, blk_d, nblk, *p, mlp, stats, s))) return r;
  } else if (stats) {
    run_update(blk_h, blk_d, nblk, e, *p, dt_d, dt, a0, a1, b, s);
    run_c2p(blk_h, blk_d, nblk, *p, e, s, stats);
  } else {
    run_update(blk_h, blk_d, nblk, e, *p, dt_d, dt, a0, a1, b, s, true);
  }
  return last_err();
}

int grmhd_dt(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
             const grmhd_params* p, double cfl, double* red, double* dt_out, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if (!red || !dt_out || !(cfl > 0.0)) return GRMHD_EINVAL;
  if ((r = check_reads(blk_h, blk_d, nblk, NEED_W | NEED_BS | NEED_ADM))) return r;
  hipStream_t s = (hipStream_t)stream;
  k_zero1<<<1, 64, 0, s>>>(red);
  {
    TIMED(T_DT, s);
    const Eos e = make_eos(*p);
    eos_dispatch(e.type, [&](auto et) {
      k_dt<decltype(et)::value><<<grid_cls(blk_h, nblk, S_INTERIOR, tpb(T_DT)), tpb(T_DT), 0, s>>>(blk_d, e, red);
    });
  }
  k_dt_final<<<1, 64, 0, s>>>(red, cfl, dt_out);
  return last_err();
}

int grmhd_mass(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk, double* partial,
               double* out, void* stream) {
  if (!partial || !out) return GRMHD_EINVAL;
  int r = check_reads(blk_h, blk_d, nblk, NEED_D);
  if (r) return r;
  hipStream_t s = (hipStream_t)stream;
  k_mass_block<<<nblk, kThreads, 0, s>>>(blk_d, partial);
  k_mass_final<<<1, 64, 0, s>>>(partial, nblk, out);
  return last_err();
}

int grmhd_mass_noalloc(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                       double* out, void* stream) {
  if (!out) return GRMHD_EINVAL;
  if (nblk > kMassNoAllocBlocks) return GRMHD_ETOOBIG;
  int r = check_reads(blk_h, blk_d, nblk, NEED_D);
  if (r) return r;
  double* part = nullptr;
  if ((r = scratch_address(&part))) return r;
  hipStream_t s = (hipStream_t)stream;
  // every partial[0..nblk) is written by k_mass_block before k_mass_final
  // reads it (stream order): nothing to clear
  k_mass_block<<<nblk, kThreads, 0, s>>>(blk_d, part);
  k_mass_final<<<1, 64, 0, s>>>(part, nblk, out);
  return last_err();
}

int32_t grmhd_mass_noalloc_max_blocks(void) { return kMassNoAllocBlocks; }

int prim2con(int64_t n, double* const w[5], double* const bt[3], double* const gam[6], double* u[5],
             const grmhd_params* p, void* stream) {
  int r = check_params(p);
  if (r) return r;
  // an empty batch is valid whatever its (possibly NULL) pointers
  if (n < 0) return GRMHD_EINVAL;
  if (n == 0) return GRMHD_OK;
  if (!w || !bt || !gam || !u) return GRMHD_EINVAL;
  Ptrs5 pw, pu;
  Ptrs3 pb;
  Ptrs6 pg;
  for (int v = 0; v < 5; ++v) { pw.p[v] = w[v]; pu.p[v] = u[v]; if (!w[v] || !u[v]) return GRMHD_EINVAL; }
  for (int v = 0; v < 3; ++v) { pb.p[v] = bt[v]; if (!bt[v]) return GRMHD_EINVAL; }
  for (int v = 0; v < 6; ++v) { pg.p[v] = gam[v]; if (!gam[v]) return GRMHD_EINVAL; }
  const Eos e = make_eos(*p);
  eos_dispatch(e.type, [&](auto et) {
    k_prim2con<decltype(et)::value><<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0,
                                      (hipStream_t)stream>>>(n, pw, pb, pg, pu, e);
  });
  return last_err();
}

int c2p_batch(int64_t n, double* u[5], double* const bt[3], double* const gam[6], double* w[5],
              uint16_t* flags, const grmhd_params* p, const c2p_mlp* mlp, c2p_stats* stats,
              double* mu_out, int32_t* nev_out, void* stream) {
  int r = check_params(p);
  if (r) return r;
  // an empty batch is valid whatever its (possibly NULL) pointers
  if (n < 0) return GRMHD_EINVAL;
  if (n == 0) return GRMHD_OK;
  if (!u || !bt || !gam || !w || !flags) return GRMHD_EINVAL;
  if (mlp) return c2p_batch_learned(n, u, bt, gam, w, flags, p, mlp, stats, mu_out, nev_out, stream);
  for (int v = 0; v < 5; ++v) if (!w[v] || !u[v]) return GRMHD_EINVAL;
  for (int v = 0; v < 3; ++v) if (!bt[v]) return GRMHD_EINVAL;
  for (int v = 0; v < 6; ++v) if (!gam[v]) return GRMHD_EINVAL;
  launch_c2p_batch(n, u, bt, gam, w, flags, *p, nullptr, nullptr, mu_out, nev_out, stats,
                   (hipStream_t)stream);
  return last_err();
}

int grmhd_prim2con_blocks(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                          const grmhd_params* p, void* stream) {
  int r = check_params(p);
  if (r) return r;
  if ((r = check_reads(blk_h, blk_d, nblk, NEED_W | NEED_BS | NEED_ADM | NEED_US))) return r;
  const Eos e = make_eos(*p);
  eos_dispatch(e.type, [&](auto et) {
    k_p2c_block<decltype(et)::value><<<grid_cls(blk_h, nblk, S_CELLS, tpb(T_BCC)), tpb(T_BCC), 0,
                                       (hipStream_t)stream>>>(blk_d, e);
  });
  return last_err();
}

const char* grmhd_version(void) { return "grmhd 0.2 gfx950 fp64"; }

int32_t grmhd_launch_shapes(void) { return (int32_t)S_COUNT; }

int grmhd_timing(int32_t on) {
  if (on) {
    if (!g_tm.created) {
      for (int x = 0; x < kEventPool; ++x)
        if (hipEventCreate(&g_tm.ev[x]) != hipSuccess) return GRMHD_EHIP;
      g_tm.created = 1;
    }
    g_tm.used = 0;
    for (int f = 0; f < kFamilies; ++f) { g_tm.ms[f] = 0.0; g_tm.cnt[f] = 0; }
  }
  g_tm.on = on ? 1 : 0;
  return GRMHD_OK;
}

int grmhd_timing_read(int32_t family, double* ms, int64_t* launches) {
  if (family < 0 || family >= kFamilies || !ms || !launches) return GRMHD_EINVAL;
  for (int x = 0; x < g_tm.used; x += 2) {
    if (hipEventSynchronize(g_tm.ev[x + 1]) != hipSuccess) return GRMHD_EHIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_tm.ev[x], g_tm.ev[x + 1]) != hipSuccess) return GRMHD_EHIP;
    g_tm.ms[g_tm.fam[x / 2]] += t;
    g_tm.cnt[g_tm.fam[x / 2]] += 1;
  }
  g_tm.used = 0;
  *ms = g_tm.ms[family];
  *launches = g_tm.cnt[family];
  return GRMHD_OK;
}

int grmhd_copy(const double* src, double* dst, int64_t n, void* stream) {
  if (n < 0) return GRMHD_EINVAL;
  if (n == 0) return GRMHD_OK;
  if (!src || !dst) return GRMHD_EINVAL;
  k_copy<<<4096, kThreads, 0, (hipStream_t)stream>>>(src, dst, n);
  return last_err();
}

int grmhd_c2p_pairs(const grmhd_block* blk_h, const grmhd_block* blk_d, int32_t nblk,
                    int32_t stride, const int64_t* base, double* const u[5], double* const bt[3],
                    double* const gam[6], double* const w[5], void* stream) {
  if (stride < 1 || !base || !u || !bt || !gam || !w) return GRMHD_EINVAL;
  int r = check_reads(blk_h, blk_d, nblk, NEED_W | NEED_BS | NEED_ADM | NEED_US);
  if (r) return r;
  Ptrs5 pu, pw;
  Ptrs3 pb;
  Ptrs6 pg;
  for (int v = 0; v < 5; ++v) {
    if (!u[v] || !w[v]) return GRMHD_EINVAL;
    pu.p[v] = u[v];
    pw.p[v] = w[v];
  }
  for (int v = 0; v < 3; ++v) {
    if (!bt[v]) return GRMHD_EINVAL;
    pb.p[v] = bt[v];
  }
  for (int v = 0; v < 6; ++v) {
    if (!gam[v]) return GRMHD_EINVAL;
    pg.p[v] = gam[v];
  }
  k_c2p_pairs<<<grid_cls(blk_h, nblk, S_INTERIOR, kThreads), kThreads, 0, (hipStream_t)stream>>>(
      blk_d, stride, base, pu, pb, pg, pw);
  return last_err();
}

int grmhd_rk2_step(const grmhd_rk2_tables* t, int32_t nblk, const grmhd_params* p, double cfl,
                   double* red, double* dt_out, void* stream) {
  if (!t) return GRMHD_EINVAL;
  int r;
  // the CFL dt of set A, reduced in the first stage's field kernel
  if ((r = grmhd_stage_cfl(t->ab_h, t->ab_d, nblk, p, cfl, red, dt_out, 0.0, 1.0, 1.0, stream)))
    return r;
  if ((r = grmhd_ghost_fill(t->b_h, t->b_d, nblk, 7, stream))) return r;
  if ((r = grmhd_stage(t->ba_h, t->ba_d, nblk, p, dt_out, 0.0, 0.5, 0.5, 0.5, stream))) return r;
  return grmhd_ghost_fill(t->a_h, t->a_d, nblk, 7, stream);
}

struct grmhd_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int grmhd_graph_build(const grmhd_rk2_tables* t, int32_t nblk, const grmhd_params* p, double cfl,
                      double* red, double* dt_out, void* stream, grmhd_graph** out) {
  if (!t || !out || !stream || g_tm.on) return GRMHD_EINVAL;
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return GRMHD_EHIP;
  const int r = grmhd_rk2_step(t, nblk, p, cfl, red, dt_out, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (r || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return r ? r : GRMHD_EHIP;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return GRMHD_EHIP;
  }
  *out = new grmhd_graph{g, x};
  return GRMHD_OK;
}

int grmhd_graph_launch(grmhd_graph* g, void* stream) {
  if (!g) return GRMHD_EINVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? GRMHD_OK : GRMHD_EHIP;
}

int grmhd_graph_destroy(grmhd_graph* g) {
  if (!g) return GRMHD_EINVAL;
  const bool ok = hipGraphExecDestroy(g->exec) == hipSuccess && hipGraphDestroy(g->graph) == hipSuccess;
  delete g;
  return ok ? GRMHD_OK : GRMHD_EHIP;
}

int grmhd_autotune(const grmhd_block* ab_h, const grmhd_block* ab_d, int32_t nblk,
                   const grmhd_params* p, double dt, int32_t reps, int32_t* threads_out,
                   double* ms_out, void* stream) {
  constexpr int kTuned = 8;            // families 0..7: T_FLUX_X .. T_C2P
  constexpr int kSizes[4] = {64, 128, 256, 512};
  if (!threads_out || reps < 1 || !(dt > 0.0)) return GRMHD_EINVAL;
  int r = check_params(p);
  if (r) return r;
  if ((r = check_blocks(ab_h, ab_d, nblk))) return r;
  hipStream_t s = (hipStream_t)stream;
  for (int fam = 0; fam < kTuned; ++fam) {
    double best = 0.0;
    int best_th = g_threads[fam];
    bool launched = false;
    for (int c = 0; c < 4; ++c) {
      g_threads[fam] = kSizes[c];
      // warm launch outside the timed region, then reps timed stages
      if ((r = grmhd_stage_learned(ab_h, ab_d, nblk, p, nullptr, dt, 0.0, 1.0, 1.0, nullptr, nullptr,
                                   stream)))
        break;
      if ((r = grmhd_timing(1))) break;
      for (int k = 0; k < reps && !r; ++k)
        r = grmhd_stage_learned(ab_h, ab_d, nblk, p, nullptr, dt, 0.0, 1.0, 1.0, nullptr, nullptr,
                                stream);
      double ms = 0.0;
      int64_t n = 0;
      if (!r) r = grmhd_timing_read(fam, &ms, &n);
      (void)grmhd_timing(0);
      if (r) break;
      // a family the stage does not launch (the separate inversion when it
      // is fused into the update) keeps its size
      const double per = n > 0 ? ms / (double)n : 0.0;
      if (ms_out) ms_out[fam * 4 + c] = per;
      if (n > 0 && (!launched || per < best)) {
        best = per;
        best_th = kSizes[c];
        launched = true;
      }
    }
    if (!launched) best_th = 256;
    g_threads[fam] = best_th;
    threads_out[fam] = best_th;
    if (r) return r;
  }
  return hipStreamSynchronize(s) == hipSuccess ? GRMHD_OK : GRMHD_EHIP;
}

int grmhd_set_threads(int32_t family, int32_t threads) {
  if (family < 0 || family >= kFamilies) return GRMHD_EINVAL;
  if (threads < 64 || threads > kMaxThreads || (threads % 64)) return GRMHD_EINVAL;
  g_threads[family] = threads;
  return GRMHD_OK;
}

int32_t grmhd_struct_size(int32_t which) {
  switch (which) {
    case 0: return (int32_t)sizeof(grmhd_params);
    case 1: return (int32_t)sizeof(grmhd_block);
    case 2: return (int32_t)sizeof(c2p_mlp);
    case 3: return (int32_t)sizeof(c2p_stats);
    default: return -1;
  }
}

}  // extern "C"
