// amr.hip -- the inter-level transfer of block-based mesh refinement (Sec. I;
// prolongation and restriction, Sec. V-A): the host-side links of a leaf
// mesh, the ghost fill across levels, and the flux and EMF corrections at
// level boundaries of a stage.  The rules are stated in include/grmhd.h.
//
// Every kernel item finds its source leaf from its block's link: the item's
// neighbour region (after outflow clamping) names at most 4 candidate leaves
// of one level, and the item takes the candidate whose range holds it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "blocks.hpp"
#include "grmhd.h"
#include "timing.hpp"

using namespace gk;

namespace {

constexpr int kAmrThreads = 256;
constexpr int kMaxThreads = 512;   // ghost kernels run with the ghost family's workgroup size

__device__ __forceinline__ int dir_of(const int o[3]) {
  return (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1);
}

// the candidate leaf of region dir of link lk that holds global cell I (of
// lk's level; for a finer region its child 2I), -1 if none
__device__ __forceinline__ int amr_pick(const grmhd_amr_link* __restrict__ L,
                                        const grmhd_amr_link& lk, int dir, const int I[3],
                                        int nb) {
  const int rel = lk.rel[dir];
  if (rel < -1 || rel > 1) return -1;
  if (rel == -1) return lk.src[dir][0];   // one coarser leaf covers the region
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int s = lk.src[dir][c];
    if (s < 0) return -1;
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int J = rel == 1 ? 2 * I[a] : I[a];
      in = in && J >= L[s].org[a] && J < L[s].org[a] + nb;
    }
    if (in) return s;
  }
  return -1;
}

// global cell index at lk's level of padded cell position x along axis a,
// with its region offset o; outflow positions beyond the domain are clamped
// to its last cell (o = 0 then: the block touches that boundary)
__device__ __forceinline__ void amr_axis(const grmhd_amr_link& lk, const Geo& q, int a, int x,
                                         int& I, int& o) {
  const int n = a == 0 ? q.nx : (a == 1 ? q.ny : q.nz);
  int G = lk.org[a] + x - q.g;
  o = x < q.g ? -1 : (x >= q.g + n ? 1 : 0);
  const int N = lk.N[a];
  if (G < 0 || G >= N) {
    if ((lk.periodic >> a) & 1) {
      G = G < 0 ? G + N : G - N;
    } else {
      G = G < 0 ? 0 : N - 1;
      o = 0;
    }
  }
  I = G;
}

// block and item of this thread for launch shape cls over the blocks
// b0..b1 of the list (a contiguous range: the leaves of one level), as
// locate() does over the whole list
__device__ __forceinline__ bool locate_range(const grmhd_block* __restrict__ blks, int cls, int b0,
                                             int b1, int& bi, int64_t& t) {
  const int64_t g = (int64_t)xcd_linear() * blockDim.x + threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane((int)(g >> 6)) + blks[b0].wave0[cls];
  int lo = b0, hi = b1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blks[mid].wave0[cls] <= w) lo = mid; else hi = mid - 1;
  }
  bi = lo;
  const Geo q = geo_of(blks[bi]);
  if (bi == b1 && w >= blks[b1].wave0[cls] + (int)((shape_items(q, cls) + 63) >> 6)) return false;
  t = (int64_t)(w - blks[bi].wave0[cls]) * 64 + (threadIdx.x & 63);
  return t < shape_items(q, cls);
}

__device__ __forceinline__ double minmod2(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

// padded cell index in leaf s (geometry q) of global cell J of its level
__device__ __forceinline__ int64_t leaf_cell(const grmhd_amr_link& ls, const Geo& q,
                                             const int J[3]) {
  return cell(q, J[0] - ls.org[0] + q.g, J[1] - ls.org[1] + q.g, J[2] - ls.org[2] + q.g);
}

// prolongation of padded cell array f of leaf s to its child I (one level finer)
__device__ __forceinline__ double prolong(const grmhd_amr_link& ls, const Geo& q,
                                          gptr<const double> f, const int I[3]) {
  const int P[3] = {I[0] >> 1, I[1] >> 1, I[2] >> 1};
  const int64_t c = leaf_cell(ls, q, P);
  const double v = f[c];
  const int64_t st[3] = {1, (int64_t)q.sx, (int64_t)q.sx * q.sy};
  double out = v;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double s = minmod2(f[c + st[a]] - v, v - f[c - st[a]]);
    out += (I[a] & 1) ? 0.25 * s : -0.25 * s;
  }
  return out;
}

// Ghost cells of the w (mask 1), us (2) and flags (8) slots over launch
// shape S_GCELLS, or (list != 0: the flag exchange of a stage) the flags of
// the first ghost shell S_GSHELL, whose flagged cells join the block's FOFC
// list.  pass 0: copies and restrictions; pass p > 0: the prolongations of
// the blocks at level p; pass -1: all (flags only: a prolonged flag is the
// parent's, which is an interior cell).
__global__ __launch_bounds__(kMaxThreads) void k_ghost_cells_amr(
    const grmhd_block* __restrict__ blks, const grmhd_amr_link* __restrict__ L, int mask, int list,
    int pass, int b0, int b1) {
  int ib;
  int64_t t;
  const int cls = list ? S_GSHELL : S_GCELLS;
  if (!locate_range(blks, cls, b0, b1, ib, t)) return;
  const grmhd_amr_link& lk = L[ib];
  if (pass > 0 && lk.level != pass) return;
  const GB b = gview(blks[ib]);
  const Geo q = geo_of(b);
  int x[3];
  ghost_ring(q, cls).at(t, x[0], x[1], x[2]);
  if (list) {
    x[0] += q.g - 1; x[1] += q.g - 1; x[2] += q.g - 1;
  }
  const int64_t c = cell(q, x[0], x[1], x[2]);
  int I[3], o[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) amr_axis(lk, q, a, x[a], I[a], o[a]);
  const int dir = dir_of(o);
  const int rel = lk.rel[dir];
  const int s = amr_pick(L, lk, dir, I, q.nx);
  bool take = false;
  if (s >= 0 && (pass < 0 || (pass == 0 && rel >= 0) || (pass > 0 && rel == -1))) {
    const GB src = gview(blks[s]);
    const Geo qs = geo_of(src);
    const grmhd_amr_link& ls = L[s];
    uint16_t f = 0;
    if (rel == 0) {
      const int64_t sc = leaf_cell(ls, qs, I);
      if (mask & 1)
#pragma unroll
        for (int v = 0; v < 5; ++v) b.w[v][c] = src.w[v][sc];
      if (mask & 2)
#pragma unroll
        for (int v = 0; v < 5; ++v) b.us[v][c] = src.us[v][sc];
      f = src.flags[sc];
    } else if (rel == 1) {
      // the 8 children, x fastest
      const int C0[3] = {2 * I[0], 2 * I[1], 2 * I[2]};
      const int64_t c0 = leaf_cell(ls, qs, C0);
      const int64_t st[3] = {1, (int64_t)qs.sx, (int64_t)qs.sx * qs.sy};
      if (mask & 1)
        for (int v = 0; v < 5; ++v) {
          double sum = 0.0;
#pragma unroll
          for (int k8 = 0; k8 < 8; ++k8)
            sum += src.w[v][c0 + (k8 & 1) * st[0] + ((k8 >> 1) & 1) * st[1] + (k8 >> 2) * st[2]];
          b.w[v][c] = 0.125 * sum;
        }
      if (mask & 2)
        for (int v = 0; v < 5; ++v) {
          double sum = 0.0;
#pragma unroll
          for (int k8 = 0; k8 < 8; ++k8)
            sum += src.us[v][c0 + (k8 & 1) * st[0] + ((k8 >> 1) & 1) * st[1] + (k8 >> 2) * st[2]];
          b.us[v][c] = 0.125 * sum;
        }
#pragma unroll
      for (int k8 = 0; k8 < 8; ++k8)
        f |= src.flags[c0 + (k8 & 1) * st[0] + ((k8 >> 1) & 1) * st[1] + (k8 >> 2) * st[2]];
    } else {
      if (mask & 1)
        for (int v = 0; v < 5; ++v) b.w[v][c] = prolong(ls, qs, src.w[v], I);
      if (mask & 2)
        for (int v = 0; v < 5; ++v) b.us[v][c] = prolong(ls, qs, src.us[v], I);
      const int P[3] = {I[0] >> 1, I[1] >> 1, I[2] >> 1};
      f = src.flags[leaf_cell(ls, qs, P)];
    }
    if (mask & 8) {
      b.flags[c] = f;
      take = (f & (GRMHD_F_FOFC | GRMHD_F_DMP)) != 0;
    }
  }
  if (list) fofc_append(b, q, take, c);
}

// face value of leaf s (geometry q) in direction d at global face index J
// (J[d] the face index along d, the others cell indices) of its level
__device__ __forceinline__ double leaf_face(const grmhd_block& bs, const grmhd_amr_link& ls,
                                            const Geo& q, int d, const int J[3]) {
  const gptr<const double> f = (gptr<const double>)bs.bs[d];
  return f[face_rt(q, d, J[0] - ls.org[0] + q.g, J[1] - ls.org[1] + q.g, J[2] - ls.org[2] + q.g)];
}

// Ghost faces of direction d (launch shape S_GXFACE + d); passes as for the
// cells.
__global__ __launch_bounds__(kMaxThreads) void k_ghost_faces_amr(
    const grmhd_block* __restrict__ blks, const grmhd_amr_link* __restrict__ L, int d, int pass,
    int b0, int b1) {
  int ib;
  int64_t t;
  if (!locate_range(blks, S_GXFACE + d, b0, b1, ib, t)) return;
  const grmhd_amr_link& lk = L[ib];
  if (pass > 0 && lk.level != pass) return;
  const Geo q = geo_of(blks[ib]);
  int x[3];
  ghost_ring(q, S_GXFACE + d).at(t, x[0], x[1], x[2]);
  const int64_t dst = face_rt(q, d, x[0], x[1], x[2]);
  const int n[3] = {q.nx, q.ny, q.nz};
  // across d: cells as in the cell fill; along d: the face index (periodic:
  // modulo N; outflow: clamped to the boundary faces 0 and N, the padded
  // position moved with it)
  int F[3], o[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a != d) amr_axis(lk, q, a, x[a], F[a], o[a]);
  const int N = lk.N[d];
  int xd = x[d];
  int Fd = lk.org[d] + x[d] - q.g;
  if (Fd < 0 || Fd >= N) {
    if ((lk.periodic >> d) & 1) {
      Fd = Fd < 0 ? Fd + N : Fd - N;
    } else if (Fd < 0 || Fd > N) {
      Fd = Fd < 0 ? 0 : N;
      xd = Fd - lk.org[d] + q.g;
    }
  }
  F[d] = Fd;
  // the two sides: the cell above (padded xd, global Fd) and below (xd - 1,
  // Fd - 1); for each its leaf and the face's index along d in its numbering
  // (the upper face of the cell below is Fd - 1 + 1, N across a periodic
  // boundary)
  const bool per = (lk.periodic >> d) & 1;
  int leaf[2], lev[2], fidx[2];
  const bool first_m = x[d] == q.g + n[d];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const bool below = first_m ? side == 0 : side == 1;
    const int xc = below ? xd - 1 : xd;
    int Gc = below ? Fd - 1 : Fd;
    bool exists = true;
    if (Gc < 0) {
      if (per) Gc += N; else exists = false;
    }
    if (Gc >= N) exists = false;
    leaf[side] = -1;
    lev[side] = -100;
    fidx[side] = below ? Gc + 1 : Gc;
    if (!exists) continue;
    int oo[3] = {o[0], o[1], o[2]};
    oo[d] = xc < q.g ? -1 : (xc >= q.g + n[d] ? 1 : 0);
    int I[3] = {F[0], F[1], F[2]};
    I[d] = Gc;
    const int dir = dir_of(oo);
    const int s = amr_pick(L, lk, dir, I, q.nx);
    if (s < 0) continue;
    leaf[side] = s;
    lev[side] = lk.level + lk.rel[dir];
  }
  // same level first, then finer, then coarser; the first side in order
  int pick = -1, kind = -1;
#pragma unroll
  for (int want = 0; want < 3; ++want) {
    const int lw = want == 0 ? lk.level : (want == 1 ? lk.level + 1 : lk.level - 1);
    for (int side = 0; side < 2; ++side)
      if (pick < 0 && lev[side] == lw) {
        pick = side;
        kind = want;
      }
  }
  if (pick < 0) return;
  if ((kind < 2 && pass > 0) || (kind == 2 && pass == 0)) return;
  const int s = leaf[pick];
  const grmhd_block& sb = blks[s];
  const grmhd_amr_link& ls = L[s];
  const Geo qs = geo_of(sb);
  const int Fs = fidx[pick];
  double val;
  if (kind == 0) {
    int J[3] = {F[0], F[1], F[2]};
    J[d] = Fs;
    val = leaf_face(sb, ls, qs, d, J);
  } else if (kind == 1) {
    double sum = 0.0;
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      int J[3];
      int tt = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a == d) {
          J[a] = 2 * Fs;
        } else {
          J[a] = 2 * F[a] + ((c4 >> tt) & 1);
          ++tt;
        }
      }
      sum += leaf_face(sb, ls, qs, d, J);
    }
    val = 0.25 * sum;
  } else {
    int J[3] = {F[0] >> 1, F[1] >> 1, F[2] >> 1};
    J[d] = Fs >> 1;
    if ((Fs & 1) == 0) {
      val = leaf_face(sb, ls, qs, d, J);
    } else {
      int J1[3] = {J[0], J[1], J[2]};
      J1[d] += 1;
      val = 0.5 * (leaf_face(sb, ls, qs, d, J) + leaf_face(sb, ls, qs, d, J1));
    }
  }
  ((gptr<double>)blks[ib].bs[d])[dst] = val;
}

// Flux correction: items (block, side of 6, boundary face of nb^2); a
// block's boundary face next to a finer leaf takes the mean of that leaf's
// 4 fluxes there (all 7 components).
__global__ __launch_bounds__(kAmrThreads) void k_amr_flux_fix(
    const grmhd_block* __restrict__ blks, const grmhd_amr_link* __restrict__ L, int nblk, int nb) {
  const int64_t per = 6 * (int64_t)nb * nb;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nblk) return;
  const int ib = (int)(t / per);
  const int r = (int)(t - (int64_t)ib * per);
  const int side6 = r / (nb * nb), qf = r - side6 * nb * nb;
  const int d = side6 >> 1, up = side6 & 1;
  const grmhd_amr_link& lk = L[ib];
  int o[3] = {0, 0, 0};
  o[d] = up ? 1 : -1;
  const int dir = dir_of(o);
  if (lk.rel[dir] != 1) return;
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const int q1 = qf % nb, q2 = qf / nb;
  int I[3];
  const int N = lk.N[d];
  int Gd = lk.org[d] + (up ? nb : -1);
  Gd = Gd < 0 ? Gd + N : (Gd >= N ? Gd - N : Gd);   // a finer region is never beyond an outflow edge
  I[d] = Gd;
  I[t1] = lk.org[t1] + q1;
  I[t2] = lk.org[t2] + q2;
  const int s = amr_pick(L, lk, dir, I, nb);
  if (s < 0) return;
  const grmhd_block& fb = blks[s];
  const grmhd_amr_link& ls = L[s];
  const Geo qs = geo_of(fb);
  const Geo q = geo_of(blks[ib]);
  const gptr<const double> FS = (gptr<const double>)fb.scratch;
  gptr<double> FB = (gptr<double>)blks[ib].scratch;
  int64_t ff[4];
#pragma unroll
  for (int c4 = 0; c4 < 4; ++c4) {
    int J[3];
    // across the lower face: the upper faces of the children 2I + 1; across
    // the upper face: the lower faces of the children 2I
    J[d] = up ? 2 * I[d] : 2 * I[d] + 2;
    J[t1] = 2 * I[t1] + (c4 & 1);
    J[t2] = 2 * I[t2] + (c4 >> 1);
    ff[c4] = face_rt(qs, d, J[0] - ls.org[0] + qs.g, J[1] - ls.org[1] + qs.g, J[2] - ls.org[2] + qs.g);
  }
  int x[3];
  x[d] = up ? q.g + nb : q.g;
  x[t1] = q.g + q1;
  x[t2] = q.g + q2;
  const int64_t f0 = face_rt(q, d, x[0], x[1], x[2]);
  for (int v = 0; v < 7; ++v) {
    const gptr<const double> a = FS + off_flux(qs, d, v);
    double sum = 0.0;
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) sum += a[ff[c4]];
    FB[off_flux(q, d, v) + f0] = 0.25 * sum;
  }
}

// EMF correction: items (block, component of 3, perimeter position of 4 nb
// on the plane across the component, position along it of nb); a block's
// boundary edge EMF where one of the 4 cells around the edge lies in a finer
// leaf takes the mean of that leaf's 2 EMFs along the edge.
__global__ __launch_bounds__(kAmrThreads) void k_amr_emf_fix(
    const grmhd_block* __restrict__ blks, const grmhd_amr_link* __restrict__ L, int nblk, int nb) {
  const int64_t per = 12 * (int64_t)nb * nb;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nblk) return;
  const int ib = (int)(t / per);
  int r = (int)(t - (int64_t)ib * per);
  const int comp = r / (4 * nb * nb);
  r -= comp * 4 * nb * nb;
  const int p = r / nb, uc = r - p * nb;
  const int side = p / nb, u = p - side * nb;
  const grmhd_amr_link& lk = L[ib];
  const Geo q = geo_of(blks[ib]);
  const int g = q.g;
  const int A = (comp + 1) % 3, B = (comp + 2) % 3;
  int x[3];
  x[comp] = g + uc;
  x[A] = side == 0 ? g + u : (side == 1 ? g + nb : (side == 2 ? g + nb - u : g));
  x[B] = side == 0 ? g : (side == 1 ? g + u : (side == 2 ? g + nb : g + nb - u));
  for (int cl = 0; cl < 4; ++cl) {
    const int oa = cl & 1, ob = cl >> 1;   // the cell (a - oa, b - ob)
    int I[3], o[3];
    bool outside = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int xc = x[a] - (a == A ? oa : 0) - (a == B ? ob : 0);
      int G = lk.org[a] + xc - g;
      o[a] = xc < g ? -1 : (xc >= g + nb ? 1 : 0);
      const int N = lk.N[a];
      if (G < 0 || G >= N) {
        if ((lk.periodic >> a) & 1) G = G < 0 ? G + N : G - N;
        else outside = true;
      }
      I[a] = G;
    }
    if (outside) continue;
    const int dir = dir_of(o);
    if (lk.rel[dir] != 1) continue;
    const int s = amr_pick(L, lk, dir, I, nb);
    if (s < 0) continue;
    const grmhd_amr_link& ls = L[s];
    const Geo qs = geo_of(blks[s]);
    const gptr<const double> E =
        (gptr<const double>)blks[s].scratch + off_edge(qs) + comp * n_edges(qs);
    double sum = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int J[3];
      J[comp] = 2 * I[comp] + h;
      J[A] = 2 * (I[A] + oa);
      J[B] = 2 * (I[B] + ob);
      sum += E[edge(qs, J[0] - ls.org[0] + qs.g, J[1] - ls.org[1] + qs.g, J[2] - ls.org[2] + qs.g)];
    }
    ((gptr<double>)blks[ib].scratch)[off_edge(q) + comp * n_edges(q) + edge(q, x[0], x[1], x[2])] =
        0.5 * sum;
    return;
  }
}

// ---------------------------------------------------------------------------
// host: links
// ---------------------------------------------------------------------------
// interval [lo, hi] of level lv as an interval of level lt
void to_level(int64_t lo, int64_t hi, int lv, int lt, int64_t& a, int64_t& b) {
  if (lt >= lv) {
    a = lo << (lt - lv);
    b = ((hi + 1) << (lt - lv)) - 1;
  } else {
    a = lo >> (lv - lt);
    b = hi >> (lv - lt);
  }
}

}  // namespace

namespace gk {

int amr_max_level(const grmhd_amr_link* h, int nblk) {
  int m = 0;
  for (int i = 0; i < nblk; ++i) m = std::max(m, (int)h[i].level);
  return m;
}

// blocks of one size (nb^3, nb >= 2 ng + 2) and ghosts filled (bc == 1)
int amr_check(const grmhd_block* h, const grmhd_amr_link* lh, int nblk) {
  if (!h || !lh || nblk < 1) return GRMHD_EINVAL;
  const int nb = h[0].nx, ng = h[0].ng;
  if (nb < 2 * ng + 2 || (nb & 1) || ng < 1) return GRMHD_EINVAL;
  for (int i = 0; i < nblk; ++i) {
    if (h[i].nx != nb || h[i].ny != nb || h[i].nz != nb || h[i].ng != ng || h[i].bc != 1)
      return GRMHD_EINVAL;
    if (lh[i].level < 0 || lh[i].level > 24) return GRMHD_EINVAL;
    for (int dir = 0; dir < 27; ++dir)
      for (int c = 0; c < 4; ++c)
        if (lh[i].src[dir][c] < -1 || lh[i].src[dir][c] >= nblk) return GRMHD_EINVAL;
  }
  return GRMHD_OK;
}

// the blocks of pass `pass` (all for pass <= 0; the leaves of that level
// for pass > 0, a contiguous range when the list is ordered by level, else
// all of them) and the workgroups covering their items of shape cls
static bool pass_range(const grmhd_block* h, const grmhd_amr_link* lh, int nblk, int pass, int cls,
                       int threads, int& b0, int& b1, unsigned& grid) {
  b0 = 0;
  b1 = nblk - 1;
  if (pass > 0) {
    int first = -1, last = -1, count = 0;
    for (int i = 0; i < nblk; ++i)
      if (lh[i].level == pass) {
        if (first < 0) first = i;
        last = i;
        ++count;
      }
    if (count == 0) return false;
    if (last - first + 1 == count) {
      b0 = first;
      b1 = last;
    }
  }
  const int64_t waves = (int64_t)h[b1].wave0[cls] + (shape_items(geo_of(h[b1]), cls) + 63) / 64 -
                        h[b0].wave0[cls];
  grid = (unsigned)((waves * 64 + threads - 1) / threads);
  return waves > 0;
}

void launch_ghost_cells_amr(const grmhd_block* h, const grmhd_block* d, int nblk,
                            const grmhd_amr_link* lh, const grmhd_amr_link* ld, int mask, int list,
                            int pass, int threads, hipStream_t s) {
  int b0, b1;
  unsigned grid;
  if (!pass_range(h, lh, nblk, pass, list ? S_GSHELL : S_GCELLS, threads, b0, b1, grid)) return;
  k_ghost_cells_amr<<<grid, threads, 0, s>>>(d, ld, mask, list, pass, b0, b1);
}

void launch_ghost_faces_amr(const grmhd_block* h, const grmhd_block* d, int nblk,
                            const grmhd_amr_link* lh, const grmhd_amr_link* ld, int dir, int pass,
                            int threads, hipStream_t s) {
  int b0, b1;
  unsigned grid;
  if (!pass_range(h, lh, nblk, pass, S_GXFACE + dir, threads, b0, b1, grid)) return;
  k_ghost_faces_amr<<<grid, threads, 0, s>>>(d, ld, dir, pass, b0, b1);
}

void launch_amr_flux_fix(const grmhd_block* d, const grmhd_amr_link* ld, int nblk, int nb,
                         hipStream_t s) {
  const int64_t items = 6 * (int64_t)nb * nb * nblk;
  k_amr_flux_fix<<<(unsigned)((items + kAmrThreads - 1) / kAmrThreads), kAmrThreads, 0, s>>>(d, ld, nblk, nb);
}

void launch_amr_emf_fix(const grmhd_block* d, const grmhd_amr_link* ld, int nblk, int nb,
                        hipStream_t s) {
  const int64_t items = 12 * (int64_t)nb * nb * nblk;
  k_amr_emf_fix<<<(unsigned)((items + kAmrThreads - 1) / kAmrThreads), kAmrThreads, 0, s>>>(d, ld, nblk, nb);
}

}  // namespace gk

extern "C" int grmhd_amr_links(int32_t nblk, const int32_t* level, const int32_t* org, int32_t nb,
                               int32_t ng, const int32_t n0[3], const int32_t periodic[3],
                               grmhd_amr_link* links) {
  if (nblk < 1 || !level || !org || !n0 || !periodic || !links) return GRMHD_EINVAL;
  if (ng < 1 || nb < 2 * ng + 2 || (nb & 1)) return GRMHD_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (n0[a] < nb || n0[a] % nb) return GRMHD_EINVAL;
  for (int i = 0; i < nblk; ++i) {
    if (level[i] < 0 || level[i] > 24) return GRMHD_EINVAL;
    for (int a = 0; a < 3; ++a) {
      const int64_t N = (int64_t)n0[a] << level[i];
      if (org[3 * i + a] < 0 || org[3 * i + a] + nb > N || org[3 * i + a] % nb) return GRMHD_EINVAL;
    }
  }
  // no two leaves overlap (pairwise, at the finer of the two levels)
  for (int i = 0; i < nblk; ++i)
    for (int j = i + 1; j < nblk; ++j) {
      bool ov = true;
      const int lt = std::max(level[i], level[j]);
      for (int a = 0; a < 3 && ov; ++a) {
        int64_t ai, bi, aj, bj;
        to_level(org[3 * i + a], org[3 * i + a] + nb - 1, level[i], lt, ai, bi);
        to_level(org[3 * j + a], org[3 * j + a] + nb - 1, level[j], lt, aj, bj);
        ov = ai <= bj && aj <= bi;
      }
      if (ov) return GRMHD_EINVAL;
    }
  for (int i = 0; i < nblk; ++i) {
    grmhd_amr_link& lk = links[i];
    const int lv = level[i];
    lk.level = lv;
    lk.periodic = 0;
    for (int a = 0; a < 3; ++a) {
      lk.org[a] = org[3 * i + a];
      lk.N[a] = n0[a] << lv;
      if (periodic[a]) lk.periodic |= 1 << a;
    }
    for (int dir = 0; dir < 27; ++dir) {
      const int o[3] = {dir % 3 - 1, (dir / 3) % 3 - 1, dir / 9 - 1};
      for (int c = 0; c < 4; ++c) lk.src[dir][c] = -1;
      lk.rel[dir] = GRMHD_AMR_NONE;
      if (dir == 13) {
        lk.rel[dir] = 0;
        lk.src[dir][0] = i;
        continue;
      }
      // the region, ng + 1 cells deep, wrapped across periodic boundaries
      int64_t lo[3], hi[3];
      bool beyond = false;
      for (int a = 0; a < 3; ++a) {
        const int64_t N = lk.N[a], og = lk.org[a];
        lo[a] = o[a] < 0 ? og - ng - 1 : (o[a] > 0 ? og + nb : og);
        hi[a] = o[a] < 0 ? og - 1 : (o[a] > 0 ? og + nb + ng : og + nb - 1);
        if (lo[a] < 0 || hi[a] >= N) {
          if (!periodic[a]) beyond = true;
          else if (lo[a] < 0) { lo[a] += N; hi[a] += N; }
          else { lo[a] -= N; hi[a] -= N; }
        }
      }
      if (beyond) continue;
      int cnt = 0, lvl = -1;
      for (int j = 0; j < nblk; ++j) {
        bool ov = true;
        for (int a = 0; a < 3 && ov; ++a) {
          int64_t ra, rb;
          to_level(lo[a], hi[a], lv, level[j], ra, rb);
          ov = ra <= org[3 * j + a] + nb - 1 && org[3 * j + a] <= rb;
        }
        if (!ov) continue;
        if (cnt == 4) return GRMHD_EINVAL;
        if (lvl >= 0 && level[j] != lvl) return GRMHD_EINVAL;
        lvl = level[j];
        lk.src[dir][cnt++] = j;
      }
      if (cnt == 0 || lvl < lv - 1 || lvl > lv + 1) return GRMHD_EINVAL;
      lk.rel[dir] = lvl - lv;
    }
  }
  return GRMHD_OK;
}
