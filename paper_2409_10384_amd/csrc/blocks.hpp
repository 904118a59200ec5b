// blocks.hpp -- MeshBlock geometry, scratch layout and the flattened launch
// layout shared by the stage kernels and the learned-bracket kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grmhd.h"
#include "physics.hpp"

namespace gk {

// ---------------------------------------------------------------------------
// block geometry helpers
// ---------------------------------------------------------------------------
struct Geo {
  int nx, ny, nz, g, sx, sy, sz;
};

__host__ __device__ __forceinline__ Geo geo_of(const grmhd_block& b) {
  Geo q;
  q.nx = b.nx; q.ny = b.ny; q.nz = b.nz; q.g = b.ng;
  q.sx = b.nx + 2 * b.ng; q.sy = b.ny + 2 * b.ng; q.sz = b.nz + 2 * b.ng;
  return q;
}

// A pointer into global memory (address space 1).
template <class T>
using gptr = __attribute__((address_space(1))) T*;

// Device view of a block: its sizes and arrays, with every array typed as
// global memory.  Through the plain pointers of the C struct the compiler
// cannot tell global memory from LDS and emits flat loads, each with its own
// 64-bit address; through these it emits global loads from a scalar base
// plus a 32-bit offset.  (The neighbour table and the launch layout stay in
// the C struct, read from there where needed.)
struct GB {
  int nx, ny, nz, ng;
  double dx[3];
  gptr<double> w[5], un[5], us[5], bn[3], bs[3], uo[5], bo[3], wo[5];
  gptr<const double> adm[16];
  gptr<uint16_t> flags;
  gptr<double> scratch;
};

__device__ __forceinline__ GB gview(const grmhd_block& b) {
  GB g;
  g.nx = b.nx; g.ny = b.ny; g.nz = b.nz; g.ng = b.ng;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g.dx[a] = b.dx[a];
    g.bn[a] = (gptr<double>)b.bn[a];
    g.bs[a] = (gptr<double>)b.bs[a];
    g.bo[a] = (gptr<double>)b.bo[a];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    g.w[v] = (gptr<double>)b.w[v];
    g.un[v] = (gptr<double>)b.un[v];
    g.us[v] = (gptr<double>)b.us[v];
    g.uo[v] = (gptr<double>)b.uo[v];
    g.wo[v] = (gptr<double>)b.wo[v];
  }
#pragma unroll
  for (int n = 0; n < 16; ++n) g.adm[n] = (gptr<const double>)b.adm[n];
  g.flags = (gptr<uint16_t>)b.flags;
  g.scratch = (gptr<double>)b.scratch;
  return g;
}

__device__ __forceinline__ Geo geo_of(const GB& b) {
  Geo q;
  q.nx = b.nx; q.ny = b.ny; q.nz = b.nz; q.g = b.ng;
  q.sx = b.nx + 2 * b.ng; q.sy = b.ny + 2 * b.ng; q.sz = b.nz + 2 * b.ng;
  return q;
}
__host__ __device__ __forceinline__ int64_t n_cells(const Geo& q) {
  return (int64_t)q.sx * q.sy * q.sz;
}
__host__ __device__ __forceinline__ int64_t n_faces(const Geo& q, int d) {
  return (int64_t)(q.sx + (d == 0)) * (q.sy + (d == 1)) * (q.sz + (d == 2));
}
__host__ __device__ __forceinline__ int64_t n_edges(const Geo& q) {
  return (int64_t)(q.sx + 1) * (q.sy + 1) * (q.sz + 1);
}
__device__ __forceinline__ int64_t cell(const Geo& q, int i, int j, int k) {
  return ((int64_t)k * q.sy + j) * q.sx + i;
}
template <int D>
__device__ __forceinline__ int64_t face(const Geo& q, int i, int j, int k) {
  const int ex = q.sx + (D == 0), ey = q.sy + (D == 1);
  return ((int64_t)k * ey + j) * ex + i;
}
__device__ __forceinline__ int64_t face_rt(const Geo& q, int d, int i, int j, int k) {
  const int ex = q.sx + (d == 0), ey = q.sy + (d == 1);
  return ((int64_t)k * ey + j) * ex + i;
}
__device__ __forceinline__ int64_t edge(const Geo& q, int i, int j, int k) {
  return ((int64_t)k * (q.sy + 1) + j) * (q.sx + 1) + i;
}

// scratch layout (doubles): flux[d][c] | Bcc[3] | Ecc[3] | Eedge[3] | wave stats | FOFC list
__host__ __device__ __forceinline__ int64_t off_flux(const Geo& q, int d, int c) {
  int64_t o = 0;
  for (int dd = 0; dd < d; ++dd) o += 7 * n_faces(q, dd);
  return o + c * n_faces(q, d);
}
__host__ __device__ __forceinline__ int64_t off_bcc(const Geo& q) {
  return off_flux(q, 3, 0);
}
__host__ __device__ __forceinline__ int64_t off_ecc(const Geo& q) {
  return off_bcc(q) + 3 * n_cells(q);
}
__host__ __device__ __forceinline__ int64_t off_edge(const Geo& q) {
  return off_ecc(q) + 3 * n_cells(q);
}
// statistics of the stage inversion: per 64-cell wave of the interior shape,
// the wave's solves, evaluations, fallbacks and failures (4 uint64), summed
// by a reduction kernel (room for 2 doubles per padded cell)
__host__ __device__ __forceinline__ int64_t off_wstat(const Geo& q) {
  return off_edge(q) + 3 * n_edges(q);
}
// FOFC cell list: the flagged cells of [g-1, g+n]^3 (interior cells and the
// first ghost shell), int32 padded-cell indices after a uint32 counter
__host__ __device__ __forceinline__ int64_t fofc_cap(const Geo& q) {
  return (int64_t)(q.nx + 2) * (q.ny + 2) * (q.nz + 2);
}
__host__ __device__ __forceinline__ int64_t off_fofc(const Geo& q) {
  return off_wstat(q) + 2 * n_cells(q);
}
__host__ __device__ __forceinline__ int64_t scratch_total(const Geo& q) {
  return off_fofc(q) + (fofc_cap(q) + 2 + 1) / 2;
}
__device__ __forceinline__ gptr<unsigned int> fofc_count(const GB& b, const Geo& q) {
  return (gptr<unsigned int>)(b.scratch + off_fofc(q));
}
__device__ __forceinline__ gptr<int> fofc_list(const GB& b, const Geo& q) {
  return (gptr<int>)(b.scratch + off_fofc(q)) + 2;
}

// Sum (solves, evaluations, fallbacks, failures) over the wave and store it
// in the block's per-wave slot (lane 0; item index t of the interior shape).
// Inactive lanes must not call this; every lane of a live wave does.
__device__ __forceinline__ void wave_stats_store(const GB& b, const Geo& q, int64_t t,
                                                 unsigned long long n, unsigned long long ev,
                                                 unsigned long long fb, unsigned long long fail) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    n += __shfl_xor(n, o, 64);
    ev += __shfl_xor(ev, o, 64);
    fb += __shfl_xor(fb, o, 64);
    fail += __shfl_xor(fail, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    gptr<unsigned long long> ws = (gptr<unsigned long long>)(b.scratch + off_wstat(q)) + 4 * (t >> 6);
    ws[0] = n; ws[1] = ev; ws[2] = fb; ws[3] = fail;
  }
}

// Append cell c to the block's FOFC list when `take`; all lanes of the wave
// belong to one block.  One atomic per wave; entries beyond the capacity are
// dropped (cannot happen when the counter is cleared every stage).
__device__ __forceinline__ void fofc_append(const GB& b, const Geo& q, bool take,
                                            int64_t c) {
  const unsigned long long m = __ballot(take);
  if (!m) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd((unsigned int*)fofc_count(b, q), (unsigned int)__popcll(m));
  base = __shfl(base, leader, 64);
  if (take) {
    const unsigned int below = (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
    const unsigned int idx = base + below;
    if ((int64_t)idx < fofc_cap(q)) fofc_list(b, q)[idx] = (int)c;
  }
}

// Launch shapes: every kernel runs over one "shape" of items per block,
// flattened over the whole block list in 64-item waves (a wave never spans
// two blocks; the host stores each block's first wave per shape in wave0).
enum {
  S_CELLS = 0,    // padded cells
  S_INTERIOR,     // interior cells
  S_EXT,          // cells [g-1, g+n] (cell-centre EMF)
  S_XFACE,        // extended face ranges of direction x, y, z (fluxes)
  S_YFACE,
  S_ZFACE,
  S_XEDGE,        // corner-EMF ranges of component x, y, z
  S_YEDGE,
  S_ZEDGE,
  S_XIFACE,       // interior faces of direction x, y, z (CT update)
  S_YIFACE,
  S_ZIFACE,
  S_XPFACE,       // padded faces of direction x, y, z
  S_YPFACE,
  S_ZPFACE,
  S_GCELLS,       // ghost cells: padded cells minus the interior (ghost fill)
  S_GSHELL,       // first ghost shell [g-1, g+n]^3 minus the interior (flag exchange)
  S_GXFACE,       // ghost faces of direction x, y, z: padded faces minus the
  S_GYFACE,       // interior ones (faces g..g+n along the direction, cells
  S_GZFACE,       // g..g+n-1 across; ghost-face fill)
  S_CORNER,       // cell corners [g, g+n]^3 (corner EMFs and face update of CT)
  S_COUNT
};
// the descriptor's wave0 table has one slot per launch shape
static_assert(S_COUNT <= (int)(sizeof(((grmhd_block*)0)->wave0) / sizeof(int32_t)),
              "grmhd_block.wave0 needs a slot for every launch shape");

// A box with a box-shaped hole: the extents e[3] of an outer box, and the
// hole at offset l[3] (relative to the outer origin) with counts c[3] inside
// it.  Items run over the outer box minus the hole, x fastest: the planes
// below the hole, then each plane through the hole (rows below it, the rows
// through it without the hole's cells, rows above it), then the planes
// above it.
struct Ring {
  int e[3], l[3], c[3];
  __host__ __device__ __forceinline__ int64_t size() const {
    return (int64_t)e[0] * e[1] * e[2] - (int64_t)c[0] * c[1] * c[2];
  }
  // position (i, j, k) relative to the outer origin of item t < size()
  __host__ __device__ __forceinline__ void at(int64_t t, int& i, int& j, int& k) const {
    const int64_t plane = (int64_t)e[0] * e[1];
    const int64_t below = (int64_t)l[2] * plane;
    if (t < below) {
      k = (int)(t / plane);
      const int64_t r = t - (int64_t)k * plane;
      j = (int)(r / e[0]);
      i = (int)(r - (int64_t)j * e[0]);
      return;
    }
    t -= below;
    const int64_t ring = plane - (int64_t)c[0] * c[1];
    const int64_t mid = (int64_t)c[2] * ring;
    if (t >= mid) {
      t -= mid;
      const int kk = (int)(t / plane);
      const int64_t r = t - (int64_t)kk * plane;
      k = l[2] + c[2] + kk;
      j = (int)(r / e[0]);
      i = (int)(r - (int64_t)j * e[0]);
      return;
    }
    const int kk = (int)(t / ring);
    int64_t r = t - (int64_t)kk * ring;
    k = l[2] + kk;
    const int64_t rows_lo = (int64_t)l[1] * e[0];
    if (r < rows_lo) {
      j = (int)(r / e[0]);
      i = (int)(r - (int64_t)j * e[0]);
      return;
    }
    r -= rows_lo;
    const int side = e[0] - c[0];
    const int64_t rows_mid = (int64_t)c[1] * side;
    if (r < rows_mid) {
      const int jj = (int)(r / side);
      const int s = (int)(r - (int64_t)jj * side);
      j = l[1] + jj;
      i = s < l[0] ? s : s + c[0];
      return;
    }
    r -= rows_mid;
    const int jj = (int)(r / e[0]);
    j = l[1] + c[1] + jj;
    i = (int)(r - (int64_t)jj * e[0]);
  }
};

// the ghost region of launch shape cls (S_GCELLS .. S_GZFACE), in padded
// cell or face coordinates
__host__ __device__ __forceinline__ Ring ghost_ring(const Geo& q, int cls) {
  Ring r;
  const int n[3] = {q.nx, q.ny, q.nz};
  const int s[3] = {q.sx, q.sy, q.sz};
  if (cls == S_GSHELL) {
    // offset g-1 is added by the caller
    for (int a = 0; a < 3; ++a) { r.e[a] = n[a] + 2; r.l[a] = 1; r.c[a] = n[a]; }
    return r;
  }
  const int d = cls - S_GXFACE;   // -1.. for S_GCELLS: no face direction
  for (int a = 0; a < 3; ++a) {
    const int f = (cls != S_GCELLS && a == d) ? 1 : 0;
    r.e[a] = s[a] + f;
    r.l[a] = q.g;
    r.c[a] = n[a] + f;
  }
  return r;
}

__host__ __device__ __forceinline__ int64_t shape_items(const Geo& q, int cls) {
  const int n[3] = {q.nx, q.ny, q.nz};
  int64_t c = 1;
  switch (cls) {
    case S_CELLS: return n_cells(q);
    case S_INTERIOR: return (int64_t)n[0] * n[1] * n[2];
    case S_EXT: return (int64_t)(n[0] + 2) * (n[1] + 2) * (n[2] + 2);
    case S_XFACE: case S_YFACE: case S_ZFACE:
      for (int a = 0; a < 3; ++a) c *= a == cls - S_XFACE ? n[a] + 1 : n[a] + 2;
      return c;
    case S_XEDGE: case S_YEDGE: case S_ZEDGE:
      for (int a = 0; a < 3; ++a) c *= a == cls - S_XEDGE ? n[a] : n[a] + 1;
      return c;
    case S_XIFACE: case S_YIFACE: case S_ZIFACE:
      for (int a = 0; a < 3; ++a) c *= a == cls - S_XIFACE ? n[a] + 1 : n[a];
      return c;
    case S_XPFACE: case S_YPFACE: case S_ZPFACE: return n_faces(q, cls - S_XPFACE);
    case S_CORNER: return (int64_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
    default: return ghost_ring(q, cls).size();
  }
}

// XCD-aware order.  Workgroups are dealt round-robin to the 8 XCDs by
// linear id L; each XCD has its own L2.  Renumber so that XCD x owns a
// contiguous range of tiles (its y/z stencil neighbours then share that L2):
// L -> start(L % 8) + L / 8, a bijection of [0, N) for any N.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_linear() {
  const int n = gridDim.x;
  const int L = blockIdx.x;
  const int x = L % kXcds, i = L / kXcds;
  const int q = n / kXcds, r = n % kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// block and item of this thread for launch shape cls; false when the thread
// has no item (past the last wave, or in the padding of a block's last wave)
__device__ __forceinline__ bool locate(const grmhd_block* __restrict__ blks, int cls, int& bi,
                                       int64_t& t) {
  const int64_t g = (int64_t)xcd_linear() * blockDim.x + threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane((int)(g >> 6));
  const int nb = blks[0].nblk;
  const int last = blks[nb - 1].wave0[cls];
  // binary search: largest b with wave0[b] <= w
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blks[mid].wave0[cls] <= w) lo = mid; else hi = mid - 1;
  }
  bi = lo;
  const Geo q = geo_of(blks[bi]);
  if (bi == nb - 1 && w >= last + (int)((shape_items(q, cls) + 63) >> 6)) return false;
  t = (int64_t)(w - blks[bi].wave0[cls]) * 64 + (threadIdx.x & 63);
  return t < shape_items(q, cls);
}

// decompose a linear item index over a box [lo, lo+cnt)
struct Box {
  int lo[3], cnt[3];
  __device__ __forceinline__ int64_t size() const { return (int64_t)cnt[0] * cnt[1] * cnt[2]; }
  __device__ __forceinline__ void at(int64_t t, int& i, int& j, int& k) const {
    i = lo[0] + (int)(t % cnt[0]);
    const int64_t r = t / cnt[0];
    j = lo[1] + (int)(r % cnt[1]);
    k = lo[2] + (int)(r / cnt[1]);
  }
};

// extended face range of direction D: faces [g, g+n_D] along D, cells
// [g-1, g+n_t] across (one ghost column each side for the corner EMFs)
template <int D>
__device__ __forceinline__ Box face_box(const Geo& q) {
  Box b;
  const int n[3] = {q.nx, q.ny, q.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a == D) { b.lo[a] = q.g; b.cnt[a] = n[a] + 1; }
    else { b.lo[a] = q.g - 1; b.cnt[a] = n[a] + 2; }
  }
  return b;
}
__device__ __forceinline__ Box interior_box(const Geo& q) {
  Box b;
  b.lo[0] = b.lo[1] = b.lo[2] = q.g;
  b.cnt[0] = q.nx; b.cnt[1] = q.ny; b.cnt[2] = q.nz;
  return b;
}

__device__ __forceinline__ double dt_of(const double* dt_d, double dt) {
  return dt_d ? *dt_d : dt;
}

__device__ __forceinline__ void cell_metric(const GB& b, int64_t c, M3& m) {
  metric_build(m, b.adm[4][c], b.adm[5][c], b.adm[6][c], b.adm[7][c], b.adm[8][c], b.adm[9][c]);
}

// densitized cell-centred field from the faces of slot f
template <class P>
__device__ __forceinline__ void cell_bt(const Geo& q, const P* f, int i, int j, int k,
                                        double Bt[3]) {
  Bt[0] = 0.5 * (f[0][face<0>(q, i, j, k)] + f[0][face<0>(q, i + 1, j, k)]);
  Bt[1] = 0.5 * (f[1][face<1>(q, i, j, k)] + f[1][face<1>(q, i, j + 1, k)]);
  Bt[2] = 0.5 * (f[2][face<2>(q, i, j, k)] + f[2][face<2>(q, i, j, k + 1)]);
}

}  // namespace gk
