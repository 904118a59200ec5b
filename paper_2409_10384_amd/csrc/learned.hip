// learned.hip -- learned initial guess and bracket for the inversion (not in
// the paper): feature extraction, MLP inference fused with the FP64 root
// solve, and MLP training (forward, backward, Adam) on the MFMA units.
//
// The FP64 bracketed root solve of the paper's inversion always finishes:
// the network only chooses the starting bracket; when that bracket holds no
// sign change the full bracket is used (flag GRMHD_F_BRACKET_FALLBACK).
// Built without contraction to fused multiply-adds (the rest of the library
// fuses within expressions): with it the fused network + root-solve kernel
// of the piecewise polytrope needs 258 registers (VGPRs + AGPRs) and drops
// to one wave per SIMD.
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "blocks.hpp"
#include "grmhd.h"
#include "mlp.hpp"
#include "physics.hpp"
#include "timing.hpp"

using namespace gk;

namespace gk {
Eos make_eos_host(const grmhd_params& p);
unsigned stage_grid(const grmhd_block* h, int nblk, int cls, int threads);
void launch_stats_sum(const grmhd_block* d, int nblk, c2p_stats* stats, hipStream_t s);
int check_params_host(const grmhd_params* p);
void launch_c2p_batch(int64_t n, double* const* u, double* const* bt, double* const* gam, double* const* w,
                      uint16_t* flags, const grmhd_params& p, const double* blo, const double* bhi,
                      double* mu_out, int32_t* nev_out, c2p_stats* stats, hipStream_t s);
}  // namespace gk

namespace {

constexpr int kT = 256;   // threads per workgroup of the fused inversion

struct P5 { double* p[5]; };
struct P3 { double* p[3]; };
struct P6 { double* p[6]; };
struct Feat { float mean[5], scale[5]; };

// invariant features of the scaled state (the oracle's definition), in fp32:
// they are rounded to bf16 on entry to the network anyway.  log10 D from the
// FP64 exponent plus the fp32 log of the mantissa, so any D > 0 is in range.
__device__ __forceinline__ void features(const KState& k, const Feat& f, float x[5]) {
  constexpr float kLog10_2 = 0.30102999566398120f;
  int ex;
  const double man = frexp(k.D, &ex);
  const float iq1 = __builtin_amdgcn_rcpf((float)(1.0 + k.q));
  const float den = (float)(k.r2 * k.b2);
  float raw[5];
  raw[0] = ((float)ex + __log2f((float)man)) * kLog10_2;
  raw[1] = log1pf((float)k.q) * 0.43429448190325182f;   // log10(1 + q)
  raw[2] = __builtin_sqrtf((float)k.r2) * iq1;
  raw[3] = (float)k.b2 * iq1;
  raw[4] = den > 1e-30f ? fminf((float)(k.s * k.s) * __builtin_amdgcn_rcpf(den), 1.0f) : 0.0f;
#pragma unroll
  for (int c = 0; c < 5; ++c) x[c] = (raw[c] - f.mean[c]) * f.scale[c];
}

__device__ __forceinline__ void load_metric(const P6& gm, int64_t t, M3& m) {
  metric_build(m, gm.p[0][t], gm.p[1][t], gm.p[2][t], gm.p[3][t], gm.p[4][t], gm.p[5][t]);
}

// bracket [lo, hi] of mu from the network outputs: logistic(y0 -/+ half),
// half = k exp(y1) + delta_min (exponentials in fp32, the logistic's division
// in FP64 so that brackets near mu = 1 stay distinct)
__device__ __forceinline__ void bracket_of(float y0, float y1, float width_k, float width_min,
                                           double& lo, double& hi) {
  const float half = width_k * __expf(fminf(y1, 30.0f)) + width_min;
  lo = 1.0 / (1.0 + (double)__expf(-(y0 - half)));
  hi = 1.0 / (1.0 + (double)__expf(-(y0 + half)));
}

// Persistent wave loop: wave w of the grid handles states [64 w', 64 w' + 64)
// for w' = w, w + (waves in grid), ...; the loop bound is wave-uniform so
// that every lane reaches the MFMA chain.
struct WaveLoop {
  int64_t first, stride;
  __device__ WaveLoop() {
    const int wpb = blockDim.x >> 6;
    first = ((int64_t)blockIdx.x * wpb + (threadIdx.x >> 6)) * 64;
    stride = (int64_t)gridDim.x * wpb * 64;
  }
};

// ---------------------------------------------------------------------------
// inversion with the learned bracket, fused: per wave, the conserved-floor
// rules and features in FP64, the network on the MFMA units (activations in
// registers), then the FP64 bracketed root solve
// ---------------------------------------------------------------------------
template <int ET>
__global__ __launch_bounds__(kT) void k_c2p_learned(int64_t n, P5 u, P3 bt, P6 gm, P5 wout,
                                                    uint16_t* flags, Eos e_in, grmhd_params p_in,
                                                    const uint16_t* wh, const float* wf, Feat ft,
                                                    float width_k, float width_min, double* mu_out,
                                                    int32_t* nev_out, c2p_stats* stats) {
  const Eos e0 = eos_fixed<ET>(e_in);
  const grmhd_params p0 = p_in;
  __shared__ MlpLds s;
  mlp_load(s, wh, wf);
  __syncthreads();
  const int l = threadIdx.x & 63;
  unsigned long long c_solves = 0, c_nev = 0, c_fb = 0, c_fail = 0;
  const WaveLoop wl;
  for (int64_t base = wl.first; base < n; base += wl.stride) {
    const int64_t t = base + l;
    const bool live = t < n;
    Eos e = e0;
    grmhd_params p = p0;
    consts_per_pass(e, p);
    double w[5];
    C2PWork cw;
    float x[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (live) {
      M3 m;
      double U[5], B[3];
      load_metric(gm, t, m);
#pragma unroll
      for (int v = 0; v < 5; ++v) U[v] = u.p[v][t];
#pragma unroll
      for (int v = 0; v < 3; ++v) B[v] = bt.p[v][t];
      cw = c2p_prepare(e, p, m, U, B, w);
      if (cw.done) {
#pragma unroll
        for (int v = 0; v < 5; ++v) u.p[v][t] = U[v];
      } else {
        features(cw.k, ft, x);
      }
    } else {
      cw.done = true;
      cw.fl = 0;
    }
    float y0, y1;
    mlp_wave(s, x, y0, y1);
    if (live) {
      uint32_t r = cw.fl;
      int nev = 0;
      double mu = 0.0;
      if (!cw.done) {
        double lo, hi;
        bracket_of(y0, y1, width_k, width_min, lo, hi);
        r = c2p_lean(e, p, cw, w, true, lo, hi, nev, mu);
        if (r & kFloorBits) {
          // U from the final primitives, metric and field loaded again
          __asm__ volatile("" ::: "memory");
          M3 m;
          load_metric(gm, t, m);
          const double B[3] = {bt.p[0][t], bt.p[1][t], bt.p[2][t]};
          double U[5];
          prim_to_cons(e, m, w, B, U);
#pragma unroll
          for (int v = 0; v < 5; ++v) u.p[v][t] = U[v];
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) wout.p[v][t] = w[v];
      flags[t] = (uint16_t)r;
      if (mu_out) mu_out[t] = mu;
      if (nev_out) nev_out[t] = nev;
      c_solves += 1;
      c_nev += (unsigned long long)nev;
      c_fb += (r & GRMHD_F_BRACKET_FALLBACK) ? 1 : 0;
      c_fail += (r & GRMHD_F_C2P_FAIL) ? 1 : 0;
    }
  }
  if (stats) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      c_solves += __shfl_xor(c_solves, o, 64);
      c_nev += __shfl_xor(c_nev, o, 64);
      c_fb += __shfl_xor(c_fb, o, 64);
      c_fail += __shfl_xor(c_fail, o, 64);
    }
    if (l == 0) {
      atomicAdd(&stats->solves, c_solves);
      atomicAdd(&stats->evaluations, c_nev);
      atomicAdd(&stats->fallbacks, c_fb);
      atomicAdd(&stats->failures, c_fail);
    }
  }
}

// ---------------------------------------------------------------------------
// the network alone: bracket [lo, hi] of every state into br[0..n), br[n..2n)
// (states that an atmosphere rule settles get an empty bracket)
// ---------------------------------------------------------------------------
template <int ET>
__global__ __launch_bounds__(kT) void k_mlp_bracket(int64_t n, P5 u, P3 bt, P6 gm, Eos e_in,
                                                    grmhd_params p, const uint16_t* wh,
                                                    const float* wf, Feat ft, float width_k,
                                                    float width_min, double* br) {
  const Eos e = eos_fixed<ET>(e_in);
  __shared__ MlpLds s;
  mlp_load(s, wh, wf);
  __syncthreads();
  const int l = threadIdx.x & 63;
  const WaveLoop wl;
  for (int64_t base = wl.first; base < n; base += wl.stride) {
    const int64_t t = base + l;
    float x[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    bool done = true;
    if (t < n) {
      M3 m;
      load_metric(gm, t, m);
      double U[5], B[3], w[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) U[v] = u.p[v][t];
#pragma unroll
      for (int v = 0; v < 3; ++v) B[v] = bt.p[v][t];
      const C2PWork cw = c2p_prepare(e, p, m, U, B, w);
      done = cw.done;
      if (!done) features(cw.k, ft, x);
    }
    float y0, y1;
    mlp_wave(s, x, y0, y1);
    if (t < n) {
      double lo = 0.0, hi = 0.0;
      if (!done) bracket_of(y0, y1, width_k, width_min, lo, hi);
      br[t] = lo;
      br[n + t] = hi;
    }
  }
}

// ---------------------------------------------------------------------------
// a8 with the learned bracket: the stage's inversion over the interior cells
// of every block (flattened wave layout).  Lanes without a cell still run the
// network with their wave; the root solve, the atmosphere rules and the
// flags are those of the plain stage inversion.
// ---------------------------------------------------------------------------
template <int ET>
__global__ __launch_bounds__(kT) void k_stage_c2p_learned(const grmhd_block* __restrict__ blks,
                                                          Eos e_in, grmhd_params p,
                                                          const uint16_t* wh, const float* wf,
                                                          Feat ft, float width_k, float width_min,
                                                          c2p_stats* stats) {
  const Eos e = eos_fixed<ET>(e_in);
  __shared__ MlpLds s;
  mlp_load(s, wh, wf);
  __syncthreads();
  int bi = 0;
  int64_t t = 0;
  const bool live = locate(blks, S_INTERIOR, bi, t);
  const GB b = gview(blks[bi]);
  const Geo q = geo_of(b);
  int i = 0, j = 0, k = 0;
  int64_t c = 0;
  double w[5];
  C2PWork cw;
  cw.done = true;
  cw.fl = 0;
  float x[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (live) {
    interior_box(q).at(t, i, j, k);
    c = cell(q, i, j, k);
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
    } else {
      features(cw.k, ft, x);
    }
  }
  float y0, y1;
  mlp_wave(s, x, y0, y1);
  unsigned long long c_n = 0, c_ev = 0, c_fb = 0, c_fail = 0;
  if (live) {
    uint32_t r = cw.fl;
    int nev = 0;
    if (!cw.done) {
      double lo, hi, mu;
      bracket_of(y0, y1, width_k, width_min, lo, hi);
      r = c2p_lean(e, p, cw, w, true, lo, hi, nev, mu);
      if (r & kFloorBits) {
        // U from the final primitives, metric and field loaded again
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
    c_fb = (r & GRMHD_F_BRACKET_FALLBACK) ? 1 : 0;
    c_fail = (r & GRMHD_F_C2P_FAIL) ? 1 : 0;
  }
  // per-wave sums into the block's scratch, summed by the stats reduction
  if (stats && __shfl((int)live, 0, 64)) wave_stats_store(b, q, t, c_n, c_ev, c_fb, c_fail);
}

// ---------------------------------------------------------------------------
// training data: standardised features of conserved states (after the
// conserved-floor rules) and the target logit(mu*), mu* = 1/(h W) of the
// primitives that generated the state
// ---------------------------------------------------------------------------
template <int ET>
__global__ __launch_bounds__(kT) void k_mlp_features(int64_t n, P5 u, P3 bt, P6 gm, P5 wtrue,
                                                     int has_target, Eos e_in, grmhd_params p, Feat ft,
                                                     float* feats, float* target) {
  const Eos e = eos_fixed<ET>(e_in);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  M3 m;
  load_metric(gm, t, m);
  double U[5], B[3], w[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) U[v] = u.p[v][t];
#pragma unroll
  for (int v = 0; v < 3; ++v) B[v] = bt.p[v][t];
  C2PWork cw = c2p_prepare(e, p, m, U, B, w);
  float x[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (!cw.done) features(cw.k, ft, x);
#pragma unroll
  for (int c = 0; c < 5; ++c) feats[c * n + t] = x[c];
  if (has_target) {
    const double rho = wtrue.p[0][t], P = wtrue.p[4][t];
    double ul[3];
    lower(m.g, wtrue.p[1][t], wtrue.p[2][t], wtrue.p[3][t], ul[0], ul[1], ul[2]);
    const double W = sqrt(1.0 + wtrue.p[1][t] * ul[0] + wtrue.p[2][t] * ul[1] + wtrue.p[3][t] * ul[2]);
    const double h = 1.0 + eos_eps_from_P(e, rho, P) + P / rho;
    const double mu = 1.0 / (h * W);
    target[t] = (float)log(mu / (1.0 - mu));
  }
}

// ---------------------------------------------------------------------------
// forward only (n states, standardised features [5][n]) -> y [2][n]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_mlp_forward(int64_t n, const float* feats, float* y,
                                                    const uint16_t* wh, const float* wf) {
  __shared__ MlpLds s;
  mlp_load(s, wh, wf);
  __syncthreads();
  const int l = threadIdx.x & 63;
  const WaveLoop wl;
  for (int64_t base = wl.first; base < n; base += wl.stride) {
    const int64_t t = base + l;
    float x[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) x[c] = t < n ? feats[c * n + t] : 0.f;
    float y0, y1;
    mlp_wave(s, x, y0, y1);
    if (t < n) {
      y[t] = y0;
      y[n + t] = y1;
    }
  }
}

// |y0 - target| / exp(y1): the bracket half-width, in units of the network's
// own error estimate, that the label needs (y1 clamped at 30)
__global__ __launch_bounds__(kT) void k_width_ratio(int64_t n, const float* y, const float* target,
                                                    float* ratio) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  ratio[t] = fabsf(y[t] - target[t]) / expf(fminf(y[n + t], 30.0f));
}

// ---------------------------------------------------------------------------
// training: one wave per workgroup runs forward + backward on 64 samples and
// writes its partial gradient (fp32, parameter layout) to partial[wg]
// ---------------------------------------------------------------------------
struct TrainLds {
  MlpLds w;
  uint16_t x0[64 * kLdIn];
  uint16_t h[3][64 * kLdH];     // h1, h2, h3 (bf16)
  float d[3][64 * 64];          // act'(z_l), then the fp32 gradient g_l in place
  uint16_t ga[64 * kLdH];       // bf16 copies of g_l for the MFMA (ping-pong)
  uint16_t gb[64 * kLdH];
  float y[64 * 2];
  float dy[64 * 2];
};

// dW[o][i] = sum_r G[r][o] X[r][i] over the 64 rows (M = o, N = i, K = r)
template <int NT>
__device__ __forceinline__ void grad_w(const uint16_t* G, const uint16_t* X, int ldx, float* out,
                                       int in_dim) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
#pragma unroll 1
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll 1
    for (int nt = 0; nt < NT; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        // A[o][k] = G[k][o], B[k][i] = X[k][i]
        const bf16x4 a = ld4s(G + (ks * 16 + 4 * q) * kLdH + mt * 16 + r, kLdH);
        const bf16x4 b = ld4s(X + (ks * 16 + 4 * q) * ldx + nt * 16 + r, ldx);
        acc = mfma16(a, b, acc);
      }
      const int i = nt * 16 + r;
      if (i < in_dim) {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[(mt * 16 + 4 * q + e) * in_dim + i] = acc[e];
      }
    }
}

// dX[r][i] = sum_o G[r][o] W[o][i] (M = r, N = i, K = o), times act'(z) in
// place into d (fp32), bf16 copy into gnext
__device__ __forceinline__ void grad_x(const uint16_t* G, const uint16_t* W, float* d,
                                       uint16_t* gnext) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
#pragma unroll 1
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bf16x4 a = ld4(G + (mt * 16 + r) * kLdH + ks * 16 + 4 * q);
        const bf16x4 b = ld4s(W + (ks * 16 + 4 * q) * kLdH + nt * 16 + r, kLdH);
        acc = mfma16(a, b, acc);
      }
      const int col = nt * 16 + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = mt * 16 + 4 * q + e;
        const float g = acc[e] * d[row * 64 + col];
        d[row * 64 + col] = g;
        gnext[row * kLdH + col] = f2bf(g);
      }
    }
}

// column sums over the 64 rows of an fp32 [64][64] gradient -> bias gradient
__device__ __forceinline__ void grad_b(const float* d, float* out) {
  const int l = threadIdx.x & 63;
  float s = 0.f;
  for (int r = 0; r < 64; ++r) s += d[r * 64 + l];
  out[l] = s;
}

__global__ __launch_bounds__(64) void k_mlp_train(int64_t nbatch, const float* feats,
                                                  const float* target, const uint16_t* wh,
                                                  const float* wf, float* partial, float* loss_part) {
  __shared__ TrainLds s;
  mlp_load(s.w, wh, wf);
  const int l = threadIdx.x;
  const int64_t t = (int64_t)blockIdx.x * 64 + l;
  float* pg = partial + (int64_t)blockIdx.x * kNParam;
  // inputs
#pragma unroll
  for (int c = 0; c < 16; ++c) s.x0[l * kLdIn + c] = c < 5 ? f2bf(feats[c * nbatch + t]) : (uint16_t)0;
  __syncthreads();
  // forward, keeping act'(z) for each hidden layer
#pragma unroll 1
  for (int mt = 0; mt < 4; ++mt) {
    mlp_hidden<1>(s.x0 + mt * 16 * kLdIn, kLdIn, s.w.W1, kLdIn, s.w.b1, s.h[0] + mt * 16 * kLdH,
                  s.d[0] + mt * 16 * 64);
  }
  __syncthreads();
#pragma unroll 1
  for (int mt = 0; mt < 4; ++mt)
    mlp_hidden<4>(s.h[0] + mt * 16 * kLdH, kLdH, s.w.W2, kLdH, s.w.b2, s.h[1] + mt * 16 * kLdH,
                  s.d[1] + mt * 16 * 64);
  __syncthreads();
#pragma unroll 1
  for (int mt = 0; mt < 4; ++mt)
    mlp_hidden<4>(s.h[1] + mt * 16 * kLdH, kLdH, s.w.W3, kLdH, s.w.b3, s.h[2] + mt * 16 * kLdH,
                  s.d[2] + mt * 16 * 64);
  __syncthreads();
#pragma unroll 1
  for (int mt = 0; mt < 4; ++mt) mlp_out(s.h[2] + mt * 16 * kLdH, s.w.W4, s.w.b4, s.y + mt * 32);
  __syncthreads();
  // loss 0.5 (y0 - t)^2 + 0.5 (y1 - log(|y0 - t| + c))^2, averaged over the batch
  {
    const float tg = target[t];
    const float e0 = s.y[l * 2] - tg;
    const float t1 = logf(fabsf(e0) + 1e-4f);
    const float e1 = s.y[l * 2 + 1] - t1;
    const float inv = 1.0f / (float)nbatch;
    s.dy[l * 2] = e0 * inv;
    s.dy[l * 2 + 1] = e1 * inv;
    float ls = 0.5f * (e0 * e0 + e1 * e1) * inv;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) ls += __shfl_xor(ls, o, 64);
    if (l == 0 && loss_part) loss_part[blockIdx.x] = ls;
  }
  __syncthreads();
  // output layer in fp32 (two outputs): dW4, db4 and dh3 = dy0 W4[0], g3 = dh3 * act'(z3)
  {
    // dW4[o][i] = sum_r dy[r][o] h3[r][i]; lane l owns column i = l
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
    for (int r = 0; r < 64; ++r) {
      const float hv = bf2f(s.h[2][r * kLdH + l]);
      a0 += s.dy[r * 2] * hv;
      a1 += s.dy[r * 2 + 1] * hv;
    }
    pg[kOffW4 + l] = a0;
    pg[kOffW4 + 64 + l] = a1;
    if (l == 0) {
      for (int r = 0; r < 64; ++r) { b0 += s.dy[r * 2]; b1 += s.dy[r * 2 + 1]; }
      pg[kOffB4] = b0;
      pg[kOffB4 + 1] = b1;
    }
    // only the guess output trains the hidden layers: the error-scale output
    // is a linear read-out of the last hidden layer (its gradient stops there)
    const float w0 = bf2f(s.w.W4[0 * kLdH + l]);
    for (int r = 0; r < 64; ++r) {
      const float g = s.dy[r * 2] * w0 * s.d[2][r * 64 + l];
      s.d[2][r * 64 + l] = g;
      s.ga[r * kLdH + l] = f2bf(g);
    }
  }
  __syncthreads();
  // layer 3: dW3 = g3^T h2, db3, g2 = (g3 W3) * act'(z2)
  grad_w<4>(s.ga, s.h[1], kLdH, pg + kOffW3, 64);
  grad_b(s.d[2], pg + kOffB3);
  grad_x(s.ga, s.w.W3, s.d[1], s.gb);
  __syncthreads();
  // layer 2
  grad_w<4>(s.gb, s.h[0], kLdH, pg + kOffW2, 64);
  grad_b(s.d[1], pg + kOffB2);
  grad_x(s.gb, s.w.W2, s.d[0], s.ga);
  __syncthreads();
  // layer 1 (5 inputs)
  grad_w<1>(s.ga, s.x0, kLdIn, pg + kOffW1, 5);
  grad_b(s.d[0], pg + kOffB1);
}

// deterministic reduction of the partial gradients (fixed order) and Adam
__global__ __launch_bounds__(kT) void k_mlp_adam(int nwg, const float* partial, float* theta,
                                                 float* m1, float* m2, uint16_t* theta_h, float lr,
                                                 float c1, float c2, int apply, float* grad_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= kNParam) return;
  float g = 0.f;
  for (int w = 0; w < nwg; ++w) g += partial[(int64_t)w * kNParam + x];
  if (grad_out) grad_out[x] = g;
  if (!apply) return;
  // decay rates 0.9 and 0.999 with their complements written out: 1.f - 0.999f
  // would be 1.3e-5 off 0.001 (0.999 is not exact in fp32)
  const float b1 = 0.9f, b2 = 0.999f, ob1 = 0.1f, ob2 = 0.001f, eps = 1e-8f;
  const float a = b1 * m1[x] + ob1 * g;
  const float v = b2 * m2[x] + ob2 * g * g;
  m1[x] = a;
  m2[x] = v;
  const float th = theta[x] - lr * (a / c1) / (sqrtf(v / c2) + eps);
  theta[x] = th;
  theta_h[x] = f2bf(th);
}

__global__ void k_sum_loss(int nwg, const float* loss_part, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < nwg; ++w) s += loss_part[w];
    loss[0] = s;
  }
}

__global__ void k_to_bf16(int n, const float* a, uint16_t* b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) b[x] = f2bf(a[x]);
}

int learned_err() { return hipGetLastError() == hipSuccess ? GRMHD_OK : GRMHD_EHIP; }

int fill_ptrs(double* const* a, int n, double** out) {
  if (!a) return GRMHD_EINVAL;
  for (int v = 0; v < n; ++v) {
    if (!a[v]) return GRMHD_EINVAL;
    out[v] = a[v];
  }
  return GRMHD_OK;
}

unsigned persistent_grid(int64_t n) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) == hipSuccess) cus = pr.multiProcessorCount;
  }
  const int64_t tiles = (n + kT - 1) / kT;
  const int64_t g = (int64_t)cus * 8;   // enough resident waves at any occupancy
  return (unsigned)(tiles < g ? tiles : g);
}

}  // namespace

namespace gk {
// the stage inversion with the learned bracket over every block's interior
int launch_stage_c2p_learned(const grmhd_block* h, const grmhd_block* d, int nblk,
                             const grmhd_params& p, const c2p_mlp* mlp, c2p_stats* stats,
                             hipStream_t s) {
  if (!mlp || !mlp->w_bf16 || !mlp->w_f32) return GRMHD_EINVAL;
  Feat ft;
  for (int c = 0; c < 5; ++c) { ft.mean[c] = mlp->feat_mean[c]; ft.scale[c] = mlp->feat_scale[c]; }
  const Eos e = make_eos_host(p);
  TIMED(T_STAGE_C2P_LEARNED, s);
  eos_dispatch(e.type, [&](auto et) {
    k_stage_c2p_learned<decltype(et)::value><<<stage_grid(h, nblk, S_INTERIOR, kT), kT, 0, s>>>(
        d, e, p, mlp->w_bf16, mlp->w_f32, ft, mlp->width_k, mlp->width_min, stats);
  });
  if (stats) launch_stats_sum(d, nblk, stats, s);
  return learned_err();
}
}  // namespace gk

extern "C" {

int c2p_batch_learned(int64_t n, double* u[5], double* const bt[3], double* const gam[6],
                      double* w[5], uint16_t* flags, const grmhd_params* p, const c2p_mlp* mlp,
                      c2p_stats* stats, double* mu_out, int32_t* nev_out, void* stream) {
  int r = check_params_host(p);
  if (r) return r;
  // an empty batch is valid whatever its (possibly NULL) pointers
  if (n < 0) return GRMHD_EINVAL;
  if (n == 0) return GRMHD_OK;
  if (!flags || !mlp || !mlp->w_bf16 || !mlp->w_f32) return GRMHD_EINVAL;
  P5 pu, pw;
  P3 pb;
  P6 pg;
  if (fill_ptrs(u, 5, pu.p) || fill_ptrs(w, 5, pw.p) || fill_ptrs(bt, 3, pb.p) || fill_ptrs(gam, 6, pg.p))
    return GRMHD_EINVAL;
  Feat ft;
  for (int c = 0; c < 5; ++c) { ft.mean[c] = mlp->feat_mean[c]; ft.scale[c] = mlp->feat_scale[c]; }
  if (mlp->bracket_ws) {
    // network as its own MFMA kernel, then the lean FP64 root kernel
    {
      TIMED(T_MLP_BRACKET, (hipStream_t)stream);
      const Eos e = make_eos_host(*p);
      eos_dispatch(e.type, [&](auto et) {
        k_mlp_bracket<decltype(et)::value><<<persistent_grid(n), kT, 0, (hipStream_t)stream>>>(
            n, pu, pb, pg, e, *p, mlp->w_bf16, mlp->w_f32, ft, mlp->width_k, mlp->width_min,
            mlp->bracket_ws);
      });
    }
    launch_c2p_batch(n, u, bt, gam, w, flags, *p, mlp->bracket_ws, mlp->bracket_ws + n, mu_out,
                     nev_out, stats, (hipStream_t)stream);
    return learned_err();
  }
  TIMED(T_C2P_LEARNED, (hipStream_t)stream);
  const Eos e = make_eos_host(*p);
  eos_dispatch(e.type, [&](auto et) {
    k_c2p_learned<decltype(et)::value><<<persistent_grid(n), kT, 0, (hipStream_t)stream>>>(
        n, pu, pb, pg, pw, flags, e, *p, mlp->w_bf16, mlp->w_f32, ft, mlp->width_k,
        mlp->width_min, mu_out, nev_out, stats);
  });
  return learned_err();
}

int c2p_mlp_features(int64_t n, double* const u[5], double* const bt[3], double* const gam[6],
                     double* const w_true[5], const grmhd_params* p, const float mean[5],
                     const float scale[5], float* feats, float* target, void* stream) {
  int r = check_params_host(p);
  if (r) return r;
  if (n < 1 || !feats || !mean || !scale || (w_true && !target)) return GRMHD_EINVAL;
  P5 pu, pw;
  P3 pb;
  P6 pg;
  if (fill_ptrs(u, 5, pu.p) || fill_ptrs(bt, 3, pb.p) || fill_ptrs(gam, 6, pg.p)) return GRMHD_EINVAL;
  if (w_true) {
    if (fill_ptrs(w_true, 5, pw.p)) return GRMHD_EINVAL;
  } else {
    for (int v = 0; v < 5; ++v) pw.p[v] = nullptr;
  }
  Feat ft;
  for (int c = 0; c < 5; ++c) { ft.mean[c] = mean[c]; ft.scale[c] = scale[c]; }
  const Eos e = make_eos_host(*p);
  eos_dispatch(e.type, [&](auto et) {
    k_mlp_features<decltype(et)::value><<<(unsigned)((n + kT - 1) / kT), kT, 0, (hipStream_t)stream>>>(
        n, pu, pb, pg, pw, w_true ? 1 : 0, e, *p, ft, feats, target);
  });
  return learned_err();
}

int c2p_mlp_forward(const c2p_mlp* mlp, int64_t n, const float* feats, float* y, void* stream) {
  if (!mlp || !mlp->w_bf16 || !mlp->w_f32 || n < 1 || !feats || !y) return GRMHD_EINVAL;
  k_mlp_forward<<<persistent_grid(n), kT, 0, (hipStream_t)stream>>>(n, feats, y, mlp->w_bf16,
                                                                    mlp->w_f32);
  return learned_err();
}

int c2p_mlp_calibrate_width(c2p_mlp* mlp, int64_t n, const float* feats, const float* target,
                            double q, float width_min, float* ws, void* stream) {
  if (!mlp || !mlp->w_bf16 || !mlp->w_f32 || n < 1 || !feats || !target || !ws || !(q > 0.0) ||
      !(q <= 1.0) || !(width_min >= 0.0f))
    return GRMHD_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  float* y = ws;
  float* ratio = ws + 2 * n;
  k_mlp_forward<<<persistent_grid(n), kT, 0, s>>>(n, feats, y, mlp->w_bf16, mlp->w_f32);
  k_width_ratio<<<(unsigned)((n + kT - 1) / kT), kT, 0, s>>>(n, y, target, ratio);
  if (hipGetLastError() != hipSuccess) return GRMHD_EHIP;
  // the q-quantile of the ratios: the order statistic at q (n - 1), linear
  // interpolation between its two neighbours (setup, not the hot path)
  std::vector<float> h((size_t)n);
  if (hipMemcpyAsync(h.data(), ratio, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return GRMHD_EHIP;
  const double pos = q * (double)(n - 1);
  const int64_t lo = (int64_t)pos;
  const int64_t hi = lo + 1 < n ? lo + 1 : lo;
  std::nth_element(h.begin(), h.begin() + lo, h.end());
  const double a = h[(size_t)lo];
  double b = a;
  if (hi != lo) b = *std::min_element(h.begin() + lo + 1, h.end());
  mlp->width_k = (float)(a + (pos - (double)lo) * (b - a));
  mlp->width_min = width_min;
  return GRMHD_OK;
}

int c2p_mlp_to_bf16(const float* theta, uint16_t* theta_bf16, void* stream) {
  if (!theta || !theta_bf16) return GRMHD_EINVAL;
  k_to_bf16<<<(kNParam + kT - 1) / kT, kT, 0, (hipStream_t)stream>>>(kNParam, theta, theta_bf16);
  return learned_err();
}

int c2p_mlp_train_step(float* theta, float* adam_m, float* adam_v, uint16_t* theta_bf16,
                       const float* feats, const float* target, int64_t nbatch, float lr,
                       int32_t step, float* partial, float* loss_part, float* loss_out,
                       float* grad_out, void* stream) {
  if (!theta || !theta_bf16 || !feats || !target || !partial || nbatch < 64 || (nbatch % 64))
    return GRMHD_EINVAL;
  const int apply = step > 0;
  if (apply && (!adam_m || !adam_v)) return GRMHD_EINVAL;
  const int nwg = (int)(nbatch / 64);
  hipStream_t s = (hipStream_t)stream;
  TIMED(T_MLP_TRAIN, s);
  k_mlp_train<<<nwg, 64, 0, s>>>(nbatch, feats, target, theta_bf16, theta, partial, loss_part);
  // bias corrections 1 - 0.9^t and 1 - 0.999^t in double, then rounded once
  const float c1 = apply ? (float)(1.0 - pow(0.9, (double)step)) : 1.f;
  const float c2 = apply ? (float)(1.0 - pow(0.999, (double)step)) : 1.f;
  k_mlp_adam<<<(kNParam + kT - 1) / kT, kT, 0, s>>>(nwg, partial, theta, adam_m, adam_v, theta_bf16,
                                                   lr, c1, c2, apply, grad_out);
  if (loss_part && loss_out) k_sum_loss<<<1, 64, 0, s>>>(nwg, loss_part, loss_out);
  return learned_err();
}

}  // extern "C"
