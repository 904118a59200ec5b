// mlp.hpp -- device pieces of the learned C2P guess network (not in the paper):
// a 5-64-64-64-2 perceptron with hard-swish activations, bf16 operands on the MFMA units with
// fp32 accumulation.
//
// Parameter vector (fp32 master copy and bf16 copy share this layout):
//   W1 [64][5] | b1 [64] | W2 [64][64] | b2 [64] | W3 [64][64] | b3 [64] |
//   W4 [2][64] | b4 [2]                         (8834 values, row-major [out][in])
//
// MFMA v_mfma_f32_16x16x16_bf16 fragments (64 lanes, lane l, e = 0..3):
//   A (16x16, rows x k):  A[l % 16][4 (l / 16) + e]
//   B (16x16, k x cols):  B[4 (l / 16) + e][l % 16]
//   D (16x16, rows x cols): D[4 (l / 16) + e][l % 16]
// The inference pass takes its 64-deep layers in 32-deep steps of
// v_mfma_f32_16x16x32_bf16 (8 bf16 of A and of B per lane, same D fragment):
// a lane's 8 k-slots are the same in A and B, so which neuron sits in which
// slot is free as long as both operands agree.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kOffW1 = 0, kOffB1 = 320, kOffW2 = 384, kOffB2 = 4480, kOffW3 = 4544, kOffB3 = 8640,
              kOffW4 = 8704, kOffB4 = 8832, kNParam = 8834;

// LDS strides (bf16 elements) chosen to spread rows over the LDS banks
constexpr int kLdIn = 24;   // input tile / W1: 16 used
constexpr int kLdH = 72;    // hidden activations / W2, W3, W4: 64 used

// fp32 -> bf16, round to nearest even (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// hard-swish activation (Howard et al. 2019), z clamp(z / 6 + 1/2, 0, 1):
// one fused multiply-add with a clamp to [0, 1] and one multiply, where a
// logistic-based activation needs an exponential and a reciprocal (quarter
// rate) per neuron, which would cost several times the matrix products
__device__ __forceinline__ float act_f(float z) {
  return z * __builtin_amdgcn_fmed3f(fmaf(z, 1.0f / 6.0f, 0.5f), 0.0f, 1.0f);
}
__device__ __forceinline__ float dact_f(float z) {
  return z <= -3.0f ? 0.0f : (z >= 3.0f ? 1.0f : fmaf(z, 1.0f / 3.0f, 0.5f));
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// contiguous 4 bf16 (8 bytes) from LDS
__device__ __forceinline__ bf16x4 ld4(const uint16_t* p) { return *(const bf16x4*)p; }
// 4 bf16 at stride ld
__device__ __forceinline__ bf16x4 ld4s(const uint16_t* p, int ld) {
  bf16x4 r;
  r[0] = (short)p[0];
  r[1] = (short)p[ld];
  r[2] = (short)p[2 * ld];
  r[3] = (short)p[3 * ld];
  return r;
}

// Shared weights of one workgroup in LDS
struct MlpLds {
  uint16_t W1[64 * kLdIn];
  uint16_t W2[64 * kLdH];
  uint16_t W3[64 * kLdH];
  uint16_t W4[16 * kLdH];
  alignas(16) float b1[64];
  alignas(16) float b2[64];
  alignas(16) float b3[64];
  alignas(16) float b4[4];
};

// cooperative load of the bf16 weights (padded) and fp32 biases into LDS
__device__ __forceinline__ void mlp_load(MlpLds& s, const uint16_t* wh, const float* wf) {
  for (int x = threadIdx.x; x < 64 * kLdIn; x += blockDim.x) {
    const int o = x / kLdIn, i = x % kLdIn;
    s.W1[x] = i < 5 ? wh[kOffW1 + o * 5 + i] : (uint16_t)0;
  }
  for (int x = threadIdx.x; x < 64 * kLdH; x += blockDim.x) {
    const int o = x / kLdH, i = x % kLdH;
    s.W2[x] = i < 64 ? wh[kOffW2 + o * 64 + i] : (uint16_t)0;
    s.W3[x] = i < 64 ? wh[kOffW3 + o * 64 + i] : (uint16_t)0;
  }
  for (int x = threadIdx.x; x < 16 * kLdH; x += blockDim.x) {
    const int o = x / kLdH, i = x % kLdH;
    s.W4[x] = (o < 2 && i < 64) ? wh[kOffW4 + o * 64 + i] : (uint16_t)0;
  }
  for (int x = threadIdx.x; x < 64; x += blockDim.x) {
    s.b1[x] = wf[kOffB1 + x];
    s.b2[x] = wf[kOffB2 + x];
    s.b3[x] = wf[kOffB3 + x];
  }
  if (threadIdx.x < 2) s.b4[threadIdx.x] = wf[kOffB4 + threadIdx.x];
}

// One hidden layer on a 16-row tile: out = act(in W^T + b), in [16][ld_in]
// with KT k-steps of 16, out [16][kLdH] (64 columns).  Optionally keeps the
// pre-activation derivative act'(z) (fp32 [16][64]) for the backward pass.
template <int KT>
__device__ __forceinline__ void mlp_hidden(const uint16_t* in, int ld_in, const uint16_t* W, int ldw,
                                           const float* bias, uint16_t* out, float* dz) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) {
      const bf16x4 a = ld4(in + r * ld_in + ks * 16 + 4 * q);
      const bf16x4 b = ld4(W + (nt * 16 + r) * ldw + ks * 16 + 4 * q);
      acc = mfma16(a, b, acc);
    }
    const int col = nt * 16 + r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 4 * q + e;
      const float z = acc[e] + bias[col];
      out[row * kLdH + col] = f2bf(act_f(z));
      if (dz) dz[row * 64 + col] = dact_f(z);
    }
  }
}

// Output layer on a 16-row tile: y[16][2] (fp32) = in W4^T + b4
__device__ __forceinline__ void mlp_out(const uint16_t* in, const uint16_t* W4, const float* b4,
                                        float* y) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const bf16x4 a = ld4(in + r * kLdH + ks * 16 + 4 * q);
    const bf16x4 b = ld4(W4 + r * kLdH + ks * 16 + 4 * q);
    acc = mfma16(a, b, acc);
  }
  if (r < 2) {
#pragma unroll
    for (int e = 0; e < 4; ++e) y[(4 * q + e) * 2 + r] = acc[e] + b4[r];
  }
}

// ---------------------------------------------------------------------------
// Register-resident forward pass of one wave over its 64 lanes' states.
//
// Each layer is computed transposed, H^T = W X^T, on 16-state tiles: the
// weights are the A operand (rows = output neurons), the previous layer's
// activations the B operand (k = input neuron, column = state).  The MFMA
// result D[4 (l / 16) + e][l % 16] (neuron, state) is then exactly the B
// fragment of the next layer's k-step, so activations never leave the
// registers.  A 32-deep step joins two such fragments: slots 0..3 of lane
// group q hold neurons 32 s + 4 q + e, slots 4..7 neurons 32 s + 16 + 4 q + e,
// and the weight fragment reads the same two column groups.  Lane l
// contributes its own state's 5 features x and receives (y0, y1) of its own
// state.  All 64 lanes must call this together.
// ---------------------------------------------------------------------------

// activation of an MFMA output fragment (bias already in the accumulator),
// packed to bf16 two values per conversion (one v_cvt_pk_bf16_f32 per pair;
// a 4-wide conversion is split by the compiler into one per value plus
// byte permutes)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  const f32x2 h = {act_f(a), act_f(b)};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(h, bf16x2v));
}
__device__ __forceinline__ bf16x4 act_frag(f32x4 acc) {
  const u32x2 r = {bf16_pair(acc[0], acc[1]), bf16_pair(acc[2], acc[3])};
  return __builtin_bit_cast(bf16x4, r);
}

// accumulator start: the biases of this lane's 4 fragment rows (neurons)
__device__ __forceinline__ f32x4 bias_frag(const float* bias) {
  return *(const f32x4*)bias;
}

typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
// two 4-wide fragments as the 8 k-slots of one 32-deep step
__device__ __forceinline__ bf16x8v cat8(bf16x4 a, bf16x4 b) {
  const s16x8 r = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
  return __builtin_bit_cast(bf16x8v, r);
}
// weight columns c + 0..3 and c + 16..19 of one row: the neurons of cat8
__device__ __forceinline__ bf16x8v ld8(const uint16_t* p) { return cat8(ld4(p), ld4(p + 16)); }
__device__ __forceinline__ f32x4 mfma32(bf16x8v a, bf16x8v b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16-state tiles that one pass of the forward runs side by side: all four
// of the wave's (four chains for the matrix cores; one and two were 9% and
// 3% slower in the fused inversion)
constexpr int kTilesPerPass = 4;

__device__ __forceinline__ void mlp_wave(const MlpLds& w, const float x[5], float& y0, float& y1) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
  y0 = 0.f;
  y1 = 0.f;
#pragma unroll 1
  for (int t0 = 0; t0 < 4; t0 += kTilesPerPass) {
    // keep the weight fragments in LDS: re-read them per pass instead of
    // letting them be hoisted into ~80 live VGPRs across the caller's loop
    __asm__ volatile("" ::: "memory");
    // independent 16-state tiles per pass share each weight fragment and
    // give the matrix cores as many dependency chains to interleave
    bf16x4 xb[kTilesPerPass];
#pragma unroll
    for (int u = 0; u < kTilesPerPass; ++u) {
      // B operand of layer 1: features 4q..4q+3 of state 16 (t0 + u) + r
      const int src = (t0 + u) * 16 + r;
      float f[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) f[c] = __shfl(x[c], src, 64);
      xb[u][0] = (short)(q == 0 ? f2bf(f[0]) : (q == 1 ? f2bf(f[4]) : 0));
      xb[u][1] = (short)(q == 0 ? f2bf(f[1]) : 0);
      xb[u][2] = (short)(q == 0 ? f2bf(f[2]) : 0);
      xb[u][3] = (short)(q == 0 ? f2bf(f[3]) : 0);
    }
    bf16x4 h1[kTilesPerPass][4], h2[kTilesPerPass][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 b0 = bias_frag(w.b1 + nt * 16 + 4 * q);
      const bf16x4 a = ld4(w.W1 + (nt * 16 + r) * kLdIn + 4 * q);
#pragma unroll
      for (int u = 0; u < kTilesPerPass; ++u) h1[u][nt] = act_frag(mfma16(a, xb[u], b0));
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 b0 = bias_frag(w.b2 + nt * 16 + 4 * q);
      f32x4 acc[kTilesPerPass];
#pragma unroll
      for (int u = 0; u < kTilesPerPass; ++u) acc[u] = b0;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const bf16x8v a = ld8(w.W2 + (nt * 16 + r) * kLdH + ks * 32 + 4 * q);
#pragma unroll
        for (int u = 0; u < kTilesPerPass; ++u)
          acc[u] = mfma32(a, cat8(h1[u][2 * ks], h1[u][2 * ks + 1]), acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kTilesPerPass; ++u) h2[u][nt] = act_frag(acc[u]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 b0 = bias_frag(w.b3 + nt * 16 + 4 * q);
      f32x4 acc[kTilesPerPass];
#pragma unroll
      for (int u = 0; u < kTilesPerPass; ++u) acc[u] = b0;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const bf16x8v a = ld8(w.W3 + (nt * 16 + r) * kLdH + ks * 32 + 4 * q);
#pragma unroll
        for (int u = 0; u < kTilesPerPass; ++u)
          acc[u] = mfma32(a, cat8(h2[u][2 * ks], h2[u][2 * ks + 1]), acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kTilesPerPass; ++u) h1[u][nt] = act_frag(acc[u]);
    }
    f32x4 acc[kTilesPerPass];
#pragma unroll
    for (int u = 0; u < kTilesPerPass; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const bf16x8v a = ld8(w.W4 + r * kLdH + ks * 32 + 4 * q);
#pragma unroll
      for (int u = 0; u < kTilesPerPass; ++u)
        acc[u] = mfma32(a, cat8(h1[u][2 * ks], h1[u][2 * ks + 1]), acc[u]);
    }
#pragma unroll
    for (int u = 0; u < kTilesPerPass; ++u) {
      // rows 0 and 1 (lanes 0..15, e = 0, 1) hold the two outputs of state 16 (t0 + u) + r
      const float o0 = __shfl(acc[u][0], r, 64), o1 = __shfl(acc[u][1], r, 64);
      if (q == t0 + u) {
        y0 = o0 + w.b4[0];
        y1 = o1 + w.b4[1];
      }
    }
  }
}

}  // namespace gk
