// mlp.hpp -- the learned star-pressure guess: a 6 -> 32 -> 32 -> 1 network
// with ReLU activations, BF16 weights and activations on the MFMA units,
// FP32 accumulation.  One wave evaluates 64 samples (one per lane).
//
// The network corrects the two-rarefaction guess p_ptr.  Features of an
// interface (all dimensionless, FP32):
//   a = ln(rho_L / rho_bar), b = ln(p_L / p_bar), w = asinh((u_L - u_bar) / c_bar),
//   q = ln(p_ptr / p_bar),   x = (a, b, w, q, -a, -b)
// with rho_bar = sqrt(rho_L rho_R), p_bar = sqrt(p_L p_R), u_bar = (u_L+u_R)/2,
// c_bar = sqrt(gamma p_bar / rho_bar) (-a, -b are the right state's
// ln rho_R/rho_bar, ln p_R/p_bar).  asinh keeps strong velocity jumps
// (|u_L - u_R| >> c_bar) on the logarithmic scale of the other features.
// Target y = ln(p* / p_ptr); guess p_ptr exp(y).  The correction is small
// where the two-rarefaction guess is good, so the network's BF16 rounding
// (about 1e-2 relative on its inputs) scales with the correction rather than
// with ln p* itself.
//
// Network (W row-major [out][in]; bf16() rounds to nearest even):
//   z1 = W1 bf16(x) + b1,  a1 = bf16(relu(z1))
//   z2 = W2 a1 + b2,       a2 = relu(z2)
//   y  = W3 . a2 + b3
// Layers 1 and 2 run as v_mfma_f32_16x16x16_bf16 / v_mfma_f32_16x16x32_bf16
// with samples as the N dimension.  In the result layout lane l holds units
// 16m + 4g + e (g = l/16, e = 0..3) of sample 16t + (l mod 16) for tiles
// m, t; the layer-2 contraction index is permuted so that these values are
// the B operand directly (no cross-lane traffic between layers).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "godunov.hpp"

namespace hydro {

constexpr int kMlpIn = 6;
constexpr int kMlpHidden = 32;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden + 1;  // 1313

// FP32 master parameters, flat: W1[32][6], b1[32], W2[32][32], b2[32], W3[32], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHidden * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden;

// Device-side packed network (bf16 bits in lane-ready orders).
struct MlpDev {
  unsigned short w1[32][16];   // W1[unit][feature], features >= 6 zero
  unsigned short w2p[32][32];  // W2[i][unit2(k')]: layer-2 rows, permuted K
  unsigned short w2tp[32][32]; // W2[unit2(k')][r]: transposed rows, permuted K
  float b1[32];
  float b2[32];
  float w3[32];                // bf16-rounded W3, widened
  float b3;
  int valid;                   // 0: weights absent / non-finite -> guess invalid
};

// The part of the packed network inference reads: layer-1 and layer-2 A
// operands, biases, output weights (3.4 KB).  A sweep kernel with the learned
// guess stages it in LDS once per block (mlp_stage), so the four sample tiles
// of a call read their weight fragments from LDS.
struct MlpInfer {
  unsigned short w1[32][16];
  unsigned short w2p[32][32];
  float b1[32];
  float b2[32];
  float w3[32];
  float b3;
  int valid;
};

// Block-wide copy of the inference part of the network into LDS; every
// thread of the block must call it (it ends with a barrier).
__device__ __forceinline__ void mlp_stage(const MlpDev* __restrict__ m, MlpInfer* s) {
  const unsigned* w1 = reinterpret_cast<const unsigned*>(m->w1);
  const unsigned* w2 = reinterpret_cast<const unsigned*>(m->w2p);
  unsigned* d1 = reinterpret_cast<unsigned*>(s->w1);
  unsigned* d2 = reinterpret_cast<unsigned*>(s->w2p);
  for (int i = threadIdx.x; i < 32 * 16 / 2; i += blockDim.x) d1[i] = w1[i];
  for (int i = threadIdx.x; i < 32 * 32 / 2; i += blockDim.x) d2[i] = w2[i];
  for (int i = threadIdx.x; i < 32; i += blockDim.x) {
    s->b1[i] = m->b1[i];
    s->b2[i] = m->b2[i];
    s->w3[i] = m->w3[i];
  }
  if (threadIdx.x == 0) {
    s->b3 = m->b3;
    s->valid = m->valid;
  }
  __syncthreads();
}

// Unit held at position k' = 8 g + e' of the permuted 32-wide K order.
__host__ __device__ inline int mlp_unit_of(int kp) {
  const int g = kp >> 3, e = kp & 7;
  return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4);
}

typedef short mlp_v4s __attribute__((ext_vector_type(4)));
typedef float mlp_v4f __attribute__((ext_vector_type(4)));
typedef __bf16 mlp_v8bf __attribute__((ext_vector_type(8)));

// round-to-nearest-even float -> bf16 bits
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) {
  return __uint_as_float(((unsigned)b) << 16);
}

// Per-lane copy of the weights a lane feeds to the MFMA units, loaded once.
struct MlpRegs {
  mlp_v4s w1[2];     // A operands of layer 1 (tiles m = 0, 1)
  mlp_v8bf w2[2];    // A operands of layer 2
  float b1[8], b2[8], w3[8];  // per held unit: index 4m + e -> unit 16m + 4g + e
  float b3;
  int valid;
};

__device__ __forceinline__ void mlp_load(const MlpDev* m, MlpRegs& r) {
  const int l = threadIdx.x & 63, g = l >> 4, row = l & 15;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
#pragma unroll
    for (int e = 0; e < 4; ++e) r.w1[t][e] = (short)m->w1[16 * t + row][4 * g + e];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      r.w2[t][e] = __builtin_bit_cast(__bf16, m->w2p[16 * t + row][8 * g + e]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      r.b1[4 * t + e] = m->b1[16 * t + 4 * g + e];
      r.b2[4 * t + e] = m->b2[16 * t + 4 * g + e];
      r.w3[4 * t + e] = m->w3[16 * t + 4 * g + e];
    }
  }
  r.b3 = m->b3;
  r.valid = m->valid;
}

// asinh in FP32: odd Taylor polynomial below 1/16 (truncation < 3e-9
// relative), ln(|w| + sqrt(w^2 + 1)) above, |w| capped at 1e18.
__device__ __forceinline__ float mlp_asinh(float w) {
  const float a = fminf(fabsf(w), 1e18f);
  const float a2 = a * a;
  const float small = a * (1.0f + a2 * (-1.0f / 6.0f + a2 * (3.0f / 40.0f)));
  const float large = fm::log2(a + fm::sqrt(a2 + 1.0f)) * 0.69314718055994531f;
  return copysignf(a < 0.0625f ? small : large, w);
}

// Features of one interface (FP32) from its states and the two-rarefaction
// guess p_ptr.
template <typename T>
__device__ __forceinline__ void mlp_features(const Prim<T>& L, const Prim<T>& R, T p_ptr,
                                             float gamma, float x[6]) {
  const float l2rl = fm::log2((float)L.r), l2rr = fm::log2((float)R.r);
  const float l2pl = fm::log2((float)L.p), l2pr = fm::log2((float)R.p);
  const float ln2 = 0.69314718055994531f;
  const float a = 0.5f * (l2rl - l2rr) * ln2;
  const float b = 0.5f * (l2pl - l2pr) * ln2;
  // c_bar = sqrt(gamma p_bar / rho_bar) = 2^(0.5 log2 gamma + 0.25 (log2 pL pR - log2 rL rR))
  const float l2c = 0.5f * fm::log2(gamma) + 0.25f * ((l2pl + l2pr) - (l2rl + l2rr));
  const float w = mlp_asinh(0.5f * ((float)L.u - (float)R.u) * fm::exp2(-l2c));
  const float q = (fm::log2((float)p_ptr) - 0.5f * (l2pl + l2pr)) * ln2;
  x[0] = a;
  x[1] = b;
  x[2] = w;
  x[3] = q;
  x[4] = -a;
  x[5] = -b;
}

// Layer outputs a lane keeps for the backward pass.
struct MlpAct {
  float z1[2][4][4];  // [m][t][e] pre-activation of layer 1 (bias included)
  float z2[2][4][4];
  mlp_v8bf a1[4];     // B operands of layer 2 (bf16 relu(z1)) per sample tile
  float y;            // own sample
};

// Whole-wave forward pass: lane l supplies the features of its sample and
// receives the network output for it.  Must be called by all 64 lanes.
template <bool KEEP>
__device__ __forceinline__ float mlp_forward(const MlpRegs& r, const float x[6], MlpAct* act) {
  const int l = threadIdx.x & 63, g = l >> 4, col = l & 15;
  // layer 1: B operand of sample tile t holds features 4g..4g+3 of sample 16t + col
  mlp_v8bf b2op[4];
  float z1k[2][4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int src = 16 * t + col;
    float v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = __shfl(x[k], src);
    mlp_v4s b1op;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float f = g == 0 ? v[e] : (g == 1 && e < 2 ? v[4 + e] : 0.0f);
      b1op[e] = (short)bf16_bits(f);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      // the bias is the accumulator's initial value
      mlp_v4f c = {r.b1[4 * m], r.b1[4 * m + 1], r.b1[4 * m + 2], r.b1[4 * m + 3]};
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r.w1[m], b1op, c, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float z = c[e];
        z1k[m][t][e] = z;
        b2op[t][4 * m + e] = __builtin_bit_cast(__bf16, bf16_bits(fmaxf(z, 0.0f)));
      }
    }
  }
  // layer 2 and the output dot product
  float py[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      mlp_v4f c = {r.b2[4 * m], r.b2[4 * m + 1], r.b2[4 * m + 2], r.b2[4 * m + 3]};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(r.w2[m], b2op[t], c, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float z = c[e];
        if (KEEP) act->z2[m][t][e] = z;
        s = fmaf(r.w3[4 * m + e], fmaxf(z, 0.0f), s);
      }
    }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    py[t] = s;
  }
  if (KEEP) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) act->z1[m][t][e] = z1k[m][t][e];
#pragma unroll
    for (int t = 0; t < 4; ++t) act->a1[t] = b2op[t];
  }
  const int own = l >> 4;
  float y = own == 0 ? py[0] : own == 1 ? py[1] : own == 2 ? py[2] : py[3];
  y += r.b3;
  if (KEEP) act->y = y;
  return y;
}

// Inference inside the sweeps: the same arithmetic as mlp_forward<false>,
// one 16-sample tile at a time, from the network staged in LDS.  Every lane
// packs its six features into three BF16 pairs once (v_cvt_pk_bf16_f32) and a
// tile's B operand takes them with three shuffles; biases enter as the MFMA
// accumulator's initial value; activations are packed the same way.  Each
// tile reads its weight fragments from LDS rather than holding all of them
// (36 registers) across the four tiles, so the branch that evaluates the
// network keeps few registers live next to the sweep's own state.  Must be
// called by all 64 lanes.
typedef unsigned mlp_v2u __attribute__((ext_vector_type(2)));
typedef __bf16 mlp_v2bf __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned mlp_pack2(float lo, float hi) {
  mlp_v2bf v;
  v[0] = (__bf16)lo;
  v[1] = (__bf16)hi;
  return __builtin_bit_cast(unsigned, v);
}

__device__ __forceinline__ float mlp_infer(const MlpInfer* m, const float x[6]) {
  const int l = threadIdx.x & 63, g = l >> 4, col = l & 15;
  const int p01 = (int)mlp_pack2(x[0], x[1]);
  const int p23 = (int)mlp_pack2(x[2], x[3]);
  const int p45 = (int)mlp_pack2(x[4], x[5]);
  float y = 0.0f;
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    // lane offsets of the weight fragments, opaque to the optimiser so that
    // the LDS reads stay in the tile loop instead of being hoisted and held
    // across all four tiles
    unsigned ow1 = (unsigned)(col * 16 + 4 * g), ow2 = (unsigned)(col * 32 + 8 * g);
    unsigned ov = (unsigned)(4 * g);
    __asm__("" : "+v"(ow1), "+v"(ow2), "+v"(ov));
    // B operand of layer 1: features 4g .. 4g+3 of sample 16t + col
    const int src = 16 * t + col;
    const int f01 = __shfl(p01, src), f23 = __shfl(p23, src), f45 = __shfl(p45, src);
    mlp_v2u bw;
    bw[0] = (unsigned)(g == 0 ? f01 : (g == 1 ? f45 : 0));
    bw[1] = (unsigned)(g == 0 ? f23 : 0);
    const mlp_v4s b1op = __builtin_bit_cast(mlp_v4s, bw);
    mlp_v8bf b2op;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const mlp_v4s w1 = *reinterpret_cast<const mlp_v4s*>(&m->w1[16 * mt][0] + ow1);
      const mlp_v4f b1 = *reinterpret_cast<const mlp_v4f*>(&m->b1[16 * mt] + ov);
      const mlp_v4f c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1, b1op, b1, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) b2op[4 * mt + e] = (__bf16)fmaxf(c[e], 0.0f);
    }
    float s = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const mlp_v8bf w2 = *reinterpret_cast<const mlp_v8bf*>(&m->w2p[16 * mt][0] + ow2);
      const mlp_v4f b2 = *reinterpret_cast<const mlp_v4f*>(&m->b2[16 * mt] + ov);
      const mlp_v4f w3 = *reinterpret_cast<const mlp_v4f*>(&m->w3[16 * mt] + ov);
      const mlp_v4f c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2, b2op, b2, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) s = fmaf(w3[e], fmaxf(c[e], 0.0f), s);
    }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == t) y = s;
  }
  return y + m->b3;
}

// Strength test of the learned guess: a pressure jump above the factor kappa
// or a velocity jump of the order of theta times the sound speed.  kappa = 0
// selects every interface.
template <typename T>
__device__ __forceinline__ bool learned_wanted(const Prim<T>& L, const Prim<T>& R, float gamma,
                                               float kappa, float theta2) {
  if (!(kappa > 0.0f)) return true;
  const float pl = (float)L.p, pr = (float)R.p;
  const float du = (float)(R.u - L.u);
  return fmaxf(pl, pr) > kappa * fminf(pl, pr) ||
         du * du * ((float)L.r + (float)R.r) > theta2 * gamma * (pl + pr);
}

// The learned starting guess, called by riemann_flux with the
// two-rarefaction guess p_ptr: 0 when the strength test keeps p_ptr, the
// network's correction p_ptr exp(y) otherwise, or -1 when the network is
// invalid or its guess is not a finite positive pressure.  A wave evaluates
// the network only if one of its lanes passes the test (the branch is
// wave-uniform).  Called by all 64 lanes.
struct LearnedGuess {
  static constexpr bool enabled = true;
  const MlpInfer* mlp;  // the network staged in LDS
  float gamma, kappa, theta2;
  template <typename T>
  __device__ __forceinline__ T operator()(const Prim<T>& L, const Prim<T>& R, T p_ptr) const {
    const bool want = learned_wanted(L, R, gamma, kappa, theta2);
    if (__ballot(want) == 0ull) return T(0);
    float x[6];
    mlp_features(L, R, p_ptr, gamma, x);
    const float y = mlp_infer(mlp, x);
    if (!want) return T(0);
    const float f = fm::exp2(y * 1.4426950408889634f);
    const T p = p_ptr * T(f);
    return (mlp->valid && f > 0.0f && p > T(0) && p < T(INFINITY)) ? p : T(-1);
  }
};

}  // namespace hydro
