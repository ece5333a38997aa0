// mlp.hpp -- the learned star-pressure guess: a 6 -> 32 -> 32 -> 1 network
// with ReLU activations, BF16 weights and activations on the MFMA units,
// FP32 accumulation.  One wave evaluates 64 samples (one per lane).
//
// Features of an interface (all dimensionless, FP32):
//   a = ln(rho_L / rho_bar), b = ln(p_L / p_bar), w = asinh((u_L - u_bar) / c_bar)
//   x = (a, b, w, -a, -b, -w)
// with rho_bar = sqrt(rho_L rho_R), p_bar = sqrt(p_L p_R), u_bar = (u_L+u_R)/2,
// c_bar = sqrt(gamma p_bar / rho_bar); the second triple is the right
// state's (ln rho_R/rho_bar = -a, ...).  asinh keeps strong velocity jumps
// (|u_L - u_R| >> c_bar) on the logarithmic scale of the other two features.  Target y = ln(p* / p_bar); guess
// p_bar exp(y).
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

// Features of one interface (FP32) and ln(p_bar).
template <typename T>
__device__ __forceinline__ void mlp_features(const Prim<T>& L, const Prim<T>& R, float gamma,
                                             float x[6], float& lpbar) {
  const float l2rl = fm::log2((float)L.r), l2rr = fm::log2((float)R.r);
  const float l2pl = fm::log2((float)L.p), l2pr = fm::log2((float)R.p);
  const float ln2 = 0.69314718055994531f;
  const float a = 0.5f * (l2rl - l2rr) * ln2;
  const float b = 0.5f * (l2pl - l2pr) * ln2;
  // c_bar = sqrt(gamma p_bar / rho_bar) = 2^(0.5 log2 gamma + 0.25 (log2 pL pR - log2 rL rR))
  const float l2c = 0.5f * fm::log2(gamma) + 0.25f * ((l2pl + l2pr) - (l2rl + l2rr));
  const float w = mlp_asinh(0.5f * ((float)L.u - (float)R.u) * fm::exp2(-l2c));
  x[0] = a;
  x[1] = b;
  x[2] = w;
  x[3] = -a;
  x[4] = -b;
  x[5] = -w;
  lpbar = 0.5f * (l2pl + l2pr) * ln2;
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
      mlp_v4f c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r.w1[m], b1op, c, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float z = c[e] + r.b1[4 * m + e];
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
      mlp_v4f c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(r.w2[m], b2op[t], c, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float z = c[e] + r.b2[4 * m + e];
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
// one 16-sample tile at a time.  Each tile re-reads its weight fragments
// (6 KB, cache-resident) through one wave-uniform base and three lane
// offsets, so the branch that evaluates the network keeps few registers live
// next to the sweep's own state.  Must be called by all 64 lanes.
__device__ __forceinline__ float mlp_infer(const MlpDev* __restrict__ m, const float x[6]) {
  const int l = threadIdx.x & 63, g = l >> 4, col = l & 15;
  const char* base = reinterpret_cast<const char*>(m);
  float y = 0.0f;
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    unsigned ow1 = (unsigned)(offsetof(MlpDev, w1) + col * 32 + g * 8);   // w1[col][4g]
    unsigned ow2 = (unsigned)(offsetof(MlpDev, w2p) + col * 64 + g * 16); // w2p[col][8g]
    unsigned ov = (unsigned)(g * 16);                                    // b1/b2/w3[4g]
    // opaque to the optimiser: the loads below stay in the tile loop rather
    // than being hoisted and held across all four tiles
    __asm__("" : "+v"(ow1), "+v"(ow2), "+v"(ov));
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
    mlp_v8bf b2op;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const mlp_v4s w1 = *reinterpret_cast<const mlp_v4s*>(base + ow1 + mt * 16 * 32);
      const mlp_v4f b1 =
          *reinterpret_cast<const mlp_v4f*>(base + offsetof(MlpDev, b1) + ov + mt * 64);
      mlp_v4f c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1, b1op, c, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        b2op[4 * mt + e] = __builtin_bit_cast(__bf16, bf16_bits(fmaxf(c[e] + b1[e], 0.0f)));
    }
    float s = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const mlp_v8bf w2 = *reinterpret_cast<const mlp_v8bf*>(base + ow2 + mt * 16 * 64);
      const mlp_v4f b2 =
          *reinterpret_cast<const mlp_v4f*>(base + offsetof(MlpDev, b2) + ov + mt * 64);
      const mlp_v4f w3 =
          *reinterpret_cast<const mlp_v4f*>(base + offsetof(MlpDev, w3) + ov + mt * 64);
      mlp_v4f c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2, b2op, c, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) s = fmaf(w3[e], fmaxf(c[e] + b2[e], 0.0f), s);
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

// Starting guess of this lane's Riemann problem: 0 when the strength test
// keeps the two-rarefaction guess, the network's p* otherwise, or -1 when the
// network is invalid or its output is not a finite positive pressure.  A wave
// evaluates the network only if one of its lanes passes the test (the branch
// is wave-uniform).  Must be called by all 64 lanes.
template <typename T>
__device__ __forceinline__ T learned_guess(const MlpDev* m, const Prim<T>& L, const Prim<T>& R,
                                          float gamma, float kappa, float theta2) {
  const bool want = learned_wanted(L, R, gamma, kappa, theta2);
  if (__ballot(want) == 0ull) return T(0);
  float x[6], lpbar;
  mlp_features(L, R, gamma, x, lpbar);
  const float y = mlp_infer(m, x);
  const float p = fm::exp2((y + lpbar) * 1.4426950408889634f);
  if (!want) return T(0);
  return (m->valid && p > 0.0f && p < INFINITY) ? T(p) : T(-1);
}

}  // namespace hydro
