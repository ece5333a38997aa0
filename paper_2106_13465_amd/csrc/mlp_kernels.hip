// mlp_kernels.hip -- training and evaluation kernels of the learned
// star-pressure guess (network in mlp.hpp).
//
// Loss over n samples: L = (1/n) sum_s (y_s - t_s)^2.  Backward, with the
// bf16 rounding points of the MFMA operands:
//   gy = 2 (y - t) / n;  gb3 = sum gy;  gW3 = sum gy a2
//   gz2 = gy W3 [z2 > 0];  gb2 = sum gz2;  gW2 = sum bf16(gz2) a1^T
//   ga1 = W2^T bf16(gz2);  gz1 = ga1 [z1 > 0];  gb1 = sum gz1
//   gW1 = sum bf16(gz1) bf16(x)^T
// ga1 runs on the MFMA units in the forward pass's register layout; the two
// weight gradients contract over samples, so each wave stages its 64 samples'
// bf16(gz2), a1, bf16(gz1) and bf16(x) in LDS (unit-major) and reads them back
// in MFMA operand order.  Each block adds its waves' gradients in LDS and
// writes one partial; a second kernel sums the partials in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_state.hpp"
#include "mlp.hpp"
#include "mlp_launch.hpp"
#include "plan.hpp"

namespace hydro {

namespace {

constexpr int kGradSlots = kMlpParams + 1;  // + loss

__global__ void k_mlp_pack(const float* __restrict__ p, MlpDev* m) {
  const int t = threadIdx.x;  // 1024 threads
  __shared__ int finite;
  if (t == 0) finite = 1;
  __syncthreads();
  for (int i = t; i < kMlpParams; i += blockDim.x)
    if (!(fabsf(p[i]) < INFINITY)) finite = 0;
  // W1 [32][6] -> w1 [32][16]
  for (int i = t; i < 32 * 16; i += blockDim.x) {
    const int u = i / 16, f = i % 16;
    m->w1[u][f] = f < kMlpIn ? bf16_bits(p[kOffW1 + u * kMlpIn + f]) : 0;
  }
  for (int i = t; i < 32 * 32; i += blockDim.x) {
    const int r = i / 32, kp = i % 32;
    m->w2p[r][kp] = bf16_bits(p[kOffW2 + r * 32 + mlp_unit_of(kp)]);   // W2[r][unit]
    m->w2tp[r][kp] = bf16_bits(p[kOffW2 + mlp_unit_of(kp) * 32 + r]);  // W2[unit][r]
  }
  for (int i = t; i < 32; i += blockDim.x) {
    m->b1[i] = p[kOffB1 + i];
    m->b2[i] = p[kOffB2 + i];
    m->w3[i] = bf16_float(bf16_bits(p[kOffW3 + i]));
  }
  __syncthreads();
  if (t == 0) {
    m->b3 = p[kOffB3];
    m->valid = finite;
  }
}

// records [n][8] (rho_L, u_L, p_L, rho_R, u_R, p_R, p*, strength) ->
// features X [n][6] and targets Y [n] = ln(p* / p_ptr), with the
// two-rarefaction guess p_ptr of the record's states in FP64 (the FP64
// sweep's arithmetic)
__global__ void k_mlp_features(const float* __restrict__ rec, long long n, Gas<double> G, float* X,
                               float* Y) {
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const float* r = rec + s * kLogFields;
    const Prim<double> L{r[0], r[1], 0.0, r[2]}, R{r[3], r[4], 0.0, r[5]};
    const double p_ptr = two_rarefaction_of(L, R, G);
    float x[6];
    mlp_features(L, R, p_ptr, (float)G.g, x);
#pragma unroll
    for (int k = 0; k < 6; ++k) X[s * 6 + k] = x[k];
    if (Y) Y[s] = (float)log((double)r[6] / p_ptr);
  }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const MlpDev* m, const float* __restrict__ X,
                                                     float* Y, long long n) {
  MlpRegs r;
  mlp_load(m, r);
  const int l = threadIdx.x & 63;
  const long long waves = (long long)gridDim.x * 4;
  for (long long w = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); w * 64 < n; w += waves) {
    const long long s = w * 64 + l;
    float x[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = s < n ? X[s * 6 + k] : 0.0f;
    const float y = mlp_forward<false>(r, x, nullptr);
    if (s < n) Y[s] = y;
  }
}

// One block = 4 waves = 256 samples per iteration; all waves of a block run
// the same number of iterations (the grid stride is in whole blocks).
__global__ __launch_bounds__(256) void k_mlp_grad(const MlpDev* m, const float* __restrict__ X,
                                                  const float* __restrict__ Tg, long long n,
                                                  float inv_n, float* partials) {
  __shared__ float acc[kGradSlots];
  __shared__ unsigned short gz2s[4][32][64];  // [wave][unit][sample]
  __shared__ unsigned short a1s[4][32][64];
  __shared__ unsigned short gz1s[4][32][64];
  __shared__ unsigned short xs[4][16][64];    // [wave][feature][sample], features >= 6 zero

  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, g = l >> 4, col = l & 15;
  for (int i = threadIdx.x; i < kGradSlots; i += blockDim.x) acc[i] = 0.0f;
  for (int i = l; i < 16 * 64; i += 64) xs[wv][i / 64][i % 64] = 0;
  MlpRegs r;
  mlp_load(m, r);
  // A operands of ga1 = W2^T gz2: rows = layer-1 units, K = layer-2 units (permuted)
  mlp_v8bf w2t[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      w2t[t][e] = __builtin_bit_cast(__bf16, m->w2tp[16 * t + col][8 * g + e]);
  __syncthreads();

  for (long long base = (long long)blockIdx.x * 256; base < n; base += (long long)gridDim.x * 256) {
    const long long s = base + threadIdx.x;
    const bool valid = s < n;
    float x[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = valid ? X[s * 6 + k] : 0.0f;
    const float tgt = valid ? Tg[s] : 0.0f;
    MlpAct act;
    const float y = mlp_forward<true>(r, x, &act);
    const float gy = valid ? 2.0f * (y - tgt) * inv_n : 0.0f;
    float loss = valid ? (y - tgt) * (y - tgt) * inv_n : 0.0f;
#pragma unroll
    for (int k = 0; k < 6; ++k) xs[wv][k][l] = bf16_bits(x[k]);

    float gyt[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) gyt[t] = __shfl(gy, 16 * t + col);

    // layer 3 and layer-2 biases; gz2 in the forward layout [m][t][e]
    float gz2[2][4][4];
    float pw3[8], pb2[8], pb1[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) pw3[i] = pb2[i] = pb1[i] = 0.0f;
#pragma unroll
    for (int mm = 0; mm < 2; ++mm)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float z = act.z2[mm][t][e];
          const float a2 = fmaxf(z, 0.0f);
          pw3[4 * mm + e] = fmaf(gyt[t], a2, pw3[4 * mm + e]);
          const float gz = z > 0.0f ? gyt[t] * r.w3[4 * mm + e] : 0.0f;
          gz2[mm][t][e] = gz;
          pb2[4 * mm + e] += gz;
          gz2s[wv][16 * mm + 4 * g + e][16 * t + col] = bf16_bits(gz);
          a1s[wv][16 * mm + 4 * g + e][16 * t + col] = bf16_bits(fmaxf(act.z1[mm][t][e], 0.0f));
        }
    // ga1 = W2^T bf16(gz2) on the MFMA units; gz1 = ga1 [z1 > 0]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      mlp_v8bf bop;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        bop[e] = __builtin_bit_cast(__bf16, bf16_bits(e < 4 ? gz2[0][t][e] : gz2[1][t][e - 4]));
#pragma unroll
      for (int mm = 0; mm < 2; ++mm) {
        mlp_v4f c = {0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2t[mm], bop, c, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float gz = act.z1[mm][t][e] > 0.0f ? c[e] : 0.0f;
          pb1[4 * mm + e] += gz;
          gz1s[wv][16 * mm + 4 * g + e][16 * t + col] = bf16_bits(gz);
        }
      }
    }
    // per-unit sums over the 16 lanes holding the same units
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        pw3[i] += __shfl_xor(pw3[i], o);
        pb2[i] += __shfl_xor(pb2[i], o);
        pb1[i] += __shfl_xor(pb1[i], o);
      }
    }
    float sgy = gy;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      sgy += __shfl_xor(sgy, o);
      loss += __shfl_xor(loss, o);
    }
    if (col == 0) {
#pragma unroll
      for (int mm = 0; mm < 2; ++mm)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int u = 16 * mm + 4 * g + e;
          atomicAdd(&acc[kOffW3 + u], pw3[4 * mm + e]);
          atomicAdd(&acc[kOffB2 + u], pb2[4 * mm + e]);
          atomicAdd(&acc[kOffB1 + u], pb1[4 * mm + e]);
        }
    }
    if (l == 0) {
      atomicAdd(&acc[kOffB3], sgy);
      atomicAdd(&acc[kMlpParams], loss);
    }
    __syncthreads();  // LDS staging complete

    // gW2[i][k] = sum_s bf16(gz2)[i][s] a1[k][s]; K = 64 samples in two steps
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int nk = 0; nk < 2; ++nk) {
        mlp_v4f c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          mlp_v8bf aop, bop;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            aop[e] = __builtin_bit_cast(__bf16, gz2s[wv][16 * mi + col][32 * kk + 8 * g + e]);
            bop[e] = __builtin_bit_cast(__bf16, a1s[wv][16 * nk + col][32 * kk + 8 * g + e]);
          }
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, c, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
          atomicAdd(&acc[kOffW2 + (16 * mi + 4 * g + e) * 32 + 16 * nk + col], c[e]);
      }
    // gW1[u][f] = sum_s bf16(gz1)[u][s] bf16(x)[f][s]
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      mlp_v4f c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        mlp_v8bf aop, bop;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          aop[e] = __builtin_bit_cast(__bf16, gz1s[wv][16 * mi + col][32 * kk + 8 * g + e]);
          bop[e] = __builtin_bit_cast(__bf16, xs[wv][col][32 * kk + 8 * g + e]);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, c, 0, 0, 0);
      }
      if (col < kMlpIn) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          atomicAdd(&acc[kOffW1 + (16 * mi + 4 * g + e) * kMlpIn + col], c[e]);
      }
    }
    __syncthreads();  // before the staging buffers are reused
  }
  for (int i = threadIdx.x; i < kGradSlots; i += blockDim.x)
    partials[(long long)blockIdx.x * kGradSlots + i] = acc[i];
}

// grad[i] = sum over blocks of partials, in block order
__global__ void k_mlp_reduce(const float* __restrict__ partials, int nblocks, float* grad,
                             float* loss) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kGradSlots; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += partials[(long long)b * kGradSlots + i];
    if (i < kMlpParams)
      grad[i] = s;
    else if (loss)
      *loss = s;
  }
}

__global__ void k_mlp_adam(float* p, float* mo, float* ve, const float* __restrict__ grad,
                           float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  const float gi = grad[i];
  const float m = b1 * mo[i] + (1.0f - b1) * gi;
  const float v = b2 * ve[i] + (1.0f - b2) * gi * gi;
  mo[i] = m;
  ve[i] = v;
  p[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

}  // namespace

int mlp_grad_blocks(long long n) {
  long long nb = (n + 255) / 256;
  return (int)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}
size_t mlp_grad_scratch_floats(long long n) { return (size_t)mlp_grad_blocks(n) * kGradSlots; }

hipError_t launch_mlp_pack(const float* params, MlpDev* m, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(1024), 0, s, params, m);
  return hipGetLastError();
}

hipError_t launch_mlp_features(const float* rec, long long n, double gamma, float* X, float* Y,
                               hipStream_t s) {
  long long nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  const Gas<double> G = make_gas<double>(gamma, default_options());
  hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)nb), dim3(256), 0, s, rec, n, G, X, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev* m, const float* X, float* Y, long long n,
                              hipStream_t s) {
  long long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)nb), dim3(256), 0, s, m, X, Y, n);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev* m, const float* X, const float* T, long long n,
                           float* scratch, float* grad, float* loss, hipStream_t s) {
  const int nb = mlp_grad_blocks(n);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, s, m, X, T, n, 1.0f / (float)n, scratch);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(6), dim3(256), 0, s, (const float*)scratch, nb, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, float* m, float* v, const float* grad, long long step,
                           double lr, double b1, double b2, double eps, hipStream_t s) {
  const double c1 = 1.0 - std::pow(b1, (double)step);
  const double c2 = 1.0 - std::pow(b2, (double)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, p, m, v, grad,
                     (float)lr, (float)b1, (float)b2, (float)eps, (float)c1, (float)c2);
  return hipGetLastError();
}

}  // namespace hydro
