// kernels.hip -- gfx950 kernels of the split Godunov sweep and its time step,
// all working on a batch of grids (a single grid is a batch of one).
//
// Work items are waves.  A launch covers the whole batch: the global wave
// index is mapped to (grid, local item) by a binary search over the grids'
// first-item prefix table (wave-uniform, scalar loads).  Launches are
// persistent when the launcher passes fewer blocks than items: each wave then
// strides over the items.
//
// x-sweep (rows, the contiguous direction): one lane per cell.  A 64-lane
//   wave holds cells x0-2 .. x0+61 of one row, loaded coalesced with the
//   boundary rule applied in the index remap; neighbours are exchanged with
//   cross-lane shuffles (primitive variables for the slopes, left face states
//   for the Riemann problems, fluxes for the update), and lanes 2..61 write
//   the 60 updated cells.  Every interface a wave needs is solved by its own
//   lane, so there is no divergent halo pass.  An item is `seg` consecutive
//   60-cell segments of one row.
// y-sweep (columns): one thread per column marches down a segment of rows
//   with a register window of the 5-cell stencil (paper, Figure 2); lanes
//   run along x, so every load and store of the wave is one coalesced row
//   access without an LDS transpose.
// tiled y-sweep (option): the x-sweep's one-lane-per-cell code along the
//   columns of a 16 x 64 tile transposed through LDS (sweeps.hpp).
// The last sweep of a step computes the max wave speed of the new state in
// its epilogue, for the grid's next dt (fused CFL reduction).
//
// Both read the grid's stored dt from device memory, so a step launches
// without a host round trip and can be captured into a HIP graph.  The sweep
// kernels themselves live in sweeps.hpp; this file instantiates the variants
// without passive scalars (kernels_scalar.hip those with one) and holds the
// row, per-grid and totals kernels and the launchers.
#include <hip/hip_runtime.h>

#include <utility>

#include "device_state.hpp"
#include "godunov.hpp"
#include "launch.hpp"
#include "mlp.hpp"
#include "sweeps.hpp"

namespace hydro {

// ------------------------------------------------------------ row kernels
// max wave speed of every cell (first step, hydro_compute_dt): one row per item
template <typename T>
__global__ __launch_bounds__(256) void k_max_speed(Batch<T> b, Gas<T> G) {
  const int lane = threadIdx.x & (kWave - 1);
  for (long long w = first_wave(); w < b.items; w += wave_stride()) {
    const int gi = find_grid<Key::Row>(b.g, b.ngrids, w);
    const GridDesc d = b.g[gi];
    const T* rp = b.src + d.off + (w - d.r0) * d.pitch;
    const long long P = d.plane;
    double smax = 0.0;
    for (int x = lane; x < d.nx; x += kWave)
      smax = fmax(smax, (double)max_speed(rp[x], rp[P + x], rp[2 * P + x], rp[3 * P + x], G));
    smax = wave_max(smax);
    if (lane == 0) fold_max(&b.st[gi].acc, smax);
  }
}

// dst <- src over the interior (standalone sweep): one row per item
template <typename T>
__global__ __launch_bounds__(256) void k_copy(Batch<T> b) {
  const int lane = threadIdx.x & (kWave - 1);
  for (long long w = first_wave(); w < b.items; w += wave_stride()) {
    const int gi = find_grid<Key::Row>(b.g, b.ngrids, w);
    const GridDesc d = b.g[gi];
    const long long base = d.off + (w - d.r0) * d.pitch;
    for (int x = lane; x < d.nx; x += kWave) {
#pragma unroll
      for (int v = 0; v < kMaxVars; ++v)
        if (v < b.nv) b.dst[base + v * d.plane + x] = b.src[base + v * d.plane + x];
    }
  }
}

// ------------------------------------------------------------ per-grid scalars
__global__ void k_reset_acc(DevState* st, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) st[i].acc = 0ull;
}

// dt = cfl h / smax from the grid's accumulated max; optionally advance its
// clock and clear the accumulator for the next fused reduction.
__global__ void k_finalize_dt(const GridDesc* g, DevState* st, int n, int advance, int reset) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  DevState& s = st[i];
  const double smax = __longlong_as_double((long long)s.acc);
  const double dt = g[i].cfl * g[i].h / smax;
  s.dt = dt;
  s.smax = smax;
  if (advance) {
    s.t += dt;
    s.step += 1;
  }
  if (reset) s.acc = 0ull;
}

__global__ void k_set_clock(DevState* st, int i, double t, long long step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st[i].t = t;
    st[i].step = step;
  }
}

__global__ void k_clear_stats(DevState* st, int n) {
  const int gi = blockIdx.x;
  const int i = threadIdx.x;
  if (gi >= n) return;
  if (i <= kMaxIter) {
    st[gi].hist[i] = 0ull;
    st[gi].wave_hist[i] = 0ull;
  }
  if (i == 0) {
    st[gi].interfaces = 0ull;
    st[gi].fallbacks = 0ull;
  }
}

// ------------------------------------------------------------ totals
// Grid g owns partial blocks tb0 .. tb0+ntb-1; block k of a grid sums rows
// k, k+ntb, ... with each thread a fixed strided set of cells, then a
// fixed-shape tree.  The final kernel (one block per grid) adds the grid's
// partials in a fixed order.  Results do not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void k_totals(Batch<T> b, double* partials) {
  __shared__ double sh[kMaxVars][256];
  int lo = 0, hi = b.ngrids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.g[mid].tb0 <= (int)blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GridDesc d = b.g[lo];
  const int k = blockIdx.x - d.tb0;
  double s[kMaxVars] = {};
  for (int y = k; y < d.ny; y += d.ntb) {
    const T* rowp = b.src + d.off + (long long)y * d.pitch;
    for (int x = threadIdx.x; x < d.nx; x += blockDim.x) {
#pragma unroll
      for (int v = 0; v < kMaxVars; ++v)
        if (v < b.nv) s[v] += (double)rowp[v * d.plane + x];
    }
  }
#pragma unroll
  for (int v = 0; v < kMaxVars; ++v) sh[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int v = 0; v < kMaxVars; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < kMaxVars) partials[blockIdx.x * kMaxVars + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_totals_final(const GridDesc* g, const double* partials,
                                                      DevState* st) {
  __shared__ double sh[kMaxVars][256];
  const GridDesc d = g[blockIdx.x];
  double s[kMaxVars] = {};
  for (int k = threadIdx.x; k < d.ntb; k += blockDim.x) {
#pragma unroll
    for (int v = 0; v < kMaxVars; ++v) s[v] += partials[(d.tb0 + k) * kMaxVars + v];
  }
#pragma unroll
  for (int v = 0; v < kMaxVars; ++v) sh[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int v = 0; v < kMaxVars; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < kMaxVars)
    st[blockIdx.x].totals[threadIdx.x] = sh[threadIdx.x][0] * (d.h * d.h);
}

// ------------------------------------------------------------ launchers
static inline unsigned blocks_for(long long items, unsigned max_blocks) {
  long long nb = (items + kWavesPerBlock - 1) / kWavesPerBlock;
  if (max_blocks > 0 && nb > (long long)max_blocks) nb = max_blocks;
  return (unsigned)(nb > 0 ? nb : 1);
}

// The variant for the options; null for an invalid limiter, solver or
// scalar count.  With the HLLC flux the instrumentation and the learned guess
// do not apply.
// the variants with a passive scalar are instantiated in kernels_scalar.hip
extern template SweepFn<double> sweep_table_ns<double, 0, 1>(int);
extern template SweepFn<double> sweep_table_ns<double, 1, 1>(int);
extern template SweepFn<float> sweep_table_ns<float, 0, 1>(int);
extern template SweepFn<float> sweep_table_ns<float, 1, 1>(int);
extern template SweepFn<double> sweep_table_ns<double, 2, 1>(int);
extern template SweepFn<float> sweep_table_ns<float, 2, 1>(int);

template <typename T, int DIR>
SweepFn<T> sweep_kernel(bool instr, int guess, bool fuse, int limiter, int riemann, int ns) {
  if (limiter < 0 || limiter > 2 || riemann < 0 || riemann > 2 || ns < 0 || ns > kMaxScalars)
    return nullptr;
  if (riemann == 2) instr = false, guess = 0;
  const int v = (instr ? 1 : 0) + (guess ? 2 : 0) + (fuse ? 4 : 0) + 8 * limiter + 24 * riemann;
  return ns == 0 ? sweep_table_ns<T, DIR, 0>(v) : sweep_table_ns<T, DIR, 1>(v);
}

template <typename T>
hipError_t launch_sweep_x(const Batch<T>& b, const Gas<T>& G, const Extras& ex, bool instr,
                          int guess, unsigned max_blocks, hipStream_t s) {
  const SweepFn<T> k =
      sweep_kernel<T, 0>(instr, guess, ex.fuse != 0, G.limiter, G.riemann, b.nv - 4);
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(blocks_for(b.items, max_blocks)), dim3(kWave * kWavesPerBlock), 0,
                     s, b, G, ex);
  return hipGetLastError();
}

template <typename T>
int sweep_y_blocks_per_cu(bool instr, int guess, bool fuse, int limiter, int riemann, int ns) {
  const SweepFn<T> k = sweep_kernel<T, 1>(instr, guess, fuse, limiter, riemann, ns);
  if (!k) return 0;
  int nb = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kWave * kWavesPerBlock, 0);
  return e == hipSuccess ? nb : 0;
}

template <typename T>
hipError_t launch_sweep_y(const Batch<T>& b, const Gas<T>& G, const Extras& ex, bool instr,
                          int guess, unsigned max_blocks, hipStream_t s) {
  const SweepFn<T> k =
      sweep_kernel<T, 1>(instr, guess, ex.fuse != 0, G.limiter, G.riemann, b.nv - 4);
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(blocks_for(b.items, max_blocks)), dim3(kWave * kWavesPerBlock), 0,
                     s, b, G, ex);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_y_tile(const Batch<T>& b, const Gas<T>& G, const Extras& ex, bool instr,
                               int guess, unsigned max_blocks, hipStream_t s) {
  const SweepFn<T> k =
      sweep_kernel<T, 2>(instr, guess, ex.fuse != 0, G.limiter, G.riemann, b.nv - 4);
  if (!k) return hipErrorInvalidValue;
  long long nb = b.items;
  if (max_blocks > 0 && nb > (long long)max_blocks) nb = max_blocks;
  hipLaunchKernelGGL(k, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kWave * kWavesPerBlock), 0, s, b,
                     G, ex);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_max_speed(const Batch<T>& b, const Gas<T>& G, hipStream_t s) {
  hipLaunchKernelGGL((k_max_speed<T>), dim3(blocks_for(b.items, 4096)),
                     dim3(kWave * kWavesPerBlock), 0, s, b, G);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const Batch<T>& b, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<T>), dim3(blocks_for(b.items, 8192)), dim3(kWave * kWavesPerBlock),
                     0, s, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_totals(const Batch<T>& b, int total_blocks, double* partials, hipStream_t s) {
  hipLaunchKernelGGL((k_totals<T>), dim3(total_blocks), dim3(256), 0, s, b, partials);
  hipLaunchKernelGGL(k_totals_final, dim3(b.ngrids), dim3(256), 0, s, b.g,
                     (const double*)partials, b.st);
  return hipGetLastError();
}

hipError_t launch_reset_acc(DevState* st, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_acc, dim3((n + 255) / 256), dim3(256), 0, s, st, n);
  return hipGetLastError();
}

hipError_t launch_finalize_dt(const GridDesc* g, DevState* st, int n, bool advance, bool reset,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_dt, dim3((n + 255) / 256), dim3(256), 0, s, g, st, n,
                     advance ? 1 : 0, reset ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_set_clock(DevState* st, int i, double t, long long step, hipStream_t s) {
  hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, s, st, i, t, step);
  return hipGetLastError();
}

hipError_t launch_clear_stats(DevState* st, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_stats, dim3(n), dim3(64), 0, s, st, n);
  return hipGetLastError();
}

#define HYDRO_INSTANTIATE(T)                                                                   \
  template hipError_t launch_sweep_x<T>(const Batch<T>&, const Gas<T>&, const Extras&, bool,  \
                                        int, unsigned, hipStream_t);                          \
  template hipError_t launch_sweep_y<T>(const Batch<T>&, const Gas<T>&, const Extras&, bool,  \
                                        int, unsigned, hipStream_t);                          \
  template hipError_t launch_sweep_y_tile<T>(const Batch<T>&, const Gas<T>&, const Extras&,   \
                                             bool, int, unsigned, hipStream_t);               \
  template int sweep_y_blocks_per_cu<T>(bool, int, bool, int, int, int);                      \
  template hipError_t launch_max_speed<T>(const Batch<T>&, const Gas<T>&, hipStream_t);       \
  template hipError_t launch_copy<T>(const Batch<T>&, hipStream_t);                           \
  template hipError_t launch_totals<T>(const Batch<T>&, int, double*, hipStream_t);

HYDRO_INSTANTIATE(double)
HYDRO_INSTANTIATE(float)

}  // namespace hydro
