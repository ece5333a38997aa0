// kernels.hip -- gfx950 kernels of the split Godunov sweep and its time step.
//
// x-sweep (rows, the contiguous direction): one lane per cell.  A 64-lane
//   wave holds cells x0-2 .. x0+61 of one row, loaded coalesced with the
//   boundary rule applied in the index remap; neighbours are exchanged with
//   cross-lane shuffles (primitive variables for the slopes, left face states
//   for the Riemann problems, fluxes for the update), and lanes 2..61 write
//   the 60 updated cells.  Every interface a wave needs is solved by its own
//   lane, so there is no divergent halo pass.
// y-sweep (columns): one thread per column marches down a segment of rows
//   with a register window of the 5-cell stencil (paper, Figure 2); lanes
//   run along x, so every load and store of the wave is one coalesced row
//   access without an LDS transpose.  The epilogue computes the max wave
//   speed of the new state for the next step's dt (fused CFL reduction).
//
// Both read the stored dt from device memory, so a step launches without a
// host round trip and can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include "device_state.hpp"
#include "godunov.hpp"
#include "launch.hpp"

namespace hydro {

// ------------------------------------------------------------ wave helpers
// Neighbour exchange by one lane (ds_bpermute through the LDS crossbar; the
// DPP wavefront shifts measured slower on gfx950).  Edge lanes read their own
// value; the x-sweep never uses those results.
template <typename T>
__device__ __forceinline__ T from_left(T v) {
  return __shfl_up(v, 1);
}
template <typename T>
__device__ __forceinline__ T from_right(T v) {
  return __shfl_down(v, 1);
}
template <typename T>
__device__ __forceinline__ Prim<T> from_left(const Prim<T>& q) {
  return Prim<T>{from_left(q.r), from_left(q.u), from_left(q.t), from_left(q.p)};
}
template <typename T>
__device__ __forceinline__ Prim<T> from_right(const Prim<T>& q) {
  return Prim<T>{from_right(q.r), from_right(q.u), from_right(q.t), from_right(q.p)};
}
template <typename T>
__device__ __forceinline__ Flux<T> from_left(const Flux<T>& f) {
  return Flux<T>{from_left(f.m), from_left(f.n), from_left(f.t), from_left(f.e)};
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

__device__ __forceinline__ void count_newton(DevState* st, bool valid, int key) {
  const int lane = threadIdx.x & (kWave - 1);
  bool mine = valid;
  unsigned long long all = __ballot(valid);
  if (all != 0ull && lane == __ffsll((long long)all) - 1)
    atomicAdd(&st->interfaces, (unsigned long long)__popcll(all));
  while (true) {
    unsigned long long mask = __ballot(mine);
    if (mask == 0ull) break;
    int leader = __ffsll((long long)mask) - 1;
    int k = __shfl(key, leader);
    unsigned long long same = __ballot(mine && key == k);
    if (lane == leader) atomicAdd(&st->hist[k], (unsigned long long)__popcll(same));
    if (key == k) mine = false;
  }
}

template <typename T>
__device__ __forceinline__ bool nonphysical(T r, T e) {
  return !(r > T(0)) || !(fabs(e) < T(INFINITY));
}

template <typename T>
__device__ __forceinline__ T step_lambda(const DevState* st, double h) {
  return T(st->dt / h);
}

// ------------------------------------------------------------ x-sweep
template <typename T, bool STATS>
__global__ __launch_bounds__(256) void k_sweep_x(GridArgs<T> a, Gas<T> G, DevState* st,
                                                 int segs_per_wave) {
  const int lane = threadIdx.x & (kWave - 1);
  const long long wave = (long long)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int nseg = (a.nx + kXOut - 1) / kXOut;
  const int chunks = (nseg + segs_per_wave - 1) / segs_per_wave;
  if (wave >= (long long)chunks * a.ny) return;
  const int row = (int)(wave / chunks);
  const int seg0 = (int)(wave % chunks) * segs_per_wave;
  const T lam = step_lambda<T>(st, a.h);
  const T* rowp = a.src + (long long)row * a.pitch;
  T* outp = a.dst + (long long)row * a.pitch;
  const long long P = a.plane;
  int status = 0;

  for (int sgi = 0; sgi < segs_per_wave; ++sgi) {
    const int seg = seg0 + sgi;
    if (seg >= nseg) break;
    const int x0 = seg * kXOut;
    const int i = x0 - 2 + lane;  // cell of this lane, in [-2, nx+1] when used
    bool flip;
    const int src = ghost_source(min(i, a.nx + 1), a.nx, a.bc, flip);
    T u0 = rowp[src];
    T un = rowp[P + src];
    T ut = rowp[2 * P + src];
    T e = rowp[3 * P + src];
    if (flip) un = -un;

    // COMPUTE: primitive variables, slopes, half-step face states
    T ir;
    const Prim<T> q = cons_to_prim(u0, un, ut, e, G, ir);
    const Prim<T> ql = from_left(q);
    const Prim<T> qr = from_right(q);
    Prim<T> d;
    d.r = minmod(q.r - ql.r, qr.r - q.r);
    d.u = minmod(q.u - ql.u, qr.u - q.u);
    d.t = minmod(q.t - ql.t, qr.t - q.t);
    d.p = minmod(q.p - ql.p, qr.p - q.p);
    Prim<T> qm, qp;
    trace(q, ir, d, lam, G, qm, qp);

    // Riemann problem at this lane's right interface i+1/2
    const Prim<T> qm_next = from_right(qm);
    int iters;
    bool conv;
    const Flux<T> F = riemann_flux(qp, qm_next, G, iters, conv);
    const Flux<T> Fl = from_left(F);  // interface i-1/2

    if (STATS) {
      // interfaces owned by this segment: x0-1/2 (first segment only) and the
      // right interfaces of its cells
      const bool valid = (lane >= 2 || (lane == 1 && x0 == 0)) && lane < 62 && i < a.nx;
      count_newton(st, valid, conv ? iters : 0);
    }

    // WRITE: conservative update of cells x0 .. x0+59
    if (lane >= 2 && lane < 62 && i < a.nx) {
      const T nr = u0 + lam * (Fl.m - F.m);
      const T nn = un + lam * (Fl.n - F.n);
      const T nt = ut + lam * (Fl.t - F.t);
      const T ne = e + lam * (Fl.e - F.e);
      outp[i] = nr;
      outp[P + i] = nn;
      outp[2 * P + i] = nt;
      outp[3 * P + i] = ne;
      status |= nonphysical(nr, ne) ? kStatusNonPhys : 0;
    }
  }
  if (status) atomicOr(&st->status, status);
}

// ------------------------------------------------------------ y-sweep
template <typename T>
struct Cell {
  T r, n, t, e;  // conservative: density, normal (y) and transverse (x) momentum, energy
};

template <typename T, bool FUSE_DT, bool STATS>
__global__ __launch_bounds__(256) void k_sweep_y(GridArgs<T> a, Gas<T> G, DevState* st,
                                                 int seg) {
  const int lane = threadIdx.x & (kWave - 1);
  const long long wave = (long long)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int ncolg = (a.nx + kWave - 1) / kWave;
  const int nsegs = (a.ny + seg - 1) / seg;
  if (wave >= (long long)ncolg * nsegs) return;
  const int cg = (int)(wave % ncolg);
  const int sg = (int)(wave / ncolg);
  const int x = cg * kWave + lane;
  const bool xin = x < a.nx;
  const T* col = a.src + (xin ? x : a.nx - 1);
  T* out = a.dst + x;
  const long long P = a.plane;
  const int y0 = sg * seg;
  const int y1 = min(y0 + seg, a.ny);
  const T lam = step_lambda<T>(st, a.h);

  auto load = [&](int j) {
    bool flip;
    const long long off = (long long)ghost_source(j, a.ny, a.bc, flip) * a.pitch;
    Cell<T> c;
    c.r = col[off];
    c.t = col[P + off];      // rho u: transverse
    c.n = col[2 * P + off];  // rho v: normal
    c.e = col[3 * P + off];
    if (flip) c.n = -c.n;
    return c;
  };
  auto slopes = [](const Prim<T>& a_, const Prim<T>& b, const Prim<T>& c) {
    Prim<T> d;
    d.r = minmod(b.r - a_.r, c.r - b.r);
    d.u = minmod(b.u - a_.u, c.u - b.u);
    d.t = minmod(b.t - a_.t, c.t - b.t);
    d.p = minmod(b.p - a_.p, c.p - b.p);
    return d;
  };

  // One loop body does everything: iteration j READs cell j+2, traces cell
  // j+1, solves the Riemann problem at j+1/2 and WRITEs cell j.  The first
  // four iterations only fill the window (uniform guards), so every step of
  // the method exists at one code location and an interface shared by two
  // segments is computed bitwise identically by both.
  Cell<T> c0, c1 = {T(1), T(0), T(0), T(1)}, c2 = c1;
  Prim<T> q0, q1 = {T(1), T(0), T(0), T(1)}, q2 = q1;
  T ir1, ir2 = T(1);
  Prim<T> qp0 = q1, qm1 = q1, qp1 = q1;
  Flux<T> Fm = {T(0), T(0), T(0), T(0)}, F = Fm;
  double smax = 0.0;
  int status = 0;
  for (int j = y0 - 4; j < y1; ++j) {
    c0 = c1;
    c1 = c2;
    q0 = q1;
    q1 = q2;
    ir1 = ir2;
    c2 = load(j + 2);
    q2 = cons_to_prim(c2.r, c2.n, c2.t, c2.e, G, ir2);
    if (j >= y0 - 2) trace(q1, ir1, slopes(q0, q1, q2), lam, G, qm1, qp1);
    if (j >= y0 - 1) {
      int iters;
      bool conv;
      F = riemann_flux(qp0, qm1, G, iters, conv);
      if (STATS) count_newton(st, xin && (j >= y0 || y0 == 0), conv ? iters : 0);
    }
    if (j >= y0) {
      const T nr = c0.r + lam * (Fm.m - F.m);
      const T nn = c0.n + lam * (Fm.n - F.n);
      const T nt = c0.t + lam * (Fm.t - F.t);
      const T ne = c0.e + lam * (Fm.e - F.e);
      if (xin) {
        const long long off = (long long)j * a.pitch;
        out[off] = nr;
        out[P + off] = nt;
        out[2 * P + off] = nn;
        out[3 * P + off] = ne;
        status |= nonphysical(nr, ne) ? kStatusNonPhys : 0;
        if (FUSE_DT) smax = fmax(smax, (double)max_speed(nr, nn, nt, ne, G));
      }
    }
    qp0 = qp1;
    Fm = F;
  }
  if (status) atomicOr(&st->status, status);
  if (FUSE_DT) {
    smax = wave_max(smax);
    if (lane == 0) atomicMax(&st->acc, (unsigned long long)__double_as_longlong(smax));
  }
}

// ------------------------------------------------------------ dt
template <typename T>
__global__ __launch_bounds__(256) void k_max_speed(GridArgs<T> a, Gas<T> G, DevState* st) {
  double smax = 0.0;
  const long long n = (long long)a.nx * a.ny;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(c / a.nx), x = (int)(c % a.nx);
    const long long off = (long long)y * a.pitch + x;
    smax = fmax(smax, (double)max_speed(a.src[off], a.src[a.plane + off],
                                        a.src[2 * a.plane + off], a.src[3 * a.plane + off], G));
  }
  smax = wave_max(smax);
  if ((threadIdx.x & (kWave - 1)) == 0)
    atomicMax(&st->acc, (unsigned long long)__double_as_longlong(smax));
}

__global__ void k_reset_acc(DevState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->acc = 0ull;
}

// dt = cfl h / smax from the accumulated max; optionally advance the clock
// and clear the accumulator for the next fused reduction.
__global__ void k_finalize_dt(DevState* st, double cfl, double h, int advance, int reset) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double smax = __longlong_as_double((long long)st->acc);
  const double dt = cfl * h / smax;
  st->dt = dt;
  st->smax = smax;
  if (advance) {
    st->t += dt;
    st->step += 1;
  }
  if (reset) st->acc = 0ull;
}

// ------------------------------------------------------------ totals
constexpr int kTotBlocks = 512;

// Block b sums rows b, b+kTotBlocks, ...; each thread a fixed strided set of
// cells; then a fixed-shape tree.  The result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void k_totals(GridArgs<T> a, double* partials) {
  __shared__ double sh[4][256];
  double s[4] = {0, 0, 0, 0};
  for (int y = blockIdx.x; y < a.ny; y += gridDim.x) {
    const T* rowp = a.src + (long long)y * a.pitch;
    for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
#pragma unroll
      for (int v = 0; v < 4; ++v) s[v] += (double)rowp[v * a.plane + x];
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) sh[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) partials[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_totals_final(const double* partials, int nb, double h,
                                                      DevState* st) {
  __shared__ double sh[4][256];
  double s[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] += partials[b * 4 + v];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) sh[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) st->totals[threadIdx.x] = sh[threadIdx.x][0] * (h * h);
}

// dst <- src over the nx x ny interior of all four planes
template <typename T>
__global__ __launch_bounds__(256) void k_copy(GridArgs<T> a) {
  const long long n = (long long)a.nx * a.ny;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const long long off = (c / a.nx) * a.pitch + c % a.nx;
#pragma unroll
    for (int v = 0; v < 4; ++v) a.dst[v * a.plane + off] = a.src[v * a.plane + off];
  }
}

__global__ void k_set_clock(DevState* st, double t, long long step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->t = t;
    st->step = step;
  }
}

__global__ void k_clear_stats(DevState* st) {
  const int i = threadIdx.x;
  if (i <= kMaxIter) st->hist[i] = 0ull;
  if (i == 0) {
    st->interfaces = 0ull;
    st->fallbacks = 0ull;
  }
}

// ------------------------------------------------------------ launchers
static inline unsigned blocks_for(long long waves, int waves_per_block) {
  return (unsigned)((waves + waves_per_block - 1) / waves_per_block);
}

template <typename T>
hipError_t launch_sweep_x(const GridArgs<T>& a, const Gas<T>& G, DevState* st, int segs,
                          bool stats, hipStream_t s) {
  const int nseg = (a.nx + kXOut - 1) / kXOut;
  const long long waves = (long long)((nseg + segs - 1) / segs) * a.ny;
  const dim3 grid(blocks_for(waves, 4)), block(256);
  if (stats)
    hipLaunchKernelGGL((k_sweep_x<T, true>), grid, block, 0, s, a, G, st, segs);
  else
    hipLaunchKernelGGL((k_sweep_x<T, false>), grid, block, 0, s, a, G, st, segs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_y(const GridArgs<T>& a, const Gas<T>& G, DevState* st, int seg,
                          bool fuse_dt, bool stats, hipStream_t s) {
  const long long waves = (long long)((a.nx + kWave - 1) / kWave) * ((a.ny + seg - 1) / seg);
  const dim3 grid(blocks_for(waves, 4)), block(256);
  if (fuse_dt) {
    if (stats)
      hipLaunchKernelGGL((k_sweep_y<T, true, true>), grid, block, 0, s, a, G, st, seg);
    else
      hipLaunchKernelGGL((k_sweep_y<T, true, false>), grid, block, 0, s, a, G, st, seg);
  } else {
    if (stats)
      hipLaunchKernelGGL((k_sweep_y<T, false, true>), grid, block, 0, s, a, G, st, seg);
    else
      hipLaunchKernelGGL((k_sweep_y<T, false, false>), grid, block, 0, s, a, G, st, seg);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_max_speed(const GridArgs<T>& a, const Gas<T>& G, DevState* st, hipStream_t s) {
  const long long n = (long long)a.nx * a.ny;
  unsigned nb = (unsigned)((n + 255) / 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL((k_max_speed<T>), dim3(nb), dim3(256), 0, s, a, G, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const GridArgs<T>& a, hipStream_t s) {
  const long long n = (long long)a.nx * a.ny;
  unsigned nb = (unsigned)((n + 255) / 256);
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL((k_copy<T>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reset_acc(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_acc, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_finalize_dt(DevState* st, double cfl, double h, bool advance, bool reset,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_dt, dim3(1), dim3(64), 0, s, st, cfl, h, advance ? 1 : 0,
                     reset ? 1 : 0);
  return hipGetLastError();
}

int totals_blocks() { return kTotBlocks; }

template <typename T>
hipError_t launch_totals(const GridArgs<T>& a, double* partials, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_totals<T>), dim3(kTotBlocks), dim3(256), 0, s, a, partials);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(256), 0, s, (const double*)partials,
                     kTotBlocks, a.h, st);
  return hipGetLastError();
}

hipError_t launch_set_clock(DevState* st, double t, long long step, hipStream_t s) {
  hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, s, st, t, step);
  return hipGetLastError();
}

hipError_t launch_clear_stats(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_stats, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

#define HYDRO_INSTANTIATE(T)                                                                 \
  template hipError_t launch_sweep_x<T>(const GridArgs<T>&, const Gas<T>&, DevState*, int,  \
                                        bool, hipStream_t);                                 \
  template hipError_t launch_sweep_y<T>(const GridArgs<T>&, const Gas<T>&, DevState*, int,  \
                                        bool, bool, hipStream_t);                           \
  template hipError_t launch_max_speed<T>(const GridArgs<T>&, const Gas<T>&, DevState*,     \
                                          hipStream_t);                                     \
  template hipError_t launch_totals<T>(const GridArgs<T>&, double*, DevState*, hipStream_t); \
  template hipError_t launch_copy<T>(const GridArgs<T>&, hipStream_t);

HYDRO_INSTANTIATE(double)
HYDRO_INSTANTIATE(float)

}  // namespace hydro
