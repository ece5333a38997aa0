// sweeps.hpp -- the sweep kernels (x-sweep over rows, y-sweep over columns)
// and their device helpers, templated on every option that selects a
// compiled variant.  Two translation units instantiate them: kernels.hip the
// variants without passive scalars, kernels_scalar.hip those with one, so
// the two halves compile in parallel.  The kernel design is described at the
// top of kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "device_state.hpp"
#include "godunov.hpp"
#include "mlp.hpp"

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

// Fold a non-negative wave maximum into a grid's max-speed accumulator (bits
// of a double >= 0 order as unsigned integers).  Atomics on one address
// serialise in L2, so the atomic is skipped when the value read already
// covers v: the accumulator only grows within a step, so a stale read costs
// at most a redundant atomic.  Without the check a launch with one small work
// item per wave (the x-sweep: ~1.5e5 items on 8192^2) spends milliseconds on
// them.  Called by one lane.
__device__ __forceinline__ void fold_max(unsigned long long* acc, double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  if (bits > __hip_atomic_load(acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax(acc, bits);
}

// Newton statistics of one wave's interfaces (valid lanes): the histogram of
// key (iterations to convergence, 0 = unconverged) per interface, and of the
// wave's largest iteration count `iters` (iterations run, the cap for an
// unconverged interface), which is what the wave's time follows.  Both bins
// are clamped to kMaxIter: a learned start that fails its residual test adds
// up to 4 iterations to the full cap, so counts above kMaxIter land in the
// last bin instead of past the array.
__device__ __forceinline__ void count_newton(DevState* st, bool valid, int key, int iters) {
  const int lane = threadIdx.x & (kWave - 1);
  key = min(key, kMaxIter);
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
  int m = valid ? iters : 0;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = max(m, __shfl_xor(m, off));
  if (all != 0ull && lane == __ffsll((long long)all) - 1)
    atomicAdd(&st->wave_hist[min(m, kMaxIter)], 1ull);
}

__device__ __forceinline__ void count_flag(unsigned long long* counter, bool flag) {
  const unsigned long long m = __ballot(flag);
  const int lane = threadIdx.x & (kWave - 1);
  if (m != 0ull && lane == __ffsll((long long)m) - 1)
    atomicAdd(counter, (unsigned long long)__popcll(m));
}

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014): a
// counter-based hash for the logger's sampling decisions.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Interface-state logger: samples interfaces (stronger jumps at a higher
// rate) into a device buffer for training the learned guess.
template <typename T>
__device__ __forceinline__ void log_interface(const Extras& ex, bool valid, const Prim<T>& L,
                                              const Prim<T>& R, T pstar, unsigned long long key) {
  if (!valid) return;
  const float rl = (float)L.r, rr = (float)R.r, pl = (float)L.p, pr = (float)R.p;
  const float cbar = sqrtf(ex.gamma * sqrtf(pl * pr) / sqrtf(rl * rr));
  const float strength = fabsf(logf(pl / pr)) + fabsf((float)(R.u - L.u)) / cbar;
  const float rate = strength > 0.05f ? ex.rate_strong : ex.rate_smooth;
  const float u = (float)(mix64(ex.seed ^ key) >> 40) * (1.0f / 16777216.0f);
  if (!(u < rate)) return;
  const unsigned long long slot = atomicAdd(ex.log_count, 1ull);
  if ((long long)slot >= ex.log_cap) return;
  float* r = ex.log + slot * kLogFields;
  r[0] = rl;
  r[1] = (float)L.u;
  r[2] = pl;
  r[3] = rr;
  r[4] = (float)R.u;
  r[5] = pr;
  r[6] = (float)pstar;
  r[7] = strength;
}

template <typename T>
__device__ __forceinline__ bool nonphysical(T r, T e) {
  return !(r > T(0)) || !(fabs(e) < T(INFINITY));
}

// First work item of this wave and the stride between a wave's items; both
// wave-uniform.
__device__ __forceinline__ long long first_wave() {
  const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  return (long long)blockIdx.x * kWavesPerBlock + wib;
}
__device__ __forceinline__ long long wave_stride() {
  return (long long)gridDim.x * kWavesPerBlock;
}

// Last grid whose first item is <= w (prefix tables start at 0 and never
// decrease).
enum class Key { X, Y, Row };
template <Key K>
__device__ __forceinline__ long long key_of(const GridDesc& d) {
  return K == Key::X ? d.wx0 : (K == Key::Y ? d.wy0 : d.r0);
}
template <Key K>
__device__ __forceinline__ int find_grid(const GridDesc* g, int n, long long w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key_of<K>(g[mid]) <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ x-sweep
// Waves per SIMD the register allocator must leave room for, per sweep
// variant (1: no constraint).  Values above what the variant needs on its own
// trade spills of loop-invariant values for occupancy.  Timed on MI355X over
// an 8192^2 state: the FP64 y-sweep runs 1.47 -> 1.21 ms at 3 waves instead
// of 2, the FP32 y-sweep 0.69 -> 0.62 ms at 6 instead of 5, the FP32 sweeps
// with the learned guess 1.09 -> 0.92 ms (x, 6 waves) and 0.75 -> 0.67 ms
// (y, 5); asking for more (FP64 x at 5, FP32 at 8) spills inside the Newton
// loop and runs 1.3-2.5x slower.
#ifndef HYDRO_OCC
#define HYDRO_OCC 1, 1, 1, 6, 3, 1, 6, 5
#endif
constexpr int kOcc[8] = {HYDRO_OCC};  // x f64, x f64 learned, x f32, x f32 learned, then y
// The exact solver's FP64 y-sweep needs more registers than 3 waves leave
// (it spilled ~150 bytes per lane there); it asks for 2.  The HLLC FP32
// y-sweep spilled 68 bytes at 6, the FP32 sweeps with a passive scalar 40-50;
// they ask for 5.
template <typename T, int GUESS, int RS, int NS>
struct SweepOcc {
  static constexpr bool f32 = sizeof(T) == 4;
  static constexpr int v = (f32 ? 2 : 0) + (GUESS ? 1 : 0);
  static constexpr int cap_x = f32 && NS > 0 ? 5 : 8;
  static constexpr int cap_y = RS == 1 && !f32 ? 2 : f32 && (RS == 2 || NS > 0) ? 5 : 8;
  static constexpr int x = kOcc[v] < cap_x ? kOcc[v] : cap_x;
  static constexpr int y = kOcc[4 + v] < cap_y ? kOcc[4 + v] : cap_y;
};

template <typename T, bool INSTR, int GUESS, int LIM, bool FUSE, int RS, int NS>
__global__ __launch_bounds__(256, (SweepOcc<T, GUESS, RS, NS>::x)) void k_sweep_x(Batch<T> b, Gas<T> G, Extras ex) {
  const int lane = threadIdx.x & (kWave - 1);
  for (long long w = first_wave(); w < b.items; w += wave_stride()) {
    const int gi = find_grid<Key::X>(b.g, b.ngrids, w);
    const GridDesc d = b.g[gi];
    DevState* st = b.st + gi;
    const int lw = (int)(w - d.wx0);
    const int nseg = (d.nx + kXOut - 1) / kXOut;
    const int chunks = (nseg + b.seg - 1) / b.seg;
    const int row = lw / chunks;
    const int seg0 = (lw - row * chunks) * b.seg;
    const T lam = T(st->dt / d.h);
    const T* rowp = b.src + d.off + (long long)row * d.pitch;
    T* outp = b.dst + d.off + (long long)row * d.pitch;
    const long long P = d.plane;
    int status = 0;
    T smax = T(0);  // max wave speed of the written cells (FUSE)

    for (int sgi = 0; sgi < b.seg; ++sgi) {
      const int seg = seg0 + sgi;
      if (seg >= nseg) break;
      const int x0 = seg * kXOut;
      const int i = x0 - 2 + lane;  // cell of this lane, in [-2, nx+1] when used
      bool flip;
      const int src = ghost_source(min(i, d.nx + 1), d.nx, d.bc, flip);
      T u0 = rowp[src];
      T un = rowp[P + src];
      T ut = rowp[2 * P + src];
      T e = rowp[3 * P + src];
      T sx = T(0);  // rho X of the passive scalar (NS)
      if constexpr (NS > 0) sx = rowp[4 * P + src];
      if (flip) un = -un;

      // COMPUTE: primitive variables, slopes, half-step face states
      T ir;
      const Prim<T> q = cons_to_prim(u0, un, ut, e, G, ir);
      const Prim<T> ql = from_left(q);
      const Prim<T> qr = from_right(q);
      Prim<T> dq;
      dq.r = limit<LIM>(q.r - ql.r, qr.r - q.r);
      dq.u = limit<LIM>(q.u - ql.u, qr.u - q.u);
      dq.t = limit<LIM>(q.t - ql.t, qr.t - q.t);
      dq.p = limit<LIM>(q.p - ql.p, qr.p - q.p);
      Prim<T> qm, qp;
      trace(q, ir, dq, lam, G, qm, qp);
      // passive scalar X = rho X / rho: limited slope, half-step faces with
      // the advective source -u dX
      T xm = T(0), xp = T(0);
      if constexpr (NS > 0) {
        const T X = sx * ir;
        const T dX = limit<LIM>(X - from_left(X), from_right(X) - X);
        const T hs = T(-0.5) * lam * q.u * dX;
        xm = X - T(0.5) * dX + hs;
        xp = X + T(0.5) * dX + hs;
      }

      // Riemann problem at this lane's right interface i+1/2
      const Prim<T> qm_next = from_right(qm);
      T p_learned = T(0);
      if (GUESS)
        p_learned = learned_guess<T>(ex.mlp, qp, qm_next, ex.gamma, ex.gate_kappa, ex.gate_theta2);
      int iters;
      bool conv, fb, left;
      T pstar;
      // FP64: the series form of the guess's power in smooth waves (measured
      // 4% faster on the x-sweep; no gain in FP32 or in the y-sweep's loop)
      const Flux<T> F = riemann_flux<RS, T, sizeof(T) == 8>(qp, qm_next, G, p_learned, iters,
                                                            conv, fb, pstar, left);
      const Flux<T> Fl = from_left(F);  // interface i-1/2
      // scalar flux: mass flux times X on the side of the contact at x/t = 0
      T FX = T(0), FXl = T(0);
      if constexpr (NS > 0) {
        const T xm_next = from_right(xm);
        FX = F.m * (left ? xp : xm_next);
        FXl = from_left(FX);
      }

      if (INSTR) {
        // interfaces owned by this segment: x0-1/2 (first segment only) and
        // the right interfaces of its cells
        const bool valid = (lane >= 2 || (lane == 1 && x0 == 0)) && lane < 62 && i < d.nx;
        count_newton(st, valid, conv ? iters : 0, iters);
        if (GUESS) count_flag(&st->fallbacks, valid && fb);
        if (ex.log)
          log_interface(ex, valid, qp, qm_next, pstar,
                        ((unsigned long long)gi << 44) ^ ((unsigned long long)st->step << 24) ^
                            ((unsigned long long)row * (d.nx + 1) + (i + 1)) * 2ull);
      }

      // WRITE: conservative update of cells x0 .. x0+59
      if (lane >= 2 && lane < 62 && i < d.nx) {
        const T nr = u0 + lam * (Fl.m - F.m);
        const T nn = un + lam * (Fl.n - F.n);
        const T nt = ut + lam * (Fl.t - F.t);
        const T ne = e + lam * (Fl.e - F.e);
        outp[i] = nr;
        outp[P + i] = nn;
        outp[2 * P + i] = nt;
        outp[3 * P + i] = ne;
        if constexpr (NS > 0) outp[4 * P + i] = sx + lam * (FXl - FX);
        status |= nonphysical(nr, ne) ? kStatusNonPhys : 0;
        if constexpr (FUSE) smax = fmax(smax, max_speed(nr, nn, nt, ne, G));
      }
    }
    if (status) atomicOr(&st->status, status);
    if constexpr (FUSE) {
      const double wmax = wave_max((double)smax);
      if (lane == 0) fold_max(&st->acc, wmax);
    }
  }
}

// ------------------------------------------------------------ y-sweep
template <typename T>
struct Cell {
  T r, n, t, e;  // conservative: density, normal (y) and transverse (x) momentum, energy
};

template <int LIM, typename T>
__device__ __forceinline__ Prim<T> slopes(const Prim<T>& a, const Prim<T>& b, const Prim<T>& c) {
  Prim<T> d;
  d.r = limit<LIM>(b.r - a.r, c.r - b.r);
  d.u = limit<LIM>(b.u - a.u, c.u - b.u);
  d.t = limit<LIM>(b.t - a.t, c.t - b.t);
  d.p = limit<LIM>(b.p - a.p, c.p - b.p);
  return d;
}

template <typename T, bool INSTR, int GUESS, int LIM, bool FUSE, int RS, int NS>
__global__ __launch_bounds__(256, (SweepOcc<T, GUESS, RS, NS>::y)) void k_sweep_y(Batch<T> b, Gas<T> G, Extras ex) {
  const int lane = threadIdx.x & (kWave - 1);
  for (long long w = first_wave(); w < b.items; w += wave_stride()) {
    const int gi = find_grid<Key::Y>(b.g, b.ngrids, w);
    const GridDesc d = b.g[gi];
    DevState* st = b.st + gi;
    const int lw = (int)(w - d.wy0);
    const int ncolg = (d.nx + kWave - 1) / kWave;
    const int sg = lw / ncolg;
    const int cg = lw - sg * ncolg;
    const int x = cg * kWave + lane;
    const bool xin = x < d.nx;
    const T* col = b.src + d.off + (xin ? x : d.nx - 1);
    T* out = b.dst + d.off + x;
    const long long P = d.plane;
    const int y0 = sg * b.seg;
    const int y1 = min(y0 + b.seg, d.ny);
    const T lam = T(st->dt / d.h);

    auto load = [&](int j) {
      bool flip;
      const long long off = (long long)ghost_source(j, d.ny, d.bc, flip) * d.pitch;
      Cell<T> c;
      c.r = col[off];
      c.t = col[P + off];      // rho u: transverse
      c.n = col[2 * P + off];  // rho v: normal
      c.e = col[3 * P + off];
      if (flip) c.n = -c.n;
      return c;
    };
    auto load_scalar = [&](int j) {  // rho X (NS): copied at walls
      bool flip;
      return col[4 * P + (long long)ghost_source(j, d.ny, d.bc, flip) * d.pitch];
    };

    T smax = T(0);  // max of T values is exact; widened once for the atomic
    int status = 0;
    if constexpr (sizeof(T) == 8 && NS == 0 && LIM == 0 && RS == 0) {
      // FP64, minmod, two-shock solver, no passive scalar: the loop below
      // software-pipelined by one row.  Iteration j issues the READ of row
      // j+3, solves the Riemann problem at j+1/2 from faces traced in the
      // previous iteration and WRITEs row j while that load is in flight,
      // then converts row j+3 and traces row j+2, so the load's latency hides
      // behind the wave's own Riemann solve.  The loop is unrolled by 3 and
      // runs from a row index that is a multiple of 3 for a multiple of 3
      // iterations, so every row is converted, traced and solved by the same
      // unrolled copy whatever the segment bounds: results do not depend on
      // the launch shape.  (The FP32 sweep and the FP64 MC and HLLC variants
      // spill with the longer window and keep the loop below.)
      Cell<T> c0, c1 = {T(1), T(0), T(0), T(1)}, c2 = c1;
      Prim<T> q1 = {T(1), T(0), T(0), T(1)}, q2 = q1;
      T ir2 = T(1);
      Prim<T> qpA = q1, qmB = q1, qpB = q1;  // qp(j), qm(j+1), qp(j+1)
      Flux<T> Fm = {T(0), T(0), T(0), T(0)}, F = Fm;
      const int jb = y0 - 5;                   // first iteration the stencil needs
      const int j0 = jb - (((jb % 3) + 3) % 3);  // ... moved down to a multiple of 3
      const int j1 = j0 + (y1 - j0 + 2) / 3 * 3;  // >= y1, a multiple of 3 iterations
#pragma unroll 3
      for (int j = j0; j < j1; ++j) {
        // rows outside -2 .. ny+1 are never used (the clamp keeps reads in range)
        const Cell<T> cn = load(max(min(j + 3, d.ny + 1), -2));
        if (j >= y0 - 1 && j < y1) {
          T p_learned = T(0);
          if (GUESS)
            p_learned = learned_guess<T>(ex.mlp, qpA, qmB, ex.gamma, ex.gate_kappa, ex.gate_theta2);
          int iters;
          bool conv, fb, left;
          T pstar;
          F = riemann_flux<RS>(qpA, qmB, G, p_learned, iters, conv, fb, pstar, left);
          if (INSTR) {
            const bool valid = xin && (j >= y0 || y0 == 0);
            count_newton(st, valid, conv ? iters : 0, iters);
            if (GUESS) count_flag(&st->fallbacks, valid && fb);
            if (ex.log)
              log_interface(ex, valid, qpA, qmB, pstar,
                            ((unsigned long long)gi << 44) ^ ((unsigned long long)st->step << 24) ^
                                (((unsigned long long)x * (d.ny + 1) + (j + 1)) * 2ull + 1ull));
          }
        }
        if (j >= y0 && j < y1) {
          const T nr = c0.r + lam * (Fm.m - F.m);
          const T nn = c0.n + lam * (Fm.n - F.n);
          const T nt = c0.t + lam * (Fm.t - F.t);
          const T ne = c0.e + lam * (Fm.e - F.e);
          if (xin) {
            const long long off = (long long)j * d.pitch;
            __builtin_nontemporal_store(nr, out + off);
            __builtin_nontemporal_store(nt, out + P + off);
            __builtin_nontemporal_store(nn, out + 2 * P + off);
            __builtin_nontemporal_store(ne, out + 3 * P + off);
            status |= nonphysical(nr, ne) ? kStatusNonPhys : 0;
            if constexpr (FUSE) smax = fmax(smax, max_speed(nr, nn, nt, ne, G));
          }
        }
        Fm = F;
        c0 = c1;
        c1 = c2;
        c2 = cn;
        T ir3;
        const Prim<T> q3 = cons_to_prim(cn.r, cn.n, cn.t, cn.e, G, ir3);
        Prim<T> qm2, qp2;
        trace(q2, ir2, slopes<LIM>(q1, q2, q3), lam, G, qm2, qp2);
        qpA = qpB;
        qmB = qm2;
        qpB = qp2;
        q1 = q2;
        q2 = q3;
        ir2 = ir3;
      }
    } else {
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
      // passive scalar (NS): rho X and X of the window, faces, fluxes
      T s0 = T(0), s1 = T(0), s2 = T(0), X0 = T(0), X1 = T(0), X2 = T(0);
      T xm1 = T(0), xp1 = T(0), xp0 = T(0), FX = T(0), FmX = T(0);
#pragma unroll 3
      for (int j = y0 - 4; j < y1; ++j) {
        c0 = c1;
        c1 = c2;
        q0 = q1;
        q1 = q2;
        ir1 = ir2;
        c2 = load(j + 2);
        q2 = cons_to_prim(c2.r, c2.n, c2.t, c2.e, G, ir2);
        if constexpr (NS > 0) {
          s0 = s1;
          s1 = s2;
          X0 = X1;
          X1 = X2;
          s2 = load_scalar(j + 2);
          X2 = s2 * ir2;
        }
        if (j >= y0 - 2) {
          trace(q1, ir1, slopes<LIM>(q0, q1, q2), lam, G, qm1, qp1);
          if constexpr (NS > 0) {
            const T dX = limit<LIM>(X1 - X0, X2 - X1);
            const T hs = T(-0.5) * lam * q1.u * dX;
            xm1 = X1 - T(0.5) * dX + hs;
            xp1 = X1 + T(0.5) * dX + hs;
          }
        }
        if (j >= y0 - 1) {
          T p_learned = T(0);
          if (GUESS)
            p_learned = learned_guess<T>(ex.mlp, qp0, qm1, ex.gamma, ex.gate_kappa, ex.gate_theta2);
          int iters;
          bool conv, fb, left;
          T pstar;
          F = riemann_flux<RS>(qp0, qm1, G, p_learned, iters, conv, fb, pstar, left);
          if constexpr (NS > 0) FX = F.m * (left ? xp0 : xm1);
          if (INSTR) {
            const bool valid = xin && (j >= y0 || y0 == 0);
            count_newton(st, valid, conv ? iters : 0, iters);
            if (GUESS) count_flag(&st->fallbacks, valid && fb);
            if (ex.log)
              log_interface(ex, valid, qp0, qm1, pstar,
                            ((unsigned long long)gi << 44) ^ ((unsigned long long)st->step << 24) ^
                                (((unsigned long long)x * (d.ny + 1) + (j + 1)) * 2ull + 1ull));
          }
        }
        if (j >= y0) {
          const T nr = c0.r + lam * (Fm.m - F.m);
          const T nn = c0.n + lam * (Fm.n - F.n);
          const T nt = c0.t + lam * (Fm.t - F.t);
          const T ne = c0.e + lam * (Fm.e - F.e);
          if (xin) {
            const long long off = (long long)j * d.pitch;
            // streaming stores: the next sweep reads these only after the
            // whole grid (measured faster for the y-sweep, slower for the x-sweep)
            __builtin_nontemporal_store(nr, out + off);
            __builtin_nontemporal_store(nt, out + P + off);
            __builtin_nontemporal_store(nn, out + 2 * P + off);
            __builtin_nontemporal_store(ne, out + 3 * P + off);
            if constexpr (NS > 0)
              __builtin_nontemporal_store(s0 + lam * (FmX - FX), out + 4 * P + off);
            status |= nonphysical(nr, ne) ? kStatusNonPhys : 0;
            if constexpr (FUSE) smax = fmax(smax, max_speed(nr, nn, nt, ne, G));
          }
        }
        qp0 = qp1;
        Fm = F;
        if constexpr (NS > 0) {
          xp0 = xp1;
          FmX = FX;
        }
      }
    }
    if (status) atomicOr(&st->status, status);
    if constexpr (FUSE) {
      const double wmax = wave_max((double)smax);
      if (lane == 0) fold_max(&st->acc, wmax);
    }
  }
}

// ------------------------------------------------------------ variant tables
// Sweep kernel variants: instrumentation, learned guess, fused reduction,
// limiter and interface solver are template arguments; index within one
// scalar count = instr + 2 guess + 4 fuse + 8 limiter + 24 solver.  The HLLC
// flux iterates nothing, so it has neither instrumented nor learned-guess
// variants (null entries).
template <typename T>
using SweepFn = void (*)(Batch<T>, Gas<T>, Extras);
constexpr int kSweepVariants = 2 * 2 * 2 * 3 * 3;

template <typename T, int DIR, int NS, int V>
constexpr SweepFn<T> sweep_variant() {
  constexpr bool I = V & 1;
  constexpr int GS = (V >> 1) & 1;
  constexpr bool F = (V >> 2) & 1;
  constexpr int L = (V >> 3) % 3;
  constexpr int RS = V / 24;
  if constexpr (RS == 2 && (I || GS))
    return nullptr;
  else if constexpr (DIR == 0)
    return &k_sweep_x<T, I, GS, L, F, RS, NS>;
  else
    return &k_sweep_y<T, I, GS, L, F, RS, NS>;
}

template <typename T, int DIR, int NS, int... V>
SweepFn<T> sweep_table(int v, std::integer_sequence<int, V...>) {
  static const SweepFn<T> table[] = {sweep_variant<T, DIR, NS, V>()...};
  return table[v];
}

// Table lookup for NS passive scalars; each NS is instantiated in one
// translation unit (0 in kernels.hip, 1 in kernels_scalar.hip).
template <typename T, int DIR, int NS>
SweepFn<T> sweep_table_ns(int v) {
  return sweep_table<T, DIR, NS>(v, std::make_integer_sequence<int, kSweepVariants>());
}

}  // namespace hydro
