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
// value; the x-sweep never uses those results.  The byte addresses of the two
// neighbours are computed once per kernel (Nbr) rather than at every exchange.
struct Nbr {
  int left, right;  // ds_bpermute addresses of lanes l - 1 and l + 1
};
__device__ __forceinline__ Nbr lane_neighbours() {
  const int l = __lane_id();
  return Nbr{(l > 0 ? l - 1 : l) * 4, (l < kWave - 1 ? l + 1 : l) * 4};
}
__device__ __forceinline__ float bpermute(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double bpermute(int addr, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <typename T>
__device__ __forceinline__ T from_left(const Nbr& nb, T v) {
  return bpermute(nb.left, v);
}
template <typename T>
__device__ __forceinline__ T from_right(const Nbr& nb, T v) {
  return bpermute(nb.right, v);
}
template <typename T>
__device__ __forceinline__ Prim<T> from_left(const Nbr& nb, const Prim<T>& q) {
  return Prim<T>{from_left(nb, q.r), from_left(nb, q.u), from_left(nb, q.t), from_left(nb, q.p)};
}
template <typename T>
__device__ __forceinline__ Prim<T> from_right(const Nbr& nb, const Prim<T>& q) {
  return Prim<T>{from_right(nb, q.r), from_right(nb, q.u), from_right(nb, q.t),
                 from_right(nb, q.p)};
}
template <typename T>
__device__ __forceinline__ Flux<T> from_left(const Nbr& nb, const Flux<T>& f) {
  return Flux<T>{from_left(nb, f.m), from_left(nb, f.n), from_left(nb, f.t), from_left(nb, f.e)};
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

// Flux at one interface with the starting guess the variant selects: the
// network's correction of the two-rarefaction guess (GUESS; net is the
// network staged in LDS) or that guess itself.  Called by all 64 lanes.
template <int RS, bool SERIES, int GUESS, bool CARRY = false, typename T>
__device__ __forceinline__ Flux<T> interface_flux(const Prim<T>& L, const Prim<T>& R,
                                                  const Gas<T>& G, const Extras& ex,
                                                  const MlpInfer* net, int& iters, bool& conv,
                                                  bool& fb, T& pstar, bool& left) {
  if constexpr (GUESS != 0 && RS != 2)
    return riemann_flux<RS, T, SERIES, CARRY>(
        L, R, G, LearnedGuess{net, ex.gamma, ex.gate_kappa, ex.gate_theta2}, iters, conv, fb,
        pstar, left);
  else
    return riemann_flux<RS, T, SERIES, CARRY>(L, R, G, NoLearnedGuess{}, iters, conv, fb, pstar,
                                              left);
}

// A wave-uniform pointer moved to scalar registers (both halves read from the
// first active lane) as a global-memory pointer, so that per-lane accesses
// p + offset take the scalar-base form of the global load and store: a 32-bit
// per-lane byte offset and no 64-bit address arithmetic per lane and access.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ global_ptr<T> uniform_ptr(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (global_ptr<T>)(((unsigned long long)hi << 32) | lo);
}
// The element at byte offset boff (a non-negative in-range offset that fits
// 32 bits) from base.
template <typename T>
__device__ __forceinline__ T at(global_ptr<const T> base, unsigned boff) {
  return *(global_ptr<const T>)((global_ptr<const char>)base + boff);
}
template <typename T>
__device__ __forceinline__ global_ptr<T> ptr_at(global_ptr<T> base, unsigned boff) {
  return (global_ptr<T>)((global_ptr<char>)base + boff);
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
enum class Key { X, Y, Tile, Row };
template <Key K>
__device__ __forceinline__ long long key_of(const GridDesc& d) {
  return K == Key::X ? d.wx0 : (K == Key::Y ? d.wy0 : (K == Key::Tile ? d.wt0 : d.r0));
}
// Descriptor i of a batch's table.  The table is read-only while a kernel
// runs and read at wave-uniform indices, so it is read through the constant
// address space: scalar loads into scalar registers, which keeps the
// arithmetic on its fields (rows, segments, plane pointers) scalar.
__device__ __forceinline__ GridDesc load_desc(const GridDesc* g, int i) {
  static_assert(sizeof(GridDesc) % 8 == 0, "descriptor read as 64-bit words");
  typedef const __attribute__((address_space(4))) unsigned long long* const_words;
  const const_words src = (const_words)(g + i);
  unsigned long long w[sizeof(GridDesc) / 8];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(GridDesc) / 8); ++k) w[k] = src[k];
  GridDesc d;
  __builtin_memcpy(&d, w, sizeof(GridDesc));
  return d;
}
template <Key K>
__device__ __forceinline__ int find_grid(const GridDesc* g, int n, long long w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key_of<K>(load_desc(g, mid)) <= w)
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
// of 2, the FP32 y-sweep 0.69 -> 0.62 ms at 6 instead of 5; asking for more
// (FP32 at 8) spills inside the Newton loop and runs 1.3-2.5x slower.  The
// sweeps with the learned guess hold the network's tile in registers next to
// their own state: 4 (FP64 x), 3 (FP64 y) and 5 (FP32) waves fit without
// spilling (FP32 y: 3 registers).
#ifndef HYDRO_OCC
#define HYDRO_OCC 1, 4, 1, 5, 3, 3, 6, 5
#endif
constexpr int kOcc[8] = {HYDRO_OCC};  // x f64, x f64 learned, x f32, x f32 learned, then y
// The exact solver's FP64 y-sweep needs more registers than 3 waves leave
// (it spilled ~150 bytes per lane there); it asks for 2.  The HLLC FP32
// y-sweep spilled 68 bytes at 6, the FP32 sweeps with a passive scalar 40-50;
// they ask for 5.
// The plain FP64 x-sweep (two-shock or HLLC, no scalar) asks for 5 waves and
// fits 6 (77 registers); held at 7 it spills and runs 5% slower.  With the
// statistics or the fused max speed it asks for 4.
template <typename T, int GUESS, int RS, int NS, bool INSTR = false, bool FUSE = false>
struct SweepOcc {
  static constexpr bool f32 = sizeof(T) == 4;
  static constexpr int v = (f32 ? 2 : 0) + (GUESS ? 1 : 0);
  static constexpr int cap_x = f32 && NS > 0 ? 5 : 8;
  static constexpr int cap_y = RS == 1 && !f32 ? 2 : f32 && (RS == 2 || NS > 0) ? 5 : 8;
  static constexpr bool plain64 = !f32 && GUESS == 0 && RS != 1 && NS == 0;
  static constexpr int x = plain64 ? (INSTR || FUSE ? 4 : 5) : (kOcc[v] < cap_x ? kOcc[v] : cap_x);
  static constexpr int y = kOcc[4 + v] < cap_y ? kOcc[4 + v] : cap_y;
  // tiled y-sweep (the x-sweep's code plus the tile loop): the FP64 default
  // variant at 4 waves (5 spilled; the two ran within 0.4% of each other in
  // a single-grid build), the exact solver at 2, the other FP64 variants at
  // 3, FP32 as the x-sweep
  static constexpr int t = f32 ? x : (RS == 1 ? 2 : (GUESS == 0 && NS == 0 ? 4 : 3));
};

// Conservative state of the cell one lane holds: density, normal and
// transverse momentum, energy, and rho X of the passive scalar (NS).
template <typename T>
struct Lane {
  T r, n, t, e, s;
};

// One pencil segment of 64 cells held one cell per lane: lane l holds cell
// c0 - 2 + l, so lanes 2..61 are the 60 cells the segment updates and lanes
// 0, 1, 62, 63 their ghost or neighbour cells (cells past the pencil's end
// hold clamped copies that no updated cell depends on).  Neighbours come by
// cross-lane shuffles (primitive variables for the slopes, left face states
// for the Riemann problem at each lane's right interface, fluxes for the
// update).  On return c holds the lane's updated cell (meaningful in lanes
// 2..61).  iface_valid marks the lanes whose right interface this segment
// owns (statistics and logger, INSTR); log_key identifies it for the logger.
// The x-sweep runs it along rows, the tiled y-sweep along columns of a tile
// transposed through LDS.
template <typename T, bool INSTR, int GUESS, int LIM, int RS, int NS>
__device__ __forceinline__ void pencil_segment(Lane<T>& c, const Nbr& nb, T lam, const Gas<T>& G,
                                               const Extras& ex, const MlpInfer* net,
                                               DevState* st, bool iface_valid,
                                               unsigned long long log_key) {
  // COMPUTE: primitive variables, slopes, half-step face states
  T ir;
  const Prim<T> q = cons_to_prim(c.r, c.n, c.t, c.e, G, ir);
  const Prim<T> ql = from_left(nb, q);
  const Prim<T> qr = from_right(nb, q);
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
    const T X = c.s * ir;
    const T dX = limit<LIM>(X - from_left(nb, X), from_right(nb, X) - X);
    const T hs = T(-0.5) * lam * q.u * dX;
    xm = X - T(0.5) * dX + hs;
    xp = X + T(0.5) * dX + hs;
  }

  // Riemann problem at this lane's right interface
  const Prim<T> qm_next = from_right(nb, qm);
  int iters;
  bool conv, fb, left;
  T pstar;
  // FP64: the series form of the guess's power in smooth waves (measured
  // 4% faster on the x-sweep; no gain in FP32 or in the y-sweep's loop)
  // FP32: the final star state carried from the last Newton iterate (the
  // registers are there in this one-cell-per-lane form)
  const Flux<T> F = interface_flux<RS, sizeof(T) == 8, GUESS, sizeof(T) == 4>(
      qp, qm_next, G, ex, net, iters, conv, fb, pstar, left);
  const Flux<T> Fl = from_left(nb, F);  // the lane's left interface
  // scalar flux: mass flux times X on the side of the contact at x/t = 0
  T FX = T(0), FXl = T(0);
  if constexpr (NS > 0) {
    const T xm_next = from_right(nb, xm);
    FX = F.m * (left ? xp : xm_next);
    FXl = from_left(nb, FX);
  }

  if (INSTR) {
    count_newton(st, iface_valid, conv ? iters : 0, iters);
    if (GUESS) count_flag(&st->fallbacks, iface_valid && fb);
    if (ex.log) log_interface(ex, iface_valid, qp, qm_next, pstar, log_key);
  }

  // conservative update of the lane's cell
  c.r = c.r + lam * (Fl.m - F.m);
  c.n = c.n + lam * (Fl.n - F.n);
  c.t = c.t + lam * (Fl.t - F.t);
  c.e = c.e + lam * (Fl.e - F.e);
  if constexpr (NS > 0) c.s = c.s + lam * (FXl - FX);
}

template <typename T, bool INSTR, int GUESS, int LIM, bool FUSE, int RS, int NS>
__global__ __launch_bounds__(256, (SweepOcc<T, GUESS, RS, NS, INSTR, FUSE>::x)) void k_sweep_x(Batch<T> b, Gas<T> G, Extras ex) {
  const int lane = threadIdx.x & (kWave - 1);
  const Nbr nb = lane_neighbours();
  // the learned guess's network, staged in LDS once per block
  __shared__ MlpInfer net_lds;
  const MlpInfer* net = nullptr;
  if constexpr (GUESS != 0) {
    mlp_stage(ex.mlp, &net_lds);
    net = &net_lds;
  }
  // Line-aligned stores (the variants without passive scalars or learned
  // guess): a segment updates 60 cells, so its stores would start and end
  // inside 128-byte lines, and partial-line stores cost HBM time of their own
  // (a four-plane copy with every 64-cell store shifted by two cells takes
  // 10-13% longer than the aligned one, and more with streaming stores).  Each
  // wave therefore parks its updated cells in a ring of kXRing cells per
  // variable in LDS and stores whole 64-cell blocks, aligned to the output
  // address, with streaming stores; the rest of the work item's last block
  // goes out at its end (long items, seg_x 8-16, keep those few).  The ring
  // holds at most 63 + 60 pending cells.  A wave reads back only what it wrote
  // itself, and LDS executes a wave's instructions in order, so no barrier is
  // needed, only a fence against the compiler moving the LDS accesses across
  // each other.
  // (The block has at most kWavesPerBlock waves: __launch_bounds__(256).)
  constexpr bool STAGE = (NS == 0 && GUESS == 0);
  __shared__ T ring[STAGE ? kWavesPerBlock : 1][4][kXRing];
  T(*const wring)[kXRing] = ring[STAGE ? threadIdx.x / kWave : 0];
  for (long long w = first_wave(); w < b.items; w += wave_stride()) {
    const int gi = find_grid<Key::X>(b.g, b.ngrids, w);
    const GridDesc d = load_desc(b.g, gi);
    DevState* st = b.st + gi;
    const int lw = (int)(w - d.wx0);
    const int nseg = (d.nx + kXOut - 1) / kXOut;
    const int chunks = (nseg + b.seg - 1) / b.seg;
    const int row = lw / chunks;
    const int seg0 = (lw - row * chunks) * b.seg;
    const T lam = T(st->dt / d.h);
    const long long P = d.plane;
    // the row's variable planes in scalar registers
    const T* rowp = b.src + d.off + (long long)row * d.pitch;
    T* outp = b.dst + d.off + (long long)row * d.pitch;
    const auto in0 = uniform_ptr(rowp), in1 = uniform_ptr(rowp + P);
    const auto in2 = uniform_ptr(rowp + 2 * P), in3 = uniform_ptr(rowp + 3 * P);
    const auto out0 = uniform_ptr(outp), out1 = uniform_ptr(outp + P);
    const auto out2 = uniform_ptr(outp + 2 * P), out3 = uniform_ptr(outp + 3 * P);
    int status = 0;
    T smax = T(0);  // max wave speed of the written cells (FUSE)
    // STAGE: cells [flushed, produced) of the row are parked in the ring; block
    // boundaries are where the first variable's output address is a multiple
    // of 64 cells (the other planes share it when the plane stride is a
    // multiple of 64 cells; otherwise only their speed suffers)
    int flushed = seg0 * kXOut;
    const int xa = (int)(((unsigned long long)outp / sizeof(T)) & 63u);
    auto flush = [&](int produced, bool last) {
      while (flushed < produced) {
        const int bs = ((flushed + xa) & ~63) - xa;
        const int lim = min(bs + 64, produced);
        if (lim < bs + 64 && !last) break;
        const int cell = bs + lane;
        if (cell >= flushed && cell < lim) {
          const int k = cell & (kXRing - 1);
          const unsigned oo = (unsigned)cell * (unsigned)sizeof(T);
          __builtin_nontemporal_store(wring[0][k], ptr_at(out0, oo));
          __builtin_nontemporal_store(wring[1][k], ptr_at(out1, oo));
          __builtin_nontemporal_store(wring[2][k], ptr_at(out2, oo));
          __builtin_nontemporal_store(wring[3][k], ptr_at(out3, oo));
        }
        flushed = lim;
      }
    };

    for (int sgi = 0; sgi < b.seg; ++sgi) {
      const int seg = seg0 + sgi;
      if (seg >= nseg) break;
      const int x0 = seg * kXOut;
      const int i = x0 - 2 + lane;  // cell of this lane, in [-2, nx+1] when used
      // READ, with the boundary rule in the index remap
      bool flip;
      const int src = ghost_source(min(i, d.nx + 1), d.nx, d.bc, flip);
      const unsigned so = (unsigned)src * (unsigned)sizeof(T);
      Lane<T> c;
      c.r = at(in0, so);
      c.n = at(in1, so);
      c.t = at(in2, so);
      c.e = at(in3, so);
      c.s = T(0);
      if constexpr (NS > 0) c.s = rowp[4 * P + src];
      if (flip) c.n = -c.n;

      // interfaces owned by this segment: x0-1/2 (first segment only) and
      // the right interfaces of its cells
      const bool valid = (lane >= 2 || (lane == 1 && x0 == 0)) && lane < 62 && i < d.nx;
      pencil_segment<T, INSTR, GUESS, LIM, RS, NS>(
          c, nb, lam, G, ex, net, st, valid,
          ((unsigned long long)gi << 44) ^ ((unsigned long long)st->step << 24) ^
              ((unsigned long long)row * (d.nx + 1) + (i + 1)) * 2ull);

      // WRITE: cells x0 .. x0+59
      if (lane >= 2 && lane < 62 && i < d.nx) {
        if constexpr (STAGE) {
          const int k = i & (kXRing - 1);
          wring[0][k] = c.r;
          wring[1][k] = c.n;
          wring[2][k] = c.t;
          wring[3][k] = c.e;
        } else {
          const unsigned oo = (unsigned)i * (unsigned)sizeof(T);
          *ptr_at(out0, oo) = c.r;
          *ptr_at(out1, oo) = c.n;
          *ptr_at(out2, oo) = c.t;
          *ptr_at(out3, oo) = c.e;
          if constexpr (NS > 0) outp[4 * P + i] = c.s;
        }
        status |= nonphysical(c.r, c.e) ? kStatusNonPhys : 0;
        if constexpr (FUSE) smax = fmax(smax, max_speed(c.r, c.n, c.t, c.e, G));
      }
      if constexpr (STAGE) {
        __builtin_amdgcn_wave_barrier();
        flush(min(x0 + kXOut, d.nx), false);
        __builtin_amdgcn_wave_barrier();
      }
    }
    if constexpr (STAGE) {
      flush(min((seg0 + b.seg) * kXOut, d.nx), true);
      __builtin_amdgcn_wave_barrier();
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
  // the learned guess's network, staged in LDS once per block
  __shared__ MlpInfer net_lds;
  const MlpInfer* net = nullptr;
  if constexpr (GUESS != 0) {
    mlp_stage(ex.mlp, &net_lds);
    net = &net_lds;
  }
  for (long long w = first_wave(); w < b.items; w += wave_stride()) {
    const int gi = find_grid<Key::Y>(b.g, b.ngrids, w);
    const GridDesc d = load_desc(b.g, gi);
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
    // the grid's variable planes from scalar registers and the lane's column
    // as a 32-bit byte offset (the compiler folds the two into one 64-bit
    // address per plane and lane once per work item and adds each row's
    // offset to it; rows through buffer descriptors, which keep that addition
    // scalar, timed no better)
    const auto in0 = uniform_ptr(b.src + d.off), in1 = uniform_ptr(b.src + d.off + P);
    const auto in2 = uniform_ptr(b.src + d.off + 2 * P), in3 = uniform_ptr(b.src + d.off + 3 * P);
    const auto out0 = uniform_ptr(b.dst + d.off), out1 = uniform_ptr(b.dst + d.off + P);
    const auto out2 = uniform_ptr(b.dst + d.off + 2 * P), out3 = uniform_ptr(b.dst + d.off + 3 * P);
    const long long pitch = d.pitch;
    const unsigned xo_in = (unsigned)(xin ? x : d.nx - 1) * (unsigned)sizeof(T);
    const unsigned xo_out = (unsigned)x * (unsigned)sizeof(T);

    auto load = [&](int j) {
      bool flip;
      const long long off = (long long)ghost_source(j, d.ny, d.bc, flip) * pitch;
      Cell<T> c;
      c.r = at(in0 + off, xo_in);
      c.t = at(in1 + off, xo_in);  // rho u: transverse
      c.n = at(in2 + off, xo_in);  // rho v: normal
      c.e = at(in3 + off, xo_in);
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
          int iters;
          bool conv, fb, left;
          T pstar;
          F = interface_flux<RS, false, GUESS>(qpA, qmB, G, ex, net, iters, conv, fb, pstar, left);
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
            const long long off = (long long)j * pitch;
            __builtin_nontemporal_store(nr, ptr_at(out0 + off, xo_out));
            __builtin_nontemporal_store(nt, ptr_at(out1 + off, xo_out));
            __builtin_nontemporal_store(nn, ptr_at(out2 + off, xo_out));
            __builtin_nontemporal_store(ne, ptr_at(out3 + off, xo_out));
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
          int iters;
          bool conv, fb, left;
          T pstar;
          F = interface_flux<RS, false, GUESS>(qp0, qm1, G, ex, net, iters, conv, fb, pstar, left);
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
            const long long off = (long long)j * pitch;
            // streaming stores: the next sweep reads these only after the
            // whole grid (faster here; the x-sweep streams only whole aligned
            // blocks, since streaming stores that start or end inside a line
            // are slower than plain ones)
            __builtin_nontemporal_store(nr, ptr_at(out0 + off, xo_out));
            __builtin_nontemporal_store(nt, ptr_at(out1 + off, xo_out));
            __builtin_nontemporal_store(nn, ptr_at(out2 + off, xo_out));
            __builtin_nontemporal_store(ne, ptr_at(out3 + off, xo_out));
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

// ------------------------------------------------------------ tiled y-sweep
// The y-sweep in the x-sweep's form, through a tile transposed in LDS (the
// alternative to the column march above; option ysweep = tile).  A work item
// is a block-wide tile: kTileCols columns by 64 rows (the 60 rows it updates
// and two ghost rows on each side), read row-coalesced into LDS with the
// boundary rule in the row index remap.  Each wave then takes every fourth
// column of the tile as a 64-lane pencil segment (pencil_segment, one cell per
// lane), writes the updated cells back into its own column of the tile, and
// after a barrier the block stores the 60 rows row-coalesced.  Tile columns
// are XOR-swizzled by row (tile_col) so that both the row-wise fill and the
// column-wise lane reads hit distinct LDS banks.  Same numerics as the x-sweep
// (the same device code), so results equal the march to rounding; per updated
// cell it executes the 64/60 lanes of a segment and the shuffles of the x-sweep
// instead of the march's register window.
// LDS column of tile element (r, c): c XOR a function of the row, so that the
// 16 lanes of a wave that the LDS serves together (a row-wise fill: one row
// per 16 lanes; a column read: 16 consecutive rows) fall on distinct banks of
// the 32 4-byte banks.  A row of 16 FP64 values spans all 32 banks, so
// consecutive rows take different XOR keys; a row of 16 FP32 values spans
// half of them, so pairs of rows share a key.
template <typename T>
__device__ __forceinline__ int tile_col(int r, int c) {
  return c ^ ((sizeof(T) == 8 ? r : r >> 1) & (kTileCols - 1));
}

template <typename T, bool INSTR, int GUESS, int LIM, bool FUSE, int RS, int NS>
__global__ __launch_bounds__(256, (SweepOcc<T, GUESS, RS, NS>::t)) void k_sweep_y_tile(Batch<T> b, Gas<T> G, Extras ex) {
  constexpr int NV = 4 + NS;
  const Nbr nb = lane_neighbours();
  __shared__ T tile[NV][kTileRows][kTileCols];
  const int tid = threadIdx.x;
  // the learned guess's network, staged in LDS once per block
  __shared__ MlpInfer net_lds;
  const MlpInfer* net = nullptr;
  if constexpr (GUESS != 0) {
    mlp_stage(ex.mlp, &net_lds);
    net = &net_lds;
  }

  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
  int status = 0;
  T smax = T(0);  // max wave speed of the written cells (FUSE), per grid
  int gcur = -1;  // grid smax belongs to
  for (long long it = blockIdx.x; it < b.items; it += gridDim.x) {
    const int gi = find_grid<Key::Tile>(b.g, b.ngrids, it);
    const GridDesc d = load_desc(b.g, gi);
    DevState* st = b.st + gi;
    if (gi != gcur) {  // flush the previous grid's status and max speed
      if (gcur >= 0) {
        if (status) atomicOr(&b.st[gcur].status, status);
        if constexpr (FUSE) {
          const double wmax = wave_max((double)smax);
          if (lane == 0) fold_max(&b.st[gcur].acc, wmax);
        }
      }
      status = 0;
      smax = T(0);
      gcur = gi;
    }
    const int li = (int)(it - d.wt0);
    const int ncols = (d.nx + kTileCols - 1) / kTileCols;
    const int ty = li / ncols;
    const int x0 = (li - ty * ncols) * kTileCols;
    const int y0 = ty * kTileOut;
    const T lam = T(st->dt / d.h);
    const long long P = d.plane;
    // READ: rows y0-2 .. y0+61 (ghost rows by index remap, rows past ny+1
    // clamped), columns x0 .. x0+15 (past nx clamped); planes in pencil order
    // (rho, normal rho v, transverse rho u, E, rho X)
#pragma unroll
    for (int k = 0; k < kTileRows * kTileCols / 256; ++k) {
      const int e = tid + 256 * k;
      const int r = e / kTileCols, cl = e % kTileCols;
      bool flip;
      const int src = ghost_source(min(y0 - 2 + r, d.ny + 1), d.ny, d.bc, flip);
      const T* p = b.src + d.off + (long long)src * d.pitch + min(x0 + cl, d.nx - 1);
      const int cc = tile_col<T>(r, cl);
      const T vr = p[0], vu = p[P], vv = p[2 * P], ve = p[3 * P];
      tile[0][r][cc] = vr;
      tile[1][r][cc] = flip ? -vv : vv;
      tile[2][r][cc] = vu;
      tile[3][r][cc] = ve;
      if constexpr (NS > 0) tile[4][r][cc] = p[4 * P];
    }
    __syncthreads();
    // COMPUTE: wave wv takes columns wv, wv+4, ...; lane l is row y0-2+l
    const int i = y0 - 2 + lane;
    for (int cl = wv; cl < kTileCols && x0 + cl < d.nx; cl += kWavesPerBlock) {
      const int cc = tile_col<T>(lane, cl);
      Lane<T> c;
      c.r = tile[0][lane][cc];
      c.n = tile[1][lane][cc];
      c.t = tile[2][lane][cc];
      c.e = tile[3][lane][cc];
      c.s = T(0);
      if constexpr (NS > 0) c.s = tile[4][lane][cc];
      // interfaces owned: y0-1/2 (first tile only) and the right interfaces
      // of the updated rows
      const bool valid = (lane >= 2 || (lane == 1 && y0 == 0)) && lane < 62 && i < d.ny;
      const int x = x0 + cl;
      pencil_segment<T, INSTR, GUESS, LIM, RS, NS>(
          c, nb, lam, G, ex, net, st, valid,
          ((unsigned long long)gi << 44) ^ ((unsigned long long)st->step << 24) ^
              (((unsigned long long)x * (d.ny + 1) + (i + 1)) * 2ull + 1ull));
      if (lane >= 2 && lane < 62 && i < d.ny) {
        tile[0][lane][cc] = c.r;
        tile[1][lane][cc] = c.n;
        tile[2][lane][cc] = c.t;
        tile[3][lane][cc] = c.e;
        if constexpr (NS > 0) tile[4][lane][cc] = c.s;
        status |= nonphysical(c.r, c.e) ? kStatusNonPhys : 0;
        if constexpr (FUSE) smax = fmax(smax, max_speed(c.r, c.n, c.t, c.e, G));
      }
    }
    __syncthreads();
    // WRITE: rows y0 .. y0+59 (below ny), columns x0 .. x0+15 (below nx)
#pragma unroll
    for (int k = 0; k < (kTileOut * kTileCols + 255) / 256; ++k) {
      const int e = tid + 256 * k;
      const int r = e / kTileCols, cl = e % kTileCols;
      const int j = y0 + r, x = x0 + cl;
      if (e < kTileOut * kTileCols && j < d.ny && x < d.nx) {
        const int cc = tile_col<T>(r + 2, cl);
        T* p = b.dst + d.off + (long long)j * d.pitch + x;
        __builtin_nontemporal_store(tile[0][r + 2][cc], p);
        __builtin_nontemporal_store(tile[2][r + 2][cc], p + P);
        __builtin_nontemporal_store(tile[1][r + 2][cc], p + 2 * P);
        __builtin_nontemporal_store(tile[3][r + 2][cc], p + 3 * P);
        if constexpr (NS > 0) __builtin_nontemporal_store(tile[4][r + 2][cc], p + 4 * P);
      }
    }
    __syncthreads();  // the next item refills the tile
  }
  if (gcur >= 0) {
    if (status) atomicOr(&b.st[gcur].status, status);
    if constexpr (FUSE) {
      const double wmax = wave_max((double)smax);
      if (lane == 0) fold_max(&b.st[gcur].acc, wmax);
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
  else if constexpr (DIR == 1)
    return &k_sweep_y<T, I, GS, L, F, RS, NS>;
  else
    return &k_sweep_y_tile<T, I, GS, L, F, RS, NS>;
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
