// launch.hpp -- host-side launchers of the batch kernels.  All enqueue on the
// given stream and return the launch status.  max_blocks = 0 launches one
// block per four work items; a smaller positive value makes the sweep
// persistent (each wave strides over items).
#pragma once
#include <hip/hip_runtime.h>

#include "device_state.hpp"

namespace hydro {

// instr: Newton statistics and (if ex.log) the interface logger; guess: 1 =
// learned starting guess from ex.mlp.  With ex.fuse the sweep folds the max
// wave speed of its output into st[].acc (the last sweep of a step).  These,
// G.limiter, G.riemann and the passive scalars (b.nv - 4) pick a compiled
// variant of the kernel (values outside the built ones return
// hipErrorInvalidValue); with the HLLC flux instr and guess are ignored.
template <typename T>
hipError_t launch_sweep_x(const Batch<T>& b, const Gas<T>& G, const Extras& ex, bool instr,
                          int guess, unsigned max_blocks, hipStream_t s);
template <typename T>
hipError_t launch_sweep_y(const Batch<T>& b, const Gas<T>& G, const Extras& ex, bool instr,
                          int guess, unsigned max_blocks, hipStream_t s);
// The y-sweep through LDS tiles: b.items tiles (GridDesc::wt0 prefixes), one
// block per tile (max_blocks = 0) or persistent blocks.
template <typename T>
hipError_t launch_sweep_y_tile(const Batch<T>& b, const Gas<T>& G, const Extras& ex, bool instr,
                               int guess, unsigned max_blocks, hipStream_t s);
// Resident blocks per CU of the y-sweep variant (runtime occupancy query),
// for sizing its work items to whole rounds of the chip; 0 on error.
template <typename T>
int sweep_y_blocks_per_cu(bool instr, int guess, bool fuse, int limiter, int riemann, int ns);
template <typename T>
hipError_t launch_max_speed(const Batch<T>& b, const Gas<T>& G, hipStream_t s);
template <typename T>
hipError_t launch_copy(const Batch<T>& b, hipStream_t s);
template <typename T>
hipError_t launch_totals(const Batch<T>& b, int total_blocks, double* partials, hipStream_t s);

// Streaming copy of n16 16-byte words (n16 > 0; both pointers 16-byte aligned).
hipError_t launch_stream_copy(void* dst, const void* src, long long n16, hipStream_t s);
hipError_t launch_reset_acc(DevState* st, int n, hipStream_t s);
hipError_t launch_finalize_dt(const GridDesc* g, DevState* st, int n, bool advance, bool reset,
                              hipStream_t s);
hipError_t launch_set_clock(DevState* st, int i, double t, long long step, hipStream_t s);
hipError_t launch_clear_stats(DevState* st, int n, hipStream_t s);

}  // namespace hydro
