// launch.hpp -- host-side launchers of the sweep, dt and totals kernels.
// All enqueue on the given stream and return the launch status.
#pragma once
#include <hip/hip_runtime.h>

#include "device_state.hpp"

namespace hydro {

template <typename T>
hipError_t launch_sweep_x(const GridArgs<T>& a, const Gas<T>& G, DevState* st, int segs,
                          bool stats, hipStream_t s);
template <typename T>
hipError_t launch_sweep_y(const GridArgs<T>& a, const Gas<T>& G, DevState* st, int seg,
                          bool fuse_dt, bool stats, hipStream_t s);
template <typename T>
hipError_t launch_max_speed(const GridArgs<T>& a, const Gas<T>& G, DevState* st, hipStream_t s);
template <typename T>
hipError_t launch_totals(const GridArgs<T>& a, double* partials, DevState* st, hipStream_t s);

template <typename T>
hipError_t launch_copy(const GridArgs<T>& a, hipStream_t s);

hipError_t launch_reset_acc(DevState* st, hipStream_t s);
hipError_t launch_finalize_dt(DevState* st, double cfl, double h, bool advance, bool reset,
                              hipStream_t s);
hipError_t launch_set_clock(DevState* st, double t, long long step, hipStream_t s);
hipError_t launch_clear_stats(DevState* st, hipStream_t s);
int totals_blocks();

}  // namespace hydro
