// device_state.hpp -- plain structs shared by the kernels and the host side of
// the library: the per-grid kernel arguments and the small device-resident
// scratch of a handle (time step, clock, max-speed accumulator, status word,
// Riemann statistics, totals).
#pragma once
#include <stdint.h>

#include "godunov.hpp"

namespace hydro {

constexpr int kMaxIter = 32;      // largest Newton cap (HYDRO_MAX_NITER)
constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kXOut = kWave - 4;  // x-sweep cells updated per 64-lane segment

// status word bits
constexpr int kStatusNonPhys = 1;

struct DevState {
  double dt;        // time step the sweeps use
  double t;         // simulated time
  double smax;      // max wave speed dt was computed from
  long long step;   // steps taken
  unsigned long long acc;  // running max wave speed: bits of a double >= 0
  int status;       // kStatus* bits, latched
  int pad0;
  double totals[4];
  unsigned long long interfaces;          // Riemann problems counted
  unsigned long long hist[kMaxIter + 1];  // [0] unconverged, [k] k iterations
  unsigned long long fallbacks;
};

// One grid of the state: plane v of cell (x, y) at U[v * plane + y * pitch + x].
// A sweep reads src and writes dst (distinct buffers of the same layout), so
// no wave ever reads a cell another wave has already updated.
template <typename T>
struct GridArgs {
  const T* src;
  T* dst;
  long long plane;
  int pitch;
  int nx, ny;
  int bc;
  double h;    // cell size
  double cfl;
};

}  // namespace hydro
