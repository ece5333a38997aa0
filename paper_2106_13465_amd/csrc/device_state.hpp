// device_state.hpp -- plain structs shared by the kernels and the host side of
// the library: per-grid device scratch (time step, clock, max-speed
// accumulator, status word, Riemann statistics, totals), per-grid geometry and
// the kernel argument that describes a batch of grids.
//
// Every launch works on a batch: a single grid is a batch of one.  Grid g's
// state lives at offset GridDesc::off of two equally laid-out buffers; its
// variable plane v of cell (x, y) is at off + v * plane + y * pitch + x.  A
// sweep reads one buffer and writes the other, so no wave ever reads a cell
// another wave has already updated.  Planes 0..3 are rho, rho u, rho v, E;
// planes 4.. hold rho X for the passive scalars X.
#pragma once
#include <stdint.h>

#include "godunov.hpp"

namespace hydro {

constexpr int kMaxIter = 32;      // largest Newton cap (HYDRO_MAX_NITER)
constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kXOut = kWave - 4;  // x-sweep cells updated per 64-lane segment
constexpr int kXRing = 128;       // x-sweep store ring per wave and variable (> 63 + kXOut)
static_assert(kXRing >= 63 + kXOut && (kXRing & (kXRing - 1)) == 0, "ring size");
constexpr int kWavesPerBlock = 4;
constexpr int kTileCols = 16;        // tiled y-sweep: columns per tile
constexpr int kTileRows = kWave;     // ... rows held per tile (one per lane)
constexpr int kTileOut = kWave - 4;  // ... rows updated per tile
constexpr int kMaxTotBlocks = 512;  // partial-sum blocks per grid for totals
constexpr int kMaxScalars = 1;      // passive scalars (HYDRO_MAX_SCALARS)
constexpr int kMaxVars = 4 + kMaxScalars;

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
  double totals[kMaxVars];
  unsigned long long interfaces;          // Riemann problems counted
  unsigned long long hist[kMaxIter + 1];  // [0] unconverged, [k] k iterations
  unsigned long long wave_hist[kMaxIter + 1];  // waves by their largest count
  unsigned long long fallbacks;           // learned guesses rejected
};

struct MlpDev;

// Optional per-launch extras: the learned guess and the interface-state
// logger (records rho_L, u_L, p_L, rho_R, u_R, p_R, p*, jump strength along
// the sweep's normal direction).
struct Extras {
  const MlpDev* mlp;
  float* log;                      // [log_cap][8] or NULL
  unsigned long long* log_count;   // records offered so far (may exceed log_cap)
  long long log_cap;
  unsigned long long seed;
  float rate_smooth;               // sampling probability of weak jumps
  float rate_strong;               // ... of jumps with strength > 0.05
  float gamma;
  float gate_kappa;                // learned guess where pmax > kappa pmin (0: everywhere)
  float gate_theta2;               // ... or du^2 (rL+rR) > theta2 gamma (pL+pR)
  int fuse;                        // 1: fold the max wave speed of the sweep's
                                   // output into st[].acc (last sweep of a step)
};
constexpr int kLogFields = 8;

struct GridDesc {
  long long off;    // element offset of plane 0 in the state buffers
  long long plane;  // elements per variable plane (ny * pitch)
  int pitch, nx, ny, bc;
  double h;         // cell size 1/max(nx, ny)
  double cfl;
  long long wx0;    // first global wave of this grid in the x-sweep
  long long wy0;    // first global wave of this grid in the y-sweep
  long long wt0;    // first global tile of this grid in the tiled y-sweep
  long long r0;     // first global row (row-item kernels)
  int tb0;          // first partial block of the totals
  int ntb;          // partial blocks of the totals
};

// Kernel argument of one launch over a batch.
template <typename T>
struct Batch {
  const T* src;
  T* dst;
  const GridDesc* g;  // device array [ngrids]
  DevState* st;       // device array [ngrids]
  int ngrids;
  int seg;            // x-sweep: 60-cell segments per wave item; y-sweep: rows per item
  int nv;             // variable planes per grid: 4 + passive scalars
  long long items;    // waves (sweeps) or rows (row kernels) over the whole batch
};

}  // namespace hydro
