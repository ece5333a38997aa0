// plan.hpp -- host side of a batch of grids: geometry, device descriptors and
// scratch, the bound state buffers and stream, the launch shape, and the order
// in which a time step enqueues its kernels (dt, x-sweep, y-sweep; paper,
// Figure 5).  A single-grid handle is a plan with one grid.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "device_state.hpp"
#include "hydro.h"

namespace hydro {

// Launch shape of the two sweeps; results do not depend on it.
struct LaunchCfg {
  int seg_x = 8;          // 60-cell segments per x-sweep item (long items keep the
                          // x-sweep's staged stores line-aligned)
  int seg_y = 128;        // rows per y-sweep item
  unsigned blocks_x = 0;  // 0: one block per 4 items; else persistent
  unsigned blocks_y = 0;
};

struct Plan {
  // geometry
  int n = 0;
  std::vector<int> nx, ny, bc;
  std::vector<long> pitch;
  std::vector<long long> off;
  long long elems = 0;  // elements per state buffer
  double gamma = 1.4, cfl = 0.8;
  int nscalars = 0;     // passive scalars: the state has 4 + nscalars planes
  // options and launch shape
  hydro_options_t opt{};
  LaunchCfg cfg;
  bool user_seg_x = false, user_seg_y = false;
  // device
  int device = 0;
  int cus = 256;
  DevState* st = nullptr;     // [n]
  GridDesc* d_desc = nullptr;  // [n]
  std::vector<GridDesc> desc;
  double* partials = nullptr;
  int tot_blocks = 0;
  long long items_x = 0, items_y = 0, items_t = 0, rows = 0;
  // bound state
  void* U = nullptr;
  void* V = nullptr;  // second buffer (owned)
  size_t v_bytes = 0;
  int dtype = HYDRO_F64;
  hipStream_t stream = nullptr;
  bool bound = false;
  bool acc_valid = false;  // st[].acc holds the max speed of the current U
  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  // captured multi-step graph
  hipGraphExec_t gexec = nullptr;
  int graph_steps = 0;
  int graph_parity = 0;       // starting step parity the graph was captured for
  long long host_step = 0;    // steps enqueued (mirrors the device step count)
  // learned guess (borrowed device network) and interface logger
  const MlpDev* mlp = nullptr;
  float* log = nullptr;
  long long log_cap = 0;
  unsigned long long* log_count = nullptr;  // device counter (owned)
  unsigned long long log_seed = 0;
  float rate_smooth = 0.f, rate_strong = 0.f;

  ~Plan();

  // All return hipSuccess or the first HIP error.
  hipError_t init(int ngrids, const int* nx_, const int* ny_, const int* bc_, double gamma_,
                  double cfl_);
  hipError_t bind(void* U_, const long* pitches, const long long* offsets, int dtype_,
                  hipStream_t s);
  hipError_t set_options(const hydro_options_t& o);
  hipError_t set_logger(float* buf, long long cap, unsigned long long seed, double r_smooth,
                        double r_strong);
  hipError_t logger_count(unsigned long long* out);
  hipError_t upload_descriptors();  // after a change of geometry or launch shape
  void drop_graph();

  hipError_t enqueue_max_speed();          // st[].acc <- max speed of U
  hipError_t enqueue_finalize(bool advance, bool reset);
  hipError_t enqueue_sweep(int dir, bool fuse, const void* src, void* dst);
  hipError_t enqueue_step();  // dt (fused max), first sweep U->V, second V->U (fused max)
  hipError_t enqueue_single_sweep(int dir);  // U->V, copy back
  hipError_t enqueue_totals();
  hipError_t graph_launch(int nsteps);
  hipError_t sync_states(std::vector<DevState>& out);  // copies st[] after the stream drains

  // Times candidate launch shapes on the bound state (U is not modified) and
  // keeps the fastest; results are bitwise independent of the choice.
  hipError_t autotune(hydro_tune_t* out, bool use_cache);

  size_t elem_size() const { return dtype == HYDRO_F64 ? 8 : 4; }
};

// Row pitch (elements) padded to 256 bytes.
long padded_pitch(int nx, int dtype);

// Sets the calling thread's hydro_last_error message (printf format) and
// returns code.
int fail(int code, const char* fmt, ...);

// Solver options of a new handle: Newton cap 10, tolerance 1e-8, the
// two-rarefaction guess, minmod, x then y, the two-shock solver.
hydro_options_t default_options();

// Gas constants and solver settings of the sweep kernels for ratio of
// specific heats g and options o, in the kernel's arithmetic type.
template <typename T>
Gas<T> make_gas(double g, const hydro_options_t& o);

}  // namespace hydro
