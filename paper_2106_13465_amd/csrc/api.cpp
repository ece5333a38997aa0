// api.cpp -- the C ABI of include/hydro.h: handle life cycle, argument
// validation, error reporting, and the order in which a time step enqueues
// its kernels (dt, x-sweep, y-sweep; paper, Figure 5).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "hydro.h"
#include "launch.hpp"

using hydro::DevState;
using hydro::Gas;
using hydro::GridArgs;

struct hydro_s {
  int nx, ny, bc;
  double gamma, cfl, h;
  hydro_options_t opt;
  int device;
  DevState* st;       // device scratch
  double* partials;   // device, totals_blocks() * 4
  void* U;            // bound state (caller-owned)
  void* V;            // second state buffer of the same size (handle-owned)
  size_t v_bytes;
  long pitch;
  int dtype;
  hipStream_t stream;
  bool bound;
  bool acc_valid;     // st->acc holds the max speed of the current U
  // kernel timing: event pairs recorded around the phases of hydro_step
  bool profiling;
  std::vector<hipEvent_t> ev_pool;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  // captured multi-step graph
  hipGraphExec_t gexec;
  int graph_steps;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int dev_fail(hipError_t e, const char* what) {
  return fail(HYDRO_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

hydro_options_t default_options() {
  hydro_options_t o;
  std::memset(&o, 0, sizeof o);
  o.niter = 10;
  o.tol = 1e-8;
  o.guess = HYDRO_GUESS_PTR;
  o.stats = 0;
  o.seg_x = 0;
  o.seg_y = 0;
  return o;
}

template <typename T>
Gas<T> make_gas(double g, const hydro_options_t& o) {
  Gas<T> G;
  const double z = (g - 1.0) / (2.0 * g);
  G.g = T(g);
  G.gm1 = T(g - 1.0);
  G.gs = T((g + 1.0) / (2.0 * g));
  G.z = T(z);
  G.inv_z = T(1.0 / z);
  G.half_gm1 = T(0.5 * (g - 1.0));
  G.h_coef = T(g / (g - 1.0));
  G.pfloor = T(hydro::kCMin * hydro::kCMin / g);
  G.rho_min = T(hydro::kRhoMin);
  G.inv_rho_min = T(1.0 / hydro::kRhoMin);
  G.c_min = T(hydro::kCMin);
  // Convergence can only be detected above the arithmetic's rounding noise:
  // in FP32 the test is floored at 8 ulp of 1.
  const double tol_floor = sizeof(T) == 4 ? 8.0 * 1.1920928955078125e-07 : 0.0;
  G.tol = T(o.tol > tol_floor ? o.tol : tol_floor);
  G.niter = o.niter;
  // 1/z = 2 gamma / (gamma - 1); an integer exponent (7 for gamma = 1.4) lets
  // the guess use repeated squaring instead of exp2/log2
  const double k = std::nearbyint(1.0 / z);
  G.ipow_k = (k >= 1.0 && k <= 64.0 && std::fabs(1.0 / z - k) <= 1e-12 * k) ? (int)k : 0;
  return G;
}

// Sweeps never update in place: each reads one buffer and writes the other.
template <typename T>
GridArgs<T> grid_args(const hydro_t* h, const void* src, void* dst) {
  GridArgs<T> a;
  a.src = static_cast<const T*>(src);
  a.dst = static_cast<T*>(dst);
  a.pitch = (int)h->pitch;
  a.plane = (long long)h->pitch * h->ny;
  a.nx = h->nx;
  a.ny = h->ny;
  a.bc = h->bc;
  a.h = h->h;
  a.cfl = h->cfl;
  return a;
}

int seg_x_of(const hydro_t* h) { return h->opt.seg_x > 0 ? h->opt.seg_x : 1; }
int seg_y_of(const hydro_t* h) {
  int s = h->opt.seg_y > 0 ? h->opt.seg_y : 128;
  return s < h->ny ? s : h->ny;
}

template <typename T>
hipError_t enqueue_sweep(hydro_t* h, int dir, bool fuse_dt, const void* src, void* dst) {
  const GridArgs<T> a = grid_args<T>(h, src, dst);
  const Gas<T> G = make_gas<T>(h->gamma, h->opt);
  if (dir == HYDRO_DIR_X)
    return hydro::launch_sweep_x<T>(a, G, h->st, seg_x_of(h), h->opt.stats != 0, h->stream);
  return hydro::launch_sweep_y<T>(a, G, h->st, seg_y_of(h), fuse_dt, h->opt.stats != 0,
                                  h->stream);
}

template <typename T>
hipError_t enqueue_max_speed(hydro_t* h) {
  hipError_t e = hydro::launch_reset_acc(h->st, h->stream);
  if (e != hipSuccess) return e;
  return hydro::launch_max_speed<T>(grid_args<T>(h, h->U, nullptr),
                                    make_gas<T>(h->gamma, h->opt), h->st, h->stream);
}

template <typename T>
hipError_t enqueue_totals(hydro_t* h) {
  return hydro::launch_totals<T>(grid_args<T>(h, h->U, nullptr), h->partials, h->st,
                                 h->stream);
}

// One standalone sweep: U -> V, then V copied back into U.
template <typename T>
hipError_t enqueue_single_sweep(hydro_t* h, int dir) {
  hipError_t e = enqueue_sweep<T>(h, dir, false, h->U, h->V);
  if (e != hipSuccess) return e;
  return hydro::launch_copy<T>(grid_args<T>(h, h->V, h->U), h->stream);
}

// Event pair around one phase of a step (no-op unless profiling and the
// stream is not being captured).
struct PhaseTimer {
  hydro_t* h;
  int phase;
  hipEvent_t a = nullptr, b = nullptr;
  PhaseTimer(hydro_t* h_, int phase_) : h(h_), phase(phase_) {
    if (!h->profiling) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return;
    a = take();
    b = take();
    if (a && b) (void)hipEventRecord(a, h->stream);
  }
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!h->ev_pool.empty()) {
      e = h->ev_pool.back();
      h->ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  ~PhaseTimer() {
    if (a && b) {
      (void)hipEventRecord(b, h->stream);
      h->marks.push_back({phase, a, b});
    } else {
      if (a) h->ev_pool.push_back(a);
      if (b) h->ev_pool.push_back(b);
    }
  }
};

void drop_graph(hydro_t* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
  h->graph_steps = 0;
}

// The kernels of one step: dt from the accumulated max speed, x-sweep U -> V,
// y-sweep V -> U with the next max speed fused.  Requires st->acc to hold the
// max speed of U (acc_valid).
hipError_t enqueue_step_body(hydro_t* h) {
  const bool f64 = h->dtype == HYDRO_F64;
  hipError_t e;
  {
    PhaseTimer pt(h, HYDRO_PHASE_DT);
    e = hydro::launch_finalize_dt(h->st, h->cfl, h->h, true, true, h->stream);
  }
  if (e != hipSuccess) return e;
  {
    PhaseTimer pt(h, HYDRO_PHASE_SWEEP_X);
    e = f64 ? enqueue_sweep<double>(h, HYDRO_DIR_X, false, h->U, h->V)
            : enqueue_sweep<float>(h, HYDRO_DIR_X, false, h->U, h->V);
  }
  if (e != hipSuccess) return e;
  PhaseTimer pt(h, HYDRO_PHASE_SWEEP_Y);
  return f64 ? enqueue_sweep<double>(h, HYDRO_DIR_Y, true, h->V, h->U)
             : enqueue_sweep<float>(h, HYDRO_DIR_Y, true, h->V, h->U);
}

int check_bound(const hydro_t* h) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  if (!h->bound) return fail(HYDRO_ESTATE, "no state bound (call hydro_bind first)");
  return HYDRO_OK;
}

// Copies the device scratch to the host after the stream drains; reports a
// latched non-physical state once and clears it.
int sync_state(hydro_t* h, DevState* out) {
  hipError_t e = hipMemcpyAsync(out, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return dev_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_fail(e, "hipStreamSynchronize");
  if (out->status != 0) {
    int zero = 0;
    e = hipMemcpyAsync(&h->st->status, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_fail(e, "status reset");
    return fail(HYDRO_ENONPHYS, "a sweep produced a non-physical state (status 0x%x)",
                out->status);
  }
  return HYDRO_OK;
}

}  // namespace

extern "C" {

const char* hydro_last_error(void) { return g_err; }

hydro_t* hydro_create(int nx, int ny, double gamma, double cfl, int bc) {
  if (nx < 2 || ny < 2) {
    fail(HYDRO_EINVAL, "grid %d x %d: both sides must be >= 2", nx, ny);
    return nullptr;
  }
  if ((long long)nx * ny * 4 >= (1ll << 40)) {
    fail(HYDRO_EINVAL, "grid %d x %d too large", nx, ny);
    return nullptr;
  }
  if (!(gamma > 1.0) || !std::isfinite(gamma)) {
    fail(HYDRO_EINVAL, "gamma = %g: must be > 1", gamma);
    return nullptr;
  }
  if (!(cfl > 0.0 && cfl <= 1.0)) {
    fail(HYDRO_EINVAL, "cfl = %g: must be in (0, 1]", cfl);
    return nullptr;
  }
  if (bc != HYDRO_BC_REFLECT && bc != HYDRO_BC_OUTFLOW && bc != HYDRO_BC_PERIODIC) {
    fail(HYDRO_EINVAL, "bc = %d: not a HYDRO_BC_* value", bc);
    return nullptr;
  }
  hydro_t* h = new (std::nothrow) hydro_s();
  if (!h) {
    fail(HYDRO_ENOMEM, "host allocation failed");
    return nullptr;
  }
  h->nx = nx;
  h->ny = ny;
  h->bc = bc;
  h->gamma = gamma;
  h->cfl = cfl;
  h->h = 1.0 / (double)(nx > ny ? nx : ny);
  h->opt = default_options();
  h->st = nullptr;
  h->partials = nullptr;
  h->U = nullptr;
  h->V = nullptr;
  h->v_bytes = 0;
  h->bound = false;
  h->acc_valid = false;
  h->stream = nullptr;
  h->profiling = false;
  h->gexec = nullptr;
  h->graph_steps = 0;
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = hipMalloc((void**)&h->st, sizeof(DevState));
  if (e == hipSuccess)
    e = hipMalloc((void**)&h->partials, sizeof(double) * 4 * hydro::totals_blocks());
  if (e == hipSuccess) e = hipMemset(h->st, 0, sizeof(DevState));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    dev_fail(e, "hydro_create");
    hydro_destroy(h);
    return nullptr;
  }
  return h;
}

void hydro_destroy(hydro_t* h) {
  if (!h) return;
  DeviceGuard g(h->device);
  if (h->bound && h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->st) (void)hipFree(h->st);
  if (h->partials) (void)hipFree(h->partials);
  if (h->V) (void)hipFree(h->V);
  drop_graph(h);
  for (auto& m : h->marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
}

int hydro_bind(hydro_t* h, void* U, long pitch, int dtype, void* hip_stream) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  if (!U) return fail(HYDRO_EINVAL, "NULL state pointer");
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return fail(HYDRO_EINVAL, "dtype %d", dtype);
  if (pitch < h->nx) return fail(HYDRO_EINVAL, "pitch %ld < nx %d", pitch, h->nx);
  if ((long long)pitch * h->ny * 4 >= (1ll << 40) || pitch > (1l << 30))
    return fail(HYDRO_EINVAL, "pitch %ld too large", pitch);
  const size_t elem = dtype == HYDRO_F64 ? 8 : 4;
  if (((uintptr_t)U) % elem != 0) return fail(HYDRO_EINVAL, "state pointer misaligned");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, U) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(HYDRO_EINVAL, "state pointer is not device memory");
  }
  if (attr.device != h->device)
    return fail(HYDRO_EINVAL, "state on device %d, handle on device %d", attr.device, h->device);
  const size_t bytes = elem * 4 * (size_t)pitch * (size_t)h->ny;
  if (h->v_bytes != bytes) {
    DeviceGuard g(h->device);
    if (h->V) {
      if (h->bound && h->stream) (void)hipStreamSynchronize(h->stream);
      (void)hipFree(h->V);
      h->V = nullptr;
      h->v_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->V, bytes);
    if (e != hipSuccess) {
      h->V = nullptr;
      h->bound = false;
      return fail(HYDRO_ENOMEM, "second state buffer (%zu bytes): %s", bytes,
                  hipGetErrorString(e));
    }
    h->v_bytes = bytes;
  }
  drop_graph(h);
  h->U = U;
  h->pitch = pitch;
  h->dtype = dtype;
  h->stream = (hipStream_t)hip_stream;
  h->bound = true;
  h->acc_valid = false;
  return HYDRO_OK;
}

int hydro_invalidate(hydro_t* h) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  h->acc_valid = false;
  return HYDRO_OK;
}

int hydro_set_options(hydro_t* h, const hydro_options_t* o) {
  if (!h || !o) return fail(HYDRO_EINVAL, "NULL argument");
  if (o->niter < 1 || o->niter > HYDRO_MAX_NITER)
    return fail(HYDRO_EINVAL, "niter %d: must be in 1..%d", o->niter, HYDRO_MAX_NITER);
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(HYDRO_EINVAL, "tol %g", o->tol);
  if (o->guess != HYDRO_GUESS_PTR)
    return fail(HYDRO_EINVAL, "guess %d not available on this handle", o->guess);
  if (o->seg_x < 0 || o->seg_x > 4096) return fail(HYDRO_EINVAL, "seg_x %d", o->seg_x);
  if (o->seg_y < 0 || o->seg_y > (1 << 20)) return fail(HYDRO_EINVAL, "seg_y %d", o->seg_y);
  h->opt = *o;
  drop_graph(h);
  return HYDRO_OK;
}

int hydro_get_options(const hydro_t* h, hydro_options_t* o) {
  if (!h || !o) return fail(HYDRO_EINVAL, "NULL argument");
  *o = h->opt;
  return HYDRO_OK;
}

double hydro_compute_dt(hydro_t* h) {
  int rc = check_bound(h);
  if (rc) return rc;
  DeviceGuard g(h->device);
  hipError_t e = h->dtype == HYDRO_F64 ? enqueue_max_speed<double>(h) : enqueue_max_speed<float>(h);
  if (e == hipSuccess) e = hydro::launch_finalize_dt(h->st, h->cfl, h->h, false, false, h->stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_compute_dt");
  DevState s;
  rc = sync_state(h, &s);
  if (rc) {
    h->acc_valid = false;
    return rc;
  }
  h->acc_valid = true;
  return s.dt;
}

int hydro_sweep(hydro_t* h, int dir) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (dir != HYDRO_DIR_X && dir != HYDRO_DIR_Y) return fail(HYDRO_EINVAL, "dir %d", dir);
  DeviceGuard g(h->device);
  hipError_t e = h->dtype == HYDRO_F64 ? enqueue_single_sweep<double>(h, dir)
                                       : enqueue_single_sweep<float>(h, dir);
  h->acc_valid = false;
  if (e != hipSuccess) return dev_fail(e, "hydro_sweep");
  return HYDRO_OK;
}

int hydro_step(hydro_t* h) {
  int rc = check_bound(h);
  if (rc) return rc;
  DeviceGuard g(h->device);
  hipError_t e = hipSuccess;
  if (!h->acc_valid) {
    PhaseTimer pt(h, HYDRO_PHASE_DT);
    e = h->dtype == HYDRO_F64 ? enqueue_max_speed<double>(h) : enqueue_max_speed<float>(h);
  }
  if (e == hipSuccess) e = enqueue_step_body(h);
  if (e != hipSuccess) {
    h->acc_valid = false;
    return dev_fail(e, "hydro_step");
  }
  h->acc_valid = true;
  return HYDRO_OK;
}

int hydro_graph_steps(hydro_t* h, int nsteps) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (nsteps < 1 || nsteps > 4096) return fail(HYDRO_EINVAL, "nsteps %d: 1..4096", nsteps);
  if (h->stream == nullptr)
    return fail(HYDRO_ESTATE, "graph capture needs a non-default stream (hydro_bind)");
  DeviceGuard g(h->device);
  hipError_t e = hipSuccess;
  if (!h->acc_valid) {
    // the graph starts from a valid max speed; compute it eagerly once
    e = h->dtype == HYDRO_F64 ? enqueue_max_speed<double>(h) : enqueue_max_speed<float>(h);
    if (e != hipSuccess) return dev_fail(e, "hydro_graph_steps");
    h->acc_valid = true;
  }
  if (!h->gexec || h->graph_steps != nsteps) {
    drop_graph(h);
    const bool prof = h->profiling;
    h->profiling = false;
    e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
    for (int i = 0; e == hipSuccess && i < nsteps; ++i) e = enqueue_step_body(h);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
    h->profiling = prof;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      h->gexec = nullptr;
      return dev_fail(e, "graph capture");
    }
    h->graph_steps = nsteps;
  }
  e = hipGraphLaunch(h->gexec, h->stream);
  if (e != hipSuccess) return dev_fail(e, "hipGraphLaunch");
  return HYDRO_OK;
}

int hydro_conserved_totals(hydro_t* h, double out[4]) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!out) return fail(HYDRO_EINVAL, "NULL output");
  DeviceGuard g(h->device);
  hipError_t e = h->dtype == HYDRO_F64 ? enqueue_totals<double>(h) : enqueue_totals<float>(h);
  if (e != hipSuccess) return dev_fail(e, "hydro_conserved_totals");
  DevState s;
  rc = sync_state(h, &s);
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) out[k] = s.totals[k];
  return HYDRO_OK;
}

int hydro_get_clock(hydro_t* h, double* t, long* step, double* dt) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  DeviceGuard g(h->device);
  DevState s;
  hipError_t e = hipMemcpyAsync(&s, h->st, sizeof s, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_get_clock");
  if (t) *t = s.t;
  if (step) *step = (long)s.step;
  if (dt) *dt = s.dt;
  return HYDRO_OK;
}

int hydro_set_clock(hydro_t* h, double t, long step) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  if (!std::isfinite(t) || step < 0) return fail(HYDRO_EINVAL, "clock t=%g step=%ld", t, step);
  DeviceGuard g(h->device);
  hipError_t e = hydro::launch_set_clock(h->st, t, step, h->stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_set_clock");
  return HYDRO_OK;
}

int hydro_riemann_stats(hydro_t* h, hydro_stats_t* out, int reset) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  DeviceGuard g(h->device);
  DevState s;
  hipError_t e = hipMemcpyAsync(&s, h->st, sizeof s, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_riemann_stats");
  if (out) {
    std::memset(out, 0, sizeof *out);
    out->interfaces = (long long)s.interfaces;
    for (int k = 0; k <= HYDRO_MAX_NITER; ++k) out->hist[k] = (long long)s.hist[k];
    out->fallbacks = (long long)s.fallbacks;
  }
  if (reset) {
    e = hydro::launch_clear_stats(h->st, h->stream);
    if (e != hipSuccess) return dev_fail(e, "stats reset");
  }
  return HYDRO_OK;
}

int hydro_set_profiling(hydro_t* h, int enable) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  h->profiling = enable != 0;
  return HYDRO_OK;
}

int hydro_get_profile(hydro_t* h, double ms[HYDRO_NPHASES], long long launches[HYDRO_NPHASES],
                      int reset) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  DeviceGuard g(h->device);
  if (h->stream || h->bound) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return dev_fail(e, "hydro_get_profile");
  }
  double acc[HYDRO_NPHASES] = {0, 0, 0};
  long long cnt[HYDRO_NPHASES] = {0, 0, 0};
  for (const auto& m : h->marks) {
    float t = 0.f;
    hipError_t e = hipEventElapsedTime(&t, m.a, m.b);
    if (e != hipSuccess) return dev_fail(e, "hipEventElapsedTime");
    acc[m.phase] += t;
    cnt[m.phase] += 1;
  }
  for (int k = 0; k < HYDRO_NPHASES; ++k) {
    if (ms) ms[k] = acc[k];
    if (launches) launches[k] = cnt[k];
  }
  if (reset) {
    for (const auto& m : h->marks) {
      h->ev_pool.push_back(m.a);
      h->ev_pool.push_back(m.b);
    }
    h->marks.clear();
  }
  return HYDRO_OK;
}

}  // extern "C"
