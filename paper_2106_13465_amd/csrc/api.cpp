// api.cpp -- the C ABI of include/hydro.h: argument validation, error
// reporting and thin wrappers over hydro::Plan.  A single-grid handle is a
// plan with one grid bound at offset 0 with the caller's pitch; a batch handle
// binds the packed layout of hydro_batch_layout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "hydro.h"
#include "launch.hpp"
#include "mlp.hpp"
#include "mlp_launch.hpp"
#include "plan.hpp"

struct hydro_s : hydro::Plan {};
struct hydro_batch_s : hydro::Plan {};

namespace hydro {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace hydro

namespace {

using hydro::fail;
using hydro::g_err;

int dev_fail(hipError_t e, const char* what) {
  return fail(HYDRO_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Makes the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int check_grid(int nx, int ny, int bc) {
  if (nx < 2 || ny < 2) return fail(HYDRO_EINVAL, "grid %d x %d: both sides must be >= 2", nx, ny);
  if (nx > (1 << 28) || ny > (1 << 28) || (long long)nx * ny >= (1ll << 38))
    return fail(HYDRO_EINVAL, "grid %d x %d too large", nx, ny);
  if (bc != HYDRO_BC_REFLECT && bc != HYDRO_BC_OUTFLOW && bc != HYDRO_BC_PERIODIC)
    return fail(HYDRO_EINVAL, "bc = %d: not a HYDRO_BC_* value", bc);
  return HYDRO_OK;
}

int check_gas(double gamma, double cfl) {
  if (!(gamma > 1.0) || !std::isfinite(gamma))
    return fail(HYDRO_EINVAL, "gamma = %g: must be > 1", gamma);
  if (!(cfl > 0.0 && cfl <= 1.0)) return fail(HYDRO_EINVAL, "cfl = %g: must be in (0, 1]", cfl);
  return HYDRO_OK;
}

template <typename H>
H* create_plan(int n, const int* nx, const int* ny, double gamma, double cfl, const int* bc) {
  if (n < 1 || !nx || !ny || !bc) {
    fail(HYDRO_EINVAL, "batch of %d grids (or NULL sizes)", n);
    return nullptr;
  }
  for (int g = 0; g < n; ++g)
    if (check_grid(nx[g], ny[g], bc[g])) return nullptr;
  if (check_gas(gamma, cfl)) return nullptr;
  H* h = new (std::nothrow) H();
  if (!h) {
    fail(HYDRO_ENOMEM, "host allocation failed");
    return nullptr;
  }
  hipError_t e = h->init(n, nx, ny, bc, gamma, cfl);
  if (e != hipSuccess) {
    dev_fail(e, "create");
    delete h;
    return nullptr;
  }
  return h;
}

int check_bound(const hydro::Plan* p) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  if (!p->bound) return fail(HYDRO_ESTATE, "no state bound (bind first)");
  return HYDRO_OK;
}

int check_options(const hydro::Plan* p, const hydro_options_t* o) {
  if (!o) return fail(HYDRO_EINVAL, "NULL options");
  if (o->niter < 1 || o->niter > HYDRO_MAX_NITER)
    return fail(HYDRO_EINVAL, "niter %d: must be in 1..%d", o->niter, HYDRO_MAX_NITER);
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(HYDRO_EINVAL, "tol %g", o->tol);
  if (o->guess != HYDRO_GUESS_PTR && o->guess != HYDRO_GUESS_MLP)
    return fail(HYDRO_EINVAL, "guess %d", o->guess);
  if (o->guess == HYDRO_GUESS_MLP && !p->mlp)
    return fail(HYDRO_ESTATE, "learned guess requested but no network set (hydro_set_mlp)");
  if (o->seg_x < 0 || o->seg_x > 4096) return fail(HYDRO_EINVAL, "seg_x %d", o->seg_x);
  if (o->seg_y < 0 || o->seg_y > (1 << 20)) return fail(HYDRO_EINVAL, "seg_y %d", o->seg_y);
  if (!std::isfinite(o->learned_gate) || o->learned_gate > 50.0)
    return fail(HYDRO_EINVAL, "learned_gate %g: must be finite and <= 50", o->learned_gate);
  if (o->limiter < HYDRO_LIMITER_MINMOD || o->limiter > HYDRO_LIMITER_VANLEER)
    return fail(HYDRO_EINVAL, "limiter %d", o->limiter);
  if (o->order != HYDRO_ORDER_XY && o->order != HYDRO_ORDER_ALTERNATE)
    return fail(HYDRO_EINVAL, "order %d", o->order);
  if (o->riemann < HYDRO_RIEMANN_TWO_SHOCK || o->riemann > HYDRO_RIEMANN_HLLC)
    return fail(HYDRO_EINVAL, "riemann %d", o->riemann);
  if (o->ysweep != HYDRO_YSWEEP_MARCH && o->ysweep != HYDRO_YSWEEP_TILE)
    return fail(HYDRO_EINVAL, "ysweep %d", o->ysweep);
  if (o->riemann == HYDRO_RIEMANN_HLLC && o->guess == HYDRO_GUESS_MLP)
    return fail(HYDRO_EINVAL, "the learned guess needs an iterative solver, not HLLC");
  return HYDRO_OK;
}

// Copies the per-grid states after the stream drains; reports a latched
// non-physical state once and clears it.
int sync_states(hydro::Plan* p, std::vector<hydro::DevState>& s) {
  hipError_t e = p->sync_states(s);
  if (e != hipSuccess) return dev_fail(e, "synchronise");
  int bad = -1;
  for (int g = 0; g < p->n; ++g)
    if (s[g].status != 0) bad = g;
  if (bad < 0) return HYDRO_OK;
  for (int g = 0; g < p->n; ++g) {
    if (s[g].status == 0) continue;
    int zero = 0;
    e = hipMemcpyAsync(&p->st[g].status, &zero, sizeof(int), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return dev_fail(e, "status reset");
  }
  return fail(HYDRO_ENONPHYS, "a sweep produced a non-physical state (grid %d, status 0x%x)", bad,
              s[bad].status);
}

int do_compute_dt(hydro::Plan* p, double* dt) {
  int rc = check_bound(p);
  if (rc) return rc;
  DeviceGuard g(p->device);
  hipError_t e = p->enqueue_max_speed();
  if (e == hipSuccess) e = p->enqueue_finalize(false, false);
  if (e != hipSuccess) return dev_fail(e, "compute_dt");
  std::vector<hydro::DevState> s;
  rc = sync_states(p, s);
  if (rc) {
    p->acc_valid = false;
    return rc;
  }
  p->acc_valid = true;
  if (dt)
    for (int i = 0; i < p->n; ++i) dt[i] = s[i].dt;
  return HYDRO_OK;
}

int do_step(hydro::Plan* p) {
  int rc = check_bound(p);
  if (rc) return rc;
  DeviceGuard g(p->device);
  hipError_t e = p->enqueue_step();
  if (e != hipSuccess) {
    p->acc_valid = false;
    return dev_fail(e, "step");
  }
  return HYDRO_OK;
}

int do_graph_steps(hydro::Plan* p, int nsteps) {
  int rc = check_bound(p);
  if (rc) return rc;
  if (nsteps < 1 || nsteps > 4096) return fail(HYDRO_EINVAL, "nsteps %d: 1..4096", nsteps);
  if (p->stream == nullptr)
    return fail(HYDRO_ESTATE, "graph capture needs a non-default stream (bind)");
  DeviceGuard g(p->device);
  hipError_t e = p->graph_launch(nsteps);
  if (e != hipSuccess) return dev_fail(e, "graph steps");
  return HYDRO_OK;
}

int do_totals(hydro::Plan* p, double* out) {
  int rc = check_bound(p);
  if (rc) return rc;
  if (!out) return fail(HYDRO_EINVAL, "NULL output");
  DeviceGuard g(p->device);
  hipError_t e = p->enqueue_totals();
  if (e != hipSuccess) return dev_fail(e, "totals");
  std::vector<hydro::DevState> s;
  rc = sync_states(p, s);
  if (rc) return rc;
  const int nv = 4 + p->nscalars;
  for (int i = 0; i < p->n; ++i)
    for (int k = 0; k < nv; ++k) out[nv * i + k] = s[i].totals[k];
  return HYDRO_OK;
}

int do_set_scalars(hydro::Plan* p, int n) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  if (n < 0 || n > HYDRO_MAX_SCALARS)
    return fail(HYDRO_EINVAL, "%d passive scalars: must be in 0..%d", n, HYDRO_MAX_SCALARS);
  if (p->bound) return fail(HYDRO_ESTATE, "passive scalars must be set before binding");
  p->nscalars = n;
  return HYDRO_OK;
}

int do_get_clock(hydro::Plan* p, double* t, long* step, double* dt) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  DeviceGuard g(p->device);
  std::vector<hydro::DevState> s;
  hipError_t e = p->sync_states(s);
  if (e != hipSuccess) return dev_fail(e, "get_clock");
  for (int i = 0; i < p->n; ++i) {
    if (t) t[i] = s[i].t;
    if (step) step[i] = (long)s[i].step;
    if (dt) dt[i] = s[i].dt;
  }
  return HYDRO_OK;
}

int do_stats(hydro::Plan* p, hydro_stats_t* out, int reset) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  DeviceGuard g(p->device);
  std::vector<hydro::DevState> s;
  hipError_t e = p->sync_states(s);
  if (e != hipSuccess) return dev_fail(e, "riemann_stats");
  if (out) {
    std::memset(out, 0, sizeof *out);
    for (int i = 0; i < p->n; ++i) {
      out->interfaces += (long long)s[i].interfaces;
      for (int k = 0; k <= HYDRO_MAX_NITER; ++k) {
        out->hist[k] += (long long)s[i].hist[k];
        out->wave_hist[k] += (long long)s[i].wave_hist[k];
      }
      out->fallbacks += (long long)s[i].fallbacks;
    }
  }
  if (reset) {
    e = hydro::launch_clear_stats(p->st, p->n, p->stream);
    if (e != hipSuccess) return dev_fail(e, "stats reset");
  }
  return HYDRO_OK;
}

int do_set_options(hydro::Plan* p, const hydro_options_t* o) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  int rc = check_options(p, o);
  if (rc) return rc;
  DeviceGuard g(p->device);
  hipError_t e = p->set_options(*o);
  if (e != hipSuccess) return dev_fail(e, "set_options");
  return HYDRO_OK;
}

int do_autotune(hydro::Plan* p, hydro_tune_t* out, int use_cache) {
  int rc = check_bound(p);
  if (rc) return rc;
  DeviceGuard g(p->device);
  hipError_t e = p->autotune(out, use_cache != 0);
  if (e != hipSuccess) return dev_fail(e, "autotune");
  return HYDRO_OK;
}

int do_set_profiling(hydro::Plan* p, int enable) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  p->profiling = enable != 0;
  return HYDRO_OK;
}

int do_get_profile(hydro::Plan* p, double ms[HYDRO_NPHASES], long long launches[HYDRO_NPHASES],
                   int reset) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  DeviceGuard g(p->device);
  if (p->bound) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return dev_fail(e, "get_profile");
  }
  double acc[HYDRO_NPHASES] = {0, 0, 0};
  long long cnt[HYDRO_NPHASES] = {0, 0, 0};
  for (const auto& m : p->marks) {
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
    for (const auto& m : p->marks) {
      p->ev_pool.push_back(m.a);
      p->ev_pool.push_back(m.b);
    }
    p->marks.clear();
  }
  return HYDRO_OK;
}

int check_state_ptr(const hydro::Plan* p, void* U, int dtype) {
  if (!U) return fail(HYDRO_EINVAL, "NULL state pointer");
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return fail(HYDRO_EINVAL, "dtype %d", dtype);
  const size_t elem = dtype == HYDRO_F64 ? 8 : 4;
  if (((uintptr_t)U) % elem != 0) return fail(HYDRO_EINVAL, "state pointer misaligned");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, U) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(HYDRO_EINVAL, "state pointer is not device memory");
  }
  if (attr.device != p->device)
    return fail(HYDRO_EINVAL, "state on device %d, handle on device %d", attr.device, p->device);
  return HYDRO_OK;
}

int do_bind(hydro::Plan* p, void* U, const long* pitches, const long long* offsets, int dtype,
            void* stream) {
  DeviceGuard g(p->device);
  hipError_t e = p->bind(U, pitches, offsets, dtype, (hipStream_t)stream);
  if (e == hipErrorOutOfMemory) return fail(HYDRO_ENOMEM, "second state buffer: out of memory");
  if (e != hipSuccess) return dev_fail(e, "bind");
  return HYDRO_OK;
}

int do_set_mlp(hydro::Plan* p, const void* mlp) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  if (mlp) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, mlp) != hipSuccess || attr.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      return fail(HYDRO_EINVAL, "network pointer is not device memory");
    }
  }
  p->mlp = static_cast<const hydro::MlpDev*>(mlp);
  if (!mlp && p->opt.guess == HYDRO_GUESS_MLP) p->opt.guess = HYDRO_GUESS_PTR;
  p->drop_graph();
  return HYDRO_OK;
}

int do_set_logger(hydro::Plan* p, float* buf, long long cap, unsigned long long seed, double rs,
                  double rg) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  if (buf && cap < 1) return fail(HYDRO_EINVAL, "logger capacity %lld", cap);
  if (!(rs >= 0.0 && rs <= 1.0 && rg >= 0.0 && rg <= 1.0))
    return fail(HYDRO_EINVAL, "logger rates %g %g: must be in [0, 1]", rs, rg);
  DeviceGuard g(p->device);
  hipError_t e = p->set_logger(buf, cap, seed, rs, rg);
  if (e != hipSuccess) return dev_fail(e, "set_logger");
  return HYDRO_OK;
}

long long do_logger_count(hydro::Plan* p) {
  if (!p) return fail(HYDRO_EINVAL, "NULL handle");
  DeviceGuard g(p->device);
  unsigned long long c = 0;
  hipError_t e = p->logger_count(&c);
  if (e != hipSuccess) return dev_fail(e, "logger_count");
  return (long long)c;
}

}  // namespace

extern "C" {

const char* hydro_last_error(void) { return g_err; }

// ------------------------------------------------------------ single grid
hydro_t* hydro_create(int nx, int ny, double gamma, double cfl, int bc) {
  return create_plan<hydro_s>(1, &nx, &ny, gamma, cfl, &bc);
}

void hydro_destroy(hydro_t* h) { delete h; }

int hydro_bind(hydro_t* h, void* U, long pitch, int dtype, void* hip_stream) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  int rc = check_state_ptr(h, U, dtype);
  if (rc) return rc;
  if (pitch < h->nx[0]) return fail(HYDRO_EINVAL, "pitch %ld < nx %d", pitch, h->nx[0]);
  if (pitch > (1l << 30)) return fail(HYDRO_EINVAL, "pitch %ld too large", pitch);
  const long long off = 0;
  return do_bind(h, U, &pitch, &off, dtype, hip_stream);
}

int hydro_invalidate(hydro_t* h) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  h->acc_valid = false;
  return HYDRO_OK;
}

int hydro_set_options(hydro_t* h, const hydro_options_t* o) { return do_set_options(h, o); }

int hydro_get_options(const hydro_t* h, hydro_options_t* o) {
  if (!h || !o) return fail(HYDRO_EINVAL, "NULL argument");
  *o = h->opt;
  return HYDRO_OK;
}

double hydro_compute_dt(hydro_t* h) {
  double dt = 0.0;
  int rc = do_compute_dt(h, &dt);
  return rc ? (double)rc : dt;
}

int hydro_sweep(hydro_t* h, int dir) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (dir != HYDRO_DIR_X && dir != HYDRO_DIR_Y) return fail(HYDRO_EINVAL, "dir %d", dir);
  DeviceGuard g(h->device);
  hipError_t e = h->enqueue_single_sweep(dir);
  if (e != hipSuccess) return dev_fail(e, "hydro_sweep");
  return HYDRO_OK;
}

int hydro_step(hydro_t* h) { return do_step(h); }
int hydro_graph_steps(hydro_t* h, int nsteps) { return do_graph_steps(h, nsteps); }
int hydro_conserved_totals(hydro_t* h, double* out) { return do_totals(h, out); }

int hydro_set_scalars(hydro_t* h, int n) { return do_set_scalars(h, n); }

int hydro_get_clock(hydro_t* h, double* t, long* step, double* dt) {
  return do_get_clock(h, t, step, dt);
}

int hydro_set_clock(hydro_t* h, double t, long step) {
  if (!h) return fail(HYDRO_EINVAL, "NULL handle");
  if (!std::isfinite(t) || step < 0) return fail(HYDRO_EINVAL, "clock t=%g step=%ld", t, step);
  DeviceGuard g(h->device);
  hipError_t e = hydro::launch_set_clock(h->st, 0, t, step, h->stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_set_clock");
  h->host_step = step;
  return HYDRO_OK;
}

int hydro_riemann_stats(hydro_t* h, hydro_stats_t* s, int reset) { return do_stats(h, s, reset); }
int hydro_autotune(hydro_t* h, hydro_tune_t* out, int use_cache) {
  return do_autotune(h, out, use_cache);
}
int hydro_set_profiling(hydro_t* h, int enable) { return do_set_profiling(h, enable); }
int hydro_get_profile(hydro_t* h, double ms[HYDRO_NPHASES], long long launches[HYDRO_NPHASES],
                      int reset) {
  return do_get_profile(h, ms, launches, reset);
}

// ------------------------------------------------------------ batches
hydro_batch_t* hydro_batch_create(int n, const int* nx, const int* ny, double gamma, double cfl,
                                  const int* bc) {
  return create_plan<hydro_batch_s>(n, nx, ny, gamma, cfl, bc);
}

void hydro_batch_destroy(hydro_batch_t* b) { delete b; }

long long hydro_batch_layout(const hydro_batch_t* b, int dtype, long long* offsets,
                             long* pitches) {
  if (!b) return fail(HYDRO_EINVAL, "NULL handle");
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return fail(HYDRO_EINVAL, "dtype %d", dtype);
  long long total = 0;
  for (int g = 0; g < b->n; ++g) {
    const long p = hydro::padded_pitch(b->nx[g], dtype);
    if (offsets) offsets[g] = total;
    if (pitches) pitches[g] = p;
    total += (4LL + b->nscalars) * p * b->ny[g];
  }
  return total;
}

int hydro_batch_bind(hydro_batch_t* b, void* U, int dtype, void* hip_stream) {
  if (!b) return fail(HYDRO_EINVAL, "NULL handle");
  int rc = check_state_ptr(b, U, dtype);
  if (rc) return rc;
  std::vector<long long> off(b->n);
  std::vector<long> pitch(b->n);
  hydro_batch_layout(b, dtype, off.data(), pitch.data());
  return do_bind(b, U, pitch.data(), off.data(), dtype, hip_stream);
}

int hydro_batch_set_options(hydro_batch_t* b, const hydro_options_t* o) {
  return do_set_options(b, o);
}

int hydro_batch_set_scalars(hydro_batch_t* b, int n) { return do_set_scalars(b, n); }

int hydro_batch_invalidate(hydro_batch_t* b) {
  if (!b) return fail(HYDRO_EINVAL, "NULL handle");
  b->acc_valid = false;
  return HYDRO_OK;
}

int hydro_batch_compute_dt(hydro_batch_t* b, double* dt) { return do_compute_dt(b, dt); }
int hydro_batch_step(hydro_batch_t* b) { return do_step(b); }
int hydro_batch_graph_steps(hydro_batch_t* b, int nsteps) { return do_graph_steps(b, nsteps); }
int hydro_batch_totals(hydro_batch_t* b, double* out) { return do_totals(b, out); }
int hydro_batch_get_clock(hydro_batch_t* b, double* t, long* step, double* dt) {
  return do_get_clock(b, t, step, dt);
}
int hydro_batch_riemann_stats(hydro_batch_t* b, hydro_stats_t* s, int reset) {
  return do_stats(b, s, reset);
}
int hydro_batch_autotune(hydro_batch_t* b, hydro_tune_t* out, int use_cache) {
  return do_autotune(b, out, use_cache);
}
int hydro_batch_set_profiling(hydro_batch_t* b, int enable) { return do_set_profiling(b, enable); }
int hydro_batch_get_profile(hydro_batch_t* b, double ms[HYDRO_NPHASES],
                            long long launches[HYDRO_NPHASES], int reset) {
  return do_get_profile(b, ms, launches, reset);
}

int hydro_set_mlp(hydro_t* h, const void* mlp) { return do_set_mlp(h, mlp); }
int hydro_batch_set_mlp(hydro_batch_t* b, const void* mlp) { return do_set_mlp(b, mlp); }
int hydro_set_logger(hydro_t* h, float* records, long long capacity, unsigned long long seed,
                     double rate_smooth, double rate_strong) {
  return do_set_logger(h, records, capacity, seed, rate_smooth, rate_strong);
}
int hydro_batch_set_logger(hydro_batch_t* b, float* records, long long capacity,
                           unsigned long long seed, double rate_smooth, double rate_strong) {
  return do_set_logger(b, records, capacity, seed, rate_smooth, rate_strong);
}
long long hydro_logger_count(hydro_t* h) { return do_logger_count(h); }
long long hydro_batch_logger_count(hydro_batch_t* b) { return do_logger_count(b); }

// ------------------------------------------------------------ learned-guess network
size_t hydro_mlp_dev_bytes(void) { return sizeof(hydro::MlpDev); }

size_t hydro_mlp_grad_scratch_bytes(long long n) {
  return sizeof(float) * hydro::mlp_grad_scratch_floats(n < 1 ? 1 : n);
}

int hydro_stream_copy(void* dst, const void* src, long long nbytes, void* hip_stream) {
  if (!dst || !src) return fail(HYDRO_EINVAL, "NULL argument");
  if (nbytes < 0 || nbytes % 16 != 0) return fail(HYDRO_EINVAL, "nbytes %lld", nbytes);
  const uintptr_t d = reinterpret_cast<uintptr_t>(dst), s = reinterpret_cast<uintptr_t>(src);
  if (d % 16 != 0 || s % 16 != 0) return fail(HYDRO_EINVAL, "pointers not 16-byte aligned");
  if (nbytes == 0) return HYDRO_OK;
  if (d < s + (uintptr_t)nbytes && s < d + (uintptr_t)nbytes)
    return fail(HYDRO_EINVAL, "overlapping ranges");
  hipError_t e = hydro::launch_stream_copy(dst, src, nbytes / 16, (hipStream_t)hip_stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_stream_copy");
  return HYDRO_OK;
}

int hydro_mlp_pack(const float* params, void* mlp, void* stream) {
  if (!params || !mlp) return fail(HYDRO_EINVAL, "NULL argument");
  hipError_t e = hydro::launch_mlp_pack(params, static_cast<hydro::MlpDev*>(mlp),
                                        (hipStream_t)stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_mlp_pack");
  return HYDRO_OK;
}

int hydro_mlp_features(const float* records, long long n, double gamma, float* X, float* Y,
                       void* stream) {
  if (!records || !X || n < 0) return fail(HYDRO_EINVAL, "bad arguments");
  if (!(gamma > 1.0)) return fail(HYDRO_EINVAL, "gamma %g", gamma);
  if (n == 0) return HYDRO_OK;
  hipError_t e = hydro::launch_mlp_features(records, n, gamma, X, Y, (hipStream_t)stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_mlp_features");
  return HYDRO_OK;
}

int hydro_mlp_forward(const void* mlp, const float* X, float* Y, long long n, void* stream) {
  if (!mlp || !X || !Y || n < 0) return fail(HYDRO_EINVAL, "bad arguments");
  if (n == 0) return HYDRO_OK;
  hipError_t e = hydro::launch_mlp_forward(static_cast<const hydro::MlpDev*>(mlp), X, Y, n,
                                           (hipStream_t)stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_mlp_forward");
  return HYDRO_OK;
}

int hydro_mlp_grad(const void* mlp, const float* X, const float* T, long long n, float* scratch,
                   float* grad, float* loss, void* stream) {
  if (!mlp || !X || !T || !scratch || !grad || n < 1) return fail(HYDRO_EINVAL, "bad arguments");
  hipError_t e = hydro::launch_mlp_grad(static_cast<const hydro::MlpDev*>(mlp), X, T, n, scratch,
                                        grad, loss, (hipStream_t)stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_mlp_grad");
  return HYDRO_OK;
}

int hydro_mlp_adam(float* params, float* m, float* v, const float* grad, long long step,
                   double lr, double beta1, double beta2, double eps, void* stream) {
  if (!params || !m || !v || !grad || step < 1) return fail(HYDRO_EINVAL, "bad arguments");
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return fail(HYDRO_EINVAL, "Adam hyper-parameters");
  hipError_t e = hydro::launch_mlp_adam(params, m, v, grad, step, lr, beta1, beta2, eps,
                                        (hipStream_t)stream);
  if (e != hipSuccess) return dev_fail(e, "hydro_mlp_adam");
  return HYDRO_OK;
}

}  // extern "C"
