// noalloc.hip -- hydro_step_noalloc: one time step of up to
// HYDRO_NOALLOC_MAX_GRIDS grids held in caller buffers, without a handle and
// without any device allocation.
//
// The kernels of hydro_step keep per-grid device scratch: the grid
// descriptors (geometry, work-item prefixes) and the device state (dt slot,
// max-speed accumulator, status word, statistics).  Here that scratch is a
// file-scope device array of fixed size.  Each GPU holds its own copy, at its
// own address, from the first call on that GPU until the process ends; the
// host never passes the array's name to a kernel (on the host it is only a
// stand-in), it passes the device address resolved once per device with
// hipGetSymbolAddress.
//
// Every call on one GPU shares that GPU's copy and overwrites it: calls that
// overlap on one GPU (other streams, other host threads) race.  Each call
// rewrites the descriptors and clears the state with a kernel (no memset, so
// a caller may capture the call into a HIP graph).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "device_state.hpp"
#include "hydro.h"
#include "launch.hpp"
#include "plan.hpp"

namespace hydro {
namespace {

constexpr int kMaxGrids = HYDRO_NOALLOC_MAX_GRIDS;
static_assert(sizeof(DevState) % 8 == 0, "DevState is cleared as 64-bit words");

struct NoallocScratch {
  GridDesc desc[kMaxGrids];
  DevState st[kMaxGrids];
};
static_assert(sizeof(NoallocScratch) <= 16384, "the static scratch stays small");

// The scratch array: one copy per GPU.  Only its device address (per device,
// from hipGetSymbolAddress) is ever handed to a kernel.
static __device__ __align__(256) unsigned char scratch[sizeof(NoallocScratch)];

// Kernel argument carrying the descriptors (no host-to-device copy).
struct DescArg {
  GridDesc d[kMaxGrids];
  int n;
};

__global__ void k_noalloc_setup(DescArg a, GridDesc* g, DevState* st) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(st);
  const int words = a.n * (int)(sizeof(DevState) / 8);
  for (int k = threadIdx.x; k < words; k += blockDim.x) w[k] = 0ull;
  for (int k = threadIdx.x; k < a.n; k += blockDim.x) g[k] = a.d[k];
}

// dt_out[g] = the time step grid g advanced by, NaN if one of its sweeps
// produced a non-physical state.
__global__ void k_noalloc_report(const DevState* st, int n, double* dt_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dt_out[i] = st[i].status ? (double)NAN : st[i].dt;
}

// Device address of this device's copy of `scratch`, resolved once per device
// (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

hipError_t scratch_address(int dev, NoallocScratch** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[dev] = p;
  }
  *out = static_cast<NoallocScratch*>(g_addr[dev]);
  return hipSuccess;
}

template <typename T>
Batch<T> batch(const void* src, void* dst, NoallocScratch* s, int n, int seg, long long items) {
  Batch<T> b;
  b.src = static_cast<const T*>(src);
  b.dst = static_cast<T*>(dst);
  b.g = s->desc;
  b.st = s->st;
  b.ngrids = n;
  b.seg = seg;
  b.nv = 4;
  b.items = items;
  return b;
}

template <typename T>
hipError_t enqueue(const DescArg& a, NoallocScratch* s, const void* U, void* Uh, void* Uo,
                   double* dt_out, double gamma, long long items_x, long long items_y,
                   long long rows, int seg_x, int seg_y, hipStream_t stream) {
  const Gas<T> G = make_gas<T>(gamma, default_options());
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, stream, a, s->desc, s->st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // dt from the max wave speed of U, as the first step of a handle
  e = launch_max_speed<T>(batch<T>(U, nullptr, s, a.n, 0, rows), G, stream);
  if (e != hipSuccess) return e;
  e = launch_finalize_dt(s->desc, s->st, a.n, false, true, stream);
  if (e != hipSuccess) return e;
  Extras ex;
  std::memset(&ex, 0, sizeof ex);
  ex.gamma = (float)gamma;
  e = launch_sweep_x<T>(batch<T>(U, Uh, s, a.n, seg_x, items_x), G, ex, false, 0, 0, stream);
  if (e != hipSuccess) return e;
  e = launch_sweep_y<T>(batch<T>(Uh, Uo, s, a.n, seg_y, items_y), G, ex, false, 0, 0, stream);
  if (e != hipSuccess) return e;
  if (dt_out) {
    hipLaunchKernelGGL(k_noalloc_report, dim3(1), dim3(64), 0, stream, (const DevState*)s->st,
                       a.n, dt_out);
    e = hipGetLastError();
  }
  return e;
}

bool overlaps(const void* a, const void* b, size_t bytes) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bytes && pb < pa + bytes;
}

}  // namespace
}  // namespace hydro

extern "C" int hydro_step_noalloc(int n, const int* nx, const int* ny, const int* bc,
                                  const long long* offsets, const long* pitches, int dtype,
                                  double gamma, double cfl, const void* U, void* U_half,
                                  void* U_out, double* dt_out, void* hip_stream) {
  using namespace hydro;
  if (n < 1 || n > kMaxGrids)
    return fail(HYDRO_EINVAL,
                "n = %d grids: hydro_step_noalloc takes 1..%d (its static device scratch holds "
                "%d grids)",
                n, kMaxGrids, kMaxGrids);
  if (!nx || !ny || !bc || !offsets || !pitches || !U || !U_half || !U_out)
    return fail(HYDRO_EINVAL, "NULL size array or state pointer");
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return fail(HYDRO_EINVAL, "dtype %d", dtype);
  if (!(gamma > 1.0) || !std::isfinite(gamma))
    return fail(HYDRO_EINVAL, "gamma = %g: must be > 1", gamma);
  if (!(cfl > 0.0 && cfl <= 1.0)) return fail(HYDRO_EINVAL, "cfl = %g: must be in (0, 1]", cfl);
  LaunchCfg cfg;  // the default launch shape of a handle
  DescArg a;
  std::memset(&a, 0, sizeof a);
  a.n = n;
  long long items_x = 0, items_y = 0, rows = 0, elems = 0;
  for (int g = 0; g < n; ++g) {
    if (nx[g] < 2 || ny[g] < 2 || nx[g] > (1 << 28) || ny[g] > (1 << 28) ||
        (long long)nx[g] * ny[g] >= (1ll << 38))
      return fail(HYDRO_EINVAL, "grid %d: %d x %d (sides 2 .. 2^28, < 2^38 cells)", g, nx[g],
                  ny[g]);
    if (bc[g] != HYDRO_BC_REFLECT && bc[g] != HYDRO_BC_OUTFLOW && bc[g] != HYDRO_BC_PERIODIC)
      return fail(HYDRO_EINVAL, "grid %d: bc = %d is not a HYDRO_BC_* value", g, bc[g]);
    if (pitches[g] < nx[g] || pitches[g] > (1l << 30) || offsets[g] < 0)
      return fail(HYDRO_EINVAL, "grid %d: pitch %ld (>= nx = %d) or offset %lld (>= 0)", g,
                  pitches[g], nx[g], offsets[g]);
    GridDesc& d = a.d[g];
    d.off = offsets[g];
    d.pitch = (int)pitches[g];
    d.nx = nx[g];
    d.ny = ny[g];
    d.bc = bc[g];
    d.plane = (long long)d.pitch * ny[g];
    d.h = 1.0 / (double)(nx[g] > ny[g] ? nx[g] : ny[g]);
    d.cfl = cfl;
    d.r0 = rows;
    rows += ny[g];
    const int nseg = (nx[g] + kXOut - 1) / kXOut;
    d.wx0 = items_x;
    items_x += (long long)((nseg + cfg.seg_x - 1) / cfg.seg_x) * ny[g];
    d.wy0 = items_y;
    items_y += (long long)((nx[g] + kWave - 1) / kWave) * ((ny[g] + cfg.seg_y - 1) / cfg.seg_y);
    const long long end = d.off + 4 * d.plane;
    if (end > elems) elems = end;
  }
  // U_half must not overlap the input or the output; U_out is U or disjoint
  const size_t bytes = (size_t)elems * (dtype == HYDRO_F64 ? 8 : 4);
  if (overlaps(U_half, U, bytes) || overlaps(U_half, U_out, bytes))
    return fail(HYDRO_EINVAL, "U_half overlaps U or U_out");
  if (U_out != U && overlaps(U_out, U, bytes))
    return fail(HYDRO_EINVAL, "U_out must be U itself or not overlap it");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HYDRO_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(HYDRO_EDEVICE, "device %d out of range", dev);
  NoallocScratch* s = nullptr;
  e = scratch_address(dev, &s);
  if (e != hipSuccess)
    return fail(HYDRO_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  e = dtype == HYDRO_F64
          ? enqueue<double>(a, s, U, U_half, U_out, dt_out, gamma, items_x, items_y, rows,
                            cfg.seg_x, cfg.seg_y, stream)
          : enqueue<float>(a, s, U, U_half, U_out, dt_out, gamma, items_x, items_y, rows,
                           cfg.seg_x, cfg.seg_y, stream);
  if (e != hipSuccess) return fail(HYDRO_EDEVICE, "hydro_step_noalloc: %s", hipGetErrorString(e));
  return HYDRO_OK;
}
