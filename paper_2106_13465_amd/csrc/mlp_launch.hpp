// mlp_launch.hpp -- host-side launchers of the learned-guess network kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace hydro {

struct MlpDev;

int mlp_grad_blocks(long long n);
size_t mlp_grad_scratch_floats(long long n);

hipError_t launch_mlp_pack(const float* params, MlpDev* m, hipStream_t s);
hipError_t launch_mlp_features(const float* rec, long long n, double gamma, float* X, float* Y,
                               hipStream_t s);
hipError_t launch_mlp_forward(const MlpDev* m, const float* X, float* Y, long long n,
                              hipStream_t s);
hipError_t launch_mlp_grad(const MlpDev* m, const float* X, const float* T, long long n,
                           float* scratch, float* grad, float* loss, hipStream_t s);
hipError_t launch_mlp_adam(float* p, float* m, float* v, const float* grad, long long step,
                           double lr, double b1, double b2, double eps, hipStream_t s);

}  // namespace hydro
