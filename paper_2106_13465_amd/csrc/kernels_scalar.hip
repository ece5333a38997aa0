// kernels_scalar.hip -- the sweep kernel variants that carry one passive
// scalar (instantiated here so they compile in parallel with kernels.hip).
#include "sweeps.hpp"

namespace hydro {

template SweepFn<double> sweep_table_ns<double, 0, 1>(int);
template SweepFn<double> sweep_table_ns<double, 1, 1>(int);
template SweepFn<float> sweep_table_ns<float, 0, 1>(int);
template SweepFn<float> sweep_table_ns<float, 1, 1>(int);
template SweepFn<double> sweep_table_ns<double, 2, 1>(int);
template SweepFn<float> sweep_table_ns<float, 2, 1>(int);

}  // namespace hydro
