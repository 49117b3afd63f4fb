// Instantiations of the per-axis pass for double2 storage, 1 state(s) per pass.
#include "axis_pass.hpp"

namespace hom4d_impl {
dev::AxisKernel pick_axis_f64_1(int axis, int n, int vk, bool nt, int* t) {
    return dev::pick_axis<double2, 1>(axis, n, vk, nt, t);
}
}  // namespace hom4d_impl
