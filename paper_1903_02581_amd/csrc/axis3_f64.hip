// Instantiations of the three-stage per-axis pass for double2 storage.
#include "axis3_pass.hpp"

namespace hom4d_impl {
dev::AxisKernel pick_axis3_f64(int axis, int n, int vk, int nst, bool nt, bool pers, int w, int* t) {
    return dev::pick_axis3<double2>(axis, n, vk, nst, nt, pers, w, t);
}
}  // namespace hom4d_impl
