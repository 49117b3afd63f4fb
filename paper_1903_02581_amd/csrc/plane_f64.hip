// Instantiations of the fused (x2, y2)-plane pass for double2 storage.
#include "plane_pass.hpp"

namespace hom4d_impl {
namespace {
using dev::AxisKernel;
using dev::k_plane2;
using dev::plane_threads;
using dev::Shape;

template <int NX, int NY>
AxisKernel mk(int* nt, int vk) {
    constexpr int T = plane_threads(NX, NY, Shape<NX>::t, Shape<NY>::t);
    *nt = T;
    return vk == 2 ? k_plane2<double2, NX, NY, T, 2> : k_plane2<double2, NX, NY, T, 1>;
}
}  // namespace

// Plane sizes with a fused kernel: the FP64 LDS image (nx rows of ny + ny/8
// slots) must fit in 160 KB with room for a second workgroup.
AxisKernel pick_plane_f64(int nx, int ny, int vk, int* nt) {
#define HOM4D_PLANE(X, Y) \
    if (nx == X && ny == Y) return mk<X, Y>(nt, vk);
    HOM4D_PLANE(16, 16)
    HOM4D_PLANE(24, 24)
    HOM4D_PLANE(32, 32)
    HOM4D_PLANE(48, 48)
    HOM4D_PLANE(64, 64)
    HOM4D_PLANE(48, 16)
    HOM4D_PLANE(16, 48)
#undef HOM4D_PLANE
    *nt = 0;
    return nullptr;
}
}  // namespace hom4d_impl
