// Instantiations of the fused (x2, y2)-plane pass for float2 storage.
#include <cstdlib>

#include "plane_pass.hpp"

namespace hom4d_impl {
namespace {
using dev::AxisKernel;
using dev::k_plane2;
using dev::plane_threads;
using dev::Shape;

bool plane_small_blocks() {
    const char* e = std::getenv("HOM4D_PLANE_NT");
    return e && e[0] == '2';
}

template <int NX, int NY>
AxisKernel mk(int* nt, bool persist, int vk) {
    constexpr int T = plane_threads(NX, NY, Shape<NX>::t, Shape<NY>::t);
    *nt = T;
    if (vk == 2) return persist ? k_plane2<float2, NX, NY, T, true, 2> : k_plane2<float2, NX, NY, T, false, 2>;
    return persist ? k_plane2<float2, NX, NY, T, true, 1> : k_plane2<float2, NX, NY, T, false, 1>;
}
}  // namespace

AxisKernel pick_plane_f32(int nx, int ny, bool persist, int vk, int* nt) {
    if (nx == 64 && ny == 64 && !persist && plane_small_blocks()) {
        *nt = 256;
        return vk == 2 ? k_plane2<float2, 64, 64, 256, false, 2> : k_plane2<float2, 64, 64, 256, false, 1>;
    }
#define HOM4D_PLANE(X, Y) \
    if (nx == X && ny == Y) return mk<X, Y>(nt, persist, vk);
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
