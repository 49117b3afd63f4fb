// Launchers of the pass kernels and the elementwise / reduction kernels of the
// two-electron split-step propagator (gfx950, wave64).
//
// The pass kernels (axis_pass.hpp, axis3_pass.hpp, plane_pass.hpp) apply one
// batched transform round trip along a coordinate of Psi[x1][y1][x2][y2] with
// the diagonal kinetic phase of that coordinate in reciprocal space (Appendix A
// of arXiv 1903.02581: T_x diagonal in (k_x, y), T_y diagonal in k_y), and on
// the passes that carry it the real-space potential factor
// exp(-i tau (V1 + V2 + V12) / hbar) (Sec. II.C Eq. (evoloperat); Sec. III.B
// Eq. (coulomb)).  A thread loads its elements of a line straight from HBM
// (for strided axes consecutive lanes read consecutive lines, so every row
// access of a wavefront is one contiguous run), runs register DFTs, exchanges
// through LDS between radix stages, applies the phase at known wave numbers and
// runs the transposed network back to its own elements, which it stores in
// place.  All arithmetic is FP64; the state is stored as complex128 or complex64.
//
// This file also holds the launch logic (kernel choice per line length,
// storage type, state count and potential-factor form) and the FP64
// reductions, whose partial sums are combined in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_set>

#include "axis_pass.hpp"
#include "hom4d_internal.hpp"

using namespace hom4d_dev;

namespace hom4d_impl {

using dev::AxisKernel;
AxisKernel pick_axis_f64_1(int axis, int n, int vk, bool nt, int* t);
AxisKernel pick_axis_f64_2(int axis, int n, int vk, bool nt, int* t);
AxisKernel pick_axis_f32_1(int axis, int n, int vk, bool nt, int* t);
AxisKernel pick_axis_f32_2(int axis, int n, int vk, bool nt, int* t);
AxisKernel pick_axis3_f64(int axis, int n, int vk, int nst, bool nt, bool pers, int w, int* t);
AxisKernel pick_axis3_f32(int axis, int n, int vk, int nst, bool nt, bool pers, int w, int* t);
AxisKernel pick_plane_f64(int nx, int ny, int vk, int* nt);
AxisKernel pick_plane_f32(int nx, int ny, int vk, int* nt);

namespace {

using namespace dev;

// --------------------------------------------------------------------------------------
// Elementwise / reduction kernels.  Rows r1 are spread over blocks, r2 over threads, so
// the summation order depends only on the launch shape: results are bitwise repeatable.

__global__ void k_init_norm(const double2* pa, const double2* pb, int sym, int nxy, double* part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int r1 = blockIdx.x; r1 < nxy; r1 += gridDim.x) {
        const double2 a1 = pa[r1], b1 = pb[r1];
        for (int r2 = threadIdx.x; r2 < nxy; r2 += blockDim.x) {
            double2 p = cmul(a1, pb[r2]);
            if (sym != 0) {
                const double2 q = cmul(b1, pa[r2]);
                p = make_double2(p.x + sym * q.x, p.y + sym * q.y);
            }
            acc += p.x * p.x + p.y * p.y;
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <class S>
__global__ void k_init_write(S* psi, const double2* pa, const double2* pb, int sym, int nxy, double scale) {
    for (int r1 = blockIdx.x; r1 < nxy; r1 += gridDim.x) {
        const double2 a1 = pa[r1], b1 = pb[r1];
        for (int r2 = threadIdx.x; r2 < nxy; r2 += blockDim.x) {
            double2 p = cmul(a1, pb[r2]);
            if (sym != 0) {
                const double2 q = cmul(b1, pa[r2]);
                p = make_double2(p.x + sym * q.x, p.y + sym * q.y);
            }
            st<S>(psi + (int64_t)r1 * nxy + r2, cscale(p, scale));
        }
    }
}

template <class S>
__global__ void k_obs(const S* psi, const double* w, int nxy, double* part) {
    __shared__ double red[256];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r1 = blockIdx.x; r1 < nxy; r1 += gridDim.x) {
        const double w1 = w[r1];
        const S* row = psi + (int64_t)r1 * nxy;
        for (int r2 = threadIdx.x; r2 < nxy; r2 += blockDim.x) {
            const double2 p = ld<S>(row + r2);
            const double d = p.x * p.x + p.y * p.y;
            const double w2 = w[r2];
            acc[0] += d;
            acc[1] += w1 * w2 * d;
            acc[2] += w1 * (1.0 - w2) * d;
            acc[3] += (1.0 - w1) * w2 * d;
            acc[4] += (1.0 - w1) * (1.0 - w2) * d;
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double s = block_sum(acc[q], red);
        if (threadIdx.x == 0) part[blockIdx.x * 5 + q] = s;
    }
}

struct LossCoeffs {
    double c[4];
};

template <class S>
__global__ void k_loss_lambda(const S* psi, S* lam, const double* w, LossCoeffs cf, int nxy, double* part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int r1 = blockIdx.x; r1 < nxy; r1 += gridDim.x) {
        const double w1 = w[r1];
        const int64_t o = (int64_t)r1 * nxy;
        for (int r2 = threadIdx.x; r2 < nxy; r2 += blockDim.x) {
            const double2 p = ld<S>(psi + o + r2);
            const double w2 = w[r2];
            const double wl = cf.c[0] * w1 * w2 + cf.c[1] * w1 * (1.0 - w2) + cf.c[2] * (1.0 - w1) * w2 +
                              cf.c[3] * (1.0 - w1) * (1.0 - w2);
            acc += wl * (p.x * p.x + p.y * p.y);
            st<S>(lam + o + r2, cscale(p, wl));
        }
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[q] = sum_b part[b * width + q], fixed order; one block per q.
__global__ void k_reduce_parts(const double* part, int nparts, int width, double* out) {
    __shared__ double red[256];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) acc += part[(int64_t)b * width + q];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[q] = s;
}

template <class S>
__global__ void k_gather(const S* psi, const int32_t* ix1, int n1, int jy1, const int32_t* ix2, int n2, int jy2,
                         int nx, int ny, double2* out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n1 * n2) return;
    const int a = idx / n2, b = idx % n2;
    const int64_t nxy = (int64_t)nx * ny;
    const int64_t off = ((int64_t)ix1[a] * ny + jy1) * nxy + (int64_t)ix2[b] * ny + jy2;
    out[idx] = ld<S>(psi + off);
}

// out[r1] = sum_r2 |psi(r1, r2)|^2: one block per r1 over its contiguous plane.
template <class S>
__global__ void k_marginal(const S* psi, int nxy, double* out) {
    __shared__ double red[256];
    const int r1 = blockIdx.x;
    const S* row = psi + (int64_t)r1 * nxy;
    double acc = 0.0;
    for (int r2 = threadIdx.x; r2 < nxy; r2 += blockDim.x) {
        const double2 p = ld<S>(row + r2);
        acc += p.x * p.x + p.y * p.y;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[r1] = s;
}

// out[r1] = |psi(r1, r2)|^2 for one fixed r2.
template <class S>
__global__ void k_conditional(const S* psi, int nxy, int r2, double* out) {
    const int r1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (r1 >= nxy) return;
    const double2 p = ld<S>(psi + (int64_t)r1 * nxy + r2);
    out[r1] = p.x * p.x + p.y * p.y;
}

__global__ void k_c128_to_c64(const double2* in, float2* out, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

__global__ void k_c64_to_c128(const float2* in, double2* out, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = make_double2((double)in[i].x, (double)in[i].y);
}

__global__ void k_zero(double* p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_grad_finish(const double* m_x2, int bpr_x2, const double* m_y2, int bpr_y2, const double* m_y1,
                              const double* m_x1, int nx, int ny, double gscale, double* dldv) {
    const int nxy = nx * ny;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nxy) return;
    double g1 = 0.0, g2 = 0.0;
    for (int q = 0; q < bpr_x2; ++q) g1 += m_x2[(int64_t)r * bpr_x2 + q];
    for (int q = 0; q < bpr_y2; ++q) g1 += m_y2[(int64_t)r * bpr_y2 + q];
    for (int i = 0; i < nx; ++i) g2 += m_y1[(int64_t)i * nxy + r];
    for (int j = 0; j < ny; ++j) g2 += m_x1[(int64_t)j * nxy + r];
    dldv[r] = gscale * (g1 + g2);
}

inline int obs_threads() { return 256; }

}  // namespace

int axis3_threads(int n, int nst) {
    if (nst != 1 && nst != 2) return 0;
    switch (n) {
        case 96: return 8;
        case 128: return 16;
        case 256: return 32;
        default: return 0;
    }
}

bool fft_shape(int n, FftShape* out) {
    switch (n) {
        case 4: *out = {4, 1, 1}; return true;
        case 6: *out = {6, 1, 1}; return true;
        case 8: *out = {8, 1, 1}; return true;
        case 12: *out = {12, 1, 1}; return true;
        case 16: *out = {4, 4, 4}; return true;
        case 24: *out = {12, 2, 2}; return true;
        case 32: *out = {8, 4, 4}; return true;
        case 48: *out = {12, 4, 4}; return true;
        case 64: *out = {8, 8, 8}; return true;
        case 96: *out = {12, 8, 4}; return true;
        case 128: *out = {16, 8, 8}; return true;
        case 256: *out = {16, 16, 16}; return true;
        default: return false;
    }
}

// Blocks of fn (threads, dynamic LDS) resident on the whole device at once:
// blocks per CU times the CU count, cached per kernel and shape.
hipError_t resident_blocks(AxisKernel fn, int threads, size_t lds_bytes, int* out) {
    static std::mutex mu;
    static std::map<std::tuple<const void*, int, size_t>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(reinterpret_cast<const void*>(fn), threads, lds_bytes);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return hipSuccess;
    }
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), threads,
                                                         lds_bytes);
    if (e != hipSuccess) return e;
    *out = per_cu * cus;
    cache[key] = *out;
    return hipSuccess;
}

hipError_t launch_axis(int axis, int n, bool mixed, int nst, bool pers, const PassArgs& a, int64_t nlines,
                       size_t lds_bytes, hipStream_t s) {
    int t = 0;
    AxisKernel fn = nullptr;
    const int vk = a.vmode == 0 ? 0 : (a.vdirect ? 2 : 1);
    const bool nt = a.nt != 0;
    if (axis3_threads(n, nst) > 0)
        fn = mixed ? pick_axis3_f32(axis, n, vk, nst, nt, pers, a.W, &t)
                   : pick_axis3_f64(axis, n, vk, nst, nt, pers, a.W, &t);
    else if (pers)
        return hipErrorInvalidValue;  // only the three-stage passes have a persistent form
    else if (!mixed)
        fn = (nst == 2) ? pick_axis_f64_2(axis, n, vk, nt, &t) : pick_axis_f64_1(axis, n, vk, nt, &t);
    else
        fn = (nst == 2) ? pick_axis_f32_2(axis, n, vk, nt, &t) : pick_axis_f32_1(axis, n, vk, nt, &t);
    if (!fn || a.W <= 0 || nlines % a.W != 0) return hipErrorInvalidValue;
    const int64_t nblocks = nlines / a.W;
    const int max_threads = axis3_threads(n, nst) > 0 ? axis3_block_threads(axis, n, nst, mixed) : 256;
    if (nblocks > 0x7fffffff || t * a.W > max_threads || lds_bytes > 160 * 1024) return hipErrorInvalidValue;
    if (axis3_threads(n, nst) > 0) {
        if (lds_bytes < axis3_pass_lds_bytes(axis, n, a.W, nst, mixed, pers)) return hipErrorInvalidValue;
    } else {
        FftShape sh;
        if (!fft_shape(n, &sh)) return hipErrorInvalidValue;
        const size_t need = axis_xchg_bytes(sh.n2 > 1 ? n : 0, a.W, nst, axis_xchg_c64(axis, mixed)) + 3u * (size_t)n * 16u;
        if (lds_bytes < need) return hipErrorInvalidValue;
    }
    if (lds_bytes > 64 * 1024) {
        // dynamic LDS above 64 KB has to be enabled per kernel, once
        static std::mutex mu;
        static std::unordered_set<const void*> raised;
        std::lock_guard<std::mutex> lock(mu);
        const void* key = reinterpret_cast<const void*>(fn);
        if (!raised.count(key)) {
            hipError_t e = hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            raised.insert(key);
        }
    }
    int64_t grid = nblocks;
    if (pers) {
        // persistent pass: the blocks that fit the device at once walk the
        // a.ntiles tiles
        if (a.ntiles != (uint32_t)nblocks) return hipErrorInvalidValue;
        int resident = 0;
        hipError_t e = resident_blocks(fn, t * a.W, lds_bytes, &resident);
        if (e != hipSuccess) return e;
        if (resident > 0) grid = std::min<int64_t>(nblocks, resident);
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(t * a.W), lds_bytes, s, a);
    return hipGetLastError();
}

bool plane_available(int nx, int ny, bool mixed) {
    int nt = 0;
    return (mixed ? pick_plane_f32(nx, ny, 1, &nt) : pick_plane_f64(nx, ny, 1, &nt)) != nullptr;
}

hipError_t launch_plane(int nx, int ny, bool mixed, const PassArgs& a, hipStream_t s) {
    int nt = 0;
    const int vk = a.vdirect ? 2 : 1;
    AxisKernel fn = mixed ? pick_plane_f32(nx, ny, vk, &nt) : pick_plane_f64(nx, ny, vk, &nt);
    if (!fn || nt <= 0 || nt > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)(nx * ny)), dim3(nt), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init_norm(const double2* pa, const double2* pb, int sym, int nxy, double* part, int nblocks,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_init_norm, dim3(nblocks), dim3(obs_threads()), 0, s, pa, pb, sym, nxy, part);
    return hipGetLastError();
}

hipError_t launch_init_write(void* psi, bool mixed, const double2* pa, const double2* pb, int sym, int nxy,
                             double scale, hipStream_t s) {
    const int nb = nxy < 2048 ? nxy : 2048;
    if (mixed)
        hipLaunchKernelGGL(k_init_write<float2>, dim3(nb), dim3(256), 0, s, (float2*)psi, pa, pb, sym, nxy, scale);
    else
        hipLaunchKernelGGL(k_init_write<double2>, dim3(nb), dim3(256), 0, s, (double2*)psi, pa, pb, sym, nxy, scale);
    return hipGetLastError();
}

hipError_t launch_obs(const void* psi, bool mixed, const double* w, int nxy, double* part, int nblocks,
                      hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL(k_obs<float2>, dim3(nblocks), dim3(obs_threads()), 0, s, (const float2*)psi, w, nxy, part);
    else
        hipLaunchKernelGGL(k_obs<double2>, dim3(nblocks), dim3(obs_threads()), 0, s, (const double2*)psi, w, nxy,
                           part);
    return hipGetLastError();
}

hipError_t launch_loss_lambda(const void* psi, void* lam, bool mixed, const double* w, const double* coeffs, int nxy,
                              double* part, int nblocks, hipStream_t s) {
    LossCoeffs cf{{coeffs[0], coeffs[1], coeffs[2], coeffs[3]}};
    if (mixed)
        hipLaunchKernelGGL(k_loss_lambda<float2>, dim3(nblocks), dim3(obs_threads()), 0, s, (const float2*)psi,
                           (float2*)lam, w, cf, nxy, part);
    else
        hipLaunchKernelGGL(k_loss_lambda<double2>, dim3(nblocks), dim3(obs_threads()), 0, s, (const double2*)psi,
                           (double2*)lam, w, cf, nxy, part);
    return hipGetLastError();
}

hipError_t launch_reduce_parts(const double* part, int nparts, int width, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_parts, dim3(width), dim3(256), 0, s, part, nparts, width, out);
    return hipGetLastError();
}

hipError_t launch_gather(const void* psi, bool mixed, const int32_t* ix1, int n1, int jy1, const int32_t* ix2, int n2,
                         int jy2, int nx, int ny, double2* out, hipStream_t s) {
    const int tot = n1 * n2;
    const int nb = (tot + 255) / 256;
    if (mixed)
        hipLaunchKernelGGL(k_gather<float2>, dim3(nb), dim3(256), 0, s, (const float2*)psi, ix1, n1, jy1, ix2, n2,
                           jy2, nx, ny, out);
    else
        hipLaunchKernelGGL(k_gather<double2>, dim3(nb), dim3(256), 0, s, (const double2*)psi, ix1, n1, jy1, ix2, n2,
                           jy2, nx, ny, out);
    return hipGetLastError();
}

hipError_t launch_marginal(const void* psi, bool mixed, int nxy, double* out, hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL(k_marginal<float2>, dim3(nxy), dim3(256), 0, s, (const float2*)psi, nxy, out);
    else
        hipLaunchKernelGGL(k_marginal<double2>, dim3(nxy), dim3(256), 0, s, (const double2*)psi, nxy, out);
    return hipGetLastError();
}

hipError_t launch_conditional(const void* psi, bool mixed, int nxy, int r2, double* out, hipStream_t s) {
    const int nb = (nxy + 255) / 256;
    if (mixed)
        hipLaunchKernelGGL(k_conditional<float2>, dim3(nb), dim3(256), 0, s, (const float2*)psi, nxy, r2, out);
    else
        hipLaunchKernelGGL(k_conditional<double2>, dim3(nb), dim3(256), 0, s, (const double2*)psi, nxy, r2, out);
    return hipGetLastError();
}

hipError_t launch_c128_to_c64(const double2* in, float2* out, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_c128_to_c64, dim3(1024), dim3(256), 0, s, in, out, count);
    return hipGetLastError();
}

hipError_t launch_c64_to_c128(const float2* in, double2* out, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_c64_to_c128, dim3(1024), dim3(256), 0, s, in, out, count);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

// Gradient partials of the reverse sweep for callers that cannot allocate
// (hom4d_grad_backward_noalloc): a fixed array in device memory, one copy per
// GPU that loads the library.  Host code never names it: each device's address
// is taken once, with that device current, and kept in scratch_ptrs.
namespace {
static __device__ __align__(256) double scratch[kScratchDoubles];
std::mutex scratch_mu;
double* scratch_ptrs[kMaxDevices] = {};
}  // namespace

hipError_t init_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptrs[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptrs[device] = static_cast<double*>(ptr);
    return hipSuccess;
}

double* scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    return scratch_ptrs[device];
}

hipError_t launch_grad_finish(const double* m_x2, int bpr_x2, const double* m_y2, int bpr_y2, const double* m_y1,
                              const double* m_x1, int nx, int ny, double gscale, double* dldv, hipStream_t s) {
    const int nxy = nx * ny;
    hipLaunchKernelGGL(k_grad_finish, dim3((nxy + 255) / 256), dim3(256), 0, s, m_x2, bpr_x2, m_y2, bpr_y2, m_y1,
                       m_x1, nx, ny, gscale, dldv);
    return hipGetLastError();
}

}  // namespace hom4d_impl
