// Internal interface between the host driver (hom4d_host.cpp) and the device
// kernels (hom4d_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hom4d_impl {

enum Axis : int { AX_X1 = 0, AX_Y1 = 1, AX_X2 = 2, AX_Y2 = 3 };

enum GradFlags : int {
    G_GB = 1,    // accumulate dL/dB contributions in (k_x, y) space (x axes)
    G_MIN = 2,   // accumulate Im(conj(lambda) psi) marginals of the loaded real-space states
    G_MOUT = 4,  // ... of the real-space states written back
};

// Division by a grid extent d = 2^a 3^c (c <= 2; every supported nx, ny and
// nx ny has this form) without an integer divide: x / d = mulhi(x >> s1, m) >> s2,
// where m = ceil(2^33 / 3^c) for c > 0 (0xAAAAAAAB for 3, 0x38E38E39 for 9:
// m 3^c - 2^33 = 1, exact for every 32-bit dividend) with s2 = 1, and for c = 0
// m = 2^31, s1 = a - 1, s2 = 0 (a plain shift by a, a >= 1).
struct Div3 {
    uint32_t s1, m, s2, d;
    __device__ __forceinline__ uint32_t div(uint32_t x) const { return __umulhi(x >> s1, m) >> s2; }
    __device__ __forceinline__ uint32_t mod(uint32_t x, uint32_t q) const { return x - q * d; }
};

// Everything one per-axis pass needs.  Axis lines have length n = nx (x axes)
// or ny (y axes); the 4D state is row-major [x1][y1][x2][y2].
struct PassArgs {
    void* psi;                // state, complex128 or complex64
    void* lam;                // adjoint state (dual-state passes only)
    int nx, ny;
    Div3 dnx, dny, dnxy;      // division by nx, ny and nx ny (line numbers -> coordinates)
    int W;                    // lines per block
    uint32_t ntiles;          // tiles of W lines (nlines / W); a persistent pass's grid may be smaller
    const double2* tw;        // twiddles exp(-2 pi i j / n), j < n
    const double2* ktab;      // k-space factor incl. 1/n: x1 pass [ny][nx], x2 and plane passes [nx][ny], y [ny]
    const double2* tw2;       // plane pass only: twiddles of the y lines
    const double2* ktab2;     // plane pass only: y kinetic factor [ny]
    int vmode;                // 0: none, 1: potential factor before the transform, 2: after
    int nt;                   // line passes: non-temporal state loads and stores (large states)
    // potential factor, table form
    const double2* a1;        // [nx*ny]  exp(-i tau V(x,y)/hbar)
    const double2* ac;        // [(2nx-1)*(2ny-1)] exp(-i tau V12(dx,dy)/hbar), or null
    // potential factor, per-point form (vdirect = 1)
    int vdirect;
    const double* vtab;       // [nx*ny] V in meV
    double vscale;            // tau / hbar (1/meV), signed
    double dx, dy, soft2, ck, inv_screen;
    // gradient accumulation (dual-state passes)
    int gflags;
    double* gb_part;          // per block
    double* marg_part;        // per line (x1, y1 axes) or per block (x2, y2 axes)
    double db_coef;           // (tau/hbar) * kappa * 2 * (-e/hbar)
    double b_eoh;             // e B / hbar
    double kstep;             // 2 pi / Lx
    double y0, ystep;         // y grid
};

struct FftShape {
    int n1, n2, t;  // n = n1 * n2, t threads per line
};

// Supported line lengths and their register/LDS decomposition.
bool fft_shape(int n, FftShape* out);

// Threads per line of the three-stage pass kernel used for the long lines
// (n = 96, 128, 256), forward (one state) and reverse (two states); 0 where
// the two-stage kernel runs.
int axis3_threads(int n, int nst);

// Threads per block of the three-stage kernel: 1024 for the complex64 forward
// x1 pass at n = 256 (32 lines of 32 threads: 256-byte runs on its strided
// axis), 512 otherwise.
__host__ __device__ constexpr int axis3_block_threads(int axis, int n, int nst, bool mixed) {
    return (n == 256 && nst == 1 && mixed && axis == AX_X1) ? 1024 : 512;
}

// Lines per block of the three-stage kernel before the grid's divisibility
// limits (plan_axis may halve it further): the block's threads over the
// threads per line, halved until the exchange area and the staged factors fit
// the LDS budget -- 48 KB for the one-state n = 128 passes (three or more
// blocks per CU), 80 KB otherwise, counted in complex128 entries for the
// one-state passes of 256- or 512-thread blocks and in the storage's entry
// size for the 1024-thread and 32-line n = 128 complex64 blocks and the
// two-state passes.  The kernel is built with this width as a compile-time
// constant (LDS offsets become immediates) and with a run-time width.
__host__ __device__ constexpr int axis3_nominal_w(int axis, int n, int t3, int nst, bool mixed) {
    const int bt = axis3_block_threads(axis, n, nst, mixed);
    const bool wide = n != 128;
    // the complex64 x2 and (persistent) x1 and y1 passes of 128-point lines: 32 lines
    const bool c64_32 = n == 128 && nst == 1 && mixed && (axis == AX_X2 || axis == AX_Y1 || axis == AX_X1);
    int w = (bt == 1024 ? 1024 : (wide || c64_32) ? 512 : 256) / t3;
    const int cap = (bt == 1024 || c64_32) ? (81920 - 2 * n * 16) / (n * 8) - 1
                  : nst == 1 ? ((wide ? 81920 : 49152) - 2 * n * 16) / (n * 16) - 1
                             : (81920 - 2 * n * 16) / (2 * n * (mixed ? 8 : 16)) - 1;
    while (w > cap) w >>= 1;
    return w;
}

// Whether the two-stage kernel's exchanges on this axis are complex64 (with
// complex64 storage: every axis but x1).
__host__ __device__ constexpr bool axis_xchg_c64(int axis, bool mixed) { return mixed && axis != AX_X1; }

// Exchange area of the two-stage kernel: nst states x n positions x (W + 1)
// slots (n = 0 where the line needs no exchange), entries as above.
__host__ __device__ constexpr size_t axis_xchg_bytes(int n, int w, int nst, bool c64) {
    return ((size_t)nst * (size_t)n * (size_t)(w + 1) * (c64 ? 8u : 16u) + 15u) / 16u * 16u;
}

// LDS of the three-stage kernel: the exchange area (nst states x n positions x
// (W + 1) slots, complex64 entries with complex64 storage, complex128
// otherwise, rounded up to 16 bytes), then 2n staged FP64 factors.
__host__ __device__ constexpr size_t axis3_xchg_bytes(int n, int w, int nst, bool c64) {
    return ((size_t)nst * (size_t)n * (size_t)(w + 1) * (c64 ? 8u : 16u) + 15u) / 16u * 16u;
}
__host__ __device__ constexpr size_t axis3_lds_bytes(int n, int w, int nst, bool c64) {
    return axis3_xchg_bytes(n, w, nst, c64) + 2u * (size_t)n * 16u;
}
// ... of a pass: the persistent x1 pass keeps two kinetic rows after its
// twiddles, one more row of n complex128 entries
__host__ __device__ constexpr size_t axis3_pass_lds_bytes(int axis, int n, int w, int nst, bool c64, bool pers) {
    return axis3_lds_bytes(n, w, nst, c64) + ((pers && axis == AX_X1) ? (size_t)n * 16u : 0u);
}

// Launch one per-axis pass: blocks of t*W threads, nlines/W blocks; with pers
// (three-stage forward x1 and y1 passes only) the persistent form, as many
// blocks as fit the device at once, walking the a.ntiles = nlines/W tiles.
hipError_t launch_axis(int axis, int n, bool mixed, int nst, bool pers, const PassArgs& a, int64_t nlines,
                       size_t lds_bytes, hipStream_t s);

// Fused (x2, y2)-plane pass: X2(ktab) -> potential factor -> Y2(ktab2), one
// workgroup per electron-1 position.  Returns hipErrorInvalidValue when no
// kernel is built for (nx, ny, storage); plane_available() says beforehand.
bool plane_available(int nx, int ny, bool mixed);
hipError_t launch_plane(int nx, int ny, bool mixed, const PassArgs& a, hipStream_t s);

// Reductions and elementwise kernels.
hipError_t launch_init_norm(const double2* pa, const double2* pb, int sym, int nxy, double* part,
                            int nblocks, hipStream_t s);
hipError_t launch_init_write(void* psi, bool mixed, const double2* pa, const double2* pb, int sym,
                             int nxy, double scale, hipStream_t s);
hipError_t launch_obs(const void* psi, bool mixed, const double* w, int nxy, double* part, int nblocks,
                      hipStream_t s);
hipError_t launch_loss_lambda(const void* psi, void* lam, bool mixed, const double* w,
                              const double* coeffs_dev, int nxy, double* part, int nblocks,
                              hipStream_t s);
hipError_t launch_reduce_parts(const double* part, int nparts, int width, double* out, hipStream_t s);
hipError_t launch_gather(const void* psi, bool mixed, const int32_t* ix1, int n1, int jy1,
                         const int32_t* ix2, int n2, int jy2, int nx, int ny, double2* out,
                         hipStream_t s);
hipError_t launch_marginal(const void* psi, bool mixed, int nxy, double* out, hipStream_t s);
hipError_t launch_conditional(const void* psi, bool mixed, int nxy, int r2, double* out, hipStream_t s);
hipError_t launch_c128_to_c64(const double2* in, float2* out, int64_t count, hipStream_t s);
hipError_t launch_c64_to_c128(const float2* in, double2* out, int64_t count, hipStream_t s);
hipError_t launch_grad_finish(const double* m_x2, int bpr_x2, const double* m_y2, int bpr_y2,
                              const double* m_y1, const double* m_x1, int nx, int ny, double gscale,
                              double* dldv, hipStream_t s);
hipError_t launch_zero(double* p, int64_t count, hipStream_t s);

// Edge states of every grid wave number along x and one Gaussian edge-state
// packet built from them (edge_states.hip).  Device pointers: circ [ny] (first
// row of the spectral kinetic matrix), vcol [ny], kx [nx], work [2 nx ny^2],
// e1 [nx], phi [nx ny], psi [nx ny], part [nx], info [3] = (k0, E(k0), target).
struct EdgeArgs {
    const double* circ;
    const double* vcol;
    const double* kx;
    int nx, ny, top;
    double kappa, inv_lb2;   // meV nm^2, eB/hbar in 1/nm^2
    double x0, dx, y0, dy;   // grids (nm)
    double target, sigma, xc;
    double* work;
    double* e1;
    double* phi;
    double2* psi;
    double* part;
    double* info;
};
hipError_t launch_edge_packet(const EdgeArgs& e, hipStream_t s);

// Fixed device scratch of the no-allocation reverse sweep: kScratchDoubles
// FP64 values (64 MiB) per GPU.  init_scratch(device), with that device
// current, takes the array's address on it once; scratch_on(device) returns
// it afterwards (nullptr before).
constexpr size_t kScratchDoubles = (size_t(64) << 20) / sizeof(double);
constexpr int kMaxDevices = 64;
hipError_t init_scratch(int device);
double* scratch_on(int device);

}  // namespace hom4d_impl
