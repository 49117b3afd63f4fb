// Fused pass over the contiguous (x2, y2) plane of one electron-1 position.
//
// For fixed r1 = (x1, y1) the nx*ny values Psi(r1, x2, y2) are contiguous in
// the [x1][y1][x2][y2] layout.  One workgroup owns one such plane and applies,
// in one HBM read and one HBM write,
//     X2(tau):  transform along x2, kinetic phase of (k_x2, y2), inverse,
//     V(dt/2):  exp(-i dt/2 (V(r1) + V(r2) + V12(r1 - r2)) / hbar),
//     Y2(dt):   transform along y2, kinetic phase of k_y2, inverse,
// i.e. three consecutive factors of the Strang step (arXiv 1903.02581,
// Sec. II.C Eq. (evoloperat); the x and y kinetic terms of Appendix A).  The
// plane stays in LDS between the stages, in the storage precision (Xchg); the
// arithmetic is FP64.  Each line transform is the same register/LDS four-step
// network as the per-axis pass.
#pragma once

#include "axis_pass.hpp"

namespace hom4d_impl {
namespace dev {

template <int N>
struct Shape;
template <> struct Shape<4> { static constexpr int n1 = 4, n2 = 1, t = 1; };
template <> struct Shape<6> { static constexpr int n1 = 6, n2 = 1, t = 1; };
template <> struct Shape<8> { static constexpr int n1 = 8, n2 = 1, t = 1; };
template <> struct Shape<12> { static constexpr int n1 = 12, n2 = 1, t = 1; };
template <> struct Shape<16> { static constexpr int n1 = 4, n2 = 4, t = 4; };
template <> struct Shape<24> { static constexpr int n1 = 12, n2 = 2, t = 2; };
template <> struct Shape<32> { static constexpr int n1 = 8, n2 = 4, t = 4; };
template <> struct Shape<48> { static constexpr int n1 = 12, n2 = 4, t = 4; };
template <> struct Shape<64> { static constexpr int n1 = 8, n2 = 8, t = 8; };
template <> struct Shape<96> { static constexpr int n1 = 12, n2 = 8, t = 4; };
template <> struct Shape<128> { static constexpr int n1 = 16, n2 = 8, t = 8; };

// LDS row layout of the plane: element p of row r at r * row + (p ^ ((p / 8) % 8)),
// row = NY + NY / 8.  The XOR permutes each aligned group of 8 slots, so the
// image stays in bounds.  For 16-byte accesses, 16 consecutive lanes must hit
// 16 different 16-byte bank groups: the x stage (lanes along a row, stride 1),
// the y stage's row reads (8 lanes along each of two rows) and its sub-row
// reads (stride 8 along two rows) all do at 64 x 64, where row = 72 puts the
// two rows of a lane group half a bank cycle apart.
template <int NY>
struct PlaneLds {
    static_assert(NY % 8 == 0, "plane rows are whole groups of 8");
    static constexpr int row = NY + NY / 8;
    __device__ static __forceinline__ int at(int r, int p) { return r * row + (p ^ ((p >> 3) & 7)); }
};

// One plane per workgroup, grid = nx * ny.  Barriers: one after every LDS write
// that other wavefronts read back (the row exchanges of the Y2 stage stay
// inside one wavefront and only wait for its own writes); none before a write,
// because each exchange writes exactly the positions the same thread read in
// the previous one.
template <class S, int NX, int NY, int NT, int VK>
__global__ void __launch_bounds__(NT) k_plane2(const PassArgs a) {
    using SX_ = Shape<NX>;
    using SY_ = Shape<NY>;
    using LY = PlaneLds<NY>;
    constexpr int A1 = SX_::n1, A2 = SX_::n2, TX = SX_::t;
    constexpr int B1 = SY_::n1, B2 = SY_::n2, TY = SY_::t;
    constexpr int EX = NX / TX;
    constexpr int JAX = A2 / TX, IBX = A1 / TX;
    constexpr int JAY = B2 / TY, IBY = B1 / TY;
    constexpr int SLX = NY * TX, QX = (SLX + NT - 1) / NT;
    constexpr int SLY = NX * TY, QY = (SLY + NT - 1) / NT;
    using X = Xchg<S>;
    // Where the potential factor is applied: at the end of the X2 stage (FP64
    // storage) or as the Y2 stage reads its rows (complex64 storage, where the
    // smaller register footprint buys a resident wavefront per SIMD).
    constexpr bool V_IN_Y = !std::is_same<S, double2>::value;
    __shared__ typename X::T L[NX * LY::row];
    __shared__ double2 TW[NX + 2 * NY];  // x twiddles, y twiddles, y kinetic factor

    const int tid = threadIdx.x;
    const int r1 = blockIdx.x;
    const int i1 = r1 / NY, j1 = r1 % NY;
    // The one-body factor of electron 1 is one number for the whole plane, so it
    // is folded into the y kinetic factor here instead of multiplying each point.
    const double2 v1 = (VK == 1) ? a.a1[r1] : make_double2(1.0, 0.0);
    for (int i = tid; i < NX + 2 * NY; i += NT) {
        double2 v;
        if (i < NX) v = a.tw[i];
        else if (i < NX + NY) v = a.tw2[i - NX];
        else {
            v = a.ktab2[i - NX - NY];
            if constexpr (VK == 1) v = cmul(v, v1);
        }
        TW[i] = v;
    }

    // X2 stage slot of this thread: column c (= y2) and thread-in-line t
    auto slot_x = [&](int q, int* c, int* t) {
        const int s = tid + NT * q;
        *c = s % NY;
        *t = s / NY;
        return s < SLX;
    };

    S* base = reinterpret_cast<S*>(a.psi) + (int64_t)r1 * (NX * NY);
    double2 vx[QX][EX];
#pragma unroll
    for (int q = 0; q < QX; ++q) {
        int c, t;
        if (slot_x(q, &c, &t)) {
#pragma unroll
            for (int jj = 0; jj < JAX; ++jj)
#pragma unroll
                for (int n1 = 0; n1 < A1; ++n1) vx[q][jj * A1 + n1] = ld<S>(base + (n1 * A2 + t + TX * jj) * NY + c);
        }
    }
    __syncthreads();  // TW staged
    {
        const double2* twx = TW;
        const double2* twy = TW + NX;
        const double2* ky = TW + NX + NY;
        const double2* kx = a.ktab;
        const PassArgs& av = a;

        // ---------------- X2 stage A: DFT_A1 on the loaded columns, twiddles
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            int c, t;
            if (slot_x(q, &c, &t)) {
#pragma unroll
                for (int jj = 0; jj < JAX; ++jj) {
                    dft<A1, -1>(&vx[q][jj * A1]);
                    if constexpr (A2 > 1) {
                        const int jc = t + TX * jj;
#pragma unroll
                        for (int k1 = 1; k1 < A1; ++k1)
                            vx[q][jj * A1 + k1] = cmul(vx[q][jj * A1 + k1], twx[(jc * k1) % NX]);
                    }
                }
            }
        }
        double2 vb[QX][EX];  // stage-B / real-space values of the X2 stage
        if constexpr (A2 > 1) {
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                int c, t;
                if (slot_x(q, &c, &t)) {
#pragma unroll
                    for (int jj = 0; jj < JAX; ++jj)
#pragma unroll
                        for (int k1 = 0; k1 < A1; ++k1) L[LY::at(k1 * A2 + t + TX * jj, c)] = X::put(vx[q][jj * A1 + k1]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                int c, t;
                if (slot_x(q, &c, &t)) {
#pragma unroll
                    for (int ii = 0; ii < IBX; ++ii)
#pragma unroll
                        for (int j = 0; j < A2; ++j) vb[q][ii * A2 + j] = X::get(L[LY::at((t + TX * ii) * A2 + j, c)]);
#pragma unroll
                    for (int ii = 0; ii < IBX; ++ii) dft<A2, -1>(&vb[q][ii * A2]);
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < QX; ++q)
#pragma unroll
                for (int e = 0; e < EX; ++e) vb[q][e] = vx[q][e];
        }
        // kinetic x phase at (k_x2, y2), then the inverse transform
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            int c, t;
            if (slot_x(q, &c, &t)) {
                const double2* kt = kx + c;  // k-major table: [k][y2]
#pragma unroll
                for (int ii = 0; ii < IBX; ++ii)
#pragma unroll
                    for (int k2 = 0; k2 < A2; ++k2) {
                        double2 f = kt[(t + TX * ii + A1 * k2) * NY];
                        vb[q][ii * A2 + k2] = cmul(vb[q][ii * A2 + k2], f);
                    }
                if constexpr (A2 > 1) {
#pragma unroll
                    for (int ii = 0; ii < IBX; ++ii) dft<A2, 1>(&vb[q][ii * A2]);
                }
            }
        }
        if constexpr (A2 > 1) {
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                int c, t;
                if (slot_x(q, &c, &t)) {
#pragma unroll
                    for (int ii = 0; ii < IBX; ++ii)
#pragma unroll
                        for (int j = 0; j < A2; ++j) L[LY::at((t + TX * ii) * A2 + j, c)] = X::put(vb[q][ii * A2 + j]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                int c, t;
                if (slot_x(q, &c, &t)) {
#pragma unroll
                    for (int jj = 0; jj < JAX; ++jj)
#pragma unroll
                        for (int k1 = 0; k1 < A1; ++k1) vb[q][jj * A1 + k1] = X::get(L[LY::at(k1 * A2 + t + TX * jj, c)]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            int c, t;
            if (slot_x(q, &c, &t)) {
#pragma unroll
                for (int jj = 0; jj < JAX; ++jj) {
                    if constexpr (A2 > 1) {
                        const int jc = t + TX * jj;
#pragma unroll
                        for (int k1 = 1; k1 < A1; ++k1)
                            vb[q][jj * A1 + k1] = cmulc(vb[q][jj * A1 + k1], twx[(jc * k1) % NX]);
                    }
                    dft<A1, 1>(&vb[q][jj * A1]);
                }
                if constexpr (!V_IN_Y) {
                    // potential factor in real space at (x2 = n1 * A2 + t + TX * jj, y2 = c)
#pragma unroll
                    for (int jj = 0; jj < JAX; ++jj)
#pragma unroll
                        for (int n1 = 0; n1 < A1; ++n1) {
                            const double2 f = vfactor<VK == 1 ? 3 : VK, false>(av, i1, j1, n1 * A2 + t + TX * jj, c);
                            vb[q][jj * A1 + n1] = cmul(vb[q][jj * A1 + n1], f);
                        }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            int c, t;
            if (slot_x(q, &c, &t)) {
#pragma unroll
                for (int jj = 0; jj < JAX; ++jj)
#pragma unroll
                    for (int n1 = 0; n1 < A1; ++n1) L[LY::at(n1 * A2 + t + TX * jj, c)] = X::put(vb[q][jj * A1 + n1]);
            }
        }
        __syncthreads();

        // ---------------- Y2 stage: lines along y2, one per x2 (row of the plane)
        // When every row's TY threads sit in one wavefront and each wavefront owns
        // whole rows, the row exchanges stay inside the wavefront: it waits for its
        // own LDS writes before it reads (the memory clobber keeps the compiler
        // from moving or forwarding LDS accesses across the wait); no workgroup
        // barrier.  (The column exchanges of the X2 stage span wavefronts: a
        // column-per-wavefront thread mapping measured slower, 127 -> 150 us.)
        // Each sub-transform reads and writes back the same LDS slots, so the
        // stages take one sub-transform at a time and hold only its values in
        // registers.
        constexpr bool Y_WAVE = (QY == 1) && (64 % TY == 0);
        auto y_sync = [&]() {
            if constexpr (Y_WAVE)
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            else
                __syncthreads();
        };
        if constexpr (B2 > 1) {
            // stage A: DFT_B1 and twiddles, in place
#pragma unroll
            for (int q = 0; q < QY; ++q) {
                const int s = tid + NT * q;
                if (s < SLY) {
                    const int t = s % TY, row = s / TY;
#pragma unroll
                    for (int jj = 0; jj < JAY; ++jj) {
                        double2 u[B1];
#pragma unroll
                        for (int n1 = 0; n1 < B1; ++n1) u[n1] = X::get(L[LY::at(row, n1 * B2 + t + TY * jj)]);
                        if constexpr (V_IN_Y) {
                            // potential factor in real space at (x2 = row, y2)
#pragma unroll
                            for (int n1 = 0; n1 < B1; ++n1)
                                u[n1] = cmul(u[n1], vfactor<VK == 1 ? 3 : VK, false>(av, i1, j1, row, n1 * B2 + t + TY * jj));
                        }
                        dft<B1, -1>(u);
                        const int jc = t + TY * jj;
#pragma unroll
                        for (int k1 = 1; k1 < B1; ++k1) u[k1] = cmul(u[k1], twy[(jc * k1) % NY]);
#pragma unroll
                        for (int k1 = 0; k1 < B1; ++k1) L[LY::at(row, k1 * B2 + t + TY * jj)] = X::put(u[k1]);
                    }
                }
            }
            y_sync();
            // stage B: DFT_B2, kinetic y phase, inverse DFT_B2, in place
#pragma unroll
            for (int q = 0; q < QY; ++q) {
                const int s = tid + NT * q;
                if (s < SLY) {
                    const int t = s % TY, row = s / TY;
#pragma unroll
                    for (int ii = 0; ii < IBY; ++ii) {
                        double2 u[B2];
#pragma unroll
                        for (int j = 0; j < B2; ++j) u[j] = X::get(L[LY::at(row, (t + TY * ii) * B2 + j)]);
                        dft<B2, -1>(u);
#pragma unroll
                        for (int k2 = 0; k2 < B2; ++k2) u[k2] = cmul(u[k2], ky[t + TY * ii + B1 * k2]);
                        dft<B2, 1>(u);
#pragma unroll
                        for (int j = 0; j < B2; ++j) L[LY::at(row, (t + TY * ii) * B2 + j)] = X::put(u[j]);
                    }
                }
            }
            y_sync();
            // stage A inverse: conjugate twiddles, inverse DFT_B1, store
#pragma unroll
            for (int q = 0; q < QY; ++q) {
                const int s = tid + NT * q;
                if (s < SLY) {
                    const int t = s % TY, row = s / TY;
#pragma unroll
                    for (int jj = 0; jj < JAY; ++jj) {
                        double2 u[B1];
#pragma unroll
                        for (int k1 = 0; k1 < B1; ++k1) u[k1] = X::get(L[LY::at(row, k1 * B2 + t + TY * jj)]);
                        const int jc = t + TY * jj;
#pragma unroll
                        for (int k1 = 1; k1 < B1; ++k1) u[k1] = cmulc(u[k1], twy[(jc * k1) % NY]);
                        dft<B1, 1>(u);
#pragma unroll
                        for (int n1 = 0; n1 < B1; ++n1) st<S>(base + row * NY + n1 * B2 + t + TY * jj, u[n1]);
                    }
                }
            }
        } else {
            // a whole row per thread: DFT, kinetic y phase, inverse DFT
#pragma unroll
            for (int q = 0; q < QY; ++q) {
                const int s = tid + NT * q;
                if (s < SLY) {
                    const int row = s / TY;
                    double2 u[B1];
#pragma unroll
                    for (int n1 = 0; n1 < B1; ++n1) {
                        u[n1] = X::get(L[LY::at(row, n1)]);
                        if constexpr (V_IN_Y) u[n1] = cmul(u[n1], vfactor<VK == 1 ? 3 : VK, false>(av, i1, j1, row, n1));
                    }
                    dft<B1, -1>(u);
#pragma unroll
                    for (int k1 = 0; k1 < B1; ++k1) u[k1] = cmul(u[k1], ky[k1]);
                    dft<B1, 1>(u);
#pragma unroll
                    for (int n1 = 0; n1 < B1; ++n1) st<S>(base + row * NY + n1, u[n1]);
                }
            }
        }
    }
}

// Threads per plane workgroup: enough for the larger of the two stages, at most 1024.
constexpr int plane_threads(int nx, int ny, int tx, int ty) {
    const int s = (ny * tx > nx * ty) ? ny * tx : nx * ty;
    const int r = ((s + 63) / 64) * 64;
    return r > 1024 ? 1024 : r;
}

}  // namespace dev
}  // namespace hom4d_impl

