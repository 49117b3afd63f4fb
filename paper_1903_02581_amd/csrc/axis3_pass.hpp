// Per-axis pass for the long lines (n = 96, 128, 256) of the forward step:
// the same transform -> kinetic phase -> inverse round trip as k_axis
// (Sec. II.C Eq. (evoloperat); kinetic terms of Appendix A), with the line
// transform factored into three radix stages instead of two, so that every
// thread holds 8 (or 12) elements instead of 16 (or 24) and the kernels keep
// enough waves resident to stream HBM.  n = 256 takes 32 threads per line, so
// its blocks hold 16 lines in 512 threads (128-byte runs on the strided axes
// in complex64 storage), or 32 lines in 1024 threads on the complex64 x1
// pass.
//
// Line of n = R1 R2 R3 points, element m = n1 (R2 R3) + n2 R3 + j3, handled by T
// threads.  Forward:
//   stage A   DFT_R1 over n1 for each column jc = n2 R3 + j3, twiddle w_n^(jc k1);
//   stage B1  DFT_R2 over n2 for each (k1, j3), twiddle w_(R2 R3)^(j3 k2);
//   stage B2  DFT_R3 over j3 for each (k1, k2);
// giving wave number k = k1 + R1 (k2 + R2 k3).  The kinetic phase is applied
// there, and the transposed network (conjugate twiddles, inverse DFTs in the
// reverse order) brings every thread back to the elements it loaded.  Between
// stages the line is exchanged through LDS, each stage reading and writing its
// own disjoint set of positions.
//
// PERS (the forward one-state passes and the reverse sweep's x1 pass): the
// kernel is persistent: a block
// walks tiles of W lines (tile = blockIdx.x, + gridDim.x, ...) and issues the
// loads of its next tile while it transforms the current one (at its start, or
// on the wide forms in four parts between its exchanges), so that the HBM
// reads of one tile overlap the arithmetic and LDS exchanges of the previous
// one inside the block, instead of relying on other resident blocks being out
// of phase.  The two-state form loads and stores both states and takes its
// gradient partial sums per tile, with LDS-only barriers, and synchronises once
// more after them before the next tile reuses the exchange area.  Its exchanges synchronise the block on LDS alone (lds_barrier),
// leaving the prefetch loads and the stores in flight.  It pays where a pass
// has few resident blocks per CU: measured on the complex64 x1 and y1 passes
// of the 256x128 state (x1 6.07 -> 5.36 ms, y1 4.46 -> 4.20 ms); the x2 and
// y2 passes, the FP64 passes and n = 96 lines ran slower that way (128x96
// complex64 y1 0.52 -> 0.61 ms, y2 0.72 -> 0.86 ms; 128x128 FP64 x1 1.62 ->
// 1.79 ms), so they keep one tile per block.  No global load is waited for
// inside a tile's transform (the x1 pass takes its kinetic factors from LDS),
// and the first tile is peeled off the loop, so that the only wait for the
// prefetch, at the start of the next tile, leaves the stores in flight.
//
// The arithmetic is FP64 for both storage types.  With complex64 storage the
// exchange area holds complex64 too: each exchange then rounds like one more
// store of the state (random, not coherent, since the state changes every
// step), and the area takes half the LDS, so twice as many blocks fit a CU.
#pragma once

#include "axis_pass.hpp"

namespace hom4d_impl {
namespace dev {

template <int R1, int R2, int R3, int T>
struct Net3 {
    static constexpr int N = R1 * R2 * R3, N2 = R2 * R3;
    static constexpr int JA = N2 / T;        // stage-A columns per thread
    static constexpr int G1 = R1 * R3 / T;   // stage-B1 groups per thread
    static constexpr int G2 = R1 * R2 / T;   // stage-B2 groups per thread
    static constexpr int E = JA * R1;        // elements per thread
    static_assert(N2 % T == 0 && (R1 * R3) % T == 0 && (R1 * R2) % T == 0, "T must split every stage");
    static_assert(G1 * R2 == E && G2 * R3 == E, "every stage must give a thread E elements");
};

// Block-wide synchronisation on LDS only: wait for this wave's LDS accesses,
// then the barrier.  Global loads and stores stay in flight (a fence-carrying
// __syncthreads would wait for them); the memory clobber keeps the compiler
// from moving LDS accesses across it.  Exchanges along y2 with T | 64 stay
// wave-local as in line_sync.
template <int AXIS, int T>
__device__ __forceinline__ void lds_barrier() {
    if constexpr (AXIS == AX_Y2 && 64 % T == 0)
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    else
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Elements per batch of the table-form potential loads: 2 on the complex64 y2
// pass of 128- and 256-point lines (90 instead of 116 VGPRs, five waves per
// SIMD instead of four: 256x128 y2+V 4.66 -> 4.48 ms), 4 elsewhere (the
// complex64 x2 pass measured slower with 2: 5.21 -> 5.36 ms, 128x96 0.674 ->
// 0.717 ms).
constexpr int potential_batch(int axis, int n, bool c64) { return (c64 && axis == AX_Y2 && n >= 128) ? 2 : 4; }

// WC > 0: the block holds WC lines, a compile-time constant (the nominal width
// of the pass, axis3_nominal_w), so every LDS address is a per-thread base plus
// an immediate offset; WC = 0: a.W lines, for grids that allow fewer.
template <class S, int AXIS, int R1, int R2, int R3, int T, int NST, int VK, bool NT, bool PERS, int WC>
__global__ void __launch_bounds__(axis3_block_threads(AXIS, R1 * R2 * R3, NST, !std::is_same<S, double2>::value)) k_axis3(const PassArgs a) {
    static_assert(!PERS || NST == 1 || AXIS == AX_X1, "persistent: the forward passes and the reverse x1 pass");
    // the reverse sweep (two states) applies every factor conjugated
    constexpr bool CONJ = NST == 2;
    using NW = Net3<R1, R2, R3, T>;
    constexpr int N = NW::N, N2 = NW::N2, JA = NW::JA, G1 = NW::G1, G2 = NW::G2, E = NW::E;
    using X = Xchg<S>;
    extern __shared__ double2 lds_raw[];

    const int W = WC > 0 ? WC : a.W;
    const int tid = threadIdx.x;
    int t, cl;
    if constexpr (AXIS == AX_Y2) {
        t = tid % T;
        cl = tid / T;
    } else {
        cl = tid % W;
        t = tid / W;
    }

    // twiddles w_n^j (and, on y axes, the kinetic factor) staged after the exchange area
    constexpr bool KT_LDS = (AXIS == AX_Y1 || AXIS == AX_Y2);
    // persistent x1 pass: the tile's kinetic row (its lines share y1) comes from
    // one of two LDS rows after the twiddles, written at the start of the tile
    // from a register loaded with the previous tile's prefetch, so that no
    // global load is issued inside the transform (a wait for one would also wait
    // for the next tile's loads and the previous tile's stores, issued earlier)
    constexpr bool KROW = PERS && AXIS == AX_X1;
    const double2* krow = nullptr;
    const int LS = W + 1;  // padded LDS row: one line position across the block's W lines
    typename X::T* lds = reinterpret_cast<typename X::T*>(lds_raw);
    double2* twl = reinterpret_cast<double2*>(reinterpret_cast<char*>(lds_raw) +
                                              axis3_xchg_bytes(N, W, NST, sizeof(typename X::T) == 8));
    for (int i = tid; i < (KT_LDS ? 2 * N : N); i += T * W) {
        double2 w;
        if (i < N) {
            w = a.tw[i];
        } else {
            w = a.ktab[i - N];
            if constexpr (CONJ) w = conjd(w);
        }
        twl[i] = w;
    }
    __syncthreads();
    // state s, line position pos: s * N + pos rows of W + 1 slots
    auto Lw = [&](int st_, int pos, double2 v) { lds[(st_ * N + pos) * LS + cl] = X::put(v); };
    auto Lr = [&](int st_, int pos) -> double2 { return X::get(lds[(st_ * N + pos) * LS + cl]); };
    // the exchanges: LDS-only barriers in the persistent passes
    auto sync = [&]() {
        if constexpr (PERS)
            lds_barrier<AXIS, T>();
        else
            line_sync<AXIS, T>();
    };
    // element jj * R1 + n1 of a thread: line position n1 N2 + t + T jj
    // visit the thread's elements e = jj R1 + n1 of a line (line position
    // n1 N2 + t + T jj) with their addresses, stepping from one to the next by a
    // 64-bit add rather than forming each offset by multiplication
    auto walk = [&](const LineGeom<AXIS>& lg, auto* base, auto&& fn) {
        const int64_t step = (int64_t)N2 * lg.sN;
#pragma unroll
        for (int jj = 0; jj < JA; ++jj) {
            auto* p = base + (int64_t)(t + T * jj) * lg.sN;
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) {
                fn(jj * R1 + n1, p);
                p += step;
            }
        }
    };

    // elements e0 .. e1 - 1 of the walk above, each address formed directly
    auto walk_part = [&](const LineGeom<AXIS>& lg, auto* base, int e0, int e1, auto&& fn) {
#pragma unroll
        for (int e = e0; e < e1; ++e) {
            const int jj = e / R1, n1 = e % R1;
            fn(e, base + ((int64_t)(t + T * jj) + (int64_t)n1 * N2) * lg.sN);
        }
    };

    // Transform round trip of the block's tile held in v (loaded elements in,
    // the same elements out, stored in place), with the potential factor and
    // the reverse sweep's gradient terms.  between(k) runs after the k-th of the
    // four exchanges (k = 0..3).
    double2 v[NST][E];
    auto round_trip = [&](const LineGeom<AXIS>& lg, uint32_t line, uint32_t blk, S* const* ps, auto&& between) {
        // gradient accumulators of the reverse sweep: the potential marginal
        // Im(conj(lambda) psi) on the side of the potential factor the pass is told
        // to take it (before: G_MIN, after: G_MOUT), and the dL/dB term of the x
        // kinetic factor in reciprocal space
        double gm_acc = 0.0, gb_acc = 0.0;
        if constexpr (NST == 2) {
            if (a.gflags & G_MIN) {
#pragma unroll
                for (int e = 0; e < E; ++e) gm_acc += im_cl_p(v[1][e], v[0][e]);
            }
        }
        // the potential factor on the thread's elements (element e = jj R1 + n1 at
        // line position n1 N2 + t + T jj), its table entries loaded in batches
        auto potential = [&]() {
            if constexpr (VK == 1) {
                const LineTables<AXIS> tb(a, lg, t);
                const double2 f0 = tb.fixed();
                batched<E, potential_batch(AXIS, N, !std::is_same<S, double2>::value)>([&](int e) { return tb.load((e % R1) * N2 + T * (e / R1)); },
                              [&](int e, const VLoad& l) {
                                  const double2 f = tb.template combine<CONJ>(f0, l);
#pragma unroll
                                  for (int s = 0; s < NST; ++s) v[s][e] = cmul(v[s][e], f);
                              });
            } else {
                constexpr int VKF = VK == 0 ? 1 : VK;
                auto coords = [&](int e, int* c) {
                    elem_coord<AXIS>(lg.i1, lg.j1, lg.i2, lg.j2, (e % R1) * N2 + t + T * (e / R1), c);
                };
                batched<E, vbatch<VKF>()>(
                    [&](int e) {
                        int c[4];
                        coords(e, c);
                        return vload<VKF>(a, c[0], c[1], c[2], c[3]);
                    },
                    [&](int e, const VLoad& l) {
                        int c[4];
                        coords(e, c);
                        const double2 f = vcombine<VKF, CONJ>(a, l, c[0], c[1], c[2], c[3]);
#pragma unroll
                        for (int s = 0; s < NST; ++s) v[s][e] = cmul(v[s][e], f);
                    });
            }
        };
        if (VK != 0 && a.vmode == 1) potential();

        // ---- stage A (forward)
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int jj = 0; jj < JA; ++jj) {
                const int jc = t + T * jj;
                dft<R1, -1>(&v[s][jj * R1]);
#pragma unroll
                for (int k1 = 1; k1 < R1; ++k1) v[s][jj * R1 + k1] = cmul(v[s][jj * R1 + k1], twl[(uint32_t)(jc * k1) % N]);
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) Lw(s, k1 * N2 + jc, v[s][jj * R1 + k1]);
            }
        sync();
        between(0);

        // ---- stage B1 (forward), in place on its positions
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int ii = 0; ii < G1; ++ii) {
                const int q = t + T * ii, k1 = q / R3, j3 = q % R3;
#pragma unroll
                for (int n2 = 0; n2 < R2; ++n2) v[s][ii * R2 + n2] = Lr(s, k1 * N2 + n2 * R3 + j3);
                dft<R2, -1>(&v[s][ii * R2]);
#pragma unroll
                for (int k2 = 1; k2 < R2; ++k2) v[s][ii * R2 + k2] = cmul(v[s][ii * R2 + k2], twl[(uint32_t)(R1 * j3 * k2) % N]);
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) Lw(s, k1 * N2 + k2 * R3 + j3, v[s][ii * R2 + k2]);
            }
        sync();
        between(1);

        // ---- stage B2: forward, kinetic phase at k = k1 + R1 (k2 + R2 k3), inverse
        // x kinetic factor table: y-major [y][k] on the x1 pass, k-major [k][y] on the x2 pass
        const int yrow = (AXIS == AX_X1) ? lg.j1 : ((AXIS == AX_X2) ? lg.j2 : 0);
        const double2* kt = a.ktab + (AXIS == AX_X1 ? (int64_t)yrow * N : (int64_t)yrow);
        const int64_t kstride = AXIS == AX_X1 ? 1 : a.ny;
        constexpr bool GB = (NST == 2) && (AXIS == AX_X1 || AXIS == AX_X2);
        const bool gb_on = GB && (a.gflags & G_GB);
        const double yv = a.y0 + a.ystep * yrow;
        const double shift = yv * a.b_eoh;
#pragma unroll
        for (int ii = 0; ii < G2; ++ii) {
            const int q = t + T * ii, k1 = q / R2, k2 = q % R2;
            // x axes: the group's kinetic factors come from the L2-resident table;
            // their loads are issued ahead of the LDS reads and the DFT, which hide them
            double2 kf[R3];
            if constexpr (!KT_LDS) {
#pragma unroll
                for (int k3 = 0; k3 < R3; ++k3)
                    kf[k3] = KROW ? krow[k1 + R1 * (k2 + R2 * k3)] : kt[(k1 + R1 * (k2 + R2 * k3)) * kstride];
                if constexpr (!KROW) after_loads();
            }
#pragma unroll
            for (int s = 0; s < NST; ++s) {
#pragma unroll
                for (int j3 = 0; j3 < R3; ++j3) v[s][ii * R3 + j3] = Lr(s, k1 * N2 + k2 * R3 + j3);
                dft<R3, -1>(&v[s][ii * R3]);
            }
#pragma unroll
            for (int k3 = 0; k3 < R3; ++k3) {
                const int k = k1 + R1 * (k2 + R2 * k3);
                if constexpr (GB) {
                    if (gb_on) {
                        // d theta_X / dB at (k, y), on the values before the kinetic factor
                        const int m = (k < (N + 1) / 2) ? k : k - N;
                        const double dth = a.db_coef * (a.kstep * m - shift) * yv;
                        gb_acc += dth * im_cl_p(v[1][ii * R3 + k3], v[0][ii * R3 + k3]);
                    }
                }
                double2 f;
                if constexpr (KT_LDS) {
                    f = twl[N + k];
                } else {
                    f = kf[k3];
                    if constexpr (CONJ) f = conjd(f);
                }
#pragma unroll
                for (int s = 0; s < NST; ++s) v[s][ii * R3 + k3] = cmul(v[s][ii * R3 + k3], f);
            }
#pragma unroll
            for (int s = 0; s < NST; ++s) {
                dft<R3, 1>(&v[s][ii * R3]);
#pragma unroll
                for (int j3 = 0; j3 < R3; ++j3) Lw(s, k1 * N2 + k2 * R3 + j3, v[s][ii * R3 + j3]);
            }
        }
        sync();
        between(2);

        // ---- stage B1 (inverse)
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int ii = 0; ii < G1; ++ii) {
                const int q = t + T * ii, k1 = q / R3, j3 = q % R3;
#pragma unroll
                for (int k2 = 0; k2 < R2; ++k2) v[s][ii * R2 + k2] = Lr(s, k1 * N2 + k2 * R3 + j3);
#pragma unroll
                for (int k2 = 1; k2 < R2; ++k2) v[s][ii * R2 + k2] = cmulc(v[s][ii * R2 + k2], twl[(uint32_t)(R1 * j3 * k2) % N]);
                dft<R2, 1>(&v[s][ii * R2]);
#pragma unroll
                for (int n2 = 0; n2 < R2; ++n2) Lw(s, k1 * N2 + n2 * R3 + j3, v[s][ii * R2 + n2]);
            }
        sync();
        between(3);

        // ---- stage A (inverse), back on the loaded elements
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int jj = 0; jj < JA; ++jj) {
                const int jc = t + T * jj;
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) v[s][jj * R1 + k1] = Lr(s, k1 * N2 + jc);
#pragma unroll
                for (int k1 = 1; k1 < R1; ++k1) v[s][jj * R1 + k1] = cmulc(v[s][jj * R1 + k1], twl[(uint32_t)(jc * k1) % N]);
                dft<R1, 1>(&v[s][jj * R1]);
            }

        if (VK != 0 && a.vmode == 2) potential();

        if constexpr (NST == 2) {
            if (a.gflags & G_MOUT) {
#pragma unroll
                for (int e = 0; e < E; ++e) gm_acc += im_cl_p(v[1][e], v[0][e]);
            }
        }

#pragma unroll
        for (int s = 0; s < NST; ++s) walk(lg, ps[s], [&](int e, S* p) { st<S, NT>(p, v[s][e]); });

        if constexpr (NST == 2) {
            // the same partial-sum layout as the two-stage pass: dL/dB per block; the
            // marginal per line on the x1 and y1 axes (the line's threads summed in
            // fixed order), per block on x2 and y2 (a block's lines share r1)
            double* red = reinterpret_cast<double*>(lds_raw);
            // block-wide synchronisation on LDS alone in the persistent form (the
            // next tile's loads stay in flight)
            auto bsync = [&]() {
                if constexpr (PERS)
                    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                else
                    __syncthreads();
            };
            if (a.gflags & G_GB) {
                double sum;
                if constexpr (PERS) {
                    // block_sum's order: the wavefront's butterfly, then the wavefronts in turn
                    double g = gb_acc;
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) g += __shfl_xor(g, o, 64);
                    bsync();
                    if ((tid & 63) == 0) red[tid >> 6] = g;
                    bsync();
                    sum = 0.0;
                    if (tid == 0)
                        for (int w = 0; w < (T * W) / 64; ++w) sum += red[w];
                } else {
                    sum = block_sum(gb_acc, red);
                }
                if (tid == 0) a.gb_part[blk] += sum;
            }
            if (a.gflags & (G_MIN | G_MOUT)) {
                if constexpr (AXIS == AX_X1 || AXIS == AX_Y1) {
                    bsync();
                    red[t * W + cl] = gm_acc;
                    bsync();
                    if (t == 0) {
                        double sum = 0.0;
                        for (int q = 0; q < T; ++q) sum += red[q * W + cl];
                        a.marg_part[line] += sum;
                    }
                } else {
                    const double sum = block_sum(gm_acc, red);
                    if (tid == 0) a.marg_part[blk] += sum;
                }
            }
            // the next tile's first exchange reuses the area the sums were read from
            if constexpr (PERS) {
                if (a.gflags & (G_GB | G_MIN | G_MOUT)) bsync();
            }
        }
    };

    if constexpr (PERS) {
        // persistent: tiles blockIdx.x, + gridDim.x, ...; the next tile's
        // elements are loaded (as stored) before the current one is transformed
        const uint32_t ntiles = a.ntiles;
        S raw[NST][E];
        auto state = [&](int s) { return reinterpret_cast<S*>(s == 0 ? a.psi : a.lam); };
        double2 kreg = make_double2(0.0, 0.0);  // KROW: entry tid of the next tile's kinetic row
        // the kinetic row of tile tl: y1 of its lines (a tile's lines share y1)
        auto krow_of = [&](uint32_t tl) { return a.ktab + (int64_t)a.dnxy.div(tl * (uint32_t)W) * N; };
        uint32_t tile = blockIdx.x;
        if (tile < ntiles) {
            const LineGeom<AXIS> lg(a, tile * (uint32_t)W + (uint32_t)cl);
#pragma unroll
            for (int s = 0; s < NST; ++s)
                walk(lg, static_cast<const S*>(state(s)) + lg.base,
                     [&](int e, const S* p) { raw[s][e] = ld_raw<S, NT>(p); });
            if constexpr (KROW) {
                if (tid < N) kreg = krow_of(tile)[tid];
            }
        }
        uint32_t it = 0;  // the block's tile count: parity selects the kinetic row
        // The wide persistent forms -- the 256-point x1 pass (1024-thread blocks,
        // one per CU whatever their registers up to 128) and the 128-point x1 and
        // y1 passes (32-line 512-thread blocks, two per CU at up to 128 registers) -- keep
        // the thread's tile-invariant addresses in registers, and issue the next
        // tile's loads in parts while the current tile is transformed, instead of
        // all at its start (the schedule below).  Elsewhere the thread's line slot and
        // position index pass through an empty asm each tile, so that the LDS and
        // table addresses derived from them are recomputed per tile rather than
        // hoisted out of the loop and held in registers for all of it, and the
        // loads go out at once.  Hoisting: 256x128 x1 96 -> 120 VGPRs, about 8
        // fewer VALU instructions per point, 5.25 -> 5.12 ms; y1 with 32-line
        // blocks 4.28 -> 3.89 ms.  Spreading (the schedule below), 256x128: x1
        // 5.10 -> 4.41 ms, y1 3.83 -> 3.57-3.62 ms, with fewer registers held over
        // the tile; the 128-point x1 pass in 32-line blocks, hoisted and in four
        // parts from the start: 128x96 0.559 -> 0.526 ms, 128x64 0.279 -> 0.234 ms
        // (its 16-line blocks measured 0.549 -> 0.554 ms in four parts and
        // loads at once).
        constexpr bool WIDE = WC > 0 && ((AXIS == AX_X1 && (N == 256 || N == 128)) || (AXIS == AX_Y1 && N == 128));
        auto one_tile = [&](uint32_t tl) {
            if constexpr (!WIDE) asm volatile("" : "+v"(t), "+v"(cl));
            const uint32_t line = tl * (uint32_t)W + (uint32_t)cl;
            const LineGeom<AXIS> lg(a, line);
            S* ps[NST];
#pragma unroll
            for (int s = 0; s < NST; ++s) ps[s] = state(s) + lg.base;
#pragma unroll
            for (int s = 0; s < NST; ++s)
#pragma unroll
                for (int e = 0; e < E; ++e) v[s][e] = widen(raw[s][e]);
            if constexpr (KROW) {
                // visible to every thread after the first exchange barrier; the row
                // written two tiles ago was last read before this tile's barriers
                double2* row = twl + N * (1 + (it & 1));
                if (tid < N) row[tid] = kreg;
                krow = row;
            }
            const uint32_t next = tl + gridDim.x;
            if constexpr (WIDE) {
                const bool has_next = next < ntiles;
                const LineGeom<AXIS> ln(a, (has_next ? next : tl) * (uint32_t)W + (uint32_t)cl);
                const S* nbase[NST];
#pragma unroll
                for (int s = 0; s < NST; ++s) nbase[s] = state(s) + ln.base;
                if constexpr (KROW) {
                    if (has_next && tid < N) kreg = krow_of(next)[tid];
                }
                // NP parts of the E elements, part j issued at slot FIRST + j (slot -1:
                // before the first stage, slot k >= 0: after exchange k): x1 in four
                // parts from the start of the tile, y1 in two after its first two
                // exchanges, the fastest of the schedules measured (x1 four parts
                // after the four exchanges 4.56-4.65 ms, three or two from the start
                // 4.62 and 4.76 ms; y1 four parts 3.59-3.68 ms)
                constexpr int NP = AXIS == AX_X1 ? 4 : 2;
                constexpr int FIRST = AXIS == AX_X1 ? -1 : 0;
                constexpr int PART = (E + NP - 1) / NP;
                auto part = [&](int slot) {
                    const int j = slot - FIRST;
                    if (has_next && j >= 0 && j < NP) {
#pragma unroll
                        for (int s = 0; s < NST; ++s)
                            walk_part(ln, nbase[s], j * PART, (j + 1) * PART < E ? (j + 1) * PART : E,
                                      [&](int e, const S* p) { raw[s][e] = ld_raw<S, NT>(p); });
                    }
                };
                part(-1);
                round_trip(lg, line, tl, ps, part);
            } else {
                if (next < ntiles) {
                    const LineGeom<AXIS> ln(a, next * (uint32_t)W + (uint32_t)cl);
#pragma unroll
                    for (int s = 0; s < NST; ++s)
                        walk(ln, static_cast<const S*>(state(s)) + ln.base,
                             [&](int e, const S* p) { raw[s][e] = ld_raw<S, NT>(p); });
                    if constexpr (KROW) {
                        if (tid < N) kreg = krow_of(next)[tid];
                    }
                }
                round_trip(lg, line, tl, ps, [](int) {});
            }
            ++it;
        };
        // The first tile is peeled off the loop, so that the loop is entered, like
        // its back edge, with the next tile's loads followed by this tile's stores
        // outstanding: the wait for those loads (the memory counter covers loads
        // and stores in issue order) then leaves the stores in flight, where a
        // loop entered with the loads alone outstanding waits for everything.
        if (tile < ntiles) {
            one_tile(tile);
            for (tile += gridDim.x; tile < ntiles; tile += gridDim.x) one_tile(tile);
        }
    } else {
        const uint32_t line = blockIdx.x * (uint32_t)W + (uint32_t)cl;
        const LineGeom<AXIS> lg(a, line);
        // the state, and in the reverse sweep the adjoint state beside it
        S* ps[NST];
        ps[0] = reinterpret_cast<S*>(a.psi) + lg.base;
        if constexpr (NST == 2) ps[1] = reinterpret_cast<S*>(a.lam) + lg.base;
        S raw[NST][E];
#pragma unroll
        for (int s = 0; s < NST; ++s) walk(lg, ps[s], [&](int e, S* p) { raw[s][e] = ld_raw<S, NT>(p); });
        after_loads();
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int e = 0; e < E; ++e) v[s][e] = widen(raw[s][e]);
        round_trip(lg, line, blockIdx.x, ps, [](int) {});
    }
}

// Three-stage factorisations: n = R1 R2 R3 on T threads per line.
// The compile-time-width form when the block takes the pass's nominal width w.
template <class S, int AXIS, int R1, int R2, int R3, int T, int NST, int VK, bool NT, bool PERS>
AxisKernel pick_w(int w) {
    constexpr int WN = axis3_nominal_w(AXIS, R1 * R2 * R3, T, NST, !std::is_same<S, double2>::value);
    return w == WN ? k_axis3<S, AXIS, R1, R2, R3, T, NST, VK, NT, PERS, WN>
                   : k_axis3<S, AXIS, R1, R2, R3, T, NST, VK, NT, PERS, 0>;
}

template <class S, int AXIS, int NST, int VK, bool NT, bool PERS = false>
AxisKernel pick3(int n, int w, int* t) {
    switch (n) {
        case 96: *t = 8; return pick_w<S, AXIS, 12, 4, 2, 8, NST, VK, NT, PERS>(w);
        case 128: *t = 16; return pick_w<S, AXIS, 8, 4, 4, 16, NST, VK, NT, PERS>(w);
        case 256: *t = 32; return pick_w<S, AXIS, 8, 8, 4, 32, NST, VK, NT, PERS>(w);
        default: *t = 0; return nullptr;
    }
}

// Forward single-state passes: the x1 pass carries no potential factor, the
// y2 pass always carries it, x2 and y1 either.  Reverse dual-state passes: the
// x passes carry none, y1 (before its transform) and y2 (after) carry it.
// Persistent forms: the x1 and y1 passes without a potential factor.
template <class S, bool NT>
AxisKernel pick_axis3_nt(int axis, int n, int vk, int nst, bool pers, int w, int* t) {
    if (pers) {
        if (nst == 1 && vk == 0 && axis == AX_X1) return pick3<S, AX_X1, 1, 0, NT, true>(n, w, t);
        if (nst == 1 && vk == 0 && axis == AX_Y1) return pick3<S, AX_Y1, 1, 0, NT, true>(n, w, t);
        if (nst == 2 && vk == 0 && axis == AX_X1) return pick3<S, AX_X1, 2, 0, NT, true>(n, w, t);
        *t = 0;
        return nullptr;
    }
    if (nst == 2) {
        switch (axis) {
            case AX_X1:
                if (vk == 0) return pick3<S, AX_X1, 2, 0, NT>(n, w, t);
                break;
            case AX_X2:
                if (vk == 0) return pick3<S, AX_X2, 2, 0, NT>(n, w, t);
                break;
            case AX_Y1:
                if (vk == 1) return pick3<S, AX_Y1, 2, 1, NT>(n, w, t);
                if (vk == 2) return pick3<S, AX_Y1, 2, 2, NT>(n, w, t);
                break;
            case AX_Y2:
                if (vk == 1) return pick3<S, AX_Y2, 2, 1, NT>(n, w, t);
                if (vk == 2) return pick3<S, AX_Y2, 2, 2, NT>(n, w, t);
                break;
            default: break;
        }
        *t = 0;
        return nullptr;
    }
    switch (axis) {
        case AX_X1:
            if (vk == 0) return pick3<S, AX_X1, 1, 0, NT>(n, w, t);
            break;
        case AX_X2:
            if (vk == 0) return pick3<S, AX_X2, 1, 0, NT>(n, w, t);
            if (vk == 1) return pick3<S, AX_X2, 1, 1, NT>(n, w, t);
            if (vk == 2) return pick3<S, AX_X2, 1, 2, NT>(n, w, t);
            break;
        case AX_Y1:
            if (vk == 0) return pick3<S, AX_Y1, 1, 0, NT>(n, w, t);
            if (vk == 1) return pick3<S, AX_Y1, 1, 1, NT>(n, w, t);
            if (vk == 2) return pick3<S, AX_Y1, 1, 2, NT>(n, w, t);
            break;
        case AX_Y2:
            if (vk == 1) return pick3<S, AX_Y2, 1, 1, NT>(n, w, t);
            if (vk == 2) return pick3<S, AX_Y2, 1, 2, NT>(n, w, t);
            break;
        default: break;
    }
    *t = 0;
    return nullptr;
}

template <class S>
AxisKernel pick_axis3(int axis, int n, int vk, int nst, bool nt, bool pers, int w, int* t) {
    return nt ? pick_axis3_nt<S, true>(axis, n, vk, nst, pers, w, t) : pick_axis3_nt<S, false>(axis, n, vk, nst, pers, w, t);
}

}  // namespace dev
}  // namespace hom4d_impl
