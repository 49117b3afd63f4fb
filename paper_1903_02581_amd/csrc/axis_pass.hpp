// The per-axis pass kernel (template) and its device helpers; included by the
// translation units that instantiate it for one storage type and state count.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dft_regs.hpp"
#include "hom4d_internal.hpp"

namespace hom4d_impl {
namespace dev {
using namespace hom4d_dev;

// State loads and stores, widened to / narrowed from FP64.  NT marks them
// non-temporal (the nt bit of the global load/store): the passes over states
// several times the 256 MB Infinity Cache stream every element once, and
// keeping them out of the caches leaves room for the factor tables; smaller
// states keep the default policy, which lets one pass hit what the previous
// one wrote.
typedef double ntv_d2 __attribute__((ext_vector_type(2)));
typedef float ntv_f2 __attribute__((ext_vector_type(2)));
template <class S, bool NT = false>
__device__ __forceinline__ double2 ld(const S* p) {
    if constexpr (std::is_same<S, double2>::value) {
        if constexpr (NT) {
            const ntv_d2 r = __builtin_nontemporal_load(reinterpret_cast<const ntv_d2*>(p));
            return make_double2(r.x, r.y);
        } else {
            return *p;
        }
    } else {
        static_assert(std::is_same<S, float2>::value, "complex128 or complex64 storage");
        if constexpr (NT) {
            const ntv_f2 f = __builtin_nontemporal_load(reinterpret_cast<const ntv_f2*>(p));
            return make_double2((double)f.x, (double)f.y);
        } else {
            const float2 f = *p;
            return make_double2((double)f.x, (double)f.y);
        }
    }
}
template <class S, bool NT = false>
__device__ __forceinline__ void st(S* p, double2 v) {
    if constexpr (std::is_same<S, double2>::value) {
        if constexpr (NT) {
            ntv_d2 r;
            r.x = v.x;
            r.y = v.y;
            __builtin_nontemporal_store(r, reinterpret_cast<ntv_d2*>(p));
        } else {
            *p = v;
        }
    } else {
        if constexpr (NT) {
            ntv_f2 r;
            r.x = (float)v.x;
            r.y = (float)v.y;
            __builtin_nontemporal_store(r, reinterpret_cast<ntv_f2*>(p));
        } else {
            *p = make_float2((float)v.x, (float)v.y);
        }
    }
}

// State element as stored (complex128 or complex64), not widened: loads of a
// batch land here first, and the persistent passes' prefetch registers hold
// the next tile this way.
template <class S, bool NT>
__device__ __forceinline__ S ld_raw(const S* p) {
    if constexpr (NT) {
        if constexpr (std::is_same<S, double2>::value) {
            const ntv_d2 r = __builtin_nontemporal_load(reinterpret_cast<const ntv_d2*>(p));
            return make_double2(r.x, r.y);
        } else {
            const ntv_f2 r = __builtin_nontemporal_load(reinterpret_cast<const ntv_f2*>(p));
            return make_float2(r.x, r.y);
        }
    } else {
        return *p;
    }
}
__device__ __forceinline__ double2 widen(double2 v) { return v; }
__device__ __forceinline__ double2 widen(float2 v) { return make_double2((double)v.x, (double)v.y); }

// Element type of an LDS exchange of the state: complex64 with complex64
// storage (the exchange rounds like one more store of the state), complex128
// otherwise.  The arithmetic is FP64 either way.
template <class S>
struct Xchg {
    using T = double2;
    __device__ static __forceinline__ T put(double2 v) { return v; }
    __device__ static __forceinline__ double2 get(T v) { return v; }
};
template <>
struct Xchg<float2> {
    using T = float2;
    __device__ static __forceinline__ T put(double2 v) { return make_float2((float)v.x, (float)v.y); }
    __device__ static __forceinline__ double2 get(T v) { return make_double2((double)v.x, (double)v.y); }
};

__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// Im(conj(l) * p)
__device__ __forceinline__ double im_cl_p(double2 l, double2 p) { return fma(l.x, p.y, -l.y * p.x); }

// theta - 2 pi * rint(theta / 2 pi), 2 pi split in three parts (Cody & Waite);
// the first part has 9 significant bits, so q * c1 is exact for |q| < 2^44.
__device__ __forceinline__ double reduce_2pi(double th) {
    const double inv2pi = 0.15915494309189535;
    const double c1 = 6.28125;
    const double c2 = 0.001935307179586477;
    const double c3 = -1.0033115225336665e-19;
    const double q = rint(th * inv2pi);
    return fma(-q, c3, fma(-q, c2, fma(-q, c1, th)));
}

// Every load of a batch is issued before any of its values is used.  Left
// alone, the machine scheduler places each loaded value's first use right after
// its load, behind a wait for that load (s_waitcnt vmcnt(0)), so a wave keeps a
// single load in flight; this scheduling barrier keeps a batch's loads ahead of
// their uses, which then wait for the whole batch once.
__device__ __forceinline__ void after_loads() { __builtin_amdgcn_sched_barrier(0); }

// Apply use(e, load(e)) to the elements e = 0 .. E-1 in batches of G: the G
// loads of a batch are issued, then their G uses run.
template <int E, int G, class Load, class Use>
__device__ __forceinline__ void batched(Load load, Use use) {
#pragma unroll
    for (int b = 0; b < E; b += G) {
        decltype(load(0)) buf[G];
#pragma unroll
        for (int i = 0; i < G; ++i)
            if (b + i < E) buf[i] = load(b + i);
        after_loads();
#pragma unroll
        for (int i = 0; i < G; ++i)
            if (b + i < E) use(b + i, buf[i]);
    }
}

// Table entries / potential values one element's potential factor needs,
// loaded ahead of use (vload) and combined later (vcombine).  Table form
// (VK = 1, 3): p = a1(r1) (VK = 1 only), q = a1(r2), r = ac(r1 - r2); per-point
// form (VK = 2): p = (V(r1), V(r2)).
struct VLoad {
    double2 p, q, r;
};

template <int VK>
__device__ __forceinline__ VLoad vload(const PassArgs& a, int i1, int j1, int i2, int j2) {
    VLoad l;
    if constexpr (VK == 1 || VK == 3) {
        l.q = a.a1[i2 * a.ny + j2];
        if constexpr (VK == 1) l.p = a.a1[i1 * a.ny + j1];
        l.r = a.ac[(i1 - i2 + a.nx - 1) * (2 * a.ny - 1) + (j1 - j2 + a.ny - 1)];
    } else {
        l.p = make_double2(a.vtab[i1 * a.ny + j1], a.vtab[i2 * a.ny + j2]);
    }
    return l;
}

// exp(-i tau (V(r1) + V(r2) + V12(r1 - r2)) / hbar), or its conjugate, from the
// loaded entries.  VK = 1: product of the one-body and two-body factor tables;
// VK = 2: the FP64 angle evaluated here, reduced mod 2 pi, then sincos; VK = 3:
// as VK = 1 without the one-body factor of electron 1 (applied by the caller).
template <int VK, bool CONJ>
__device__ __forceinline__ double2 vcombine(const PassArgs& a, const VLoad& l, int i1, int j1, int i2, int j2) {
    double2 f;
    if constexpr (VK == 1 || VK == 3) {
        f = l.q;
        if constexpr (VK == 1) f = cmul(l.p, f);
        f = cmul(f, l.r);
        if constexpr (CONJ) f = conjd(f);
    } else {
        double v = l.p.x + l.p.y;
        if (a.ck != 0.0) {
            const double ddx = (double)(i1 - i2) * a.dx;
            const double ddy = (double)(j1 - j2) * a.dy;
            const double r2 = ddx * ddx + ddy * ddy;
            double vc = a.ck / sqrt(r2 + a.soft2);
            if (a.inv_screen > 0.0) vc *= exp(-sqrt(r2) * a.inv_screen);
            v += vc;
        }
        const double th = reduce_2pi(a.vscale * v);  // vscale carries the sign of tau
        double s, c;
        sincos(th, &s, &c);
        f = make_double2(c, -s);
    }
    return f;
}

// The same factor with its table entries loaded in place (the fused plane pass
// applies it element by element inside its LDS stages; there the batched form
// measured slower: 64x64 FP64 plane pass 104 -> 130 VGPRs, 127 -> 163 us).
template <int VK, bool CONJ>
__device__ __forceinline__ double2 vfactor(const PassArgs& a, int i1, int j1, int i2, int j2) {
    double2 f;
    if constexpr (VK == 1 || VK == 3) {
        f = a.a1[i2 * a.ny + j2];
        if constexpr (VK == 1) f = cmul(a.a1[i1 * a.ny + j1], f);
        f = cmul(f, a.ac[(i1 - i2 + a.nx - 1) * (2 * a.ny - 1) + (j1 - j2 + a.ny - 1)]);
        if constexpr (CONJ) f = conjd(f);
    } else {
        VLoad l;
        l.p = make_double2(a.vtab[i1 * a.ny + j1], a.vtab[i2 * a.ny + j2]);
        f = vcombine<VK, CONJ>(a, l, i1, j1, i2, j2);
    }
    return f;
}

// Elements per batch of potential-factor loads: 4 with three complex table
// entries per element (48 VGPRs in flight), 8 otherwise.
template <int VK>
constexpr int vbatch() { return VK == 1 ? 4 : 8; }

// Synchronisation after an LDS exchange of a line pass.  Lines along y2 put a
// line's T threads on consecutive lanes, so with T dividing 64 every wavefront
// owns whole lines: it only waits for its own LDS writes before reading (the
// memory clobber keeps the compiler from moving or forwarding LDS accesses
// across the wait).  On the other axes a line spans wavefronts.
template <int AXIS, int T>
__device__ __forceinline__ void line_sync() {
    if constexpr (AXIS == AX_Y2 && 64 % T == 0)
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    else
        __syncthreads();
}

// Sum over the block, valid in thread 0.  blockDim.x is a power of two.
__device__ inline double block_sum(double v, double* red) {
    const int tid = threadIdx.x;
    const int nb = blockDim.x;
    if (nb >= 64) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        double s = 0.0;
        if (tid == 0)
            for (int w = 0; w < (nb >> 6); ++w) s += red[w];
        return s;
    }
    __syncthreads();
    red[tid] = v;
    __syncthreads();
    for (int o = nb >> 1; o >= 1; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    return tid == 0 ? red[0] : 0.0;
}

// Coordinates (i1, j1, i2, j2) of element m of a line along AXIS.
template <int AXIS>
__device__ __forceinline__ void elem_coord(int i1, int j1, int i2, int j2, int m, int* c) {
    c[0] = i1;
    c[1] = j1;
    c[2] = i2;
    c[3] = j2;
    c[AXIS] = m;
}

// Position of line number `line` of a pass along AXIS in the [x1][y1][x2][y2]
// state: its fixed coordinates (the one along AXIS is left 0), the offset of its
// first element and the element stride.  Lines are numbered so that
// consecutive lines are adjacent in memory on the strided axes.
template <int AXIS>
struct LineGeom {
    int i1 = 0, j1 = 0, i2 = 0, j2 = 0;
    int64_t base, sN;
    __device__ __forceinline__ LineGeom(const PassArgs& a, uint32_t line) {
        const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny, nxy = nx * ny;
        if constexpr (AXIS == AX_X1) {
            const uint32_t o = a.dny.div(line);
            j1 = (int)a.dnx.div(o);
            i2 = (int)a.dnx.mod(o, (uint32_t)j1);
            j2 = (int)a.dny.mod(line, o);
            base = line;
            sN = (int64_t)ny * nxy;
        } else if constexpr (AXIS == AX_Y1) {
            i1 = (int)a.dnxy.div(line);
            const uint32_t c = a.dnxy.mod(line, (uint32_t)i1);
            i2 = (int)a.dny.div(c);
            j2 = (int)a.dny.mod(c, (uint32_t)i2);
            base = (int64_t)i1 * ny * nxy + c;
            sN = nxy;
        } else if constexpr (AXIS == AX_X2) {
            const uint32_t o = a.dny.div(line);
            i1 = (int)a.dny.div(o);
            j1 = (int)a.dny.mod(o, (uint32_t)i1);
            j2 = (int)a.dny.mod(line, o);
            base = (int64_t)o * nxy + j2;
            sN = ny;
        } else {
            const uint32_t o = a.dnx.div(line);
            i1 = (int)a.dny.div(o);
            j1 = (int)a.dny.mod(o, (uint32_t)i1);
            i2 = (int)a.dnx.mod(line, o);
            base = (int64_t)line * ny;
            sN = 1;
        }
    }
};

// VK: 0 = no potential factor on this pass, 1 = table form, 2 = per-point form.
template <class S, int AXIS, int N1, int N2, int T, int NST, int VK, bool NT>
__global__ void __launch_bounds__(256) k_axis(const PassArgs a) {
    constexpr int N = N1 * N2;
    constexpr int E = N / T;
    constexpr int JA = N2 / T;  // stage-A columns per thread
    constexpr int IB = N1 / T;  // stage-B rows per thread
    static_assert(N1 % T == 0 && N2 % T == 0, "t must divide both factors");
    // the reverse sweep (two states) applies every factor conjugated
    constexpr bool CONJ = NST == 2;
    // complex64 exchanges with complex64 storage, except on the x1 pass, which
    // measured slower with them (48x48: 27.7 -> 32.8 us)
    using X = Xchg<typename std::conditional<axis_xchg_c64(AXIS, true), S, double2>::type>;
    extern __shared__ double2 lds_raw[];
    typename X::T* lds = reinterpret_cast<typename X::T*>(lds_raw);

    const int W = a.W;
    const int tid = threadIdx.x;
    int t, cl;
    if constexpr (AXIS == AX_Y2) {
        t = tid % T;
        cl = tid / T;
    } else {
        cl = tid % W;
        t = tid / W;
    }
    // The forward y1 pass takes its blocks in reverse order: it follows the plane
    // pass, which writes the state in ascending order, so it starts on the planes
    // written last, which a state about the size of the Infinity Cache (64x64 FP64,
    // 268 MB) still holds there (steady 286-288 us per step against 288-296).
    const uint32_t blk = (AXIS == AX_Y1 && NST == 1) ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
    const uint32_t line = blk * (uint32_t)W + (uint32_t)cl;
    const LineGeom<AXIS> lg(a, line);
    const int i1 = lg.i1, j1 = lg.j1, i2 = lg.i2, j2 = lg.j2;
    const int64_t base = lg.base, sN = lg.sN;

    // twiddles (and, on y axes, the kinetic factor) staged in LDS after the exchange area
    constexpr bool KT_LDS = (AXIS == AX_Y1 || AXIS == AX_Y2);
    // On the y1 pass the block's lines share x1, so the one-body factor of
    // electron 1 along the line, exp(-i tau V(x1, y1) / hbar) for every y1, is one
    // table row: staged after the kinetic factor instead of read per element.
    constexpr bool A1_LDS = (AXIS == AX_Y1 && VK == 1);
    double2* TWL = reinterpret_cast<double2*>(reinterpret_cast<char*>(lds_raw) +
                                              axis_xchg_bytes(N2 > 1 ? N : 0, W, NST, sizeof(typename X::T) == 8));
    const int a1_row = A1_LDS ? (int)((blk * (uint32_t)W) / ((uint32_t)a.nx * (uint32_t)a.ny)) * a.ny : 0;
    for (int i = tid; i < (KT_LDS ? 2 * N : N) + (A1_LDS ? N : 0); i += T * W) {
        double2 v;
        if (i < N) {
            v = a.tw[i];
        } else if (i < 2 * N) {
            v = a.ktab[i - N];
            if constexpr (CONJ) v = conjd(v);
        } else {
            v = a.a1[a1_row + i - 2 * N];
        }
        TWL[i] = v;
    }
    __syncthreads();
    const double2* twl = TWL;
    double2 v[NST][E];  // the thread's elements of the state (and the adjoint state)
    // line position of the thread's element e = jj * N1 + n1
    auto pos = [&](int e) { return (e % N1) * N2 + t + T * (e / N1); };
    // the potential factor on the thread's elements, its table entries loaded in batches
    auto apply_potential = [&]() {
        constexpr int VKF = VK == 0 ? 1 : VK;
        if constexpr (A1_LDS) {
            const double2 f2 = a.a1[i2 * a.ny + j2];  // electron 2's factor: the same along the line
            batched<E, 8>(
                [&](int e) { return a.ac[(i1 - i2 + a.nx - 1) * (2 * a.ny - 1) + (pos(e) - j2 + a.ny - 1)]; },
                [&](int e, double2 fc) {
                    double2 f = cmul(cmul(twl[2 * N + pos(e)], f2), fc);
                    if constexpr (CONJ) f = conjd(f);
#pragma unroll
                    for (int s = 0; s < NST; ++s) v[s][e] = cmul(v[s][e], f);
                });
        } else {
            batched<E, vbatch<VKF>()>(
                [&](int e) {
                    int c[4];
                    elem_coord<AXIS>(i1, j1, i2, j2, pos(e), c);
                    return vload<VKF>(a, c[0], c[1], c[2], c[3]);
                },
                [&](int e, const VLoad& l) {
                    int c[4];
                    elem_coord<AXIS>(i1, j1, i2, j2, pos(e), c);
                    const double2 f = vcombine<VKF, CONJ>(a, l, c[0], c[1], c[2], c[3]);
#pragma unroll
                    for (int s = 0; s < NST; ++s) v[s][e] = cmul(v[s][e], f);
                });
        }
    };

    S* ps[NST];
    ps[0] = reinterpret_cast<S*>(a.psi) + base;
    if constexpr (NST == 2) ps[1] = reinterpret_cast<S*>(a.lam) + base;

    {
        S raw[NST][E];
#pragma unroll
        for (int jj = 0; jj < JA; ++jj) {
            const int jc = t + T * jj;
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) {
                const int64_t off = (int64_t)(n1 * N2 + jc) * sN;
#pragma unroll
                for (int s = 0; s < NST; ++s) raw[s][jj * N1 + n1] = ld_raw<S, NT>(ps[s] + off);
            }
        }
        after_loads();
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int e = 0; e < E; ++e) v[s][e] = widen(raw[s][e]);
    }

    double gm_acc = 0.0;  // marginal accumulator of this thread
    double gb_acc = 0.0;  // dL/dB accumulator of this thread
    if constexpr (NST == 2) {
        if (a.gflags & G_MIN) {
#pragma unroll
            for (int e = 0; e < E; ++e) gm_acc += im_cl_p(v[1][e], v[0][e]);
        }
    }

    if (VK != 0 && a.vmode == 1) apply_potential();

    // ---- forward transform, stage A: DFT_n1 over n1 for each of the thread's columns
#pragma unroll
    for (int s = 0; s < NST; ++s) {
#pragma unroll
        for (int jj = 0; jj < JA; ++jj) {
            dft<N1, -1>(&v[s][jj * N1]);
            if constexpr (N2 > 1) {
                const int jc = t + T * jj;
#pragma unroll
                for (int k1 = 1; k1 < N1; ++k1) v[s][jj * N1 + k1] = cmul(v[s][jj * N1 + k1], twl[(jc * k1) % N]);
            }
        }
    }

    const int LS = W + 1;  // padded LDS row (complex elements) for one position across W lines
    if constexpr (N2 > 1) {
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int jj = 0; jj < JA; ++jj)
#pragma unroll
                for (int k1 = 0; k1 < N1; ++k1)
                    lds[(s * N + k1 * N2 + t + T * jj) * LS + cl] = X::put(v[s][jj * N1 + k1]);
        line_sync<AXIS, T>();
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int ii = 0; ii < IB; ++ii)
#pragma unroll
                for (int j = 0; j < N2; ++j) v[s][ii * N2 + j] = X::get(lds[(s * N + (t + T * ii) * N2 + j) * LS + cl]);
        // stage B: DFT_n2 over the columns; element (ii, k2) is wave number k1 + n1 * k2
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int ii = 0; ii < IB; ++ii) dft<N2, -1>(&v[s][ii * N2]);
    }

    // ---- reciprocal space: gradient contribution and the kinetic phase
    // x kinetic factor table: y-major [y][k] on the x1 pass (all lanes of a block share y1,
    // each thread's k values are contiguous), k-major [k][y] on the x2 pass (neighbouring
    // lanes hold neighbouring y2 at the same k)
    const int yrow = (AXIS == AX_X1) ? j1 : ((AXIS == AX_X2) ? j2 : 0);
    const double2* kt = a.ktab + (AXIS == AX_X1 ? (int64_t)yrow * N : (int64_t)yrow);
    const int64_t kstride = AXIS == AX_X1 ? 1 : a.ny;
    if constexpr (NST == 2 && (AXIS == AX_X1 || AXIS == AX_X2)) {
        if (a.gflags & G_GB) {
            const double yv = a.y0 + a.ystep * yrow;
            const double shift = yv * a.b_eoh;
#pragma unroll
            for (int ii = 0; ii < IB; ++ii)
#pragma unroll
                for (int k2 = 0; k2 < N2; ++k2) {
                    const int k = t + T * ii + N1 * k2;
                    const int m = (k < (N + 1) / 2) ? k : k - N;
                    const double dth = a.db_coef * (a.kstep * m - shift) * yv;
                    gb_acc += dth * im_cl_p(v[1][ii * N2 + k2], v[0][ii * N2 + k2]);
                }
        }
    }
    // element e = ii * N2 + k2 holds wave number t + T * ii + N1 * k2; on the x axes
    // the kinetic factors come from the L2-resident table, loaded in one batch
    auto wave_number = [&](int e) { return t + T * (e / N2) + N1 * (e % N2); };
    if constexpr (KT_LDS) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double2 f = twl[N + wave_number(e)];
#pragma unroll
            for (int s = 0; s < NST; ++s) v[s][e] = cmul(v[s][e], f);
        }
    } else {
        batched<E, 8>([&](int e) { return kt[wave_number(e) * kstride]; },
                      [&](int e, double2 f) {
                          if constexpr (CONJ) f = conjd(f);
#pragma unroll
                          for (int s = 0; s < NST; ++s) v[s][e] = cmul(v[s][e], f);
                      });
    }

    // ---- inverse transform: the forward network transposed
    if constexpr (N2 > 1) {
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int ii = 0; ii < IB; ++ii) dft<N2, 1>(&v[s][ii * N2]);
        // each thread writes back exactly the positions it read for stage B: no barrier needed
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int ii = 0; ii < IB; ++ii)
#pragma unroll
                for (int j = 0; j < N2; ++j) lds[(s * N + (t + T * ii) * N2 + j) * LS + cl] = X::put(v[s][ii * N2 + j]);
        line_sync<AXIS, T>();
#pragma unroll
        for (int s = 0; s < NST; ++s)
#pragma unroll
            for (int jj = 0; jj < JA; ++jj)
#pragma unroll
                for (int k1 = 0; k1 < N1; ++k1)
                    v[s][jj * N1 + k1] = X::get(lds[(s * N + k1 * N2 + t + T * jj) * LS + cl]);
    }
#pragma unroll
    for (int s = 0; s < NST; ++s) {
#pragma unroll
        for (int jj = 0; jj < JA; ++jj) {
            if constexpr (N2 > 1) {
                const int jc = t + T * jj;
#pragma unroll
                for (int k1 = 1; k1 < N1; ++k1) v[s][jj * N1 + k1] = cmulc(v[s][jj * N1 + k1], twl[(jc * k1) % N]);
            }
            dft<N1, 1>(&v[s][jj * N1]);
        }
    }

    if (VK != 0 && a.vmode == 2) apply_potential();

    if constexpr (NST == 2) {
        if (a.gflags & G_MOUT) {
#pragma unroll
            for (int e = 0; e < E; ++e) gm_acc += im_cl_p(v[1][e], v[0][e]);
        }
    }

#pragma unroll
    for (int jj = 0; jj < JA; ++jj) {
        const int jc = t + T * jj;
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) {
            const int64_t off = (int64_t)(n1 * N2 + jc) * sN;
#pragma unroll
            for (int s = 0; s < NST; ++s) st<S, NT>(ps[s] + off, v[s][jj * N1 + n1]);
        }
    }

    if constexpr (NST == 2) {
        double* red = reinterpret_cast<double*>(lds_raw);
        if (a.gflags & G_GB) {
            const double s = block_sum(gb_acc, red);
            if (tid == 0) a.gb_part[blockIdx.x] += s;
        }
        if (a.gflags & (G_MIN | G_MOUT)) {
            if constexpr (AXIS == AX_X1 || AXIS == AX_Y1) {
                // one marginal slot per line: sum the t threads of the line in fixed order
                __syncthreads();
                red[t * W + cl] = gm_acc;
                __syncthreads();
                if (t == 0) {
                    double s = 0.0;
                    for (int q = 0; q < T; ++q) s += red[q * W + cl];
                    a.marg_part[line] += s;
                }
            } else {
                // the block's lines share r1: one slot per block
                const double s = block_sum(gm_acc, red);
                if (tid == 0) a.marg_part[blockIdx.x] += s;
            }
        }
    }
}

// Table form of the potential factor along one line (VK = 1 of vfactor, same
// products in the same order): element m of a line along AXIS reads a1 at r1(m),
// a1 at r2(m) and ac at r1(m) - r2(m), each index affine in m.  The line's
// fixed coordinates and the thread's first element m0 give three base pointers
// once; element m0 + dm then adds dm times a per-axis step, a uniform product
// when dm is a compile-time offset.
template <int AXIS>
struct LineTables {
    const double2* p1;
    const double2* p2;
    const double2* pc;
    int64_t step;  // index step of the varying electron's a1 entry (ny on x axes, 1 on y axes)
    int64_t cstep; // index step of ac (+-(2 ny - 1) on x axes, +-1 on y axes)
    __device__ __forceinline__ LineTables(const PassArgs& a, const LineGeom<AXIS>& lg, int m0) {
        int c[4];
        elem_coord<AXIS>(lg.i1, lg.j1, lg.i2, lg.j2, m0, c);
        const int64_t ny = a.ny, cy = 2 * (int64_t)a.ny - 1;
        p1 = a.a1 + (c[0] * ny + c[1]);
        p2 = a.a1 + (c[2] * ny + c[3]);
        pc = a.ac + ((int64_t)(c[0] - c[2] + a.nx - 1) * cy + (c[1] - c[3] + a.ny - 1));
        step = (AXIS == AX_X1 || AXIS == AX_X2) ? ny : 1;
        cstep = (AXIS == AX_X1) ? cy : (AXIS == AX_X2) ? -cy : (AXIS == AX_Y1) ? 1 : -1;
    }
    // the entry fixed along the line: the one-body factor of the electron the
    // line does not move
    __device__ __forceinline__ double2 fixed() const {
        return (AXIS == AX_X1 || AXIS == AX_Y1) ? p2[0] : p1[0];
    }
    // the entries of element m0 + dm: the moving electron's one-body factor (q)
    // and the two-body factor (r)
    __device__ __forceinline__ VLoad load(int dm) const {
        VLoad l;
        l.q = (AXIS == AX_X1 || AXIS == AX_Y1) ? p1[dm * step] : p2[dm * step];
        l.r = pc[dm * cstep];
        return l;
    }
    template <bool CONJ>
    __device__ __forceinline__ double2 combine(double2 f0, const VLoad& l) const {
        double2 f;
        if constexpr (AXIS == AX_X1 || AXIS == AX_Y1)
            f = cmul(l.q, f0);
        else
            f = cmul(f0, l.q);
        f = cmul(f, l.r);
        return CONJ ? conjd(f) : f;
    }
};

using AxisKernel = void (*)(const PassArgs);

// Line lengths of the two-stage kernel (96, 128 and 256 take the three-stage one).
template <class S, int AXIS, int NST, int VK, bool NT>
AxisKernel pick(int n, int* t) {
    switch (n) {
        case 4: *t = 1; return k_axis<S, AXIS, 4, 1, 1, NST, VK, NT>;
        case 6: *t = 1; return k_axis<S, AXIS, 6, 1, 1, NST, VK, NT>;
        case 8: *t = 1; return k_axis<S, AXIS, 8, 1, 1, NST, VK, NT>;
        case 12: *t = 1; return k_axis<S, AXIS, 12, 1, 1, NST, VK, NT>;
        case 16: *t = 4; return k_axis<S, AXIS, 4, 4, 4, NST, VK, NT>;
        case 24: *t = 2; return k_axis<S, AXIS, 12, 2, 2, NST, VK, NT>;
        case 32: *t = 4; return k_axis<S, AXIS, 8, 4, 4, NST, VK, NT>;
        case 48: *t = 4; return k_axis<S, AXIS, 12, 4, 4, NST, VK, NT>;
        case 64: *t = 8; return k_axis<S, AXIS, 8, 8, 8, NST, VK, NT>;
        default: *t = 0; return nullptr;
    }
}

// Variants built: vk = 0 (no potential factor), 1 (table form), 2 (per-point
// form).  The x1 pass never carries the factor; the reverse (two-state) sweep
// carries it on the y passes only; the forward plans put it on x2, y1 or y2.
template <class S, int AXIS, int NST, bool NT>
AxisKernel pick_vk(int n, int vk, int* t) {
    constexpr bool with_v = (NST == 1) ? (AXIS != AX_X1) : (AXIS == AX_Y1 || AXIS == AX_Y2);
    constexpr bool without_v = (AXIS == AX_X1 || AXIS == AX_X2 || (NST == 1 && AXIS == AX_Y1));
    if constexpr (with_v) {
        if (vk == 1) return pick<S, AXIS, NST, 1, NT>(n, t);
        if (vk == 2) return pick<S, AXIS, NST, 2, NT>(n, t);
    }
    if constexpr (without_v) {
        if (vk == 0) return pick<S, AXIS, NST, 0, NT>(n, t);
    }
    *t = 0;
    return nullptr;
}

template <class S, int NST, bool NT>
AxisKernel pick_axis_nt(int axis, int n, int vk, int* t) {
    switch (axis) {
        case AX_X1: return pick_vk<S, AX_X1, NST, NT>(n, vk, t);
        case AX_X2: return pick_vk<S, AX_X2, NST, NT>(n, vk, t);
        case AX_Y1: return pick_vk<S, AX_Y1, NST, NT>(n, vk, t);
        case AX_Y2: return pick_vk<S, AX_Y2, NST, NT>(n, vk, t);
        default: *t = 0; return nullptr;
    }
}

template <class S, int NST>
AxisKernel pick_axis(int axis, int n, int vk, bool nt, int* t) {
    return nt ? pick_axis_nt<S, NST, true>(axis, n, vk, t) : pick_axis_nt<S, NST, false>(axis, n, vk, t);
}

}  // namespace dev
}  // namespace hom4d_impl
