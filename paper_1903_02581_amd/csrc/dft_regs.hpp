// Small discrete Fourier transforms held entirely in registers (FP64).
//
// X[k] = sum_n v[n] w^(n k), w = exp(DIR * 2 pi i / R); DIR = -1 is the forward
// transform (exp(-i k x) convention), DIR = +1 the unnormalised inverse.
// Sizes R in {1, 2, 3, 4, 6, 8, 12, 16, 24}; 8 is two 4-point transforms and a
// radix-2 step; the other composite sizes use one
// Cooley-Tukey split R = A * B (A = 4, 2 or 3) with compile-time twiddles, so
// after unrolling every index and constant is known to the compiler.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace hom4d_dev {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i * DIR * a
template <int DIR>
__device__ __forceinline__ double2 imul(double2 a) {
    return DIR < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// cos(2 pi j / 48) for j = 0..12, correctly rounded; the other quadrants by symmetry.
struct C48 {
    static constexpr double q[13] = {1.0,
                                     0.9914448613738104,
                                     0.9659258262890683,
                                     0.9238795325112867,
                                     0.8660254037844386,
                                     0.7933533402912352,
                                     0.7071067811865476,
                                     0.6087614290087207,
                                     0.5,
                                     0.3826834323650898,
                                     0.25881904510252074,
                                     0.1305261922200516,
                                     0.0};
    static constexpr int md(int j) { return ((j % 48) + 48) % 48; }
    static constexpr double cosj(int j) {
        return md(j) <= 12 ? q[md(j)]
             : md(j) <= 24 ? -q[24 - md(j)]
             : md(j) <= 36 ? -q[md(j) - 24]
                           : q[48 - md(j)];
    }
    static constexpr double sinj(int j) { return cosj(j - 12); }
};

// v * exp(DIR * 2 pi i * M / R), M and R compile-time, R | 48.
template <int R, int M, int DIR>
__device__ __forceinline__ double2 twiddle(double2 v) {
    static_assert(48 % R == 0, "twiddle base must divide 48");
    constexpr int j = C48::md(M * (48 / R));
    if constexpr (j == 0) {
        return v;
    } else if constexpr (j == 24) {
        return make_double2(-v.x, -v.y);
    } else if constexpr (j == 12) {
        return imul<DIR>(v);
    } else if constexpr (j == 36) {
        return imul<-DIR>(v);
    } else {
        constexpr double c = C48::cosj(j);
        constexpr double s = DIR * C48::sinj(j);
        return make_double2(fma(v.x, c, -v.y * s), fma(v.x, s, v.y * c));
    }
}

template <int I, int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        sfor<I + 1, N>(f);
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(double2* v);

template <int DIR>
__device__ __forceinline__ void dft2(double2* v) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int DIR>
__device__ __forceinline__ void dft3(double2* v) {
    constexpr double h = 0.8660254037844386;  // sin(2 pi / 3)
    const double2 a = v[0];
    const double2 s = cadd(v[1], v[2]);
    const double2 d = csub(v[1], v[2]);
    const double2 m = make_double2(fma(-0.5, s.x, a.x), fma(-0.5, s.y, a.y));
    // the scaling by h folds into the output additions
    const double2 t = imul<DIR>(d);
    v[0] = cadd(a, s);
    v[1] = make_double2(fma(h, t.x, m.x), fma(h, t.y, m.y));
    v[2] = make_double2(fma(-h, t.x, m.x), fma(-h, t.y, m.y));
}

template <int DIR>
__device__ __forceinline__ void dft4(double2* v) {
    const double2 s0 = cadd(v[0], v[2]), d0 = csub(v[0], v[2]);
    const double2 s1 = cadd(v[1], v[3]), d1 = csub(v[1], v[3]);
    const double2 id1 = imul<DIR>(d1);
    v[0] = cadd(s0, s1);
    v[2] = csub(s0, s1);
    v[1] = cadd(d0, id1);
    v[3] = csub(d0, id1);
}

// 8 points from the 4-point transforms E, O of the even and odd elements:
// X[k] = E[k] + w^k O[k], X[k + 4] = E[k] - w^k O[k].  The odd multiples of 45
// degrees, w^1 = c (1 + DIR i) and w^3 = -c (1 - DIR i) with c = cos(pi / 4), take
// two additions each, and their scaling by c folds into the fused multiply-adds
// of the output pair (52 instead of 56 FP64 operations).
template <int DIR>
__device__ __forceinline__ void dft8(double2* v) {
    constexpr double c = 0.7071067811865476;
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    const double2 t2 = imul<DIR>(o[2]);
    v[2] = cadd(e[2], t2);
    v[6] = csub(e[2], t2);
    // w^1 (a + i b) = c (a - DIR b + i (b + DIR a))
    const double r1 = DIR < 0 ? o[1].x + o[1].y : o[1].x - o[1].y;
    const double i1 = DIR < 0 ? o[1].y - o[1].x : o[1].y + o[1].x;
    v[1] = make_double2(fma(c, r1, e[1].x), fma(c, i1, e[1].y));
    v[5] = make_double2(fma(-c, r1, e[1].x), fma(-c, i1, e[1].y));
    // w^3 (a + i b) = -c (a + DIR b + i (b - DIR a))
    const double r3 = DIR < 0 ? o[3].x - o[3].y : o[3].x + o[3].y;
    const double i3 = DIR < 0 ? o[3].y + o[3].x : o[3].y - o[3].x;
    v[3] = make_double2(fma(-c, r3, e[3].x), fma(-c, i3, e[3].y));
    v[7] = make_double2(fma(c, r3, e[3].x), fma(c, i3, e[3].y));
}

template <int R, int DIR>
__device__ __forceinline__ void dft(double2* v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        dft2<DIR>(v);
    } else if constexpr (R == 3) {
        dft3<DIR>(v);
    } else if constexpr (R == 4) {
        dft4<DIR>(v);
    } else if constexpr (R == 8) {
        dft8<DIR>(v);
    } else {
        // n = B * na + nb, k = ka + A * kb:
        //   u[nb][ka] = DFT_A over na of v[B na + nb], times w_R^(nb ka);
        //   X[ka + A kb] = DFT_B over nb of u[nb][ka].
        constexpr int A = (R % 4 == 0) ? 4 : ((R % 2 == 0) ? 2 : 3);
        constexpr int B = R / A;
        double2 u[R];
        sfor<0, B>([&](auto nbc) {
            constexpr int nb = decltype(nbc)::value;
            double2 tmp[A];
#pragma unroll
            for (int na = 0; na < A; ++na) tmp[na] = v[B * na + nb];
            dft<A, DIR>(tmp);
            sfor<0, A>([&](auto kac) {
                constexpr int ka = decltype(kac)::value;
                u[nb * A + ka] = twiddle<R, nb * ka, DIR>(tmp[ka]);
            });
        });
#pragma unroll
        for (int ka = 0; ka < A; ++ka) {
            double2 tmp[B];
#pragma unroll
            for (int nb = 0; nb < B; ++nb) tmp[nb] = u[nb * A + ka];
            dft<B, DIR>(tmp);
#pragma unroll
            for (int kb = 0; kb < B; ++kb) v[ka + A * kb] = tmp[kb];
        }
    }
}

}  // namespace hom4d_dev
