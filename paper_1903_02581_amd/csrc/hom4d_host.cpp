// Host side of the C ABI declared in include/hom4d.h: argument validation,
// FP64 phase/twiddle tables, the step driver, observables, entanglement and
// the reverse (adjoint) sweep.
//
// Method: arXiv 1903.02581, Sec. II.C Eq. (evoloperat) and Appendix A (split-
// step Fourier propagation of two electrons), Eq. (coulomb) and
// Eq. (screenedCoulomb) (two-body term), Eq. (p_bunching) (region
// probabilities), Eq. (reduced_density) (spatial entanglement).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hom4d.h"
#include "hom4d_internal.hpp"

using namespace hom4d_impl;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(HOM4D_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                \
    } while (0)

// CODATA 2018 SI values.
constexpr double kHbarSI = 1.054571817e-34;   // J s
constexpr double kQeSI = 1.602176634e-19;     // C
constexpr double kMeSI = 9.1093837015e-31;    // kg
constexpr double kEps0SI = 8.8541878128e-12;  // F/m
constexpr long double kPiL = 3.141592653589793238462643383279502884L;

struct Units {
    double hbar;    // meV fs
    double kappa;   // hbar^2 / 2m*, meV nm^2
    double kc;      // e^2 / 4 pi eps0 eps_r, meV nm
    double eoh;     // e / hbar, 1/(T nm^2)
};

Units units_for(const hom4d_cfg& c) {
    Units u;
    u.hbar = kHbarSI / kQeSI * 1e3 * 1e15;
    u.kappa = kHbarSI * kHbarSI / (2.0 * c.mstar_rel * kMeSI) / kQeSI * 1e3 * 1e18;
    u.kc = kQeSI * kQeSI / (4.0 * (double)kPiL * kEps0SI * c.eps_r) / kQeSI * 1e3 * 1e9;
    u.eoh = kQeSI / kHbarSI * 1e-18;
    return u;
}

// theta - 2 pi rint(theta / 2 pi) with a three-part 2 pi (Cody & Waite).
double reduce_2pi(double th) {
    const double c1 = 6.28125, c2 = 0.001935307179586477, c3 = -1.0033115225336665e-19;
    const double q = std::rint(th * 0.15915494309189535);
    return std::fma(-q, c3, std::fma(-q, c2, std::fma(-q, c1, th)));
}

// exp(-i theta) * scale, angle reduced first
void phase(double th, double scale, double* out) {
    const double r = reduce_2pi(th);
    out[0] = std::cos(r) * scale;
    out[1] = -std::sin(r) * scale;
}

bool supported_n(int n) {
    FftShape s;
    return fft_shape(n, &s);
}

int validate(const hom4d_cfg* c) {
    if (!c) return fail(HOM4D_EINVAL, "cfg is NULL");
    if (!supported_n(c->nx) || !supported_n(c->ny))
        return fail(HOM4D_EINVAL, "nx=%d ny=%d: each must be one of 4 6 8 12 16 24 32 48 64 96 128 256", c->nx,
                    c->ny);
    if (c->precision != HOM4D_FP64 && c->precision != HOM4D_MIXED)
        return fail(HOM4D_EINVAL, "precision=%d: use HOM4D_FP64 or HOM4D_MIXED", c->precision);
    if (c->coulomb_mode != HOM4D_COULOMB_TABLE && c->coulomb_mode != HOM4D_COULOMB_DIRECT)
        return fail(HOM4D_EINVAL, "coulomb_mode=%d", c->coulomb_mode);
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(c->lx_nm) || !pos(c->ly_nm)) return fail(HOM4D_EINVAL, "box lengths must be positive");
    if (!pos(c->mstar_rel) || !pos(c->eps_r)) return fail(HOM4D_EINVAL, "m* and eps_r must be positive");
    if (!pos(c->dt_fs)) return fail(HOM4D_EINVAL, "dt must be positive");
    if (!std::isfinite(c->b_tesla)) return fail(HOM4D_EINVAL, "B must be finite");
    if (!std::isfinite(c->coulomb_c)) return fail(HOM4D_EINVAL, "coulomb_c must be finite");
    if (c->coulomb_c != 0.0 && !pos(c->soft_nm))
        return fail(HOM4D_EINVAL, "soft_nm must be positive when the Coulomb term is on");
    if (!(std::isfinite(c->screen_nm) && c->screen_nm >= 0.0)) return fail(HOM4D_EINVAL, "screen_nm must be >= 0");
    const double pts = (double)c->nx * c->ny * (double)c->nx * c->ny;
    if (pts > 4.3e9) return fail(HOM4D_EINVAL, "state too large");
    return HOM4D_OK;
}

struct AxisPlan {
    int n, t, W;
    int64_t nlines;
    size_t lds;
    bool pers;  // persistent three-stage pass (prefetches its next tile)
};

int64_t ilog2_pow2_divisor(int64_t v) {  // largest power of two dividing v
    return v & (-v);
}

AxisPlan plan_axis(int axis, int nx, int ny, int nst, bool grad, bool mixed) {
    AxisPlan p{};
    p.n = (axis == AX_X1 || axis == AX_X2) ? nx : ny;
    FftShape sh;
    fft_shape(p.n, &sh);
    p.t = sh.t;
    const int64_t nxy = (int64_t)nx * ny;
    p.nlines = nxy * nxy / p.n;
    const int t3 = axis3_threads(p.n, nst);
    if (t3 > 0) {
        // three-stage kernel: exchange area of n (W + 1) entries plus 2n staged
        // factors.  n = 128: 16 lines (256 threads) within 48 KB, so that three
        // or more blocks share a CU; n = 96 and 256 measured faster with wider
        // blocks: 32 lines (256 threads) and 16 lines (512 threads) within 80 KB
        // (in complex128 entries).  The complex64 x1 pass at n = 256 takes 32
        // lines (1024 threads; complex64 entries, within 80 KB): 7.12 -> 6.70 ms
        // at 256 x 128, while the x2 pass measured slower that way (6.72 ->
        // 7.97 ms).  The reverse sweep's
        // dual-state blocks take two exchange areas within 80 KB, counted in
        // the storage's entry size.
        p.t = t3;
        // The complex64 x2 pass at n = 128 takes 32 lines as well (512 threads,
        // complex64 entries within 80 KB): x2+V 842 -> 812 us at 128 x 96, 317 ->
        // 310 us at 128 x 64 (the one-tile x1 pass measured slower that way, 581
        // -> 647); so do the persistent y1 and x1 passes, with their addresses
        // kept in registers and the next tile's loads issued in parts (256 x 128
        // y1: 4.28 -> 3.83 ms; 128 x 96 x1: 0.559 -> 0.526 ms).
        int64_t w = axis3_nominal_w(axis, p.n, t3, nst, mixed);
        w = std::min<int64_t>(w, ilog2_pow2_divisor(p.nlines));
        if (axis == AX_X2) w = std::min<int64_t>(w, ilog2_pow2_divisor(ny));
        if (axis == AX_Y2 && grad) w = std::min<int64_t>(w, ilog2_pow2_divisor(nx));
        p.W = (int)std::max<int64_t>(w, 1);
        // persistent form on the complex64 x1 and y1 passes of 128- and 256-point
        // lines (256x128: x1 6.07 -> 5.36 ms, y1 4.46 -> 4.20 ms); the other
        // passes, FP64 and 96-point lines measured slower that way.  The x1 form
        // stages each tile's kinetic row, so a tile's lines share y1 and the
        // block's threads cover a row.
        // The reverse sweep's two-state x1 pass of 256-point lines (one 512-thread
        // block per CU at its 143 registers, so none out of phase to hide its
        // loads) takes the persistent form too: 256 x 128 reverse sweep 0.946 ->
        // 0.880 s over 20 recorded steps, gradients unchanged to rounding.
        p.pers = mixed && p.n >= 128 && (axis == AX_X1 || axis == AX_Y1) && (nst == 1 || (axis == AX_X1 && p.n == 256));
        if (p.pers && axis == AX_X1 && (nxy % p.W != 0 || (int64_t)p.t * p.W < p.n)) p.pers = false;
        p.lds = axis3_pass_lds_bytes(axis, p.n, p.W, nst, mixed, p.pers);
        return p;
    }
    int64_t w = 256 / sh.t;
    if (sh.n2 > 1) {
        // widths from an LDS budget counted in complex128 exchange entries: 64 KB
        // for complex128 storage (W = 16 lines already gives 256-byte runs), 80 KB
        // for complex64 (W = 32 on n = 128), whose blocks then take half of it
        // since they exchange complex64
        const int64_t budget = mixed ? 81920 : 65536;
        const int64_t cap = (budget - 3 * p.n * 16) / ((int64_t)nst * p.n * 16) - 1;
        while (w > cap) w >>= 1;
    }
    w = std::min<int64_t>(w, ilog2_pow2_divisor(p.nlines));
    if (axis == AX_X2) w = std::min<int64_t>(w, ilog2_pow2_divisor(ny));
    if (axis == AX_Y2 && grad) w = std::min<int64_t>(w, ilog2_pow2_divisor(nx));
    if (axis == AX_Y1) w = std::min<int64_t>(w, ilog2_pow2_divisor(nxy));  // a block's lines share x1
    if (w < 1) w = 1;
    p.W = (int)w;
    // exchange area, then the staged twiddles, kinetic factor and (y1) one-body
    // factor row (3n entries); the dual-state reduction scratch reuses the start
    // of the allocation at the end
    const size_t ex = axis_xchg_bytes(sh.n2 > 1 ? p.n : 0, p.W, nst, axis_xchg_c64(axis, mixed));
    const size_t red = nst == 2 ? (size_t)sh.t * p.W * sizeof(double) : 0;
    p.lds = std::max(ex + (size_t)3 * p.n * sizeof(double2), red);
    return p;
}

bool env_sync_check() {
    const char* e = std::getenv("HOM4D_SYNC_CHECK");
    return e && e[0] == '1';
}

}  // namespace

struct hom4d {
    hom4d_cfg cfg;
    Units u;
    hipStream_t stream = nullptr;
    int device = 0;
    bool mixed = false;
    bool sync_check = false;
    int nxy = 0;
    int64_t npts = 0;
    size_t state_bytes = 0;
    // device tables (FP64)
    double2* tw_x = nullptr;     // [nx]
    double2* tw_y = nullptr;     // [ny]
    double2* kx_half = nullptr;  // [ny][nx] (y-major)  exp(-i theta_x(dt/2)) / nx
    double2* kx_full = nullptr;  // [ny][nx] (y-major)  exp(-i theta_x(dt)) / nx
    double2* kxt_half = nullptr; // the same two tables k-major, [nx][ny]
    double2* kxt_full = nullptr;
    double2* ky_full = nullptr;  // [ny]      exp(-i theta_y(dt)) / ny
    double2* a1_half = nullptr;  // [nx*ny]   exp(-i (dt/2) V / hbar)
    double2* ac_half = nullptr;  // [(2nx-1)(2ny-1)]
    double* v_dev = nullptr;     // [nx*ny] meV
    double* w_dev = nullptr;     // [nx*ny] region weights
    double* red_part = nullptr;  // reduction partials
    double* red_out = nullptr;   // 8 doubles
    double* host_out = nullptr;  // pinned, 8 doubles
    int red_blocks = 0;
    // slices
    int32_t* ix_dev = nullptr;   // 512 ints
    double2* slice_dev = nullptr;// 256*256
    double2* orb_dev = nullptr;  // 2 * nx*ny
    // state
    void* psi = nullptr;
    int64_t step = 0;
    bool have_v = false;
    uint64_t v_hash = 0;         // FNV-1a of the last potential table (0: none)
    double norm_tol = 1e-6;
    int pass_plan = 0;           // 0: fused plane pass where built, 1: per-axis passes only
    bool plane_built = false;    // a fused plane kernel exists for (nx, ny, precision)
    // gradient recording
    bool rec = false;
    int ckpt_every = 0;
    char* pool = nullptr;
    size_t pool_bytes = 0;
    int64_t rec_steps = 0;
    double* g_buf = nullptr;     // all gradient partials
    size_t g_len = 0;
    // pass timing (measurement): an event pair around every pass kernel launch
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pool of 2 * kEvPairs events, created at the first timed launch
    std::vector<int> ev_kind;    // pass kind of each pending pair (0..4)
    double ev_ms[5] = {};        // folded sums per kind
    int64_t ev_n[5] = {};
};

namespace {

void free_events(hom4d* h) {
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    h->ev.clear();
    h->ev_kind.clear();
}

constexpr size_t kEvPairs = 4096;

// Wait for the pending event pairs and add their times to the per-kind sums;
// the events are then free for reuse.
hipError_t fold_events(hom4d* h) {
    if (h->ev_kind.empty()) return hipSuccess;
    hipError_t err = hipStreamSynchronize(h->stream);
    if (err != hipSuccess) return err;
    for (size_t i = 0; i < h->ev_kind.size(); ++i) {
        float t = 0.0f;
        if ((err = hipEventElapsedTime(&t, h->ev[2 * i], h->ev[2 * i + 1])) != hipSuccess) return err;
        h->ev_ms[h->ev_kind[i]] += t;
        h->ev_n[h->ev_kind[i]] += 1;
    }
    h->ev_kind.clear();
    return hipSuccess;
}

// Launch one pass kernel; while timing is on, between an event pair of its own.
// kind: 0 x1, 1 y1, 2 x2, 3 y2 (the axis), 4 the fused plane pass.  The pool
// holds kEvPairs pairs; when they are all pending the stream is synchronised
// and their times folded into the sums.
template <class F>
hipError_t timed_launch(hom4d* h, int kind, F&& launch) {
    if (!h->timing) return launch();
    hipError_t err;
    while (h->ev.size() < 2 * kEvPairs) {
        hipEvent_t e;
        if ((err = hipEventCreate(&e)) != hipSuccess) return err;
        h->ev.push_back(e);
    }
    if (h->ev_kind.size() == kEvPairs && (err = fold_events(h)) != hipSuccess) return err;
    const size_t i = 2 * h->ev_kind.size();
    err = hipEventRecord(h->ev[i], h->stream);
    if (err != hipSuccess) return err;
    if ((err = launch()) != hipSuccess) return err;
    if ((err = hipEventRecord(h->ev[i + 1], h->stream)) != hipSuccess) return err;
    h->ev_kind.push_back(kind);
    return hipSuccess;
}

int upload(hom4d* h, void* dst, const void* src, size_t bytes) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return HOM4D_OK;
}

double xgrid(const hom4d_cfg& c, int i) { return -0.5 * c.lx_nm + i * (c.lx_nm / c.nx); }
double ygrid(const hom4d_cfg& c, int j) { return -0.5 * c.ly_nm + j * (c.ly_nm / c.ny); }
// angular wave number of FFT index m for n points over length L (Nyquist -> negative)
double kgrid(int n, double len, int m) {
    const int mm = (m < (n + 1) / 2) ? m : m - n;
    return 2.0 * M_PI * (mm * (1.0 / (n * (len / n))));
}

int build_twiddles(hom4d* h) {
    for (int axis = 0; axis < 2; ++axis) {
        const int n = axis == 0 ? h->cfg.nx : h->cfg.ny;
        std::vector<double2> tw(n);
        for (int j = 0; j < n; ++j) {
            const long double a = 2.0L * kPiL * (long double)j / (long double)n;
            tw[j] = make_double2((double)cosl(a), (double)-sinl(a));
        }
        int rc = upload(h, axis == 0 ? h->tw_x : h->tw_y, tw.data(), n * sizeof(double2));
        if (rc) return rc;
    }
    return HOM4D_OK;
}

int build_kinetic(hom4d* h) {
    const hom4d_cfg& c = h->cfg;
    const double eb = h->u.eoh * c.b_tesla;
    for (int which = 0; which < 2; ++which) {
        const double tau = which == 0 ? 0.5 * c.dt_fs : c.dt_fs;
        std::vector<double2> t((size_t)c.ny * c.nx), tt((size_t)c.ny * c.nx);
        for (int j = 0; j < c.ny; ++j) {
            const double shift = ygrid(c, j) * eb;
            for (int m = 0; m < c.nx; ++m) {
                const double q = kgrid(c.nx, c.lx_nm, m) - shift;
                const double th = (tau / h->u.hbar) * h->u.kappa * (q * q);
                double f[2];
                phase(th, 1.0 / c.nx, f);
                t[(size_t)j * c.nx + m] = make_double2(f[0], f[1]);   // y-major
                tt[(size_t)m * c.ny + j] = make_double2(f[0], f[1]);  // k-major
            }
        }
        int rc = upload(h, which == 0 ? h->kx_half : h->kx_full, t.data(), t.size() * sizeof(double2));
        if (rc) return rc;
        rc = upload(h, which == 0 ? h->kxt_half : h->kxt_full, tt.data(), tt.size() * sizeof(double2));
        if (rc) return rc;
    }
    std::vector<double2> ty(c.ny);
    for (int m = 0; m < c.ny; ++m) {
        const double k = kgrid(c.ny, c.ly_nm, m);
        const double th = (c.dt_fs / h->u.hbar) * h->u.kappa * (k * k);
        double f[2];
        phase(th, 1.0 / c.ny, f);
        ty[m] = make_double2(f[0], f[1]);
    }
    return upload(h, h->ky_full, ty.data(), ty.size() * sizeof(double2));
}

int build_coulomb(hom4d* h) {
    const hom4d_cfg& c = h->cfg;
    const int ax = 2 * c.nx - 1, ay = 2 * c.ny - 1;
    std::vector<double2> t((size_t)ax * ay);
    const double dx = c.lx_nm / c.nx, dy = c.ly_nm / c.ny;
    const double tau = 0.5 * c.dt_fs;
    for (int di = 0; di < ax; ++di)
        for (int dj = 0; dj < ay; ++dj) {
            const double ddx = (di - (c.nx - 1)) * dx, ddy = (dj - (c.ny - 1)) * dy;
            const double r2 = ddx * ddx + ddy * ddy;
            double v = c.coulomb_c * h->u.kc / std::sqrt(r2 + c.soft_nm * c.soft_nm);
            if (c.screen_nm > 0.0) v *= std::exp(-std::sqrt(r2) / c.screen_nm);
            double f[2];
            phase((tau / h->u.hbar) * v, 1.0, f);
            t[(size_t)di * ay + dj] = make_double2(f[0], f[1]);
        }
    return upload(h, h->ac_half, t.data(), t.size() * sizeof(double2));
}

int sync_check(hom4d* h, const char* what) {
    if (!h->sync_check) return HOM4D_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(HOM4D_EHIP, "%s: %s", what, hipGetErrorString(e));
    return HOM4D_OK;
}

// Div3 of d = 2^a 3^c, c <= 2, a >= 1 (validate() admits only such extents).
Div3 make_div3(uint32_t d) {
    uint32_t a = 0, c = 0, r = d;
    while (r % 2 == 0) { r /= 2; ++a; }
    while (r % 3 == 0) { r /= 3; ++c; }
    Div3 q{};
    q.d = d;
    if (r != 1 || c > 2 || a < 1) return q;  // not reached for supported extents
    if (c == 0) {
        q.s1 = a - 1; q.m = 0x80000000u; q.s2 = 0;
    } else {
        q.s1 = a; q.m = c == 1 ? 0xAAAAAAABu : 0x38E38E39u; q.s2 = 1;
    }
    return q;
}

enum KTab { KX_HALF, KX_FULL, KY_FULL };

struct GradCtx {
    double* gb_x1;
    double* gb_x2;
    double* m_x1;
    double* m_y1;
    double* m_x2;
    double* m_y2;
};

int run_pass(hom4d* h, int axis, KTab kt, int vmode, int nst, void* lam, bool reverse, int gflags,
             const GradCtx* g) {
    const hom4d_cfg& c = h->cfg;
    // the pass kernels conjugate every factor exactly when they carry two states
    if (reverse != (nst == 2)) return fail(HOM4D_EINVAL, "internal: a reverse pass carries the adjoint state");
    AxisPlan p = plan_axis(axis, c.nx, c.ny, nst, nst == 2, h->mixed);
    PassArgs a{};
    a.psi = h->psi;
    a.lam = lam;
    a.nx = c.nx;
    a.ny = c.ny;
    a.dnx = make_div3((uint32_t)c.nx);
    a.dny = make_div3((uint32_t)c.ny);
    a.dnxy = make_div3((uint32_t)(c.nx * c.ny));
    a.W = p.W;
    a.ntiles = (uint32_t)(p.nlines / p.W);
    a.tw = (axis == AX_X1 || axis == AX_X2) ? h->tw_x : h->tw_y;
    if (axis == AX_X2)
        a.ktab = kt == KX_HALF ? h->kxt_half : h->kxt_full;
    else
        a.ktab = kt == KX_HALF ? h->kx_half : (kt == KX_FULL ? h->kx_full : h->ky_full);
    a.vmode = vmode;
    // Non-temporal state accesses where each pass streams the state through
    // once: on every pass for states over 1 GiB (four times the 256 MB
    // Infinity Cache; 256x128 complex64 23.55 -> 22.01 ms per step, 128x128
    // FP64 7.18 -> 6.77, 128x96 FP64 3.90 -> 3.70, 128x96 complex64 2.715 ->
    // 2.667), and on the x1 pass from 512 MiB (128x64 FP64 1.572 -> 1.524 ms,
    // complex64 1.096 -> 1.083; all passes there were slower, and x1 with x2
    // let the following y1 pass lose its cache hits).  Smaller states keep
    // the default policy (64x64 FP64 288 -> 332 us with it), since one pass
    // then hits what the previous one wrote.
    a.nt = (h->state_bytes > (size_t(1) << 30) || (axis == AX_X1 && h->state_bytes >= (size_t(1) << 29))) ? 1 : 0;
    a.a1 = h->a1_half;
    a.ac = h->ac_half;  // all (1, 0) without the Coulomb term: the product is then exact
    a.vdirect = c.coulomb_mode == HOM4D_COULOMB_DIRECT ? 1 : 0;
    a.vtab = h->v_dev;
    a.vscale = (reverse ? -0.5 : 0.5) * c.dt_fs / h->u.hbar;
    a.dx = c.lx_nm / c.nx;
    a.dy = c.ly_nm / c.ny;
    a.soft2 = c.soft_nm * c.soft_nm;
    a.ck = c.coulomb_c * h->u.kc;
    a.inv_screen = c.screen_nm > 0.0 ? 1.0 / c.screen_nm : 0.0;
    a.gflags = gflags;
    if (nst == 2 && g) {
        const double tau = kt == KX_FULL ? c.dt_fs : 0.5 * c.dt_fs;
        a.db_coef = (tau / h->u.hbar) * h->u.kappa * 2.0 * (-h->u.eoh);
        a.b_eoh = h->u.eoh * c.b_tesla;
        a.kstep = 2.0 * M_PI / c.lx_nm;
        a.y0 = -0.5 * c.ly_nm;
        a.ystep = c.ly_nm / c.ny;
        if (axis == AX_X1) { a.gb_part = g->gb_x1; a.marg_part = g->m_x1; }
        if (axis == AX_X2) { a.gb_part = g->gb_x2; a.marg_part = g->m_x2; }
        if (axis == AX_Y1) { a.marg_part = g->m_y1; }
        if (axis == AX_Y2) { a.marg_part = g->m_y2; }
    }
    if (vmode && !h->have_v) return fail(HOM4D_ESTATE, "no potential set (hom4d_set_potential)");
    HIP_TRY(timed_launch(h, axis, [&] { return launch_axis(axis, p.n, h->mixed, nst, p.pers, a, p.nlines, p.lds, h->stream); }));
    return sync_check(h, "axis pass");
}

// The fused (x2, y2) plane pass: X2(kt), potential factor, Y2(dt).
int run_plane(hom4d* h, KTab kt) {
    const hom4d_cfg& c = h->cfg;
    if (!h->have_v) return fail(HOM4D_ESTATE, "no potential set (hom4d_set_potential)");
    PassArgs a{};
    a.psi = h->psi;
    a.nx = c.nx;
    a.ny = c.ny;
    a.tw = h->tw_x;
    a.ktab = kt == KX_HALF ? h->kxt_half : h->kxt_full;  // k-major
    a.tw2 = h->tw_y;
    a.ktab2 = h->ky_full;
    a.a1 = h->a1_half;
    a.ac = h->ac_half;  // all (1, 0) without the Coulomb term: the product is then exact
    a.vdirect = c.coulomb_mode == HOM4D_COULOMB_DIRECT ? 1 : 0;
    a.vtab = h->v_dev;
    a.vscale = 0.5 * c.dt_fs / h->u.hbar;
    a.dx = c.lx_nm / c.nx;
    a.dy = c.ly_nm / c.ny;
    a.soft2 = c.soft_nm * c.soft_nm;
    a.ck = c.coulomb_c * h->u.kc;
    a.inv_screen = c.screen_nm > 0.0 ? 1.0 / c.screen_nm : 0.0;
    HIP_TRY(timed_launch(h, 4, [&] { return launch_plane(c.nx, c.ny, h->mixed, a, h->stream); }));
    return sync_check(h, "plane pass");
}

bool use_plane(const hom4d* h) { return h->pass_plan == 0 && h->plane_built; }

// n whole forward steps in three passes per step:
//   X1 | [X2, V, Y2] (plane) | [Y1, V]  ...  closing X1, X2 halves.
int run_steps_plane(hom4d* h, int64_t n) {
    int rc;
    if ((rc = run_pass(h, AX_X1, KX_HALF, 0, 1, nullptr, false, 0, nullptr))) return rc;
    for (int64_t i = 0; i < n; ++i) {
        const bool last = i == n - 1;
        if ((rc = run_plane(h, i == 0 ? KX_HALF : KX_FULL))) return rc;
        if ((rc = run_pass(h, AX_Y1, KY_FULL, 2, 1, nullptr, false, 0, nullptr))) return rc;
        if ((rc = run_pass(h, AX_X1, last ? KX_HALF : KX_FULL, 0, 1, nullptr, false, 0, nullptr))) return rc;
    }
    return run_pass(h, AX_X2, KX_HALF, 0, 1, nullptr, false, 0, nullptr);
}

// n whole forward steps in four per-axis passes, the potential factor as the
// epilogue of the x2 and y2 passes:  X1 | X2, V | Y1 | Y2, V | X1 ...
int run_steps_axis(hom4d* h, int64_t n) {
    int rc;
    if ((rc = run_pass(h, AX_X1, KX_HALF, 0, 1, nullptr, false, 0, nullptr))) return rc;
    if ((rc = run_pass(h, AX_X2, KX_HALF, 2, 1, nullptr, false, 0, nullptr))) return rc;
    for (int64_t i = 0; i < n; ++i) {
        const bool last = i == n - 1;
        if ((rc = run_pass(h, AX_Y1, KY_FULL, 0, 1, nullptr, false, 0, nullptr))) return rc;
        if ((rc = run_pass(h, AX_Y2, KY_FULL, 2, 1, nullptr, false, 0, nullptr))) return rc;
        const KTab kx = last ? KX_HALF : KX_FULL;
        if ((rc = run_pass(h, AX_X1, kx, 0, 1, nullptr, false, 0, nullptr))) return rc;
        if ((rc = run_pass(h, AX_X2, kx, last ? 0 : 2, 1, nullptr, false, 0, nullptr))) return rc;
    }
    return HOM4D_OK;
}

// n whole steps with merged X halves; the state is closed at the end.
int run_steps(hom4d* h, int64_t n, int nst, void* lam, bool reverse, const GradCtx* g) {
    if (n <= 0) return HOM4D_OK;
    if (nst == 1 && !reverse) return use_plane(h) ? run_steps_plane(h, n) : run_steps_axis(h, n);
    // reverse (dual-state) sweep: X1 | X2 | V, Y1 | Y2, V -- the gradient marginals of each
    // potential factor are taken by the passes on either side of it
    const bool gr = nst == 2;
    int rc;
    if ((rc = run_pass(h, AX_X1, KX_HALF, 0, nst, lam, reverse, gr ? G_GB : 0, g))) return rc;
    if ((rc = run_pass(h, AX_X2, KX_HALF, 0, nst, lam, reverse, gr ? (G_GB | G_MOUT) : 0, g))) return rc;
    for (int64_t i = 0; i < n; ++i) {
        const bool last = i == n - 1;
        if ((rc = run_pass(h, AX_Y1, KY_FULL, 1, nst, lam, reverse, gr ? G_MIN : 0, g))) return rc;
        if ((rc = run_pass(h, AX_Y2, KY_FULL, 2, nst, lam, reverse, gr ? G_MOUT : 0, g))) return rc;
        const KTab kx = last ? KX_HALF : KX_FULL;
        if ((rc = run_pass(h, AX_X1, kx, 0, nst, lam, reverse, gr ? (G_GB | G_MIN) : 0, g))) return rc;
        if ((rc = run_pass(h, AX_X2, kx, 0, nst, lam, reverse, gr ? (G_GB | (last ? 0 : G_MOUT)) : 0, g)))
            return rc;
    }
    return HOM4D_OK;
}




int fetch_reduction(hom4d* h, int width, double* out) {
    HIP_TRY(launch_reduce_parts(h->red_part, h->red_blocks, width, h->red_out, h->stream));
    HIP_TRY(hipMemcpyAsync(h->host_out, h->red_out, width * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int q = 0; q < width; ++q) out[q] = h->host_out[q];
    return HOM4D_OK;
}

int check_weights(const double* w, int n) {
    if (!w) return fail(HOM4D_EINVAL, "w_top is NULL");
    for (int i = 0; i < n; ++i)
        if (!(w[i] >= 0.0 && w[i] <= 1.0)) return fail(HOM4D_EINVAL, "w_top[%d] = %g outside [0, 1]", i, w[i]);
    return HOM4D_OK;
}

// Eigenvalues of a real symmetric matrix (row-major, n x n, destroyed), cyclic Jacobi.
void jacobi_eigenvalues(std::vector<double>& a, int n, std::vector<double>& ev) {
    auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
    double diag2 = 0.0;
    for (int i = 0; i < n; ++i) diag2 += A(i, i) * A(i, i);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A(p, q) * A(p, q);
        if (off <= 1e-32 * std::max(diag2, 1e-300)) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                const double zeta = (A(q, q) - A(p, p)) / (2.0 * apq);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(zeta * zeta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
            }
    }
    ev.resize(n);
    for (int i = 0; i < n; ++i) ev[i] = A(i, i);
}

int slice_checks(hom4d* h, const int32_t* ix1, int32_t n1, int32_t jy1, const int32_t* ix2, int32_t n2,
                 int32_t jy2) {
    const hom4d_cfg& c = h->cfg;
    if (!ix1 || !ix2) return fail(HOM4D_EINVAL, "index array is NULL");
    if (n1 < 1 || n1 > 256 || n2 < 1 || n2 > 256) return fail(HOM4D_EINVAL, "slice sizes must be in [1, 256]");
    if (jy1 < 0 || jy1 >= c.ny || jy2 < 0 || jy2 >= c.ny) return fail(HOM4D_EINVAL, "y slice index out of range");
    for (int i = 0; i < n1; ++i)
        if (ix1[i] < 0 || ix1[i] >= c.nx) return fail(HOM4D_EINVAL, "ix1[%d] out of range", i);
    for (int i = 0; i < n2; ++i)
        if (ix2[i] < 0 || ix2[i] >= c.nx) return fail(HOM4D_EINVAL, "ix2[%d] out of range", i);
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    return HOM4D_OK;
}

int gather(hom4d* h, const int32_t* ix1, int32_t n1, int32_t jy1, const int32_t* ix2, int32_t n2, int32_t jy2,
           std::vector<double>& out) {
    int rc = slice_checks(h, ix1, n1, jy1, ix2, n2, jy2);
    if (rc) return rc;
    std::vector<int32_t> idx(512, 0);
    std::memcpy(idx.data(), ix1, n1 * sizeof(int32_t));
    std::memcpy(idx.data() + 256, ix2, n2 * sizeof(int32_t));
    HIP_TRY(hipMemcpyAsync(h->ix_dev, idx.data(), 512 * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(launch_gather(h->psi, h->mixed, h->ix_dev, n1, jy1, h->ix_dev + 256, n2, jy2, h->cfg.nx, h->cfg.ny,
                          h->slice_dev, h->stream));
    out.resize((size_t)2 * n1 * n2);
    HIP_TRY(hipMemcpyAsync(out.data(), h->slice_dev, (size_t)n1 * n2 * sizeof(double2), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return HOM4D_OK;
}

// 64-bit FNV-1a, continued from h.
uint64_t fnv1a(const void* p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

// Everything a resumed run must share with the saved one: the configuration
// fields one by one (no struct padding), the current field B and the potential.
uint64_t config_hash(const hom4d* h) {
    const hom4d_cfg& c = h->cfg;
    uint64_t x = fnv1a(&c.nx, sizeof c.nx);
    x = fnv1a(&c.ny, sizeof c.ny, x);
    x = fnv1a(&c.precision, sizeof c.precision, x);
    x = fnv1a(&c.coulomb_mode, sizeof c.coulomb_mode, x);
    const double d[] = {c.lx_nm, c.ly_nm, c.mstar_rel, c.eps_r, c.b_tesla, c.dt_fs, c.soft_nm, c.coulomb_c, c.screen_nm};
    x = fnv1a(d, sizeof d, x);
    return fnv1a(&h->v_hash, sizeof h->v_hash, x);
}

// Fletcher-style sum over 64-bit words (every single-bit change and every
// reordering of words changes it); n is a multiple of 8.
uint64_t payload_sum(const void* p, size_t n, uint64_t s1 = 0, uint64_t s2 = 0) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; i += 8) {
        uint64_t w;
        std::memcpy(&w, b + i, 8);
        s1 += w;
        s2 += s1;
    }
    return s1 ^ ((s2 << 32) | (s2 >> 32));
}

// Checkpoint image header (64 bytes), followed by the state in its storage precision.
struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t precision;
    int32_t nx, ny;
    int64_t step;
    uint64_t config_hash;
    uint64_t payload_bytes;
    uint64_t payload_sum;
    double norm;
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header is 64 bytes");
constexpr char kCkptMagic[8] = {'H', 'O', 'M', '4', 'D', 'C', 'K', '1'};

// FP64 norm of the bound state (one reduction pass).
int state_norm(hom4d* h, double* out) {
    HIP_TRY(hipMemsetAsync(h->w_dev, 0, h->nxy * sizeof(double), h->stream));
    HIP_TRY(launch_obs(h->psi, h->mixed, h->w_dev, h->nxy, h->red_part, h->red_blocks, h->stream));
    double r[5];
    int rc = fetch_reduction(h, 5, r);
    if (rc) return rc;
    *out = r[0];
    return HOM4D_OK;
}

void free_all(hom4d* h) {
    void* bufs[] = {h->tw_x, h->tw_y, h->kx_half, h->kx_full, h->kxt_half, h->kxt_full, h->ky_full, h->a1_half, h->ac_half, h->v_dev,
                    h->w_dev, h->red_part, h->red_out, h->ix_dev, h->slice_dev, h->orb_dev, h->g_buf};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (h->host_out) (void)hipHostFree(h->host_out);
}

// Argument and state checks shared by the two reverse-sweep entry points.
int grad_checks(hom4d* h, const double* w_top, const double* coeffs, void* d_lambda, double* loss, double* dL_dV,
                double* dL_dB) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!coeffs || !d_lambda || !loss || !dL_dV || !dL_dB) return fail(HOM4D_EINVAL, "NULL argument");
    if (((uintptr_t)d_lambda) % 16 != 0) return fail(HOM4D_EINVAL, "adjoint buffer must be 16-byte aligned");
    int rc = check_weights(w_top, h->nxy);
    if (rc) return rc;
    if (!h->rec) return fail(HOM4D_ESTATE, "no recorded forward run (hom4d_grad_begin + hom4d_step)");
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    if ((size_t)(h->rec_steps / h->ckpt_every + 1) * h->state_bytes > h->pool_bytes)
        return fail(HOM4D_ESTATE, "recorded checkpoints exceed the pool (%zu bytes)", h->pool_bytes);
    return HOM4D_OK;
}

// Layout of the reverse sweep's FP64 partial sums: dL/dB per block of the two x
// passes, the potential marginals per line (x1, y1) or per block (x2, y2), then
// the finished dL/dV table.
struct GradLayout {
    int64_t nb_x1, nb_x2, nb_y2, len_m_x1, len_m_y1;
    int w_x2, w_y2;
    size_t total;  // doubles
};

GradLayout grad_layout(const hom4d* h) {
    const hom4d_cfg& c = h->cfg;
    const AxisPlan px1 = plan_axis(AX_X1, c.nx, c.ny, 2, true, h->mixed);
    const AxisPlan px2 = plan_axis(AX_X2, c.nx, c.ny, 2, true, h->mixed);
    const AxisPlan py1 = plan_axis(AX_Y1, c.nx, c.ny, 2, true, h->mixed);
    const AxisPlan py2 = plan_axis(AX_Y2, c.nx, c.ny, 2, true, h->mixed);
    GradLayout l;
    l.nb_x1 = px1.nlines / px1.W;
    l.nb_x2 = px2.nlines / px2.W;
    l.nb_y2 = py2.nlines / py2.W;
    l.len_m_x1 = px1.nlines;
    l.len_m_y1 = py1.nlines;
    l.w_x2 = px2.W;
    l.w_y2 = py2.W;
    l.total = (size_t)(l.nb_x1 + l.nb_x2 + l.len_m_x1 + l.len_m_y1 + l.nb_x2 + l.nb_y2 + h->nxy);
    return l;
}

size_t grad_scratch_len(const hom4d* h) { return grad_layout(h).total; }

// The reverse sweep on the partial-sum buffer buf (grad_scratch_len doubles, cleared here).
int grad_sweep(hom4d* h, const double* w_top, const double* coeffs, void* d_lambda, double* loss, double* dL_dV,
               double* dL_dB, double* buf) {
    const hom4d_cfg& c = h->cfg;
    const GradLayout l = grad_layout(h);
    GradCtx g;
    g.gb_x1 = buf;
    g.gb_x2 = g.gb_x1 + l.nb_x1;
    g.m_x1 = g.gb_x2 + l.nb_x2;
    g.m_y1 = g.m_x1 + l.len_m_x1;
    g.m_x2 = g.m_y1 + l.len_m_y1;
    g.m_y2 = g.m_x2 + l.nb_x2;
    double* dldv_dev = g.m_y2 + l.nb_y2;
    int rc;
    HIP_TRY(launch_zero(buf, (int64_t)l.total, h->stream));
    HIP_TRY(hipMemcpyAsync(h->w_dev, w_top, h->nxy * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(launch_loss_lambda(h->psi, d_lambda, h->mixed, h->w_dev, coeffs, h->nxy, h->red_part, h->red_blocks,
                               h->stream));
    double L = 0.0;
    if ((rc = fetch_reduction(h, 1, &L))) return rc;
    // reverse sweep, segment by segment, restoring the state at every checkpoint
    int64_t seg_end = h->rec_steps;
    for (int64_t k = h->rec_steps / h->ckpt_every; k >= 0; --k) {
        const int64_t seg_start = k * h->ckpt_every;
        if (seg_end > seg_start) {
            if ((rc = run_steps(h, seg_end - seg_start, 2, d_lambda, true, &g))) return rc;
        }
        HIP_TRY(hipMemcpyAsync(h->psi, h->pool + (size_t)k * h->state_bytes, h->state_bytes, hipMemcpyDeviceToDevice,
                               h->stream));
        seg_end = seg_start;
    }
    HIP_TRY(launch_grad_finish(g.m_x2, (int)(c.ny / l.w_x2), g.m_y2, (int)(c.nx / l.w_y2), g.m_y1, g.m_x1, c.nx,
                               c.ny, c.dt_fs / h->u.hbar, dldv_dev, h->stream));
    HIP_TRY(hipMemcpyAsync(dL_dV, dldv_dev, h->nxy * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    // dL/dB: both x axes, Parseval factor 1/nx, factor 2 of 2 Im(conj(lambda) psi)
    HIP_TRY(launch_reduce_parts(g.gb_x1, (int)(l.nb_x1 + l.nb_x2), 1, h->red_out, h->stream));
    HIP_TRY(hipMemcpyAsync(h->host_out, h->red_out, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    *dL_dB = h->host_out[0] * 2.0 / c.nx;
    *loss = L;
    h->step -= h->rec_steps;
    h->rec = false;
    return HOM4D_OK;
}

}  // namespace

extern "C" {

int hom4d_validate_cfg(const hom4d_cfg* cfg) { return validate(cfg); }

size_t hom4d_state_bytes(const hom4d_cfg* cfg) {
    if (validate(cfg) != HOM4D_OK) return 0;
    const size_t nxy = (size_t)cfg->nx * cfg->ny;
    return nxy * nxy * (cfg->precision == HOM4D_MIXED ? 8 : 16);
}

int hom4d_create(const hom4d_cfg* cfg, void* hip_stream, hom4d** out) {
    if (!out) return fail(HOM4D_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    hom4d* h = new hom4d();
    h->cfg = *cfg;
    h->u = units_for(*cfg);
    h->stream = (hipStream_t)hip_stream;
    h->mixed = cfg->precision == HOM4D_MIXED;
    h->sync_check = env_sync_check();
    h->nxy = cfg->nx * cfg->ny;
    h->npts = (int64_t)h->nxy * h->nxy;
    h->state_bytes = hom4d_state_bytes(cfg);
    h->red_blocks = std::min(h->nxy, 1024);
    auto cleanup = [&](int code) {
        free_all(h);
        delete h;
        return code;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        fail(HOM4D_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
        return cleanup(HOM4D_EHIP);
    }
    const int nx = cfg->nx, ny = cfg->ny;
    struct {
        void** p;
        size_t bytes;
    } allocs[] = {
        {(void**)&h->tw_x, nx * sizeof(double2)},
        {(void**)&h->tw_y, ny * sizeof(double2)},
        {(void**)&h->kx_half, (size_t)nx * ny * sizeof(double2)},
        {(void**)&h->kx_full, (size_t)nx * ny * sizeof(double2)},
        {(void**)&h->kxt_half, (size_t)nx * ny * sizeof(double2)},
        {(void**)&h->kxt_full, (size_t)nx * ny * sizeof(double2)},
        {(void**)&h->ky_full, ny * sizeof(double2)},
        {(void**)&h->a1_half, (size_t)nx * ny * sizeof(double2)},
        {(void**)&h->ac_half, (size_t)(2 * nx - 1) * (2 * ny - 1) * sizeof(double2)},
        {(void**)&h->v_dev, (size_t)nx * ny * sizeof(double)},
        {(void**)&h->w_dev, (size_t)nx * ny * sizeof(double)},
        {(void**)&h->red_part, (size_t)h->red_blocks * 8 * sizeof(double)},
        {(void**)&h->red_out, 8 * sizeof(double)},
        {(void**)&h->ix_dev, 512 * sizeof(int32_t)},
        {(void**)&h->slice_dev, 256 * 256 * sizeof(double2)},
        {(void**)&h->orb_dev, (size_t)2 * nx * ny * sizeof(double2)},
    };
    for (auto& a : allocs) {
        e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) {
            fail(HOM4D_EHIP, "hipMalloc(%zu): %s", a.bytes, hipGetErrorString(e));
            return cleanup(HOM4D_EHIP);
        }
    }
    e = hipHostMalloc((void**)&h->host_out, 8 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        fail(HOM4D_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
        return cleanup(HOM4D_EHIP);
    }
    if ((rc = build_twiddles(h)) || (rc = build_kinetic(h)) || (rc = build_coulomb(h))) return cleanup(rc);
    // the fixed scratch of hom4d_grad_backward_noalloc: its address on this device, once
    e = init_scratch(h->device);
    if (e != hipSuccess) {
        fail(HOM4D_EHIP, "device scratch address: %s", hipGetErrorString(e));
        return cleanup(HOM4D_EHIP);
    }
    h->plane_built = plane_available(nx, ny, h->mixed);
    *out = h;
    return HOM4D_OK;
}

int hom4d_destroy(hom4d* h) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_events(h);
    free_all(h);
    delete h;
    return HOM4D_OK;
}

int hom4d_bind_state(hom4d* h, void* d_psi) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!d_psi) return fail(HOM4D_EINVAL, "state pointer is NULL");
    if (((uintptr_t)d_psi) % 16 != 0) return fail(HOM4D_EINVAL, "state pointer must be 16-byte aligned");
    h->psi = d_psi;
    h->rec = false;
    return HOM4D_OK;
}

int hom4d_set_potential(hom4d* h, const double* v) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!v) return fail(HOM4D_EINVAL, "potential is NULL");
    const hom4d_cfg& c = h->cfg;
    std::vector<double2> a1((size_t)c.nx * c.ny);
    for (int i = 0; i < c.nx * c.ny; ++i) {
        if (!std::isfinite(v[i])) return fail(HOM4D_EINVAL, "V[%d] is not finite", i);
        double f[2];
        phase((0.5 * c.dt_fs / h->u.hbar) * v[i], 1.0, f);
        a1[i] = make_double2(f[0], f[1]);
    }
    int rc = upload(h, h->a1_half, a1.data(), a1.size() * sizeof(double2));
    if (rc) return rc;
    rc = upload(h, h->v_dev, v, (size_t)c.nx * c.ny * sizeof(double));
    if (rc) return rc;
    h->have_v = true;
    h->v_hash = fnv1a(v, (size_t)c.nx * c.ny * sizeof(double));
    h->rec = false;  // a recorded forward run used the old factors
    return HOM4D_OK;
}

int hom4d_set_field(hom4d* h, double b) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!std::isfinite(b)) return fail(HOM4D_EINVAL, "B must be finite");
    h->cfg.b_tesla = b;
    h->rec = false;  // a recorded forward run used the old factors
    return build_kinetic(h);
}

int hom4d_set_norm_tol(hom4d* h, double tol) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!(tol > 0.0)) return fail(HOM4D_EINVAL, "tolerance must be positive");
    h->norm_tol = tol;
    return HOM4D_OK;
}

int hom4d_init_state(hom4d* h, const double* psi_a, const double* psi_b, int32_t sym) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!psi_a || !psi_b) return fail(HOM4D_EINVAL, "orbital is NULL");
    if (sym != -1 && sym != 0 && sym != 1) return fail(HOM4D_EINVAL, "sym=%d: use -1, 0 or +1", sym);
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    const size_t nb = (size_t)h->nxy * sizeof(double2);
    HIP_TRY(hipMemcpyAsync(h->orb_dev, psi_a, nb, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->orb_dev + h->nxy, psi_b, nb, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(launch_init_norm(h->orb_dev, h->orb_dev + h->nxy, sym, h->nxy, h->red_part, h->red_blocks, h->stream));
    double nrm = 0.0;
    int rc = fetch_reduction(h, 1, &nrm);
    if (rc) return rc;
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(HOM4D_EINVAL, "initial state has norm %g", nrm);
    HIP_TRY(launch_init_write(h->psi, h->mixed, h->orb_dev, h->orb_dev + h->nxy, sym, h->nxy, 1.0 / std::sqrt(nrm),
                              h->stream));
    h->step = 0;
    h->rec = false;
    return sync_check(h, "init");
}

int hom4d_load_state(hom4d* h, const double* psi4d) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!psi4d) return fail(HOM4D_EINVAL, "state is NULL");
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    if (!h->mixed) {
        HIP_TRY(hipMemcpyAsync(h->psi, psi4d, h->state_bytes, hipMemcpyHostToDevice, h->stream));
    } else {
        // round to complex64 on the host in chunks
        const int64_t chunk = 1 << 22;
        std::vector<float> buf((size_t)2 * chunk);
        for (int64_t o = 0; o < h->npts; o += chunk) {
            const int64_t m = std::min(chunk, h->npts - o);
            for (int64_t i = 0; i < 2 * m; ++i) buf[i] = (float)psi4d[2 * o + i];
            HIP_TRY(hipMemcpyAsync((float2*)h->psi + o, buf.data(), m * sizeof(float2), hipMemcpyHostToDevice,
                                   h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
        }
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->step = 0;
    h->rec = false;
    return HOM4D_OK;
}

int hom4d_store_state(hom4d* h, double* psi4d) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!psi4d) return fail(HOM4D_EINVAL, "output is NULL");
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    if (!h->mixed) {
        HIP_TRY(hipMemcpyAsync(psi4d, h->psi, h->state_bytes, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    } else {
        const int64_t chunk = 1 << 22;
        std::vector<float> buf((size_t)2 * chunk);
        for (int64_t o = 0; o < h->npts; o += chunk) {
            const int64_t m = std::min(chunk, h->npts - o);
            HIP_TRY(hipMemcpyAsync(buf.data(), (float2*)h->psi + o, m * sizeof(float2), hipMemcpyDeviceToHost,
                                   h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
            for (int64_t i = 0; i < 2 * m; ++i) psi4d[2 * o + i] = (double)buf[i];
        }
    }
    return HOM4D_OK;
}

size_t hom4d_checkpoint_bytes(const hom4d* h) { return h ? sizeof(CkptHeader) + h->state_bytes : 0; }

int hom4d_save_checkpoint(hom4d* h, void* buf, size_t bytes) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!buf) return fail(HOM4D_EINVAL, "buffer is NULL");
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    if (bytes < sizeof(CkptHeader) + h->state_bytes)
        return fail(HOM4D_ENOMEM, "checkpoint buffer of %zu bytes, %zu needed", bytes,
                    sizeof(CkptHeader) + h->state_bytes);
    double nrm = 0.0;
    int rc = state_norm(h, &nrm);
    if (rc) return rc;
    if (!std::isfinite(nrm)) return fail(HOM4D_ENONFINITE, "state holds non-finite values");
    char* payload = static_cast<char*>(buf) + sizeof(CkptHeader);
    HIP_TRY(hipMemcpyAsync(payload, h->psi, h->state_bytes, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    CkptHeader hd{};
    std::memcpy(hd.magic, kCkptMagic, 8);
    hd.version = 1;
    hd.precision = h->cfg.precision;
    hd.nx = h->cfg.nx;
    hd.ny = h->cfg.ny;
    hd.step = h->step;
    hd.config_hash = config_hash(h);
    hd.payload_bytes = h->state_bytes;
    hd.payload_sum = payload_sum(payload, h->state_bytes);
    hd.norm = nrm;
    std::memcpy(buf, &hd, sizeof hd);
    return HOM4D_OK;
}

int hom4d_load_checkpoint(hom4d* h, const void* buf, size_t bytes) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!buf) return fail(HOM4D_EINVAL, "buffer is NULL");
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    CkptHeader hd;
    if (bytes < sizeof hd) return fail(HOM4D_EINVAL, "%zu bytes: shorter than a checkpoint header", bytes);
    std::memcpy(&hd, buf, sizeof hd);
    if (std::memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 1)
        return fail(HOM4D_EINVAL, "not a checkpoint image of this library");
    if (hd.precision != h->cfg.precision || hd.nx != h->cfg.nx || hd.ny != h->cfg.ny ||
        hd.payload_bytes != h->state_bytes)
        return fail(HOM4D_ECONFIG, "checkpoint of a %dx%d %s state, handle is %dx%d %s", hd.nx, hd.ny,
                    hd.precision == HOM4D_MIXED ? "complex64" : "complex128", h->cfg.nx, h->cfg.ny,
                    h->mixed ? "complex64" : "complex128");
    if (hd.config_hash != config_hash(h))
        return fail(HOM4D_ECONFIG, "checkpoint taken with other parameters, field or potential");
    if (bytes < sizeof hd + hd.payload_bytes)
        return fail(HOM4D_EINVAL, "%zu bytes: the image is truncated (%zu expected)", bytes,
                    (size_t)(sizeof hd + hd.payload_bytes));
    const char* payload = static_cast<const char*>(buf) + sizeof hd;
    if (payload_sum(payload, h->state_bytes) != hd.payload_sum)
        return fail(HOM4D_ECORRUPT, "checkpoint payload does not match its checksum");
    HIP_TRY(hipMemcpyAsync(h->psi, payload, h->state_bytes, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->rec = false;
    double nrm = 0.0;
    int rc = state_norm(h, &nrm);
    if (rc) return rc;
    if (!std::isfinite(nrm)) return fail(HOM4D_ENONFINITE, "restored state holds non-finite values");
    if (!(std::fabs(nrm - hd.norm) <= 1e-12 * std::fabs(hd.norm)))
        return fail(HOM4D_ECORRUPT, "restored state has norm %.17g, the image recorded %.17g", nrm, hd.norm);
    h->step = hd.step;
    return HOM4D_OK;
}

int hom4d_step(hom4d* h, int64_t n) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (n < 0) return fail(HOM4D_EINVAL, "n=%lld must be >= 0", (long long)n);
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    if (!h->have_v) return fail(HOM4D_ESTATE, "no potential set (hom4d_set_potential)");
    if (!h->rec) {
        int rc = run_steps(h, n, 1, nullptr, false, nullptr);
        if (rc) return rc;
        h->step += n;
        return HOM4D_OK;
    }
    // recording: every checkpoint these n steps reach must fit the pool, checked
    // before anything runs, so that a refused call leaves the state, the step
    // count and the recording as they were
    // (counted in whole slots, so that no product can wrap)
    const int64_t slots = (int64_t)(h->pool_bytes / h->state_bytes);
    if (n > INT64_MAX - h->rec_steps || (h->rec_steps + n) / h->ckpt_every >= slots)
        return fail(HOM4D_ENOMEM, "the checkpoints of %lld more recorded steps do not fit the pool (%zu bytes)",
                    (long long)n, h->pool_bytes);
    // close the state on every checkpoint boundary and copy it out; a failure
    // part way closes the recording (its checkpoints no longer match the state)
    int64_t left = n;
    while (left > 0) {
        const int64_t to_ck = h->ckpt_every - (h->rec_steps % h->ckpt_every);
        const int64_t m = std::min(left, to_ck);
        int rc = run_steps(h, m, 1, nullptr, false, nullptr);
        if (rc) {
            h->rec = false;
            return rc;
        }
        h->rec_steps += m;
        h->step += m;
        left -= m;
        if (h->rec_steps % h->ckpt_every == 0) {
            const size_t slot = (size_t)(h->rec_steps / h->ckpt_every);
            const hipError_t e = hipMemcpyAsync(h->pool + slot * h->state_bytes, h->psi, h->state_bytes,
                                                hipMemcpyDeviceToDevice, h->stream);
            if (e != hipSuccess) {
                h->rec = false;
                return fail(HOM4D_EHIP, "checkpoint copy: %s", hipGetErrorString(e));
            }
        }
    }
    return HOM4D_OK;
}

int hom4d_observables(hom4d* h, const double* w_top, hom4d_obs* out) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!out) return fail(HOM4D_EINVAL, "out is NULL");
    int rc = check_weights(w_top, h->nxy);
    if (rc) return rc;
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    HIP_TRY(hipMemcpyAsync(h->w_dev, w_top, h->nxy * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(launch_obs(h->psi, h->mixed, h->w_dev, h->nxy, h->red_part, h->red_blocks, h->stream));
    double r[5];
    if ((rc = fetch_reduction(h, 5, r))) return rc;
    out->norm = r[0];
    out->p_tt = r[1];
    out->p_tb = r[2];
    out->p_bt = r[3];
    out->p_bb = r[4];
    out->p_b = r[1] + r[4];
    out->p_ab = r[2] + r[3];
    out->step = h->step;
    if (!std::isfinite(r[0])) return fail(HOM4D_ENONFINITE, "state holds non-finite values");
    if (std::fabs(r[0] - 1.0) > h->norm_tol)
        return fail(HOM4D_ENORMDRIFT, "norm %.17g drifted beyond %g", r[0], h->norm_tol);
    return HOM4D_OK;
}

int hom4d_marginal(hom4d* h, double* out) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!out) return fail(HOM4D_EINVAL, "out is NULL");
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    // the reduction partial buffer has room for red_blocks * 8 >= nx*ny doubles only if
    // nx*ny <= 8 * red_blocks; the slice buffer (256*256 complex) always does
    double* dst = reinterpret_cast<double*>(h->slice_dev);
    HIP_TRY(launch_marginal(h->psi, h->mixed, h->nxy, dst, h->stream));
    HIP_TRY(hipMemcpyAsync(out, dst, h->nxy * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return HOM4D_OK;
}

int hom4d_conditional(hom4d* h, int32_t ix2, int32_t jy2, double* out) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!out) return fail(HOM4D_EINVAL, "out is NULL");
    if (ix2 < 0 || ix2 >= h->cfg.nx || jy2 < 0 || jy2 >= h->cfg.ny)
        return fail(HOM4D_EINVAL, "(ix2, jy2) = (%d, %d) out of range", ix2, jy2);
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    double* dst = reinterpret_cast<double*>(h->slice_dev);
    HIP_TRY(launch_conditional(h->psi, h->mixed, h->nxy, ix2 * h->cfg.ny + jy2, dst, h->stream));
    HIP_TRY(hipMemcpyAsync(out, dst, h->nxy * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return HOM4D_OK;
}

int hom4d_gather_slice(hom4d* h, const int32_t* ix1, int32_t n1, int32_t jy1, const int32_t* ix2, int32_t n2,
                       int32_t jy2, double* out) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!out) return fail(HOM4D_EINVAL, "out is NULL");
    std::vector<double> phi;
    int rc = gather(h, ix1, n1, jy1, ix2, n2, jy2, phi);
    if (rc) return rc;
    std::memcpy(out, phi.data(), phi.size() * sizeof(double));
    return HOM4D_OK;
}

int hom4d_entanglement(hom4d* h, const int32_t* ix1, int32_t n1, int32_t jy1, const int32_t* ix2, int32_t n2,
                       int32_t jy2, double* s_out) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!s_out) return fail(HOM4D_EINVAL, "s_out is NULL");
    std::vector<double> phi;
    int rc = gather(h, ix1, n1, jy1, ix2, n2, jy2, phi);
    if (rc) return rc;
    double nrm = 0.0;
    for (double x : phi) nrm += x * x;
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(HOM4D_ENONFINITE, "slice norm %g", nrm);
    // rho over the smaller side: G = phi phi^dagger (n1 <= n2) or phi^dagger phi, Hermitian,
    // embedded as the real symmetric [[Re, -Im], [Im, Re]] whose spectrum is G's, doubled.
    const bool left = n1 <= n2;
    const int m = left ? n1 : n2, kdim = left ? n2 : n1;
    auto el = [&](int a, int b, double* re, double* im) {  // phi[a][b]
        *re = phi[2 * ((size_t)a * n2 + b)] / std::sqrt(nrm);
        *im = phi[2 * ((size_t)a * n2 + b) + 1] / std::sqrt(nrm);
    };
    std::vector<double> g((size_t)2 * m * 2 * m, 0.0);
    for (int p = 0; p < m; ++p)
        for (int q = 0; q < m; ++q) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < kdim; ++k) {
                double ar, ai, br, bi;
                if (left) {
                    el(p, k, &ar, &ai);
                    el(q, k, &br, &bi);
                } else {
                    el(k, p, &ar, &ai);
                    el(k, q, &br, &bi);
                    ai = -ai;
                    bi = -bi;
                }
                re += ar * br + ai * bi;  // a * conj(b)
                im += ai * br - ar * bi;
            }
            const int M = 2 * m;
            g[(size_t)p * M + q] = re;
            g[(size_t)(p + m) * M + (q + m)] = re;
            g[(size_t)p * M + (q + m)] = -im;
            g[(size_t)(p + m) * M + q] = im;
        }
    std::vector<double> ev;
    jacobi_eigenvalues(g, 2 * m, ev);
    double s = 0.0;
    for (double lam : ev)
        if (lam > 0.0) s -= lam * std::log(lam);
    *s_out = 0.5 * s;
    return HOM4D_OK;
}

int hom4d_grad_begin(hom4d* h, int32_t ckpt_every, void* d_pool, size_t pool_bytes) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (ckpt_every < 1) return fail(HOM4D_EINVAL, "ckpt_every=%d must be >= 1", ckpt_every);
    if (!d_pool) return fail(HOM4D_EINVAL, "pool is NULL");
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    if (pool_bytes < h->state_bytes) return fail(HOM4D_ENOMEM, "pool smaller than one state");
    h->ckpt_every = ckpt_every;
    h->pool = (char*)d_pool;
    h->pool_bytes = pool_bytes;
    h->rec_steps = 0;
    HIP_TRY(hipMemcpyAsync(h->pool, h->psi, h->state_bytes, hipMemcpyDeviceToDevice, h->stream));
    h->rec = true;
    return HOM4D_OK;
}

int hom4d_grad_end(hom4d* h) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    h->rec = false;
    return HOM4D_OK;
}

int hom4d_grad_backward(hom4d* h, const double* w_top, const double* coeffs, void* d_lambda, double* loss,
                        double* dL_dV, double* dL_dB) {
    int rc = grad_checks(h, w_top, coeffs, d_lambda, loss, dL_dV, dL_dB);
    if (rc) return rc;
    const size_t need = grad_scratch_len(h);
    if (need > h->g_len) {
        if (h->g_buf) HIP_TRY(hipFree(h->g_buf));
        h->g_buf = nullptr;
        h->g_len = 0;
        HIP_TRY(hipMalloc((void**)&h->g_buf, need * sizeof(double)));
        h->g_len = need;
    }
    return grad_sweep(h, w_top, coeffs, d_lambda, loss, dL_dV, dL_dB, h->g_buf);
}

int hom4d_grad_backward_noalloc(hom4d* h, const double* w_top, const double* coeffs, void* d_lambda,
                                double* loss, double* dL_dV, double* dL_dB) {
    int rc = grad_checks(h, w_top, coeffs, d_lambda, loss, dL_dV, dL_dB);
    if (rc) return rc;
    if (h->timing) return fail(HOM4D_ESTATE, "pass timing is on (its event pool is created on demand)");
    const size_t need = grad_scratch_len(h);
    if (need > kScratchDoubles)
        return fail(HOM4D_ENOMEM, "gradient partials need %zu doubles, the fixed scratch holds %zu", need,
                    kScratchDoubles);
    double* buf = scratch_on(h->device);
    if (!buf) return fail(HOM4D_EHIP, "device scratch of device %d not initialised", h->device);
    return grad_sweep(h, w_top, coeffs, d_lambda, loss, dL_dV, dL_dB, buf);
}

int hom4d_pass_timing(hom4d* h, int32_t enable) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (enable != 0 && enable != 1) return fail(HOM4D_EINVAL, "enable=%d must be 0 or 1", enable);
    if (enable) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->ev_kind.clear();  // the pool of events is kept
        for (int k = 0; k < 5; ++k) {
            h->ev_ms[k] = 0.0;
            h->ev_n[k] = 0;
        }
    }
    h->timing = enable == 1;
    return HOM4D_OK;
}

int hom4d_pass_times(hom4d* h, double* ms, int64_t* count) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!ms || !count) return fail(HOM4D_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(fold_events(h));
    for (int k = 0; k < 5; ++k) {
        ms[k] = h->ev_ms[k];
        count[k] = h->ev_n[k];
    }
    return HOM4D_OK;
}

int hom4d_set_pass_plan(hom4d* h, int32_t plan) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (plan != 0 && plan != 1) return fail(HOM4D_EINVAL, "plan=%d must be 0 or 1", plan);
    h->pass_plan = plan;
    return HOM4D_OK;
}

int hom4d_pass_plan(hom4d* h) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    return use_plane(h) ? 3 : 4;
}

int hom4d_edge_packet(hom4d* h, const double* v_col, double sigma_x_nm, double xc_nm, int32_t top,
                      double e_above_lll_mev, double* psi_out, double* info_out) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (!v_col || !psi_out) return fail(HOM4D_EINVAL, "v_col and psi_out must not be NULL");
    if (!(sigma_x_nm > 0.0) || !std::isfinite(sigma_x_nm) || !std::isfinite(xc_nm) ||
        !std::isfinite(e_above_lll_mev))
        return fail(HOM4D_EINVAL, "sigma_x=%g must be positive and finite, xc=%g and e_above=%g finite",
                    sigma_x_nm, xc_nm, e_above_lll_mev);
    if (top != 0 && top != 1) return fail(HOM4D_EINVAL, "top=%d must be 0 or 1", top);
    const hom4d_cfg& c = h->cfg;
    const int nx = c.nx, ny = c.ny;
    for (int j = 0; j < ny; ++j)
        if (!std::isfinite(v_col[j])) return fail(HOM4D_EINVAL, "v_col[%d] is not finite", j);
    // first row of the spectral kinetic matrix kappa (-d^2/dy^2) on the periodic y grid
    std::vector<double> host((size_t)2 * ny + nx);
    double* circ = host.data();
    for (int d = 0; d < ny; ++d) {
        double acc = 0.0;
        for (int m = 0; m < ny; ++m) {
            const double k = kgrid(ny, c.ly_nm, m);
            acc += k * k * std::cos(2.0 * M_PI * (double)((m * d) % ny) / ny);
        }
        circ[d] = h->u.kappa * acc / ny;
    }
    std::memcpy(host.data() + ny, v_col, ny * sizeof(double));
    for (int m = 0; m < nx; ++m) host[2 * ny + m] = kgrid(nx, c.lx_nm, m);
    // device: circ, v, kx | work 2 nx ny^2 | e1 nx | phi nx ny | psi 2 nx ny | part nx | info 3
    const size_t n_in = host.size(), n_work = (size_t)2 * nx * ny * ny;
    const size_t total = n_in + n_work + nx + (size_t)nx * ny + (size_t)2 * nx * ny + nx + 3;
    double* dev = nullptr;
    HIP_TRY(hipMalloc((void**)&dev, total * sizeof(double)));
    EdgeArgs e{};
    e.circ = dev;
    e.vcol = dev + ny;
    e.kx = dev + 2 * ny;
    e.work = dev + n_in;
    e.e1 = e.work + n_work;
    e.phi = e.e1 + nx;
    e.psi = reinterpret_cast<double2*>(e.phi + (size_t)nx * ny);
    e.part = e.phi + (size_t)nx * ny + (size_t)2 * nx * ny;
    e.info = e.part + nx;
    e.nx = nx;
    e.ny = ny;
    e.top = top;
    e.kappa = h->u.kappa;
    e.inv_lb2 = h->u.eoh * c.b_tesla;
    e.x0 = xgrid(c, 0);
    e.dx = c.lx_nm / nx;
    e.y0 = ygrid(c, 0);
    e.dy = c.ly_nm / ny;
    e.target = h->u.kappa * e.inv_lb2 + e_above_lll_mev;  // hbar omega_c / 2 = kappa eB / hbar
    e.sigma = sigma_x_nm;
    e.xc = xc_nm;
    double info[3] = {0.0, 0.0, 0.0};
    hipError_t err = hipMemcpyAsync(dev, host.data(), n_in * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (err == hipSuccess) err = launch_edge_packet(e, h->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(psi_out, e.psi, (size_t)nx * ny * sizeof(double2), hipMemcpyDeviceToHost, h->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(info, e.info, sizeof(info), hipMemcpyDeviceToHost, h->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(h->stream);
    const hipError_t ferr = hipFree(dev);
    if (err != hipSuccess) return fail(HOM4D_EHIP, "edge packet: %s", hipGetErrorString(err));
    if (ferr != hipSuccess) return fail(HOM4D_EHIP, "edge packet: %s", hipGetErrorString(ferr));
    if (info_out) std::memcpy(info_out, info, sizeof(info));
    return HOM4D_OK;
}

int hom4d_run_pass(hom4d* h, int32_t axis, int32_t reps) {
    if (!h) return fail(HOM4D_EINVAL, "handle is NULL");
    if (axis < 0 || axis > 5) return fail(HOM4D_EINVAL, "axis=%d must be 0..5", axis);
    if (axis >= 4) {
        if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
        if (axis == 4 && !use_plane(h)) return fail(HOM4D_EINVAL, "no fused plane pass for this size/precision");
        for (int32_t r = 0; r < reps; ++r) {
            int rc = axis == 4 ? run_plane(h, KX_FULL) : run_pass(h, AX_Y1, KY_FULL, 2, 1, nullptr, false, 0, nullptr);
            if (rc) return rc;
        }
        return HOM4D_OK;
    }
    if (reps < 0) return fail(HOM4D_EINVAL, "reps=%d must be >= 0", reps);
    if (!h->psi) return fail(HOM4D_EUNBOUND, "no state bound");
    if (!h->have_v) return fail(HOM4D_ESTATE, "no potential set (hom4d_set_potential)");
    const KTab kt = (axis == AX_X1 || axis == AX_X2) ? KX_FULL : KY_FULL;
    const int vmode = (axis == AX_X2 || axis == AX_Y2) ? 2 : 0;  // the four-pass plan's kernels
    for (int32_t r = 0; r < reps; ++r) {
        int rc = run_pass(h, axis, kt, vmode, 1, nullptr, false, 0, nullptr);
        if (rc) return rc;
    }
    return HOM4D_OK;
}

const char* hom4d_strerror(int status) {
    switch (status) {
        case HOM4D_OK: return "ok";
        case HOM4D_EINVAL: return "invalid argument";
        case HOM4D_EUNBOUND: return "no state bound";
        case HOM4D_ESTATE: return "call out of order";
        case HOM4D_ENOMEM: return "buffer too small or allocation failed";
        case HOM4D_EHIP: return "HIP runtime error";
        case HOM4D_ENONFINITE: return "non-finite state";
        case HOM4D_ENORMDRIFT: return "norm drift beyond tolerance";
        case HOM4D_ECONFIG: return "checkpoint from another configuration";
        case HOM4D_ECORRUPT: return "checkpoint corrupted";
        default: return "unknown status";
    }
}

const char* hom4d_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
