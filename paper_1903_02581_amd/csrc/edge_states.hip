// Edge states and Gaussian edge-state wave packets on the GPU: the one-electron
// inputs of the two-electron propagation (arXiv 1903.02581 Sec. II.A,
// Eq. (H_effective); Sec. II.B, Eq. (singlepwp)).
//
// In the gauge A = (-B y, 0) an electron with wave number k along x sees the
// transverse Hamiltonian
//     H(k) = kappa [ -d^2/dy^2 + (k - y eB/hbar)^2 ] + v(y),
// with the second derivative spectral on the periodic y grid: the circulant
// matrix c[(i - j) mod ny], c[d] = (kappa / ny) sum_m ky_m^2 cos(2 pi m d / ny),
// whose first row the host computes.  k_edge_jacobi diagonalises H(k) for every
// grid k (one workgroup per k) by the cyclic Jacobi method with the round-robin
// ordering of disjoint index pairs: each of the ny - 1 steps of a sweep rotates
// ny / 2 disjoint (p, q) planes at once, the angles all taken from the matrix
// before the step, then applied to the rows (J^T A), then to the columns (A J)
// and to the accumulated eigenvectors (V J).  Sweeps repeat until the
// off-diagonal part stops shrinking at rounding level.  The lowest diagonal
// entry and its column of V are the edge state, its sign fixed so that the
// largest-magnitude component is positive.
//
// k_edge_sum forms psi(x_i, y_j) = sum_m exp(-sigma^2 (k_m - k0)^2)
// exp(i k_m (x_i - xc)) phi_m(y_j) with the m sum in grid order, where k0 is the
// grid wave number (on the requested side: k > 0 for the top edge, k < 0 for the
// bottom) whose edge-state energy is closest to hbar omega_c / 2 + e_above;
// k_edge_scale normalises it on the grid.  All arithmetic is FP64; the matrices
// live in a device work buffer of 2 nx ny^2 doubles.
#include "hom4d_internal.hpp"

namespace hom4d_impl {
namespace {

constexpr int kEdgeThreads = 256;
constexpr int kEdgeMaxSweeps = 40;

// sums of two values over the block, valid in every thread
__device__ void block_sum2(double& a, double& b, double* red) {
    const int tid = threadIdx.x, nw = blockDim.x / 64;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    __syncthreads();
    if ((tid & 63) == 0) {
        red[2 * (tid >> 6)] = a;
        red[2 * (tid >> 6) + 1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < nw; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kEdgeThreads) k_edge_jacobi(const double* circ, const double* vcol, const double* kx,
                                                              int ny, double kappa, double inv_lb2, double y0,
                                                              double dy, double* work, double* e1, double* phi) {
    const int m = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double k = kx[m];
    double* A = work + (size_t)m * 2 * ny * ny;
    double* V = A + (size_t)ny * ny;
    __shared__ int sp[128], sq[128];
    __shared__ double sc[128], ss[128];
    __shared__ double red[2 * (kEdgeThreads / 64)];
    __shared__ int s_min, s_sign;

    for (int idx = tid; idx < ny * ny; idx += nt) {
        const int i = idx / ny, j = idx % ny;
        double a = circ[(i - j + ny) % ny];
        if (i == j) {
            const double u = k - (y0 + dy * i) * inv_lb2;
            a += kappa * u * u + vcol[i];
        }
        A[idx] = a;
        V[idx] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();

    const int half = ny / 2;
    double prev_off = -1.0;
    for (int sweep = 0; sweep < kEdgeMaxSweeps; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int idx = tid; idx < ny * ny; idx += nt) {
            const double a = A[idx];
            tot += a * a;
            if (idx / ny != idx % ny) off += a * a;
        }
        block_sum2(off, tot, red);
        // converged, or stalled at rounding level: quadratic convergence would
        // have shrunk it by far more than a factor 4, and a stall counts only once
        // the off-diagonal part is already small (where the sweeps stall, rounding
        // leaves 2e-33 to 7e-33 of the total at ny = 64 and 256), not during the
        // slower first sweeps
        if (off == 0.0 || off <= 1e-32 * tot ||
            (sweep > 3 && prev_off >= 0.0 && off > 0.25 * prev_off && off <= 1e-24 * tot))
            break;
        prev_off = off;
        for (int r = 0; r < ny - 1; ++r) {
            if (tid < half) {
                // round robin: index ny - 1 meets r, and (r + i, r - i) mod (ny - 1) meet
                int p, q;
                if (tid == 0) {
                    p = r;
                    q = ny - 1;
                } else {
                    p = (r + tid) % (ny - 1);
                    q = (r - tid + (ny - 1)) % (ny - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const double apq = A[p * ny + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    // tan of the angle that zeroes a_pq: the smaller root of t^2 + 2 theta t - 1 = 0
                    const double theta = (A[q * ny + q] - A[p * ny + p]) / (2.0 * apq);
                    const double at = fabs(theta);
                    double t = (at > 1e150) ? 0.5 / at : 1.0 / (at + sqrt(at * at + 1.0));
                    if (theta < 0.0) t = -t;
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                }
                sp[tid] = p;
                sq[tid] = q;
                sc[tid] = c;
                ss[tid] = s;
            }
            __syncthreads();
            for (int w = tid; w < half * ny; w += nt) {  // rows p, q of J^T A
                const int i = w / ny, j = w % ny;
                const int p = sp[i], q = sq[i];
                const double c = sc[i], s = ss[i];
                const double x = A[p * ny + j], y = A[q * ny + j];
                A[p * ny + j] = c * x - s * y;
                A[q * ny + j] = s * x + c * y;
            }
            __syncthreads();
            for (int w = tid; w < half * ny; w += nt) {  // columns p, q of (J^T A) J and V J
                const int i = w / ny, j = w % ny;
                const int p = sp[i], q = sq[i];
                const double c = sc[i], s = ss[i];
                const double x = A[j * ny + p], y = A[j * ny + q];
                A[j * ny + p] = c * x - s * y;
                A[j * ny + q] = s * x + c * y;
                const double vx = V[j * ny + p], vy = V[j * ny + q];
                V[j * ny + p] = c * vx - s * vy;
                V[j * ny + q] = s * vx + c * vy;
            }
            __syncthreads();
        }
    }

    if (tid == 0) {
        int b = 0;
        for (int i = 1; i < ny; ++i)
            if (A[i * ny + i] < A[b * ny + b]) b = i;
        int jm = 0;
        for (int j = 1; j < ny; ++j)
            if (fabs(V[j * ny + b]) > fabs(V[jm * ny + b])) jm = j;
        s_min = b;
        s_sign = V[jm * ny + b] < 0.0 ? -1 : 1;
        e1[m] = A[b * ny + b];
    }
    __syncthreads();
    for (int j = tid; j < ny; j += nt) phi[(size_t)m * ny + j] = s_sign * V[j * ny + s_min];
}

// block i: the row x_i of the packet, thread j: y_j
__global__ void k_edge_sum(const double* kx, const double* e1, const double* phi, int nx, int ny, int top,
                           double target, double sigma, double xc, double x0, double dx, double2* psi,
                           double* part, double* info) {
    __shared__ int s_i0;
    __shared__ double s_n2[256];
    const int i = blockIdx.x, j = threadIdx.x;
    if (j == 0) {
        // first grid index on the requested side whose level is closest to the target
        int best = -1;
        for (int m = 0; m < nx; ++m) {
            const bool side = top ? (kx[m] > 0.0) : (kx[m] < 0.0);
            if (!side) continue;
            if (best < 0 || fabs(e1[m] - target) < fabs(e1[best] - target)) best = m;
        }
        if (best < 0) best = 0;  // not reached: every supported nx has wave numbers of both signs
        s_i0 = best;
        if (i == 0) {
            info[0] = kx[best];
            info[1] = e1[best];
            info[2] = target;
        }
    }
    __syncthreads();
    const double k0 = kx[s_i0];
    const double x = x0 + dx * i;
    double re = 0.0, im = 0.0;
    for (int m = 0; m < nx; ++m) {
        const double d = kx[m] - k0;
        const double amp = exp(-sigma * sigma * d * d);
        double sn, cs;
        sincos(kx[m] * (x - xc), &sn, &cs);
        const double f = amp * phi[(size_t)m * ny + j];
        re += f * cs;
        im += f * sn;
    }
    psi[(size_t)i * ny + j] = make_double2(re, im);
    s_n2[j] = re * re + im * im;
    __syncthreads();
    if (j == 0) {  // the row's squared modulus, summed in y order
        double t = 0.0;
        for (int q = 0; q < ny; ++q) t += s_n2[q];
        part[i] = t;
    }
}

__global__ void k_edge_scale(double2* psi, const double* part, int nx, int ny) {
    __shared__ double s_inv;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < nx; ++i) t += part[i];
        s_inv = 1.0 / sqrt(t);
    }
    __syncthreads();
    const size_t idx = (size_t)blockIdx.x * ny + threadIdx.x;
    const double2 v = psi[idx];
    psi[idx] = make_double2(v.x * s_inv, v.y * s_inv);
}

}  // namespace

hipError_t launch_edge_packet(const EdgeArgs& e, hipStream_t s) {
    // even ny (the round-robin pairs), at most 256 (one thread per y in the packet kernels)
    if (e.nx <= 0 || e.ny < 4 || e.ny > 256 || (e.ny % 2) != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_edge_jacobi, dim3(e.nx), dim3(kEdgeThreads), 0, s, e.circ, e.vcol, e.kx, e.ny, e.kappa,
                       e.inv_lb2, e.y0, e.dy, e.work, e.e1, e.phi);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_edge_sum, dim3(e.nx), dim3(e.ny), 0, s, e.kx, e.e1, e.phi, e.nx, e.ny, e.top, e.target,
                       e.sigma, e.xc, e.x0, e.dx, e.psi, e.part, e.info);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_edge_scale, dim3(e.nx), dim3(e.ny), 0, s, e.psi, e.part, e.nx, e.ny);
    return hipGetLastError();
}

}  // namespace hom4d_impl
