/*
 * hom4d.h -- C ABI of the MI355X (gfx950) two-electron split-step propagator.
 *
 * The library advances the exact two-electron wavefunction Psi(x1, y1, x2, y2)
 * of a Hall-edge Hong-Ou-Mandel interferometer on a 4D grid, as in
 * L. Bellentani, P. Bordone, X. Oriols, A. Bertoni, arXiv 1903.02581:
 *   - Sec. II.C, Eq. (evoloperat) and Appendix A: split-step Fourier method for
 *     two particles in a perpendicular field, kinetic terms diagonal in mixed
 *     real/reciprocal representations, potentials diagonal in 4D real space;
 *   - Sec. III.B, Eq. (coulomb) / Eq. (screenedCoulomb): the two-body term;
 *   - Sec. III, Eq. (p_bunching): region-resolved (bunching) probabilities;
 *   - Sec. III.C, Eq. (reduced_density): spatial entanglement of 1D slices.
 *
 * Conventions (readings where the paper is silent, fixed here):
 *   - units nm, fs, meV, tesla; electron charge -e; gauge A = (-B y, 0), so the
 *     x kinetic term is (hbar k_x - e B y)^2 / 2m*, diagonal in (k_x, y), and
 *     the y kinetic term hbar^2 k_y^2 / 2m*, diagonal in k_y;
 *   - grids x_i = -Lx/2 + i Lx/nx, y_j = -Ly/2 + j Ly/ny, periodic; forward DFT
 *     exp(-i k x); wave number index m >= n/2 maps to m - n (Nyquist = -pi/dx);
 *   - one step is the symmetric product S(dt) = X(dt/2) V(dt/2) Y(dt) V(dt/2) X(dt/2)
 *     with V = V(r1) + V(r2) + V12(r1, r2); consecutive X halves are merged
 *     inside one hom4d_step call, which always ends on a whole step;
 *   - V12 = C e^2 / (4 pi eps0 eps_r sqrt(|r1 - r2|^2 + d^2)), times
 *     exp(-|r1 - r2| / sigma_c) when screen_nm = sigma_c > 0;
 *   - canonical state layout: row-major [x1][y1][x2][y2] of interleaved
 *     complex (re, im); the device state uses the same layout, in complex128
 *     (HOM4D_FP64) or complex64 (HOM4D_MIXED) storage.  All arithmetic --
 *     transforms, phase products, potential angles, reductions -- is FP64 in
 *     both precisions; HOM4D_MIXED only rounds the stored state to FP32.
 *
 * Ownership: host arrays are owned by the caller and copied during the call.
 * The state buffer (and the adjoint and checkpoint buffers) are device memory
 * owned by the caller (typically torch tensors); the library keeps only the
 * pointer while bound.  The handle owns O(nx*ny) tables and small reduction
 * scratch.  All device work is enqueued on the HIP stream given at create
 * time; calls that return host results synchronise that stream.
 *
 * Errors: every call returns 0 (HOM4D_OK) or a negative HOM4D_E* code and
 * never throws across the ABI.  hom4d_last_error() gives a thread-local
 * detail string for the last failing call on this thread.
 */
#ifndef HOM4D_H
#define HOM4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOM4D_OK 0
#define HOM4D_EINVAL (-1)      /* bad argument: size, pointer, flag, step count */
#define HOM4D_EUNBOUND (-2)    /* no state buffer bound */
#define HOM4D_ESTATE (-3)      /* call out of order (e.g. backward without a recorded forward) */
#define HOM4D_ENOMEM (-4)      /* caller-provided buffer too small, or a table allocation failed */
#define HOM4D_EHIP (-5)        /* HIP runtime error; detail in hom4d_last_error() */
#define HOM4D_ENONFINITE (-6)  /* the state holds a NaN or Inf */
#define HOM4D_ENORMDRIFT (-7)  /* |norm - 1| above the watchdog tolerance */
#define HOM4D_ECONFIG (-8)     /* checkpoint image taken with another configuration */
#define HOM4D_ECORRUPT (-9)    /* checkpoint image fails its checksum or norm check */

#define HOM4D_FP64 0           /* complex128 state */
#define HOM4D_MIXED 1          /* complex64 state, FP64 arithmetic */

#define HOM4D_COULOMB_TABLE 0  /* V12 phase from a device table over (x1-x2, y1-y2) */
#define HOM4D_COULOMB_DIRECT 1 /* V12 angle evaluated per 4D point on the fly */

typedef struct hom4d hom4d;

/* Problem definition.  nx, ny: grid points per electron, each of the form
 * 2^a 3^b in {4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256}.  Lengths in nm,
 * dt in fs, B in tesla (Appendix A: field along +z), soft_nm = d and
 * coulomb_c = C of Eq. (coulomb) (C = 0 switches the two-body term off),
 * screen_nm = sigma_c of Eq. (screenedCoulomb) (0 = unscreened). */
typedef struct {
    int32_t nx, ny;
    int32_t precision;      /* HOM4D_FP64 or HOM4D_MIXED */
    int32_t coulomb_mode;   /* HOM4D_COULOMB_TABLE or HOM4D_COULOMB_DIRECT */
    double lx_nm, ly_nm;
    double mstar_rel;       /* m* / m_e (GaAs: 0.067) */
    double eps_r;           /* relative permittivity (GaAs: 12.9) */
    double b_tesla;
    double dt_fs;
    double soft_nm;
    double coulomb_c;
    double screen_nm;
} hom4d_cfg;

/* Region-resolved probabilities of Eq. (p_bunching) as raw grid sums of
 * |Psi|^2 weighted by w(r1), w(r2) (T) and 1 - w (B); p_b = p_tt + p_bb,
 * p_ab = p_tb + p_bt; norm = sum |Psi|^2.  step counts whole steps taken
 * since the last init/load. */
typedef struct {
    double norm, p_tt, p_tb, p_bt, p_bb, p_b, p_ab;
    int64_t step;
} hom4d_obs;

/* Validate cfg, build the phase and twiddle tables and upload them.
 * hip_stream: a hipStream_t (NULL = the null stream).  On success *out owns
 * the handle.  EINVAL on an unsupported size or a non-positive length / dt /
 * mass / permittivity / softening; EHIP if no device is usable. */
int hom4d_create(const hom4d_cfg* cfg, void* hip_stream, hom4d** out);

/* Release the handle and its tables (not the bound caller buffers). */
int hom4d_destroy(hom4d* h);

/* Checks cfg without touching the GPU; returns HOM4D_OK or HOM4D_EINVAL. */
int hom4d_validate_cfg(const hom4d_cfg* cfg);

/* Bytes of one device state buffer for cfg: (nx*ny)^2 * (16 or 8); 0 if cfg is invalid. */
size_t hom4d_state_bytes(const hom4d_cfg* cfg);

/* Bind the caller-owned device state buffer (hom4d_state_bytes bytes, 16-byte
 * aligned).  Rebinding discards any gradient recording. */
int hom4d_bind_state(hom4d* h, void* d_psi);

/* External potential V(x, y) in meV, host row-major [nx][ny] FP64: the
 * one-body terms V(r1) + V(r2) of the two-particle Hamiltonian of Appendix A
 * (the same confinement and beam-splitter potential for both electrons,
 * Sec. II.B, Eq. (pot_x) / Eq. (pot_xy)), entering the real-space factor of
 * Eq. (evoloperat).  Rebuilds the potential phase tables and discards any
 * gradient recording (its forward run used the old factors).  EINVAL on a
 * NULL pointer or a non-finite entry. */
int hom4d_set_potential(hom4d* h, const double* v_meV);

/* Change B (tesla), the perpendicular field of Sec. II.A and Appendix A.  In
 * the Landau gauge A = (-B y, 0) it enters only the x kinetic term
 * (hbar k_x - e B y)^2 / 2m*, so this rebuilds the x kinetic phase tables and
 * discards any gradient recording.  EINVAL on a non-finite B. */
int hom4d_set_field(hom4d* h, double b_tesla);

/* Initial state of Sec. II.C Eq. (twopstate) from two single-electron
 * orbitals, host row-major [nx][ny] interleaved complex128:
 *   sym = -1: psi_a(r1) psi_b(r2) - psi_a(r2) psi_b(r1) (Slater determinant),
 *   sym = +1: the symmetric combination, sym = 0: the product psi_a(r1) psi_b(r2);
 * then normalised so that the 4D grid sum of |Psi|^2 is 1 (FP64 norm).
 * EINVAL on another sym or a zero-norm combination.  Resets the step count. */
int hom4d_init_state(hom4d* h, const double* psi_a, const double* psi_b, int32_t sym);

/* Copy a canonical complex128 state in/out (host, (nx*ny)^2 complex values).
 * load resets the step count; in MIXED the values are rounded to complex64. */
int hom4d_load_state(hom4d* h, const double* psi4d);
int hom4d_store_state(hom4d* h, double* psi4d);

/* Measurement: per-pass kernel timing on the stream.  enable = 1 discards
 * earlier records and brackets every pass kernel launched afterwards by a HIP
 * event pair; 0 stops recording.  hom4d_pass_times synchronises and returns,
 * per pass kind (0 x1, 1 y1, 2 x2, 3 y2, 4 the fused (x2, y2) plane pass), the
 * summed event-to-event time in ms and the number of launches (host arrays of
 * 5); reading does not reset them.  A pool of 8192 events is created at the
 * first timed launch and kept until hom4d_destroy: while timing is on, every
 * 4096 launches the stream is synchronised and the pending pairs are folded
 * into the sums, so memory stays bounded over any number of steps.  The event
 * records add a little time between kernels, so a run that measures the step
 * rate leaves timing off. */
int hom4d_pass_timing(hom4d* h, int32_t enable);
int hom4d_pass_times(hom4d* h, double* ms, int64_t* count);

/* Checkpoint images for resuming a long run (not an operation of the paper:
 * its propagations take thousands of steps, Sec. III).  An image is a 64-byte
 * header -- magic "HOM4DCK1", version 1, precision, nx, ny, step count, a
 * 64-bit hash of the configuration fields, the current B and the potential
 * table, the payload size, a Fletcher-style checksum of the payload and the
 * FP64 norm of the state -- followed by the state in its storage precision
 * ([x1][y1][x2][y2], complex128 or complex64, bit for bit).  The buffer is
 * caller-owned host memory of hom4d_checkpoint_bytes(h) bytes (0 for a NULL
 * handle).  save: ENOMEM if the buffer is smaller, ENONFINITE if the state is
 * not finite; synchronises.  load: EINVAL if the buffer is not an image or is
 * truncated, ECONFIG if it was taken with another size, precision,
 * configuration, field or potential (the bound state is then untouched),
 * ECORRUPT if the payload fails its checksum (untouched) or the norm
 * recomputed on the GPU after the copy differs from the recorded one by more
 * than 1e-12 relative (the state is then the damaged copy); on success the
 * state and the step count are the saved ones and any gradient recording is
 * discarded.  Synchronises. */
size_t hom4d_checkpoint_bytes(const hom4d* h);
int hom4d_save_checkpoint(hom4d* h, void* buf, size_t bytes);
int hom4d_load_checkpoint(hom4d* h, const void* buf, size_t bytes);

/* Advance the bound state by n >= 0 whole steps of the split-step Fourier
 * propagator of Sec. II.C, Eq. (evoloperat) and Appendix A: each step is
 * S(dt) = X(dt/2) V(dt/2) Y(dt) V(dt/2) X(dt/2), with X and Y the kinetic
 * factors of the two electrons (diagonal in (k_x, y) and k_y) and V the
 * one-body potentials plus the two-body term of Eq. (coulomb) /
 * Eq. (screenedCoulomb), diagonal in 4D real space.  Asynchronous on the
 * stream.  EUNBOUND without a state, ESTATE without a potential.  While a
 * gradient recording is open it also stores the checkpoints; a call whose
 * checkpoints would not fit the pool returns ENOMEM before taking any step
 * (state, step count and recording unchanged), and a failure part way closes
 * the recording. */
int hom4d_step(hom4d* h, int64_t n);

/* Region-resolved probabilities of the bound state for the top-region weight
 * table w_top (host [nx][ny] FP64, values in [0, 1]).  Synchronises.
 * Returns ENONFINITE if the state holds a NaN/Inf, ENORMDRIFT if
 * |norm - 1| > norm_tol (set with hom4d_set_norm_tol; default 1e-6);
 * *out is filled in either case. */
int hom4d_observables(hom4d* h, const double* w_top, hom4d_obs* out);
int hom4d_set_norm_tol(hom4d* h, double tol);

/* Von Neumann entropy of the slice phi(a, b) = Psi(ix1[a], jy1, ix2[b], jy2)
 * (Sec. III.C): phi is renormalised, rho = phi phi^dagger, S = -Tr rho ln rho
 * (natural log).  1 <= n1, n2 <= 256; indices in range.  Synchronises. */
int hom4d_entanglement(hom4d* h, const int32_t* ix1, int32_t n1, int32_t jy1,
                       const int32_t* ix2, int32_t n2, int32_t jy2, double* s_out);

/* Unconditional (marginal) probability of electron 1 (Sec. III.A, Fig. 3(b)
 * caption): out[x1][y1] = sum over (x2, y2) of |Psi(x1, y1, x2, y2)|^2, host
 * [nx][ny] FP64, FP64 accumulation in a fixed order.  Synchronises. */
int hom4d_marginal(hom4d* h, double* out);

/* Conditional probability of electron 1 with electron 2 at the grid point
 * (ix2, jy2) (Sec. II.A, Fig. 2 caption): out[x1][y1] = |Psi(x1, y1, ix2, jy2)|^2,
 * host [nx][ny] FP64, not renormalised.  EINVAL on an index out of range.
 * Synchronises. */
int hom4d_conditional(hom4d* h, int32_t ix2, int32_t jy2, double* out);

/* One electron's Gaussian edge-state wave packet on the handle's grid, the
 * input of hom4d_init_state (Sec. II.A, Eq. (H_effective); Sec. II.B,
 * Eq. (singlepwp)).  For every grid wave number k along x the lowest
 * eigenpair of the transverse Hamiltonian
 *     H(k) = kappa [ -d^2/dy^2 + (k - y eB/hbar)^2 ] + v_col(y)
 * (gauge A = (-B y, 0), second derivative spectral on the periodic y grid) is
 * found on the GPU (Jacobi, FP64), its sign fixed so that the largest-magnitude
 * component is positive; k0 is the wave number, among k > 0 (top = 1) or k < 0
 * (top = 0), whose level is closest to hbar omega_c / 2 + e_above_lll_mev; and
 *     psi(x, y) = sum_k exp(-sigma_x^2 (k - k0)^2) exp(i k (x - xc)) phi_k(y),
 * normalised on the grid.  v_col: host [ny] FP64 meV (the potential across the
 * edge where the packet starts), copied.  psi_out: host [nx][ny] interleaved
 * complex128.  info_out (may be NULL): host double[3] = (k0 in 1/nm, its level
 * in meV, the target level in meV).  The handle's state is not touched.  EINVAL
 * on NULL pointers, sigma_x <= 0, non-finite inputs or top not 0/1; EHIP
 * (allocates a work buffer of 2 nx ny^2 doubles for the call).  Synchronises. */
int hom4d_edge_packet(hom4d* h, const double* v_col, double sigma_x_nm, double xc_nm, int32_t top,
                      double e_above_lll_mev, double* psi_out, double* info_out);

/* Gather the (n1 x n2) slice above into host memory (interleaved complex128),
 * unnormalised.  Synchronises. */
int hom4d_gather_slice(hom4d* h, const int32_t* ix1, int32_t n1, int32_t jy1,
                       const int32_t* ix2, int32_t n2, int32_t jy2, double* out);

/* Start recording a forward run for the adjoint (the reverse-mode derivative
 * of the bunching probability of Eq. (p_bunching) through the unitary steps of
 * Eq. (evoloperat); not an operation of the paper itself).  The current bound
 * state is checkpoint 0; every ckpt_every steps taken by later hom4d_step calls
 * the state is copied into the caller-owned device pool (pool_bytes bytes,
 * slots of hom4d_state_bytes).  hom4d_step returns ENOMEM, without stepping,
 * when a checkpoint it would reach does not fit.  EINVAL on ckpt_every < 1 or
 * a NULL pool, ENOMEM if the pool is smaller than one state. */
int hom4d_grad_begin(hom4d* h, int32_t ckpt_every, void* d_pool, size_t pool_bytes);

/* Reverse sweep for L = sum w_L |Psi_N|^2 with
 * w_L = c[0] w1 w2 + c[1] w1 (1-w2) + c[2] (1-w1) w2 + c[3] (1-w1)(1-w2)
 * (c = {1,0,0,1}: the bunching probability).  d_lambda: caller-owned device
 * buffer of hom4d_state_bytes for the adjoint state.  The state and the
 * adjoint are carried back together by S(-dt); at every checkpoint the state
 * is replaced by the stored copy (bounds the reverse drift).  Outputs:
 * *loss = L, dL_dV (host [nx][ny] FP64, derivative with respect to the
 * potential table in 1/meV), *dL_dB (1/T).  On return the bound state holds
 * checkpoint 0 and the recording is closed.  ESTATE without a recording or
 * when the recorded checkpoints exceed the pool. */
int hom4d_grad_backward(hom4d* h, const double* w_top, const double* coeffs,
                        void* d_lambda, double* loss, double* dL_dV, double* dL_dB);

/* hom4d_grad_backward for callers that cannot allocate device memory: code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors, bit for bit the same outputs; it calls
 * no hipMalloc, hipFree or allocating library routine.  The reverse sweep's
 * FP64 partial sums go to a fixed 64 MiB array in device memory instead of a
 * buffer the handle allocates on first use: one copy per GPU, shared by every
 * handle on that GPU, its address taken by hom4d_create, kept until the
 * process ends, cleared (by a fill kernel) at the start of every call.  Calls
 * that overlap on one GPU race on it.  ENOMEM when the partial sums of the
 * handle's grid exceed the array (8M doubles: grids up to 128x128 per
 * electron fit, 256x128 does not); ESTATE also while pass timing is on (its
 * event pool is created on demand). */
int hom4d_grad_backward_noalloc(hom4d* h, const double* w_top, const double* coeffs, void* d_lambda,
                                double* loss, double* dL_dV, double* dL_dB);

/* Abandon an open recording. */
int hom4d_grad_end(hom4d* h);

/* Pass plan.  plan = 0 (default): where a fused kernel is built for (nx, ny)
 * and the precision, one step is three state passes -- x1 line transforms;
 * the (x2, y2) plane of each r1 with X2, V and Y2 fused; y1 line transforms
 * with V fused.  plan = 1: four per-axis passes (x1; x2 then V; y1; y2 then V).
 * Both apply the same factors in the same order (Sec. II.C Eq. (evoloperat)).
 * The reverse (adjoint) sweep always uses the per-axis passes.
 * hom4d_pass_plan returns the number of passes per step in use (3 or 4). */
int hom4d_set_pass_plan(hom4d* h, int32_t plan);
int hom4d_pass_plan(hom4d* h);

/* Measurement entry point: launch one pass kernel reps times on the bound
 * state, asynchronously.  axis: 0 = x1, 1 = y1, 2 = x2 then potential factor,
 * 3 = y2 then potential factor -- the kernels of the four-pass plan (kinetic
 * factors of a full dt); 4 = the fused (x2, y2) plane pass and 5 = y1 then
 * potential factor -- the kernels of the three-pass plan (with 0).  Each
 * launch applies a unitary factor, so the state stays normalised but no
 * longer follows the step sequence; the step count is not changed. */
int hom4d_run_pass(hom4d* h, int32_t axis, int32_t reps);

/* Static string for a status code. */
const char* hom4d_strerror(int status);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char* hom4d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HOM4D_H */
