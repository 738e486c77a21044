/*
 * dmdmi.h - C ABI of the MI355X (gfx950) DMD hot path.
 *
 * Method: Dynamic Mode Decomposition as used by Chen et al., "Fast Subspace
 * Fluid Simulation with a Temporally-Aware Basis" (ACM TOG 2025):
 *   - snapshot pair X = [u_0 .. u_{T-1}], X' = [u_1 .. u_T]     (Sec. 3.1, eq. reduced_koopman)
 *   - K = X' V S^-1 U^T from the thin SVD X = U S V^T, truncated to rank r,
 *     reduced operator Atilde = U_r^T X' V_r S_r^-1, its eigen-decomposition
 *     Atilde W = W Lambda                                        (Sec. 3.1, eq. reduced_koopman_solution)
 *   - randomized SVD: X ~ Q Q^T X, B = Q^T X, SVD of the small B (Sec. 4.3)
 *   - amplitudes z = Phi^+ u                                     (Sec. 3.1, eq. projection)
 *   - u(t + k dt) = Phi Lambda^k z(t) in one product             (Sec. 4.4, eq. large_time_step)
 *   - u(t) = Phi exp(Omega t) z with Omega = Log(Lambda)/dt      (Sec. 6.1, eq. edit_temporal)
 *   - Lambda^-1 runs the reduced model backwards                 (Sec. 6.2, eq. reverse_simulation)
 *
 * Conventions shared by every call
 *   - All device memory (inputs, outputs, model arrays, workspace) is owned by
 *     the caller.  The library never allocates or frees device memory; each
 *     call that needs scratch memory has a *_workspace_size query.
 *   - `stream` is a hipStream_t passed as void*.  Every call only enqueues work
 *     on that stream, except dmd_fit without DMD_FIT_ASYNC, which waits for the
 *     stream to reach the end of the fit and returns the fit's device status.
 *   - Host arrays are borrowed for the duration of the call only.
 *   - Inputs are never modified.
 *   - Matrices are column-major unless stated otherwise; leading dimensions and
 *     sizes are 64-bit and counted in elements.
 *   - Errors: every call returns a dmd_status.  Argument validation happens on
 *     the host before any HIP call; on error nothing is enqueued.  Errors found
 *     on the device during a fit (Cholesky breakdown, rank loss, eigen-solver
 *     non-convergence) are written to model->info[0] and returned by the
 *     synchronous dmd_fit.  Domain and overflow errors of the powers lambda^k
 *     (evaluation calls) are written to a status word at the start of the
 *     call's workspace, read by dmd_status_word.  No exception or exit() crosses
 *     the ABI.  On error the outputs are unspecified and nothing leaks.
 *
 * Model storage (real "folded" modes).  For real snapshots the DMD eigenvalues
 * and modes come in exact complex-conjugate pairs.  The model stores each pair
 * (phi, conj(phi)) as two real columns [Re phi, Im phi] and each real mode as
 * one real column, the storage LAPACK uses for real eigenvectors.  kind[i] = 0
 * marks a real mode, kind[i] = 1 / kind[i+1] = 2 a conjugate pair whose complex
 * modes are phi_i = P[:, i] + 1j P[:, i+1] and phi_{i+1} = conj(phi_i).
 * lam[] and b[] hold all r complex values (both members of each pair), so
 * they can be edited independently; Re() of the mode sum is always taken.
 * Mode order: ascending |arg lambda|, ties by descending |lambda|, the member
 * with Im lambda > 0 first (the paper orders modes by the size of their
 * imaginary part, Sec. 6.3.1).
 */
#ifndef DMDMI_H
#define DMDMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DMDMI_ABI_VERSION 3

/* Status codes. */
typedef enum dmd_status {
    DMD_OK = 0,
    DMD_ERR_ARG = 1,            /* null pointer, bad enum, misaligned pointer or leading dimension */
    DMD_ERR_SHAPE = 2,          /* r > m-1, l > m-1, l > N, K <= 0, ... */
    DMD_ERR_WORKSPACE = 3,      /* workspace smaller than the *_workspace_size query */
    DMD_ERR_NONFINITE = 4,      /* NaN or Inf in the input (only with DMD_FIT_CHECK_FINITE) */
    DMD_ERR_CHOL_BREAKDOWN = 5, /* CholeskyQR failed even after the shifted retry */
    DMD_ERR_RANK = 6,           /* sigma_r <= rank_tol * sigma_1 */
    DMD_ERR_EIG_NOCONV = 7,     /* an eigenvalue iteration reached its limit */
    DMD_ERR_DOMAIN = 8,         /* lambda = 0 raised to a negative or fractional power (device
                                   status word, see dmd_status_word) */
    DMD_ERR_OVERFLOW = 9,       /* |b| |lambda|^k beyond the output type's finite range (device
                                   status word, see dmd_status_word) */
    DMD_ERR_HIP = 10,           /* a HIP runtime call failed */
    DMD_ERR_UNSUPPORTED = 11,   /* size beyond what a single-workgroup small-matrix kernel holds */
    DMD_ERR_IO = 12             /* model file missing, unwritable, truncated or failing its checks */
} dmd_status;

/* Element types. */
typedef enum dmd_dtype { DMD_F32 = 0, DMD_F64 = 1 } dmd_dtype;

/* Fit precision. */
typedef enum dmd_fit_precision {
    /* Randomized SVD; FP32 streaming GEMMs (MFMA, FP32 accumulate); FP64 Gram
     * products, Cholesky, small SVD, eigen-decomposition; FP32 modes. X is FP32. */
    DMD_FIT_MIXED = 0,
    /* The same randomized algorithm entirely in FP64 (the plain path). X is FP64. */
    DMD_FIT_FP64_RANDOMIZED = 1,
    /* Exact thin SVD of X (no sketch; Sec. 3.1), X FP64, m-1 <= DMD_MAX_SMALL.  For
     * m-1 <= DMD_EXACT_QR_MAX through a triangular factor: Q R = [X X'] by shifted
     * CholeskyQR in FP64, then the singular values and right vectors of R from the
     * symmetric eigen-decomposition of [[0, R], [R^T, 0]] (relative accuracy u kappa for
     * the small singular values; the workspace holds an N x m FP64 copy of the snapshots).
     * Above it, through the FP64 Gram of the snapshots (method of snapshots), which
     * squares the condition number. */
    DMD_FIT_FP64_EXACT = 2
} dmd_fit_precision;

/* Reconstruction arithmetic. */
typedef enum dmd_recon_mode {
    DMD_RECON_FP64 = 0,   /* FP64 modes, FP64 MFMA, FP64 output */
    DMD_RECON_FP32 = 1,   /* FP32 modes, FP32 MFMA, FP32 output */
    DMD_RECON_BF16 = 2,   /* modes and coefficients rounded to BF16, FP32 accumulate/output */
    DMD_RECON_BF16X3 = 3  /* split-BF16 (hi+lo, three products), FP32 accumulate/output */
} dmd_recon_mode;

/* Limits of the single-workgroup FP64 kernels (packed matrices held in LDS).  A fit
 * beyond them returns DMD_ERR_UNSUPPORTED. */
#define DMD_MAX_SMALL 192   /* m-1 for DMD_FIT_FP64_EXACT (symmetric eigen-solver) */
#define DMD_EXACT_QR_MAX 96 /* m-1 up to which DMD_FIT_FP64_EXACT takes the triangular-factor
                               route (the symmetric solver takes 2(m-1) <= DMD_MAX_SMALL) */
#define DMD_MAX_SKETCH 160  /* l = r + p on the randomized paths (Cholesky of the l x l Gram) */
#define DMD_MAX_RANK 160    /* r (nonsymmetric eigen-solver) */

/* Fit flags. */
#define DMD_FIT_ASYNC 1u         /* do not wait for the stream; status stays in model->info[0] */
#define DMD_FIT_CHECK_FINITE 2u  /* scan X and X' for NaN/Inf first */
#define DMD_FIT_OPTDMD 4u        /* OptDMD (Sec. 4.2): refine lambda and the modes by variable
                                    projection on all snapshots of X (eq. variable_projection,
                                    eq. phi_optdmd), starting from the fit's eigenvalues, by
                                    Levenberg-Marquardt steps decided on the device.  Without
                                    DMD_FIT_ASYNC the call runs the iteration to its stopping
                                    rule (it reads a device flag after every 8 trial points);
                                    with DMD_FIT_ASYNC, and in dmd_fit_batched, it enqueues
                                    opts.optdmd_trials trial points (a fixed launch sequence
                                    that can be captured; trial points after the stop cost
                                    their launches only).  info[4..6] report the outcome */
#define DMD_MAX_OPTDMD_TRIALS 100000

/* Options of a fit. */
typedef struct dmd_fit_opts {
    int32_t r;          /* rank (number of modes), 1 <= r */
    int32_t p;          /* oversampling, l = r + p columns in the sketch (randomized) */
    int32_t q;          /* power iterations (randomized), >= 0 */
    int32_t precision;  /* dmd_fit_precision */
    double dt;          /* time between snapshots (> 0), stored in the model */
    double rank_tol;    /* > 0: fail with DMD_ERR_RANK when sigma_r <= rank_tol * sigma_1 */
    const void* omega;  /* device (m-1) x l Gaussian sketch, column-major, ld = m-1, same
                           element type as X; NULL for DMD_FIT_FP64_EXACT.  The sketch is an
                           input so that a reference implementation can use the same draw. */
    uint32_t flags;     /* DMD_FIT_* */
    int32_t optdmd_trials;  /* DMD_FIT_OPTDMD with DMD_FIT_ASYNC or in dmd_fit_batched: trial
                               points enqueued (0: 64); 0 <= optdmd_trials <=
                               DMD_MAX_OPTDMD_TRIALS, else DMD_ERR_ARG; otherwise unused */
} dmd_fit_opts;

/* Number of int32 words in model->info. */
#define DMD_INFO_WORDS 8
/* info[0] status, [1] bisection rounds of the symmetric eigenvalues, [2] Ehrlich-Aberth
 * iterations of the eigenvalues
 * of Atilde, [3] shifted CholeskyQR retries, [4] OptDMD Levenberg-Marquardt steps kept,
 * [5] OptDMD trial points evaluated, [6] OptDMD outcome: 0 stopped by its rule (a kept step
 * gained at most 1e-13 of the cost, 200 kept steps, 40 rejections in a row or the damping
 * past 1e20), 1 still running when the enqueued trial points ran out (the model holds the
 * last kept point), 2 not applied (the starting basis was singular or its cost not finite;
 * the model is the plain fit's), [7] reserved. */

/* A DMD model; every pointer is device memory owned by the caller. */
typedef struct dmd_model {
    int64_t n;        /* rows N (grid DOFs) */
    int32_t r;        /* number of modes */
    int32_t dtype;    /* dmd_dtype of phi */
    double dt;        /* time step of the snapshots */
    void* phi;        /* N x ldphi, ROW-major (the r mode values of a grid point are
                         contiguous), folded real storage; columns r..ldphi-1 are zero */
    int64_t ldphi;    /* >= dmd_phi_ld(r), a multiple of 32, at most 192 */
    double* lam;      /* r complex eigenvalues, interleaved (re, im) */
    double* b;        /* r complex amplitudes, interleaved (re, im) */
    double* sigma;    /* r singular values kept by the fit (written by dmd_fit) */
    int32_t* kind;    /* r entries, 0 real / 1 first of pair / 2 second of pair */
    int32_t* info;    /* DMD_INFO_WORDS status / diagnostic words (written by dmd_fit) */
} dmd_model;

/* One scene of a batched fit. */
typedef struct dmd_scene {
    const void* x;    /* device X, N x ncols */
    const void* xp;   /* device X', N x ncols */
    int64_t n;
    int32_t ncols;    /* m - 1 */
    int32_t xdtype;   /* dmd_dtype of X and X' */
    int64_t ldx;
    int64_t ldxp;
    dmd_fit_opts opts;
    void* ws;         /* this scene's workspace (dmd_fit_workspace_size) */
    size_t ws_bytes;
} dmd_scene;

typedef struct dmd_graph dmd_graph;  /* opaque captured launch graph */

/* ABI version (DMDMI_ABI_VERSION). */
int32_t dmd_abi_version(void);

/* Static description of a status code (never NULL). */
const char* dmd_status_string(int32_t status);

/* Minimal leading dimension of phi for r modes: r rounded up to 32. */
int64_t dmd_phi_ld(int32_t r);

/* Workspace bytes for dmd_fit on an N x ncols snapshot pair of element type xdtype. */
int32_t dmd_fit_workspace_size(int64_t n, int32_t ncols, int32_t xdtype,
                               const dmd_fit_opts* opts, size_t* bytes);

/*
 * Fit a rank-r DMD model to the snapshot pair (X, X').
 *   x, xp    device, N x ncols (ncols = m-1), column-major with leading dimensions
 *            ldx, ldxp >= N.  When xp == x + ldx elements and ldxp == ldx (the two
 *            shifted views of one snapshot buffer Z, eq. reduced_koopman) the
 *            projection reads Z in one pass.
 *   xdtype   DMD_F32 for DMD_FIT_MIXED, DMD_F64 otherwise.
 *   model    caller-filled: n, phi (N x ldphi, dtype = F32 for MIXED else F64),
 *            ldphi, lam, b, sigma, kind, info; the fit sets r, dtype, dt and writes
 *            every array.
 * Steps (Sec. 4.3 then Sec. 3.1): sketch Y = X Omega; CholeskyQR2 (FP64 Gram);
 * q power iterations W = orth(X^T Q), Y = X W; B = Q^T [X X']; eigen-decomposition
 * of the FP64 Gram B B^T (Householder tridiagonalisation, bisection on Sturm counts,
 * inverse iteration: singular values and left vectors of B);
 * Atilde = U_r^T B' V_r S_r^-1; Hessenberg reduction, eigenvalues as the roots of
 * det(zI - H) by the Ehrlich-Aberth iteration, eigenvectors W by inverse iteration;
 * exact modes Phi = X' V_r S_r^-1 W; b = Phi^+ x_0.
 * Sizes: 1 <= r <= min(ncols, N, DMD_MAX_RANK); on the randomized paths
 * l = r + p <= min(ncols, N, DMD_MAX_SKETCH); on DMD_FIT_FP64_EXACT
 * ncols <= DMD_MAX_SMALL.  Violations return DMD_ERR_SHAPE (inconsistent sizes) or
 * DMD_ERR_UNSUPPORTED (beyond a limit) before any device work.
 * Returns the device status unless DMD_FIT_ASYNC is set.
 */
int32_t dmd_fit(void* stream, const void* x, const void* xp, int64_t n, int32_t ncols,
                int64_t ldx, int64_t ldxp, int32_t xdtype, const dmd_fit_opts* opts,
                void* ws, size_t ws_bytes, dmd_model* model);

/* Workspace bytes for dmd_reconstruct / dmd_integrate of K frames at rank r. */
int32_t dmd_reconstruct_workspace_size(int32_t r, int32_t K, int32_t mode, size_t* bytes);

/*
 * U[:, j] = Re( Phi diag(lambda^{k_j}) b ), j = 0..K-1 (Sec. 4.4, eq. large_time_step;
 * negative k runs the model backwards, Sec. 6.2).
 *   k_host  host, K integer exponents (copied to the workspace, stream-ordered)
 *   mode    dmd_recon_mode; DMD_RECON_FP64 needs an F64 model and an FP64 U,
 *           the other modes an F32 model and an FP32 U
 *   U       device, N x K column-major (frame j contiguous), ldu >= N
 * lambda^k is evaluated in FP64 as exp(k Log lambda) (0^0 = 1, 0^k = 0 for k > 0).
 * Sec. 6.1 takes Omega = Log(lambda) / dt, which has no value at lambda = 0: a power of
 * lambda = 0 with a negative or fractional exponent, and a term |b_i| |lambda_i|^k beyond the
 * largest finite value of the output type (FP64 for DMD_RECON_FP64, FP32 otherwise), are
 * recorded in the device status word at the start of the workspace (the call itself stays
 * asynchronous and returns DMD_OK); dmd_status_word reads it.
 */
int32_t dmd_reconstruct(void* stream, const dmd_model* model, const int64_t* k_host,
                        int32_t K, int32_t mode, void* U, int64_t ldu, void* ws,
                        size_t ws_bytes);

/*
 * dmd_reconstruct with no workspace argument and no allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, layout and result as dmd_reconstruct; the
 * exponents and packed coefficients go to a library-owned device array of
 * DMD_NOALLOC_SCRATCH_BYTES per GPU, held from the first call (or library set-up) on
 * that GPU until the process ends.  A call needs dmd_reconstruct_workspace_size(r, K,
 * mode) bytes of it (with r = 160: about 6,400 frames in DMD_RECON_FP64, 12,800 in
 * DMD_RECON_BF16X3); a larger request returns DMD_ERR_WORKSPACE before any device work.
 * Every call on one GPU uses the same array and leaves its contents there: calls that
 * overlap on one GPU (other streams, other host threads) race and must be serialised by
 * the caller.  status: NULL, or a device int32 that receives the coefficient pass's
 * status bits (bit 0: a power of lambda = 0 outside its domain, DMD_ERR_DOMAIN; bit 1: a
 * term beyond the output type's range, DMD_ERR_OVERFLOW), stream-ordered.  Calls no
 * hipMalloc, hipFree or allocating library routine.
 */
#define DMD_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
int32_t dmd_reconstruct_noalloc(void* stream, const dmd_model* model, const int64_t* k_host,
                                int32_t K, int32_t mode, void* U, int64_t ldu, int32_t* status);

/*
 * The two halves of dmd_reconstruct, for callers that evaluate one exponent list
 * many times (the coefficients depend only on lambda, b and the exponents):
 *   prepare: exponents (k_host integers, or t_host / dt when k_host is NULL) and the
 *            FP64 coefficients b lambda^e, packed for `mode`, into the workspace;
 *   apply:   the reconstruction GEMM from a workspace filled by prepare with the
 *            same model, K and mode (nothing is checked across the two calls).
 */
int32_t dmd_reconstruct_prepare(void* stream, const dmd_model* model, const int64_t* k_host,
                                const double* t_host, int32_t K, int32_t mode, void* ws,
                                size_t ws_bytes);
int32_t dmd_reconstruct_apply(void* stream, const dmd_model* model, int32_t K, int32_t mode,
                              void* U, int64_t ldu, void* ws, size_t ws_bytes);

/*
 * U[:, j] = Re( Phi exp(Omega t_j) b ), Omega = Log(Lambda) / dt (Sec. 6.1,
 * eq. edit_temporal), principal branch, for real times t_host[0..T-1].
 * Same layout, modes and workspace as dmd_reconstruct (K = T).
 */
int32_t dmd_integrate(void* stream, const dmd_model* model, const double* t_host,
                      int32_t T, int32_t mode, void* U, int64_t ldu, void* ws,
                      size_t ws_bytes);

/* Temporal edit of the modes by frequency cluster (Sec. 6.1, eq. edit_temporal). */
typedef struct dmd_edit {
    double freq_cut;     /* a mode with |Im Omega| < freq_cut is in cluster 0 (low frequency),
                            the others in cluster 1; Sec. 6.1 uses 0.01 */
    double weight[2];    /* amplitude factor w of cluster 0 / 1: b' = w b */
    double re_scale[2];  /* Re Omega' = re_scale * Re Omega + re_shift (decay / growth rate) */
    double re_shift[2];
    double im_scale[2];  /* Im Omega' = im_scale * Im Omega (angular frequency) */
} dmd_edit;

/*
 * Edited eigenvalues and amplitudes for playback (Sec. 6.1, eq. edit_temporal).
 * With Omega = Log(lambda) / dt = (log|lambda| + i arg lambda) / dt (principal branch,
 * dt = model->dt), each mode gets
 *   lambda' = exp(Omega' dt),  Re Omega' = re_scale Re Omega + re_shift,
 *   Im Omega' = im_scale Im Omega,  b' = w b,
 * with its cluster's parameters, or with its own row of mode_edit when that is not NULL.
 * lambda = 0 gives lambda' = 0.  Reconstructing a model whose lam / b point at
 * lam_out / b_out (same phi and kind) plays back the edited flow; re_scale = im_scale = -1
 * gives lambda^-1, the reversed dynamics of Sec. 6.2.  A conjugate pair keeps conjugate
 * eigenvalues under cluster edits (both members have the same |Im Omega|).
 *   model       reads r, dt, lam, b (device); phi is not read
 *   edit        host; every field finite, freq_cut >= 0
 *   mode_edit   device, r rows of 4 doubles (w, re_scale, re_shift, im_scale), row-major,
 *               or NULL to use the cluster parameters
 *   lam_out     device, r complex (interleaved); may be model->lam (in-place edit)
 *   b_out       device, r complex; may be model->b
 *   cluster_out device, r int32 cluster labels, or NULL
 * Errors: DMD_ERR_ARG for a missing pointer, dt <= 0 or a non-finite / negative field of
 * edit; nothing is enqueued then.  Stream-ordered, no workspace, no synchronisation.
 */
int32_t dmd_edit_modes(void* stream, const dmd_model* model, const dmd_edit* edit,
                       const double* mode_edit, double* lam_out, double* b_out,
                       int32_t* cluster_out);

/* Workspace bytes for dmd_project. */
int32_t dmd_project_workspace_size(int64_t n, int32_t r, size_t* bytes);

/*
 * z = Phi^+ u (Sec. 3.1, eq. projection): least-squares reduced state of a full
 * state u (device, N values of the model's dtype).  z: device, r complex
 * (interleaved), conjugate-paired like lam.  FP64 Gram of Phi + Cholesky solve.
 */
int32_t dmd_project(void* stream, const dmd_model* model, const void* u, double* z,
                    void* ws, size_t ws_bytes);

/* Workspace bytes for dmd_rollout of T forced steps (any f / U / z_out combination). */
int32_t dmd_rollout_workspace_size(int64_t n, int32_t r, int32_t T, int32_t mode, size_t* bytes);

/*
 * Forced roll-out in the reduced space (Sec. 4.6, eq. external_forces, DMD with control):
 *   z_0 = z0,   z_{s+1} = Lambda z_s + dt Phi^+ f_s   (s = 0 .. T-1, dt = model->dt),
 * and the frames u_s = Re(Phi z_s), s = 0 .. T.
 *   z0      device, r complex (interleaved), conjugate-paired like lam; NULL starts from
 *           model->b (the fitted state at k = 0)
 *   f       device, N x T column-major (ldf >= N), the model's dtype: column s is the
 *           full-space forcing of step s, i.e. the paper's sum of B_i q_i(t) and f_j(t),
 *           formed by the caller; NULL runs the unforced recurrence (lambda^s z0)
 *   mode    dmd_recon_mode of U, as for dmd_reconstruct (checked also when U is NULL)
 *   U       device, N x (T+1) column-major (ldu >= N), frame s in column s; or NULL
 *   z_out   device, (T+1) x r complex, state s at z_out + 2 r s; or NULL
 * Phi^+ f_s is the least-squares projection of eq. projection: the FP64 Gram of Phi, its
 * Cholesky inverse, then R^-1 R^-T Phi^T F over all steps (Phi^T F in the model's precision,
 * split-N partial sums in FP64).  The recurrence runs in FP64,
 * one scan per mode; the frames are one reconstruction GEMM over the T+1 states.
 * Errors: DMD_ERR_SHAPE for T < 1, DMD_ERR_ARG for dt <= 0, ldf < N, a bad mode or a
 * mode / dtype / ldu mismatch of U, DMD_ERR_WORKSPACE; nothing is enqueued then.
 */
int32_t dmd_rollout(void* stream, const dmd_model* model, const double* z0, const void* f,
                    int64_t ldf, int32_t T, int32_t mode, void* U, int64_t ldu, double* z_out,
                    void* ws, size_t ws_bytes);

/* Workspace bytes for dmd_upsample of T guide frames. */
int32_t dmd_upsample_workspace_size(int64_t n, int32_t r, int32_t T, int32_t mode, size_t* bytes);

/*
 * Upsampling evolution (Sec. 6.3.1): a high-res model adds its high-order modes to a
 * low-res guide.  R_0 = Phi^+ h0; for t = 1 .. T, R*_t = Lambda R_{t-1},
 * P_t = Phi^+ l_t and R_t = S^L P_t + S^H R*_t (low-order modes from the guide, the
 * others evolved, i.e. lambda^t R_0); frames H_t = Re(Phi R_t), t = 0 .. T.
 *   h0        device, N values (model dtype): the high-res initial field
 *   l         device, N x T column-major (ldl >= N): guide frames l_1 .. l_T on the
 *             high-res grid (the caller prolongs the low-res frames)
 *   low_host  host, r int32 flags, non-zero = low-order mode (taken from the guide); a
 *             conjugate pair follows its first member's flag
 *   mode, U, ldu   frames as for dmd_rollout (U may be NULL)
 *   r_out     device, (T+1) x r complex states, or NULL
 * Projections as in dmd_rollout (FP64 Gram and Cholesky inverse, MFMA products).
 * Errors: DMD_ERR_SHAPE for T < 1; DMD_ERR_ARG for missing h0 / l / low_host,
 * ldl < N, a bad mode or U mismatch; DMD_ERR_WORKSPACE.
 */
int32_t dmd_upsample(void* stream, const dmd_model* model, const void* h0, const void* l,
                     int64_t ldl, int32_t T, const int32_t* low_host, int32_t mode, void* U,
                     int64_t ldu, double* r_out, void* ws, size_t ws_bytes);

/*
 * Projection onto the fields that match a low-res guide (Sec. 6.3.2):
 *   x = argmin ||x - h||^2  subject to  A x = l,
 * A = average over factor x factor (x factor) blocks of a regular grid, per component.
 * A A^T = factor^-d I, so the KKT solution is x = h - A^T factor^d (A h - l): every fine
 * cell moves by its block's mean mismatch.  One pass over h, l and x.
 *   dtype        DMD_F32 or DMD_F64 (h, l, x)
 *   h, x         device, nframes frames of N = ncomp * nz * ny * nx values, component-major
 *                (c, z, y, x) with x fastest, frame f at h + f ldh (ldh, ldx >= N); x may be h
 *   l            device, nframes coarse frames of ncomp * (nz/fz) * (ny/factor) * (nx/factor)
 *                values in the same order, ld ldl; fz = factor, or 1 when nz = 1 (2D)
 * Errors: DMD_ERR_SHAPE for non-positive sizes or dimensions not divisible by factor,
 * DMD_ERR_ARG for a bad dtype, null pointer or short leading dimension.
 */
int32_t dmd_lowres_project(void* stream, int32_t dtype, const void* h, int64_t ldh, const void* l,
                           int64_t ldl, void* x, int64_t ldx, int64_t nframes, int32_t ncomp,
                           int32_t nz, int32_t ny, int32_t nx, int32_t factor);

/* Workspace bytes for dmd_loss_grad. */
int32_t dmd_loss_grad_workspace_size(int64_t n, int32_t r, int32_t ncols, int32_t dtype,
                                     size_t* bytes);

/*
 * Device status of the last coefficient pass that used workspace `ws` (dmd_reconstruct,
 * dmd_reconstruct_prepare, dmd_integrate, dmd_rollout, dmd_upsample, dmd_loss_grad all
 * clear it and then record into it): waits for `stream`, then stores in *status
 * DMD_ERR_DOMAIN when a power of lambda = 0 had a negative or fractional exponent (Sec. 6.1:
 * Omega = Log(lambda) / dt is undefined there), else DMD_ERR_OVERFLOW when a coefficient
 * b_i lambda_i^k (or a reduced state of a roll-out) exceeded the output type's finite range,
 * else DMD_OK.  The affected outputs hold zeros (domain) or non-finite values (overflow).
 *   ws      device, the workspace passed to that call (its first 4 bytes hold the word)
 * Returns DMD_ERR_ARG for null pointers, DMD_ERR_HIP when the copy fails.
 */
int32_t dmd_status_word(void* stream, const void* ws, int32_t* status);

/*
 * Loss and adjoint of the full-space reconstruction with the modes held fixed:
 *   L(lambda, b) = sum_j || x_j - Re(Phi (b .* lambda^{k_j})) ||^2
 *   G = Phi^T R (transpose), grad_b = -2 conj(sum_j G_ij lambda_i^{k_j}),
 *   grad_lambda = -2 conj(sum_j G_ij k_j b_i lambda_i^{k_j - 1})
 * (gradients as dL/dRe + i dL/dIm, the complex-autograd convention).
 *   lam, b   device, r complex each (the variables; the model's lam/b are ignored)
 *   xt       device target frames, N x ncols column-major, ldxt >= N, model dtype
 *   k_host   host, ncols exponents (frame j of xt is compared with lambda^{k_j})
 *   out      device, 1 + 4r doubles: loss, grad_lambda (r complex), grad_b (r complex)
 * The residual and G run as MFMA GEMMs in the model's precision; loss, lambda^k
 * and the r-reductions are FP64.
 * Limits: r * ncols <= 102400 (the G = Phi^T R product's output, e.g. 682 frames at
 * r = 150); larger calls return DMD_ERR_UNSUPPORTED before anything is enqueued.
 * Domain and overflow of lambda^k are recorded as for dmd_reconstruct (dmd_status_word).
 */
int32_t dmd_loss_grad(void* stream, const dmd_model* model, const double* lam,
                      const double* b, const void* xt, int64_t ldxt, const int64_t* k_host,
                      int32_t ncols, double* out, void* ws, size_t ws_bytes);

/*
 * Refit statistics: the loss and adjoint of dmd_loss_grad for many (lambda, b) with the
 * same modes and target frames.  With the modes fixed the loss needs the frames only
 * through G0 = Phi_f^T X (r x ncols), M = Phi_f^T Phi_f (r x r) and ||X||^2 (folded real
 * modes Phi_f, FP64 sums of the model's data); with the folded FP64 coefficients C of
 * (lambda, b),  G_f = G0 - M C = Phi_f^T R  and  L = ||X||^2 - <C, G0 + G_f>, so each
 * evaluation is O(r^2 ncols) and the residual R is never formed (the objective of Sec. 4.2
 * with the modes fixed, as in dmd_loss_grad).
 *   dmd_refit_prepare:   reads xt (N x ncols, ldxt >= N, model dtype) and the exponents
 *                        k_host once, stores the statistics in the workspace;
 *   dmd_refit_loss_grad: out (device, 1 + 4r doubles, the layout of dmd_loss_grad) for
 *                        lam, b (device, r complex each), from a workspace prepared with
 *                        the same model and ncols (nothing is checked across the calls).
 * Both are asynchronous.  The loss loses accuracy by cancellation when it is far below
 * ||X||^2 (relative error about 1e-16 ||X||^2 / L).  Limits as dmd_loss_grad
 * (r * ncols <= 102400).  Domain and overflow of lambda^k are recorded in the workspace's
 * status word (dmd_status_word).
 */
int32_t dmd_refit_workspace_size(int64_t n, int32_t r, int32_t ncols, size_t* bytes);
int32_t dmd_refit_prepare(void* stream, const dmd_model* model, const void* xt, int64_t ldxt,
                          const int64_t* k_host, int32_t ncols, void* ws, size_t ws_bytes);
int32_t dmd_refit_loss_grad(void* stream, const dmd_model* model, const double* lam,
                            const double* b, int32_t ncols, double* out, void* ws,
                            size_t ws_bytes);

/*
 * Fit several independent scenes.  Each scene's fit runs on its own forked
 * stream (default priority) joined back into `stream`, so the latency-bound
 * small-matrix stages of different scenes overlap.  With capture != 0 the batch
 * first runs once (the call waits for it: the runtime loads each kernel's code on
 * its first launch, which a capturing stream does not allow), then is captured into
 * a HIP graph returned in *graph for dmd_graph_launch; capture needs a created
 * stream (the null stream is refused with DMD_ERR_ARG).  Without capture the batch
 * runs and the call waits for it.
 * Scenes use DMD_FIT_ASYNC semantics (statuses land in each model's info[0]).
 */
int32_t dmd_fit_batched(void* stream, int32_t nscenes, const dmd_scene* scenes,
                        dmd_model* models, int32_t capture, dmd_graph** graph);

/* Launch a captured batch on `stream`. */
int32_t dmd_graph_launch(dmd_graph* graph, void* stream);

/* Destroy a captured batch and the streams it forked. */
int32_t dmd_graph_destroy(dmd_graph* graph);

/*
 * Autotuner for the reconstruction kernel: times each candidate tile shape on
 * the given model and output, keeps the fastest for this (mode, r, N, K) class
 * in the in-process table (used by later dmd_reconstruct calls) and appends it
 * to the text cache file `cache_path` (may be NULL).  best_cfg receives the
 * chosen candidate index.
 */
int32_t dmd_autotune_reconstruct(void* stream, const dmd_model* model, int32_t K,
                                 int32_t mode, void* U, int64_t ldu, void* ws,
                                 size_t ws_bytes, const char* cache_path,
                                 int32_t* best_cfg);

/*
 * Fit-product autotuner.  Runs the fit of dmd_fit (same arguments; the model receives
 * its result) while recording every streaming TN product of the fit (X^T Q, Q^T Z, the
 * Grams that do not take the triangle-only kernel), then times each recorded shape
 * class (input and compute type, row chunk, output blocks, log2 N) with every tile
 * candidate of the TN kernel, three launches each, keeps the fastest for later fits and
 * products of the same class in this process, and appends one line per class to
 * `cache_path` (may be NULL).  The replays rewrite workspace buffers only.  Without an
 * entry a product takes its tile from a cost model.  Synchronous; errors as dmd_fit.
 */
int32_t dmd_autotune_fit(void* stream, const void* x, const void* xp, int64_t n, int32_t ncols,
                         int64_t ldx, int64_t ldxp, int32_t xdtype, const dmd_fit_opts* opts,
                         void* ws, size_t ws_bytes, dmd_model* model, const char* cache_path);

/* Load autotuner entries (reconstruction and fit products) from a cache file written by
 * dmd_autotune_reconstruct or dmd_autotune_fit. */
int32_t dmd_autotune_load(const char* cache_path);

/*
 * Model files.  The fit is the offline precomputation whose result the run-time
 * evaluation loads (Sec. 4.4: the reduced model is stepped, or evaluated for many frames
 * in one product).  A file holds a 64-byte versioned header (magic "DMDMODEL", format
 * version 1, N, r, dtype, dt, payload size, FNV-1a 64 hash of the payload, writer ABI
 * version), then lambda, b (2r FP64 each, interleaved), sigma (r FP64), kind (r int32)
 * and Phi (N x r, row-major, the model's dtype; padding columns are not stored).
 *
 * dmd_model_save: waits for `stream`, copies the model's device arrays through host
 *   memory (staging buffers of at most 65536 rows) and writes `path`.  Returns
 *   DMD_ERR_IO when the file cannot be written.
 * dmd_model_file_info: host only, no HIP call; reads and checks the header and the payload
 *   hash and returns N, r, dtype and dt, so the caller can allocate the model's arrays.
 * dmd_model_load: fills the caller's model (n and dtype must match the file; phi holds
 *   N x ldphi with ldphi >= dmd_phi_ld(r), a multiple of 32; lam, b: r complex; sigma: r;
 *   kind: r; info may be NULL, else it is zeroed) and sets r and dt; the padding columns of
 *   phi are written as zeros.  Waits for `stream` before returning.
 * Errors: DMD_ERR_ARG (null pointer, dtype / ldphi mismatch), DMD_ERR_SHAPE (N differs),
 * DMD_ERR_IO (missing, truncated, foreign or corrupted file), DMD_ERR_HIP.
 */
int32_t dmd_model_save(void* stream, const dmd_model* model, const char* path);
int32_t dmd_model_file_info(const char* path, int64_t* n, int32_t* r, int32_t* dtype, double* dt);
int32_t dmd_model_load(void* stream, const char* path, dmd_model* model);

#ifdef __cplusplus
}
#endif

#endif /* DMDMI_H */
