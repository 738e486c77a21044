// Internal launchers of the gfx950 kernels (host-callable, enqueue only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dmdmi.h"

namespace dmd {

constexpr int NN_MAX_CB = 12;          // gemm_nn: n <= 192 output columns
constexpr int TN_MAX_SPLITS = 1024;    // gemm_tn: row splits (FP64 partials), at most
constexpr int64_t TN_MAX_OUT = 320 * 320;
constexpr int RECON_MAX_RP = 160;      // padded rank held in registers by the reconstruction
constexpr int RECON_KPAD = 64;         // frame padding of the coefficient matrix
constexpr int SMALL_MAX = DMD_MAX_SMALL;
constexpr int EXACT_QR_MAX = DMD_EXACT_QR_MAX;
constexpr int EIG_MAX = DMD_MAX_RANK;

__global__ void fill_f64_kernel(double* p, int64_t n, double v);
__global__ void fill_f32_kernel(float* p, int64_t n, float v);
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v);

int device_cu_count();
hipError_t fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
// One-time per-kernel attributes (LDS above 64 KiB); called before any capture.
hipError_t prepare_kernels();
hipError_t gemm_prepare();
hipError_t small_prepare();
hipError_t eig_prepare();

// ---- tall-skinny GEMMs (gemm.hip)
// b_upper: B is upper triangular (B(k, j) = 0 for k > j), its zero part is not multiplied
hipError_t gemm_nn(hipStream_t s, int dtype, const void* A, int64_t lda, const void* B, int64_t ldb,
                   void* C, int64_t ldc, int c_rowmajor, int64_t N, int K, int n,
                   const int32_t* skip_unless, int b_upper = 0);
hipError_t gemm_tn(hipStream_t s, int in_dtype, int compute_dtype, const void* A, int64_t lda,
                   int a_rowmajor, int ka, const void* B, int64_t ldb, int b_rowmajor, int nb,
                   int sym, int64_t N, double* P, double* out, int64_t ldo, float* out32,
                   int64_t ldo32, const int32_t* skip_unless);
size_t gemm_tn_partial_bytes(int64_t N, int ka, int nb);
// Tile tuner of gemm_tn: record the products that reach the tile choice (tn_record(true)
// ... tn_record(false)), then time every candidate of each recorded shape class and keep
// the fastest (lines: one cache line "tn ..." per class); tn_table_set loads a choice.
void tn_record(bool on);
hipError_t tn_tune_recorded(hipStream_t s, std::vector<std::string>* lines);
void tn_table_set(int in_dt, int c_dt, int rc, int nbi, int nbj, int ln, int cand);
size_t tn_table_size();
int tn_max_splits(int64_t N);          // row splits (FP64 partial products) gemm_tn uses for N rows

// ---- reconstruction (recon.hip)
struct ReconArgs {
    int mode;
    const void* phi; int64_t ldphi; int64_t N; int rp;
    const void* c_hi; const void* c_lo; int K;
    void* U; int64_t ldu; int vec_store;
    const void* xt; int64_t ldxt; double* ss_partial;   // residual epilogue (adjoint)
    int* grid_out;
};
constexpr int RECON_NCFG = 6;
constexpr int RECON_MAX_WG_PER_CU = 4;  // the largest work-groups-per-CU of any tile candidate
constexpr int LG_SS_SLOTS = 4096;       // loss partials (one per work-group) of the residual launch
inline int recon_max_grid() { return device_cu_count() * RECON_MAX_WG_PER_CU; }
hipError_t recon_launch(hipStream_t s, const ReconArgs& ra, int cfg);
// status (may be null): COEF_DOMAIN / COEF_OVERFLOW bits or-ed in (common.h)
hipError_t powers_pack(hipStream_t s, const double* lam, const double* b, const int32_t* kind, int r,
                       const double* expo, int K, int Kp, int rp, int mode, void* hi, void* lo, int32_t* status);
hipError_t exponents(hipStream_t s, const int64_t* k, const double* t, double inv_dt, int K, double* e);

// ---- small FP64 matrices (small.hip)
// Cholesky G = R^T R of an n x n SPD matrix and R^-1 (upper).  On breakdown retry
// once with a diagonal shift (flagging *shifted = 1 and run_next[0..nnext-1] = 1, the
// run flags of the passes that must follow a shifted one); a failure without a shift,
// or of the shifted retry, writes DMD_ERR_CHOL_BREAKDOWN to info[0] and an identity R^-1.
hipError_t chol_inv(hipStream_t s, const double* G, int64_t ldg, int n, double* Rinv, int64_t ldr,
                    float* Rinv32, int64_t ldr32, double shift_scale, int32_t* shifted,
                    int32_t* info, const int32_t* skip_unless, int32_t* run_next = nullptr, int nnext = 0);
// Symmetric eigen-decomposition (eig.hip): all n eigenvalues of the symmetric n x n
// matrix S (n <= 192) in descending order, and unit eigenvectors of the nv largest in the
// columns of Vout (ld ldv).  Eigenvectors of clustered eigenvalues are independent but not
// orthogonal to working precision.  info[1] receives the bisection rounds.
size_t sym_eig_workspace_bytes(int n);
hipError_t sym_eig(hipStream_t s, const double* S, int64_t lds, int n, int nv, double* evals, double* Vout,
                   int64_t ldv, void* ws, int32_t* info);
// C = alpha op(A) op(B) + beta C, all FP64 column-major, small sizes.  A launcher's
// `run` (where present, may be null): the kernel does nothing when *run == 0.
hipError_t small_gemm(hipStream_t s, int ta, int tb, int m, int n, int k, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                      double* C, int64_t ldc, const int32_t* run = nullptr);
// Scale column j of A (m x n) by d[j] (or 1/d[j] with inv): A(:, j) *= f(d[j]).
hipError_t scale_cols(hipStream_t s, int m, int n, double* A, int64_t lda, const double* d, int mode);
// sigma = sqrt(max(evals, 0))[0..r) (squared = 1: evals are squares) or max(evals, 0)
// (squared = 0), rank check against rank_tol.
hipError_t sigma_from_evals(hipStream_t s, const double* evals, int r, double rank_tol, double* sigma,
                            double* sigma_out, int32_t* info, int squared = 1);
// J = [[0, R], [R^T, 0]] (2n x 2n, ld 2n) from the n x n block R (ld ldr).
hipError_t jw_build(hipStream_t s, int n, const double* R, int64_t ldr, double* J);
// Copy a double matrix into float (m x n), zero-filling columns n..n_pad-1.
hipError_t to_f32(hipStream_t s, int m, int n, int n_pad, const double* A, int64_t lda, float* B,
                  int64_t ldb);
hipError_t copy_f64(hipStream_t s, int m, int n, int n_pad, const double* A, int64_t lda, double* B,
                    int64_t ldb, double scale = 1.0, const int32_t* run = nullptr);   // B = scale A
// Least-squares amplitudes from the Gram of the folded modes: beta = G^-1 rhs via
// Rinv (beta_ws: r doubles), then complex b for each (real | pair) mode.
hipError_t amplitudes(hipStream_t s, int r, const double* Rinv, int64_t ldr, const double* rhs,
                      const int32_t* kind, double* b, double* beta_ws);
hipError_t normal_solve(hipStream_t s, int r, const double* Rinv, int64_t ldr, const double* rhs, double* beta,
                        int accumulate, const int32_t* run = nullptr);
hipError_t beta_to_b(hipStream_t s, int r, const double* beta, const int32_t* kind, double* b);
// res = x - Phi beta (one FP64 dot per row), in the model's element type
hipError_t residual(hipStream_t s, int dtype, int64_t N, int r, const void* phi, int64_t ldphi, const double* beta,
                    const void* x, void* res);
hipError_t check_finite(hipStream_t s, int dtype, const void* X, int64_t ld, int64_t N, int ncols,
                        int32_t* info);

// ---- nonsymmetric eigen-decomposition (eig.hip)
size_t eig_workspace_bytes(int n);
// lam (2n doubles), kind (n), W (n x n folded real eigenvectors, ld n) sorted in
// the canonical order.  tol: an eigenvalue approximation is converged once its
// correction falls below tol relative to its size (at least 4e-16).  info[2] receives
// the number of eigenvalue iterations.
hipError_t nonsym_eig(hipStream_t s, const double* A, int64_t lda, int n, void* ws, double* lam,
                      int32_t* kind, double* W, int32_t* info, double tol);

// ---- temporal editing (edit.hip)
// lam_out / b_out may alias lam / b; mode_edit (r x 4, row-major) overrides the cluster
// parameters when not null; cluster_out may be null.
hipError_t edit_modes(hipStream_t s, int r, double dt, const dmd_edit& e, const double* mode_edit,
                      const double* lam, const double* b, double* lam_out, double* b_out, int32_t* cluster_out);

// ---- forced roll-out (rollout.hip)
// states: (T+1) x r complex, state s at states + 2 r s; beta (r x T, ld ldb) may be null
// (unforced).
hipError_t rollout_scan(hipStream_t s, int r, int T, const double* lam, const double* z0, const double* beta,
                        int64_t ldb, const int32_t* kind, double dt, double* states);
hipError_t pack_states(hipStream_t s, const double* states, const int32_t* kind, int r, int K, int Kp, int rp,
                       int mode, void* hi, void* lo, int32_t* status);

// ---- upsampling (upsample.hip)
hipError_t upsample_states(hipStream_t s, int r, int T, const double* lam, const double* beta0, const double* beta,
                           int64_t ldb, const int32_t* kind, const int32_t* low, double* states);
hipError_t lowres_project(hipStream_t s, int dtype, const void* h, int64_t ldh, const void* l, int64_t ldl, void* x,
                          int64_t ldx, int64_t nframes, int ncomp, int nz, int ny, int nx, int f);

// ---- OptDMD by variable projection (optdmd.hip), real folded parameters theta
// Levenberg-Marquardt state on the device: ist (VP_IST_WORDS int32), vst (2 doubles)
constexpr int VP_RUN = 0, VP_ACCEPT = 1, VP_STEPS = 2, VP_TRIES = 3, VP_TRIALS = 4, VP_DAMPED = 5,
              VP_APPLY = 6, VP_FIT_OK = 7, VP_IST_WORDS = 8;
constexpr int VP_COST = 0, VP_MU = 1;
constexpr int VP_MAX_STEPS = 200;      // kept steps (the oracle's cap)
constexpr int VP_MAX_TRIES = 40;       // rejected trial points in a row
constexpr double VP_MU0 = 1e-3, VP_MU_MIN = 1e-12, VP_MU_MAX = 1e20, VP_GAIN_TOL = 1e-13;
hipError_t vp_theta_init(hipStream_t s, int r, const double* lam, const int32_t* kind, double* theta);
hipError_t vp_basis(hipStream_t s, int T, int r, const double* theta, const int32_t* kind, double* Phi, double* E,
                    const int32_t* run);
hipError_t vp_assemble(hipStream_t s, int r, const int32_t* kind, const double* K, const double* W, const double* H,
                       double* G, double* g, const int32_t* run);
hipError_t vp_sumsq(hipStream_t s, int m, int n, const double* A, int64_t lda, double* out, const int32_t* run);
hipError_t vp_damp(hipStream_t s, int r, const double* G, const double* mu, double* A, const int32_t* run,
                   int32_t* scr);
hipError_t vp_update(hipStream_t s, int r, const double* theta, const double* delta, double* out, const int32_t* run,
                     int32_t* scr, int32_t* ist);
hipError_t vp_lift(hipStream_t s, int r, const int32_t* kind, const double* theta, const double* B, double* lam,
                   double* b, double* scale, const int32_t* run);
hipError_t vp_begin(hipStream_t s, const int32_t* fit_info, int32_t* ist, int32_t* scr);
hipError_t vp_start(hipStream_t s, const double* cost0, const int32_t* scr, int32_t* ist, double* vst);
hipError_t vp_decide(hipStream_t s, const double* cost_t, const int32_t* scr, int32_t* ist, double* vst);
hipError_t vp_commit(hipStream_t s, int r, const int32_t* ist, const double* theta_t, double* theta_c,
                     const double* bf_t, double* bf_c, const double* G_t, double* G_c, const double* g_t, double* g_c);
hipError_t vp_finish(hipStream_t s, const int32_t* ist, int32_t* info);

// ---- adjoint (adjoint.hip)
// Refit statistics (adjoint.hip): FP64 sum of squares of an N x ncols matrix as at most
// SQ_MAX_PARTS partials (*nparts of them), and loss[0] = sum(xxp) - <C, G0 + Gf>.
constexpr int SQ_MAX_PARTS = 512;
inline int64_t sumsq_rows_per(int64_t N) { return std::max<int64_t>((N + SQ_MAX_PARTS - 1) / SQ_MAX_PARTS, 1024); }
inline int sumsq_parts(int64_t N) { return (int)((N + sumsq_rows_per(N) - 1) / sumsq_rows_per(N)); }
hipError_t sumsq(hipStream_t s, int dtype, const void* X, int64_t ld, int64_t N, int ncols, double* partial,
                 int* nparts);
hipError_t refit_loss(hipStream_t s, int r, int ncols, const double* C, const double* G0, const double* Gf,
                      const double* xxp, int nxx, double* loss);
hipError_t grad_reduce(hipStream_t s, int r, int ncols, const double* G, const double* lam,
                       const double* b, const int32_t* kind, const double* expo,
                       const double* ss_partial, int nss, double* out);

}  // namespace dmd
