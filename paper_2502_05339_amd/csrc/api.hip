// Host orchestration and the extern "C" boundary of the DMD hot path.
//
// Every entry point validates its arguments on the host before the first HIP
// call, carves the caller's workspace with the same routine that answers the
// size query, and only enqueues kernels on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "kernels.h"

using namespace dmd;

namespace {

// ---------------------------------------------------------------- workspace carving
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T> T* take(size_t count) {
        off = (size_t)round_up((int64_t)off, 256);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (size_t)round_up((int64_t)off, 256); }
};

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return DMD_ERR_HIP;   \
    } while (0)

size_t esize(int dt) { return dt == DMD_F32 ? 4 : 8; }

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

std::once_flag g_init_once;
hipError_t g_init_error = hipSuccess;
void lib_init();
hipError_t scratch_address(void** out);
// one-time set-up (kernel LDS limits, autotune cache); its failure fails every call
static int32_t ensure_init()
{
    std::call_once(g_init_once, lib_init);
    return g_init_error == hipSuccess ? DMD_OK : DMD_ERR_HIP;
}

// ---------------------------------------------------------------- fit plan
struct FitArgs {
    const void* x;
    const void* xp;
    int64_t n;
    int ncols;
    int64_t ldx, ldxp;
    int xdtype;
    dmd_fit_opts o;
    bool shifted;   // X' is the one-column shift of X inside one snapshot buffer Z
};

bool is_shifted_view(const void* x, const void* xp, int64_t ldx, int64_t ldxp, int dt)
{
    return x && ldx == ldxp && (uintptr_t)xp == (uintptr_t)x + (uintptr_t)(ldx * (dt == DMD_F32 ? 4 : 8));
}

int32_t validate_fit(const FitArgs& a, const dmd_model* model, bool need_ptrs)
{
    const dmd_fit_opts& o = a.o;
    if (a.n < 1 || a.ncols < 1) return DMD_ERR_SHAPE;
    if (o.precision < DMD_FIT_MIXED || o.precision > DMD_FIT_FP64_EXACT) return DMD_ERR_ARG;
    if (a.xdtype != (o.precision == DMD_FIT_MIXED ? DMD_F32 : DMD_F64)) return DMD_ERR_ARG;
    if (o.r < 1 || o.r > a.ncols || o.r > a.n) return DMD_ERR_SHAPE;
    if (o.r > DMD_MAX_RANK) return DMD_ERR_UNSUPPORTED;
    if (!(o.dt > 0.0) || !isfinite(o.dt)) return DMD_ERR_ARG;
    if (o.rank_tol < 0.0 || !isfinite(o.rank_tol)) return DMD_ERR_ARG;
    if (o.optdmd_trials < 0 || o.optdmd_trials > DMD_MAX_OPTDMD_TRIALS) return DMD_ERR_ARG;
    if (o.precision == DMD_FIT_FP64_EXACT) {
        if (a.ncols > DMD_MAX_SMALL) return DMD_ERR_UNSUPPORTED;
    } else {
        if (o.p < 0 || o.q < 0 || o.q > 64) return DMD_ERR_ARG;
        const int l = o.r + o.p;
        if (l > a.ncols || l > a.n) return DMD_ERR_SHAPE;
        if (l > DMD_MAX_SKETCH) return DMD_ERR_UNSUPPORTED;
        if (need_ptrs && !o.omega) return DMD_ERR_ARG;
    }
    if (need_ptrs) {
        if (!a.x || !a.xp || !model) return DMD_ERR_ARG;
        if (a.ldx < a.n || a.ldxp < a.n) return DMD_ERR_ARG;
        if (!model->phi || !model->lam || !model->b || !model->sigma || !model->kind || !model->info)
            return DMD_ERR_ARG;
        if (model->n != a.n) return DMD_ERR_SHAPE;
        const int64_t rp = dmd_phi_ld(o.r);
        if (model->ldphi < rp || model->ldphi % 32 != 0 || model->ldphi > 16 * NN_MAX_CB) return DMD_ERR_ARG;
        if (!aligned16(model->phi)) return DMD_ERR_ARG;
    }
    return DMD_OK;
}

// OptDMD buffers (variable projection on the T x r data Y = V_r S_r); two slots hold the
// current and the trial point of the Levenberg-Marquardt iteration
struct OptPlan {
    double *YE, *RE, *Phi;                  // T x 2r: [Y | E] and [R | E~]; T x r
    double *PtP, *Rv, *K, *Wm, *ER, *H;     // r x r
    double *PtYE, *tmp;                     // r x 2r
    double *BF[2], *G[2], *g[2], *theta[2]; // current (0) and trial (1) point: r x 2r (B | Phi^+ E), r x r, r, r
    double *cost;                           // 2
    double *A, *RinvA, *delta, *scale;      // r x r, r x r, r, r
    double *C;                              // rows x r (rows = l, or T on the exact path)
    void* Cf;                               // rows x ldphi in the data type
    int32_t* scr;                           // 16: status words of the r x r factorisations
    int32_t* ist;                           // the iteration's integer state (VP_*)
    double* vst;                            // cost and mu of the current point
    double* Ptn;                            // split partial products of the T-reductions
};

OptPlan opt_carve(Carver& cv, int T, int r, int rows, int64_t ldphi, int fdt)
{
    OptPlan o;
    const size_t tr = (size_t)T * r, rr = (size_t)r * r;
    o.YE = cv.take<double>(2 * tr); o.RE = cv.take<double>(2 * tr); o.Phi = cv.take<double>(tr);
    o.PtP = cv.take<double>(rr); o.Rv = cv.take<double>(rr); o.K = cv.take<double>(rr);
    o.Wm = cv.take<double>(rr); o.ER = cv.take<double>(rr); o.H = cv.take<double>(rr);
    o.PtYE = cv.take<double>(2 * rr); o.tmp = cv.take<double>(2 * rr);
    for (int k = 0; k < 2; ++k) {
        o.BF[k] = cv.take<double>(2 * rr); o.G[k] = cv.take<double>(rr);
        o.g[k] = cv.take<double>((size_t)r); o.theta[k] = cv.take<double>((size_t)r);
    }
    o.cost = cv.take<double>(2);
    o.A = cv.take<double>(rr); o.RinvA = cv.take<double>(rr);
    o.delta = cv.take<double>((size_t)r); o.scale = cv.take<double>((size_t)r);
    o.C = cv.take<double>((size_t)rows * r);
    o.Cf = cv.take<char>((size_t)rows * ldphi * esize(fdt));
    o.scr = cv.take<int32_t>(16);
    o.ist = cv.take<int32_t>(VP_IST_WORDS);
    o.vst = cv.take<double>(2);
    o.Ptn = cv.take<double>((size_t)tn_max_splits(T) * 2 * rr);   // the widest T-reduction is r x 2r
    return o;
}

// what the OptDMD refinement reads from a finished fit
struct FitBufs {
    const void* Q; int64_t ldq;   // orthonormal basis (randomized paths)
    double* Bx;                   // l x (m-1): Q^T X
    double* Ueig;                 // eigenvectors of B B^T (l x l) or of X^T X (m-1 x m-1)
    double* sigma;                // r singular values
    int l;
    OptPlan op;
};

// Carves (and, with base != nullptr, enqueues) the whole fit.
int32_t fit_plan(Carver& cv, hipStream_t st, const FitArgs& a, dmd_model* model, FitBufs* fb = nullptr)
{
    const bool run = cv.base != nullptr;
    const dmd_fit_opts& o = a.o;
    const int r = o.r, mm = a.ncols;
    const int64_t n = a.n;
    const int fdt = a.xdtype;
    const bool mixed = o.precision == DMD_FIT_MIXED;
    const bool exact = o.precision == DMD_FIT_FP64_EXACT;
    const int l = exact ? mm : r + o.p;
    const bool shifted = a.shifted;
    const int64_t ldphi = model ? model->ldphi : dmd_phi_ld(r);
    // staging of the mode coefficients is carved for the largest ldphi the header allows,
    // so the size query (which has no model) covers every valid model
    const int64_t ldphi_ws = 16 * NN_MAX_CB;
    const int64_t ldy = round_up(n, 4);
    const double u = 1.1102230246251565e-16;
    // Convergence of the eigenvalue iteration: full FP64 accuracy on the FP64 paths; on the
    // mixed path (FP32 data, 1e-5 eigenvalue target) a last correction below 1e-10
    // relative, almost three orders below the rounding of the FP32 data (6e-8); the
    // iteration converges cubically, so the eigenvalues themselves are far closer.
    const double defl_tol = mixed ? 1e-10 : 2.220446049250313e-16;

    // attempt/run flags: 16 words per CholeskyQR call (the sketch basis, then W and Y of
    // each power iteration), 16 for the shifted Cholesky of the mode Gram; all cleared by
    // one fill at the start of the fit
    const int qf = exact ? 0 : std::max(o.q, 0);     // validated <= 64 on the randomized paths
    const int nflags = 16 * (2 + 2 * qf);
    int32_t* flags = cv.take<int32_t>((size_t)nflags);
    int32_t* info = model ? model->info : nullptr;
    // partial buffer: largest TN product of the fit
    const int wide = shifted ? mm + 1 : mm;
    int64_t maxprod = (int64_t)std::max({(int64_t)l * wide, (int64_t)mm * l, (int64_t)l * l,
                                         (int64_t)r * r, (int64_t)r, (int64_t)wide * wide});
    double* P = cv.take<double>((size_t)tn_max_splits(n) * maxprod);
    double* G = cv.take<double>((size_t)std::max(l, wide) * std::max(l, wide));
    double* Rinv = cv.take<double>((size_t)std::max(l, wide) * std::max(l, wide));
    float* Rinv32 = cv.take<float>((size_t)l * l);
    double* evals = cv.take<double>((size_t)std::max(l, mm));
    double* Ueig = cv.take<double>((size_t)std::max(l, mm) * std::max(l, mm));
    double* sigma = cv.take<double>((size_t)r);
    double* Vs = cv.take<double>((size_t)mm * r);
    double* T1 = cv.take<double>((size_t)std::max(l, mm) * r);
    double* At = cv.take<double>((size_t)r * r);
    double* W = cv.take<double>((size_t)r * r);
    double* M = cv.take<double>((size_t)mm * r);
    void* Mf = cv.take<char>((size_t)mm * ldphi_ws * esize(fdt));
    double* PhiG = cv.take<double>((size_t)r * r);
    double* rhs = cv.take<double>((size_t)r);
    double* RinvPhi = cv.take<double>((size_t)r * r);
    double* beta = cv.take<double>((size_t)r);
    double* rhs2 = cv.take<double>((size_t)r);
    void* res = cv.take<char>((size_t)n * esize(fdt));
    void* eigws = cv.take<char>(eig_workspace_bytes(r));
    // exact path by the QR route (m - 1 <= EXACT_QR_MAX): an FP64 copy of [X X'] factored by
    // CholeskyQR, its triangular factor, and the 2(m-1) x 2(m-1) matrix [[0, R], [R^T, 0]]
    const bool qr_route = exact && mm <= EXACT_QR_MAX && n <= INT32_MAX;
    const int nc = shifted ? mm + 1 : mm;
    void* symws = cv.take<char>(sym_eig_workspace_bytes(qr_route ? 2 * mm : std::max(l, mm)));
    double* Gxp2 = (exact && !shifted && !qr_route) ? cv.take<double>((size_t)mm * mm) : nullptr;
    double* Qb = qr_route ? cv.take<double>((size_t)ldy * nc) : nullptr;
    double* RZ = qr_route ? cv.take<double>((size_t)nc * nc) : nullptr;
    double* RP = (qr_route && !shifted) ? cv.take<double>((size_t)mm * mm) : nullptr;
    double* Jm = qr_route ? cv.take<double>((size_t)4 * mm * mm) : nullptr;
    double* Ujw = qr_route ? cv.take<double>((size_t)2 * mm * r) : nullptr;
    double* Ys = qr_route ? cv.take<double>((size_t)nc * r) : nullptr;
    double* Yp = qr_route ? cv.take<double>((size_t)nc * r) : nullptr;
    void* Y = nullptr;
    double* Wt = nullptr;
    void* Wtf = nullptr;
    double* Bx = nullptr;
    double* Bp = nullptr;
    if (!exact) {
        Y = cv.take<char>((size_t)ldy * l * esize(fdt));
        Wt = cv.take<double>((size_t)mm * l);
        Wtf = cv.take<char>((size_t)mm * l * esize(fdt));
        if (shifted) {
            Bx = cv.take<double>((size_t)l * (mm + 1));
            Bp = Bx ? Bx + l : nullptr;          // a size query carves from a null base
        } else {
            Bx = cv.take<double>((size_t)l * mm);
            Bp = cv.take<double>((size_t)l * mm);
        }
    }
    OptPlan op{};
    if (o.flags & DMD_FIT_OPTDMD) op = opt_carve(cv, mm, r, exact ? mm : l, ldphi_ws, fdt);
    if (fb) {
        fb->Q = Y; fb->ldq = ldy; fb->Bx = Bx; fb->Ueig = Ueig; fb->sigma = sigma; fb->l = l;
        fb->op = op;
    }
    if (!run) return DMD_OK;

    HIPCHK(fill_i32(st, info, DMD_INFO_WORDS, 0));
    HIPCHK(fill_i32(st, flags, nflags, 0));
    if (o.flags & DMD_FIT_CHECK_FINITE) {
        HIPCHK(check_finite(st, fdt, a.x, a.ldx, n, mm, info));
        HIPCHK(check_finite(st, fdt, a.xp, a.ldxp, n, mm, info));
    }
    const void* Xp = a.xp;
    const int64_t ldxp = a.ldxp;

    // CholeskyQR2 of an N x nq (or mm x nq) matrix in place (`two`), or one pass for an
    // intermediate basis of the power iteration (it only has to be well conditioned;
    // the next pass re-orthonormalises it).  A pass whose Cholesky breaks down retries
    // with a diagonal shift (shifted CholeskyQR); a shifted pass leaves a basis of
    // condition up to about u^-1/2, so it is followed by as many clean passes as the
    // mode asks for (two, or one), which run only when their run flag is set.  Shifts
    // are allowed in the first npass - need passes, so a sketch too ill-conditioned even
    // for one shifted pass (condition past u^-1) gets a second one; a breakdown in a
    // pass without a shift is DMD_ERR_CHOL_BREAKDOWN.
    // fl[0..npass): attempt flags of the passes; fl[8..8+npass): their run flags.
    auto cholqr = [&](void* Yb, int64_t ld, int64_t rows, int dtype, int32_t* fl, bool two, int nq) -> int32_t {
        const int need = two ? 2 : 1, npass = two ? 4 : 2;
        const double shift_scale = 11.0 * ((double)rows * nq + (double)nq * (nq + 1)) * u;
        for (int pass = 0; pass < npass; ++pass) {
            const int32_t* skip = pass < need ? nullptr : fl + 8 + pass;
            const bool can_shift = pass < npass - need;
            HIPCHK(gemm_tn(st, dtype, DMD_F64, Yb, ld, 0, nq, Yb, ld, 0, nq, 1, rows, P, G, nq, nullptr, 0, skip));
            HIPCHK(chol_inv(st, G, nq, nq, Rinv, nq, dtype == DMD_F32 ? Rinv32 : nullptr, nq,
                            can_shift ? shift_scale : 0.0, can_shift ? fl + pass : nullptr, info, skip,
                            fl + 8 + pass + 1, can_shift ? need : 0));
            HIPCHK(gemm_nn(st, dtype, Yb, ld, dtype == DMD_F32 ? (const void*)Rinv32 : (const void*)Rinv, nq,
                           Yb, ld, 0, rows, nq, nq, skip, 1));
        }
        return DMD_OK;
    };
    if (!exact) {
        const int cdt = mixed ? DMD_F32 : DMD_F64;   // MFMA type of the streaming products
        // sketch Y = X Omega (Sec. 4.3)
        HIPCHK(gemm_nn(st, fdt, a.x, a.ldx, o.omega, mm, Y, ldy, 0, n, mm, l, nullptr));
        if (int32_t e = cholqr(Y, ldy, n, fdt, flags + 0, o.q == 0, l)) return e;
        // power iterations: W = orth(X^T Q), Y = X W, Q = orth(Y)
        for (int it = 0; it < o.q; ++it) {
            HIPCHK(gemm_tn(st, fdt, cdt, a.x, a.ldx, 0, mm, Y, ldy, 0, l, 0, n, P, Wt, mm, nullptr, 0, nullptr));
            if (int32_t e = cholqr(Wt, mm, mm, DMD_F64, flags + 16 * (1 + 2 * it), false, l)) return e;
            if (fdt == DMD_F32) HIPCHK(to_f32(st, mm, l, l, Wt, mm, (float*)Wtf, mm));
            else HIPCHK(copy_f64(st, mm, l, l, Wt, mm, (double*)Wtf, mm));
            HIPCHK(gemm_nn(st, fdt, a.x, a.ldx, Wtf, mm, Y, ldy, 0, n, mm, l, nullptr));
            if (int32_t e = cholqr(Y, ldy, n, fdt, flags + 16 * (2 + 2 * it), it == o.q - 1, l)) return e;
        }
        // projection B = Q^T X, B' = Q^T X' (one pass over Z when X' is the shifted view).
        // Its sums over N run on the FP64 MFMA on both paths: B feeds the small factors
        // directly, and FP32 accumulation over the rows of a split was the largest error
        // of the mixed path's eigenvalues (FP32 sums: amplitude-weighted 1.5e-5 on an
        // 289,536-row scene of 32 pairs; FP64 sums: 6.9e-6).
        if (shifted) {
            HIPCHK(gemm_tn(st, fdt, DMD_F64, Y, ldy, 0, l, a.x, a.ldx, 0, mm + 1, 0, n, P, Bx, l, nullptr, 0, nullptr));
        } else {
            HIPCHK(gemm_tn(st, fdt, DMD_F64, Y, ldy, 0, l, a.x, a.ldx, 0, mm, 0, n, P, Bx, l, nullptr, 0, nullptr));
            HIPCHK(gemm_tn(st, fdt, DMD_F64, Y, ldy, 0, l, Xp, ldxp, 0, mm, 0, n, P, Bp, l, nullptr, 0, nullptr));
        }
        // SVD of B through the symmetric eigen-decomposition of B B^T: sigma_i^2 and the
        // left vectors U_r of the r largest
        HIPCHK(small_gemm(st, 0, 1, l, l, mm, 1.0, Bx, l, Bx, l, 0.0, G, l));
        HIPCHK(sym_eig(st, G, l, l, r, evals, Ueig, l, symws, info));
        HIPCHK(sigma_from_evals(st, evals, r, o.rank_tol, sigma, model->sigma, info));
        // Vs = V_r S_r^-1, written for the computed U_r as B^T U_r (U_r^T B B^T U_r)^-1 (the
        // same matrix when U_r holds exact singular vectors; for any basis of their span it
        // gives a reduced operator similar to the exact one and the same modes).  With
        // C = B^T U_r S_r^-1 (close to V_r) and C^T C = R^T R:  Vs = C R^-1 R^-T S_r^-1.
        HIPCHK(small_gemm(st, 1, 0, mm, r, l, 1.0, Bx, l, Ueig, l, 0.0, Vs, mm));
        HIPCHK(scale_cols(st, mm, r, Vs, mm, sigma, 1));
        HIPCHK(small_gemm(st, 1, 0, r, r, mm, 1.0, Vs, mm, Vs, mm, 0.0, G, r));
        HIPCHK(chol_inv(st, G, r, r, Rinv, r, nullptr, 0, 0.0, nullptr, info, nullptr));
        HIPCHK(small_gemm(st, 0, 0, mm, r, r, 1.0, Vs, mm, Rinv, r, 0.0, T1, mm));
        HIPCHK(small_gemm(st, 0, 1, mm, r, r, 1.0, T1, mm, Rinv, r, 0.0, Vs, mm));
        HIPCHK(scale_cols(st, mm, r, Vs, mm, sigma, 1));
        // Atilde = U_r^T B' V_r S_r^-1
        HIPCHK(small_gemm(st, 0, 0, l, r, mm, 1.0, Bp, l, Vs, mm, 0.0, T1, l));
        HIPCHK(small_gemm(st, 1, 0, r, r, l, 1.0, Ueig, l, T1, l, 0.0, At, r));
    } else if (qr_route) {
        // Q R_Z = [X X'] (or X) by shifted CholeskyQR in FP64, R_Z = Q^T [X X'] (one more pass,
        // exact up to rounding), and the singular values and right vectors of R = R_Z(0:m-1,
        // 0:m-1), X's own, from the symmetric matrix [[0, R], [R^T, 0]]: its eigenvalues are
        // +-sigma_i, so the small singular values keep relative accuracy u kappa (the Gram
        // X^T X would square kappa), and the eigenvector of +sigma_i is [u_i; v_i] / sqrt(2).
        HIPCHK(copy_f64(st, (int)n, nc, nc, (const double*)a.x, a.ldx, Qb, ldy));
        if (int32_t e = cholqr(Qb, ldy, n, DMD_F64, flags + 0, true, nc)) return e;
        HIPCHK(gemm_tn(st, DMD_F64, DMD_F64, Qb, ldy, 0, nc, a.x, a.ldx, 0, nc, 0, n, P, RZ, nc, nullptr, 0, nullptr));
        if (!shifted)
            HIPCHK(gemm_tn(st, DMD_F64, DMD_F64, Qb, ldy, 0, mm, Xp, ldxp, 0, mm, 0, n, P, RP, mm, nullptr, 0, nullptr));
        HIPCHK(jw_build(st, mm, RZ, nc, Jm));
        HIPCHK(sym_eig(st, Jm, 2 * mm, 2 * mm, r, evals, Ujw, 2 * mm, symws, info));
        HIPCHK(sigma_from_evals(st, evals, r, o.rank_tol, sigma, model->sigma, info, 0));
        // V_r (unit columns, also read by the OptDMD refinement), then Vs = V_r S_r^-1
        HIPCHK(copy_f64(st, mm, r, r, Ujw + mm, 2 * mm, Ueig, mm, 1.4142135623730951));
        HIPCHK(copy_f64(st, mm, r, r, Ueig, mm, Vs, mm));
        HIPCHK(scale_cols(st, mm, r, Vs, mm, sigma, 1));
        // X Vs = Q Ys and X' Vs = Q Yp with Ys = R_Z(:, 0:m-1) Vs, Yp = R_Z(:, 1:m) Vs (or
        // Q^T X' Vs); Atilde = (Ys^T Ys)^-1 Ys^T Yp, the operator on the span of X Vs in that
        // basis (similar to the exact one for any basis of the span, the same modes X' Vs W).
        HIPCHK(small_gemm(st, 0, 0, nc, r, mm, 1.0, RZ, nc, Vs, mm, 0.0, Ys, nc));
        if (shifted) HIPCHK(small_gemm(st, 0, 0, nc, r, mm, 1.0, RZ + nc, nc, Vs, mm, 0.0, Yp, nc));
        else HIPCHK(small_gemm(st, 0, 0, mm, r, mm, 1.0, RP, mm, Vs, mm, 0.0, Yp, mm));
        HIPCHK(small_gemm(st, 1, 0, r, r, nc, 1.0, Ys, nc, Ys, nc, 0.0, PhiG, r));
        HIPCHK(chol_inv(st, PhiG, r, r, Rinv, r, nullptr, 0, 0.0, nullptr, info, nullptr));
        HIPCHK(small_gemm(st, 1, 0, r, r, nc, 1.0, Ys, nc, Yp, nc, 0.0, W, r));
        HIPCHK(small_gemm(st, 1, 0, r, r, r, 1.0, Rinv, r, W, r, 0.0, PhiG, r));
        HIPCHK(small_gemm(st, 0, 0, r, r, r, 1.0, Rinv, r, PhiG, r, 0.0, At, r));
    } else {
        // method of snapshots (m - 1 > EXACT_QR_MAX): Gram of [X X'] in FP64
        double* Gxx;
        double* Gxp;
        int64_t ldg;
        if (shifted) {
            HIPCHK(gemm_tn(st, DMD_F64, DMD_F64, a.x, a.ldx, 0, mm + 1, a.x, a.ldx, 0, mm + 1, 1, n, P, G, mm + 1,
                           nullptr, 0, nullptr));
            Gxx = G;
            Gxp = G + (mm + 1);
            ldg = mm + 1;
        } else {
            HIPCHK(gemm_tn(st, DMD_F64, DMD_F64, a.x, a.ldx, 0, mm, a.x, a.ldx, 0, mm, 1, n, P, G, mm, nullptr, 0, nullptr));
            HIPCHK(gemm_tn(st, DMD_F64, DMD_F64, a.x, a.ldx, 0, mm, Xp, ldxp, 0, mm, 0, n, P, Gxp2, mm, nullptr, 0, nullptr));
            Gxx = G;
            Gxp = Gxp2;
            ldg = mm;
        }
        HIPCHK(sym_eig(st, Gxx, ldg, mm, r, evals, Ueig, mm, symws, info));
        HIPCHK(sigma_from_evals(st, evals, r, o.rank_tol, sigma, model->sigma, info));
        HIPCHK(copy_f64(st, mm, r, r, Ueig, mm, Vs, mm));
        HIPCHK(scale_cols(st, mm, r, Vs, mm, sigma, 1));
        // Atilde = (Vs^T X^T X Vs)^-1 Vs^T (X^T X') Vs with Vs = V_r S_r^-1: the operator on
        // the span of X Vs in that basis (the inverse is the identity for exact singular
        // vectors; for any basis of their span the operator is the same).  The modes are
        // X' Vs W.  Vs^T X^T X Vs = R^T R.
        double* T2 = M;   // scratch (mm x r), overwritten below
        HIPCHK(small_gemm(st, 0, 0, mm, r, mm, 1.0, Gxx, ldg, Vs, mm, 0.0, T2, mm));
        HIPCHK(small_gemm(st, 1, 0, r, r, mm, 1.0, Vs, mm, T2, mm, 0.0, PhiG, r));
        HIPCHK(chol_inv(st, PhiG, r, r, Rinv, r, nullptr, 0, 0.0, nullptr, info, nullptr));
        HIPCHK(small_gemm(st, 0, 0, mm, r, mm, 1.0, Gxp, ldg, Vs, mm, 0.0, T2, mm));
        HIPCHK(small_gemm(st, 1, 0, r, r, mm, 1.0, Vs, mm, T2, mm, 0.0, W, r));
        HIPCHK(small_gemm(st, 1, 0, r, r, r, 1.0, Rinv, r, W, r, 0.0, PhiG, r));
        HIPCHK(small_gemm(st, 0, 0, r, r, r, 1.0, Rinv, r, PhiG, r, 0.0, At, r));
    }
    // eigen-decomposition, canonical order, folded eigenvectors
    HIPCHK(nonsym_eig(st, At, r, r, eigws, model->lam, model->kind, W, info, defl_tol));
    // exact modes Phi = X' V_r S_r^-1 W
    HIPCHK(small_gemm(st, 0, 0, mm, r, r, 1.0, Vs, mm, W, r, 0.0, M, mm));
    if (fdt == DMD_F32) HIPCHK(to_f32(st, mm, r, (int)ldphi, M, mm, (float*)Mf, mm));
    else HIPCHK(copy_f64(st, mm, r, (int)ldphi, M, mm, (double*)Mf, mm));
    HIPCHK(gemm_nn(st, fdt, Xp, ldxp, Mf, mm, model->phi, ldphi, 1, n, mm, (int)ldphi, nullptr));
    // amplitudes b = Phi^+ x0 from the FP64 Gram of Phi
    HIPCHK(gemm_tn(st, fdt, DMD_F64, model->phi, ldphi, 1, r, model->phi, ldphi, 1, r, 1, n, P, PhiG, r, nullptr, 0, nullptr));
    HIPCHK(gemm_tn(st, fdt, DMD_F64, model->phi, ldphi, 1, r, a.x, a.ldx, 0, 1, 0, n, P, rhs, r, nullptr, 0, nullptr));
    HIPCHK(chol_inv(st, PhiG, r, r, RinvPhi, r, nullptr, 0, 11.0 * ((double)n * r + (double)r * (r + 1)) * u,
                    flags + 16 * (1 + 2 * qf), info, nullptr));
    HIPCHK(normal_solve(st, r, RinvPhi, r, rhs, beta, 0));
    if (fdt == DMD_F64) {
        // one step of iterative refinement: beta += G^-1 Phi^T (x0 - Phi beta)
        HIPCHK(residual(st, fdt, n, r, model->phi, ldphi, beta, a.x, res));
        HIPCHK(gemm_tn(st, fdt, DMD_F64, model->phi, ldphi, 1, r, res, n, 0, 1, 0, n, P, rhs2, r, nullptr, 0, nullptr));
        HIPCHK(normal_solve(st, r, RinvPhi, r, rhs2, beta, 1));
    }
    HIPCHK(beta_to_b(st, r, beta, model->kind, model->b));
    return DMD_OK;
}

// ---------------------------------------------------------------- OptDMD refinement
// Levenberg-Marquardt on theta (real folded parameters, one per column) for
// min ||Y - Phi(theta) B||_F with B = Phi^+ Y eliminated (eq. variable_projection), then
// the modes of eq. phi_optdmd written into the model.  Driven from the device: every
// trial point is the same fixed sequence of launches, run only while the iteration goes
// on (ist[VP_RUN]); vp_decide keeps a trial point when it lowers the cost (mu / 4), else
// mu * 4, and stops the iteration when a kept step gains at most 1e-13 of the cost, after
// 200 kept steps, after 40 rejections in a row, or when mu passes 1e20.  A waiting call
// enqueues trial points in groups of VP_GROUP and reads the run flag after each group;
// an asynchronous one (or a scene of dmd_fit_batched) enqueues a fixed number of them.
constexpr int VP_GROUP = 8;
constexpr int VP_DEFAULT_TRIALS = 64;

int32_t optdmd_refine(hipStream_t st, const FitArgs& a, dmd_model* model, FitBufs& fb, bool wait)
{
    const dmd_fit_opts& o = a.o;
    const bool exact = o.precision == DMD_FIT_FP64_EXACT;
    const int T = a.ncols, r = o.r, l = fb.l;
    const int rows = exact ? T : l;
    OptPlan& op = fb.op;
    const double u = 1.1102230246251565e-16;
    const double shift_scale = 11.0 * ((double)T * r + (double)r * (r + 1)) * u;
    const size_t tr = (size_t)T * r;
    double* Yd = op.YE;              // Y
    double* E = op.YE + tr;          // t alpha^(t-1) columns
    double* R = op.RE;               // Y - Phi B
    double* Et = op.RE + tr;         // E - Phi F
    int32_t* run = op.ist + VP_RUN;
    const int32_t* apply = op.ist + VP_APPLY;
    HIPCHK(vp_begin(st, model->info, op.ist, op.scr));
    // data Y = V_r S_r: B^T U_r on the randomized paths (B = Q^T X), V_r S_r on the exact one
    if (!exact) {
        HIPCHK(small_gemm(st, 1, 0, T, r, l, 1.0, fb.Bx, l, fb.Ueig, l, 0.0, Yd, T, apply));
    } else {
        HIPCHK(copy_f64(st, T, r, r, fb.Ueig, T, Yd, T, 1.0, apply));
        HIPCHK(scale_cols(st, T, r, Yd, T, fb.sigma, 0));
    }
    HIPCHK(vp_theta_init(st, r, model->lam, model->kind, op.theta[0]));
    // out (r x nb) = A^T B for T x r A and T x nb B, column-major
    auto tn64 = [&](const double* A, const double* B, int nb, int sym, double* out, const int32_t* gate) {
        return gemm_tn(st, DMD_F64, DMD_F64, A, T, 0, r, B, T, 0, nb, sym, T, op.Ptn, out, r, nullptr, 0, gate);
    };
    // cost, B, J^T J and J^T r at theta[k], into slot k
    auto evaluate = [&](int k, const int32_t* gate) -> hipError_t {
        hipError_t e;
        if ((e = vp_basis(st, T, r, op.theta[k], model->kind, op.Phi, E, gate))) return e;
        // products over the T snapshots as FP64 MFMA reductions
        if ((e = tn64(op.Phi, op.Phi, r, 1, op.PtP, gate))) return e;
        if ((e = tn64(op.Phi, op.YE, 2 * r, 0, op.PtYE, gate))) return e;     // Phi^T [Y | E]
        if ((e = chol_inv(st, op.PtP, r, r, op.Rv, r, nullptr, 0, shift_scale, op.scr + 1, op.scr, gate))) return e;
        // [B | F] = (Phi^T Phi)^-1 Phi^T [Y | E]
        if ((e = small_gemm(st, 1, 0, r, 2 * r, r, 1.0, op.Rv, r, op.PtYE, r, 0.0, op.tmp, r, gate))) return e;
        if ((e = small_gemm(st, 0, 0, r, 2 * r, r, 1.0, op.Rv, r, op.tmp, r, 0.0, op.BF[k], r, gate))) return e;
        // [R | E~] = [Y | E] - Phi [B | F]
        if ((e = copy_f64(st, T, 2 * r, 2 * r, op.YE, T, op.RE, T, 1.0, gate))) return e;
        if ((e = small_gemm(st, 0, 0, T, 2 * r, r, -1.0, op.Phi, T, op.BF[k], r, 1.0, op.RE, T, gate))) return e;
        // K = E~^T E~, W = B B^T, H = E^T R B^T
        if ((e = tn64(Et, Et, r, 1, op.K, gate))) return e;
        if ((e = small_gemm(st, 0, 1, r, r, r, 1.0, op.BF[k], r, op.BF[k], r, 0.0, op.Wm, r, gate))) return e;
        if ((e = tn64(E, R, r, 0, op.ER, gate))) return e;
        if ((e = small_gemm(st, 0, 1, r, r, r, 1.0, op.ER, r, op.BF[k], r, 0.0, op.H, r, gate))) return e;
        if ((e = vp_sumsq(st, T, r, R, T, op.cost + k, gate))) return e;
        return vp_assemble(st, r, model->kind, op.K, op.Wm, op.H, op.G[k], op.g[k], gate);
    };
    // one trial point from the current point (slot 0) into slot 1, then the decision
    auto trial = [&]() -> hipError_t {
        hipError_t e;
        if ((e = vp_damp(st, r, op.G[0], op.vst + VP_MU, op.A, run, op.scr))) return e;
        if ((e = chol_inv(st, op.A, r, r, op.RinvA, r, nullptr, 0, 0.0, nullptr, op.scr, run))) return e;
        if ((e = normal_solve(st, r, op.RinvA, r, op.g[0], op.delta, 0, run))) return e;
        if ((e = vp_update(st, r, op.theta[0], op.delta, op.theta[1], run, op.scr, op.ist))) return e;
        if ((e = evaluate(1, run))) return e;
        if ((e = vp_decide(st, op.cost + 1, op.scr, op.ist, op.vst))) return e;
        return vp_commit(st, r, op.ist, op.theta[1], op.theta[0], op.BF[1], op.BF[0], op.G[1], op.G[0], op.g[1],
                         op.g[0]);
    };
    HIPCHK(evaluate(0, apply));
    HIPCHK(vp_start(st, op.cost, op.scr, op.ist, op.vst));
    if (wait) {
        // the device stops the iteration after at most VP_MAX_STEPS (VP_MAX_TRIES + 1) trial points
        const int cap = VP_MAX_STEPS * (VP_MAX_TRIES + 1) + VP_GROUP;
        for (int done = 0; done < cap; done += VP_GROUP) {
            for (int t = 0; t < VP_GROUP; ++t) HIPCHK(trial());
            int32_t going = 0;
            HIPCHK(hipMemcpyAsync(&going, run, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (!going) break;
        }
    } else {
        const int n_trials = o.optdmd_trials > 0 ? o.optdmd_trials : VP_DEFAULT_TRIALS;
        for (int t = 0; t < n_trials; ++t) HIPCHK(trial());
    }
    // modes of eq. phi_optdmd: Phi = basis C with C = U_B,r B^T (randomized; basis Q) or
    // V_r S_r^-1 B^T (exact; basis X), columns scaled into the folded unit-norm form; a
    // refinement that did not apply leaves the fit's model as it is
    const double* B = op.BF[0];
    HIPCHK(vp_lift(st, r, model->kind, op.theta[0], B, model->lam, model->b, op.scale, apply));
    if (!exact) {
        HIPCHK(small_gemm(st, 0, 1, l, r, r, 1.0, fb.Ueig, l, B, r, 0.0, op.C, l, apply));
    } else {
        HIPCHK(copy_f64(st, T, r, r, fb.Ueig, T, Et, T, 1.0, apply));          // V_r S_r^-1 (scratch)
        HIPCHK(scale_cols(st, T, r, Et, T, fb.sigma, 1));
        HIPCHK(small_gemm(st, 0, 1, T, r, r, 1.0, Et, T, B, r, 0.0, op.C, T, apply));
    }
    HIPCHK(scale_cols(st, rows, r, op.C, rows, op.scale, 0));
    const int64_t ldphi = model->ldphi;
    if (a.xdtype == DMD_F32) HIPCHK(to_f32(st, rows, r, (int)ldphi, op.C, rows, (float*)op.Cf, rows));
    else HIPCHK(copy_f64(st, rows, r, (int)ldphi, op.C, rows, (double*)op.Cf, rows));
    if (!exact) HIPCHK(gemm_nn(st, a.xdtype, fb.Q, fb.ldq, op.Cf, rows, model->phi, ldphi, 1, a.n, rows, (int)ldphi, apply));
    else HIPCHK(gemm_nn(st, a.xdtype, a.x, a.ldx, op.Cf, rows, model->phi, ldphi, 1, a.n, rows, (int)ldphi, apply));
    HIPCHK(vp_finish(st, op.ist, model->info));
    return DMD_OK;
}

// ---------------------------------------------------------------- reconstruction plan
struct ReconPlan {
    int32_t* status;   // COEF_DOMAIN / COEF_OVERFLOW bits of the last coefficient pass
    int64_t* kdev;
    double* expo;
    void* chi;
    void* clo;
};

size_t c_elem(int mode) { return mode == DMD_RECON_FP64 ? 8 : (mode == DMD_RECON_FP32 ? 4 : 2); }

ReconPlan recon_carve(Carver& cv, int r, int K, int mode)
{
    ReconPlan p;
    const int rp = (int)dmd_phi_ld(r);
    const int Kp = (int)round_up(K, RECON_KPAD);
    p.status = cv.take<int32_t>(64);
    p.kdev = cv.take<int64_t>((size_t)K);
    p.expo = cv.take<double>((size_t)K);
    p.chi = cv.take<char>((size_t)Kp * rp * c_elem(mode));
    p.clo = mode == DMD_RECON_BF16X3 ? cv.take<char>((size_t)Kp * rp * 2) : nullptr;
    return p;
}

int32_t validate_model(const dmd_model* m)
{
    if (!m || !m->phi || !m->lam || !m->b || !m->kind) return DMD_ERR_ARG;
    if (m->n < 1 || m->r < 1) return DMD_ERR_SHAPE;
    if (m->r > RECON_MAX_RP) return DMD_ERR_UNSUPPORTED;
    if (m->dtype != DMD_F32 && m->dtype != DMD_F64) return DMD_ERR_ARG;
    if (m->ldphi < dmd_phi_ld(m->r) || m->ldphi % 32 != 0) return DMD_ERR_ARG;
    if (!aligned16(m->phi)) return DMD_ERR_ARG;
    return DMD_OK;
}

// ---------------------------------------------------------------- autotuner table
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;

std::tuple<int, int, int, int> tune_key(int mode, int rp, int64_t N, int K)
{
    int ln = 0, lk = 0;
    while ((int64_t(1) << (ln + 1)) <= N) ++ln;
    while ((1 << (lk + 1)) <= K) ++lk;
    return std::make_tuple(mode, rp, ln, lk);
}

int tune_lookup(int mode, int rp, int64_t N, int K)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(tune_key(mode, rp, N, K));
    return it == g_tune.end() ? 0 : it->second;
}

int32_t load_cache(const char* path)
{
    FILE* f = fopen(path, "r");
    if (!f) return DMD_ERR_ARG;
    char line[256];
    std::lock_guard<std::mutex> g(g_tune_mu);
    while (fgets(line, sizeof line, f)) {
        int mode, rp, ln, lk, cfg;
        double us;
        if (line[0] == '#') continue;
        if (line[0] == 't' && line[1] == 'n') {
            int in_dt, c_dt, rc, nbi, nbj, lnn, cand;
            if (sscanf(line + 2, "%d %d %d %d %d %d %d %lf", &in_dt, &c_dt, &rc, &nbi, &nbj, &lnn, &cand, &us) == 8 &&
                cand >= 0 && cand < 64)
                tn_table_set(in_dt, c_dt, rc, nbi, nbj, lnn, cand);
            continue;
        }
        if (sscanf(line, "%d %d %d %d %d %lf", &mode, &rp, &ln, &lk, &cfg, &us) == 6 && cfg >= 0 && cfg < RECON_NCFG)
            g_tune[std::make_tuple(mode, rp, ln, lk)] = cfg;
    }
    fclose(f);
    return DMD_OK;
}

void lib_init()
{
    (void)device_cu_count();
    g_init_error = prepare_kernels();
    if (g_init_error == hipSuccess) {
        void* p = nullptr;
        g_init_error = scratch_address(&p);
    }
    const char* c = getenv("DMDMI_AUTOTUNE_CACHE");
    if (c && *c) load_cache(c);
}

int32_t recon_validate(const dmd_model* m, int K, int mode, size_t ws_bytes, const void* ws)
{
    if (int32_t e = validate_model(m)) return e;
    if (K < 1) return DMD_ERR_SHAPE;
    if (mode < DMD_RECON_FP64 || mode > DMD_RECON_BF16X3) return DMD_ERR_ARG;
    if ((mode == DMD_RECON_FP64) != (m->dtype == DMD_F64)) return DMD_ERR_ARG;
    Carver dry(nullptr);
    recon_carve(dry, m->r, K, mode);
    if (!ws || ws_bytes < dry.bytes()) return DMD_ERR_WORKSPACE;
    return DMD_OK;
}

// exponents + packed coefficients into the workspace
int32_t recon_prepare(hipStream_t st, const dmd_model* m, const int64_t* k_host, const double* t_host, int K,
                      int mode, void* ws, size_t ws_bytes)
{
    if (!k_host && !t_host) return DMD_ERR_ARG;
    if (int32_t e = recon_validate(m, K, mode, ws_bytes, ws)) return e;
    if (!k_host && !(m->dt > 0.0)) return DMD_ERR_ARG;
    if (int32_t e0 = ensure_init()) return e0;
    Carver cv(ws);
    ReconPlan p = recon_carve(cv, m->r, K, mode);
    const int rp = (int)dmd_phi_ld(m->r);
    const int Kp = (int)round_up(K, RECON_KPAD);
    if (k_host) {
        HIPCHK(hipMemcpyAsync(p.kdev, k_host, (size_t)K * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HIPCHK(exponents(st, p.kdev, nullptr, 1.0, K, p.expo));
    } else {
        HIPCHK(hipMemcpyAsync(p.expo, t_host, (size_t)K * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(exponents(st, nullptr, p.expo, 1.0 / m->dt, K, p.expo));
    }
    HIPCHK(fill_i32(st, p.status, 1, 0));
    HIPCHK(powers_pack(st, m->lam, m->b, m->kind, m->r, p.expo, K, Kp, rp, mode, p.chi, p.clo, p.status));
    return DMD_OK;
}

// the reconstruction GEMM from prepared coefficients
int32_t recon_apply(hipStream_t st, const dmd_model* m, int K, int mode, void* U, int64_t ldu, void* ws,
                    size_t ws_bytes, int cfg_override)
{
    if (int32_t e = recon_validate(m, K, mode, ws_bytes, ws)) return e;
    if (!U || ldu < m->n) return DMD_ERR_ARG;
    if (int32_t e0 = ensure_init()) return e0;
    Carver cv(ws);
    ReconPlan p = recon_carve(cv, m->r, K, mode);
    const int rp = (int)dmd_phi_ld(m->r);
    ReconArgs ra{};
    ra.mode = mode;
    ra.phi = m->phi; ra.ldphi = m->ldphi; ra.N = m->n; ra.rp = rp;
    ra.c_hi = p.chi; ra.c_lo = p.clo; ra.K = K;
    ra.U = U; ra.ldu = ldu;
    const int vw = mode == DMD_RECON_FP64 ? 2 : 4;
    ra.vec_store = (ldu % vw == 0) && aligned16(U);
    const int cfg = cfg_override >= 0 ? cfg_override : tune_lookup(mode, rp, m->n, K);
    HIPCHK(recon_launch(st, ra, cfg));
    return DMD_OK;
}

int32_t recon_enqueue(hipStream_t st, const dmd_model* m, const int64_t* k_host, const double* t_host,
                      int K, int mode, void* U, int64_t ldu, void* ws, size_t ws_bytes, int cfg_override)
{
    if (int32_t e = recon_validate(m, K, mode, ws_bytes, ws)) return e;
    if (!U || ldu < m->n) return DMD_ERR_ARG;
    if (int32_t e = recon_prepare(st, m, k_host, t_host, K, mode, ws, ws_bytes)) return e;
    return recon_apply(st, m, K, mode, U, ldu, ws, ws_bytes, cfg_override);
}

// ---------------------------------------------------------------- allocation-free reconstruction
// The workspace of dmd_reconstruct_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  In host code `scratch`
// names a host-side stand-in, so the array is reached only through the device address
// hipGetSymbolAddress gives for each device, taken once per device (at set-up for the
// device current then, else at the first call on a device) and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[DMD_NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

hipError_t scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// ---- forced roll-out workspace
// forcing columns per projection GEMM: 12 output blocks of 16, which the 5 x 3 wave tile
// covers without recomputed blocks for r up to 160
constexpr int ROLL_TC = 192;

struct RollPlan {
    double* P;        // split-N partial products
    double* PhiG;     // r x r FP64 Gram of Phi
    double* Rinv;     // r x r
    int32_t* scratch;
    double* rhs;      // r x T: Phi^T F
    double* tmp;      // r x T: R^-T rhs, then beta
    double* states;   // (T+1) x r complex
    ReconPlan rec;    // coefficients of the T+1 frames
};

RollPlan roll_carve(Carver& cv, int64_t n, int r, int T, int mode)
{
    RollPlan p;
    p.rec = recon_carve(cv, r, T + 1, mode);   // first: its status word opens the workspace
    const int tc = std::min(T, ROLL_TC);
    p.P = cv.take<double>((size_t)tn_max_splits(n) * r * std::max(r, tc));
    p.PhiG = cv.take<double>((size_t)r * r);
    p.Rinv = cv.take<double>((size_t)r * r);
    p.scratch = cv.take<int32_t>(16);
    p.rhs = cv.take<double>((size_t)r * T);
    p.tmp = cv.take<double>((size_t)r * T);
    p.states = cv.take<double>((size_t)2 * r * (T + 1));
    return p;
}

// beta (r x T, ld r) = least-squares coefficients of the folded basis for the T columns of
// F (N x T, ld ldf): FP64 Gram of Phi and its Cholesky inverse, Phi^T F as split-N MFMA
// products in chunks of ROLL_TC columns, then R^-1 R^-T (Phi^T F).  The result lands in
// p.rhs; p.tmp is scratch.
hipError_t project_columns(hipStream_t st, const dmd_model* m, const void* F, int64_t ldf, int T, const RollPlan& p,
                           bool have_rinv)
{
    const int r = m->r;
    const int64_t n = m->n;
    const size_t esz = m->dtype == DMD_F64 ? 8 : 4;
    hipError_t e;
    if (!have_rinv) {
        if ((e = gemm_tn(st, m->dtype, DMD_F64, m->phi, m->ldphi, 1, r, m->phi, m->ldphi, 1, r, 1, n, p.P, p.PhiG, r,
                         nullptr, 0, nullptr)) != hipSuccess) return e;
        if ((e = fill_i32(st, p.scratch, 16, 0)) != hipSuccess) return e;
        if ((e = chol_inv(st, p.PhiG, r, r, p.Rinv, r, nullptr, 0, 0.0, nullptr, p.scratch, nullptr)) != hipSuccess)
            return e;
    }
    for (int c0 = 0; c0 < T; c0 += ROLL_TC) {
        const int nc = std::min(ROLL_TC, T - c0);
        const void* fc = (const char*)F + (size_t)c0 * (size_t)ldf * esz;
        // FP32 models: FP32 MFMA products, split-N partials summed in FP64 (as the fit's X^T Q)
        if ((e = gemm_tn(st, m->dtype, m->dtype, m->phi, m->ldphi, 1, r, fc, ldf, 0, nc, 0, n, p.P,
                         p.rhs + (size_t)c0 * r, r, nullptr, 0, nullptr)) != hipSuccess) return e;
    }
    if ((e = small_gemm(st, 1, 0, r, T, r, 1.0, p.Rinv, r, p.rhs, r, 0.0, p.tmp, r)) != hipSuccess) return e;
    return small_gemm(st, 0, 0, r, T, r, 1.0, p.Rinv, r, p.tmp, r, 0.0, p.rhs, r);
}

struct UpPlan {
    RollPlan rp;
    double* beta0;    // r: coefficients of h0
    double* tmp0;     // r
    int32_t* low;     // r flags
};

UpPlan up_carve(Carver& cv, int64_t n, int r, int T, int mode)
{
    UpPlan u;
    u.rp = roll_carve(cv, n, r, T, mode);
    u.beta0 = cv.take<double>((size_t)r);
    u.tmp0 = cv.take<double>((size_t)r);
    u.low = cv.take<int32_t>((size_t)r);
    return u;
}

// frames Re(Phi z_s), s = 0 .. K-1, from K reduced states
hipError_t frames_from_states(hipStream_t st, const dmd_model* m, const double* states, int K, int mode,
                              const ReconPlan& rec, void* U, int64_t ldu)
{
    const int rp = (int)dmd_phi_ld(m->r);
    const int Kp = (int)round_up(K, RECON_KPAD);
    hipError_t e = pack_states(st, states, m->kind, m->r, K, Kp, rp, mode, rec.chi, rec.clo, rec.status);
    if (e != hipSuccess) return e;
    ReconArgs ra{};
    ra.mode = mode;
    ra.phi = m->phi; ra.ldphi = m->ldphi; ra.N = m->n; ra.rp = rp;
    ra.c_hi = rec.chi; ra.c_lo = rec.clo; ra.K = K;
    ra.U = U; ra.ldu = ldu;
    const int vw = mode == DMD_RECON_FP64 ? 2 : 4;
    ra.vec_store = (ldu % vw == 0) && aligned16(U);
    return recon_launch(st, ra, tune_lookup(mode, rp, m->n, K));
}

}  // namespace

// ====================================================================== extern "C"
extern "C" {

int32_t dmd_abi_version(void) { return DMDMI_ABI_VERSION; }

const char* dmd_status_string(int32_t s)
{
    switch (s) {
    case DMD_OK: return "ok";
    case DMD_ERR_ARG: return "invalid argument (null pointer, enum, alignment or leading dimension)";
    case DMD_ERR_SHAPE: return "inconsistent or unsupported shape";
    case DMD_ERR_WORKSPACE: return "workspace too small";
    case DMD_ERR_NONFINITE: return "non-finite value in the input";
    case DMD_ERR_CHOL_BREAKDOWN: return "CholeskyQR breakdown (sketch numerically rank deficient)";
    case DMD_ERR_RANK: return "sigma_r below the rank tolerance";
    case DMD_ERR_EIG_NOCONV: return "eigen-solver did not converge";
    case DMD_ERR_DOMAIN: return "lambda = 0 raised to a negative or fractional power";
    case DMD_ERR_OVERFLOW: return "result outside the output type's range";
    case DMD_ERR_HIP: return "HIP runtime error";
    case DMD_ERR_UNSUPPORTED: return "size beyond the small-matrix kernels' limits";
    case DMD_ERR_IO: return "model file missing, unwritable, truncated or corrupted";
    default: return "unknown status";
    }
}

int64_t dmd_phi_ld(int32_t r) { return round_up(std::max(r, 1), 32); }

int32_t dmd_fit_workspace_size(int64_t n, int32_t ncols, int32_t xdtype, const dmd_fit_opts* opts, size_t* bytes)
{
    if (!opts || !bytes) return DMD_ERR_ARG;
    FitArgs a{nullptr, nullptr, n, ncols, n, n, xdtype, *opts, false};
    if (int32_t e = validate_fit(a, nullptr, false)) return e;
    // size for the larger of the two projection layouts
    Carver c1(nullptr);
    fit_plan(c1, nullptr, a, nullptr);
    a.shifted = true;
    Carver c2(nullptr);
    fit_plan(c2, nullptr, a, nullptr);
    *bytes = std::max(c1.bytes(), c2.bytes());
    return DMD_OK;
}

int32_t dmd_fit(void* stream, const void* x, const void* xp, int64_t n, int32_t ncols, int64_t ldx,
                int64_t ldxp, int32_t xdtype, const dmd_fit_opts* opts, void* ws, size_t ws_bytes,
                dmd_model* model)
{
    if (!opts) return DMD_ERR_ARG;
    FitArgs a{x, xp, n, ncols, ldx, ldxp, xdtype, *opts, is_shifted_view(x, xp, ldx, ldxp, xdtype)};
    if (int32_t e = validate_fit(a, model, true)) return e;
    size_t need = 0;
    if (int32_t e = dmd_fit_workspace_size(n, ncols, xdtype, opts, &need)) return e;
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    {
        // the carve of this very call (its layout and the caller's ldphi) must fit as well
        Carver dry(nullptr);
        fit_plan(dry, nullptr, a, model);
        if (dry.bytes() > ws_bytes) return DMD_ERR_WORKSPACE;
    }
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    model->r = opts->r;
    model->dtype = xdtype;
    model->dt = opts->dt;
    Carver cv(ws);
    FitBufs fb{};
    if (int32_t e = fit_plan(cv, st, a, model, &fb)) return e;
    if (opts->flags & DMD_FIT_OPTDMD)
        if (int32_t e = optdmd_refine(st, a, model, fb, !(opts->flags & DMD_FIT_ASYNC))) return e;
    if (opts->flags & DMD_FIT_ASYNC) return DMD_OK;
    int32_t status = 0;
    HIPCHK(hipMemcpyAsync(&status, model->info, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return status;
}

int32_t dmd_autotune_fit(void* stream, const void* x, const void* xp, int64_t n, int32_t ncols, int64_t ldx,
                         int64_t ldxp, int32_t xdtype, const dmd_fit_opts* opts, void* ws, size_t ws_bytes,
                         dmd_model* model, const char* cache_path)
{
    if (!opts) return DMD_ERR_ARG;
    dmd_fit_opts o = *opts;
    o.flags &= ~(DMD_FIT_ASYNC | DMD_FIT_OPTDMD);
    FitArgs a{x, xp, n, ncols, ldx, ldxp, xdtype, o, is_shifted_view(x, xp, ldx, ldxp, xdtype)};
    if (int32_t e = validate_fit(a, model, true)) return e;
    size_t need = 0;
    if (int32_t e = dmd_fit_workspace_size(n, ncols, xdtype, &o, &need)) return e;
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    {
        Carver dry(nullptr);
        fit_plan(dry, nullptr, a, model);
        if (dry.bytes() > ws_bytes) return DMD_ERR_WORKSPACE;
    }
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    model->r = o.r;
    model->dtype = xdtype;
    model->dt = o.dt;
    Carver cv(ws);
    tn_record(true);
    const int32_t fe = fit_plan(cv, st, a, model);
    tn_record(false);
    if (fe) return fe;
    HIPCHK(hipStreamSynchronize(st));
    std::vector<std::string> lines;
    HIPCHK(tn_tune_recorded(st, &lines));
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (!f) return DMD_ERR_IO;
        for (auto& l : lines) fprintf(f, "%s\n", l.c_str());
        fclose(f);
    }
    int32_t status = 0;
    HIPCHK(hipMemcpyAsync(&status, model->info, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return status;
}

int32_t dmd_reconstruct_workspace_size(int32_t r, int32_t K, int32_t mode, size_t* bytes)
{
    if (!bytes) return DMD_ERR_ARG;
    if (r < 1 || K < 1) return DMD_ERR_SHAPE;
    if (mode < DMD_RECON_FP64 || mode > DMD_RECON_BF16X3) return DMD_ERR_ARG;
    Carver c(nullptr);
    recon_carve(c, r, K, mode);
    *bytes = c.bytes();
    return DMD_OK;
}

int32_t dmd_reconstruct(void* stream, const dmd_model* model, const int64_t* k_host, int32_t K, int32_t mode,
                        void* U, int64_t ldu, void* ws, size_t ws_bytes)
{
    if (!k_host) return DMD_ERR_ARG;
    return recon_enqueue((hipStream_t)stream, model, k_host, nullptr, K, mode, U, ldu, ws, ws_bytes, -1);
}

int32_t dmd_reconstruct_noalloc(void* stream, const dmd_model* model, const int64_t* k_host, int32_t K, int32_t mode,
                                void* U, int64_t ldu, int32_t* status)
{
    if (!k_host) return DMD_ERR_ARG;
    if (int32_t e = validate_model(model)) return e;
    if (K < 1) return DMD_ERR_SHAPE;
    if (mode < DMD_RECON_FP64 || mode > DMD_RECON_BF16X3) return DMD_ERR_ARG;
    Carver dry(nullptr);
    recon_carve(dry, model->r, K, mode);
    if (dry.bytes() > DMD_NOALLOC_SCRATCH_BYTES) return DMD_ERR_WORKSPACE;
    if (int32_t e0 = ensure_init()) return e0;
    void* ws = nullptr;
    HIPCHK(scratch_address(&ws));
    hipStream_t st = (hipStream_t)stream;
    if (int32_t e = recon_enqueue(st, model, k_host, nullptr, K, mode, U, ldu, ws, DMD_NOALLOC_SCRATCH_BYTES, -1))
        return e;
    // the status word sits at the start of the scratch (as at the start of a workspace)
    if (status) HIPCHK(hipMemcpyAsync(status, ws, sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    return DMD_OK;
}

int32_t dmd_reconstruct_prepare(void* stream, const dmd_model* model, const int64_t* k_host, const double* t_host,
                                int32_t K, int32_t mode, void* ws, size_t ws_bytes)
{
    for (int32_t j = 0; !k_host && t_host && j < K; ++j)
        if (!isfinite(t_host[j])) return DMD_ERR_ARG;
    return recon_prepare((hipStream_t)stream, model, k_host, t_host, K, mode, ws, ws_bytes);
}

int32_t dmd_reconstruct_apply(void* stream, const dmd_model* model, int32_t K, int32_t mode, void* U, int64_t ldu,
                              void* ws, size_t ws_bytes)
{
    return recon_apply((hipStream_t)stream, model, K, mode, U, ldu, ws, ws_bytes, -1);
}

int32_t dmd_integrate(void* stream, const dmd_model* model, const double* t_host, int32_t T, int32_t mode,
                      void* U, int64_t ldu, void* ws, size_t ws_bytes)
{
    if (!t_host) return DMD_ERR_ARG;
    if (model && !(model->dt > 0.0)) return DMD_ERR_ARG;
    for (int32_t j = 0; t_host && j < T; ++j)
        if (!isfinite(t_host[j])) return DMD_ERR_ARG;
    return recon_enqueue((hipStream_t)stream, model, nullptr, t_host, T, mode, U, ldu, ws, ws_bytes, -1);
}

int32_t dmd_edit_modes(void* stream, const dmd_model* model, const dmd_edit* edit, const double* mode_edit,
                       double* lam_out, double* b_out, int32_t* cluster_out)
{
    if (int32_t e = validate_model(model)) return e;
    if (!edit || !lam_out || !b_out) return DMD_ERR_ARG;
    if (!(model->dt > 0.0) || !isfinite(model->dt)) return DMD_ERR_ARG;
    if (!isfinite(edit->freq_cut) || edit->freq_cut < 0.0) return DMD_ERR_ARG;
    for (int c = 0; c < 2; ++c)
        if (!isfinite(edit->weight[c]) || !isfinite(edit->re_scale[c]) || !isfinite(edit->re_shift[c]) ||
            !isfinite(edit->im_scale[c]))
            return DMD_ERR_ARG;
    if (int32_t e0 = ensure_init()) return e0;
    HIPCHK(edit_modes((hipStream_t)stream, model->r, model->dt, *edit, mode_edit, model->lam, model->b, lam_out,
                      b_out, cluster_out));
    return DMD_OK;
}

int32_t dmd_project_workspace_size(int64_t n, int32_t r, size_t* bytes)
{
    if (!bytes) return DMD_ERR_ARG;
    if (n < 1 || r < 1) return DMD_ERR_SHAPE;
    Carver c(nullptr);
    c.take<double>((size_t)tn_max_splits(n) * r * r);
    c.take<double>((size_t)r * r);
    c.take<double>((size_t)r);
    c.take<double>((size_t)r * r);
    c.take<int32_t>(16);
    c.take<double>((size_t)r);
    c.take<double>((size_t)r);
    c.take<double>((size_t)n);
    *bytes = c.bytes();
    return DMD_OK;
}

int32_t dmd_project(void* stream, const dmd_model* model, const void* u, double* z, void* ws, size_t ws_bytes)
{
    if (int32_t e = validate_model(model)) return e;
    if (!u || !z) return DMD_ERR_ARG;
    size_t need = 0;
    dmd_project_workspace_size(model->n, model->r, &need);
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    const int r = model->r;
    const int64_t n = model->n;
    Carver cv(ws);
    double* P = cv.take<double>((size_t)tn_max_splits(n) * r * r);
    double* PhiG = cv.take<double>((size_t)r * r);
    double* rhs = cv.take<double>((size_t)r);
    double* Rinv = cv.take<double>((size_t)r * r);
    int32_t* scratch = cv.take<int32_t>(16);
    double* beta = cv.take<double>((size_t)r);
    double* rhs2 = cv.take<double>((size_t)r);
    void* res = cv.take<double>((size_t)n);
    HIPCHK(gemm_tn(st, model->dtype, DMD_F64, model->phi, model->ldphi, 1, r, model->phi, model->ldphi, 1, r, 1, n,
                   P, PhiG, r, nullptr, 0, nullptr));
    HIPCHK(gemm_tn(st, model->dtype, DMD_F64, model->phi, model->ldphi, 1, r, u, n, 0, 1, 0, n, P, rhs, r, nullptr,
                   0, nullptr));
    HIPCHK(fill_i32(st, scratch, 16, 0));
    HIPCHK(chol_inv(st, PhiG, r, r, Rinv, r, nullptr, 0, 0.0, nullptr, scratch, nullptr));
    HIPCHK(normal_solve(st, r, Rinv, r, rhs, beta, 0));
    if (model->dtype == DMD_F64) {   // one step of iterative refinement
        HIPCHK(residual(st, model->dtype, n, r, model->phi, model->ldphi, beta, u, res));
        HIPCHK(gemm_tn(st, model->dtype, DMD_F64, model->phi, model->ldphi, 1, r, res, n, 0, 1, 0, n, P, rhs2, r,
                       nullptr, 0, nullptr));
        HIPCHK(normal_solve(st, r, Rinv, r, rhs2, beta, 1));
    }
    HIPCHK(beta_to_b(st, r, beta, model->kind, z));
    return DMD_OK;
}

int32_t dmd_rollout_workspace_size(int64_t n, int32_t r, int32_t T, int32_t mode, size_t* bytes)
{
    if (!bytes) return DMD_ERR_ARG;
    if (n < 1 || r < 1 || T < 1) return DMD_ERR_SHAPE;
    if (mode < DMD_RECON_FP64 || mode > DMD_RECON_BF16X3) return DMD_ERR_ARG;
    Carver c(nullptr);
    roll_carve(c, n, r, T, mode);
    *bytes = c.bytes();
    return DMD_OK;
}

int32_t dmd_rollout(void* stream, const dmd_model* model, const double* z0, const void* f, int64_t ldf, int32_t T,
                    int32_t mode, void* U, int64_t ldu, double* z_out, void* ws, size_t ws_bytes)
{
    if (int32_t e = validate_model(model)) return e;
    if (T < 1) return DMD_ERR_SHAPE;
    if (!(model->dt > 0.0) || !isfinite(model->dt)) return DMD_ERR_ARG;
    if (f && ldf < model->n) return DMD_ERR_ARG;
    if (mode < DMD_RECON_FP64 || mode > DMD_RECON_BF16X3) return DMD_ERR_ARG;
    if (U && ((mode == DMD_RECON_FP64) != (model->dtype == DMD_F64) || ldu < model->n)) return DMD_ERR_ARG;
    size_t need = 0;
    if (int32_t e = dmd_rollout_workspace_size(model->n, model->r, T, mode, &need)) return e;
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    const int r = model->r;
    const int64_t n = model->n;
    Carver cv(ws);
    RollPlan p = roll_carve(cv, n, r, T, mode);
    double* states = z_out ? z_out : p.states;
    const double* beta = nullptr;
    HIPCHK(fill_i32(st, p.rec.status, 1, 0));
    if (f) {
        HIPCHK(project_columns(st, model, f, ldf, T, p, false));   // g_s = Phi^+ f_s, every step
        beta = p.rhs;
    }
    HIPCHK(rollout_scan(st, r, T, model->lam, z0 ? z0 : model->b, beta, r, model->kind, model->dt, states));
    if (U) HIPCHK(frames_from_states(st, model, states, T + 1, mode, p.rec, U, ldu));
    return DMD_OK;
}

int32_t dmd_upsample_workspace_size(int64_t n, int32_t r, int32_t T, int32_t mode, size_t* bytes)
{
    if (!bytes) return DMD_ERR_ARG;
    if (n < 1 || r < 1 || T < 1) return DMD_ERR_SHAPE;
    if (mode < DMD_RECON_FP64 || mode > DMD_RECON_BF16X3) return DMD_ERR_ARG;
    Carver c(nullptr);
    up_carve(c, n, r, T, mode);
    *bytes = c.bytes();
    return DMD_OK;
}

int32_t dmd_upsample(void* stream, const dmd_model* model, const void* h0, const void* l, int64_t ldl, int32_t T,
                     const int32_t* low_host, int32_t mode, void* U, int64_t ldu, double* r_out, void* ws,
                     size_t ws_bytes)
{
    if (int32_t e = validate_model(model)) return e;
    if (T < 1) return DMD_ERR_SHAPE;
    if (!h0 || !l || !low_host || ldl < model->n) return DMD_ERR_ARG;
    if (mode < DMD_RECON_FP64 || mode > DMD_RECON_BF16X3) return DMD_ERR_ARG;
    if (U && ((mode == DMD_RECON_FP64) != (model->dtype == DMD_F64) || ldu < model->n)) return DMD_ERR_ARG;
    size_t need = 0;
    if (int32_t e = dmd_upsample_workspace_size(model->n, model->r, T, mode, &need)) return e;
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    const int r = model->r;
    Carver cv(ws);
    UpPlan u = up_carve(cv, model->n, r, T, mode);
    HIPCHK(fill_i32(st, u.rp.rec.status, 1, 0));
    RollPlan p0 = u.rp;                 // h0 uses the same Gram and inverse, its own coefficients
    p0.rhs = u.beta0;
    p0.tmp = u.tmp0;
    HIPCHK(project_columns(st, model, h0, model->n, 1, p0, false));
    HIPCHK(project_columns(st, model, l, ldl, T, u.rp, true));
    HIPCHK(hipMemcpyAsync(u.low, low_host, (size_t)r * sizeof(int32_t), hipMemcpyHostToDevice, st));
    double* states = r_out ? r_out : u.rp.states;
    HIPCHK(upsample_states(st, r, T, model->lam, u.beta0, u.rp.rhs, r, model->kind, u.low, states));
    if (U) HIPCHK(frames_from_states(st, model, states, T + 1, mode, u.rp.rec, U, ldu));
    return DMD_OK;
}

int32_t dmd_lowres_project(void* stream, int32_t dtype, const void* h, int64_t ldh, const void* l, int64_t ldl,
                           void* x, int64_t ldx, int64_t nframes, int32_t ncomp, int32_t nz, int32_t ny, int32_t nx,
                           int32_t factor)
{
    if (dtype != DMD_F32 && dtype != DMD_F64) return DMD_ERR_ARG;
    if (!h || !l || !x) return DMD_ERR_ARG;
    if (nframes < 0 || ncomp < 1 || nz < 1 || ny < 1 || nx < 1 || factor < 1) return DMD_ERR_SHAPE;
    if (ny % factor || nx % factor || (nz > 1 && nz % factor)) return DMD_ERR_SHAPE;
    const int fz = nz == 1 ? 1 : factor;
    const int64_t nfine = (int64_t)ncomp * nz * ny * nx;
    const int64_t ncoarse = (int64_t)ncomp * (nz / fz) * (ny / factor) * (nx / factor);
    if (ldh < nfine || ldx < nfine || ldl < ncoarse) return DMD_ERR_ARG;
    if (nframes == 0) return DMD_OK;
    if (int32_t e0 = ensure_init()) return e0;
    HIPCHK(lowres_project((hipStream_t)stream, dtype, h, ldh, l, ldl, x, ldx, nframes, ncomp, nz, ny, nx, factor));
    return DMD_OK;
}

int32_t dmd_loss_grad_workspace_size(int64_t n, int32_t r, int32_t ncols, int32_t dtype, size_t* bytes)
{
    if (!bytes) return DMD_ERR_ARG;
    if (n < 1 || r < 1 || ncols < 1) return DMD_ERR_SHAPE;
    if (dtype != DMD_F32 && dtype != DMD_F64) return DMD_ERR_ARG;
    const int mode = dtype == DMD_F64 ? DMD_RECON_FP64 : DMD_RECON_FP32;
    Carver c(nullptr);
    recon_carve(c, r, ncols, mode);
    c.take<char>((size_t)round_up(n, 4) * ncols * esize(dtype));
    c.take<double>(LG_SS_SLOTS);
    c.take<double>((size_t)tn_max_splits(n) * r * ncols);
    c.take<double>((size_t)r * ncols);
    *bytes = c.bytes();
    return DMD_OK;
}

int32_t dmd_loss_grad(void* stream, const dmd_model* model, const double* lam, const double* b, const void* xt,
                      int64_t ldxt, const int64_t* k_host, int32_t ncols, double* out, void* ws, size_t ws_bytes)
{
    if (int32_t e = validate_model(model)) return e;
    if (!lam || !b || !xt || !k_host || !out) return DMD_ERR_ARG;
    if (ncols < 1) return DMD_ERR_SHAPE;
    if (ldxt < model->n) return DMD_ERR_ARG;
    if ((int64_t)model->r * ncols > TN_MAX_OUT) return DMD_ERR_UNSUPPORTED;
    size_t need = 0;
    dmd_loss_grad_workspace_size(model->n, model->r, ncols, model->dtype, &need);
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    if (int32_t e0 = ensure_init()) return e0;
    // one FP64 loss partial per work-group of the residual launch: its largest grid must fit
    if (recon_max_grid() > LG_SS_SLOTS) return DMD_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const int r = model->r, rp = (int)dmd_phi_ld(r);
    const int64_t n = model->n, ldr = round_up(n, 4);
    const int mode = model->dtype == DMD_F64 ? DMD_RECON_FP64 : DMD_RECON_FP32;
    Carver cv(ws);
    ReconPlan p = recon_carve(cv, r, ncols, mode);
    void* R = cv.take<char>((size_t)ldr * ncols * esize(model->dtype));
    double* ss = cv.take<double>(LG_SS_SLOTS);
    double* P = cv.take<double>((size_t)tn_max_splits(n) * r * ncols);
    double* G = cv.take<double>((size_t)r * ncols);
    HIPCHK(fill_i32(st, p.status, 1, 0));
    HIPCHK(hipMemcpyAsync(p.kdev, k_host, (size_t)ncols * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(exponents(st, p.kdev, nullptr, 1.0, ncols, p.expo));
    HIPCHK(powers_pack(st, lam, b, model->kind, r, p.expo, ncols, (int)round_up(ncols, RECON_KPAD), rp, mode, p.chi,
                       nullptr, p.status));
    int grid = 0;
    ReconArgs ra{};
    ra.mode = mode;
    ra.phi = model->phi; ra.ldphi = model->ldphi; ra.N = n; ra.rp = rp;
    ra.c_hi = p.chi; ra.c_lo = nullptr; ra.K = ncols;
    ra.U = R; ra.ldu = ldr; ra.vec_store = 1;
    ra.xt = xt; ra.ldxt = ldxt; ra.ss_partial = ss; ra.grid_out = &grid;
    HIPCHK(recon_launch(st, ra, 0));
    HIPCHK(gemm_tn(st, model->dtype, model->dtype, model->phi, model->ldphi, 1, r, R, ldr, 0, ncols, 0, n, P, G, r,
                   nullptr, 0, nullptr));
    HIPCHK(grad_reduce(st, r, ncols, G, lam, b, model->kind, p.expo, ss, grid, out));
    return DMD_OK;
}

// ---------------------------------------------------------------- refit statistics
struct RefitPlan {
    int32_t* status;
    int64_t* kdev;
    double* expo;
    double* G0;     // Phi_f^T X (r x ncols)
    double* M;      // Phi_f^T Phi_f (r x r)
    double* xxp;    // ||X||^2 partials
    double* P;      // split partials of the two products
    double* C;      // folded FP64 coefficients (r x ncols)
    double* Gf;     // Phi_f^T R (r x ncols)
    double* loss;
};

static RefitPlan refit_carve(Carver& cv, int64_t n, int r, int ncols)
{
    RefitPlan p;
    p.status = cv.take<int32_t>(64);
    p.kdev = cv.take<int64_t>((size_t)ncols);
    p.expo = cv.take<double>((size_t)ncols);
    p.G0 = cv.take<double>((size_t)r * ncols);
    p.M = cv.take<double>((size_t)r * r);
    p.xxp = cv.take<double>(SQ_MAX_PARTS);
    p.P = cv.take<double>((size_t)tn_max_splits(n) * std::max<int64_t>((int64_t)r * ncols, (int64_t)r * r));
    p.C = cv.take<double>((size_t)r * ncols);
    p.Gf = cv.take<double>((size_t)r * ncols);
    p.loss = cv.take<double>(8);
    return p;
}

int32_t dmd_refit_workspace_size(int64_t n, int32_t r, int32_t ncols, size_t* bytes)
{
    if (!bytes) return DMD_ERR_ARG;
    if (n < 1 || r < 1 || ncols < 1) return DMD_ERR_SHAPE;
    Carver c(nullptr);
    refit_carve(c, n, r, ncols);
    *bytes = c.bytes();
    return DMD_OK;
}

int32_t dmd_refit_prepare(void* stream, const dmd_model* model, const void* xt, int64_t ldxt, const int64_t* k_host,
                          int32_t ncols, void* ws, size_t ws_bytes)
{
    if (int32_t e = validate_model(model)) return e;
    if (!xt || !k_host) return DMD_ERR_ARG;
    if (ncols < 1) return DMD_ERR_SHAPE;
    if (ldxt < model->n) return DMD_ERR_ARG;
    if ((int64_t)model->r * ncols > TN_MAX_OUT) return DMD_ERR_UNSUPPORTED;
    size_t need = 0;
    dmd_refit_workspace_size(model->n, model->r, ncols, &need);
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    const int r = model->r;
    const int64_t n = model->n;
    Carver cv(ws);
    RefitPlan p = refit_carve(cv, n, r, ncols);
    HIPCHK(hipMemcpyAsync(p.kdev, k_host, (size_t)ncols * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(exponents(st, p.kdev, nullptr, 1.0, ncols, p.expo));
    // G0 = Phi_f^T X and M = Phi_f^T Phi_f with FP64 sums (FP64 MFMA on the model's data)
    HIPCHK(gemm_tn(st, model->dtype, DMD_F64, model->phi, model->ldphi, 1, r, xt, ldxt, 0, ncols, 0, n, p.P, p.G0, r,
                   nullptr, 0, nullptr));
    HIPCHK(gemm_tn(st, model->dtype, DMD_F64, model->phi, model->ldphi, 1, r, model->phi, model->ldphi, 1, r, 1, n, p.P,
                   p.M, r, nullptr, 0, nullptr));
    int nparts = 0;
    HIPCHK(sumsq(st, model->dtype, xt, ldxt, n, ncols, p.xxp, &nparts));
    return DMD_OK;
}

int32_t dmd_refit_loss_grad(void* stream, const dmd_model* model, const double* lam, const double* b, int32_t ncols,
                            double* out, void* ws, size_t ws_bytes)
{
    if (int32_t e = validate_model(model)) return e;
    if (!lam || !b || !out) return DMD_ERR_ARG;
    if (ncols < 1) return DMD_ERR_SHAPE;
    if ((int64_t)model->r * ncols > TN_MAX_OUT) return DMD_ERR_UNSUPPORTED;
    size_t need = 0;
    dmd_refit_workspace_size(model->n, model->r, ncols, &need);
    if (!ws || ws_bytes < need) return DMD_ERR_WORKSPACE;
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    const int r = model->r;
    Carver cv(ws);
    RefitPlan p = refit_carve(cv, model->n, r, ncols);
    HIPCHK(fill_i32(st, p.status, 1, 0));
    HIPCHK(powers_pack(st, lam, b, model->kind, r, p.expo, ncols, ncols, r, DMD_RECON_FP64, p.C, nullptr, p.status));
    // G_f = G0 - M C, L = ||X||^2 - <C, G0 + G_f>
    HIPCHK(copy_f64(st, r, ncols, ncols, p.G0, r, p.Gf, r));
    HIPCHK(small_gemm(st, 0, 0, r, ncols, r, -1.0, p.M, r, p.C, r, 1.0, p.Gf, r));
    HIPCHK(refit_loss(st, r, ncols, p.C, p.G0, p.Gf, p.xxp, sumsq_parts(model->n), p.loss));
    HIPCHK(grad_reduce(st, r, ncols, p.Gf, lam, b, model->kind, p.expo, p.loss, 1, out));
    return DMD_OK;
}

int32_t dmd_status_word(void* stream, const void* ws, int32_t* status)
{
    if (!ws || !status) return DMD_ERR_ARG;
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t st = (hipStream_t)stream;
    int32_t bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, ws, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *status = (bits & COEF_DOMAIN) ? DMD_ERR_DOMAIN : ((bits & COEF_OVERFLOW) ? DMD_ERR_OVERFLOW : DMD_OK);
    return DMD_OK;
}

}  // extern "C"

// ====================================================================== batched fit + graphs
struct dmd_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
};

extern "C" {

int32_t dmd_fit_batched(void* stream, int32_t nscenes, const dmd_scene* scenes, dmd_model* models, int32_t capture,
                        dmd_graph** graph)
{
    if (nscenes < 1 || !scenes || !models) return DMD_ERR_ARG;
    if (capture && !graph) return DMD_ERR_ARG;
    if (capture && !stream) return DMD_ERR_ARG;   // the legacy null stream cannot be captured
    for (int i = 0; i < nscenes; ++i) {
        const dmd_scene& sc = scenes[i];
        FitArgs a{sc.x, sc.xp, sc.n, sc.ncols, sc.ldx, sc.ldxp, sc.xdtype, sc.opts,
                  is_shifted_view(sc.x, sc.xp, sc.ldx, sc.ldxp, sc.xdtype)};
        if (int32_t e = validate_fit(a, &models[i], true)) return e;
        size_t need = 0;
        if (int32_t e = dmd_fit_workspace_size(sc.n, sc.ncols, sc.xdtype, &sc.opts, &need)) return e;
        if (!sc.ws || sc.ws_bytes < need) return DMD_ERR_WORKSPACE;
        Carver dry(nullptr);
        fit_plan(dry, nullptr, a, &models[i]);
        if (dry.bytes() > sc.ws_bytes) return DMD_ERR_WORKSPACE;
    }
    if (int32_t e0 = ensure_init()) return e0;
    hipStream_t origin = (hipStream_t)stream;
    dmd_graph* g = new dmd_graph();
    auto cleanup = [&](int32_t code) {
        for (auto e : g->events) hipEventDestroy(e);
        for (auto s : g->streams) hipStreamDestroy(s);
        if (g->exec) hipGraphExecDestroy(g->exec);
        if (g->graph) hipGraphDestroy(g->graph);
        delete g;
        return code;
    };
    g->events.resize(nscenes + 1, nullptr);
    g->streams.resize(nscenes, nullptr);
    for (int i = 0; i <= nscenes; ++i)
        if (hipEventCreateWithFlags(&g->events[i], hipEventDisableTiming) != hipSuccess) return cleanup(DMD_ERR_HIP);
    for (int i = 0; i < nscenes; ++i)
        if (hipStreamCreateWithFlags(&g->streams[i], hipStreamNonBlocking) != hipSuccess) return cleanup(DMD_ERR_HIP);
    // fork: every scene on its own stream after the origin's prior work, joined back into origin
    auto enqueue_all = [&]() -> int32_t {
        if (hipEventRecord(g->events[nscenes], origin) != hipSuccess) return DMD_ERR_HIP;
        for (int i = 0; i < nscenes; ++i) {
            const dmd_scene& sc = scenes[i];
            FitArgs a{sc.x, sc.xp, sc.n, sc.ncols, sc.ldx, sc.ldxp, sc.xdtype, sc.opts,
                      is_shifted_view(sc.x, sc.xp, sc.ldx, sc.ldxp, sc.xdtype)};
            a.o.flags |= DMD_FIT_ASYNC;
            models[i].r = sc.opts.r;
            models[i].dtype = sc.xdtype;
            models[i].dt = sc.opts.dt;
            if (hipStreamWaitEvent(g->streams[i], g->events[nscenes], 0) != hipSuccess) return DMD_ERR_HIP;
            Carver cv(sc.ws);
            FitBufs fb{};
            if (int32_t st = fit_plan(cv, g->streams[i], a, &models[i], &fb)) return st;
            if (a.o.flags & DMD_FIT_OPTDMD)
                if (int32_t st = optdmd_refine(g->streams[i], a, &models[i], fb, false)) return st;
            if (hipEventRecord(g->events[i], g->streams[i]) != hipSuccess) return DMD_ERR_HIP;
            if (hipStreamWaitEvent(origin, g->events[i], 0) != hipSuccess) return DMD_ERR_HIP;
        }
        return DMD_OK;
    };
    int32_t status = DMD_OK;
    if (capture) {
        // one eager pass first: the runtime loads a kernel's code on its first launch, which
        // is not allowed while a stream is being captured
        status = enqueue_all();
        if (hipStreamSynchronize(origin) != hipSuccess && status == DMD_OK) status = DMD_ERR_HIP;
        if (status != DMD_OK) return cleanup(status);
        if (hipStreamBeginCapture(origin, hipStreamCaptureModeGlobal) != hipSuccess) return cleanup(DMD_ERR_HIP);
    }
    status = enqueue_all();
    if (capture) {
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(origin, &gr);
        g->graph = gr;
        if (status != DMD_OK) return cleanup(status);
        if (e != hipSuccess || !gr) return cleanup(DMD_ERR_HIP);
        if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) return cleanup(DMD_ERR_HIP);
        *graph = g;
        return DMD_OK;
    }
    if (status != DMD_OK) { hipStreamSynchronize(origin); return cleanup(status); }
    if (hipStreamSynchronize(origin) != hipSuccess) return cleanup(DMD_ERR_HIP);
    return cleanup(DMD_OK);
}

int32_t dmd_graph_launch(dmd_graph* graph, void* stream)
{
    if (!graph || !graph->exec) return DMD_ERR_ARG;
    HIPCHK(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return DMD_OK;
}

int32_t dmd_graph_destroy(dmd_graph* graph)
{
    if (!graph) return DMD_ERR_ARG;
    if (graph->exec) hipGraphExecDestroy(graph->exec);
    if (graph->graph) hipGraphDestroy(graph->graph);
    for (auto e : graph->events) hipEventDestroy(e);
    for (auto s : graph->streams) hipStreamDestroy(s);
    delete graph;
    return DMD_OK;
}

int32_t dmd_autotune_reconstruct(void* stream, const dmd_model* model, int32_t K, int32_t mode, void* U, int64_t ldu,
                                 void* ws, size_t ws_bytes, const char* cache_path, int32_t* best_cfg)
{
    if (int32_t e = validate_model(model)) return e;
    if (K < 1) return DMD_ERR_SHAPE;
    std::vector<int64_t> ks((size_t)K);
    for (int j = 0; j < K; ++j) ks[j] = j;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return DMD_ERR_HIP; }
    int best = 0;
    float best_ms = 1e30f;
    int32_t status = DMD_OK;
    status = recon_prepare(st, model, ks.data(), nullptr, K, mode, ws, ws_bytes);
    for (int cfg = 0; cfg < RECON_NCFG && status == DMD_OK; ++cfg) {
        status = recon_apply(st, model, K, mode, U, ldu, ws, ws_bytes, cfg);   // warm-up
        if (status) break;
        hipEventRecord(e0, st);
        for (int rep = 0; rep < 3 && status == DMD_OK; ++rep)
            status = recon_apply(st, model, K, mode, U, ldu, ws, ws_bytes, cfg);
        hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { status = DMD_ERR_HIP; break; }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) { best_ms = ms; best = cfg; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (status != DMD_OK) return status;
    const int rp = (int)dmd_phi_ld(model->r);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[tune_key(mode, rp, model->n, K)] = best;
    }
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            auto k = tune_key(mode, rp, model->n, K);
            fprintf(f, "%d %d %d %d %d %.3f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), best,
                    best_ms / 3.0f * 1000.0f);
            fclose(f);
        }
    }
    if (best_cfg) *best_cfg = best;
    return DMD_OK;
}

int32_t dmd_autotune_load(const char* cache_path)
{
    if (!cache_path) return DMD_ERR_ARG;
    return load_cache(cache_path);
}

}  // extern "C"
