// FP64 eigen-decomposition of the reduced operator Atilde W = W Lambda (Sec. 3.1).
//
// Real nonsymmetric n x n matrix (n <= DMD_MAX_RANK), five kernels:
//  1. hessenberg_kernel (1 work-group): Householder reduction A = Q H Q^T, H in
//     registers across the work-group, the reflectors (v_k, tau_k) kept for
//     rebuilding Q; H is written row-major with its trace and squared Frobenius norm.
//  2. aberth_kernel (one wave per eigenvalue, four per work-group sharing H in LDS):
//     the eigenvalues as the roots of det(zI - H), all refined at once by the
//     Ehrlich-Aberth iteration, each Newton ratio from Hyman's method (the determinant of
//     a Hessenberg matrix by back-substitution on its sub-diagonal) differentiated in z.
//  2b. eig_pair_kernel (1 work-group): real eigenvalues and conjugate pairs told apart
//     and made exact (real, or exactly conjugate).
//  2c. invit_kernel (one wave per real eigenvalue or pair, up to four per work-group
//     sharing H in LDS): the eigenvector by inverse iteration on H, taken through Q,
//     normalised to unit 2-norm (folded: [Re, Im] for a conjugate pair).
//  3. sort_modes_kernel (1 work-group): canonical order (ascending |arg lambda|,
//     ties by descending |lambda|, Im > 0 member of a pair first), lambda, kind
//     and the permuted folded eigenvectors (pair -> [Re w, Im w], LAPACK storage).
#include "common.h"
#include "kernels.h"

namespace dmd {

// workspace layout (doubles unless noted)
struct EigWs {
    double* H;        // n x n row-major Hessenberg matrix, then trace(H) and ||H||_F^2
    double* V;        // n x n reflector vectors (column k: rows k+1..n-1)
    double* tau;      // n
    double* Wraw;     // n x n unsorted folded eigenvectors
    double* wr;       // n
    double* wi;       // n
    double* zbuf;     // 2 x 2n: two iterates of the eigenvalue approximations (re, im)
    double* zfin;     // 2n: converged approximations
    int32_t* kind0;   // n
    int32_t* conv;    // 2 x n: converged flags of the two iterates
    uint32_t* counter;
};

size_t eig_workspace_bytes(int n)
{
    const size_t nn = (size_t)n * n;
    const size_t dbl = (nn + 2) + nn + n + nn + 2 * (size_t)n + 4 * (size_t)n + 2 * (size_t)n;
    return dbl * sizeof(double) + 3 * (size_t)round_up((int64_t)n * sizeof(int32_t), 64) + 64 + 256;
}

static EigWs eig_carve(void* ws, int n)
{
    EigWs w;
    double* p = (double*)ws;
    const size_t nn = (size_t)n * n;
    w.H = p; p += nn + 2;
    w.V = p; p += nn;
    w.tau = p; p += n;
    w.Wraw = p; p += nn;
    w.wr = p; p += n;
    w.wi = p; p += n;
    w.zbuf = p; p += 4 * (size_t)n;
    w.zfin = p; p += 2 * (size_t)n;
    char* q = (char*)p;
    w.kind0 = (int32_t*)q; q += round_up((int64_t)n * sizeof(int32_t), 64);
    w.conv = (int32_t*)q; q += 2 * round_up((int64_t)n * sizeof(int32_t), 64);
    w.counter = (uint32_t*)q;
    return w;
}

// ====================================================================== 1. Hessenberg
// Householder reduction A = Q H Q^T, H held in registers: thread (ib, jb) of a 32 x 32
// grid keeps H(ib + 32 a, jb + 32 c), a, c < HN (n <= 32 HN).  Step k, reflector P = I - tau v v^T of
// column k (rows k+1..):  with u = H v, w = H^T v and gamma = v^T H v taken from H before
// the step, P H P = H - tau (v w^T + u v^T) + tau^2 gamma v v^T on columns > k, and column
// k becomes (.., beta, 0, ..).  u, w and gamma are summed from per-thread partials in LDS
// (fixed order).  While the others update their entries, wave 0 forms the next column and
// the next reflector.  Three barriers per step.  SYMM (a symmetric A, whose reduction is
// tridiagonal): u = H v equals w = H^T v, so only w is summed and serves for both.
template <int HN, bool SYMM = false>
__global__ void __launch_bounds__(1024)
hessenberg_kernel(const double* __restrict__ A, int64_t lda, int n, double* H, double* V, double* tau)
{
    constexpr int HS_N = HN, NMAX = 32 * HN;
    __shared__ double col[NMAX];              // column k of H (rows > k), for v
    __shared__ double colpre[NMAX];           // column k + 1 before step k
    __shared__ double us[NMAX], ws[NMAX];
    // partial u per column group jb; rows of odd length so that the 32 lanes of a store
    // (32 column groups, one row) fall in different banks
    constexpr int UPS = NMAX + 1;
    __shared__ double upart[32 * UPS];
    __shared__ double wpart[32 * NMAX];       // partial w per row group ib
    __shared__ double gpart[1024];
    __shared__ double refl[4];                // tau, beta, 1 / (alpha - beta), gamma
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ib = 2 * wave + (lane >> 5), jb = lane & 31;

    double h[HS_N][HS_N];
#pragma unroll
    for (int a = 0; a < HS_N; ++a)
#pragma unroll
        for (int c = 0; c < HS_N; ++c) {
            const int i = ib + 32 * a, j = jb + 32 * c;
            h[a][c] = (i < n && j < n) ? A[(int64_t)j * lda + i] : 0.0;
        }
    for (int e = tid; e < n * n; e += 1024) V[e] = 0.0;
    for (int i = tid; i < n; i += 1024) tau[i] = 0.0;
    // reflector data of column k from the column in col[]: (tau, beta, scale); wave-wide
    auto reflector = [&](int k) {
        double x2 = 0.0;
        for (int i = k + 2 + lane; i < n; i += 64) { const double x = col[i]; x2 = fma(x, x, x2); }
        x2 = wave_sum_dpp(x2);
        const double alpha = col[k + 1];
        double tk = 0.0, beta = alpha, sc = 0.0;
        if (x2 != 0.0) {
            const double nrm = sqrt(alpha * alpha + x2);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tk = (beta - alpha) / beta;
            sc = 1.0 / (alpha - beta);
        }
        if (lane == 0) { refl[0] = tk; refl[1] = beta; refl[2] = sc; }
    };
    if (n > 2 && jb == 0)
#pragma unroll
        for (int a = 0; a < HS_N; ++a)
            if (ib + 32 * a < n) col[ib + 32 * a] = h[a][0];
    __syncthreads();
    if (n > 2 && wave == 0) reflector(0);
    __syncthreads();

    for (int k = 0; k + 2 < n; ++k) {
        const double tk = refl[0], beta = refl[1], sc = refl[2];
        // v_i without branches: every lane reads col[i] (i < NMAX) and selects
        auto vof = [&](int i) {
            const double cv = col[i] * sc;
            return i == k + 1 ? 1.0 : (i > k + 1 && i < n ? cv : 0.0);
        };
        double vr[HS_N], vc[HS_N];
#pragma unroll
        for (int a = 0; a < HS_N; ++a) { vr[a] = vof(ib + 32 * a); vc[a] = vof(jb + 32 * a); }
        if (wave == 1) {
            for (int i = k + 1 + lane; i < n; i += 64) V[(int64_t)k * n + i] = vof(i);
            if (lane == 0) tau[k] = tk;
        }
        // ---- partials of u = H v, w = H^T v, gamma = v^T H v; column k + 1 before the step.
        // Column blocks c < k / 32 lie left of column k: v is 0 there, so they add nothing
        // to u or gamma, and their entries of w are not used; they are skipped (a uniform
        // test per block).  Rows and columns past n hold zeros: partials stored unguarded.
        const int cb_k = k >> 5;
        double g = 0.0;
        if constexpr (!SYMM) {
            double tu[HS_N];
#pragma unroll
            for (int a = 0; a < HS_N; ++a) tu[a] = 0.0;
#pragma unroll
            for (int c = 0; c < HS_N; ++c) {
                if (c < cb_k) continue;
#pragma unroll
                for (int a = 0; a < HS_N; ++a) tu[a] = fma(h[a][c], vc[c], tu[a]);
            }
#pragma unroll
            for (int a = 0; a < HS_N; ++a) upart[jb * UPS + ib + 32 * a] = tu[a];
        }
#pragma unroll
        for (int c = 0; c < HS_N; ++c) {
            if (c < cb_k) continue;
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < HS_N; ++a) t = fma(vr[a], h[a][c], t);
            g = fma(t, vc[c], g);
            const int j = jb + 32 * c;
            wpart[ib * NMAX + j] = t;
            if (c == ((k + 1) >> 5) && jb == ((k + 1) & 31))       // j == k + 1
#pragma unroll
                for (int a = 0; a < HS_N; ++a) colpre[ib + 32 * a] = h[a][c];
        }
        gpart[tid] = g;
        __syncthreads();
        // ---- sums in a fixed order: four interleaved chains of eight, then pairwise (the
        // dependent-add chain is 10 long instead of 32)
        auto sum32 = [](const double* p, int stride) {
            double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int h = 0; h < 4; ++h) c[h] += p[(8 * h + q) * stride];
            return (c[0] + c[1]) + (c[2] + c[3]);
        };
        if (!SYMM && tid < n) {
            us[tid] = sum32(upart + tid, UPS);
        } else if (tid >= 256 && tid - 256 < n) {
            const int j = tid - 256;
            ws[j] = sum32(wpart + j, NMAX);
        } else if (wave == 15) {
            double t0 = 0.0, t1 = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) { t0 += gpart[q * 64 + lane]; t1 += gpart[(q + 8) * 64 + lane]; }
            const double t = wave_sum_dpp(t0 + t1);
            if (lane == 0) refl[3] = t;
        }
        __syncthreads();
        const double* uv = SYMM ? ws : us;      // u = H v
        const double tg = tk * tk * refl[3];
        // ---- wave 0 first: column k + 1 after the step, and the reflector of step k + 1 (a
        // latency chain that the other waves' updates hide; it reads no entry of h)
        if (wave == 0 && k + 3 < n) {
            const double wk = ws[k + 1], vk = k + 1 < n ? 1.0 : 0.0;    // v_{k+1} = 1
            for (int i = k + 2 + lane; i < n; i += 64) {
                const double vi = vof(i);
                col[i] = colpre[i] - (tk * fma(vi, wk, uv[i] * vk) - tg * vi * vk);
            }
            wave_sync_lds();
            reflector(k + 1);
        }
        // ---- H <- P H P on columns > k; column k -> (.., beta, 0, ..).  Per entry
        // tau (v_i w_j + u_i v_j) - tau^2 gamma v_i v_j = v_i A_j + v_j B_i with
        // A_j = tau w_j and B_i = tau u_i - tau^2 gamma v_i: two FMAs; columns <= k and
        // past n take A = v = 0 and rows past n take B = v = 0, which leaves them unchanged
        // Column blocks c < k / 32 are skipped (A = v = 0 there).  SYMM: the rows of those
        // blocks lie above row k, where u (= w, not summed for them) is 0 in exact arithmetic
        // (row i < k of the symmetric iterate is 0 right of column i + 1), so B = 0 there.
        double Aj[HS_N], vcm[HS_N], Bi[HS_N];
#pragma unroll
        for (int c = 0; c < HS_N; ++c) {
            const int j = jb + 32 * c;
            const bool upd = j > k && j < n;
            Aj[c] = upd ? tk * ws[j] : 0.0;
            vcm[c] = upd ? vc[c] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < HS_N; ++a) {
            const int i = ib + 32 * a;
            const bool row = i < n && (!SYMM || a >= cb_k);         // padding rows stay as they are
            Bi[a] = row ? fma(tk, uv[i], -tg * vr[a]) : 0.0;
        }
        const bool colk = jb == (k & 31);
#pragma unroll
        for (int c = 0; c < HS_N; ++c) {
            if (c < cb_k) continue;
#pragma unroll
            for (int a = 0; a < HS_N; ++a) h[a][c] = fma(-vr[a], Aj[c], fma(-vcm[c], Bi[a], h[a][c]));
            if (c == cb_k) {                    // the block holding column k: (.., beta, 0, ..)
#pragma unroll
                for (int a = 0; a < HS_N; ++a) {
                    const int i = ib + 32 * a;
                    if (colk && tk != 0.0 && i == k + 1) h[a][c] = beta;
                    if (colk && i > k + 1) h[a][c] = 0.0;
                }
            }
        }
        __syncthreads();
    }
    // H row-major, then its trace and squared Frobenius norm (fixed-order sums)
    double tr = 0.0, f2 = 0.0;
#pragma unroll
    for (int a = 0; a < HS_N; ++a)
#pragma unroll
        for (int c = 0; c < HS_N; ++c) {
            const int i = ib + 32 * a, j = jb + 32 * c;
            if (i < n && j < n) {
                H[(int64_t)i * n + j] = h[a][c];
                f2 = fma(h[a][c], h[a][c], f2);
                if (i == j) tr += h[a][c];
            }
        }
    gpart[tid] = f2;
    upart[tid] = tr;
    __syncthreads();
    if (wave == 0) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) { a += gpart[q * 64 + lane]; b += upart[q * 64 + lane]; }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) { H[(int64_t)n * n] = b; H[(int64_t)n * n + 1] = a; }
    }
}

// ====================================================================== 2. eigenvalues
// Ehrlich-Aberth iteration on p(z) = det(zI - H), all n approximations at once:
//   z_i <- z_i - 1 / (p'(z_i)/p(z_i) - sum_{j != i} 1 / (z_i - z_j)),
// with p'/p from Hyman's method (ab_logdet_deriv below).  Each wave refines one
// approximation, lanes over the rows; the four waves of a work-group share one copy of H
// in LDS (column-packed, scaled by the power of two that brings ||H||_F near 1).
// Iterations are separated by a grid-wide barrier (a counter in the workspace), so every
// approximation is updated from the same previous iterate and the result does not depend
// on scheduling.  The barrier's wait is bounded: a wave that waits past the bound reports
// DMD_ERR_EIG_NOCONV and leaves, which ends the other waves' waits too.
// Start: n points on the circle about trace(H)/n whose radius is the spread
// (||H||_F^2 / n - |trace(H)/n|^2)^(1/2) that bounds the eigenvalues' deviation from their
// mean (Schur's inequality).  A root is converged when its correction falls below tol
// relative to |z| (the next correction of a simple root is of the cube of that size), or
// below 1e-9 |z| without shrinking by a factor 4 any more (the rounding floor of the
// evaluation, reached by clustered roots).
constexpr int AB_SLOTS = 3;                 // columns (rows) per lane: n <= 192
static_assert(EIG_MAX <= 64 * AB_SLOTS, "aberth_kernel keeps at most 3 columns per lane");
constexpr int AB_MAX_IT = 200;
constexpr uint32_t AB_SPIN_CAP = 1u << 22;
constexpr int AB_WAVES = 4;                 // approximations (waves) per work-group

__device__ __forceinline__ double bcast(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Column-packed Hessenberg: column c holds rows 0 .. min(c + 1, n - 1).
__host__ __device__ __forceinline__ int hcol_off(int c) { return (c * (c + 3)) / 2; }
__host__ __device__ __forceinline__ int hcol_size(int n) { return n <= 1 ? n : hcol_off(n - 1) + n; }
// Packed reflectors: column k (k <= n - 3) holds v_k on rows k + 1 .. n - 1.
__host__ __device__ __forceinline__ int vcol_off(int k, int n) { return k * (n - 1) - (k * (k - 1)) / 2; }
__host__ __device__ __forceinline__ int vcol_size(int n) { return n < 3 ? 0 : vcol_off(n - 2, n); }

// ---- LDS staging of the small factors with eight global loads in flight per thread.
// Element e of an n x n source (thread tid takes e = tid, tid + nthr, ...) is read in a
// batch of eight independent loads, then stored: a loop that stored each value before
// loading the next waited a full memory latency per element.
constexpr int STAGE_B = 8;

// H (row-major, n x n) times sc, column-packed (column c holds rows 0 .. c + 1); with
// inv_sub, also 1 / h_{r,r-1} with the sub-diagonal raised to at least floor_sub
__device__ __forceinline__ void stage_hessenberg(const double* __restrict__ Hr, int n, double sc, double* Hs,
                                                 double* inv_sub, double floor_sub, int tid, int nthr)
{
    const int tot = n * n;
    for (int e0 = tid; e0 < tot; e0 += STAGE_B * nthr) {
        double v[STAGE_B];
        int rr[STAGE_B], cc[STAGE_B];
#pragma unroll
        for (int u = 0; u < STAGE_B; ++u) {
            const int e = e0 + u * nthr;
            rr[u] = e / n;
            cc[u] = e - rr[u] * n;
            v[u] = (e < tot && cc[u] + 1 >= rr[u]) ? Hr[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < STAGE_B; ++u) {
            const int e = e0 + u * nthr, r = rr[u], c = cc[u];
            if (e < tot && c + 1 >= r) {
                const double x = v[u] * sc;
                Hs[hcol_off(c) + r] = x;
                if (inv_sub && c == r - 1)
                    inv_sub[r] = 1.0 / (fabs(x) >= floor_sub ? x : (x < 0.0 ? -floor_sub : floor_sub));
            }
        }
    }
}

// the reflectors v_k (column k of V, n x n column-major, rows k + 1 .. n - 1, k <= n - 3)
// packed at vcol_off(k, n), and their tau
__device__ __forceinline__ void stage_reflectors(const double* __restrict__ Vg, const double* __restrict__ taug, int n,
                                                 double* Vs, double* taus, int tid, int nthr)
{
    if (n <= 2) return;
    const int tot = (n - 2) * n;
    for (int e0 = tid; e0 < tot; e0 += STAGE_B * nthr) {
        double v[STAGE_B];
        int kk[STAGE_B], ii[STAGE_B];
#pragma unroll
        for (int u = 0; u < STAGE_B; ++u) {
            const int e = e0 + u * nthr;
            kk[u] = e / n;
            ii[u] = e - kk[u] * n;
            v[u] = (e < tot && ii[u] > kk[u]) ? Vg[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < STAGE_B; ++u) {
            const int e = e0 + u * nthr, k = kk[u], i = ii[u];
            if (e < tot && i > k) Vs[vcol_off(k, n) + i - k - 1] = v[u];
        }
    }
    for (int k = tid; k + 2 < n; k += nthr) taus[k] = taug[k];
}

// Start point j of the iteration (the same formula on every wave).
__device__ __forceinline__ void ab_start(int j, int n, double cr, double rho, double* zr, double* zi)
{
    double s, c;
    sincospi(2.0 * (j + 0.4) / n, &s, &c);
    *zr = fma(rho, c, cr);
    *zi = rho * s;
}

// 1/a for complex a: conj(a) / |a|^2 with the hardware reciprocal refined by two Newton
// steps (a few ulp); a = 0 gives a non-finite result.
__device__ __forceinline__ void crcp(double ar, double ai, double* rr, double* ri)
{
    const double im2 = rcp_nr(fma(ar, ar, ai * ai));
    *rr = ar * im2;
    *ri = -ai * im2;
}

// p'/p(z) for p(z) = det(zI - H) by Hyman's method.  With x_{n-1} = 1, rows n-1 .. 1 of
// (zI - H) x = 0 give x_{j-1} = r_j / h_{j,j-1}, where r_j = sum_{c >= j} (z d_jc - h_jc) x_c
// is complete once x_j is known; row 0 is left with r_0, and det(zI - H) = r_0 times the
// product of the sub-diagonal entries, which do not depend on z, so p'/p = r'_0 / r_0
// (r' and x' carried along).  Column-oriented: each lane keeps r and r' of its rows and
// adds column j times x_j to them; the only divisions are the precomputed reciprocals of
// the sub-diagonal.  Sub-diagonal entries below eps ||H||_F have been raised to that size
// (a backward-stable perturbation), so one step multiplies |x| by at most about
// n (|z| + ||H||) / (eps ||H||) < 1e19; every eight steps, once |x| passes 1e100, x, x',
// r and r' are scaled by the power of two that brings |x| to [1, 2) (exact, and the ratio
// does not change), which keeps them below 1e260.
// Slot s of a lane holds row i = lane + 64 s.  In steps j with j >> 6 == JS the rows still
// accumulating (i <= j) lie in slots 0 .. JS; the rows of those slots take the update
// without a lane mask (column j is zero below row j + 1 in the packed layout, read as 0).
// The steps run without branches: eight per block, the next column and reciprocal loaded
// one step ahead by every lane (its own row, clamped into the column, then zeroed below
// the diagonal), and the rescaling applied by a factor that is 1 when not needed.
struct HyState {
    double rr[AB_SLOTS], ri[AB_SLOTS], pr[AB_SLOTS], pi[AB_SLOTS];   // r and r' of the rows
    double hc[AB_SLOTS];                                             // column j of H
    double is;                                                       // 1 / h_{j,j-1}
    double xr, xi, xpr, xpi;                                         // x_j and x'_j
};

// column c (rows 0 .. c of slots 0 .. JS; the rest 0) into hc
template <int JS>
__device__ __forceinline__ void hy_load_col(const double* Hs, int c, int lane, double (&hc)[AB_SLOTS])
{
    const double* col = Hs + hcol_off(c);
#pragma unroll
    for (int s = 0; s <= JS; ++s) {
        const int i = lane + 64 * s;
        const double v = col[min(i, c)];
        hc[s] = (s < JS || i <= c) ? v : 0.0;
    }
}

// step j (j >= 1): add column j to the rows, then x_{j-1} = r_j / h_{j,j-1}
template <int JS>
__device__ __forceinline__ void hy_step(const double* Hs, const double* inv_sub, int lane, double zr, double zi,
                                        int j, HyState& st)
{
    double hc[AB_SLOTS];
#pragma unroll
    for (int s = 0; s <= JS; ++s) hc[s] = st.hc[s];
    const double is = st.is;
    hy_load_col<JS>(Hs, j - 1, lane, st.hc);     // rows of slot JS lie below column j - 1 at a segment's end
    st.is = inv_sub[j - 1];                      // inv_sub[0] is 0 (not used)
    const double xr = st.xr, xi = st.xi, xpr = st.xpr, xpi = st.xpi;
    // z x and x + z x' for the diagonal row j
    const double zxr = fma(zr, xr, -zi * xi), zxi = fma(zr, xi, zi * xr);
    const double zpr = xr + fma(zr, xpr, -zi * xpi), zpi = xi + fma(zr, xpi, zi * xpr);
#pragma unroll
    for (int s = 0; s <= JS; ++s) {
        st.rr[s] = fma(-hc[s], xr, st.rr[s]);
        st.ri[s] = fma(-hc[s], xi, st.ri[s]);
        st.pr[s] = fma(-hc[s], xpr, st.pr[s]);
        st.pi[s] = fma(-hc[s], xpi, st.pi[s]);
    }
    // row j is complete: its diagonal term z x_j (and x_j + z x'_j) is added to the
    // broadcast value only; the lane's own copy of row j is not read again
    const int jl = j & 63;
    st.xr = (bcast(st.rr[JS], jl) + zxr) * is;
    st.xi = (bcast(st.ri[JS], jl) + zxi) * is;
    st.xpr = (bcast(st.pr[JS], jl) + zpr) * is;
    st.xpi = (bcast(st.pi[JS], jl) + zpi) * is;
}

template <int JS>
__device__ __forceinline__ void hy_rescale(HyState& st)
{
    const double big = fabs(st.xr) + fabs(st.xi);
    const double f = big > 1e100 ? ldexp(1.0, -ilogb(big)) : 1.0;     // exact: a power of two
    st.xr *= f; st.xi *= f; st.xpr *= f; st.xpi *= f;
#pragma unroll
    for (int s = 0; s <= JS; ++s) { st.rr[s] *= f; st.ri[s] *= f; st.pr[s] *= f; st.pi[s] *= f; }
}

// steps j = j_hi down to j_lo (all with j >> 6 == JS, j_lo >= 1)
template <int JS>
__device__ void hy_segment(const double* Hs, const double* inv_sub, int lane, double zr, double zi, int j_hi,
                           int j_lo, HyState& st)
{
    int j = j_hi;
    for (; j - 7 >= j_lo; j -= 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) hy_step<JS>(Hs, inv_sub, lane, zr, zi, j - u, st);
        hy_rescale<JS>(st);
    }
    for (; j >= j_lo; --j) hy_step<JS>(Hs, inv_sub, lane, zr, zi, j, st);
    hy_rescale<JS>(st);
}

// p'/p at z for the column-packed Hessenberg matrix Hs in LDS (inv_sub[j] = 1 / h_{j,j-1});
// false when the ratio is not finite (r_0 = 0: z is an eigenvalue to working precision).
__device__ bool ab_logdet_deriv(const double* Hs, const double* inv_sub, int n, int lane, double zr, double zi,
                                double* sr_out, double* si_out)
{
    HyState st;
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) { st.rr[s] = 0.0; st.ri[s] = 0.0; st.pr[s] = 0.0; st.pi[s] = 0.0; st.hc[s] = 0.0; }
    st.xr = 1.0; st.xi = 0.0; st.xpr = 0.0; st.xpi = 0.0;
    const int j0 = n - 1;
    if ((j0 >> 6) == 2) hy_load_col<2>(Hs, j0, lane, st.hc);
    else if ((j0 >> 6) == 1) hy_load_col<1>(Hs, j0, lane, st.hc);
    else hy_load_col<0>(Hs, j0, lane, st.hc);
    st.is = inv_sub[j0];
    if (j0 >= 128) hy_segment<2>(Hs, inv_sub, lane, zr, zi, j0, 128, st);
    if (j0 >= 64) hy_segment<1>(Hs, inv_sub, lane, zr, zi, min(j0, 127), 64, st);
    if (j0 >= 1) hy_segment<0>(Hs, inv_sub, lane, zr, zi, min(j0, 63), 1, st);
    // column 0 into row 0
    {
        const double hv = st.hc[0];
        const bool l0 = lane == 0;
        const double zxr = fma(zr, st.xr, -zi * st.xi), zxi = fma(zr, st.xi, zi * st.xr);
        const double zpr = st.xr + fma(zr, st.xpr, -zi * st.xpi), zpi = st.xi + fma(zr, st.xpi, zi * st.xpr);
        st.rr[0] = fma(-hv, st.xr, st.rr[0]) + (l0 ? zxr : 0.0);
        st.ri[0] = fma(-hv, st.xi, st.ri[0]) + (l0 ? zxi : 0.0);
        st.pr[0] = fma(-hv, st.xpr, st.pr[0]) + (l0 ? zpr : 0.0);
        st.pi[0] = fma(-hv, st.xpi, st.pi[0]) + (l0 ? zpi : 0.0);
    }
    const double r0r = bcast(st.rr[0], 0), r0i = bcast(st.ri[0], 0);
    const double p0r = bcast(st.pr[0], 0), p0i = bcast(st.pi[0], 0);
    double ir, ii;
    crcp(r0r, r0i, &ir, &ii);
    *sr_out = fma(p0r, ir, -p0i * ii);
    *si_out = fma(p0r, ii, p0i * ir);
    return isfinite(*sr_out) && isfinite(*si_out);
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, DMD_WAVE);
    return v;
}

__global__ void __launch_bounds__(64 * AB_WAVES)
aberth_kernel(int n, const double* __restrict__ Hr, double* zbuf, int32_t* conv, uint32_t* counter,
              double* zfin, int32_t* info, double tol, int max_it)
{
    extern __shared__ __align__(16) double ab_sm[];
    double* Hs = ab_sm;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i = blockIdx.x * AB_WAVES + wave;
    // H / 2^e into LDS, column-packed, with 2^e near ||H||_F (exact scaling: the eigenvalues
    // scale by the same power of two), then the reciprocals of its sub-diagonal; row r is
    // read whole (coalesced) and entry (r, c) stored at column c
    const double f2raw = Hr[(int64_t)n * n + 1];
    const double sc = f2raw > 0.0 ? ldexp(1.0, -ilogb(sqrt(f2raw))) : 1.0;
    double* inv_sub = Hs + hcol_size(n);
    const double floor_sub = 2.220446049250313e-16 * sqrt(f2raw) * sc;
    stage_hessenberg(Hr, n, sc, Hs, inv_sub, floor_sub, tid, 64 * AB_WAVES);
    if (tid == 0) inv_sub[0] = 0.0;
    __syncthreads();
    if (i >= n) return;                     // no approximation for this wave (no barrier below)
    const double tr = Hr[(int64_t)n * n] * sc, f2 = f2raw * sc * sc;
    const double cr = tr / n;
    const double hscale = sqrt(f2 / n);
    const double rho = sqrt(fmax(f2 / n - cr * cr, 1e-30 * (f2 / n) + 1e-300));
    double zr, zi;
    ab_start(i, n, cr, rho, &zr, &zi);
    bool done = false, timeout = false;
    double wp = __builtin_inf();
    int it = 0;
    for (;; ++it) {
        const double* zc = zbuf + (size_t)(it & 1) * 2 * n;     // iterate it (it >= 1)
        if (!done) {
            double sr = 0.0, si = 0.0;
            const bool ok = ab_logdet_deriv(Hs, inv_sub, n, lane, zr, zi, &sr, &si);
            // sum over j != i of 1 / (z_i - z_j), fixed-order
            double qr = 0.0, qi = 0.0;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) {
                const int j = lane + 64 * s;
                if (j >= n || j == i) continue;
                double zjr, zji;
                if (it == 0) {
                    ab_start(j, n, cr, rho, &zjr, &zji);
                } else {
                    zjr = __hip_atomic_load(zc + 2 * j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    zji = __hip_atomic_load(zc + 2 * j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                const double ddr = zr - zjr, ddi = zi - zji;
                if (ddr != 0.0 || ddi != 0.0) {
                    double tr_, ti_;
                    crcp(ddr, ddi, &tr_, &ti_);
                    qr += tr_;
                    qi += ti_;
                }
            }
            qr = wave_sum_dpp(qr);
            qi = wave_sum_dpp(qi);
            double wr = 0.0, wi = 0.0;
            if (ok) {
                const double er = sr - qr, ei = si - qi;
                const double m = fma(er, er, ei * ei);
                if (m > 0.0 && m < __builtin_inf()) { wr = er / m; wi = -ei / m; }
            }
            zr -= wr;
            zi -= wi;
            const double aw = hypot(wr, wi), az = hypot(zr, zi) + 1e-6 * hscale;
            if (!ok || aw <= tol * az || (aw <= 1e-9 * az && aw > 0.25 * wp)) done = true;
            wp = aw;
        }
        // publish iterate it + 1 and its converged flag (both double-buffered: a wave that
        // is already one iteration ahead writes the other copy), then wait for every wave
        // to have done the same.  Everything exchanged between waves (iterates, flags, the
        // counter) is written and read by device-scope atomic accesses, which are coherent
        // across the XCDs' L2 caches on their own; so the release needs only the completion
        // of the three stores before the count (vmcnt(0)), and the acquire nothing: the
        // fences of the memory model would write back and invalidate the whole L2 of the
        // XCD on every iteration for data that is not cached there
        double* zn = zbuf + (size_t)((it + 1) & 1) * 2 * n;
        int32_t* cn = conv + (size_t)((it + 1) & 1) * n;
        if (lane == 0) {
            __hip_atomic_store(zn + 2 * i, zr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(zn + 2 * i + 1, zi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(cn + i, done ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_s_waitcnt(0x0F70);    // vmcnt(0): the stores above have completed
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t target = (uint32_t)(it + 1) * (uint32_t)n;
            uint32_t polls = 0;
            while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++polls > AB_SPIN_CAP) { timeout = true; break; }
            }
        }
        timeout = __shfl(timeout ? 1 : 0, 0, 64) != 0;
        if (timeout) break;
        int nc = 0;
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) {
            const int j = lane + 64 * s;
            if (j < n) nc += __hip_atomic_load(cn + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        nc = wave_sum_i(nc);
        if (nc == n || it + 1 >= max_it) break;
    }
    if (lane == 0) {
        zfin[2 * i] = zr / sc;
        zfin[2 * i + 1] = zi / sc;
        if (timeout || (!done && wp > 1e-6 * (hypot(zr, zi) + 1e-6 * hscale))) set_status(info, DMD_ERR_EIG_NOCONV);
        if (i == 0 && info) info[2] = it + 1;
    }
}

// ====================================================================== 2b. pairs
// A real matrix has real eigenvalues and conjugate pairs; the independent approximations
// carry rounding-level imaginary parts and asymmetries.  An approximation is real when
// |Im z| <= tau (|z| + 1e-6 ||H||_F / sqrt(n)), tau = 1e-12, raised tenfold until as
// many approximations lie above the real axis as below it; each upper one is paired with
// the lower one nearest to its conjugate (mutually nearest, else in index order), and a
// pair becomes (z_i + conj(z_j)) / 2 and its conjugate.  Output positions follow the index
// of the real root or of the upper member (a pair takes two adjacent positions).
constexpr int EP_THREADS = 256;
static_assert(EIG_MAX <= EP_THREADS, "eig_pair_kernel: one thread per approximation");

__global__ void __launch_bounds__(EP_THREADS)
eig_pair_kernel(int n, const double* __restrict__ zfin, const double* __restrict__ Hr, double* wr, double* wi,
                int32_t* kind0, int32_t* info)
{
    __shared__ double zs[2 * EIG_MAX];
    __shared__ int cls[EIG_MAX];
    __shared__ int mate[EIG_MAX], back[EIG_MAX];
    __shared__ int cnt[2], ok;
    const int tid = threadIdx.x;
    for (int e = tid; e < 2 * n; e += EP_THREADS) zs[e] = zfin[e];
    const double hscale = sqrt(Hr[(int64_t)n * n + 1] / n);
    __syncthreads();
    double tau = 1e-12;
    for (int t = 0; t < 9; ++t) {
        if (tid < 2) cnt[tid] = 0;
        __syncthreads();
        if (tid < n) {
            const double re = zs[2 * tid], im = zs[2 * tid + 1];
            const int c = fabs(im) <= tau * (hypot(re, im) + 1e-6 * hscale) ? 0 : (im > 0.0 ? 1 : -1);
            cls[tid] = c;
            if (c != 0) atomicAdd(&cnt[c > 0 ? 0 : 1], 1);
        }
        __syncthreads();
        const bool even = cnt[0] == cnt[1];
        __syncthreads();
        if (even) break;
        tau *= 10.0;
    }
    if (cnt[0] != cnt[1]) {
        if (tid == 0) set_status(info, DMD_ERR_EIG_NOCONV);
        return;
    }
    // nearest partner of every upper root among the lower ones, and back
    if (tid < n) {
        mate[tid] = -1;
        back[tid] = -1;
        const int c = cls[tid];
        if (c != 0) {
            const double re = zs[2 * tid], im = -zs[2 * tid + 1];     // conjugate
            double best = __builtin_inf();
            int bj = -1;
            for (int j = 0; j < n; ++j) {
                if (cls[j] != -c) continue;
                const double dr = zs[2 * j] - re, di = zs[2 * j + 1] - im;
                const double d = fma(dr, dr, di * di);
                if (d < best) { best = d; bj = j; }
            }
            if (c > 0) mate[tid] = bj; else back[tid] = bj;
        }
    }
    if (tid == 0) ok = 1;
    __syncthreads();
    if (tid < n && cls[tid] > 0 && back[mate[tid]] != tid) ok = 0;
    __syncthreads();
    if (tid == 0) {
        if (!ok) {
            // greedy in index order over the upper roots
            for (int j = 0; j < n; ++j) back[j] = 0;
            for (int u = 0; u < n; ++u) {
                if (cls[u] <= 0) continue;
                const double re = zs[2 * u], im = -zs[2 * u + 1];
                double best = __builtin_inf();
                int bj = -1;
                for (int j = 0; j < n; ++j) {
                    if (cls[j] >= 0 || back[j]) continue;
                    const double dr = zs[2 * j] - re, di = zs[2 * j + 1] - im;
                    const double d = fma(dr, dr, di * di);
                    if (d < best) { best = d; bj = j; }
                }
                mate[u] = bj;
                back[bj] = 1;
            }
        }
        int p = 0;
        for (int u = 0; u < n; ++u) {
            if (cls[u] == 0) {
                wr[p] = zs[2 * u]; wi[p] = 0.0; kind0[p] = 0;
                ++p;
            } else if (cls[u] > 0) {
                const int j = mate[u];
                const double re = 0.5 * (zs[2 * u] + zs[2 * j]);
                const double im = 0.5 * (zs[2 * u + 1] - zs[2 * j + 1]);
                wr[p] = re; wi[p] = im; kind0[p] = 1;
                wr[p + 1] = re; wi[p + 1] = -im; kind0[p + 1] = 2;
                p += 2;
            }
        }
    }
}

// ====================================================================== 2c. eigenvectors
// Inverse iteration on the Hessenberg matrix: x = (H - lambda I)^-1 (1, .., 1)^T, one wave
// per real eigenvalue or pair.  The factorisation eliminates the sub-diagonal from the
// bottom with column operations and partial pivoting: (H - lambda I) E_{n-1} .. E_1 = R,
// where E_j combines (and may swap) columns j - 1 and j.  Column j of R is final at step
// j, and R y = 1 is solved along with it (y_j from the running sums of the finished
// columns), so neither R nor the factors are stored; x = E_{n-1} .. E_1 y then follows
// from the kept multipliers and swaps.  H and lambda are scaled by the power of two that
// brings ||H||_F near 1; pivots below eps ||H||_F are raised to that value, and y is
// rescaled when it grows past 1e100.  x, normalised to unit 2-norm, is taken
// through the Hessenberg reflectors (A = Q H Q^T) to the eigenvector Q x of A; a pair
// stores [Re, Im] in its two columns.  The waves of a work-group share H (column-packed)
// in LDS, then the reflectors in the same space.
constexpr int IV_MAXW = 4;
static int invit_big(int n) { return std::max(hcol_size(n), vcol_size(n) + n); }
static size_t invit_lds_bytes(int n, int waves)
{
    return ((size_t)invit_big(n) + (size_t)waves * 5 * n) * sizeof(double) + (size_t)waves * round_up(n, 2) * sizeof(int);
}
static int invit_waves(int n)
{
    for (int w = IV_MAXW; w > 1; w >>= 1)
        if (invit_lds_bytes(n, w) <= 160 * 1024 - 256) return w;
    return 1;
}

// Slot s of a lane holds row i = lane + 64 s.  In steps j with j >> 6 == JS, rows i < j
// (the ones still updated) lie in slots 0 .. JS, all of them in slots below JS.  The rows
// of those slots take the update without a lane mask: rows i >= j are never read again.
struct IvState {
    double acr[AB_SLOTS], aci[AB_SLOTS];   // active column
    double rhr[AB_SLOTS], rhi[AB_SLOTS];   // rho_i = sum over finished columns c of R(i, c) y_c
    double ncr[AB_SLOTS];                  // column j - 1 of H, rows < j (the next step's)
    double hsub;                           // H(j, j - 1)
    double rs;                             // right-hand side scale
};

// column jn - 1 of H (rows 0 .. jn) for step jn: rows i < jn of slots 0 .. JS (the rest 0),
// read without branches (every lane reads a row of the column, clamped, and selects), and
// the sub-diagonal H(jn, jn - 1)
template <int JS>
__device__ __forceinline__ void iv_load_col(const double* Hs, int jn, int lane, double (&ncr)[AB_SLOTS], double& hsub)
{
    const double* nc = Hs + hcol_off(jn - 1);                      // column jn - 1: rows 0 .. jn
#pragma unroll
    for (int s = 0; s <= JS; ++s) {
        const int i = lane + 64 * s;
        const double v = nc[min(i, jn)];
        ncr[s] = i < jn ? v : 0.0;
    }
    hsub = nc[jn];
}

// step j of the column elimination (see invit_kernel)
template <int JS>
__device__ __forceinline__ void iv_step(const double* Hs, int lane, double lr, double li, double eps3, int j,
                                        IvState& st, double* yv, double* mu, double* fs, int* swp)
{
    double ncr[AB_SLOTS];
    const double hs = st.hsub;
#pragma unroll
    for (int s = 0; s <= JS; ++s) ncr[s] = st.ncr[s];
    iv_load_col<JS>(Hs, max(j - 1, 1), lane, st.ncr, st.hsub);    // the next step's (unused after j = 1)
    const int jl = j & 63;
    const double ajr = bcast(st.acr[JS], jl), aji = bcast(st.aci[JS], jl);
    const double qjr = bcast(st.rhr[JS], jl), qji = bcast(st.rhi[JS], jl);
    double nci[AB_SLOTS];
#pragma unroll
    for (int s = 0; s <= JS; ++s) {
        const int i = lane + 64 * s;
        const bool dg = i == j - 1;
        ncr[s] = dg ? ncr[s] - lr : ncr[s];
        nci[s] = dg ? -li : 0.0;
    }
    // pivot: H(j, j - 1) of the new column when it is larger, else the active column's
    // entry (a select, not a branch); raised to eps3 when below it
    const bool swap = fabs(hs) > fabs(ajr) + fabs(aji);
    double pvr = swap ? hs : ajr, pvi = swap ? 0.0 : aji;
    const bool tiny = fabs(pvr) + fabs(pvi) < eps3;
    pvr = tiny ? (pvr < 0.0 ? -eps3 : eps3) : pvr;
    pvi = tiny ? 0.0 : pvi;
    const double orr = swap ? ajr : hs, oi = swap ? aji : 0.0;
    double ipr, ipi;
    crcp(pvr, pvi, &ipr, &ipi);
    const double mur = fma(orr, ipr, -oi * ipi), mui = fma(orr, ipi, oi * ipr);
    // y_j = (rs - rho_j) / pivot
    const double tr = st.rs - qjr, ti = -qji;
    double yr = fma(tr, ipr, -ti * ipi), yi = fma(tr, ipi, ti * ipr);
    // growth guard without a branch: past 1e100 this step's y, the right-hand side and
    // the running sums take a factor 1e-100, kept in fs[j]; the y stored before are
    // brought to the same scale when x is formed
    const double f = fabs(yr) + fabs(yi) > 1e100 ? 1e-100 : 1.0;
    yr *= f; yi *= f; st.rs *= f;
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) { st.rhr[s] *= f; st.rhi[s] *= f; }
#pragma unroll
    for (int s = 0; s <= JS; ++s) {
        const double rcr = swap ? ncr[s] : st.acr[s], rci = swap ? nci[s] : st.aci[s];   // R(i, j)
        const double ocr = swap ? st.acr[s] : ncr[s], oci = swap ? st.aci[s] : nci[s];
        st.rhr[s] += fma(rcr, yr, -rci * yi);
        st.rhi[s] += fma(rcr, yi, rci * yr);
        st.acr[s] = ocr - fma(mur, rcr, -mui * rci);
        st.aci[s] = oci - fma(mur, rci, mui * rcr);
    }
    if (lane == 0) {
        yv[2 * j] = yr; yv[2 * j + 1] = yi;
        mu[2 * j] = mur; mu[2 * j + 1] = mui;
        fs[j] = f;
        swp[j] = swap ? 1 : 0;
    }
}

// steps j = j_hi down to j_lo (all with j >> 6 == JS, j_lo >= 1), in blocks of eight
template <int JS>
__device__ void iv_segment(const double* Hs, int lane, double lr, double li, double eps3, int j_hi, int j_lo,
                           IvState& st, double* yv, double* mu, double* fs, int* swp)
{
    int j = j_hi;
    for (; j - 7 >= j_lo; j -= 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) iv_step<JS>(Hs, lane, lr, li, eps3, j - u, st, yv, mu, fs, swp);
    }
    for (; j >= j_lo; --j) iv_step<JS>(Hs, lane, lr, li, eps3, j, st, yv, mu, fs, swp);
}

__global__ void __launch_bounds__(64 * IV_MAXW)
invit_kernel(int n, int waves, const double* __restrict__ Hr, const double* __restrict__ Vg,
             const double* __restrict__ taug, const double* __restrict__ wr, const double* __restrict__ wi,
             const int32_t* __restrict__ kind0, double* Wraw)
{
    extern __shared__ __align__(16) double iv_sm[];
    const int big = max(hcol_size(n), vcol_size(n) + n);
    double* Hs = iv_sm;                                   // column-packed H, later the reflectors
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double* yv = iv_sm + big + (size_t)wave * 5 * n;      // y, then x (re, im interleaved)
    double* mu = yv + 2 * n;                              // multipliers (re, im)
    double* fs = mu + 2 * n;                              // growth-guard factors
    int* swp = reinterpret_cast<int*>(iv_sm + big + (size_t)waves * 5 * n) + wave * round_up(n, 2);
    const int p = blockIdx.x * waves + wave;
    const int nthr = 64 * waves;
    // H / 2^e column-packed (2^e near ||H||_F, as in the eigenvalue iteration): row r read
    // whole (coalesced), entry (r, c) stored at column c
    const double f2raw = Hr[(int64_t)n * n + 1];
    const double sc = f2raw > 0.0 ? ldexp(1.0, -ilogb(sqrt(f2raw))) : 1.0;
    stage_hessenberg(Hr, n, sc, Hs, nullptr, 0.0, tid, nthr);
    __syncthreads();
    const bool valid = p < n && kind0[p] != 2;
    const bool pair = valid && kind0[p] == 1;
    double xr[AB_SLOTS], xi[AB_SLOTS];
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) { xr[s] = 0.0; xi[s] = 0.0; }
    if (valid) {
        const double lr = wr[p] * sc, li = pair ? wi[p] * sc : 0.0;
        const double eps3 = 2.220446049250313e-16 * sqrt(f2raw) * sc + 1e-300;
        IvState st;
        const double* cl = Hs + hcol_off(n - 1);
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) {
            const int i = lane + 64 * s;
            st.acr[s] = i < n ? cl[i] : 0.0;
            st.aci[s] = 0.0;
            if (i == n - 1) { st.acr[s] -= lr; st.aci[s] = -li; }
            st.rhr[s] = 0.0;
            st.rhi[s] = 0.0;
            st.ncr[s] = 0.0;
        }
        st.rs = 1.0;
        st.hsub = 0.0;
        if (n > 1) {
            const int j0 = n - 1;                              // first step's column j0 - 1
            if ((j0 >> 6) == 2) iv_load_col<2>(Hs, j0, lane, st.ncr, st.hsub);
            else if ((j0 >> 6) == 1) iv_load_col<1>(Hs, j0, lane, st.ncr, st.hsub);
            else iv_load_col<0>(Hs, j0, lane, st.ncr, st.hsub);
        }
        // steps j = n - 1 .. 1 by segments of 64
        if (n - 1 >= 128) iv_segment<2>(Hs, lane, lr, li, eps3, n - 1, 128, st, yv, mu, fs, swp);
        if (n - 1 >= 64) iv_segment<1>(Hs, lane, lr, li, eps3, min(n - 1, 127), 64, st, yv, mu, fs, swp);
        if (n - 1 >= 1) iv_segment<0>(Hs, lane, lr, li, eps3, min(n - 1, 63), 1, st, yv, mu, fs, swp);
        {
            double pvr = bcast(st.acr[0], 0), pvi = bcast(st.aci[0], 0);
            if (fabs(pvr) + fabs(pvi) < eps3) { pvr = eps3; pvi = 0.0; }
            const double qr = bcast(st.rhr[0], 0), qi = bcast(st.rhi[0], 0);
            const double tr = st.rs - qr, ti = -qi;
            double ipr, ipi;
            crcp(pvr, pvi, &ipr, &ipi);
            if (lane == 0) { yv[0] = fma(tr, ipr, -ti * ipi); yv[1] = fma(tr, ipi, ti * ipr); }
        }
        wave_sync_lds();
        // x = E_{n-1} .. E_1 y: E_j takes v_j -= mu_j v_{j-1}, then swaps v_{j-1}, v_j if
        // the step pivoted; component j - 1 is final after E_j.  y_j is brought to the scale
        // of y_0 by the factors of the steps after it (steps run from j = n - 1 down).
        if (lane == 0) {
            double cr = yv[0], ci = yv[1];
            double g = 1.0;
            for (int j = 1; j < n; ++j) {                     // branch-free: selects
                g *= j >= 2 ? fs[j - 1] : 1.0;                // factors of steps 1 .. j - 1
                const double yr_ = yv[2 * j] * g, yi_ = yv[2 * j + 1] * g;
                const double vr = yr_ - fma(mu[2 * j], cr, -mu[2 * j + 1] * ci);
                const double vi = yi_ - fma(mu[2 * j], ci, mu[2 * j + 1] * cr);
                const bool sj = swp[j] != 0;
                yv[2 * (j - 1)] = sj ? vr : cr;
                yv[2 * (j - 1) + 1] = sj ? vi : ci;
                cr = sj ? cr : vr;
                ci = sj ? ci : vi;
            }
            yv[2 * (n - 1)] = cr; yv[2 * (n - 1) + 1] = ci;
        }
        wave_sync_lds();
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) {
            const int i = lane + 64 * s;
            xr[s] = i < n ? yv[2 * i] : 0.0;
            xi[s] = i < n ? yv[2 * i + 1] : 0.0;
        }
        double nn2 = 0.0;
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) nn2 = fma(xr[s], xr[s], fma(xi[s], xi[s], nn2));
        nn2 = wave_sum_dpp(nn2);
        const double inv = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 0.0;
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) { xr[s] *= inv; xi[s] *= inv; }
    }
    // reflectors into the space H held: column k (rows k + 1 ..) packed, then tau
    __syncthreads();
    stage_reflectors(Vg, taug, n, Hs, Hs + vcol_size(n), tid, nthr);
    __syncthreads();
    if (!valid) return;
    // y = Q x with Q = P_0 P_1 .. P_{n-3}: P_k = I - tau_k v_k v_k^T (v_k rows k+1.., v_{k+1} = 1)
    if (n > 2) {
        const double* taus = Hs + vcol_size(n);
        for (int k = n - 3; k >= 0; --k) {
            const double* v = Hs + vcol_off(k, n) - (k + 1);      // entry i at v[i]
            double vv[AB_SLOTS];
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) {
                const int i = lane + 64 * s;
                const double vi = v[min(max(i, k + 1), n - 1)];   // in the column; selected below
                vv[s] = (i > k && i < n) ? vi : 0.0;
            }
            double gr = 0.0, gi = 0.0;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) { gr = fma(vv[s], xr[s], gr); gi = fma(vv[s], xi[s], gi); }
            const double t = taus[k];
            gr = wave_sum_dpp(gr) * t;
            gi = wave_sum_dpp(gi) * t;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) { xr[s] = fma(-gr, vv[s], xr[s]); xi[s] = fma(-gi, vv[s], xi[s]); }
        }
    }
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) {
        const int row = lane + 64 * s;
        if (row >= n) continue;
        Wraw[(int64_t)p * n + row] = xr[s];
        if (pair) Wraw[(int64_t)(p + 1) * n + row] = xi[s];
    }
}

// ====================================================================== 3. canonical order
constexpr int SM_THREADS = 1024;
__global__ void __launch_bounds__(SM_THREADS)
sort_modes_kernel(int n, const double* __restrict__ wr, const double* __restrict__ wi,
                  const int32_t* __restrict__ kind0, const double* __restrict__ Wraw, double* lam,
                  int32_t* kind, double* W)
{
    // LDS: the sort keys |arg|, modulus (n doubles each), then the kinds and the output
    // position of each unit head (n ints each)
    extern __shared__ double skey[];
    double* ang = skey;
    double* mag = skey + n;
    int* k0 = reinterpret_cast<int*>(skey + 2 * n);
    int* pos = k0 + n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = SM_THREADS >> 6;
    for (int u = tid; u < n; u += SM_THREADS) {
        k0[u] = kind0[u];
        ang[u] = fabs(atan2(wi[u], wr[u]));
        mag[u] = hypot(wr[u], wi[u]);
    }
    __syncthreads();
    // position of unit u: four lanes per unit, each counting the units v = q mod 4 placed
    // before it, then a sum over the four lanes
    for (int t = tid; t < 4 * round_up(n, 16); t += SM_THREADS) {
        const int u = t >> 2, q = t & 3;
        int p = 0;
        const bool head = u < n && k0[u] != 2;
        if (head) {
            const double au = ang[u], mu = mag[u];
            for (int v = q; v < n; v += 4) {
                if (k0[v] == 2 || v == u) continue;
                const double av = ang[v], mv = mag[v];
                const bool before = (av < au) || (av == au && mv > mu) || (av == au && mv == mu && v < u);
                if (before) p += (k0[v] == 1) ? 2 : 1;
            }
        }
        p += __shfl_xor(p, 1, 64);
        p += __shfl_xor(p, 2, 64);
        if (q == 0 && u < n) pos[u] = head ? p : -1;
    }
    __syncthreads();
    for (int u = tid; u < n; u += SM_THREADS) {
        const int p = pos[u];
        if (p < 0) continue;
        if (k0[u] == 0) {
            lam[2 * p] = wr[u]; lam[2 * p + 1] = 0.0; kind[p] = 0;
        } else {
            lam[2 * p] = wr[u]; lam[2 * p + 1] = fabs(wi[u]);
            lam[2 * p + 2] = wr[u]; lam[2 * p + 3] = -fabs(wi[u]);
            kind[p] = 1; kind[p + 1] = 2;
        }
    }
    // permuted eigenvector columns: one source column (and its partner) per wave at a time,
    // every row of it loaded before the stores
    static_assert(EIG_MAX <= 3 * 64, "sort_modes_kernel keeps 3 rows per lane");
    for (int u = wave; u < n; u += nw) {
        const int p = pos[u];
        if (p < 0) continue;
        const bool pair = k0[u] == 1;
        double a[3], b[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int row = lane + 64 * s;
            a[s] = row < n ? Wraw[(int64_t)u * n + row] : 0.0;
            b[s] = (pair && row < n) ? Wraw[(int64_t)(u + 1) * n + row] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int row = lane + 64 * s;
            if (row < n) {
                W[(int64_t)p * n + row] = a[s];
                if (pair) W[(int64_t)(p + 1) * n + row] = b[s];
            }
        }
    }
}

// ====================================================================== 4. symmetric
// Eigen-decomposition of a symmetric n x n matrix S (n <= DMD_MAX_SMALL): every eigenvalue
// (descending) and the eigenvectors of the nv largest, in three launches:
//  1. hessenberg_kernel: the Householder reduction of a symmetric matrix is tridiagonal,
//     S = Q T Q^T; its diagonal d and sub-diagonal e are read from H (the entries above
//     the super-diagonal are rounding-level and dropped).
//  2. tri_bisect_kernel (one wave per eigenvalue): bisection on Sturm counts, the number
//     of negative pivots of the LDL^T factorisation of T - xI, with the 64 lanes counting
//     at 64 points of the current interval, so one round narrows it 65-fold; from the
//     Gershgorin interval down to 4 eps max|x| (the absolute accuracy eps ||T|| that any
//     backward-stable method reaches).
//  3. tri_invit_kernel (one wave per wanted eigenvector): inverse iteration on T, two
//     solves of (T - lambda I) x = b by Gaussian elimination with partial pivoting (three
//     bands of U kept in LDS), from a start vector that differs between eigenvalues, so
//     equal or close eigenvalues still get independent vectors; then Q x through the
//     reflectors.  The vectors are unit-norm but, inside clusters of close eigenvalues,
//     only as orthogonal as inverse iteration makes them: callers that need an exact
//     basis form it from their span.
// T is scaled by the power of two that brings ||S||_F near 1 (exact), so pivots and Sturm
// recurrences stay in range.
constexpr int TB_WAVES = 4;
constexpr int TB_MAX_ROUNDS = 40;
constexpr double TB_PIVMIN = 1e-290;

__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x)
{
    double q = d[0] - x;
    q = fabs(q) < TB_PIVMIN ? -TB_PIVMIN : q;
    int c = q < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] * rcp_nr(q);
        q = fabs(q) < TB_PIVMIN ? -TB_PIVMIN : q;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

__device__ __forceinline__ double tb_scale(const double* Hr, int n)
{
    const double f2 = Hr[(int64_t)n * n + 1];
    return f2 > 0.0 ? ldexp(1.0, -ilogb(sqrt(f2))) : 1.0;
}

__global__ void __launch_bounds__(64 * TB_WAVES)
tri_bisect_kernel(int n, const double* __restrict__ Hr, double* evals, int32_t* info)
{
    extern __shared__ __align__(16) double tb_sm[];
    double* d = tb_sm;               // diagonal
    double* e2 = tb_sm + n;          // squared sub-diagonal
    double* ea = tb_sm + 2 * n;      // |sub-diagonal|
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double sc = tb_scale(Hr, n);
    for (int i = tid; i < n; i += 64 * TB_WAVES) {
        d[i] = Hr[(int64_t)i * n + i] * sc;
        const double b = i + 1 < n ? Hr[(int64_t)(i + 1) * n + i] * sc : 0.0;
        e2[i] = b * b;
        ea[i] = fabs(b);
    }
    __syncthreads();
    const int k = blockIdx.x * TB_WAVES + wave;          // k-th largest
    if (k >= n) return;
    // Gershgorin interval, widened by the rounding of its sums
    double glo = __builtin_inf(), ghi = -__builtin_inf();
    for (int i = lane; i < n; i += 64) {
        const double rad = (i > 0 ? ea[i - 1] : 0.0) + ea[i];
        glo = fmin(glo, d[i] - rad);
        ghi = fmax(ghi, d[i] + rad);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        glo = fmin(glo, __shfl_xor(glo, o, 64));
        ghi = fmax(ghi, __shfl_xor(ghi, o, 64));
    }
    const double tnorm = fmax(fabs(glo), fabs(ghi));
    double lo = glo - 4.0 * 2.220446049250313e-16 * n * tnorm - 2.0 * TB_PIVMIN;
    double hi = ghi + 4.0 * 2.220446049250313e-16 * n * tnorm + 2.0 * TB_PIVMIN;
    const int j = n - 1 - k;                             // j-th smallest: count(lo) <= j < count(hi)
    const double atol = 4.0 * 2.220446049250313e-16 * tnorm + TB_PIVMIN;
    int round = 0;
    for (; round < TB_MAX_ROUNDS; ++round) {
        const double w = hi - lo;
        if (w <= fmax(4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)), atol)) break;
        const double x = fma(w, (lane + 1) * (1.0 / 65.0), lo);
        const int c = sturm_count(d, e2, n, x);
        const uint64_t m = __ballot(c <= j);
        const int t = m ? 63 - __clzll((long long)m) : -1;   // last point with count <= j
        const double nlo = t >= 0 ? bcast(x, t) : lo;
        const double nhi = t < 63 ? bcast(x, t + 1) : hi;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) {
        evals[k] = 0.5 * (lo + hi) / sc;
        if (info) atomicMax(&info[1], round);
    }
}

// per-wave LDS of tri_invit_kernel: the bands of U (u0 the reciprocals of its diagonal, u1, u2), the multipliers,
// the row swaps and the right-hand side / solution
constexpr int TI_ARR = 6;
__host__ __device__ __forceinline__ int tinv_big(int n) { return vcol_size(n) + n; }
static size_t tinv_lds_bytes(int n, int waves)
{
    return ((size_t)2 * n + tinv_big(n) + (size_t)waves * TI_ARR * n) * sizeof(double);
}
static int tinv_waves(int n)
{
    for (int w = IV_MAXW; w > 1; w >>= 1)
        if (tinv_lds_bytes(n, w) <= 160 * 1024 - 256) return w;
    return 1;
}

// start vector entry i of eigenvector k: a fixed pseudo-random value in (-1, 1)
__device__ __forceinline__ double ti_start(int k, int i)
{
    uint64_t z = (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull + (uint64_t)(i + 1) * 0xD1B54A32D192ED03ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void __launch_bounds__(64 * IV_MAXW)
tri_invit_kernel(int n, int nv, int waves, const double* __restrict__ Hr, const double* __restrict__ Vg,
                 const double* __restrict__ taug, const double* __restrict__ evals, double* Vout, int64_t ldv)
{
    extern __shared__ __align__(16) double ti_sm[];
    double* d = ti_sm;                                   // diagonal (scaled)
    double* e = ti_sm + n;                               // sub-diagonal (scaled, signed)
    double* Vs = ti_sm + 2 * n;                          // packed reflectors, then tau
    double* taus = Vs + vcol_size(n);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nthr = 64 * waves;
    double* u0 = ti_sm + 2 * n + tinv_big(n) + (size_t)wave * TI_ARR * n;
    double* u1 = u0 + n;
    double* u2 = u1 + n;
    double* mu = u2 + n;
    double* sw = mu + n;                                 // 1.0 where rows i, i + 1 swapped
    double* y = sw + n;
    const double sc = tb_scale(Hr, n);
    for (int i = tid; i < n; i += nthr) {
        d[i] = Hr[(int64_t)i * n + i] * sc;
        e[i] = i + 1 < n ? Hr[(int64_t)(i + 1) * n + i] * sc : 0.0;
    }
    stage_reflectors(Vg, taug, n, Vs, taus, tid, nthr);
    __syncthreads();
    const int kv = blockIdx.x * waves + wave;
    if (kv >= nv) return;
    const double lam = evals[kv] * sc;
    const double eps3 = 2.220446049250313e-16 * sqrt(Hr[(int64_t)n * n + 1]) * sc + 1e-300;
    if (lane == 0) {
        // factorisation of T - lam I with partial pivoting; rows enter as (cu, cv) = the
        // entries of the current row at columns i, i + 1
        double cu = d[0] - lam, cv = n > 1 ? e[0] : 0.0;
        for (int i = 0; i + 1 < n; ++i) {
            const double bsub = e[i];                                    // T(i + 1, i)
            const double an = d[i + 1] - lam, gn = i + 2 < n ? e[i + 1] : 0.0;   // row i + 1 at i + 1, i + 2
            const bool s = fabs(bsub) > fabs(cu);
            double p = s ? bsub : cu;
            p = fabs(p) < eps3 ? (p < 0.0 ? -eps3 : eps3) : p;
            const double ip = rcp_nr(p);
            const double m = (s ? cu : bsub) * ip;
            u0[i] = ip;                                                  // 1 / pivot
            u1[i] = s ? an : cv;
            u2[i] = s ? gn : 0.0;
            mu[i] = m;
            sw[i] = s ? 1.0 : 0.0;
            const double ncu = s ? cv - m * an : an - m * cv;
            const double ncv = s ? -m * gn : gn;
            cu = ncu;
            cv = ncv;
        }
        u0[n - 1] = rcp_nr(fabs(cu) < eps3 ? (cu < 0.0 ? -eps3 : eps3) : cu);
#pragma unroll 8
        for (int i = 0; i < n; ++i) y[i] = ti_start(kv, i);
        for (int pass = 0; pass < 2; ++pass) {
            // forward: the row swaps and multipliers on the right-hand side; the running
            // entry is carried in a register (no LDS round trip on the chain), swaps by select
            double cur = y[0];
            for (int i = 0; i + 1 < n; ++i) {
                const double b = y[i + 1];
                const bool s = sw[i] != 0.0;
                const double a2 = s ? b : cur, b2 = s ? cur : b;
                y[i] = a2;
                cur = b2 - mu[i] * a2;
            }
            y[n - 1] = cur;
            // back-substitution with the three bands of U, then unit 2-norm
            double x1 = 0.0, x2 = 0.0, nrm = 0.0;
            for (int i = n - 1; i >= 0; --i) {
                const double xi = (y[i] - u1[i] * x1 - u2[i] * x2) * u0[i];
                y[i] = xi;
                x2 = x1;
                x1 = xi;
                nrm = fma(xi, xi, nrm);
            }
            const double inv = nrm > 0.0 ? rsqrt_nr(nrm) : 0.0;
#pragma unroll 8
            for (int i = 0; i < n; ++i) y[i] *= inv;
        }
    }
    wave_sync_lds();
    double xr[AB_SLOTS];
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) {
        const int i = lane + 64 * s;
        xr[s] = i < n ? y[i] : 0.0;
    }
    // y = Q x with Q = P_0 P_1 .. P_{n-3}
    if (n > 2) {
        for (int k = n - 3; k >= 0; --k) {
            const double* v = Vs + vcol_off(k, n) - (k + 1);
            double vv[AB_SLOTS];
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) {
                const int i = lane + 64 * s;
                const double vi = v[min(max(i, k + 1), n - 1)];   // in the column; selected below
                vv[s] = (i > k && i < n) ? vi : 0.0;
            }
            double g = 0.0;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) g = fma(vv[s], xr[s], g);
            g = wave_sum_dpp(g) * taus[k];
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) xr[s] = fma(-g, vv[s], xr[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) {
        const int row = lane + 64 * s;
        if (row < n) Vout[(int64_t)kv * ldv + row] = xr[s];
    }
}

size_t sym_eig_workspace_bytes(int n) { return ((size_t)2 * n * n + n + 2) * sizeof(double) + 256; }

hipError_t sym_eig(hipStream_t s, const double* S, int64_t lds, int n, int nv, double* evals, double* Vout,
                   int64_t ldv, void* ws, int32_t* info)
{
    if (n <= 0) return hipSuccess;
    if (n > 192 || nv > n) return hipErrorInvalidValue;
    double* H = (double*)ws;
    double* V = H + (size_t)n * n + 2;
    double* tau = V + (size_t)n * n;
    if (n <= 160) hipLaunchKernelGGL((hessenberg_kernel<5, true>), dim3(1), dim3(1024), 0, s, S, lds, n, H, V, tau);
    else hipLaunchKernelGGL((hessenberg_kernel<6, true>), dim3(1), dim3(1024), 0, s, S, lds, n, H, V, tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tri_bisect_kernel, dim3((unsigned)ceil_div(n, TB_WAVES)), dim3(64 * TB_WAVES),
                       (size_t)3 * n * sizeof(double), s, n, H, evals, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nv <= 0) return hipSuccess;
    const int w = tinv_waves(n);
    hipLaunchKernelGGL(tri_invit_kernel, dim3((unsigned)ceil_div(nv, w)), dim3(64 * w), tinv_lds_bytes(n, w), s, n, nv,
                       w, H, V, tau, evals, Vout, ldv);
    return hipGetLastError();
}

hipError_t nonsym_eig(hipStream_t s, const double* A, int64_t lda, int n, void* ws, double* lam,
                      int32_t* kind, double* W, int32_t* info, double tol)
{
    if (n <= 0) return hipSuccess;
    if (n > EIG_MAX) return hipErrorInvalidValue;
    EigWs w = eig_carve(ws, n);
    hipLaunchKernelGGL(hessenberg_kernel<5>, dim3(1), dim3(1024), 0, s, A, lda, n, w.H, w.V, w.tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = fill_i32(s, (int32_t*)w.counter, 1, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(aberth_kernel, dim3((unsigned)ceil_div(n, AB_WAVES)), dim3(64 * AB_WAVES),
                       (size_t)(hcol_size(n) + n) * sizeof(double), s, n, w.H, w.zbuf, w.conv, w.counter, w.zfin, info,
                       fmax(tol, 4e-16), AB_MAX_IT);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(eig_pair_kernel, dim3(1), dim3(EP_THREADS), 0, s, n, w.zfin, w.H, w.wr, w.wi, w.kind0, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int iw = invit_waves(n);
    hipLaunchKernelGGL(invit_kernel, dim3((unsigned)ceil_div(n, iw)), dim3(64 * iw), invit_lds_bytes(n, iw), s, n, iw,
                       w.H, w.V, w.tau, w.wr, w.wi, w.kind0, w.Wraw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(sort_modes_kernel, dim3(1), dim3(SM_THREADS), (size_t)n * (2 * sizeof(double) + 2 * sizeof(int)),
                       s, n, w.wr, w.wi, w.kind0, w.Wraw, lam, kind, W);
    return hipGetLastError();
}

hipError_t eig_prepare()
{
    hipError_t e = hipFuncSetAttribute((const void*)aberth_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024 - 256);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)tri_invit_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)invit_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
}

hipError_t prepare_kernels()
{
    hipError_t e = gemm_prepare();
    if (e != hipSuccess) return e;
    e = small_prepare();
    if (e != hipSuccess) return e;
    return eig_prepare();
}

}  // namespace dmd
