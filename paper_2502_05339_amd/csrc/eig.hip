// FP64 eigen-decomposition of the reduced operator Atilde W = W Lambda (Sec. 3.1).
//
// Real nonsymmetric n x n matrix (n <= DMD_MAX_RANK), five kernels:
//  1. hessenberg_kernel (1 work-group): Householder reduction A = Q H Q^T, H in
//     registers across the work-group, the reflectors (v_k, tau_k) kept for
//     rebuilding Q; H is written row-major with its trace and squared Frobenius norm.
//  2. aberth_kernel (n single-wave work-groups): the eigenvalues as the roots of
//     det(zI - H), all refined at once by the Ehrlich-Aberth iteration, each Newton
//     ratio from a pivoted LU factorisation of H - zI differentiated in z.
//  2b. eig_pair_kernel (1 work-group): real eigenvalues and conjugate pairs told apart
//     and made exact (real, or exactly conjugate).
//  2c. invit_kernel (one single-wave work-group per real eigenvalue or pair): the
//     eigenvector by inverse iteration on H, taken through Q, normalised to unit 2-norm
//     (folded: [Re, Im] for a conjugate pair).
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
    double* Us;       // per output position, the packed rows of U (complex): n * n(n+1)/2 * 2
    int32_t* kind0;   // n
    int32_t* conv;    // 2 x n: converged flags of the two iterates
    uint32_t* counter;
};

static size_t eig_upk(int n) { return (size_t)n * (n + 1) / 2; }

size_t eig_workspace_bytes(int n)
{
    const size_t nn = (size_t)n * n;
    const size_t dbl = (nn + 2) + nn + n + nn + 2 * (size_t)n + 4 * (size_t)n + 2 * (size_t)n + (size_t)n * 2 * eig_upk(n);
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
    w.Us = p; p += (size_t)n * 2 * eig_upk(n);
    char* q = (char*)p;
    w.kind0 = (int32_t*)q; q += round_up((int64_t)n * sizeof(int32_t), 64);
    w.conv = (int32_t*)q; q += 2 * round_up((int64_t)n * sizeof(int32_t), 64);
    w.counter = (uint32_t*)q;
    return w;
}

// ====================================================================== 1. Hessenberg
// Householder reduction A = Q H Q^T, H held in registers: thread (ib, jb) of a 32 x 32
// grid keeps H(ib + 32 a, jb + 32 c), a, c < HS_N.  Step k, reflector P = I - tau v v^T of
// column k (rows k+1..):  with u = H v, w = H^T v and gamma = v^T H v taken from H before
// the step, P H P = H - tau (v w^T + u v^T) + tau^2 gamma v v^T on columns > k, and column
// k becomes (.., beta, 0, ..).  u, w and gamma are summed from per-thread partials in LDS
// (fixed order).  While the others update their entries, wave 0 forms the next column and
// the next reflector.  Three barriers per step.
constexpr int HS_N = (EIG_MAX + 31) / 32;

__global__ void __launch_bounds__(1024)
hessenberg_kernel(const double* __restrict__ A, int64_t lda, int n, double* H, double* V, double* tau)
{
    __shared__ double col[EIG_MAX];           // column k of H (rows > k), for v
    __shared__ double colpre[EIG_MAX];        // column k + 1 before step k
    __shared__ double us[EIG_MAX], ws[EIG_MAX];
    // partial u per column group jb; rows of odd length so that the 32 lanes of a store
    // (32 column groups, one row) fall in different banks
    constexpr int UPS = EIG_MAX + 1;
    __shared__ double upart[32 * UPS];
    __shared__ double wpart[32 * EIG_MAX];    // partial w per row group ib
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
        x2 = wave_sum(x2);
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
        auto vof = [&](int i) { return i == k + 1 ? 1.0 : (i > k + 1 && i < n ? col[i] * sc : 0.0); };
        double vr[HS_N], vc[HS_N];
#pragma unroll
        for (int a = 0; a < HS_N; ++a) { vr[a] = vof(ib + 32 * a); vc[a] = vof(jb + 32 * a); }
        if (wave == 1) {
            for (int i = k + 1 + lane; i < n; i += 64) V[(int64_t)k * n + i] = vof(i);
            if (lane == 0) tau[k] = tk;
        }
        // ---- partials of u = H v, w = H^T v, gamma = v^T H v; column k + 1 before the step
        double g = 0.0;
#pragma unroll
        for (int a = 0; a < HS_N; ++a) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < HS_N; ++c) t = fma(h[a][c], vc[c], t);
            const int i = ib + 32 * a;
            if (i < n) upart[jb * UPS + i] = t;
        }
#pragma unroll
        for (int c = 0; c < HS_N; ++c) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < HS_N; ++a) t = fma(vr[a], h[a][c], t);
            g = fma(t, vc[c], g);
            const int j = jb + 32 * c;
            if (j < n) wpart[ib * EIG_MAX + j] = t;
            if (j == k + 1)
#pragma unroll
                for (int a = 0; a < HS_N; ++a)
                    if (ib + 32 * a < n) colpre[ib + 32 * a] = h[a][c];
        }
        gpart[tid] = g;
        __syncthreads();
        // ---- sums in a fixed order
        if (tid < n) {
            double t = 0.0;
            for (int q = 0; q < 32; ++q) t += upart[q * UPS + tid];
            us[tid] = t;
        } else if (tid >= 256 && tid - 256 < n) {
            const int j = tid - 256;
            double t = 0.0;
            for (int q = 0; q < 32; ++q) t += wpart[q * EIG_MAX + j];
            ws[j] = t;
        } else if (wave == 15) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) t += gpart[q * 64 + lane];
            t = wave_sum(t);
            if (lane == 0) refl[3] = t;
        }
        __syncthreads();
        const double tg = tk * tk * refl[3];
        // ---- wave 0 first: column k + 1 after the step, and the reflector of step k + 1 (a
        // latency chain that the other waves' updates hide; it reads no entry of h)
        if (wave == 0 && k + 3 < n) {
            const double wk = ws[k + 1], vk = k + 1 < n ? 1.0 : 0.0;    // v_{k+1} = 1
            for (int i = k + 2 + lane; i < n; i += 64) {
                const double vi = vof(i);
                col[i] = colpre[i] - (tk * fma(vi, wk, us[i] * vk) - tg * vi * vk);
            }
            wave_sync_lds();
            reflector(k + 1);
        }
        // ---- H <- P H P on columns > k; column k -> (.., beta, 0, ..).  Per entry
        // tau (v_i w_j + u_i v_j) - tau^2 gamma v_i v_j = v_i A_j + v_j B_i with
        // A_j = tau w_j and B_i = tau u_i - tau^2 gamma v_i: two FMAs; columns <= k and
        // past n take A = v = 0 and rows past n take B = v = 0, which leaves them unchanged
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
            Bi[a] = i < n ? fma(tk, us[i], -tg * vr[a]) : 0.0;    // padding rows stay as they are
        }
#pragma unroll
        for (int a = 0; a < HS_N; ++a) {
            const int i = ib + 32 * a;
#pragma unroll
            for (int c = 0; c < HS_N; ++c) {
                const int j = jb + 32 * c;
                h[a][c] = fma(-vr[a], Aj[c], fma(-vcm[c], Bi[a], h[a][c]));
                if (j == k && tk != 0.0 && i == k + 1) h[a][c] = beta;
                if (j == k && i > k + 1) h[a][c] = 0.0;
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
//   z_i <- z_i - 1 / (p'(z_i)/p(z_i) - sum_{j != i} 1 / (z_i - z_j)).
// p'/p(z) = d/dz log det(H - zI) = sum_k u'_kk / u_kk over the pivots of the LU
// factorisation of H - zI with partial pivoting, differentiated in z alongside.  A
// Hessenberg matrix has one candidate row below each pivot, so the elimination carries a
// single active row (and its derivative) and reads row k + 1 of H at step k.
// One single-wave work-group per approximation, lanes over the columns of the active row.
// Iterations are separated by a grid-wide barrier (a counter in the workspace), so every
// approximation is updated from the same previous iterate and the result does not depend
// on scheduling.  The barrier's wait is bounded: a work-group that waits past the bound
// reports DMD_ERR_EIG_NOCONV and leaves, which ends the other work-groups' waits too.
// Start: n points on the circle about trace(H)/n whose radius is the spread
// (||H||_F^2 / n - |trace(H)/n|^2)^(1/2) that bounds the eigenvalues' deviation from their
// mean (Schur's inequality).  A root is converged when its correction falls below tol
// relative to |z| (the next correction of a simple root is of the cube of that size), or
// below 1e-9 |z| without shrinking by a factor 4 any more (the rounding floor of the
// evaluation, reached by clustered roots).
constexpr int AB_SLOTS = (EIG_MAX + 63) / 64;
static_assert(AB_SLOTS <= 4, "aberth_kernel keeps at most 4 columns per lane");
// columns of one lane, as one vector value: a run-time element index on a vector stays in
// registers, where the same index on a private array would put it in scratch
typedef double dvec4 __attribute__((ext_vector_type(4)));
constexpr int AB_MAX_IT = 200;
constexpr uint32_t AB_SPIN_CAP = 1u << 22;

__device__ __forceinline__ double bcast(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Start point j of the iteration (the same formula on every work-group).
__device__ __forceinline__ void ab_start(int j, int n, double cr, double rho, double* zr, double* zi)
{
    double s, c;
    sincospi(2.0 * (j + 0.4) / n, &s, &c);
    *zr = fma(rho, c, cr);
    *zi = rho * s;
}

// Row k + 1 of H for the lane's columns c > k (zero elsewhere), and the sub-diagonal
// entry H(k + 1, k): the operands of elimination step k.
struct AbRow {
    dvec4 v;
    double sub;
};
__device__ __forceinline__ AbRow ab_load_row(const double* __restrict__ Hr, int n, int k, int lane)
{
    AbRow r;
    const double* row = Hr + (int64_t)(k + 1) * n;
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) {
        const int c = lane + 64 * s;
        r.v[s] = (c > k && c < n) ? row[c] : 0.0;
    }
    r.sub = row[k];
    return r;
}

// p'/p at z for the row-major Hessenberg matrix Hr; false when H - zI has an exactly zero
// pivot (z is an eigenvalue).  Row k + 2 is loaded while step k runs.
__device__ bool ab_logdet_deriv(const double* __restrict__ Hr, int n, int lane, double zr, double zi,
                                double* sr_out, double* si_out)
{
    dvec4 ar, ai, dr, di;
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) {
        const int c = lane + 64 * s;
        ar[s] = c < n ? Hr[c] : 0.0;
        ai[s] = 0.0;
        dr[s] = 0.0;
        di[s] = 0.0;
        if (c == 0) { ar[s] -= zr; ai[s] = -zi; dr[s] = -1.0; }
    }
    double sr = 0.0, si = 0.0;
    bool sing = false;
    AbRow nxt = ab_load_row(Hr, n, 0, lane);
    for (int k = 0; k + 1 < n; ++k) {
        const AbRow cur = nxt;
        if (k + 2 < n) nxt = ab_load_row(Hr, n, k + 1, lane);
        const int ks = k >> 6, kl = k & 63;
        const double akr = bcast(ar[ks], kl), aki = bcast(ai[ks], kl);
        const double dkr = bcast(dr[ks], kl), dki = bcast(di[ks], kl);
        const double bk = cur.sub;
        if (fabs(bk) > fabs(akr) + fabs(aki)) {
            // pivot on row k + 1 (real pivot, no z at column k): a <- a - l b, l = a_k / b_k
            const double ib = 1.0 / bk;
            const double lr = akr * ib, li = aki * ib;
            const double dlr = dkr * ib, dli = dki * ib;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) {
                const int c = lane + 64 * s;
                if (c <= k || c >= n) continue;
                double bcr = cur.v[s], bci = 0.0, dbr = 0.0;
                if (c == k + 1) { bcr -= zr; bci = -zi; dbr = -1.0; }
                const double nr = ar[s] - fma(lr, bcr, -li * bci), ni = ai[s] - fma(lr, bci, li * bcr);
                const double ndr = dr[s] - fma(dlr, bcr, -dli * bci) - lr * dbr;
                const double ndi = di[s] - fma(dlr, bci, dli * bcr) - li * dbr;
                ar[s] = nr; ai[s] = ni; dr[s] = ndr; di[s] = ndi;
            }
        } else {
            // pivot on the active row: a <- b - l a, l = b_k / a_k, p'/p += a'_k / a_k
            const double m2 = fma(akr, akr, aki * aki);
            if (m2 == 0.0) { sing = true; break; }
            const double im2 = 1.0 / m2;
            const double ir = akr * im2, ii = -aki * im2;                   // 1 / a_k
            sr += fma(dkr, ir, -dki * ii);
            si += fma(dkr, ii, dki * ir);
            const double lr = bk * ir, li = bk * ii;
            const double tr = fma(lr, dkr, -li * dki), ti = fma(lr, dki, li * dkr);   // l a'_k
            const double dlr = -fma(tr, ir, -ti * ii), dli = -fma(tr, ii, ti * ir);  // l' = -l a'_k / a_k
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) {
                const int c = lane + 64 * s;
                if (c <= k || c >= n) continue;
                double bcr = cur.v[s], bci = 0.0, dbr = 0.0;
                if (c == k + 1) { bcr -= zr; bci = -zi; dbr = -1.0; }
                const double xr = ar[s], xi = ai[s], yr = dr[s], yi = di[s];
                ar[s] = bcr - fma(lr, xr, -li * xi);
                ai[s] = bci - fma(lr, xi, li * xr);
                dr[s] = dbr - fma(dlr, xr, -dli * xi) - fma(lr, yr, -li * yi);
                di[s] = -fma(dlr, xi, dli * xr) - fma(lr, yi, li * yr);
            }
        }
    }
    if (!sing) {
        const int ks = (n - 1) >> 6, kl = (n - 1) & 63;
        const double akr = bcast(ar[ks], kl), aki = bcast(ai[ks], kl);
        const double dkr = bcast(dr[ks], kl), dki = bcast(di[ks], kl);
        const double m2 = fma(akr, akr, aki * aki);
        if (m2 == 0.0) {
            sing = true;
        } else {
            const double ir = akr / m2, ii = -aki / m2;
            sr += fma(dkr, ir, -dki * ii);
            si += fma(dkr, ii, dki * ir);
        }
    }
    *sr_out = sr;
    *si_out = si;
    return !sing;
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, DMD_WAVE);
    return v;
}

__global__ void __launch_bounds__(64)
aberth_kernel(int n, const double* __restrict__ Hr, double* zbuf, int32_t* conv, uint32_t* counter,
              double* zfin, int32_t* info, double tol, int max_it)
{
    const int i = blockIdx.x, lane = threadIdx.x;
    const double tr = Hr[(int64_t)n * n], f2 = Hr[(int64_t)n * n + 1];
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
            const bool ok = ab_logdet_deriv(Hr, n, lane, zr, zi, &sr, &si);
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
                const double m = fma(ddr, ddr, ddi * ddi);
                if (m > 0.0) { qr += ddr / m; qi -= ddi / m; }
            }
            qr = wave_sum(qr);
            qi = wave_sum(qi);
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
        // publish iterate it + 1 and its converged flag (both double-buffered: a work-group
        // that is already one iteration ahead writes the other copy), then wait for every
        // work-group to have done the same
        double* zn = zbuf + (size_t)((it + 1) & 1) * 2 * n;
        int32_t* cn = conv + (size_t)((it + 1) & 1) * n;
        if (lane == 0) {
            __hip_atomic_store(zn + 2 * i, zr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(zn + 2 * i + 1, zi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(cn + i, done ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t target = (uint32_t)(it + 1) * (uint32_t)n;
            uint32_t polls = 0;
            while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(2);
                if (++polls > AB_SPIN_CAP) { timeout = true; break; }
            }
        }
        timeout = __shfl(timeout ? 1 : 0, 0, 64) != 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
        zfin[2 * i] = zr;
        zfin[2 * i + 1] = zi;
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
// Inverse iteration on the Hessenberg matrix, one single-wave work-group per real
// eigenvalue or pair: the LU factorisation of H - lambda I with partial pivoting (as in
// the eigenvalue iteration, pivots below eps ||H||_F raised to that value) writes the
// rows of U to the workspace; x = U^-1 (1, .., 1)^T by back-substitution (one dot product
// per row, rescaled when it grows past 1e100) is the eigenvector of H, normalised to unit
// 2-norm; the Hessenberg reflectors (A = Q H Q^T) then give the eigenvector Q x of A.
// A pair stores [Re, Im] in its two columns.
__global__ void __launch_bounds__(64)
invit_kernel(int n, const double* __restrict__ Hr, const double* __restrict__ Vg, const double* __restrict__ taug,
             const double* __restrict__ wr, const double* __restrict__ wi, const int32_t* __restrict__ kind0,
             double* Us, double* Wraw)
{
    const int p = blockIdx.x, lane = threadIdx.x;
    const int kd = kind0[p];
    if (kd == 2) return;
    const bool pair = kd == 1;
    const double lr = wr[p], li = pair ? wi[p] : 0.0;
    const double eps3 = 2.220446049250313e-16 * sqrt(Hr[(int64_t)n * n + 1]) + 1e-300;
    const int64_t npk = (int64_t)n * (n + 1) / 2;
    double* U = Us + (size_t)p * 2 * npk;                         // packed rows, complex
    auto rowoff = [&](int k) -> int64_t { return (int64_t)k * n - (int64_t)k * (k - 1) / 2; };
    dvec4 ar, ai;
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) {
        const int c = lane + 64 * s;
        ar[s] = c < n ? Hr[c] : 0.0;
        ai[s] = 0.0;
        if (c == 0) { ar[s] -= lr; ai[s] = -li; }
    }
    AbRow nxt = ab_load_row(Hr, n, 0, lane);
    for (int k = 0; k + 1 < n; ++k) {
        const AbRow cur = nxt;
        if (k + 2 < n) nxt = ab_load_row(Hr, n, k + 1, lane);
        const int ks = k >> 6, kl = k & 63;
        const double akr = bcast(ar[ks], kl), aki = bcast(ai[ks], kl);
        const double bk = cur.sub;
        double* Urow = U + 2 * rowoff(k);
        if (fabs(bk) > fabs(akr) + fabs(aki)) {
            const double piv = fabs(bk) < eps3 ? (bk < 0.0 ? -eps3 : eps3) : bk;
            const double ib = 1.0 / piv;
            const double l_r = akr * ib, l_i = aki * ib;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) {
                const int c = lane + 64 * s;
                if (c < k || c >= n) continue;
                double bcr = c == k ? piv : cur.v[s], bci = 0.0;
                if (c == k + 1) { bcr -= lr; bci = -li; }
                Urow[2 * (c - k)] = bcr;
                Urow[2 * (c - k) + 1] = bci;
                if (c == k) continue;
                const double nr = ar[s] - fma(l_r, bcr, -l_i * bci), ni = ai[s] - fma(l_r, bci, l_i * bcr);
                ar[s] = nr; ai[s] = ni;
            }
        } else {
            double pr = akr, pi = aki;
            if (fabs(pr) + fabs(pi) < eps3) { pr = eps3; pi = 0.0; }
            const double m2 = fma(pr, pr, pi * pi);
            const double ir = pr / m2, ii = -pi / m2;
            const double l_r = bk * ir, l_i = bk * ii;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) {
                const int c = lane + 64 * s;
                if (c < k || c >= n) continue;
                const double xr = c == k ? pr : ar[s], xi = c == k ? pi : ai[s];
                Urow[2 * (c - k)] = xr;
                Urow[2 * (c - k) + 1] = xi;
                if (c == k) continue;
                double bcr = cur.v[s], bci = 0.0;
                if (c == k + 1) { bcr -= lr; bci = -li; }
                ar[s] = bcr - fma(l_r, xr, -l_i * xi);
                ai[s] = bci - fma(l_r, xi, l_i * xr);
            }
        }
    }
    {
        const int k = n - 1, ks = k >> 6, kl = k & 63;
        double pr = bcast(ar[ks], kl), pi = bcast(ai[ks], kl);
        if (fabs(pr) + fabs(pi) < eps3) { pr = eps3; pi = 0.0; }
        if (lane == kl) { U[2 * rowoff(k)] = pr; U[2 * rowoff(k) + 1] = pi; }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");    // the rows of U are read back below
    // back-substitution U x = rs (1, .., 1)^T, rows from the last; row k - 1 loaded while
    // row k is solved
    dvec4 xr, xi;
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) { xr[s] = 0.0; xi[s] = 0.0; }
    double rs = 1.0;
    auto load_u = [&](int k, dvec4& vr, dvec4& vi) {
        const double* Urow = U + 2 * rowoff(k);
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) {
            const int c = lane + 64 * s;
            const bool in = c >= k && c < n;
            vr[s] = in ? Urow[2 * (c - k)] : 0.0;
            vi[s] = in ? Urow[2 * (c - k) + 1] : 0.0;
        }
    };
    dvec4 nur, nui;
    load_u(n - 1, nur, nui);
    for (int k = n - 1; k >= 0; --k) {
        const dvec4 ur = nur, ui = nui;
        if (k > 0) load_u(k - 1, nur, nui);
        const int ks = k >> 6, kl = k & 63;
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) {
            const int c = lane + 64 * s;
            if (c <= k) continue;
            tr += fma(ur[s], xr[s], -ui[s] * xi[s]);
            ti += fma(ur[s], xi[s], ui[s] * xr[s]);
        }
        tr = wave_sum(tr);
        ti = wave_sum(ti);
        const double dr = bcast(ur[ks], kl), di = bcast(ui[ks], kl);
        const double nr = rs - tr, ni = -ti;
        const double m2 = fma(dr, dr, di * di);
        double vr = fma(nr, dr, ni * di) / m2, vi = fma(ni, dr, -nr * di) / m2;
        if (fabs(vr) + fabs(vi) > 1e100) {
            xr *= 1e-100; xi *= 1e-100; rs *= 1e-100;
            vr *= 1e-100; vi *= 1e-100;
        }
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s)
            if (s == ks && lane == kl) { xr[s] = vr; xi[s] = vi; }
    }
    // unit 2-norm
    double nn2 = 0.0;
#pragma unroll
    for (int s = 0; s < AB_SLOTS; ++s) nn2 = fma(xr[s], xr[s], fma(xi[s], xi[s], nn2));
    nn2 = wave_sum(nn2);
    const double inv = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 0.0;
    xr *= inv;
    xi *= inv;
    // y = Q x with Q = P_0 P_1 .. P_{n-3}: P_k = I - tau_k v_k v_k^T (v_k rows k+1.., v_{k+1} = 1)
    auto load_v = [&](int k, dvec4& v) {
#pragma unroll
        for (int s = 0; s < AB_SLOTS; ++s) {
            const int c = lane + 64 * s;
            v[s] = (c > k && c < n) ? Vg[(int64_t)k * n + c] : 0.0;
        }
    };
    if (n > 2) {
        dvec4 nv;
        load_v(n - 3, nv);
        for (int k = n - 3; k >= 0; --k) {
            const dvec4 v = nv;
            if (k > 0) load_v(k - 1, nv);
            const double t = taug[k];
            double gr = 0.0, gi = 0.0;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) { gr = fma(v[s], xr[s], gr); gi = fma(v[s], xi[s], gi); }
            gr = wave_sum(gr) * t;
            gi = wave_sum(gi) * t;
#pragma unroll
            for (int s = 0; s < AB_SLOTS; ++s) { xr[s] = fma(-gr, v[s], xr[s]); xi[s] = fma(-gi, v[s], xi[s]); }
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

hipError_t nonsym_eig(hipStream_t s, const double* A, int64_t lda, int n, void* ws, double* lam,
                      int32_t* kind, double* W, int32_t* info, double tol)
{
    if (n <= 0) return hipSuccess;
    if (n > EIG_MAX) return hipErrorInvalidValue;
    EigWs w = eig_carve(ws, n);
    hipLaunchKernelGGL(hessenberg_kernel, dim3(1), dim3(1024), 0, s, A, lda, n, w.H, w.V, w.tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = fill_i32(s, (int32_t*)w.counter, 1, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(aberth_kernel, dim3(n), dim3(64), 0, s, n, w.H, w.zbuf, w.conv, w.counter, w.zfin, info,
                       fmax(tol, 4e-16), AB_MAX_IT);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(eig_pair_kernel, dim3(1), dim3(EP_THREADS), 0, s, n, w.zfin, w.H, w.wr, w.wi, w.kind0, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(invit_kernel, dim3(n), dim3(64), 0, s, n, w.H, w.V, w.tau, w.wr, w.wi, w.kind0, w.Us, w.Wraw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(sort_modes_kernel, dim3(1), dim3(SM_THREADS), (size_t)n * (2 * sizeof(double) + 2 * sizeof(int)),
                       s, n, w.wr, w.wi, w.kind0, w.Wraw, lam, kind, W);
    return hipGetLastError();
}

hipError_t eig_prepare() { return hipSuccess; }
hipError_t prepare_kernels()
{
    hipError_t e = gemm_prepare();
    if (e != hipSuccess) return e;
    e = small_prepare();
    if (e != hipSuccess) return e;
    return eig_prepare();
}

}  // namespace dmd
