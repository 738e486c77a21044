// FP64 eigen-decomposition of the reduced operator Atilde W = W Lambda (Sec. 3.1).
//
// Real nonsymmetric n x n matrix (n <= DMD_MAX_RANK), three kernels:
//  1. hessenberg_kernel (1 work-group): Householder reduction A = Q H Q^T, H in
//     registers across the work-group, the reflectors (v_k, tau_k) kept for
//     rebuilding Q.
//  2. francis_kernel (ceil(n / nr) work-groups): every work-group holds H packed
//     in LDS (upper Hessenberg plus the two extra sub-diagonals a double-shift
//     bulge needs) and runs the same implicit double-shift QR iteration with
//     deflation, producing the real Schur form T; each work-group rebuilds and
//     updates only its own nr rows of the Schur vectors Z (Z = Q * product of
//     the QR reflectors), so no work-group ever waits for another.  2 x 2
//     diagonal blocks with real eigenvalues are split by a rotation.  T, its block
//     structure and Z go to global scratch.
//  2b. eigvec_kernel (one single-wave work-group per eigenvalue): the eigenvector x
//     of T by back-substitution, column by column (each lane keeps the residual of
//     its rows, so a row costs one complex product and a broadcast), normalised to
//     unit 2-norm (Z is orthogonal, so the norm carries over), then the column
//     Z x of the eigenvector matrix (folded: [Re, Im] for a conjugate pair).
//  3. sort_modes_kernel (1 work-group): canonical order (ascending |arg lambda|,
//     ties by descending |lambda|, Im > 0 member of a pair first), lambda, kind
//     and the permuted folded eigenvectors (pair -> [Re w, Im w], LAPACK storage).
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace dmd {

// workspace layout (doubles unless noted)
struct EigWs {
    double* H;      // n x n
    double* V;      // n x n reflector vectors (column k: rows k+1..n-1)
    double* tau;    // n
    double* Wraw;   // n x n unsorted folded eigenvectors
    double* wr;     // n
    double* wi;     // n
    int32_t* kind0; // n
    double* Z;      // n x n Schur vectors, column-major
    double* T;      // real Schur form, packed as in francis_kernel (<= n x n), then max |T_ij|
    int32_t* blk;   // n: 0 real eigenvalue, 1/2 first/second of a 2 x 2 block
};

static int eig_rows_per_wg(int n) { return n <= 64 ? 8 : 16; }
static int eig_grid(int n) { return (int)ceil_div(n, eig_rows_per_wg(n)); }

size_t eig_workspace_bytes(int n)
{
    size_t nn = (size_t)n * n;
    return (5 * nn + 2 + 4 * (size_t)n) * sizeof(double) + 2 * (size_t)round_up((int64_t)n * sizeof(int32_t), 64) + 256;
}

static EigWs eig_carve(void* ws, int n)
{
    EigWs w;
    double* p = (double*)ws;
    size_t nn = (size_t)n * n;
    w.H = p; p += nn;
    w.V = p; p += nn;
    w.Wraw = p; p += nn;
    w.Z = p; p += nn;
    w.T = p; p += nn + 2;                // + max |T_ij|
    w.tau = p; p += n;
    w.wr = p; p += n;
    w.wi = p; p += n;
    p += n;
    w.kind0 = (int32_t*)p;
    p = (double*)((char*)p + round_up((int64_t)n * sizeof(int32_t), 64));
    w.blk = (int32_t*)p;
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
#pragma unroll
    for (int a = 0; a < HS_N; ++a)
#pragma unroll
        for (int c = 0; c < HS_N; ++c) {
            const int i = ib + 32 * a, j = jb + 32 * c;
            if (i < n && j < n) H[(int64_t)j * n + i] = h[a][c];
        }
}

// ====================================================================== 2. Francis QR
// Packed Hessenberg with 3 sub-diagonals: column j holds rows 0..min(j+3, n-1), i.e.
// min(j+4, n) entries; the offset of column j is computed, not looked up.
__host__ __device__ __forceinline__ int hp_col(int j, int n) {
    const int head = (j * (j + 7)) >> 1;                             // columns 0..j-1 all hold i+4 rows
    const int tail = (((n - 3) * (n + 4)) >> 1) + (j - (n - 3)) * n;  // full columns from n-3 on
    return n <= 4 ? j * n : (j <= n - 3 ? head : tail);
}
constexpr int FR_THREADS = 256;
constexpr int FR_VCH = 16;    // reflectors staged in LDS at a time in the Z-slab setup
// row-update roles use threads 1..n, Z-slab roles the last 16, plus one deferred-write thread
static_assert(EIG_MAX + 1 + 1 + 16 <= FR_THREADS, "francis_kernel thread roles overlap");

struct HP {
    double* a;
    int n;
    __device__ __forceinline__ double& operator()(int i, int j) const { return a[hp_col(j, n) + i]; }
};


__device__ __forceinline__ void house3(double x, double y, double z, double* v1, double* v2, double* tau, double* beta)
{
    const double nrm = sqrt(x * x + y * y + z * z);
    if (nrm == 0.0 || (y == 0.0 && z == 0.0)) { *tau = 0.0; *v1 = 0.0; *v2 = 0.0; *beta = x; return; }
    const double b = x >= 0.0 ? -nrm : nrm;
    const double d = x - b;                 // |d| >= |x|, never zero here
    const double ibd = 1.0 / (b * d);       // one division gives 1/b and 1/d
    *tau = -d * d * ibd;                    // (b - x) / b
    const double sc = b * ibd;              // 1 / (x - b)
    *v1 = y * sc;
    *v2 = z * sc;
    *beta = b;
}

// Reflector of the bulge step in unnormalised form: P = I - t u u^T with u = (d, y, z),
// d = x - beta, beta = -sign(x) ||(x, y, z)||, and t = 2 / (u^T u) taken from the u that
// is actually used, so P is orthogonal to rounding whatever the error of the norm.
// P (x, y, z)^T = (beta, 0, 0)^T.  t = 0 when y = z = 0 (P = I).
__device__ __forceinline__ void reflector3(double x, double y, double z, double* d, double* t, double* beta)
{
    const double yz = fma(y, y, z * z);
    const double sig = fma(x, x, yz);
    if (yz == 0.0 || !(sig >= 1e-280)) {      // nothing to annihilate, or too small to scale safely
        if (yz == 0.0) { *t = 0.0; *d = 0.0; *beta = x; return; }
        double v1, v2, tau, b;
        house3(x, y, z, &v1, &v2, &tau, &b);
        // same reflector: u = (x - b) (1, v1, v2), t = tau / (x - b)^2
        const double dd = x - b;
        *d = dd; *t = tau / (dd * dd); *beta = b;
        return;
    }
    const double r = rsqrt_nr(sig);
    const double nrm = sig * r;
    const double dd = x >= 0.0 ? x + nrm : x - nrm;
    *d = dd;
    *beta = x >= 0.0 ? -nrm : nrm;
    *t = 2.0 * rcp_nr(fma(dd, dd, yz));
}

__global__ void __launch_bounds__(FR_THREADS)
francis_kernel(int n, int nr, const double* __restrict__ Hg, const double* __restrict__ Vg,
               const double* __restrict__ taug, double* Zg, double* Tg, int32_t* blkg, double* wr, double* wi,
               int32_t* kind0, int32_t* info, double defl_tol)
{
    extern __shared__ double sm[];
    int* blk = reinterpret_cast<int*>(sm);                      // n ints
    const int ioff = (int)round_up(n, 2) / 2;                   // in doubles
    double* Hs = sm + ioff;
    __shared__ int sh_l, sh_stop, sh_iter_total;
    __shared__ double sh_v[4];   // rotation of a 2x2 block split
    __shared__ int sh_lc[2];     // deflation search result (double-buffered)
    __shared__ double sh_red[4];

    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, nw = nt >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: wave-level branches stay scalar
    const int hsize = hp_col(n, n);
    double* Zs = Hs + hsize;                                    // nr x n
    HP H{Hs, n};
    const int r0 = blockIdx.x * nr;
    const int nrows = min(nr, n - r0);

    // packed H, eight columns at a time with their loads in flight (nt > n + 3: one entry
    // of a column per thread)
    static_assert(FR_THREADS > EIG_MAX + 3, "francis_kernel loads one entry per column and thread");
    for (int j0 = 0; j0 < n; j0 += 8) {
        double hv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u;
            hv[u] = (j < n && tid <= j + 1 && tid < n) ? Hg[(int64_t)j * n + tid] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u;
            if (j < n && tid <= min(j + 3, n - 1)) H(tid, j) = hv[u];
        }
    }
    // Z slab = rows r0.. of Q = P_0 P_1 ... P_{n-3}: identity rows with the reflectors applied
    // on the right (below)
    __syncthreads();
    // Each group of 16 lanes keeps one row of the slab in registers (entries gl + 16 s) and
    // takes it through the reflectors in order: per reflector a 16-lane dot product (a
    // fixed-shape sum inside the group) and an update.  The reflectors come in chunks of
    // FR_VCH columns of V (and their tau) copied to LDS by the whole work-group with all
    // loads in flight.  V is zero above the start of each reflector, so every slot takes part.
    {
        constexpr int ZS = (EIG_MAX + 15) / 16;                     // row entries per lane
        static_assert(FR_THREADS / 16 >= 16, "one 16-lane group per Z-slab row (16 rows at most)");
        const int grp = tid >> 4, gl = tid & 15;
        double zr[ZS];
#pragma unroll
        for (int sl = 0; sl < ZS; ++sl) {
            const int j = gl + 16 * sl;
            zr[sl] = (grp < nrows && j < n && r0 + grp == j) ? 1.0 : 0.0;
        }
        double* Vst = Zs + nr * n;                                  // FR_VCH x n
        double* tst = Vst + FR_VCH * n;                             // FR_VCH
        for (int k0 = 0; k0 + 2 < n; k0 += FR_VCH) {
            const int kc = min(FR_VCH, n - 2 - k0);
            __syncthreads();                                        // the previous chunk is consumed
            for (int e0 = tid; e0 < kc * n; e0 += 4 * nt) {
                double t4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * nt;
                    t4[u] = e < kc * n ? Vg[(int64_t)k0 * n + e] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (e0 + u * nt < kc * n) Vst[e0 + u * nt] = t4[u];
            }
            if (tid < kc) tst[tid] = taug[k0 + tid];
            __syncthreads();
            for (int kk = 0; kk < kc; ++kk) {
                const double tk = tst[kk];
                if (tk == 0.0) continue;                            // uniform
                const double* v = Vst + kk * n;
                double vv[ZS];
                double d = 0.0;
#pragma unroll
                for (int sl = 0; sl < ZS; ++sl) {
                    const int j = gl + 16 * sl;
                    vv[sl] = j < n ? v[j] : 0.0;
                    d = fma(zr[sl], vv[sl], d);
                }
                d += __shfl_xor(d, 8, 16);
                d += __shfl_xor(d, 4, 16);
                d += __shfl_xor(d, 2, 16);
                d += __shfl_xor(d, 1, 16);
                d *= tk;
#pragma unroll
                for (int sl = 0; sl < ZS; ++sl) zr[sl] -= d * vv[sl];
            }
        }
        // the slab into LDS for the QR iteration (rows past nrows are zero)
        if (grp < nr)
#pragma unroll
            for (int sl = 0; sl < ZS; ++sl) {
                const int j = gl + 16 * sl;
                if (j < n) Zs[grp * n + j] = zr[sl];
            }
    }
    __syncthreads();

    // max |H_ij| (used when a diagonal pair is exactly zero, and for the pivot floor)
    {
        double mx = 0.0;
        for (int j = tid; j < n; j += nt)
            for (int i = 0; i <= min(j + 1, n - 1); ++i) mx = fmax(mx, fabs(H(i, j)));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) sh_red[wave] = mx;
        __syncthreads();
        if (tid == 0) { double m = 0.0; for (int w = 0; w < nw; ++w) m = fmax(m, sh_red[w]); sh_red[0] = m; }
        __syncthreads();
    }
    const double hnorm = sh_red[0];
    const double eps = defl_tol;             // deflation: |h(k,k-1)| <= eps (|h(k-1,k-1)| + |h(k,k)|)
    if (tid == 0) { sh_stop = 0; sh_iter_total = 0; }
    __syncthreads();
    // ---- implicit double-shift QR (all waves; one barrier per bulge step)
    // Roles within bulge step k (reflector P_k on rows/columns k .. k+m-1, m = 3, or 2
    // for the final step of a sweep), fixed by the thread index:
    //   tid <= min(k+3, hi)      column update of row tid; the rows k .. k+m-1 first
    //                            apply the row update to their corner entries
    //   k+m <= tid-1 < n         row update of column tid-1
    //   tid >= nt - nrows        column update of one row of this work-group's Z slab
    //   tid == nt - nrows - 1    deferred write of the column that step k-1 reduced
    // The roles touch disjoint entries, so the only barrier is the one that ends the step.
    {
        int hi = n - 1, its = 0, total = 0, parity = 0;
        bool stop = false;
        const int zt0 = nt - nrows;              // first Z-role thread
        const int pend_t = zt0 - 1;              // thread doing the deferred writes
        const bool zrole = tid >= zt0;
        // offset (from Hs) of this thread's row-update column tid-1 or Z-slab row
        const int base_t = (tid >= 1 && tid <= n) ? hp_col(tid - 1, n) : (zrole ? hsize + (tid - zt0) * n : 0);
        if (tid == 0) { sh_lc[0] = 0; sh_lc[1] = 0; }
        __syncthreads();
        while (hi >= 0) {
            // deflation point: largest l <= hi with negligible H(l, l-1), searched in parallel
            for (int k = hi - tid; k >= 1; k -= nt) {
                double sd = fabs(H(k - 1, k - 1)) + fabs(H(k, k));
                if (sd == 0.0) sd = hnorm;
                if (fabs(H(k, k - 1)) <= eps * sd) { atomicMax(&sh_lc[parity], k); break; }
            }
            __syncthreads();
            const int l = sh_lc[parity];
            if (tid == 0) {
                sh_lc[parity ^ 1] = 0;
                if (l > 0) H(l, l - 1) = 0.0;   // deflate exactly (read again only after a barrier)
            }
            parity ^= 1;
            if (l == hi) { hi -= 1; its = 0; __syncthreads(); continue; }
            if (l == hi - 1) {
                // 2x2 block (p, q): split it if its eigenvalues are real
                const int p = hi - 1, q = hi;
                const double a = H(p, p), b = H(p, q), c = H(q, p), d = H(q, q);
                double cs_ = 1.0, sn_ = 0.0;
                bool rot = false;
                if (c != 0.0) {
                    const double hp = 0.5 * (a - d);
                    const double disc = hp * hp + b * c;
                    if (disc >= 0.0) {
                        const double sq = sqrt(disc);
                        const double mu = 0.5 * (a + d) + (hp >= 0.0 ? sq : -sq);
                        double e1 = b, e2 = mu - a;             // eigenvector (b, mu - a)
                        double f1 = mu - d, f2 = c;             // or (mu - d, c)
                        if (e1 * e1 + e2 * e2 < f1 * f1 + f2 * f2) { e1 = f1; e2 = f2; }
                        const double nr_ = sqrt(e1 * e1 + e2 * e2);
                        if (nr_ > 0.0) { cs_ = e1 / nr_; sn_ = e2 / nr_; rot = true; }
                    }
                }
                __syncthreads();
                if (rot) {
                    for (int j = p + tid; j < n; j += nt) {          // rows p, q <- G^T rows
                        const double x = H(p, j), y = H(q, j);
                        H(p, j) = cs_ * x + sn_ * y;
                        H(q, j) = -sn_ * x + cs_ * y;
                    }
                    __syncthreads();
                    for (int i = tid; i <= q; i += nt) {             // columns p, q <- columns G
                        const double x = H(i, p), y = H(i, q);
                        H(i, p) = cs_ * x + sn_ * y;
                        H(i, q) = -sn_ * x + cs_ * y;
                    }
                    for (int rl = tid; rl < nrows; rl += nt) {
                        const double x = Zs[rl * n + p], y = Zs[rl * n + q];
                        Zs[rl * n + p] = cs_ * x + sn_ * y;
                        Zs[rl * n + q] = -sn_ * x + cs_ * y;
                    }
                    __syncthreads();
                    if (tid == 0) H(q, p) = 0.0;
                }
                hi -= 2; its = 0;
                __syncthreads();
                continue;
            }
            ++its;
            if (++total > 40 * n) { stop = true; break; }   // uniform: every thread counts alike
            // shifts: eigenvalues of the trailing 2x2 block (exceptional shifts at 10 and 20)
            double s, t;
            if (its == 10 || its == 20) {
                const double w = fabs(H(hi, hi - 1)) + (hi >= 2 ? fabs(H(hi - 1, hi - 2)) : 0.0);
                s = 2.0 * H(hi, hi) + 1.5 * w;
                t = (H(hi, hi) + 0.75 * w) * (H(hi, hi) + 0.75 * w);
            } else {
                s = H(hi - 1, hi - 1) + H(hi, hi);
                t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
            }
            // first column of (H - mu1)(H - mu2) on the active block
            const double x0 = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
            const double y0 = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
            const double z0 = H(l + 1, l) * H(l + 2, l + 1);
            __syncthreads();   // every thread has read the shift inputs before H changes
            int pk = -1;       // column reduced by the previous step, written one step late
            int poff = 0;      // its packed offset
            double pbeta = 0.0;
            // packed offsets of columns k-1 .. k+2, advanced by the column lengths min(j+4, n)
            int hm = hp_col(max(l - 1, 0), n), hk0 = hp_col(l, n), hk1 = hp_col(l + 1, n), hk2 = hp_col(l + 2, n);
            double e0 = 0.0, e1 = 0.0, e2 = 0.0;   // this thread's operands, carried between steps
            int prole = 0;
            // One bulge step k.  G (general) covers the first step of the sweep (vector from
            // the shift polynomial) and the last two (the block ends: m = 2 or rows past
            // hi); every other step takes the lean path with m = 3 and rows up to k+3.
            auto step = [&](const int k, auto general) {
                constexpr bool G = decltype(general)::value;
                const int m = G ? ((k == hi - 1) ? 2 : 3) : 3;
                const int crow = G ? min(k + 3, hi) : k + 3;
                if (!G || k > l) { hm = hk0; hk0 = hk1; hk1 = hk2; hk2 += min(k + 5, n); }
                // ---- loads, all issued before the reflector is formed
                double x, y, z;
                if (G && k == l) { x = x0; y = y0; z = z0; }
                else { x = Hs[hm + k]; y = Hs[hm + k + 1]; z = Hs[hm + k + 2]; }
                // role: 1 column update of row tid, 2 row update of column tid-1, 3 Z row
                const bool colr = tid <= crow;
                const int role = colr ? 1 : (zrole ? 3 : ((tid - 1 >= k + m && tid <= n) ? 2 : 0));
                const int o0 = colr ? hk0 + tid : base_t + k;
                const int o1 = colr ? hk1 + tid : base_t + k + 1;
                const int o2 = colr ? hk2 + tid : base_t + k + 2;
                // a thread that keeps its role finds two of its operands in registers (the
                // entries it updated in the previous step); only the third is new
                if (role != prole || (G && k == l)) { e0 = Hs[o0]; e1 = Hs[o1]; }
                e2 = Hs[o2];
                prole = role;
                // the corner C(a, b) = H(k+a, k+b) is needed only by the waves holding rows k..k+m-1
                const bool cw = (wave == (k >> 6)) || (wave == ((k + m - 1) >> 6));
                double c00, c10, c20, c01, c11, c21, c02, c12, c22;   // read only where cw
                if (cw) {
                    c00 = Hs[hk0 + k]; c10 = Hs[hk0 + k + 1]; c20 = Hs[hk0 + k + 2];
                    c01 = Hs[hk1 + k]; c11 = Hs[hk1 + k + 1]; c21 = Hs[hk1 + k + 2];
                    c02 = Hs[hk2 + k]; c12 = Hs[hk2 + k + 1]; c22 = Hs[hk2 + k + 2];
                }
                if (G && m == 2) {
                    z = 0.0; e2 = 0.0;
                    if (cw) { c20 = 0.0; c21 = 0.0; c02 = 0.0; c12 = 0.0; c22 = 0.0; }
                }
                double d, t, beta;
                reflector3(x, y, z, &d, &t, &beta);
                // ---- P_k = I - t u u^T, u = (d, y, z), applied to the operands: rows k..k+m-1
                // of the corner first take the row update (s_b), then every role applies the
                // same formula (P is symmetric, so rows and columns transform alike)
                if (t != 0.0) {
                    if (cw) {
                        const double s0 = (d * c00 + y * c10 + z * c20) * t;
                        const double s1 = (d * c01 + y * c11 + z * c21) * t;
                        const double s2 = (d * c02 + y * c12 + z * c22) * t;
                        const int a = tid - k;
                        const double ua = !colr ? 0.0 : (a == 0 ? d : (a == 1 ? y : (a == 2 ? z : 0.0)));
                        e0 -= ua * s0;
                        e1 -= ua * s1;
                        e2 -= ua * s2;
                    }
                    const double w = (d * e0 + y * e1 + z * e2) * t;
                    e0 -= w * d;
                    e1 -= w * y;
                    e2 -= w * z;
                    if (role != 0) {
                        Hs[o0] = e0;
                        Hs[o1] = e1;
                        if (!G || m == 3) Hs[o2] = e2;
                    }
                }
                if (tid == pend_t && pk >= 0) {             // column pk: (beta, 0, 0) below its subdiagonal
                    Hs[poff + pk + 1] = pbeta; Hs[poff + pk + 2] = 0.0;
                    if (pk + 3 <= hi) Hs[poff + pk + 3] = 0.0;
                }
                if (!G || k > l) { pk = k - 1; poff = hm; pbeta = beta; }
                // operands of the next step: this step's second and third entries
                e0 = e1; e1 = e2;
                __syncthreads();
            };
            step(l, std::true_type{});
            for (int k = l + 1; k <= hi - 3; ++k) step(k, std::false_type{});
            for (int k = max(l + 1, hi - 2); k <= hi - 1; ++k) step(k, std::true_type{});
            if (tid == pend_t && pk >= 0) {
                Hs[poff + pk + 1] = pbeta; Hs[poff + pk + 2] = 0.0;
                if (pk + 3 <= hi) Hs[poff + pk + 3] = 0.0;
            }
            __syncthreads();
        }
        if (tid == 0) { sh_stop = stop ? 1 : 0; sh_iter_total = total; }
    }
    __syncthreads();
    if (sh_stop) {
        if (blockIdx.x == 0 && tid == 0) set_status(info, DMD_ERR_EIG_NOCONV);
    }
    if (blockIdx.x == 0 && tid == 0 && info) atomicAdd(&info[2], sh_iter_total);

    // ---- block structure of T and eigenvalues
    if (tid == 0) {
        int k = 0;
        while (k < n) {
            if (k + 1 < n && H(k + 1, k) != 0.0) { blk[k] = 1; blk[k + 1] = 2; k += 2; }
            else { blk[k] = 0; k += 1; }
        }
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int k = tid; k < n; k += nt) {
            if (blk[k] == 0) { wr[k] = H(k, k); wi[k] = 0.0; kind0[k] = 0; }
            else {
                const int p = blk[k] == 1 ? k : k - 1;
                const double a = H(p, p), b = H(p, p + 1), c = H(p + 1, p), d = H(p + 1, p + 1);
                const double hp = 0.5 * (a - d);
                const double im = sqrt(fmax(-(hp * hp + b * c), 0.0));
                wr[k] = 0.5 * (a + d);
                wi[k] = blk[k] == 1 ? im : -im;
                kind0[k] = blk[k];
            }
        }
    }
    // ---- T, max |T_ij| (stored after T), the block structure and this work-group's rows
    // of Z to global scratch
    if (blockIdx.x == 0) {
        double mx = 0.0;
        for (int j = tid; j < n; j += nt)
            for (int i = 0; i <= min(j + 1, n - 1); ++i) mx = fmax(mx, fabs(H(i, j)));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        __syncthreads();
        if (lane == 0) sh_red[wave] = mx;
        __syncthreads();
        if (tid == 0) { double m = 0.0; for (int w = 0; w < nw; ++w) m = fmax(m, sh_red[w]); Tg[hsize] = m; }
        for (int e = tid; e < hsize; e += nt) Tg[e] = Hs[e];
        for (int k = tid; k < n; k += nt) blkg[k] = blk[k];
    }
    for (int e = tid; e < nrows * n; e += nt) {
        const int rl = e % nrows, c = e / nrows;
        Zg[(int64_t)c * n + r0 + rl] = Zs[rl * n + c];
    }
}

// ====================================================================== 2b. eigenvectors
// Eigenvector of the quasi-triangular T for eigenvalue index k (lambda = lre + i lim; a
// pair's first member has lim > 0), by back-substitution on (T - lambda) x = 0 with x_j = 0
// for j > top.  Column-oriented: lane l keeps the residuals r_i = -sum_{j > i} T(i, j) x_j
// of rows i = l, l + 64, l + 128; once x_i (or the pair x_ia, x_i of a 2 x 2 block) is known
// from the owner lane's residual, every lane subtracts T(i', i) x_i from its rows i' above.
// Tiny pivots are raised to smin; entries past 1e100 rescale x and r.
constexpr int EV_SLOTS = (EIG_MAX + 63) / 64;
static_assert(EV_SLOTS <= 4, "eigvec_kernel keeps at most 4 rows per lane");
// rows of one lane, as one vector value: a run-time element index on a vector stays in
// registers, where the same index on a private array would put it in scratch
typedef double evrow __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double bcast(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

__global__ void __launch_bounds__(64)
eigvec_kernel(int n, const double* __restrict__ Tg, const int32_t* __restrict__ blkg,
              const double* __restrict__ Zg, double* __restrict__ Wraw, double eps)
{
    extern __shared__ __align__(16) double evs[];
    const int k = blockIdx.x, lane = threadIdx.x;
    const int bk = blkg[k];
    if (bk == 2) return;                                   // second member: done with the first
    const bool pair = bk == 1;
    const int top = pair ? k + 1 : k;
    const int tsize = hp_col(top + 1, n);                  // columns 0..top of T
    double* Ts = evs;
    double* xs = evs + round_up(hp_col(n, n), 2);          // 2n: normalised Re, Im of x
    int* bs = reinterpret_cast<int*>(xs + 2 * n);          // n: block structure
    for (int e0 = lane; e0 < tsize; e0 += 8 * 64) {          // eight loads in flight per lane
        double tv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) tv[u] = e0 + 64 * u < tsize ? Tg[e0 + 64 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e0 + 64 * u < tsize) Ts[e0 + 64 * u] = tv[u];
    }
    for (int e = lane; e < n; e += 64) bs[e] = blkg[e];
    __syncthreads();
    HP T{Ts, n};

    const double smin = fmax(eps * Tg[hp_col(n, n)], 1e-290);   // max |T_ij| is stored after T
    double lre, lim;
    cplx xk, xk1 = {0.0, 0.0};
    if (!pair) { lre = T(k, k); lim = 0.0; xk = {1.0, 0.0}; }
    else {
        const double a = T(k, k), b = T(k, k + 1), c = T(k + 1, k), d = T(k + 1, k + 1);
        const double hp = 0.5 * (a - d);
        lre = 0.5 * (a + d);
        lim = sqrt(fmax(-(hp * hp + b * c), 0.0));
        // eigenvector of [[a b][c d]] for lre + i lim: (b, lambda - a) or (lambda - d, c)
        double e1r = b, e1i = 0.0, e2r = lre - a, e2i = lim;
        const double f1r = lre - d, f1i = lim, f2r = c, f2i = 0.0;
        if (e1r * e1r + e2r * e2r + e2i * e2i < f1r * f1r + f1i * f1i + f2r * f2r) {
            e1r = f1r; e1i = f1i; e2r = f2r; e2i = f2i;
        }
        xk = {e1r, e1i};
        xk1 = {e2r, e2i};
    }
    // this lane's rows: residuals and solution entries
    evrow rr, ri, xr, xi;
#pragma unroll
    for (int s = 0; s < EV_SLOTS; ++s) {
        const int row = lane + 64 * s;
        rr[s] = 0.0; ri[s] = 0.0;
        xr[s] = row == k ? xk.re : (pair && row == k + 1 ? xk1.re : 0.0);
        xi[s] = row == k ? xk.im : (pair && row == k + 1 ? xk1.im : 0.0);
        if (row < k) {
            const double t0 = T(row, k);
            rr[s] = -t0 * xk.re; ri[s] = -t0 * xk.im;
            if (pair) { const double t1 = T(row, k + 1); rr[s] -= t1 * xk1.re; ri[s] -= t1 * xk1.im; }
        }
    }
    int i = k - 1;
    while (i >= 0) {
        const bool two = bs[i] == 2;
        const int ia = two ? i - 1 : i;
        // residuals of rows ia, i from their owner lanes
        auto slot_val = [&](const evrow& v, int row) { return bcast(v[row >> 6], row & 63); };
        cplx x1, x0 = {0.0, 0.0};
        const cplx s1 = {slot_val(rr, i), slot_val(ri, i)};
        if (!two) {
            cplx d = {T(i, i) - lre, -lim};
            if (fabs(d.re) + fabs(d.im) < smin) d = {smin, 0.0};
            x1 = cdiv(s1, d);
        } else {
            const cplx s0 = {slot_val(rr, ia), slot_val(ri, ia)};
            // [[T(ia,ia)-lam, T(ia,i)], [T(i,ia), T(i,i)-lam]] [x_ia; x_i] = [s0; s1]
            const cplx a11 = {T(ia, ia) - lre, -lim}, a12 = {T(ia, i), 0.0};
            const cplx a21 = {T(i, ia), 0.0}, a22 = {T(i, i) - lre, -lim};
            cplx det = csub(cmul(a11, a22), cmul(a12, a21));
            if (fabs(det.re) + fabs(det.im) < smin * smin) det = {smin * smin, 0.0};
            x0 = cdiv(csub(cmul(s0, a22), cmul(a12, s1)), det);
            x1 = cdiv(csub(cmul(a11, s1), cmul(a21, s0)), det);
        }
        // guard against overflow: rescale x and r when the new entries grow large
        const double big = fmax(fabs(x1.re) + fabs(x1.im), fabs(x0.re) + fabs(x0.im));
        const double sc = big > 1e100 ? 1e-100 : 1.0;
        x1.re *= sc; x1.im *= sc; x0.re *= sc; x0.im *= sc;
#pragma unroll
        for (int s = 0; s < EV_SLOTS; ++s) {
            const int row = lane + 64 * s;
            rr[s] *= sc; ri[s] *= sc; xr[s] *= sc; xi[s] *= sc;
            if (row == i) { xr[s] = x1.re; xi[s] = x1.im; }
            if (two && row == ia) { xr[s] = x0.re; xi[s] = x0.im; }
            if (row < ia) {
                const double t1 = T(row, i);
                rr[s] -= t1 * x1.re; ri[s] -= t1 * x1.im;
                if (two) { const double t0 = T(row, ia); rr[s] -= t0 * x0.re; ri[s] -= t0 * x0.im; }
            }
        }
        i = ia - 1;
    }
    // normalise (complex 2-norm) and stage x for the product with Z
    double nn2 = 0.0;
#pragma unroll
    for (int s = 0; s < EV_SLOTS; ++s) nn2 += xr[s] * xr[s] + xi[s] * xi[s];
    nn2 = wave_sum(nn2);
    const double inv = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 0.0;
#pragma unroll
    for (int s = 0; s < EV_SLOTS; ++s) {
        const int row = lane + 64 * s;
        if (row < n) { xs[row] = xr[s] * inv; xs[n + row] = xi[s] * inv; }
    }
    __syncthreads();
    // W[:, k] = Z Re(x) (and W[:, k+1] = Z Im(x) for a pair); Z is column-major.  Columns
    // of Z are taken eight at a time, every row slot's entries loaded before the FMAs (each
    // sum still runs over j in ascending order)
    double wre[EV_SLOTS], wim[EV_SLOTS];
#pragma unroll
    for (int s = 0; s < EV_SLOTS; ++s) { wre[s] = 0.0; wim[s] = 0.0; }
    int j = 0;
    for (; j + 7 <= top; j += 8) {
        double z[8][EV_SLOTS];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int s = 0; s < EV_SLOTS; ++s) {
                const int row = lane + 64 * s;
                z[u][s] = row < n ? Zg[(int64_t)(j + u) * n + row] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double xre = xs[j + u], xim = xs[n + j + u];
#pragma unroll
            for (int s = 0; s < EV_SLOTS; ++s) { wre[s] += z[u][s] * xre; wim[s] += z[u][s] * xim; }
        }
    }
    for (; j <= top; ++j) {
        const double xre = xs[j], xim = xs[n + j];
#pragma unroll
        for (int s = 0; s < EV_SLOTS; ++s) {
            const int row = lane + 64 * s;
            const double z = row < n ? Zg[(int64_t)j * n + row] : 0.0;
            wre[s] += z * xre;
            wim[s] += z * xim;
        }
    }
#pragma unroll
    for (int s = 0; s < EV_SLOTS; ++s) {
        const int row = lane + 64 * s;
        if (row >= n) continue;
        Wraw[(int64_t)k * n + row] = wre[s];
        if (pair) Wraw[(int64_t)(k + 1) * n + row] = wim[s];
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
                      int32_t* kind, double* W, int32_t* info, double defl_tol)
{
    if (n <= 0) return hipSuccess;
    if (n > EIG_MAX) return hipErrorInvalidValue;
    EigWs w = eig_carve(ws, n);
    hipLaunchKernelGGL(hessenberg_kernel, dim3(1), dim3(1024), 0, s, A, lda, n, w.H, w.V, w.tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nr = eig_rows_per_wg(n);
    const int grid = eig_grid(n);
    const int hsize = hp_col(n, n);
    const int nw = FR_THREADS / 64;
    // blk ints, packed H, the Z slab, then the staged reflectors (FR_VCH columns and their tau)
    const size_t lds = (size_t)(round_up(n, 2) / 2) * 8 + (size_t)hsize * 8 + (size_t)nr * n * 8 +
                       (size_t)FR_VCH * (n + 1) * 8;
    if (lds > 160 * 1024 - 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL(francis_kernel, dim3(grid), dim3(64 * nw), lds, s, n, nr, w.H, w.V, w.tau, w.Z, w.T,
                       w.blk, w.wr, w.wi, w.kind0, info, defl_tol);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t evlds = ((size_t)round_up(hsize, 2) + 2 * (size_t)n) * 8 + (size_t)n * 4;
    hipLaunchKernelGGL(eigvec_kernel, dim3(n), dim3(64), evlds, s, n, w.T, w.blk, w.Z, w.Wraw, defl_tol);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_modes_kernel, dim3(1), dim3(SM_THREADS), (size_t)n * (2 * sizeof(double) + 2 * sizeof(int)),
                       s, n, w.wr, w.wi, w.kind0, w.Wraw, lam, kind, W);
    return hipGetLastError();
}

hipError_t eig_prepare()
{
    hipError_t e = hipFuncSetAttribute((const void*)eigvec_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024 - 256);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)francis_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
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
