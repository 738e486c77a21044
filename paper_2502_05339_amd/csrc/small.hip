// Small FP64 dense kernels of the fit (latency-bound, single or few work-groups).
//
//  chol_inv   Cholesky factor of a Gram matrix and the inverse of the factor, for
//             CholeskyQR (Q = Y R^-1).  One work-group; 16 x 16 blocks in LDS,
//             FP64 MFMA block updates, block column by block column.
//             Breakdown -> one retry with a diagonal shift (shifted CholeskyQR),
//             then a status code.
//  small_gemm, scale_cols, sigma_from_evals, conversions, amplitudes, check_finite.
#include "common.h"
#include "kernels.h"

namespace dmd {


// ====================================================================== Cholesky
// G = L L^T and X = L^-1 by 16 x 16 blocks in one work-group of 16 waves, every block in
// LDS (padded rows): the lower blocks of G (those below the diagonal overwritten by L and
// then by X), and the inverses S_p = L_pp^-1 of the diagonal blocks.  Cholesky, for each
// block column p:
//   D  one wave forms S_p = L_pp^-1 by a column sweep on [G_pp | I] held in its registers
//      (unscaled entries times 1/d, rows of S scaled by 1/sqrt(d)); L_pp itself is never
//      needed again (P uses S_p, the inverse uses S_p and the blocks below the diagonal);
//   P  L_ip = G_ip S_p^T (i > p), one wave per block, FP64 MFMA, in place;
//   U  G_ij -= L_ip L_jp^T (i >= j > p), FP64 MFMA; wave 0 takes block (p+1, p+1) alone
//      and runs D for p+1 right after it.
// Inverse, in place, block column j from the last to the first (the blocks right of j
// already hold X):  X_jj = S_j,  X_ij = -(sum_{k=j+1..i} X_ik L_kj) S_j  (i > j), computed
// into registers, written after a barrier.  R^-1 = L^-T = X^T.  Rows and columns past n
// are padded with the identity.
constexpr int CM_THREADS = 1024;
constexpr int CM_NW = CM_THREADS / 64;
constexpr int CM_T = (SMALL_MAX + 15) / 16;                  // block rows
constexpr int CM_LD = 17;                                    // padded row stride of LDS blocks
constexpr int CM_BLK = 16 * CM_LD;

__host__ __device__ __forceinline__ int cm_g(int I, int J) { return I * (I + 1) / 2 + J; }   // I >= J

// dynamic LDS of chol_inv_kernel for n
static size_t cm_lds_bytes(int n)
{
    const int T = (n + 15) / 16;
    return (size_t)(T * (T + 1) / 2 + T) * CM_BLK * sizeof(double);
}

// column sweep of one 16 x 16 diagonal block by one wave: Db (G'_pp) is read, Sb receives
// S = L_pp^-1.  The block and S live in registers (lane: row i = lane / 4, columns
// 4 (lane % 4) .. + 3); each round of two pivots takes the 2 x 2 pivot block by readlane
// and columns j, j + 1 and rows j, j + 1 of S by lane shuffles, so no round waits on
// LDS.  Returns false on a non-positive or
// non-finite pivot (tested once after the sweep: a branch per pivot costs more than the
// sweep's arithmetic on values that are then discarded).
__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ bool cm_diag(const double* Db, double* Sb, int lane)
{
    const int i = lane >> 2, q = lane & 3, c0 = q * 4;
    double dv[4], sv[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        dv[b] = Db[i * CM_LD + c0 + b];
        sv[b] = (i == c0 + b) ? 1.0 : 0.0;
    }
    bool bad = false;                                      // uniform; checked once after the sweep
    // two pivots (j, j + 1) per round: the 2 x 2 pivot block is factored from three
    // broadcast values, and each lane applies both eliminations to its entries at once, so
    // a round waits on one set of lane shuffles instead of two
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
        const int g = j >> 2;                              // lane column group of columns j, j + 1
        const double x0 = dv[j & 3], x1 = dv[(j & 3) + 1]; // columns j, j + 1 (in the lanes with q = g)
        const double d0 = readlane_f64(x0, (j << 2) | g);            // D(j, j)
        const double e = readlane_f64(x0, ((j + 1) << 2) | g);       // D(j + 1, j)
        const double f = readlane_f64(x1, ((j + 1) << 2) | g);       // D(j + 1, j + 1)
        const double a = __shfl(x0, (i << 2) | g, 64);               // D(i, j)
        const double bb = __shfl(x1, (i << 2) | g, 64);              // D(i, j + 1)
        double gc0[4], gc1[4], xr0[4], xr1[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gc0[b] = __shfl(x0, ((c0 + b) << 2) | g, 64);            // D(c0 + b, j)
            gc1[b] = __shfl(x1, ((c0 + b) << 2) | g, 64);            // D(c0 + b, j + 1)
            xr0[b] = __shfl(sv[b], (j << 2) | q, 64);                // S(j, c0 + b)
            xr1[b] = __shfl(sv[b], ((j + 1) << 2) | q, 64);          // S(j + 1, c0 + b)
        }
        const double s0 = rsqrt_nr(d0), inv0 = s0 * s0;
        const double l10 = e * inv0;
        const double d1 = f - l10 * e;                    // D(j + 1, j + 1) after pivot j
        const double s1 = rsqrt_nr(d1), inv1 = s1 * s1;
        bad = bad || !(d0 > 0.0) || !isfinite(d0) || !(d1 > 0.0) || !isfinite(d1);
        const double li0 = a * inv0;                       // row i's multipliers (used for i > j + 1)
        const double li1 = (bb - li0 * e) * inv1;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int c = c0 + b;
            const double sp = xr1[b] - l10 * xr0[b];      // S(j + 1, c) after pivot j
            const double dp = gc1[b] - (gc0[b] * inv0) * e;   // D(c, j + 1) after pivot j
            if (i > j + 1 && c > j + 1 && c <= i) dv[b] = (dv[b] - li0 * gc0[b]) - li1 * dp;
            if (i > j + 1 && c <= j + 1) sv[b] = (sv[b] - li0 * xr0[b]) - li1 * sp;
            if (i == j + 1 && c <= j + 1) sv[b] = sp * s1;
            if (i == j && c <= j) sv[b] = xr0[b] * s0;
        }
    }
    if (bad) return false;
#pragma unroll
    for (int b = 0; b < 4; ++b) Sb[i * CM_LD + c0 + b] = sv[b];
    return true;
}

// A operand of block M (row-major, padded) for k-group kk: M[l16][4 kk + lg]; its B
// operand: M[4 kk + lg][l16].  Accumulators hold rows acc_row(lane, v), column l16.
__device__ __forceinline__ double cm_a(const double* M, int kk, int l16, int lg) { return M[l16 * CM_LD + 4 * kk + lg]; }
__device__ __forceinline__ double cm_b(const double* M, int kk, int l16, int lg) { return M[(4 * kk + lg) * CM_LD + l16]; }

// attempt 0 factors G as given; when it breaks down and shift_scale > 0 it only sets
// *shifted (and the nnext run flags of the passes a shifted pass needs after it), and
// attempt 1 (launched right after, a no-op unless *shifted is set) factors
// G + shift_scale * trace(G) * I.  A breakdown without a further attempt reports
// DMD_ERR_CHOL_BREAKDOWN and leaves the identity.
__global__ void __launch_bounds__(CM_THREADS)
chol_inv_kernel(const double* __restrict__ G, int64_t ldg, int n, double* Rinv, int64_t ldr,
                float* Rinv32, int64_t ldr32, double shift_scale, int attempt, int32_t* shifted,
                int32_t* info, const int32_t* skip_unless, int32_t* run_next, int nnext)
{
    if (skip_unless && *skip_unless == 0) return;
    if (attempt == 1 && (!shifted || *shifted == 0)) return;
    extern __shared__ __align__(16) double cm_sm[];
    __shared__ double shift;
    __shared__ int sh_fail;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, lg = lane >> 4;
    const int T = (n + 15) / 16, NG = T * (T + 1) / 2;
    double* Gs = cm_sm;                     // NG blocks, block (I, J) at cm_g(I, J)
    double* Ss = cm_sm + NG * CM_BLK;       // T blocks
    auto gblk = [&](int I, int J) { return Gs + cm_g(I, J) * CM_BLK; };

    if (tid == 0) {
        double tr = 0.0;
        if (attempt == 1)
            for (int j = 0; j < n; ++j) tr += fabs(G[(int64_t)j * ldg + j]);
        shift = shift_scale * tr;
        sh_fail = 0;
    }
    __syncthreads();
    const double sh = shift;
    // lower blocks of G (the lower triangle only, also for both halves of a diagonal block)
    // one block per wave at a time (block index and its (I, J) uniform), four entries per lane
    for (int b = wave; b < NG; b += CM_NW) {
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= b) ++I;
        const int J = b - I * (I + 1) / 2;
        double xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = lane + 64 * u, r = e >> 4, c = e & 15;
            const int row = I * 16 + c, col = J * 16 + r;       // consecutive lanes: consecutive rows
            const int rlo = max(row, col), clo = min(row, col);
            xv[u] = (row < n && col < n) ? G[(int64_t)clo * ldg + rlo] + (row == col ? sh : 0.0)
                                         : (row == col ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = lane + 64 * u;
            Gs[b * CM_BLK + (e & 15) * CM_LD + (e >> 4)] = xv[u];
        }
    }
    __syncthreads();
    if (wave == 0 && !cm_diag(gblk(0, 0), Ss, lane) && lane == 0) sh_fail = 1;
    __syncthreads();

    for (int p = 0; p < T && !sh_fail; ++p) {
        const double* Sp = Ss + p * CM_BLK;
        // ---- P: L_ip = G_ip S_p^T, one wave per block, in place
        for (int I = p + 1 + wave; I < T; I += CM_NW) {
            double* M = gblk(I, p);
            doublex4 c = zero_acc<doublex4>();
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) c = mfma_f64(cm_a(M, kk, l16, lg), cm_a(Sp, kk, l16, lg), c);
#pragma unroll
            for (int v = 0; v < 4; ++v) M[acc_row<doublex4>(lane, v) * CM_LD + l16] = c[v];
        }
        __syncthreads();
        // ---- U: G_ij -= L_ip L_jp^T for i >= j > p; block (p+1, p+1) and D(p+1) on wave 0
        const int h = T - p - 1;                              // block rows below p
        const int nu = h * (h + 1) / 2;                       // blocks (i, j), i >= j > p
        for (int e = (wave == 0 ? 0 : wave); e < (wave == 0 ? min(nu, 1) : nu); e += (wave == 0 ? 1 : CM_NW - 1)) {
            // e -> (J, I): block columns J = p+1.. in turn, rows I = J..T-1 (e = 0 is (p+1, p+1))
            int J = p + 1, r = e;
            while (r >= T - J) { r -= T - J; ++J; }
            const int I = J + r;
            double* M = gblk(I, J);
            const double* La = gblk(I, p);
            const double* Lb = gblk(J, p);
            doublex4 c;
#pragma unroll
            for (int v = 0; v < 4; ++v) c[v] = M[acc_row<doublex4>(lane, v) * CM_LD + l16];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) c = mfma_f64(-cm_a(La, kk, l16, lg), cm_a(Lb, kk, l16, lg), c);
#pragma unroll
            for (int v = 0; v < 4; ++v) M[acc_row<doublex4>(lane, v) * CM_LD + l16] = c[v];
        }
        if (wave == 0 && p + 1 < T) {
            wave_sync_lds();
            if (!cm_diag(gblk(p + 1, p + 1), Ss + (p + 1) * CM_BLK, lane) && lane == 0) sh_fail = 1;
        }
        __syncthreads();
    }
    const bool fail = sh_fail != 0;
    if (fail && attempt == 0 && shift_scale > 0.0 && shifted) {
        if (tid == 0) {
            *shifted = 1;
            for (int j = 0; j < nnext; ++j) run_next[j] = 1;
            if (info) atomicAdd(&info[3], 1);
        }
        return;
    }
    if (fail) {
        // breakdown: report, and leave an identity so that later stages stay finite
        if (tid == 0) set_status(info, DMD_ERR_CHOL_BREAKDOWN);
        for (int e = tid; e < n * n; e += CM_THREADS) {
            const int i = e % n, j = e / n;
            const double v = i == j ? 1.0 : 0.0;
            Rinv[(int64_t)j * ldr + i] = v;
            if (Rinv32) Rinv32[(int64_t)j * ldr32 + i] = (float)v;
        }
        return;
    }
    // ---- X = L^-1 in place, block column j from the last to the first
    for (int j = T - 2; j >= 0; --j) {
        const int I = j + 1 + wave;                           // one block row per wave (T - 1 <= 16)
        doublex4 x = zero_acc<doublex4>();
        if (I < T) {
            // W^T = sum_k L_kj^T X_ik^T (X_ii = S_i), then X_ij = -W S_j
            // two independent accumulation chains (K - j odd / even), added at the end
            doublex4 wa = zero_acc<doublex4>(), wb = zero_acc<doublex4>();
            for (int K = j + 1; K <= I; K += 2) {
                const double* Lk = gblk(K, j);
                const double* Xk = K == I ? Ss + I * CM_BLK : gblk(I, K);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) wa = mfma_f64(cm_b(Lk, kk, l16, lg), cm_a(Xk, kk, l16, lg), wa);
                if (K + 1 <= I) {
                    const double* Lk1 = gblk(K + 1, j);
                    const double* Xk1 = K + 1 == I ? Ss + I * CM_BLK : gblk(I, K + 1);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) wb = mfma_f64(cm_b(Lk1, kk, l16, lg), cm_a(Xk1, kk, l16, lg), wb);
                }
            }
            doublex4 wt;
#pragma unroll
            for (int v = 0; v < 4; ++v) wt[v] = wa[v] + wb[v];
            const double* Sj = Ss + j * CM_BLK;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) x = mfma_f64(-wt[kk], cm_b(Sj, kk, l16, lg), x);
        }
        __syncthreads();                                       // every read of column j is done
        if (I < T) {
            double* M = gblk(I, j);
#pragma unroll
            for (int v = 0; v < 4; ++v) M[acc_row<doublex4>(lane, v) * CM_LD + l16] = x[v];
        }
        __syncthreads();
    }
    // R^-1(r, c) = X(c, r) for r <= c, zero below: one column per wave at a time
    for (int c = wave; c < n; c += CM_NW) {
        const int I = c >> 4;
        for (int r = lane; r < n; r += 64) {
            double v = 0.0;
            if (r <= c) {
                const int J = r >> 4;
                const double* M = I == J ? Ss + I * CM_BLK : gblk(I, J);
                v = M[(c & 15) * CM_LD + (r & 15)];
            }
            Rinv[(int64_t)c * ldr + r] = v;
            if (Rinv32) Rinv32[(int64_t)c * ldr32 + r] = (float)v;
        }
    }
}

hipError_t chol_inv(hipStream_t s, const double* G, int64_t ldg, int n, double* Rinv, int64_t ldr,
                    float* Rinv32, int64_t ldr32, double shift_scale, int32_t* shifted,
                    int32_t* info, const int32_t* skip_unless, int32_t* run_next, int nnext)
{
    if (n <= 0) return hipSuccess;
    if (nnext > 0 && !run_next) return hipErrorInvalidValue;
    if (n > SMALL_MAX) return hipErrorInvalidValue;
    static_assert(CM_T - 1 <= CM_NW, "chol_inv_kernel: one block row per wave in the inverse");
    const size_t lds = cm_lds_bytes(n);
    if (lds > 160 * 1024 - 1024) return hipErrorInvalidValue;
    const int attempts = (shift_scale > 0.0 && shifted) ? 2 : 1;
    for (int at = 0; at < attempts; ++at) {
        hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(CM_THREADS), lds, s, G, ldg, n, Rinv, ldr, Rinv32, ldr32,
                           shift_scale, at, shifted, info, skip_unless, run_next, nnext);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}


// ====================================================================== helpers
// C = alpha op(A) op(B) + beta C by 32 x 32 output tiles: 256 threads, each owning a 2 x 2
// block (rows 2 tx, 2 tx + 1, columns 2 ty, 2 ty + 1), over k in chunks of 32 staged in
// LDS as [k][row] and [k][column] panels (the transposes are taken while staging, with
// the contiguous index of either layout on consecutive threads).  Each k step is two
// 16-byte LDS reads and four FMAs; every output sums its products in ascending k.
constexpr int SG_T = 32;
constexpr int SG_KC = 32;
constexpr int SG_LD = SG_T + 2;   // 16-byte aligned rows
__global__ void __launch_bounds__(256)
small_gemm_kernel(int ta, int tb, int m, int n, int k, double alpha, const double* __restrict__ A, int64_t lda,
                  const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
                  const int32_t* __restrict__ run)
{
    if (run && *run == 0) return;
    __shared__ __align__(16) double As[SG_KC * SG_LD];
    __shared__ __align__(16) double Bs[SG_KC * SG_LD];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int i0 = blockIdx.x * SG_T, j0 = blockIdx.y * SG_T;
    double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
    // the next chunk's operands are loaded into registers while the current one is
    // multiplied (its memory latency overlaps the FMAs); every load reads an in-bounds
    // entry (clamped indices) and zero is selected outside the matrices
    constexpr int SG_U = SG_KC * SG_T / 256;
    double pa[SG_U], pb[SG_U];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < SG_U; ++u) {
            const int e = tid + 256 * u;
            int ii, qa, jj, qb;
            if (ta) { qa = e % SG_KC; ii = e / SG_KC; } else { ii = e % SG_T; qa = e / SG_T; }
            if (tb) { jj = e % SG_T; qb = e / SG_T; } else { qb = e % SG_KC; jj = e / SG_KC; }
            const int gi = i0 + ii, gka = k0 + qa, gj = j0 + jj, gkb = k0 + qb;
            const int ci = min(gi, m - 1), cka = min(gka, k - 1), cj = min(gj, n - 1), ckb = min(gkb, k - 1);
            const double a = ta ? A[(int64_t)ci * lda + cka] : A[(int64_t)cka * lda + ci];
            const double b = tb ? B[(int64_t)ckb * ldb + cj] : B[(int64_t)cj * ldb + ckb];
            pa[u] = (gi < m && gka < k) ? a : 0.0;
            pb[u] = (gj < n && gkb < k) ? b : 0.0;
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int u = 0; u < SG_U; ++u) {
            const int e = tid + 256 * u;
            int ii, qa, jj, qb;
            if (ta) { qa = e % SG_KC; ii = e / SG_KC; } else { ii = e % SG_T; qa = e / SG_T; }
            if (tb) { jj = e % SG_T; qb = e / SG_T; } else { qb = e % SG_KC; jj = e / SG_KC; }
            As[qa * SG_LD + ii] = pa[u];
            Bs[qb * SG_LD + jj] = pb[u];
        }
    };
    if (k > 0) fetch(0);
    for (int k0 = 0; k0 < k; k0 += SG_KC) {
        put();
        __syncthreads();
        if (k0 + SG_KC < k) fetch(k0 + SG_KC);
        const int kc = min(SG_KC, k - k0);
        for (int q = 0; q < kc; ++q) {
            const double2 a = *reinterpret_cast<const double2*>(As + q * SG_LD + 2 * tx);
            const double2 b = *reinterpret_cast<const double2*>(Bs + q * SG_LD + 2 * ty);
            c00 = fma(a.x, b.x, c00);
            c10 = fma(a.y, b.x, c10);
            c01 = fma(a.x, b.y, c01);
            c11 = fma(a.y, b.y, c11);
        }
        __syncthreads();
    }
    const int i = i0 + 2 * tx, j = j0 + 2 * ty;
    auto out = [&](int ii, int jj, double v) {
        if (ii < m && jj < n) {
            double* c = C + (int64_t)jj * ldc + ii;
            *c = alpha * v + (beta == 0.0 ? 0.0 : beta * *c);
        }
    };
    out(i, j, c00);
    out(i + 1, j, c10);
    out(i, j + 1, c01);
    out(i + 1, j + 1, c11);
}

hipError_t small_gemm(hipStream_t s, int ta, int tb, int m, int n, int k, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                      double* C, int64_t ldc, const int32_t* run)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)ceil_div(m, SG_T), (unsigned)ceil_div(n, SG_T));
    hipLaunchKernelGGL(small_gemm_kernel, grid, dim3(256), 0, s, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                       run);
    return hipGetLastError();
}

__global__ void scale_cols_kernel(int m, int n, double* A, int64_t lda, const double* d, int mode)
{
    const int64_t tot = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        A[(int64_t)j * lda + i] = mode ? A[(int64_t)j * lda + i] / d[j] : A[(int64_t)j * lda + i] * d[j];
    }
}

hipError_t scale_cols(hipStream_t s, int m, int n, double* A, int64_t lda, const double* d, int mode)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)m * n, 256), 1024)), dim3(256), 0, s,
                       m, n, A, lda, d, mode);
    return hipGetLastError();
}

__global__ void sigma_kernel(const double* ev, int r, double rank_tol, double* sigma, double* sigma_out,
                             int32_t* info, int squared)
{
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    auto sv = [&](double e) { return squared ? sqrt(fmax(e, 0.0)) : fmax(e, 0.0); };
    if (i < r) {
        const double v = sv(ev[i]);
        sigma[i] = v;
        if (sigma_out) sigma_out[i] = v;
    }
    if (i == 0) {
        const double s1 = sv(ev[0]), sr = sv(ev[r - 1]);
        if (!(sr > 0.0) || (rank_tol > 0.0 && sr <= rank_tol * s1)) set_status(info, DMD_ERR_RANK);
    }
}

hipError_t sigma_from_evals(hipStream_t s, const double* evals, int r, double rank_tol, double* sigma,
                            double* sigma_out, int32_t* info, int squared)
{
    hipLaunchKernelGGL(sigma_kernel, dim3((unsigned)ceil_div(r, 256)), dim3(256), 0, s, evals, r, rank_tol,
                       sigma, sigma_out, info, squared);
    return hipGetLastError();
}

// J = [[0, R], [R^T, 0]] (2n x 2n, column-major, ld 2n) from the n x n block R (ld ldr):
// its eigenvalues are +-sigma_i(R), with eigenvectors [u_i; v_i] / sqrt(2) for +sigma_i.
__global__ void jw_build_kernel(int n, const double* __restrict__ R, int64_t ldr, double* __restrict__ J)
{
    const int64_t m = 2 * (int64_t)n;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < m * m;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % m, j = idx / m;          // J(i, j)
        double v = 0.0;
        if (i < n && j >= n) v = R[(j - n) * ldr + i];                 // R(i, j - n)
        else if (i >= n && j < n) v = R[(i - n) * ldr + j];            // R^T(i - n, j) = R(j, i - n)
        J[idx] = v;
    }
}

hipError_t jw_build(hipStream_t s, int n, const double* R, int64_t ldr, double* J)
{
    const int64_t tot = 4 * (int64_t)n * n;
    hipLaunchKernelGGL(jw_build_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(tot, 256), 1024)), dim3(256), 0, s,
                       n, R, ldr, J);
    return hipGetLastError();
}

__global__ void to_f32_kernel(int m, int n, int n_pad, const double* A, int64_t lda, float* B, int64_t ldb)
{
    const int64_t tot = (int64_t)m * n_pad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        B[(int64_t)j * ldb + i] = j < n ? (float)A[(int64_t)j * lda + i] : 0.0f;
    }
}
__global__ void copy_f64_kernel(int m, int n, int n_pad, const double* A, int64_t lda, double* B, int64_t ldb,
                                double scale, const int32_t* run)
{
    if (run && *run == 0) return;
    const int64_t tot = (int64_t)m * n_pad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        B[(int64_t)j * ldb + i] = j < n ? scale * A[(int64_t)j * lda + i] : 0.0;
    }
}

hipError_t to_f32(hipStream_t s, int m, int n, int n_pad, const double* A, int64_t lda, float* B, int64_t ldb)
{
    if (m <= 0 || n_pad <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)m * n_pad, 256), 1024)), dim3(256), 0, s,
                       m, n, n_pad, A, lda, B, ldb);
    return hipGetLastError();
}
hipError_t copy_f64(hipStream_t s, int m, int n, int n_pad, const double* A, int64_t lda, double* B, int64_t ldb,
                    double scale, const int32_t* run)
{
    if (m <= 0 || n_pad <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)m * n_pad, 256), 1024)), dim3(256), 0, s,
                       m, n, n_pad, A, lda, B, ldb, scale, run);
    return hipGetLastError();
}

// beta (+)= R^-1 R^-T rhs  (the normal equations G beta = rhs with G = R^T R)
// beta = R^-1 R^-T rhs (R^-1 upper triangular, column-major): t = R^-T rhs, then
// beta = R^-1 t, one wave per row (rows w, w + 16, ...), lanes over the row's terms and a
// fixed-shape wave sum; t is kept in LDS.
constexpr int NS_THREADS = 1024;
__global__ void __launch_bounds__(NS_THREADS)
normal_solve_kernel(int r, const double* __restrict__ Rinv, int64_t ldr, const double* __restrict__ rhs,
                    double* __restrict__ beta, int accumulate, const int32_t* __restrict__ run)
{
    if (run && *run == 0) return;
    extern __shared__ double sh[];
    double* x = sh;          // rhs (r)
    double* t = sh + r;      // R^-T rhs (r)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = NS_THREADS / 64;
    for (int i = tid; i < r; i += NS_THREADS) x[i] = rhs[i];
    __syncthreads();
    for (int i = wave; i < r; i += nw) {                 // t_i = sum_{j <= i} R^-1(j, i) rhs_j
        const double* col = Rinv + (int64_t)i * ldr;
        double s = 0.0;
        for (int j = lane; j <= i; j += 64) s = fma(col[j], x[j], s);
        s = wave_sum(s);
        if (lane == 0) t[i] = s;
    }
    __syncthreads();
    for (int i = wave; i < r; i += nw) {                 // beta_i = sum_{j >= i} R^-1(i, j) t_j
        double s = 0.0;
        for (int j = i + lane; j < r; j += 64) s = fma(Rinv[(int64_t)j * ldr + i], t[j], s);
        s = wave_sum(s);
        if (lane == 0) beta[i] = accumulate ? beta[i] + s : s;
    }
}

// Complex amplitudes of the folded basis from the real coefficients beta: a pair
// (i, i+1) contributes Re(phi) beta_i + Im(phi) beta_{i+1} = 2 Re(phi b_i) with
// b_i = (beta_i - i beta_{i+1}) / 2 and b_{i+1} = conj(b_i).
__global__ void beta_to_b_kernel(int r, const double* __restrict__ beta, const int32_t* __restrict__ kind,
                                 double* __restrict__ b)
{
    for (int i = threadIdx.x; i < r; i += blockDim.x) {
        int kd = kind[i];
        if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;
        if (kd == 0) { b[2 * i] = beta[i]; b[2 * i + 1] = 0.0; }
        else if (kd == 1) { b[2 * i] = 0.5 * beta[i]; b[2 * i + 1] = -0.5 * beta[i + 1]; }
        else { b[2 * i] = 0.5 * beta[i - 1]; b[2 * i + 1] = 0.5 * beta[i]; }
    }
}

// res = x - Phi beta  (Phi row-major N x r with leading dimension ldphi), FP64 sums
template <typename T>
__global__ void residual_kernel(int64_t N, int r, const T* __restrict__ phi, int64_t ldphi,
                                const double* __restrict__ beta, const T* __restrict__ x, T* __restrict__ res)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const T* row = phi + i * ldphi;
        double s = 0.0;
        for (int c = 0; c < r; ++c) s += (double)row[c] * beta[c];
        res[i] = (T)((double)x[i] - s);
    }
}

hipError_t normal_solve(hipStream_t s, int r, const double* Rinv, int64_t ldr, const double* rhs, double* beta,
                        int accumulate, const int32_t* run)
{
    hipLaunchKernelGGL(normal_solve_kernel, dim3(1), dim3(NS_THREADS), 2 * r * sizeof(double), s, r, Rinv, ldr, rhs,
                       beta, accumulate, run);
    return hipGetLastError();
}

hipError_t beta_to_b(hipStream_t s, int r, const double* beta, const int32_t* kind, double* b)
{
    hipLaunchKernelGGL(beta_to_b_kernel, dim3(1), dim3(256), 0, s, r, beta, kind, b);
    return hipGetLastError();
}

hipError_t residual(hipStream_t s, int dtype, int64_t N, int r, const void* phi, int64_t ldphi, const double* beta,
                    const void* x, void* res)
{
    const int blocks = (int)std::min<int64_t>(ceil_div(N, 256), 2048);
    if (dtype == DMD_F32)
        hipLaunchKernelGGL(residual_kernel<float>, dim3(blocks), dim3(256), 0, s, N, r, (const float*)phi, ldphi,
                           beta, (const float*)x, (float*)res);
    else
        hipLaunchKernelGGL(residual_kernel<double>, dim3(blocks), dim3(256), 0, s, N, r, (const double*)phi, ldphi,
                           beta, (const double*)x, (double*)res);
    return hipGetLastError();
}

// project / amplitudes helper used outside the fit: beta = G^-1 rhs then complex b
hipError_t amplitudes(hipStream_t s, int r, const double* Rinv, int64_t ldr, const double* rhs,
                      const int32_t* kind, double* b, double* beta_ws)
{
    hipError_t e = normal_solve(s, r, Rinv, ldr, rhs, beta_ws, 0);
    if (e != hipSuccess) return e;
    return beta_to_b(s, r, beta_ws, kind, b);
}

template <typename T>
__global__ void check_finite_kernel(const T* __restrict__ X, int64_t ld, int64_t N, int ncols, int32_t* info)
{
    int bad = 0;
    const int64_t tot = N * ncols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % N, j = e / N;
        if (!isfinite((double)X[j * ld + i])) bad = 1;
    }
    if (bad) set_status(info, DMD_ERR_NONFINITE);
}

hipError_t check_finite(hipStream_t s, int dtype, const void* X, int64_t ld, int64_t N, int ncols, int32_t* info)
{
    if (N <= 0 || ncols <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(ceil_div(N * ncols, 256), 4096);
    if (dtype == DMD_F32)
        hipLaunchKernelGGL(check_finite_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)X, ld, N, ncols, info);
    else
        hipLaunchKernelGGL(check_finite_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)X, ld, N, ncols, info);
    return hipGetLastError();
}

hipError_t small_prepare()
{
    return hipFuncSetAttribute((const void*)chol_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024 - 1024);
}

}  // namespace dmd
