// Small FP64 dense kernels of the fit (latency-bound, single or few work-groups).
//
//  chol_inv   Cholesky factor of a Gram matrix and the inverse of the factor, for
//             CholeskyQR (Q = Y R^-1).  One work-group; the factor lives packed in
//             LDS; the inverse is formed by 16x16 blocks (diagonal blocks first,
//             then one wave per block column).  Breakdown -> one retry with a
//             diagonal shift (shifted CholeskyQR), then a status code.
//  sym_eig    cyclic Jacobi eigen-decomposition of a symmetric matrix with a
//             round-robin parallel ordering.  Every work-group holds the whole
//             (packed) matrix in LDS and performs the same rotations; each one
//             owns a slice of rows of the eigenvector matrix, so rotating the
//             eigenvectors needs no communication between work-groups.
//  small_gemm, scale_cols, sigma_from_evals, conversions, amplitudes, check_finite.
#include "common.h"
#include "kernels.h"

namespace dmd {

// ====================================================================== Cholesky
__device__ __forceinline__ int64_t lp_idx(int i, int j, int n) {   // packed lower, i >= j
    return (int64_t)j * n - (int64_t)j * (j - 1) / 2 + (i - j);
}

__global__ void __launch_bounds__(1024)
chol_inv_kernel(const double* __restrict__ G, int64_t ldg, int n, double* Rinv, int64_t ldr,
                float* Rinv32, int64_t ldr32, double shift_scale, int32_t* shifted,
                int32_t* info, const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    extern __shared__ double L[];
    __shared__ int fail;
    __shared__ double shift;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;

    // R^-1 starts as zero (its strictly lower part stays zero)
    for (int64_t e = tid; e < (int64_t)n * n; e += nt) Rinv[(e / n) * ldr + (e % n)] = 0.0;

    int attempt = 0;
    for (;;) {
        if (tid == 0) {
            fail = 0;
            if (attempt == 1) {
                double tr = 0.0;
                for (int j = 0; j < n; ++j) tr += fabs(G[(int64_t)j * ldg + j]);
                shift = shift_scale * tr;
            } else {
                shift = 0.0;
            }
        }
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)n * n; e += nt) {
            const int i = (int)(e % n), j = (int)(e / n);
            if (i >= j) L[lp_idx(i, j, n)] = G[(int64_t)j * ldg + i] + (i == j ? shift : 0.0);
        }
        __syncthreads();
        for (int j = 0; j < n; ++j) {
            if (tid == 0) {
                const double d = L[lp_idx(j, j, n)];
                if (!(d > 0.0) || !isfinite(d)) fail = 1;
                else L[lp_idx(j, j, n)] = sqrt(d);
            }
            __syncthreads();
            if (fail) break;
            const double inv = 1.0 / L[lp_idx(j, j, n)];
            for (int i = j + 1 + tid; i < n; i += nt) L[lp_idx(i, j, n)] *= inv;
            __syncthreads();
            const int m = n - j - 1;
            for (int idx = tid; idx < m * m; idx += nt) {
                const int c = j + 1 + idx / m, i = j + 1 + idx % m;
                if (i >= c) L[lp_idx(i, c, n)] -= L[lp_idx(i, j, n)] * L[lp_idx(c, j, n)];
            }
            __syncthreads();
        }
        if (!fail) break;
        if (attempt == 0 && shift_scale > 0.0) {
            attempt = 1;
            if (tid == 0 && shifted) *shifted = 1;
            if (tid == 0 && info) atomicAdd(&info[3], 1);
            __syncthreads();
            continue;
        }
        // breakdown: report, and leave an identity so that later stages stay finite
        if (tid == 0) set_status(info, DMD_ERR_CHOL_BREAKDOWN);
        __syncthreads();
        for (int i = tid; i < n; i += nt) Rinv[(int64_t)i * ldr + i] = 1.0;
        __syncthreads();
        __threadfence_block();
        if (Rinv32)
            for (int64_t e = tid; e < (int64_t)n * n; e += nt)
                Rinv32[(e / n) * ldr32 + (e % n)] = (float)Rinv[(e / n) * ldr + (e % n)];
        return;
    }

    // ---- inverse of the lower factor L by 16 x 16 blocks; R^-1 = (L^-1)^T is stored:
    //      Linv(a, b) lives at Rinv[a * ldr + b]  (i.e. R^-1(b, a)).
    const int nb = (n + 15) / 16;
    // step 1: diagonal blocks, one wave per block, lane c < 16 computes column c
    if (wave < nb && lane < 16) {
        const int b0 = wave * 16, c = lane;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int gi = b0 + i;
            if (gi >= n || i < c || b0 + c >= n) { x[i] = 0.0; continue; }
            if (i == c) { x[i] = 1.0 / L[lp_idx(gi, gi, n)]; continue; }
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k)
                if (k >= c) s += L[lp_idx(gi, b0 + k, n)] * x[k];
            x[i] = -s / L[lp_idx(gi, gi, n)];
        }
        if (b0 + c < n) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (b0 + i < n) Rinv[(int64_t)(b0 + i) * ldr + (b0 + c)] = x[i];
        }
    }
    __syncthreads();
    __threadfence_block();
    // step 2: wave j computes block column j: Linv_ij = -Dinv_i * sum_{c=j}^{i-1} L_ic Linv_cj
    if (wave < nb) {
        const int j = wave;
        const int tj = lane & 15, tg = lane >> 4;       // entries (tg + 4q, tj), q = 0..3
        for (int i = j + 1; i < nb; ++i) {
            double T[4] = {0.0, 0.0, 0.0, 0.0};
            for (int c = j; c < i; ++c) {
                for (int k = 0; k < 16; ++k) {
                    const int col = 16 * c + k;
                    if (col >= n) break;
                    const double lv = (16 * j + tj < n) ? Rinv[(int64_t)col * ldr + 16 * j + tj] : 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int row = 16 * i + tg + 4 * q;
                        if (row < n) T[q] += L[lp_idx(row, col, n)] * lv;
                    }
                }
            }
            // gather column tj of T: T[k][tj] sits in lane tj + 16 * (k % 4), slot k / 4
            double Tc[16];
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int q = 0; q < 4; ++q) Tc[g + 4 * q] = __shfl(T[q], tj + 16 * g, 64);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ti = tg + 4 * q;
                const int row = 16 * i + ti;
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int kr = 16 * i + k;
                    if (kr < n && row < n) s += Rinv[(int64_t)row * ldr + kr] * Tc[k];
                }
                if (row < n && 16 * j + tj < n) Rinv[(int64_t)row * ldr + 16 * j + tj] = -s;
            }
            __threadfence_block();
        }
    }
    __syncthreads();
    __threadfence_block();
    if (Rinv32)
        for (int64_t e = tid; e < (int64_t)n * n; e += nt)
            Rinv32[(e / n) * ldr32 + (e % n)] = (float)Rinv[(e / n) * ldr + (e % n)];
}

hipError_t chol_inv(hipStream_t s, const double* G, int64_t ldg, int n, double* Rinv, int64_t ldr,
                    float* Rinv32, int64_t ldr32, double shift_scale, int32_t* shifted,
                    int32_t* info, const int32_t* skip_unless)
{
    if (n <= 0) return hipSuccess;
    if (n > SMALL_MAX) return hipErrorInvalidValue;
    const size_t lds = (size_t)n * (n + 1) / 2 * sizeof(double);
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), lds, s, G, ldg, n, Rinv, ldr, Rinv32,
                       ldr32, shift_scale, shifted, info, skip_unless);
    return hipGetLastError();
}

// ====================================================================== Jacobi
__device__ __forceinline__ int64_t up_idx(int i, int j) {   // packed upper, i <= j
    return (int64_t)j * (j + 1) / 2 + i;
}
__device__ __forceinline__ double sym_get(const double* A, int i, int j) {
    return i <= j ? A[up_idx(i, j)] : A[up_idx(j, i)];
}
__device__ __forceinline__ void sym_set(double* A, int i, int j, double v) {
    if (i <= j) A[up_idx(i, j)] = v; else A[up_idx(j, i)] = v;
}
// Round-robin (circle) schedule on n2 (even) players: in round t, pair k.
__device__ __forceinline__ void rr_pair(int k, int t, int n2, int* p, int* q) {
    const int m = n2 - 1;
    int a, b;
    if (k == 0) { a = 0; b = 1 + (t % m); }
    else { a = 1 + ((t + k) % m); b = 1 + ((t - k + m) % m); }
    *p = min(a, b);
    *q = max(a, b);
}

__global__ void __launch_bounds__(1024)
jacobi_kernel(const double* __restrict__ S, int64_t lds, int n, int nr, double* evals,
              double* Vout, int32_t* info)
{
    extern __shared__ double sm[];
    const int n2 = n + (n & 1);
    const int np = n2 / 2;
    double* A = sm;                                   // n(n+1)/2
    double* Vs = A + (int64_t)n * (n + 1) / 2;        // nr x n
    double* cs = Vs + (int64_t)nr * n;                // np
    double* sn = cs + np;                             // np
    double* tn = sn + np;                             // np
    int* pp = reinterpret_cast<int*>(tn + np);        // np
    int* qq = pp + np;                                // np
    int* rank = qq + np;                              // n
    __shared__ int rot_count;
    __shared__ double dmax_s;

    const int tid = threadIdx.x, nt = blockDim.x;
    const int r0 = blockIdx.x * nr;
    const int nrows = min(nr, n - r0);

    for (int64_t e = tid; e < (int64_t)n * n; e += nt) {
        const int i = (int)(e % n), j = (int)(e / n);
        if (i <= j) A[up_idx(i, j)] = S[(int64_t)j * lds + i];
    }
    for (int e = tid; e < nr * n; e += nt) {
        const int rl = e / n, c = e % n;
        Vs[e] = (rl < nrows && r0 + rl == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double d = 0.0;
        for (int i = 0; i < n; ++i) d = fmax(d, fabs(A[up_idx(i, i)]));
        dmax_s = d;
    }
    __syncthreads();
    const double floor_abs = 1e-17 * dmax_s;
    const int nblk = np * (np + 1) / 2;

    int sweep = 0;
    bool converged = false;
    for (; sweep < 40; ++sweep) {
        if (tid == 0) rot_count = 0;
        __syncthreads();
        for (int t = 0; t < n2 - 1; ++t) {
            for (int k = tid; k < np; k += nt) {
                int p, q;
                rr_pair(k, t, n2, &p, &q);
                double c = 1.0, s = 0.0, tt = 0.0;
                if (q < n) {
                    const double apq = A[up_idx(p, q)];
                    const double app = A[up_idx(p, p)], aqq = A[up_idx(q, q)];
                    if (fabs(apq) > floor_abs && fabs(apq) > 1e-15 * sqrt(fabs(app) * fabs(aqq))) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                        atomicAdd(&rot_count, 1);
                    }
                }
                pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s; tn[k] = tt;
            }
            __syncthreads();
            // 2x2 blocks of every pair of pairs: B' = J1^T B J2 (independent, disjoint entries)
            for (int bidx = tid; bidx < nblk; bidx += nt) {
                int k2 = (int)((sqrtf(8.0f * (float)bidx + 1.0f) - 1.0f) * 0.5f);
                while (k2 * (k2 + 1) / 2 > bidx) --k2;
                while ((k2 + 1) * (k2 + 2) / 2 <= bidx) ++k2;
                const int k1 = bidx - k2 * (k2 + 1) / 2;
                const int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
                if (q1 >= n || q2 >= n) {
                    // one pair involves the padding player: only its real index rotates
                    if (k1 == k2) continue;
                    const bool r1 = q1 < n, r2 = q2 < n;
                    if (!r1 && !r2) continue;
                    if (r1) {   // pair 1 real, pair 2 = (p2, pad): rotate column p2 against rows p1, q1
                        const double c1 = cs[k1], s1 = sn[k1];
                        const double x = sym_get(A, p1, p2), y = sym_get(A, q1, p2);
                        sym_set(A, p1, p2, c1 * x - s1 * y);
                        sym_set(A, q1, p2, s1 * x + c1 * y);
                    } else {
                        const double c2 = cs[k2], s2 = sn[k2];
                        const double x = sym_get(A, p1, p2), y = sym_get(A, p1, q2);
                        sym_set(A, p1, p2, c2 * x - s2 * y);
                        sym_set(A, p1, q2, s2 * x + c2 * y);
                    }
                    continue;
                }
                if (k1 == k2) {
                    const double t1 = tn[k1];
                    if (t1 == 0.0) continue;
                    const double apq = A[up_idx(p1, q1)];
                    A[up_idx(p1, p1)] -= t1 * apq;
                    A[up_idx(q1, q1)] += t1 * apq;
                    A[up_idx(p1, q1)] = 0.0;
                    continue;
                }
                const double c1 = cs[k1], s1 = sn[k1], c2 = cs[k2], s2 = sn[k2];
                const double b00 = sym_get(A, p1, p2), b01 = sym_get(A, p1, q2);
                const double b10 = sym_get(A, q1, p2), b11 = sym_get(A, q1, q2);
                const double x00 = c2 * b00 - s2 * b01, x01 = s2 * b00 + c2 * b01;
                const double x10 = c2 * b10 - s2 * b11, x11 = s2 * b10 + c2 * b11;
                sym_set(A, p1, p2, c1 * x00 - s1 * x10);
                sym_set(A, p1, q2, c1 * x01 - s1 * x11);
                sym_set(A, q1, p2, s1 * x00 + c1 * x10);
                sym_set(A, q1, q2, s1 * x01 + c1 * x11);
            }
            // eigenvector rows owned by this work-group: V <- V J
            for (int e = tid; e < nrows * np; e += nt) {
                const int rl = e / np, k = e % np;
                const int p = pp[k], q = qq[k];
                if (q >= n || tn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double vp = Vs[rl * n + p], vq = Vs[rl * n + q];
                Vs[rl * n + p] = c * vp - s * vq;
                Vs[rl * n + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
        if (rot_count == 0) { converged = true; break; }
        __syncthreads();
    }
    // order: descending eigenvalue, ties by index (NaN last)
    for (int i = tid; i < n; i += nt) {
        const double di = A[up_idx(i, i)];
        const double ki = isnan(di) ? -__builtin_inf() : di;
        int rk = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = A[up_idx(j, j)];
            const double kj = isnan(dj) ? -__builtin_inf() : dj;
            if (kj > ki || (kj == ki && j < i)) ++rk;
        }
        rank[i] = rk;
    }
    __syncthreads();
    for (int e = tid; e < nrows * n; e += nt) {
        const int rl = e / n, i = e % n;
        Vout[(int64_t)rank[i] * n + r0 + rl] = Vs[rl * n + i];
    }
    if (blockIdx.x == 0) {
        for (int i = tid; i < n; i += nt) evals[rank[i]] = A[up_idx(i, i)];
        if (tid == 0 && info) {
            info[1] += sweep + 1;
            if (!converged) set_status(info, DMD_ERR_EIG_NOCONV);
        }
    }
}

hipError_t sym_eig(hipStream_t s, const double* S, int64_t lds, int n, double* evals, double* Vout,
                   int32_t* info)
{
    if (n <= 0) return hipSuccess;
    if (n > SMALL_MAX) return hipErrorInvalidValue;
    const int n2 = n + (n & 1), np = n2 / 2;
    const size_t fixed = (size_t)n * (n + 1) / 2 * 8 + (size_t)np * (3 * 8 + 2 * 4) + (size_t)n * 4 + 64;
    const size_t budget = 160 * 1024 - 512;
    if (fixed + (size_t)n * 8 > budget) return hipErrorInvalidValue;
    int nr = (int)((budget - fixed) / ((size_t)n * 8));
    if (nr > 32) nr = 32;
    if (nr > n) nr = n;
    const int grid = (int)ceil_div(n, nr);
    const size_t lds_bytes = fixed + (size_t)nr * n * 8;
    hipLaunchKernelGGL(jacobi_kernel, dim3(grid), dim3(1024), lds_bytes, s, S, lds, n, nr, evals, Vout, info);
    return hipGetLastError();
}

// ====================================================================== helpers
__global__ void small_gemm_kernel(int ta, int tb, int m, int n, int k, double alpha,
                                  const double* __restrict__ A, int64_t lda,
                                  const double* __restrict__ B, int64_t ldb, double beta,
                                  double* __restrict__ C, int64_t ldc)
{
    const int64_t tot = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        double s = 0.0;
        for (int kk = 0; kk < k; ++kk) {
            const double a = ta ? A[(int64_t)i * lda + kk] : A[(int64_t)kk * lda + i];
            const double b = tb ? B[(int64_t)kk * ldb + j] : B[(int64_t)j * ldb + kk];
            s += a * b;
        }
        double* c = C + (int64_t)j * ldc + i;
        *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
    }
}

hipError_t small_gemm(hipStream_t s, int ta, int tb, int m, int n, int k, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                      double* C, int64_t ldc)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t tot = (int64_t)m * n;
    hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(tot, 128), 1024)), dim3(128), 0, s,
                       ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
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
                             int32_t* info)
{
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i < r) {
        const double v = sqrt(fmax(ev[i], 0.0));
        sigma[i] = v;
        if (sigma_out) sigma_out[i] = v;
    }
    if (i == 0) {
        const double s1 = sqrt(fmax(ev[0], 0.0)), sr = sqrt(fmax(ev[r - 1], 0.0));
        if (!(sr > 0.0) || (rank_tol > 0.0 && sr <= rank_tol * s1)) set_status(info, DMD_ERR_RANK);
    }
}

hipError_t sigma_from_evals(hipStream_t s, const double* evals, int r, double rank_tol, double* sigma,
                            double* sigma_out, int32_t* info)
{
    hipLaunchKernelGGL(sigma_kernel, dim3((unsigned)ceil_div(r, 256)), dim3(256), 0, s, evals, r, rank_tol,
                       sigma, sigma_out, info);
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
__global__ void copy_f64_kernel(int m, int n, int n_pad, const double* A, int64_t lda, double* B, int64_t ldb)
{
    const int64_t tot = (int64_t)m * n_pad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        B[(int64_t)j * ldb + i] = j < n ? A[(int64_t)j * lda + i] : 0.0;
    }
}

hipError_t to_f32(hipStream_t s, int m, int n, int n_pad, const double* A, int64_t lda, float* B, int64_t ldb)
{
    if (m <= 0 || n_pad <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)m * n_pad, 256), 1024)), dim3(256), 0, s,
                       m, n, n_pad, A, lda, B, ldb);
    return hipGetLastError();
}
hipError_t copy_f64(hipStream_t s, int m, int n, int n_pad, const double* A, int64_t lda, double* B, int64_t ldb)
{
    if (m <= 0 || n_pad <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)m * n_pad, 256), 1024)), dim3(256), 0, s,
                       m, n, n_pad, A, lda, B, ldb);
    return hipGetLastError();
}

// beta = R^-1 R^-T rhs  (the normal equations G beta = rhs with G = R^T R), then the
// complex amplitudes of the folded basis: a pair (i, i+1) contributes
// Re(phi) beta_i + Im(phi) beta_{i+1} = 2 Re(phi b_i) with b_i = (beta_i - i beta_{i+1}) / 2.
__global__ void amplitudes_kernel(int r, const double* __restrict__ Rinv, int64_t ldr,
                                  const double* __restrict__ rhs, const int32_t* __restrict__ kind,
                                  double* __restrict__ b)
{
    extern __shared__ double sh[];
    double* t = sh;          // r
    double* beta = sh + r;   // r
    const int tid = threadIdx.x;
    for (int i = tid; i < r; i += blockDim.x) {          // t = R^-T rhs
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += Rinv[(int64_t)i * ldr + j] * rhs[j];
        t[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < r; i += blockDim.x) {          // beta = R^-1 t
        double s = 0.0;
        for (int j = i; j < r; ++j) s += Rinv[(int64_t)j * ldr + i] * t[j];
        beta[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < r; i += blockDim.x) {
        int kd = kind[i];
        if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;
        if (kd == 0) { b[2 * i] = beta[i]; b[2 * i + 1] = 0.0; }
        else if (kd == 1) { b[2 * i] = 0.5 * beta[i]; b[2 * i + 1] = -0.5 * beta[i + 1]; }
        else { b[2 * i] = 0.5 * beta[i - 1]; b[2 * i + 1] = 0.5 * beta[i]; }
    }
}

hipError_t amplitudes(hipStream_t s, int r, const double* Rinv, int64_t ldr, const double* rhs,
                      const int32_t* kind, double* b)
{
    hipLaunchKernelGGL(amplitudes_kernel, dim3(1), dim3(256), 2 * r * sizeof(double), s, r, Rinv, ldr, rhs, kind, b);
    return hipGetLastError();
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
    hipError_t e = hipFuncSetAttribute((const void*)chol_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
}

}  // namespace dmd
