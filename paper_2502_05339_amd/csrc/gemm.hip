// Tall-skinny GEMMs of the fit on MFMA (gfx950).
//
//  gemm_nn : C (N x n) = A (N x k) B (k x n), A streamed, the small B staged in LDS.
//            Used for the sketch Y = X Omega and Y = X W (Sec. 4.3), the CholeskyQR
//            apply Q = Y R^-1, and the exact modes Phi = X' M (Sec. 3.1).
//  gemm_tn : P_s = A[rows_s]^T B[rows_s] over a split of the N rows, written as FP64
//            partials; reduce_partials sums them in a fixed order (deterministic).
//            Used for the Gram products of CholeskyQR (FP64 MFMA), X^T Q, the
//            projection Q^T Z (one pass over both X and X'), Phi^T Phi, Phi^T x0 and
//            the adjoint's Phi^T R.
#include "common.h"
#include "kernels.h"

namespace dmd {

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------------ NN
// Work-group: 256 threads = 4 waves stacked in rows; each wave owns 16*RB rows
// and all n (<= 16*NBW) columns; the work-group tile is 64*RB rows x n.  The k
// dimension is consumed in chunks of KC = 16, each staged through LDS (A as
// [k][row], B as [k][col]) so that MFMA operand reads are bank-conflict free.
template <typename T, int RB, int NBW, bool VEC>
__global__ void __launch_bounds__(256)
gemm_nn_kernel(const T* A, int64_t lda, const T* __restrict__ B, int64_t ldb,
               T* C, int64_t ldc, int c_rowmajor, int64_t N, int K, int n,
               const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    constexpr int KC = 16;
    constexpr int BM = 64 * RB;
    constexpr int PADA = (sizeof(T) == 4) ? 4 : 2;
    constexpr int NP = 16 * NBW;
    __shared__ T As[KC][BM + PADA];
    __shared__ T Bs[KC][NP + PADA];

    typedef typename Acc<T>::type V;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * BM;
    const int ncb = (n + 15) / 16;

    V acc[RB][NBW];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb) acc[rb][cb] = zero_acc<V>();

    for (int k0 = 0; k0 < K; k0 += KC) {
        // ---- stage A chunk: BM rows x KC columns (column-major in global)
        if constexpr (VEC) {
            constexpr int VW = 16 / sizeof(T);          // elements per 16-byte load
            constexpr int NV = BM / VW * KC;
            for (int idx = tid; idx < NV; idx += 256) {
                int i = (idx % (BM / VW)) * VW;
                int kk = idx / (BM / VW);
                int64_t row = row0 + i;
                int kcol = k0 + kk;
                const T* src = A + (int64_t)kcol * lda + row;
                if (kcol < K && row + VW <= N) {
                    if constexpr (sizeof(T) == 4) {
                        float4 v = *reinterpret_cast<const float4*>(src);
                        As[kk][i] = v.x; As[kk][i + 1] = v.y; As[kk][i + 2] = v.z; As[kk][i + 3] = v.w;
                    } else {
                        double2 v = *reinterpret_cast<const double2*>(src);
                        As[kk][i] = v.x; As[kk][i + 1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        As[kk][i + e] = (kcol < K && row + e < N) ? src[e] : T(0);
                }
            }
        } else {
            for (int idx = tid; idx < BM * KC; idx += 256) {
                int i = idx % BM, kk = idx / BM;
                int64_t row = row0 + i;
                int kcol = k0 + kk;
                As[kk][i] = (kcol < K && row < N) ? A[(int64_t)kcol * lda + row] : T(0);
            }
        }
        // ---- stage B chunk: KC x NP
        for (int idx = tid; idx < KC * NP; idx += 256) {
            int kk = idx % KC, j = idx / KC;
            int kr = k0 + kk;
            Bs[kk][j] = (kr < K && j < n) ? B[(int64_t)j * ldb + kr] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            T a[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) a[rb] = As[kk][wave * 16 * RB + rb * 16 + (lane & 15)];
#pragma unroll
            for (int cb = 0; cb < NBW; ++cb) {
                if (cb < ncb) {
                    T bv = Bs[kk][cb * 16 + (lane & 15)];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) acc[rb][cb] = mfma(a[rb], bv, acc[rb][cb]);
                }
            }
        }
        __syncthreads();
    }

    // ---- epilogue
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int64_t tile0 = row0 + wave * 16 * RB + rb * 16;
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb) {
            if (cb >= ncb) continue;
            const int col = cb * 16 + (lane & 15);
            if (col >= n) continue;
            if constexpr (sizeof(T) == 4) {
                const int64_t rbase = tile0 + 4 * (lane >> 4);     // 4 consecutive rows
                if (!c_rowmajor && VEC && rbase + 4 <= N) {
                    float4 o = make_float4(acc[rb][cb][0], acc[rb][cb][1], acc[rb][cb][2], acc[rb][cb][3]);
                    *reinterpret_cast<float4*>(C + (int64_t)col * ldc + rbase) = o;
                    continue;
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = tile0 + acc_row<V>(lane, v);
                if (row < N) {
                    if (c_rowmajor) C[row * ldc + col] = acc[rb][cb][v];
                    else C[(int64_t)col * ldc + row] = acc[rb][cb][v];
                }
            }
        }
    }
}

template <typename T, int RB, int NBW>
static hipError_t launch_nn_t(hipStream_t s, const T* A, int64_t lda, const T* B, int64_t ldb,
                              T* C, int64_t ldc, int c_rowmajor, int64_t N, int K, int n,
                              const int32_t* skip_unless)
{
    constexpr int BM = 64 * RB;
    dim3 grid((unsigned)ceil_div(N, BM));
    const int vw = 16 / sizeof(T);
    bool vec = (lda % vw == 0) && ((uintptr_t)A % 16 == 0) && (c_rowmajor || ((ldc % vw == 0) && ((uintptr_t)C % 16 == 0)));
    if (vec)
        hipLaunchKernelGGL((gemm_nn_kernel<T, RB, NBW, true>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, c_rowmajor, N, K, n, skip_unless);
    else
        hipLaunchKernelGGL((gemm_nn_kernel<T, RB, NBW, false>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, c_rowmajor, N, K, n, skip_unless);
    return hipGetLastError();
}

hipError_t gemm_nn(hipStream_t s, int dtype, const void* A, int64_t lda, const void* B, int64_t ldb,
                   void* C, int64_t ldc, int c_rowmajor, int64_t N, int K, int n,
                   const int32_t* skip_unless)
{
    if (N <= 0 || n <= 0) return hipSuccess;
    if (n > 16 * NN_MAX_CB) return hipErrorInvalidValue;
    if (dtype == DMD_F32) {
        const float* a = (const float*)A; const float* b = (const float*)B; float* c = (float*)C;
        if (n <= 64)  return launch_nn_t<float, 2, 4>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless);
        if (n <= 128) return launch_nn_t<float, 2, 8>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless);
        return launch_nn_t<float, 2, NN_MAX_CB>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless);
    } else {
        const double* a = (const double*)A; const double* b = (const double*)B; double* c = (double*)C;
        if (n <= 64)  return launch_nn_t<double, 1, 4>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless);
        if (n <= 128) return launch_nn_t<double, 1, 8>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless);
        return launch_nn_t<double, 1, NN_MAX_CB>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless);
    }
}

// ------------------------------------------------------------------------ TN
// Block b of the output, enumerated column-major over 16x16 blocks; in symmetric
// mode only the upper block triangle (bi <= bj) is enumerated.
__device__ __forceinline__ void block_decode(int b, int sym, int nbi, int* bi, int* bj) {
    if (!sym) { *bi = b % nbi; *bj = b / nbi; return; }
    int j = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
    while (j * (j + 1) / 2 > b) --j;
    while ((j + 1) * (j + 2) / 2 <= b) ++j;
    *bj = j;
    *bi = b - j * (j + 1) / 2;
}

// Work-group: 512 threads = 8 waves.  Rows are consumed in chunks of RC staged in
// LDS as [row][col]; the output's 16x16 blocks are dealt round-robin to the waves
// (each wave holds up to MAXB accumulators).  gridDim.x = row splits, gridDim.y =
// groups of 8*MAXB output blocks.
template <typename Tin, typename Tc, int RC, int MAXB>
__global__ void __launch_bounds__(512)
gemm_tn_kernel(const Tin* __restrict__ A, int64_t lda, int a_rowmajor, int ka,
               const Tin* __restrict__ B, int64_t ldb, int b_rowmajor, int nb,
               int sym, int64_t N, int64_t rows_per_split, double* __restrict__ P,
               const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Tc* smem = reinterpret_cast<Tc*>(smem_raw);
    typedef typename Acc<Tc>::type V;
    constexpr int PAD = (sizeof(Tc) == 4) ? 16 : 8;
    const int ka_p = (int)round_up(ka, 16), nb_p = (int)round_up(nb, 16);
    const int lda_s = ka_p + PAD, ldb_s = nb_p + PAD;
    Tc* As = smem;
    Tc* Bs = sym ? smem : smem + RC * lda_s;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform -> scalar registers
    const int nbi = ka_p / 16, nbj = nb_p / 16;
    // enumerate blocks: column-major over (bi, bj); symmetric keeps bi <= bj
    const int64_t split = blockIdx.x;
    const int64_t r_begin = split * rows_per_split;
    const int64_t r_end = min(N, r_begin + rows_per_split);

    const int nblocks = sym ? nbj * (nbj + 1) / 2 : nbi * nbj;
    const int first = blockIdx.y * 8 * MAXB;
    int aoff[MAXB], boff[MAXB];
    uint32_t valid = 0;
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        const int b = first + wave + 8 * t;
        int bi, bj;
        block_decode(b, sym, nbi, &bi, &bj);
        if (b < nblocks) valid |= 1u << t;
        aoff[t] = __builtin_amdgcn_readfirstlane(bi * 16);
        boff[t] = __builtin_amdgcn_readfirstlane(bj * 16);
    }
    V acc[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) acc[t] = zero_acc<V>();

    for (int64_t c0 = r_begin; c0 < r_end; c0 += RC) {
        // ---- stage A rows [c0, c0+RC) x ka_p
        if (a_rowmajor) {
            for (int idx = tid; idx < RC * ka_p; idx += 512) {
                int c = idx % ka_p, rr = idx / ka_p;
                int64_t row = c0 + rr;
                As[rr * lda_s + c] = (row < r_end && c < ka) ? (Tc)A[row * lda + c] : Tc(0);
            }
        } else {
            for (int idx = tid; idx < RC * ka_p; idx += 512) {
                int rr = idx % RC, c = idx / RC;
                int64_t row = c0 + rr;
                As[rr * lda_s + c] = (row < r_end && c < ka) ? (Tc)A[(int64_t)c * lda + row] : Tc(0);
            }
        }
        if (!sym) {
            if (b_rowmajor) {
                for (int idx = tid; idx < RC * nb_p; idx += 512) {
                    int c = idx % nb_p, rr = idx / nb_p;
                    int64_t row = c0 + rr;
                    Bs[rr * ldb_s + c] = (row < r_end && c < nb) ? (Tc)B[row * ldb + c] : Tc(0);
                }
            } else {
                for (int idx = tid; idx < RC * nb_p; idx += 512) {
                    int rr = idx % RC, c = idx / RC;
                    int64_t row = c0 + rr;
                    Bs[rr * ldb_s + c] = (row < r_end && c < nb) ? (Tc)B[(int64_t)c * ldb + row] : Tc(0);
                }
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int ks = 0; ks < RC / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            const Tc* arow = As + kk * lda_s + (lane & 15);
            const Tc* brow = Bs + kk * (sym ? lda_s : ldb_s) + (lane & 15);
#pragma unroll
            for (int t = 0; t < MAXB; ++t) {
                if (valid & (1u << t)) {
                    Tc av = arow[aoff[t]];
                    Tc bv = brow[boff[t]];
                    acc[t] = mfma(av, bv, acc[t]);
                }
            }
        }
        __syncthreads();
    }

    double* out = P + split * (int64_t)ka * nb;
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        if (valid & (1u << t)) {
            const int j = boff[t] + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = aoff[t] + acc_row<V>(lane, v);
                if (i < ka && j < nb) out[(int64_t)j * ka + i] = (double)acc[t][v];
            }
        }
    }
}

// out(i, j) = sum_s P_s(i, j), summed in split order.  In symmetric mode only the
// upper block triangle of P is valid and the rest is mirrored.
__global__ void reduce_partials_kernel(const double* __restrict__ P, int nsplit, int ka, int nb,
                                       int sym, double* out, int64_t ldo, float* out32,
                                       int64_t ldo32, const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    const int64_t tot = (int64_t)ka * nb;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(e % ka), j = (int)(e / ka);
        int si = i, sj = j;
        if (sym && (i / 16) > (j / 16)) { si = j; sj = i; }
        const double* p = P + (int64_t)sj * ka + si;
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += p[(int64_t)k * tot];
        if (out) out[(int64_t)j * ldo + i] = s;
        if (out32) out32[(int64_t)j * ldo32 + i] = (float)s;
    }
}

static int tn_splits(int64_t N, int rc) {
    int64_t s = N / (int64_t)(rc * 16);
    if (s < 1) s = 1;
    if (s > TN_MAX_SPLITS) s = TN_MAX_SPLITS;
    return (int)s;
}

hipError_t gemm_prepare()
{
    hipError_t e;
    e = hipFuncSetAttribute((const void*)gemm_tn_kernel<float, float, 32, 24>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)gemm_tn_kernel<float, double, 16, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)gemm_tn_kernel<double, double, 16, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

size_t gemm_tn_partial_bytes(int64_t N, int ka, int nb) {
    return (size_t)TN_MAX_SPLITS * (size_t)ka * (size_t)nb * sizeof(double);
}

template <typename Tin, typename Tc>
static hipError_t launch_tn_t(hipStream_t s, const Tin* A, int64_t lda, int a_rm, int ka,
                              const Tin* B, int64_t ldb, int b_rm, int nb, int sym, int64_t N,
                              double* P, int* nsplit_out, const int32_t* skip_unless)
{
    constexpr int RC = (sizeof(Tc) == 4) ? 32 : 16;
    constexpr int MAXB = (sizeof(Tc) == 4) ? 24 : 16;
    constexpr int PAD = (sizeof(Tc) == 4) ? 16 : 8;
    const int ka_p = (int)round_up(ka, 16), nb_p = (int)round_up(nb, 16);
    const int nbi = ka_p / 16, nbj = nb_p / 16;
    const int nblocks = sym ? nbj * (nbj + 1) / 2 : nbi * nbj;
    const int gy = (int)ceil_div(nblocks, 8 * MAXB);
    const int ns = tn_splits(N, RC);
    const int64_t rps = round_up(ceil_div(N, ns), RC);
    const int ns_eff = (int)ceil_div(N, rps);
    size_t lds = (size_t)RC * (ka_p + PAD) * sizeof(Tc);
    if (!sym) lds += (size_t)RC * (nb_p + PAD) * sizeof(Tc);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_tn_kernel<Tin, Tc, RC, MAXB>), dim3(ns_eff, gy), dim3(512), lds, s,
                       A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, rps, P, skip_unless);
    *nsplit_out = ns_eff;
    return hipGetLastError();
}

hipError_t gemm_tn(hipStream_t s, int in_dtype, int compute_dtype, const void* A, int64_t lda,
                   int a_rowmajor, int ka, const void* B, int64_t ldb, int b_rowmajor, int nb,
                   int sym, int64_t N, double* P, double* out, int64_t ldo, float* out32,
                   int64_t ldo32, const int32_t* skip_unless)
{
    if (ka <= 0 || nb <= 0) return hipSuccess;
    if ((int64_t)ka * nb > TN_MAX_OUT) return hipErrorInvalidValue;
    int ns = 1;
    hipError_t e;
    if (N <= 0) {
        // empty reduction: zero output
        hipLaunchKernelGGL(fill_f64_kernel, dim3(64), dim3(256), 0, s, P, (int64_t)ka * nb, 0.0);
        ns = 1;
        e = hipGetLastError();
    } else if (in_dtype == DMD_F32 && compute_dtype == DMD_F32) {
        e = launch_tn_t<float, float>(s, (const float*)A, lda, a_rowmajor, ka, (const float*)B, ldb, b_rowmajor, nb, sym, N, P, &ns, skip_unless);
    } else if (in_dtype == DMD_F32) {
        e = launch_tn_t<float, double>(s, (const float*)A, lda, a_rowmajor, ka, (const float*)B, ldb, b_rowmajor, nb, sym, N, P, &ns, skip_unless);
    } else {
        e = launch_tn_t<double, double>(s, (const double*)A, lda, a_rowmajor, ka, (const double*)B, ldb, b_rowmajor, nb, sym, N, P, &ns, skip_unless);
    }
    if (e != hipSuccess) return e;
    const int64_t tot = (int64_t)ka * nb;
    int blocks = (int)std::min<int64_t>(ceil_div(tot, 256), 1024);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(blocks), dim3(256), 0, s, P, ns, ka, nb, sym,
                       out, ldo, out32, ldo32, skip_unless);
    return hipGetLastError();
}

}  // namespace dmd
