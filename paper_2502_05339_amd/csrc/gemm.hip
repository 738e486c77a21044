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
#include <algorithm>
#include <type_traits>

#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

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
// Work-group: 256 threads = 4 waves; the waves form (4 / CS) row groups x CS column
// groups.  Each wave owns WR = 16*VW consecutive rows (VW = 16 / sizeof(T): 4 FP32 or
// 2 FP64 rows per 16-byte load) and NB / CS of the 16-column blocks, so that its
// accumulators leave room for several waves per SIMD (the A operand streams from
// memory; other waves cover its latency).  The A operand comes straight from memory: in
// k-step s, lane l loads the VW consecutive rows r0 + VW*(l%16) .. of column
// k0 + 4s + l/16 with one vector load, and element e of that vector is lane l's A
// operand of MFMA row-block e.  Row-block e of a wave therefore holds the rows
// {r0 + VW*i + e}, i = 0..15: a permutation of the wave's rows that the epilogue undoes,
// since it puts VW consecutive rows of one column in one lane again (vector stores of
// C).  B is staged through LDS in chunks of KB rows as [k][col], two buffers: chunk c+1
// (B and the A operands) is fetched into registers while chunk c feeds the MFMAs, one
// barrier per chunk.  C may alias A (every wave reads all of its rows of A before any
// wave writes them: the last chunk's reads precede the final barrier), which the
// in-place CholeskyQR apply Q = Y R^-1 relies on.  Column block b belongs to column group
// b % CS, so with an upper-triangular B (b_upper: B(k, j) = 0 for k > j, as R^-1), where
// block b takes only the chunks c <= b, the groups get nearly equal MFMA work and skip the
// rest (about 45% of the products at n = 160).
template <typename T, int NB, int CS, bool VEC>
__global__ void __launch_bounds__(256)
gemm_nn_kernel(const T* A, int64_t lda, const T* __restrict__ B, int64_t ldb,
               T* C, int64_t ldc, int c_rowmajor, int64_t N, int K, int n,
               const int32_t* skip_unless, int b_upper)
{
    if (skip_unless && *skip_unless == 0) return;
    constexpr int VW = 16 / sizeof(T);
    constexpr int WR = 16 * VW;
    constexpr int KB = 16;
    constexpr int NP = 16 * NB;
    constexpr int NBW = NB / CS;                 // column blocks per wave
    constexpr int RG = 4 / CS;                   // row groups per work-group
    static_assert(NB % CS == 0 && 4 % CS == 0, "column split must divide the blocks and the waves");
    constexpr int PADB = (sizeof(T) == 4) ? 4 : 2;
    constexpr int BPT = (KB * NP + 255) / 256;   // staged B elements per thread and chunk
    constexpr int NKS = KB / 4;                  // k-steps per chunk
    __shared__ T Bs[2][KB][NP + PADB];
    typedef typename Acc<T>::type V;
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type VT;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int kq = lane >> 4;
    const int cg = wave % CS;                    // column group
    const int64_t r0 = ((int64_t)blockIdx.x * RG + wave / CS) * WR;
    const int64_t rl = r0 + VW * (lane & 15);

    V acc[VW][NBW];
#pragma unroll
    for (int e = 0; e < VW; ++e)
#pragma unroll
        for (int cb = 0; cb < NBW; ++cb) acc[e][cb] = zero_acc<V>();

    // Software pipeline: while chunk c feeds the MFMAs, chunk c+1's B (to the other LDS
    // buffer after the MFMAs) and its A operands (registers) are in flight.
    T bpre[BPT];
    VT apre[NKS], acur[NKS];
    auto fetch_b = [&](int k0) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int idx = tid + q * 256;
            const int kk = idx % KB, j = idx / KB;
            const int kr = k0 + kk;
            bpre[q] = (idx < KB * NP && kr < K && j < n) ? B[(int64_t)j * ldb + kr] : T(0);
        }
    };
    auto put_b = [&](int buf) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int idx = tid + q * 256;
            if (idx < KB * NP) Bs[buf][idx % KB][idx / KB] = bpre[q];
        }
    };
    // VEC (N a multiple of VW): one unguarded load per k-step from an address clamped into
    // the matrix, so the loads of a chunk are all in flight together; operands of columns
    // past K or rows past N are zeroed when the chunk is consumed (take_a), after the wait
    // that precedes it anyway.  A guard per load would make each wait for the one before.
    auto fetch_a = [&](int k0) {
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            const int k = k0 + 4 * ks + kq;
            if constexpr (VEC) {
                apre[ks] = *reinterpret_cast<const VT*>(A + (int64_t)min(k, K - 1) * lda + min(rl, N - VW));
            } else {
                const T* src = A + (int64_t)k * lda + rl;
                VT v;
                T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
                for (int e = 0; e < VW; ++e) pv[e] = (k < K && rl + e < N) ? src[e] : T(0);
                apre[ks] = v;
            }
        }
    };
    auto take_a = [&](int k0) {
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            acur[ks] = apre[ks];
            if constexpr (VEC) {
                const bool valid = k0 + 4 * ks + kq < K && rl < N;
                T* pv = reinterpret_cast<T*>(&acur[ks]);
#pragma unroll
                for (int e = 0; e < VW; ++e) pv[e] = valid ? pv[e] : T(0);
            }
        }
    };

    const int nchunk = (K + KB - 1) / KB;
    fetch_b(0);
    fetch_a(0);
    put_b(0);
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        const bool more = c + 1 < nchunk;
        take_a(c * KB);
        if (more) { fetch_b((c + 1) * KB); fetch_a((c + 1) * KB); }
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            const T* av = reinterpret_cast<const T*>(&acur[ks]);
            T bv[NBW];
#pragma unroll
            for (int cb = 0; cb < NBW; ++cb) bv[cb] = Bs[buf][4 * ks + kq][(cb * CS + cg) * 16 + (lane & 15)];
#pragma unroll
            for (int e = 0; e < VW; ++e)
#pragma unroll
                for (int cb = 0; cb < NBW; ++cb)
                    if (!b_upper || c <= cb * CS + cg) acc[e][cb] = mfma(av[e], bv[cb], acc[e][cb]);
        }
        if (more) put_b(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogue: row-block e, tile row i  ->  row r0 + VW*i + e
#pragma unroll
    for (int cb = 0; cb < NBW; ++cb) {
        const int col = (cb * CS + cg) * 16 + (lane & 15);
        if (col >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + VW * acc_row<V>(lane, v);
            if (!c_rowmajor && VEC && row + VW <= N) {
                VT o;
                if constexpr (VW == 4) { o.x = acc[0][cb][v]; o.y = acc[1][cb][v]; o.z = acc[2][cb][v]; o.w = acc[3][cb][v]; }
                else { o.x = acc[0][cb][v]; o.y = acc[1][cb][v]; }
                *reinterpret_cast<VT*>(C + (int64_t)col * ldc + row) = o;
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    if (row + e < N) {
                        if (c_rowmajor) C[(row + e) * ldc + col] = acc[e][cb][v];
                        else C[(int64_t)col * ldc + row + e] = acc[e][cb][v];
                    }
                }
            }
        }
    }
}

template <typename T, int NB, int CS>
static hipError_t launch_nn_t(hipStream_t s, const T* A, int64_t lda, const T* B, int64_t ldb,
                              T* C, int64_t ldc, int c_rowmajor, int64_t N, int K, int n,
                              const int32_t* skip_unless, int b_upper)
{
    constexpr int BM = (4 / CS) * 16 * (16 / sizeof(T));
    dim3 grid((unsigned)ceil_div(N, BM));
    const int vw = 16 / sizeof(T);
    bool vec = (lda % vw == 0) && ((uintptr_t)A % 16 == 0) && N % vw == 0 &&
               (c_rowmajor || ((ldc % vw == 0) && ((uintptr_t)C % 16 == 0)));
    if (vec)
        hipLaunchKernelGGL((gemm_nn_kernel<T, NB, CS, true>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, c_rowmajor, N, K, n, skip_unless,
                           b_upper);
    else
        hipLaunchKernelGGL((gemm_nn_kernel<T, NB, CS, false>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, c_rowmajor, N, K, n, skip_unless,
                           b_upper);
    return hipGetLastError();
}

// Column blocks NB >= 4 are split over two waves (CS = 2).
template <typename T>
static hipError_t launch_nn_any(hipStream_t s, const T* a, int64_t lda, const T* b, int64_t ldb, T* c, int64_t ldc,
                                int c_rowmajor, int64_t N, int K, int n, const int32_t* skip_unless, int b_upper)
{
    const int ncb = (n + 15) / 16;
    if (ncb <= 2)  return launch_nn_t<T, 2, 1>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless, b_upper);
    if (ncb <= 4)  return launch_nn_t<T, 4, 2>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless, b_upper);
    if (ncb <= 6)  return launch_nn_t<T, 6, 2>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless, b_upper);
    if (ncb <= 8)  return launch_nn_t<T, 8, 2>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless, b_upper);
    if (ncb <= 10) return launch_nn_t<T, 10, 2>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless, b_upper);
    return launch_nn_t<T, NN_MAX_CB, 2>(s, a, lda, b, ldb, c, ldc, c_rowmajor, N, K, n, skip_unless, b_upper);
}

hipError_t gemm_nn(hipStream_t s, int dtype, const void* A, int64_t lda, const void* B, int64_t ldb,
                   void* C, int64_t ldc, int c_rowmajor, int64_t N, int K, int n,
                   const int32_t* skip_unless, int b_upper)
{
    if (N <= 0 || n <= 0) return hipSuccess;
    if (n > 16 * NN_MAX_CB) return hipErrorInvalidValue;
    if (dtype == DMD_F32)
        return launch_nn_any<float>(s, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc, c_rowmajor, N, K, n,
                                    skip_unless, b_upper);
    return launch_nn_any<double>(s, (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc, c_rowmajor, N, K, n,
                                 skip_unless, b_upper);
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

// Work-group: 512 threads = 8 waves.  Rows are consumed in chunks of RC, staged in
// LDS as [row][col] (so each MFMA operand read is 16 consecutive columns of one row)
// in the input type (FP32 inputs of an FP64-summed product are widened as each
// fragment is read, which is exact and keeps the LDS footprint of the FP32 products)
// with two buffers: the next chunk is fetched from memory into registers with 16-byte
// loads while the current one feeds the MFMAs, then written to the other buffer, one
// barrier per chunk.  Output tiling: the 16x16 blocks of C form an nbi x nbj grid; a
// work-group (blockIdx.y) takes a 2RI x 4RJ tile of it and each of its 8 waves a
// RI x RJ piece, so a row step of a wave reads RI + RJ operand fragments for RI*RJ
// MFMAs.
// Blocks past the grid edge are clamped onto the last block (recomputed, not stored),
// which keeps the MFMA loop free of branches.  A symmetric product (B = A) stages A
// only and computes the full square.  gridDim.x = row splits.
constexpr int TN_THREADS = 512;
constexpr int TN_MAXT = 4;     // staged 16-byte vectors per thread and chunk

__host__ __device__ constexpr int tn_ld(int ncol_p, int esz) {
    // row stride of a staged chunk: 16 elements past a multiple of 64 (FP32) or 32
    // (FP64) so that the four k-rows of one operand read fall in different banks
    return esz == 4 ? ((ncol_p + 63) / 64) * 64 + 16 : ((ncol_p + 31) / 32) * 32 + 16;
}

// One staging task moves VWI consecutive elements of one operand: VWI rows of a
// column (column-major operand) or VWI columns of a row (row-major operand).  The
// tasks of a thread are the same for every chunk, so they are decoded once; each keeps
// one running pointer into the next chunk to fetch, advanced after every fetch (one
// pointer per task for both the whole-chunk and the ragged-chunk loop).
template <typename Tin, typename Tc>
struct TnStage {
    static constexpr int VWI = 16 / sizeof(Tin);
    typedef typename std::conditional<sizeof(Tin) == 4, float4, double2>::type VT;
    __host__ __device__ static int ntasks(int rowmajor, int ncol, int ncol_p, int rc) {
        return rowmajor ? rc * (ncol_p / VWI) : ncol * (rc / VWI);
    }
    const Tin* p;       // first element of the task in the next chunk to fetch
    int64_t adv;        // elements from one chunk to the next (rc, or rc ld if row-major)
    int soff;           // LDS element offset of the first element (buffer-relative)
    int sstride;        // LDS stride between the VWI elements
    int roff;           // row of the task inside the chunk (first of VWI rows if column-major)
    int rowmajor;       // 0 / 1
    int cvalid;         // row-major: number of the VWI columns that exist (guard of the scalar path)
    __device__ void init(const Tin* X, int64_t ld, int rm, int ncol, int ncol_p, int rc, int t, int ldsld, int base) {
        rowmajor = rm;
        if (rm) {
            const int per = ncol_p / VWI;
            const int rr = t / per, cq = t % per;
            p = X + (int64_t)rr * ld + VWI * cq;
            adv = (int64_t)rc * ld;
            soff = base + rr * ldsld + VWI * cq;
            sstride = 1;
            roff = rr;
            cvalid = min(VWI, max(0, ncol - VWI * cq));
        } else {
            const int per = rc / VWI;
            const int c = t / per, q = t % per;
            p = X + (int64_t)c * ld + VWI * q;
            adv = rc;
            soff = base + VWI * q * ldsld + c;
            sstride = ldsld;
            roff = VWI * q;
            cvalid = VWI;
        }
    }
    // c0: offset of the chunk at p inside the split (for the row guards)
    __device__ VT load(int64_t c0, int64_t r_end, int vec) const {
        VT v;
        Tin* pv = reinterpret_cast<Tin*>(&v);
        const int64_t row = c0 + roff;
        if (rowmajor) {
            if (vec && row < r_end) v = *reinterpret_cast<const VT*>(p);
            else {
#pragma unroll
                for (int e = 0; e < VWI; ++e) pv[e] = (row < r_end && e < cvalid) ? p[e] : Tin(0);
            }
        } else {
            if (vec && row + VWI <= r_end) v = *reinterpret_cast<const VT*>(p);
            else {
#pragma unroll
                for (int e = 0; e < VWI; ++e) pv[e] = (row + e < r_end) ? p[e] : Tin(0);
            }
        }
        return v;
    }
    // every row of the chunk exists and the operand allows 16-byte loads: one load (the
    // columns past the last of a row-major operand are cleared by store)
    __device__ VT load_full() const { return *reinterpret_cast<const VT*>(p); }
    __device__ void next() { p += adv; }
    __device__ void store(Tin* buf, const VT& v) const {
        const Tin* pv = reinterpret_cast<const Tin*>(&v);
#pragma unroll
        for (int e = 0; e < VWI; ++e) buf[soff + e * sstride] = e < cvalid ? pv[e] : Tin(0);
    }
};

template <typename Tin, typename Tc, int RC, int RI, int RJ, int WI>
__global__ void __launch_bounds__(256 * WI)
gemm_tn_kernel(const Tin* __restrict__ A, int64_t lda, int a_rowmajor, int ka,
               const Tin* __restrict__ B, int64_t ldb, int b_rowmajor, int nb,
               int sym, int64_t N, int64_t rows_per_split, int vec, double* __restrict__ P,
               const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    typedef TnStage<Tin, Tc> St;
    typedef typename St::VT VT;
    typedef typename Acc<Tc>::type V;
    const int ka_p = (int)round_up(ka, 16), nb_p = (int)round_up(nb, 16);
    const int lda_s = tn_ld(ka_p, sizeof(Tin)), ldb_s = tn_ld(nb_p, sizeof(Tin));
    const int bufsz = RC * lda_s + (sym ? 0 : RC * ldb_s);
    Tin* buf0 = reinterpret_cast<Tin*>(smem_raw);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform -> scalar registers
    const int nbi = ka_p / 16, nbj = nb_p / 16;
    const int64_t split = blockIdx.x;
    const int64_t r_begin = split * rows_per_split;
    const int64_t r_end = min(N, r_begin + rows_per_split);

    // this wave's RI x RJ piece of the work-group's (WI RI) x (4 RJ) tile
    constexpr int NT = 256 * WI;
    const int ntj = (int)ceil_div(nbj, 4 * RJ);
    const int ti = blockIdx.y / ntj, tj = blockIdx.y % ntj;
    const int bi0 = ti * WI * RI + (wave >> 2) * RI;
    const int bj0 = tj * 4 * RJ + (wave & 3) * RJ;
    V acc[RI][RJ];
#pragma unroll
    for (int i = 0; i < RI; ++i)
#pragma unroll
        for (int j = 0; j < RJ; ++j) acc[i][j] = zero_acc<V>();

    const int na = St::ntasks(a_rowmajor, ka, ka_p, RC);
    const int nbt = sym ? 0 : St::ntasks(b_rowmajor, nb, nb_p, RC);
    const int ntask = na + nbt;
    St task[TN_MAXT];
    bool has[TN_MAXT];
#pragma unroll
    for (int q = 0; q < TN_MAXT; ++q) {
        const int t = tid + q * NT;
        has[q] = t < ntask;
        if (t < na) task[q].init(A + r_begin * (a_rowmajor ? lda : 1), lda, a_rowmajor, ka, ka_p, RC, t, lda_s, 0);
        else task[q].init(B + r_begin * (b_rowmajor ? ldb : 1), ldb, b_rowmajor, nb, nb_p, RC,
                          has[q] ? t - na : 0, ldb_s, RC * lda_s);
    }
    VT pre[TN_MAXT];
    // the next chunk of every task into registers: fetch_whole for a chunk whose rows all
    // exist, fetch (c0 = the chunk's row offset inside the split) with row guards
    auto fetch_whole = [&]() {
#pragma unroll
        for (int q = 0; q < TN_MAXT; ++q)
            if (has[q]) { pre[q] = task[q].load_full(); task[q].next(); }
    };
    auto fetch = [&](int64_t c0) {
#pragma unroll
        for (int q = 0; q < TN_MAXT; ++q)
            if (has[q]) { pre[q] = task[q].load(c0, r_end - r_begin, vec); task[q].next(); }
    };
    auto put = [&](Tin* buf) {
#pragma unroll
        for (int q = 0; q < TN_MAXT; ++q)
            if (has[q]) task[q].store(buf, pre[q]);
    };

    const int64_t nchunk = ceil_div(r_end - r_begin, (int64_t)RC);
    const int64_t nwhole = vec ? (r_end - r_begin) / RC : 0;   // chunks read by 16-byte loads
    if (nchunk > 0) {
        fetch(0);
        put(buf0);
    }
    __syncthreads();
    // clamped fragment columns (in elements)
    const int amax = (nbi - 1) * 16, bmax = (nbj - 1) * 16;
    // one chunk: fetch the next one into registers, MFMAs on the current one, then the
    // next one into the other buffer.  The loop whose next chunk is whole has only the
    // unguarded loads, which all stay in flight together; the guarded per-element loads
    // of a ragged chunk run in a loop of their own, since in the same loop they write
    // the same registers and make each load wait for the one before.
    auto step = [&](int64_t ci, auto whole_next) {
        Tin* cur = buf0 + (ci & 1) * bufsz;
        Tin* nxt = buf0 + ((ci + 1) & 1) * bufsz;
        const bool more = ci + 1 < nchunk;
        if constexpr (decltype(whole_next)::value) fetch_whole();
        else if (more) fetch((ci + 1) * RC);
        const Tin* As = cur;
        const Tin* Bs = sym ? cur : cur + RC * lda_s;
        const int bld = sym ? lda_s : ldb_s;
#pragma unroll
        for (int ks = 0; ks < RC / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            const Tin* arow = As + kk * lda_s + (lane & 15);
            const Tin* brow = Bs + kk * bld + (lane & 15);
            Tc av[RI], bv[RJ];
#pragma unroll
            for (int i = 0; i < RI; ++i) av[i] = (Tc)arow[min((bi0 + i) * 16, amax)];
#pragma unroll
            for (int j = 0; j < RJ; ++j) bv[j] = (Tc)brow[min((bj0 + j) * 16, bmax)];
#pragma unroll
            for (int i = 0; i < RI; ++i)
#pragma unroll
                for (int j = 0; j < RJ; ++j) acc[i][j] = mfma(av[i], bv[j], acc[i][j]);
        }
        if (more) put(nxt);
        __syncthreads();
    };
    int64_t ci = 0;
    for (; ci + 1 < nwhole; ++ci) step(ci, std::true_type{});
    for (; ci < nchunk; ++ci) step(ci, std::false_type{});

    double* out = P + split * (int64_t)ka * nb;
#pragma unroll
    for (int i = 0; i < RI; ++i) {
#pragma unroll
        for (int j = 0; j < RJ; ++j) {
            if (bi0 + i >= nbi || bj0 + j >= nbj) continue;
            const int jj = (bj0 + j) * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ii = (bi0 + i) * 16 + acc_row<V>(lane, v);
                if (ii < ka && jj < nb) out[(int64_t)jj * ka + ii] = (double)acc[i][j][v];
            }
        }
    }
}

// Symmetric product P_s = A[rows_s]^T A[rows_s] (the Gram matrices), nbi <= 2*SB_MAXW*8
// block rows: only the upper block triangle is formed (the reduction mirrors it).  The
// 16x16 blocks are grouped in 2x2 super-blocks; the upper super-blocks (si <= sj) are
// dealt to the 8 waves, at most SB_MAXW each, so no wave forms more than 4*SB_MAXW
// blocks.  Staging as in gemm_tn_kernel (two LDS buffers, one barrier per chunk).
constexpr int SB_MAXW = 2;
template <typename Tin, typename Tc, int RC>
__global__ void __launch_bounds__(TN_THREADS)
gemm_sym_kernel(const Tin* __restrict__ A, int64_t lda, int a_rowmajor, int ka,
                int64_t N, int64_t rows_per_split, int vec, double* __restrict__ P,
                const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    typedef TnStage<Tin, Tc> St;
    typedef typename St::VT VT;
    typedef typename Acc<Tc>::type V;
    const int ka_p = (int)round_up(ka, 16);
    const int lda_s = tn_ld(ka_p, sizeof(Tin));
    const int bufsz = RC * lda_s;
    Tin* buf0 = reinterpret_cast<Tin*>(smem_raw);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nbi = ka_p / 16, sbn = (nbi + 1) / 2, nsb = sbn * (sbn + 1) / 2;
    const int64_t split = blockIdx.x;
    const int64_t r_begin = split * rows_per_split;
    const int64_t r_end = min(N, r_begin + rows_per_split);

    // this wave's super-blocks (column-major over the upper triangle): block rows 2si, 2si+1
    // and block columns 2sj, 2sj+1, clamped to the last block (recomputed, not stored)
    int sr[SB_MAXW], sc[SB_MAXW];
    bool sv[SB_MAXW];
#pragma unroll
    for (int q = 0; q < SB_MAXW; ++q) {
        const int sb = wave + q * (TN_THREADS / 64);
        sv[q] = sb < nsb;
        int si = 0, sj = 0;
        if (sv[q]) block_decode(sb, 1, sbn, &si, &sj);
        sr[q] = si; sc[q] = sj;
    }
    V acc[SB_MAXW][2][2];
#pragma unroll
    for (int q = 0; q < SB_MAXW; ++q)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[q][a][b] = zero_acc<V>();

    const int ntask = St::ntasks(a_rowmajor, ka, ka_p, RC);
    St task[TN_MAXT];
    bool has[TN_MAXT];
#pragma unroll
    for (int q = 0; q < TN_MAXT; ++q) {
        const int t = tid + q * TN_THREADS;
        has[q] = t < ntask;
        task[q].init(A + r_begin * (a_rowmajor ? lda : 1), lda, a_rowmajor, ka, ka_p, RC, has[q] ? t : 0, lda_s, 0);
    }
    VT pre[TN_MAXT];
    auto fetch_whole = [&]() {
#pragma unroll
        for (int q = 0; q < TN_MAXT; ++q)
            if (has[q]) { pre[q] = task[q].load_full(); task[q].next(); }
    };
    auto fetch = [&](int64_t c0) {
#pragma unroll
        for (int q = 0; q < TN_MAXT; ++q)
            if (has[q]) { pre[q] = task[q].load(c0, r_end - r_begin, vec); task[q].next(); }
    };
    auto put = [&](Tin* buf) {
#pragma unroll
        for (int q = 0; q < TN_MAXT; ++q)
            if (has[q]) task[q].store(buf, pre[q]);
    };

    const int64_t nchunk = ceil_div(r_end - r_begin, (int64_t)RC);
    const int64_t nwhole = vec ? (r_end - r_begin) / RC : 0;
    if (nchunk > 0) {
        fetch(0);
        put(buf0);
    }
    __syncthreads();
    const int amax = (nbi - 1) * 16;
    // whole next chunks and the ragged rest in loops of their own, as in gemm_tn_kernel
    auto step = [&](int64_t ci, auto whole_next) {
        Tin* cur = buf0 + (ci & 1) * bufsz;
        Tin* nxt = buf0 + ((ci + 1) & 1) * bufsz;
        const bool more = ci + 1 < nchunk;
        if constexpr (decltype(whole_next)::value) fetch_whole();
        else if (more) fetch((ci + 1) * RC);
#pragma unroll
        for (int ks = 0; ks < RC / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            const Tin* row = cur + kk * lda_s + (lane & 15);
#pragma unroll
            for (int q = 0; q < SB_MAXW; ++q) {
                if (!sv[q]) continue;                                 // wave-uniform
                Tc av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = (Tc)row[min((2 * sr[q] + a) * 16, amax)];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = (Tc)row[min((2 * sc[q] + b) * 16, amax)];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) acc[q][a][b] = mfma(av[a], bv[b], acc[q][a][b]);
            }
        }
        if (more) put(nxt);
        __syncthreads();
    };
    int64_t ci = 0;
    for (; ci + 1 < nwhole; ++ci) step(ci, std::true_type{});
    for (; ci < nchunk; ++ci) step(ci, std::false_type{});

    double* out = P + split * (int64_t)ka * ka;
#pragma unroll
    for (int q = 0; q < SB_MAXW; ++q) {
        if (!sv[q]) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int bi = 2 * sr[q] + a, bj = 2 * sc[q] + b;
                if (bi >= nbi || bj >= nbi || bi > bj) continue;
                const int jj = bj * 16 + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ii = bi * 16 + acc_row<V>(lane, v);
                    if (ii < ka && jj < ka) out[(int64_t)jj * ka + ii] = (double)acc[q][a][b][v];
                }
            }
    }
}

// out(i, j) = sum_s P_s(i, j) in a fixed order: work-group = 64 consecutive rows i of one
// column j (blockIdx.y) x RQ split ranges; thread (o, q) sums the splits s = q, q + RQ, ...
// of row o, and the RQ partial sums are added in q order.  Every read of a split is 64
// consecutive entries of a column.  In symmetric mode the products hold the upper block
// triangle only: a column is summed down to the end of its diagonal block and each sum
// above the diagonal block is written to (i, j) and to the mirror (j, i), which keeps the
// output exactly symmetric.
constexpr int RQ = 8;
__global__ void __launch_bounds__(64 * RQ)
reduce_partials_kernel(const double* __restrict__ P, int nsplit, int ka, int nb,
                       int sym, double* out, int64_t ldo, float* out32,
                       int64_t ldo32, const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    __shared__ double part[RQ][64];
    const int64_t tot = (int64_t)ka * nb;
    const int o = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int j = blockIdx.y;
    const int i = blockIdx.x * 64 + o;
    const int limit = sym ? min(ka, (j / 16 + 1) * 16) : ka;
    if (blockIdx.x * 64 >= limit) return;                // the whole work-group: uniform
    double s = 0.0;
    if (i < limit) {
        const double* p = P + (int64_t)j * ka + i;
        // eight loads in flight per lane, added in the same (split) order as one at a time
        int k = q;
        for (; k + 7 * RQ < nsplit; k += 8 * RQ) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(k + u * RQ) * tot];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; k < nsplit; k += RQ) s += p[(int64_t)k * tot];
    }
    part[q][o] = s;
    __syncthreads();
    if (q == 0 && i < limit) {
        double t = part[0][o];
#pragma unroll
        for (int k = 1; k < RQ; ++k) t += part[k][o];
        if (out) out[(int64_t)j * ldo + i] = t;
        if (out32) out32[(int64_t)j * ldo32 + i] = (float)t;
        if (sym && i / 16 < j / 16) {
            if (out) out[(int64_t)i * ldo + j] = t;
            if (out32) out32[(int64_t)i * ldo32 + j] = (float)t;
        }
    }
}

// Row splits: one chunk or more per split up to 256 splits, and for long products at
// least 32 chunks per split up to TN_MAX_SPLITS (more work-groups in flight per CU).
static int tn_splits(int64_t N, int rc) {
    const int64_t chunks = ceil_div(N, (int64_t)rc);
    int64_t s = std::max(std::min<int64_t>(chunks, 256), std::min<int64_t>(ceil_div(chunks, (int64_t)32), TN_MAX_SPLITS));
    return (int)std::max<int64_t>(s, 1);
}
// largest split count over the chunk sizes used (8 and 16 rows)
int tn_max_splits(int64_t N) { return std::max(tn_splits(N, 8), tn_splits(N, 16)); }

template <typename Tin, typename Tc>
static size_t tn_lds(int rc, int ka, int nb, int sym) {
    const size_t per = (size_t)rc * tn_ld((int)round_up(ka, 16), sizeof(Tin)) +
                       (sym ? 0 : (size_t)rc * tn_ld((int)round_up(nb, 16), sizeof(Tin)));
    return 2 * per * sizeof(Tin);
}

// wave tiles (RI x RJ output blocks) instantiated per accumulator type
#define TN_TILES_F32(X, Ti, Tc, RC) X(Ti, Tc, RC, 2, 2) X(Ti, Tc, RC, 3, 3) X(Ti, Tc, RC, 5, 1) \
    X(Ti, Tc, RC, 5, 3) X(Ti, Tc, RC, 5, 4) X(Ti, Tc, RC, 5, 5) X(Ti, Tc, RC, 7, 3) X(Ti, Tc, RC, 10, 3)
#define TN_TILES_F64(X, Ti, Tc, RC) X(Ti, Tc, RC, 2, 2) X(Ti, Tc, RC, 3, 3) X(Ti, Tc, RC, 4, 4) \
    X(Ti, Tc, RC, 5, 1) X(Ti, Tc, RC, 5, 3)
// FP32 products with 16 waves (4 x 4): smaller wave tiles, four waves per SIMD
#define TN_TILES_F32_W4(X) X(3, 3) X(3, 4) X(3, 5) X(4, 3) X(5, 3)
#define TN_INSTANCES(X) \
    TN_TILES_F32(X, float, float, 16) TN_TILES_F32(X, float, float, 8) \
    TN_TILES_F64(X, float, double, 16) TN_TILES_F64(X, float, double, 8) \
    TN_TILES_F64(X, double, double, 16) TN_TILES_F64(X, double, double, 8)

hipError_t gemm_prepare()
{
    hipError_t e = hipSuccess;
#define TN_ATTR(Ti, Tc, RC, RI, RJ) \
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)gemm_tn_kernel<Ti, Tc, RC, RI, RJ, 2>, \
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    TN_INSTANCES(TN_ATTR)
#undef TN_ATTR
#define TN_ATTR4(RI, RJ) \
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)gemm_tn_kernel<float, float, 16, RI, RJ, 4>, \
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    TN_TILES_F32_W4(TN_ATTR4)
#undef TN_ATTR4
#define SYM_ATTR(Ti, Tc, RC) \
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)gemm_sym_kernel<Ti, Tc, RC>, \
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    SYM_ATTR(float, float, 16) SYM_ATTR(float, float, 8) SYM_ATTR(float, double, 16) SYM_ATTR(float, double, 8)
    SYM_ATTR(double, double, 16) SYM_ATTR(double, double, 8)
#undef SYM_ATTR
    return e;
}

size_t gemm_tn_partial_bytes(int64_t N, int ka, int nb) {
    return (size_t)tn_max_splits(N) * (size_t)ka * (size_t)nb * sizeof(double);
}

template <typename Tin, typename Tc, int RC, int RI, int RJ, int WI = 2>
static hipError_t launch_tn_k(hipStream_t s, const Tin* A, int64_t lda, int a_rm, int ka,
                              const Tin* B, int64_t ldb, int b_rm, int nb, int sym, int64_t N, int vec,
                              double* P, int* nsplit_out, const int32_t* skip_unless)
{
    const int nbi = (int)ceil_div(ka, 16), nbj = (int)ceil_div(nb, 16);
    const int gy = (int)(ceil_div(nbi, WI * RI) * ceil_div(nbj, 4 * RJ));
    const int ns = tn_splits(N, RC);
    const int64_t rps = round_up(ceil_div(N, ns), RC);
    const int ns_eff = (int)ceil_div(N, rps);
    const size_t lds = tn_lds<Tin, Tc>(RC, ka, nb, sym);
    hipLaunchKernelGGL((gemm_tn_kernel<Tin, Tc, RC, RI, RJ, WI>), dim3(ns_eff, gy), dim3(256 * WI), lds, s,
                       A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, rps, vec, P, skip_unless);
    *nsplit_out = ns_eff;
    return hipGetLastError();
}

// Wave tile: the instantiated shape that covers the block grid with the fewest
// work-groups per row split, then the least recomputed (clamped) blocks.
template <typename Tin, typename Tc, int RC>
static hipError_t launch_sym_k(hipStream_t s, const Tin* A, int64_t lda, int a_rm, int ka, int64_t N, int vec,
                               double* P, int* nsplit_out, const int32_t* skip_unless)
{
    const int ns = tn_splits(N, RC);
    const int64_t rps = round_up(ceil_div(N, ns), RC);
    const int ns_eff = (int)ceil_div(N, rps);
    const size_t lds = tn_lds<Tin, Tc>(RC, ka, ka, 1);
    hipLaunchKernelGGL((gemm_sym_kernel<Tin, Tc, RC>), dim3(ns_eff), dim3(TN_THREADS), lds, s,
                       A, lda, a_rm, ka, N, rps, vec, P, skip_unless);
    *nsplit_out = ns_eff;
    return hipGetLastError();
}

// ---- tile choice of the TN products: the cost model below, or a timed choice per shape
// class (input and compute type, row chunk, output blocks, log2 N) from tn_tune_recorded.
// While recording, each product that reaches the tile choice is kept (its arguments by
// value) so the tuner can replay it with every candidate forced.
typedef std::tuple<int, int, int, int, int, int> TnKey;
static std::mutex g_tn_mu;
static std::map<TnKey, int> g_tn_table;
typedef std::vector<std::pair<TnKey, std::function<hipError_t(hipStream_t, int)>>> TnCalls;
static bool g_tn_recording = false;
static TnCalls g_tn_calls;
static thread_local int g_tn_force = -1;

template <typename T> constexpr int tn_type_code() { return sizeof(T) == 4 ? DMD_F32 : DMD_F64; }

// The candidate to launch among ncand: the forced one during a tuner replay (a force past
// the last candidate is hipErrorNotFound, nothing launched), else the tuned one, else the
// cost model's *best.
static hipError_t tn_pick(const TnKey& key, int ncand, int* best)
{
    if (g_tn_force >= 0) {
        if (g_tn_force >= ncand) return hipErrorNotFound;
        *best = g_tn_force;
        return hipSuccess;
    }
    std::lock_guard<std::mutex> g(g_tn_mu);
    auto it = g_tn_table.find(key);
    if (it != g_tn_table.end() && it->second >= 0 && it->second < ncand) *best = it->second;
    return hipSuccess;
}
static int tn_log2(int64_t n) { int l = 0; while ((int64_t(1) << (l + 1)) <= n) ++l; return l; }

template <typename Tin, typename Tc, int RC>
static hipError_t launch_tn_rc(hipStream_t s, const Tin* A, int64_t lda, int a_rm, int ka,
                               const Tin* B, int64_t ldb, int b_rm, int nb, int sym, int64_t N, int vec,
                               double* P, int* nsplit_out, const int32_t* skip_unless)
{
    const int nbi = (int)ceil_div(ka, 16), nbj = (int)ceil_div(nb, 16);
    // symmetric products whose upper super-blocks fit the waves: triangle-only kernel
    if (sym && ((nbi + 1) / 2) * ((nbi + 1) / 2 + 1) / 2 <= SB_MAXW * (TN_THREADS / 64))
        return launch_sym_k<Tin, Tc, RC>(s, A, lda, a_rm, ka, N, vec, P, nsplit_out, skip_unless);
    const TnKey key{tn_type_code<Tin>(), tn_type_code<Tc>(), RC, nbi, nbj, tn_log2(N)};
    if (g_tn_force < 0) {
        std::lock_guard<std::mutex> g(g_tn_mu);
        if (g_tn_recording)
            g_tn_calls.emplace_back(key, [=](hipStream_t s2, int force) {
                int ns = 0;
                g_tn_force = force;
                const hipError_t e = launch_tn_rc<Tin, Tc, RC>(s2, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P,
                                                              &ns, skip_unless);
                g_tn_force = -1;
                return e;
            });
    }
    int best = -1;
    int64_t best_cost = INT64_MAX;
    int idx = 0;
    // fewest work-groups per row split (each re-reads the panels) first, then MFMA work
    // (recomputed clamped blocks); 16-wave tiles count half, for their occupancy
    auto consider = [&](int ri, int rj, int wi) {
        const int64_t gy = ceil_div(nbi, wi * ri) * ceil_div(nbj, 4 * rj);
        const int64_t cost = gy * 100000 + gy * 4 * wi * ri * rj * (wi == 4 ? 5 : 10);
        if (cost < best_cost) { best_cost = cost; best = idx; }
        ++idx;
    };
#define TN_CASE(k, RI, RJ) \
    case k: return launch_tn_k<Tin, Tc, RC, RI, RJ>(s, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P, nsplit_out, skip_unless);
#define TN_CASE4(k, RI, RJ) \
    case k: return launch_tn_k<Tin, Tc, RC, RI, RJ, 4>(s, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P, nsplit_out, skip_unless);
    if constexpr (sizeof(Tc) == 4 && sizeof(Tin) == 4 && RC == 16) {
        consider(2, 2, 2); consider(3, 3, 2); consider(5, 1, 2); consider(5, 3, 2); consider(5, 4, 2); consider(5, 5, 2);
        consider(7, 3, 2); consider(10, 3, 2);
        consider(3, 3, 4); consider(3, 4, 4); consider(3, 5, 4); consider(4, 3, 4); consider(5, 3, 4);
        if (hipError_t e = tn_pick(key, idx, &best)) return e;
        switch (best) {
            TN_CASE(0, 2, 2) TN_CASE(1, 3, 3) TN_CASE(2, 5, 1) TN_CASE(3, 5, 3) TN_CASE(4, 5, 4) TN_CASE(5, 5, 5)
            TN_CASE(6, 7, 3) TN_CASE(7, 10, 3)
            TN_CASE4(8, 3, 3) TN_CASE4(9, 3, 4) TN_CASE4(10, 3, 5) TN_CASE4(11, 4, 3)
            default: return launch_tn_k<Tin, Tc, RC, 5, 3, 4>(s, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P, nsplit_out, skip_unless);
        }
    } else if constexpr (sizeof(Tc) == 4) {
        consider(2, 2, 2); consider(3, 3, 2); consider(5, 1, 2); consider(5, 3, 2); consider(5, 4, 2); consider(5, 5, 2);
        consider(7, 3, 2); consider(10, 3, 2);
        if (hipError_t e = tn_pick(key, idx, &best)) return e;
        switch (best) {
            TN_CASE(0, 2, 2) TN_CASE(1, 3, 3) TN_CASE(2, 5, 1) TN_CASE(3, 5, 3) TN_CASE(4, 5, 4) TN_CASE(5, 5, 5)
            TN_CASE(6, 7, 3)
            default: return launch_tn_k<Tin, Tc, RC, 10, 3>(s, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P, nsplit_out, skip_unless);
        }
    } else {
        consider(2, 2, 2); consider(3, 3, 2); consider(4, 4, 2); consider(5, 1, 2); consider(5, 3, 2);
        if (hipError_t e = tn_pick(key, idx, &best)) return e;
        switch (best) {
            TN_CASE(0, 2, 2) TN_CASE(1, 3, 3) TN_CASE(2, 4, 4) TN_CASE(3, 5, 1)
            default: return launch_tn_k<Tin, Tc, RC, 5, 3>(s, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P, nsplit_out, skip_unless);
        }
    }
#undef TN_CASE
#undef TN_CASE4
}

// Largest row chunk whose two LDS buffers and staging registers fit.
template <typename Tin, typename Tc>
static hipError_t launch_tn_t(hipStream_t s, const Tin* A, int64_t lda, int a_rm, int ka,
                              const Tin* B, int64_t ldb, int b_rm, int nb, int sym, int64_t N,
                              double* P, int* nsplit_out, const int32_t* skip_unless)
{
    typedef TnStage<Tin, Tc> St;
    constexpr int VWI = St::VWI;
    // 16-byte loads need aligned bases and leading dimensions; row-major operands are
    // read up to the padded width, so they also need ld >= that width
    auto ok = [&](const Tin* X, int64_t ld, int rm, int nc) {
        if ((uintptr_t)X % 16 || ld % VWI) return false;
        return !rm || ld >= round_up(nc, 16);
    };
    const int vec = ok(A, lda, a_rm, ka) && (sym || ok(B, ldb, b_rm, nb)) ? 1 : 0;
    const int ka_p = (int)round_up(ka, 16), nb_p = (int)round_up(nb, 16);
    auto fits = [&](int rc) {
        const int64_t tasks = (int64_t)St::ntasks(a_rm, ka, ka_p, rc) + (sym ? 0 : St::ntasks(b_rm, nb, nb_p, rc));
        return tn_lds<Tin, Tc>(rc, ka, nb, sym) <= 160 * 1024 && tasks <= (int64_t)TN_THREADS * TN_MAXT;
    };
    if (fits(16)) return launch_tn_rc<Tin, Tc, 16>(s, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P, nsplit_out, skip_unless);
    if (fits(8)) return launch_tn_rc<Tin, Tc, 8>(s, A, lda, a_rm, ka, B, ldb, b_rm, nb, sym, N, vec, P, nsplit_out, skip_unless);
    return hipErrorInvalidValue;
}

// A^T b for a row-major A (N x ka, ka <= 192, 16-byte aligned rows) and one column b: a
// memory-bound pass, so no MFMA and no staging.  A row is cut into chunks of 64 VW
// columns; in chunk h, lane l reads the VW consecutive columns 64 VW h + VW l .. + VW-1 as
// one 16-byte load (each chunk of a row is one contiguous read across the wave) and
// accumulates them in FP64.  FP32 rows (VW = 4) need one chunk for 192 columns, FP64 rows
// (VW = 2) two.  Each wave walks its rows GEMV_ROWS_UNROLL at a time; the four waves of a
// work-group sum in LDS, one FP64 partial per split.
constexpr int GEMV_ROWS_UNROLL = 8;
constexpr int GEMV_MAX_KA = 192;
template <typename T>
__global__ void __launch_bounds__(256)
gemv_tn_kernel(const T* __restrict__ A, int64_t lda, int ka, const T* __restrict__ b, int64_t N,
               int64_t rows_per_split, double* __restrict__ P, const int32_t* skip_unless)
{
    if (skip_unless && *skip_unless == 0) return;
    constexpr int VW = 16 / sizeof(T);
    constexpr int NCH = (GEMV_MAX_KA + 64 * VW - 1) / (64 * VW);
    typedef T vec __attribute__((ext_vector_type(VW)));
    __shared__ double part[4][GEMV_MAX_KA];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = blockIdx.x * rows_per_split;
    const int64_t r1 = min(N, r0 + rows_per_split);
    bool act[NCH];
    int col[NCH];
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
        const int c = (64 * h + lane) * VW;
        act[h] = c < ka;
        col[h] = act[h] ? c : 0;
    }
    // the first chunk is read by every lane (inactive lanes re-read column 0, in bounds);
    // later chunks only where they hold columns
    auto load = [&](int64_t rw, int h) -> vec {
        if (h == 0 || act[h]) return *reinterpret_cast<const vec*>(A + rw * lda + col[h]);
        return vec{};
    };
    double acc[NCH][VW];
#pragma unroll
    for (int h = 0; h < NCH; ++h)
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[h][e] = 0.0;
    int64_t row = r0 + wave;
    for (; row + 4 * (GEMV_ROWS_UNROLL - 1) < r1; row += 4 * GEMV_ROWS_UNROLL) {
        vec a[GEMV_ROWS_UNROLL][NCH];
        T bv[GEMV_ROWS_UNROLL];
#pragma unroll
        for (int u = 0; u < GEMV_ROWS_UNROLL; ++u) {
#pragma unroll
            for (int h = 0; h < NCH; ++h) a[u][h] = load(row + 4 * u, h);
            bv[u] = b[row + 4 * u];
        }
#pragma unroll
        for (int u = 0; u < GEMV_ROWS_UNROLL; ++u)
#pragma unroll
            for (int h = 0; h < NCH; ++h)
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[h][e] = fma((double)a[u][h][e], (double)bv[u], acc[h][e]);
    }
    for (; row < r1; row += 4) {
        const double bb = (double)b[row];
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
            const vec a = load(row, h);
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[h][e] = fma((double)a[e], bb, acc[h][e]);
        }
    }
#pragma unroll
    for (int h = 0; h < NCH; ++h)
        if (act[h])
#pragma unroll
            for (int e = 0; e < VW; ++e) part[wave][col[h] + e] = acc[h][e];
    __syncthreads();
    for (int c = threadIdx.x; c < ka; c += blockDim.x)
        P[blockIdx.x * (int64_t)ka + c] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
}

template <typename T>
static hipError_t launch_gemv_tn(hipStream_t s, const T* A, int64_t lda, int ka, const T* b, int64_t N, double* P,
                                 int* nsplit_out, const int32_t* skip_unless)
{
    // at least 4 rows per wave per split, at most the split count the partial buffer holds
    const int64_t ns = std::max<int64_t>(1, std::min<int64_t>(tn_max_splits(N), ceil_div(N, (int64_t)64)));
    const int64_t rps = ceil_div(N, ns);
    const int ns_eff = (int)ceil_div(N, rps);
    hipLaunchKernelGGL(gemv_tn_kernel<T>, dim3(ns_eff), dim3(256), 0, s, A, lda, ka, b, N, rps, P, skip_unless);
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
    } else if (nb == 1 && a_rowmajor && !sym && ka <= GEMV_MAX_KA && !b_rowmajor && (uintptr_t)A % 16 == 0 &&
               lda % (in_dtype == DMD_F32 ? 4 : 2) == 0 && lda >= round_up(ka, in_dtype == DMD_F32 ? 4 : 2)) {
        // one column against a row-major panel: FP64 accumulation for either compute type
        if (in_dtype == DMD_F32) e = launch_gemv_tn<float>(s, (const float*)A, lda, ka, (const float*)B, N, P, &ns, skip_unless);
        else e = launch_gemv_tn<double>(s, (const double*)A, lda, ka, (const double*)B, N, P, &ns, skip_unless);
    } else if (in_dtype == DMD_F32 && compute_dtype == DMD_F32) {
        e = launch_tn_t<float, float>(s, (const float*)A, lda, a_rowmajor, ka, (const float*)B, ldb, b_rowmajor, nb, sym, N, P, &ns, skip_unless);
    } else if (in_dtype == DMD_F32) {
        e = launch_tn_t<float, double>(s, (const float*)A, lda, a_rowmajor, ka, (const float*)B, ldb, b_rowmajor, nb, sym, N, P, &ns, skip_unless);
    } else {
        e = launch_tn_t<double, double>(s, (const double*)A, lda, a_rowmajor, ka, (const double*)B, ldb, b_rowmajor, nb, sym, N, P, &ns, skip_unless);
    }
    if (e != hipSuccess) return e;
    const int64_t tot = (int64_t)ka * nb;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)ceil_div(ka, 64), (unsigned)nb), dim3(64 * RQ), 0, s, P, ns,
                       ka, nb, sym, out, ldo, out32, ldo32, skip_unless);
    return hipGetLastError();
}


// ---- TN tile tuner
void tn_record(bool on)
{
    std::lock_guard<std::mutex> g(g_tn_mu);
    if (on) g_tn_calls.clear();
    g_tn_recording = on;
}

hipError_t tn_tune_recorded(hipStream_t s, std::vector<std::string>* lines)
{
    TnCalls calls;
    {
        std::lock_guard<std::mutex> g(g_tn_mu);
        calls.swap(g_tn_calls);
    }
    std::map<TnKey, std::pair<int, float>> done;
    hipEvent_t e0, e1;
    hipError_t err = hipEventCreate(&e0);
    if (err != hipSuccess) return err;
    if ((err = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return err; }
    for (auto& rec : calls) {
        if (done.count(rec.first)) continue;
        int best = -1;
        float best_ms = 1e30f;
        for (int c = 0; c < 64; ++c) {
            err = rec.second(s, c);                                   // warm-up
            if (err == hipErrorNotFound) { err = hipSuccess; break; }
            if (err != hipSuccess) break;
            (void)hipEventRecord(e0, s);
            for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) err = rec.second(s, c);
            (void)hipEventRecord(e1, s);
            if (err != hipSuccess || (err = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) { best_ms = ms; best = c; }
        }
        if (err != hipSuccess) break;
        done[rec.first] = {best, best_ms / 3.0f};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return err;
    std::lock_guard<std::mutex> g(g_tn_mu);
    for (auto& kv : done) {
        if (kv.second.first < 0) continue;
        g_tn_table[kv.first] = kv.second.first;
        if (lines) {
            char buf[160];
            const TnKey& k = kv.first;
            snprintf(buf, sizeof buf, "tn %d %d %d %d %d %d %d %.3f", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                     std::get<3>(k), std::get<4>(k), std::get<5>(k), kv.second.first, kv.second.second * 1000.0f);
            lines->push_back(buf);
        }
    }
    return hipSuccess;
}

void tn_table_set(int in_dt, int c_dt, int rc, int nbi, int nbj, int ln, int cand)
{
    std::lock_guard<std::mutex> g(g_tn_mu);
    g_tn_table[TnKey{in_dt, c_dt, rc, nbi, nbj, ln}] = cand;
}

size_t tn_table_size()
{
    std::lock_guard<std::mutex> g(g_tn_mu);
    return g_tn_table.size();
}

}  // namespace dmd
