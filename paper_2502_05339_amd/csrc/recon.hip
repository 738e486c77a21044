// Batched evaluation of the fitted model on MFMA (gfx950).
//
//  powers_pack : the coefficient matrix C (frame-major, [Kp][rp]) of
//                U = Re(Phi diag(lambda^e) b) in the folded real mode basis, with
//                lambda^e evaluated in FP64 as exp(e Log lambda)
//                (Sec. 4.4, eq. large_time_step; Sec. 6.1, eq. edit_temporal).
//  recon       : U (N x K, column-major) = Phi (N x rp, row-major) * C^T, as one
//                persistent GEMM over (row tile, frame chunk) work items.  The
//                row tile of Phi stays in registers while the frames stream
//                through LDS-staged chunks of C; every output element is written
//                exactly once with non-temporal 16-byte stores, after a pass through
//                LDS that makes each store instruction cover whole row runs of a frame.
//                With RESID the epilogue forms R = Xt - U instead, and the FP64
//                sum of squares of R (the adjoint's loss) per work-group.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace dmd {

// ---------------------------------------------------------------- coefficients
// Folded basis: kind 0 -> C = Re(b lambda^e); a pair (i, i+1) with members
// c1 = b_i lambda_i^e and c2 = b_{i+1} lambda_{i+1}^e has
//   C_i = Re c1 + Re c2,   C_{i+1} = Im c2 - Im c1
// because Re(phi c1 + conj(phi) c2) = Re(phi)(Re c1 + Re c2) + Im(phi)(Im c2 - Im c1).
// Each member also reports, in *flags, a power of lambda = 0 with a negative or
// fractional exponent (COEF_DOMAIN: Omega = Log(lambda) / dt has no value there) and a
// magnitude |b| |lambda|^e beyond vmax, the largest finite value of the output type
// (COEF_OVERFLOW).
__device__ __forceinline__ cplx checked_member(const double* lam, const double* b, int i, double e, double vmax,
                                               int* flags)
{
    const cplx l = {lam[2 * i], lam[2 * i + 1]};
    if (l.re == 0.0 && l.im == 0.0 && (e < 0.0 || e != floor(e))) { *flags |= COEF_DOMAIN; return {0.0, 0.0}; }
    const cplx c = cmul({b[2 * i], b[2 * i + 1]}, cpow_real(l, e));
    if (!(hypot(c.re, c.im) <= vmax)) *flags |= COEF_OVERFLOW;   // also catches NaN
    return c;
}

__device__ __forceinline__ double folded_coeff(const double* lam, const double* b,
                                               const int32_t* kind, int r, int i, double e, double vmax,
                                               int* flags)
{
    int kd = kind[i];
    if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;   // malformed pair marker
    if (kd == 0) return checked_member(lam, b, i, e, vmax, flags).re;
    const int i1 = (kd == 1) ? i : i - 1;
    const int i2 = i1 + 1;
    const cplx c1 = checked_member(lam, b, i1, e, vmax, flags);
    const cplx c2 = checked_member(lam, b, i2, e, vmax, flags);
    const double v = (kd == 1) ? (c1.re + c2.re) : (c2.im - c1.im);
    if (!(fabs(v) <= vmax)) *flags |= COEF_OVERFLOW;
    return v;
}

// Largest finite value of the coefficient / output type of a reconstruction mode.
__device__ __forceinline__ double mode_vmax(int mode)
{
    return mode == DMD_RECON_FP64 ? 1.7976931348623157e308 : 3.4028234663852886e38;
}

__global__ void powers_pack_kernel(const double* __restrict__ lam, const double* __restrict__ b,
                                   const int32_t* __restrict__ kind, int r,
                                   const double* __restrict__ expo, int K, int Kp, int rp,
                                   int mode, void* out_hi, void* out_lo, int32_t* status)
{
    const int64_t tot = (int64_t)Kp * rp;
    const double vmax = mode_vmax(mode);
    int flags = 0;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % rp);
        const int j = (int)(idx / rp);
        double v = 0.0;
        if (i < r && j < K) v = folded_coeff(lam, b, kind, r, i, expo[j], vmax, &flags);
        switch (mode) {
        case DMD_RECON_FP64: ((double*)out_hi)[idx] = v; break;
        case DMD_RECON_FP32: ((float*)out_hi)[idx] = (float)v; break;
        case DMD_RECON_BF16: ((__bf16*)out_hi)[idx] = (__bf16)(float)v; break;
        default: {
            const float f = (float)v;
            const __bf16 h = (__bf16)f;
            ((__bf16*)out_hi)[idx] = h;
            ((__bf16*)out_lo)[idx] = (__bf16)(f - (float)h);
        }
        }
    }
    if (flags && status) atomicOr(status, flags);
}

// Integer exponents to doubles; real times t to t / dt.
__global__ void exponents_kernel(const int64_t* __restrict__ k, const double* __restrict__ t,
                                 double inv_dt, int K, double* __restrict__ e)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < K; j += gridDim.x * blockDim.x)
        e[j] = k ? (double)k[j] : t[j] * inv_dt;
}

// ---------------------------------------------------------------- reconstruction
template <int MODE> struct RTraits;
template <> struct RTraits<DMD_RECON_FP64> {
    typedef double Tphi; typedef double Tc; typedef double Tout; typedef doublex4 V;
    static constexpr int KW = 16;   // modes per k-group
};
template <> struct RTraits<DMD_RECON_FP32> {
    typedef float Tphi; typedef float Tc; typedef float Tout; typedef floatx4 V;
    static constexpr int KW = 16;
};
template <> struct RTraits<DMD_RECON_BF16> {
    typedef float Tphi; typedef __bf16 Tc; typedef float Tout; typedef floatx4 V;
    static constexpr int KW = 32;
};
template <> struct RTraits<DMD_RECON_BF16X3> {
    typedef float Tphi; typedef __bf16 Tc; typedef float Tout; typedef floatx4 V;
    static constexpr int KW = 32;
};

template <int MODE> struct AFrag;
template <> struct AFrag<DMD_RECON_FP64> { double v[4]; };
template <> struct AFrag<DMD_RECON_FP32> { float v[4]; };
template <> struct AFrag<DMD_RECON_BF16> { bf16x8 hi; };
template <> struct AFrag<DMD_RECON_BF16X3> { bf16x8 hi, lo; };

// The A fragments of a row tile.  FP64 and FP32: one row block at a time, the loads of
// the block's nkg fragments are issued together (rows past N read row 0, which exists),
// then the values are zeroed for those rows; loading fragment by fragment made each load
// wait for the one before, a chain of memory latencies at every new row tile.  Fragments
// past nkg are set to zero, so every fragment is redefined and the previous tile's values
// are dead while the new ones load.  BF16 modes load and split fragment by fragment: the
// batched form needs about 50 more registers there, and the bf16x3 kernel ran 25% slower
// with them.
template <int MODE> struct ARaw;
template <> struct ARaw<DMD_RECON_FP64> { double2 x, y; };
template <> struct ARaw<DMD_RECON_FP32> { float4 x; };
template <> struct ARaw<DMD_RECON_BF16> { float4 x, y; };
template <> struct ARaw<DMD_RECON_BF16X3> { float4 x, y; };

template <int MODE>
__device__ __forceinline__ void load_a_raw(ARaw<MODE>& r, const typename RTraits<MODE>::Tphi* p)
{
    if constexpr (MODE == DMD_RECON_FP64) {
        r.x = reinterpret_cast<const double2*>(p)[0];
        r.y = reinterpret_cast<const double2*>(p)[1];
    } else if constexpr (MODE == DMD_RECON_FP32) {
        r.x = reinterpret_cast<const float4*>(p)[0];
    } else {
        r.x = reinterpret_cast<const float4*>(p)[0];
        r.y = reinterpret_cast<const float4*>(p)[1];
    }
}

template <int MODE>
__device__ __forceinline__ void finish_a(AFrag<MODE>& f, const ARaw<MODE>& r, bool ok)
{
    if constexpr (MODE == DMD_RECON_FP64) {
        f.v[0] = ok ? r.x.x : 0.0; f.v[1] = ok ? r.x.y : 0.0;
        f.v[2] = ok ? r.y.x : 0.0; f.v[3] = ok ? r.y.y : 0.0;
    } else if constexpr (MODE == DMD_RECON_FP32) {
        f.v[0] = ok ? r.x.x : 0.f; f.v[1] = ok ? r.x.y : 0.f;
        f.v[2] = ok ? r.x.z : 0.f; f.v[3] = ok ? r.x.w : 0.f;
    } else {
        const float xs[8] = {r.x.x, r.x.y, r.x.z, r.x.w, r.y.x, r.y.y, r.y.z, r.y.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float v = ok ? xs[e] : 0.f;
            const __bf16 h = (__bf16)v;
            f.hi[e] = h;
            if constexpr (MODE == DMD_RECON_BF16X3) f.lo[e] = (__bf16)(v - (float)h);
        }
    }
}

template <int MODE, int RBW, int KGMAX>
__device__ __forceinline__ void load_tile_a(AFrag<MODE> (&a)[RBW][KGMAX], const typename RTraits<MODE>::Tphi* phi,
                                            int64_t ldphi, int64_t N, int64_t tile_row0, int nkg, int l16, int lg)
{
    constexpr int KW = RTraits<MODE>::KW;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
        const int64_t row = tile_row0 + rb * 16 + l16;
        const bool ok = row < N;
        const typename RTraits<MODE>::Tphi* prow = phi + (ok ? row : 0) * ldphi;
        if constexpr (MODE == DMD_RECON_FP64 || MODE == DMD_RECON_FP32) {
            ARaw<MODE> raw[KGMAX] = {};
#pragma unroll
            for (int kg = 0; kg < KGMAX; ++kg)
                if (kg < nkg) load_a_raw<MODE>(raw[kg], prow + kg * 16 + 4 * lg);
#pragma unroll
            for (int kg = 0; kg < KGMAX; ++kg) finish_a<MODE>(a[rb][kg], raw[kg], ok && kg < nkg);
        } else {
#pragma unroll
            for (int kg = 0; kg < KGMAX; ++kg) {
                if (kg < nkg) {
                    ARaw<MODE> raw;
                    if (ok) load_a_raw<MODE>(raw, prow + kg * 32 + 8 * lg);
                    else raw.x = raw.y = make_float4(0.f, 0.f, 0.f, 0.f);
                    finish_a<MODE>(a[rb][kg], raw, true);
                }
            }
        }
    }
}

// Coefficient rows of FC frames (16-byte moves, thread-strided) from global memory to
// registers, and from registers to an LDS buffer with row stride cld (>= rp + 16 bytes).
// The moves in flight live in one vector value of 4*PREF floats, not an array: private
// arrays share the compiler's register budget with the fragment array a[][], and past it
// they go to scratch.  Both copies are straight-line code.
template <int PREF> using PrefV = float __attribute__((ext_vector_type(4 * PREF)));

template <int PREF>
__device__ __forceinline__ float4 pref_get(const PrefV<PREF>& v, int q)
{
    return make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}
template <int PREF>
__device__ __forceinline__ void pref_set(PrefV<PREF>& v, int q, float4 x)
{
    v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
}

template <int PREF, bool X3, typename Tc>
__device__ __forceinline__ void recon_fetch(PrefV<PREF>& hi, PrefV<PREF>& lo, const Tc* __restrict__ Chi,
                                            const Tc* __restrict__ Clo, int tid, int per_row, int f0, int rp,
                                            int FC, int VE)
{
#pragma unroll
    for (int q = 0; q < PREF; ++q) {
        // a move past the chunk re-reads its first piece (recon_put drops it)
        const int idx = tid + q * 256 < FC * per_row ? tid + q * 256 : 0;
        const int fr = idx / per_row, c = (idx % per_row) * VE;
        const int64_t src = (int64_t)(f0 + fr) * rp + c;
        pref_set<PREF>(hi, q, *reinterpret_cast<const float4*>(&Chi[src]));
        if constexpr (X3) pref_set<PREF>(lo, q, *reinterpret_cast<const float4*>(&Clo[src]));
    }
}
template <int PREF, bool X3, typename Tc>
__device__ __forceinline__ void recon_put(const PrefV<PREF>& hi, const PrefV<PREF>& lo, Tc* Sh, Tc* Sl,
                                          int tid, int per_row, int cld, int FC, int VE)
{
#pragma unroll
    for (int q = 0; q < PREF; ++q) {
        // a move past the chunk lands in the row pad of frame 0, which no MFMA operand
        // reads (columns >= rp = per_row * VE)
        const int idx = tid + q * 256;
        const bool ok = idx < FC * per_row;
        const int fr = idx / per_row, c = (idx % per_row) * VE;
        const int off = ok ? fr * cld + c : per_row * VE;
        *reinterpret_cast<float4*>(&Sh[off]) = pref_get<PREF>(hi, q);
        if constexpr (X3) *reinterpret_cast<float4*>(&Sl[off]) = pref_get<PREF>(lo, q);
    }
}

// Epilogue of one 16-frame block.  The wave holds RW = 16*RBW consecutive rows of
// frames fb .. fb+15, in the MFMA layout (lane l: frame fb + l%16, 16-row pieces).
// Stored as is, one store instruction would write 16 frames x 64 bytes, half of a
// 128-byte line per frame.  The block goes through the wave's own LDS tile st
// (16 x (RW + pad) elements) and comes back frame-major: each lane then holds 16
// contiguous bytes of one frame and each instruction writes 4*RW (FP32) or 8*RW (FP64)
// contiguous bytes per frame.  With RESID the stored value is Xt - U and its square
// is added to ss.  Frames >= f_end and rows >= N are not written.
template <typename Tout, typename V, int RBW, bool RESID>
__device__ __forceinline__ void recon_store(const V (&acc)[RBW], Tout* st, int lane, int fb, int f_end,
                                            int64_t row0, int64_t N, Tout* U, int64_t ldu, int vec_store,
                                            const Tout* __restrict__ Xt, int64_t ldxt, double& ss)
{
    constexpr int RW = 16 * RBW;
    constexpr int VEC = 16 / sizeof(Tout);    // elements per 16-byte piece
    constexpr int SLD = RW + VEC;             // tile row stride (one piece of pad)
    constexpr int LPF = RW / VEC;             // lanes per frame on the way out
    constexpr int FPI = 64 / LPF;             // frames per store instruction
    typedef typename std::conditional<sizeof(Tout) == 4, floatx4, doublex2>::type OV;
    const int l16 = lane & 15;
    wave_sync_lds();                          // the previous block's reads are done
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
        Tout* t = st + l16 * SLD + rb * 16;
        if constexpr (sizeof(Tout) == 4) {
            *reinterpret_cast<floatx4*>(t + acc_row<V>(lane, 0)) = acc[rb];
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) t[acc_row<V>(lane, v)] = acc[rb][v];
        }
    }
    wave_sync_lds();
#pragma unroll
    for (int q = 0; q < 16 / FPI; ++q) {
        const int fl = q * FPI + lane / LPF;
        const int rr = (lane % LPF) * VEC;
        const int frame = fb + fl;
        const int64_t row = row0 + rr;
        // a vector, not an array: private arrays count against the compiler's budget for
        // keeping such arrays in registers, which the fragment array a[][] nearly fills
        OV o = *reinterpret_cast<const OV*>(st + fl * SLD + rr);
        if (frame >= f_end || row >= N) continue;
        Tout* dst = U + (int64_t)frame * ldu + row;
        const bool full = vec_store && row + VEC <= N;
        if constexpr (RESID) {
            const Tout* src = Xt + (int64_t)frame * ldxt + row;
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                if (row + v < N) {
                    o[v] = src[v] - o[v];
                    ss += (double)o[v] * (double)o[v];
                }
            }
        }
        if (full) {
            if constexpr (RESID) *reinterpret_cast<OV*>(dst) = o;
            else __builtin_nontemporal_store(o, reinterpret_cast<OV*>(dst));
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                if (row + v < N) dst[v] = o[v];
        }
    }
}

// Work items are (row tile, chunk of FC frames) pairs, numbered row tile major; work-
// group g takes the contiguous run [g*ipw, (g+1)*ipw), so consecutive items mostly
// share their row tile (the tile of Phi is loaded into registers once per tile).  The
// coefficients of the next item are fetched into registers while the current item's
// MFMAs run, then stored to the other of two LDS buffers: one barrier per item.
template <int MODE, int RBW, int FCB, bool RESID>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
recon_kernel(const typename RTraits<MODE>::Tphi* __restrict__ phi, int64_t ldphi, int64_t N, int rp,
             const typename RTraits<MODE>::Tc* __restrict__ Chi,
             const typename RTraits<MODE>::Tc* __restrict__ Clo, int K,
             typename RTraits<MODE>::Tout* U, int64_t ldu, int vec_store,
             const typename RTraits<MODE>::Tout* __restrict__ Xt, int64_t ldxt,
             double* __restrict__ ss_partial,
             int n_rowtiles, int n_fchunks, int items_per_wg)
{
    typedef RTraits<MODE> Tr;
    typedef typename Tr::Tc Tc;
    typedef typename Tr::Tout Tout;
    typedef typename Tr::V V;
    constexpr int KW = Tr::KW;
    constexpr int KGMAX = RECON_MAX_RP / KW;
    constexpr int FC = FCB * 16;
    constexpr int CPAD = 16 / sizeof(Tc);               // 16-byte row pad in LDS
    constexpr int CLD = RECON_MAX_RP + CPAD;
    constexpr bool X3 = (MODE == DMD_RECON_BF16X3);
    constexpr int WG_ROWS = 4 * RBW * 16;
    constexpr int VE = 16 / sizeof(Tc);                 // elements per 16-byte move
    constexpr int PREF = (FC * (RECON_MAX_RP / VE) + 255) / 256;   // 16-byte moves per thread

    __shared__ __align__(16) Tc Cs_hi[2][FC * CLD];
    __shared__ __align__(16) Tc Cs_lo[X3 ? 2 : 1][X3 ? FC * CLD : 1];
    __shared__ __align__(16) Tout Ost[4][16 * (16 * RBW + 16 / sizeof(Tout))];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lg = lane >> 4;
    const int nkg = rp / KW;
    const int cld = rp + CPAD;          // LDS leading dimension actually used
    const int per_row = rp / VE;

    AFrag<MODE> a[RBW][KGMAX];
    int cur_rt = -1;
    double ss = 0.0;
    const int64_t n_items = (int64_t)n_rowtiles * n_fchunks;
    const int64_t it_begin = (int64_t)blockIdx.x * items_per_wg;
    const int64_t it_end = min(n_items, it_begin + items_per_wg);

    PrefV<PREF> pre_hi, pre_lo;
    if (it_begin < it_end) {
        recon_fetch<PREF, X3>(pre_hi, pre_lo, Chi, Clo, tid, per_row, (int)(it_begin % n_fchunks) * FC, rp, FC, VE);
        recon_put<PREF, X3>(pre_hi, pre_lo, Cs_hi[0], Cs_lo[0], tid, per_row, cld, FC, VE);
    }
    __syncthreads();
    for (int64_t item = it_begin; item < it_end; ++item) {
        const int buf = (int)((item - it_begin) & 1);
        const bool more = item + 1 < it_end;
        if (more) recon_fetch<PREF, X3>(pre_hi, pre_lo, Chi, Clo, tid, per_row, (int)((item + 1) % n_fchunks) * FC, rp, FC, VE);
        const int rt = (int)(item / n_fchunks);
        const int f0 = (int)(item % n_fchunks) * FC;
        const int f_end = min(K, f0 + FC);
        const int64_t tile_row0 = (int64_t)rt * WG_ROWS + wave * RBW * 16;
        if (rt != cur_rt) {
            load_tile_a<MODE, RBW, KGMAX>(a, phi, ldphi, N, tile_row0, nkg, l16, lg);
            cur_rt = rt;
        }
        {
#pragma unroll
            for (int cb = 0; cb < FCB; ++cb) {
                V acc[RBW];
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb) acc[rb] = zero_acc<V>();
                const Tc* crow_hi = Cs_hi[buf] + (cb * 16 + l16) * cld;
                const Tc* crow_lo = Cs_lo[X3 ? buf : 0] + (cb * 16 + l16) * cld;
#pragma unroll
                for (int kg = 0; kg < KGMAX; ++kg) {
                    if (kg < nkg) {
                        if constexpr (MODE == DMD_RECON_FP32 || MODE == DMD_RECON_FP64) {
                            const Tc* bp = crow_hi + kg * 16 + 4 * lg;
                            Tc bv[4];
                            if constexpr (MODE == DMD_RECON_FP32) {
                                float4 x = *reinterpret_cast<const float4*>(bp);
                                bv[0] = x.x; bv[1] = x.y; bv[2] = x.z; bv[3] = x.w;
                            } else {
                                double2 x = reinterpret_cast<const double2*>(bp)[0];
                                double2 y = reinterpret_cast<const double2*>(bp)[1];
                                bv[0] = x.x; bv[1] = x.y; bv[2] = y.x; bv[3] = y.y;
                            }
#pragma unroll
                            for (int s = 0; s < 4; ++s)
#pragma unroll
                                for (int rb = 0; rb < RBW; ++rb)
                                    acc[rb] = mfma(a[rb][kg].v[s], bv[s], acc[rb]);
                        } else {
                            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(crow_hi + kg * 32 + 8 * lg);
                            if constexpr (X3) {
                                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(crow_lo + kg * 32 + 8 * lg);
#pragma unroll
                                for (int rb = 0; rb < RBW; ++rb) {
                                    acc[rb] = mfma_bf16(a[rb][kg].lo, bh, acc[rb]);
                                    acc[rb] = mfma_bf16(a[rb][kg].hi, bl, acc[rb]);
                                    acc[rb] = mfma_bf16(a[rb][kg].hi, bh, acc[rb]);
                                }
                            } else {
#pragma unroll
                                for (int rb = 0; rb < RBW; ++rb)
                                    acc[rb] = mfma_bf16(a[rb][kg].hi, bh, acc[rb]);
                            }
                        }
                    }
                }
                recon_store<Tout, V, RBW, RESID>(acc, Ost[wave], lane, f0 + cb * 16, f_end, tile_row0, N,
                                                 U, ldu, vec_store, Xt, ldxt, ss);
            }
        }
        if (more) recon_put<PREF, X3>(pre_hi, pre_lo, Cs_hi[buf ^ 1], Cs_lo[X3 ? (buf ^ 1) : 0], tid, per_row, cld, FC, VE);
        __syncthreads();
    }
    if constexpr (RESID) {
        __shared__ double red[4];
        ss = wave_sum(ss);
        if (lane == 0) red[wave] = ss;
        __syncthreads();
        if (tid == 0) ss_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// Single-buffered variant (an autotuner candidate): each work item is a row tile and a
// range of frames; the coefficients of each FC-frame chunk are staged between two
// barriers.  It suits very long frame ranges in plain BF16 better than the prefetching
// kernel above on some shapes, so the autotuner times both.
template <int MODE, int RBW, int FCB, bool RESID>
__global__ void __launch_bounds__(256)
recon_kernel_sb(const typename RTraits<MODE>::Tphi* __restrict__ phi, int64_t ldphi, int64_t N, int rp,
             const typename RTraits<MODE>::Tc* __restrict__ Chi,
             const typename RTraits<MODE>::Tc* __restrict__ Clo, int K,
             typename RTraits<MODE>::Tout* U, int64_t ldu, int vec_store,
             const typename RTraits<MODE>::Tout* __restrict__ Xt, int64_t ldxt,
             double* __restrict__ ss_partial,
             int n_rowtiles, int n_fchunks, int frames_per_chunk)
{
    typedef RTraits<MODE> Tr;
    typedef typename Tr::Tc Tc;
    typedef typename Tr::Tout Tout;
    typedef typename Tr::V V;
    constexpr int KW = Tr::KW;
    constexpr int KGMAX = RECON_MAX_RP / KW;
    constexpr int FC = FCB * 16;
    constexpr int CPAD = 16 / sizeof(Tc);               // 16-byte row pad in LDS
    constexpr int CLD = RECON_MAX_RP + CPAD;
    constexpr bool X3 = (MODE == DMD_RECON_BF16X3);
    constexpr int WG_ROWS = 4 * RBW * 16;

    __shared__ __align__(16) Tc Cs_hi[FC * CLD];
    __shared__ __align__(16) Tc Cs_lo[X3 ? FC * CLD : 1];
    __shared__ __align__(16) Tout Ost[4][16 * (16 * RBW + 16 / sizeof(Tout))];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lg = lane >> 4;
    const int nkg = rp / KW;
    const int cld = rp + CPAD;          // LDS leading dimension actually used

    AFrag<MODE> a[RBW][KGMAX];
    int cur_rt = -1;
    double ss = 0.0;
    const int64_t n_items = (int64_t)n_rowtiles * n_fchunks;

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int rt = (int)(item / n_fchunks);
        const int fc = (int)(item % n_fchunks);
        const int64_t tile_row0 = (int64_t)rt * WG_ROWS + wave * RBW * 16;
        if (rt != cur_rt) {
            load_tile_a<MODE, RBW, KGMAX>(a, phi, ldphi, N, tile_row0, nkg, l16, lg);
            cur_rt = rt;
        }
        const int f_begin = fc * frames_per_chunk;
        const int f_end = min(K, f_begin + frames_per_chunk);
        for (int f0 = f_begin; f0 < f_end; f0 += FC) {
            __syncthreads();
            // ---- stage coefficients of frames [f0, f0 + FC) (zero-padded rows exist up to Kp)
            {
                constexpr int VE = 16 / sizeof(Tc);       // elements per 16-byte move
                const int per_row = rp / VE;
                for (int idx = tid; idx < FC * per_row; idx += 256) {
                    const int fr = idx / per_row, c = (idx % per_row) * VE;
                    const int64_t src = (int64_t)(f0 + fr) * rp + c;
                    *reinterpret_cast<float4*>(&Cs_hi[fr * cld + c]) = *reinterpret_cast<const float4*>(&Chi[src]);
                    if constexpr (X3)
                        *reinterpret_cast<float4*>(&Cs_lo[fr * cld + c]) = *reinterpret_cast<const float4*>(&Clo[src]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int cb = 0; cb < FCB; ++cb) {
                V acc[RBW];
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb) acc[rb] = zero_acc<V>();
                const Tc* crow_hi = Cs_hi + (cb * 16 + l16) * cld;
                const Tc* crow_lo = Cs_lo + (cb * 16 + l16) * cld;
#pragma unroll
                for (int kg = 0; kg < KGMAX; ++kg) {
                    if (kg < nkg) {
                        if constexpr (MODE == DMD_RECON_FP32 || MODE == DMD_RECON_FP64) {
                            const Tc* bp = crow_hi + kg * 16 + 4 * lg;
                            Tc bv[4];
                            if constexpr (MODE == DMD_RECON_FP32) {
                                float4 x = *reinterpret_cast<const float4*>(bp);
                                bv[0] = x.x; bv[1] = x.y; bv[2] = x.z; bv[3] = x.w;
                            } else {
                                double2 x = reinterpret_cast<const double2*>(bp)[0];
                                double2 y = reinterpret_cast<const double2*>(bp)[1];
                                bv[0] = x.x; bv[1] = x.y; bv[2] = y.x; bv[3] = y.y;
                            }
#pragma unroll
                            for (int s = 0; s < 4; ++s)
#pragma unroll
                                for (int rb = 0; rb < RBW; ++rb)
                                    acc[rb] = mfma(a[rb][kg].v[s], bv[s], acc[rb]);
                        } else {
                            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(crow_hi + kg * 32 + 8 * lg);
                            if constexpr (X3) {
                                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(crow_lo + kg * 32 + 8 * lg);
#pragma unroll
                                for (int rb = 0; rb < RBW; ++rb) {
                                    acc[rb] = mfma_bf16(a[rb][kg].lo, bh, acc[rb]);
                                    acc[rb] = mfma_bf16(a[rb][kg].hi, bl, acc[rb]);
                                    acc[rb] = mfma_bf16(a[rb][kg].hi, bh, acc[rb]);
                                }
                            } else {
#pragma unroll
                                for (int rb = 0; rb < RBW; ++rb)
                                    acc[rb] = mfma_bf16(a[rb][kg].hi, bh, acc[rb]);
                            }
                        }
                    }
                }
                recon_store<Tout, V, RBW, RESID>(acc, Ost[wave], lane, f0 + cb * 16, f_end, tile_row0, N,
                                                 U, ldu, vec_store, Xt, ldxt, ss);
            }
        }
    }
    if constexpr (RESID) {
        __shared__ double red[4];
        ss = wave_sum(ss);
        if (lane == 0) red[wave] = ss;
        __syncthreads();
        if (tid == 0) ss_partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// ---------------------------------------------------------------- launch
static int g_cu_count = 0;
int device_cu_count()
{
    if (g_cu_count == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 256;
        g_cu_count = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
    }
    return g_cu_count;
}

template <int MODE, int RBW, int FCB, bool RESID>
static hipError_t launch_recon_t(hipStream_t s, const ReconArgs& ra, int grid_per_cu)
{
    typedef RTraits<MODE> Tr;
    constexpr int WG_ROWS = 4 * RBW * 16;
    constexpr int FC = FCB * 16;
    const int n_rowtiles = (int)ceil_div(ra.N, WG_ROWS);
    const int max_grid = device_cu_count() * grid_per_cu;
    const int n_fc = (int)ceil_div(ra.K, FC);               // items are single chunks of FC frames
    const int64_t items = (int64_t)n_rowtiles * n_fc;
    const int64_t ipw = ceil_div(items, (int64_t)max_grid);
    const int grid = (int)ceil_div(items, ipw);
    hipLaunchKernelGGL((recon_kernel<MODE, RBW, FCB, RESID>), dim3(grid), dim3(256), 0, s,
                       (const typename Tr::Tphi*)ra.phi, ra.ldphi, ra.N, ra.rp,
                       (const typename Tr::Tc*)ra.c_hi, (const typename Tr::Tc*)ra.c_lo, ra.K,
                       (typename Tr::Tout*)ra.U, ra.ldu, ra.vec_store,
                       (const typename Tr::Tout*)ra.xt, ra.ldxt, ra.ss_partial,
                       n_rowtiles, n_fc, (int)ipw);
    if (ra.grid_out) *ra.grid_out = grid;
    return hipGetLastError();
}

template <int MODE, int RBW, int FCB, bool RESID>
static hipError_t launch_recon_sb(hipStream_t s, const ReconArgs& ra, int grid_per_cu)
{
    typedef RTraits<MODE> Tr;
    constexpr int WG_ROWS = 4 * RBW * 16;
    constexpr int FC = FCB * 16;
    const int n_rowtiles = (int)ceil_div(ra.N, WG_ROWS);
    const int max_grid = device_cu_count() * grid_per_cu;
    int n_fchunks = 1;
    const int max_fchunks = (int)ceil_div(ra.K, FC);
    if (n_rowtiles < 2 * max_grid) n_fchunks = (int)std::min<int64_t>(max_fchunks, ceil_div(2 * max_grid, n_rowtiles));
    if (n_fchunks < 1) n_fchunks = 1;
    const int fpc = (int)round_up(ceil_div(ra.K, n_fchunks), FC);
    n_fchunks = (int)ceil_div(ra.K, fpc);
    const int64_t items = (int64_t)n_rowtiles * n_fchunks;
    const int grid = (int)std::min<int64_t>(items, max_grid);
    hipLaunchKernelGGL((recon_kernel_sb<MODE, RBW, FCB, RESID>), dim3(grid), dim3(256), 0, s,
                       (const typename Tr::Tphi*)ra.phi, ra.ldphi, ra.N, ra.rp,
                       (const typename Tr::Tc*)ra.c_hi, (const typename Tr::Tc*)ra.c_lo, ra.K,
                       (typename Tr::Tout*)ra.U, ra.ldu, ra.vec_store,
                       (const typename Tr::Tout*)ra.xt, ra.ldxt, ra.ss_partial,
                       n_rowtiles, n_fchunks, fpc);
    if (ra.grid_out) *ra.grid_out = grid;
    return hipGetLastError();
}

// Tile-shape candidates (index = autotuner config id): <row blocks per wave, frame
// blocks per item>, work-groups per CU.
template <bool RESID>
static hipError_t dispatch_recon(hipStream_t s, const ReconArgs& ra, int cfg)
{
    switch (ra.mode) {
    case DMD_RECON_FP64:
        switch (cfg) {
        case 1: return launch_recon_t<DMD_RECON_FP64, 1, 1, RESID>(s, ra, 2);
        case 2: return launch_recon_t<DMD_RECON_FP64, 2, 2, RESID>(s, ra, 1);
        case 3: return launch_recon_t<DMD_RECON_FP64, 1, 2, RESID>(s, ra, 1);
        case 4: return launch_recon_t<DMD_RECON_FP64, 1, 1, RESID>(s, ra, 4);
        case 5: return launch_recon_sb<DMD_RECON_FP64, 1, 2, RESID>(s, ra, 2);
        default: return launch_recon_t<DMD_RECON_FP64, 1, 2, RESID>(s, ra, 2);
        }
    case DMD_RECON_FP32:
        switch (cfg) {
        case 1: return launch_recon_t<DMD_RECON_FP32, 1, 2, RESID>(s, ra, 4);
        case 2: return launch_recon_t<DMD_RECON_FP32, 2, 4, RESID>(s, ra, 2);
        case 3: return launch_recon_t<DMD_RECON_FP32, 2, 2, RESID>(s, ra, 1);
        case 4: return launch_recon_t<DMD_RECON_FP32, 1, 4, RESID>(s, ra, 3);
        case 5: return launch_recon_sb<DMD_RECON_FP32, 2, 2, RESID>(s, ra, 2);
        default: return launch_recon_t<DMD_RECON_FP32, 2, 2, RESID>(s, ra, 2);
        }
    case DMD_RECON_BF16:
        switch (cfg) {
        case 1: return launch_recon_t<DMD_RECON_BF16, 2, 2, RESID>(s, ra, 4);
        case 2: return launch_recon_t<DMD_RECON_BF16, 4, 4, RESID>(s, ra, 2);
        case 3: return launch_recon_t<DMD_RECON_BF16, 2, 4, RESID>(s, ra, 3);
        case 4: return launch_recon_t<DMD_RECON_BF16, 4, 2, RESID>(s, ra, 1);
        case 5: return launch_recon_sb<DMD_RECON_BF16, 4, 2, RESID>(s, ra, 2);
        default: return launch_recon_t<DMD_RECON_BF16, 4, 2, RESID>(s, ra, 2);
        }
    default:
        switch (cfg) {
        case 1: return launch_recon_t<DMD_RECON_BF16X3, 2, 2, RESID>(s, ra, 4);
        case 2: return launch_recon_t<DMD_RECON_BF16X3, 4, 4, RESID>(s, ra, 2);
        case 3: return launch_recon_t<DMD_RECON_BF16X3, 2, 4, RESID>(s, ra, 3);
        case 4: return launch_recon_t<DMD_RECON_BF16X3, 4, 2, RESID>(s, ra, 1);
        case 5: return launch_recon_sb<DMD_RECON_BF16X3, 4, 2, RESID>(s, ra, 2);
        default: return launch_recon_t<DMD_RECON_BF16X3, 4, 2, RESID>(s, ra, 2);
        }
    }
}

hipError_t recon_launch(hipStream_t s, const ReconArgs& ra, int cfg)
{
    if (ra.N <= 0 || ra.K <= 0) return hipSuccess;
    return ra.xt ? dispatch_recon<true>(s, ra, cfg) : dispatch_recon<false>(s, ra, cfg);
}

hipError_t powers_pack(hipStream_t s, const double* lam, const double* b, const int32_t* kind, int r,
                       const double* expo, int K, int Kp, int rp, int mode, void* hi, void* lo, int32_t* status)
{
    const int64_t tot = (int64_t)Kp * rp;
    const int blocks = (int)std::min<int64_t>(ceil_div(tot, 256), 2048);
    hipLaunchKernelGGL(powers_pack_kernel, dim3(blocks), dim3(256), 0, s, lam, b, kind, r, expo, K,
                       Kp, rp, mode, hi, lo, status);
    return hipGetLastError();
}

hipError_t exponents(hipStream_t s, const int64_t* k, const double* t, double inv_dt, int K, double* e)
{
    hipLaunchKernelGGL(exponents_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(K, 256), 256)), dim3(256), 0, s,
                       k, t, inv_dt, K, e);
    return hipGetLastError();
}

}  // namespace dmd
