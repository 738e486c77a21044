// Forced reduced roll-out (Sec. 4.6, eq. external_forces, DMD with control):
// z_{s+1} = Lambda z_s + dt g_s with g_s = Phi^+ f_s, then frames Re(Phi z_s).
#include "common.h"
#include "kernels.h"

namespace dmd {

// Complex projection g_s of mode i from the real least-squares coefficients beta(:, s)
// of the folded basis (a pair (i, i+1) has b_i = (beta_i - i beta_{i+1}) / 2).
__device__ __forceinline__ cplx proj_coeff(const double* beta, int64_t ldb, const int32_t* kind, int r, int i,
                                           int s)
{
    const double* bc = beta + (int64_t)s * ldb;
    int kd = kind[i];
    if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;
    if (kd == 0) return {bc[i], 0.0};
    if (kd == 1) return {0.5 * bc[i], -0.5 * bc[i + 1]};
    return {0.5 * bc[i - 1], 0.5 * bc[i]};
}

// One 64-lane work-group per mode.  Lane l owns steps [l C, (l+1) C), C = ceil(T / 64):
// it first runs its steps from a zero state, giving the affine map z -> lambda^len z + w
// of its chunk; lane 0 chains the 64 maps from z_0 into each chunk's incoming state;
// then every lane reruns its steps from that state and writes z_{s+1}.
__global__ void __launch_bounds__(64)
rollout_scan_kernel(int r, int T, const double* __restrict__ lam, const double* __restrict__ z0,
                    const double* __restrict__ beta, int64_t ldb, const int32_t* __restrict__ kind, double dt,
                    double* __restrict__ states)
{
    __shared__ cplx amap[64], wmap[64], cin[64];
    const int i = blockIdx.x, lane = threadIdx.x;
    const cplx lm = {lam[2 * i], lam[2 * i + 1]};
    const int C = (T + 63) / 64;
    const int s0 = min(lane * C, T), s1 = min(s0 + C, T);
    cplx a = {1.0, 0.0}, w = {0.0, 0.0};
    for (int s = s0; s < s1; ++s) {
        w = cmul(lm, w);
        if (beta) {
            const cplx g = proj_coeff(beta, ldb, kind, r, i, s);
            w.re = fma(dt, g.re, w.re);
            w.im = fma(dt, g.im, w.im);
        }
        a = cmul(lm, a);
    }
    amap[lane] = a;
    wmap[lane] = w;
    __syncthreads();
    if (lane == 0) {
        cplx z = {z0[2 * i], z0[2 * i + 1]};
        for (int l = 0; l < 64; ++l) {
            cin[l] = z;
            z = cadd(cmul(amap[l], z), wmap[l]);
        }
    }
    __syncthreads();
    cplx z = cin[lane];
    if (lane == 0) {
        states[2 * i] = z.re;
        states[2 * i + 1] = z.im;
    }
    for (int s = s0; s < s1; ++s) {
        z = cmul(lm, z);
        if (beta) {
            const cplx g = proj_coeff(beta, ldb, kind, r, i, s);
            z.re = fma(dt, g.re, z.re);
            z.im = fma(dt, g.im, z.im);
        }
        double* o = states + 2 * ((int64_t)(s + 1) * r + i);
        o[0] = z.re;
        o[1] = z.im;
    }
}

// Coefficients of the reconstruction GEMM from reduced states (frame j = state j), in
// the folded basis: kind 0 -> Re z_i; a pair (i, i+1) -> Re z_i + Re z_{i+1} and
// Im z_{i+1} - Im z_i, so that Re(Phi z) = sum_i phi_folded_i C_i.  A coefficient beyond
// the output type's finite range sets COEF_OVERFLOW in *status.
__global__ void pack_states_kernel(const double* __restrict__ states, const int32_t* __restrict__ kind, int r,
                                   int K, int Kp, int rp, int mode, void* out_hi, void* out_lo, int32_t* status)
{
    const int64_t tot = (int64_t)Kp * rp;
    const double vmax = mode == DMD_RECON_FP64 ? 1.7976931348623157e308 : 3.4028234663852886e38;
    int flags = 0;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % rp);
        const int j = (int)(idx / rp);
        double v = 0.0;
        if (i < r && j < K) {
            const double* z = states + 2 * (int64_t)j * r;
            int kd = kind[i];
            if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;
            if (kd == 0) v = z[2 * i];
            else if (kd == 1) v = z[2 * i] + z[2 * i + 2];
            else v = z[2 * i + 1] - z[2 * i - 1];
            if (!(fabs(v) <= vmax)) flags |= COEF_OVERFLOW;
        }
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

hipError_t rollout_scan(hipStream_t s, int r, int T, const double* lam, const double* z0, const double* beta,
                        int64_t ldb, const int32_t* kind, double dt, double* states)
{
    hipLaunchKernelGGL(rollout_scan_kernel, dim3(r), dim3(64), 0, s, r, T, lam, z0, beta, ldb, kind, dt, states);
    return hipGetLastError();
}

hipError_t pack_states(hipStream_t s, const double* states, const int32_t* kind, int r, int K, int Kp, int rp,
                       int mode, void* hi, void* lo, int32_t* status)
{
    const int64_t tot = (int64_t)Kp * rp;
    const int blocks = (int)std::min<int64_t>(ceil_div(tot, 256), 2048);
    hipLaunchKernelGGL(pack_states_kernel, dim3(blocks), dim3(256), 0, s, states, kind, r, K, Kp, rp, mode, hi, lo,
                       status);
    return hipGetLastError();
}

}  // namespace dmd
