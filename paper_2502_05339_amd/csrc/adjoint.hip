// Adjoint of the full-space reconstruction loss with the modes held fixed.
//
//   L(lambda, b) = sum_j || x_j - Re(Phi (b .* lambda^{k_j})) ||^2
//
// The residual R = X - Phi C (C the folded coefficients) and its FP64 sum of squares
// come from the reconstruction kernel's residual epilogue; G_f = Phi_f^T R (folded,
// r x ncols) from the TN GEMM.  grad_reduce_kernel turns G_f into the complex
// G = Phi^T R of every mode (a pair's second member has the conjugate column) and
// does the FP64 r-reductions
//   grad_b_i      = -2 conj( sum_j G_ij lambda_i^{k_j} )
//   grad_lambda_i = -2 conj( sum_j G_ij k_j b_i lambda_i^{k_j - 1} )
// in the complex-autograd convention (dL/dRe + i dL/dIm).
#include "common.h"
#include "kernels.h"

namespace dmd {

// One wave per mode, lanes over the frames: lane t takes frames t, t + 64, .. and the two
// sums finish with a fixed-shape wave reduction (the result does not depend on timing).
// Wave 0 of work-group 0 also sums the loss partials of the residual launch, in a fixed
// order.  lambda^e and e lambda^(e-1) are formed in FP64 as exp(e Log lambda) (the
// principal branch of the reconstruction); e lambda^(e-1) is zero for e = 0.
constexpr int GR_WAVES = 4;

__global__ void __launch_bounds__(64 * GR_WAVES)
grad_reduce_kernel(int r, int ncols, const double* __restrict__ G, const double* __restrict__ lam,
                   const double* __restrict__ b, const int32_t* __restrict__ kind, const double* __restrict__ expo,
                   const double* __restrict__ ss_partial, int nss, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * GR_WAVES + (threadIdx.x >> 6);
    if (blockIdx.x == 0 && (threadIdx.x >> 6) == 0) {
        double s = 0.0;
        for (int k = lane; k < nss; k += 64) s += ss_partial[k];
        s = wave_sum(s);
        if (lane == 0) out[0] = s;
    }
    if (i >= r) return;
    int kd = kind[i];
    if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;   // malformed pair marker
    const cplx li = {lam[2 * i], lam[2 * i + 1]};
    const cplx bi = {b[2 * i], b[2 * i + 1]};
    cplx sb = {0.0, 0.0}, sl = {0.0, 0.0};
    for (int j = lane; j < ncols; j += 64) {
        cplx g;
        if (kd == 0) g = {G[(int64_t)j * r + i], 0.0};
        else if (kd == 1) g = {G[(int64_t)j * r + i], G[(int64_t)j * r + i + 1]};
        else g = {G[(int64_t)j * r + i - 1], -G[(int64_t)j * r + i]};
        const double e = expo[j];
        sb = cadd(sb, cmul(g, cpow_real(li, e)));
        if (e != 0.0) {
            const cplx d = cmul({e, 0.0}, cpow_real(li, e - 1.0));
            sl = cadd(sl, cmul(g, d));
        }
    }
    sb.re = wave_sum(sb.re);
    sb.im = wave_sum(sb.im);
    sl.re = wave_sum(sl.re);
    sl.im = wave_sum(sl.im);
    if (lane == 0) {
        const cplx gl = cconj(cmul(sl, bi));
        out[1 + 2 * i] = -2.0 * gl.re;
        out[2 + 2 * i] = -2.0 * gl.im;
        out[1 + 2 * r + 2 * i] = -2.0 * sb.re;
        out[2 + 2 * r + 2 * i] = 2.0 * sb.im;
    }
}

hipError_t grad_reduce(hipStream_t s, int r, int ncols, const double* G, const double* lam,
                       const double* b, const int32_t* kind, const double* expo,
                       const double* ss_partial, int nss, double* out)
{
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)ceil_div(std::max(r, 1), GR_WAVES)), dim3(64 * GR_WAVES), 0, s,
                       r, ncols, G, lam, b, kind, expo, ss_partial, nss, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- refit statistics
// With the modes fixed, the loss and its adjoint need X only through G0 = Phi_f^T X,
// M = Phi_f^T Phi_f and ||X||^2:  with the folded FP64 coefficients C (r x ncols),
//   G_f = Phi_f^T (X - Phi_f C) = G0 - M C,
//   L   = ||X||^2 - 2 <C, G0> + <C, M C> = ||X||^2 - <C, G0 + G_f>,
// so a refit step costs O(r^2 ncols) once the three are formed (R is never formed).

// Sum of squares of an N x ncols column-major matrix: one FP64 partial per work-group
// (rows split into contiguous ranges, every column of a range in turn), summed in a
// fixed order inside the work-group.
constexpr int SQ_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(SQ_THREADS)
sumsq_kernel(const T* __restrict__ X, int64_t ld, int64_t N, int ncols, int64_t rows_per, double* partial)
{
    __shared__ double red[SQ_THREADS];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per;
    const int64_t r1 = min(N, r0 + rows_per);
    double s = 0.0;
    for (int j = 0; j < ncols; ++j) {
        const T* col = X + (int64_t)j * ld;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += SQ_THREADS) {
            const double v = (double)col[i];
            s = fma(v, v, s);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = SQ_THREADS / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t sumsq(hipStream_t s, int dtype, const void* X, int64_t ld, int64_t N, int ncols, double* partial,
                 int* nparts)
{
    const int64_t rows_per = sumsq_rows_per(N);
    const int nb = sumsq_parts(N);
    *nparts = nb;
    if (dtype == DMD_F32)
        hipLaunchKernelGGL(sumsq_kernel<float>, dim3(nb), dim3(SQ_THREADS), 0, s, (const float*)X, ld, N, ncols,
                           rows_per, partial);
    else
        hipLaunchKernelGGL(sumsq_kernel<double>, dim3(nb), dim3(SQ_THREADS), 0, s, (const double*)X, ld, N, ncols,
                           rows_per, partial);
    return hipGetLastError();
}

// loss[0] = sum(xx partials) - <C, G0 + Gf>, fixed-order
__global__ void __launch_bounds__(SQ_THREADS)
refit_loss_kernel(int r, int ncols, const double* __restrict__ C, const double* __restrict__ G0,
                  const double* __restrict__ Gf, const double* __restrict__ xxp, int nxx, double* loss)
{
    __shared__ double red[SQ_THREADS];
    const int64_t tot = (int64_t)r * ncols;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < tot; e += SQ_THREADS) s = fma(C[e], G0[e] + Gf[e], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = SQ_THREADS / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double xx = 0.0;
        for (int k = 0; k < nxx; ++k) xx += xxp[k];
        loss[0] = xx - red[0];
    }
}

hipError_t refit_loss(hipStream_t s, int r, int ncols, const double* C, const double* G0, const double* Gf,
                      const double* xxp, int nxx, double* loss)
{
    hipLaunchKernelGGL(refit_loss_kernel, dim3(1), dim3(SQ_THREADS), 0, s, r, ncols, C, G0, Gf, xxp, nxx, loss);
    return hipGetLastError();
}

}  // namespace dmd
