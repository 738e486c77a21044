// Adjoint of the full-space reconstruction loss with the modes held fixed.
//
//   L(lambda, b) = sum_j || x_j - Re(Phi (b .* lambda^{k_j})) ||^2
//
// The residual R = X - Phi C (C the folded coefficients) and its FP64 sum of squares
// come from the reconstruction kernel's residual epilogue; G_f = Phi_f^T R (folded,
// r x ncols) from the TN GEMM.  This kernel turns G_f into the complex
// G = Phi^T R of every mode (a pair's second member has the conjugate column) and
// does the FP64 r-reductions
//   grad_b_i      = -2 conj( sum_j G_ij lambda_i^{k_j} )
//   grad_lambda_i = -2 conj( sum_j G_ij k_j b_i lambda_i^{k_j - 1} )
// in the complex-autograd convention (dL/dRe + i dL/dIm).
#include "common.h"
#include "kernels.h"

namespace dmd {

__global__ void grad_reduce_kernel(int r, int ncols, const double* __restrict__ G,
                                   const double* __restrict__ lam, const double* __restrict__ b,
                                   const int32_t* __restrict__ kind, const double* __restrict__ expo,
                                   const double* __restrict__ ss_partial, int nss, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        double s = 0.0;
        for (int k = 0; k < nss; ++k) s += ss_partial[k];
        out[0] = s;
    }
    if (i >= r) return;
    int kd = kind[i];
    if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;   // malformed pair marker
    const cplx li = {lam[2 * i], lam[2 * i + 1]};
    const cplx bi = {b[2 * i], b[2 * i + 1]};
    cplx sb = {0.0, 0.0}, sl = {0.0, 0.0};
    for (int j = 0; j < ncols; ++j) {
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
    const cplx gl = cconj(cmul(sl, bi));
    out[1 + 2 * i] = -2.0 * gl.re;
    out[2 + 2 * i] = -2.0 * gl.im;
    out[1 + 2 * r + 2 * i] = -2.0 * sb.re;
    out[2 + 2 * r + 2 * i] = 2.0 * sb.im;
}

hipError_t grad_reduce(hipStream_t s, int r, int ncols, const double* G, const double* lam,
                       const double* b, const int32_t* kind, const double* expo,
                       const double* ss_partial, int nss, double* out)
{
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)ceil_div(r, 64)), dim3(64), 0, s, r, ncols, G,
                       lam, b, kind, expo, ss_partial, nss, out);
    return hipGetLastError();
}

}  // namespace dmd
