// OptDMD by variable projection (Sec. 4.2, eq. variable_projection and eq. phi_optdmd),
// in real arithmetic on the folded basis.  For real data the eigenvalues come in
// conjugate pairs, so the T x r basis Phi(theta) holds, per pair (c, c+1) led by
// alpha = theta_c + i theta_{c+1}, the columns Re(alpha^t) and Im(alpha^t), and per real
// eigenvalue a the column a^t (t = 0 .. T-1).  theta has one entry per column.  With
// E the matching columns of t alpha^(t-1), the derivative of Phi with respect to
//   theta_c (real mode):      E_c in column c;
//   theta_c (pair, Re alpha): E_c in column c, E_{c+1} in column c+1;
//   theta_{c+1} (Im alpha):   -E_{c+1} in column c, E_c in column c+1.
// The Kaufman Jacobian of the projected residual is J_p = -P_perp (dPhi/dtheta_p) B, a
// sum of rank-one terms, so with E~ = P_perp E, K = E~^T E~, W = B B^T and H = E^T R B^T
//   (J^T J)_pq = sum g1 g2 K[s1, s2] W[c1, c2],   (J^T r)_p = -sum g H[s, c]
// over the (column c, source s, sign g) terms of p and q.
#include "common.h"
#include "kernels.h"

namespace dmd {

// the (column, source, sign) terms of parameter p; returns their number (1 or 2)
__device__ __forceinline__ int vp_terms(const int32_t* kind, int r, int p, int* col, int* src, double* sg)
{
    int kd = kind[p];
    if ((kd == 1 && p + 1 >= r) || (kd == 2 && p == 0) || kd < 0 || kd > 2) kd = 0;
    if (kd == 0) { col[0] = p; src[0] = p; sg[0] = 1.0; return 1; }
    if (kd == 1) {                                   // Re alpha of the pair (p, p+1)
        col[0] = p; src[0] = p; sg[0] = 1.0;
        col[1] = p + 1; src[1] = p + 1; sg[1] = 1.0;
        return 2;
    }
    col[0] = p - 1; src[0] = p; sg[0] = -1.0;        // Im alpha of the pair (p-1, p)
    col[1] = p; src[1] = p - 1; sg[1] = 1.0;
    return 2;
}

__global__ void vp_theta_init_kernel(int r, const double* __restrict__ lam, const int32_t* __restrict__ kind,
                                     double* __restrict__ theta)
{
    for (int c = threadIdx.x; c < r; c += blockDim.x) {
        int kd = kind[c];
        if ((kd == 1 && c + 1 >= r) || (kd == 2 && c == 0) || kd < 0 || kd > 2) kd = 0;
        theta[c] = kd == 2 ? lam[2 * (c - 1) + 1] : lam[2 * c];
    }
}

// Phi(theta) and E(theta), T x r column-major (ld T)
__global__ void vp_basis_kernel(int T, int r, const double* __restrict__ theta, const int32_t* __restrict__ kind,
                                double* __restrict__ Phi, double* __restrict__ E)
{
    const int64_t tot = (int64_t)T * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e % T), c = (int)(e / T);
        int kd = kind[c];
        if ((kd == 1 && c + 1 >= r) || (kd == 2 && c == 0) || kd < 0 || kd > 2) kd = 0;
        const int lead = kd == 2 ? c - 1 : c;
        const cplx al = {theta[lead], kd == 0 ? 0.0 : theta[lead + 1]};
        const cplx z = cpow_real(al, (double)t);
        const cplx w = t == 0 ? cplx{0.0, 0.0} : cpow_real(al, (double)(t - 1));
        const bool im = kd == 2;
        Phi[e] = im ? z.im : z.re;
        E[e] = (double)t * (im ? w.im : w.re);
    }
}

// G = J^T J and g = J^T r from K, W, H (r x r, column-major); one thread per entry of G
__global__ void vp_assemble_kernel(int r, const int32_t* __restrict__ kind, const double* __restrict__ K,
                                   const double* __restrict__ W, const double* __restrict__ H,
                                   double* __restrict__ G, double* __restrict__ g)
{
    const int64_t tot = (int64_t)r * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(e % r), q = (int)(e / r);
        int cp[2], sp[2], cq[2], sq[2];
        double gp[2], gq[2];
        const int np_ = vp_terms(kind, r, p, cp, sp, gp);
        const int nq = vp_terms(kind, r, q, cq, sq, gq);
        double s = 0.0;
        for (int a = 0; a < np_; ++a)
            for (int b = 0; b < nq; ++b)
                s += gp[a] * gq[b] * K[(int64_t)sq[b] * r + sp[a]] * W[(int64_t)cq[b] * r + cp[a]];
        G[e] = s;
        if (q == 0) {
            double h = 0.0;
            for (int a = 0; a < np_; ++a) h -= gp[a] * H[(int64_t)cp[a] * r + sp[a]];
            g[p] = h;
        }
    }
}

// sum of squares of an m x n column-major matrix into *out (one work-group of 1024
// threads, four loads in flight per thread, fixed-order combination)
constexpr int VP_SS_THREADS = 1024;
__global__ void __launch_bounds__(VP_SS_THREADS) vp_sumsq_kernel(int m, int n, const double* __restrict__ A,
                                                                 int64_t lda, double* __restrict__ out)
{
    __shared__ double part[VP_SS_THREADS / 64];
    const int64_t tot = (int64_t)m * n;
    double s = 0.0;
    for (int64_t e0 = threadIdx.x; e0 < tot; e0 += 4 * VP_SS_THREADS) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = e0 + (int64_t)u * VP_SS_THREADS;
            v[u] = e < tot ? A[(e / m) * lda + e % m] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s = fma(v[u], v[u], s);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < VP_SS_THREADS / 64; ++w) t += part[w];
        *out = t;
    }
}

// A = G + mu diag(G) (a small floor keeps the diagonal positive)
__global__ void __launch_bounds__(256) vp_damp_kernel(int r, const double* __restrict__ G, double mu,
                                                      double* __restrict__ A)
{
    __shared__ double part[4];
    const int64_t tot = (int64_t)r * r;
    double dm = 0.0;                                     // max of the diagonal, per work-group
    for (int i = threadIdx.x; i < r; i += blockDim.x) dm = fmax(dm, G[(int64_t)i * r + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = dm;
    __syncthreads();
    const double dmax = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % r), j = (int)(e / r);
        double v = G[e];
        if (i == j) v += mu * fmax(v, 1e-14 * dmax);
        A[e] = v;
    }
}

__global__ void vp_update_kernel(int r, const double* __restrict__ theta, const double* __restrict__ delta,
                                 double* __restrict__ out)
{
    for (int c = threadIdx.x; c < r; c += blockDim.x) out[c] = theta[c] - delta[c];
}

// eigenvalues, amplitudes and column scales of the lifted modes (eq. phi_optdmd): with
// M = U_r B^T, a pair's complex mode times amplitude is w = (M_c - i M_{c+1}) / 2, so
// b = ||w|| = sqrt(||B_c||^2 + ||B_{c+1}||^2) / 2 (U_r has orthonormal columns) and the
// folded columns are M_c / (2 b) and -M_{c+1} / (2 b); a real mode has b = ||B_c||.
__global__ void vp_lift_kernel(int r, const int32_t* __restrict__ kind, const double* __restrict__ theta,
                               const double* __restrict__ B, double* __restrict__ lam, double* __restrict__ b,
                               double* __restrict__ scale)
{
    for (int c = threadIdx.x; c < r; c += blockDim.x) {
        int kd = kind[c];
        if ((kd == 1 && c + 1 >= r) || (kd == 2 && c == 0) || kd < 0 || kd > 2) kd = 0;
        const int lead = kd == 2 ? c - 1 : c;
        double n2 = 0.0;
        for (int j = 0; j < r; ++j) n2 = fma(B[(int64_t)j * r + lead], B[(int64_t)j * r + lead], n2);
        if (kd != 0)
            for (int j = 0; j < r; ++j) n2 = fma(B[(int64_t)j * r + lead + 1], B[(int64_t)j * r + lead + 1], n2);
        const double amp = kd == 0 ? sqrt(n2) : 0.5 * sqrt(n2);
        const double inv = amp > 0.0 ? 1.0 / amp : 0.0;
        lam[2 * c] = theta[lead];
        lam[2 * c + 1] = kd == 0 ? 0.0 : (kd == 1 ? theta[lead + 1] : -theta[lead + 1]);
        b[2 * c] = amp;
        b[2 * c + 1] = 0.0;
        scale[c] = kd == 0 ? inv : (kd == 1 ? 0.5 * inv : -0.5 * inv);
    }
}

hipError_t vp_theta_init(hipStream_t s, int r, const double* lam, const int32_t* kind, double* theta)
{
    hipLaunchKernelGGL(vp_theta_init_kernel, dim3(1), dim3(256), 0, s, r, lam, kind, theta);
    return hipGetLastError();
}
hipError_t vp_basis(hipStream_t s, int T, int r, const double* theta, const int32_t* kind, double* Phi, double* E)
{
    const int blocks = (int)std::min<int64_t>(ceil_div((int64_t)T * r, 256), 1024);
    hipLaunchKernelGGL(vp_basis_kernel, dim3(blocks), dim3(256), 0, s, T, r, theta, kind, Phi, E);
    return hipGetLastError();
}
hipError_t vp_assemble(hipStream_t s, int r, const int32_t* kind, const double* K, const double* W, const double* H,
                       double* G, double* g)
{
    const int blocks = (int)ceil_div((int64_t)r * r, 256);
    hipLaunchKernelGGL(vp_assemble_kernel, dim3(blocks), dim3(256), 0, s, r, kind, K, W, H, G, g);
    return hipGetLastError();
}
hipError_t vp_sumsq(hipStream_t s, int m, int n, const double* A, int64_t lda, double* out)
{
    hipLaunchKernelGGL(vp_sumsq_kernel, dim3(1), dim3(VP_SS_THREADS), 0, s, m, n, A, lda, out);
    return hipGetLastError();
}
hipError_t vp_damp(hipStream_t s, int r, const double* G, double mu, double* A)
{
    const int blocks = (int)ceil_div((int64_t)r * r, 256);
    hipLaunchKernelGGL(vp_damp_kernel, dim3(blocks), dim3(256), 0, s, r, G, mu, A);
    return hipGetLastError();
}
hipError_t vp_update(hipStream_t s, int r, const double* theta, const double* delta, double* out)
{
    hipLaunchKernelGGL(vp_update_kernel, dim3(1), dim3(256), 0, s, r, theta, delta, out);
    return hipGetLastError();
}
hipError_t vp_lift(hipStream_t s, int r, const int32_t* kind, const double* theta, const double* B, double* lam,
                   double* b, double* scale)
{
    hipLaunchKernelGGL(vp_lift_kernel, dim3(1), dim3(256), 0, s, r, kind, theta, B, lam, b, scale);
    return hipGetLastError();
}

}  // namespace dmd
