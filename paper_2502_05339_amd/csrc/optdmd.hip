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
                                double* __restrict__ Phi, double* __restrict__ E, const int32_t* __restrict__ run)
{
    if (*run == 0) return;
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
                                   double* __restrict__ G, double* __restrict__ g, const int32_t* __restrict__ run)
{
    if (*run == 0) return;
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
                                                                 int64_t lda, double* __restrict__ out,
                                                                 const int32_t* __restrict__ run)
{
    if (*run == 0) return;
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

// A = G + mu diag(G) (a small floor keeps the diagonal positive); clears the status
// words of the Cholesky factorisation that follows
__global__ void __launch_bounds__(256) vp_damp_kernel(int r, const double* __restrict__ G,
                                                      const double* __restrict__ mu_p, double* __restrict__ A,
                                                      const int32_t* __restrict__ run, int32_t* __restrict__ scr)
{
    if (*run == 0) return;
    if (blockIdx.x == 0 && threadIdx.x < 2) scr[threadIdx.x] = 0;
    const double mu = *mu_p;
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

// trial point theta - delta; keeps the status of the damped solve and clears the status
// words for the trial's own factorisation
__global__ void vp_update_kernel(int r, const double* __restrict__ theta, const double* __restrict__ delta,
                                 double* __restrict__ out, const int32_t* __restrict__ run,
                                 int32_t* __restrict__ scr, int32_t* __restrict__ ist)
{
    if (*run == 0) return;
    for (int c = threadIdx.x; c < r; c += blockDim.x) out[c] = theta[c] - delta[c];
    if (threadIdx.x == 0) {
        ist[VP_DAMPED] = scr[0];
        scr[0] = 0;
        scr[1] = 0;
    }
}

// ---- the iteration's control, on the device.  A trial point is evaluated only while
// ist[VP_RUN] is set; vp_decide_kernel takes the keep / reject decision and the stopping
// rule from the device values alone, so the sequence of launches is the same whatever
// the outcome (and can be captured).
__global__ void vp_begin_kernel(const int32_t* __restrict__ fit_info, int32_t* __restrict__ ist,
                                int32_t* __restrict__ scr)
{
    const int i = threadIdx.x;
    if (i < VP_IST_WORDS) ist[i] = i == VP_FIT_OK || i == VP_APPLY ? (fit_info[0] == 0 ? 1 : 0) : 0;
    if (i < 16) scr[i] = 0;
}

__global__ void vp_start_kernel(const double* __restrict__ cost0, const int32_t* __restrict__ scr,
                                int32_t* __restrict__ ist, double* __restrict__ vst)
{
    if (threadIdx.x != 0 || ist[VP_APPLY] == 0) return;
    const double c = *cost0;
    const bool ok = scr[0] == 0 && isfinite(c);
    ist[VP_APPLY] = ok ? 1 : 0;      // a singular or non-finite start leaves the plain fit
    ist[VP_RUN] = ok ? 1 : 0;
    vst[VP_COST] = c;
    vst[VP_MU] = VP_MU0;
}

__global__ void vp_decide_kernel(const double* __restrict__ cost_t, const int32_t* __restrict__ scr,
                                 int32_t* __restrict__ ist, double* __restrict__ vst)
{
    if (threadIdx.x != 0) return;
    if (ist[VP_RUN] == 0) { ist[VP_ACCEPT] = 0; return; }
    ist[VP_TRIALS] += 1;
    const double c_new = *cost_t, cost = vst[VP_COST];
    double mu = vst[VP_MU];
    if (ist[VP_DAMPED] == 0 && scr[0] == 0 && isfinite(c_new) && c_new < cost) {
        const double gain = cost - c_new;
        vst[VP_COST] = c_new;
        vst[VP_MU] = fmax(mu * 0.25, VP_MU_MIN);
        ist[VP_ACCEPT] = 1;
        ist[VP_TRIES] = 0;
        ist[VP_STEPS] += 1;
        if (gain <= VP_GAIN_TOL * c_new || ist[VP_STEPS] >= VP_MAX_STEPS) ist[VP_RUN] = 0;
    } else {
        mu *= 4.0;
        vst[VP_MU] = mu;
        ist[VP_ACCEPT] = 0;
        ist[VP_TRIES] += 1;
        if (ist[VP_TRIES] >= VP_MAX_TRIES || mu > VP_MU_MAX) ist[VP_RUN] = 0;
    }
}

// a kept trial point becomes the current one: theta, [B | F], J^T J and J^T r
__global__ void vp_commit_kernel(int r, const int32_t* __restrict__ ist, const double* __restrict__ theta_t,
                                 double* __restrict__ theta_c, const double* __restrict__ bf_t,
                                 double* __restrict__ bf_c, const double* __restrict__ G_t, double* __restrict__ G_c,
                                 const double* __restrict__ g_t, double* __restrict__ g_c)
{
    if (ist[VP_ACCEPT] == 0) return;
    const int64_t rr = (int64_t)r * r, tot = 3 * rr + 2 * (int64_t)r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < 2 * rr) bf_c[e] = bf_t[e];
        else if (e < 3 * rr) G_c[e - 2 * rr] = G_t[e - 2 * rr];
        else if (e < 3 * rr + r) g_c[e - 3 * rr] = g_t[e - 3 * rr];
        else theta_c[e - 3 * rr - r] = theta_t[e - 3 * rr - r];
    }
}

// info[4] kept steps, info[5] trial points, info[6] outcome (0 stopped by its rule, 1 still
// running when the trial points ran out, 2 not applied: singular or non-finite start)
__global__ void vp_finish_kernel(const int32_t* __restrict__ ist, int32_t* __restrict__ info)
{
    if (threadIdx.x != 0 || ist[VP_FIT_OK] == 0) return;
    info[4] = ist[VP_STEPS];
    info[5] = ist[VP_TRIALS];
    info[6] = ist[VP_APPLY] == 0 ? 2 : (ist[VP_RUN] != 0 ? 1 : 0);
}

// eigenvalues, amplitudes and column scales of the lifted modes (eq. phi_optdmd): with
// M = U_r B^T, a pair's complex mode times amplitude is w = (M_c - i M_{c+1}) / 2, so
// b = ||w|| = sqrt(||B_c||^2 + ||B_{c+1}||^2) / 2 (U_r has orthonormal columns) and the
// folded columns are M_c / (2 b) and -M_{c+1} / (2 b); a real mode has b = ||B_c||.
__global__ void vp_lift_kernel(int r, const int32_t* __restrict__ kind, const double* __restrict__ theta,
                               const double* __restrict__ B, double* __restrict__ lam, double* __restrict__ b,
                               double* __restrict__ scale, const int32_t* __restrict__ run)
{
    if (*run == 0) return;
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
hipError_t vp_basis(hipStream_t s, int T, int r, const double* theta, const int32_t* kind, double* Phi, double* E,
                    const int32_t* run)
{
    const int blocks = (int)std::min<int64_t>(ceil_div((int64_t)T * r, 256), 1024);
    hipLaunchKernelGGL(vp_basis_kernel, dim3(blocks), dim3(256), 0, s, T, r, theta, kind, Phi, E, run);
    return hipGetLastError();
}
hipError_t vp_assemble(hipStream_t s, int r, const int32_t* kind, const double* K, const double* W, const double* H,
                       double* G, double* g, const int32_t* run)
{
    const int blocks = (int)ceil_div((int64_t)r * r, 256);
    hipLaunchKernelGGL(vp_assemble_kernel, dim3(blocks), dim3(256), 0, s, r, kind, K, W, H, G, g, run);
    return hipGetLastError();
}
hipError_t vp_sumsq(hipStream_t s, int m, int n, const double* A, int64_t lda, double* out, const int32_t* run)
{
    hipLaunchKernelGGL(vp_sumsq_kernel, dim3(1), dim3(VP_SS_THREADS), 0, s, m, n, A, lda, out, run);
    return hipGetLastError();
}
hipError_t vp_damp(hipStream_t s, int r, const double* G, const double* mu, double* A, const int32_t* run,
                   int32_t* scr)
{
    const int blocks = (int)ceil_div((int64_t)r * r, 256);
    hipLaunchKernelGGL(vp_damp_kernel, dim3(blocks), dim3(256), 0, s, r, G, mu, A, run, scr);
    return hipGetLastError();
}
hipError_t vp_update(hipStream_t s, int r, const double* theta, const double* delta, double* out, const int32_t* run,
                     int32_t* scr, int32_t* ist)
{
    hipLaunchKernelGGL(vp_update_kernel, dim3(1), dim3(256), 0, s, r, theta, delta, out, run, scr, ist);
    return hipGetLastError();
}
hipError_t vp_lift(hipStream_t s, int r, const int32_t* kind, const double* theta, const double* B, double* lam,
                   double* b, double* scale, const int32_t* run)
{
    hipLaunchKernelGGL(vp_lift_kernel, dim3(1), dim3(256), 0, s, r, kind, theta, B, lam, b, scale, run);
    return hipGetLastError();
}
hipError_t vp_begin(hipStream_t s, const int32_t* fit_info, int32_t* ist, int32_t* scr)
{
    hipLaunchKernelGGL(vp_begin_kernel, dim3(1), dim3(64), 0, s, fit_info, ist, scr);
    return hipGetLastError();
}
hipError_t vp_start(hipStream_t s, const double* cost0, const int32_t* scr, int32_t* ist, double* vst)
{
    hipLaunchKernelGGL(vp_start_kernel, dim3(1), dim3(64), 0, s, cost0, scr, ist, vst);
    return hipGetLastError();
}
hipError_t vp_decide(hipStream_t s, const double* cost_t, const int32_t* scr, int32_t* ist, double* vst)
{
    hipLaunchKernelGGL(vp_decide_kernel, dim3(1), dim3(64), 0, s, cost_t, scr, ist, vst);
    return hipGetLastError();
}
hipError_t vp_commit(hipStream_t s, int r, const int32_t* ist, const double* theta_t, double* theta_c,
                     const double* bf_t, double* bf_c, const double* G_t, double* G_c, const double* g_t, double* g_c)
{
    const int blocks = (int)std::min<int64_t>(ceil_div(3 * (int64_t)r * r + 2 * r, 256), 256);
    hipLaunchKernelGGL(vp_commit_kernel, dim3(blocks), dim3(256), 0, s, r, ist, theta_t, theta_c, bf_t, bf_c, G_t, G_c,
                       g_t, g_c);
    return hipGetLastError();
}
hipError_t vp_finish(hipStream_t s, const int32_t* ist, int32_t* info)
{
    hipLaunchKernelGGL(vp_finish_kernel, dim3(1), dim3(64), 0, s, ist, info);
    return hipGetLastError();
}

}  // namespace dmd
