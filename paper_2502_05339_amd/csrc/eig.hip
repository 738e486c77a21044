// FP64 eigen-decomposition of the reduced operator Atilde W = W Lambda (Sec. 3.1).
//
// Real nonsymmetric n x n matrix (n <= DMD_MAX_RANK), three kernels:
//  1. hessenberg_kernel (1 work-group): Householder reduction A = Q H Q^T, H in
//     global scratch, the reflectors (v_k, tau_k) kept for rebuilding Q.
//  2. francis_kernel (ceil(n / nr) work-groups): every work-group holds H packed
//     in LDS (upper Hessenberg plus the two extra sub-diagonals a double-shift
//     bulge needs) and runs the same implicit double-shift QR iteration with
//     deflation, producing the real Schur form T; each work-group rebuilds and
//     updates only its own nr rows of the Schur vectors Z (Z = Q * product of
//     the QR reflectors), so no work-group ever waits for another.  2 x 2
//     diagonal blocks with real eigenvalues are split by a rotation.  Then the
//     eigenvectors of T are found by back-substitution (one wave per eigenvalue,
//     complex arithmetic for conjugate pairs), normalised to unit 2-norm (Z is
//     orthogonal, so the norm carries over) and multiplied by the work-group's
//     rows of Z.
//  3. sort_modes_kernel (1 work-group): canonical order (ascending |arg lambda|,
//     ties by descending |lambda|, Im > 0 member of a pair first), lambda, kind
//     and the permuted folded eigenvectors (pair -> [Re w, Im w], LAPACK storage).
#include "common.h"
#include "kernels.h"

namespace dmd {

// workspace layout (doubles unless noted)
struct EigWs {
    double* H;      // n x n
    double* V;      // n x n reflector vectors (column k: rows k+1..n-1)
    double* tau;    // n
    double* Wraw;   // n x n unsorted folded eigenvectors
    double* wr;     // n
    double* wi;     // n
    int32_t* kind0; // n
    double* X;      // grid x n x n per-work-group eigenvectors of T
};

static int eig_rows_per_wg(int n) { return n <= 64 ? 8 : 16; }
static int eig_grid(int n) { return (int)ceil_div(n, eig_rows_per_wg(n)); }

size_t eig_workspace_bytes(int n)
{
    size_t nn = (size_t)n * n;
    return (3 * nn + 4 * (size_t)n) * sizeof(double) + (size_t)n * sizeof(int32_t) + 64 +
           (size_t)eig_grid(n) * nn * sizeof(double) + 256;
}

static EigWs eig_carve(void* ws, int n)
{
    EigWs w;
    double* p = (double*)ws;
    size_t nn = (size_t)n * n;
    w.H = p; p += nn;
    w.V = p; p += nn;
    w.Wraw = p; p += nn;
    w.tau = p; p += n;
    w.wr = p; p += n;
    w.wi = p; p += n;
    p += n;
    w.kind0 = (int32_t*)p;
    p = (double*)((char*)p + round_up((int64_t)n * sizeof(int32_t), 64));
    w.X = p;
    return w;
}

// ====================================================================== 1. Hessenberg
__global__ void __launch_bounds__(1024)
hessenberg_kernel(const double* __restrict__ A, int64_t lda, int n, double* H, double* V, double* tau)
{
    __shared__ double sh_beta, sh_tau, sh_scale;
    __shared__ double red[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int64_t e = tid; e < (int64_t)n * n; e += blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        H[e] = A[(int64_t)j * lda + i];
        V[e] = 0.0;
    }
    for (int i = tid; i < n; i += blockDim.x) tau[i] = 0.0;
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        // reflector for x = H[k+1..n-1, k]
        double part = 0.0;
        for (int i = k + 2 + tid; i < n; i += blockDim.x) { const double v = H[(int64_t)k * n + i]; part += v * v; }
        part = wave_sum(part);
        if (lane == 0) red[wave] = part;
        __syncthreads();
        if (tid == 0) {
            double xn2 = 0.0;
            for (int w = 0; w < nw; ++w) xn2 += red[w];
            const double alpha = H[(int64_t)k * n + k + 1];
            if (xn2 == 0.0) {
                sh_tau = 0.0; sh_beta = alpha; sh_scale = 0.0;
            } else {
                const double nrm = sqrt(alpha * alpha + xn2);
                const double beta = alpha >= 0.0 ? -nrm : nrm;
                sh_tau = (beta - alpha) / beta;
                sh_scale = 1.0 / (alpha - beta);
                sh_beta = beta;
            }
        }
        __syncthreads();
        const double tk = sh_tau, sc = sh_scale;
        // v (v_0 = 1) into column k of V; H[k+1, k] = beta, below = 0
        for (int i = k + 1 + tid; i < n; i += blockDim.x)
            V[(int64_t)k * n + i] = (i == k + 1) ? 1.0 : H[(int64_t)k * n + i] * sc;
        __syncthreads();
        __threadfence_block();
        if (tk != 0.0) {
            const double* v = V + (int64_t)k * n;
            // left: H[k+1.., j] -= tau v (v^T H[k+1.., j]),  j = k+1 .. n-1  (one wave per column)
            for (int j = k + 1 + wave; j < n; j += nw) {
                double* col = H + (int64_t)j * n;
                double s = 0.0;
                for (int i = k + 1 + lane; i < n; i += 64) s += v[i] * col[i];
                s = wave_sum(s) * tk;
                for (int i = k + 1 + lane; i < n; i += 64) col[i] -= s * v[i];
            }
            __syncthreads();
            __threadfence_block();
            // right: H[i, k+1..] -= tau (H[i, k+1..] v) v^T,  all rows  (one wave per row)
            for (int i = wave; i < n; i += nw) {
                double s = 0.0;
                for (int j = k + 1 + lane; j < n; j += 64) s += H[(int64_t)j * n + i] * v[j];
                s = wave_sum(s) * tk;
                for (int j = k + 1 + lane; j < n; j += 64) H[(int64_t)j * n + i] -= s * v[j];
            }
            __syncthreads();
            __threadfence_block();
        }
        if (tid == 0) {
            tau[k] = tk;
            if (tk != 0.0) H[(int64_t)k * n + k + 1] = sh_beta;
        }
        for (int i = k + 2 + tid; i < n; i += blockDim.x) H[(int64_t)k * n + i] = 0.0;
        __syncthreads();
        __threadfence_block();
    }
}

// ====================================================================== 2. Francis QR
struct HP {   // packed Hessenberg with 3 sub-diagonals: column j holds rows 0..min(j+3, n-1)
    double* a;
    const int* cs;
    __device__ __forceinline__ double& operator()(int i, int j) const { return a[cs[j] + i]; }
};

__device__ __forceinline__ void house3(double x, double y, double z, double* v1, double* v2, double* tau, double* beta)
{
    const double nrm = sqrt(x * x + y * y + z * z);
    if (nrm == 0.0 || (y == 0.0 && z == 0.0)) { *tau = 0.0; *v1 = 0.0; *v2 = 0.0; *beta = x; return; }
    const double b = x >= 0.0 ? -nrm : nrm;
    *tau = (b - x) / b;
    const double sc = 1.0 / (x - b);
    *v1 = y * sc;
    *v2 = z * sc;
    *beta = b;
}

__global__ void __launch_bounds__(256)
francis_kernel(int n, int nr, const double* __restrict__ Hg, const double* __restrict__ Vg,
               const double* __restrict__ taug, double* Wraw, double* wr, double* wi, int32_t* kind0,
               double* Xall, int32_t* info)
{
    extern __shared__ double sm[];
    int* cs = reinterpret_cast<int*>(sm);                       // n + 1 ints
    int* blk = cs + (n + 1);                                    // n ints
    const int ioff = (int)round_up(2 * n + 1, 2) / 2;           // in doubles
    double* Hs = sm + ioff;
    __shared__ int sh_l, sh_stop, sh_iter_total;
    __shared__ double sh_v[4];   // rotation of a 2x2 block split
    __shared__ double sh_nxt[3]; // vector of the next bulge reflector
    __shared__ double sh_red[4];

    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    if (tid == 0) {
        int acc = 0;
        for (int j = 0; j < n; ++j) { cs[j] = acc; acc += min(j + 4, n); }
        cs[n] = acc;
    }
    __syncthreads();
    const int hsize = cs[n];
    double* Zs = Hs + hsize;                                    // nr x n
    double* xs = Zs + (int64_t)nr * n;                          // nw x 2n (eigenvector scratch)
    HP H{Hs, cs};
    const int r0 = blockIdx.x * nr;
    const int nrows = min(nr, n - r0);

    for (int j = 0; j < n; ++j)
        for (int i = tid; i <= min(j + 3, n - 1); i += nt) H(i, j) = (i <= j + 1) ? Hg[(int64_t)j * n + i] : 0.0;
    // Z slab = rows r0.. of Q = P_0 P_1 ... P_{n-3}: start from identity rows, apply reflectors on the right
    for (int e = tid; e < nr * n; e += nt) { const int rl = e / n, c = e % n; Zs[e] = (rl < nrows && r0 + rl == c) ? 1.0 : 0.0; }
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        const double tk = taug[k];
        if (tk == 0.0) continue;
        const double* v = Vg + (int64_t)k * n;
        for (int rl = wave; rl < nrows; rl += nw) {
            double* z = Zs + rl * n;
            double s = 0.0;
            for (int j = k + 1 + lane; j < n; j += 64) s += z[j] * v[j];
            s = wave_sum(s) * tk;
            for (int j = k + 1 + lane; j < n; j += 64) z[j] -= s * v[j];
        }
    }
    __syncthreads();

    // max |H_ij| (used when a diagonal pair is exactly zero, and for the pivot floor)
    {
        double mx = 0.0;
        for (int j = tid; j < n; j += nt)
            for (int i = 0; i <= min(j + 1, n - 1); ++i) mx = fmax(mx, fabs(H(i, j)));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) sh_red[wave] = mx;
        __syncthreads();
        if (tid == 0) { double m = 0.0; for (int w = 0; w < nw; ++w) m = fmax(m, sh_red[w]); sh_red[0] = m; }
        __syncthreads();
    }
    const double hnorm = sh_red[0];
    const double eps = 2.220446049250313e-16;
    int hi = n - 1;
    int its = 0;
    if (tid == 0) { sh_stop = 0; sh_iter_total = 0; }
    __syncthreads();
    while (hi >= 0) {
        // deflation point: largest l <= hi with negligible H(l, l-1)
        if (tid == 0) {
            int l = 0;
            for (int k = hi; k >= 1; --k) {
                double s = fabs(H(k - 1, k - 1)) + fabs(H(k, k));
                if (s == 0.0) s = hnorm;
                if (fabs(H(k, k - 1)) <= eps * s) { H(k, k - 1) = 0.0; l = k; break; }
            }
            sh_l = l;
        }
        __syncthreads();
        const int l = sh_l;
        if (l == hi) { hi -= 1; its = 0; __syncthreads(); continue; }
        if (l == hi - 1) {
            // 2x2 block (p, q): split it if its eigenvalues are real
            const int p = hi - 1, q = hi;
            if (tid == 0) {
                const double a = H(p, p), b = H(p, q), c = H(q, p), d = H(q, q);
                double cs_ = 1.0, sn_ = 0.0;
                bool rot = false;
                if (c != 0.0) {
                    const double hp = 0.5 * (a - d);
                    const double disc = hp * hp + b * c;
                    if (disc >= 0.0) {
                        const double sq = sqrt(disc);
                        const double mu = 0.5 * (a + d) + (hp >= 0.0 ? sq : -sq);
                        double e1 = b, e2 = mu - a;             // eigenvector (b, mu - a)
                        double f1 = mu - d, f2 = c;             // or (mu - d, c)
                        if (e1 * e1 + e2 * e2 < f1 * f1 + f2 * f2) { e1 = f1; e2 = f2; }
                        const double nr_ = sqrt(e1 * e1 + e2 * e2);
                        if (nr_ > 0.0) { cs_ = e1 / nr_; sn_ = e2 / nr_; rot = true; }
                    }
                }
                sh_v[0] = cs_; sh_v[1] = sn_; sh_v[2] = rot ? 1.0 : 0.0;
            }
            __syncthreads();
            if (sh_v[2] != 0.0) {
                const double c = sh_v[0], s = sh_v[1];
                // rows p, q <- G^T rows (columns p..n-1)
                for (int j = p + tid; j < n; j += nt) {
                    const double x = H(p, j), y = H(q, j);
                    H(p, j) = c * x + s * y;
                    H(q, j) = -s * x + c * y;
                }
                __syncthreads();
                // columns p, q <- columns G (rows 0..q)
                for (int i = tid; i <= q; i += nt) {
                    const double x = H(i, p), y = H(i, q);
                    H(i, p) = c * x + s * y;
                    H(i, q) = -s * x + c * y;
                }
                for (int rl = tid; rl < nrows; rl += nt) {
                    const double x = Zs[rl * n + p], y = Zs[rl * n + q];
                    Zs[rl * n + p] = c * x + s * y;
                    Zs[rl * n + q] = -s * x + c * y;
                }
                __syncthreads();
                if (tid == 0) H(q, p) = 0.0;
            }
            hi -= 2; its = 0;
            __syncthreads();
            continue;
        }
        ++its;
        if (tid == 0) { ++sh_iter_total; if (sh_iter_total > 40 * n) sh_stop = 1; }
        __syncthreads();
        if (sh_stop) break;
        // shifts: eigenvalues of the trailing 2x2 block (exceptional shifts at 10 and 20)
        double s, t;
        if (its == 10 || its == 20) {
            const double w = fabs(H(hi, hi - 1)) + (hi >= 2 ? fabs(H(hi - 1, hi - 2)) : 0.0);
            s = 2.0 * H(hi, hi) + 1.5 * w;
            t = (H(hi, hi) + 0.75 * w) * (H(hi, hi) + 0.75 * w);
        } else {
            s = H(hi - 1, hi - 1) + H(hi, hi);
            t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
        }
        // first column of (H - mu1)(H - mu2) on the active block
        double x = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
        double y = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
        double z = H(l + 1, l) * H(l + 2, l + 1);
        __syncthreads();   // every thread has read the shift inputs before H changes
        for (int k = l; k <= hi - 2; ++k) {
            if (k > l) { x = sh_nxt[0]; y = sh_nxt[1]; z = sh_nxt[2]; }
            double v1, v2, tk, beta;
            house3(x, y, z, &v1, &v2, &tk, &beta);
            if (tk != 0.0) {
                const int c0 = max(l, k - 1);
                // left: rows k..k+2, columns c0..n-1
                for (int j = c0 + tid; j < n; j += nt) {
                    double* hk = &H(k, j);
                    const double w = (hk[0] + v1 * hk[1] + v2 * hk[2]) * tk;
                    hk[0] -= w; hk[1] -= w * v1; hk[2] -= w * v2;
                }
            }
            __syncthreads();
            if (tk != 0.0) {
                if (tid == 0 && k > l) { H(k, k - 1) = beta; H(k + 1, k - 1) = 0.0; H(k + 2, k - 1) = 0.0; }
                // right: columns k..k+2, rows 0..min(k+3, hi)
                const int rmax = min(k + 3, hi);
                for (int i = tid; i <= rmax; i += nt) {
                    double& a0 = H(i, k);
                    double& a1 = H(i, k + 1);
                    double& a2 = H(i, k + 2);
                    const double w = (a0 + v1 * a1 + v2 * a2) * tk;
                    a0 -= w; a1 -= w * v1; a2 -= w * v2;
                }
                for (int rl = tid; rl < nrows; rl += nt) {
                    double* zr = Zs + rl * n + k;
                    const double w = (zr[0] + v1 * zr[1] + v2 * zr[2]) * tk;
                    zr[0] -= w; zr[1] -= w * v1; zr[2] -= w * v2;
                }
            }
            // the next reflector's vector is column k, rows k+1..k+3 (copied so that the
            // next left update may overwrite H while slower threads still read it)
            for (int i = tid; i <= min(k + 3, n - 1); i += nt)   // same row mapping as the update
                if (i >= k + 1) sh_nxt[i - k - 1] = (i <= hi) ? H(i, k) : 0.0;
            __syncthreads();
        }
        // final 2-vector reflector on rows / columns hi-1, hi
        {
            const int k = hi - 1;
            double xx, yy;
            if (k > l) { xx = sh_nxt[0]; yy = sh_nxt[1]; }
            else { xx = x; yy = y; }
            double v1, v2, tk, beta;
            house3(xx, yy, 0.0, &v1, &v2, &tk, &beta);
            if (tk != 0.0) {
                const int c0 = max(l, k - 1);
                for (int j = c0 + tid; j < n; j += nt) {
                    double* hk = &H(k, j);
                    const double w = (hk[0] + v1 * hk[1]) * tk;
                    hk[0] -= w; hk[1] -= w * v1;
                }
            }
            __syncthreads();
            if (tk != 0.0) {
                if (tid == 0 && k > l) { H(k, k - 1) = beta; H(k + 1, k - 1) = 0.0; }
                for (int i = tid; i <= hi; i += nt) {
                    double& a0 = H(i, k);
                    double& a1 = H(i, k + 1);
                    const double w = (a0 + v1 * a1) * tk;
                    a0 -= w; a1 -= w * v1;
                }
                for (int rl = tid; rl < nrows; rl += nt) {
                    double* zr = Zs + rl * n + k;
                    const double w = (zr[0] + v1 * zr[1]) * tk;
                    zr[0] -= w; zr[1] -= w * v1;
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    if (sh_stop) {
        if (blockIdx.x == 0 && tid == 0) set_status(info, DMD_ERR_EIG_NOCONV);
    }
    if (blockIdx.x == 0 && tid == 0 && info) atomicAdd(&info[2], sh_iter_total);

    // ---- block structure of T and eigenvalues
    if (tid == 0) {
        int k = 0;
        while (k < n) {
            if (k + 1 < n && H(k + 1, k) != 0.0) { blk[k] = 1; blk[k + 1] = 2; k += 2; }
            else { blk[k] = 0; k += 1; }
        }
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int k = tid; k < n; k += nt) {
            if (blk[k] == 0) { wr[k] = H(k, k); wi[k] = 0.0; kind0[k] = 0; }
            else {
                const int p = blk[k] == 1 ? k : k - 1;
                const double a = H(p, p), b = H(p, p + 1), c = H(p + 1, p), d = H(p + 1, p + 1);
                const double hp = 0.5 * (a - d);
                const double im = sqrt(fmax(-(hp * hp + b * c), 0.0));
                wr[k] = 0.5 * (a + d);
                wi[k] = blk[k] == 1 ? im : -im;
                kind0[k] = blk[k];
            }
        }
    }
    // ---- eigenvectors of T, one wave per eigenvalue unit; x in LDS scratch (re, im)
    double* X = Xall + (int64_t)blockIdx.x * n * n;
    __syncthreads();
    {
        double mx = 0.0;
        for (int j = tid; j < n; j += nt)
            for (int i = 0; i <= min(j + 1, n - 1); ++i) mx = fmax(mx, fabs(H(i, j)));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) sh_red[wave] = mx;
        __syncthreads();
        if (tid == 0) { double m = 0.0; for (int w = 0; w < nw; ++w) m = fmax(m, sh_red[w]); sh_red[0] = m; }
        __syncthreads();
    }
    const double tnorm = sh_red[0];
    const double smin = fmax(eps * tnorm, 1e-290);
    double* xr = xs + (int64_t)wave * 2 * n;
    double* xi = xr + n;
    for (int k = 0; k < n; ++k) {
        if (blk[k] == 2) continue;
        // unit owner: round-robin over units by wave
        int unit = 0;
        for (int u = 0; u < k; ++u) if (blk[u] != 2) ++unit;
        if (unit % nw != wave) continue;
        const bool pair = blk[k] == 1;
        const int top = pair ? k + 1 : k;
        double lre, lim;
        if (!pair) { lre = H(k, k); lim = 0.0; }
        else {
            const double a = H(k, k), b = H(k, k + 1), c = H(k + 1, k), d = H(k + 1, k + 1);
            const double hp = 0.5 * (a - d);
            lre = 0.5 * (a + d);
            lim = sqrt(fmax(-(hp * hp + b * c), 0.0));
        }
        for (int i = lane; i < n; i += 64) { xr[i] = 0.0; xi[i] = 0.0; }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            if (!pair) { xr[k] = 1.0; }
            else {
                const double a = H(k, k), b = H(k, k + 1), c = H(k + 1, k), d = H(k + 1, k + 1);
                // eigenvector of [[a b][c d]] for lre + i lim: (b, lambda - a) or (lambda - d, c)
                double e1r = b, e1i = 0.0, e2r = lre - a, e2i = lim;
                double f1r = lre - d, f1i = lim, f2r = c, f2i = 0.0;
                if (e1r * e1r + e2r * e2r + e2i * e2i < f1r * f1r + f1i * f1i + f2r * f2r) {
                    e1r = f1r; e1i = f1i; e2r = f2r; e2i = f2i;
                }
                xr[k] = e1r; xi[k] = e1i; xr[k + 1] = e2r; xi[k + 1] = e2i;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int i = k - 1;
        while (i >= 0) {
            const bool two = (blk[i] == 2);
            const int ia = two ? i - 1 : i;
            // r_row = -sum_{j = i+1 .. top} T(row, j) x_j   for row in {ia, i}
            double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
            for (int j = i + 1 + lane; j <= top; j += 64) {
                const double t1 = H(i, j);
                s1r += t1 * xr[j]; s1i += t1 * xi[j];
                if (two) { const double t0 = H(ia, j); s0r += t0 * xr[j]; s0i += t0 * xi[j]; }
            }
            s1r = -wave_sum(s1r); s1i = -wave_sum(s1i);
            if (two) { s0r = -wave_sum(s0r); s0i = -wave_sum(s0i); }
            if (lane == 0) {
                if (!two) {
                    cplx dd = {H(i, i) - lre, -lim};
                    if (fabs(dd.re) + fabs(dd.im) < smin) dd = {smin, 0.0};
                    cplx v = cdiv({s1r, s1i}, dd);
                    xr[i] = v.re; xi[i] = v.im;
                } else {
                    // [[T(ia,ia)-lam, T(ia,i)], [T(i,ia), T(i,i)-lam]] [x_ia; x_i] = [s0; s1]
                    cplx a11 = {H(ia, ia) - lre, -lim}, a12 = {H(ia, i), 0.0};
                    cplx a21 = {H(i, ia), 0.0}, a22 = {H(i, i) - lre, -lim};
                    cplx det = csub(cmul(a11, a22), cmul(a12, a21));
                    if (fabs(det.re) + fabs(det.im) < smin * smin) det = {smin * smin, 0.0};
                    cplx x0 = cdiv(csub(cmul({s0r, s0i}, a22), cmul(a12, {s1r, s1i})), det);
                    cplx x1 = cdiv(csub(cmul(a11, {s1r, s1i}), cmul(a21, {s0r, s0i})), det);
                    xr[ia] = x0.re; xi[ia] = x0.im; xr[i] = x1.re; xi[i] = x1.im;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // guard against overflow: rescale when the entries grow large
            double mx = 0.0;
            for (int j = ia + lane; j <= top; j += 64) mx = fmax(mx, fabs(xr[j]) + fabs(xi[j]));
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
            if (mx > 1e100) {
                for (int j = ia + lane; j <= top; j += 64) { xr[j] *= 1e-100; xi[j] *= 1e-100; }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            i = ia - 1;
        }
        // normalise (complex 2-norm) and store the folded columns
        double nn2 = 0.0;
        for (int j = lane; j <= top; j += 64) nn2 += xr[j] * xr[j] + xi[j] * xi[j];
        nn2 = wave_sum(nn2);
        const double inv = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 0.0;
        for (int j = lane; j < n; j += 64) {
            X[(int64_t)k * n + j] = xr[j] * inv;
            if (pair) X[(int64_t)(k + 1) * n + j] = xi[j] * inv;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    __threadfence_block();
    // ---- W rows of this work-group = Z_slab X
    for (int e = tid; e < nrows * n; e += nt) {
        const int rl = e % nrows, c = e / nrows;
        const double* xc = X + (int64_t)c * n;
        const double* z = Zs + rl * n;
        double s = 0.0;
        for (int m = 0; m < n; ++m) s += z[m] * xc[m];
        Wraw[(int64_t)c * n + r0 + rl] = s;
    }
}

// ====================================================================== 3. canonical order
__global__ void sort_modes_kernel(int n, const double* __restrict__ wr, const double* __restrict__ wi,
                                  const int32_t* __restrict__ kind0, const double* __restrict__ Wraw,
                                  double* lam, int32_t* kind, double* W)
{
    extern __shared__ int pos[];   // n: output position of each unit head
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int u = tid; u < n; u += nt) {
        pos[u] = -1;
        if (kind0[u] == 2) continue;
        const double au = fabs(atan2(wi[u], wr[u])), mu = hypot(wr[u], wi[u]);
        int p = 0;
        for (int v = 0; v < n; ++v) {
            if (kind0[v] == 2 || v == u) continue;
            const double av = fabs(atan2(wi[v], wr[v])), mv = hypot(wr[v], wi[v]);
            const bool before = (av < au) || (av == au && mv > mu) || (av == au && mv == mu && v < u);
            if (before) p += (kind0[v] == 1) ? 2 : 1;
        }
        pos[u] = p;
    }
    __syncthreads();
    for (int u = tid; u < n; u += nt) {
        const int p = pos[u];
        if (p < 0) continue;
        if (kind0[u] == 0) {
            lam[2 * p] = wr[u]; lam[2 * p + 1] = 0.0; kind[p] = 0;
        } else {
            lam[2 * p] = wr[u]; lam[2 * p + 1] = fabs(wi[u]);
            lam[2 * p + 2] = wr[u]; lam[2 * p + 3] = -fabs(wi[u]);
            kind[p] = 1; kind[p + 1] = 2;
        }
    }
    for (int64_t e = tid; e < (int64_t)n * n; e += nt) {
        const int row = (int)(e % n), u = (int)(e / n);
        const int p = pos[u];
        if (p < 0) continue;
        W[(int64_t)p * n + row] = Wraw[(int64_t)u * n + row];
        if (kind0[u] == 1) W[(int64_t)(p + 1) * n + row] = Wraw[(int64_t)(u + 1) * n + row];
    }
}

hipError_t nonsym_eig(hipStream_t s, const double* A, int64_t lda, int n, void* ws, double* lam,
                      int32_t* kind, double* W, int32_t* info)
{
    if (n <= 0) return hipSuccess;
    if (n > EIG_MAX) return hipErrorInvalidValue;
    EigWs w = eig_carve(ws, n);
    hipLaunchKernelGGL(hessenberg_kernel, dim3(1), dim3(1024), 0, s, A, lda, n, w.H, w.V, w.tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nr = eig_rows_per_wg(n);
    const int grid = eig_grid(n);
    int hsize = 0;
    for (int j = 0; j < n; ++j) hsize += std::min(j + 4, n);
    const int nw = 4;
    const size_t lds = (size_t)(round_up(2 * n + 1, 2) / 2) * 8 + (size_t)hsize * 8 + (size_t)nr * n * 8 +
                       (size_t)nw * 2 * n * 8;
    if (lds > 160 * 1024 - 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL(francis_kernel, dim3(grid), dim3(64 * nw), lds, s, n, nr, w.H, w.V, w.tau, w.Wraw,
                       w.wr, w.wi, w.kind0, w.X, info);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_modes_kernel, dim3(1), dim3(256), n * sizeof(int), s, n, w.wr, w.wi, w.kind0,
                       w.Wraw, lam, kind, W);
    return hipGetLastError();
}

hipError_t eig_prepare()
{
    return hipFuncSetAttribute((const void*)francis_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 256);
}

hipError_t prepare_kernels()
{
    hipError_t e = gemm_prepare();
    if (e != hipSuccess) return e;
    e = small_prepare();
    if (e != hipSuccess) return e;
    return eig_prepare();
}

}  // namespace dmd
