// Upsampling with the reduced Koopman operator (Sec. 6.3): the evolution that keeps the
// low-order modes of a low-res guide and evolves the others (Sec. 6.3.1), and the
// projection onto fields whose block average equals the guide (Sec. 6.3.2).
#include "common.h"
#include "kernels.h"

namespace dmd {

// Complex coefficient of mode i from the real least-squares coefficients of the folded
// basis (a pair (i, i+1) has z_i = (beta_i - i beta_{i+1}) / 2, z_{i+1} its conjugate).
__device__ __forceinline__ cplx folded_to_complex(const double* bc, const int32_t* kind, int r, int i)
{
    int kd = kind[i];
    if ((kd == 1 && i + 1 >= r) || (kd == 2 && i == 0) || kd < 0 || kd > 2) kd = 0;
    if (kd == 0) return {bc[i], 0.0};
    if (kd == 1) return {0.5 * bc[i], -0.5 * bc[i + 1]};
    return {0.5 * bc[i - 1], 0.5 * bc[i]};
}

// R_0 = Phi^+ h0; R_t = the guide's projection for low-order modes and lambda^t R_0 for
// the others (the recurrence R*_t = Lambda R_{t-1} applied t times).  A pair follows the
// flag of its first member.  One thread per (t, i); states (T+1) x r complex.
__global__ void upsample_states_kernel(int r, int T, const double* __restrict__ lam, const double* __restrict__ beta0,
                                       const double* __restrict__ beta, int64_t ldb,
                                       const int32_t* __restrict__ kind, const int32_t* __restrict__ low,
                                       double* __restrict__ states)
{
    const int64_t tot = (int64_t)(T + 1) * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % r), t = (int)(e / r);
        const int lead = (kind[i] == 2 && i > 0) ? i - 1 : i;
        cplx z;
        if (t == 0) z = folded_to_complex(beta0, kind, r, i);
        else if (low[lead]) z = folded_to_complex(beta + (int64_t)(t - 1) * ldb, kind, r, i);
        else z = cmul(cpow_real({lam[2 * i], lam[2 * i + 1]}, (double)t), folded_to_complex(beta0, kind, r, i));
        states[2 * e] = z.re;
        states[2 * e + 1] = z.im;
    }
}

// x = h - (A h - l) spread over each block: the minimiser of ||x - h|| subject to A x = l
// when A averages f x f (x f) blocks (A A^T = f^-d I, so x = h - A^T (A A^T)^-1 (A h - l)).
// One thread per coarse cell of one component of one frame; x may alias h.  FX > 0 fixes
// the block width at compile time so that each block row moves as 16-byte vectors
// (consecutive lanes take consecutive blocks, so every access instruction is contiguous).
template <typename T, int FX> struct RowIO {
    static constexpr int VW = 16 / sizeof(T);
    static constexpr int NV = FX / VW;
    typedef T vec __attribute__((ext_vector_type(VW)));
    __device__ static double sum(const T* p) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const vec a = reinterpret_cast<const vec*>(p)[v];
#pragma unroll
            for (int e = 0; e < VW; ++e) s += (double)a[e];
        }
        return s;
    }
    __device__ static void shift(const T* src, T* dst, double d) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            vec a = reinterpret_cast<const vec*>(src)[v];
#pragma unroll
            for (int e = 0; e < VW; ++e) a[e] = (T)((double)a[e] - d);
            reinterpret_cast<vec*>(dst)[v] = a;
        }
    }
};

template <typename T, int FX>
__global__ void lowres_project_kernel(const T* h, int64_t ldh, const T* __restrict__ l, int64_t ldl, T* x,
                                      int64_t ldx, int64_t nframes, int ncomp, int nz, int ny, int nx, int fr_,
                                      int fz)
{
    const int f = FX > 0 ? FX : fr_;
    const int cz = nz / fz, cy = ny / f, cx = nx / f;
    const int64_t per_frame = (int64_t)ncomp * cz * cy * cx;
    const int64_t tot = per_frame * nframes;
    const double inv = 1.0 / ((double)fz * f * f);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t fr = e / per_frame;
        const int64_t cell = e % per_frame;                  // coarse index (comp, z, y, x), x fastest
        int64_t c = cell;
        const int ix = (int)(c % cx); c /= cx;
        const int iy = (int)(c % cy); c /= cy;
        const int iz = (int)(c % cz);
        const int comp = (int)(c / cz);
        const int64_t base = (((int64_t)comp * nz + (int64_t)iz * fz) * ny + (int64_t)iy * f) * nx + (int64_t)ix * f;
        const T* hf = h + fr * ldh + base;
        T* xf = x + fr * ldx + base;
        double s = 0.0;
        for (int dz = 0; dz < fz; ++dz)
            for (int dy = 0; dy < f; ++dy) {
                const T* row = hf + ((int64_t)dz * ny + dy) * nx;
                if constexpr (FX > 0) s += RowIO<T, FX>::sum(row);
                else for (int dx = 0; dx < f; ++dx) s += (double)row[dx];
            }
        const double d = s * inv - (double)l[fr * ldl + cell];
        for (int dz = 0; dz < fz; ++dz)
            for (int dy = 0; dy < f; ++dy) {
                const int64_t o = ((int64_t)dz * ny + dy) * nx;
                if constexpr (FX > 0) RowIO<T, FX>::shift(hf + o, xf + o, d);
                else for (int dx = 0; dx < f; ++dx) xf[o + dx] = (T)((double)hf[o + dx] - d);
            }
    }
}

hipError_t upsample_states(hipStream_t s, int r, int T, const double* lam, const double* beta0, const double* beta,
                           int64_t ldb, const int32_t* kind, const int32_t* low, double* states)
{
    const int64_t tot = (int64_t)(T + 1) * r;
    const int blocks = (int)std::min<int64_t>(ceil_div(tot, 256), 4096);
    hipLaunchKernelGGL(upsample_states_kernel, dim3(blocks), dim3(256), 0, s, r, T, lam, beta0, beta, ldb, kind, low,
                       states);
    return hipGetLastError();
}

template <typename T>
static hipError_t lowres_launch(hipStream_t s, const T* h, int64_t ldh, const T* l, int64_t ldl, T* x, int64_t ldx,
                                int64_t nframes, int ncomp, int nz, int ny, int nx, int f, int fz, int blocks)
{
    // 16-byte block rows need aligned frames: base pointers, leading dimensions and nx
    constexpr int VW = 16 / sizeof(T);
    const bool al = (uintptr_t)h % 16 == 0 && (uintptr_t)x % 16 == 0 && ldh % VW == 0 && ldx % VW == 0 && nx % VW == 0;
    if (al && f == 4)
        hipLaunchKernelGGL((lowres_project_kernel<T, 4>), dim3(blocks), dim3(256), 0, s, h, ldh, l, ldl, x, ldx,
                           nframes, ncomp, nz, ny, nx, f, fz);
    else if (al && f == 8)
        hipLaunchKernelGGL((lowres_project_kernel<T, 8>), dim3(blocks), dim3(256), 0, s, h, ldh, l, ldl, x, ldx,
                           nframes, ncomp, nz, ny, nx, f, fz);
    else if (al && f == 2 && VW == 2)
        hipLaunchKernelGGL((lowres_project_kernel<T, 2>), dim3(blocks), dim3(256), 0, s, h, ldh, l, ldl, x, ldx,
                           nframes, ncomp, nz, ny, nx, f, fz);
    else
        hipLaunchKernelGGL((lowres_project_kernel<T, 0>), dim3(blocks), dim3(256), 0, s, h, ldh, l, ldl, x, ldx,
                           nframes, ncomp, nz, ny, nx, f, fz);
    return hipGetLastError();
}

hipError_t lowres_project(hipStream_t s, int dtype, const void* h, int64_t ldh, const void* l, int64_t ldl, void* x,
                          int64_t ldx, int64_t nframes, int ncomp, int nz, int ny, int nx, int f)
{
    const int fz = nz == 1 ? 1 : f;
    const int64_t tot = (int64_t)ncomp * (nz / fz) * (ny / f) * (nx / f) * nframes;
    if (tot == 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(ceil_div(tot, 256), (int64_t)device_cu_count() * 16);
    if (dtype == DMD_F32)
        return lowres_launch<float>(s, (const float*)h, ldh, (const float*)l, ldl, (float*)x, ldx, nframes, ncomp, nz,
                                    ny, nx, f, fz, blocks);
    return lowres_launch<double>(s, (const double*)h, ldh, (const double*)l, ldl, (double*)x, ldx, nframes, ncomp, nz,
                                 ny, nx, f, fz, blocks);
}

}  // namespace dmd
