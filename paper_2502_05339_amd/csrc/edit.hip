// Temporal editing of DMD modes (Sec. 6.1, eq. edit_temporal): per-mode rate,
// frequency and weight edits on Omega = Log(lambda) / dt, by frequency cluster.
#include "common.h"
#include "kernels.h"

namespace dmd {

// One thread per mode.  lam / b may alias lam_out / b_out: each thread reads its own
// entries before writing them.
__global__ void edit_modes_kernel(int r, double dt, dmd_edit e, const double* mode_edit,
                                  const double* lam, const double* b, double* lam_out, double* b_out,
                                  int32_t* cluster_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const double lr = lam[2 * i], li = lam[2 * i + 1];
    const double br = b[2 * i], bi = b[2 * i + 1];
    const double theta = atan2(li, lr);               // arg lambda in (-pi, pi]
    const int c = (fabs(theta / dt) < e.freq_cut) ? 0 : 1;
    double w, s_re, c_re, s_im;
    if (mode_edit) {
        w = mode_edit[4 * i];
        s_re = mode_edit[4 * i + 1];
        c_re = mode_edit[4 * i + 2];
        s_im = mode_edit[4 * i + 3];
    } else {
        w = e.weight[c];
        s_re = e.re_scale[c];
        c_re = e.re_shift[c];
        s_im = e.im_scale[c];
    }
    const double mod = hypot(lr, li);
    double nr = 0.0, ni = 0.0;
    if (mod != 0.0) {
        const double om_re = log(mod) / dt;           // Re Omega: log-modulus rate
        const double om_im = theta / dt;              // Im Omega: angular frequency
        const double mod_new = exp((s_re * om_re + c_re) * dt);
        const double th_new = (s_im * om_im) * dt;
        double sn, cs;
        sincos(th_new, &sn, &cs);
        nr = mod_new * cs;
        ni = mod_new * sn;
    }
    lam_out[2 * i] = nr;
    lam_out[2 * i + 1] = ni;
    b_out[2 * i] = w * br;
    b_out[2 * i + 1] = w * bi;
    if (cluster_out) cluster_out[i] = c;
}

hipError_t edit_modes(hipStream_t s, int r, double dt, const dmd_edit& e, const double* mode_edit,
                      const double* lam, const double* b, double* lam_out, double* b_out, int32_t* cluster_out)
{
    const int threads = 64;
    const int blocks = (int)ceil_div(r, threads);
    hipLaunchKernelGGL(edit_modes_kernel, dim3(blocks), dim3(threads), 0, s, r, dt, e, mode_edit, lam, b,
                       lam_out, b_out, cluster_out);
    return hipGetLastError();
}

}  // namespace dmd
