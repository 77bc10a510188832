// psc_scale.hip -- the damped update of the beam-width scales, a generalised
// antenna parameter solved with the same sums as the pointing offsets
// (Eq. DA with a_i = sigma_i, Eq. DCHIDD; Sec. 5.3 solves the beam's shape
// with this machinery).
#include "psc_internal.h"

namespace psc {

// One block per interval: sigma += gain g / H for every (pol, antenna) with
// H > 0, finite sums and a result above min_scale (0, or the narrowest beam
// the support holds); others are left as they are and flagged.  The block's largest |delta sigma| goes to max_step[s].  With
// solve state (done, iters non-null): a finished interval is skipped, and an
// interval whose step falls below tol is marked finished.
__global__ void __launch_bounds__(256)
k_scale_step(int n_pol, int n_ant, const double* __restrict__ acc3, double gain, double* __restrict__ scale,
             int32_t* __restrict__ not_updated, double* __restrict__ max_step, int32_t* __restrict__ done,
             int32_t* __restrict__ iters, double tol, double min_scale)
{
    __shared__ double smax[256];
    const int s = blockIdx.x, tid = threadIdx.x;
    if (done != nullptr && done[s]) {
        if (tid == 0 && max_step != nullptr) max_step[s] = 0.0;
        return;
    }
    const int npa = n_pol * n_ant;
    double mx = 0.0;
    for (int k = tid; k < npa; k += 256) {
        const size_t i = (size_t)s * npa + k;
        const double g = acc3[3 * i + 1], h = acc3[3 * i + 2];
        const double cur = scale[i];
        const double nxt = cur + gain * g / h;
        const bool ok = h > 0.0 && isfinite(g) && isfinite(h) && isfinite(nxt) && nxt > 0.0 && nxt >= min_scale;
        if (ok) {
            mx = fmax(mx, fabs(nxt - cur));
            scale[i] = nxt;
        }
        if (not_updated != nullptr) not_updated[i] = ok ? 0 : 1;
    }
    smax[tid] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) smax[tid] = fmax(smax[tid], smax[tid + w]);
        __syncthreads();
    }
    if (tid == 0) {
        if (max_step != nullptr) max_step[s] = smax[0];
        if (iters != nullptr) iters[s] += 1;
        if (done != nullptr) done[s] = smax[0] < tol ? 1 : 0;
    }
}

hipError_t launch_scale_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* scale,
                             int32_t* not_updated, double* max_step, int32_t* done, int32_t* iters, double tol,
                             double min_scale, hipStream_t s)
{
    if (n_int <= 0) return hipSuccess;
    k_scale_step<<<n_int, 256, 0, s>>>(n_pol, n_ant, acc3, gain, scale, not_updated, max_step, done, iters, tol, min_scale);
    return hipGetLastError();
}

// The uniform disc's radial moments for the aperture defocus: with the
// illumination times exp(i delta t^2) (t = r / R) the pattern is
//   E(x; delta) = 2 int_0^1 J0(x t) exp(i delta t^2) t dt
//               = sum_n (i delta)^n / n! M_n(x),  M_n(x) = 2 int_0^1 J0(x t) t^(2n+1) dt,
// dM_n/dx = -2 int_0^1 J1(x t) t^(2n+2) dt; Gauss-Legendre quadrature on
// [0, 1] in float64, stored (M_n, dx dM_n/dx) per x node, [node][n].
__global__ void k_moment_table(float2* __restrict__ tab, int n_tab, int n_mom, double dx,
                               const double* __restrict__ gl_t, const double* __restrict__ gl_w, int n_gl)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_tab * n_mom) return;
    const int i = idx / n_mom, n = idx - i * n_mom;
    const double x = i * dx;
    double m = 0.0, dm = 0.0;
    for (int q = 0; q < n_gl; ++q) {
        const double t = gl_t[q], w = gl_w[q];
        const double tp = pow(t, 2 * n + 1);
        m += w * j0(x * t) * tp;
        dm -= w * j1(x * t) * tp * t;
    }
    tab[idx] = make_float2((float)(2.0 * m), (float)(2.0 * dm * dx));
}

// One block per interval: delta += gain g / H where H > 0, the sums are
// finite and the result stays within |delta| <= kMaxDefocus; others are left
// as they are and flagged.  max_step[s]: the block's largest |step|.
__global__ void __launch_bounds__(256)
k_defocus_step(int n_pol, int n_ant, const double* __restrict__ acc3, double gain, double* __restrict__ defocus,
               int32_t* __restrict__ not_updated, double* __restrict__ max_step)
{
    __shared__ double smax[256];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int npa = n_pol * n_ant;
    double mx = 0.0;
    for (int k = tid; k < npa; k += 256) {
        const size_t i = (size_t)s * npa + k;
        const double g = acc3[3 * i + 1], h = acc3[3 * i + 2];
        const double step = gain * g / h;
        const double nxt = defocus[i] + step;
        const bool ok = h > 0.0 && isfinite(g) && isfinite(h) && isfinite(nxt) && fabs(nxt) <= kMaxDefocus;
        if (ok) {
            mx = fmax(mx, fabs(step));
            defocus[i] = nxt;
        }
        if (not_updated != nullptr) not_updated[i] = ok ? 0 : 1;
    }
    smax[tid] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) smax[tid] = fmax(smax[tid], smax[tid + w]);
        __syncthreads();
    }
    if (tid == 0 && max_step != nullptr) max_step[s] = smax[0];
}

hipError_t launch_moment_table(float2* tab, int n_tab, int n_mom, double dx, const double* gl_t, const double* gl_w,
                               int n_gl, hipStream_t s)
{
    const int tot = n_tab * n_mom;
    k_moment_table<<<(tot + 255) / 256, 256, 0, s>>>(tab, n_tab, n_mom, dx, gl_t, gl_w, n_gl);
    return hipGetLastError();
}

hipError_t launch_defocus_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* defocus,
                               int32_t* not_updated, double* max_step, hipStream_t s)
{
    if (n_int <= 0) return hipSuccess;
    k_defocus_step<<<n_int, 256, 0, s>>>(n_pol, n_ant, acc3, gain, defocus, not_updated, max_step);
    return hipGetLastError();
}

}  // namespace psc
