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

}  // namespace psc
