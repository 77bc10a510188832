// psc_aperture.hip -- the far-field pattern of a measured aperture
// illumination, tabulated for the window-form kernels (setup work).
//
// A dish's voltage pattern is the Fourier transform of its aperture
// illumination (Sec. 1 and Sec. 3: blockage, feed support shadows and taper
// all enter through the illumination).  For a real, even illumination the
// transform is real.  In units of lambda/D the pattern of a given
// illumination is the same at every frequency, so one table serves every
// channel; the kernels scale the sky displacement by D / lambda.
#include "psc_internal.h"

namespace psc {

// One node per thread: T(u, v) = sum_k w_k cos(2 pi (xi_k u + eta_k v)) and
// its derivatives, (xi, eta) the cell centre in units of D and w its weight
// (normalised so that T(0) = 1), by the direct sum in float64.  Stored as
// float32 (T, s T_u, s T_v, s^2 T_uv), s the node step, the slopes the cubic
// Hermite interpolation takes per node.
__global__ void __launch_bounds__(256)
k_aperture_table(const double* __restrict__ cells, int n_cells, float4* __restrict__ tab, int n, double c,
                 double step)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * n) return;
    const int i = idx / n, j = idx - (idx / n) * n;
    const double u = (i - c) * step, v = (j - c) * step;
    double t = 0.0, tu = 0.0, tv = 0.0, tuv = 0.0;
    for (int k = 0; k < n_cells; ++k) {
        const double xi = cells[3 * k], eta = cells[3 * k + 1], w = cells[3 * k + 2];
        double sn, cs;
        sincospi(2.0 * (xi * u + eta * v), &sn, &cs);
        t = fma(w, cs, t);
        tu = fma(-w * xi, sn, tu);
        tv = fma(-w * eta, sn, tv);
        tuv = fma(-w * xi * eta, cs, tuv);
    }
    const double tp = 2.0 * kPi * step;
    tab[idx] = make_float4((float)t, (float)(tp * tu), (float)(tp * tv), (float)(tp * tp * tuv));
}

hipError_t launch_aperture_table(const double* cells, int n_cells, float4* tab, int n, double c, double step,
                                 hipStream_t s)
{
    const long long nodes = (long long)n * n;
    if (n < 2 || nodes > 2147483647LL || n_cells < 1) return hipErrorInvalidValue;
    const int blocks = (int)((nodes + 255) / 256);
    k_aperture_table<<<blocks, 256, 0, s>>>(cells, n_cells, tab, n, c, step);
    return hipGetLastError();
}

}  // namespace psc
