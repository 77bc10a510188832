// psc_kernels.hip -- gfx950 kernels of the Pointing SelfCal hot path.
//
// Notation (Bhatnagar & Cornwell 2017): V^{M0} is the gridded transform of
// the model image (Eq. MEDD), A_ij the uv kernel of baseline (i,j) -- the
// convolution of the two antennas' aperture functions, each carrying its
// pointing offset as a phase gradient (Eq. MEDD, Sec. 3) -- and dA_ij/dp its
// derivative (Eq. DA).  Degridding evaluates V = A_ij * V^{M0} and dV/dp
// (Algorithm 1, "use A-Projection") at every sample; the residual sums of
// Eq. DCHIDD are accumulated per antenna in float64.
//
// Kernel construction.  With an anti-aliasing taper c(l) (exponential of a
// semicircle in the uv plane, W cells wide), the grid holds V^{M0} = F[I/c]
// and the kernel of baseline (i,j) is the transform of E_i E_j c, sampled on
// the 1/O lattice.  E_i E_j c is band-limited to S cells, so its transform is
// exactly the DFT of image-plane samples at spacing FoV/S; the samples reach
// |l| < M/2 * FoV/S, beyond which c is negligible.  Writing a lattice index
// as f + O b (0 <= f < O), the DFT splits into a twiddle by exp(2 pi i f n/(SO)),
// a fold of n modulo S, and an S-point DFT over b: each S x S sub-table is one
// small 2-D FFT.  Only sub-tables that some sample of the item uses are built.
#include <type_traits>

#include "psc_device.h"

namespace psc {

// ---------------------------------------------------------------------------
// Model transform (setup): V^{M0}[k] = sum_n I[n]/c[n] exp(+2 pi i k.(n - N/2)/N)
// ---------------------------------------------------------------------------
__global__ void k_taper_image(const double* __restrict__ img, const double* __restrict__ tp,
                              double2* __restrict__ out, int n)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int ix = (int)(idx / n), iy = (int)(idx % n);
    out[idx] = make_double2(img[idx] / (tp[ix] * tp[iy]), 0.0);
}

// In-place radix-2 DFT with exponent +2 pi i along each row (one block per row).
__global__ void k_fft_rows(double2* __restrict__ data, int n, int log2n)
{
    extern __shared__ double2 sh[];
    double2* row = data + (size_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int r = 0;
        for (int b = 0; b < log2n; ++b)
            if (i & (1 << b)) r |= 1 << (log2n - 1 - b);
        sh[r] = row[i];
    }
    __syncthreads();
    for (int st = 1; st <= log2n; ++st) {
        const int mlen = 1 << st, half = mlen >> 1;
        for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
            const int grp = b / half, j = b % half;
            const int i0 = grp * mlen + j, i1 = i0 + half;
            double s, c;
            sincospi(2.0 * (double)j / (double)mlen, &s, &c);
            const double2 v = sh[i1];
            const double2 t = make_double2(c * v.x - s * v.y, c * v.y + s * v.x);
            const double2 u = sh[i0];
            sh[i0] = make_double2(u.x + t.x, u.y + t.y);
            sh[i1] = make_double2(u.x - t.x, u.y - t.y);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) row[i] = sh[i];
}

__global__ void k_transpose(const double2* __restrict__ in, double2* __restrict__ out, int n)
{
    __shared__ double2 tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int j = threadIdx.y; j < 32; j += blockDim.y)
        tile[j][threadIdx.x] = in[(size_t)(by + j) * n + bx + threadIdx.x];
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += blockDim.y)
        out[(size_t)(bx + j) * n + by + threadIdx.x] = tile[threadIdx.x][j];
}

// Writes V^{M0} into a (N+pad) x (N+pad) array whose last `pad` rows and
// columns repeat the first ones (V^{M0} is N-periodic because the sky lies on
// the pixel lattice), so an S x S window starting anywhere in [0, N) never wraps.
// The tapered image of one w-plane: (I / c) exp(2 pi i w (n - 1)) with the
// pixel's direction cosines l = (ix - N/2) cell, m = (iy - N/2) cell and
// n - 1 = -x / (1 + sqrt(1 - x)), x = l^2 + m^2 (Eq. ME with the baseline's w),
// in float64.
__global__ void k_wplane_image(const double* __restrict__ img, const double* __restrict__ tp,
                               double2* __restrict__ out, int n, double cell, double w)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int ix = (int)(idx / n), iy = (int)(idx % n);
    const double v = img[idx] / (tp[ix] * tp[iy]);
    if (v == 0.0) {
        out[idx] = make_double2(0.0, 0.0);
        return;
    }
    const double l = (ix - n / 2) * cell, m = (iy - n / 2) * cell;
    const double x = l * l + m * m;
    const double nm1 = -x / (1.0 + sqrt(1.0 - x));
    double sn, cs;
    sincospi(2.0 * w * nm1, &sn, &cs);
    out[idx] = make_double2(v * cs, v * sn);
}

__global__ void k_finish_grid(const double2* __restrict__ in, float2* __restrict__ out, int n, int pad)
{
    const int p = n + pad;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)p * p) return;
    const int kx = (int)(idx / p) % n, ky = (int)(idx % p) % n;
    const double sgn = ((kx + ky) & 1) ? -1.0 : 1.0;  // exp(-i pi (kx + ky)) from the N/2 shift
    const double2 v = in[(size_t)kx * n + ky];
    out[idx] = make_float2((float)(sgn * v.x), (float)(sgn * v.y));
}

// ---------------------------------------------------------------------------
// Image gradient (the adjoint of the model transform and degrid)
// ---------------------------------------------------------------------------
// Zero fill: a kernel rather than a memset, so that it can sit in a graph.
__global__ void k_zero(double2* __restrict__ p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_double2(0.0, 0.0);
}

// Folds the (N+pad)^2 residual grid back onto N x N (its last `pad` rows and
// columns are the first ones again) and applies the sign of the N/2 shift:
// out[k] = (-1)^(kx+ky) sum of the copies of cell k.
__global__ void k_unpad_grid(const double2* __restrict__ g, double2* __restrict__ out, int n, int pad)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int kx = (int)(idx / n), ky = (int)(idx % n);
    const size_t p = (size_t)n + pad;
    double2 v = g[kx * p + ky];
    if (kx < pad) {
        const double2 w = g[(kx + n) * p + ky];
        v.x += w.x;
        v.y += w.y;
    }
    if (ky < pad) {
        const double2 w = g[kx * p + ky + n];
        v.x += w.x;
        v.y += w.y;
    }
    if (kx < pad && ky < pad) {
        const double2 w = g[(kx + n) * p + ky + n];
        v.x += w.x;
        v.y += w.y;
    }
    const double sgn = ((kx + ky) & 1) ? -1.0 : 1.0;
    out[idx] = make_double2(sgn * v.x, sgn * v.y);
}

// d chi^2 / d I[n] = -2 Re(F[n]) / c[n]: F is the transform of the unpadded
// residual grid, c the taper response the model was divided by.
__global__ void k_image_grad(const double2* __restrict__ f, const double* __restrict__ tp,
                             double* __restrict__ out, int n)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int ix = (int)(idx / n), iy = (int)(idx % n);
    out[idx] = -2.0 * f[idx].x / (tp[ix] * tp[iy]);
}

// ---------------------------------------------------------------------------
// Airy pattern table: A(x) = 2 J1(x)/x, B(x) = 2 J2(x)/x^2 and their slopes
// (A' = -x B, B' = (A - 4B)/x), for cubic Hermite interpolation.
// ---------------------------------------------------------------------------
__global__ void k_airy_table(float4* __restrict__ tab, int n_tab, double dx)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tab) return;
    const double x = i * dx;
    double A, B, Bp;
    if (x < 1e-2) {
        const double x2 = x * x;
        A = 1.0 - x2 / 8.0 + x2 * x2 / 192.0;
        B = 0.25 - x2 / 48.0 + x2 * x2 / 1536.0;
        Bp = -x / 24.0 + x * x2 / 384.0;
    } else {
        A = 2.0 * j1(x) / x;
        B = 2.0 * jn(2, x) / (x * x);
        Bp = (A - 4.0 * B) / x;
    }
    // slopes pre-multiplied by the spacing, as the Hermite form uses them
    tab[i] = make_float4((float)A, (float)(-x * B * dx), (float)B, (float)(Bp * dx));
}

// ---------------------------------------------------------------------------
// Fused kernel build + degrid + per-item float64 partial sums (table form).
// One block (4 wavefronts) per item; the wavefronts share the image-plane
// products and take the item's sub-table groups in turn.  Inside a group, a
// wavefront builds the five S x S sub-tables in its own LDS buffer and
// degrids SPL * 64/S samples at a time: lane a_m of each S-lane slot reads
// column a_m of its samples' S x S windows of V^{M0} and of the sub-tables.
// ---------------------------------------------------------------------------
// LDS holds two blocks per CU, i.e. two wavefronts per SIMD; telling the
// compiler so lets it keep every window load of an iteration in flight.
template <int S, int MODE, int SPL, bool MX>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) k_item(ItemArgs a)
{
    constexpr int NV = mode_nv(MODE);
    constexpr int NC = mode_nc(MODE);
    constexpr int SP = S + 1;
    constexpr int SPW = 64 / S;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float2 twsh[S * 16];  // exp(+2 pi i t / (S O)), O <= 16
    __shared__ float2 phsh[kWaves][64];  // per-wave phase vectors of the current group
    __shared__ int next_group;
    __shared__ float2 zrow[4];  // zero kernel coefficients for unused MFMA columns

    const int m = a.m, half_m = m >> 1, m2 = m * m;
    const int m2p = (m2 + 3) & ~3;
    // dynamic LDS: per-group float64 sums | image-plane products | sub-tables
    double* gpart = reinterpret_cast<double*>(smem);
    const int O2 = a.oversample * a.oversample;
    float* gsh = reinterpret_cast<float*>(smem + sizeof(double) * (NC > 0 ? NC : 1) * O2);
    float2* ush = reinterpret_cast<float2*>(reinterpret_cast<unsigned char*>(gsh) + sizeof(float) * NV * m2p);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = item_of_block();
    if (li >= a.n_items) return;
    const int item_idx = a.item_begin + li;
    const Item it = a.items[item_idx];
    if (a.done != nullptr && a.done[it.interval]) return;

    const int N = a.grid_n;
    const int O = a.oversample, so = S * O;
    const float inv_s = 1.0f / (float)S;
    const int P = N + S;  // pitch of the padded grid
    const int rowbytes = P * (int)sizeof(float2);
    const __amdgpu_buffer_rsrc_t grsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.grid, (short)0, P * P * (int)sizeof(float2), 0x00020000);

    for (int t = tid; t < so; t += kBlock) twsh[t] = a.tw[t];
    if (tid < 4) zrow[tid] = make_float2(0.f, 0.f);

    for (int pol = 0; pol < a.n_pol; ++pol) {
        if (tid == 0) next_group = it.grp_begin + kWaves;
        image_products<MODE>(a, it, pol, gsh, m2p, tid, kBlock);
        __syncthreads();

        double acc64 = 0.0;
        float2* uw = ush + (size_t)wave * NV * S * SP;
        float2* phw = phsh[wave];
        // groups are handed out to wavefronts dynamically, first one each
        const int slot = lane / S;
        const int am = lane - slot * S;
        int gi = it.grp_begin + wave;
        Group g = a.groups[gi < it.grp_end ? gi : it.grp_begin];
        while (gi < it.grp_end) {
            // claim the next group and start fetching its descriptor and this
            // group's first samples; both loads complete behind the fold/FFT
            int nxt_g = 0;
            if (lane == 0) nxt_g = atomicAdd(&next_group, 1);
            nxt_g = __shfl(nxt_g, 0);
            const Group gnext = a.groups[nxt_g < it.grp_end ? nxt_g : gi];
            constexpr int STEP = SPW * SPL;
            const int nv = g.n_vis;
            const uint32_t vb = g.vis_begin;
            VisEnt ent[SPL];
#pragma unroll
            for (int j = 0; j < SPL; ++j) {
                const int v = slot + SPW * j;
                ent[j] = a.vis[vb + (v < nv ? v : nv - 1)];
            }
            const int fl = g.f / O, fm = g.f - fl * O;

            // ---- per-axis phases (-1)^n exp(2 pi i f n / (S O)) / S, n in [-M/2, M/2)
            if (lane < m) {
                const int n = lane - half_m;
                float2 p = twsh[(fl * n) & (so - 1)];
                const float sg = (n & 1) ? -inv_s : inv_s;
                phw[lane] = make_float2(p.x * sg, p.y * sg);
            } else if (lane >= 32 && lane - 32 < m) {
                const int n = lane - 32 - half_m;
                float2 p = twsh[(fm * n) & (so - 1)];
                const float sg = (n & 1) ? -inv_s : inv_s;
                phw[lane] = make_float2(p.x * sg, p.y * sg);
            }
            wave_sync();

            // ---- twiddle and fold: U[r] = sum_{n = r mod S} phase_l(n_l) phase_m(n_m) g[n]
            for (int r = lane; r < S * S; r += 64) {
                const int rl = r / S, rm = r - rl * S;
                float2 u[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) u[k] = make_float2(0.f, 0.f);
#pragma unroll
                for (int el = 0; el < 2; ++el) {
                    const int nl = rl - el * S;
                    if (nl < -half_m || nl >= half_m) continue;
                    // inner fold along m for this n_l, then one complex twiddle
                    float2 x[NV];
#pragma unroll
                    for (int k = 0; k < NV; ++k) x[k] = make_float2(0.f, 0.f);
#pragma unroll
                    for (int em = 0; em < 2; ++em) {
                        const int nmv = rm - em * S;
                        if (nmv < -half_m || nmv >= half_m) continue;
                        const float2 pm = phw[32 + nmv + half_m];
                        const int gidx = (nl + half_m) * m + (nmv + half_m);
#pragma unroll
                        for (int k = 0; k < NV; ++k) {
                            const float gv = gsh[k * m2p + gidx];
                            x[k].x = fmaf(gv, pm.x, x[k].x);
                            x[k].y = fmaf(gv, pm.y, x[k].y);
                        }
                    }
                    const float2 pl = phw[nl + half_m];
#pragma unroll
                    for (int k = 0; k < NV; ++k) cmac(u[k], pl, x[k]);
                }
#pragma unroll
                for (int k = 0; k < NV; ++k) uw[(k * S + rl) * SP + rm] = u[k];
            }
            wave_sync();

            // ---- 2-D DFT of each sub-table: rows, then columns.  For the five
            // gradient variants the 80 row and 80 column transforms run as 160
            // tasks in three passes of 64 lanes (a variant's columns start one
            // pass after its rows end) instead of four passes, two of them a
            // quarter full.
            constexpr bool kPacked = !MX && NV * S == 80 && S == 16;
            if constexpr (kPacked) {
#pragma unroll 1
                for (int pass = 0; pass < 3; ++pass) {
                    const int t = pass * 64 + lane;
                    if (t < 2 * NV * S) {
                        const bool is_row = t < NV * S;
                        const int tt = is_row ? t : t - NV * S;
                        const int k = tt / S, rc = tt - k * S;
                        // row task: x[i] = U[k][rc][i]; column task: x[i] = U[k][i][rc]
                        float2* base = uw + (size_t)k * S * SP + (is_row ? rc * SP : rc);
                        const int step = is_row ? 1 : SP;
                        float2 x[S];
#pragma unroll
                        for (int i = 0; i < S; ++i) x[i] = base[i * step];
                        fft_reg<S>(x);
#pragma unroll
                        for (int i = 0; i < S; ++i) base[i * step] = x[i];
                    }
                    wave_sync();
                }
            } else {
            for (int t = lane; t < NV * S; t += 64) {
                const int k = t / S, row = t - k * S;
                float2 x[S];
#pragma unroll
                for (int i = 0; i < S; ++i) x[i] = uw[(k * S + row) * SP + i];
                fft_reg<S>(x);
#pragma unroll
                for (int i = 0; i < S; ++i) uw[(k * S + row) * SP + i] = x[i];
            }
            wave_sync();
            if constexpr (!MX) {
                for (int t = lane; t < NV * S; t += 64) {
                    const int k = t / S, col = t - k * S;
                    float2 x[S];
#pragma unroll
                    for (int i = 0; i < S; ++i) x[i] = uw[(k * S + i) * SP + col];
                    fft_reg<S>(x);
#pragma unroll
                    for (int i = 0; i < S; ++i) uw[(k * S + i) * SP + col] = x[i];
                }
            } else {
                // column DFTs written in the order the MFMA B operand reads them:
                // entry (b_l, b_m) of variant k goes to tap row a_l = S-1-b_l,
                // column group g = (S-1-b_m)/4, position m = (S-1-b_m)%4 of
                //   [a_l][g][k][m]
                // so a lane's four coefficients of a tap row are 32 contiguous
                // bytes and the lanes of a row read one contiguous block.  Every
                // column is read before any is rewritten (NV*S > 64 tasks).
                static_assert(NV * S <= 128, "two column tasks per lane at most");
                const int t0 = lane, t1 = lane + 64;
                const bool has1 = t1 < NV * S;
                float2 x0[S], x1[S];
                {
                    const int k = t0 / S, col = t0 - k * S;
#pragma unroll
                    for (int i = 0; i < S; ++i) x0[i] = uw[(k * S + i) * SP + col];
                }
                if (has1) {
                    const int k = t1 / S, col = t1 - k * S;
#pragma unroll
                    for (int i = 0; i < S; ++i) x1[i] = uw[(k * S + i) * SP + col];
                }
                // one wavefront's LDS operations run in issue order, so every
                // column above is read before the first write below lands
                fft_reg<S>(x0);
                {
                    const int k = t0 / S, col = t0 - k * S;
                    const int gq = (S - 1 - col) >> 2, mq = (S - 1 - col) & 3;
#pragma unroll
                    for (int i = 0; i < S; ++i)
                        uw[(((S - 1 - i) * (S / 4) + gq) * NV + k) * 4 + mq] = x0[i];
                }
                if (has1) fft_reg<S>(x1);
                if (has1) {
                    const int k = t1 / S, col = t1 - k * S;
                    const int gq = (S - 1 - col) >> 2, mq = (S - 1 - col) & 3;
#pragma unroll
                    for (int i = 0; i < S; ++i)
                        uw[(((S - 1 - i) * (S / 4) + gq) * NV + k) * 4 + mq] = x1[i];
                }
            }
            wave_sync();
            }  // kPacked

            // ---- degrid.  Lane (slot, a_m) of the wavefront reads column a_m of
            // every S x S window it handles; tap (a_l, a_m) uses lattice index
            // b = (S-1-a_l, S-1-a_m) of the sub-tables, read from LDS (the four
            // slots read the same addresses).  Each lane carries SPL samples.
            const int t = am;
            // which term lane t accumulates (see the gradient branch below)
            const TermSel tsel(t);
            const bool t_end = tsel.end, t_xr = tsel.xr, t_xl = tsel.xl, t_yr = tsel.yr, t_yl = tsel.yl;
            // D columns (MFMA path): V = 0,1; d/dl_i = 2,3; d/dm_i = 4,5; d/dl_j = 6,7; d/dm_j = 8,9
            const int t_dl = t_end ? 6 : 2, t_dm = t_end ? 8 : 4;
            const int t_xcol = t_xr ? 0 : (t_xl ? t_dl : t_dm);
            const int t_ycol = t_yr ? 0 : (t_yl ? t_dl : t_dm);
            // A pass degrids L * 64/S samples from v0 on (L per lane).  Full
            // passes (L = SPL) run while more than (SPL - 1) 64/S samples
            // remain; the remainder takes passes with L = 1 (one at SPL = 2),
            // so the partly filled last pass of a part costs less.
            auto degrid = [&](uint32_t vb, int nv, VisEnt (&ent)[SPL]) {
            auto pass = [&](int v0, auto l_const) {
                constexpr int L = decltype(l_const)::value;
                // re-read the sub-tables from LDS every iteration instead of
                // letting the compiler keep all S*NV values in registers
                int kofs = S - 1 - am;
                asm volatile("" : "+v"(kofs));
                const float2* kcol = uw + kofs;
                VisEnt nxt[L];
                int voff[L];
                float2 vin[L];
                float wgt[L];
#pragma unroll
                for (int j = 0; j < L; ++j) {
                    if (L == SPL) {  // the next full pass, early
                        const int vn = v0 + STEP + slot + SPW * j;
                        nxt[j] = a.vis[vb + (vn < nv ? vn : nv - 1)];
                    }
                    const int row0 = (int)(ent[j].klo >> 16);
                    const int col0 = (int)(ent[j].klo & 0xffffu);
                    voff[j] = (row0 * P + col0 + am) * (int)sizeof(float2);
                    // this iteration's data, fetched before the multiply-adds
                    const size_t o = (size_t)ent[j].vidx * a.n_pol + pol;
                    if (MODE != kPredict) vin[j] = a.vis_in[o];
                    if (MODE == kGrad || MODE == kGrid) wgt[j] = a.weight[o];
                }
                float2 s[L][NV];
#pragma unroll
                for (int j = 0; j < L; ++j)
#pragma unroll
                    for (int k = 0; k < NV; ++k) s[j][k] = make_float2(0.f, 0.f);
                // every window row of the iteration is requested up front
                float2 gwin[L][S];
#pragma unroll
                for (int j = 0; j < L; ++j)
#pragma unroll
                    for (int al = 0; al < S; ++al)
                        gwin[j][al] = __builtin_bit_cast(
                            float2, __builtin_amdgcn_raw_buffer_load_b64(grsrc, voff[j], al * rowbytes, 0));
                // kernel rows from LDS, one row ahead of the multiply-adds
                float2 kv[NV], kvn[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) kv[k] = kcol[(k * S + (S - 1)) * SP];
#pragma unroll
                for (int al = 0; al < S; ++al) {
                    if (al + 1 < S) {
#pragma unroll
                        for (int k = 0; k < NV; ++k) kvn[k] = kcol[(k * S + (S - 2 - al)) * SP];
                    }
#pragma unroll
                    for (int j = 0; j < L; ++j)
#pragma unroll
                        for (int k = 0; k < NV; ++k) cmac(s[j][k], kv[k], gwin[j][al]);
#pragma unroll
                    for (int k = 0; k < NV; ++k) kv[k] = kvn[k];
                }
#pragma unroll
                for (int j = 0; j < L; ++j)
#pragma unroll
                    for (int k = 0; k < NV; ++k) {
                        s[j][k].x = row16_sum(s[j][k].x);
                        s[j][k].y = row16_sum(s[j][k].y);
                    }
#pragma unroll
                for (int j = 0; j < L; ++j) {
                    const int v = v0 + slot + SPW * j;
                    if (v >= nv) continue;
                    const size_t o = (size_t)ent[j].vidx * a.n_pol + pol;
                    if constexpr (MODE == kPredict) {
                        if (t == 0) a.vis_out[o] = s[j][0];
                    } else if constexpr (MODE == kGrad) {
                        if (a.vis_out != nullptr && t == 0) a.vis_out[o] = s[j][0];
                        grad_term(tsel, s[j], vin[j], wgt[j], acc64);
                    } else if constexpr (MODE == kVjp) {
                        vjp_term(t, s[j], vin[j], acc64);
                    } else {
                        // adjoint of the degrid: w conj(R) spread back over the
                        // window with the coefficients that produced V, summed
                        // in float64 on the residual grid
                        if (a.vis_out != nullptr && t == 0) a.vis_out[o] = s[j][0];
                        const float rr = (float)((double)vin[j].x - (double)s[j][0].x);
                        const float ri = (float)((double)vin[j].y - (double)s[j][0].y);
                        const float cr = wgt[j] * rr, ci = -wgt[j] * ri;
                        double2* gdst = a.grid_acc + voff[j] / (int)sizeof(float2);
#pragma unroll
                        for (int al = 0; al < S; ++al) {
                            const float2 kv = kcol[(S - 1 - al) * SP];
                            unsafeAtomicAdd(&gdst[(size_t)al * P].x, (double)(cr * kv.x - ci * kv.y));
                            unsafeAtomicAdd(&gdst[(size_t)al * P].y, (double)(cr * kv.y + ci * kv.x));
                        }
                    }
                }
                if constexpr (L == SPL) {
#pragma unroll
                    for (int j = 0; j < SPL; ++j) ent[j] = nxt[j];
                }
            };
            int v0 = 0;
            for (; nv - v0 > SPW * (SPL - 1); v0 += STEP) pass(v0, std::integral_constant<int, SPL>{});
            for (int q = 0; v0 < nv; v0 += SPW, ++q) {
                // the first remainder pass has its entry from the last full
                // pass; later ones (SPL > 2) fetch theirs
                if (q > 0) ent[0] = a.vis[vb + (v0 + slot < nv ? v0 + slot : nv - 1)];
                pass(v0, std::integral_constant<int, 1>{});
            }
            };  // degrid

            if constexpr (MX) {
                // ---- degrid on the matrix cores.  A tile is 16 samples of the
                // group (offset f, then offset -f); per tile the wavefront runs
                // 128 MFMA 16x16x4 f32 over k = (tap, re/im) with
                //   A[sample][k] = window value, B[k][n] = kernel coefficient,
                //   n = 2v + c: real (c = 0) / imaginary (c = 1) part of variant v.
                // Lane (g4, i16) feeds sample i16 at the 4 tap columns 4 g4 .. 4 g4 + 3
                // of each tap row, and gets D columns n = i16 for samples 4 g4 + r.
                // A sample at -f reads its window reflected (b -> S-1-b on an axis
                // with f != 0, b -> -b mod S with f = 0) and conjugated, which is
                // the same as using -f's conjugate-reflected sub-tables; its
                // result is conjugated back.
                const int i16 = lane & 15, g4 = lane >> 4;
                const int ntot = nv + g.n_vis2;
                const bool bzero = i16 >= 2 * NV;
                const bool bd = (i16 & 1) != 0;
                // [a_l][g][k][m] layout (see the column DFTs): tap row a_l starts at
                // a_l * (S/4) * NV * 4; this lane's 4 coefficients are contiguous
                const float2* bbase = bzero ? zrow : uw + (size_t)(g4 * NV + (i16 >> 1)) * 4;
                const int bstride = bzero ? 0 : (S / 4) * NV * 4;
                // Tiles are software-pipelined: while tile t runs its MFMAs, the
                // sample entries of tile t+1 arrive and, during t's last chunk,
                // t+1's first window rows are requested.
                struct TileAddr {
                    bool partner, wrapc;
                    int cbase, wbase;
                    float csg;
                };
                constexpr int HR = 4;  // tap rows per chunk
                typedef float f4v __attribute__((ext_vector_type(4)));
                auto tile_addr = [&](int t0, const VisEnt& e) {
                    const int q = t0 + i16;
                    TileAddr ta;
                    ta.partner = q < ntot && q >= nv;
                    const int row0 = (int)(e.klo >> 16);
                    const int col0 = (int)(e.klo & 0xffffu);
                    // this lane's 4 tap columns 4 g4 .. 4 g4 + 3 as one 32-byte chunk of
                    // the window row (reversed for a sample at -f; with f_m = 0 the last
                    // column of the last group wraps to window column S-1)
                    const int lo = ta.partner ? (fm ? (S - 4 - 4 * g4) : (S - 5 - 4 * g4)) : 4 * g4;
                    ta.wrapc = ta.partner && fm == 0 && g4 == 3;
                    ta.cbase = (row0 * P + col0 + lo) * (int)sizeof(float2);
                    ta.wbase = (row0 * P + col0 + (S - 1)) * (int)sizeof(float2);
                    ta.csg = ta.partner ? -1.f : 1.f;
                    return ta;
                };
                auto load_chunk = [&](const TileAddr& ta, int a0, float2 (&wv)[HR][4]) {
#pragma unroll
                    for (int ah = 0; ah < HR; ++ah) {
                        const int al = a0 + ah;
                        const int wr = ta.partner ? (fl ? (S - 1 - al) : ((S - 2 - al) & (S - 1))) : al;
                        const int roff = wr * rowbytes;
                        const f4v c01 = __builtin_bit_cast(
                            f4v, __builtin_amdgcn_raw_buffer_load_b128(grsrc, ta.cbase + roff, 0, 0));
                        const f4v c23 = __builtin_bit_cast(
                            f4v, __builtin_amdgcn_raw_buffer_load_b128(grsrc, ta.cbase + roff + 16, 0, 0));
                        float2 ch[4] = {make_float2(c01[0], c01[1]), make_float2(c01[2], c01[3]),
                                        make_float2(c23[0], c23[1]), make_float2(c23[2], c23[3])};
                        if (ta.wrapc)
                            ch[0] = __builtin_bit_cast(
                                float2, __builtin_amdgcn_raw_buffer_load_b64(grsrc, ta.wbase + roff, 0, 0));
#pragma unroll
                        for (int mm = 0; mm < 4; ++mm) wv[ah][mm] = ta.partner ? ch[3 - mm] : ch[mm];
                    }
                };
                auto tile_entries = [&](int t0, VisEnt& e, VisEnt (&es)[4]) {
                    const int q = t0 + i16;
                    e = a.vis[vb + (q < ntot ? q : 0)];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int qs = t0 + 4 * g4 + r;
                        es[r] = a.vis[vb + (qs < ntot ? qs : 0)];
                    }
                };
                auto tile_data = [&](const VisEnt (&es)[4], float2 (&tv)[4], float (&tw)[4]) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const size_t o = (size_t)es[r].vidx * a.n_pol + pol;
                        tv[r] = a.vis_in[o];
                        tw[r] = (MODE == kGrad) ? a.weight[o] : 0.f;
                    }
                };
                VisEnt e_cur, es[4];
                tile_entries(0, e_cur, es);
                TileAddr ta = tile_addr(0, e_cur);
                float2 cur[HR][4], nxt[HR][4];
                load_chunk(ta, 0, cur);
                float2 tv[4];
                float tw[4];
                tile_data(es, tv, tw);
                for (int t0 = 0; t0 < ntot; t0 += 16) {
                    const int t1 = t0 + 16;
                    const bool more = t1 < ntot;
                    VisEnt e_nx = e_cur, es_nx[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) es_nx[r] = es[r];
                    if (more) tile_entries(t1, e_nx, es_nx);
                    TileAddr ta_nx = ta;
                    mfma_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
                    for (int a0 = 0; a0 < S; a0 += HR) {
                        if (a0 + HR < S) {
                            load_chunk(ta, a0 + HR, nxt);
                        } else if (more) {
                            ta_nx = tile_addr(t1, e_nx);
                            load_chunk(ta_nx, 0, nxt);
                        }
#pragma unroll
                        for (int ah = 0; ah < HR; ++ah) {
                            const int al = a0 + ah;
                            const float2* br = bbase + al * bstride;
                            float2 kk[4];
#pragma unroll
                            for (int mm = 0; mm < 4; ++mm) kk[mm] = br[mm];
#pragma unroll
                            for (int mm = 0; mm < 4; ++mm) {
                                const float ar = cur[ah][mm].x, ai = ta.csg * cur[ah][mm].y;
                                const float b0 = bd ? kk[mm].y : kk[mm].x;
                                const float b1 = bd ? kk[mm].x : -kk[mm].y;
                                acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b0, acc0, 0, 0, 0);
                                acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b1, acc1, 0, 0, 0);
                            }
                        }
#pragma unroll
                        for (int ah = 0; ah < HR; ++ah)
#pragma unroll
                            for (int mm = 0; mm < 4; ++mm) cur[ah][mm] = nxt[ah][mm];
                    }
                    float2 tv_nx[4];
                    float tw_nx[4];
                    if (more) tile_data(es_nx, tv_nx, tw_nx);
                    const mfma_f4 acc = acc0 + acc1;
                    // ---- per-sample terms: lane n < NC of row group g4 adds term n
                    const int src0 = 16 * g4;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int qs = t0 + 4 * g4 + r;
                        const bool vr = qs < ntot;
                        const bool pr = vr && qs >= nv;
                        const float cval = (pr && bd) ? -acc[r] : acc[r];
                        const size_t o = (size_t)es[r].vidx * a.n_pol + pol;
                        if (MODE == kGrad) {
                            const int t = i16;
                            const float v_re = __shfl(cval, src0 + 0);
                            const float v_im = __shfl(cval, src0 + 1);
                            const float xr0 = __shfl(cval, src0 + t_xcol);
                            const float xi0 = __shfl(cval, src0 + t_xcol + 1);
                            const float yr0 = __shfl(cval, src0 + t_ycol);
                            const float yi0 = __shfl(cval, src0 + t_ycol + 1);
                            if (vr) {
                                if (a.vis_out != nullptr && t == 0) a.vis_out[o] = make_float2(v_re, v_im);
                                const float2 vo = tv[r];
                                const float rr = (float)((double)vo.x - (double)v_re);
                                const float ri = (float)((double)vo.y - (double)v_im);
                                const float xr = t_xr ? rr : xr0, xi = t_xr ? ri : xi0;
                                const float yr = t_yr ? rr : yr0, yi = t_yr ? ri : yi0;
                                const float val = fmaf(xr, yr, xi * yi);
                                if (t < 12) acc64 = fma((double)tw[r], (double)val, acc64);
                            }
                        } else {
                            const int t = i16 < 4 ? i16 : 0;
                            const float dr = __shfl(cval, src0 + 2 * t);
                            const float di = __shfl(cval, src0 + 2 * t + 1);
                            if (vr && i16 < 4) {
                                const float2 gv = tv[r];
                                acc64 += (double)gv.x * (double)dr + (double)gv.y * (double)di;
                            }
                        }
                    }
                    // the next tile's state becomes current
                    if (more) {
                        e_cur = e_nx;
                        ta = ta_nx;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            es[r] = es_nx[r];
                            tv[r] = tv_nx[r];
                            tw[r] = tw_nx[r];
                        }
                    }
                }
            } else {
                degrid(vb, nv, ent);
                if (g.n_vis2 > 0) {
                    // partner offset f' = -f: its sub-tables are the conjugates of
                    // these, reflected (b -> S-1-b on an axis with f != 0, b -> -b mod S
                    // on an axis with f = 0); rewrite them in place and degrid f'
                    const uint32_t vb2 = vb + (uint32_t)nv;
                    const int nv2 = g.n_vis2;
    #pragma unroll
                    for (int j = 0; j < SPL; ++j) {
                        const int v = slot + SPW * j;
                        ent[j] = a.vis[vb2 + (v < nv2 ? v : nv2 - 1)];
                    }
                    constexpr int PER = (NV * S * S) / 64;
                    float2 tmp[PER];
    #pragma unroll
                    for (int q = 0; q < PER; ++q) {
                        const int e = lane + 64 * q;
                        const int k = e / (S * S), b = e - k * S * S;
                        const int bl = b / S, bm = b - bl * S;
                        const int sl = fl ? (S - 1 - bl) : ((S - bl) & (S - 1));
                        const int sm = fm ? (S - 1 - bm) : ((S - bm) & (S - 1));
                        tmp[q] = uw[(k * S + sl) * SP + sm];
                    }
                    wave_sync();
    #pragma unroll
                    for (int q = 0; q < PER; ++q) {
                        const int e = lane + 64 * q;
                        const int k = e / (S * S), b = e - k * S * S;
                        const int bl = b / S, bm = b - bl * S;
                        uw[(k * S + bl) * SP + bm] = make_float2(tmp[q].x, -tmp[q].y);
                    }
                    wave_sync();
                    degrid(vb2, nv2, ent);
                }
            }
            wave_sync();  // the sub-table buffer is rewritten by the next group
            if (NC > 0) {
                // the group's own sums, in a fixed order, kept per group so the
                // item total does not depend on which wavefront took the group
#pragma unroll
                for (int off = S; off < 64; off <<= 1) acc64 += __shfl_xor(acc64, off);
                if (lane < NC) gpart[(gi - it.grp_begin) * NC + lane] = acc64;
                acc64 = 0.0;
            }
            gi = nxt_g;
            g = gnext;
        }

        // ---- per-item partial sums: groups added in group order
        __syncthreads();
        if (NC > 0 && tid < NC) {
            double sum = 0.0;
            for (int gg = 0; gg < it.grp_end - it.grp_begin; ++gg) sum += gpart[gg * NC + tid];
            a.partials[((size_t)item_idx * a.n_pol + pol) * NC + tid] = sum;
        }
        __syncthreads();
    }
}

// Per (interval, pol, antenna): sum the partials of every item touching the
// antenna, in a fixed order.  One wavefront each.
template <int NC>
__global__ void __launch_bounds__(64) k_reduce(ReduceArgs a)
{
    constexpr int NH = NC / 2;
    const int b = blockIdx.x;
    const int ant = b % a.n_ant;
    const int pol = (b / a.n_ant) % a.n_pol;
    const int s = a.int_begin + b / (a.n_ant * a.n_pol);
    if (a.done != nullptr && a.done[s]) return;
    const int lane = threadIdx.x;
    double sum[NH];
#pragma unroll
    for (int c = 0; c < NH; ++c) sum[c] = 0.0;
    const uint32_t e0 = a.ant_ptr[(size_t)s * a.n_ant + ant];
    const uint32_t e1 = a.ant_ptr[(size_t)s * a.n_ant + ant + 1];
    for (uint32_t e = e0 + lane; e < e1; e += 64) {
        const uint32_t ent = a.ant_ent[e];
        const uint32_t item = ent >> 1, end = ent & 1u;
        const double* p = a.partials + ((size_t)item * a.n_pol + pol) * NC + end * NH;
#pragma unroll
        for (int c = 0; c < NH; ++c) sum[c] += p[c];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < NH; ++c) sum[c] += __shfl_xor(sum[c], off);
    if (lane == 0) {
        double* o = a.out + (((size_t)s * a.n_pol + pol) * a.n_ant + ant) * NH;
#pragma unroll
        for (int c = 0; c < NH; ++c) o[c] = sum[c];
    }
}

// Damped 2x2 Gauss-Newton step per antenna, one block per interval.
__global__ void __launch_bounds__(256) k_solve(SolveArgs a)
{
    __shared__ double smax[256];
    const int s = a.int_begin + blockIdx.x;
    const int tid = threadIdx.x;
    if (a.done != nullptr && a.done[s]) {
        if (tid == 0 && a.max_step != nullptr) a.max_step[s] = 0.0;
        return;
    }
    double mx = 0.0;
    const int npa = a.n_pol * a.n_ant;
    for (int pa = tid; pa < npa; pa += blockDim.x) {
        const size_t k = (size_t)s * npa + pa;
        const double* t = a.acc + 6 * k;
        // H + mu diag(H) (mu = 0: the plain Gauss-Newton step)
        const double gl = t[1], gm = t[2], hll = t[3] * (1.0 + a.lm_mu), hlm = t[4];
        const double hmm = t[5] * (1.0 + a.lm_mu);
        const double tr = hll + hmm;
        const bool bad = !(isfinite(gl) && isfinite(gm) && isfinite(hll) && isfinite(hlm) &&
                           isfinite(hmm)) || !(tr > 0.0);
        if (a.not_updated != nullptr) a.not_updated[k] = bad ? 1 : 0;
        if (bad) continue;
        const double det = hll * hmm - hlm * hlm;
        double dl, dm;
        if (det > 1e-12 * tr * tr) {
            dl = (hmm * gl - hlm * gm) / det;
            dm = (hll * gm - hlm * gl) / det;
        } else {
            dl = hll > 0.0 ? gl / hll : 0.0;
            dm = hmm > 0.0 ? gm / hmm : 0.0;
        }
        dl *= a.gain;
        dm *= a.gain;
        a.offsets[2 * k] += dl;
        a.offsets[2 * k + 1] += dm;
        mx = fmax(mx, sqrt(dl * dl + dm * dm));
    }
    smax[tid] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) smax[tid] = fmax(smax[tid], smax[tid + w]);
        __syncthreads();
    }
    if (tid == 0) {
        const double m = smax[0];
        if (a.max_step != nullptr) a.max_step[s] = m;
        if (a.iters != nullptr) a.iters[s] += 1;
        if (a.done != nullptr) a.done[s] = (m < a.tol) ? 1 : 0;
    }
}

__global__ void k_init_state(int32_t* done, int32_t* iters, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        done[i] = 0;
        iters[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_taper_image(const double* img, const double* taper_pix, double2* out, int n,
                              hipStream_t s)
{
    const size_t tot = (size_t)n * n;
    k_taper_image<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(img, taper_pix, out, n);
    return hipGetLastError();
}

hipError_t launch_wplane_image(const double* img, const double* taper_pix, double2* out, int n, double cell,
                               double w, hipStream_t s)
{
    const size_t tot = (size_t)n * n;
    k_wplane_image<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(img, taper_pix, out, n, cell, w);
    return hipGetLastError();
}

hipError_t launch_fft_rows(double2* data, int n, int log2n, hipStream_t s)
{
    const size_t sh = sizeof(double2) * (size_t)n;
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_rows,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    k_fft_rows<<<n, 256, sh, s>>>(data, n, log2n);
    return hipGetLastError();
}

hipError_t launch_transpose(const double2* in, double2* out, int n, hipStream_t s)
{
    dim3 grid(n / 32, n / 32), block(32, 8);
    k_transpose<<<grid, block, 0, s>>>(in, out, n);
    return hipGetLastError();
}

hipError_t launch_finish_grid(const double2* in, float2* out, int n, int pad, hipStream_t s)
{
    const size_t tot = (size_t)(n + pad) * (n + pad);
    k_finish_grid<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(in, out, n, pad);
    return hipGetLastError();
}

hipError_t launch_zero(double2* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_zero<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_unpad_grid(const double2* g, double2* out, int n, int pad, hipStream_t s)
{
    const size_t tot = (size_t)n * n;
    k_unpad_grid<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(g, out, n, pad);
    return hipGetLastError();
}

hipError_t launch_image_grad(const double2* f, const double* taper_pix, double* out, int n, hipStream_t s)
{
    const size_t tot = (size_t)n * n;
    k_image_grad<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(f, taper_pix, out, n);
    return hipGetLastError();
}

hipError_t launch_airy_table(float4* tab, int n_tab, double dx, hipStream_t s)
{
    k_airy_table<<<(n_tab + 255) / 256, 256, 0, s>>>(tab, n_tab, dx);
    return hipGetLastError();
}

template <int S, int MODE, int SPL, bool MX>
static hipError_t launch_items_t(const ItemArgs& a, hipStream_t s)
{
    constexpr int NV = mode_nv(MODE);
    constexpr int NC = mode_nc(MODE) > 0 ? mode_nc(MODE) : 1;
    const int m2p = (a.m * a.m + 3) & ~3;
    const size_t gp = sizeof(double) * NC * a.oversample * a.oversample;
    const size_t sh = gp + sizeof(float) * NV * m2p + sizeof(float2) * kWaves * NV * S * (S + 1);
    // raise the dynamic LDS limit once, to the largest size any image_samples can need
    static const hipError_t attr = [] {
        const int mmax = 2 * S;
        const size_t shmax = sizeof(double) * NC * 256 + sizeof(float) * NV * ((mmax * mmax + 3) & ~3) +
                             sizeof(float2) * kWaves * NV * S * (S + 1);
        return hipFuncSetAttribute((const void*)k_item<S, MODE, SPL, MX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmax);
    }();
    if (attr != hipSuccess) return attr;
    const int blocks = (int)item_blocks(a.n_items);
    k_item<S, MODE, SPL, MX><<<blocks, kBlock, sh, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_items(int mode, int support, const ItemArgs& a, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    if (support != 16) return hipErrorInvalidValue;
    const bool mx = a.use_mfma != 0;
    switch (mode) {
    case kPredict: return launch_items_t<16, kPredict, 2, false>(a, s);
    case kGrid: return launch_items_t<16, kGrid, 2, false>(a, s);
    case kGrad:
        return mx ? launch_items_t<16, kGrad, 2, true>(a, s) : launch_items_t<16, kGrad, 2, false>(a, s);
    case kVjp:
        return mx ? launch_items_t<16, kVjp, 2, true>(a, s) : launch_items_t<16, kVjp, 2, false>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce(int ncontrib, const ReduceArgs& a, hipStream_t s)
{
    const int nb = (a.int_end - a.int_begin) * a.n_pol * a.n_ant;
    if (nb <= 0) return hipSuccess;
    if (ncontrib == 12)
        k_reduce<12><<<nb, 64, 0, s>>>(a);
    else if (ncontrib == 6)
        k_reduce<6><<<nb, 64, 0, s>>>(a);
    else if (ncontrib == 4)
        k_reduce<4><<<nb, 64, 0, s>>>(a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s)
{
    const int nb = a.int_end - a.int_begin;
    if (nb <= 0) return hipSuccess;
    k_solve<<<nb, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_init_state(int32_t* done, int32_t* iters, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_init_state<<<(n + 255) / 256, 256, 0, s>>>(done, iters, n);
    return hipGetLastError();
}

}  // namespace psc
