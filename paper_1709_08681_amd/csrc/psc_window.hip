// psc_window.hip -- degridding in the window form (supports 16 and 32).
//
// The table form (psc_kernels.hip) evaluates each sample as
//     V = sum_a V^{M0}[k_lo + a] T_f[S-1-a],
// where the sub-table T_f is the S-point 2-D DFT of the folded, twiddled
// image-plane products U_f[r] = sum_{n = r mod S} phi_f(n) g[n], with the
// per-axis phase phi_f(n) = exp(2 pi i f n / (S O)) (-1)^n / S.  Moving the DFT
// from the kernel onto the window (Parseval) and undoing the fold gives
//     V = sum_n g[n] phi_f(n) What[n mod S],
//     What[b] = sum_a' V^{M0}[k_lo + S-1-a'] exp(+2 pi i a'.b / S),
// the sum running over the M x M image samples.  This is the same quantity,
// term for term, as the A-projection degrid of Algorithm 1 with the kernel of
// Eq. MEDD; only the order of the sums differs.  Per sample it costs one S x S
// FFT of the window and an M x M dot product for all derivative variants
// (Eq. DA) at once, instead of NV S x S FFTs per sub-table, and it stores no
// sub-table: the form for few samples per sub-table (fine oversampling, short
// solution intervals) and for support 32, whose five sub-tables would not fit
// in LDS beside the image-plane products.
#include <algorithm>

#include "psc_device.h"

namespace psc {

// Image-plane factors per sample of the window form (sky frame): for predict,
// adjoint, gradient and beam scale.
__host__ __device__ constexpr int win_ng(int mode)
{
    return mode == kGrad || mode == kScale ? 3 : mode == kVjp ? 2 : 1;
}

// kFrameSkyAperture (psc_internal.h): a measured aperture in the sky frame
// (no parallactic angles); the pattern is fixed for the item, so its
// image-plane products are stored per image sample like the radial factors,
// but one per variant (the pattern is not radial, so the derivative sums do
// not factor).

// Factors stored per image sample by a window kernel of the given frame and
// mode (0: none, the mount frames evaluate them per sample).
__host__ __device__ constexpr int win_factors(int frame, int mode)
{
    return frame == kFrameSky           ? win_ng(mode)
           : frame == kFrameSkyAperture ? mode_nv(mode)
           : frame == kFrameSkyComplex  ? 2 * mode_nv(mode)
                                        : 0;
}

// A pattern with aperture defocus delta at displacement (dl, dm) from its
// beam centre, e = E and, with DERIV, de = dE/ddelta (complex).  Uniform disc:
// E = sum_n (i delta)^n / n! M_n(x), dE/ddelta = sum_n i^(n+1) delta^n / n!
// M_{n+1}(x), x = kk rho, M_n from the moment table (cubic Hermite).
// Gaussian mode: E = z exp(-z rho^2 / (2 s^2)), z = 1 / (1 - i kappa), kappa =
// kgd delta, dE/ddelta = kgd i z E (1 - z rho^2 / (2 s^2)).
template <bool DERIV>
__device__ __forceinline__ void efd(const ItemArgs& a, float kk, float inv_s2, float kgd, float delta, float dl,
                                    float dm, float2& e, float2& de)
{
    const float rho2 = fmaf(dl, dl, dm * dm);
    if (a.illum == 1) {
        const float kap = kgd * delta;
        const float den = __builtin_amdgcn_rcpf(fmaf(kap, kap, 1.f));
        const float zr = den, zi = kap * den;
        const float ah = 0.5f * rho2 * inv_s2;
        const float mag = __expf(-ah * zr);
        float sn, cs;
        __sincosf(-ah * zi, &sn, &cs);
        const float er = mag * cs, ei = mag * sn;
        e = make_float2(zr * er - zi * ei, zr * ei + zi * er);
        if (DERIV) {
            const float tr = fmaf(-ah, zr, 1.f), ti = -ah * zi;
            const float ur = zr * e.x - zi * e.y, ui = zr * e.y + zi * e.x;
            const float vr = ur * tr - ui * ti, vi = ur * ti + ui * tr;
            de = make_float2(-vi * kgd, vr * kgd);
        }
        return;
    }
    const float x = kk * __builtin_amdgcn_sqrtf(rho2);
    const float xs = x * a.inv_dx;
    int i0 = (int)xs;
    i0 = i0 < a.n_tab - 2 ? i0 : a.n_tab - 2;
    const float u = fminf(xs - (float)i0, 1.f);
    const float u1 = 1.f - u;
    const float h00 = (1.f + 2.f * u) * u1 * u1, h10 = u * u1 * u1, h01 = u * u * (3.f - 2.f * u),
                h11 = u * u * (u - 1.f);
    const float2* r0 = a.mtab + (size_t)i0 * kMoments;
    const float2* r1 = r0 + kMoments;
    float er = 0.f, ei = 0.f, dr = 0.f, di = 0.f, coef = 1.f;
    float mn;
    {
        const float2 p0 = r0[0], p1 = r1[0];
        mn = fmaf(h00, p0.x, fmaf(h10, p0.y, fmaf(h01, p1.x, h11 * p1.y)));
    }
#pragma unroll
    for (int n = 0; n < kMoments - 1; ++n) {
        const float2 p0 = r0[n + 1], p1 = r1[n + 1];
        const float mn1 = fmaf(h00, p0.x, fmaf(h10, p0.y, fmaf(h01, p1.x, h11 * p1.y)));
        // (i delta)^n / n! = i^n coef: the powers of i cycle 1, i, -1, -i
        switch (n & 3) {
        case 0: er = fmaf(coef, mn, er); if (DERIV) di = fmaf(coef, mn1, di); break;
        case 1: ei = fmaf(coef, mn, ei); if (DERIV) dr = fmaf(-coef, mn1, dr); break;
        case 2: er = fmaf(-coef, mn, er); if (DERIV) di = fmaf(-coef, mn1, di); break;
        default: ei = fmaf(-coef, mn, ei); if (DERIV) dr = fmaf(coef, mn1, dr); break;
        }
        coef *= delta * (1.f / (float)(n + 1));
        mn = mn1;
    }
    e = make_float2(er, ei);
    if (DERIV) de = make_float2(dr, di);
}

// Image-plane products of an item with complex patterns (aperture defocus,
// sky frame), [n][2 NV] (re, im): g = E_i conj(E_j) c, and for the defocus
// sums dE_i/ddelta_i conj(E_j) c and E_i conj(dE_j/ddelta_j) c.
template <int MODE>
__device__ __forceinline__ void image_factors_cx(const ItemArgs& a, float* gsh, float kk, float inv_s2, float kgd,
                                                 float di, float dj, float pil, float pim, float pjl, float pjm,
                                                 int tid, int nthr)
{
    constexpr bool D = MODE == kScale;
    constexpr int NG = 2 * mode_nv(MODE);
    const int m = a.m, half_m = m >> 1, m2 = m * m;
    const float hstep = (float)a.h;
    for (int idx = tid; idx < m2; idx += nthr) {
        const int il = idx / m, im = idx - il * m;
        const float l = (float)(il - half_m) * hstep, mm = (float)(im - half_m) * hstep;
        const float c = a.taper_img[il] * a.taper_img[im];
        float2 ei, dei, ej, dej;
        efd<D>(a, kk, inv_s2, kgd, di, l - pil, mm - pim, ei, dei);
        efd<D>(a, kk, inv_s2, kgd, dj, l - pjl, mm - pjm, ej, dej);
        float* gn = gsh + idx * NG;
        // x conj(y) c
        auto xcy = [&](float2 x, float2 y, float* o) {
            o[0] = c * fmaf(x.x, y.x, x.y * y.y);
            o[1] = c * fmaf(x.y, y.x, -x.x * y.y);
        };
        xcy(ei, ej, gn);
        if constexpr (D) {
            xcy(dei, ej, gn + 2);
            xcy(ei, dej, gn + 4);
        }
    }
}

// Image-plane factors of an item at the M x M samples, [n][NG]: g = E_i E_j c
// and, for the offsets' derivatives, the gradient factors q_i E_j c and
// E_i q_j c (dE/dp = q (l - p)), from which the sum forms the four derivative
// variants of Eq. DA; for the beam scales, dE/dsigma = q |l - p|^2 / sigma in
// place of q.  AP: a measured aperture, one stored product per variant (as
// mf_products_ap at angle zero).  bi, bj: each antenna's beam constants (its
// width scale applied).  HW: the hardware square root in the beam lookups
// (2.6% faster at support 32, 16% slower at 16).  pi, pj: the two antennas'
// tabulated (E, q) at the image samples (k_ant_beams), or null to evaluate
// them here from the Airy table tab.
template <int MODE, bool AP, bool HW>
__device__ __forceinline__ void image_factors(const ItemArgs& a, const float4* tab, const float2* pi,
                                              const float2* pj, int ai, int aj, float* gsh, const BeamK& bi,
                                              const BeamK& bj, float pil, float pim, float pjl, float pjm, int tid,
                                              int nthr)
{
    constexpr int NG = AP ? mode_nv(MODE) : win_ng(MODE);
    const int m = a.m, half_m = m >> 1, m2 = m * m;
    const float hstep = (float)a.h;
    const float inv_m = 1.f / (float)m;
    for (int idx = tid; idx < m2; idx += nthr) {
        // idx / m without an integer division: (idx + 1/2) / m lies at least
        // 1/(2m) from an integer, far beyond the float product's error
        const int il = (int)(((float)idx + 0.5f) * inv_m), im = idx - il * m;
        const float l = (float)(il - half_m) * hstep, mm = (float)(im - half_m) * hstep;
        const float dli = l - pil, dmi = mm - pim, dlj = l - pjl, dmj = mm - pjm;
        const float c = a.taper_img[il] * a.taper_img[im];
        float* gn = gsh + idx * NG;
        if constexpr (AP) {
            // the sky frame is the mount frame at angle zero
            float g[mode_nv(MODE)];
            mf_products_ap<MODE>(a, ap_table(a, ai), ap_table(a, aj), bi, bj, 1.f, 0.f, dli, dmi, dlj, dmj, c, g);
#pragma unroll
            for (int k = 0; k < NG; ++k) gn[k] = g[k];
        } else {
            float ei, qi, ej, qj;
            if (pi != nullptr) {
                const float2 ti = pi[idx], tj = pj[idx];
                ei = ti.x;
                qi = ti.y;
                ej = tj.x;
                qj = tj.y;
            } else {
                efq<HW>(a, tab, bi.kk, bi.inv_s2, dli, dmi, ei, qi);
                efq<HW>(a, tab, bj.kk, bj.inv_s2, dlj, dmj, ej, qj);
            }
            if constexpr (MODE == kPredict) {
                gn[0] = ei * ej * c;
            } else if constexpr (MODE == kScale) {
                gn[0] = ei * ej * c;
                gn[1] = qi * fmaf(dli, dli, dmi * dmi) * bi.rsig * ej * c;
                gn[2] = ei * qj * fmaf(dlj, dlj, dmj * dmj) * bj.rsig * c;
            } else {
                constexpr int o = MODE == kGrad ? 1 : 0;
                if constexpr (MODE == kGrad) gn[0] = ei * ej * c;
                gn[o] = qi * ej * c;
                gn[o + 1] = ei * qj * c;
            }
        }
    }
}

// Cross-half exchanges without the LDS crossbar.  v_permlane32_swap(v, v)
// returns (lanes 0-31 of v in both halves, lanes 32-63 of v in both halves);
// v_permlane16_swap(a, b) swaps the odd 16-lane rows of a with the even rows
// of b: it returns (a's rows 0 and 2 each followed by b's, a's rows 1 and 3
// each followed by b's), so with a = b the sum of its two results is the sum
// of lane l and lane l ^ 16.
__device__ __forceinline__ void halves32(float v, float& lo, float& hi)
{
    const unsigned u = __builtin_bit_cast(unsigned, v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    lo = __builtin_bit_cast(float, (unsigned)r[0]);
    hi = __builtin_bit_cast(float, (unsigned)r[1]);
}
// Sums over the 2S lanes of a worker of two values at once, each total in
// every lane of the worker.  One row swap pairs a's and b's partial sums of
// the two (at support 32: four) 16-lane rows so that the rows hold a and b
// alternately; one 16-lane reduction then serves both values, and a last
// swap hands each row the other's total.  Seven instructions for two values
// at support 16 against six for each one alone.
template <int S>
__device__ __forceinline__ void worker_sum2(float& a, float& b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a),
                                                    __builtin_bit_cast(unsigned, b), false, false);
    // rows (a0 + a1, b0 + b1, a2 + a3, b2 + b3)
    float p = __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
    if constexpr (S == 32) {
        float lo, hi;
        halves32(p, lo, hi);
        p = lo + hi;
    }
    p = row16_sum(p);
    const auto q = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, p),
                                                    __builtin_bit_cast(unsigned, p), false, false);
    a = __builtin_bit_cast(float, (unsigned)q[0]);
    b = __builtin_bit_cast(float, (unsigned)q[1]);
}

// The two halves of a worker of 2S lanes: (value of lane (0, c), value of
// lane (1, c)) in every lane (h, c).
template <int S>
__device__ __forceinline__ void halves(float v, float& lo, float& hi)
{
    if constexpr (S == 32) {
        halves32(v, lo, hi);
    } else {
        static_assert(S == 16, "supports 16 and 32");
        const unsigned u = __builtin_bit_cast(unsigned, v);
        const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        lo = __builtin_bit_cast(float, (unsigned)r[0]);
        hi = __builtin_bit_cast(float, (unsigned)r[1]);
    }
}

// Wavefronts per SIMD the window kernel asks the compiler to fit.
__host__ __device__ constexpr int win_min_waves(int S, int MF, bool WT)
{
    return S == 16 && (MF == kFrameMount || (WT && MF == kFrameSky)) ? 3
         : S == 32 && MF == kFrameMount && !WT ? 2 : 1;
}

// ---------------------------------------------------------------------------
// Workers of 2S lanes: a wavefront per sample at support 32, half a wavefront
// at support 16.
//
// One block of W wavefronts per item (in the sky frame at support 32, per
// run of win_items_per_block consecutive items, taken one after another and
// sharing the block's set-up).  The item's n samples, in row order (time
// order along the baseline's uv track), are split among the workers in
// contiguous shares: worker w takes [w n / NW, (w + 1) n / NW).  A worker
// loads its next sample's entry, window and inputs while it transforms and
// sums the current one, so the chain of dependent loads (entry, then
// window) stays off the critical path, and it keeps its window transform
// while consecutive samples share a window; the float64 sums are kept per
// worker and added in worker order.
//
// Lane (h, c) of a worker loads rows [Hh, Hh + H) of column c of the reversed
// window, H = S/2.  Each S-point transform is split in its first radix-2
// step: the half h = 0 keeps the sum of the two halves' points, h = 1 their
// difference times exp(+2 pi i r / S), and each finishes with an H-point
// transform, giving the outputs 2b + h.  Along l the columns go through the
// worker's LDS tile; along m lane (h, c) reads row c, and multiplies it by the
// l-axis phase phi_l(n) of the image-sample index n in [-M/2, S - M/2)
// congruent to c before writing it back, so the sum needs no phase per image
// sample: the samples n + S carry the common factor exp(2 pi i f_l / O), and
// the m-axis phase is the lane's own.  In the sum lane (h, c) takes the
// image-sample m index n_m = c - S h (M/2 of the S lanes of each half have
// one).
//
// MT: the image-sample count per axis when fixed at compile time (the
// default 3S/2, sky frame), 0 to read it from the arguments; fixed, the
// image-sample sums run with constant trip counts.  The mount frame at
// support 16 asks for three wavefronts per SIMD (a few registers spill;
// 13% faster on the single-interval workload than two), and so does the
// sky frame's w-term, which needs a register or two more than three allow;
// the mount frame at support 32 asks for two (without the bound its
// gradient spills into accumulation registers and runs at one).
template <int S, int MODE, int MF, int W, bool WT, int MT = 0>
__global__ void __launch_bounds__(64 * W, win_min_waves(S, MF, WT)) k_winw(ItemArgs a)
{
    constexpr int H = S / 2, SP = S + 1;
    constexpr int SL = 2 * S;    // lanes per worker
    constexpr int SPW = 64 / SL;  // workers per wavefront
    constexpr int NW = W * SPW;   // workers per block
    constexpr int NV = mode_nv(MODE);
    constexpr int NC = mode_nc(MODE);
    constexpr int NCP = NC > 0 ? NC : 1;
    constexpr bool CPLX = MF == kFrameSkyComplex;  // complex patterns: complex products
    constexpr bool SKY = MF == kFrameSky || MF == kFrameSkyAperture || CPLX;  // factors stored per image sample
    // one stored factor per variant, summed plainly (no factored derivatives)
    constexpr bool PLAIN = MODE == kScale || MF == kFrameSkyAperture || CPLX;
    constexpr int NG = SKY ? win_factors(MF, MODE) : 1;  // image-plane factors per image sample
    constexpr int kBlock = 64 * W;
    static_assert(NC <= SL, "one term per lane");

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float2 twsh[S * 16];  // exp(+2 pi i t / (S O)), S O <= 16 S

    const int m = MT > 0 ? MT : a.m, half_m = m >> 1;
    const int m2p = (m * m + 3) & ~3;
    constexpr int kUnroll = 4;
    const int O = a.oversample, so = S * O;
    // dynamic LDS: per-worker float64 sums | image-plane factors [n][NG]
    // (sky frame) | window tiles | Airy table (mount frame)
    double* gpart = reinterpret_cast<double*>(smem);  // [NW][NCP]
    float* gsh = reinterpret_cast<float*>(gpart + NW * NCP);
    float2* wtile = reinterpret_cast<float2*>(gsh + (SKY ? NG * m2p : 0));
    // each lane's share of its worker's current window transform, before the
    // sample's phases, kept while samples share the window: in LDS at
    // support 16 ([H][block lanes]; in registers it would cost a wavefront
    // per SIMD), in registers at 32 (whose blocks are bound by LDS)
    constexpr bool YLDS = S == 16;
    float2* ybuf = wtile + (size_t)NW * S * SP;
    float4* airy_sh = reinterpret_cast<float4*>(ybuf + (YLDS ? (size_t)H * kBlock : 0));

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the block's items: in the sky frame at support 32, unit_items
    // consecutive ones, which share the block's set-up below (the twiddles
    // and the Airy table in LDS); otherwise one (a loop over items costs the
    // other variants registers, and some of them a wavefront per SIMD)
    constexpr bool MULTI = win_multi_item(S, MF);
    const int R = MULTI && a.unit_items > 1 ? a.unit_items : 1;
    const long long li0_wide = (long long)item_of_block() * R;
    if (li0_wide >= a.n_items) return;
    const int li0 = (int)li0_wide;

    const int N = a.grid_n;
    const float inv_s = 1.0f / (float)S;
    const int P = N + S;  // pitch of the padded grid
    const int rowbytes = P * (int)sizeof(float2);
    // the model grid, or with w-stacking the stack of its w-planes (each
    // (N+S)^2, at most 2 GiB together)
    const bool stacked = WT && a.w_nk > 0;
    const int plane_bytes = P * P * (int)sizeof(float2);
    const __amdgpu_buffer_rsrc_t grsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(stacked ? a.wgrid : a.grid), (short)0, (stacked ? a.w_nk : 1) * plane_bytes, 0x00020000);

    for (int t = tid; t < so; t += kBlock) twsh[t] = a.tw[t];
    // the Airy table: in LDS for the mount frame's per-sample lookups, and
    // for the sky frame's image-plane factors when it fits beside two blocks
    // (support 32) and the antennas' patterns are not tabulated
    const bool btab = MF == kFrameSky && S == 16 && a.beams != nullptr;
    const bool tlds = MF == kFrameMount || (MF == kFrameSky && S == 32 && a.tab_lds && !btab);
    if (tlds)
        for (int t = tid; t < a.n_tab; t += kBlock) airy_sh[t] = a.airy[t];
    __syncthreads();
    auto one_item = [&](const int li) {
        if (li >= a.n_items) return;
        const int item_idx = a.item_begin + li;
        const Item it = a.items[item_idx];
        if (a.done != nullptr && a.done[it.interval]) return;

        const int sl = lane & (SL - 1);  // lane within the worker
        const int worker = wave * SPW + lane / SL;
        const int c = sl & (S - 1), hh = sl / S;
        float2* wt = wtile + (size_t)worker * S * SP;  // this worker's tile
        const TermSel tsel(sl);
        const float2 zero = make_float2(0.f, 0.f);
        // the lane's image-sample m index, and the l index its transform row c
        // stands for
        const int nm = c - hh * S;
        const bool m_ok = nm >= -half_m && nm < half_m;
        const int jm = m_ok ? nm + half_m : 0;
        const int nl_row = ((c + half_m) & (S - 1)) - half_m;
        // first radix-2 step of an S-point transform: half h keeps
        // (x_r + (-1)^h x_{H+r}) exp(+2 pi i h r / S)
        const float sgn = hh ? -1.f : 1.f;
        float2 tw1[H];
    #pragma unroll
        for (int r = 0; r < H; ++r)
            tw1[r] = hh ? make_float2(kTw.re[(64 / S) * r], kTw.im[(64 / S) * r]) : make_float2(1.f, 0.f);

        // (-1)^n exp(2 pi i f n / (S O)) / S
        auto phase = [&](int f, int n) {
            const float2 t = twsh[(f * n) & (so - 1)];
            const float sg = (n & 1) ? -inv_s : inv_s;
            return make_float2(t.x * sg, t.y * sg);
        };
        // The item's samples in row order (time order along the baseline's uv
        // track), each worker a contiguous share [k_lo, k_hi): consecutive
        // samples of one worker often fall in the same window (a track moves a
        // fraction of a cell per integration), whose transform is then reused.
        const int n_s = it.n_vis;
        const int k_lo = (int)(((long long)worker * n_s) / NW), k_hi = (int)(((long long)(worker + 1) * n_s) / NW);
        const VisEnt* went = a.wvis + it.vis_begin;
        const uint8_t* wfp = a.wf + it.vis_begin;
        // rows H hh + r of the reversed column c: grid row k_lo_l + S-1-(H hh + r),
        // of w-plane `plane` when stacked
        auto load_window = [&](const VisEnt& e, int plane, float2 (&x)[H]) {
            const int row0 = (int)(e.klo >> 16);
            const int col0 = (int)(e.klo & 0xffffu);
            const int voff = plane * plane_bytes + (row0 * P + col0 + (S - 1 - c)) * (int)sizeof(float2) +
                             (1 - hh) * H * rowbytes;
    #pragma unroll
            for (int r = 0; r < H; ++r)
                x[r] = __builtin_bit_cast(
                    float2, __builtin_amdgcn_raw_buffer_load_b64(grsrc, voff, (H - 1 - r) * rowbytes, 0));
        };

        // mount frame: beam constants of the item's channel, the lane's
        // image-sample m coordinate and taper value
        const double lam = kCLight / a.freq[it.chan];
        const float kk = (float)(kPi * a.dish / lam);
        const double sigma = a.gauss_sigma_ld * lam / a.dish;
        const float inv_s2 = (float)(1.0 / (sigma * sigma));
        const float aps = (float)(a.dish / lam * a.ap_inv_step);  // aperture table nodes per radian
        const float hstep = (float)a.h;
        const float mmy = (float)nm * hstep;
        // w-term: w in wavelengths per metre at the item's channel, and the
        // lane's m^2
        const double w_per_m = a.freq[it.chan] / kCLight;
        const float mm2 = mmy * mmy;
        // exp(2 pi i w (n - 1)) at (l, lane's m), n - 1 = -x / (1 + sqrt(1 - x)),
        // from the hardware sine and cosine of the phase in turns reduced to
        // [0, 1) (the phase itself is a float32 product; the parity tests bound
        // the result)
        // a sample's w in wavelengths, and with w-stacking its plane k (the one
        // nearest, w_k = k dw) and the residual w - w_k that the kernel carries
        auto wsel = [&](const VisEnt& e, float& wr, int& plane) {
            const double wl = a.w_m[e.vidx / (uint32_t)a.n_chan] * w_per_m;
            if (stacked) {
                const int k = min(max((int)rint(wl / a.w_dw), a.w_k0), a.w_k0 + a.w_nk - 1);
                wr = (float)(wl - (double)k * a.w_dw);
                plane = k - a.w_k0;
            } else {
                wr = (float)wl;
                plane = 0;
            }
        };
        auto wphase = [&](float wl, float l) {
            const float x = fmaf(l, l, mm2);
            const float nm1 = -x * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_sqrtf(1.f - x));
            const float r = __builtin_amdgcn_fractf(wl * nm1);
            return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
        };
        const float ctm = a.taper_img[jm];

        for (int pol = 0; pol < a.n_pol; ++pol) {
            // this worker's first sample and the entry after it, the first window
            int k0 = k_lo;
            VisEnt e0 = {0u, 0u}, e1 = {0u, 0u};
            int f0 = 0, f1 = 0;
            float2 x0[H];
            float2 vin0 = zero;
            float wgt0 = 0.f, w0 = 0.f;
            int pl0 = 0;
            if (k0 < k_hi) {
                e0 = went[k0];
                f0 = wfp[k0];
                const int k1 = k0 + 1 < k_hi ? k0 + 1 : k0;  // past the end: the last (loads stay in bounds)
                e1 = went[k1];
                f1 = wfp[k1];
                if constexpr (WT) wsel(e0, w0, pl0);
                load_window(e0, pl0, x0);
                const size_t o0 = (size_t)e0.vidx * a.n_pol + pol;
                if (MODE != kPredict) vin0 = a.vis_in[o0];
                if (MODE == kGrad || MODE == kScale) wgt0 = a.weight[o0];
            }

            // offsets plus squint (along l, or along the mount's first axis)
            const double sq = (pol == 0 ? 1.0 : -1.0) * a.squint_frac * 1.02899 * lam / a.dish;
            const double* oi = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.ai) * 2;
            const double* oj = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.aj) * 2;
            const double qil = oi[0] + sq, qim = oi[1], qjl = oj[0] + sq, qjm = oj[1];
            // each antenna's beam constants with its width scale
            BeamK bki = beam_k(kk, inv_s2, aps, 1.f), bkj = bki;
            if (a.scale != nullptr) {
                const double* sc = a.scale + ((size_t)it.interval * a.n_pol + pol) * a.n_ant;
                bki = beam_k(kk, inv_s2, aps, (float)sc[it.ai]);
                bkj = beam_k(kk, inv_s2, aps, (float)sc[it.aj]);
            }
            if constexpr (CPLX) {
                const double* dfp = a.defocus + ((size_t)it.interval * a.n_pol + pol) * a.n_ant;
                const float kgd = (float)(2.0 / (kPi * kPi * a.gauss_sigma_ld * a.gauss_sigma_ld));
                image_factors_cx<MODE>(a, gsh, kk, inv_s2, kgd, (float)dfp[it.ai], (float)dfp[it.aj], (float)qil,
                                       (float)qim, (float)qjl, (float)qjm, tid, kBlock);
            } else if constexpr (SKY) {
                const float2 *pi = nullptr, *pj = nullptr;
                if constexpr (S == 16) {  // tables only at support 16 (none compiled at 32)
                    if (btab) {
                        const size_t t0 = (((size_t)it.interval * a.n_pol + pol) * a.n_chan + it.chan) * a.n_ant;
                        pi = a.beams + (t0 + it.ai) * (size_t)(a.m * a.m);
                        pj = a.beams + (t0 + it.aj) * (size_t)(a.m * a.m);
                    }
                }
                image_factors<MODE, MF == kFrameSkyAperture, S == 32>(a, tlds ? airy_sh : a.airy, pi, pj, it.ai, it.aj,
                                                                       gsh, bki, bkj, (float)qil, (float)qim,
                                                                       (float)qjl, (float)qjm, tid, kBlock);
            }
            __syncthreads();

            double acc64 = 0.0;
            bool need0 = true;
            float2 y[H];
            while (k0 < k_hi) {
                // ---- fetch ahead: the next sample's window (when it differs), its
                // inputs, the entry after it
                const bool more = k0 + 1 < k_hi;
                float w1 = 0.f;
                int pl1 = 0;
                if constexpr (WT) wsel(e1, w1, pl1);
                const bool need1 = more && (e1.klo != e0.klo || pl1 != pl0);
                float2 x1[H];
                if (need1) load_window(e1, pl1, x1);
                const size_t o1 = (size_t)e1.vidx * a.n_pol + pol;
                float2 vin1 = zero;
                float wgt1 = 0.f;
                if (MODE != kPredict) vin1 = a.vis_in[o1];
                if (MODE == kGrad || MODE == kScale) wgt1 = a.weight[o1];
                const int k2 = k0 + 2 < k_hi ? k0 + 2 : k_hi - 1;
                const VisEnt e2 = went[k2];
                const int f2 = wfp[k2];

                // ---- the current sample's sub-lattice offset per axis
                const int fl = f0 >> 4, fm = f0 & 15;

                if (need0) {
                    // ---- along l: first radix-2 step across the halves, then H points
    #pragma unroll
                    for (int r = 0; r < H; ++r) {
                        // the column's rows r (half 0) and H + r (half 1), in every lane
                        float tx, bx, ty, by;
                        halves<S>(x0[r].x, tx, bx);
                        halves<S>(x0[r].y, ty, by);
                        y[r] = make_float2(fmaf(sgn, bx, tx), fmaf(sgn, by, ty));
                        if (r > 0) y[r] = cmul(y[r], tw1[r]);
                    }
                    fft_reg<H>(y);
                    wave_sync();  // the previous sample's tile has been read
    #pragma unroll
                    for (int b = 0; b < H; ++b) wt[(2 * b + hh) * SP + c] = y[b];
                    wave_sync();
                    // ---- along m: row c, the same split
    #pragma unroll
                    for (int r = 0; r < H; ++r) {
                        const float2 t0 = wt[c * SP + r], t1 = wt[c * SP + H + r];
                        y[r] = make_float2(fmaf(sgn, t1.x, t0.x), fmaf(sgn, t1.y, t0.y));
                        if (r > 0) y[r] = cmul(y[r], tw1[r]);
                    }
                    fft_reg<H>(y);
                    if constexpr (YLDS) {
    #pragma unroll
                        for (int b = 0; b < H; ++b) ybuf[b * kBlock + tid] = y[b];
                    }
                } else if constexpr (YLDS) {
    #pragma unroll
                    for (int b = 0; b < H; ++b) y[b] = ybuf[b * kBlock + tid];
                }
                // ---- row c times the sample's l-axis phase of the row's index
                const float2 prow = phase(fl, nl_row);
                wave_sync();  // the tile (the previous sample's, or the transpose) has been read
    #pragma unroll
                for (int b = 0; b < H; ++b) wt[c * SP + 2 * b + hh] = cmul(y[b], prow);
                wave_sync();
                // ---- A_k, B_k: sums over l of g_k[n_l][n_m] T[n_l mod 32][c] for
                // n_l below and above 32 - M/2
                float2 A[NV], B[NV];
    #pragma unroll
                for (int k = 0; k < NV; ++k) A[k] = B[k] = zero;
                float cs = 1.f, sn = 0.f;
                if constexpr (!SKY) {
                    // this row's beam centres on the sky
                    sincosf((float)a.par_angle[e0.vidx / (uint32_t)a.n_chan], &sn, &cs);
                    const float pil = (float)(cs * qil - sn * qim), pim = (float)(sn * qil + cs * qim);
                    const float pjl = (float)(cs * qjl - sn * qjm), pjm = (float)(sn * qjl + cs * qjm);
                    const float4 *api = nullptr, *apj = nullptr;  // the two antennas' aperture tables
                    if constexpr (MF == kFrameAperture) {
                        api = ap_table(a, it.ai);
                        apj = ap_table(a, it.aj);
                    }
                    auto term = [&](int jl, float2 (&acc)[NV]) {
                        const float l = (float)(jl - half_m) * hstep;
                        float2 t = wt[((jl - half_m) & (S - 1)) * SP + c];
                        if constexpr (WT) t = cmul(t, wphase(w0, l));
                        float g[NV];
                        if constexpr (MF == kFrameAperture)
                            mf_products_ap<MODE>(a, api, apj, bki, bkj, cs, sn, l - pil, mmy - pim, l - pjl,
                                                 mmy - pjm, a.taper_img[jl] * ctm, g);
                        else
                            mf_products<MODE>(a, airy_sh, bki, bkj, l - pil, mmy - pim, l - pjl, mmy - pjm,
                                              a.taper_img[jl] * ctm, g);
    #pragma unroll
                        for (int k = 0; k < NV; ++k) {
                            acc[k].x = fmaf(g[k], t.x, acc[k].x);
                            acc[k].y = fmaf(g[k], t.y, acc[k].y);
                        }
                    };
    #pragma unroll 2
                    for (int jl = 0; jl < S; ++jl) term(jl, A);
    #pragma unroll 2
                    for (int jl = S; jl < m; ++jl) term(jl, B);
                } else {
                    // factored sums: the value sum g T, and per antenna Q = sum q T
                    // and L = sum q l T, l the image-sample l coordinate (the
                    // variant dV/dp_l = L - p_l Q, dV/dp_m = (m - p_m) Q).  L comes
                    // from running sums: over the part's rows n < j1 in order,
                    // Q += q T and then P += Q leave P = sum (j1 - n) q T, so with
                    // l = (n - M/2) h, L = h ((j1 - M/2) Q - P): no product by l
                    // per row (the float32 error stays within twice that of the
                    // direct sum, coherent rows included).
                    const float* gp = gsh + jm * NG;
                    // the halves read factors S samples apart, S NG words: an odd
                    // multiple of 32 for NG odd, so they use disjoint banks
                    // image-sample rows [j0, j1) at tile rows b0, b0 + 1, ... (no wrap)
                    auto seg = [&](int j0, int j1, int b0, float2 (&acc)[NV]) {
                        const float2* tp = wt + b0 * SP + c;
                        const float* g = gp + j0 * m * NG;
    #pragma unroll kUnroll
                        for (int jl = j0; jl < j1; ++jl, tp += SP, g += m * NG) {
                            float2 t = *tp;
                            if constexpr (WT) t = cmul(t, wphase(w0, (float)(jl - half_m) * hstep));
                            if constexpr (CPLX) {
                                // one plain sum per variant, complex products
    #pragma unroll
                                for (int k = 0; k < NV; ++k) {
                                    const float gr = g[2 * k], gi = g[2 * k + 1];
                                    acc[k].x = fmaf(gr, t.x, fmaf(-gi, t.y, acc[k].x));
                                    acc[k].y = fmaf(gr, t.y, fmaf(gi, t.x, acc[k].y));
                                }
                            } else if constexpr (PLAIN) {
                                // one plain sum per variant
    #pragma unroll
                                for (int k = 0; k < NV; ++k) {
                                    acc[k].x = fmaf(g[k], t.x, acc[k].x);
                                    acc[k].y = fmaf(g[k], t.y, acc[k].y);
                                }
                            }
                            if constexpr (MODE != kVjp && !PLAIN) {
                                acc[0].x = fmaf(g[0], t.x, acc[0].x);
                                acc[0].y = fmaf(g[0], t.y, acc[0].y);
                            }
                            if constexpr (MODE != kPredict && !PLAIN) {
                                constexpr int o = MODE == kGrad ? 1 : 0;
    #pragma unroll
                                for (int end = 0; end < 2; ++end) {
                                    const float q = g[o + end];
                                    float2& P = acc[o + 2 * end];
                                    float2& Q = acc[o + 2 * end + 1];
                                    Q.x = fmaf(q, t.x, Q.x);
                                    Q.y = fmaf(q, t.y, Q.y);
                                    P.x += Q.x;
                                    P.y += Q.y;
                                }
                            }
                        }
                    };
                    // n_l in [-M/2, 0) is tile row n_l + 32 and [0, 32 - M/2) row
                    // n_l (the A part); [32 - M/2, M/2) is row n_l, the row of
                    // n_l - 32 (the B part)
                    seg(0, half_m, S - half_m, A);
                    seg(half_m, S, 0, A);
                    seg(S, m, S - half_m, B);
                    if constexpr (MODE != kPredict && !PLAIN) {
                        // L from P and Q: the A part ends at row S, the B part at M
                        constexpr int o = MODE == kGrad ? 1 : 0;
                        const float ca = (float)(S - half_m), cb = (float)(m - half_m);
    #pragma unroll
                        for (int end = 0; end < 2; ++end) {
                            float2& pa = A[o + 2 * end];
                            float2& pb = B[o + 2 * end];
                            const float2 qa = A[o + 2 * end + 1], qb = B[o + 2 * end + 1];
                            pa = make_float2(hstep * fmaf(ca, qa.x, -pa.x), hstep * fmaf(ca, qa.y, -pa.y));
                            pb = make_float2(hstep * fmaf(cb, qb.x, -pb.x), hstep * fmaf(cb, qb.y, -pb.y));
                        }
                    }
                }
                // ---- s_k = phi_m(n_m) (A_k + exp(2 pi i f_l / O) B_k), summed over the worker
                const float2 rho = twsh[(fl * S) & (so - 1)];
                const float2 pm = m_ok ? phase(fm, nm) : zero;
                float2 s[NV];
    #pragma unroll
                for (int k = 0; k < NV; ++k) {
                    const float2 rb = cmul(rho, B[k]);
                    s[k] = cmul(pm, make_float2(A[k].x + rb.x, A[k].y + rb.y));
                }
                if constexpr (SKY && !PLAIN && MODE != kPredict) {
                    // derivative variants from the factored sums (the lane's m coordinate is mmy)
                    constexpr int o = MODE == kGrad ? 1 : 0;
                    const float pl[2] = {(float)qil, (float)qjl}, pmm[2] = {(float)qim, (float)qjm};
    #pragma unroll
                    for (int end = 0; end < 2; ++end) {
                        const float2 L = s[o + 2 * end], Q = s[o + 2 * end + 1];
                        const float dm = mmy - pmm[end];
                        s[o + 2 * end] = make_float2(fmaf(-pl[end], Q.x, L.x), fmaf(-pl[end], Q.y, L.y));
                        s[o + 2 * end + 1] = make_float2(dm * Q.x, dm * Q.y);
                    }
                }
    #pragma unroll
                for (int k = 0; k < NV; ++k) worker_sum2<S>(s[k].x, s[k].y);
                if constexpr (MF == kFrameMount && MODE != kPredict && MODE != kScale) {
                    // derivatives with respect to the mount-frame offsets
                    constexpr int d0 = (MODE == kGrad) ? 1 : 0;
    #pragma unroll
                    for (int end = 0; end < 2; ++end) {
                        const float2 dl = s[d0 + 2 * end], dm = s[d0 + 2 * end + 1];
                        s[d0 + 2 * end] = make_float2(cs * dl.x + sn * dm.x, cs * dl.y + sn * dm.y);
                        s[d0 + 2 * end + 1] = make_float2(cs * dm.x - sn * dl.x, cs * dm.y - sn * dl.y);
                    }
                }
                const size_t o0 = (size_t)e0.vidx * a.n_pol + pol;
                if constexpr (MODE == kPredict) {
                    if (sl == 0) a.vis_out[o0] = s[0];
                } else if constexpr (MODE == kGrad) {
                    if (a.vis_out != nullptr && sl == 0) a.vis_out[o0] = s[0];
                    grad_term(tsel, s, vin0, wgt0, acc64);
                } else if constexpr (MODE == kScale) {
                    scale_term(sl, s, vin0, wgt0, acc64);
                } else {
                    vjp_term(sl, s, vin0, acc64);
                }

                // ---- move on
                if (need1) {
    #pragma unroll
                    for (int r = 0; r < H; ++r) x0[r] = x1[r];
                }
                need0 = need1;
                vin0 = vin1;
                wgt0 = wgt1;
                w0 = w1;
                pl0 = pl1;
                e0 = e1;
                f0 = f1;
                e1 = e2;
                f1 = f2;
                ++k0;
            }

            // ---- per-item partial sums: workers added in order
            if (NC > 0 && sl < NC) gpart[worker * NCP + sl] = acc64;
            __syncthreads();
            if (NC > 0 && tid < NC) {
                double sum = 0.0;
    #pragma unroll
                for (int w = 0; w < NW; ++w) sum += gpart[w * NCP + tid];
                a.partials[((size_t)item_idx * a.n_pol + pol) * NC + tid] = sum;
            }
            __syncthreads();
        }
    };
    if constexpr (MULTI) {
        for (int r = 0; r < R && r < a.n_items - li0; ++r) one_item(li0 + r);
    } else {
        one_item(li0);
    }
}

// Whether a sky-frame block at support 32 stages the Airy table in LDS: when
// a four-wavefront block with it still leaves room for a second block on the
// compute unit (the lookups of the image-plane factors then stay on chip).
static bool sky_tab_lds(int support, int mode, int frame, int m, int oversample, int n_tab)
{
    if (frame != kFrameSky || support != 32) return false;
    const size_t b4 = winw_lds_bytes(support, 4, mode, m, oversample, -1) + sizeof(float4) * (size_t)n_tab;
    return 2 * (b4 + (160 * 1024 - win_lds_budget(support))) <= 160 * 1024;
}

// Dynamic LDS of a k_winw block of the given frame: winw_lds_bytes, with the
// stored factors counted per frame.
static size_t winw_frame_lds(int support, int waves, int mode, int frame, int m, int oversample, int n_tab)
{
    const size_t m2p = (size_t)((m * m + 3) & ~3);
    const int tab = frame == kFrameMount ? n_tab : frame == kFrameSky ? -1 : 0;
    size_t b = winw_lds_bytes(support, waves, mode, m, oversample, tab);
    if (sky_tab_lds(support, mode, frame, m, oversample, n_tab)) b += sizeof(float4) * (size_t)n_tab;
    // frames with stored products other than the radial factors: the base
    // size counts none (tab = 0), so all of them are added here
    if (frame == kFrameSkyAperture || frame == kFrameSkyComplex)
        b += sizeof(float) * (size_t)win_factors(frame, mode) * m2p;
    return b;
}

int win_block_waves(int support, int mode, int frame, int m, int oversample, int n_tab, int plan_waves)
{
    // items of few samples at support 16: one or two wavefronts (two or four
    // workers) per block, as the plan chose
    if (support == 16 && (plan_waves == 1 || plan_waves == 2)) return plan_waves;
    // four wavefronts when two blocks fit a compute unit's LDS, else eight
    // (support 32 with many image samples)
    const size_t budget = win_lds_budget(support);
    const size_t sh4 = winw_frame_lds(support, 4, mode, frame, m, oversample, n_tab);
    if (2 * (sh4 + (160 * 1024 - budget)) <= 160 * 1024) return 4;
    if (support == 32 && winw_frame_lds(support, 8, mode, frame, m, oversample, n_tab) <= budget) return 8;
    return 0;
}

// The dynamic LDS a k_winw<S, MODE, MF, W> block lays out (the kernel's own
// arithmetic): float64 sums, stored products, tiles, the transform kept for
// reuse, the Airy table.  A launch whose allocation is smaller is refused.
template <int S, int MODE, int MF, int W>
static size_t winw_layout_bytes(int m, int n_tab, bool tab_lds)
{
    constexpr int NW = W * (64 / (2 * S));
    constexpr int NC = mode_nc(MODE);
    constexpr bool SKY = MF == kFrameSky || MF == kFrameSkyAperture || MF == kFrameSkyComplex;
    const size_t m2p = (size_t)((m * m + 3) & ~3);
    size_t b = sizeof(double) * NW * (NC > 0 ? NC : 1);
    b += SKY ? sizeof(float) * (size_t)win_factors(MF, MODE) * m2p : 0;
    b += sizeof(float2) * (size_t)NW * S * (S + 1);
    b += S == 16 ? sizeof(float2) * (size_t)(S / 2) * 64 * W : 0;
    b += MF == kFrameMount || (MF == kFrameSky && S == 32 && tab_lds) ? sizeof(float4) * (size_t)n_tab : 0;
    return b;
}

template <int S, int MODE, int MF, int W, bool WT, int MT>
static hipError_t launch_win_wm(const ItemArgs& a, hipStream_t s)
{
    // raise the dynamic LDS limit once, to what one compute unit allows
    static const hipError_t attr = hipFuncSetAttribute(
        (const void*)k_winw<S, MODE, MF, W, WT, MT>, hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)win_lds_budget(S));
    if (attr != hipSuccess) return attr;
    ItemArgs b = a;
    b.tab_lds = sky_tab_lds(S, MODE, MF, a.m, a.oversample, a.n_tab);
    // many items, sky frame at support 32: 32 consecutive ones per block,
    // sharing its set-up (a launch of one interval of the large workload,
    // 260k items, keeps one per block)
    b.unit_items = win_items_per_block(S, MF, a.n_items);
    const int blocks = (int)item_blocks((a.n_items + b.unit_items - 1) / b.unit_items);
    const size_t sh = winw_frame_lds(S, W, MODE, MF, a.m, a.oversample, a.n_tab);
    if (sh < winw_layout_bytes<S, MODE, MF, W>(a.m, a.n_tab, b.tab_lds)) return hipErrorInvalidValue;
    k_winw<S, MODE, MF, W, WT, MT><<<blocks, 64 * W, sh, s>>>(b);
    return hipGetLastError();
}

template <int S, int MODE, int MF, int W, bool WT>
static hipError_t launch_win_w(const ItemArgs& a, hipStream_t s)
{
    // the default image-sample count fixed at compile time: at support 32,
    // sky frame (1% on the large workload; at 16 it costs registers and 2%)
    if constexpr (MF == kFrameSky && S == 32)
        if (a.m == 3 * S / 2) return launch_win_wm<S, MODE, MF, W, WT, 3 * S / 2>(a, s);
    return launch_win_wm<S, MODE, MF, W, WT, 0>(a, s);
}

template <int S, int MODE, int MF, bool WT>
static hipError_t launch_win_t(const ItemArgs& a, hipStream_t s)
{
    switch (win_block_waves(S, MODE, MF, a.m, a.oversample, a.n_tab, a.win_waves)) {
    case 4: return launch_win_w<S, MODE, MF, 4, WT>(a, s);
    case 1:
        if constexpr (S == 16) return launch_win_w<S, MODE, MF, 1, WT>(a, s);
        break;
    case 2:
        if constexpr (S == 16) return launch_win_w<S, MODE, MF, 2, WT>(a, s);
        break;
    case 8:
        if constexpr (S == 32) return launch_win_w<S, MODE, MF, 8, WT>(a, s);
        break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <int S, int MODE>
static hipError_t launch_win_m(const ItemArgs& a, hipStream_t s)
{
    const bool wt = a.w_m != nullptr;
    if (a.defocus != nullptr) {
        // complex patterns: prediction, and the defocus sums (the scale mode's terms)
        if constexpr (MODE == kPredict || MODE == kScale)
            return wt ? launch_win_t<S, MODE, kFrameSkyComplex, true>(a, s)
                      : launch_win_t<S, MODE, kFrameSkyComplex, false>(a, s);
        return hipErrorInvalidValue;
    }
    if (a.ap_tab != nullptr && a.par_angle != nullptr)
        return wt ? launch_win_t<S, MODE, kFrameAperture, true>(a, s)
                  : launch_win_t<S, MODE, kFrameAperture, false>(a, s);
    if (a.ap_tab != nullptr)
        return wt ? launch_win_t<S, MODE, kFrameSkyAperture, true>(a, s)
                  : launch_win_t<S, MODE, kFrameSkyAperture, false>(a, s);
    if (a.par_angle != nullptr)
        return wt ? launch_win_t<S, MODE, kFrameMount, true>(a, s) : launch_win_t<S, MODE, kFrameMount, false>(a, s);
    return wt ? launch_win_t<S, MODE, kFrameSky, true>(a, s) : launch_win_t<S, MODE, kFrameSky, false>(a, s);
}

size_t win_lds_bytes(int support, int mode, int m, int oversample, int mount_frame_tab)
{
    // the larger block: what must fit for every launch to be possible
    return winw_lds_bytes(support, 8, mode, m, oversample, mount_frame_tab);
}

size_t winw_lds_bytes(int support, int waves, int mode, int m, int oversample, int mount_frame_tab)
{
    const int workers = waves * (64 / (2 * support));
    const int nc = mode_nc(mode) > 0 ? mode_nc(mode) : 1;
    const size_t m2p = (size_t)((m * m + 3) & ~3);
    const bool mf = mount_frame_tab >= 0;
    const int ng = win_ng(mode);  // image-plane factors per sample (sky frame)
    (void)oversample;
    return sizeof(double) * nc * workers + (mf ? 0 : sizeof(float) * ng * m2p) +
           sizeof(float2) * (size_t)workers * support * (support + 1) +
           (support == 16 ? sizeof(float2) * (size_t)(support / 2) * 64 * waves : 0) +
           (mf ? sizeof(float4) * mount_frame_tab : 0);
}

size_t win_lds_budget(int support)
{
    // static LDS of k_winw: the twiddles
    return 160 * 1024 - sizeof(float2) * support * 16;
}

// Every antenna's pattern E and gradient factor q (dE/dp = q (l - p)) at the
// image samples, per interval, polarisation and channel (Eq. DA): what each
// item of the sky frame otherwise evaluates for its two antennas, once per
// antenna instead of once per baseline.  One block per table; the same
// offsets, squint and width scale as the degrid kernel's items, evaluated
// by the same efq (support 16: the correctly rounded square root).
// Intervals already converged (done) are skipped.
__global__ void __launch_bounds__(256) k_ant_beams(ItemArgs a)
{
    const int t = (int)blockIdx.x;
    const int ant = t % a.n_ant;
    const int chan = (t / a.n_ant) % a.n_chan;
    const int pol = (t / (a.n_ant * a.n_chan)) % a.n_pol;
    const int k = a.beam_int0 + t / (a.n_ant * a.n_chan * a.n_pol);
    if (a.done != nullptr && a.done[k]) return;
    const double lam = kCLight / a.freq[chan];
    const float kk = (float)(kPi * a.dish / lam);
    const double sigma = a.gauss_sigma_ld * lam / a.dish;
    const float inv_s2 = (float)(1.0 / (sigma * sigma));
    const float aps = (float)(a.dish / lam * a.ap_inv_step);
    const double sq = (pol == 0 ? 1.0 : -1.0) * a.squint_frac * 1.02899 * lam / a.dish;
    const double* o = a.offsets + (((size_t)k * a.n_pol + pol) * a.n_ant + ant) * 2;
    const float pl = (float)(o[0] + sq), pm = (float)o[1];
    BeamK b = beam_k(kk, inv_s2, aps, 1.f);
    if (a.scale != nullptr) b = beam_k(kk, inv_s2, aps, (float)a.scale[((size_t)k * a.n_pol + pol) * a.n_ant + ant]);
    const int m = a.m, half_m = m >> 1, m2 = m * m;
    const float hstep = (float)a.h;
    const float inv_m = 1.f / (float)m;
    float2* out = a.beams + (((size_t)k * a.n_pol + pol) * a.n_chan + chan) * a.n_ant * (size_t)m2 + (size_t)ant * m2;
    for (int idx = threadIdx.x; idx < m2; idx += 256) {
        const int il = (int)(((float)idx + 0.5f) * inv_m), im = idx - il * m;
        const float l = (float)(il - half_m) * hstep, mm = (float)(im - half_m) * hstep;
        float e, q;
        efq<false>(a, a.airy, b.kk, b.inv_s2, l - pl, mm - pm, e, q);
        out[idx] = make_float2(e, q);
    }
}

hipError_t launch_ant_beams(const ItemArgs& a, hipStream_t s)
{
    const long long n = (long long)(a.beam_int1 - a.beam_int0) * a.n_pol * a.n_chan * a.n_ant;
    if (n <= 0) return hipSuccess;
    if (n > 0x7fffffffLL) return hipErrorInvalidValue;
    k_ant_beams<<<(unsigned)n, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_win(int mode, int support, const ItemArgs& a, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    // the sky frame with radial beams at support 16: tabulate each
    // antenna's pattern first
    if (support == 16 && a.beams != nullptr && a.par_angle == nullptr && a.ap_tab == nullptr &&
        a.defocus == nullptr) {
        const hipError_t e = launch_ant_beams(a, s);
        if (e != hipSuccess) return e;
    }
    if (support == 16) {
        switch (mode) {
        case kPredict: return launch_win_m<16, kPredict>(a, s);
        case kGrad: return launch_win_m<16, kGrad>(a, s);
        case kVjp: return launch_win_m<16, kVjp>(a, s);
        case kScale: return launch_win_m<16, kScale>(a, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (support == 32) {
        switch (mode) {
        case kPredict: return launch_win_m<32, kPredict>(a, s);
        case kGrad: return launch_win_m<32, kGrad>(a, s);
        case kVjp: return launch_win_m<32, kVjp>(a, s);
        case kScale: return launch_win_m<32, kScale>(a, s);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace psc
