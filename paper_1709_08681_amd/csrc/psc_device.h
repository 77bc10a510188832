// psc_device.h -- device helpers shared by the kernels of libpsc: complex
// arithmetic, wavefront-level ordering and reductions, the in-register FFT and
// the antenna voltage pattern.
#pragma once

#include "psc_internal.h"

namespace psc {

// exp(+2 pi i j / 64), j = 0..63, evaluated at compile time (Taylor series on
// [-pi, pi], exact on the axes) so that the unrolled FFT sees literal twiddles.
struct TwTable {
    float re[64];
    float im[64];
    constexpr TwTable() : re(), im()
    {
        for (int j = 0; j < 64; ++j) {
            const int jj = j > 32 ? j - 64 : j;
            const double x = kPi * jj / 32.0;
            double sn = x, cs = 1.0, ts = x, tc = 1.0;
            for (int k = 1; k < 30; ++k) {
                ts *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
                sn += ts;
                tc *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
                cs += tc;
            }
            if (j % 16 == 0) {
                const int q = j / 16;
                cs = (q == 0) ? 1.0 : (q == 2) ? -1.0 : 0.0;
                sn = (q == 1) ? 1.0 : (q == 3) ? -1.0 : 0.0;
            }
            re[j] = (float)cs;
            im[j] = (float)sn;
        }
    }
};
constexpr TwTable kTw{};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b)
{
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over each row of 16 lanes with DPP moves (quad swaps, then half-row and
// row mirrors); every lane of the row ends with the row's total.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, true));
}

__device__ __forceinline__ float row16_sum(float v)
{
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    v += dpp_mov<0x140>(v);  // row_mirror
    return v;
}

template <int LOG>
__host__ __device__ constexpr int bitrev(int i)
{
    int r = 0;
    for (int b = 0; b < LOG; ++b)
        if (i & (1 << b)) r |= 1 << (LOG - 1 - b);
    return r;
}

// t = w * v for the twiddle w = exp(+2 pi i j / 64) (j known after unrolling);
// multiplications by 1, i, -1, -i are dropped.
__device__ __forceinline__ float2 twmul(int j, float2 v)
{
    if (j == 0) return v;
    if (j == 16) return make_float2(-v.y, v.x);
    if (j == 32) return make_float2(-v.x, -v.y);
    if (j == 48) return make_float2(v.y, -v.x);
    const float wr = kTw.re[j], wi = kTw.im[j];
    return make_float2(v.x * wr - v.y * wi, v.x * wi + v.y * wr);
}

// In-register radix-2 DFT X[b] = sum_r x[r] exp(+2 pi i b r / S), S <= 64.
template <int S>
__device__ __forceinline__ void fft_reg(float2 (&x)[S])
{
    constexpr int LOG = (S == 8) ? 3 : (S == 16) ? 4 : (S == 32) ? 5 : 6;
    float2 y[S];
#pragma unroll
    for (int i = 0; i < S; ++i) y[bitrev<LOG>(i)] = x[i];
#pragma unroll
    for (int st = 1; st <= LOG; ++st) {
        const int mlen = 1 << st, half = mlen >> 1;
#pragma unroll
        for (int k = 0; k < S; k += mlen) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const float2 t = twmul(j * (64 / mlen), y[k + j + half]);
                const float2 u = y[k + j];
                y[k + j] = make_float2(u.x + t.x, u.y + t.y);
                y[k + j + half] = make_float2(u.x - t.x, u.y - t.y);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < S; ++i) x[i] = y[i];
}

// Far-field voltage pattern of one antenna at sky offset (dl, dm) = l - p and
// its derivatives with respect to the pointing offset p (float32; the Airy
// pattern from the cubic Hermite table, the Gaussian in closed form).
__device__ __forceinline__ void efp(const ItemArgs& a, const float4* tab, float kk, float inv_s2, float dl,
                                    float dm, float& e, float& el, float& em)
{
    if (a.illum == 1) {
        e = expf(-0.5f * (dl * dl + dm * dm) * inv_s2);
        el = e * dl * inv_s2;
        em = e * dm * inv_s2;
        return;
    }
    // the hardware square root (about 1 ulp; the correctly rounded sqrtf adds
    // some fifteen instructions, which the per-sample mount-frame products
    // pay at every image sample)
    const float x = kk * __builtin_amdgcn_sqrtf(fmaf(dl, dl, dm * dm));
    float u = x * a.inv_dx;
    int i;
    if (!(u < (float)(a.n_tab - 2))) {  // beyond the table, or not finite: clamp
        i = a.n_tab - 2;
        u = (float)i + 1.0f;
    } else {
        i = (int)u;
    }
    const float t = u - (float)i;
    const float4 p0 = tab[i], p1 = tab[i + 1];
    const float t2 = t * t, t3 = t2 * t;
    const float h00 = 2.f * t3 - 3.f * t2 + 1.f, h10 = t3 - 2.f * t2 + t, h01 = -2.f * t3 + 3.f * t2,
                h11 = t3 - t2;
    const float A = h00 * p0.x + h10 * p0.y + h01 * p1.x + h11 * p1.y;
    const float B = h00 * p0.z + h10 * p0.w + h01 * p1.z + h11 * p1.w;
    e = A;
    const float k2 = kk * kk * B;
    el = k2 * dl;
    em = k2 * dm;
}

// The same pattern in factored form: E and the factor q of its gradient with
// respect to the pointing offset, dE/dp = q (dl, dm) (the pattern depends on
// |l - p| alone, so the gradient points along l - p).  HW: the hardware square
// root instead of the correctly rounded one (faster in some kernels, slower
// in others through register allocation: chosen by measurement).
template <bool HW = false>
__device__ __forceinline__ void efq(const ItemArgs& a, const float4* tab, float kk, float inv_s2, float dl,
                                    float dm, float& e, float& q)
{
    if (a.illum == 1) {
        e = expf(-0.5f * (dl * dl + dm * dm) * inv_s2);
        q = e * inv_s2;
        return;
    }
    const float x = HW ? kk * __builtin_amdgcn_sqrtf(fmaf(dl, dl, dm * dm)) : kk * sqrtf(dl * dl + dm * dm);
    float u = x * a.inv_dx;
    int i;
    if (!(u < (float)(a.n_tab - 2))) {  // beyond the table, or not finite: clamp
        i = a.n_tab - 2;
        u = (float)i + 1.0f;
    } else {
        i = (int)u;
    }
    const float t = u - (float)i;
    const float4 p0 = tab[i], p1 = tab[i + 1];
    const float t2 = t * t, t3 = t2 * t;
    const float h00 = 2.f * t3 - 3.f * t2 + 1.f, h10 = t3 - 2.f * t2 + t, h01 = -2.f * t3 + 3.f * t2,
                h11 = t3 - t2;
    e = h00 * p0.x + h10 * p0.y + h01 * p1.x + h11 * p1.y;
    q = kk * kk * (h00 * p0.z + h10 * p0.w + h01 * p1.z + h11 * p1.w);
}

// Image-plane products E_i E_j c at the M x M samples (spacing FoV/S, centred)
// for one item and polarisation, and for the gradient and adjoint the offset
// derivatives dE_i/dp_i E_j c and E_i dE_j/dp_j c (Eq. DA).  Variant k of
// sample n goes to gsh[k * m2p + n] (variant-major); threads tid, tid + nthr,
// ... of the block share the work.
template <int MODE>
__device__ __forceinline__ void image_products(const ItemArgs& a, const Item& it, int pol, float* gsh,
                                               int m2p, int tid, int nthr)
{
    constexpr int NV = mode_nv(MODE);
    const int ks = m2p;  // stride between variants
    const int m = a.m, half_m = m >> 1, m2 = m * m;
    const double lam = kCLight / a.freq[it.chan];
    const float kk = (float)(kPi * a.dish / lam);
    const double sigma = a.gauss_sigma_ld * lam / a.dish;
    const float inv_s2 = (float)(1.0 / (sigma * sigma));
    const double hp = 1.02899 * lam / a.dish;
    const float hstep = (float)a.h;
    // beam squint: opposite shifts along l for the two polarisations
    const double sq = (pol == 0 ? 1.0 : -1.0) * a.squint_frac * hp;
    const double* oi = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.ai) * 2;
    const double* oj = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.aj) * 2;
    const float pil = (float)(oi[0] + sq), pim = (float)oi[1];
    const float pjl = (float)(oj[0] + sq), pjm = (float)oj[1];
    for (int idx = tid; idx < m2; idx += nthr) {
        const int il = idx / m, im = idx - il * m;
        const float l = (float)(il - half_m) * hstep, mm = (float)(im - half_m) * hstep;
        float ei, eil, eim, ej, ejl, ejm;
        efp(a, a.airy, kk, inv_s2, l - pil, mm - pim, ei, eil, eim);
        efp(a, a.airy, kk, inv_s2, l - pjl, mm - pjm, ej, ejl, ejm);
        const float c = a.taper_img[il] * a.taper_img[im];
        float* gn = gsh + idx;
        if (NV == 1) {
            gn[0] = ei * ej * c;
        } else {
            constexpr int o = (MODE == kGrad) ? 1 : 0;
            if (MODE == kGrad) gn[0] = ei * ej * c;
            gn[(o + 0) * ks] = eil * ej * c;
            gn[(o + 1) * ks] = eim * ej * c;
            gn[(o + 2) * ks] = ei * ejl * c;
            gn[(o + 3) * ks] = ei * ejm * c;
        }
    }
}

// The pattern table of antenna ant's measured aperture (a heterogeneous
// array gives each antenna one of several).
__device__ __forceinline__ const float4* ap_table(const ItemArgs& a, int ant)
{
    return a.ap_ant == nullptr ? a.ap_tab : a.ap_tab + (size_t)a.ap_ant[ant] * a.ap_n * a.ap_n;
}

// A measured aperture's pattern and gradient at table coordinates (x, y)
// (nodes, along the mount frame's l and m), by bicubic Hermite interpolation
// of the node values and derivatives of table tab: E, and dE/dx, dE/dy per
// node step.  Coordinates beyond the table, or not finite, are clamped to
// its edge.
template <bool DERIV>
__device__ __forceinline__ void ap_eval(const ItemArgs& a, const float4* tab, float x, float y, float& e,
                                        float& ex, float& ey)
{
    const float top = (float)(a.ap_n - 1);
    x = fminf(fmaxf(x, 0.f), top);  // fmaxf(NaN, 0) = 0
    y = fminf(fmaxf(y, 0.f), top);
    const int i = min((int)x, a.ap_n - 2), j = min((int)y, a.ap_n - 2);
    const float t = x - (float)i, u = y - (float)j;
    const float4* p = tab + (size_t)i * a.ap_n + j;
    const float4 f00 = p[0], f01 = p[1], f10 = p[a.ap_n], f11 = p[a.ap_n + 1];
    // cubic Hermite basis: value at 0 / 1 (h0, h1), slope at 0 / 1 (g0, g1)
    const float t2 = t * t, t3 = t2 * t, u2 = u * u, u3 = u2 * u;
    const float th0 = 2.f * t3 - 3.f * t2 + 1.f, th1 = 3.f * t2 - 2.f * t3;
    const float tg0 = t3 - 2.f * t2 + t, tg1 = t3 - t2;
    const float uh0 = 2.f * u3 - 3.f * u2 + 1.f, uh1 = 3.f * u2 - 2.f * u3;
    const float ug0 = u3 - 2.f * u2 + u, ug1 = u3 - u2;
    // along x at columns j and j + 1: the value (G) and the y slope (Q)
    const float G0 = th0 * f00.x + tg0 * f00.y + th1 * f10.x + tg1 * f10.y;
    const float G1 = th0 * f01.x + tg0 * f01.y + th1 * f11.x + tg1 * f11.y;
    const float Q0 = th0 * f00.z + tg0 * f00.w + th1 * f10.z + tg1 * f10.w;
    const float Q1 = th0 * f01.z + tg0 * f01.w + th1 * f11.z + tg1 * f11.w;
    e = uh0 * G0 + ug0 * Q0 + uh1 * G1 + ug1 * Q1;
    if constexpr (DERIV) {
        const float dth0 = 6.f * (t2 - t), dtg0 = 3.f * t2 - 4.f * t + 1.f, dtg1 = 3.f * t2 - 2.f * t;
        const float duh0 = 6.f * (u2 - u), dug0 = 3.f * u2 - 4.f * u + 1.f, dug1 = 3.f * u2 - 2.f * u;
        const float Gx0 = dth0 * (f00.x - f10.x) + dtg0 * f00.y + dtg1 * f10.y;
        const float Gx1 = dth0 * (f01.x - f11.x) + dtg0 * f01.y + dtg1 * f11.y;
        const float Qx0 = dth0 * (f00.z - f10.z) + dtg0 * f00.w + dtg1 * f10.w;
        const float Qx1 = dth0 * (f01.z - f11.z) + dtg0 * f01.w + dtg1 * f11.w;
        ex = uh0 * Gx0 + ug0 * Qx0 + uh1 * Gx1 + ug1 * Qx1;
        ey = duh0 * (G0 - G1) + dug0 * Q0 + dug1 * Q1;
    }
}

// A measured aperture's pattern towards sky-frame displacement d = (dl, dm)
// from a beam centre, for a row rotated by (cs, sn) = (cos, sin) of its
// parallactic angle: E = T(R^T d D / lambda), the pattern fixed to the
// mount; the derivatives are those with respect to the beam centre in the
// mount frame, -grad T there.  s = D / (lambda * table step).
template <bool DERIV>
__device__ __forceinline__ void efp_ap(const ItemArgs& a, const float4* tab, float s, float cs, float sn, float dl,
                                       float dm, float& e, float& el, float& em)
{
    const float x = fmaf(cs * dl + sn * dm, s, a.ap_c), y = fmaf(cs * dm - sn * dl, s, a.ap_c);
    float ex = 0.f, ey = 0.f;
    ap_eval<DERIV>(a, tab, x, y, e, ex, ey);
    if constexpr (DERIV) {
        el = -s * ex;
        em = -s * ey;
    }
}

// Beam constants of one antenna at an item's channel, its width scale sigma
// applied: the Airy argument per radian kk = pi D / (lambda sigma), the
// Gaussian 1 / (s sigma)^2, the aperture table's nodes per radian over
// sigma, and 1 / sigma (for the scale derivative).
struct BeamK {
    float kk, inv_s2, aps, rsig;
};

__device__ __forceinline__ BeamK beam_k(float kk, float inv_s2, float aps, float sigma)
{
    const float r = 1.f / sigma;
    return BeamK{kk * r, inv_s2 * r * r, aps * r, r};
}

// Image-plane products as mf_products, for measured apertures (antenna i's
// table ti, antenna j's tj), with the derivative variants already with
// respect to the mount-frame offsets (and dE/dsigma = (d . dE/dc) / sigma
// with d in the mount frame).
template <int MODE>
__device__ __forceinline__ void mf_products_ap(const ItemArgs& a, const float4* ti, const float4* tj,
                                               const BeamK& bi, const BeamK& bj, float cs, float sn, float dli,
                                               float dmi, float dlj, float dmj, float c, float (&g)[mode_nv(MODE)])
{
    constexpr bool D = mode_nv(MODE) > 1;
    float ei, eil = 0.f, eim = 0.f, ej, ejl = 0.f, ejm = 0.f;
    efp_ap<D>(a, ti, bi.aps, cs, sn, dli, dmi, ei, eil, eim);
    efp_ap<D>(a, tj, bj.aps, cs, sn, dlj, dmj, ej, ejl, ejm);
    if constexpr (!D) {
        g[0] = ei * ej * c;
    } else if constexpr (MODE == kScale) {
        const float si = ((cs * dli + sn * dmi) * eil + (cs * dmi - sn * dli) * eim) * bi.rsig;
        const float sj = ((cs * dlj + sn * dmj) * ejl + (cs * dmj - sn * dlj) * ejm) * bj.rsig;
        g[0] = ei * ej * c;
        g[1] = si * ej * c;
        g[2] = ei * sj * c;
    } else {
        constexpr int o = (MODE == kGrad) ? 1 : 0;
        if constexpr (MODE == kGrad) g[0] = ei * ej * c;
        g[o + 0] = eil * ej * c;
        g[o + 1] = eim * ej * c;
        g[o + 2] = ei * ejl * c;
        g[o + 3] = ei * ejm * c;
    }
}

// Image-plane products at one image sample for one visibility, from the two
// antennas' offsets relative to the sample (dl_i, dm_i), (dl_j, dm_j) and the
// taper value c there, in the variant order of image_products.
template <int MODE>
__device__ __forceinline__ void mf_products(const ItemArgs& a, const float4* tab, const BeamK& bi,
                                            const BeamK& bj, float dli, float dmi, float dlj, float dmj, float c,
                                            float (&g)[mode_nv(MODE)])
{
    float ei, eil, eim, ej, ejl, ejm;
    efp(a, tab, bi.kk, bi.inv_s2, dli, dmi, ei, eil, eim);
    efp(a, tab, bj.kk, bj.inv_s2, dlj, dmj, ej, ejl, ejm);
    if constexpr (mode_nv(MODE) == 1) {
        g[0] = ei * ej * c;
    } else if constexpr (MODE == kScale) {
        // dE/dsigma = (d . dE/dp) / sigma
        g[0] = ei * ej * c;
        g[1] = (dli * eil + dmi * eim) * bi.rsig * ej * c;
        g[2] = ei * (dlj * ejl + dmj * ejm) * bj.rsig * c;
    } else {
        constexpr int o = (MODE == kGrad) ? 1 : 0;
        if constexpr (MODE == kGrad) g[0] = ei * ej * c;
        g[o + 0] = eil * ej * c;
        g[o + 1] = eim * ej * c;
        g[o + 2] = ei * ejl * c;
        g[o + 3] = ei * ejm * c;
    }
}

// Per-sample terms of the float64 sums.  Gradient: lane t < 12 of a sample's
// lane group adds term t = 6 * end + c, end 0 for antenna i and 1 for j, c
// indexing chi, g_l, g_m, H_ll, H_lm, H_mm = w Re(conj(x) y) with
// (x, y) = (R,R) (R,dl) (R,dm) (dl,dl) (dl,dm) (dm,dm) (Eq. DCHIDD and the
// 2 x 2 normal matrix); the residual R = V^Obs - V^M is formed exactly, the
// product in float32 and the running sum in float64.
struct TermSel {
    bool on, end, xr, xl, yr, yl;
    __device__ explicit TermSel(int t)
    {
        const int c = t % 6;
        on = t < 12;
        end = t >= 6 && t < 12;
        xr = c < 3;
        xl = c == 3 || c == 4;
        yr = c == 0;
        yl = c == 1 || c == 3;
    }
};

// s[0] = V^M, s[1..4] = dV/d(l_i, m_i, l_j, m_j).
template <int NV>
__device__ __forceinline__ void grad_term(const TermSel& ts, const float2 (&s)[NV], float2 vo, float wgt,
                                          double& acc)
{
    const float rr = (float)((double)vo.x - (double)s[0].x);
    const float ri = (float)((double)vo.y - (double)s[0].y);
    const float2 dl = ts.end ? s[3] : s[1];
    const float2 dm = ts.end ? s[4] : s[2];
    const float xr = ts.xr ? rr : (ts.xl ? dl.x : dm.x);
    const float xi = ts.xr ? ri : (ts.xl ? dl.y : dm.y);
    const float yr = ts.yr ? rr : (ts.yl ? dl.x : dm.x);
    const float yi = ts.yr ? ri : (ts.yl ? dl.y : dm.y);
    const float val = fmaf(xr, yr, xi * yi);
    if (ts.on) acc = fma((double)wgt, (double)val, acc);
}

// Adjoint: lane t < 4 adds Re(conj(G) dV/dp_t), s[0..3] = dV/d(l_i, m_i, l_j, m_j).
template <int NV>
__device__ __forceinline__ void vjp_term(int t, const float2 (&s)[NV], float2 gv, double& acc)
{
    const int tt = t < 4 ? t : 0;
    float2 dv = s[0];
#pragma unroll
    for (int k = 1; k < 4; ++k)
        if (tt == k) dv = s[k];
    if (t < 4) acc += (double)gv.x * (double)dv.x + (double)gv.y * (double)dv.y;
}

// Beam-scale sums: lane t < 6 adds term t = 3 * end + c, c indexing chi,
// g_sigma, H_sigma = w |R|^2, w Re(conj(R) dV/dsigma_end), w |dV/dsigma_end|^2
// (Eq. DCHIDD with the scale as the antenna parameter); s[0] = V^M,
// s[1], s[2] = dV/dsigma_i, dV/dsigma_j.
__device__ __forceinline__ void scale_term(int t, const float2 (&s)[3], float2 vo, float wgt, double& acc)
{
    const float rr = (float)((double)vo.x - (double)s[0].x);
    const float ri = (float)((double)vo.y - (double)s[0].y);
    const int c = t % 3;
    const float2 d = t >= 3 ? s[2] : s[1];
    const float xr = c == 2 ? d.x : rr, xi = c == 2 ? d.y : ri;
    const float yr = c == 0 ? rr : d.x, yi = c == 0 ? ri : d.y;
    const float val = fmaf(xr, yr, xi * yi);
    if (t < 6) acc = fma((double)wgt, (double)val, acc);
}

}  // namespace psc
