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

// ---------------------------------------------------------------------------
// Support 16: S-lane workers.
//
// One block (W wavefronts) per item, as in the table form: the wavefronts
// share the item's image-plane products in LDS.  Each S-lane slot of a
// wavefront is an independent worker.  The item's work is cut into units of
// kChunks per sample group (unit u: group u / kChunks, chunk u % kChunks of
// its samples, both offsets f and -f counted), which the slots claim in turn
// and whose samples they handle one at a time; groups of one or two samples
// (fine oversampling, short intervals) and large groups both keep every slot
// busy.  For a sample, lane c of the slot loads column c of the reversed
// window, the slot transforms it through its own S x (S+1) LDS tile (columns,
// then rows), and lane c then sums over the image samples n whose m index is
// congruent to c modulo S.  Sums are kept per unit and added in unit order.
//
// MF: offsets in the antenna mount frame.  Each row has its own parallactic
// angle chi, so each sample has its own beam centres p = R(chi) (q + squint)
// and its own image-plane products: they are evaluated inside the image-sample
// sum instead of once per item, and the offset derivatives are rotated back to
// the mount frame, dV/dq = R(chi)^T dV/dp.
template <int S, int MODE, int W, bool MF>
__global__ void __launch_bounds__(64 * W) k_win(ItemArgs a)
{
    constexpr int NV = mode_nv(MODE);
    constexpr int NC = mode_nc(MODE);
    constexpr int SP = S + 1;
    constexpr int SPW = 64 / S;
    constexpr int kBlock = 64 * W;
    static_assert(NC <= S, "one term per lane of a slot");
    static_assert(S == 16, "support 32 runs k_winw");

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float2 twsh[S * 16];       // exp(+2 pi i t / (S O)), S O <= 16 S
    constexpr int NW = W * SPW;            // workers (slots) per block
    __shared__ float2 phsh[128][NW];       // slot w's l-axis phases at [0, M)[w], m axis at [64, 64 + M)[w]
    __shared__ int next_group;

    const int m = a.m, half_m = m >> 1;
    const int m2p = (m * m + 3) & ~3;
    // dynamic LDS: per-unit float64 sums | image-plane products | window tiles
    constexpr int kChunks = kWinChunks;
    double* gpart = reinterpret_cast<double*>(smem);  // [unit][NC]
    float* gsh = reinterpret_cast<float*>(smem + sizeof(double) * (NC > 0 ? NC : 1) * win_max_units(a.oversample));
    float2* wtile = reinterpret_cast<float2*>(reinterpret_cast<unsigned char*>(gsh) +
                                              (MF ? 0 : sizeof(float) * NV * m2p));
    // mount frame: the Airy table, read at every image sample of every sample
    float4* airy_sh = reinterpret_cast<float4*>(wtile + (size_t)W * 64 * SP);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per_xcd = gridDim.x >> 3;
    const int li = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
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
    if constexpr (MF)
        for (int t = tid; t < a.n_tab; t += kBlock) airy_sh[t] = a.airy[t];

    const int slot = lane / S;
    const int c = lane - slot * S;
    const int worker = wave * SPW + slot;
    float2* wt = wtile + (size_t)worker * S * SP;  // this slot's tile
    float2* ph = &phsh[0][worker];  // phase j of this slot at ph[j * NW]
    const TermSel tsel(c);
    const float2 zero = make_float2(0.f, 0.f);
    // the two image-sample m indices congruent to c modulo S: c and c - S
    const bool m0_ok = c < half_m, m1_ok = c >= S - half_m;
    const int jm0 = m0_ok ? c + half_m : 0;
    const int jm1 = m1_ok ? c - S + half_m : 0;
    float2 pm0 = zero, pm1 = zero;

    // mount frame: beam constants of the item's channel, and the lane's two
    // image-sample m coordinates with their taper values
    const double lam = kCLight / a.freq[it.chan];
    const float kk = (float)(kPi * a.dish / lam);
    const double sigma = a.gauss_sigma_ld * lam / a.dish;
    const float inv_s2 = (float)(1.0 / (sigma * sigma));
    const float hstep = (float)a.h;
    const float mm0 = (float)(jm0 - half_m) * hstep, mm1 = (float)(jm1 - half_m) * hstep;
    const float ctm0 = a.taper_img[jm0], ctm1 = a.taper_img[jm1];
    double qil = 0, qim = 0, qjl = 0, qjm = 0;

    // per-axis phases (-1)^n exp(2 pi i f n / (S O)) / S, n in [-M/2, M/2), of
    // the group's offset f (part 0) or of -f (part 1), written by the slot
    auto set_phases = [&](int f, int part) {
        int fl = f / O, fm = f - (f / O) * O;
        if (part) {
            fl = (O - fl) & (O - 1);
            fm = (O - fm) & (O - 1);
        }
        wave_sync();  // earlier readers of this slot's phases are done
        for (int j = c; j < m; j += S) {
            const int n = j - half_m;
            const float sg = (n & 1) ? -inv_s : inv_s;
            const float2 pl = twsh[(fl * n) & (so - 1)];
            const float2 pm = twsh[(fm * n) & (so - 1)];
            ph[j * NW] = make_float2(pl.x * sg, pl.y * sg);
            ph[(64 + j) * NW] = make_float2(pm.x * sg, pm.y * sg);
        }
        wave_sync();
        pm0 = m0_ok ? ph[(64 + jm0) * NW] : zero;
        pm1 = m1_ok ? ph[(64 + jm1) * NW] : zero;
    };

    for (int pol = 0; pol < a.n_pol; ++pol) {
        if (tid == 0) next_group = NW;
        if constexpr (MF) {
            // mount-frame offsets plus squint (along the mount's first axis)
            const double sq = (pol == 0 ? 1.0 : -1.0) * a.squint_frac * 1.02899 * lam / a.dish;
            const double* oi = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.ai) * 2;
            const double* oj = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.aj) * 2;
            qil = oi[0] + sq;
            qim = oi[1];
            qjl = oj[0] + sq;
            qjm = oj[1];
        } else {
            image_products<MODE>(a, it, pol, gsh, m2p, tid, kBlock);
        }
        __syncthreads();

        const int n_units = (it.grp_end - it.grp_begin) * kChunks;
        double acc64 = 0.0;
        // claim units until one has samples; v in [v, v_end) of group g, part
        // = whether the current sample is at -f
        int u = -1, v = 0, v_end = 0, part = 0;
        Group g;
        bool active = true;
        auto next_unit = [&]() {
            while (true) {
                if (u >= 0) {  // close the finished (or empty) unit, claim the next
                    if (NC > 0 && c < NC) gpart[u * NC + c] = acc64;
                    acc64 = 0.0;
                    int nx = 0;
                    if (c == 0) nx = atomicAdd(&next_group, 1);
                    u = __shfl(nx, slot * S);
                } else {
                    u = worker;  // units 0 .. NW-1 go to the slots in order
                }
                if (u >= n_units) {
                    active = false;
                    return;
                }
                g = a.groups[it.grp_begin + u / kChunks];
                const int total = g.n_vis + g.n_vis2;
                const int len = (total + kChunks - 1) / kChunks;
                v = (u % kChunks) * len;
                v_end = min(total, v + len);
                if (v < v_end) break;
            }
            part = v >= g.n_vis;
            set_phases(g.f, part);
        };
        next_unit();
        while (__any(active)) {
            if (active) {
                const uint32_t vb = g.vis_begin;
                const VisEnt e = a.vis[vb + v];
                const size_t o = (size_t)e.vidx * a.n_pol + pol;
                float2 vin = zero;
                float wgt = 0.f;
                if (MODE != kPredict) vin = a.vis_in[o];
                if (MODE == kGrad) wgt = a.weight[o];
                // ---- reversed window column c: x[i] = V^{M0}[k_lo_l + S-1-i][k_lo_m + S-1-c]
                const int row0 = (int)(e.klo >> 16);
                const int col0 = (int)(e.klo & 0xffffu);
                const int voff = (row0 * P + col0 + (S - 1 - c)) * (int)sizeof(float2);
                float2 x[S];
#pragma unroll
                for (int i = 0; i < S; ++i)
                    x[i] = __builtin_bit_cast(
                        float2, __builtin_amdgcn_raw_buffer_load_b64(grsrc, voff, (S - 1 - i) * rowbytes, 0));
                // ---- 2-D DFT of the window: along l in registers, then along m
                fft_reg<S>(x);
                wave_sync();  // the previous sample's tile has been read
#pragma unroll
                for (int i = 0; i < S; ++i) wt[i * SP + c] = x[i];
                wave_sync();
#pragma unroll
                for (int i = 0; i < S; ++i) x[i] = wt[c * SP + i];
                fft_reg<S>(x);
#pragma unroll
                for (int i = 0; i < S; ++i) wt[c * SP + i] = x[i];
                wave_sync();

                // ---- V_k = sum_n g_k[n] phi_l(n_l) phi_m(n_m) What[n_l mod S][n_m mod S]
                float2 s[NV];
#pragma unroll
                for (int k = 0; k < NV; ++k) s[k] = zero;
                float cs = 1.f, sn = 0.f;
                if constexpr (MF) {
                    // this row's beam centres on the sky
                    sincosf((float)a.par_angle[e.vidx / (uint32_t)a.n_chan], &sn, &cs);
                    const float pil = (float)(cs * qil - sn * qim), pim = (float)(sn * qil + cs * qim);
                    const float pjl = (float)(cs * qjl - sn * qjm), pjm = (float)(sn * qjl + cs * qjm);
#pragma unroll 2
                    for (int jl = 0; jl < m; ++jl) {
                        const int bl = (jl - half_m) & (S - 1);
                        const float2 t = cmul(ph[jl * NW], wt[bl * SP + c]);
                        const float2 z0 = cmul(t, pm0), z1 = cmul(t, pm1);
                        const float l = (float)(jl - half_m) * hstep;
                        const float ctl = a.taper_img[jl];
                        float g0[NV], g1[NV];
                        mf_products<MODE>(a, airy_sh, kk, inv_s2, l - pil, mm0 - pim, l - pjl, mm0 - pjm,
                                          ctl * ctm0, g0);
                        mf_products<MODE>(a, airy_sh, kk, inv_s2, l - pil, mm1 - pim, l - pjl, mm1 - pjm,
                                          ctl * ctm1, g1);
#pragma unroll
                        for (int k = 0; k < NV; ++k) {
                            s[k].x = fmaf(g0[k], z0.x, fmaf(g1[k], z1.x, s[k].x));
                            s[k].y = fmaf(g0[k], z0.y, fmaf(g1[k], z1.y, s[k].y));
                        }
                    }
                } else {
#pragma unroll 4
                for (int jl = 0; jl < m; ++jl) {
                    const int bl = (jl - half_m) & (S - 1);
                    const float2 t = cmul(ph[jl * NW], wt[bl * SP + c]);
                    const float2 z0 = cmul(t, pm0), z1 = cmul(t, pm1);
                    // variant k of samples (jl, jm0) and (jl, jm1)
                    const float* g0p = gsh + jl * m + jm0;
                    const float* g1p = gsh + jl * m + jm1;
#pragma unroll
                    for (int k = 0; k < NV; ++k) {
                        const float g0 = g0p[k * m2p], g1 = g1p[k * m2p];
                        s[k].x = fmaf(g0, z0.x, fmaf(g1, z1.x, s[k].x));
                        s[k].y = fmaf(g0, z0.y, fmaf(g1, z1.y, s[k].y));
                    }
                }
                }
                // sum over the slot's S lanes
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    s[k].x = row16_sum(s[k].x);
                    s[k].y = row16_sum(s[k].y);
                }
                if constexpr (MF && MODE != kPredict) {
                    // derivatives with respect to the mount-frame offsets
                    constexpr int d0 = (MODE == kGrad) ? 1 : 0;
#pragma unroll
                    for (int end = 0; end < 2; ++end) {
                        const float2 dl = s[d0 + 2 * end], dm = s[d0 + 2 * end + 1];
                        s[d0 + 2 * end] = make_float2(cs * dl.x + sn * dm.x, cs * dl.y + sn * dm.y);
                        s[d0 + 2 * end + 1] = make_float2(cs * dm.x - sn * dl.x, cs * dm.y - sn * dl.y);
                    }
                }
                if (MODE == kPredict) {
                    if (c == 0) a.vis_out[o] = s[0];
                } else if (MODE == kGrad) {
                    if (a.vis_out != nullptr && c == 0) a.vis_out[o] = s[0];
                    grad_term(tsel, s, vin, wgt, acc64);
                } else {
                    vjp_term(c, s, vin, acc64);
                }

                // ---- next sample: same part, the partner part, or the next unit
                if (++v == v_end) {
                    next_unit();
                } else if (part == 0 && v == g.n_vis) {
                    part = 1;
                    set_phases(g.f, 1);
                }
            }
        }

        // ---- per-item partial sums: units added in unit order
        __syncthreads();
        if (NC > 0 && tid < NC) {
            double sum = 0.0;
            for (int uu = 0; uu < n_units; ++uu) sum += gpart[uu * NC + tid];
            a.partials[((size_t)item_idx * a.n_pol + pol) * NC + tid] = sum;
        }
        __syncthreads();
    }
}

// Image-plane factors of an item at the M x M samples, [n][NG] with NG = 1, 2, 3
// for predict, adjoint, gradient: g = E_i E_j c and, for the derivatives,
// the gradient factors q_i E_j c and E_i q_j c (dE/dp = q (l - p)), from
// which the sum forms the four derivative variants of Eq. DA.
template <int MODE>
__device__ __forceinline__ void image_factors(const ItemArgs& a, float* gsh, float kk, float inv_s2, float pil,
                                              float pim, float pjl, float pjm, int tid, int nthr)
{
    constexpr int NG = MODE == kGrad ? 3 : MODE == kVjp ? 2 : 1;
    const int m = a.m, half_m = m >> 1, m2 = m * m;
    const float hstep = (float)a.h;
    for (int idx = tid; idx < m2; idx += nthr) {
        const int il = idx / m, im = idx - il * m;
        const float l = (float)(il - half_m) * hstep, mm = (float)(im - half_m) * hstep;
        float ei, qi, ej, qj;
        efq(a, a.airy, kk, inv_s2, l - pil, mm - pim, ei, qi);
        efq(a, a.airy, kk, inv_s2, l - pjl, mm - pjm, ej, qj);
        const float c = a.taper_img[il] * a.taper_img[im];
        float* gn = gsh + idx * NG;
        if constexpr (MODE == kPredict) {
            gn[0] = ei * ej * c;
        } else {
            constexpr int o = MODE == kGrad ? 1 : 0;
            if constexpr (MODE == kGrad) gn[0] = ei * ej * c;
            gn[o] = qi * ej * c;
            gn[o + 1] = ei * qj * c;
        }
    }
}

// Cross-half exchanges without the LDS crossbar.  v_permlane32_swap(v, v)
// returns (lanes 0-31 of v in both halves, lanes 32-63 of v in both halves);
// v_permlane16_swap(v, v) returns (rows 0 and 2 of v, each in its own and the
// next row; rows 1 and 3 likewise), so the sum of its two results is the sum
// of lane l and lane l ^ 16.
__device__ __forceinline__ void halves32(float v, float& lo, float& hi)
{
    const unsigned u = __builtin_bit_cast(unsigned, v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    lo = __builtin_bit_cast(float, (unsigned)r[0]);
    hi = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ float sum_xor16(float v)
{
    const unsigned u = __builtin_bit_cast(unsigned, v);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __builtin_bit_cast(float, (unsigned)r[0]) + __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ float sum_xor32(float v)
{
    float lo, hi;
    halves32(v, lo, hi);
    return lo + hi;
}

// ---------------------------------------------------------------------------
// Support 32: a wavefront per sample.
//
// One block of eight wavefronts per item.  The item's samples, numbered group
// by group (each group's samples at f, then those at -f), are dealt to the
// wavefronts in turn: wavefront w takes samples w, w + 8, w + 16, ...  With
// the assignment fixed, a wavefront loads its next sample's entry, window and
// inputs while it transforms and sums the current one, so the chain of
// dependent loads (entry, then window) stays off the critical path; the
// float64 sums are kept per wavefront and added in wavefront order.
//
// Lane (h, c) loads rows [16h, 16h + 16) of column c of the reversed window.
// Each 32-point transform is split in its first radix-2 step: the half h = 0
// keeps the sum of the two halves' points, h = 1 their difference times
// exp(+2 pi i r / 32), and each finishes with a 16-point transform, giving
// the outputs 2b + h.  Along l the columns go through the wavefront's LDS
// tile; along m lane (h, c) reads row c, and multiplies it by the l-axis phase
// phi_l(n) of the image-sample index n in [-M/2, 32 - M/2) congruent to c
// before writing it back, so the sum needs no phase per image sample: the
// samples n + 32 carry the common factor exp(2 pi i f_l / O), and the m-axis
// phase is the lane's own.  In the sum lane (h, c) takes the image-sample m
// index n_m = c - 32 h (M/2 of the 32 lanes of each half have one).
template <int MODE, bool MF, int W>
__global__ void __launch_bounds__(64 * W) k_winw(ItemArgs a)
{
    constexpr int S = 32, H = S / 2, SP = S + 1;
    constexpr int NV = mode_nv(MODE);
    constexpr int NC = mode_nc(MODE);
    constexpr int NCP = NC > 0 ? NC : 1;
    constexpr int NG = MODE == kGrad ? 3 : MODE == kVjp ? 2 : 1;  // image-plane factors per sample
    constexpr int kBlock = 64 * W;
    static_assert(NC <= 64, "one term per lane");

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float2 twsh[S * 16];  // exp(+2 pi i t / (S O)), S O <= 16 S

    const int m = a.m, half_m = m >> 1;
    const int m2p = (m * m + 3) & ~3;
    const int O = a.oversample, so = S * O;
    // dynamic LDS: per-wavefront float64 sums | the item's groups |
    // image-plane products [n][NV] | window tiles | Airy table (MF)
    double* gpart = reinterpret_cast<double*>(smem);  // [W][NCP]
    Group* grp = reinterpret_cast<Group*>(gpart + W * NCP);
    float* gsh = reinterpret_cast<float*>(grp + win_max_groups(O));
    float2* wtile = reinterpret_cast<float2*>(gsh + (MF ? 0 : NG * m2p));
    float4* airy_sh = reinterpret_cast<float4*>(wtile + (size_t)W * S * SP);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per_xcd = gridDim.x >> 3;
    const int li = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (li >= a.n_items) return;
    const int item_idx = a.item_begin + li;
    const Item it = a.items[item_idx];
    if (a.done != nullptr && a.done[it.interval]) return;

    const int N = a.grid_n;
    const float inv_s = 1.0f / (float)S;
    const int P = N + S;  // pitch of the padded grid
    const int rowbytes = P * (int)sizeof(float2);
    const __amdgpu_buffer_rsrc_t grsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.grid, (short)0, P * P * (int)sizeof(float2), 0x00020000);

    const int n_grp = it.grp_end - it.grp_begin;
    for (int t = tid; t < so; t += kBlock) twsh[t] = a.tw[t];
    for (int t = tid; t < n_grp; t += kBlock) grp[t] = a.groups[it.grp_begin + t];
    if constexpr (MF)
        for (int t = tid; t < a.n_tab; t += kBlock) airy_sh[t] = a.airy[t];
    __syncthreads();

    const int c = lane & (S - 1), hh = lane >> 5;
    float2* wt = wtile + (size_t)wave * S * SP;  // this wavefront's tile
    const TermSel tsel(lane);
    const float2 zero = make_float2(0.f, 0.f);
    // the lane's image-sample m index, and the l index its transform row c
    // stands for
    const int nm = c - hh * S;
    const bool m_ok = nm >= -half_m && nm < half_m;
    const int jm = m_ok ? nm + half_m : 0;
    const int nl_row = ((c + half_m) & (S - 1)) - half_m;
    // first radix-2 step of a 32-point transform: half h keeps
    // (x_r + (-1)^h x_{16+r}) exp(+2 pi i h r / 32)
    const float sgn = hh ? -1.f : 1.f;
    float2 tw1[H];
#pragma unroll
    for (int r = 0; r < H; ++r) tw1[r] = hh ? make_float2(kTw.re[2 * r], kTw.im[2 * r]) : make_float2(1.f, 0.f);

    // (-1)^n exp(2 pi i f n / (S O)) / S
    auto phase = [&](int f, int n) {
        const float2 t = twsh[(f * n) & (so - 1)];
        const float sg = (n & 1) ? -inv_s : inv_s;
        return make_float2(t.x * sg, t.y * sg);
    };
    // the sample v positions on from (gi, v) in the item's numbering
    auto advance = [&](int& gi, int& v, int step) {
        v += step;
        while (gi < n_grp) {
            const int tot = grp[gi].n_vis + grp[gi].n_vis2;
            if (v < tot) break;
            v -= tot;
            ++gi;
        }
    };
    // a sample's entry; past the end, the item's first (loads stay in bounds)
    auto entry = [&](int gi, int v) {
        return gi < n_grp ? a.vis[grp[gi].vis_begin + v] : a.vis[grp[0].vis_begin];
    };
    // rows H hh + r of the reversed column c: grid row k_lo_l + S-1-(H hh + r)
    auto load_window = [&](const VisEnt& e, float2 (&x)[H]) {
        const int row0 = (int)(e.klo >> 16);
        const int col0 = (int)(e.klo & 0xffffu);
        const int voff = (row0 * P + col0 + (S - 1 - c)) * (int)sizeof(float2) + (1 - hh) * H * rowbytes;
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
    const float hstep = (float)a.h;
    const float mmy = (float)nm * hstep;
    const float ctm = a.taper_img[jm];

    for (int pol = 0; pol < a.n_pol; ++pol) {
        // this wavefront's first two samples, their entries, the first window
        int gi0 = 0, v0 = wave;
        advance(gi0, v0, 0);
        int gi1 = gi0, v1 = v0;
        if (gi0 < n_grp) advance(gi1, v1, W);
        float2 x0[H];
        VisEnt e0 = {0u, 0u}, e1 = {0u, 0u};
        float2 vin0 = zero;
        float wgt0 = 0.f;
        if (gi0 < n_grp) {
            e0 = entry(gi0, v0);
            e1 = entry(gi1, v1);
            load_window(e0, x0);
            const size_t o0 = (size_t)e0.vidx * a.n_pol + pol;
            if (MODE != kPredict) vin0 = a.vis_in[o0];
            if (MODE == kGrad) wgt0 = a.weight[o0];
        }

        // offsets plus squint (along l, or along the mount's first axis)
        const double sq = (pol == 0 ? 1.0 : -1.0) * a.squint_frac * 1.02899 * lam / a.dish;
        const double* oi = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.ai) * 2;
        const double* oj = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.aj) * 2;
        const double qil = oi[0] + sq, qim = oi[1], qjl = oj[0] + sq, qjm = oj[1];
        if constexpr (!MF)
            image_factors<MODE>(a, gsh, kk, inv_s2, (float)qil, (float)qim, (float)qjl, (float)qjm, tid, kBlock);
        __syncthreads();

        double acc64 = 0.0;
        while (gi0 < n_grp) {
            // ---- fetch ahead: the next sample's window and inputs, the entry after it
            float2 x1[H];
            load_window(e1, x1);
            const size_t o1 = (size_t)e1.vidx * a.n_pol + pol;
            float2 vin1 = zero;
            float wgt1 = 0.f;
            if (MODE != kPredict) vin1 = a.vis_in[o1];
            if (MODE == kGrad) wgt1 = a.weight[o1];
            int gi2 = gi1, v2 = v1;
            if (gi1 < n_grp) advance(gi2, v2, W);
            const VisEnt e2 = entry(gi2, v2);

            // ---- the current sample's offset per axis: f, or -f after the group's first part
            const Group g0 = grp[gi0];
            int fl = g0.f / O, fm = g0.f - (g0.f / O) * O;
            if (v0 >= g0.n_vis) {
                fl = (O - fl) & (O - 1);
                fm = (O - fm) & (O - 1);
            }

            // ---- along l: first radix-2 step across the halves, then 16 points
            float2 y[H];
#pragma unroll
            for (int r = 0; r < H; ++r) {
                // the column's rows r (half 0) and 16 + r (half 1), in every lane
                float tx, bx, ty, by;
                halves32(x0[r].x, tx, bx);
                halves32(x0[r].y, ty, by);
                y[r] = make_float2(fmaf(sgn, bx, tx), fmaf(sgn, by, ty));
                if (r > 0) y[r] = cmul(y[r], tw1[r]);
            }
            fft_reg<H>(y);
            wave_sync();  // the previous sample's tile has been read
#pragma unroll
            for (int b = 0; b < H; ++b) wt[(2 * b + hh) * SP + c] = y[b];
            wave_sync();
            // ---- along m: row c, the same split; times the row's l-axis phase
#pragma unroll
            for (int r = 0; r < H; ++r) {
                const float2 t0 = wt[c * SP + r], t1 = wt[c * SP + H + r];
                y[r] = make_float2(fmaf(sgn, t1.x, t0.x), fmaf(sgn, t1.y, t0.y));
                if (r > 0) y[r] = cmul(y[r], tw1[r]);
            }
            fft_reg<H>(y);
            const float2 prow = phase(fl, nl_row);
#pragma unroll
            for (int b = 0; b < H; ++b) wt[c * SP + 2 * b + hh] = cmul(y[b], prow);
            wave_sync();

            // ---- A_k, B_k: sums over l of g_k[n_l][n_m] T[n_l mod 32][c] for
            // n_l below and above 32 - M/2
            float2 A[NV], B[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) A[k] = B[k] = zero;
            float cs = 1.f, sn = 0.f;
            if constexpr (MF) {
                // this row's beam centres on the sky
                sincosf((float)a.par_angle[e0.vidx / (uint32_t)a.n_chan], &sn, &cs);
                const float pil = (float)(cs * qil - sn * qim), pim = (float)(sn * qil + cs * qim);
                const float pjl = (float)(cs * qjl - sn * qjm), pjm = (float)(sn * qjl + cs * qjm);
                auto term = [&](int jl, float2 (&acc)[NV]) {
                    const float2 t = wt[((jl - half_m) & (S - 1)) * SP + c];
                    const float l = (float)(jl - half_m) * hstep;
                    float g[NV];
                    mf_products<MODE>(a, airy_sh, kk, inv_s2, l - pil, mmy - pim, l - pjl, mmy - pjm,
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
                // variant dV/dp_l = L - p_l Q, dV/dp_m = (m - p_m) Q)
                const float* gp = gsh + jm * NG;
                // the halves read factors S samples apart, S NG words: an odd
                // multiple of 32 for NG odd, so they use disjoint banks
                // image-sample rows [j0, j1) at tile rows b0, b0 + 1, ... (no wrap)
                auto seg = [&](int j0, int j1, int b0, float2 (&acc)[NV]) {
                    const float2* tp = wt + b0 * SP + c;
                    const float* g = gp + j0 * m * NG;
#pragma unroll 4
                    for (int jl = j0; jl < j1; ++jl, tp += SP, g += m * NG) {
                        const float2 t = *tp;
                        if constexpr (MODE != kVjp) {
                            acc[0].x = fmaf(g[0], t.x, acc[0].x);
                            acc[0].y = fmaf(g[0], t.y, acc[0].y);
                        }
                        if constexpr (MODE != kPredict) {
                            constexpr int o = MODE == kGrad ? 1 : 0;
                            const float l = (float)(jl - half_m) * hstep;
                            const float2 tl = make_float2(t.x * l, t.y * l);
#pragma unroll
                            for (int end = 0; end < 2; ++end) {
                                const float q = g[o + end];
                                float2& L = acc[o + 2 * end];
                                float2& Q = acc[o + 2 * end + 1];
                                L.x = fmaf(q, tl.x, L.x);
                                L.y = fmaf(q, tl.y, L.y);
                                Q.x = fmaf(q, t.x, Q.x);
                                Q.y = fmaf(q, t.y, Q.y);
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
            }
            // ---- s_k = phi_m(n_m) (A_k + exp(2 pi i f_l / O) B_k), summed over the wavefront
            const float2 rho = twsh[(fl * S) & (so - 1)];
            const float2 pm = m_ok ? phase(fm, nm) : zero;
            float2 s[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const float2 rb = cmul(rho, B[k]);
                s[k] = cmul(pm, make_float2(A[k].x + rb.x, A[k].y + rb.y));
            }
            if constexpr (!MF && MODE != kPredict) {
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
            for (int k = 0; k < NV; ++k) {
                s[k].x = row16_sum(s[k].x);
                s[k].y = row16_sum(s[k].y);
                s[k].x = sum_xor32(sum_xor16(s[k].x));
                s[k].y = sum_xor32(sum_xor16(s[k].y));
            }
            if constexpr (MF && MODE != kPredict) {
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
            if (MODE == kPredict) {
                if (lane == 0) a.vis_out[o0] = s[0];
            } else if (MODE == kGrad) {
                if (a.vis_out != nullptr && lane == 0) a.vis_out[o0] = s[0];
                grad_term(tsel, s, vin0, wgt0, acc64);
            } else {
                vjp_term(lane, s, vin0, acc64);
            }

            // ---- move on
#pragma unroll
            for (int r = 0; r < H; ++r) x0[r] = x1[r];
            vin0 = vin1;
            wgt0 = wgt1;
            e0 = e1;
            e1 = e2;
            gi0 = gi1;
            v0 = v1;
            gi1 = gi2;
            v1 = v2;
        }

        // ---- per-item partial sums: wavefronts added in order
        if (NC > 0 && lane < NC) gpart[wave * NCP + lane] = acc64;
        __syncthreads();
        if (NC > 0 && tid < NC) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) sum += gpart[w * NCP + tid];
            a.partials[((size_t)item_idx * a.n_pol + pol) * NC + tid] = sum;
        }
        __syncthreads();
    }
}

template <int S, int MODE, bool MF>
static hipError_t launch_win_t(const ItemArgs& a, hipStream_t s)
{
    const size_t sh = win_lds_bytes(S, MODE, a.m, a.oversample, MF ? a.n_tab : -1);
    if (sh > win_lds_budget(S)) return hipErrorInvalidValue;
    if constexpr (S == 16) {
        constexpr int W = kWinWaves;
        // raise the dynamic LDS limit once, to what one compute unit allows
        static const hipError_t attr = hipFuncSetAttribute(
            (const void*)k_win<S, MODE, W, MF>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)win_lds_budget(S));
        if (attr != hipSuccess) return attr;
        const int blocks = 8 * ((a.n_items + 7) / 8);
        k_win<S, MODE, W, MF><<<blocks, 64 * W, sh, s>>>(a);
    } else {
        static const hipError_t attr8 = hipFuncSetAttribute(
            (const void*)k_winw<MODE, MF, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)win_lds_budget(S));
        static const hipError_t attr4 = hipFuncSetAttribute(
            (const void*)k_winw<MODE, MF, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)win_lds_budget(S));
        if (attr8 != hipSuccess) return attr8;
        if (attr4 != hipSuccess) return attr4;
        const int blocks = 8 * ((a.n_items + 7) / 8);
        // four wavefronts when two blocks fit a compute unit's LDS, else eight
        const size_t sh4 = winw_lds_bytes(4, MODE, a.m, a.oversample, MF ? a.n_tab : -1);
        if (2 * (sh4 + (160 * 1024 - win_lds_budget(S))) <= 160 * 1024)
            k_winw<MODE, MF, 4><<<blocks, 64 * 4, sh4, s>>>(a);
        else
            k_winw<MODE, MF, 8><<<blocks, 64 * 8, sh, s>>>(a);
    }
    return hipGetLastError();
}

size_t win_lds_bytes(int support, int mode, int m, int oversample, int mount_frame_tab)
{
    const int nv = mode_nv(mode);
    const int nc = mode_nc(mode) > 0 ? mode_nc(mode) : 1;
    const size_t m2p = (size_t)((m * m + 3) & ~3);
    const bool mf = mount_frame_tab >= 0;
    const size_t prod = mf ? 0 : sizeof(float) * nv * m2p;
    const size_t tab = mf ? sizeof(float4) * mount_frame_tab : 0;
    if (support == 16)
        return sizeof(double) * nc * win_max_units(oversample) + prod +
               sizeof(float2) * (size_t)kWinWaves * 64 * (support + 1) + tab;
    return winw_lds_bytes(kWinwWaves, mode, m, oversample, mount_frame_tab);
}

size_t winw_lds_bytes(int waves, int mode, int m, int oversample, int mount_frame_tab)
{
    constexpr int S = 32;
    const int nc = mode_nc(mode) > 0 ? mode_nc(mode) : 1;
    const size_t m2p = (size_t)((m * m + 3) & ~3);
    const bool mf = mount_frame_tab >= 0;
    const int ng = mode == kGrad ? 3 : mode == kVjp ? 2 : 1;  // image-plane factors per sample
    return sizeof(double) * nc * waves + sizeof(Group) * win_max_groups(oversample) +
           (mf ? 0 : sizeof(float) * ng * m2p) + sizeof(float2) * (size_t)waves * S * (S + 1) +
           (mf ? sizeof(float4) * mount_frame_tab : 0);
}

size_t win_lds_budget(int support)
{
    // static LDS: twiddles, and at support 16 the per-slot phases and the
    // group counter
    const size_t stat = support == 16
        ? sizeof(float2) * support * 16 + sizeof(float2) * kWinWaves * (64 / support) * 128 + 16
        : sizeof(float2) * support * 16;
    return 160 * 1024 - stat;
}

hipError_t launch_win(int mode, int support, const ItemArgs& a, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const bool mf = a.par_angle != nullptr;
    if (support == 16) {
        switch (mode) {
        case kPredict: return mf ? launch_win_t<16, kPredict, true>(a, s) : launch_win_t<16, kPredict, false>(a, s);
        case kGrad: return mf ? launch_win_t<16, kGrad, true>(a, s) : launch_win_t<16, kGrad, false>(a, s);
        case kVjp: return mf ? launch_win_t<16, kVjp, true>(a, s) : launch_win_t<16, kVjp, false>(a, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (support == 32) {
        switch (mode) {
        case kPredict: return mf ? launch_win_t<32, kPredict, true>(a, s) : launch_win_t<32, kPredict, false>(a, s);
        case kGrad: return mf ? launch_win_t<32, kGrad, true>(a, s) : launch_win_t<32, kGrad, false>(a, s);
        case kVjp: return mf ? launch_win_t<32, kVjp, true>(a, s) : launch_win_t<32, kVjp, false>(a, s);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace psc
