// psc_grid.hip -- the adjoint of the degrid with respect to the model grid.
//
// d chi^2 / d V^{M0}: every sample spreads w conj(R) over its S x S window
// with the kernel coefficients that produced its V = sum_a V^{M0}[k_lo + a]
// T_f[S-1-a] (table form, Eq. MEDD), R = V^Obs - V from a preceding predict.
// The residual grid is then folded, transformed and divided by the taper
// (psc_kernels.hip) to give the image gradient.
//
// A sample's window touches S^2 cells; added one by one with float64
// atomics that is 2 S^2 global atomics per sample.  Here one block takes an
// item (a baseline at one channel in one interval), builds the sub-tables of
// every sub-lattice offset the item uses (f and its partner -f) in LDS, and
// walks the item's samples in time order: consecutive samples move by a
// fraction of a cell along the uv track, so a chunk of them covers a small
// box of the grid.  The chunk's taps are summed into an LDS patch covering
// that box (float32, sample by sample), and the patch is added to the
// residual grid once (float64 atomics), cutting the global atomics by the
// ratio of the chunk's taps to its box.  A chunk whose box does not fit the patch (a track
// crossing the grid's edge) adds its taps directly.
#include <climits>

#include "psc_device.h"

namespace psc {

template <int S>
__global__ void __launch_bounds__(kGridThreads) k_grid(ItemArgs a)
{
    constexpr int SP = S + 1, NT = S * S, W = kGridThreads / 64;
    constexpr int PB = kGridPatch, CH = kGridChunk;
    static_assert(NT == kGridThreads, "a thread per tap");

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float2 twsh[S * 16];      // exp(+2 pi i t / (S O)), O <= 16
    __shared__ float2 phsh[W][64];       // per-wave phases: l axis at [0, M), m axis at [32, 32 + M)
    __shared__ int box[4];               // chunk's rows [0], [1] and columns [2], [3] (min, max)
    __shared__ float4 rec[CH];           // chunk samples: k_lo, w conj(R), table slot

    const int m = a.m, half_m = m >> 1;
    const int m2p = (m * m + 3) & ~3;
    const int O = a.oversample, so = S * O;
    // dynamic LDS: sub-tables [2 groups][S][SP] | image-plane products | patch [PB][PB]
    float2* tab = reinterpret_cast<float2*>(smem);
    float* gsh = reinterpret_cast<float*>(tab + (size_t)2 * win_max_groups(O) * S * SP);
    float2* patch = reinterpret_cast<float2*>(gsh + m2p);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = item_of_block();
    if (li >= a.n_items) return;
    const Item it = a.items[a.item_begin + li];

    const int P = a.grid_n + S;  // pitch of the padded grid
    const float inv_s = 1.0f / (float)S;
    for (int t = tid; t < so; t += kGridThreads) twsh[t] = a.tw[t];

    // the item's samples: one contiguous range of the sample array
    const int n_grp = it.grp_end - it.grp_begin;
    uint32_t s_lo = UINT_MAX, s_n = 0;
    for (int gl = 0; gl < n_grp; ++gl) {
        const Group g = a.groups[it.grp_begin + gl];
        s_lo = min(s_lo, g.vis_begin);
        s_n += (uint32_t)(g.n_vis + g.n_vis2);
    }
    // this thread's tap (a_l, a_m) and its sub-table index b = (S-1-a_l, S-1-a_m)
    const int al = tid / S, am = tid - (tid / S) * S;
    const int boff = (S - 1 - al) * SP + (S - 1 - am);

    for (int pol = 0; pol < a.n_pol; ++pol) {
        image_products<kPredict>(a, it, pol, gsh, m2p, tid, kGridThreads);
        __syncthreads();

        // ---- sub-tables: wavefront w builds the groups w, w + W, ... (f at
        // slot 2 gl, its partner -f at slot 2 gl + 1)
        for (int gl = wave; gl < n_grp; gl += W) {
            const Group g = a.groups[it.grp_begin + gl];
            const int fl = g.f / O, fm = g.f - (g.f / O) * O;
            float2* ph = phsh[wave];
            if (lane < m) {
                const int n = lane - half_m;
                const float2 p = twsh[(fl * n) & (so - 1)];
                const float sg = (n & 1) ? -inv_s : inv_s;
                ph[lane] = make_float2(p.x * sg, p.y * sg);
            } else if (lane >= 32 && lane - 32 < m) {
                const int n = lane - 32 - half_m;
                const float2 p = twsh[(fm * n) & (so - 1)];
                const float sg = (n & 1) ? -inv_s : inv_s;
                ph[lane] = make_float2(p.x * sg, p.y * sg);
            }
            wave_sync();
            // fold: U[r] = sum over n = r mod S of phi_l(n_l) phi_m(n_m) g[n]
            float2* T = tab + (size_t)(2 * gl) * S * SP;
            for (int r = lane; r < NT; r += 64) {
                const int rl = r / S, rm = r - (r / S) * S;
                float2 u = make_float2(0.f, 0.f);
#pragma unroll
                for (int el = 0; el < 2; ++el) {
                    const int nl = rl - el * S;
                    if (nl < -half_m || nl >= half_m) continue;
                    float2 x = make_float2(0.f, 0.f);
#pragma unroll
                    for (int em = 0; em < 2; ++em) {
                        const int nmv = rm - em * S;
                        if (nmv < -half_m || nmv >= half_m) continue;
                        const float gv = gsh[(nl + half_m) * m + nmv + half_m];
                        const float2 pm = ph[32 + nmv + half_m];
                        x.x = fmaf(gv, pm.x, x.x);
                        x.y = fmaf(gv, pm.y, x.y);
                    }
                    cmac(u, ph[nl + half_m], x);
                }
                T[rl * SP + rm] = u;
            }
            wave_sync();
            // S x S DFT: rows, then columns
            if (lane < S) {
                float2 x[S];
#pragma unroll
                for (int i = 0; i < S; ++i) x[i] = T[lane * SP + i];
                fft_reg<S>(x);
#pragma unroll
                for (int i = 0; i < S; ++i) T[lane * SP + i] = x[i];
            }
            wave_sync();
            if (lane < S) {
                float2 x[S];
#pragma unroll
                for (int i = 0; i < S; ++i) x[i] = T[i * SP + lane];
                fft_reg<S>(x);
#pragma unroll
                for (int i = 0; i < S; ++i) T[i * SP + lane] = x[i];
            }
            wave_sync();
            if (g.n_vis2 > 0) {
                // partner -f: the conjugate, reflected (b -> S-1-b on an axis
                // with f != 0, b -> -b mod S on an axis with f = 0)
                float2* T2 = T + S * SP;
                for (int e = lane; e < NT; e += 64) {
                    const int bl = e / S, bm = e - (e / S) * S;
                    const int sl = fl ? (S - 1 - bl) : ((S - bl) & (S - 1));
                    const int sm = fm ? (S - 1 - bm) : ((S - bm) & (S - 1));
                    const float2 v = T[sl * SP + sm];
                    T2[bl * SP + bm] = make_float2(v.x, -v.y);
                }
            }
            wave_sync();  // the phases are rewritten by the wavefront's next group
        }
        __syncthreads();

        // ---- chunks of CH samples in time order
        for (uint32_t base = 0; base < s_n; base += CH) {
            const int nch = (int)min((uint32_t)CH, s_n - base);
            if (tid == 0) {
                box[0] = INT_MAX;
                box[1] = INT_MIN;
                box[2] = INT_MAX;
                box[3] = INT_MIN;
            }
            __syncthreads();
            if (tid < nch) {
                const uint2 od = a.ig_ord[s_lo + base + tid];
                const VisEnt e = a.vis[od.x];
                const size_t o = (size_t)e.vidx * a.n_pol + pol;
                const float2 vo = a.vis_in[o], vm = a.vis_model[o];
                const float wgt = a.weight[o];
                // w conj(R), R = V^Obs - V formed in float64
                const float rr = (float)((double)vo.x - (double)vm.x);
                const float ri = (float)((double)vo.y - (double)vm.y);
                rec[tid] = make_float4(__builtin_bit_cast(float, e.klo), wgt * rr, -wgt * ri,
                                       __builtin_bit_cast(float, od.y));
                const int row = (int)(e.klo >> 16), col = (int)(e.klo & 0xffffu);
                atomicMin(&box[0], row);
                atomicMax(&box[1], row);
                atomicMin(&box[2], col);
                atomicMax(&box[3], col);
            }
            __syncthreads();
            const int r0 = box[0], c0 = box[2];
            const int hgt = box[1] - r0 + S, wid = box[3] - c0 + S;
            const bool fits = hgt <= PB && wid <= PB;
            if (fits)
                for (int t = tid; t < hgt * PB; t += kGridThreads) patch[t] = make_float2(0.f, 0.f);
            __syncthreads();
            // the chunk's samples one after another: a sample's taps are
            // distinct cells, so each adds without atomics, in sample order
            // (float32 sums that do not depend on the schedule)
            for (int k = 0; k < nch; ++k) {
                const float4 rc = rec[k];
                const uint32_t klo = __builtin_bit_cast(uint32_t, rc.x);
                const int row = (int)(klo >> 16), col = (int)(klo & 0xffffu);
                const float2 kv = tab[(size_t)__builtin_bit_cast(uint32_t, rc.w) * S * SP + boff];
                const float vr = rc.y * kv.x - rc.z * kv.y, vi = rc.y * kv.y + rc.z * kv.x;
                if (fits) {
                    float2* pc = patch + (row - r0 + al) * PB + (col - c0 + am);
                    const float2 p0 = *pc;
                    *pc = make_float2(p0.x + vr, p0.y + vi);
                    __syncthreads();
                } else {
                    double2* gd = a.grid_acc + (size_t)(row + al) * P + (col + am);
                    unsafeAtomicAdd(&gd->x, (double)vr);
                    unsafeAtomicAdd(&gd->y, (double)vi);
                }
            }
            __syncthreads();
            if (fits) {
                for (int t = tid; t < hgt * wid; t += kGridThreads) {
                    const int r = t / wid, cc = t - (t / wid) * wid;
                    const float2 v = patch[r * PB + cc];
                    double2* gd = a.grid_acc + (size_t)(r0 + r) * P + (c0 + cc);
                    // cells no window of the chunk touched hold exact zeros
                    if (v.x != 0.f) unsafeAtomicAdd(&gd->x, (double)v.x);
                    if (v.y != 0.f) unsafeAtomicAdd(&gd->y, (double)v.y);
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Per-sample kernels: support 32, offsets in the mount frame, the w-term.
//
// Where an item's sub-tables do not fit in LDS (support 32), or every sample
// has a kernel of its own (mount frame: each row's parallactic angle rotates
// the beams), each wavefront builds the kernel of one sample at a time: the
// fold of the image-plane products with the sample's own phases (its offset
// f, or -f for a partner sample) and an S x S DFT through the wavefront's
// tile, exactly the sub-table the degrid used for it.  The block then adds
// the round's kernels, times w conj(R), to an LDS patch covering the item's
// windows, one sample after another in a fixed order, and adds the patch to
// the residual grid once at the end of the item; an item whose windows span
// more than a patch adds every tap directly with float64 atomics.
template <int S, int MF, bool WT>
__global__ void __launch_bounds__(kGridThreads) k_gridw(ItemArgs a)
{
    constexpr int SP = S + 1, NT = S * S, W = kGridThreads / 64;
    constexpr int PB = kGridPatch;

    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float2 twsh[S * 16];  // exp(+2 pi i t / (S O)), S O <= 16 S
    __shared__ float2 phsh[W][128];  // per wavefront: l-axis phases at [0, M), m axis at [64, 64 + M)
    __shared__ int box[4];           // item windows' first rows [0], [1] and columns [2], [3] (min, max)
    __shared__ float4 crec[W];       // per wavefront: w conj(R), k_lo, whether it has a sample

    const int m = a.m, half_m = m >> 1;
    const int m2p = (m * m + 3) & ~3;
    const int O = a.oversample, so = S * O;
    // dynamic LDS: image-plane products (sky frame) | tiles [W][S][SP] | patch [PB][PB] | Airy table
    // (mount frame)
    float* gsh = reinterpret_cast<float*>(smem);
    float2* tiles = reinterpret_cast<float2*>(gsh + (MF != kFrameSky ? 0 : m2p));
    float2* patch = tiles + (size_t)W * S * SP;
    float4* airy_sh = reinterpret_cast<float4*>(patch + PB * PB);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = item_of_block();
    if (li >= a.n_items) return;
    const Item it = a.items[a.item_begin + li];

    const int P = a.grid_n + S;  // pitch of the padded grid
    const float inv_s = 1.0f / (float)S;
    for (int t = tid; t < so; t += kGridThreads) twsh[t] = a.tw[t];
    if constexpr (MF == kFrameMount)
        for (int t = tid; t < a.n_tab; t += kGridThreads) airy_sh[t] = a.airy[t];
    if (tid == 0) {
        box[0] = INT_MAX;
        box[1] = INT_MIN;
        box[2] = INT_MAX;
        box[3] = INT_MIN;
    }
    // the item's samples: one contiguous range of the sample array
    const int n_grp = it.grp_end - it.grp_begin;
    uint32_t s_lo = UINT_MAX, s_n = 0;
    for (int gl = 0; gl < n_grp; ++gl) {
        const Group g = a.groups[it.grp_begin + gl];
        s_lo = min(s_lo, g.vis_begin);
        s_n += (uint32_t)(g.n_vis + g.n_vis2);
    }
    __syncthreads();
    for (uint32_t k = tid; k < s_n; k += kGridThreads) {
        const uint32_t klo = a.vis[s_lo + k].klo;
        const int row = (int)(klo >> 16), col = (int)(klo & 0xffffu);
        atomicMin(&box[0], row);
        atomicMax(&box[1], row);
        atomicMin(&box[2], col);
        atomicMax(&box[3], col);
    }
    __syncthreads();
    const int r0 = box[0], c0 = box[2];
    const int hgt = box[1] - r0 + S, wid = box[3] - c0 + S;
    const bool fits = s_n > 0 && hgt <= PB && wid <= PB;

    // beam constants of the item's channel (mount frame)
    const double lam = kCLight / a.freq[it.chan];
    const float kk = (float)(kPi * a.dish / lam);
    const double sigma = a.gauss_sigma_ld * lam / a.dish;
    const float inv_s2 = (float)(1.0 / (sigma * sigma));
    const float aps = (float)(a.dish / lam * a.ap_inv_step);  // aperture table nodes per radian
    const float hstep = (float)a.h;
    const double w_per_m = a.freq[it.chan] / kCLight;  // w-term: wavelengths per metre
    float2* wt = tiles + (size_t)wave * S * SP;
    float2* ph = phsh[wave];

    for (int pol = 0; pol < a.n_pol; ++pol) {
        const double sq = (pol == 0 ? 1.0 : -1.0) * a.squint_frac * 1.02899 * lam / a.dish;
        const double* oi = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.ai) * 2;
        const double* oj = a.offsets + (((size_t)it.interval * a.n_pol + pol) * a.n_ant + it.aj) * 2;
        const double qil = oi[0] + sq, qim = oi[1], qjl = oj[0] + sq, qjm = oj[1];
        if constexpr (MF == kFrameSky) image_products<kPredict>(a, it, pol, gsh, m2p, tid, kGridThreads);
        // each antenna's beam constants with its width scale (mount-frame paths)
        BeamK bki = beam_k(kk, inv_s2, aps, 1.f), bkj = bki;
        if (MF != kFrameSky && a.scale != nullptr) {
            const double* sc = a.scale + ((size_t)it.interval * a.n_pol + pol) * a.n_ant;
            bki = beam_k(kk, inv_s2, aps, (float)sc[it.ai]);
            bkj = beam_k(kk, inv_s2, aps, (float)sc[it.aj]);
        }
        if (fits)
            for (int t = tid; t < hgt * PB; t += kGridThreads) patch[t] = make_float2(0.f, 0.f);
        __syncthreads();

        for (uint32_t base = 0; base < s_n; base += W) {
            // ---- wavefront w builds the kernel of the item's sample base + w
            const uint32_t k = base + wave;
            if (k < s_n) {
                const uint32_t idx = s_lo + k;
                // its group and part
                int fl = 0, fm = 0;
                for (int gl = 0; gl < n_grp; ++gl) {
                    const Group g = a.groups[it.grp_begin + gl];
                    if (idx >= g.vis_begin && idx < g.vis_begin + (uint32_t)(g.n_vis + g.n_vis2)) {
                        fl = g.f / O;
                        fm = g.f - (g.f / O) * O;
                        if (idx >= g.vis_begin + (uint32_t)g.n_vis) {
                            fl = (O - fl) & (O - 1);
                            fm = (O - fm) & (O - 1);
                        }
                    }
                }
                const VisEnt e = a.vis[idx];
                const size_t o = (size_t)e.vidx * a.n_pol + pol;
                // per-axis phases (-1)^n exp(2 pi i f n / (S O)) / S of the sample's offset
                for (int j = lane; j < m; j += 64) {
                    const int n = j - half_m;
                    const float sg = (n & 1) ? -inv_s : inv_s;
                    const float2 pl = twsh[(fl * n) & (so - 1)], pm = twsh[(fm * n) & (so - 1)];
                    ph[j] = make_float2(pl.x * sg, pl.y * sg);
                    ph[64 + j] = make_float2(pm.x * sg, pm.y * sg);
                }
                float pil = (float)qil, pim = (float)qim, pjl = (float)qjl, pjm = (float)qjm;
                const float wl = WT ? (float)(a.w_m[e.vidx / (uint32_t)a.n_chan] * w_per_m) : 0.f;
                float sn = 0.f, cs = 1.f;
                if constexpr (MF != kFrameSky) {
                    // this row's beam centres on the sky
                    sincosf((float)a.par_angle[e.vidx / (uint32_t)a.n_chan], &sn, &cs);
                    pil = (float)(cs * qil - sn * qim);
                    pim = (float)(sn * qil + cs * qim);
                    pjl = (float)(cs * qjl - sn * qjm);
                    pjm = (float)(sn * qjl + cs * qjm);
                }
                wave_sync();
                // fold: U[r] = sum over n = r mod S of phi_l(n_l) phi_m(n_m) g[n]
                for (int r = lane; r < NT; r += 64) {
                    const int rl = r / S, rm = r - (r / S) * S;
                    float2 u = make_float2(0.f, 0.f);
#pragma unroll
                    for (int el = 0; el < 2; ++el) {
                        const int nl = rl - el * S;
                        if (nl < -half_m || nl >= half_m) continue;
                        float2 x = make_float2(0.f, 0.f);
#pragma unroll
                        for (int em = 0; em < 2; ++em) {
                            const int nmv = rm - em * S;
                            if (nmv < -half_m || nmv >= half_m) continue;
                            float gv;
                            const float l = (float)nl * hstep, mm = (float)nmv * hstep;
                            if constexpr (MF == kFrameAperture) {
                                float ei, ej, unused;
                                efp_ap<false>(a, ap_table(a, it.ai), bki.aps, cs, sn, l - pil, mm - pim, ei,
                                              unused, unused);
                                efp_ap<false>(a, ap_table(a, it.aj), bkj.aps, cs, sn, l - pjl, mm - pjm, ej,
                                              unused, unused);
                                gv = ei * ej * (a.taper_img[nl + half_m] * a.taper_img[nmv + half_m]);
                            } else if constexpr (MF == kFrameMount) {
                                float ei, qi, ej, qj;
                                efq(a, airy_sh, bki.kk, bki.inv_s2, l - pil, mm - pim, ei, qi);
                                efq(a, airy_sh, bkj.kk, bkj.inv_s2, l - pjl, mm - pjm, ej, qj);
                                gv = ei * ej * (a.taper_img[nl + half_m] * a.taper_img[nmv + half_m]);
                            } else {
                                gv = gsh[(nl + half_m) * m + nmv + half_m];
                            }
                            const float2 pm = ph[64 + nmv + half_m];
                            if constexpr (WT) {
                                // times exp(2 pi i w (n - 1)), n - 1 = -x / (1 + sqrt(1 - x)),
                                // the phase in turns reduced to [0, 1) for the hardware sine
                                const float xx = fmaf(l, l, mm * mm);
                                const float nm1 = -xx * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_sqrtf(1.f - xx));
                                const float rv = __builtin_amdgcn_fractf(wl * nm1);
                                const float sn = __builtin_amdgcn_sinf(rv), cs = __builtin_amdgcn_cosf(rv);
                                cmac(x, make_float2(gv * cs, gv * sn), pm);
                            } else {
                                x.x = fmaf(gv, pm.x, x.x);
                                x.y = fmaf(gv, pm.y, x.y);
                            }
                        }
                        cmac(u, ph[nl + half_m], x);
                    }
                    wt[rl * SP + rm] = u;
                }
                wave_sync();
                // S x S DFT: rows, then columns
                if (lane < S) {
                    float2 x[S];
#pragma unroll
                    for (int i = 0; i < S; ++i) x[i] = wt[lane * SP + i];
                    fft_reg<S>(x);
#pragma unroll
                    for (int i = 0; i < S; ++i) wt[lane * SP + i] = x[i];
                }
                wave_sync();
                if (lane < S) {
                    float2 x[S];
#pragma unroll
                    for (int i = 0; i < S; ++i) x[i] = wt[i * SP + lane];
                    fft_reg<S>(x);
#pragma unroll
                    for (int i = 0; i < S; ++i) wt[i * SP + lane] = x[i];
                }
                if (lane == 0) {
                    // w conj(R), R = V^Obs - V formed in float64
                    const float2 vo = a.vis_in[o], vm = a.vis_model[o];
                    const float wgt = a.weight[o];
                    const float rr = (float)((double)vo.x - (double)vm.x);
                    const float ri = (float)((double)vo.y - (double)vm.y);
                    crec[wave] = make_float4(wgt * rr, -wgt * ri, __builtin_bit_cast(float, e.klo), 1.f);
                }
            } else if (lane == 0) {
                crec[wave] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            __syncthreads();

            // ---- the round's kernels times w conj(R), in wavefront order
            for (int w2 = 0; w2 < W; ++w2) {
                const float4 rc = crec[w2];
                if (rc.w == 0.f) continue;
                const uint32_t klo = __builtin_bit_cast(uint32_t, rc.z);
                const int row = (int)(klo >> 16), col = (int)(klo & 0xffffu);
                const float2* T = tiles + (size_t)w2 * S * SP;
                for (int t = tid; t < NT; t += kGridThreads) {
                    // tap (a_l, a_m) at sub-table index (S-1-a_l, S-1-a_m)
                    const int al = t / S, am = t - (t / S) * S;
                    const float2 kv = T[(S - 1 - al) * SP + (S - 1 - am)];
                    const float vr = rc.x * kv.x - rc.y * kv.y, vi = rc.x * kv.y + rc.y * kv.x;
                    if (fits) {
                        float2* pc = patch + (row - r0 + al) * PB + (col - c0 + am);
                        const float2 p0 = *pc;
                        *pc = make_float2(p0.x + vr, p0.y + vi);
                    } else {
                        double2* gd = a.grid_acc + (size_t)(row + al) * P + (col + am);
                        unsafeAtomicAdd(&gd->x, (double)vr);
                        unsafeAtomicAdd(&gd->y, (double)vi);
                    }
                }
                if (fits) __syncthreads();  // the next sample's taps may reach the same cells
            }
            __syncthreads();  // tiles and records are rewritten by the next round
        }

        if (fits) {
            for (int t = tid; t < hgt * wid; t += kGridThreads) {
                const int r = t / wid, cc = t - (t / wid) * wid;
                const float2 v = patch[r * PB + cc];
                double2* gd = a.grid_acc + (size_t)(r0 + r) * P + (c0 + cc);
                // cells no window of the item touched hold exact zeros
                if (v.x != 0.f) unsafeAtomicAdd(&gd->x, (double)v.x);
                if (v.y != 0.f) unsafeAtomicAdd(&gd->y, (double)v.y);
            }
        }
        __syncthreads();  // the patch and products are rewritten for the next polarisation
    }
}

size_t gridw_lds_bytes(int support, int m, int mount_frame_tab)
{
    const bool mf = mount_frame_tab >= 0;
    const size_t m2p = (size_t)((m * m + 3) & ~3);
    return (mf ? 0 : sizeof(float) * m2p) + sizeof(float2) * (kGridThreads / 64) * support * (support + 1) +
           sizeof(float2) * kGridPatch * kGridPatch + (mf ? sizeof(float4) * mount_frame_tab : 0);
}

template <int S, int MF, bool WT>
static hipError_t launch_gridw_t(const ItemArgs& a, hipStream_t s)
{
    const size_t sh = gridw_lds_bytes(S, a.m, MF == kFrameMount ? a.n_tab : MF == kFrameAperture ? 0 : -1);
    if (sh > kGridLdsMax) return hipErrorInvalidValue;
    static const hipError_t attr = hipFuncSetAttribute(
        (const void*)k_gridw<S, MF, WT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGridLdsMax);
    if (attr != hipSuccess) return attr;
    const int blocks = (int)item_blocks(a.n_items);
    k_gridw<S, MF, WT><<<blocks, kGridThreads, sh, s>>>(a);
    return hipGetLastError();
}

template <int S>
static hipError_t launch_gridw_f(int frame, bool wt, const ItemArgs& a, hipStream_t s)
{
    switch (frame) {
    case kFrameSky: return wt ? launch_gridw_t<S, kFrameSky, true>(a, s) : launch_gridw_t<S, kFrameSky, false>(a, s);
    case kFrameMount:
        return wt ? launch_gridw_t<S, kFrameMount, true>(a, s) : launch_gridw_t<S, kFrameMount, false>(a, s);
    default:
        return wt ? launch_gridw_t<S, kFrameAperture, true>(a, s) : launch_gridw_t<S, kFrameAperture, false>(a, s);
    }
}

hipError_t launch_gridw(int support, const ItemArgs& a, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const int fr = a.ap_tab != nullptr ? kFrameAperture : a.par_angle != nullptr ? kFrameMount : kFrameSky;
    const bool wt = a.w_m != nullptr;
    if (support == 16) return launch_gridw_f<16>(fr, wt, a, s);
    if (support == 32) return launch_gridw_f<32>(fr, wt, a, s);
    return hipErrorInvalidValue;
}

size_t grid_lds_bytes(int support, int m, int oversample)
{
    const size_t m2p = (size_t)((m * m + 3) & ~3);
    return sizeof(float2) * 2 * win_max_groups(oversample) * support * (support + 1) + sizeof(float) * m2p +
           sizeof(float2) * kGridPatch * kGridPatch;
}

hipError_t launch_grid(int support, const ItemArgs& a, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    if (support != 16) return hipErrorInvalidValue;
    const size_t sh = grid_lds_bytes(support, a.m, a.oversample);
    if (sh > kGridLdsMax) return hipErrorInvalidValue;
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)k_grid<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kGridLdsMax);
    if (attr != hipSuccess) return attr;
    const int blocks = (int)item_blocks(a.n_items);
    k_grid<16><<<blocks, kGridThreads, sh, s>>>(a);
    return hipGetLastError();
}

}  // namespace psc
