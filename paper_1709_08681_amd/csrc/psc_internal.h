// psc_internal.h -- types shared by the host API and the kernels of libpsc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psc {

constexpr double kCLight = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 256;  // threads per work-item block (4 wavefronts)
constexpr int kWaves = kBlock / 64;

// One work item: the samples of one baseline in one solution interval at one
// channel.  Its samples are split into groups by sub-lattice offset f.
struct Item {
    int32_t interval;
    int32_t ai, aj;  // antennas, ai < aj
    int32_t chan;
    int32_t grp_begin, grp_end;  // [begin, end) into the group array
    uint32_t vis_begin;          // the item's samples: [vis_begin, vis_begin + n_vis) of the
    int32_t n_vis;               // sample arrays (grouped by offset, or in row order)
};

// Samples of an item sharing the sub-lattice offset f = fl * O + fm, which
// selects one S x S sub-table of the oversampled kernel, followed by the
// samples of the opposite offset -f (mod O per axis), whose sub-table is the
// reflected conjugate of f's because the image-plane products are real.
struct Group {
    int32_t f;
    uint32_t vis_begin;  // into the sample array
    int32_t n_vis;       // samples at offset f
    int32_t n_vis2;      // samples at offset -f that follow them (0 if -f == f)
};

// One visibility sample: vidx = row * n_chan + chan (vis arrays are
// [vidx][pol]), klo = first grid row/column of its S x S window, packed as
// (row << 16) | column, both already reduced modulo N.  The table form reads
// an item's samples grouped by sub-lattice offset (Group); the window form
// reads them in row order (time order within a baseline), each with its own
// offset (fl << 4) | fm in a byte array beside.
struct VisEnt {
    uint32_t vidx;
    uint32_t klo;
};

enum Mode { kPredict = 0, kGrad = 1, kVjp = 2, kGrid = 3, kScale = 4 };

// Beam frame of the window-form kernels: radial beams on the sky (factored
// image-plane products), radial beams in the mount frame (per-sample
// products at each row's rotated centres), or a measured aperture's pattern
// in the mount frame (per-sample products from its tabulated transform).
enum Frame { kFrameSky = 0, kFrameMount = 1, kFrameAperture = 2 };

// Kernel variants a mode degrids (V, its four offset derivatives, or its two
// beam-scale derivatives) and the float64 sums it keeps per item.
__host__ __device__ constexpr int mode_nv(int mode)
{
    return mode == kGrad ? 5 : mode == kVjp ? 4 : mode == kScale ? 3 : 1;
}
__host__ __device__ constexpr int mode_nc(int mode)
{
    return mode == kGrad ? 12 : mode == kVjp ? 4 : mode == kScale ? 6 : 0;
}

// Work items per launch are spread over the eight XCDs (each with its own
// L2) in chunks of kXcdChunk consecutive items dealt round-robin: the
// hardware hands block b to XCD b mod 8, so the k-th block an XCD runs takes
// item ((k / C) 8 + b mod 8) C + k mod C.  Consecutive items (the channels of
// one baseline, which read the same rows of the visibility arrays) stay on
// one XCD, while every XCD sees every part of the item list, so a launch
// whose items differ in cost along the list (uneven solution intervals)
// stays balanced.  Launch item_blocks(n) blocks and skip li >= n.
constexpr int kXcdChunk = 32;
__host__ __device__ inline long long item_blocks(long long n_items)
{
    return 8LL * kXcdChunk * ((n_items + 8LL * kXcdChunk - 1) / (8LL * kXcdChunk));
}
__device__ __forceinline__ int item_of_block()
{
    const int b = (int)blockIdx.x, k = b >> 3;
    return (((k / kXcdChunk) << 3) + (b & 7)) * kXcdChunk + (k % kXcdChunk);
}

// Arguments of the fused kernel-build + degrid kernel.
struct ItemArgs {
    const Item* items;
    const Group* groups;
    const VisEnt* vis;
    const VisEnt* wvis;         // window form: each item's samples in row order
    const uint8_t* wf;          // window form: each sample's offset (fl << 4) | fm
    int32_t item_begin, n_items;
    int32_t n_ant, n_pol, n_chan;
    const double* offsets;      // [n_int][n_pol][n_ant][2]
    const double* freq;         // [n_chan]
    const float2* grid;         // V^{M0}, [N+S][N+S], last S rows/columns repeat the first
    int32_t grid_n;
    int32_t oversample;
    int32_t m;                  // image samples per axis
    double h;                   // image sample spacing (FoV / S)
    const float* taper_img;     // [m] taper response at the image samples
    const float2* tw;           // [S*O] exp(+2 pi i t / (S O))
    double dish;
    int32_t illum;
    double gauss_sigma_ld;
    double squint_frac;
    const float4* airy;         // [n_tab] (A, dx A', B, dx B') at x = i * dx
    int32_t n_tab;
    float inv_dx;
    // mode-specific
    float2* vis_out;            // predict: V^M; grad: optional V^M
    const float2* vis_in;       // grad: V^Obs; vjp: G
    const float* weight;        // grad
    double* partials;           // [item][pol][ncontrib]
    const int32_t* done;        // nullable: per-interval skip flags
    double2* grid_acc;          // grid mode: residual grid, (N+S) x (N+S), float64 sums
    const double* par_angle;    // nullable [n_row]: offsets in the mount frame (window form)
    const double* w_m;          // nullable [n_row]: baseline w in metres, the w-term (window form)
    // w-stacking (w_nk > 0): the model grid again for w = w_k, k = w_k0 ..
    // w_k0 + w_nk - 1, w_k = k w_dw wavelengths, each (N+S)^2 and padded like
    // the grid: the transform of I exp(2 pi i w_k (n - 1)) / c
    const float2* wgrid;
    double w_dw;
    int32_t w_k0, w_nk;
    // measured apertures (illum 2): each one's transform on [ap_n][ap_n]
    // nodes in lambda/D units, (T, s dT/du, s dT/dv, s^2 d2T/dudv) at
    // u = (i - ap_c) s, s = 1 / ap_inv_step, i along the mount frame's l
    // axis, stacked [n_apertures][ap_n][ap_n]; ap_ant (nullable [n_ant])
    // names each antenna's (null: the first)
    const float4* ap_tab;
    const int32_t* ap_ant;
    int32_t ap_n;
    float ap_c;
    float ap_inv_step;
    // nullable [n_int][n_pol][n_ant]: beam-width scale sigma of each antenna,
    // pattern E0(d / sigma) (per-sample products: mount-frame paths only)
    const double* scale;
    // nullable [n_int][n_pol][n_ant]: aperture defocus delta of each antenna
    // (radians of phase at the rim; complex patterns, sky frame): with
    // illum 0 the pattern is sum_n (i delta)^n / n! M_n(x) from the moment
    // table mtab [x node][n_mom] (M_n(x) = 2 int_0^1 J0(x t) t^(2n+1) dt,
    // (value, dx slope) at x = node / 16), with illum 1 a closed form
    const double* defocus;
    const float2* mtab;
    int32_t n_mom;
    // window form at support 16: 1 or 2 for blocks of one or two wavefronts
    // (items of few samples, where four would leave workers idle), 0 to size
    // blocks by LDS alone
    int32_t win_waves;
    int32_t tab_lds;            // window form: the Airy table is staged in LDS (set by the launcher)
    int32_t unit_items;         // window form: consecutive items per block (set by the launcher)
    // window form, sky frame, radial beams: every antenna's pattern and
    // gradient factor (E, q) at the image samples, [n_int][n_pol][n_chan]
    // [n_ant][m^2], filled for intervals [beam_int0, beam_int1) before the
    // degrid (null: each item evaluates its two antennas' patterns itself)
    float2* beams;
    int32_t beam_int0, beam_int1;
    int32_t use_mfma;           // degrid on the matrix cores (gradient and adjoint)
    // image-gradient scatter (k_grid)
    const uint2* ig_ord;        // per item, its samples in time order: (sample index, sub-table slot)
    const float2* vis_model;    // V from the preceding predict
};

struct ReduceArgs {
    const uint32_t* ant_ptr;    // [(n_int * n_ant) + 1]
    const uint32_t* ant_ent;    // item * 2 + end
    const Item* items;
    const double* partials;
    int32_t n_int, n_pol, n_ant;
    int32_t int_begin, int_end;
    double* out;                // [n_int][n_pol][n_ant][ncontrib/2]
    const int32_t* done;
};

struct SolveArgs {
    int32_t n_int, n_pol, n_ant;
    int32_t int_begin, int_end;
    const double* acc;          // [n_int][n_pol][n_ant][6]
    double gain;
    double lm_mu;               // Levenberg-Marquardt damping of diag(H), >= 0
    double* offsets;
    int32_t* not_updated;       // nullable
    double* max_step;           // nullable
    int32_t* done;              // nullable (solve loop state)
    int32_t* iters;             // nullable
    double tol;
};

// Kernel launchers (psc_kernels.hip).  Each returns the launch's hipError_t.
hipError_t launch_taper_image(const double* img, const double* taper_pix, double2* out, int n,
                              hipStream_t s);
hipError_t launch_wplane_image(const double* img, const double* taper_pix, double2* out, int n, double cell,
                               double w, hipStream_t s);
hipError_t launch_fft_rows(double2* data, int n, int log2n, hipStream_t s);
hipError_t launch_transpose(const double2* in, double2* out, int n, hipStream_t s);
hipError_t launch_finish_grid(const double2* in, float2* out, int n, int pad, hipStream_t s);
hipError_t launch_airy_table(float4* tab, int n_tab, double dx, hipStream_t s);
// Measured-aperture pattern table (psc_aperture.hip): n x n nodes at
// u = (i - c) step (lambda/D units) from the aperture's non-zero cells
// [n_cells][3] = (xi, eta, weight), xi and eta in units of D.
hipError_t launch_aperture_table(const double* cells, int n_cells, float4* tab, int n, double c, double step,
                                 hipStream_t s);
// Damped step of the beam-width scales (psc_scale.hip): per (interval, pol,
// antenna) sigma += gain g / H from acc3 = (chi, g, H); one block per interval.
// done, iters (nullable): solve state, as for the offsets' step.
hipError_t launch_scale_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* scale,
                             int32_t* not_updated, double* max_step, int32_t* done, int32_t* iters, double tol,
                             double min_scale, hipStream_t s);
hipError_t launch_zero(double2* p, size_t n, hipStream_t s);
// Aperture defocus (psc_scale.hip): the uniform disc's moment table, and the
// damped step delta += gain g / H per (interval, pol, antenna), kept within
// |delta| <= kMaxDefocus (steps beyond are not taken and flagged).
hipError_t launch_moment_table(float2* tab, int n_tab, int n_mom, double dx, const double* gl_t, const double* gl_w,
                               int n_gl, hipStream_t s);
hipError_t launch_defocus_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* defocus,
                               int32_t* not_updated, double* max_step, hipStream_t s);
hipError_t launch_unpad_grid(const double2* g, double2* out, int n, int pad, hipStream_t s);
hipError_t launch_image_grad(const double2* f, const double* taper_pix, double* out, int n, hipStream_t s);
hipError_t launch_items(int mode, int support, const ItemArgs& a, hipStream_t s);
// Window-form degrid (psc_window.hip), k_winw: workers of 2S lanes (a
// wavefront at support 32, half a wavefront at 16), four or eight wavefronts
// per block.  win_lds_bytes is the dynamic LDS of the larger block,
// winw_lds_bytes that of a block of the given wavefronts, win_lds_budget the
// most a block may use (160 KiB per compute unit less the static twiddles).
// Groups of an item, at most: they pair offsets f and -f, so O^2/2 + 2 (the
// four self-paired offsets on their own).
__host__ __device__ inline int win_max_groups(int oversample)
{
    return oversample == 1 ? 1 : oversample * oversample / 2 + 2;
}
hipError_t launch_win(int mode, int support, const ItemArgs& a, hipStream_t s);
// mount_frame_tab: -1 for sky-frame offsets, else the Airy table length the
// mount-frame kernel keeps in LDS
size_t win_lds_bytes(int support, int mode, int m, int oversample, int mount_frame_tab = -1);
size_t winw_lds_bytes(int support, int waves, int mode, int m, int oversample, int mount_frame_tab = -1);
size_t win_lds_budget(int support);
// Wavefronts per block of a window-form launch (frame: a kFrame* value, or
// kFrameSkyAperture for a measured aperture without parallactic angles),
// given the plan's choice for items of few samples (ItemArgs::win_waves); 0
// when no block fits.
constexpr int kFrameSkyAperture = 3;
// Complex patterns in the sky frame (an aperture phase term): complex
// image-plane products per image sample, summed plainly.
constexpr int kFrameSkyComplex = 4;
// Aperture defocus: moments M_0 .. M_{kMoments-1} of the uniform disc, enough
// for the pattern's series to 1e-13 at |delta| <= kMaxDefocus.
constexpr int kMoments = 27;
constexpr double kMaxDefocus = 3.14159265358979323846;
int win_block_waves(int support, int mode, int frame, int m, int oversample, int n_tab, int plan_waves);
// Items per block of a window-form launch over n_items items: the sky-frame
// variants at support 32, whose set-up (twiddles, Airy table in LDS) is
// largest against an item's work, take kWinItemsPerBlock consecutive items
// when a launch has at least kWinMultiItemMin; every other launch one.
constexpr int kWinItemsPerBlock = 32;
constexpr long long kWinMultiItemMin = 1LL << 19;
__host__ __device__ constexpr bool win_multi_item(int support, int frame)
{
    return support == 32 && frame == kFrameSky;
}
__host__ __device__ constexpr int win_items_per_block(int support, int frame, long long n_items)
{
    return win_multi_item(support, frame) && n_items >= kWinMultiItemMin ? kWinItemsPerBlock : 1;
}
// Image-gradient scatter with per-item LDS patches (psc_grid.hip), support
// 16: one thread per tap, chunks of kGridChunk samples, patches of
// kGridPatch^2 cells.  grid_lds_bytes is its dynamic LDS; launch_grid refuses
// more than kGridLdsMax (the caller then uses the table-form scatter).
constexpr int kGridThreads = 256;
constexpr int kGridPatch = 48;
constexpr int kGridChunk = 32;
constexpr size_t kGridLdsMax = 150 * 1024;
size_t grid_lds_bytes(int support, int m, int oversample);
hipError_t launch_grid(int support, const ItemArgs& a, hipStream_t s);
// The same scatter with a kernel built per sample (support 32, mount frame):
// gridw_lds_bytes is its dynamic LDS (mount_frame_tab as for win_lds_bytes).
size_t gridw_lds_bytes(int support, int m, int mount_frame_tab = -1);
hipError_t launch_gridw(int support, const ItemArgs& a, hipStream_t s);
hipError_t launch_reduce(int ncontrib, const ReduceArgs& a, hipStream_t s);
hipError_t launch_solve(const SolveArgs& a, hipStream_t s);
hipError_t launch_init_state(int32_t* done, int32_t* iters, int n, hipStream_t s);

}  // namespace psc
