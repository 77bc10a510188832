// psc_api.hip -- host side of libpsc: the C ABI declared in include/psc.h,
// argument checking, the anti-aliasing taper, observation planning and the
// three execution forms of the solver loop (Algorithm 1).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/psc.h"
#include "psc_internal.h"

using namespace psc;

struct psc_ctx {
    psc_config cfg{};
    int n = 0, s = 0, o = 0, m = 0;
    double fov = 0, h = 0, snap = 0;
    float2* grid = nullptr;        // V^{M0}, (N+S) x (N+S) complex64, periodic padding
    double* taper_pix = nullptr;   // [N]
    float* taper_img = nullptr;    // [M]
    float2* tw = nullptr;          // [S*O]
    // image-gradient scratch, allocated by its first call
    double2* rgrid = nullptr;      // residual grid, (N+S) x (N+S)
    double2* fa = nullptr;         // [N][N] transform work
    double2* fb = nullptr;
    // measured apertures (illum 2), each as its non-zero cells (xi, eta,
    // weight), xi and eta in units of D, weights summing to one
    std::vector<std::vector<double>> ap_cells;
    double* image = nullptr;            // the model image [N][N] float64, kept for w-planes
    std::vector<psc_obs*> stacked;      // observations with w-planes, rebuilt with the model
    bool model_set = false;
    std::string err;
};

struct psc_obs {
    psc_ctx* ctx = nullptr;
    int32_t n_ant = 0, n_chan = 0, n_pol = 0, n_int = 0;
    int64_t n_row = 0;
    std::vector<int32_t> int_item_ptr;  // host copy, [n_int+1]
    int64_t n_items = 0, n_groups = 0, n_vis = 0;
    Item* items = nullptr;
    Group* groups = nullptr;
    VisEnt* vis = nullptr;
    VisEnt* wvis = nullptr;    // the same samples, per item in row order (window form)
    uint8_t* wf = nullptr;     // their offsets (fl << 4) | fm
    // w-stacking: the model grid for w_k = k w_dw wavelengths, k = w_k0 ..
    // w_k0 + w_nk - 1, [w_nk][(N+S)^2] complex64 (w_nk = 0: none)
    float2* wplanes = nullptr;
    int32_t w_k0 = 0, w_nk = 0;
    double w_dw = 0;
    uint32_t* ant_ptr = nullptr;
    uint32_t* ant_ent = nullptr;
    double* freq = nullptr;
    double* par_angle = nullptr;  // [n_row] or null (sky-frame offsets)
    double* w_m = nullptr;        // [n_row] or null (no w-term)
    float4* airy = nullptr;
    int32_t n_tab = 0;
    double inv_dx = 0;
    double fmax = 0;           // highest channel frequency (Hz)
    float4* ap_tab = nullptr;  // measured apertures: pattern tables [n_apertures][ap_n][ap_n]
    int32_t* ap_ant = nullptr; // [n_ant] each antenna's aperture (null: all the first)
    float2* beams = nullptr;   // sky frame, radial beams: per-antenna (E, q) tables (ItemArgs::beams)
    double* scale = nullptr;   // beam-width scales [n_int][n_pol][n_ant] (null: all 1)
    double* defocus = nullptr; // aperture defocus [n_int][n_pol][n_ant] (null: none; complex patterns)
    float2* mtab = nullptr;    // the uniform disc's moment table [n_tab][kMoments] (defocus, illum 0)
    double* zero_pa = nullptr; // [n_row] zeros: the per-sample scatter's angles with scales, sky frame
    int32_t win_waves = 0;     // window-form block size at support 16 (see ItemArgs)
    double plan_ms = 0;        // wall time psc_obs_create took
    double capture_ms = 0;     // wall time of the last solve graph's capture + instantiation
    int32_t ap_n = 0;
    double ap_c = 0, ap_step = 0;
    // the tables' ranges at beam scale 1 (Airy argument x, aperture radius in
    // lambda/D), and the smallest scale they cover
    double tab_x1 = 0, ap_r1 = 0, tab_scale = 1.0;
    double* partials = nullptr;  // [n_items][n_pol][12]
    double* acc = nullptr;       // [n_int][n_pol][n_ant][6]
    double* max_step = nullptr;  // [n_int]
    int32_t* done = nullptr;     // [n_int]
    int32_t* iters = nullptr;    // [n_int]
    uint2* ig_ord = nullptr;     // image gradient: per item, samples in time order (built on first use)
    float2* ig_vm = nullptr;     // image gradient: model visibilities when the caller passes none
    int32_t degrid = PSC_DEGRID_VALU;  // variant for gradient / adjoint
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    // arguments the captured graph was built with
    const void* g_vis = nullptr;
    const float* g_w = nullptr;
    double* g_off = nullptr;
    double g_gain = 0, g_tol = 0;
    int32_t g_nmax = -1;
};

namespace {

thread_local std::string g_create_err;

psc_status fail(psc_ctx* ctx, psc_status st, const std::string& msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_create_err = msg;
    return st;
}

psc_status hip_fail(psc_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, PSC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define PSC_HIP(ctx, call)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

template <class T>
hipError_t dmalloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, sizeof(T) * count);
}

template <class T>
void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Image-plane response of the exponential-of-semicircle taper
// phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| <= 1, spanning W uv cells:
//   c(x) = (W/2) int_{-1}^{1} phi(z) cos(pi W x z) dz,  x = l / FoV,
// integrated with z = sin(theta), which removes the end-point square root.
struct Taper {
    int width;
    double beta;
    std::vector<double> gx, gw;
    Taper(int w, double b) : width(w), beta(b) { gauss_legendre(256, gx, gw); }
    double operator()(double x) const
    {
        double acc = 0.0;
        for (size_t i = 0; i < gx.size(); ++i) {
            const double th = 0.5 * kPi * gx[i];
            const double z = sin(th);
            acc += gw[i] * exp(beta * (cos(th) - 1.0)) * cos(kPi * width * x * z) * cos(th);
        }
        return 0.5 * width * 0.5 * kPi * acc;
    }
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Largest |w| FoV / D the window form takes with the w-term: the kernel
// spread of the w phase over a beam width, in uv cells (measured against the
// direct sum: relative error below 1e-5 up to about 1.8 at both supports).
constexpr double kMaxWCells = 1.5;
// w-stacking: the residual w - w_k a sample's kernel carries widens it by at
// most this many cells.
constexpr double kWStackCells = 1.0;

int floor_div(long long a, int b)
{
    long long q = a / b;
    if ((a % b) != 0 && ((a < 0) != (b < 0))) --q;
    return (int)q;
}

}  // namespace

// Per-antenna pattern tables are used while one interval's tables (all
// polarisations, channels and antennas) stay within 8 MiB, about two XCDs'
// L2: items run interval by interval, and an item reads its second
// antenna's tables cold.  The batched workload needs 2 MB per interval
// (2.4% faster per gradient); one GPU's share of the large workload would
// need 75 MB per interval and fetched 734 GB per launch from HBM for no
// gain, so its items evaluate their own patterns.  The whole allocation is
// capped at 16 GiB.
constexpr size_t kBeamTabIntervalBytes = size_t(8) << 20;
constexpr size_t kBeamTabBytes = size_t(16) << 30;

// Scratch of the allocation-free gradient (psc_gradient_noalloc): the
// per-item float64 partial sums, kept in a file-scope device array so that
// the call allocates nothing.  Every GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not a device address: host code uses only the per-device address
// that hipGetSymbolAddress returns (scratch_address).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch, looked up once per
// device (the device `dev` must be current).
hipError_t scratch_address(int dev, double** out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

PSC_API const char* psc_version(void) { return "psc 0.1 (gfx950)"; }

PSC_API const char* psc_last_error(const psc_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

static psc_status create_impl(const psc_config* cfg, psc_ctx** out)
{
    g_create_err.clear();
    if (!cfg || !out) return fail(nullptr, PSC_E_ARG, "null config or output pointer");
    *out = nullptr;
    const psc_config& c = *cfg;
    if (!is_pow2(c.grid_n) || c.grid_n < 64 || c.grid_n > 8192)
        return fail(nullptr, PSC_E_ARG, "grid_n must be a power of two in [64, 8192]");
    if (c.support != 16 && c.support != 32)
        return fail(nullptr, PSC_E_ARG, "support must be 16 or 32");
    if (c.oversample < 1 || c.oversample > 16 || !is_pow2(c.oversample) || c.support * c.oversample > 512)
        return fail(nullptr, PSC_E_ARG, "oversample must be a power of two in [1, 16] with support*oversample <= 512");
    const int m = c.image_samples ? c.image_samples : 3 * c.support / 2;
    if (m < c.support || m > 2 * c.support || (m & 1))
        return fail(nullptr, PSC_E_ARG, "image_samples must be even and in [support, 2*support]");
    const int tw = c.taper_width ? c.taper_width : 8;
    const double tb = c.taper_beta > 0 ? c.taper_beta : 2.30 * tw;
    if (tw < 2 || tw >= c.support) return fail(nullptr, PSC_E_ARG, "taper_width must be in [2, support)");
    if (!(c.cell_rad > 0) || !(c.dish_diam_m > 0) || !isfinite(c.cell_rad))
        return fail(nullptr, PSC_E_ARG, "cell_rad and dish_diam_m must be positive");
    if (c.illum < 0 || c.illum > 2) return fail(nullptr, PSC_E_ARG, "illum must be 0, 1 or 2");
    // each aperture as its non-zero cells (x, y in units of D, weight over
    // the aperture's sum)
    std::vector<std::vector<double>> ap_cells;
    if (c.illum == 2) {
        const int an = c.aperture_n;
        const int n_ap = c.aperture_count > 0 ? c.aperture_count : 1;
        if (!c.aperture || an < 1 || an > 256)
            return fail(nullptr, PSC_E_ARG, "illum 2 needs an aperture of aperture_n in [1, 256] cells per side");
        if (n_ap > 256) return fail(nullptr, PSC_E_ARG, "aperture_count above 256");
        for (int k = 0; k < n_ap; ++k) {
            const double* A = c.aperture + (size_t)k * an * an;
            double sum = 0.0;
            for (int i = 0; i < an; ++i)
                for (int j = 0; j < an; ++j) {
                    const double v = A[(size_t)i * an + j];
                    if (!isfinite(v) || v != A[(size_t)(an - 1 - i) * an + (an - 1 - j)])
                        return fail(nullptr, PSC_E_ARG,
                                    "every aperture must be finite and even (A[i][j] = A[n-1-i][n-1-j])");
                    sum += v;
                }
            if (!(sum > 0.0)) return fail(nullptr, PSC_E_ARG, "every aperture's sum must be positive");
            std::vector<double> cells;
            for (int i = 0; i < an; ++i)
                for (int j = 0; j < an; ++j) {
                    const double v = A[(size_t)i * an + j];
                    if (v == 0.0) continue;
                    cells.push_back((i - 0.5 * (an - 1)) / an);
                    cells.push_back((j - 0.5 * (an - 1)) / an);
                    cells.push_back(v / sum);
                }
            ap_cells.push_back(std::move(cells));
        }
    }
    if (c.illum == 1 && !(c.gauss_sigma_ld > 0))
        return fail(nullptr, PSC_E_ARG, "gauss_sigma_ld must be positive in Gaussian mode");
    if (!isfinite(c.squint_frac)) return fail(nullptr, PSC_E_ARG, "squint_frac must be finite");
    if (c.support == 32 && win_lds_bytes(32, kGrad, m, c.oversample) > win_lds_budget(32))
        return fail(nullptr, PSC_E_UNSUPPORTED, "support 32: the window form exceeds the LDS of one compute unit");
    if (hipSetDevice(c.device) != hipSuccess) return fail(nullptr, PSC_E_ARG, "invalid device");

    double* scratch_dev = nullptr;
    if (scratch_address(c.device, &scratch_dev) != hipSuccess)
        return fail(nullptr, PSC_E_HIP, "hipGetSymbolAddress of the allocation-free scratch failed");

    psc_ctx* ctx = new psc_ctx();
    ctx->cfg = c;
    ctx->cfg.aperture = nullptr;  // read here only; the cells are kept instead
    ctx->ap_cells = std::move(ap_cells);
    ctx->cfg.image_samples = m;
    ctx->cfg.taper_width = tw;
    ctx->cfg.taper_beta = tb;
    ctx->n = c.grid_n;
    ctx->s = c.support;
    ctx->o = c.oversample;
    ctx->m = m;
    ctx->fov = (double)c.grid_n * c.cell_rad;
    ctx->h = ctx->fov / c.support;
    ctx->snap = (double)c.oversample * ctx->fov;

    Taper taper(tw, tb);
    std::vector<double> tp(ctx->n);
    std::vector<float> ti(m);
    for (int i = 0; i < ctx->n; ++i) tp[i] = taper((double)(i - ctx->n / 2) / ctx->n);
    for (int i = 0; i < m; ++i) ti[i] = (float)taper((double)(i - m / 2) / c.support);
    const int so = c.support * c.oversample;
    std::vector<float2> twh(so);
    for (int t = 0; t < so; ++t) {
        double sv, cv;
        if ((4 * t) % so == 0) {  // exact on the axes
            const int q = (4 * t) / so;
            cv = (q == 0) ? 1 : (q == 2) ? -1 : 0;
            sv = (q == 1) ? 1 : (q == 3) ? -1 : 0;
        } else {
            cv = cos(2.0 * kPi * t / so);
            sv = sin(2.0 * kPi * t / so);
        }
        twh[t] = make_float2((float)cv, (float)sv);
    }
    hipError_t e = dmalloc(&ctx->grid, (size_t)(ctx->n + ctx->s) * (ctx->n + ctx->s));
    if (e == hipSuccess) e = dmalloc(&ctx->taper_pix, ctx->n);
    if (e == hipSuccess) e = dmalloc(&ctx->taper_img, m);
    if (e == hipSuccess) e = dmalloc(&ctx->tw, so);
    if (e == hipSuccess) e = hipMemcpy(ctx->taper_pix, tp.data(), sizeof(double) * ctx->n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->taper_img, ti.data(), sizeof(float) * m, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->tw, twh.data(), sizeof(float2) * so, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        std::string msg = std::string("context allocation: ") + hipGetErrorString(e);
        psc_destroy(ctx);
        return fail(nullptr, e == hipErrorOutOfMemory ? PSC_E_OOM : PSC_E_HIP, msg);
    }
    *out = ctx;
    return PSC_OK;
}

PSC_API psc_status psc_destroy(psc_ctx* ctx)
{
    if (!ctx) return PSC_OK;
    (void)hipSetDevice(ctx->cfg.device);
    dfree(ctx->grid);
    dfree(ctx->image);
    dfree(ctx->taper_pix);
    dfree(ctx->taper_img);
    dfree(ctx->tw);
    dfree(ctx->rgrid);
    dfree(ctx->fa);
    dfree(ctx->fb);
    delete ctx;
    return PSC_OK;
}

// V^{M0} = F[I/c] (w = 0: the model grid) or, for a w-plane, F[I e^{2 pi i
// w (n-1)} / c], float64 FFT, stored padded as complex64 (N+S)^2 at `out`.
static hipError_t model_transform(psc_ctx* ctx, const double* image, bool wplane, double w, float2* out,
                                  double2* a, double2* b, hipStream_t st)
{
    const int n = ctx->n;
    int log2n = 0;
    while ((1 << log2n) < n) ++log2n;
    hipError_t e = wplane ? launch_wplane_image(image, ctx->taper_pix, a, n, ctx->cfg.cell_rad, w, st)
                          : launch_taper_image(image, ctx->taper_pix, a, n, st);
    if (e == hipSuccess) e = launch_fft_rows(a, n, log2n, st);
    if (e == hipSuccess) e = launch_transpose(a, b, n, st);
    if (e == hipSuccess) e = launch_fft_rows(b, n, log2n, st);
    if (e == hipSuccess) e = launch_transpose(b, a, n, st);
    if (e == hipSuccess) e = launch_finish_grid(a, out, n, ctx->s, st);
    return e;
}

// The w-planes of one observation from the kept model image.
static hipError_t build_wplanes(psc_ctx* ctx, psc_obs* obs, hipStream_t st)
{
    const size_t n2 = (size_t)ctx->n * ctx->n, p2 = (size_t)(ctx->n + ctx->s) * (ctx->n + ctx->s);
    double2 *a = nullptr, *b = nullptr;
    hipError_t e = dmalloc(&a, n2);
    if (e == hipSuccess) e = dmalloc(&b, n2);
    for (int k = 0; k < obs->w_nk && e == hipSuccess; ++k)
        e = model_transform(ctx, ctx->image, true, (double)(obs->w_k0 + k) * obs->w_dw, obs->wplanes + k * p2, a,
                            b, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(a);
    dfree(b);
    return e;
}

PSC_API psc_status psc_set_model(psc_ctx* ctx, const double* image_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    if (!image_dev) return fail(ctx, PSC_E_ARG, "null image");
    ctx->err.clear();
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t st = (hipStream_t)stream;
    const size_t n2 = (size_t)ctx->n * ctx->n;
    double2 *a = nullptr, *b = nullptr;
    hipError_t e = ctx->image ? hipSuccess : dmalloc(&ctx->image, n2);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->image, image_dev, sizeof(double) * n2, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = dmalloc(&a, n2);
    if (e == hipSuccess) e = dmalloc(&b, n2);
    if (e == hipSuccess) e = model_transform(ctx, ctx->image, false, 0.0, ctx->grid, a, b, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(a);
    dfree(b);
    // observations with w-stacking follow the model
    for (psc_obs* obs : ctx->stacked)
        if (e == hipSuccess) e = build_wplanes(ctx, obs, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "psc_set_model");
    ctx->model_set = true;
    return PSC_OK;
}

PSC_API psc_status psc_obs_destroy(psc_obs* obs)
{
    if (!obs) return PSC_OK;
    if (obs->ctx) (void)hipSetDevice(obs->ctx->cfg.device);
    if (obs->graph) (void)hipGraphExecDestroy(obs->graph);
    if (obs->cap_stream) (void)hipStreamDestroy(obs->cap_stream);
    dfree(obs->items);
    dfree(obs->groups);
    if (obs->ctx) {
        auto& v = obs->ctx->stacked;
        v.erase(std::remove(v.begin(), v.end(), obs), v.end());
    }
    dfree(obs->wplanes);
    dfree(obs->defocus);
    dfree(obs->mtab);
    dfree(obs->vis);
    dfree(obs->wvis);
    dfree(obs->wf);
    dfree(obs->ant_ptr);
    dfree(obs->ant_ent);
    dfree(obs->freq);
    dfree(obs->par_angle);
    dfree(obs->w_m);
    dfree(obs->airy);
    dfree(obs->ap_tab);
    dfree(obs->ap_ant);
    dfree(obs->beams);
    dfree(obs->scale);
    dfree(obs->zero_pa);
    dfree(obs->partials);
    dfree(obs->acc);
    dfree(obs->max_step);
    dfree(obs->done);
    dfree(obs->iters);
    dfree(obs->ig_ord);
    dfree(obs->ig_vm);
    delete obs;
    return PSC_OK;
}

// Pattern tables of the context's measured apertures, [n][ap_n][ap_n]
// (launch_aperture_table per aperture; synchronous).
static hipError_t aperture_tables(const psc_ctx* ctx, int ap_n, int ap_half, double ap_step, float4** out)
{
    const size_t n2 = (size_t)ap_n * ap_n;
    float4* tab = nullptr;
    hipError_t e = dmalloc(&tab, n2 * ctx->ap_cells.size());
    for (size_t k = 0; k < ctx->ap_cells.size() && e == hipSuccess; ++k) {
        const std::vector<double>& c = ctx->ap_cells[k];
        double* cells = nullptr;
        e = dmalloc(&cells, c.size());
        if (e == hipSuccess) e = hipMemcpy(cells, c.data(), sizeof(double) * c.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_aperture_table(cells, (int)(c.size() / 3), tab + k * n2, ap_n, ap_half, ap_step, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        dfree(cells);
    }
    if (e != hipSuccess) {
        dfree(tab);
        return e;
    }
    *out = tab;
    return hipSuccess;
}

static psc_status obs_create_impl(psc_ctx* ctx, const psc_obs_desc* d, psc_obs** out)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!d || !out) return fail(ctx, PSC_E_ARG, "null descriptor or output pointer");
    *out = nullptr;
    if (d->n_ant < 2 || d->n_chan < 1 || d->n_pol < 1 || d->n_pol > 2 || d->n_int < 1 || d->n_row < 0)
        return fail(ctx, PSC_E_ARG, "bad sizes (need n_ant >= 2, n_chan >= 1, n_pol in {1,2}, n_int >= 1)");
    if (d->n_ant > 4096) return fail(ctx, PSC_E_UNSUPPORTED, "n_ant above 4096");
    if ((d->n_row > 0 && (!d->ant1 || !d->ant2 || !d->uv_m)) || !d->int_row_ptr || !d->freq_hz)
        return fail(ctx, PSC_E_ARG, "null array in descriptor");
    if ((double)d->n_row * d->n_chan >= 4294967295.0)
        return fail(ctx, PSC_E_UNSUPPORTED, "n_row * n_chan must stay below 2^32");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));

    const int n_ant = d->n_ant, n_chan = d->n_chan, n_int = d->n_int;
    const int64_t n_row = d->n_row;
    std::vector<int64_t> rp(n_int + 1);
    std::vector<int32_t> a1(n_row), a2(n_row);
    std::vector<double> uv(2 * n_row), fr(n_chan);
    PSC_HIP(ctx, hipMemcpy(rp.data(), d->int_row_ptr, sizeof(int64_t) * (n_int + 1), hipMemcpyDeviceToHost));
    if (n_row > 0) {
        PSC_HIP(ctx, hipMemcpy(a1.data(), d->ant1, sizeof(int32_t) * n_row, hipMemcpyDeviceToHost));
        PSC_HIP(ctx, hipMemcpy(a2.data(), d->ant2, sizeof(int32_t) * n_row, hipMemcpyDeviceToHost));
        PSC_HIP(ctx, hipMemcpy(uv.data(), d->uv_m, sizeof(double) * 2 * n_row, hipMemcpyDeviceToHost));
    }
    PSC_HIP(ctx, hipMemcpy(fr.data(), d->freq_hz, sizeof(double) * n_chan, hipMemcpyDeviceToHost));
    if (rp[0] != 0 || rp[n_int] != n_row) return fail(ctx, PSC_E_ARG, "int_row_ptr must run from 0 to n_row");
    for (int s = 0; s < n_int; ++s)
        if (rp[s + 1] < rp[s]) return fail(ctx, PSC_E_ARG, "int_row_ptr must be non-decreasing");
    for (int64_t r = 0; r < n_row; ++r)
        if (a1[r] < 0 || a2[r] >= n_ant || a1[r] >= a2[r])
            return fail(ctx, PSC_E_ARG, "antenna indices must satisfy 0 <= ant1 < ant2 < n_ant");
    double fmax = 0;
    for (int c = 0; c < n_chan; ++c) {
        if (!(fr[c] > 0) || !isfinite(fr[c])) return fail(ctx, PSC_E_ARG, "frequencies must be positive");
        fmax = std::max(fmax, fr[c]);
    }
    for (int64_t i = 0; i < 2 * n_row; ++i)
        if (!isfinite(uv[i])) return fail(ctx, PSC_E_ARG, "uv_m must be finite");
    std::vector<int32_t> apa;
    if (d->ant_aperture) {
        if (ctx->cfg.illum != 2) return fail(ctx, PSC_E_ARG, "ant_aperture needs the measured-aperture mode (illum 2)");
        apa.resize(n_ant);
        PSC_HIP(ctx, hipMemcpy(apa.data(), d->ant_aperture, sizeof(int32_t) * n_ant, hipMemcpyDeviceToHost));
        for (int a = 0; a < n_ant; ++a)
            if (apa[a] < 0 || apa[a] >= (int)ctx->ap_cells.size())
                return fail(ctx, PSC_E_ARG, "ant_aperture: every index must be in [0, aperture_count)");
    }
    std::vector<double> pa;
    if (d->par_angle && n_row > 0) {
        pa.resize(n_row);
        PSC_HIP(ctx, hipMemcpy(pa.data(), d->par_angle, sizeof(double) * n_row, hipMemcpyDeviceToHost));
        for (int64_t r = 0; r < n_row; ++r)
            if (!isfinite(pa[r])) return fail(ctx, PSC_E_ARG, "par_angle must be finite");
    }
    std::vector<double> wv;
    bool w_stack = false;
    if (d->w_m && n_row > 0) {
        wv.resize(n_row);
        PSC_HIP(ctx, hipMemcpy(wv.data(), d->w_m, sizeof(double) * n_row, hipMemcpyDeviceToHost));
        double w_max = 0.0;
        for (int64_t r = 0; r < n_row; ++r) {
            if (!isfinite(wv[r])) return fail(ctx, PSC_E_ARG, "w_m must be finite");
            w_max = std::max(w_max, fabs(wv[r]));
        }
        // the w phase widens each kernel by about |w| l / lambda wavelengths
        // at sky offset l; over the beam (l ~ lambda / D) that is |w| FoV / D
        // uv cells, which must stay within what the support leaves.  Beyond
        // that the observation is w-stacked (see below).
        w_stack = w_max * ctx->fov / ctx->cfg.dish_diam_m > kMaxWCells;
    }
    // the kernel support must hold both apertures plus the taper
    const double lam_min = kCLight / fmax;
    const double need = 2.0 * ctx->cfg.dish_diam_m * ctx->fov / lam_min + ctx->cfg.taper_width;
    if (ctx->cfg.illum != 1 && need > ctx->s)
        return fail(ctx, PSC_E_ARG, "support too small for the dish at the highest frequency "
                                    "(need 2 D FoV / lambda + taper_width <= support)");

    const int S = ctx->s, O = ctx->o, N = ctx->n;
    const int n_bl = n_ant * (n_ant - 1) / 2;
    auto bl_of = [n_ant](int i, int j) { return i * (2 * n_ant - i - 1) / 2 + (j - i - 1); };

    // The plan of a run of intervals [s0, s1): its items, groups and samples,
    // with indices local to the run (made global when the runs are joined).
    struct PlanPart {
        std::vector<Item> items;
        std::vector<Group> groups;
        std::vector<VisEnt> vis, wvis;
        std::vector<uint8_t> wf;
        std::vector<int32_t> n_items;  // per interval of the run
        bool failed = false;
    };
    auto plan_run = [&](int s0, int s1, PlanPart& pp) {
        std::vector<Item>& items = pp.items;
        std::vector<Group>& groups = pp.groups;
        std::vector<VisEnt>& vis = pp.vis;
        std::vector<VisEnt>& wvis = pp.wvis;
        std::vector<uint8_t>& wf = pp.wf;
        const size_t n_samp = (size_t)(rp[s1] - rp[s0]) * n_chan;
        vis.reserve(n_samp);
        wvis.reserve(n_samp);
        wf.reserve(n_samp);
        pp.n_items.assign(s1 - s0, 0);
        std::vector<int64_t> bl_count(n_bl + 1), bl_start(n_bl + 1);
        std::vector<int64_t> bl_rows;
        std::vector<int32_t> fcount(O * O), fpos(O * O);
        std::vector<int32_t> fq(0);
        std::vector<uint32_t> kq(0);
        for (int s = s0; s < s1; ++s) {
            const int64_t r0 = rp[s], r1 = rp[s + 1];
            const size_t items_before = items.size();
            std::fill(bl_count.begin(), bl_count.end(), 0);
            for (int64_t r = r0; r < r1; ++r) bl_count[bl_of(a1[r], a2[r]) + 1]++;
            bl_start[0] = 0;
            for (int b = 0; b < n_bl; ++b) bl_start[b + 1] = bl_start[b] + bl_count[b + 1];
            bl_rows.assign(r1 - r0, 0);
            {
                std::vector<int64_t> pos(bl_start.begin(), bl_start.end());
                for (int64_t r = r0; r < r1; ++r) bl_rows[pos[bl_of(a1[r], a2[r])]++] = r;
            }
            for (int b = 0; b < n_bl; ++b) {
                const int64_t nb = bl_start[b + 1] - bl_start[b];
                if (nb == 0) continue;
                const int64_t* rows = bl_rows.data() + bl_start[b];
                fq.resize(nb);
                kq.resize(nb);
                for (int c = 0; c < n_chan; ++c) {
                    Item it;
                    it.interval = s;
                    it.ai = a1[rows[0]];
                    it.aj = a2[rows[0]];
                    it.chan = c;
                    it.grp_begin = (int32_t)groups.size();
                    std::fill(fcount.begin(), fcount.end(), 0);
                    for (int64_t k = 0; k < nb; ++k) {
                        const int64_t r = rows[k];
                        // uv in wavelengths, rounded to the 1/O lattice
                        const double uu = uv[2 * r] * fr[c] / kCLight;
                        const double vv = uv[2 * r + 1] * fr[c] / kCLight;
                        const long long ql = llround(uu * ctx->snap);
                        const long long qm = llround(vv * ctx->snap);
                        const int bl_l = floor_div(ql, O), bl_m = floor_div(qm, O);
                        const int f = (int)(ql - (long long)bl_l * O) * O + (int)(qm - (long long)bl_m * O);
                        int kl = (bl_l - S / 2 + 1) % N;
                        int km = (bl_m - S / 2 + 1) % N;
                        kl += kl < 0 ? N : 0;
                        km += km < 0 ? N : 0;
                        fq[k] = f;
                        kq[k] = ((uint32_t)kl << 16) | (uint32_t)km;
                        fcount[f]++;
                    }
                    // one group per pair of opposite offsets {f, -f}
                    const size_t base = vis.size();
                    int32_t acc = 0;
                    for (int f = 0; f < O * O; ++f) {
                        const int fl = f / O, fm = f % O;
                        const int pf = ((O - fl) % O) * O + (O - fm) % O;
                        if (pf < f) continue;  // handled with its partner
                        int prim = f, sec = (pf != f) ? pf : -1;
                        if (fcount[prim] == 0) {
                            if (sec < 0 || fcount[sec] == 0) continue;
                            prim = sec;
                            sec = -1;
                        }
                        Group g;
                        g.f = prim;
                        g.vis_begin = (uint32_t)(base + acc);
                        g.n_vis = fcount[prim];
                        g.n_vis2 = (sec >= 0) ? fcount[sec] : 0;
                        fpos[prim] = acc;
                        acc += g.n_vis;
                        if (g.n_vis2 > 0) {
                            fpos[sec] = acc;
                            acc += g.n_vis2;
                        }
                        groups.push_back(g);
                    }
                    vis.resize(base + nb);
                    for (int64_t k = 0; k < nb; ++k) {
                        VisEnt ve;
                        ve.vidx = (uint32_t)(rows[k] * n_chan + c);
                        ve.klo = kq[k];
                        vis[base + fpos[fq[k]]++] = ve;
                        wvis.push_back(ve);
                        wf.push_back((uint8_t)(((fq[k] / O) << 4) | (fq[k] % O)));
                    }
                    it.vis_begin = (uint32_t)base;
                    it.n_vis = (int32_t)nb;
                    it.grp_end = (int32_t)groups.size();
                    // largest groups first: the block's wavefronts claim groups in
                    // this order, so the long ones start early and the item's
                    // wavefronts finish together
                    std::stable_sort(groups.begin() + it.grp_begin, groups.end(),
                                     [](const Group& x, const Group& y) {
                                         const int cx = (x.n_vis + 7) / 8 + (x.n_vis2 + 7) / 8;
                                         const int cy = (y.n_vis + 7) / 8 + (y.n_vis2 + 7) / 8;
                                         return cx > cy;
                                     });
                    items.push_back(it);
                }
            }
            pp.n_items[s - s0] = (int32_t)(items.size() - items_before);
        }
    };

    // Intervals are planned independently: runs of them on host threads,
    // split by row count, then joined in interval order (the result does not
    // depend on the split).
    const int n_thr = (int)std::max<int64_t>(1, std::min<int64_t>(
        {(int64_t)std::max(1u, std::thread::hardware_concurrency()), 16, (int64_t)n_int,
         1 + n_row * n_chan / 200000}));
    std::vector<int> cut(n_thr + 1, n_int);
    cut[0] = 0;
    for (int t = 1; t < n_thr; ++t) {
        const int64_t target = n_row * t / n_thr;
        cut[t] = std::max(cut[t - 1], (int)(std::upper_bound(rp.begin(), rp.end(), target) - rp.begin()) - 1);
        cut[t] = std::min(cut[t], n_int);
    }
    std::vector<PlanPart> parts(n_thr);
    {
        std::vector<std::thread> pool;
        for (int t = 1; t < n_thr; ++t)
            pool.emplace_back([&, t] {
                try {
                    plan_run(cut[t], cut[t + 1], parts[t]);
                } catch (...) {
                    parts[t].failed = true;
                }
            });
        try {
            plan_run(cut[0], cut[1], parts[0]);
        } catch (...) {
            parts[0].failed = true;
        }
        for (auto& th : pool) th.join();
    }
    size_t tot_items = 0, tot_groups = 0, tot_vis = 0;
    for (const PlanPart& pp : parts) {
        if (pp.failed) return fail(ctx, PSC_E_OOM, "host memory allocation failed while planning");
        tot_items += pp.items.size();
        tot_groups += pp.groups.size();
        tot_vis += pp.vis.size();
    }
    if (tot_groups > 2147483647u || tot_vis > 4294967295u || tot_items > 2000000000u)
        return fail(ctx, PSC_E_UNSUPPORTED, "too many samples for one observation");
    std::vector<Item> items;
    std::vector<Group> groups;
    std::vector<VisEnt> vis, wvis;
    std::vector<uint8_t> wf;
    items.reserve(tot_items);
    groups.reserve(tot_groups);
    vis.reserve(tot_vis);
    wvis.reserve(tot_vis);
    wf.reserve(tot_vis);
    std::vector<int32_t> item_ptr(n_int + 1, 0);
    for (int t = 0; t < n_thr; ++t) {
        PlanPart& pp = parts[t];
        const uint32_t g_off = (uint32_t)groups.size(), v_off = (uint32_t)vis.size();
        for (Item it : pp.items) {
            it.grp_begin += (int32_t)g_off;
            it.grp_end += (int32_t)g_off;
            it.vis_begin += v_off;
            items.push_back(it);
        }
        for (Group g : pp.groups) {
            g.vis_begin += v_off;
            groups.push_back(g);
        }
        vis.insert(vis.end(), pp.vis.begin(), pp.vis.end());
        wvis.insert(wvis.end(), pp.wvis.begin(), pp.wvis.end());
        wf.insert(wf.end(), pp.wf.begin(), pp.wf.end());
        for (int s = cut[t]; s < cut[t + 1]; ++s) item_ptr[s + 1] = item_ptr[s] + pp.n_items[s - cut[t]];
        std::vector<Item>().swap(pp.items);  // release the run's memory as it is joined
        std::vector<Group>().swap(pp.groups);
        std::vector<VisEnt>().swap(pp.vis);
        std::vector<VisEnt>().swap(pp.wvis);
        std::vector<uint8_t>().swap(pp.wf);
    }

    // per (interval, antenna) list of (item, end) in item order
    std::vector<uint32_t> ant_ptr((size_t)n_int * n_ant + 1, 0), ant_ent(2 * items.size());
    for (const Item& it : items) {
        ant_ptr[(size_t)it.interval * n_ant + it.ai + 1]++;
        ant_ptr[(size_t)it.interval * n_ant + it.aj + 1]++;
    }
    for (size_t k = 0; k < (size_t)n_int * n_ant; ++k) ant_ptr[k + 1] += ant_ptr[k];
    {
        std::vector<uint32_t> pos(ant_ptr.begin(), ant_ptr.end() - 1);
        for (size_t i = 0; i < items.size(); ++i) {
            const Item& it = items[i];
            ant_ent[pos[(size_t)it.interval * n_ant + it.ai]++] = (uint32_t)(2 * i);
            ant_ent[pos[(size_t)it.interval * n_ant + it.aj]++] = (uint32_t)(2 * i + 1);
        }
    }

    // Airy table range: largest x = pi D nu |l - p| over the image samples,
    // with room for offsets and squint up to a quarter of the field of view.
    const double rho_max = sqrt(2.0) * (ctx->m / 2) * ctx->h + 0.25 * ctx->fov;
    const double x_max = kPi * ctx->cfg.dish_diam_m / lam_min * rho_max;
    // cubic Hermite with exact slopes: error below 5e-9 at this spacing
    const double dx = 1.0 / 16.0;
    const int n_tab = (int)ceil(x_max / dx) + 3;
    // measured aperture: its pattern over the same range, in lambda/D units,
    // at 32 nodes per lambda/D (the window form stores its products per item
    // in the sky frame and evaluates them per sample in the mount frame)
    const bool ap = ctx->cfg.illum == 2;
    const double ap_step = 1.0 / 32.0;
    const int ap_half = ap ? (int)ceil(rho_max * ctx->cfg.dish_diam_m / lam_min / ap_step) + 2 : 0;
    const int ap_n = 2 * ap_half + 1;

    psc_obs* obs = new psc_obs();
    obs->ctx = ctx;
    obs->fmax = fmax;
    obs->degrid = (S == 16 && pa.empty() && wv.empty() && !ap) ? PSC_DEGRID_VALU : PSC_DEGRID_WINDOW;
    obs->n_ant = n_ant;
    obs->n_chan = n_chan;
    obs->n_pol = d->n_pol;
    obs->n_int = n_int;
    obs->n_row = n_row;
    obs->int_item_ptr = item_ptr;
    obs->n_items = (int64_t)items.size();
    obs->n_groups = (int64_t)groups.size();
    obs->n_vis = (int64_t)vis.size();
    obs->n_tab = n_tab;
    obs->inv_dx = 1.0 / dx;
    obs->tab_x1 = x_max;
    obs->ap_r1 = rho_max * ctx->cfg.dish_diam_m / lam_min;
    // items of few samples on average: window-form blocks of one wavefront
    // below 16 samples per item, of two below 128 (measured on the batched
    // array: at 4.6 samples per item 36.3 ms per gradient with one, 42.8
    // with two, 60.0 with four wavefronts; at 65, 68.5 with two against 69
    // with one and 72.3 with four; at 360 two were 6% slower than four)
    const double per_item = items.empty() ? 0.0 : (double)vis.size() / (double)items.size();
    obs->win_waves = S != 16 || items.empty() ? 0 : per_item < 16.0 ? 1 : per_item < 128.0 ? 2 : 0;
    hipError_t e = dmalloc(&obs->items, items.size());
    if (e == hipSuccess) e = dmalloc(&obs->groups, groups.size());
    if (e == hipSuccess) e = dmalloc(&obs->vis, vis.size());
    if (e == hipSuccess) e = dmalloc(&obs->wvis, wvis.size());
    if (e == hipSuccess) e = dmalloc(&obs->wf, wf.size());
    if (e == hipSuccess) e = dmalloc(&obs->ant_ptr, ant_ptr.size());
    if (e == hipSuccess) e = dmalloc(&obs->ant_ent, ant_ent.size());
    if (e == hipSuccess) e = dmalloc(&obs->freq, n_chan);
    if (e == hipSuccess && !pa.empty()) e = dmalloc(&obs->par_angle, pa.size());
    if (e == hipSuccess && !wv.empty()) e = dmalloc(&obs->w_m, wv.size());
    if (e == hipSuccess) e = dmalloc(&obs->airy, n_tab);
    // sky-frame radial beams: room for every antenna's pattern at the image
    // samples per interval, polarisation and channel, which the window form
    // fills before each degrid (within kBeamTabIntervalBytes per interval
    // and kBeamTabBytes in all; beyond that each item evaluates its
    // antennas' patterns itself)
    {
        const size_t per_int = (size_t)d->n_pol * n_chan * n_ant * (size_t)ctx->m * ctx->m;
        const size_t nb = (size_t)n_int * per_int;
        if (e == hipSuccess && pa.empty() && !ap && nb > 0 && per_int * sizeof(float2) <= kBeamTabIntervalBytes &&
            nb * sizeof(float2) <= kBeamTabBytes)
            e = dmalloc(&obs->beams, nb);
    }
    if (e == hipSuccess) e = dmalloc(&obs->partials, items.size() * d->n_pol * 12);
    if (e == hipSuccess) e = dmalloc(&obs->acc, (size_t)n_int * d->n_pol * n_ant * 6);
    if (e == hipSuccess) e = dmalloc(&obs->max_step, n_int);
    if (e == hipSuccess) e = dmalloc(&obs->done, n_int);
    if (e == hipSuccess) e = dmalloc(&obs->iters, n_int);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(obs->items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !groups.empty())
        e = hipMemcpy(obs->groups, groups.data(), sizeof(Group) * groups.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !vis.empty())
        e = hipMemcpy(obs->vis, vis.data(), sizeof(VisEnt) * vis.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !wvis.empty())
        e = hipMemcpy(obs->wvis, wvis.data(), sizeof(VisEnt) * wvis.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !wf.empty())
        e = hipMemcpy(obs->wf, wf.data(), wf.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(obs->ant_ptr, ant_ptr.data(), sizeof(uint32_t) * ant_ptr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ant_ent.empty())
        e = hipMemcpy(obs->ant_ent, ant_ent.data(), sizeof(uint32_t) * ant_ent.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(obs->freq, fr.data(), sizeof(double) * n_chan, hipMemcpyHostToDevice);
    if (e == hipSuccess && !pa.empty())
        e = hipMemcpy(obs->par_angle, pa.data(), sizeof(double) * pa.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !wv.empty())
        e = hipMemcpy(obs->w_m, wv.data(), sizeof(double) * wv.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_airy_table(obs->airy, n_tab, dx, nullptr);
    if (ap) {
        obs->ap_n = ap_n;
        obs->ap_c = ap_half;
        obs->ap_step = ap_step;
        if (e == hipSuccess) e = aperture_tables(ctx, ap_n, ap_half, ap_step, &obs->ap_tab);
        if (e == hipSuccess && !apa.empty()) e = dmalloc(&obs->ap_ant, apa.size());
        if (e == hipSuccess && !apa.empty())
            e = hipMemcpy(obs->ap_ant, apa.data(), sizeof(int32_t) * apa.size(), hipMemcpyHostToDevice);
        // the image gradient's scatter builds each sample's kernel: in the
        // sky frame at angle zero
        if (e == hipSuccess && pa.empty()) {
            const size_t nr = n_row > 0 ? (size_t)n_row : 1;
            e = dmalloc(&obs->zero_pa, nr);
            if (e == hipSuccess) e = hipMemset(obs->zero_pa, 0, sizeof(double) * nr);
        }
    }
    if (w_stack) {
        // w-stacking (Sec. 5.1: non-coplanar arrays, beyond what one kernel
        // holds): the model transformed again for planes w_k = k dw
        // wavelengths; each sample reads the plane nearest its w and carries
        // the residual w - w_k in its kernel.  dw keeps that residual's
        // widening at most kWStackCells cells at the lowest frequency.
        double fmin = fr[0];
        for (int c = 1; c < n_chan; ++c) fmin = std::min(fmin, fr[c]);
        const double dw = 2.0 * kWStackCells * ctx->cfg.dish_diam_m / (ctx->fov * (kCLight / fmin));
        const double w_lo = *std::min_element(wv.begin(), wv.end());
        const double w_hi = *std::max_element(wv.begin(), wv.end());
        int k_lo = 0, k_hi = 0;
        bool first = true;
        for (int c = 0; c < n_chan; ++c) {
            const double w_per_m = fr[c] / kCLight;  // as the kernels form it
            for (double w : {w_lo, w_hi}) {
                const int k = (int)rint((w * w_per_m) / dw);
                k_lo = first ? k : std::min(k_lo, k);
                k_hi = first ? k : std::max(k_hi, k);
                first = false;
            }
        }
        const size_t p2 = (size_t)(N + S) * (N + S);
        const size_t bytes = (size_t)(k_hi - k_lo + 1) * p2 * sizeof(float2);
        if (bytes > (size_t)2147483647) {
            psc_obs_destroy(obs);
            return fail(ctx, PSC_E_UNSUPPORTED,
                        "w-term: the w-stacked model grids would exceed 2 GiB (w range too wide for the grid)");
        }
        obs->w_k0 = k_lo;
        obs->w_nk = k_hi - k_lo + 1;
        obs->w_dw = dw;
        if (e == hipSuccess) e = dmalloc(&obs->wplanes, (size_t)obs->w_nk * p2);
        if (e == hipSuccess && ctx->model_set) e = build_wplanes(ctx, obs, nullptr);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&obs->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        psc_status st = e == hipErrorOutOfMemory ? PSC_E_OOM : PSC_E_HIP;
        std::string msg = std::string("psc_obs_create: ") + hipGetErrorString(e);
        psc_obs_destroy(obs);
        return fail(ctx, st, msg);
    }
    if (obs->w_nk > 0) ctx->stacked.push_back(obs);
    *out = obs;
    return PSC_OK;
}

PSC_API psc_status psc_obs_launch_info(const psc_obs* obs, psc_launch_info* out)
{
    if (!obs) return fail(nullptr, PSC_E_ARG, "null observation");
    if (!out) return fail(obs->ctx, PSC_E_ARG, "null output");
    const psc_ctx* ctx = obs->ctx;
    const int frame = obs->ap_tab ? (obs->par_angle ? kFrameAperture : kFrameSkyAperture)
                                  : (obs->par_angle ? kFrameMount : kFrameSky);
    out->degrid = obs->degrid;
    out->window_waves = win_block_waves(ctx->s, kGrad, frame, ctx->m, ctx->o, obs->n_tab, obs->win_waves);
    out->samples_per_item = obs->n_items > 0 ? (double)obs->n_vis / (double)obs->n_items : 0.0;
    out->plan_ms = obs->plan_ms;
    out->w_planes = obs->w_nk;
    out->tab_nodes = obs->n_tab;
    out->capture_ms = obs->capture_ms;
    out->pattern_tables = (obs->beams != nullptr && ctx->s == 16 && !obs->par_angle && !obs->ap_tab) ? 1 : 0;
    // the whole-batch launch's blocks (the window form's rule on every item,
    // complex patterns while a defocus is set; the table form takes one item
    // per block)
    out->items_per_block = obs->degrid == PSC_DEGRID_WINDOW
                               ? win_items_per_block(ctx->s, obs->defocus ? kFrameSkyComplex : frame, obs->n_items)
                               : 1;
    return PSC_OK;
}

PSC_API psc_status psc_obs_info(const psc_obs* obs, int64_t* n_items, int64_t* n_groups, int64_t* n_vis)
{
    if (!obs) return fail(nullptr, PSC_E_ARG, "null observation");
    if (n_items) *n_items = obs->n_items;
    if (n_groups) *n_groups = obs->n_groups;
    if (n_vis) *n_vis = obs->n_vis;
    return PSC_OK;
}

}  // extern "C"

namespace {

ItemArgs item_args(psc_ctx* ctx, psc_obs* obs, const double* offsets, int item_begin, int n_items,
                   const int32_t* done)
{
    ItemArgs a{};
    a.items = obs->items;
    a.groups = obs->groups;
    a.vis = obs->vis;
    a.wvis = obs->wvis;
    a.wf = obs->wf;
    a.item_begin = item_begin;
    a.n_items = n_items;
    a.n_ant = obs->n_ant;
    a.n_pol = obs->n_pol;
    a.n_chan = obs->n_chan;
    a.par_angle = obs->par_angle;
    a.w_m = obs->w_m;
    a.wgrid = obs->wplanes;
    a.w_dw = obs->w_dw;
    a.w_k0 = obs->w_k0;
    a.w_nk = obs->w_nk;
    a.offsets = offsets;
    a.freq = obs->freq;
    a.grid = ctx->grid;
    a.grid_n = ctx->n;
    a.oversample = ctx->o;
    a.m = ctx->m;
    a.h = ctx->h;
    a.taper_img = ctx->taper_img;
    a.tw = ctx->tw;
    a.dish = ctx->cfg.dish_diam_m;
    a.illum = ctx->cfg.illum;
    a.gauss_sigma_ld = ctx->cfg.gauss_sigma_ld;
    a.squint_frac = ctx->cfg.squint_frac;
    a.airy = obs->airy;
    a.n_tab = obs->n_tab;
    a.inv_dx = (float)obs->inv_dx;
    a.ap_tab = obs->ap_tab;
    a.ap_ant = obs->ap_ant;
    a.ap_n = obs->ap_n;
    a.ap_c = (float)obs->ap_c;
    a.ap_inv_step = obs->ap_step > 0 ? (float)(1.0 / obs->ap_step) : 0.f;
    a.scale = obs->scale;
    a.defocus = obs->defocus;
    a.mtab = obs->mtab;
    a.n_mom = kMoments;
    a.win_waves = obs->win_waves;
    a.partials = obs->partials;
    a.done = done;
    // the intervals the items span: the pattern tables filled for them
    a.beams = obs->beams;
    {
        const int32_t* p = obs->int_item_ptr.data();
        a.beam_int0 = (int)(std::upper_bound(p, p + obs->n_int + 1, item_begin) - p) - 1;
        a.beam_int1 = (int)(std::lower_bound(p, p + obs->n_int + 1, item_begin + n_items) - p);
        a.beam_int0 = std::max(0, std::min(a.beam_int0, obs->n_int));
        a.beam_int1 = std::max(a.beam_int0, std::min(a.beam_int1, obs->n_int));
    }
    a.use_mfma = obs->degrid == PSC_DEGRID_MFMA ? 1 : 0;
    return a;
}

ReduceArgs reduce_args(psc_obs* obs, int int_begin, int int_end, double* out, const int32_t* done)
{
    ReduceArgs r{};
    r.ant_ptr = obs->ant_ptr;
    r.ant_ent = obs->ant_ent;
    r.items = obs->items;
    r.partials = obs->partials;
    r.n_int = obs->n_int;
    r.n_pol = obs->n_pol;
    r.n_ant = obs->n_ant;
    r.int_begin = int_begin;
    r.int_end = int_end;
    r.out = out;
    r.done = done;
    return r;
}

psc_status check_call(psc_ctx* ctx, psc_obs* obs, const double* offsets)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!obs || obs->ctx != ctx) return fail(ctx, PSC_E_ARG, "observation missing or from another context");
    if (!offsets) return fail(ctx, PSC_E_ARG, "null offsets");
    if (!ctx->model_set) return fail(ctx, PSC_E_STATE, "psc_set_model has not been called");
    if (hipSetDevice(ctx->cfg.device) != hipSuccess) return fail(ctx, PSC_E_HIP, "hipSetDevice");
    return PSC_OK;
}

// Calls whose kernels take real patterns only: refused while an aperture
// defocus is set.
psc_status no_defocus(psc_ctx* ctx, const psc_obs* obs, const char* what)
{
    if (obs->defocus)
        return fail(ctx, PSC_E_UNSUPPORTED,
                    std::string(what) + ": not available with an aperture defocus set (psc_set_defocus)");
    return PSC_OK;
}

// Degrid launch in the observation's current form.
hipError_t launch_degrid(int mode, const psc_ctx* ctx, const psc_obs* obs, const ItemArgs& a, hipStream_t st)
{
    if (obs->degrid == PSC_DEGRID_WINDOW) return launch_win(mode, ctx->s, a, st);
    return launch_items(mode, ctx->s, a, st);
}

// One iteration of the solver over intervals [s0, s1): gradient sums, reduce, step.
hipError_t enqueue_iteration(psc_ctx* ctx, psc_obs* obs, const void* vis_obs, const float* w,
                             double* offsets, double gain, double tol, int s0, int s1,
                             const int32_t* done_for_items, hipStream_t st)
{
    const int i0 = obs->int_item_ptr[s0], i1 = obs->int_item_ptr[s1];
    ItemArgs a = item_args(ctx, obs, offsets, i0, i1 - i0, done_for_items);
    a.vis_in = (const float2*)vis_obs;
    a.weight = w;
    hipError_t e = launch_degrid(kGrad, ctx, obs, a, st);
    if (e != hipSuccess) return e;
    e = launch_reduce(12, reduce_args(obs, s0, s1, obs->acc, done_for_items), st);
    if (e != hipSuccess) return e;
    SolveArgs sa{};
    sa.n_int = obs->n_int;
    sa.n_pol = obs->n_pol;
    sa.n_ant = obs->n_ant;
    sa.int_begin = s0;
    sa.int_end = s1;
    sa.acc = obs->acc;
    sa.gain = gain;
    sa.offsets = offsets;
    sa.max_step = obs->max_step;
    sa.done = obs->done;
    sa.iters = obs->iters;
    sa.tol = tol;
    return launch_solve(sa, st);
}

}  // namespace

extern "C" {

PSC_API psc_status psc_predict(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev, void* vis_out_dev,
                               void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if (!vis_out_dev && obs->n_vis > 0) return fail(ctx, PSC_E_ARG, "null output");
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
    a.vis_out = (float2*)vis_out_dev;
    PSC_HIP(ctx, launch_degrid(kPredict, ctx, obs, a, (hipStream_t)stream));
    return PSC_OK;
}

PSC_API psc_status psc_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                const void* vis_obs_dev, const float* weight_dev, double* acc_out_dev,
                                void* vis_model_dev, void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if (!acc_out_dev || ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0))
        return fail(ctx, PSC_E_ARG, "null data or output");
    if ((st = no_defocus(ctx, obs, "psc_gradient")) != PSC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
    a.vis_in = (const float2*)vis_obs_dev;
    a.weight = weight_dev;
    a.vis_out = (float2*)vis_model_dev;
    PSC_HIP(ctx, launch_degrid(kGrad, ctx, obs, a, s));
    PSC_HIP(ctx, launch_reduce(12, reduce_args(obs, 0, obs->n_int, acc_out_dev, nullptr), s));
    return PSC_OK;
}

PSC_API psc_status psc_gradient_noalloc(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                        const void* vis_obs_dev, const float* weight_dev, double* acc_out_dev,
                                        void* vis_model_dev, void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if ((st = no_defocus(ctx, obs, "psc_gradient_noalloc")) != PSC_OK) return st;
    if (!acc_out_dev || ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0))
        return fail(ctx, PSC_E_ARG, "null data or output");
    if ((size_t)obs->n_items * (size_t)obs->n_pol * 12 > kScratchDoubles)
        return fail(ctx, PSC_E_UNSUPPORTED,
                    "psc_gradient_noalloc: the observation's partial sums (12 float64 per work item and "
                    "polarisation) exceed its 64 MiB scratch; use psc_gradient");
    double* part = nullptr;
    PSC_HIP(ctx, scratch_address(ctx->cfg.device, &part));
    hipStream_t s = (hipStream_t)stream;
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
    a.vis_in = (const float2*)vis_obs_dev;
    a.weight = weight_dev;
    a.vis_out = (float2*)vis_model_dev;
    a.partials = part;  // every item writes all of its sums: nothing to clear
    PSC_HIP(ctx, launch_degrid(kGrad, ctx, obs, a, s));
    ReduceArgs r = reduce_args(obs, 0, obs->n_int, acc_out_dev, nullptr);
    r.partials = part;
    PSC_HIP(ctx, launch_reduce(12, r, s));
    return PSC_OK;
}

PSC_API psc_status psc_predict_vjp(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                   const void* grad_vis_dev, double* grad_offsets_out_dev, void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if ((st = no_defocus(ctx, obs, "psc_predict_vjp")) != PSC_OK) return st;
    if (!grad_offsets_out_dev || (!grad_vis_dev && obs->n_vis > 0))
        return fail(ctx, PSC_E_ARG, "null data or output");
    hipStream_t s = (hipStream_t)stream;
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
    a.vis_in = (const float2*)grad_vis_dev;
    PSC_HIP(ctx, launch_degrid(kVjp, ctx, obs, a, s));
    PSC_HIP(ctx, launch_reduce(4, reduce_args(obs, 0, obs->n_int, grad_offsets_out_dev, nullptr), s));
    return PSC_OK;
}

// Per item, its samples in time order (the sample index within a group
// grows with the row, and rows grow with time within an interval), each with
// its sub-table slot: 2 g + 0 for group g's offset f, 2 g + 1 for -f.  Built
// on the host from the device plan on first use; entries of an item occupy
// the item's own range of the sample array.
static psc_status build_time_order(psc_ctx* ctx, psc_obs* obs)
{
    try {
        std::vector<Item> items((size_t)obs->n_items);
        std::vector<Group> groups((size_t)obs->n_groups);
        std::vector<VisEnt> vis((size_t)obs->n_vis);
        PSC_HIP(ctx, hipMemcpy(items.data(), obs->items, items.size() * sizeof(Item), hipMemcpyDeviceToHost));
        PSC_HIP(ctx, hipMemcpy(groups.data(), obs->groups, groups.size() * sizeof(Group), hipMemcpyDeviceToHost));
        PSC_HIP(ctx, hipMemcpy(vis.data(), obs->vis, vis.size() * sizeof(VisEnt), hipMemcpyDeviceToHost));
        std::vector<uint2> ord(vis.size());
        struct Ent {
            uint32_t vidx, idx, slot;
        };
        std::vector<Ent> ents;
        for (const Item& it : items) {
            ents.clear();
            uint32_t lo = UINT32_MAX;
            for (int gl = 0; gl < it.grp_end - it.grp_begin; ++gl) {
                const Group& g = groups[(size_t)it.grp_begin + gl];
                lo = std::min(lo, g.vis_begin);
                for (int v = 0; v < g.n_vis + g.n_vis2; ++v) {
                    const uint32_t idx = g.vis_begin + (uint32_t)v;
                    ents.push_back({vis[idx].vidx, idx, (uint32_t)(2 * gl + (v >= g.n_vis ? 1 : 0))});
                }
            }
            std::sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) { return x.vidx < y.vidx; });
            for (size_t k = 0; k < ents.size(); ++k) ord[lo + k] = make_uint2(ents[k].idx, ents[k].slot);
        }
        if (dmalloc(&obs->ig_ord, ord.size()) != hipSuccess) return fail(ctx, PSC_E_OOM, "image-gradient order");
        PSC_HIP(ctx, hipMemcpy(obs->ig_ord, ord.data(), ord.size() * sizeof(uint2), hipMemcpyHostToDevice));
    } catch (const std::bad_alloc&) {
        return fail(ctx, PSC_E_OOM, "host memory for the image-gradient order");
    }
    return PSC_OK;
}

PSC_API psc_status psc_image_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                      const void* vis_obs_dev, const float* weight_dev,
                                      double* image_grad_out_dev, void* vis_model_dev, void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if ((st = no_defocus(ctx, obs, "psc_image_gradient")) != PSC_OK) return st;
    if (!image_grad_out_dev || ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0))
        return fail(ctx, PSC_E_ARG, "null data or output");
    if (obs->w_nk > 0)
        return fail(ctx, PSC_E_UNSUPPORTED, "psc_image_gradient: not available for a w-stacked observation");
    const int n = ctx->n;
    const size_t np = (size_t)(n + ctx->s) * (n + ctx->s);
    if (!ctx->rgrid) {
        hipError_t e = dmalloc(&ctx->rgrid, np);
        if (e == hipSuccess) e = dmalloc(&ctx->fa, (size_t)n * n);
        if (e == hipSuccess) e = dmalloc(&ctx->fb, (size_t)n * n);
        if (e != hipSuccess) {
            dfree(ctx->rgrid);
            dfree(ctx->fa);
            dfree(ctx->fb);
            ctx->rgrid = ctx->fa = ctx->fb = nullptr;
            return fail(ctx, PSC_E_OOM, "image-gradient scratch");
        }
    }
    int log2n = 0;
    while ((1 << log2n) < n) ++log2n;
    hipStream_t s = (hipStream_t)stream;
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
    a.vis_in = (const float2*)vis_obs_dev;
    a.weight = weight_dev;
    a.vis_out = (float2*)vis_model_dev;
    a.grid_acc = ctx->rgrid;
    a.use_mfma = 0;
    PSC_HIP(ctx, launch_zero(ctx->rgrid, np, s));
    const bool table_patch = ctx->s == 16 && !obs->par_angle && !obs->w_m && !obs->scale && !obs->ap_tab &&
                             grid_lds_bytes(ctx->s, ctx->m, ctx->o) <= kGridLdsMax;
    if (table_patch || ctx->s == 32 || obs->par_angle || obs->w_m || obs->scale || obs->ap_tab) {
        // predict, then a patch scatter: per item with its sub-tables and its
        // samples in time order (support 16, sky frame), or with a kernel per
        // sample (support 32, mount frame, w-term)
        if (table_patch && !obs->ig_ord && obs->n_vis > 0) {
            psc_status bs = build_time_order(ctx, obs);
            if (bs != PSC_OK) return bs;
        }
        float2* vm = (float2*)vis_model_dev;
        if (!vm && obs->n_vis > 0) {
            if (!obs->ig_vm && dmalloc(&obs->ig_vm, (size_t)obs->n_row * obs->n_chan * obs->n_pol) != hipSuccess)
                return fail(ctx, PSC_E_OOM, "image-gradient model visibilities");
            vm = obs->ig_vm;
        }
        a.vis_out = vm;
        PSC_HIP(ctx, launch_degrid(kPredict, ctx, obs, a, s));
        a.vis_model = vm;
        a.ig_ord = obs->ig_ord;
        if (table_patch) {
            PSC_HIP(ctx, launch_grid(ctx->s, a, s));
        } else {
            // scaled beams or a measured aperture in the sky frame: the
            // per-sample kernels at angle zero
            if ((obs->scale || obs->ap_tab) && !a.par_angle) a.par_angle = obs->zero_pa;
            PSC_HIP(ctx, launch_gridw(ctx->s, a, s));
        }
    } else {
        // the table-form scatter: degrid and spread in one pass, a float64
        // atomic per tap
        PSC_HIP(ctx, launch_items(kGrid, ctx->s, a, s));
    }
    PSC_HIP(ctx, launch_unpad_grid(ctx->rgrid, ctx->fa, n, ctx->s, s));
    PSC_HIP(ctx, launch_fft_rows(ctx->fa, n, log2n, s));
    PSC_HIP(ctx, launch_transpose(ctx->fa, ctx->fb, n, s));
    PSC_HIP(ctx, launch_fft_rows(ctx->fb, n, log2n, s));
    PSC_HIP(ctx, launch_transpose(ctx->fb, ctx->fa, n, s));
    PSC_HIP(ctx, launch_image_grad(ctx->fa, ctx->taper_pix, image_grad_out_dev, n, s));
    return PSC_OK;
}

PSC_API psc_status psc_solve_step(psc_ctx* ctx, int32_t n_int, int32_t n_pol, int32_t n_ant,
                                  const double* acc_dev, double gain, double lm_mu, double* offsets_io_dev,
                                  int32_t* not_updated_dev, double* max_step_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (n_int < 1 || n_pol < 1 || n_pol > 2 || n_ant < 1) return fail(ctx, PSC_E_ARG, "bad sizes");
    if (!acc_dev || !offsets_io_dev) return fail(ctx, PSC_E_ARG, "null array");
    if (!(gain > 0.0) || !(gain <= 1.0)) return fail(ctx, PSC_E_ARG, "gain must be in (0, 1]");
    if (!(lm_mu >= 0.0) || !isfinite(lm_mu)) return fail(ctx, PSC_E_ARG, "lm_mu must be finite and >= 0");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    SolveArgs sa{};
    sa.n_int = n_int;
    sa.n_pol = n_pol;
    sa.n_ant = n_ant;
    sa.int_begin = 0;
    sa.int_end = n_int;
    sa.acc = acc_dev;
    sa.gain = gain;
    sa.lm_mu = lm_mu;
    sa.offsets = offsets_io_dev;
    sa.not_updated = not_updated_dev;
    sa.max_step = max_step_dev;
    PSC_HIP(ctx, launch_solve(sa, (hipStream_t)stream));
    return PSC_OK;
}

PSC_API psc_status psc_set_degrid(psc_obs* obs, int32_t variant)
{
    if (!obs) return fail(nullptr, PSC_E_ARG, "null observation");
    if (variant != PSC_DEGRID_VALU && variant != PSC_DEGRID_MFMA && variant != PSC_DEGRID_WINDOW)
        return fail(obs->ctx, PSC_E_ARG, "unknown degrid variant");
    if (obs->ctx->s != 16 && variant != PSC_DEGRID_WINDOW)
        return fail(obs->ctx, PSC_E_UNSUPPORTED, "support 32 degrids in the window form only");
    if (obs->par_angle && variant != PSC_DEGRID_WINDOW)
        return fail(obs->ctx, PSC_E_UNSUPPORTED,
                    "mount-frame offsets (parallactic angles) degrid in the window form only");
    if (obs->w_m && variant != PSC_DEGRID_WINDOW)
        return fail(obs->ctx, PSC_E_UNSUPPORTED, "the w-term degrids in the window form only");
    if (obs->scale && variant != PSC_DEGRID_WINDOW)
        return fail(obs->ctx, PSC_E_UNSUPPORTED, "beam-width scales degrid in the window form only");
    if (obs->ap_tab && variant != PSC_DEGRID_WINDOW)
        return fail(obs->ctx, PSC_E_UNSUPPORTED, "a measured aperture degrids in the window form only");
    if (obs->defocus && variant != PSC_DEGRID_WINDOW)
        return fail(obs->ctx, PSC_E_UNSUPPORTED, "an aperture defocus degrids in the window form only");
    if (obs->graph) {  // a captured solve graph holds the old kernels
        (void)hipGraphExecDestroy(obs->graph);
        obs->graph = nullptr;
    }
    obs->degrid = variant;
    return PSC_OK;
}

PSC_API psc_status psc_get_degrid(const psc_obs* obs, int32_t* variant)
{
    if (!obs || !variant) return fail(nullptr, PSC_E_ARG, "null argument");
    *variant = obs->degrid;
    return PSC_OK;
}

// The narrowest beam the support holds: a scale below 1 widens the aperture
// to D / sigma, and each baseline kernel with it, to 2 (D / sigma) FoV /
// lambda cells at the highest frequency.  The window form stays within the
// parity tolerance while that leaves about half the taper's width of the
// support free (on a 1.4 GHz array whose aperture term is 8 cells of 16 at
// sigma = 1: float32 rounding down to sigma = 0.8, 7e-6 on the visibilities
// and 6e-5 on the sums at 0.7).  No bound for the Gaussian test mode.
static double scale_floor(const psc_ctx* ctx, const psc_obs* obs)
{
    if (ctx->cfg.illum == 1) return 0.0;
    const double ap_cells = 2.0 * ctx->cfg.dish_diam_m * ctx->fov * obs->fmax / kCLight;
    return ap_cells / (ctx->s - 0.5 * ctx->cfg.taper_width - 0.5);
}

// A beam scale sigma < 1 stretches every pattern lookup to |l - p| / sigma:
// the Airy table (and a measured aperture's pattern table) built at
// psc_obs_create for sigma = 1 is rebuilt to cover the range over smin.
// The moment table of the defocus mode follows the Airy table's nodes, so it
// is dropped (scales and a defocus are not set together; psc_set_defocus
// builds it again).  The caller has synchronised the device.
static hipError_t grow_tables(const psc_ctx* ctx, psc_obs* obs, double smin)
{
    const double dx = 1.0 / obs->inv_dx;
    const int n_tab = (int)ceil(obs->tab_x1 / smin / dx) + 3;
    float4* airy = nullptr;
    hipError_t e = dmalloc(&airy, n_tab);
    if (e == hipSuccess) e = launch_airy_table(airy, n_tab, dx, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        dfree(airy);
        return e;
    }
    dfree(obs->airy);
    dfree(obs->mtab);
    obs->airy = airy;
    obs->n_tab = n_tab;
    if (obs->ap_tab) {
        const int ap_half = (int)ceil(obs->ap_r1 / smin / obs->ap_step) + 2;
        const int ap_n = 2 * ap_half + 1;
        float4* tab = nullptr;
        e = aperture_tables(ctx, ap_n, ap_half, obs->ap_step, &tab);
        if (e != hipSuccess) return e;
        dfree(obs->ap_tab);
        obs->ap_tab = tab;
        obs->ap_n = ap_n;
        obs->ap_c = ap_half;
    }
    obs->tab_scale = smin;
    return hipSuccess;
}

PSC_API psc_status psc_set_beam_scale(psc_ctx* ctx, psc_obs* obs, const double* scale_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!obs || obs->ctx != ctx) return fail(ctx, PSC_E_ARG, "observation missing or from another context");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t st = (hipStream_t)stream;
    if (!scale_dev) {  // back to the nominal beams
        if (obs->scale) {
            PSC_HIP(ctx, hipDeviceSynchronize());  // no launch may still read them
            dfree(obs->scale);
            if (obs->graph) {  // a captured solve graph holds the freed scales
                (void)hipGraphExecDestroy(obs->graph);
                obs->graph = nullptr;
            }
        }
        return PSC_OK;
    }
    if (obs->defocus)
        return fail(ctx, PSC_E_UNSUPPORTED, "beam scales and an aperture defocus cannot be set together");
    const size_t n = (size_t)obs->n_int * obs->n_pol * obs->n_ant;
    std::vector<double> h(n);
    PSC_HIP(ctx, hipMemcpyAsync(h.data(), scale_dev, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    PSC_HIP(ctx, hipStreamSynchronize(st));
    double smin = 1.0;
    for (size_t k = 0; k < n; ++k) {
        if (!(h[k] > 0.0) || !isfinite(h[k])) return fail(ctx, PSC_E_ARG, "beam scales must be positive and finite");
        smin = std::min(smin, h[k]);
    }
    if (smin < scale_floor(ctx, obs))
        return fail(ctx, PSC_E_UNSUPPORTED, "beam scale too small: the widened aperture's kernel "
                                            "(2 D FoV / (sigma lambda) cells) outgrows the support");
    // the pattern tables cover every scale the observation can reach: the
    // scale step narrows beams on the device, down to the same floor
    const double cover = std::min(1.0, scale_floor(ctx, obs));
    if (ctx->cfg.illum != 1 && cover < obs->tab_scale) {
        PSC_HIP(ctx, hipDeviceSynchronize());  // no launch may still read the tables
        const hipError_t e = grow_tables(ctx, obs, cover);
        if (e != hipSuccess) return hip_fail(ctx, e, "psc_set_beam_scale: pattern tables");
    }
    // the image gradient's scatter builds each sample's kernel when the
    // beams are scaled: in the sky frame it runs at angle zero
    if (!obs->par_angle && !obs->zero_pa) {
        const size_t nr = obs->n_row > 0 ? (size_t)obs->n_row : 1;
        PSC_HIP(ctx, dmalloc(&obs->zero_pa, nr));
        PSC_HIP(ctx, hipMemsetAsync(obs->zero_pa, 0, sizeof(double) * nr, st));
    }
    if (!obs->scale) PSC_HIP(ctx, dmalloc(&obs->scale, n));
    PSC_HIP(ctx, hipMemcpyAsync(obs->scale, scale_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    PSC_HIP(ctx, hipStreamSynchronize(st));
    obs->degrid = PSC_DEGRID_WINDOW;
    if (obs->graph) {  // a captured solve graph holds the old kernels
        (void)hipGraphExecDestroy(obs->graph);
        obs->graph = nullptr;
    }
    return PSC_OK;
}

PSC_API psc_status psc_get_beam_scale(psc_ctx* ctx, const psc_obs* obs, double* scale_out_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!obs || obs->ctx != ctx || !scale_out_dev) return fail(ctx, PSC_E_ARG, "null argument");
    if (!obs->scale) return fail(ctx, PSC_E_STATE, "no beam scales set (psc_set_beam_scale)");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    const size_t n = (size_t)obs->n_int * obs->n_pol * obs->n_ant;
    PSC_HIP(ctx, hipMemcpyAsync(scale_out_dev, obs->scale, sizeof(double) * n, hipMemcpyDeviceToDevice,
                                (hipStream_t)stream));
    return PSC_OK;
}

PSC_API psc_status psc_scale_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                      const void* vis_obs_dev, const float* weight_dev, double* acc_out_dev,
                                      void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if ((st = no_defocus(ctx, obs, "psc_scale_gradient")) != PSC_OK) return st;
    if (!acc_out_dev || ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0))
        return fail(ctx, PSC_E_ARG, "null data or output");
    if (!obs->scale) return fail(ctx, PSC_E_STATE, "no beam scales set (psc_set_beam_scale)");
    hipStream_t s = (hipStream_t)stream;
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
    a.vis_in = (const float2*)vis_obs_dev;
    a.weight = weight_dev;
    PSC_HIP(ctx, launch_win(kScale, ctx->s, a, s));
    PSC_HIP(ctx, launch_reduce(6, reduce_args(obs, 0, obs->n_int, acc_out_dev, nullptr), s));
    return PSC_OK;
}

PSC_API psc_status psc_scale_step(psc_ctx* ctx, psc_obs* obs, const double* acc_dev, double gain,
                                  int32_t* not_updated_dev, double* max_step_out_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!obs || obs->ctx != ctx || !acc_dev) return fail(ctx, PSC_E_ARG, "null argument");
    if (!(gain > 0.0) || !(gain <= 1.0)) return fail(ctx, PSC_E_ARG, "gain must be in (0, 1]");
    if (!obs->scale) return fail(ctx, PSC_E_STATE, "no beam scales set (psc_set_beam_scale)");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    PSC_HIP(ctx, launch_scale_step(obs->n_int, obs->n_pol, obs->n_ant, acc_dev, gain, obs->scale, not_updated_dev,
                                   max_step_out_dev, nullptr, nullptr, 0.0, scale_floor(ctx, obs),
                                   (hipStream_t)stream));
    return PSC_OK;
}

PSC_API psc_status psc_solve_scale(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev, const void* vis_obs_dev,
                                   const float* weight_dev, double gain, int32_t n_max, double tol,
                                   int32_t* iters_out_dev, void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if ((st = no_defocus(ctx, obs, "psc_solve_scale")) != PSC_OK) return st;
    if ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0) return fail(ctx, PSC_E_ARG, "null data");
    if (!(gain > 0.0) || !(gain <= 1.0)) return fail(ctx, PSC_E_ARG, "gain must be in (0, 1]");
    if (n_max < 0 || !(tol >= 0.0)) return fail(ctx, PSC_E_ARG, "n_max must be >= 0 and tol >= 0");
    if (!obs->scale) return fail(ctx, PSC_E_STATE, "no beam scales set (psc_set_beam_scale)");
    hipStream_t s = (hipStream_t)stream;
    PSC_HIP(ctx, launch_init_state(obs->done, obs->iters, obs->n_int, s));
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, obs->done);
    a.vis_in = (const float2*)vis_obs_dev;
    a.weight = weight_dev;
    const double sfloor = scale_floor(ctx, obs);
    // every interval in one launch set per iteration; finished intervals are
    // skipped by every kernel (their items, sums and steps)
    for (int it = 0; it < n_max; ++it) {
        PSC_HIP(ctx, launch_win(kScale, ctx->s, a, s));
        PSC_HIP(ctx, launch_reduce(6, reduce_args(obs, 0, obs->n_int, obs->acc, obs->done), s));
        PSC_HIP(ctx, launch_scale_step(obs->n_int, obs->n_pol, obs->n_ant, obs->acc, gain, obs->scale, nullptr,
                                       obs->max_step, obs->done, obs->iters, tol, sfloor, s));
    }
    if (iters_out_dev)
        PSC_HIP(ctx, hipMemcpyAsync(iters_out_dev, obs->iters, sizeof(int32_t) * obs->n_int, hipMemcpyDeviceToDevice, s));
    return PSC_OK;
}

PSC_API psc_status psc_set_defocus(psc_ctx* ctx, psc_obs* obs, const double* defocus_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!obs || obs->ctx != ctx) return fail(ctx, PSC_E_ARG, "observation missing or from another context");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    hipStream_t st = (hipStream_t)stream;
    if (!defocus_dev) {  // back to real patterns
        if (obs->defocus) {
            PSC_HIP(ctx, hipDeviceSynchronize());  // no launch may still read them
            dfree(obs->defocus);
        }
        return PSC_OK;
    }
    if (ctx->cfg.illum == 2 || obs->par_angle || obs->scale)
        return fail(ctx, PSC_E_UNSUPPORTED, "aperture defocus: uniform disc or Gaussian patterns, sky-frame "
                                            "offsets and no beam scales only");
    const size_t n = (size_t)obs->n_int * obs->n_pol * obs->n_ant;
    std::vector<double> h(n);
    PSC_HIP(ctx, hipMemcpyAsync(h.data(), defocus_dev, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    PSC_HIP(ctx, hipStreamSynchronize(st));
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(h[k]) || fabs(h[k]) > kMaxDefocus)
            return fail(ctx, PSC_E_ARG, "defocus must be finite and within [-pi, pi] radians");
    if (ctx->cfg.illum == 0 && !obs->mtab) {
        // the uniform disc's moments on the Airy table's nodes
        std::vector<double> gx, gw;
        gauss_legendre(96, gx, gw);
        for (size_t q = 0; q < gx.size(); ++q) {
            gx[q] = 0.5 * (gx[q] + 1.0);
            gw[q] *= 0.5;
        }
        double *dt = nullptr, *dw = nullptr;
        hipError_t e = dmalloc(&obs->mtab, (size_t)obs->n_tab * kMoments);
        if (e == hipSuccess) e = dmalloc(&dt, gx.size());
        if (e == hipSuccess) e = dmalloc(&dw, gw.size());
        if (e == hipSuccess) e = hipMemcpy(dt, gx.data(), sizeof(double) * gx.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dw, gw.data(), sizeof(double) * gw.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_moment_table(obs->mtab, obs->n_tab, kMoments, 1.0 / obs->inv_dx, dt, dw, (int)gx.size(), st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        dfree(dt);
        dfree(dw);
        if (e != hipSuccess) {
            dfree(obs->mtab);
            return hip_fail(ctx, e, "psc_set_defocus: moment table");
        }
    }
    if (!obs->defocus) PSC_HIP(ctx, dmalloc(&obs->defocus, n));
    PSC_HIP(ctx, hipMemcpyAsync(obs->defocus, defocus_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    PSC_HIP(ctx, hipStreamSynchronize(st));
    obs->degrid = PSC_DEGRID_WINDOW;
    if (obs->graph) {  // a captured solve graph holds the old kernels
        (void)hipGraphExecDestroy(obs->graph);
        obs->graph = nullptr;
    }
    return PSC_OK;
}

PSC_API psc_status psc_get_defocus(psc_ctx* ctx, const psc_obs* obs, double* defocus_out_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!obs || obs->ctx != ctx || !defocus_out_dev) return fail(ctx, PSC_E_ARG, "null argument");
    if (!obs->defocus) return fail(ctx, PSC_E_STATE, "no aperture defocus set (psc_set_defocus)");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    const size_t n = (size_t)obs->n_int * obs->n_pol * obs->n_ant;
    PSC_HIP(ctx, hipMemcpyAsync(defocus_out_dev, obs->defocus, sizeof(double) * n, hipMemcpyDeviceToDevice,
                                (hipStream_t)stream));
    return PSC_OK;
}

PSC_API psc_status psc_defocus_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                        const void* vis_obs_dev, const float* weight_dev, double* acc_out_dev,
                                        void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if (!acc_out_dev || ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0))
        return fail(ctx, PSC_E_ARG, "null data or output");
    if (!obs->defocus) return fail(ctx, PSC_E_STATE, "no aperture defocus set (psc_set_defocus)");
    hipStream_t s = (hipStream_t)stream;
    ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
    a.vis_in = (const float2*)vis_obs_dev;
    a.weight = weight_dev;
    // the scale mode's sums (chi, Re(conj(R) w dV/da), w |dV/da|^2 per end)
    // with the defocus derivatives in place of the scale's
    PSC_HIP(ctx, launch_win(kScale, ctx->s, a, s));
    PSC_HIP(ctx, launch_reduce(6, reduce_args(obs, 0, obs->n_int, acc_out_dev, nullptr), s));
    return PSC_OK;
}

PSC_API psc_status psc_defocus_step(psc_ctx* ctx, psc_obs* obs, const double* acc_dev, double gain,
                                    int32_t* not_updated_dev, double* max_step_out_dev, void* stream)
{
    if (!ctx) return fail(nullptr, PSC_E_ARG, "null context");
    ctx->err.clear();
    if (!obs || obs->ctx != ctx || !acc_dev) return fail(ctx, PSC_E_ARG, "null argument");
    if (!(gain > 0.0) || !(gain <= 1.0)) return fail(ctx, PSC_E_ARG, "gain must be in (0, 1]");
    if (!obs->defocus) return fail(ctx, PSC_E_STATE, "no aperture defocus set (psc_set_defocus)");
    PSC_HIP(ctx, hipSetDevice(ctx->cfg.device));
    PSC_HIP(ctx, launch_defocus_step(obs->n_int, obs->n_pol, obs->n_ant, acc_dev, gain, obs->defocus,
                                     not_updated_dev, max_step_out_dev, (hipStream_t)stream));
    return PSC_OK;
}

PSC_API psc_status psc_tune(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev, const void* vis_obs_dev,
                            const float* weight_dev, int32_t repeats, double* times_us_out, void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_dev);
    if (st != PSC_OK) return st;
    if ((st = no_defocus(ctx, obs, "psc_tune")) != PSC_OK) return st;
    if ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0) return fail(ctx, PSC_E_ARG, "null data");
    if (repeats < 1 || repeats > 1000) return fail(ctx, PSC_E_ARG, "repeats must be in [1, 1000]");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PSC_HIP(ctx, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    double best = 1e300;
    int32_t best_v = obs->degrid;
    const int32_t keep = obs->degrid;
    for (int32_t v = PSC_DEGRID_VALU; v <= PSC_DEGRID_WINDOW && e == hipSuccess; ++v) {
        if ((ctx->s != 16 || obs->par_angle || obs->w_m || obs->scale || obs->ap_tab) && v != PSC_DEGRID_WINDOW) {
            if (times_us_out) times_us_out[v] = -1.0;  // not available at this support
            continue;
        }
        obs->degrid = v;
        ItemArgs a = item_args(ctx, obs, offsets_dev, 0, (int)obs->n_items, nullptr);
        a.vis_in = (const float2*)vis_obs_dev;
        a.weight = weight_dev;
        e = launch_degrid(kGrad, ctx, obs, a, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < repeats && e == hipSuccess; ++r) e = launch_degrid(kGrad, ctx, obs, a, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const double us = 1e3 * ms / repeats;
        if (times_us_out) times_us_out[v] = us;
        if (e == hipSuccess && us < best) {
            best = us;
            best_v = v;
        }
    }
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    obs->degrid = keep;
    if (e != hipSuccess) return hip_fail(ctx, e, "psc_tune");
    return psc_set_degrid(obs, best_v);
}

static psc_status solve_impl(psc_ctx* ctx, psc_obs* obs, const void* vis_obs_dev, const float* weight_dev,
                             double* offsets_io_dev, double gain, int32_t n_max, double tol_rad,
                             int32_t form, int32_t* iters_out_dev, void* stream)
{
    psc_status st = check_call(ctx, obs, offsets_io_dev);
    if (st != PSC_OK) return st;
    if ((st = no_defocus(ctx, obs, "psc_solve")) != PSC_OK) return st;
    if ((!vis_obs_dev || !weight_dev) && obs->n_vis > 0) return fail(ctx, PSC_E_ARG, "null data");
    if (!(gain > 0.0) || !(gain <= 1.0)) return fail(ctx, PSC_E_ARG, "gain must be in (0, 1]");
    if (n_max < 0 || !(tol_rad >= 0.0)) return fail(ctx, PSC_E_ARG, "n_max must be >= 0 and tol_rad >= 0");
    if (form != PSC_SOLVE_PLAIN && form != PSC_SOLVE_BATCHED && form != PSC_SOLVE_GRAPH)
        return fail(ctx, PSC_E_ARG, "unknown solve form");
    hipStream_t s = (hipStream_t)stream;
    PSC_HIP(ctx, launch_init_state(obs->done, obs->iters, obs->n_int, s));
    if (form == PSC_SOLVE_PLAIN) {
        for (int iv = 0; iv < obs->n_int; ++iv) {
            for (int it = 0; it < n_max; ++it) {
                PSC_HIP(ctx, enqueue_iteration(ctx, obs, vis_obs_dev, weight_dev, offsets_io_dev, gain,
                                               tol_rad, iv, iv + 1, nullptr, s));
                double mx = 0.0;
                PSC_HIP(ctx, hipMemcpyAsync(&mx, obs->max_step + iv, sizeof(double), hipMemcpyDeviceToHost, s));
                PSC_HIP(ctx, hipStreamSynchronize(s));
                if (mx < tol_rad) break;
            }
        }
    } else if (form == PSC_SOLVE_BATCHED) {
        for (int it = 0; it < n_max; ++it)
            PSC_HIP(ctx, enqueue_iteration(ctx, obs, vis_obs_dev, weight_dev, offsets_io_dev, gain, tol_rad,
                                           0, obs->n_int, obs->done, s));
    } else {
        const bool same = obs->graph && obs->g_vis == vis_obs_dev && obs->g_w == weight_dev &&
                          obs->g_off == offsets_io_dev && obs->g_gain == gain && obs->g_tol == tol_rad &&
                          obs->g_nmax == n_max;
        if (!same) {
            const auto t0 = std::chrono::steady_clock::now();
            if (obs->graph) {
                (void)hipGraphExecDestroy(obs->graph);
                obs->graph = nullptr;
            }
            PSC_HIP(ctx, hipStreamBeginCapture(obs->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int it = 0; it < n_max && e == hipSuccess; ++it)
                e = enqueue_iteration(ctx, obs, vis_obs_dev, weight_dev, offsets_io_dev, gain, tol_rad, 0,
                                      obs->n_int, obs->done, obs->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(obs->cap_stream, &g);
            if (e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(ctx, e, "graph capture");
            }
            if (e2 != hipSuccess) return hip_fail(ctx, e2, "hipStreamEndCapture");
            e = hipGraphInstantiate(&obs->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                obs->graph = nullptr;
                return hip_fail(ctx, e, "hipGraphInstantiate");
            }
            obs->g_vis = vis_obs_dev;
            obs->g_w = weight_dev;
            obs->g_off = offsets_io_dev;
            obs->g_gain = gain;
            obs->g_tol = tol_rad;
            obs->g_nmax = n_max;
            obs->capture_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        // the graph runs on the capture stream after the caller's queued work
        PSC_HIP(ctx, hipStreamSynchronize(s));
        PSC_HIP(ctx, hipGraphLaunch(obs->graph, obs->cap_stream));
        PSC_HIP(ctx, hipStreamSynchronize(obs->cap_stream));
    }
    if (iters_out_dev)
        PSC_HIP(ctx, hipMemcpyAsync(iters_out_dev, obs->iters, sizeof(int32_t) * obs->n_int,
                                    hipMemcpyDeviceToDevice, s));
    PSC_HIP(ctx, hipStreamSynchronize(s));
    return PSC_OK;
}

// Host allocations in planning and solving may throw; no exception crosses the
// C boundary.
static psc_status host_oom(psc_ctx* ctx)
{
    try {
        return fail(ctx, PSC_E_OOM, "host memory allocation failed");
    } catch (...) {
        return PSC_E_OOM;
    }
}

PSC_API psc_status psc_create(const psc_config* cfg, psc_ctx** out)
{
    try {
        return create_impl(cfg, out);
    } catch (...) {
        return host_oom(nullptr);
    }
}

PSC_API psc_status psc_obs_create(psc_ctx* ctx, const psc_obs_desc* d, psc_obs** out)
{
    try {
        const auto t0 = std::chrono::steady_clock::now();
        const psc_status st = obs_create_impl(ctx, d, out);
        if (st == PSC_OK)
            (*out)->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return st;
    } catch (...) {
        return host_oom(ctx);
    }
}

PSC_API psc_status psc_solve(psc_ctx* ctx, psc_obs* obs, const void* vis_obs_dev, const float* weight_dev,
                             double* offsets_io_dev, double gain, int32_t n_max, double tol_rad,
                             int32_t form, int32_t* iters_out_dev, void* stream)
{
    try {
        return solve_impl(ctx, obs, vis_obs_dev, weight_dev, offsets_io_dev, gain, n_max, tol_rad, form,
                          iters_out_dev, stream);
    } catch (...) {
        return host_oom(ctx);
    }
}

}  // extern "C"
