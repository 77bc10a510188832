/*
 * psc.h -- C ABI of libpsc, the MI355X (gfx950) implementation of the
 * Pointing SelfCal predict / gradient / update hot path
 * (Bhatnagar & Cornwell 2017, "The Pointing Self Calibration algorithm for
 * aperture synthesis radio telescopes", arXiv:1709.08681).
 *
 * General rules
 *  - Every call returns a psc_status; nothing throws or prints.  On failure
 *    psc_last_error() describes the first problem found.
 *  - Array arguments named *_dev are DEVICE pointers on the context's GPU,
 *    owned by the caller and only borrowed for the duration of the call
 *    (asynchronous calls: until the work queued on `stream` has finished).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls marked
 *    "async" only enqueue work; calls marked "sync" block until done.
 *  - One context/observation pair must not be used from two streams at once:
 *    they own scratch memory that concurrent calls would share.
 *  - Units: angles and direction cosines in radians, baselines in metres,
 *    frequencies in Hz, flux in Jy.  Complex arrays are interleaved
 *    (re, im) float32 pairs ("complex64") unless stated otherwise.
 *
 * Symbols follow the paper: V^{M0} is the Fourier transform of the model
 * image on the grid (Sec. 2.2, Eq. MEDD), A_ij the aperture-plane kernel of
 * baseline (i,j) (Eq. ME), l_i = (l_i, m_i) the pointing offset of antenna i
 * (Sec. 3), R = V^Obs - V^M the residual (Eq. Res), W the inverse-variance
 * weights (Eq. Chisq).
 */
#ifndef PSC_H
#define PSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSC_API __attribute__((visibility("default")))

typedef enum {
    PSC_OK = 0,
    PSC_E_ARG = -1,          /* invalid argument (shape, range, null pointer) */
    PSC_E_HIP = -2,          /* a HIP runtime call failed */
    PSC_E_OOM = -3,          /* device or host allocation failed */
    PSC_E_UNSUPPORTED = -4,  /* valid request outside what the library implements */
    PSC_E_STATE = -5         /* call out of order (e.g. predict before set_model) */
} psc_status;

typedef struct psc_ctx psc_ctx;
typedef struct psc_obs psc_obs;

/*
 * Geometry of the model grid and of the antenna model; fixed per context.
 *
 *  grid_n        N, edge of the N x N model grid V^{M0}; power of two, 64..8192.
 *  cell_rad      pixel size of the model image (direction cosine per pixel);
 *                FoV = N * cell_rad, uv cell = 1 / FoV wavelengths.
 *  support       S, width of every baseline kernel in uv cells (16 or 32).
 *                The kernel of baseline (i,j) is the convolution of the two
 *                antennas' aperture functions (Eq. MEDD), whose width is
 *                2 D / lambda, with the anti-aliasing taper (taper_width
 *                cells); it must fit: 2 D FoV / lambda + taper_width < S.
 *  oversample    O, kernel samples per uv cell (1..16, S*O <= 512).  Each
 *                visibility's uv is rounded to the nearest 1/O cell.
 *  image_samples M, image-plane samples per axis used to build kernels, at
 *                spacing FoV/S (0 = default 3S/2; even, S..2S).
 *  dish_diam_m   D of the dishes (uniformly illuminated circular ones for
 *                illum 0).
 *  illum         0: far-field voltage pattern 2 J1(x)/x, x = pi D |l| / lambda;
 *                1: the Gaussian main-lobe model of Sec. 3,
 *                   exp(-|l|^2 / (2 s^2)), s = gauss_sigma_ld * lambda / D.
 *                   Its aperture is not compactly supported: the kernel fits
 *                   the S-cell window only for gauss_sigma_ld >~ 1.5.
 *                2: a measured aperture (below): the far-field pattern is
 *                   the Fourier transform of the aperture illumination (Sec. 1
 *                   and Sec. 3: blockage, feed-support shadows and taper enter
 *                   through it), fixed to the antenna mount (turned by each
 *                   row's par_angle when given).  Observations degrid in the
 *                   window form; psc_set_degrid refuses the table forms.
 *  squint_frac   beam squint: polarisation 0 (1) is centred at
 *                +(-) squint_frac * HPBW(nu) along +l, HPBW = 1.02899 lambda/D
 *                (Sec. 4.2: the two parallel hands are solved separately).
 *  taper_width   width W of the exponential-of-semicircle anti-aliasing taper
 *                in uv cells (0 = default 8); taper_beta its shape
 *                (0 = default 2.30 * W).
 *  device        HIP device ordinal.
 *  aperture_n,   illum 2 only: the aperture illumination, a HOST array of
 *  aperture      aperture_n x aperture_n float64 (1..256 per side) over the
 *                square of side D centred on the dish axis, [x][y] row-major
 *                with x along the mount frame's l axis; cell (i, j) is
 *                centred at ((i - (n-1)/2) D/n, (j - (n-1)/2) D/n).  It must
 *                be real, finite and even (A[i][j] = A[n-1-i][n-1-j], so the
 *                pattern is real) with a positive sum; otherwise PSC_E_ARG.
 *                Read by psc_create only (not retained).  The pattern is
 *                normalised to one on axis, tabulated per observation on
 *                32 nodes per lambda/D over the image samples plus a quarter
 *                of the field of view, and interpolated bicubically (values
 *                and slopes); displacements beyond the table take its edge
 *                value.
 *  aperture_count  apertures stacked in `aperture`, [count][n][n], each
 *                under the same rules (0 counts as 1); an observation's
 *                ant_aperture gives each antenna one of them (Sec. 3: a
 *                heterogeneous array).  Each is tabulated per observation.
 */
typedef struct {
    int32_t grid_n;
    int32_t support;
    int32_t oversample;
    int32_t image_samples;
    double cell_rad;
    double dish_diam_m;
    int32_t illum;
    double gauss_sigma_ld;
    double squint_frac;
    int32_t taper_width;
    double taper_beta;
    int32_t device;
    int32_t aperture_n;
    const double* aperture;
    int32_t aperture_count;
} psc_config;

/*
 * Description of the visibility data (read once by psc_obs_create).
 * Rows are (time, baseline) samples.  Every pointer is a DEVICE pointer.
 *
 *  int_row_ptr [n_int+1] int64: rows of solution interval s are
 *              [int_row_ptr[s], int_row_ptr[s+1]); intervals may be uneven
 *              or empty (Algorithm 1 solves each interval separately).
 *  ant1, ant2  [n_row] int32 antenna indices, 0 <= ant1 < ant2 < n_ant.
 *  uv_m        [n_row][2] float64 baseline (u, v) in metres.
 *  freq_hz     [n_chan] float64 channel frequencies.
 *  n_pol       1 or 2 parallel-hand polarisations.
 *  par_angle   nullable [n_row] float64 parallactic angle chi of each row
 *              (rad).  When given, offsets (and squint) are in the antenna
 *              mount frame, as the paper solves its VLA data (Sec. 4): a
 *              row's beam centre on the sky is R(chi) (offset + squint) with
 *              R = [[cos, -sin], [sin, cos]], and every derivative, sum and
 *              update is with respect to the mount-frame offsets.  The
 *              kernels then differ from sample to sample: the observation
 *              degrids in the window form with per-sample image-plane
 *              products (psc_set_degrid refuses the table forms).
 *  w_m         nullable [n_row] float64 baseline w in metres (the component
 *              along the phase centre).  When given, the measurement
 *              equation carries the w-term, phase 2 pi w (n - 1) with
 *              n = sqrt(1 - l^2 - m^2) beside u l + v m (w-projection: each
 *              sample's kernel is the transform of the aperture products
 *              times that phase, so it must still fit the support); the
 *              observation degrids in the window form, and psc_set_degrid
 *              refuses the table forms.  The phase widens each kernel by
 *              about |w| FoV / D uv cells over the beam; when max |w| FoV / D
 *              exceeds 1.5 the observation w-stacks (Sec. 5.1): the model is
 *              transformed again for planes w_k = k dw, each sample reads the
 *              plane nearest its w and carries the residual in its kernel
 *              (PSC_E_UNSUPPORTED when the planes would exceed 2 GiB).
 *              Null: w = 0.
 *  ant_aperture nullable [n_ant] int32: with illum 2 and several apertures
 *              (psc_config::aperture_count), the aperture of each antenna,
 *              0 <= index < aperture_count (Sec. 3: the heterogeneous
 *              array); null: every antenna takes aperture 0.  PSC_E_ARG for
 *              an index out of range, or for a map without illum 2.
 *
 * Visibility-shaped arrays used by the calls below are laid out
 * [n_row][n_chan][n_pol]; offsets are [n_int][n_pol][n_ant][2] float64 (l, m).
 */
typedef struct {
    int32_t n_ant;
    int32_t n_chan;
    int32_t n_pol;
    int32_t n_int;
    int64_t n_row;
    const int64_t* int_row_ptr;
    const int32_t* ant1;
    const int32_t* ant2;
    const double* uv_m;
    const double* freq_hz;
    const double* par_angle;
    const double* w_m;
    const int32_t* ant_aperture;
} psc_obs_desc;

/* Library version string. */
PSC_API const char* psc_version(void);

/* Create a context (sync).  Fails with PSC_E_ARG on an invalid config. */
PSC_API psc_status psc_create(const psc_config* cfg, psc_ctx** out);

/* Destroy a context and free its device memory (sync).  NULL is allowed. */
PSC_API psc_status psc_destroy(psc_ctx* ctx);

/* Message describing the last failure on this context ("" if none); valid
 * until the next call on the context.  ctx may be NULL (creation errors). */
PSC_API const char* psc_last_error(const psc_ctx* ctx);

/*
 * Model transform, Algorithm 1 step 1 (V^{M0} = F[I^M], Eq. MEDD) (sync).
 * image_dev: [N][N] float64 real model image, pixel (ix, iy) at direction
 * cosines ((ix - N/2) cell, (iy - N/2) cell).  The library divides by the
 * taper's image-plane response, transforms in float64 and keeps V^{M0} as a
 * complex64 grid.  Emission must lie in the central N/2 x N/2 pixels.
 */
PSC_API psc_status psc_set_model(psc_ctx* ctx, const double* image_dev, void* stream);

/*
 * Plan the visibility data (sync).  Copies the geometry, rounds every
 * (row, channel) uv to the kernel lattice, groups samples into work items
 * (interval, baseline, channel) and allocates the observation's scratch.
 * Without parallactic angles or a measured aperture (sky-frame offsets,
 * radial beams) the scratch includes every antenna's pattern and gradient
 * factor at the M x M image samples per interval, polarisation and channel,
 * n_int n_pol n_chan n_ant M^2 x 8 bytes, which the window form fills before
 * each degrid (Eq. DA per antenna, shared by its baselines) while one
 * interval's share stays within 8 MiB (its tables then stay in L2) and the
 * whole within 16 GiB; otherwise it is left out and each work item
 * evaluates its two antennas' patterns.
 * Calls on one observation share this scratch and must not overlap.
 * Returns PSC_E_ARG for inconsistent indices (ant1 >= ant2, out of range,
 * non-monotone int_row_ptr).
 */
PSC_API psc_status psc_obs_create(psc_ctx* ctx, const psc_obs_desc* desc, psc_obs** out);
PSC_API psc_status psc_obs_destroy(psc_obs* obs);

/* Sizes of a planned observation (host pointers, each nullable). */
PSC_API psc_status psc_obs_info(const psc_obs* obs, int64_t* n_items, int64_t* n_groups,
                                int64_t* n_vis);

/*
 * How the observation's gradient launches (host struct, filled by
 * psc_obs_launch_info; sync, no device work).  Describes the launch shape
 * of the A-Projection degrid of Algorithm 1 as planned for this data, so a
 * caller can see which kernel the autotuner kept and how the plan split it.
 *   degrid            PSC_DEGRID_* the gradient and adjoint run in
 *   window_waves      wavefronts per block of the window-form gradient
 *                     kernel (1 or 2 for items of few samples at support
 *                     16, else 4, or 8 at support 32 when two blocks of four
 *                     do not fit a compute unit's LDS)
 *   samples_per_item  mean samples per work item (interval, baseline,
 *                     channel): what the block shape is chosen from
 *   plan_ms           host wall time psc_obs_create took (planning, uploads
 *                     and setup kernels)
 *   w_planes          model grids of a w-stacked observation (0 when the
 *                     w-term, if any, fits one kernel)
 *   tab_nodes         nodes of the Airy table (grown by psc_set_beam_scale
 *                     for scales below 1)
 *   capture_ms        host wall time the last graph-form psc_solve spent
 *                     capturing and instantiating its graph (0 before any)
 *   pattern_tables    1 when the window form reads every antenna's pattern
 *                     from per-antenna tables filled before each degrid
 *                     (sky frame, radial beams, support 16, one interval's
 *                     tables within 8 MiB; see psc_obs_create), else 0
 *   items_per_block   consecutive work items each block of a gradient
 *                     launch over all intervals takes: 32 for the window
 *                     form in the sky frame at support 32 with at least
 *                     2^19 items (the block's set-up, twiddles and Airy
 *                     table into LDS, is then paid once per 32 items),
 *                     else 1; a launch of fewer items (one interval of the
 *                     plain solve form) takes one each
 * PSC_E_ARG for a null observation or output.
 */
typedef struct {
    int32_t degrid;
    int32_t window_waves;
    double samples_per_item;
    double plan_ms;
    int32_t w_planes;
    int32_t tab_nodes;
    double capture_ms;
    int32_t pattern_tables;
    int32_t items_per_block;
} psc_launch_info;
PSC_API psc_status psc_obs_launch_info(const psc_obs* obs, psc_launch_info* out);

/*
 * Predict (async): V^M_ij = [A_i (x) A_j*] * V^{M0} (Eq. MEDD, Eq. ME with the
 * direction-independent term equal to one), where A_i carries antenna i's
 * pointing offset as an aperture phase gradient (Sec. 3, Eq. AIJPOINTING
 * generalised to the exact two-aperture kernel).
 *  offsets_dev [n_int][n_pol][n_ant][2] float64
 *  vis_out_dev [n_row][n_chan][n_pol] complex64 (written)
 */
PSC_API psc_status psc_predict(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                               void* vis_out_dev, void* stream);

/*
 * Residual, chi^2, gradient and 2x2 normal matrix per antenna (async):
 * Eq. DCHIDD with a = (l_i, m_i) and Algorithm 1's accumulation step.  For
 * every visibility of baseline (i, j) and both ends a in {i, j}:
 *   chi_a += w |R|^2,  g_a += w Re(conj(R) dV/dp_a),
 *   H_a   += w Re(conj(dV/dp_a) dV/dp_a^T)        (R = V^Obs - V^M)
 * so g_a = -1/2 d chi^2 / d p_a, and chi_a counts each visibility once per end.
 *  vis_obs_dev  [n_row][n_chan][n_pol] complex64
 *  weight_dev   [n_row][n_chan][n_pol] float32 inverse variance, 0 = flagged
 *  acc_out_dev  [n_int][n_pol][n_ant][6] float64: chi, g_l, g_m, H_ll, H_lm, H_mm
 *  vis_model_dev nullable [n_row][n_chan][n_pol] complex64: V^M if not NULL
 * The sums are accumulated in float64 in a fixed order: repeated calls give
 * bit-identical results.
 */
PSC_API psc_status psc_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                const void* vis_obs_dev, const float* weight_dev,
                                double* acc_out_dev, void* vis_model_dev, void* stream);

/*
 * psc_gradient for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, arguments, results and errors as psc_gradient, but
 * the per-item float64 partial sums go to a fixed scratch array inside the
 * library instead of the observation's own buffer, and the call makes no
 * allocation of any kind.  The scratch is 64 MiB per GPU, held from the
 * library's load until the process ends: observations with n_items * n_pol
 * * 12 float64 sums beyond it are refused with PSC_E_UNSUPPORTED (about
 * 699,000 work items per polarisation; n_items from psc_obs_info).  Every
 * call on one GPU shares that GPU's scratch: calls that overlap on one GPU
 * (different streams, or threads without ordering) race and give wrong sums.
 * Every work item rewrites all of its sums, so nothing needs clearing.
 */
PSC_API psc_status psc_gradient_noalloc(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                        const void* vis_obs_dev, const float* weight_dev,
                                        double* acc_out_dev, void* vis_model_dev, void* stream);

/*
 * Vector-Jacobian product of psc_predict (async), the adjoint used by
 * automatic differentiation: for every (interval, pol, antenna a)
 *   grad[a] = sum over visibilities touching a of Re(conj(G) dV/dp_a)
 * with G = grad_vis (the gradient of a real loss with respect to Re V + i Im V).
 * Kernels are rebuilt from the offsets; nothing is kept from the forward call.
 *  grad_vis_dev  [n_row][n_chan][n_pol] complex64
 *  grad_offsets_out_dev [n_int][n_pol][n_ant][2] float64 (written)
 */
PSC_API psc_status psc_predict_vjp(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                   const void* grad_vis_dev, double* grad_offsets_out_dev,
                                   void* stream);

/*
 * Gradient of chi^2 with respect to the model image (async): the direction of
 * the model update that alternates with the antenna solve in the
 * self-calibration loop (Sec. 2), i.e. the residual image seen through both
 * offset beams of every baseline:
 *   image_grad[n] = d chi^2 / d I[n]
 *                 = -2 sum w Re( conj(R) E_i(l_n - p_i) E_j(l_n - p_j) exp(+2 pi i u.l_n) )
 * with R = V^Obs - V^M at the given offsets.  Computed as the exact adjoint of
 * this library's predict: w conj(R) is spread back over each sample's window
 * with the kernel coefficients that produced V^M (float64 sums on a residual
 * grid), transformed like the model (float64 FFT) and divided by the taper.
 *  vis_obs_dev, weight_dev  as for psc_gradient
 *  image_grad_out_dev [N][N] float64, indexed like the image of psc_set_model
 *  vis_model_dev      nullable; receives V^M
 * At support 16 with sky-frame offsets the scatter uses the item's
 * sub-tables; at 32, and with offsets in the mount frame (where each row's
 * beams differ), it builds each sample's kernel.  The first call allocates the context's scratch, (N+S)^2 + 2 N^2
 * complex float64; at support 16 with oversampling up to 4 (where every
 * sub-table of an item fits in LDS) the observation's time order of each
 * item's samples (8 bytes per sample, built on the host from a copy of the
 * plan: a blocking call); and, when vis_model_dev is null, room for V^M
 * (complex64 per visibility).  Taps are summed in float32 LDS patches in a
 * fixed order and the patches added to the residual grid with float64
 * atomics, so results agree between runs to float64 rounding, not bit for
 * bit.
 */
PSC_API psc_status psc_image_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                      const void* vis_obs_dev, const float* weight_dev,
                                      double* image_grad_out_dev, void* vis_model_dev,
                                      void* stream);

/*
 * Damped per-antenna update (async), Sec. 2.2 (a_n = a_{n-1} + f(grad)) with
 * f read as a 2x2 Gauss-Newton step scaled by the loop gain 0 < gain <= 1 of
 * Eq. SelfCal, on the Levenberg-Marquardt damped normal matrix
 * H'_a = H_a + lm_mu diag(H_a) (lm_mu >= 0; 0 is plain Gauss-Newton):
 * p_a += gain * H'_a^-1 g_a  when det H'_a > 1e-12 (tr H'_a)^2, else
 * p_a += gain * g_k / H'_kk per axis with H'_kk > 0.  Antennas with
 * tr H_a <= 0 or non-finite sums keep their offsets and get not_updated = 1.
 * psc_solve uses lm_mu = 0.
 *  acc_dev        [n_int][n_pol][n_ant][6] float64 (from psc_gradient)
 *  offsets_io_dev [n_int][n_pol][n_ant][2] float64 (updated in place)
 *  not_updated_dev nullable [n_int][n_pol][n_ant] int32
 *  max_step_dev    nullable [n_int] float64: largest |delta p| per interval
 */
PSC_API psc_status psc_solve_step(psc_ctx* ctx, int32_t n_int, int32_t n_pol, int32_t n_ant,
                                  const double* acc_dev, double gain, double lm_mu,
                                  double* offsets_io_dev, int32_t* not_updated_dev,
                                  double* max_step_dev, void* stream);

/*
 * Degrid variants (results agree to float32 rounding; each is deterministic
 * on its own):
 *  PSC_DEGRID_VALU    table form: per sub-lattice offset, the five S x S
 *                     sub-tables (kernel and its four offset derivatives,
 *                     Eq. MEDD and Eq. DA) are built by FFT in LDS and read by
 *                     vector FP32 multiply-adds; support 16;
 *  PSC_DEGRID_MFMA    table form on the FP32 matrix cores (16x16x4), 16
 *                     samples of one sub-table per tile (gradient and adjoint;
 *                     prediction uses VALU); support 16;
 *  PSC_DEGRID_WINDOW  window form: each sample's S x S window of V^{M0} is
 *                     transformed instead of the kernels, and the sum runs
 *                     over the image-plane samples; no sub-table is stored.
 *                     Cheaper when sub-tables serve few samples each; the only
 *                     form for support 32.
 * A new observation starts with PSC_DEGRID_VALU at support 16 and
 * PSC_DEGRID_WINDOW at support 32; psc_set_degrid returns PSC_E_UNSUPPORTED
 * for a table form at support 32.  The variant applies to psc_predict,
 * psc_gradient, psc_predict_vjp and psc_solve.
 */
#define PSC_DEGRID_VALU 0
#define PSC_DEGRID_MFMA 1
#define PSC_DEGRID_WINDOW 2
PSC_API psc_status psc_set_degrid(psc_obs* obs, int32_t variant);
PSC_API psc_status psc_get_degrid(const psc_obs* obs, int32_t* variant);

/*
 * Autotuner (sync): times psc_gradient on the caller's data with every degrid
 * variant (`repeats` launches each, after one warm-up) and keeps the fastest
 * for this observation.  times_us_out (host, nullable) receives the mean
 * launch time of each variant, indexed by PSC_DEGRID_* (-1 for a variant the
 * support does not allow; 3 entries).
 */
PSC_API psc_status psc_tune(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                            const void* vis_obs_dev, const float* weight_dev, int32_t repeats,
                            double* times_us_out, void* stream);

/*
 * Beam-width scale, a generalised antenna parameter (Eq. DA holds for any
 * antenna parameter a_i; Sec. 5.3 solves the beam's shape with the same
 * machinery as the offsets).  Antenna a's pattern becomes E0(d / sigma_a),
 * d its displacement from the beam centre: sigma > 1 widens the beam.
 *
 * psc_set_beam_scale (sync): copies scale_dev, [n_int][n_pol][n_ant]
 * float64 (device, borrowed), into the observation; every later predict,
 * gradient, adjoint, solve and image gradient uses it.  Values must be
 * positive and finite (PSC_E_ARG, the observation unchanged).  A scale
 * below 1 widens the aperture to D / sigma and the baseline kernel with it;
 * unless illum = 1, the smallest scale must keep 2 D FoV / (sigma lambda_min)
 * <= support - taper_width / 2 - 1/2 cells (PSC_E_UNSUPPORTED otherwise, the
 * observation unchanged; about sigma >= 0.68 when the field of view is
 * chosen so that the aperture term is half of a 16-cell support).  The scales
 * enter through the window form's image-plane products (per antenna), so
 * the observation then degrids in the window form (psc_set_degrid refuses
 * the table forms); the image gradient then builds each sample's kernel
 * (in the sky frame at angle zero, from [n_row] zeros the first call
 * allocates).  A scale below 1 stretches every pattern lookup to
 * |l - p| / sigma, so the first call rebuilds the beam tables (Airy, and a
 * measured aperture's pattern) over the range at the smallest scale allowed,
 * which the scale step cannot pass either (device memory reallocated; the
 * defocus moment table is dropped with them).  A null scale_dev drops the
 * scales (sigma = 1 again; the window form and the tables stay).  A
 * captured solve graph is discarded.
 * psc_get_beam_scale (async): copies the observation's scales to
 * scale_out_dev; PSC_E_STATE when none are set.
 */
PSC_API psc_status psc_set_beam_scale(psc_ctx* ctx, psc_obs* obs, const double* scale_dev, void* stream);
PSC_API psc_status psc_get_beam_scale(psc_ctx* ctx, const psc_obs* obs, double* scale_out_dev, void* stream);

/*
 * Sums of Eq. DCHIDD for the beam-width scales (async): per (interval, pol,
 * antenna), over both ends of every baseline,
 *   acc_out_dev[..][3] = chi = sum w |R|^2, g = sum Re(conj(R) w dV/dsigma_a),
 *                        H = sum w |dV/dsigma_a|^2,
 * with R = V^Obs - V^M at the given offsets and the observation's scales;
 * float64 sums of float32 terms, like psc_gradient.  Arguments as for
 * psc_gradient.  PSC_E_STATE without scales set.
 */
PSC_API psc_status psc_scale_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                      const void* vis_obs_dev, const float* weight_dev, double* acc_out_dev,
                                      void* stream);

/*
 * Damped update of the observation's scales (async): sigma += gain g / H per
 * (interval, pol, antenna) from acc_dev ([n_int][n_pol][n_ant][3], from
 * psc_scale_gradient), 0 < gain <= 1 (the loop gain of Eq. SelfCal; all
 * antennas move together, as for the offsets, and gain 1 makes the two ends
 * of a baseline overshoot together).  Antennas with H <= 0, non-finite sums,
 * or a step that would leave sigma non-positive or below the narrowest beam
 * the support holds (the bound of psc_set_beam_scale) keep their scale and
 * get not_updated = 1.
 *  not_updated_dev  nullable [n_int][n_pol][n_ant] int32
 *  max_step_out_dev nullable [n_int] float64: largest |delta sigma| per interval
 */
PSC_API psc_status psc_scale_step(psc_ctx* ctx, psc_obs* obs, const double* acc_dev, double gain,
                                  int32_t* not_updated_dev, double* max_step_out_dev, void* stream);

/*
 * Solve for the observation's beam scales at fixed offsets (async), as
 * Algorithm 1 solves for the offsets, with every interval in one launch set
 * per iteration: up to n_max rounds of psc_scale_gradient and psc_scale_step
 * on the device; an interval stops once its largest |delta sigma| is below
 * tol (finished intervals are skipped by every kernel).  The scales are
 * updated in place on the observation (psc_get_beam_scale reads them).
 *  offsets_dev      [n_int][n_pol][n_ant][2] float64, not changed
 *  vis_obs_dev, weight_dev  as for psc_gradient
 *  iters_out_dev    nullable [n_int] int32: steps taken per interval
 * PSC_E_STATE without scales set.
 */
PSC_API psc_status psc_solve_scale(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev, const void* vis_obs_dev,
                                   const float* weight_dev, double gain, int32_t n_max, double tol,
                                   int32_t* iters_out_dev, void* stream);

/*
 * Aperture defocus, a complex generalised antenna parameter (Eq. DA with a
 * complex a_i; Sec. 5.3 names aperture phase terms such as defocus as the
 * first shape parameters to solve for).  A defocus delta (radians of
 * aperture phase at the dish rim) multiplies antenna a's illumination by
 * exp(i delta (r/R)^2), R = D/2, so its pattern is complex:
 *   uniform disc (illum 0): E = 2 int_0^1 J0(pi D rho t / lambda)
 *                            exp(i delta t^2) t dt, rho the distance from
 *                            the beam centre (2 J1(x)/x at delta = 0);
 *   Gaussian mode (illum 1): E = z exp(-z rho^2 / (2 s^2)), z = 1 / (1 - i
 *                            kappa), kappa = 2 delta / (pi^2 gauss_sigma_ld^2).
 * Visibilities carry E_i conj(E_j) (Eq. ME).  Available for illum 0 and 1,
 * sky-frame offsets, without beam scales; the window form predicts with it.
 *
 * psc_set_defocus (sync): defocus_dev [n_int][n_pol][n_ant] float64 device
 *   array, copied; each value finite with |delta| <= pi (PSC_E_ARG
 *   otherwise).  NULL removes it (real patterns again).  PSC_E_UNSUPPORTED
 *   with a measured aperture, parallactic angles or beam scales.  While set,
 *   psc_predict uses the complex patterns; psc_gradient, psc_gradient_noalloc,
 *   psc_predict_vjp, psc_image_gradient, psc_solve, psc_tune and the
 *   beam-scale calls return PSC_E_UNSUPPORTED.
 * psc_get_defocus (async): copies the current values to defocus_out_dev.
 * psc_defocus_gradient (async): the Eq. DCHIDD sums for the defocus, per
 *   (interval, pol, antenna) acc_out_dev[3] = (chi, g = sum Re(conj(R) w
 *   dV/ddelta_a), H = sum w |dV/ddelta_a|^2) over both ends of every
 *   baseline, R = V^Obs - V^M, at the given offsets.
 * psc_defocus_step (async): delta += gain g / H on the device for every
 *   (interval, pol, antenna) with H > 0 and finite sums whose result stays
 *   within |delta| <= pi; the others are kept and flagged in
 *   not_updated_dev (nullable, int32 [n_int][n_pol][n_ant]); max_step_out_dev
 *   (nullable, [n_int]) gets each interval's largest |step|.  gain in (0, 1].
 * The three calls after psc_set_defocus return PSC_E_STATE without it.
 */
PSC_API psc_status psc_set_defocus(psc_ctx* ctx, psc_obs* obs, const double* defocus_dev, void* stream);
PSC_API psc_status psc_get_defocus(psc_ctx* ctx, const psc_obs* obs, double* defocus_out_dev, void* stream);
PSC_API psc_status psc_defocus_gradient(psc_ctx* ctx, psc_obs* obs, const double* offsets_dev,
                                        const void* vis_obs_dev, const float* weight_dev, double* acc_out_dev,
                                        void* stream);
PSC_API psc_status psc_defocus_step(psc_ctx* ctx, psc_obs* obs, const double* acc_dev, double gain,
                                    int32_t* not_updated_dev, double* max_step_out_dev, void* stream);

/* Execution forms of psc_solve. */
#define PSC_SOLVE_PLAIN 0    /* host loop over intervals, one launch set per interval */
#define PSC_SOLVE_BATCHED 1  /* every interval in one launch set per iteration */
#define PSC_SOLVE_GRAPH 2    /* BATCHED, with the n_max iterations captured in one HIP graph */

/*
 * Algorithm 1 (sync): for every solution interval, up to n_max iterations of
 * (gradient at the current offsets, damped update); an interval stops
 * iterating after the first step whose largest |delta p| is below tol_rad.
 *  offsets_io_dev [n_int][n_pol][n_ant][2] float64: start values in, solutions out
 *  iters_out_dev  nullable [n_int] int32: iterations run per interval
 * All three forms give bit-identical offsets.
 */
PSC_API psc_status psc_solve(psc_ctx* ctx, psc_obs* obs, const void* vis_obs_dev,
                             const float* weight_dev, double* offsets_io_dev, double gain,
                             int32_t n_max, double tol_rad, int32_t form, int32_t* iters_out_dev,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PSC_H */
