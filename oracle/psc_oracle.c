/*
 * psc_oracle.c -- plain FP64 CPU oracle for the Pointing SelfCal predict,
 * gradient and update (Bhatnagar & Cornwell 2017, arXiv:1709.08681).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * What it computes (everything in double precision, by definition, with no
 * gridding, tables, tapers or FFTs):
 *
 *  - predict: the measurement equation (Sec. 2, Eq. ME) with the
 *    direction-independent term set to one, evaluated by direct summation over
 *    the non-zero sky pixels.  The direction-dependent term of baseline (i,j)
 *    is the product of the two antennas' far-field patterns (Eq. MEDD), each
 *    shifted by that antenna's pointing offset (Sec. 3):
 *        V_ij(u) = sum_p I_p E_i(l_p) E_j(l_p) exp(+2 pi i u.l_p)
 *    E is the voltage pattern of a uniformly illuminated circular dish,
 *    2 J1(x)/x with x = pi D |l| / lambda, or, in the Gaussian test mode, the
 *    main-lobe model of Sec. 3, exp(-|l|^2 alpha^2) with alpha^2 = 1/(2 s^2),
 *    or the transform of a measured aperture illumination (below).
 *  - gradient: the analytic derivative of V with respect to the two offsets
 *    of each end of the baseline (Eq. DA with a = (l_i, m_i)), and the
 *    per-antenna sums of Eq. DCHIDD together with chi^2 (Eq. Chisq) and the
 *    2x2 Gauss-Newton normal matrix.
 *  - image gradient: the derivative of chi^2 with respect to the flux of
 *    chosen sky pixels, the residual image seen through both offset beams,
 *    which drives the model update of the self-calibration loop (Sec. 2).
 *  - solve step: the damped update of Sec. 2.2 (a_n = a_{n-1} + f(grad)),
 *    read as a per-antenna 2x2 Gauss-Newton step scaled by the loop gain
 *    0 < gamma < 1 of Eq. SelfCal.
 *
 * Readings taken where the paper is silent or garbled (all listed in the
 * design notes):
 *  - Algorithm 1 accumulates into antenna j but updates antenna i; here every
 *    stored baseline (i<j) contributes to both of its antennas.
 *  - chi^2 is summed over stored baselines once; g_a = sum Re(conj(R) w dV/dp_a)
 *    is minus one half of d chi^2 / d p_a, so p <- p + gamma H^-1 g descends.
 *  - All antennas are updated together (Jacobi) from sums taken at the
 *    previous iterate.
 *  - Visibility uv coordinates (in wavelengths) are rounded to the lattice of
 *    spacing 1/snap_scale before evaluation when snap_scale > 0; this is the
 *    nearest-sample lookup of an oversampled A-Projection kernel.
 *  - Polarisation p of antenna i has its beam centred at
 *    offset + sgn(p) * squint_frac * HPBW(nu) along +l, sgn = (+1, -1),
 *    HPBW = 1.02899 lambda / D.
 *  - With parallactic angles (one per row, optional), offsets and squint are
 *    in the antenna mount's frame and reach the sky rotated by the row's
 *    angle chi: p_sky = R(chi) (offset + squint), R = [[cos, -sin],
 *    [sin, cos]]; derivatives are taken with respect to the mount-frame
 *    offsets.  The paper solves in this frame for its VLA data (Sec. 4).
 *  - An optional beam-width scale sigma per (interval, pol, antenna), a
 *    generalised antenna parameter besides the offsets (Eq. DA with a_i =
 *    sigma_i; Sec. 5.3 treats the shape of the beam as parameters solved by
 *    the same machinery): the antenna's pattern is E0(d / sigma), d the
 *    displacement from its beam centre; sigma = 1 is the nominal beam.
 *  - A measured aperture (illum 2) is a real, even illumination on a square
 *    grid of cells across the dish; its far-field pattern is the aperture's
 *    Fourier transform (Sec. 1 and Sec. 3: the pattern of a dish follows
 *    from its illumination, with blockage and taper), fixed to the mount:
 *    towards sky position l a row sees E(R(chi)^T l - q), q the mount-frame
 *    offset plus squint (chi = 0 without parallactic angles).  A
 *    heterogeneous array (Sec. 3) gives each antenna one of several
 *    apertures: a baseline's visibility then carries E_i of antenna i's
 *    illumination and E_j of antenna j's.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "psc_oracle.h"

#define ORC_C_LIGHT 299792458.0
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Far-field pattern of one antenna and its derivative with respect to the  */
/* antenna's pointing offset.                                               */
/* ------------------------------------------------------------------------ */

/*
 * Airy voltage pattern of a uniformly illuminated circular aperture of
 * diameter D: E = 2 J1(x)/x, x = k rho, k = pi D / lambda, rho = |l - p|.
 * dE/dx = -2 J2(x)/x (Bessel recurrence), so
 *   dE/dp_l = 2 J2(x)/x * k * (l - p_l)/rho = k^2 (l - p_l) * 2 J2(x)/x^2.
 * 2 J2(x)/x^2 tends to 1/4 at x = 0.
 */
static void efp_airy(double k, double dl, double dm, double* e, double* de_dpl, double* de_dpm)
{
    double rho = sqrt(dl * dl + dm * dm);
    double x = k * rho;
    double e0, j2x2;
    if (x == 0.0) {
        e0 = 1.0;
        j2x2 = 0.25;
    } else if (x < 1e-4) {
        /* leading terms of the power series of J1 and J2 */
        e0 = 1.0 - x * x / 8.0;
        j2x2 = 0.25 - x * x / 48.0;
    } else {
        e0 = 2.0 * j1(x) / x;
        j2x2 = 2.0 * jn(2, x) / (x * x);
    }
    *e = e0;
    *de_dpl = k * k * dl * j2x2;
    *de_dpm = k * k * dm * j2x2;
}

/* Gaussian main-lobe model E = exp(-(dl^2+dm^2) alpha^2), alpha^2 = 1/(2 s^2). */
static void efp_gauss(double s, double dl, double dm, double* e, double* de_dpl, double* de_dpm)
{
    double a2 = 1.0 / (2.0 * s * s);
    double e0 = exp(-(dl * dl + dm * dm) * a2);
    *e = e0;
    *de_dpl = 2.0 * a2 * dl * e0;
    *de_dpm = 2.0 * a2 * dm * e0;
}

/*
 * Far-field pattern of a measured aperture: the Fourier transform of the
 * illumination A, summed directly over its cells and normalised to one on
 * the beam axis,
 *   E(d) = sum_k A_k cos(2 pi x_k . d / lambda) / sum_k A_k,
 * x_k the cell centres in metres, x_a = (a - (n - 1)/2) D / n per axis, and d
 * the displacement from the beam centre in the mount frame.  A is even, so
 * the sine part of the transform cancels and E is real.  The derivatives
 * with respect to the beam centre c (d = l - c) are
 *   dE/dc = sum_k A_k (2 pi x_k / lambda) sin(2 pi x_k . d / lambda) / sum_k A_k.
 */
static void efp_aperture(int n, const double* ap, double dish, double lambda, double dl, double dm,
                         double* e, double* de_dcl, double* de_dcm)
{
    double cell = dish / n, s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int a = 0; a < n; ++a) {
        double x = (a - 0.5 * (n - 1)) * cell;
        for (int b = 0; b < n; ++b) {
            double amp = ap[(size_t)a * n + b];
            if (amp == 0.0) continue;
            double y = (b - 0.5 * (n - 1)) * cell;
            double ph = 2.0 * ORC_PI * (x * dl + y * dm) / lambda;
            double sn = sin(ph);
            s0 += amp;
            s1 += amp * cos(ph);
            s2 += amp * (2.0 * ORC_PI * x / lambda) * sn;
            s3 += amp * (2.0 * ORC_PI * y / lambda) * sn;
        }
    }
    *e = s1 / s0;
    *de_dcl = s2 / s0;
    *de_dcm = s3 / s0;
}

void oracle_efp_aperture(int aperture_n, const double* aperture, double dish_diam_m, double freq_hz,
                         double dl, double dm, double* out3)
{
    efp_aperture(aperture_n, aperture, dish_diam_m, ORC_C_LIGHT / freq_hz, dl, dm, &out3[0], &out3[1],
                 &out3[2]);
}

/* The measured aperture of antenna a (illum 2): the first of the stack
 * unless the problem names one per antenna (Sec. 3: the heterogeneous
 * array, each antenna with its own illumination). */
static const double* aperture_of(const orc_problem* p, int a)
{
    const size_t n2 = (size_t)p->aperture_n * p->aperture_n;
    return p->aperture + (p->ant_aperture ? (size_t)p->ant_aperture[a] * n2 : 0);
}

/* The pattern of antenna a at displacement (dl, dm) from its beam centre at
 * channel c: (E, dE/dc_l, dE/dc_m). */
static void efp_problem(const orc_problem* p, int c, int a, double dl, double dm, double* out3)
{
    if (p->illum == 2)
        efp_aperture(p->aperture_n, aperture_of(p, a), p->dish_diam_m, ORC_C_LIGHT / p->freq_hz[c], dl, dm,
                     &out3[0], &out3[1], &out3[2]);
    else
        oracle_efp(p->illum, p->dish_diam_m, p->gauss_sigma_ld, p->freq_hz[c], dl, dm, out3);
}

/* The pattern widened by sigma, E(d) = E0(d / sigma), at displacement d
 * from the beam centre: out4 = (E, dE/dc_l, dE/dc_m, dE/dsigma).  The centre
 * derivatives are E0's at d / sigma divided by sigma, and
 * dE/dsigma = -(d / sigma^2) . grad E0 = (d . dE/dc) / sigma. */
static void efp_scaled(const orc_problem* p, int c, int a, double sigma, double dl, double dm, double* out4)
{
    double e[3];
    efp_problem(p, c, a, dl / sigma, dm / sigma, e);
    out4[0] = e[0];
    out4[1] = e[1] / sigma;
    out4[2] = e[2] / sigma;
    out4[3] = (dl * out4[1] + dm * out4[2]) / sigma;
}

/* sigma of antenna a, pol pol in one interval's scales (null: 1) */
static double sigma_of(const orc_problem* p, const double* scl_int, int pol, int a)
{
    return scl_int ? scl_int[pol * p->n_ant + a] : 1.0;
}

static double hpbw_rad(double lambda, double dish)
{
    return 1.02899 * lambda / dish;
}

void oracle_efp(int illum, double dish_diam_m, double gauss_sigma_ld, double freq_hz,
                double dl, double dm, double* out3)
{
    double lambda = ORC_C_LIGHT / freq_hz;
    if (illum == 1)
        efp_gauss(gauss_sigma_ld * lambda / dish_diam_m, dl, dm, &out3[0], &out3[1], &out3[2]);
    else
        efp_airy(ORC_PI * dish_diam_m / lambda, dl, dm, &out3[0], &out3[1], &out3[2]);
}

double oracle_hpbw(double freq_hz, double dish_diam_m)
{
    return hpbw_rad(ORC_C_LIGHT / freq_hz, dish_diam_m);
}

/* uv in wavelengths of one row at one frequency, optionally snapped. */
static void row_uv(const orc_problem* p, int64_t r, int c, double* u, double* v)
{
    double f = p->freq_hz[c];
    double uu = p->uv_m[2 * r] * f / ORC_C_LIGHT;
    double vv = p->uv_m[2 * r + 1] * f / ORC_C_LIGHT;
    if (p->snap_scale > 0.0) {
        uu = (double)llround(uu * p->snap_scale) / p->snap_scale;
        vv = (double)llround(vv * p->snap_scale) / p->snap_scale;
    }
    *u = uu;
    *v = vv;
}

/* w of row r at channel c in wavelengths (not rounded: it enters only the
 * phase), 0 without the w-term */
static double row_w(const orc_problem* p, int64_t r, int c)
{
    return p->w_m ? p->w_m[r] * p->freq_hz[c] / ORC_C_LIGHT : 0.0;
}

/* Phase of the measurement equation for a source at (l, m): 2 pi (u l + v m
 * + w (n - 1)), n = sqrt(1 - l^2 - m^2), with n - 1 = -x / (1 + sqrt(1 - x)),
 * x = l^2 + m^2, free of the cancellation of sqrt(1 - x) - 1. */
static double me_phase(double u, double v, double w, double l, double m)
{
    double x = l * l + m * m;
    double nm1 = -x / (1.0 + sqrt(1.0 - x));
    return 2.0 * ORC_PI * (u * l + v * m + w * nm1);
}

void oracle_snap_uv(const orc_problem* p, int64_t row, int chan, double* uv_out)
{
    row_uv(p, row, chan, &uv_out[0], &uv_out[1]);
}

/*
 * Beam values of every antenna towards every source, for one interval:
 * tab[((pol*n_ant + a)*n_chan + c)*n_src + s][4] = (E, dE/dl_a, dE/dm_a,
 * dE/dsigma_a).
 */
static double* beam_table(const orc_problem* p, const double* offs_int /* [n_pol][n_ant][2] */,
                          const double* scl_int /* nullable [n_pol][n_ant] */)
{
    size_t n = (size_t)p->n_pol * p->n_ant * p->n_chan * p->n_src;
    double* tab = (double*)malloc(n * 4 * sizeof(double));
    if (!tab) return NULL;
    for (int pol = 0; pol < p->n_pol; ++pol) {
        double sgn = (pol == 0) ? 1.0 : -1.0;
#pragma omp parallel for schedule(dynamic, 1)
        for (int a = 0; a < p->n_ant; ++a) {
            for (int c = 0; c < p->n_chan; ++c) {
                double lambda = ORC_C_LIGHT / p->freq_hz[c];
                double sq = sgn * p->squint_frac * hpbw_rad(lambda, p->dish_diam_m);
                double pl = offs_int[(pol * p->n_ant + a) * 2 + 0] + sq;
                double pm = offs_int[(pol * p->n_ant + a) * 2 + 1];
                double sig = sigma_of(p, scl_int, pol, a);
                for (int s = 0; s < p->n_src; ++s) {
                    double* t = tab + 4 * ((((size_t)pol * p->n_ant + a) * p->n_chan + c) * p->n_src + s);
                    efp_scaled(p, c, a, sig, p->src_l[s] - pl, p->src_m[s] - pm, t);
                }
            }
        }
    }
    return tab;
}

/*
 * Beam values of antenna a towards every source for one row when offsets are
 * given in the antenna frame: the offset plus squint q is carried onto the
 * sky by the row's parallactic angle chi, p = R(chi) q with
 * R = [[cos, -sin], [sin, cos]], and the derivatives are taken with respect
 * to q, dE/dq = R^T dE/dp.  t[4 s .. 4 s + 3] = (E, dE/dq_l, dE/dq_m,
 * dE/dsigma).
 */
static void beam_row(const orc_problem* p, const double* offs_int, const double* scl_int, int pol, int a,
                     int c, double chi, double* t)
{
    double sig = sigma_of(p, scl_int, pol, a);
    double lambda = ORC_C_LIGHT / p->freq_hz[c];
    double sq = (pol == 0 ? 1.0 : -1.0) * p->squint_frac * hpbw_rad(lambda, p->dish_diam_m);
    double ql = offs_int[(pol * p->n_ant + a) * 2 + 0] + sq;
    double qm = offs_int[(pol * p->n_ant + a) * 2 + 1];
    double cs = cos(chi), sn = sin(chi);
    if (p->illum == 2) {
        /* the pattern is fixed to the mount: evaluate it at the source's
         * mount-frame position R^T l minus q, where its derivatives are
         * already those with respect to q */
        for (int s = 0; s < p->n_src; ++s) {
            double dl = cs * p->src_l[s] + sn * p->src_m[s] - ql;
            double dm = -sn * p->src_l[s] + cs * p->src_m[s] - qm;
            efp_scaled(p, c, a, sig, dl, dm, t + 4 * s);
        }
        return;
    }
    double pl = cs * ql - sn * qm, pm = sn * ql + cs * qm;
    for (int s = 0; s < p->n_src; ++s) {
        double e[4];
        efp_scaled(p, c, a, sig, p->src_l[s] - pl, p->src_m[s] - pm, e);
        t[4 * s] = e[0];
        t[4 * s + 1] = cs * e[1] + sn * e[2];
        t[4 * s + 2] = -sn * e[1] + cs * e[2];
        t[4 * s + 3] = e[3];
    }
}

/*
 * Model visibility and its derivatives for one (row, chan, pol) from the two
 * antennas' beam values ti, tj ([n_src][4] each): out[0..1] = V,
 * out[2..9] = dV/dl_i, dV/dm_i, dV/dl_j, dV/dm_j, out[10..13] =
 * dV/dsigma_i, dV/dsigma_j (re, im each).
 */
static void vis_from_beams(const orc_problem* p, const double* ti, const double* tj, double u, double v,
                           double w, double* out, int want_grad)
{
    double acc[14] = {0};
    for (int s = 0; s < p->n_src; ++s) {
        double ph = me_phase(u, v, w, p->src_l[s], p->src_m[s]);
        double cr = cos(ph), ci = sin(ph);
        double fi = p->src_flux[s];
        double ei = ti[4 * s], ej = tj[4 * s];
        double a0 = fi * ei * ej;
        acc[0] += a0 * cr;
        acc[1] += a0 * ci;
        if (want_grad) {
            double d[6] = {fi * ti[4 * s + 1] * ej, fi * ti[4 * s + 2] * ej,
                           fi * ei * tj[4 * s + 1], fi * ei * tj[4 * s + 2],
                           fi * ti[4 * s + 3] * ej, fi * ei * tj[4 * s + 3]};
            for (int k = 0; k < 6; ++k) {
                acc[2 + 2 * k] += d[k] * cr;
                acc[3 + 2 * k] += d[k] * ci;
            }
        }
    }
    memcpy(out, acc, sizeof(acc));
}

/* The same from the interval's beam table (offsets in the sky frame). */
static void vis_one(const orc_problem* p, const double* tab, int pol, int ai, int aj, int c,
                    double u, double v, double w, double* out, int want_grad)
{
    const double* ti = tab + 4 * ((((size_t)pol * p->n_ant + ai) * p->n_chan + c) * p->n_src);
    const double* tj = tab + 4 * ((((size_t)pol * p->n_ant + aj) * p->n_chan + c) * p->n_src);
    vis_from_beams(p, ti, tj, u, v, w, out, want_grad);
}

/*
 * One (row, chan, pol): from the interval's beam table, or, when the problem
 * carries parallactic angles, from beams evaluated for this row into the
 * caller's scratch bi, bj ([n_src][4] each).  out has 14 entries.
 */
static void vis_row(const orc_problem* p, const double* tab, const double* offs_int, const double* scl_int,
                    int64_t r, int pol, int c, double u, double v, double w, double* bi, double* bj, double* out,
                    int want_grad)
{
    if (p->par_angle) {
        beam_row(p, offs_int, scl_int, pol, p->ant1[r], c, p->par_angle[r], bi);
        beam_row(p, offs_int, scl_int, pol, p->ant2[r], c, p->par_angle[r], bj);
        vis_from_beams(p, bi, bj, u, v, w, out, want_grad);
    } else {
        vis_one(p, tab, pol, p->ant1[r], p->ant2[r], c, u, v, w, out, want_grad);
    }
}

static int check_problem(const orc_problem* p)
{
    if (!p || p->n_ant < 2 || p->n_chan < 1 || p->n_pol < 1 || p->n_pol > 2 || p->n_int < 1)
        return -1;
    if (p->n_row < 0 || p->n_src < 0) return -1;
    if (p->int_row_ptr[0] != 0 || p->int_row_ptr[p->n_int] != p->n_row) return -1;
    for (int s = 0; s < p->n_int; ++s)
        if (p->int_row_ptr[s + 1] < p->int_row_ptr[s]) return -1;
    for (int64_t r = 0; r < p->n_row; ++r) {
        if (p->ant1[r] < 0 || p->ant2[r] < 0 || p->ant1[r] >= p->n_ant || p->ant2[r] >= p->n_ant ||
            p->ant1[r] == p->ant2[r])
            return -1;
    }
    if (p->illum < 0 || p->illum > 2) return -1;
    if (p->beam_scale)
        for (size_t k = 0; k < (size_t)p->n_int * p->n_pol * p->n_ant; ++k)
            if (!(p->beam_scale[k] > 0.0) || !isfinite(p->beam_scale[k])) return -1;
    if (p->illum == 2) {
        /* real, even apertures with a non-zero on-axis response, and every
         * antenna's index among them */
        int n = p->aperture_n, n_ap = p->n_apertures > 0 ? p->n_apertures : 1;
        if (n < 1 || !p->aperture) return -1;
        if (p->ant_aperture)
            for (int a = 0; a < p->n_ant; ++a)
                if (p->ant_aperture[a] < 0 || p->ant_aperture[a] >= n_ap) return -1;
        for (int k = 0; k < n_ap; ++k) {
            const double* ap = p->aperture + (size_t)k * n * n;
            double s0 = 0.0;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    double v = ap[(size_t)a * n + b];
                    if (!isfinite(v) || v != ap[(size_t)(n - 1 - a) * n + (n - 1 - b)]) return -1;
                    s0 += v;
                }
            if (!(s0 > 0.0)) return -1;
        }
    }
    return 0;
}

/* Predict, with the offset derivatives [n_vis][4][re, im] in dvis_out and the
 * beam-scale derivatives [n_vis][2][re, im] (antenna i, then j) in dscale_out
 * when they are not NULL. */
static int predict_impl(const orc_problem* p, const double* offsets, double* vis_out, double* dvis_out,
                        double* dscale_out)
{
    if (check_problem(p)) return -1;
    for (int s = 0; s < p->n_int; ++s) {
        int64_t r0 = p->int_row_ptr[s], r1 = p->int_row_ptr[s + 1];
        if (r0 == r1) continue; /* an empty interval predicts nothing */
        const double* offs_int = offsets + (size_t)s * p->n_pol * p->n_ant * 2;
        const double* scl_int = p->beam_scale ? p->beam_scale + (size_t)s * p->n_pol * p->n_ant : NULL;
        double* tab = p->par_angle ? NULL : beam_table(p, offs_int, scl_int);
        if (!p->par_angle && !tab) return -2;
#pragma omp parallel
        {
            double* bi = (double*)malloc(sizeof(double) * 8 * (p->n_src + 1));
            double* bj = bi + 4 * (p->n_src + 1);
#pragma omp for schedule(dynamic, 16)
            for (int64_t r = r0; r < r1; ++r) {
                for (int c = 0; c < p->n_chan; ++c) {
                    double u, v;
                    row_uv(p, r, c, &u, &v);
                    for (int pol = 0; pol < p->n_pol; ++pol) {
                        double out[14];
                        vis_row(p, tab, offs_int, scl_int, r, pol, c, u, v, row_w(p, r, c), bi, bj, out,
                                dvis_out != NULL || dscale_out != NULL);
                        size_t idx = ((size_t)r * p->n_chan + c) * p->n_pol + pol;
                        vis_out[2 * idx] = out[0];
                        vis_out[2 * idx + 1] = out[1];
                        if (dvis_out) memcpy(dvis_out + 8 * idx, out + 2, 8 * sizeof(double));
                        if (dscale_out) memcpy(dscale_out + 4 * idx, out + 10, 4 * sizeof(double));
                    }
                }
            }
            free(bi);
        }
        free(tab);
    }
    return 0;
}

int oracle_predict(const orc_problem* p, const double* offsets, double* vis_out, double* dvis_out)
{
    return predict_impl(p, offsets, vis_out, dvis_out, NULL);
}

int oracle_predict_scale(const orc_problem* p, const double* offsets, double* vis_out, double* dscale_out)
{
    return predict_impl(p, offsets, vis_out, NULL, dscale_out);
}

/*
 * The sums of Eq. DCHIDD for the beam-width scale, a generalised antenna
 * parameter (Eq. DA with a_i = sigma_i): per (interval, pol, antenna)
 * acc3[k], k = chi, g_sigma = sum Re(conj(R) w dV/dsigma_a),
 * H_sigma = sum w |dV/dsigma_a|^2, over both ends of every baseline.
 */
int oracle_scale_gradient(const orc_problem* p, const double* offsets, const double* vis_obs,
                          const double* weight, double* acc3)
{
    if (check_problem(p)) return -1;
    size_t n_vis = (size_t)p->n_row * p->n_chan * p->n_pol;
    double* vm = (double*)malloc((n_vis ? n_vis : 1) * 2 * sizeof(double));
    double* ds = (double*)malloc((n_vis ? n_vis : 1) * 4 * sizeof(double));
    if (!vm || !ds) {
        free(vm);
        free(ds);
        return -2;
    }
    int rc = predict_impl(p, offsets, vm, NULL, ds);
    memset(acc3, 0, (size_t)p->n_int * p->n_pol * p->n_ant * 3 * sizeof(double));
    for (int s = 0; s < p->n_int && rc == 0; ++s) {
        for (int64_t r = p->int_row_ptr[s]; r < p->int_row_ptr[s + 1]; ++r) {
            for (int c = 0; c < p->n_chan; ++c) {
                for (int pol = 0; pol < p->n_pol; ++pol) {
                    size_t idx = ((size_t)r * p->n_chan + c) * p->n_pol + pol;
                    double w = weight[idx];
                    double rr = vis_obs[2 * idx] - vm[2 * idx];
                    double ri = vis_obs[2 * idx + 1] - vm[2 * idx + 1];
                    for (int end = 0; end < 2; ++end) {
                        int a = end ? p->ant2[r] : p->ant1[r];
                        const double* d = ds + 4 * idx + 2 * end;
                        double* t = acc3 + (((size_t)s * p->n_pol + pol) * p->n_ant + a) * 3;
                        t[0] += w * (rr * rr + ri * ri);
                        t[1] += w * (rr * d[0] + ri * d[1]);
                        t[2] += w * (d[0] * d[0] + d[1] * d[1]);
                    }
                }
            }
        }
    }
    free(vm);
    free(ds);
    return rc;
}

/*
 * Damped Gauss-Newton step of the beam-width scale per (interval, pol,
 * antenna): sigma += gamma g_sigma / H_sigma, as the offsets' update with
 * one parameter.  An antenna with H_sigma <= 0, non-finite sums, or a step
 * that would leave sigma non-positive is left as is and marked in
 * not_updated (nullable).  max_step_out[s] (nullable) receives the largest
 * |delta sigma| of interval s.
 */
int oracle_scale_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* scale_io,
                      int32_t* not_updated, double* max_step_out)
{
    if (n_int < 0 || n_pol < 1 || n_ant < 1 || !(gain > 0.0)) return -1;
    for (int s = 0; s < n_int; ++s) {
        double mx = 0.0;
        for (int k = 0; k < n_pol * n_ant; ++k) {
            size_t i = (size_t)s * n_pol * n_ant + k;
            double g = acc3[3 * i + 1], h = acc3[3 * i + 2];
            double nxt = scale_io[i] + gain * g / h;
            int ok = h > 0.0 && isfinite(g) && isfinite(h) && isfinite(nxt) && nxt > 0.0;
            if (ok) {
                mx = fmax(mx, fabs(nxt - scale_io[i]));
                scale_io[i] = nxt;
            }
            if (not_updated) not_updated[i] = !ok;
        }
        if (max_step_out) max_step_out[s] = mx;
    }
    return 0;
}

/*
 * Per-antenna accumulation of Eq. DCHIDD for every interval and polarisation:
 * acc[((s*n_pol + pol)*n_ant + a)*6 + k], k = chi, g_l, g_m, H_ll, H_lm, H_mm.
 * Also returns the model visibilities when vis_model_out is not NULL.
 */
int oracle_gradient(const orc_problem* p, const double* offsets, const double* vis_obs,
                    const double* weight, double* acc, double* vis_model_out)
{
    if (check_problem(p)) return -1;
    size_t n_acc = (size_t)p->n_int * p->n_pol * p->n_ant * 6;
    memset(acc, 0, n_acc * sizeof(double));
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    size_t per = (size_t)p->n_pol * p->n_ant * 6;
    double* part = (double*)calloc((size_t)nthr * per, sizeof(double));
    if (!part) return -2;
    for (int s = 0; s < p->n_int; ++s) {
        int64_t r0 = p->int_row_ptr[s], r1 = p->int_row_ptr[s + 1];
        if (r0 == r1) continue; /* no samples: every sum of the interval stays 0 */
        const double* offs_int = offsets + (size_t)s * p->n_pol * p->n_ant * 2;
        const double* scl_int = p->beam_scale ? p->beam_scale + (size_t)s * p->n_pol * p->n_ant : NULL;
        double* tab = p->par_angle ? NULL : beam_table(p, offs_int, scl_int);
        if (!p->par_angle && !tab) {
            free(part);
            return -2;
        }
        memset(part, 0, (size_t)nthr * per * sizeof(double));
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* mine = part + (size_t)tid * per;
            double* bi = (double*)malloc(sizeof(double) * 8 * (p->n_src + 1));
            double* bj = bi + 4 * (p->n_src + 1);
#pragma omp for schedule(static)
            for (int64_t r = r0; r < r1; ++r) {
                int ai = p->ant1[r], aj = p->ant2[r];
                for (int c = 0; c < p->n_chan; ++c) {
                    double u, v;
                    row_uv(p, r, c, &u, &v);
                    for (int pol = 0; pol < p->n_pol; ++pol) {
                        size_t idx = ((size_t)r * p->n_chan + c) * p->n_pol + pol;
                        double out[14];
                        vis_row(p, tab, offs_int, scl_int, r, pol, c, u, v, row_w(p, r, c), bi, bj, out, 1);
                        if (vis_model_out) {
                            vis_model_out[2 * idx] = out[0];
                            vis_model_out[2 * idx + 1] = out[1];
                        }
                        double w = weight[idx];
                        double rr = vis_obs[2 * idx] - out[0];
                        double ri = vis_obs[2 * idx + 1] - out[1];
                        double chi = w * (rr * rr + ri * ri);
                        for (int end = 0; end < 2; ++end) {
                            int a = end ? aj : ai;
                            const double* dl = out + 2 + 4 * end; /* dV/dl_a */
                            const double* dm = out + 4 + 4 * end; /* dV/dm_a */
                            double* t = mine + ((size_t)pol * p->n_ant + a) * 6;
                            t[0] += chi;
                            t[1] += w * (rr * dl[0] + ri * dl[1]);
                            t[2] += w * (rr * dm[0] + ri * dm[1]);
                            t[3] += w * (dl[0] * dl[0] + dl[1] * dl[1]);
                            t[4] += w * (dl[0] * dm[0] + dl[1] * dm[1]);
                            t[5] += w * (dm[0] * dm[0] + dm[1] * dm[1]);
                        }
                    }
                }
            }
            free(bi);
        }
        double* dst = acc + (size_t)s * per;
        for (int t = 0; t < nthr; ++t)
            for (size_t k = 0; k < per; ++k) dst[k] += part[(size_t)t * per + k];
        free(tab);
    }
    free(part);
    return 0;
}

/*
 * d chi^2 / d I at each of n_pix sky positions (pix_l[k], pix_m[k]):
 *   out[k] = -2 sum w Re( conj(R) E_i(l_k - p_i) E_j(l_k - p_j) exp(+2 pi i u.l_k) ),
 * over every interval, row, channel and polarisation, R = V^Obs - V^M with
 * V^M the direct sum of Eq. ME at the given offsets.  Each term is the
 * derivative of one visibility with respect to one pixel's flux, so out is
 * exact for pixels on or off the model's support.
 */
/* The pattern of antenna a at sky position (l, m) in a row with parallactic
 * angle chi, for offsets in the mount frame: the beam centre on the sky is
 * R(chi) (q + squint), as in beam_row. */
static double beam_at_row(const orc_problem* p, const double* offs_int, const double* scl_int, int pol, int a,
                          int c, double chi, double l, double m)
{
    double sig = sigma_of(p, scl_int, pol, a);
    double lambda = ORC_C_LIGHT / p->freq_hz[c];
    double sq = (pol == 0 ? 1.0 : -1.0) * p->squint_frac * hpbw_rad(lambda, p->dish_diam_m);
    double ql = offs_int[(pol * p->n_ant + a) * 2 + 0] + sq;
    double qm = offs_int[(pol * p->n_ant + a) * 2 + 1];
    double cs = cos(chi), sn = sin(chi);
    double e[4];
    if (p->illum == 2)
        efp_scaled(p, c, a, sig, cs * l + sn * m - ql, -sn * l + cs * m - qm, e);
    else
        efp_scaled(p, c, a, sig, l - (cs * ql - sn * qm), m - (sn * ql + cs * qm), e);
    return e[0];
}

int oracle_image_gradient(const orc_problem* p, const double* offsets, const double* vis_obs,
                          const double* weight, int n_pix, const double* pix_l, const double* pix_m,
                          double* out)
{
    if (check_problem(p) || n_pix < 0) return -1;
    size_t n_vis = (size_t)p->n_row * p->n_chan * p->n_pol;
    double* vm = (double*)malloc((n_vis ? n_vis : 1) * 2 * sizeof(double));
    double* ones = (double*)malloc((n_pix ? n_pix : 1) * sizeof(double));
    if (!vm || !ones) {
        free(vm);
        free(ones);
        return -2;
    }
    int rc = oracle_predict(p, offsets, vm, NULL);
    for (int k = 0; k < n_pix; ++k) {
        out[k] = 0.0;
        ones[k] = 1.0;
    }
    /* the same problem with the requested pixels as its sky, for the beams */
    orc_problem q = *p;
    q.n_src = n_pix;
    q.src_l = pix_l;
    q.src_m = pix_m;
    q.src_flux = ones;
    for (int s = 0; s < p->n_int && rc == 0; ++s) {
        int64_t r0 = p->int_row_ptr[s], r1 = p->int_row_ptr[s + 1];
        if (r0 == r1) continue;
        const double* offs_int = offsets + (size_t)s * p->n_pol * p->n_ant * 2;
        const double* scl_int = p->beam_scale ? p->beam_scale + (size_t)s * p->n_pol * p->n_ant : NULL;
        /* sky frame: every row of the interval sees the same beams */
        double* tab = p->par_angle ? NULL : beam_table(&q, offs_int, scl_int);
        if (!p->par_angle && !tab) {
            rc = -2;
            break;
        }
#pragma omp parallel for schedule(dynamic, 4)
        for (int k = 0; k < n_pix; ++k) {
            double acc = 0.0;
            for (int64_t r = r0; r < r1; ++r) {
                int ai = p->ant1[r], aj = p->ant2[r];
                for (int c = 0; c < p->n_chan; ++c) {
                    double u, v;
                    row_uv(p, r, c, &u, &v);
                    double ph = me_phase(u, v, row_w(p, r, c), pix_l[k], pix_m[k]);
                    double cr = cos(ph), ci = sin(ph);
                    for (int pol = 0; pol < p->n_pol; ++pol) {
                        size_t idx = ((size_t)r * p->n_chan + c) * p->n_pol + pol;
                        double ei, ej;
                        if (p->par_angle) {
                            ei = beam_at_row(p, offs_int, scl_int, pol, ai, c, p->par_angle[r], pix_l[k],
                                             pix_m[k]);
                            ej = beam_at_row(p, offs_int, scl_int, pol, aj, c, p->par_angle[r], pix_l[k],
                                             pix_m[k]);
                        } else {
                            ei = tab[4 * ((((size_t)pol * p->n_ant + ai) * p->n_chan + c) * n_pix + k)];
                            ej = tab[4 * ((((size_t)pol * p->n_ant + aj) * p->n_chan + c) * n_pix + k)];
                        }
                        double rr = vis_obs[2 * idx] - vm[2 * idx];
                        double ri = vis_obs[2 * idx + 1] - vm[2 * idx + 1];
                        acc += weight[idx] * ei * ej * (rr * cr + ri * ci);
                    }
                }
            }
            out[k] += -2.0 * acc;
        }
        free(tab);
    }
    free(vm);
    free(ones);
    return rc;
}

/*
 * Damped per-antenna update.  For each (interval, pol, antenna) with sums
 * (chi, g, H), H' = H + mu diag(H) (mu >= 0, Levenberg-Marquardt damping; 0
 * is the plain Gauss-Newton step): delta = gamma H'^-1 g when H' is well
 * conditioned (det > 1e-12 tr^2), else gamma g_k / H'_kk per axis with
 * H'_kk > 0; an
 * antenna with tr H <= 0 (no unflagged data) or non-finite sums is left as is
 * and marked in not_updated.  max_step_out[s] receives the largest |delta| of
 * interval s.  Intervals whose done[s] is non-zero are skipped.
 */
int oracle_solve_step(int n_int, int n_pol, int n_ant, const double* acc, double gain, double mu,
                      double* offsets_io, int32_t* not_updated, double* max_step_out,
                      const int32_t* done)
{
    if (n_int < 1 || n_pol < 1 || n_ant < 1 || !(gain > 0.0) || !(mu >= 0.0) || !isfinite(mu)) return -1;
    for (int s = 0; s < n_int; ++s) {
        double mx = 0.0;
        for (int pol = 0; pol < n_pol; ++pol) {
            for (int a = 0; a < n_ant; ++a) {
                size_t k = ((size_t)s * n_pol + pol) * n_ant + a;
                const double* t = acc + 6 * k;
                /* Levenberg-Marquardt damping of the diagonal: H + mu diag(H) */
                double gl = t[1], gm = t[2], hll = t[3] * (1.0 + mu), hlm = t[4], hmm = t[5] * (1.0 + mu);
                int skip = (done && done[s]);
                double tr = hll + hmm;
                int bad = !(isfinite(gl) && isfinite(gm) && isfinite(hll) && isfinite(hlm) &&
                            isfinite(hmm)) || !(tr > 0.0);
                if (not_updated) not_updated[k] = (bad && !skip) ? 1 : 0;
                if (skip || bad) continue;
                double det = hll * hmm - hlm * hlm;
                double dl, dm;
                if (det > 1e-12 * tr * tr) {
                    dl = (hmm * gl - hlm * gm) / det;
                    dm = (hll * gm - hlm * gl) / det;
                } else {
                    dl = hll > 0.0 ? gl / hll : 0.0;
                    dm = hmm > 0.0 ? gm / hmm : 0.0;
                }
                dl *= gain;
                dm *= gain;
                offsets_io[2 * k] += dl;
                offsets_io[2 * k + 1] += dm;
                double st = sqrt(dl * dl + dm * dm);
                if (st > mx) mx = st;
            }
        }
        if (max_step_out) max_step_out[s] = (done && done[s]) ? 0.0 : mx;
    }
    return 0;
}

/*
 * Algorithm 1 for every interval: at most n_max iterations of
 * (accumulate at current offsets, damped update); an interval stops once its
 * largest step is below tol_rad.  iters_out[s] gets the iterations it ran.
 */
int oracle_solve(const orc_problem* p, const double* vis_obs, const double* weight,
                 double* offsets_io, double gain, int n_max, double tol_rad, int32_t* iters_out)
{
    if (check_problem(p) || n_max < 0) return -1;
    size_t n_acc = (size_t)p->n_int * p->n_pol * p->n_ant * 6;
    double* acc = (double*)malloc(n_acc * sizeof(double));
    double* mx = (double*)malloc(p->n_int * sizeof(double));
    int32_t* done = (int32_t*)calloc(p->n_int, sizeof(int32_t));
    if (!acc || !mx || !done) {
        free(acc);
        free(mx);
        free(done);
        return -2;
    }
    for (int s = 0; s < p->n_int; ++s) iters_out[s] = 0;
    int rc = 0;
    for (int it = 0; it < n_max; ++it) {
        rc = oracle_gradient(p, offsets_io, vis_obs, weight, acc, NULL);
        if (rc) break;
        rc = oracle_solve_step(p->n_int, p->n_pol, p->n_ant, acc, gain, 0.0, offsets_io, NULL, mx, done);
        if (rc) break;
        int all = 1;
        for (int s = 0; s < p->n_int; ++s) {
            if (done[s]) continue;
            iters_out[s] += 1;
            if (mx[s] < tol_rad) done[s] = 1;
            else all = 0;
        }
        if (all) break;
    }
    free(acc);
    free(mx);
    free(done);
    return rc;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Aperture phase term: defocus, a complex generalised antenna parameter.   */
/* ------------------------------------------------------------------------ */
/*
 * Eq. DA holds for any antenna parameter a_i, complex patterns included, and
 * Sec. 5.3 names phase terms of the aperture illumination (defocus,
 * astigmatism) as the first shape parameters to solve for with the same
 * machinery.  A defocus delta (radians of aperture phase at the rim)
 * multiplies the illumination by exp(i delta (r/R)^2), R = D/2, and the
 * far-field pattern becomes complex:
 *   uniform disc:  E(rho; delta) = 2 int_0^1 J0(k rho t) exp(i delta t^2) t dt,
 *                  k = pi D / lambda, so that E = 2 J1(x)/x, x = k rho, at
 *                  delta = 0 (a Hankel transform of order zero);
 *   Gaussian mode: the illumination exp(-2 pi^2 s^2 |x|^2 / lambda^2) of the
 *                  pattern exp(-rho^2/(2 s^2)), s = gauss_sigma_ld lambda/D,
 *                  times the phase, transforms in closed form:
 *                  E = z exp(-z rho^2 / (2 s^2)), z = 1 / (1 - i kappa),
 *                  kappa = 2 delta / (pi^2 gauss_sigma_ld^2)
 *                  (frequency-independent, since s and R both scale with D).
 * The visibility carries the first antenna's pattern and the conjugate of the
 * second's (Eq. ME: E_i E_j^*), which real patterns do not show:
 *   V_ij = sum_p I_p E_i(l_p - p_i) conj(E_j(l_p - p_j)) exp(+2 pi i u.l_p).
 * dV/ddelta_i takes dE_i/ddelta in place of E_i; dV/ddelta_j takes
 * conj(dE_j/ddelta) in place of conj(E_j).
 */

/* Gauss-Legendre nodes and weights on [0, 1]: Newton's method on P_n from
 * the Chebyshev-like first guesses cos(pi (i + 3/4) / (n + 1/2)). */
#define ORC_NGL 128
static double g_gl_t[ORC_NGL], g_gl_w[ORC_NGL];
static int g_gl_ready = 0;
static void gl_nodes(void)
{
    if (g_gl_ready) return;
    const int n = ORC_NGL;
    for (int i = 0; i < n; ++i) {
        double x = cos(ORC_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        g_gl_t[i] = 0.5 * (1.0 - x);
        g_gl_w[i] = 1.0 / ((1.0 - x * x) * dp * dp);  /* 2/((1-x^2) P'^2), halved for [0, 1] */
    }
    g_gl_ready = 1;
}

/* Pattern with defocus delta at displacement (dl, dm) from the beam centre:
 * out4 = (Re E, Im E, Re dE/ddelta, Im dE/ddelta). */
static void efp_defocus(int illum, double dish, double sigma_ld, double lambda, double delta, double dl,
                        double dm, double* out4)
{
    double rho2 = dl * dl + dm * dm;
    if (illum == 1) {
        double s = sigma_ld * lambda / dish;
        double kap = 2.0 * delta / (ORC_PI * ORC_PI * sigma_ld * sigma_ld);
        /* z = 1/(1 - i kappa) = (1 + i kappa)/(1 + kappa^2) */
        double den = 1.0 + kap * kap, zr = 1.0 / den, zi = kap / den;
        double a = rho2 / (2.0 * s * s);
        /* E = z exp(-a z) */
        double mag = exp(-a * zr), ph = -a * zi;
        double er = mag * cos(ph), ei = mag * sin(ph);
        double Er = zr * er - zi * ei, Ei = zr * ei + zi * er;
        /* dE/dkappa = i z E (1 - a z) */
        double tr = 1.0 - a * zr, ti = -a * zi;           /* 1 - a z */
        double ur = zr * Er - zi * Ei, ui = zr * Ei + zi * Er; /* z E */
        double vr = ur * tr - ui * ti, vi = ur * ti + ui * tr; /* z E (1 - a z) */
        double dk = 2.0 / (ORC_PI * ORC_PI * sigma_ld * sigma_ld);
        out4[0] = Er;
        out4[1] = Ei;
        out4[2] = -vi * dk; /* i (vr + i vi) = -vi + i vr */
        out4[3] = vr * dk;
        return;
    }
    gl_nodes();
    double x = ORC_PI * dish / lambda * sqrt(rho2);
    double er = 0.0, ei = 0.0, dr = 0.0, di = 0.0;
    for (int q = 0; q < ORC_NGL; ++q) {
        double t = g_gl_t[q], w = 2.0 * g_gl_w[q] * t * j0(x * t);
        double c = cos(delta * t * t), sn = sin(delta * t * t);
        er += w * c;
        ei += w * sn;
        /* d/ddelta of exp(i delta t^2) = i t^2 exp(i delta t^2) */
        dr -= w * t * t * sn;
        di += w * t * t * c;
    }
    out4[0] = er;
    out4[1] = ei;
    out4[2] = dr;
    out4[3] = di;
}

void oracle_efp_defocus(int illum, double dish_diam_m, double gauss_sigma_ld, double freq_hz, double delta,
                        double dl, double dm, double* out4)
{
    efp_defocus(illum, dish_diam_m, gauss_sigma_ld, ORC_C_LIGHT / freq_hz, delta, dl, dm, out4);
}

static int check_defocus(const orc_problem* p, const double* defocus)
{
    gl_nodes(); /* before any parallel region reads them */
    if (check_problem(p) || p->illum == 2 || p->par_angle || p->beam_scale || !defocus) return -1;
    for (size_t k = 0; k < (size_t)p->n_int * p->n_pol * p->n_ant; ++k)
        if (!isfinite(defocus[k])) return -1;
    return 0;
}

/* V [n_vis][re, im] and, when ddef_out is not NULL, dV/ddelta_i and
 * dV/ddelta_j [n_vis][2][re, im] with every antenna's defocus
 * [n_int][n_pol][n_ant] (sky-frame offsets). */
int oracle_predict_defocus(const orc_problem* p, const double* offsets, const double* defocus, double* vis_out,
                           double* ddef_out)
{
    if (check_defocus(p, defocus)) return -1;
    for (int s = 0; s < p->n_int; ++s) {
        int64_t r0 = p->int_row_ptr[s], r1 = p->int_row_ptr[s + 1];
        if (r0 == r1) continue;
        const double* offs_int = offsets + (size_t)s * p->n_pol * p->n_ant * 2;
        const double* def_int = defocus + (size_t)s * p->n_pol * p->n_ant;
        /* beams: tab[((pol * n_ant + a) * n_chan + c) * n_src + src][4] */
        size_t nt = (size_t)p->n_pol * p->n_ant * p->n_chan * p->n_src;
        double* tab = (double*)malloc((nt ? nt : 1) * 4 * sizeof(double));
        if (!tab) return -2;
        for (int pol = 0; pol < p->n_pol; ++pol) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int a = 0; a < p->n_ant; ++a) {
                for (int c = 0; c < p->n_chan; ++c) {
                    double lambda = ORC_C_LIGHT / p->freq_hz[c];
                    double sq = (pol == 0 ? 1.0 : -1.0) * p->squint_frac * hpbw_rad(lambda, p->dish_diam_m);
                    double pl = offs_int[(pol * p->n_ant + a) * 2 + 0] + sq;
                    double pm = offs_int[(pol * p->n_ant + a) * 2 + 1];
                    for (int k = 0; k < p->n_src; ++k)
                        efp_defocus(p->illum, p->dish_diam_m, p->gauss_sigma_ld, lambda,
                                    def_int[pol * p->n_ant + a], p->src_l[k] - pl, p->src_m[k] - pm,
                                    tab + 4 * ((((size_t)pol * p->n_ant + a) * p->n_chan + c) * p->n_src + k));
                }
            }
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t r = r0; r < r1; ++r) {
            for (int c = 0; c < p->n_chan; ++c) {
                double u, v;
                row_uv(p, r, c, &u, &v);
                double w = row_w(p, r, c);
                for (int pol = 0; pol < p->n_pol; ++pol) {
                    const double* ti = tab + 4 * ((((size_t)pol * p->n_ant + p->ant1[r]) * p->n_chan + c) * p->n_src);
                    const double* tj = tab + 4 * ((((size_t)pol * p->n_ant + p->ant2[r]) * p->n_chan + c) * p->n_src);
                    double acc[6] = {0};
                    for (int k = 0; k < p->n_src; ++k) {
                        double ph = me_phase(u, v, w, p->src_l[k], p->src_m[k]);
                        double fr = p->src_flux[k] * cos(ph), fi = p->src_flux[k] * sin(ph);
                        const double* a = ti + 4 * k;
                        const double* b = tj + 4 * k;
                        /* E_i conj(E_j), dE_i conj(E_j), E_i conj(dE_j) */
                        double pr[3], pi_[3];
                        pr[0] = a[0] * b[0] + a[1] * b[1];
                        pi_[0] = a[1] * b[0] - a[0] * b[1];
                        pr[1] = a[2] * b[0] + a[3] * b[1];
                        pi_[1] = a[3] * b[0] - a[2] * b[1];
                        pr[2] = a[0] * b[2] + a[1] * b[3];
                        pi_[2] = a[1] * b[2] - a[0] * b[3];
                        for (int q = 0; q < 3; ++q) {
                            acc[2 * q] += fr * pr[q] - fi * pi_[q];
                            acc[2 * q + 1] += fr * pi_[q] + fi * pr[q];
                        }
                    }
                    size_t idx = ((size_t)r * p->n_chan + c) * p->n_pol + pol;
                    vis_out[2 * idx] = acc[0];
                    vis_out[2 * idx + 1] = acc[1];
                    if (ddef_out) memcpy(ddef_out + 4 * idx, acc + 2, 4 * sizeof(double));
                }
            }
        }
        free(tab);
    }
    return 0;
}

/* The sums of Eq. DCHIDD for the defocus: per (interval, pol, antenna)
 * acc3 = (chi, g = sum Re(conj(R) w dV/ddelta_a), H = sum w |dV/ddelta_a|^2)
 * over both ends of every baseline. */
int oracle_defocus_gradient(const orc_problem* p, const double* offsets, const double* defocus,
                            const double* vis_obs, const double* weight, double* acc3)
{
    if (check_defocus(p, defocus)) return -1;
    size_t n_vis = (size_t)p->n_row * p->n_chan * p->n_pol;
    double* vm = (double*)malloc((n_vis ? n_vis : 1) * 2 * sizeof(double));
    double* dd = (double*)malloc((n_vis ? n_vis : 1) * 4 * sizeof(double));
    if (!vm || !dd) {
        free(vm);
        free(dd);
        return -2;
    }
    int rc = oracle_predict_defocus(p, offsets, defocus, vm, dd);
    memset(acc3, 0, (size_t)p->n_int * p->n_pol * p->n_ant * 3 * sizeof(double));
    for (int s = 0; s < p->n_int && rc == 0; ++s) {
        for (int64_t r = p->int_row_ptr[s]; r < p->int_row_ptr[s + 1]; ++r) {
            for (int c = 0; c < p->n_chan; ++c) {
                for (int pol = 0; pol < p->n_pol; ++pol) {
                    size_t idx = ((size_t)r * p->n_chan + c) * p->n_pol + pol;
                    double w = weight[idx];
                    double rr = vis_obs[2 * idx] - vm[2 * idx];
                    double ri = vis_obs[2 * idx + 1] - vm[2 * idx + 1];
                    for (int end = 0; end < 2; ++end) {
                        int a = end ? p->ant2[r] : p->ant1[r];
                        const double* d = dd + 4 * idx + 2 * end;
                        double* t = acc3 + (((size_t)s * p->n_pol + pol) * p->n_ant + a) * 3;
                        t[0] += w * (rr * rr + ri * ri);
                        t[1] += w * (rr * d[0] + ri * d[1]);
                        t[2] += w * (d[0] * d[0] + d[1] * d[1]);
                    }
                }
            }
        }
    }
    free(vm);
    free(dd);
    return rc;
}

/* Damped Gauss-Newton step of the defocus per (interval, pol, antenna):
 * delta += gamma g / H; an antenna with H <= 0 or non-finite sums is left
 * as is and marked in not_updated (nullable); max_step_out[s] (nullable) is
 * the largest |delta step| of interval s. */
int oracle_defocus_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* defocus_io,
                        int32_t* not_updated, double* max_step_out)
{
    if (n_int < 0 || n_pol < 1 || n_ant < 1 || !(gain > 0.0)) return -1;
    for (int s = 0; s < n_int; ++s) {
        double mx = 0.0;
        for (int k = 0; k < n_pol * n_ant; ++k) {
            size_t i = (size_t)s * n_pol * n_ant + k;
            double g = acc3[3 * i + 1], h = acc3[3 * i + 2];
            double step = gain * g / h;
            int ok = h > 0.0 && isfinite(g) && isfinite(h) && isfinite(step);
            if (ok) {
                mx = fmax(mx, fabs(step));
                defocus_io[i] += step;
            }
            if (not_updated) not_updated[i] = !ok;
        }
        if (max_step_out) max_step_out[s] = mx;
    }
    return 0;
}
