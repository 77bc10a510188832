/*
 * psc_oracle.h -- interface of the FP64 direct-summation oracle.
 * TEST INFRASTRUCTURE ONLY; see psc_oracle.c.  Host pointers throughout.
 */
#ifndef PSC_ORACLE_H
#define PSC_ORACLE_H
#include <stdint.h>

typedef struct {
    /* sky: non-zero pixels of the model image (direction cosines, Jy) */
    int32_t n_src;
    const double* src_l;
    const double* src_m;
    const double* src_flux;
    /* array and data layout */
    int32_t n_ant, n_chan, n_pol, n_int;
    int64_t n_row;
    const int64_t* int_row_ptr; /* [n_int+1] rows of interval s: [ptr[s], ptr[s+1]) */
    const int32_t* ant1;        /* [n_row] */
    const int32_t* ant2;        /* [n_row] */
    const double* uv_m;         /* [n_row][2] baseline (u,v) in metres */
    const double* freq_hz;      /* [n_chan] */
    /* antenna model */
    double dish_diam_m;
    int32_t illum;          /* 0 = uniform circular (Airy), 1 = Gaussian main lobe,
                               2 = measured aperture (below) */
    double gauss_sigma_ld;  /* Gaussian mode: sigma of E in units of lambda/D */
    double squint_frac;     /* beam squint of pol 0 (+) and pol 1 (-), in HPBW */
    double snap_scale;      /* >0: uv (wavelengths) rounded to multiples of 1/snap_scale */
    const double* par_angle; /* nullable [n_row]: offsets in the mount frame, rotated by this angle */
    const double* w_m;       /* nullable [n_row]: baseline w in metres (the w-term); null: w = 0 */
    /* illum 2: aperture illumination on aperture_n x aperture_n cells over the
     * square of side D centred on the dish axis, [x][y] row-major (x along
     * the mount frame's l axis), real and even: A[a][b] = A[n-1-a][n-1-b].
     * A heterogeneous array stacks n_apertures of them, [n_apertures][n][n],
     * and ant_aperture (nullable [n_ant]) names each antenna's (null: all
     * antennas take the first; n_apertures 0 counts as 1) */
    int32_t aperture_n;
    const double* aperture;
    int32_t n_apertures;
    const int32_t* ant_aperture;
    /* nullable [n_int][n_pol][n_ant]: beam-width scale sigma > 0 of each
     * antenna, E = E0(d / sigma) (null: 1) */
    const double* beam_scale;
} orc_problem;

void oracle_efp(int illum, double dish_diam_m, double gauss_sigma_ld, double freq_hz,
                double dl, double dm, double* out3);
void oracle_efp_aperture(int aperture_n, const double* aperture, double dish_diam_m, double freq_hz,
                         double dl, double dm, double* out3);
double oracle_hpbw(double freq_hz, double dish_diam_m);
void oracle_snap_uv(const orc_problem* p, int64_t row, int chan, double* uv_out);
int oracle_predict(const orc_problem* p, const double* offsets, double* vis_out, double* dvis_out);
int oracle_predict_scale(const orc_problem* p, const double* offsets, double* vis_out, double* dscale_out);
int oracle_scale_gradient(const orc_problem* p, const double* offsets, const double* vis_obs,
                          const double* weight, double* acc3);
int oracle_scale_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* scale_io,
                      int32_t* not_updated, double* max_step_out);
int oracle_gradient(const orc_problem* p, const double* offsets, const double* vis_obs,
                    const double* weight, double* acc, double* vis_model_out);
int oracle_image_gradient(const orc_problem* p, const double* offsets, const double* vis_obs,
                          const double* weight, int n_pix, const double* pix_l, const double* pix_m,
                          double* out);
int oracle_solve_step(int n_int, int n_pol, int n_ant, const double* acc, double gain, double mu,
                      double* offsets_io, int32_t* not_updated, double* max_step_out,
                      const int32_t* done);
int oracle_solve(const orc_problem* p, const double* vis_obs, const double* weight,
                 double* offsets_io, double gain, int n_max, double tol_rad, int32_t* iters_out);
/* Aperture phase term (defocus delta per [n_int][n_pol][n_ant], radians of
 * phase at the dish rim): complex patterns; illum 0 or 1, sky-frame
 * offsets, no beam scales.  out4 = (Re E, Im E, Re dE/ddelta, Im dE/ddelta);
 * ddef_out [n_vis][2][re, im] = dV/ddelta_i, dV/ddelta_j; acc3 = (chi, g, H). */
void oracle_efp_defocus(int illum, double dish_diam_m, double gauss_sigma_ld, double freq_hz, double delta,
                        double dl, double dm, double* out4);
int oracle_predict_defocus(const orc_problem* p, const double* offsets, const double* defocus, double* vis_out,
                           double* ddef_out);
int oracle_defocus_gradient(const orc_problem* p, const double* offsets, const double* defocus,
                            const double* vis_obs, const double* weight, double* acc3);
int oracle_defocus_step(int n_int, int n_pol, int n_ant, const double* acc3, double gain, double* defocus_io,
                        int32_t* not_updated, double* max_step_out);
int oracle_num_threads(void);

#endif
