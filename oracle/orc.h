/*
 * orc.h -- plain, slow, FP64 CPU oracle of the boosted-frame PIC step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path.
 *
 * What it computes (paper sections / equations in brackets):
 *   - Maxwell curl equations with electron and ion currents [sec. 1, Eq. Max1,
 *     Max2], on a Yee grid in normalised units (c = 1, cell edge = 1);
 *   - charge-conserving current weighting [sec. 1, Eq. Max3, Max4], here
 *     Esirkepov's scheme with quadratic B-spline shapes;
 *   - leap-frog relativistic push [sec. 1, text after Eq. Vprime], Boris or Vay;
 *   - Lorentz transform of the lab-defined beam [sec. 1, Eq. Lor1, Lor2,
 *     RRFVel, BGauss, Belon], of the undulator field [Eq. M1-M4] and of the
 *     plasma density [Eq. Nnormi]; lab elements drift at -c beta_R [Eq. Vprime];
 *   - moving window, absorbing z faces, beam particles dropped outside the
 *     window, plasma entering at the front and leaving at the back, ion
 *     current computed directly [sec. 1, last paragraphs]: immobile ions as
 *     rigid lattice sheets, or mobile ions as a species of their own on the
 *     electrons' lattice with the same shape;
 *   - diagnostics (beam moments, bunching factor, Gauss residual);
 *   - the exact discrete adjoint of one step (not in the paper; used to pin
 *     gradients of the final bunching factor w.r.t. undulator K and density).
 *
 * Compiled twice from the same source: with real == double (liborc.so) and
 * with real == double _Complex (liborc_cs.so, -DORC_CSTEP) for complex-step
 * derivatives; in the complex build every discrete decision uses the real part.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef ORC_CSTEP
#include <complex.h>
typedef double _Complex real;
#else
typedef double real;
#endif

typedef struct {
    int32_t nx, ny, nz, bc_z;      /* bc_z: 0 open z + moving window, 1 periodic z (closed-form tests) */
    double dx_m, cfl, dt_override; /* dt_override > 0 replaces cfl/sqrt(3) */
    double gamma_boost, window_beta; /* window_beta < 0: mean beam beta_z at t'=0 */
    int64_t n_beam;
    double charge_C, gamma_lab, espread, sigma[3], emit[2], zc_cells;
    double n0_cm3, pl_z0_m, pl_len_m, pl_ramp_m; /* pl_len_m <= 0: uniform */
    int32_t ppc[3], ions;          /* ions: 0 none, 1 immobile, 2 mobile (species 2, mass ion_mass) */
    int32_t und_kind, pusher;      /* und: 0 none 1 helical 2 planar; pusher: 0 Boris 1 Vay */
    double K, lu_m, und_z0_m, und_len_m, und_ramp_periods;
    double hK, hn0;                /* complex-step: imaginary parts added to K and n0 (cs build only) */
    double ion_mass;               /* mobile ions: mass in electron masses (<= 0: the proton's) */
} orc_config;

typedef struct {
    double dt, gR, bR, uR, bw, nref_m3, wbeam, ku, B0, n0n, zoff, F_elong, sig_zlab;
    int64_t k0, step, n_beam, n_plasma, sheet_lo, sheet_hi, beam_lost, plasma_removed;
    int64_t n_ions; /* mobile ion slots (n_plasma counts electron slots) */
    double ion_mass;
    double window_x; /* window position (cells) at the current time */
} orc_info_t;

typedef struct {
    double t, n_beam_alive, wsum;
    double mean[3], sigma[3], umean[3], usigma[3], emit[2];
    double b1_re, b1_im, b2_re, b2_im, b1_abs, b2_abs;
    double field_energy, kin_beam, kin_plasma;
} orc_diag_t;

typedef struct orc_sim orc_sim;

/* lifecycle: normals = 6*n_beam standard normals (rows x, y, z, ux, uy, energy) */
orc_sim *orc_new(const orc_config *c, const double *normals);
void orc_free(orc_sim *s);
void orc_step(orc_sim *s, int32_t n);
void orc_set_window_beta(orc_sim *s, double beta); /* window speed from now on */
void orc_info(const orc_sim *s, orc_info_t *out);
void orc_diag(orc_sim *s, double kb, orc_diag_t *out);

/* array access: which = 0..8 -> Ex Ey Ez Bx By Bz Jx Jy Jz (logical window order i + nx(j + ny l)) */
real *orc_field(orc_sim *s, int32_t which);
/* species 0 beam, 1 plasma electrons, 2 mobile ions; which 0..2 position, 3..5 momentum, 6 weight */
real *orc_particles(orc_sim *s, int32_t species, int32_t which);
int32_t *orc_alive(orc_sim *s, int32_t species);

/* component routines (closed-form pins) */
real orc_shape(real d);
real orc_dshape(real d);
void orc_push(int32_t pusher, double qm, double dt, const real u[3], const real E[3], const real B[3], real out[3]);
void orc_gather(const orc_sim *s, const real X[3], real E[3], real B[3]); /* grid only, no external field */
void orc_ext_field(const orc_sim *s, real z, double t, real E[3], real B[3]);
void orc_deposit(orc_sim *s, const real X0[3], const real X1[3], real qw); /* adds into J */
void orc_ion_current(orc_sim *s, double t0, double t1, int32_t unit_weight); /* adds ion J_z into J */
void orc_b_half(orc_sim *s);
void orc_e_update(orc_sim *s);
void orc_rho(orc_sim *s, int32_t mask, real *rho);   /* mask: 1 beam, 2 plasma electrons, 4 ions, 8 neutraliser */
/* neutralising charge -rho (node charge of the window at its current origin) faded linearly over
 * fade_s seconds (boosted frame), removed by the current -E d/dt(fade), E its field (div E = rho) */
void orc_set_fading_charge(orc_sim *s, const real *rho, const real *Ex, const real *Ey, const real *Ez,
                           double fade_s);
void orc_gauss(orc_sim *s, real *r);                 /* r = div E - rho on every node */
void orc_zero_J(orc_sim *s);

/* frame helpers from the paper's section 1 */
double orc_beta(double gamma);
double orc_elongation(double gamma_beam, double gamma_frame);
double orc_fel_wavelength(double lu, double K, double gamma_beam);
double orc_doppler(double lam, double gamma_frame);
void orc_lab_to_boosted(double gR, const double lab[4], const double ulab[3], double out[4], double uout[3]);

/* adjoint */
int64_t orc_state_len(const orc_sim *s);
void orc_get_state(const orc_sim *s, real *v);
void orc_set_state(orc_sim *s, const real *v);
real orc_seed_bunching(orc_sim *s, double kb, real *lam);
void orc_adjoint_step(orc_sim *s, const real *lam_in, real *lam_out, real *gK_log, real *gn_log);
void orc_grad_bunching(const orc_config *c, const double *normals, int32_t nsteps, double kb, double out[3]);
void orc_loss_bunching(const orc_config *c, const double *normals, int32_t nsteps, double kb, double out[2]);

#endif
