/*
 * orc.c -- plain FP64 CPU oracle of the boosted-frame (relativistic reference
 * frame) PIC step.  TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg; never by the product.
 *
 * Normalised units: length = cell edge D (boosted frame, cubic), time = D/c,
 * momentum u = gamma*beta, E in m c^2/(e D), B in m c/(e D), density in
 * n_ref = eps0 m c^2/(e^2 D^2).  The paper's Gaussian-unit Maxwell system
 * [sec. 1, Eq. Max1-Max4] becomes dE/dt = curl B - J, dB/dt = -curl E,
 * div E = rho, du/dt = (q/m)(E + v x B) with q/m = -1 for electrons.
 *
 * The code favours the obvious over the fast: every stencil is a plain loop
 * over its nodes, fields move physically when the window shifts, particles
 * are never reordered (removed ones are flagged), and the adjoint is the
 * step written backwards one sub-operation at a time.
 */
#include "orc.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_CSTEP
#define RE(a) creal(a)
#define RSQRT(a) csqrt(a)
#define RSIN(a) csin(a)
#define RCOS(a) ccos(a)
#else
#define RE(a) (a)
#define RSQRT(a) sqrt(a)
#define RSIN(a) sin(a)
#define RCOS(a) cos(a)
#endif

/* CODATA 2018 */
#define C_LIGHT 299792458.0
#define Q_E 1.602176634e-19
#define M_E 9.1093837015e-31
#define EPS0 8.8541878128e-12
#define PI_D 3.14159265358979323846
#define MP_OVER_ME 1836.15267343 /* proton / electron mass (CODATA 2018) */

typedef struct {
    real *x[3], *u[3], *w;
    int32_t *alive;
    int64_t n, cap;
} orc_sp;

struct orc_sim {
    orc_config c;
    int nx, ny, nz, periodic_z;
    int64_t nc;
    double dt, gR, bR, uR, bw, nref, zoff;
    double win_x0, win_t0; /* window position at time t: win_x0 + bw (t - win_t0) (cells) */
    /* neutralising charge of the beam at t' = 0, faded linearly over fc_T (section 3):
     * charge -fc_rho f(t), f = max(0, 1 - t / fc_T), carried off by the current -fc_E f'(t),
     * fc_E the field of the beam's charge (div fc_E = fc_rho); absolute planes from fc_k0 */
    real *fc_rho, *fc_E[3];
    double fc_T;
    int64_t fc_k0;
    double ku, z0u, Lu, Ru;      /* undulator (lab cells) */
    double z0p, Lp, Rp;          /* plasma (lab cells) */
    double F, sig_zlab;
    real K, n0n, wbeam, B0;
    real *E[3], *B[3], *J[3];
    int64_t k0, step, sh_lo, sh_hi, beam_lost, plasma_removed;
    /* species 0 beam electrons, 1 plasma electrons, 2 mobile plasma ions
     * (ions == 2): charge and mass in units of e and m_e */
    orc_sp sp[3];
    double q[3], m[3];
};

/* ------------------------------------------------------------------ */
/* frame helpers [sec. 1]                                               */
/* ------------------------------------------------------------------ */

/* Eq. RRFVel / Eq. beta: beta = sqrt(1 - 1/gamma^2) */
double orc_beta(double g) { return sqrt(1.0 - 1.0 / (g * g)); }

/* Eq. Belon: sigma' / sigma = gamma_B / (gamma_B gamma_R - sqrt(gamma_B^2-1) sqrt(gamma_R^2-1)) */
double orc_elongation(double gB, double gR) {
    return gB / (gB * gR - sqrt(gB * gB - 1.0) * sqrt(gR * gR - 1.0));
}

/* Eq. RadLambda: lambda_l = lambda_u (1 + K^2/2) / (2 gamma_B^2) */
double orc_fel_wavelength(double lu, double K, double gB) { return lu * (1.0 + 0.5 * K * K) / (2.0 * gB * gB); }

/* Eq. Uelon: lambda' = lambda sqrt((1 + beta_R)/(1 - beta_R)) */
double orc_doppler(double lam, double gR) {
    double b = orc_beta(gR);
    return lam * sqrt((1.0 + b) / (1.0 - b));
}

/* Eq. Lor1, Lor2 for an event (x, y, z, t) and the momentum boost of a particle:
 * z' = gR (z - bR t), t' = gR (t - bR z); u'_z = gR (u_z - bR gamma), gamma' = gR (gamma - bR u_z). */
void orc_lab_to_boosted(double gR, const double lab[4], const double ulab[3], double out[4], double uout[3]) {
    double bR = orc_beta(gR);
    double g = sqrt(1.0 + ulab[0] * ulab[0] + ulab[1] * ulab[1] + ulab[2] * ulab[2]);
    out[0] = lab[0];
    out[1] = lab[1];
    out[2] = gR * (lab[2] - bR * lab[3]);
    out[3] = gR * (lab[3] - bR * lab[2]);
    uout[0] = ulab[0];
    uout[1] = ulab[1];
    uout[2] = gR * (ulab[2] - bR * g);
}

/* ------------------------------------------------------------------ */
/* shapes: quadratic B-spline and its derivative                        */
/* ------------------------------------------------------------------ */
real orc_shape(real d) {
    double a = fabs(RE(d));
    if (a <= 0.5) return 0.75 - d * d;
    if (a < 1.5) {
        real t = 1.5 - (RE(d) >= 0 ? d : -d);
        return 0.5 * t * t;
    }
    return 0.0;
}

real orc_dshape(real d) {
    double a = fabs(RE(d));
    if (a <= 0.5) return -2.0 * d;
    if (a < 1.5) return RE(d) >= 0 ? -(1.5 - d) : (1.5 + d);
    return 0.0;
}

/* ------------------------------------------------------------------ */
/* indexing                                                             */
/* ------------------------------------------------------------------ */
static void die(const char *m) {
    fprintf(stderr, "oracle: %s\n", m);
    abort();
}

static int wrapi(int64_t i, int n) {
    int64_t r = i % n;
    return (int)(r < 0 ? r + n : r);
}

/* field index of node (i, j, k): i, j periodic; k absolute plane -> logical window plane */
static int64_t fidx(const orc_sim *s, int64_t i, int64_t j, int64_t k) {
    int64_t l;
    if (s->periodic_z)
        l = wrapi(k, s->nz);
    else {
        l = k - s->k0;
        if (l < 0 || l >= s->nz) die("stencil outside the window");
    }
    return wrapi(i, s->nx) + (int64_t)s->nx * (wrapi(j, s->ny) + (int64_t)s->ny * l);
}

static int64_t lidx(const orc_sim *s, int i, int j, int l) {
    return wrapi(i, s->nx) + (int64_t)s->nx * (wrapi(j, s->ny) + (int64_t)s->ny * wrapi(l, s->nz));
}

/* staggering of the Yee components: Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2),
 * Bx(i,j+1/2,k+1/2) By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k) */
static const double STAG_E[3][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
static const double STAG_B[3][3] = {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

/* ------------------------------------------------------------------ */
/* lab profiles                                                         */
/* ------------------------------------------------------------------ */

/* plasma longitudinal lab profile in [0,1]: linear up-ramp then flat, zero outside */
static double plasma_profile(const orc_sim *s, double zl) {
    if (s->Lp <= 0) return 1.0;
    double a = zl - s->z0p;
    if (a < 0 || a >= s->Lp) return 0.0;
    if (s->Rp > 0 && a < s->Rp) return a / s->Rp;
    return 1.0;
}

/* undulator envelope and its derivative in the lab coordinate a = z_lab - z_start:
 * linear entrance ramp over Ru, symmetric exit ramp, zero outside [0, Lu] */
static void und_envelope(const orc_sim *s, real a, real *env, real *denv) {
    double ar = RE(a);
    *env = 0.0;
    *denv = 0.0;
    if (ar < 0 || ar > s->Lu) return;
    if (s->Ru <= 0) {
        *env = 1.0;
        return;
    }
    double up = ar / s->Ru, dn = (s->Lu - ar) / s->Ru;
    if (up < 1.0 && up <= dn) {
        *env = a / s->Ru;
        *denv = 1.0 / s->Ru;
    } else if (dn < 1.0) {
        *env = (s->Lu - a) / s->Ru;
        *denv = -1.0 / s->Ru;
    } else
        *env = 1.0;
}

/* sheet l of the plasma lattice: boosted position at time t (lab-static -> drifts at -beta_R, Eq. Vprime) */
static double sheet_z(const orc_sim *s, int64_t l, double t) {
    return ((double)l + 0.5) / s->c.ppc[2] - s->bR * t;
}

/* lab position of a boosted point: inverse of Eq. Lor1 with t' -> z = gR (z' + bR t') */
static double zlab_of(const orc_sim *s, double zb, double t) { return s->gR * (zb - s->zoff + s->bR * t); }

/* per-particle weight of sheet l: density gR n(z_lab) [Eq. Nnormi] split over the lattice */
static real sheet_weight(const orc_sim *s, int64_t l) {
    double prof = plasma_profile(s, zlab_of(s, sheet_z(s, l, 0.0), 0.0));
    int ptot = s->c.ppc[0] * s->c.ppc[1] * s->c.ppc[2];
    return s->gR * s->n0n * prof / ptot;
}

/* ------------------------------------------------------------------ */
/* external undulator field in the boosted frame [Eq. M1-M4]            */
/* ------------------------------------------------------------------ */

/* Lab field B = B0 env (cos phi, sin phi, 0) (helical) or (0, sin phi, 0) (planar),
 * phi = k_u (z_lab - z_start), no lab E.  Boosted: B'_perp = gR B_perp,
 * E'_perp = gR (v_frame x B) = gR bR (zhat x B), parallel components unchanged (zero). */
static void ext_field_d(const orc_sim *s, real z, double t, real E[3], real B[3], real dE[3], real dB[3]) {
    for (int d = 0; d < 3; ++d) E[d] = B[d] = dE[d] = dB[d] = 0.0;
    if (s->c.und_kind == 0) return;
    real a = s->gR * (z - s->zoff + s->bR * t) - s->z0u;
    real env, denv;
    und_envelope(s, a, &env, &denv);
    real ph = s->ku * a, c = RCOS(ph), sn = RSIN(ph);
    real bx, by, dbx, dby; /* lab field and d/da */
    if (s->c.und_kind == 1) {
        bx = s->B0 * env * c;
        by = s->B0 * env * sn;
        dbx = s->B0 * (denv * c - env * s->ku * sn);
        dby = s->B0 * (denv * sn + env * s->ku * c);
    } else {
        bx = 0.0;
        dbx = 0.0;
        by = s->B0 * env * sn;
        dby = s->B0 * (denv * sn + env * s->ku * c);
    }
    double ge = s->gR * s->bR;
    E[0] = -ge * by;
    E[1] = ge * bx;
    B[0] = s->gR * bx;
    B[1] = s->gR * by;
    /* da/dz = gR */
    dE[0] = -ge * s->gR * dby;
    dE[1] = ge * s->gR * dbx;
    dB[0] = s->gR * s->gR * dbx;
    dB[1] = s->gR * s->gR * dby;
}

void orc_ext_field(const orc_sim *s, real z, double t, real E[3], real B[3]) {
    real dE[3], dB[3];
    ext_field_d(s, z, t, E, B, dE, dB);
}

/* ------------------------------------------------------------------ */
/* gather: each component with the quadratic shape at its own Yee site  */
/* ------------------------------------------------------------------ */
static real interp(const orc_sim *s, const real *F, const real X[3], const double off[3]) {
    int64_t lo[3];
    for (int d = 0; d < 3; ++d) lo[d] = (int64_t)floor(RE(X[d]) - off[d] + 0.5) - 1;
    real sum = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                int64_t i = lo[0] + a, j = lo[1] + b, k = lo[2] + c;
                real wt = orc_shape(X[0] - (i + off[0])) * orc_shape(X[1] - (j + off[1])) *
                          orc_shape(X[2] - (k + off[2]));
                sum += wt * F[fidx(s, i, j, k)];
            }
    return sum;
}

void orc_gather(const orc_sim *s, const real X[3], real E[3], real B[3]) {
    for (int c = 0; c < 3; ++c) {
        E[c] = interp(s, s->E[c], X, STAG_E[c]);
        B[c] = interp(s, s->B[c], X, STAG_B[c]);
    }
}

/* ------------------------------------------------------------------ */
/* leap-frog pushers                                                    */
/* ------------------------------------------------------------------ */
static real dot3(const real a[3], const real b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const real a[3], const real b[3], real o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Boris (1970): half electric kick, magnetic rotation, half electric kick. */
static void push_boris(double qm, double dt, const real u[3], const real E[3], const real B[3], real out[3]) {
    double a = 0.5 * qm * dt;
    real um[3], T[3], S[3], up[3], c[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + a * E[d];
    real gm = RSQRT(1.0 + dot3(um, um));
    for (int d = 0; d < 3; ++d) T[d] = a * B[d] / gm;
    real tt = dot3(T, T);
    for (int d = 0; d < 3; ++d) S[d] = 2.0 * T[d] / (1.0 + tt);
    cross3(um, T, c);
    for (int d = 0; d < 3; ++d) up[d] = um[d] + c[d];
    cross3(up, S, c);
    for (int d = 0; d < 3; ++d) out[d] = um[d] + c[d] + a * E[d];
}

/* Vay (2008): implicit average of the velocities in the magnetic term, solved
 * in closed form for the new Lorentz factor. */
static void push_vay(double qm, double dt, const real u[3], const real E[3], const real B[3], real out[3]) {
    double a = 0.5 * qm * dt;
    real g0 = RSQRT(1.0 + dot3(u, u));
    real v0[3], c[3], u1[3], tau[3], t[3];
    for (int d = 0; d < 3; ++d) v0[d] = u[d] / g0;
    cross3(v0, B, c);
    for (int d = 0; d < 3; ++d) u1[d] = u[d] + 2.0 * a * E[d] + a * c[d];
    for (int d = 0; d < 3; ++d) tau[d] = a * B[d];
    real us = dot3(u1, tau), tau2 = dot3(tau, tau);
    real sig = 1.0 + dot3(u1, u1) - tau2;
    real D = RSQRT(sig * sig + 4.0 * (tau2 + us * us));
    real gn = RSQRT(0.5 * (sig + D));
    for (int d = 0; d < 3; ++d) t[d] = tau[d] / gn;
    real sf = 1.0 / (1.0 + dot3(t, t));
    real ut = dot3(u1, t);
    cross3(u1, t, c);
    for (int d = 0; d < 3; ++d) out[d] = sf * (u1[d] + ut * t[d] + c[d]);
}

void orc_push(int32_t pusher, double qm, double dt, const real u[3], const real E[3], const real B[3], real out[3]) {
    if (pusher == 1)
        push_vay(qm, dt, u, E, B, out);
    else
        push_boris(qm, dt, u, E, B, out);
}

/* ------------------------------------------------------------------ */
/* Esirkepov (2001) charge-conserving deposition, quadratic shapes      */
/* ------------------------------------------------------------------ */

/* J index of component c at per-dimension indices id[3] (half-node index along c) */
static real *jref(orc_sim *s, int c, const int64_t id[3]) { return &s->J[c][fidx(s, id[0], id[1], id[2])]; }

/* For a move X0 -> X1 (|dX| < 1 per dimension), with S0, S1 the node shapes on
 * a five-node window starting at b_d = round(X0_d) - 2 and DS = S1 - S0,
 *   W_c = DS_c (S0_a S0_b + DS_a S0_b / 2 + S0_a DS_b / 2 + DS_a DS_b / 3)
 * ((c, a, b) cyclic), and J_c on the half nodes along c is the running sum
 *   J_c(m + 1/2) = J_c(m - 1/2) - q w W_c(m) / dt
 * starting from zero below the window.  The last running sum is zero. */
void orc_deposit(orc_sim *s, const real X0[3], const real X1[3], real qw) {
    int64_t b[3];
    real S0[3][5], DS[3][5];
    for (int d = 0; d < 3; ++d) {
        b[d] = (int64_t)floor(RE(X0[d]) + 0.5) - 2;
        for (int m = 0; m < 5; ++m) {
            S0[d][m] = orc_shape(X0[d] - (double)(b[d] + m));
            DS[d][m] = orc_shape(X1[d] - (double)(b[d] + m)) - S0[d][m];
        }
    }
    real f = -qw / s->dt;
    for (int c = 0; c < 3; ++c) {
        int ca = (c + 1) % 3, cb = (c + 2) % 3;
        for (int ma = 0; ma < 5; ++ma)
            for (int mb = 0; mb < 5; ++mb) {
                real acc = 0.0;
                for (int m = 0; m < 4; ++m) {
                    real W = DS[c][m] * (S0[ca][ma] * S0[cb][mb] + 0.5 * DS[ca][ma] * S0[cb][mb] +
                                         0.5 * S0[ca][ma] * DS[cb][mb] + DS[ca][ma] * DS[cb][mb] / 3.0);
                    acc += W;
                    int64_t id[3];
                    id[c] = b[c] + m;
                    id[ca] = b[ca] + ma;
                    id[cb] = b[cb] + mb;
                    *jref(s, c, id) += f * acc;
                }
            }
    }
}

/* Immobile lab ions = the plasma lattice drifting rigidly at -beta_R.  A
 * lattice that is uniform across x and y sums the transverse shapes to
 * ppc_x ppc_y on every node, so the ions' Esirkepov current is purely J_z and
 * depends on z only: the 1D running sum of -q w (S1 - S0) / dt per sheet. */
void orc_ion_current(orc_sim *s, double t0, double t1, int32_t unit_weight) {
    if (s->c.ions != 1) return;
    int ptr = s->c.ppc[0] * s->c.ppc[1];
    for (int64_t l = s->sh_lo; l < s->sh_hi; ++l) {
        real w = sheet_weight(s, l);
        if (RE(w) == 0.0) continue;
        if (unit_weight) w = w / s->n0n;
        double z0 = sheet_z(s, l, t0), z1 = sheet_z(s, l, t1);
        int64_t b = (int64_t)floor(z0 + 0.5) - 2;
        real acc = 0.0;
        for (int m = 0; m < 4; ++m) {
            acc += orc_shape(z1 - (double)(b + m)) - orc_shape(z0 - (double)(b + m));
            real jz = -(+1.0) * w * ptr / s->dt * acc;
            for (int j = 0; j < s->ny; ++j)
                for (int i = 0; i < s->nx; ++i) s->J[2][fidx(s, i, j, b + m)] += jz;
        }
    }
}

void orc_zero_J(orc_sim *s) {
    for (int c = 0; c < 3; ++c) memset(s->J[c], 0, sizeof(real) * s->nc);
}

/* ------------------------------------------------------------------ */
/* Yee FDTD [Eq. Max1, Max2]; x, y periodic; z open with Mur-1 faces    */
/* ------------------------------------------------------------------ */

/* B <- B - (dt/2) curl E.  In an open z box the half planes l = nz-1 of Bx, By
 * lie outside the window and stay untouched. */
void orc_b_half(orc_sim *s) {
    double h = 0.5 * s->dt;
    real *Ex = s->E[0], *Ey = s->E[1], *Ez = s->E[2];
    for (int l = 0; l < s->nz; ++l)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                int64_t o = lidx(s, i, j, l);
                int top = !s->periodic_z && l == s->nz - 1;
                if (!top) {
                    s->B[0][o] -= h * ((Ez[lidx(s, i, j + 1, l)] - Ez[o]) - (Ey[lidx(s, i, j, l + 1)] - Ey[o]));
                    s->B[1][o] -= h * ((Ex[lidx(s, i, j, l + 1)] - Ex[o]) - (Ez[lidx(s, i + 1, j, l)] - Ez[o]));
                }
                s->B[2][o] -= h * ((Ey[lidx(s, i + 1, j, l)] - Ey[o]) - (Ex[lidx(s, i, j + 1, l)] - Ex[o]));
            }
}

/* E <- E + dt (curl B - J).  Open z: Ex, Ey on the back face l = 0 come from
 * the first-order Mur condition
 *   E(0)^{n+1} = E(1)^n + (dt - 1)/(dt + 1) (E(1)^{n+1} - E(0)^n),
 * and on the front face l = nz-1 from its mirror when the window is at rest.
 * A moving window's front face keeps its tangential E (zero: the planes enter
 * empty) -- fields reach it only by outrunning a window moving at nearly c,
 * and a static-face Mur condition at a face that jumps forward every step or
 * two is unstable with plasma streaming in.  Ez on the outside half plane
 * nz-1 stays untouched. */
void orc_e_update(orc_sim *s) {
    real *Bx = s->B[0], *By = s->B[1], *Bz = s->B[2];
    int64_t pl = (int64_t)s->nx * s->ny;
    real *keep = NULL;
    if (!s->periodic_z) {
        keep = (real *)malloc(sizeof(real) * 8 * pl);
        int planes[4] = {0, 1, s->nz - 2, s->nz - 1};
        for (int q = 0; q < 4; ++q)
            for (int c = 0; c < 2; ++c) memcpy(keep + (2 * q + c) * pl, s->E[c] + planes[q] * pl, sizeof(real) * pl);
    }
    for (int l = 0; l < s->nz; ++l)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                int64_t o = lidx(s, i, j, l);
                int face = !s->periodic_z && (l == 0 || l == s->nz - 1);
                if (!face) {
                    s->E[0][o] += s->dt * ((Bz[o] - Bz[lidx(s, i, j - 1, l)]) - (By[o] - By[lidx(s, i, j, l - 1)]) - s->J[0][o]);
                    s->E[1][o] += s->dt * ((Bx[o] - Bx[lidx(s, i, j, l - 1)]) - (Bz[o] - Bz[lidx(s, i - 1, j, l)]) - s->J[1][o]);
                }
                if (s->periodic_z || l != s->nz - 1)
                    s->E[2][o] += s->dt * ((By[o] - By[lidx(s, i - 1, j, l)]) - (Bx[o] - Bx[lidx(s, i, j - 1, l)]) - s->J[2][o]);
            }
    if (!s->periodic_z) {
        double cm = (s->dt - 1.0) / (s->dt + 1.0);
        int front_mur = s->bw <= 0.0;
        for (int c = 0; c < 2; ++c) {
            real *o0 = keep + (0 + c) * pl, *o1 = keep + (2 + c) * pl;
            real *o2 = keep + (4 + c) * pl, *o3 = keep + (6 + c) * pl;
            real *F = s->E[c];
            for (int64_t q = 0; q < pl; ++q) {
                F[q] = o1[q] + cm * (F[pl + q] - o0[q]);
                if (front_mur) F[(s->nz - 1) * pl + q] = o2[q] + cm * (F[(s->nz - 2) * pl + q] - o3[q]);
            }
        }
        free(keep);
    }
}

/* ------------------------------------------------------------------ */
/* species storage                                                      */
/* ------------------------------------------------------------------ */
static void sp_reserve(orc_sp *p, int64_t n) {
    if (n <= p->cap) return;
    int64_t cap = p->cap ? p->cap : 1024;
    while (cap < n) cap *= 2;
    for (int d = 0; d < 3; ++d) {
        p->x[d] = (real *)realloc(p->x[d], sizeof(real) * cap);
        p->u[d] = (real *)realloc(p->u[d], sizeof(real) * cap);
    }
    p->w = (real *)realloc(p->w, sizeof(real) * cap);
    p->alive = (int32_t *)realloc(p->alive, sizeof(int32_t) * cap);
    if (!p->w || !p->alive) die("out of memory");
    p->cap = cap;
}

static void sp_free(orc_sp *p) {
    for (int d = 0; d < 3; ++d) {
        free(p->x[d]);
        free(p->u[d]);
    }
    free(p->w);
    free(p->alive);
}

/* plasma sheet: nx ny ppc_x ppc_y cold electrons at rest in the lab
 * (u = -gR bR zhat in the boosted frame), order (j, b, i, a); with mobile
 * ions, as many ions at the same places with the same velocity and weight
 * (a neutral plasma, both populations on one lattice and one shape, sec. 1) */
static void inject_sheet(orc_sim *s, int64_t l, double t) {
    real w = sheet_weight(s, l);
    if (RE(w) == 0.0) return;
    int px = s->c.ppc[0], py = s->c.ppc[1];
    int64_t add = (int64_t)s->nx * s->ny * px * py;
    double z = sheet_z(s, l, t);
    for (int sp = 1; sp <= (s->c.ions == 2 ? 2 : 1); ++sp) {
        orc_sp *p = &s->sp[sp];
        sp_reserve(p, p->n + add);
        for (int j = 0; j < s->ny; ++j)
            for (int bb = 0; bb < py; ++bb)
                for (int i = 0; i < s->nx; ++i)
                    for (int aa = 0; aa < px; ++aa) {
                        int64_t q = p->n++;
                        p->x[0][q] = i + (aa + 0.5) / px;
                        p->x[1][q] = j + (bb + 0.5) / py;
                        p->x[2][q] = z;
                        p->u[0][q] = 0.0;
                        p->u[1][q] = 0.0;
                        p->u[2][q] = -s->uR;
                        p->w[q] = w;
                        p->alive[q] = 1;
                    }
    }
}

static double zlo_of(const orc_sim *s) { return (double)(s->k0 + 3); }
static double zhi_of(const orc_sim *s) { return (double)(s->k0 + s->nz - 4); }

/* ------------------------------------------------------------------ */
/* construction                                                         */
/* ------------------------------------------------------------------ */
orc_sim *orc_new(const orc_config *c, const double *normals) {
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->c = *c;
    s->nx = c->nx;
    s->ny = c->ny;
    s->nz = c->nz;
    s->periodic_z = c->bc_z == 1;
    s->nc = (int64_t)c->nx * c->ny * c->nz;
    double D = c->dx_m;
    s->dt = c->dt_override > 0 ? c->dt_override : c->cfl / sqrt(3.0);
    s->gR = c->gamma_boost;
    s->bR = orc_beta(s->gR);
    s->uR = s->gR * s->bR;
    s->nref = EPS0 * M_E * C_LIGHT * C_LIGHT / (Q_E * Q_E * D * D);
    s->zoff = c->zc_cells;
    s->q[0] = s->q[1] = -1.0;
    s->m[0] = s->m[1] = 1.0;
    s->q[2] = 1.0;
    s->m[2] = c->ion_mass > 0 ? c->ion_mass : MP_OVER_ME;
    for (int q = 0; q < 3; ++q) {
        s->E[q] = (real *)calloc(s->nc, sizeof(real));
        s->B[q] = (real *)calloc(s->nc, sizeof(real));
        s->J[q] = (real *)calloc(s->nc, sizeof(real));
    }
    s->K = c->K;
    s->n0n = c->n0_cm3 * 1e6 / s->nref;
#ifdef ORC_CSTEP
    s->K += I * c->hK;
    s->n0n += I * (c->hn0 * 1e6 / s->nref);
#endif
    /* undulator, lab cells; B0 = K m c k_u / e -> normalised K k_u D */
    if (c->und_kind != 0) {
        double lu = c->lu_m / D;
        s->ku = 2.0 * PI_D / lu;
        s->z0u = c->und_z0_m / D;
        s->Lu = c->und_len_m / D;
        s->Ru = c->und_ramp_periods * lu;
        s->B0 = s->K * s->ku;
    }
    s->z0p = c->pl_z0_m / D;
    s->Lp = c->pl_len_m / D;
    s->Rp = c->pl_ramp_m / D;

    /* beam: lab-frame Gaussian at t = 0 around the box axis, then the
     * per-particle Lorentz transform and a ballistic drift to t' = 0 */
    orc_sp *bp = &s->sp[0];
    int64_t nb = c->n_beam;
    sp_reserve(bp, nb > 0 ? nb : 1);
    s->F = orc_elongation(c->gamma_lab, s->gR);
    s->sig_zlab = c->sigma[2] / s->F;
    s->wbeam = (c->charge_C / Q_E) / (double)(nb > 0 ? nb : 1) / (s->nref * D * D * D);
    double sux = c->emit[0] / (c->sigma[0] * D), suy = c->emit[1] / (c->sigma[1] * D);
    double wsum = 0.0, wvz = 0.0;
    for (int64_t p = 0; p < nb; ++p) {
        const double *g = normals;
        double lab[4] = {0.5 * c->nx + c->sigma[0] * g[p], 0.5 * c->ny + c->sigma[1] * g[nb + p],
                         s->sig_zlab * g[2 * nb + p], 0.0};
        double ulab[3], gam = c->gamma_lab * (1.0 + c->espread * g[5 * nb + p]);
        ulab[0] = sux * g[3 * nb + p];
        ulab[1] = suy * g[4 * nb + p];
        ulab[2] = sqrt(gam * gam - 1.0 - ulab[0] * ulab[0] - ulab[1] * ulab[1]);
        double ev[4], ub[3];
        orc_lab_to_boosted(s->gR, lab, ulab, ev, ub);
        double gb = sqrt(1.0 + ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
        double drift = -ev[3];
        double x = ev[0] + ub[0] / gb * drift, y = ev[1] + ub[1] / gb * drift;
        double z = ev[2] + ub[2] / gb * drift + s->zoff;
        x = fmod(x, c->nx);
        if (x < 0) x += c->nx;
        y = fmod(y, c->ny);
        if (y < 0) y += c->ny;
        bp->x[0][p] = x;
        bp->x[1][p] = y;
        bp->x[2][p] = z;
        for (int d = 0; d < 3; ++d) bp->u[d][p] = ub[d];
        bp->w[p] = s->wbeam;
        bp->alive[p] = s->periodic_z || (z >= zlo_of(s) && z < zhi_of(s));
        if (!bp->alive[p]) s->beam_lost++;
        if (bp->alive[p]) {
            wsum += 1.0;
            wvz += ub[2] / gb;
        }
    }
    bp->n = nb;
    s->bw = c->window_beta >= 0 ? c->window_beta : (wsum > 0 ? wvz / wsum : 0.0);

    /* plasma lattice in the window at t' = 0; ion sheets on the same lattice */
    if (c->n0_cm3 > 0) {
        int p2 = c->ppc[2];
        if (s->periodic_z) {
            s->sh_lo = 0;
            s->sh_hi = (int64_t)s->nz * p2;
        } else {
            s->sh_lo = (int64_t)(zlo_of(s) * p2);
            s->sh_hi = (int64_t)(zhi_of(s) * p2);
        }
        for (int64_t l = s->sh_lo; l < s->sh_hi; ++l) inject_sheet(s, l, 0.0);
    }
    return s;
}

void orc_free(orc_sim *s) {
    if (!s) return;
    for (int q = 0; q < 3; ++q) {
        free(s->E[q]);
        free(s->B[q]);
        free(s->J[q]);
    }
    for (int sp = 0; sp < 3; ++sp) sp_free(&s->sp[sp]);
    free(s->fc_rho);
    for (int c = 0; c < 3; ++c) free(s->fc_E[c]);
    free(s);
}

/* ------------------------------------------------------------------ */
/* one step                                                             */
/* ------------------------------------------------------------------ */
static void wrap_pos(const orc_sim *s, real X[3]) {
    if (RE(X[0]) < 0) X[0] += s->nx;
    if (RE(X[0]) >= s->nx) X[0] -= s->nx;
    if (RE(X[1]) < 0) X[1] += s->ny;
    if (RE(X[1]) >= s->ny) X[1] -= s->ny;
    if (s->periodic_z) {
        if (RE(X[2]) < 0) X[2] += s->nz;
        if (RE(X[2]) >= s->nz) X[2] -= s->nz;
    }
}

/* gather + external field -> push -> move -> deposit for one particle of species sp */
static void particle_update(orc_sim *s, int sp, int64_t q, double t) {
    orc_sp *p = &s->sp[sp];
    real X[3] = {p->x[0][q], p->x[1][q], p->x[2][q]};
    real U[3] = {p->u[0][q], p->u[1][q], p->u[2][q]};
    real Ep[3], Bp[3], Ee[3], Be[3], Un[3], X1[3];
    orc_gather(s, X, Ep, Bp);
    orc_ext_field(s, X[2], t, Ee, Be);
    for (int d = 0; d < 3; ++d) {
        Ep[d] += Ee[d];
        Bp[d] += Be[d];
    }
    orc_push(s->c.pusher, s->q[sp] / s->m[sp], s->dt, U, Ep, Bp, Un);
    real g = RSQRT(1.0 + dot3(Un, Un));
    for (int d = 0; d < 3; ++d) X1[d] = X[d] + s->dt * Un[d] / g;
    orc_deposit(s, X, X1, s->q[sp] * p->w[q]);
    wrap_pos(s, X1);
    for (int d = 0; d < 3; ++d) {
        p->x[d][q] = X1[d];
        p->u[d][q] = Un[d];
    }
}

/* shift the fields one plane back: new(l) = old(l+1), new front plane zero */
static void shift_fields(orc_sim *s) {
    int64_t pl = (int64_t)s->nx * s->ny;
    for (int c = 0; c < 3; ++c) {
        memmove(s->E[c], s->E[c] + pl, sizeof(real) * pl * (s->nz - 1));
        memmove(s->B[c], s->B[c] + pl, sizeof(real) * pl * (s->nz - 1));
        memset(s->E[c] + pl * (s->nz - 1), 0, sizeof(real) * pl);
        memset(s->B[c] + pl * (s->nz - 1), 0, sizeof(real) * pl);
    }
    s->k0 += 1;
}

/* end of step: window shift (one cell whenever the accumulated travel
 * beta_w t' passes the next whole cell), removal of particles outside the
 * active band, ion-sheet bookkeeping, injection of new lattice sheets at the
 * front.  Returns whether the window shifted. */
static int window_events(orc_sim *s, double t1) {
    int shifted = 0;
    int64_t target = (int64_t)floor(s->win_x0 + s->bw * (t1 - s->win_t0));
    while (s->k0 < target) {
        shift_fields(s);
        shifted = 1;
    }
    double lo = zlo_of(s), hi = zhi_of(s);
    for (int sp = 0; sp < 3; ++sp) {
        orc_sp *p = &s->sp[sp];
        for (int64_t q = 0; q < p->n; ++q)
            if (p->alive[q] && (RE(p->x[2][q]) < lo || RE(p->x[2][q]) >= hi)) {
                p->alive[q] = 0;
                if (sp == 0)
                    s->beam_lost++;
                else
                    s->plasma_removed++;
            }
    }
    if (s->c.n0_cm3 > 0) {
        while (s->sh_lo < s->sh_hi && sheet_z(s, s->sh_lo, t1) < lo) s->sh_lo++;
        while (sheet_z(s, s->sh_hi, t1) < hi) {
            inject_sheet(s, s->sh_hi, t1);
            s->sh_hi++;
        }
        if (s->sh_lo > s->sh_hi) s->sh_lo = s->sh_hi;
    }
    return shifted;
}

/* remaining fraction of the neutralising charge at time t */
static double fade_of(const orc_sim *s, double t) {
    if (!(s->fc_T > 0.0)) return 0.0;
    double f = 1.0 - t / s->fc_T;
    return f > 0.0 ? f : 0.0;
}

/* the current that removes the neutralising charge between t and t1: the charge drops by
 * fc_rho (f(t) - f(t1)), so -fc_E (f(t) - f(t1)) / dt satisfies continuity node by node */
static void fading_charge_current(orc_sim *s, double t, double t1) {
    double a = (fade_of(s, t) - fade_of(s, t1)) / s->dt;
    if (a == 0.0) return;
    int64_t pl = (int64_t)s->nx * s->ny;
    for (int l = 0; l < s->nz; ++l) {
        int64_t k = s->k0 + l - s->fc_k0; /* the plane where the charge was laid down */
        if (k < 0 || k >= s->nz) continue;
        for (int c = 0; c < 3; ++c)
            for (int64_t q = 0; q < pl; ++q) s->J[c][l * pl + q] -= a * s->fc_E[c][k * pl + q];
    }
}

void orc_set_fading_charge(orc_sim *s, const real *rho, const real *Ex, const real *Ey, const real *Ez,
                           double fade_s) {
    const real *E[3] = {Ex, Ey, Ez};
    if (!s->fc_rho) {
        s->fc_rho = (real *)malloc(sizeof(real) * s->nc);
        for (int c = 0; c < 3; ++c) s->fc_E[c] = (real *)malloc(sizeof(real) * s->nc);
    }
    memcpy(s->fc_rho, rho, sizeof(real) * s->nc);
    for (int c = 0; c < 3; ++c) memcpy(s->fc_E[c], E[c], sizeof(real) * s->nc);
    s->fc_T = fade_s * C_LIGHT / s->c.dx_m;
    s->fc_k0 = s->k0;
}

static void step_once(orc_sim *s) {
    double t = s->step * s->dt, t1 = (s->step + 1) * s->dt;
    orc_b_half(s); /* B^n */
    orc_zero_J(s);
    for (int sp = 0; sp < 3; ++sp) {
        orc_sp *p = &s->sp[sp];
        for (int64_t q = 0; q < p->n; ++q)
            if (p->alive[q]) particle_update(s, sp, q, t);
    }
    orc_ion_current(s, t, t1, 0);
    fading_charge_current(s, t, t1);
    orc_b_half(s); /* B^{n+1/2} */
    orc_e_update(s);
    s->step += 1;
    if (!s->periodic_z) window_events(s, t1);
}

void orc_step(orc_sim *s, int32_t n) {
    for (int32_t i = 0; i < n; ++i) step_once(s);
}

/* the window moves at beta from the current time on (section 3: the window's speed is
 * adjusted to the beam's); its position stays continuous in time */
void orc_set_window_beta(orc_sim *s, double beta) {
    double t = s->step * s->dt;
    s->win_x0 = s->win_x0 + s->bw * (t - s->win_t0);
    s->win_t0 = t;
    s->bw = beta;
}

/* ------------------------------------------------------------------ */
/* accessors                                                            */
/* ------------------------------------------------------------------ */
void orc_info(const orc_sim *s, orc_info_t *o) {
    o->dt = s->dt;
    o->gR = s->gR;
    o->bR = s->bR;
    o->uR = s->uR;
    o->bw = s->bw;
    o->nref_m3 = s->nref;
    o->wbeam = RE(s->wbeam);
    o->ku = s->ku;
    o->B0 = RE(s->B0);
    o->n0n = RE(s->n0n);
    o->zoff = s->zoff;
    o->F_elong = s->F;
    o->sig_zlab = s->sig_zlab;
    o->k0 = s->k0;
    o->step = s->step;
    o->n_beam = s->sp[0].n;
    o->n_plasma = s->sp[1].n;
    o->sheet_lo = s->sh_lo;
    o->sheet_hi = s->sh_hi;
    o->beam_lost = s->beam_lost;
    o->plasma_removed = s->plasma_removed;
    o->n_ions = s->sp[2].n;
    o->ion_mass = s->m[2];
    o->window_x = s->win_x0 + s->bw * (s->step * s->dt - s->win_t0);
}

real *orc_field(orc_sim *s, int32_t which) {
    if (which < 3) return s->E[which];
    if (which < 6) return s->B[which - 3];
    return s->J[which - 6];
}

real *orc_particles(orc_sim *s, int32_t sp, int32_t which) {
    orc_sp *p = &s->sp[sp];
    if (which < 3) return p->x[which];
    if (which < 6) return p->u[which - 3];
    return p->w;
}

int32_t *orc_alive(orc_sim *s, int32_t sp) { return s->sp[sp].alive; }

/* ------------------------------------------------------------------ */
/* diagnostics                                                          */
/* ------------------------------------------------------------------ */
void orc_rho(orc_sim *s, int32_t mask, real *rho) {
    memset(rho, 0, sizeof(real) * s->nc);
    for (int sp = 0; sp < 3; ++sp) {
        if (!(mask & (1 << sp))) continue;
        orc_sp *p = &s->sp[sp];
        for (int64_t q = 0; q < p->n; ++q) {
            if (!p->alive[q]) continue;
            real X[3] = {p->x[0][q], p->x[1][q], p->x[2][q]};
            int64_t lo[3];
            for (int d = 0; d < 3; ++d) lo[d] = (int64_t)floor(RE(X[d]) + 0.5) - 1;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    for (int c = 0; c < 3; ++c) {
                        int64_t i = lo[0] + a, j = lo[1] + b, k = lo[2] + c;
                        rho[fidx(s, i, j, k)] += s->q[sp] * p->w[q] * orc_shape(X[0] - (double)i) *
                                                 orc_shape(X[1] - (double)j) * orc_shape(X[2] - (double)k);
                    }
        }
    }
    if ((mask & 8) && s->fc_rho) {
        double f = fade_of(s, s->step * s->dt);
        int64_t pl = (int64_t)s->nx * s->ny;
        for (int l = 0; l < s->nz; ++l) {
            int64_t k = s->k0 + l - s->fc_k0;
            if (f == 0.0 || k < 0 || k >= s->nz) continue;
            for (int64_t q = 0; q < pl; ++q) rho[l * pl + q] -= f * s->fc_rho[k * pl + q];
        }
    }
    if ((mask & 4) && s->c.ions == 1) {
        double t = s->step * s->dt;
        int ptr = s->c.ppc[0] * s->c.ppc[1];
        for (int64_t l = s->sh_lo; l < s->sh_hi; ++l) {
            real w = sheet_weight(s, l);
            if (RE(w) == 0.0) continue;
            double z = sheet_z(s, l, t);
            int64_t lo = (int64_t)floor(z + 0.5) - 1;
            for (int c = 0; c < 3; ++c) {
                real v = w * ptr * orc_shape(z - (double)(lo + c));
                for (int j = 0; j < s->ny; ++j)
                    for (int i = 0; i < s->nx; ++i) rho[fidx(s, i, j, lo + c)] += v;
            }
        }
    }
}

/* r = div E - rho on every node (div of the edge-centred E at the node) */
void orc_gauss(orc_sim *s, real *r) {
    orc_rho(s, 15, r);
    for (int l = 0; l < s->nz; ++l)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                int64_t o = lidx(s, i, j, l);
                real dv = (s->E[0][o] - s->E[0][lidx(s, i - 1, j, l)]) + (s->E[1][o] - s->E[1][lidx(s, i, j - 1, l)]);
                if (s->periodic_z || l > 0) dv += s->E[2][o] - s->E[2][lidx(s, i, j, l - 1)];
                else dv += s->E[2][o];
                r[o] = dv - r[o];
            }
}

void orc_diag(orc_sim *s, double kb, orc_diag_t *o) {
    memset(o, 0, sizeof(*o));
    o->t = s->step * s->dt;
    orc_sp *p = &s->sp[0];
    double W = 0, m[3] = {0}, um[3] = {0};
    for (int64_t q = 0; q < p->n; ++q) {
        if (!p->alive[q]) continue;
        double w = RE(p->w[q]);
        W += w;
        o->n_beam_alive += 1;
        for (int d = 0; d < 3; ++d) {
            m[d] += w * RE(p->x[d][q]);
            um[d] += w * RE(p->u[d][q]);
        }
    }
    o->wsum = W;
    if (W > 0) {
        for (int d = 0; d < 3; ++d) {
            m[d] /= W;
            um[d] /= W;
        }
        double sx[3] = {0}, su[3] = {0}, sxu[2] = {0};
        double c1 = 0, s1 = 0, c2 = 0, s2 = 0, kin = 0;
        for (int64_t q = 0; q < p->n; ++q) {
            if (!p->alive[q]) continue;
            double w = RE(p->w[q]);
            double dx[3], du[3];
            for (int d = 0; d < 3; ++d) {
                dx[d] = RE(p->x[d][q]) - m[d];
                du[d] = RE(p->u[d][q]) - um[d];
                sx[d] += w * dx[d] * dx[d];
                su[d] += w * du[d] * du[d];
            }
            sxu[0] += w * dx[0] * du[0];
            sxu[1] += w * dx[1] * du[1];
            double z = RE(p->x[2][q]);
            c1 += w * cos(kb * z);
            s1 += w * sin(kb * z);
            c2 += w * cos(2 * kb * z);
            s2 += w * sin(2 * kb * z);
            double uu = RE(p->u[0][q]) * RE(p->u[0][q]) + RE(p->u[1][q]) * RE(p->u[1][q]) + RE(p->u[2][q]) * RE(p->u[2][q]);
            kin += w * (sqrt(1.0 + uu) - 1.0);
        }
        for (int d = 0; d < 3; ++d) {
            o->mean[d] = m[d];
            o->umean[d] = um[d];
            o->sigma[d] = sqrt(sx[d] / W);
            o->usigma[d] = sqrt(su[d] / W);
        }
        for (int d = 0; d < 2; ++d) o->emit[d] = sqrt(fmax(0.0, (sx[d] / W) * (su[d] / W) - (sxu[d] / W) * (sxu[d] / W)));
        o->b1_re = c1 / W;
        o->b1_im = s1 / W;
        o->b2_re = c2 / W;
        o->b2_im = s2 / W;
        o->b1_abs = sqrt(c1 * c1 + s1 * s1) / W;
        o->b2_abs = sqrt(c2 * c2 + s2 * s2) / W;
        o->kin_beam = kin;
    }
    double kp = 0; /* plasma electrons and mobile ions: m w (gamma - 1) */
    for (int sp = 1; sp < 3; ++sp) {
        orc_sp *pp = &s->sp[sp];
        for (int64_t q = 0; q < pp->n; ++q) {
            if (!pp->alive[q]) continue;
            double uu = RE(pp->u[0][q]) * RE(pp->u[0][q]) + RE(pp->u[1][q]) * RE(pp->u[1][q]) +
                        RE(pp->u[2][q]) * RE(pp->u[2][q]);
            kp += s->m[sp] * RE(pp->w[q]) * (sqrt(1.0 + uu) - 1.0);
        }
    }
    o->kin_plasma = kp;
    double fe = 0;
    for (int c = 0; c < 3; ++c)
        for (int64_t q = 0; q < s->nc; ++q) fe += RE(s->E[c][q]) * RE(s->E[c][q]) + RE(s->B[c][q]) * RE(s->B[c][q]);
    o->field_energy = 0.5 * fe;
}

/* ------------------------------------------------------------------ */
/* adjoint                                                              */
/* ------------------------------------------------------------------ */
/* state vector: [beam x,y,z,ux,uy,uz (n_beam each)] [plasma 6 x n_plasma] [E 3 x nc] [B 3 x nc] */
int64_t orc_state_len(const orc_sim *s) {
    if (s->c.ions == 2) die("adjoint state: mobile ions are not modelled");
    return 6 * (s->sp[0].n + s->sp[1].n) + 6 * s->nc;
}

void orc_get_state(const orc_sim *s, real *v) {
    if (s->c.ions == 2) die("adjoint state: mobile ions are not modelled");
    int64_t o = 0;
    for (int sp = 0; sp < 2; ++sp) {
        const orc_sp *p = &s->sp[sp];
        for (int d = 0; d < 3; ++d, o += p->n) memcpy(v + o, p->x[d], sizeof(real) * p->n);
        for (int d = 0; d < 3; ++d, o += p->n) memcpy(v + o, p->u[d], sizeof(real) * p->n);
    }
    for (int c = 0; c < 3; ++c, o += s->nc) memcpy(v + o, s->E[c], sizeof(real) * s->nc);
    for (int c = 0; c < 3; ++c, o += s->nc) memcpy(v + o, s->B[c], sizeof(real) * s->nc);
}

void orc_set_state(orc_sim *s, const real *v) {
    if (s->c.ions == 2) die("adjoint state: mobile ions are not modelled");
    int64_t o = 0;
    for (int sp = 0; sp < 2; ++sp) {
        orc_sp *p = &s->sp[sp];
        for (int d = 0; d < 3; ++d, o += p->n) memcpy(p->x[d], v + o, sizeof(real) * p->n);
        for (int d = 0; d < 3; ++d, o += p->n) memcpy(p->u[d], v + o, sizeof(real) * p->n);
    }
    for (int c = 0; c < 3; ++c, o += s->nc) memcpy(s->E[c], v + o, sizeof(real) * s->nc);
    for (int c = 0; c < 3; ++c, o += s->nc) memcpy(s->B[c], v + o, sizeof(real) * s->nc);
}

/* full copy of the dynamic state (for recomputation in the adjoint) */
typedef struct {
    orc_sp sp[2];
    real *E[3], *B[3];
    int64_t k0, step, sh_lo, sh_hi, beam_lost, plasma_removed;
} orc_snap;

static void snap_take(const orc_sim *s, orc_snap *z) {
    memset(z, 0, sizeof(*z));
    for (int sp = 0; sp < 2; ++sp) {
        const orc_sp *p = &s->sp[sp];
        orc_sp *q = &z->sp[sp];
        sp_reserve(q, p->n > 0 ? p->n : 1);
        q->n = p->n;
        for (int d = 0; d < 3; ++d) {
            memcpy(q->x[d], p->x[d], sizeof(real) * p->n);
            memcpy(q->u[d], p->u[d], sizeof(real) * p->n);
        }
        memcpy(q->w, p->w, sizeof(real) * p->n);
        memcpy(q->alive, p->alive, sizeof(int32_t) * p->n);
    }
    for (int c = 0; c < 3; ++c) {
        z->E[c] = (real *)malloc(sizeof(real) * s->nc);
        z->B[c] = (real *)malloc(sizeof(real) * s->nc);
        memcpy(z->E[c], s->E[c], sizeof(real) * s->nc);
        memcpy(z->B[c], s->B[c], sizeof(real) * s->nc);
    }
    z->k0 = s->k0;
    z->step = s->step;
    z->sh_lo = s->sh_lo;
    z->sh_hi = s->sh_hi;
    z->beam_lost = s->beam_lost;
    z->plasma_removed = s->plasma_removed;
}

static void snap_restore(orc_sim *s, const orc_snap *z) {
    for (int sp = 0; sp < 2; ++sp) {
        orc_sp *p = &s->sp[sp];
        const orc_sp *q = &z->sp[sp];
        p->n = q->n;
        for (int d = 0; d < 3; ++d) {
            memcpy(p->x[d], q->x[d], sizeof(real) * q->n);
            memcpy(p->u[d], q->u[d], sizeof(real) * q->n);
        }
        memcpy(p->w, q->w, sizeof(real) * q->n);
        memcpy(p->alive, q->alive, sizeof(int32_t) * q->n);
    }
    for (int c = 0; c < 3; ++c) {
        memcpy(s->E[c], z->E[c], sizeof(real) * s->nc);
        memcpy(s->B[c], z->B[c], sizeof(real) * s->nc);
    }
    s->k0 = z->k0;
    s->step = z->step;
    s->sh_lo = z->sh_lo;
    s->sh_hi = z->sh_hi;
    s->beam_lost = z->beam_lost;
    s->plasma_removed = z->plasma_removed;
}

static void snap_free(orc_snap *z) {
    sp_free(&z->sp[0]);
    sp_free(&z->sp[1]);
    for (int c = 0; c < 3; ++c) {
        free(z->E[c]);
        free(z->B[c]);
    }
}

/* transpose of B <- B - h curl E, acting on the adjoints: lE += -h curl_E^T(lB) */
static void b_half_adj(const orc_sim *s, real *const lB[3], real *lE[3], double h) {
    for (int l = 0; l < s->nz; ++l)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                int64_t o = lidx(s, i, j, l);
                int top = !s->periodic_z && l == s->nz - 1;
                if (!top) {
                    real g = lB[0][o]; /* Bx -= h((Ez[j+1]-Ez) - (Ey[l+1]-Ey)) */
                    lE[2][lidx(s, i, j + 1, l)] -= h * g;
                    lE[2][o] += h * g;
                    lE[1][lidx(s, i, j, l + 1)] += h * g;
                    lE[1][o] -= h * g;
                    g = lB[1][o]; /* By -= h((Ex[l+1]-Ex) - (Ez[i+1]-Ez)) */
                    lE[0][lidx(s, i, j, l + 1)] -= h * g;
                    lE[0][o] += h * g;
                    lE[2][lidx(s, i + 1, j, l)] += h * g;
                    lE[2][o] -= h * g;
                }
                real g = lB[2][o]; /* Bz -= h((Ey[i+1]-Ey) - (Ex[j+1]-Ex)) */
                lE[1][lidx(s, i + 1, j, l)] -= h * g;
                lE[1][o] += h * g;
                lE[0][lidx(s, i, j + 1, l)] += h * g;
                lE[0][o] -= h * g;
            }
}

/* transpose of the E update with Mur faces.  In: lE holds the adjoint of
 * E^{n+1}.  Out: lE the adjoint of E^n, lB += adjoint of B^{n+1/2}, lJ set. */
static void e_update_adj(const orc_sim *s, real *lE[3], real *lB[3], real *lJ[3]) {
    int64_t pl = (int64_t)s->nx * s->ny;
    double dt = s->dt;
    real *lEn[3];
    for (int c = 0; c < 3; ++c) {
        lEn[c] = (real *)calloc(s->nc, sizeof(real));
        memset(lJ[c], 0, sizeof(real) * s->nc);
    }
    if (!s->periodic_z) {
        double cm = (dt - 1.0) / (dt + 1.0);
        int front_mur = s->bw <= 0.0;
        for (int c = 0; c < 2; ++c)
            for (int64_t q = 0; q < pl; ++q) {
                real g0 = lE[c][q]; /* E(0) = E^n(1) + cm (E^{n+1}(1) - E^n(0)) */
                lE[c][pl + q] += cm * g0;
                lEn[c][pl + q] += g0;
                lEn[c][q] += -cm * g0;
                lE[c][q] = 0.0;
                int64_t t = (s->nz - 1) * pl + q, u = (s->nz - 2) * pl + q;
                real g1 = lE[c][t];
                if (front_mur) {
                    lE[c][u] += cm * g1;
                    lEn[c][u] += g1;
                    lEn[c][t] += -cm * g1;
                } else
                    lEn[c][t] += g1; /* front face kept */
                lE[c][t] = 0.0;
            }
    }
    for (int l = 0; l < s->nz; ++l)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                int64_t o = lidx(s, i, j, l);
                int face = !s->periodic_z && (l == 0 || l == s->nz - 1);
                if (!face) {
                    real g = lE[0][o]; /* Ex += dt((Bz - Bz[j-1]) - (By - By[l-1]) - Jx) */
                    lEn[0][o] += g;
                    lB[2][o] += dt * g;
                    lB[2][lidx(s, i, j - 1, l)] -= dt * g;
                    lB[1][o] -= dt * g;
                    lB[1][lidx(s, i, j, l - 1)] += dt * g;
                    lJ[0][o] = -dt * g;
                    g = lE[1][o]; /* Ey += dt((Bx - Bx[l-1]) - (Bz - Bz[i-1]) - Jy) */
                    lEn[1][o] += g;
                    lB[0][o] += dt * g;
                    lB[0][lidx(s, i, j, l - 1)] -= dt * g;
                    lB[2][o] -= dt * g;
                    lB[2][lidx(s, i - 1, j, l)] += dt * g;
                    lJ[1][o] = -dt * g;
                }
                if (s->periodic_z || l != s->nz - 1) {
                    real g = lE[2][o]; /* Ez += dt((By - By[i-1]) - (Bx - Bx[j-1]) - Jz) */
                    lEn[2][o] += g;
                    lB[1][o] += dt * g;
                    lB[1][lidx(s, i - 1, j, l)] -= dt * g;
                    lB[0][o] -= dt * g;
                    lB[0][lidx(s, i, j - 1, l)] += dt * g;
                    lJ[2][o] = -dt * g;
                } else
                    lEn[2][o] += lE[2][o]; /* untouched outside half plane */
            }
    for (int c = 0; c < 3; ++c) {
        memcpy(lE[c], lEn[c], sizeof(real) * s->nc);
        free(lEn[c]);
    }
}

/* adjoint of the Esirkepov deposit of one particle: given lJ on the grid,
 * accumulate d<lJ, J_p>/dX0 and /dX1; return <lJ, J_p>. */
static real deposit_adj(const orc_sim *s, real *const lJ[3], const real X0[3], const real X1[3], real qw,
                        real gX0[3], real gX1[3]) {
    int64_t b[3];
    real S0[3][5], S1[3][5], DS[3][5], dS0[3][5], dS1[3][5];
    for (int d = 0; d < 3; ++d) {
        b[d] = (int64_t)floor(RE(X0[d]) + 0.5) - 2;
        for (int m = 0; m < 5; ++m) {
            real d0 = X0[d] - (double)(b[d] + m), d1 = X1[d] - (double)(b[d] + m);
            S0[d][m] = orc_shape(d0);
            S1[d][m] = orc_shape(d1);
            DS[d][m] = S1[d][m] - S0[d][m];
            dS0[d][m] = orc_dshape(d0);
            dS1[d][m] = orc_dshape(d1);
        }
    }
    real f = -qw / s->dt;
    real gS0[3][5], gDS[3][5];
    memset(gS0, 0, sizeof(gS0));
    memset(gDS, 0, sizeof(gDS));
    real val = 0.0;
    for (int c = 0; c < 3; ++c) {
        int ca = (c + 1) % 3, cb = (c + 2) % 3;
        for (int ma = 0; ma < 5; ++ma)
            for (int mb = 0; mb < 5; ++mb) {
                /* L = sum_m f * lJ(m) * sum_{m'<=m} W(m') = sum_m' W(m') * Lam(m'), Lam = f * suffix sum of lJ */
                real lam[4];
                real suf = 0.0;
                for (int m = 3; m >= 0; --m) {
                    int64_t id[3];
                    id[c] = b[c] + m;
                    id[ca] = b[ca] + ma;
                    id[cb] = b[cb] + mb;
                    suf += lJ[c][fidx(s, id[0], id[1], id[2])];
                    lam[m] = f * suf;
                }
                real A = S0[ca][ma] * S0[cb][mb] + 0.5 * DS[ca][ma] * S0[cb][mb] + 0.5 * S0[ca][ma] * DS[cb][mb] +
                         DS[ca][ma] * DS[cb][mb] / 3.0;
                real gA = 0.0;
                for (int m = 0; m < 4; ++m) {
                    val += DS[c][m] * A * lam[m];
                    gDS[c][m] += A * lam[m];
                    gA += DS[c][m] * lam[m];
                }
                gS0[ca][ma] += gA * (S0[cb][mb] + 0.5 * DS[cb][mb]);
                gDS[ca][ma] += gA * (0.5 * S0[cb][mb] + DS[cb][mb] / 3.0);
                gS0[cb][mb] += gA * (S0[ca][ma] + 0.5 * DS[ca][ma]);
                gDS[cb][mb] += gA * (0.5 * S0[ca][ma] + DS[ca][ma] / 3.0);
            }
    }
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < 5; ++m) {
            /* S0 = S(X0 - node), DS = S(X1 - node) - S0 */
            gX0[d] += (gS0[d][m] - gDS[d][m]) * dS0[d][m];
            gX1[d] += gDS[d][m] * dS1[d][m];
        }
    return val;
}

/* reverse of Boris: given lo = adjoint of the output, return adjoints of u, E, B */
static void push_boris_adj(double qm, double dt, const real u[3], const real E[3], const real B[3], const real lo[3],
                           real lu[3], real lE[3], real lB[3]) {
    double a = 0.5 * qm * dt;
    real um[3], T[3], S[3], up[3], c[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + a * E[d];
    real gm = RSQRT(1.0 + dot3(um, um));
    for (int d = 0; d < 3; ++d) T[d] = a * B[d] / gm;
    real tt = dot3(T, T);
    for (int d = 0; d < 3; ++d) S[d] = 2.0 * T[d] / (1.0 + tt);
    cross3(um, T, c);
    for (int d = 0; d < 3; ++d) up[d] = um[d] + c[d];
    /* out = uplus + a E, uplus = um + up x S */
    real lum[3], lup[3], lS[3], lT[3], tmp[3];
    for (int d = 0; d < 3; ++d) {
        lE[d] = a * lo[d];
        lum[d] = lo[d];
    }
    cross3(S, lo, lup);   /* d(lo.(up x S))/dup = S x lo */
    cross3(lo, up, lS);   /* d/dS = lo x up */
    /* up = um + um x T */
    cross3(T, lup, tmp);  /* d(lup.(um x T))/dum = T x lup */
    for (int d = 0; d < 3; ++d) lum[d] += lup[d] + tmp[d];
    cross3(lup, um, lT);  /* d/dT = lup x um */
    /* S = 2T/(1+tt) */
    real TS = dot3(T, lS), den = 1.0 + tt;
    for (int d = 0; d < 3; ++d) lT[d] += 2.0 * lS[d] / den - 4.0 * T[d] * TS / (den * den);
    /* T = a B / gm */
    real lgm = -a * dot3(B, lT) / (gm * gm);
    for (int d = 0; d < 3; ++d) lB[d] = a * lT[d] / gm;
    /* gm = sqrt(1 + um.um) */
    for (int d = 0; d < 3; ++d) lum[d] += lgm * um[d] / gm;
    /* um = u + a E */
    for (int d = 0; d < 3; ++d) {
        lu[d] = lum[d];
        lE[d] += a * lum[d];
    }
}

/* reverse of Vay */
static void push_vay_adj(double qm, double dt, const real u[3], const real E[3], const real B[3], const real lo[3],
                         real lu[3], real lE[3], real lB[3]) {
    double a = 0.5 * qm * dt;
    real g0 = RSQRT(1.0 + dot3(u, u));
    real v0[3], c[3], u1[3], tau[3], t[3], w[3];
    for (int d = 0; d < 3; ++d) v0[d] = u[d] / g0;
    cross3(v0, B, c);
    for (int d = 0; d < 3; ++d) u1[d] = u[d] + 2.0 * a * E[d] + a * c[d];
    for (int d = 0; d < 3; ++d) tau[d] = a * B[d];
    real us = dot3(u1, tau), tau2 = dot3(tau, tau);
    real sig = 1.0 + dot3(u1, u1) - tau2;
    real D = RSQRT(sig * sig + 4.0 * (tau2 + us * us));
    real gn = RSQRT(0.5 * (sig + D));
    for (int d = 0; d < 3; ++d) t[d] = tau[d] / gn;
    real sf = 1.0 / (1.0 + dot3(t, t));
    real ut = dot3(u1, t);
    cross3(u1, t, c);
    for (int d = 0; d < 3; ++d) w[d] = u1[d] + ut * t[d] + c[d];
    /* out = sf w */
    real lsf = dot3(lo, w), lw[3], lu1[3], lt[3], ltau[3], tmp[3];
    for (int d = 0; d < 3; ++d) lw[d] = sf * lo[d];
    /* w = u1 + (u1.t) t + u1 x t */
    real tlw = dot3(t, lw);
    cross3(t, lw, tmp);
    for (int d = 0; d < 3; ++d) lu1[d] = lw[d] + tlw * t[d] + tmp[d];
    cross3(lw, u1, tmp);
    for (int d = 0; d < 3; ++d) lt[d] = tlw * u1[d] + ut * lw[d] + tmp[d];
    /* sf = 1/(1 + t.t) */
    for (int d = 0; d < 3; ++d) lt[d] += -2.0 * lsf * sf * sf * t[d];
    /* t = tau / gn */
    real lgn = -dot3(tau, lt) / (gn * gn);
    for (int d = 0; d < 3; ++d) ltau[d] = lt[d] / gn;
    /* gn = sqrt((sig + D)/2) */
    real lsig = lgn / (4.0 * gn), lD = lgn / (4.0 * gn);
    /* D = sqrt(sig^2 + 4 (tau2 + us^2)) */
    lsig += lD * sig / D;
    real ltau2 = lD * 2.0 / D, lus = lD * 4.0 * us / D;
    /* sig = 1 + u1.u1 - tau2 */
    ltau2 += -lsig;
    for (int d = 0; d < 3; ++d) lu1[d] += 2.0 * lsig * u1[d];
    /* tau2 = tau.tau, us = u1.tau */
    for (int d = 0; d < 3; ++d) {
        ltau[d] += 2.0 * ltau2 * tau[d] + lus * u1[d];
        lu1[d] += lus * tau[d];
    }
    /* tau = a B */
    for (int d = 0; d < 3; ++d) lB[d] = a * ltau[d];
    /* u1 = u + 2 a E + a v0 x B */
    real lv0[3];
    cross3(B, lu1, lv0);
    cross3(lu1, v0, tmp);
    for (int d = 0; d < 3; ++d) {
        lv0[d] *= a;
        lB[d] += a * tmp[d];
        lE[d] = 2.0 * a * lu1[d];
        lu[d] = lu1[d];
    }
    /* v0 = u / g0 */
    real uv = dot3(u, lv0);
    for (int d = 0; d < 3; ++d) lu[d] += lv0[d] / g0 - u[d] * uv / (g0 * g0 * g0);
}

/* scatter lam * shape into the adjoint field (transpose of interp); return d(lam * interp)/dX added to gX */
static void interp_adj(const orc_sim *s, const real *F, real *lF, const real X[3], const double off[3], real lam,
                       real gX[3]) {
    int64_t lo[3];
    for (int d = 0; d < 3; ++d) lo[d] = (int64_t)floor(RE(X[d]) - off[d] + 0.5) - 1;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                int64_t i = lo[0] + a, j = lo[1] + b, k = lo[2] + c;
                real dx = X[0] - (i + off[0]), dy = X[1] - (j + off[1]), dz = X[2] - (k + off[2]);
                real sx = orc_shape(dx), sy = orc_shape(dy), sz = orc_shape(dz);
                int64_t o = fidx(s, i, j, k);
                lF[o] += lam * sx * sy * sz;
                real f = F[o] * lam;
                gX[0] += f * orc_dshape(dx) * sy * sz;
                gX[1] += f * sx * orc_dshape(dy) * sz;
                gX[2] += f * sx * sy * orc_dshape(dz);
            }
}

/* seed of L = |sum_beam w exp(i k z)| / sum_beam w at the current state */
real orc_seed_bunching(orc_sim *s, double kb, real *lam) {
    memset(lam, 0, sizeof(real) * orc_state_len(s));
    orc_sp *p = &s->sp[0];
    real W = 0, C = 0, S = 0;
    for (int64_t q = 0; q < p->n; ++q) {
        if (!p->alive[q]) continue;
        W += p->w[q];
        C += p->w[q] * RCOS(kb * p->x[2][q]);
        S += p->w[q] * RSIN(kb * p->x[2][q]);
    }
    real A = RSQRT(C * C + S * S);
    real *lz = lam + 2 * p->n;
    for (int64_t q = 0; q < p->n; ++q) {
        if (!p->alive[q]) continue;
        real z = p->x[2][q];
        lz[q] = p->w[q] * kb * (-C * RSIN(kb * z) + S * RCOS(kb * z)) / (A * W);
    }
    return A / W;
}

/* One reverse step.  On entry the sim holds the forward state n; lam_in is the
 * adjoint of state n+1 (layout of state n+1), lam_out receives the adjoint of
 * state n.  gK_log += K dL/dK and gn_log += n0 dL/dn0 contributions of the
 * step.  Discrete events (window shift, removal, injection) are those the
 * forward step takes from state n.  The sim is left at state n. */
void orc_adjoint_step(orc_sim *s, const real *lam_in, real *lam_out, real *gK_log, real *gn_log) {
    if (s->c.ions == 2) die("adjoint: mobile ions are not modelled");
    orc_snap z0;
    snap_take(s, &z0);
    double t = s->step * s->dt, t1 = (s->step + 1) * s->dt, dt = s->dt;
    int64_t nc = s->nc, nsp[2] = {s->sp[0].n, s->sp[1].n};

    /* forward recompute: B^n, per-particle X1 (unwrapped) and u^{n+1/2}, events */
    orc_b_half(s);
    real *Bn[3];
    for (int c = 0; c < 3; ++c) {
        Bn[c] = (real *)malloc(sizeof(real) * nc);
        memcpy(Bn[c], s->B[c], sizeof(real) * nc);
    }
    real *X1[2][3], *Un[2][3];
    for (int sp = 0; sp < 2; ++sp)
        for (int d = 0; d < 3; ++d) {
            X1[sp][d] = (real *)calloc(nsp[sp] ? nsp[sp] : 1, sizeof(real));
            Un[sp][d] = (real *)calloc(nsp[sp] ? nsp[sp] : 1, sizeof(real));
        }
    for (int sp = 0; sp < 2; ++sp) {
        orc_sp *p = &s->sp[sp];
        for (int64_t q = 0; q < p->n; ++q) {
            if (!p->alive[q]) continue;
            real X[3] = {p->x[0][q], p->x[1][q], p->x[2][q]}, U[3] = {p->u[0][q], p->u[1][q], p->u[2][q]};
            real Ep[3], Bp[3], Ee[3], Be[3], un[3];
            orc_gather(s, X, Ep, Bp);
            orc_ext_field(s, X[2], t, Ee, Be);
            for (int d = 0; d < 3; ++d) {
                Ep[d] += Ee[d];
                Bp[d] += Be[d];
            }
            orc_push(s->c.pusher, -1.0, dt, U, Ep, Bp, un);
            real g = RSQRT(1.0 + dot3(un, un));
            for (int d = 0; d < 3; ++d) {
                Un[sp][d][q] = un[d];
                X1[sp][d][q] = X[d] + dt * un[d] / g;
            }
        }
    }
    /* events: run the whole forward step on the sim, read alive flags and counts */
    snap_restore(s, &z0);
    int64_t k0_before = s->k0;
    step_once(s);
    int shifted = s->k0 != k0_before;
    int64_t nsp1[2] = {s->sp[0].n, s->sp[1].n};
    int32_t *alive1[2];
    for (int sp = 0; sp < 2; ++sp) {
        alive1[sp] = (int32_t *)malloc(sizeof(int32_t) * (nsp[sp] ? nsp[sp] : 1));
        memcpy(alive1[sp], s->sp[sp].alive, sizeof(int32_t) * nsp[sp]);
    }
    snap_restore(s, &z0);

    /* unpack lam_in (layout of state n+1) */
    real *lX1[2][3], *lUn[2][3], *lE[3], *lB[3], *lJ[3];
    int64_t o = 0;
    for (int sp = 0; sp < 2; ++sp) {
        for (int d = 0; d < 3; ++d) {
            lX1[sp][d] = (real *)calloc(nsp[sp] ? nsp[sp] : 1, sizeof(real));
            lUn[sp][d] = (real *)calloc(nsp[sp] ? nsp[sp] : 1, sizeof(real));
        }
        for (int d = 0; d < 3; ++d, o += nsp1[sp])
            for (int64_t q = 0; q < nsp[sp]; ++q)
                if (alive1[sp][q]) lX1[sp][d][q] = lam_in[o + q];
        for (int d = 0; d < 3; ++d, o += nsp1[sp])
            for (int64_t q = 0; q < nsp[sp]; ++q)
                if (alive1[sp][q]) lUn[sp][d][q] = lam_in[o + q];
    }
    for (int c = 0; c < 3; ++c, o += nc) {
        lE[c] = (real *)malloc(sizeof(real) * nc);
        memcpy(lE[c], lam_in + o, sizeof(real) * nc);
    }
    for (int c = 0; c < 3; ++c, o += nc) {
        lB[c] = (real *)malloc(sizeof(real) * nc);
        memcpy(lB[c], lam_in + o, sizeof(real) * nc);
    }
    for (int c = 0; c < 3; ++c) lJ[c] = (real *)calloc(nc, sizeof(real));

    /* reverse window shift: new(l) = old(l+1) -> lold(l+1) = lnew(l), lold(0) = 0 */
    if (shifted) {
        int64_t pl = (int64_t)s->nx * s->ny;
        for (int c = 0; c < 3; ++c) {
            memmove(lE[c] + pl, lE[c], sizeof(real) * pl * (s->nz - 1));
            memmove(lB[c] + pl, lB[c], sizeof(real) * pl * (s->nz - 1));
            memset(lE[c], 0, sizeof(real) * pl);
            memset(lB[c], 0, sizeof(real) * pl);
        }
    }
    /* reverse E update: lE -> adjoint of E^n, lB -> adjoint of B^{n+1/2}, lJ */
    e_update_adj(s, lE, lB, lJ);
    /* reverse second half step: B^{n+1/2} = B^n - h curl E^n (lB now adjoint of B^n) */
    b_half_adj(s, lB, lE, 0.5 * dt);
    /* reverse ion current */
    if (s->c.ions && s->c.n0_cm3 > 0) {
        real *Jsave[3];
        for (int c = 0; c < 3; ++c) {
            Jsave[c] = s->J[c];
            s->J[c] = (real *)calloc(nc, sizeof(real));
        }
        orc_ion_current(s, t, t1, 0);
        real v = 0.0;
        for (int64_t q = 0; q < nc; ++q) v += lJ[2][q] * s->J[2][q];
        *gn_log += v;
        for (int c = 0; c < 3; ++c) {
            free(s->J[c]);
            s->J[c] = Jsave[c];
        }
    }
    /* reverse particles: deposit, move, push, gather (+ external field) */
    real *lXo[2][3], *lUo[2][3];
    for (int sp = 0; sp < 2; ++sp) {
        orc_sp *p = &s->sp[sp];
        for (int d = 0; d < 3; ++d) {
            lXo[sp][d] = (real *)calloc(nsp[sp] ? nsp[sp] : 1, sizeof(real));
            lUo[sp][d] = (real *)calloc(nsp[sp] ? nsp[sp] : 1, sizeof(real));
        }
        for (int64_t q = 0; q < p->n; ++q) {
            if (!p->alive[q]) continue;
            real X[3] = {p->x[0][q], p->x[1][q], p->x[2][q]}, U[3] = {p->u[0][q], p->u[1][q], p->u[2][q]};
            real x1[3] = {X1[sp][0][q], X1[sp][1][q], X1[sp][2][q]}, un[3] = {Un[sp][0][q], Un[sp][1][q], Un[sp][2][q]};
            real gX[3] = {0, 0, 0}, gX1[3] = {lX1[sp][0][q], lX1[sp][1][q], lX1[sp][2][q]};
            real lun[3] = {lUn[sp][0][q], lUn[sp][1][q], lUn[sp][2][q]};
            real val = deposit_adj(s, lJ, X, x1, -p->w[q], gX, gX1);
            if (sp == 1) *gn_log += val;
            /* X1 = X + dt un / g */
            real g = RSQRT(1.0 + dot3(un, un)), ug = dot3(un, gX1);
            for (int d = 0; d < 3; ++d) {
                gX[d] += gX1[d];
                lun[d] += dt * (gX1[d] / g - un[d] * ug / (g * g * g));
            }
            /* push */
            real Ep[3], Bp[3], Ee[3], Be[3], dEe[3], dBe[3], lu[3], lEp[3], lBp[3];
            orc_gather(s, X, Ep, Bp); /* s->B holds B^{n-1/2}: use B^n copies below */
            for (int c = 0; c < 3; ++c) Bp[c] = interp(s, Bn[c], X, STAG_B[c]);
            ext_field_d(s, X[2], t, Ee, Be, dEe, dBe);
            for (int d = 0; d < 3; ++d) {
                Ep[d] += Ee[d];
                Bp[d] += Be[d];
            }
            if (s->c.pusher == 1)
                push_vay_adj(-1.0, dt, U, Ep, Bp, lun, lu, lEp, lBp);
            else
                push_boris_adj(-1.0, dt, U, Ep, Bp, lun, lu, lEp, lBp);
            /* external field: linear in K; z derivative */
            *gK_log += dot3(lEp, Ee) + dot3(lBp, Be);
            gX[2] += dot3(lEp, dEe) + dot3(lBp, dBe);
            /* gather: scatter into the field adjoints, position derivative */
            for (int c = 0; c < 3; ++c) {
                interp_adj(s, s->E[c], lE[c], X, STAG_E[c], lEp[c], gX);
                interp_adj(s, Bn[c], lB[c], X, STAG_B[c], lBp[c], gX);
            }
            for (int d = 0; d < 3; ++d) {
                lXo[sp][d][q] = gX[d];
                lUo[sp][d][q] = lu[d];
            }
        }
    }
    /* reverse first half step: B^n = B^{n-1/2} - h curl E^n */
    b_half_adj(s, lB, lE, 0.5 * dt);

    /* pack lam_out (layout of state n) */
    o = 0;
    for (int sp = 0; sp < 2; ++sp) {
        for (int d = 0; d < 3; ++d, o += nsp[sp]) memcpy(lam_out + o, lXo[sp][d], sizeof(real) * nsp[sp]);
        for (int d = 0; d < 3; ++d, o += nsp[sp]) memcpy(lam_out + o, lUo[sp][d], sizeof(real) * nsp[sp]);
    }
    for (int c = 0; c < 3; ++c, o += nc) memcpy(lam_out + o, lE[c], sizeof(real) * nc);
    for (int c = 0; c < 3; ++c, o += nc) memcpy(lam_out + o, lB[c], sizeof(real) * nc);

    for (int sp = 0; sp < 2; ++sp) {
        for (int d = 0; d < 3; ++d) {
            free(X1[sp][d]);
            free(Un[sp][d]);
            free(lX1[sp][d]);
            free(lUn[sp][d]);
            free(lXo[sp][d]);
            free(lUo[sp][d]);
        }
        free(alive1[sp]);
    }
    for (int c = 0; c < 3; ++c) {
        free(Bn[c]);
        free(lE[c]);
        free(lB[c]);
        free(lJ[c]);
    }
    snap_free(&z0);
}

/* forward run + bunching loss (the complex build returns real and imaginary parts) */
void orc_loss_bunching(const orc_config *c, const double *normals, int32_t nsteps, double kb, double out[2]) {
    orc_sim *s = orc_new(c, normals);
    orc_step(s, nsteps);
    real *lam = (real *)malloc(sizeof(real) * orc_state_len(s));
    real L = orc_seed_bunching(s, kb, lam);
    out[0] = RE(L);
#ifdef ORC_CSTEP
    out[1] = cimag(L);
#else
    out[1] = 0.0;
#endif
    free(lam);
    orc_free(s);
}

/* L, K dL/dK, n0 dL/dn0 by storing every state and stepping back */
void orc_grad_bunching(const orc_config *c, const double *normals, int32_t nsteps, double kb, double out[3]) {
    orc_sim *s = orc_new(c, normals);
    orc_snap *snaps = (orc_snap *)malloc(sizeof(orc_snap) * (nsteps > 0 ? nsteps : 1));
    for (int32_t n = 0; n < nsteps; ++n) {
        snap_take(s, &snaps[n]);
        step_once(s);
    }
    int64_t len = orc_state_len(s);
    real *lam = (real *)malloc(sizeof(real) * len);
    real L = orc_seed_bunching(s, kb, lam);
    real gK = 0.0, gn = 0.0;
    for (int32_t n = nsteps - 1; n >= 0; --n) {
        snap_restore(s, &snaps[n]);
        real *lo = (real *)malloc(sizeof(real) * orc_state_len(s));
        orc_adjoint_step(s, lam, lo, &gK, &gn);
        free(lam);
        lam = lo;
        snap_free(&snaps[n]);
    }
    out[0] = RE(L);
    out[1] = RE(gK);
    out[2] = RE(gn);
    free(lam);
    free(snaps);
    orc_free(s);
}
