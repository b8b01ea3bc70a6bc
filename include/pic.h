/*
 * pic.h -- C-ABI of the MI355X boosted-frame PIC hot path.
 *
 * The library advances an electron beam (and optionally a cold plasma with
 * immobile ions, and an external undulator field) in a reference frame that
 * moves with Lorentz factor gamma_R along +z, following the method of
 * "Relativistic reference frame PIC simulations for electron beam dynamics
 * with meter-scale propagation inside plasma and under external fields":
 * Maxwell's curl equations with electron and ion currents (section 1,
 * Eq. Max1, Max2) on a Yee grid, charge-conserving current weighting
 * (Eq. Max3, Max4; Esirkepov's scheme with quadratic shapes), a leap-frog
 * relativistic push (section 1, after Eq. Vprime), the beam, field and
 * density transforms of section 1 (Eq. Lor1-Belon, M1-M4, Nnormi, Vprime)
 * and a moving window with absorbing z faces and plasma streaming through it
 * (end of section 1).
 *
 * Conventions
 *   - Units: all arguments are physical SI (m, C, T via K) or dimensionless;
 *     internally length = cell edge D, time = D/c, u = gamma*beta.
 *   - Memory: the caller owns all device memory.  pic_query_layout() reports
 *     how many bytes the context needs; the caller allocates ONE device
 *     buffer of at least that size (256-byte aligned) and passes it to
 *     pic_init(), which borrows it until pic_free().  The context allocates
 *     no device memory of its own and never frees caller memory.
 *   - Streams: every launch goes to options.stream (a hipStream_t, NULL for
 *     the null stream).  pic_step() is asynchronous; pic_diag(), pic_read(),
 *     pic_get_state() and pic_sync() synchronise the stream.
 *   - Errors: functions return pic_status; no exception or abort crosses the
 *     ABI.  pic_last_error() returns a context-owned message.  Device-side
 *     error flags (fixed-point overflow, non-finite momentum, bin overflow
 *     without room) are raised at the next synchronising call.
 *   - Threads: one context per host thread; a context is not re-entrant.
 */
#ifndef PIC_H
#define PIC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define PIC_API __attribute__((visibility("default")))
#else
#define PIC_API
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,  /* invalid argument or configuration */
    PIC_ENOMEM = -2,  /* caller buffer too small / capacity exceeded */
    PIC_EDEVICE = -3, /* HIP runtime error */
    PIC_ESTATE = -4,  /* non-finite state detected, or call not valid in this state */
    PIC_ERANGE = -5   /* fixed-point current overflow */
} pic_status;

enum { PIC_FP64_PLAIN = 0, PIC_FP32_SPLIT = 1 };
enum { PIC_BORIS = 0, PIC_VAY = 1, PIC_PUSHER_AUTO = -1 };
enum { PIC_UND_NONE = 0, PIC_UND_HELICAL = 1, PIC_UND_PLANAR = 2 };

/* Boosted-frame grid: nx x ny x nz cubic cells of edge dx_m; x, y periodic,
 * z open (first-order Mur faces) with a moving window.  dt = cfl dx / (c sqrt 3),
 * 0 < cfl <= 1, nz <= 65535.  cfl = sqrt(3)/2 (c dt = dx / 2) is where the Yee
 * grid's numerical Cherenkov growth of a plasma drifting along z is slowest. */
typedef struct {
    int32_t nx, ny, nz, reserved;
    double dx_m, cfl;
} pic_grid;

/* gamma_boost: Lorentz factor of the frame (Eq. RRFVel).  window_beta: window
 * speed in units of c; < 0 selects the mean beam velocity at t' = 0. */
typedef struct {
    double gamma_boost, window_beta;
} pic_frame;

/* Electron beam defined in the lab at lab time 0 and converted by the library
 * into the boosted frame (as section 3 describes).  Gaussian with rms
 * sizes sigma_cells[0..1] (transverse, frame invariant, cells) and sigma_cells[2]
 * (longitudinal, boosted-frame cells; the lab rms length follows from Eq. Belon),
 * lab Lorentz factor gamma_lab with relative rms spread, normalised rms emittances
 * emit_n_m (m).  normals: HOST pointer to 6 x n_macro standard-normal draws in
 * rows (x, y, z, ux, uy, energy), read during pic_init only; or NULL: pic_init
 * then draws them on the device from seed.  The draw for particle p: two blocks
 * of the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011), counters
 * (p mod 2^32, p div 2^32, j, 0) for j = 0, 1 under the key (seed mod 2^32,
 * seed div 2^32), give eight 32-bit words w0..w7; the pairs (w0, w1), (w2, w3),
 * (w4, w5) become rows (0, 1), (2, 3), (4, 5) by the Box-Muller transform in
 * FP64: U = (w + 1/2) 2^-32, n = sqrt(-2 ln U_a) cos(2 pi U_b),
 * n' = sqrt(-2 ln U_a) sin(2 pi U_b).  The beam centre sits on the box axis,
 * z_center_cells from the window's back face at t' = 0. */
typedef struct {
    int64_t n_macro;
    double charge_C, gamma_lab, rel_energy_spread_rms;
    double sigma_cells[3], emit_n_m[2], z_center_cells;
    const double *normals;
    uint64_t seed;
} pic_beam;

/* Cold plasma at rest in the lab with lab density n0 (cm^-3) on a regular
 * lattice of ppc[0] x ppc[1] x ppc[2] particles per cell; boosted density
 * gamma_R n0 (Eq. Nnormi).  Longitudinal lab profile: zero before z_start,
 * linear up-ramp over ramp_up, flat to z_start + length, zero after;
 * length <= 0 means uniform everywhere.  Lab positions are measured from the
 * beam centre at lab time 0.  Ions (section 1 computes their current
 * directly and gives them the electrons' weighting):
 *   ions = 0  none;
 *   ions = 1  immobile lab ions on the same lattice, a rigid background whose
 *             current j_i = v_R rho_i is a 1D profile along z;
 *   ions = 2  mobile ions of charge +e and mass ion_mass electron masses
 *             (0: the proton's), loaded with every sheet at the electrons'
 *             places with their velocity and weight, pushed with q/m = +1/M
 *             and deposited with the same shape.  They are stored among the
 *             plasma particles with a negated weight (pic_read
 *             returns them so); the adjoint refuses them (PIC_EINVAL).
 * ion_mass must be finite and >= 0 (PIC_EINVAL otherwise). */
typedef struct {
    double n0_lab_cm3;
    int32_t ppc[3], ions;
    double z_start_lab_m, length_lab_m, ramp_up_lab_m;
    double ion_mass;
} pic_plasma;

/* Ideal undulator in the lab: B = B0 env (cos phi, sin phi, 0) (helical) or
 * (0, sin phi, 0) (planar), phi = 2 pi (z - z_start) / period, B0 from the
 * deflection parameter K; linear entrance and exit ramps of
 * entrance_ramp_periods periods.  Transformed to the boosted frame with
 * Eq. M1-M4 and applied analytically at the particles. */
typedef struct {
    int32_t kind, reserved;
    double K, period_lab_m, z_start_lab_m, length_lab_m, entrance_ramp_periods;
} pic_undulator;

/* precision: PIC_FP64_PLAIN (absolute FP64 positions, FP64 fields, FP64 atomics)
 *            or PIC_FP32_SPLIT (int32 cell + FP32 offset, FP32 fields, 64-bit
 *            fixed-point current, particles binned by cell tile).
 * pusher: PIC_BORIS, PIC_VAY or PIC_PUSHER_AUTO (Vay when an undulator is on).
 * fp64_gamma_threshold: FP32 mode pushes particles above this Lorentz factor in FP64.
 * fixed_point_frac_bits: 0 = automatic from the peak current bound (room for 64 times
 *              the peak density: within 2^62 in FP64 mode, within 2^47 in FP32 mode,
 *              whose per-tile LDS sums are 48-bit); a larger value than the FP32
 *              mode's bound returns PIC_ERANGE.
 * check_every: FP32 mode re-lays out its bins when needed, checked every this
 *              many steps (a host synchronisation); 0 = 64.
 * tile: cell tile of the FP32 binned kernels, one of 8x8x4, 8x8x8, 8x8x16, 16x8x4,
 *       16x16x4, 16x8x8, and 16x1x16 for two-dimensional x-z grids (ny = 1)
 *       (edges divide the grid); 0,0,0 = the first of 16x8x8, 16x16x4, 8x8x16,
 *       8x8x8, 16x8x4, 8x8x4, 16x1x16 that divides the grid.
 * max_steps: sizing of the plasma capacity of the FP64 mode (injection between
 *            compactions, or over the whole run when record = 1).
 * record: FP64 mode: 1 keeps particle slots stable (no compaction) so that
 *         pic_adjoint_step() can follow them.  FP32 mode: 1 gives every
 *         particle a 4-byte id, its slot in the FP64 record layout of the same
 *         configuration, so that pic_state_to_fp64() can hand the state to an
 *         FP64 record context (the adjoint of an FP32 run).
 * variant: current deposition of the FP32 particle kernel: 0 = the Esirkepov
 *          window pruned per wave of 64 particles (its last node along an axis
 *          only when some particle of the wave crosses a half cell there),
 *          1 = every contribution of a moving component, 2 = nonzero
 *          contributions only, one branch each.  All give identical results.
 * wg_per_cu: resident workgroups per compute unit of the FP32 particle kernel's
 *            persistent grid; 0 = as many as registers and LDS allow.
 * init_fields: 0 = E = B = 0 at t' = 0 (a frozen neutralising background);
 *              2 = E = B = 0 at t' = 0 with the neutralising charge made explicit
 *              and faded out (section 3's artificial ions): a charge equal and
 *              opposite to the beam's at t' = 0, at rest, that falls linearly to
 *              zero over neutral_fade_s seconds (boosted frame); the current that
 *              removes it is -E_b d/dt(fraction left), E_b the charge's
 *              electrostatic field (the problem below with gamma_b = 1), so the
 *              charge leaves as continuity demands and Gauss's law keeps its
 *              residual; the Gauss diagnostic counts the charge.  Transverse
 *              grid edges up to 2048;
 *              1 = the beam's self-field: its rest-frame electrostatic field
 *              carried into the boosted frame (section 1 field
 *              transformation), i.e. (d_xx + d_yy + d_zz / gamma_b^2) phi =
 *              -rho solved in FP64 on the grid (periodic x, y; phi = 0 beyond
 *              the z faces; gamma_b from the beam's mean boosted beta_z),
 *              E = -(d_x, d_y, d_z / gamma_b^2) phi, B = beta_b z x E at
 *              t' = -dt/2.  Transverse grid edges up to 2048.
 * stream: hipStream_t for all launches (NULL: null stream).
 * neutral_fade_s: the fade time of init_fields = 2 (> 0); ignored otherwise. */
typedef struct {
    int32_t precision, pusher;
    double fp64_gamma_threshold;
    int32_t fixed_point_frac_bits, check_every;
    int32_t tile[3], max_steps;
    int32_t record, variant;
    int32_t wg_per_cu, init_fields;
    void *stream;
    double neutral_fade_s;
} pic_options;

typedef struct {
    uint64_t arena_bytes;    /* device bytes the caller must provide */
    uint64_t state_bytes;    /* device bytes of one pic_get_state() snapshot */
    int64_t beam_capacity;   /* particle slots */
    int64_t plasma_capacity;
} pic_layout;

/* Sizes of the caller-owned buffers for this configuration.  Host only, no GPU. */
PIC_API pic_status pic_query_layout(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                            const pic_undulator *u, const pic_options *o, pic_layout *out);

/* Derived normalised constants (host only, no GPU): for checking the host logic. */
typedef struct {
    double dt, gamma_R, beta_R, u_R, n_ref_m3, w_beam, n0_norm, k_u_lab, B0_norm, k_bunch;
    double elongation, sigma_z_lab_cells, z_offset_cells;
    int32_t frac_bits, pusher;
    int32_t tile[3], reserved;   /* FP32 mode: the cell tile in use */
} pic_derived;
PIC_API pic_status pic_derive(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                      const pic_undulator *u, const pic_options *o, pic_derived *out);

/* Create a context on the current HIP device, borrowing arena (device memory of
 * at least layout.arena_bytes).  Samples and transforms the beam (FP64, on the
 * device), loads the plasma lattice, zeroes the fields.  *out is NULL on error. */
PIC_API pic_status pic_init(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                    const pic_undulator *u, const pic_options *o, void *arena, uint64_t arena_bytes,
                    pic_ctx **out);

/* Advance nsteps steps of the boosted-frame PIC loop of section 1: field
 * gather at the particles, leap-frog push (after Eq. Vprime; Boris or Vay),
 * charge-conserving current deposit (Eq. Max3 by current weighting), the
 * immobile ions' current v_R rho_i (after Eq. Max4), the Yee update of the
 * curl equations (Eq. Max1, Max2), then the window shift and plasma
 * injection of a window co-moving with the beam (section 3).  nsteps >= 0
 * (PIC_EINVAL otherwise).  Errors found at the flag checks (every
 * check_every steps in FP32 mode): PIC_ERANGE for a fixed-point current
 * overflow or a plasma count past the capacity, PIC_ESTATE for a non-finite
 * momentum, PIC_ENOMEM when full bins lost particles; the state is then not
 * to be continued (restore a snapshot).  Asynchronous on the context stream. */
PIC_API pic_status pic_step(pic_ctx *c, int32_t nsteps);

/* Diagnostics (synchronising).  mask: PIC_DIAG_MOMENTS | PIC_DIAG_BUNCHING |
 * PIC_DIAG_ENERGY | PIC_DIAG_GAUSS.  The quantities sections 3 and 4 follow:
 * beam sizes, momenta and emittances (moments), the density modulation the
 * beam picks up (bunching) and the energy bookkeeping; the Gauss residual
 * checks Eq. Max3's constraint div E = rho, which the charge-conserving
 * deposit keeps.  Bunching b(k) = |sum_beam w exp(i k z')| /
 * sum w at k = 2 pi / bunch_period_cells and 2k (boosted frame, fixed t').
 * Gauss: r = div E - rho on nodes at least 8 planes from the z faces; reports
 * max |r| and max |r - r_prev| against the previous Gauss call (planes aligned
 * by the window shift).  n_plasma counts plasma electrons and mobile ions;
 * kin_plasma sums m w (gamma - 1) over both, m = 1 or ion_mass.  All sums in
 * FP64. */
enum { PIC_DIAG_MOMENTS = 1, PIC_DIAG_BUNCHING = 2, PIC_DIAG_ENERGY = 4, PIC_DIAG_GAUSS = 8 };
typedef struct {
    double t, step, k0, n_beam, n_plasma, beam_lost, wsum;
    double mean[3], sigma[3], umean[3], usigma[3], emit[2]; /* cells; emit in cells (x D for metres) */
    double b1_re, b1_im, b1_abs, b2_re, b2_im, b2_abs;
    double field_energy, kin_beam, kin_plasma;
    double gauss_max, gauss_drift, rho_max;
    double window_beta, frac_bits, error_flags;
    double window_x; /* window position (cells) at t; k0 is its floor, or lags it by the one shift a step allows */
} pic_diag_out;
PIC_API pic_status pic_diag(pic_ctx *c, uint32_t mask, double bunch_period_cells, pic_diag_out *out);

/* pic_diag for callers that cannot allocate device memory at all (code under
 * graph capture, serving loops, harnesses that forbid it): the same
 * diagnostics, bit for bit, with their per-block partial sums in a static
 * device array of the library (4 MiB per GPU, PIC_DIAG_STATIC_DOUBLES
 * doubles, set up by pic_init once per device and held until the process
 * ends) instead of the context's arena.  Allocates nothing.  Needs the
 * context's device current (PIC_EINVAL otherwise); PIC_ERANGE when the mask
 * needs more partials than the array holds (13 per 256 beam particles, 2
 * per 256 plasma slots or per FP32 bin, 3 per 256 cells with
 * PIC_DIAG_GAUSS).  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU, from several threads or streams, race; serialise
 * them.  Synchronising. */
enum { PIC_DIAG_STATIC_DOUBLES = 1 << 19 };
PIC_API pic_status pic_diag_static(pic_ctx *c, uint32_t mask, double bunch_period_cells, pic_diag_out *out);

/* Named arrays in canonical order (fields: logical window planes, x fastest;
 * particles: FP64 mode in slot order, FP32 mode in bin order; FP32 positions
 * are returned as absolute FP64 coordinates).  dst: DEVICE buffer.  count
 * receives the element count (dst may be NULL to query).  Synchronising. */
enum {
    PIC_A_EX = 0, PIC_A_EY, PIC_A_EZ, PIC_A_BX, PIC_A_BY, PIC_A_BZ, /* double */
    PIC_A_BEAM = 16,   /* double [7][n]: x y z ux uy uz w  (n = slots) */
    PIC_A_BEAM_ALIVE,  /* int32 [n] */
    PIC_A_PLASMA,      /* double [7][n] */
    PIC_A_PLASMA_ALIVE, /* int32 [n] */
    /* the beam in the lab frame at the current boosted time t' (section 2, the inverse of
     * Eq. Lor1, Lor2; each particle at its own lab time): double [8][n], rows x, y, z_lab,
     * t_lab, ux, uy, uz_lab, gamma_lab, with t_lab = gR (t' + bR (z' - z0)),
     * z_lab = gR (z' - z0 + bR t'), uz_lab = gR (uz' + bR gamma'), gamma_lab = gR (gamma' + bR uz'),
     * z0 = pic_derived.z_offset_cells; slots and alive flags as PIC_A_BEAM */
    PIC_A_BEAM_LAB
};
PIC_API pic_status pic_read(pic_ctx *c, int32_t which, void *dst, int64_t *count);

/* Overwrite named arrays (same layouts as pic_read, src on the DEVICE):
 * fields, and particle phase space of existing slots (FP64 mode). */
PIC_API pic_status pic_write(pic_ctx *c, int32_t which, const void *src, int64_t count);

/* FP32-mode adjoint support: overwrite the dynamic state of dst (FP64 mode,
 * record = 1) with the state of src (FP32 mode, record = 1, same
 * configuration): fields widened to FP64, every particle written to its slot
 * (its id) as absolute position, momentum and weight, slots without a particle
 * dead, window origin, step and injection cursors copied.  dst's
 * options.max_steps must cover src's run (PIC_ENOMEM otherwise); PIC_EINVAL
 * for other precisions or a differing configuration.  Synchronous.  After it,
 * pic_adjoint_seed_bunching() / pic_adjoint_step() on dst linearise about the
 * FP32 trajectory. */
PIC_API pic_status pic_state_to_fp64(const pic_ctx *src, pic_ctx *dst);

/* Lab-frame probe (section 2, relating the boosted run to the lab frame).  A
 * particle at boosted position z' (cells) and time t' is at lab time
 * t = gR (t' + bR (z' - z0)) and lab position z_lab = gR (z' - z0 + bR t'),
 * z0 = pic_derived.z_offset_cells (lab origin: the beam centre at lab time 0;
 * lengths in boosted cells, times in cells / c).  pic_lab_probe arms the probe
 * for lab time t_lab and lab wavenumber k_lab and clears its sums; each later
 * pic_step then samples every live beam particle once, at the instant its lab
 * time passes t_lab on its straight move of that step, and adds w, w cos(k z_lab),
 * w sin(k z_lab), w z_lab and w z_lab^2 to the sums.  pic_lab_probe_read
 * (synchronous) returns the five sums; the probe stays armed until re-armed or
 * pic_lab_probe(c, NAN, 0) disarms it.  Sums are FP64 atomics (order-dependent
 * rounding). */
PIC_API pic_status pic_lab_probe(pic_ctx *c, double t_lab, double k_lab);
PIC_API pic_status pic_lab_probe_read(pic_ctx *c, double out[5]);

/* Lab-frame groups of the beam (section 2): at one boosted instant t' the beam's
 * particles sit at lab times spread over gR bR dz' for a slice dz' along z (Eq. DT),
 * and particles of unequal u'_z move their lab times on unequally; grouping them by
 * slices of z' (absolute boosted cells, as pic_read returns them) and of u'_z keeps
 * each group's lab-time span small.  Group (iz, iu), iz = floor((z' - z_lo) / dz) in
 * [0, nz), iu = floor((u'_z - u_lo) / du) in [0, nu), is entry iz nu + iu of dst
 * (DEVICE, nz nu x 16 doubles): count, sum w, sum w t_lab, min t_lab, max t_lab,
 * sum w z_lab, sum w z_lab^2, sum w x, sum w x^2, sum w y, sum w y^2, sum w ux,
 * sum w ux^2, sum w uy, sum w uy^2, sum w gamma_lab (lab quantities as
 * PIC_A_BEAM_LAB); particles outside every group are left out.  At most 256 groups
 * (PIC_EINVAL otherwise).  Synchronising; FP64 sums in an order that depends on the
 * particles' (rounding at 1e-16). */
typedef struct {
    double z_lo, dz, u_lo, du;
    int32_t nz, nu;
} pic_lab_groups_spec;
enum { PIC_LAB_GROUP_VALUES = 16 };
PIC_API pic_status pic_lab_groups(pic_ctx *c, const pic_lab_groups_spec *spec, void *dst);

/* Checkpoint (the paper describes none; the step of section 1 depends on
 * nothing outside this state): copy the full dynamic state (particles, fields, window origin,
 * step counter, injection cursors; FP32 mode also its bin layout) into / out
 * of a DEVICE buffer of layout.state_bytes, between steps.  A snapshot
 * restores into any context of the same configuration and continues
 * identically (bit for bit in FP32 mode).  Used for resume and by the
 * adjoint's recomputation (FP64 mode). */
PIC_API pic_status pic_get_state(pic_ctx *c, void *dst);
PIC_API pic_status pic_set_state(pic_ctx *c, const void *src);

/* Adjoint (FP64 mode with record = 1; the paper gives none): the exact
 * reverse-mode derivative of one step of pic_step's discrete scheme (section 1:
 * gather, push, deposit, ion current, Yee update; window shift and injection
 * as index maps), for gradients of the bunching factor of sections 3 and 4
 * with respect to the undulator parameter K (Eq. M1-M4's field amplitude)
 * and the plasma density n0 (Eq. Nnormi).  The adjoint vector has the layout of
 * the forward state: [beam x,y,z,ux,uy,uz (beam slots each)] [plasma 6 x plasma
 * slots] [E 3 x cells] [B 3 x cells], doubles on the DEVICE, particle blocks
 * sized by pic_lambda_len().  pic_adjoint_seed_bunching() writes dL/dstate of
 * L = |b(2 pi / bunch_period)| for the current state and returns L.
 * pic_adjoint_step(): precondition -- the context holds forward state n (e.g.
 * restored with pic_set_state); lam holds the adjoint of state n+1 and is
 * overwritten with the adjoint of state n (slots injected during step n are
 * dropped); grad[0] += K dL/dK and grad[1] += n0 dL/dn0 contributions of the
 * step (host doubles).  The forward state is left unchanged. */
PIC_API int64_t pic_lambda_len(const pic_ctx *c);
PIC_API pic_status pic_adjoint_seed_bunching(pic_ctx *c, double bunch_period_cells, void *lam, double *loss);
PIC_API pic_status pic_adjoint_step(pic_ctx *c, void *lam, double grad[2]);

/* Kernel timing with HIP events recorded on the context stream around each
 * launch class: [0] fused particle kernels (gather, push, deposit), [1] FDTD
 * (both B half steps, E update, Mur faces), [2] window, ion current,
 * injection and binning, [3] whole steps.  pic_timing(c, 1) clears and starts
 * collecting, pic_timing(c, 0) stops.  pic_timing_read() synchronises and
 * returns the summed milliseconds and the number of timed launches per class. */
PIC_API pic_status pic_timing(pic_ctx *c, int32_t enable);
PIC_API pic_status pic_timing_read(pic_ctx *c, double ms[4], int64_t launches[4]);

/* Window speed (section 3: a beam whose mean velocity changes, e.g. on entering
 * an undulator, drifts through a window at a fixed speed; the window's speed is
 * adjusted to keep it).  From the current step on the window moves at beta
 * (units of c): its position is x0 + beta (t' - t0), x0 its position at the
 * call's time t0, and it shifts one cell whenever that position passes the next
 * whole cell (at most one shift per step).  beta in [0, 1]; a moving window
 * must keep moving (beta > 0) and a window at rest stays at rest (PIC_EINVAL
 * otherwise).  Host only, no synchronisation; the setting is part of the
 * checkpointed state.  The adjoint's recomputation replays checkpoints, so a
 * run whose window speed was changed between checkpoints is not
 * differentiated. */
PIC_API pic_status pic_set_window_beta(pic_ctx *c, double beta);

PIC_API pic_status pic_sync(pic_ctx *c);
PIC_API void pic_free(pic_ctx *c);
PIC_API const char *pic_last_error(const pic_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
