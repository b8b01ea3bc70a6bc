// pic_api.hip -- host side of the C-ABI: configuration checks, normalised
// units, arena layout, initialisation, the step loop, state I/O.
#include <math.h>

#include <cmath>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pic_internal.h"

namespace pic {

// CODATA 2018
static const double kC = 299792458.0, kQe = 1.602176634e-19, kMe = 9.1093837015e-31,
                    kEps0 = 8.8541878128e-12, kPi = 3.14159265358979323846,
                    kProtonMass = 1836.15267343;  // proton / electron mass

pic_status hip_check(Ctx &c, hipError_t e, const char *what) {
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    c.err = buf;
    return e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE;
}

static pic_status fail(std::string *err, pic_status s, const std::string &msg) {
    if (err) *err = msg;
    return s;
}

// ---------------------------------------------------------------- derivation
struct Plan {
    Params P;
    pic_derived d;
    int precision, record, check_every;
    int64_t cap_b, cap_p, ovf_b, ovf_p;
    uint64_t off[40];
    uint64_t arena, state;
};

static double beta_of(double g) { return sqrt(1.0 - 1.0 / (g * g)); }

static pic_status derive_params(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                                const pic_undulator *u, const pic_options *o, Params &P, pic_derived &d,
                                std::string *err) {
    if (!g || !f || !b || !p || !u || !o) return fail(err, PIC_EINVAL, "null configuration pointer");
    if (g->nx < 1 || g->ny < 1 || g->nz < 16) return fail(err, PIC_EINVAL, "grid: need nx, ny >= 1 and nz >= 16");
    if ((int64_t)g->nx * g->ny * g->nz > (int64_t)1 << 31)
        return fail(err, PIC_EINVAL, "grid: more than 2^31 cells");
    if (g->nz > 65535) return fail(err, PIC_EINVAL, "grid: nz <= 65535 (one launch row per plane)");
    if (!(g->dx_m > 0) || !(g->cfl > 0 && g->cfl <= 1.0)) return fail(err, PIC_EINVAL, "grid: dx_m > 0, 0 < cfl <= 1");
    if (!(f->gamma_boost >= 1.0)) return fail(err, PIC_EINVAL, "frame: gamma_boost >= 1");
    if (f->window_beta >= 1.0) return fail(err, PIC_EINVAL, "frame: window_beta < 1");
    if (b->n_macro < 0) return fail(err, PIC_EINVAL, "beam: n_macro >= 0");
    if (b->n_macro > 0) {
        if (!(b->gamma_lab > 1.0)) return fail(err, PIC_EINVAL, "beam: gamma_lab > 1");
        if (!(b->sigma_cells[0] > 0 && b->sigma_cells[1] > 0 && b->sigma_cells[2] > 0))
            return fail(err, PIC_EINVAL, "beam: sigma_cells > 0");
        if (!(b->charge_C >= 0)) return fail(err, PIC_EINVAL, "beam: charge_C >= 0");
        if (b->emit_n_m[0] < 0 || b->emit_n_m[1] < 0 || b->rel_energy_spread_rms < 0)
            return fail(err, PIC_EINVAL, "beam: emittance and energy spread >= 0");
    }
    if (p->n0_lab_cm3 < 0) return fail(err, PIC_EINVAL, "plasma: n0 >= 0");
    if (p->n0_lab_cm3 > 0 && (p->ppc[0] < 1 || p->ppc[1] < 1 || p->ppc[2] < 1))
        return fail(err, PIC_EINVAL, "plasma: ppc >= 1");
    if (p->ions < 0 || p->ions > 2) return fail(err, PIC_EINVAL, "plasma: ions is 0 (none), 1 (immobile) or 2 (mobile)");
    if (!(p->ion_mass >= 0.0) || std::isinf(p->ion_mass))
        return fail(err, PIC_EINVAL, "plasma: ion_mass >= 0 (0: the proton's)");
    if (u->kind < 0 || u->kind > 2) return fail(err, PIC_EINVAL, "undulator: kind 0, 1 or 2");
    if (u->kind != 0 && !(u->period_lab_m > 0)) return fail(err, PIC_EINVAL, "undulator: period > 0");
    if (o->precision != PIC_FP64_PLAIN && o->precision != PIC_FP32_SPLIT)
        return fail(err, PIC_EINVAL, "options: precision");
    if (o->pusher < -1 || o->pusher > 1) return fail(err, PIC_EINVAL, "options: pusher");
    if (o->variant < 0 || o->variant > 2) return fail(err, PIC_EINVAL, "options: variant 0, 1 or 2");
    if (o->wg_per_cu < 0 || o->wg_per_cu > 8) return fail(err, PIC_EINVAL, "options: wg_per_cu in [0, 8]");
    if (o->init_fields < 0 || o->init_fields > 2) return fail(err, PIC_EINVAL, "options: init_fields is 0, 1 or 2");
    if (o->init_fields == 2 && !(o->neutral_fade_s > 0.0 && std::isfinite(o->neutral_fade_s)))
        return fail(err, PIC_EINVAL, "options: init_fields = 2 needs neutral_fade_s > 0");
    if (o->init_fields && (g->nx > 2048 || g->ny > 2048))
        return fail(err, PIC_EINVAL, "options: init_fields needs transverse grid edges <= 2048");

    memset(&P, 0, sizeof P);
    memset(&d, 0, sizeof d);
    double D = g->dx_m;
    P.nx = g->nx;
    P.ny = g->ny;
    P.nz = g->nz;
    P.plane = g->nx * g->ny;
    P.nc = (int64_t)P.plane * g->nz;
    P.dt = g->cfl / sqrt(3.0);
    P.gR = f->gamma_boost;
    P.bR = beta_of(P.gR);
    P.uR = P.gR * P.bR;
    P.zoff = b->z_center_cells;
    double nref = kEps0 * kMe * kC * kC / (kQe * kQe * D * D);
    int64_t nb = b->n_macro > 0 ? b->n_macro : 1;
    P.wbeam = (b->charge_C / kQe) / (double)nb / (nref * D * D * D);
    P.und_kind = u->kind;
    if (u->kind) {
        double lu = u->period_lab_m / D;
        P.ku = 2.0 * kPi / lu;
        P.z0u = u->z_start_lab_m / D;
        P.Lu = u->length_lab_m / D;
        P.Ru = u->entrance_ramp_periods * lu;
        P.B0 = u->K * P.ku;
    }
    P.has_plasma = p->n0_lab_cm3 > 0;
    P.ions = P.has_plasma && p->ions == 1;
    P.mobile = P.has_plasma && p->ions == 2;
    P.mi = p->ion_mass > 0 ? p->ion_mass : kProtonMass;
    P.ahi = 0.5 * P.dt / P.mi;
    P.ppx = std::max(1, p->ppc[0]);
    P.ppy = std::max(1, p->ppc[1]);
    P.ppz = std::max(1, p->ppc[2]);
    P.n0n = p->n0_lab_cm3 * 1e6 / nref;
    P.wsheet = P.gR * P.n0n / (double)(P.ppx * P.ppy * P.ppz);
    P.z0p = p->z_start_lab_m / D;
    P.Lp = p->length_lab_m / D;
    P.Rp = p->ramp_up_lab_m / D;
    P.pusher = o->pusher == PIC_PUSHER_AUTO ? (u->kind ? PIC_VAY : PIC_BORIS) : o->pusher;
    P.gthr = o->fp64_gamma_threshold > 0 ? o->fp64_gamma_threshold : 100.0;
    // fixed point: room for 64 times the peak |charge density| (electrons + ions + beam)
    double F = b->n_macro > 0 ? b->gamma_lab / (b->gamma_lab * P.gR - sqrt(b->gamma_lab * b->gamma_lab - 1.0) *
                                                                          sqrt(P.gR * P.gR - 1.0))
                              : 1.0;
    double beam_peak = b->n_macro > 0 ? (double)b->n_macro * P.wbeam /
                                            (pow(2.0 * kPi, 1.5) * b->sigma_cells[0] * b->sigma_cells[1] *
                                             b->sigma_cells[2])
                                      : 0.0;
    double jb = 2.0 * P.gR * P.n0n + beam_peak + 1e-6;
    // a single contribution is at most w / dt: FP32 mode converts it exactly while below 2^51
    double vmax = 2.0 * std::max(P.wsheet, P.wbeam) / P.dt + 1e-6;
    int fb = o->fixed_point_frac_bits;
    // the FP32 mode's LDS tiles hold their sums in 48 bits (biased adds): 64 times the peak density
    // within 2^47 instead of 2^62, a quantum still far below the FP32 rounding of the contributions
    const int fb_tile = 47 - (int)ceil(log2(64.0 * jb));
    const bool split = o->precision == PIC_FP32_SPLIT;
    if (fb == 0) fb = std::min(split ? fb_tile : 62 - (int)ceil(log2(64.0 * jb)), 51 - (int)ceil(log2(vmax)));
    fb = std::min(56, std::max(20, fb));
    if (o->fixed_point_frac_bits > 60) return fail(err, PIC_ERANGE, "options: fixed_point_frac_bits > 60");
    if (split && fb > fb_tile)
        return fail(err, PIC_ERANGE,
                    "options: FP32 mode fixed point needs frac_bits <= " + std::to_string(fb_tile) +
                        " for this peak density (48-bit tile sums)");
    P.frac_bits = fb;
    P.fscale = ldexp(1.0, fb);
    P.finv = ldexp(1.0, -fb);
    if (o->precision == PIC_FP32_SPLIT) {
        int t[3] = {o->tile[0], o->tile[1], o->tile[2]};
        if (!t[0] && !t[1] && !t[2]) {
            // the first tile that divides the grid, in order of measured speed (16 x 8 x 8 is
            // 1.5-2.7 % faster than 16 x 16 x 4 on the 128x128x512 to 512x512x2048 workloads;
            // 16 x 1 x 16: two-dimensional x-z grids, ny = 1)
            static const int pref[7][3] = {{16, 8, 8}, {16, 16, 4}, {8, 8, 16}, {8, 8, 8}, {16, 8, 4}, {8, 8, 4},
                                           {16, 1, 16}};
            for (int k = 0; k < 7; ++k)
                if (g->nx % pref[k][0] == 0 && g->ny % pref[k][1] == 0 && g->nz % pref[k][2] == 0) {
                    t[0] = pref[k][0];
                    t[1] = pref[k][1];
                    t[2] = pref[k][2];
                    break;
                }
            if (!t[0])
                return fail(err, PIC_EINVAL, "FP32 mode: grid edges must be multiples of 8, 8, 4 (or 16, 1, 16)");
        }
        if (g->nx % t[0] || g->ny % t[1] || g->nz % t[2])
            return fail(err, PIC_EINVAL, "options: tile must divide the grid");
        if (t[0] < 4 || t[2] < 4 || (t[1] < 4 && !(t[1] == 1 && g->ny == 1)))
            return fail(err, PIC_EINVAL, "options: tile edges >= 4 (y edge 1 on a grid with ny = 1)");
        auto lg = [](int v) { int k = 0; while ((1 << k) < v) ++k; return k; };
        for (int d3 = 0; d3 < 3; ++d3)
            if (t[d3] != (1 << lg(t[d3]))) return fail(err, PIC_EINVAL, "options: tile edges must be powers of two");
        P.cbx = lg(g->nx);
        P.cby = lg(g->ny);
        if (P.cbx + P.cby + lg(g->nz) > 31) return fail(err, PIC_EINVAL, "FP32 mode: grid needs more than 31 cell bits");
        if (!split_tile_supported(t[0], t[1], t[2]))
            return fail(err, PIC_EINVAL,
                        "options: FP32 tile must be one of 8x8x4, 8x8x8, 8x8x16, 16x8x4, 16x16x4, 16x8x8, 16x1x16");
        P.lgx = lg(t[0]);
        P.lgy = lg(t[1]);
        P.lgz = lg(t[2]);
        // LDS of one workgroup: staged E, B (+halo) in FP32, int64 current boxes, field table
        if (split_lds_bytes(t[0], t[1], t[2]) > 160 * 1024)
            return fail(err, PIC_EINVAL, "options: tile too large for 160 KiB of LDS");
        P.tx = t[0];
        P.ty = t[1];
        P.tz = t[2];
        P.ntx = g->nx / t[0];
        P.nty = g->ny / t[1];
        P.ntz = g->nz / t[2];
        P.nbins = P.ntx * P.nty * P.ntz;
    }
    d.dt = P.dt;
    d.gamma_R = P.gR;
    d.beta_R = P.bR;
    d.u_R = P.uR;
    d.n_ref_m3 = nref;
    d.w_beam = P.wbeam;
    d.n0_norm = P.n0n;
    d.k_u_lab = P.ku;
    d.B0_norm = P.B0;
    d.k_bunch = u->kind ? P.ku * P.gR : 2.0 * kPi / 20.0;
    d.elongation = F;
    d.sigma_z_lab_cells = b->n_macro > 0 ? b->sigma_cells[2] / F : 0.0;
    d.z_offset_cells = P.zoff;
    d.frac_bits = fb;
    d.pusher = P.pusher;
    d.tile[0] = P.tx;
    d.tile[1] = P.ty;
    d.tile[2] = P.tz;
    return PIC_OK;
}

static uint64_t al256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

// plasma sheets crossing the front per step (upper bound) times the sheet size
static int64_t sheets_per_step(const Params &P) { return (int64_t)ceil(2.0 * P.dt * P.ppz) + 1; }

static pic_status make_plan(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                            const pic_undulator *u, const pic_options *o, Plan &pl, std::string *err) {
    pic_status s = derive_params(g, f, b, p, u, o, pl.P, pl.d, err);
    if (s != PIC_OK) return s;
    const Params &P = pl.P;
    pl.precision = o->precision;
    pl.record = o->record;
    pl.check_every = o->check_every > 0 ? o->check_every : 64;
    int64_t sheet = sheet_particles(P);
    int64_t fill = P.has_plasma ? (int64_t)P.nz * P.ppz * sheet : 0;
    int64_t maxs = o->max_steps > 0 ? o->max_steps : 0;
    pl.cap_b = b->n_macro;
    uint64_t *off = pl.off;
    memset(off, 0, sizeof pl.off);
    uint64_t a = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t r = a;
        a += al256(bytes);
        return r;
    };
    if (o->precision == PIC_FP64_PLAIN) {
        int64_t between = pl.record ? maxs : pl.check_every;
        pl.cap_p = P.has_plasma ? fill + (between + 2) * sheets_per_step(P) * sheet : 0;
        for (int k = 0; k < 9; ++k) off[k] = take(8 * P.nc);             // E B J
        off[9] = take(8 * P.nz);                                          // jion
        off[10] = take(8 * 8 * (uint64_t)P.plane);                        // Mur planes
        off[11] = take(60 * (uint64_t)std::max<int64_t>(pl.cap_b, 1));   // beam
        off[12] = take(60 * (uint64_t)std::max<int64_t>(pl.cap_p, 1));   // plasma
        off[13] = pl.record ? 0 : take(60 * (uint64_t)std::max<int64_t>(pl.cap_p, 1));  // plasma (compaction)
    } else {
        pl.cap_p = P.has_plasma ? fill : 0;
        for (int k = 0; k < 6; ++k) off[k] = take(4 * P.nc);  // E B float
        for (int k = 6; k < 9; ++k) off[k] = take(8 * P.nc);  // J int64
        off[9] = take(8 * P.nz);
        off[10] = take(4 * 8 * (uint64_t)P.plane);
        // particle double buffers with bin slack and an overflow tail (k_split32.hip)
        int64_t nbins = P.nbins;
        // bin slack: the beam pinches and moves between re-layouts, so its bins get 1/2 of their count as
        // headroom and an overflow tail as large as the beam (it can never lose particles); the plasma
        // gets 1/8 and a tail of 1/8 of its lattice
        int64_t cb = pl.cap_b + pl.cap_b / 2 + 32 * nbins + 4096;
        int64_t cp = pl.cap_p + pl.cap_p / 4 + 32 * nbins + 4096;
        pl.ovf_b = std::max<int64_t>(8192, pl.cap_b);
        pl.ovf_p = std::max<int64_t>(8192, pl.cap_p / 8);
        pl.cap_b = b->n_macro;
        const uint64_t sb = pl.record ? 36 : 32;  // record mode: + the particle id
        off[11] = take(sb * (uint64_t)(cb + pl.ovf_b) * 2);
        off[12] = take(sb * (uint64_t)(cp + pl.ovf_p) * 2);
        uint64_t bins_bytes = 8 * (uint64_t)(nbins + 1) * 4 + 4 * (uint64_t)nbins * 4 + 256;
        off[13] = take(bins_bytes);
        int64_t items_cap = (cb + cp + pl.ovf_b + pl.ovf_p) / 4096 + 2 * nbins + 64;
        uint64_t wl_bytes = 16 * (uint64_t)(P.nz + 8) + 256 + 16 * (uint64_t)items_cap + 8 * (uint64_t)((2 * nbins) / 512 + 16) +
                            4 * (uint64_t)(2 * nbins + 8) + 8 * (uint64_t)(nbins + 8) + 4096 + 4096;
        off[14] = take(wl_bytes);
        off[20] = cb;  // slot capacities (not offsets)
        off[21] = cp;
        off[23] = bins_bytes;
        off[24] = items_cap;
    }
    int64_t nmax = std::max<int64_t>({pl.cap_b, pl.cap_p, P.nc, 1});
    off[15] = take(8 * 32 * (uint64_t)(nblocks(nmax, 256) + 16));  // reduction partials
    off[16] = take(8 * P.nc);                                       // previous Gauss residual
    off[17] = pl.record ? take(8 * 6 * P.nc) : 0;                   // adjoint scratch
    off[18] = take(8 * 6 * (uint64_t)std::max<int64_t>(b->n_macro, 1));  // normals staging
    off[19] = take(256);                                            // device flags + lab-probe sums
    off[22] = take(8 * 2 * (uint64_t)(nblocks(nmax, 256) + 4));     // scan scratch
    if (o->init_fields == 2) {
        off[25] = take(8 * 3 * (uint64_t)P.nc);  // neutralising charge: its field
        off[26] = take(8 * (uint64_t)P.nc);      // and its node charge
    }
    pl.arena = a;
    // state: header + E, B + particles
    uint64_t fb = o->precision == PIC_FP64_PLAIN ? 8 : 4;
    uint64_t st = 256 + al256(6 * fb * P.nc);
    if (o->precision == PIC_FP64_PLAIN)
        st += al256(60 * (uint64_t)std::max<int64_t>(pl.cap_b, 1)) + al256(60 * (uint64_t)std::max<int64_t>(pl.cap_p, 1));
    else
        st = 256 + split_state_payload(P.nc, (int64_t)off[20] + pl.ovf_b, (int64_t)off[21] + pl.ovf_p, off[23],
                                       pl.record);
    pl.state = st;
    return PIC_OK;
}

static Part64 carve64(char *base, int64_t cap) {
    Part64 p;
    double *d = (double *)base;
    uint64_t c = (uint64_t)std::max<int64_t>(cap, 1);
    p.x = d;
    p.y = d + c;
    p.z = d + 2 * c;
    p.ux = d + 3 * c;
    p.uy = d + 4 * c;
    p.uz = d + 5 * c;
    p.w = d + 6 * c;
    p.alive = (int32_t *)(d + 7 * c);
    return p;
}

StepCtx make_step_ctx(const Ctx &c) {
    StepCtx S;
    memset(&S, 0, sizeof S);
    S.step = c.step;
    S.t = (double)c.step * c.P.dt;
    S.t1 = (double)(c.step + 1) * c.P.dt;
    S.k0 = c.k0;
    int64_t target = (int64_t)floor(c.win_x0 + c.bw * (S.t1 - c.win_t0));
    S.shift = c.k0 < target ? 1 : 0;
    S.k0n = c.k0 + S.shift;
    S.k0r = (int)(S.k0 % c.P.nz);
    S.k0nr = (int)(S.k0n % c.P.nz);
    return S;
}

// inject the nonzero-weight sheets of [l0, l1) at time t (FP64 mode slots)
static pic_status inject_range64(Ctx &c, int64_t l0, int64_t l1, double t) {
    int64_t sheet = sheet_particles(c.P);
    int64_t l = l0;
    while (l < l1) {
        while (l < l1 && sheet_weight(c.P, l) == 0.0) ++l;
        int64_t a = l;
        while (l < l1 && sheet_weight(c.P, l) != 0.0) ++l;
        if (l > a) {
            int64_t need = c.np_slots + (l - a) * sheet;
            if (need > c.cap_p) {
                c.err = "plasma capacity exceeded: raise options.max_steps (record mode) or check_every";
                return PIC_ENOMEM;
            }
            launch_inject64(c.P, a, l - a, t, c.p64, c.np_slots, c.st);
            c.np_slots = need;
        }
    }
    return PIC_OK;
}

static pic_status end_of_step_sheets(Ctx &c, const StepCtx &S) {
    int64_t l0 = c.sh_hi;
    if (c.P.has_plasma) {
        double lo = (double)(S.k0n + 3), hi = (double)(S.k0n + c.P.nz - 4);
        while (c.sh_lo < c.sh_hi && sheet_z(c.sh_lo, c.P.ppz, c.P.bR, S.t1) < lo) c.sh_lo++;
        while (sheet_z(c.sh_hi, c.P.ppz, c.P.bR, S.t1) < hi) c.sh_hi++;
        if (c.sh_lo > c.sh_hi) c.sh_lo = c.sh_hi;
    }
    if (c.precision == PIC_FP64_PLAIN) return c.P.has_plasma ? inject_range64(c, l0, c.sh_hi, S.t1) : PIC_OK;
    return split_inject_and_swap(c, l0, c.sh_hi, S.t1, S.k0n);  // FP32: append to the output bins, then swap
}

static pic_status check_flags(Ctx &c) {
    int32_t h = 0;
    PIC_HIP(c, hipMemcpyAsync(&h, c.dflags, sizeof h, hipMemcpyDeviceToHost, c.st));
    PIC_HIP(c, hipStreamSynchronize(c.st));
    if (h & DFLAG_FIXED_OVERFLOW) {
        c.err = "fixed-point current overflow: lower fixed_point_frac_bits";
        return PIC_ERANGE;
    }
    if (h & DFLAG_NONFINITE) {
        c.err = "non-finite particle momentum";
        return PIC_ESTATE;
    }
    if (h & DFLAG_BIN_LOST) {
        c.err = "particle bins and overflow area full: particles were lost";
        return PIC_ENOMEM;
    }
    return PIC_OK;
}

static hipEvent_t pool_get(Ctx &c) {
    if (c.ev_pool.empty()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = c.ev_pool.back();
    c.ev_pool.pop_back();
    return e;
}

hipEvent_t timing_begin(Ctx &c) {
    if (!c.timing) return nullptr;
    hipEvent_t e = pool_get(c);
    if (e) (void)hipEventRecord(e, c.st);
    return e;
}

void timing_end(Ctx &c, int cls, hipEvent_t start) {
    if (!c.timing || !start) return;
    hipEvent_t e = pool_get(c);
    if (!e) return;
    (void)hipEventRecord(e, c.st);
    c.ev_used.push_back({cls, {start, e}});
}

static pic_status step64(Ctx &c) {
    StepCtx S = make_step_ctx(c);
    FieldsT<double> f;
    for (int k = 0; k < 3; ++k) {
        f.E[k] = c.E64[k];
        f.B[k] = c.B64[k];
    }
    const Params &P = c.P;
    hipEvent_t t0 = timing_begin(c);
    launch_bhalf<double>(P, S.k0r, f, 0.5 * P.dt, nullptr, c.st);
    timing_end(c, 1, t0);
    hipEvent_t t1 = timing_begin(c);
    launch_step64(P, S, c.b64, c.nb_slots, f, c.J64, c.dflags, c.st);
    launch_step64(P, S, c.p64, c.np_slots, f, c.J64, c.dflags, c.st);
    timing_end(c, 0, t1);
    hipEvent_t t2 = timing_begin(c);
    if (P.ions) launch_ion64(P, c.sh_lo, c.sh_hi - c.sh_lo, S.t, S.t1, S.k0, c.jion64, c.st);
    launch_neutraliser_current(c, S);
    timing_end(c, 2, t2);
    hipEvent_t t3 = timing_begin(c);
    launch_bhalf<double>(P, S.k0r, f, 0.5 * P.dt, (double *)c.murbuf, c.st);
    launch_eupdate<double, double>(P, S.k0r, f, c.J64, c.jion64, P.dt, c.st);
    launch_mur_shift<double, double>(P, S.k0r, S.shift, c.bw <= 0.0, f, (const double *)c.murbuf, c.jion64, P.dt,
                                     c.st);
    timing_end(c, 1, t3);
    c.step += 1;
    c.k0 = S.k0n;
    hipEvent_t t4 = timing_begin(c);
    pic_status s = end_of_step_sheets(c, S);
    timing_end(c, 2, t4);
    if (s != PIC_OK) return s;
    if (!c.record && c.P.has_plasma && (c.step % c.check_every == 0 || c.cap_p - c.np_slots < 4 * sheets_per_step(P) * sheet_particles(P))) {
        int64_t n = compact64(c, c.p64, c.p64alt, c.np_slots);
        std::swap(c.p64, c.p64alt);
        c.np_slots = n;
    }
    return PIC_OK;
}

// ---------------------------------------------------------------- beam draws from a seed
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds, each two 32 x 32 -> 64-bit
// products of counter words with fixed multipliers whose high halves are mixed (xor) with the
// other two counter words and the key; the key advances by two Weyl constants between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
    }
}

// the beam's standard normals from the seed, as pic_beam defines them: row r of particle p at
// out[r n + p] (rows x, y, z, ux, uy, energy), one thread per particle
__global__ void __launch_bounds__(256) k_beam_normals(uint64_t seed, int64_t n, double *out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t w[8];
    for (int j = 0; j < 2; ++j) {
        uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), (uint32_t)j, 0u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        for (int q = 0; q < 4; ++q) w[4 * j + q] = c[q];
    }
    const double two_m32 = 2.3283064365386963e-10;  // 2^-32: U in (0, 1), never 0 or 1
    for (int r = 0; r < 3; ++r) {
        const double ua = ((double)w[2 * r] + 0.5) * two_m32, ub = ((double)w[2 * r + 1] + 0.5) * two_m32;
        const double rad = sqrt(-2.0 * log(ua));
        double s, co;
        sincospi(2.0 * ub, &s, &co);  // sin and cos of 2 pi ub
        out[(2 * r) * n + p] = rad * co;
        out[(2 * r + 1) * n + p] = rad * s;
    }
}

}  // namespace pic

using namespace pic;

struct pic_ctx : public Ctx {};

extern "C" {

pic_status pic_query_layout(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                            const pic_undulator *u, const pic_options *o, pic_layout *out) {
    if (!out) return PIC_EINVAL;
    Plan pl;
    pic_status s = make_plan(g, f, b, p, u, o, pl, nullptr);
    if (s != PIC_OK) return s;
    out->arena_bytes = pl.arena;
    out->state_bytes = pl.state;
    out->beam_capacity = o->precision == PIC_FP64_PLAIN ? pl.cap_b : (int64_t)pl.off[20] + pl.ovf_b;
    out->plasma_capacity = o->precision == PIC_FP64_PLAIN ? pl.cap_p : (int64_t)pl.off[21] + pl.ovf_p;
    return PIC_OK;
}

pic_status pic_derive(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                      const pic_undulator *u, const pic_options *o, pic_derived *out) {
    if (!out) return PIC_EINVAL;
    Params P;
    return derive_params(g, f, b, p, u, o, P, *out, nullptr);
}

const char *pic_last_error(const pic_ctx *c) { return c ? c->err.c_str() : "null context"; }

pic_status pic_init(const pic_grid *g, const pic_frame *f, const pic_beam *b, const pic_plasma *p,
                    const pic_undulator *u, const pic_options *o, void *arena, uint64_t arena_bytes,
                    pic_ctx **out) {
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    Plan pl;
    std::string err;
    pic_status s = make_plan(g, f, b, p, u, o, pl, &err);
    if (s != PIC_OK) {
        fprintf(stderr, "pic_init: %s\n", err.c_str());
        return s;
    }
    if (!arena || arena_bytes < pl.arena || ((uintptr_t)arena & 255)) {
        fprintf(stderr, "pic_init: arena missing, misaligned or smaller than %llu bytes\n",
                (unsigned long long)pl.arena);
        return PIC_ENOMEM;
    }
    pic_ctx *c = new pic_ctx();
    c->P = pl.P;
    c->precision = pl.precision;
    c->record = pl.record;
    c->check_every = pl.check_every;
    c->grid = *g;
    c->frame = *f;
    c->beam = *b;
    c->beam.normals = nullptr;
    c->plasma = *p;
    c->und = *u;
    c->opt = *o;
    c->st = (hipStream_t)o->stream;
    c->arena = (char *)arena;
    c->arena_bytes = arena_bytes;
    c->state_bytes = pl.state;
    c->cap_b = pl.cap_b;
    c->cap_p = pl.cap_p;
    c->k_bunch_default = pl.d.k_bunch;
    hipGetDevice(&c->device);
    if (static_scratch_setup(*c) != PIC_OK) {  // the device address of pic_diag_static's array, once per device
        fprintf(stderr, "pic_init: %s\n", c->err.c_str());
        delete c;
        return PIC_EDEVICE;
    }
    const Params &P = c->P;
    char *A = c->arena;
    uint64_t *off = pl.off;
    c->red = (double *)(A + off[15]);
    c->red_cap = (int64_t)(32 * (nblocks(std::max<int64_t>({pl.cap_b, pl.cap_p, P.nc, 1}), 256) + 16));
    c->rprev = (double *)(A + off[16]);
    c->adj = pl.record ? (double *)(A + off[17]) : nullptr;
    c->stage = (double *)(A + off[18]);
    c->dflags = (int32_t *)(A + off[19]);
    c->probe_acc = (double *)(A + off[19] + 64);  // same 256-byte block: flags, then the probe's sums
    c->i64scratch = (int64_t *)(A + off[22]);
    c->murbuf = A + off[10];
    if (o->init_fields == 2) {
        for (int k = 0; k < 3; ++k) c->fc_E[k] = (double *)(A + off[25]) + k * P.nc;
        c->fc_rho = (double *)(A + off[26]);
    }
    hipError_t e = hipMemsetAsync(c->dflags, 0, 256, c->st);
    if (e == hipSuccess) e = hipMemsetAsync(A + off[9], 0, 8 * P.nz, c->st);
    if (pl.precision == PIC_FP64_PLAIN) {
        for (int k = 0; k < 3; ++k) {
            c->E64[k] = (double *)(A + off[k]);
            c->B64[k] = (double *)(A + off[3 + k]);
            c->J64[k] = (double *)(A + off[6 + k]);
        }
        c->jion64 = (double *)(A + off[9]);
        if (e == hipSuccess) e = hipMemsetAsync(A + off[0], 0, off[9] - off[0], c->st);
        c->b64 = carve64(A + off[11], c->cap_b);
        c->p64 = carve64(A + off[12], c->cap_p);
        if (!pl.record) c->p64alt = carve64(A + off[13], c->cap_p);
        if (e == hipSuccess) e = hipMemsetAsync(c->b64.alive, 0, 4 * std::max<int64_t>(c->cap_b, 1), c->st);
    } else {
        for (int k = 0; k < 3; ++k) {
            c->E32[k] = (float *)(A + off[k]);
            c->B32[k] = (float *)(A + off[3 + k]);
            c->Ji[k] = (long long *)(A + off[6 + k]);
        }
        c->jioni = (long long *)(A + off[9]);
        if (e == hipSuccess) e = hipMemsetAsync(A + off[0], 0, off[9] - off[0], c->st);
    }
    if (e != hipSuccess) {
        hip_check(*c, e, "pic_init memset");
        fprintf(stderr, "pic_init: %s\n", c->err.c_str());
        delete c;
        return PIC_EDEVICE;
    }
    // beam: normals to the device (or drawn there from the seed), FP64 transform
    double bw = 0.0;
    if (b->n_macro > 0) {
        if (b->normals) {
            e = hipMemcpyAsync(c->stage, b->normals, 8 * 6 * (uint64_t)b->n_macro, hipMemcpyHostToDevice, c->st);
        } else {
            hipLaunchKernelGGL(k_beam_normals, dim3(nblocks(b->n_macro, 256)), dim3(256), 0, c->st, b->seed,
                               b->n_macro, c->stage);
            e = hipGetLastError();
        }
        if (e != hipSuccess) {
            hip_check(*c, e, b->normals ? "normals upload" : "normals from the seed");
            delete c;
            return PIC_EDEVICE;
        }
    }
    if (pl.precision == PIC_FP64_PLAIN) {
        c->nb_slots = b->n_macro;
        if (b->n_macro > 0) {
            double D = g->dx_m;
            double sig[5] = {b->sigma_cells[0], b->sigma_cells[1], pl.d.sigma_z_lab_cells,
                             b->emit_n_m[0] / (b->sigma_cells[0] * D), b->emit_n_m[1] / (b->sigma_cells[1] * D)};
            int nblk = nblocks(b->n_macro, 256);
            launch_beam_init64(P, c->stage, b->n_macro, sig, b->gamma_lab, b->rel_energy_spread_rms, c->b64, c->red,
                               nblk, c->st);
            std::vector<double> h(2 * (size_t)nblk);
            hipMemcpyAsync(h.data(), c->red, 16 * (uint64_t)nblk, hipMemcpyDeviceToHost, c->st);
            hipStreamSynchronize(c->st);
            double cnt = 0, vz = 0;
            for (int k = 0; k < nblk; ++k) {
                cnt += h[2 * k];
                vz += h[2 * k + 1];
            }
            bw = cnt > 0 ? vz / cnt : 0.0;
        }
        c->beam_beta0 = bw;
    } else {
        c->split_slots_b = (int64_t)off[20];
        c->split_slots_p = (int64_t)off[21];
        c->ovf_cap_b = pl.ovf_b;
        c->ovf_cap_p = pl.ovf_p;
        c->split_off_b = off[11];
        c->split_off_p = off[12];
        c->split_off_bins = off[13];
        c->split_bins_bytes = off[23];
        c->split_off_wl = off[14];
        c->split_items_cap = (int64_t)off[24];
        c->nb_slots = b->n_macro;  // ids: beam particle k is FP64 record slot k; plasma ids count up
        c->np_slots = 0;
        split_setup(*c);
        if (b->n_macro > 0) split_beam_init(*c, c->stage);
        c->beam_beta0 = c->bw;
    }
    c->bw = f->window_beta >= 0 ? f->window_beta : (pl.precision == PIC_FP64_PLAIN ? bw : c->bw);
    // plasma lattice at t' = 0 inside the active band
    if (P.has_plasma) {
        c->sh_lo = (int64_t)3 * P.ppz;
        c->sh_hi = (int64_t)(P.nz - 4) * P.ppz;
    }
    if (pl.precision == PIC_FP64_PLAIN) {
        if (P.has_plasma) s = inject_range64(*c, c->sh_lo, c->sh_hi, 0.0);
    } else {
        s = split_plasma_fill(*c);
    }
    if (s == PIC_OK && o->init_fields == 1 && b->n_macro > 0) s = init_beam_fields(*c);
    if (s == PIC_OK && o->init_fields == 2 && b->n_macro > 0) {
        c->fc_T = o->neutral_fade_s * kC / g->dx_m;
        s = init_neutraliser(*c);
    }
    if (s != PIC_OK) {
        fprintf(stderr, "pic_init: %s\n", c->err.c_str());
        if (c->split) split_free(*c);
        delete c;
        return s;
    }
    e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        hip_check(*c, e, "pic_init");
        fprintf(stderr, "pic_init: %s\n", c->err.c_str());
        delete c;
        return PIC_EDEVICE;
    }
    *out = c;
    return PIC_OK;
}

pic_status pic_step(pic_ctx *c, int32_t nsteps) {
    if (!c || nsteps < 0) return PIC_EINVAL;
    for (int32_t n = 0; n < nsteps; ++n) {
        pic_status s;
        hipEvent_t ts = timing_begin(*c);
        if (c->precision == PIC_FP64_PLAIN) {
            s = step64(*c);
        } else {
            StepCtx S = make_step_ctx(*c);
            split_step(*c, S);
            c->step += 1;
            c->k0 = S.k0n;
            hipEvent_t ti = timing_begin(*c);
            s = end_of_step_sheets(*c, S);
            timing_end(*c, 2, ti);
            if (s == PIC_OK && c->step % c->check_every == 0) s = split_check(*c);
        }
        if (s == PIC_OK && c->probe_on) probe_step(*c);
        timing_end(*c, 3, ts);
        if (s != PIC_OK) return s;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_check(*c, e, "pic_step launch");
    return PIC_OK;
}

pic_status pic_lab_probe(pic_ctx *c, double t_lab, double k_lab) {
    if (!c) return PIC_EINVAL;
    if (!std::isfinite(k_lab)) {
        c->err = "pic_lab_probe: k_lab must be finite";
        return PIC_EINVAL;
    }
    c->probe_on = std::isfinite(t_lab) ? 1 : 0;
    c->probe_t = t_lab;
    c->probe_k = k_lab;
    PIC_HIP(*c, hipMemsetAsync(c->probe_acc, 0, 5 * sizeof(double), c->st));
    return PIC_OK;
}

pic_status pic_lab_probe_read(pic_ctx *c, double out[5]) {
    if (!c || !out) return PIC_EINVAL;
    PIC_HIP(*c, hipMemcpyAsync(out, c->probe_acc, 5 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    PIC_HIP(*c, hipStreamSynchronize(c->st));
    return PIC_OK;
}

pic_status pic_timing(pic_ctx *c, int32_t enable) {
    if (!c) return PIC_EINVAL;
    PIC_HIP(*c, hipStreamSynchronize(c->st));
    for (auto &u : c->ev_used) {
        c->ev_pool.push_back(u.second.first);
        c->ev_pool.push_back(u.second.second);
    }
    c->ev_used.clear();
    c->timing = enable ? 1 : 0;
    return PIC_OK;
}

pic_status pic_timing_read(pic_ctx *c, double ms[4], int64_t launches[4]) {
    if (!c || !ms || !launches) return PIC_EINVAL;
    PIC_HIP(*c, hipStreamSynchronize(c->st));
    for (int k = 0; k < 4; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &u : c->ev_used) {
        float t = 0.f;
        PIC_HIP(*c, hipEventElapsedTime(&t, u.second.first, u.second.second));
        ms[u.first] += t;
        launches[u.first] += 1;
    }
    return PIC_OK;
}

pic_status pic_set_window_beta(pic_ctx *c, double beta) {
    if (!c) return PIC_EINVAL;
    if (!(beta >= 0.0 && beta <= 1.0)) {
        c->err = "pic_set_window_beta: beta must lie in [0, 1]";
        return PIC_EINVAL;
    }
    if ((c->bw > 0.0) != (beta > 0.0)) {
        c->err = "pic_set_window_beta: a moving window cannot stop, nor a window at rest start moving";
        return PIC_EINVAL;
    }
    const double t = (double)c->step * c->P.dt;
    c->win_x0 = c->win_x0 + c->bw * (t - c->win_t0);
    c->win_t0 = t;
    c->bw = beta;
    return PIC_OK;
}

pic_status pic_sync(pic_ctx *c) {
    if (!c) return PIC_EINVAL;
    PIC_HIP(*c, hipStreamSynchronize(c->st));
    return check_flags(*c);
}

pic_status pic_diag(pic_ctx *c, uint32_t mask, double bunch_period_cells, pic_diag_out *out) {
    if (!c || !out) return PIC_EINVAL;
    pic_status s = pic_sync(c);
    if (s != PIC_OK) return s;
    double kb = bunch_period_cells > 0 ? 2.0 * kPi / bunch_period_cells : c->k_bunch_default;
    return run_diag(*c, mask, kb, out, c->red, c->red_cap);
}

pic_status pic_diag_static(pic_ctx *c, uint32_t mask, double bunch_period_cells, pic_diag_out *out) {
    if (!c || !out) return PIC_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
        c->err = "pic_diag_static: the context's device must be current";
        return PIC_EINVAL;
    }
    double *red = static_scratch(c->device);
    if (!red) {
        c->err = "pic_diag_static: no static scratch on this device";
        return PIC_EDEVICE;
    }
    const int64_t need = diag_partials(*c, mask);
    if (need > DIAG_STATIC_DOUBLES) {
        char msg[160];
        snprintf(msg, sizeof msg, "pic_diag_static: %lld partial sums exceed the static scratch of %lld doubles",
                 (long long)need, (long long)DIAG_STATIC_DOUBLES);
        c->err = msg;
        return PIC_ERANGE;
    }
    pic_status s = pic_sync(c);
    if (s != PIC_OK) return s;
    double kb = bunch_period_cells > 0 ? 2.0 * kPi / bunch_period_cells : c->k_bunch_default;
    return run_diag(*c, mask, kb, out, red, DIAG_STATIC_DOUBLES);
}

// copy logical planes of a field into dst (double), un-rotating the ring
__global__ void k_f2d(const float *a, double *b, int64_t n) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) b[q] = (double)a[q];
}

__global__ void k_field_out(const void *src, int isfloat, double *dst, int64_t plane, int nz, int k0r) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= plane * nz) return;
    int l = (int)(q / plane);
    int64_t s = q % plane;
    int64_t o = (int64_t)ring_plane(l, k0r, nz) * plane + s;
    dst[q] = isfloat ? (double)((const float *)src)[o] : ((const double *)src)[o];
}

__global__ void k_field_in(void *dst, int isfloat, const double *src, int64_t plane, int nz, int k0r) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= plane * nz) return;
    int l = (int)(q / plane);
    int64_t s = q % plane;
    int64_t o = (int64_t)ring_plane(l, k0r, nz) * plane + s;
    if (isfloat)
        ((float *)dst)[o] = (float)src[q];
    else
        ((double *)dst)[o] = src[q];
}

pic_status pic_read(pic_ctx *c, int32_t which, void *dst, int64_t *count) {
    if (!c) return PIC_EINVAL;
    const Params &P = c->P;
    int k0r = (int)(c->k0 % P.nz);
    if (which >= PIC_A_EX && which <= PIC_A_BZ) {
        if (count) *count = P.nc;
        if (!dst) return PIC_OK;
        const void *src = c->precision == PIC_FP64_PLAIN
                              ? (const void *)(which < 3 ? c->E64[which] : c->B64[which - 3])
                              : (const void *)(which < 3 ? c->E32[which] : c->B32[which - 3]);
        hipLaunchKernelGGL(k_field_out, dim3(nblocks(P.nc, 256)), dim3(256), 0, c->st, src,
                           c->precision == PIC_FP32_SPLIT, (double *)dst, (int64_t)P.plane, P.nz, k0r);
        PIC_HIP(*c, hipStreamSynchronize(c->st));
        return PIC_OK;
    }
    if (which >= PIC_A_BEAM && which <= PIC_A_PLASMA_ALIVE) {
        int sp = which >= PIC_A_PLASMA;
        int alive = (which - PIC_A_BEAM) % 2;
        if (c->precision == PIC_FP64_PLAIN) {
            int64_t n = sp ? c->np_slots : c->nb_slots;
            if (count) *count = n;
            if (!dst || n == 0) return PIC_OK;
            Part64 p = sp ? c->p64 : c->b64;
            if (alive) {
                PIC_HIP(*c, hipMemcpyAsync(dst, p.alive, 4 * n, hipMemcpyDeviceToDevice, c->st));
            } else {
                double *arr[7] = {p.x, p.y, p.z, p.ux, p.uy, p.uz, p.w};
                for (int k = 0; k < 7; ++k)
                    PIC_HIP(*c, hipMemcpyAsync((double *)dst + (uint64_t)k * n, arr[k], 8 * n,
                                               hipMemcpyDeviceToDevice, c->st));
            }
            PIC_HIP(*c, hipStreamSynchronize(c->st));
            return PIC_OK;
        }
        int64_t n = 0;
        split_read(*c, sp, nullptr, nullptr, &n);
        if (count) *count = n;
        if (!dst || n == 0) return PIC_OK;
        if (alive)
            split_read(*c, sp, nullptr, (int32_t *)dst, &n);
        else
            split_read(*c, sp, (double *)dst, nullptr, &n);
        PIC_HIP(*c, hipStreamSynchronize(c->st));
        return PIC_OK;
    }
    if (which == PIC_A_BEAM_LAB) {
        int64_t n = 0;
        pic_status st = lab_beam(*c, nullptr, &n);
        if (count) *count = n;
        if (st != PIC_OK || !dst || n == 0) return st;
        return lab_beam(*c, (double *)dst, &n);
    }
    c->err = "pic_read: unknown array";
    return PIC_EINVAL;
}

pic_status pic_lab_groups(pic_ctx *c, const pic_lab_groups_spec *spec, void *dst) {
    if (!c || !spec || !dst) return PIC_EINVAL;
    if (spec->nz < 1 || spec->nu < 1 || (int64_t)spec->nz * spec->nu > LAB_GROUPS_MAX || !(spec->dz > 0.0) ||
        !(spec->du > 0.0) || !std::isfinite(spec->z_lo) || !std::isfinite(spec->u_lo)) {
        c->err = "pic_lab_groups: need dz, du > 0, finite lower edges and 1 <= nz * nu <= 256 groups";
        return PIC_EINVAL;
    }
    LabGroupSpec G{spec->z_lo, spec->dz, spec->u_lo, spec->du, spec->nz, spec->nu};
    return lab_groups(*c, G, (double *)dst);
}

pic_status pic_write(pic_ctx *c, int32_t which, const void *src, int64_t count) {
    if (!c || !src) return PIC_EINVAL;
    const Params &P = c->P;
    int k0r = (int)(c->k0 % P.nz);
    if (which >= PIC_A_EX && which <= PIC_A_BZ) {
        if (count != P.nc) return PIC_EINVAL;
        void *d = c->precision == PIC_FP64_PLAIN ? (void *)(which < 3 ? c->E64[which] : c->B64[which - 3])
                                                 : (void *)(which < 3 ? c->E32[which] : c->B32[which - 3]);
        hipLaunchKernelGGL(k_field_in, dim3(nblocks(P.nc, 256)), dim3(256), 0, c->st, d,
                           c->precision == PIC_FP32_SPLIT, (const double *)src, (int64_t)P.plane, P.nz, k0r);
        PIC_HIP(*c, hipStreamSynchronize(c->st));
        return PIC_OK;
    }
    if ((which == PIC_A_BEAM || which == PIC_A_PLASMA) && c->precision == PIC_FP64_PLAIN) {
        int sp = which == PIC_A_PLASMA;
        int64_t n = sp ? c->np_slots : c->nb_slots;
        if (count != n) {
            c->err = "pic_write: count must equal the slot count";
            return PIC_EINVAL;
        }
        Part64 p = sp ? c->p64 : c->b64;
        double *arr[7] = {p.x, p.y, p.z, p.ux, p.uy, p.uz, p.w};
        for (int k = 0; k < 7; ++k)
            PIC_HIP(*c, hipMemcpyAsync(arr[k], (const double *)src + (uint64_t)k * n, 8 * n,
                                       hipMemcpyDeviceToDevice, c->st));
        PIC_HIP(*c, hipStreamSynchronize(c->st));
        return PIC_OK;
    }
    c->err = "pic_write: unsupported array for this precision";
    return PIC_EINVAL;
}

// state header (host scalars)
struct StateHeader {
    uint64_t magic, bytes;
    int64_t step, k0, sh_lo, sh_hi, nb_slots, np_slots;
    int32_t cur32, precision;
    double bw, win_x0, win_t0;
};

pic_status pic_get_state(pic_ctx *c, void *dst) {
    if (!c || !dst) return PIC_EINVAL;
    char *d = (char *)dst;
    StateHeader h = {0x5049435354415445ull, c->state_bytes, c->step, c->k0, c->sh_lo, c->sh_hi,
                     c->nb_slots, c->np_slots, c->cur32, c->precision, c->bw, c->win_x0, c->win_t0};
    PIC_HIP(*c, hipMemcpyAsync(d, &h, sizeof h, hipMemcpyHostToDevice, c->st));
    uint64_t o = 256;
    const Params &P = c->P;
    if (c->precision == PIC_FP64_PLAIN) {
        PIC_HIP(*c, hipMemcpyAsync(d + o, c->E64[0], 8 * 6 * P.nc, hipMemcpyDeviceToDevice, c->st));
        o += al256(8 * 6 * P.nc);
        uint64_t bb = 60 * (uint64_t)std::max<int64_t>(c->cap_b, 1), pb = 60 * (uint64_t)std::max<int64_t>(c->cap_p, 1);
        PIC_HIP(*c, hipMemcpyAsync(d + o, c->b64.x, bb, hipMemcpyDeviceToDevice, c->st));
        o += al256(bb);
        PIC_HIP(*c, hipMemcpyAsync(d + o, c->p64.x, pb, hipMemcpyDeviceToDevice, c->st));
    } else {
        pic_status st = split_copy_state(*c, d + o, true);
        if (st != PIC_OK) return st;
    }
    PIC_HIP(*c, hipStreamSynchronize(c->st));
    return PIC_OK;
}

pic_status pic_set_state(pic_ctx *c, const void *src) {
    if (!c || !src) return PIC_EINVAL;
    const char *d = (const char *)src;
    StateHeader h;
    PIC_HIP(*c, hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, c->st));
    PIC_HIP(*c, hipStreamSynchronize(c->st));
    if (h.magic != 0x5049435354415445ull || h.bytes != c->state_bytes || h.precision != c->precision) {
        c->err = "pic_set_state: snapshot does not belong to this configuration";
        return PIC_ESTATE;
    }
    const Params &P = c->P;
    uint64_t o = 256;
    if (c->precision == PIC_FP64_PLAIN) {
        PIC_HIP(*c, hipMemcpyAsync(c->E64[0], d + o, 8 * 6 * P.nc, hipMemcpyDeviceToDevice, c->st));
        o += al256(8 * 6 * P.nc);
        uint64_t bb = 60 * (uint64_t)std::max<int64_t>(c->cap_b, 1), pb = 60 * (uint64_t)std::max<int64_t>(c->cap_p, 1);
        PIC_HIP(*c, hipMemcpyAsync(c->b64.x, d + o, bb, hipMemcpyDeviceToDevice, c->st));
        o += al256(bb);
        PIC_HIP(*c, hipMemcpyAsync(c->p64.x, d + o, pb, hipMemcpyDeviceToDevice, c->st));
    } else {
        c->cur32 = h.cur32;  // the snapshot's particles go to the buffer they came from
        pic_status st = split_copy_state(*c, (char *)d + o, false);
        if (st != PIC_OK) return st;
    }
    c->step = h.step;
    c->k0 = h.k0;
    c->sh_lo = h.sh_lo;
    c->sh_hi = h.sh_hi;
    c->nb_slots = h.nb_slots;
    c->np_slots = h.np_slots;
    c->cur32 = h.cur32;
    c->bw = h.bw;
    c->win_x0 = h.win_x0;
    c->win_t0 = h.win_t0;
    PIC_HIP(*c, hipStreamSynchronize(c->st));
    return PIC_OK;
}

int64_t pic_lambda_len(const pic_ctx *c) {
    if (!c) return 0;
    return 6 * (std::max<int64_t>(c->cap_b, 1) + std::max<int64_t>(c->cap_p, 1)) + 6 * c->P.nc;
}

pic_status pic_adjoint_seed_bunching(pic_ctx *c, double bunch_period_cells, void *lam, double *loss) {
    if (!c || !lam) return PIC_EINVAL;
    if (!c->record || c->precision != PIC_FP64_PLAIN) {
        c->err = "adjoint needs FP64 mode with record = 1";
        return PIC_ESTATE;
    }
    if (c->P.mobile) {
        c->err = "adjoint: mobile ions are not supported";
        return PIC_EINVAL;
    }
    double kb = bunch_period_cells > 0 ? 2.0 * kPi / bunch_period_cells : c->k_bunch_default;
    return adjoint_seed(*c, kb, (double *)lam, loss);
}

pic_status pic_adjoint_step(pic_ctx *c, void *lam, double grad[2]) {
    if (!c || !lam || !grad) return PIC_EINVAL;
    if (!c->record || c->precision != PIC_FP64_PLAIN) {
        c->err = "adjoint needs FP64 mode with record = 1";
        return PIC_ESTATE;
    }
    if (c->P.mobile) {
        c->err = "adjoint: mobile ions are not supported";
        return PIC_EINVAL;
    }
    return adjoint_step(*c, (double *)lam, grad);
}

pic_status pic_state_to_fp64(const pic_ctx *src, pic_ctx *dst) {
    if (!src || !dst) return PIC_EINVAL;
    if (src->precision != PIC_FP32_SPLIT || !src->record || dst->precision != PIC_FP64_PLAIN || !dst->record) {
        dst->err = "pic_state_to_fp64: needs an FP32 context and an FP64 context, both with record = 1";
        return PIC_EINVAL;
    }
    const Params &A = src->P, &B = dst->P;
    if (A.nx != B.nx || A.ny != B.ny || A.nz != B.nz || A.dt != B.dt || A.gR != B.gR || A.wbeam != B.wbeam ||
        A.wsheet != B.wsheet || A.und_kind != B.und_kind || A.pusher != B.pusher) {
        dst->err = "pic_state_to_fp64: the two contexts differ in configuration";
        return PIC_EINVAL;
    }
    if (src->nb_slots > dst->cap_b || src->np_slots > dst->cap_p) {
        dst->err = "pic_state_to_fp64: FP64 slot capacity too small: raise its options.max_steps";
        return PIC_ENOMEM;
    }
    Ctx &d = *dst;
    // fields: same ring layout once the window origin is copied
    for (int k = 0; k < 3; ++k) {
        hipLaunchKernelGGL(k_f2d, dim3(nblocks(B.nc, 256)), dim3(256), 0, d.st, (const float *)src->E32[k], d.E64[k],
                           B.nc);
        hipLaunchKernelGGL(k_f2d, dim3(nblocks(B.nc, 256)), dim3(256), 0, d.st, (const float *)src->B32[k], d.B64[k],
                           B.nc);
        PIC_HIP(d, hipMemsetAsync(d.J64[k], 0, 8 * (uint64_t)B.nc, d.st));
    }
    PIC_HIP(d, hipMemsetAsync(d.jion64, 0, 8 * (uint64_t)B.nz, d.st));
    // particles to their slots; slots without a particle are dead
    PIC_HIP(d, hipMemsetAsync(d.b64.alive, 0, 4 * (uint64_t)std::max<int64_t>(d.cap_b, 1), d.st));
    PIC_HIP(d, hipMemsetAsync(d.p64.alive, 0, 4 * (uint64_t)std::max<int64_t>(d.cap_p, 1), d.st));
    split_export64(*src, d.b64, d.p64, d.st);
    d.step = src->step;
    d.k0 = src->k0;
    d.sh_lo = src->sh_lo;
    d.sh_hi = src->sh_hi;
    d.nb_slots = src->nb_slots;
    d.np_slots = src->np_slots;
    d.bw = src->bw;
    d.win_x0 = src->win_x0;
    d.win_t0 = src->win_t0;
    PIC_HIP(d, hipStreamSynchronize(d.st));
    return PIC_OK;
}

void pic_free(pic_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    for (auto &u : c->ev_used) {
        (void)hipEventDestroy(u.second.first);
        (void)hipEventDestroy(u.second.second);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->split) split_free(*c);
    delete c;
}

}  // extern "C"
