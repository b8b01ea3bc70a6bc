// dev_common.h -- device-side building blocks shared by the HIP kernels:
// run parameters, ring-buffer indexing of the moving window, quadratic
// B-spline weights, the boosted-frame undulator field and the pushers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// Normalised run constants (length = cell edge D, time = D / c).
struct Params {
    int nx, ny, nz, plane;      // plane = nx * ny
    int64_t nc;                 // cells
    double dt, gR, bR, uR;      // time step, frame gamma, beta, gamma*beta
    double zoff;                // z_lab = gR (z - zoff + bR t)
    // undulator (lab cells)
    int und_kind, pusher;
    double ku, z0u, Lu, Ru, B0;
    // plasma (lab cells)
    int has_plasma, ions, ppx, ppy, ppz, mobile;  // ions: immobile lab ions; mobile: ions as particles
    double n0n, z0p, Lp, Rp, wsheet; // wsheet = gR n0n / (ppx ppy ppz)
    double wbeam;
    double gthr;                // FP32 mode: FP64 push above this gamma
    int frac_bits, pad1;
    double fscale, finv;        // 2^frac_bits and its inverse
    int tx, ty, tz, ntx, nty, ntz, nbins, pad2;
    // FP32 mode: packed cell = i | j << cbx | l << (cbx + cby); tile edges 2^lgx, 2^lgy, 2^lgz
    int cbx, cby, lgx, lgy, lgz, pad3;
    // mobile ions: mass in electron masses, and the pusher's half-step factor 0.5 (q/m) dt = 0.5 dt / mi
    double mi, ahi;
    int pad4;
};

// Window position during one step (host-decided, deterministic from the step count).
struct StepCtx {
    int64_t step;
    double t, t1;       // t' at the start and end of the step
    int64_t k0;         // absolute plane of logical plane 0 during the step
    int64_t k0n;        // after the end-of-step shift
    int k0r, k0nr;      // ring offsets: k0 mod nz, k0n mod nz
    int shift, pad;
};

// Lab-frame probe of one particle after a step ending at boosted time t1: its
// position before the step is z1 - dt v_z (a straight move); if its lab time
// gR (t' + bR (z - zoff)) passes T during the step, its lab position there is
// added (w, w cos k z_lab, w sin k z_lab, w z_lab, w z_lab^2) to v.
__device__ inline void probe_particle(const Params &P, double z1, double ux, double uy, double uz, double w,
                                      double t1, double T, double k, double v[5]) {
    const double z0 = z1 - P.dt * uz / sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    const double t0 = t1 - P.dt;
    const double a = P.gR * (t0 + P.bR * (z0 - P.zoff)), b = P.gR * (t1 + P.bR * (z1 - P.zoff));
    if (!(a <= T && T < b)) return;
    const double f = (T - a) / (b - a);
    const double zl = P.gR * (z0 + f * (z1 - z0) - P.zoff + P.bR * (t0 + f * P.dt));
    double s, c;
    sincos(k * zl, &s, &c);
    v[0] += w;
    v[1] += w * c;
    v[2] += w * s;
    v[3] += w * zl;
    v[4] += w * zl * zl;
}

// Lab-frame phase space of a particle at boosted time t (section 2, the inverse
// of Eq. Lor1, Lor2): lab time gR (t + bR (z - zoff)), lab position
// gR (z - zoff + bR t), u_z,lab = gR (u_z + bR gamma), gamma_lab = gR (gamma + bR u_z);
// x, y, u_x, u_y are frame invariant.  Out: x y z_lab t_lab ux uy uz_lab gamma_lab.
__device__ inline void lab_of(const Params &P, double t, double x, double y, double z, double ux, double uy, double uz,
                              double out[8]) {
    const double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz), zr = z - P.zoff;
    out[0] = x;
    out[1] = y;
    out[2] = P.gR * (zr + P.bR * t);
    out[3] = P.gR * (t + P.bR * zr);
    out[4] = ux;
    out[5] = uy;
    out[6] = P.gR * (uz + P.bR * g);
    out[7] = P.gR * (g + P.bR * uz);
}

// Grouping of the beam (section 2: at one boosted instant a beam spans a lab
// time gR bR dz' over a slice dz' along the propagation direction, Eq. DT, and
// particles of unequal u'_z advance their lab time unequally): group of a
// particle by its boosted z' and u'_z slices; per group 16 values:
// count, sum w, sum w t_lab, min t_lab, max t_lab, sum w z_lab, sum w z_lab^2,
// sum w x, sum w x^2, sum w y, sum w y^2, sum w ux, sum w ux^2, sum w uy,
// sum w uy^2, sum w gamma_lab.
enum { LAB_GROUP_VALUES = 16, LAB_GROUPS_MAX = 256 };
struct LabGroupSpec {
    double z_lo, dz, u_lo, du;
    int nz, nu;
};
__device__ inline int lab_group_of(const LabGroupSpec &G, double z, double uz) {
    const double fz = floor((z - G.z_lo) / G.dz), fu = floor((uz - G.u_lo) / G.du);
    if (!(fz >= 0.0 && fz < G.nz && fu >= 0.0 && fu < G.nu)) return -1;
    return (int)fz * G.nu + (int)fu;
}

// a block's LDS table of groups (cleared by the block: counts and sums 0, min +inf, max -inf)
__device__ inline void lab_table_clear(double *tab, int ng) {
    for (int k = threadIdx.x; k < LAB_GROUP_VALUES * ng; k += blockDim.x) {
        const int v = k % LAB_GROUP_VALUES;
        tab[k] = v == 3 ? INFINITY : (v == 4 ? -INFINITY : 0.0);
    }
}
__device__ inline void lab_group_add(double *tab, const LabGroupSpec &G, const Params &P, double t, double x, double y,
                                     double z, double ux, double uy, double uz, double w) {
    const int g = lab_group_of(G, z, uz);
    if (g < 0) return;
    double L[8];
    lab_of(P, t, x, y, z, ux, uy, uz, L);
    double *e = tab + LAB_GROUP_VALUES * g;
    atomicAdd(&e[0], 1.0);
    atomicAdd(&e[1], w);
    atomicAdd(&e[2], w * L[3]);
    atomicMin(&e[3], L[3]);
    atomicMax(&e[4], L[3]);
    atomicAdd(&e[5], w * L[2]);
    atomicAdd(&e[6], w * L[2] * L[2]);
    atomicAdd(&e[7], w * L[0]);
    atomicAdd(&e[8], w * L[0] * L[0]);
    atomicAdd(&e[9], w * L[1]);
    atomicAdd(&e[10], w * L[1] * L[1]);
    atomicAdd(&e[11], w * L[4]);
    atomicAdd(&e[12], w * L[4] * L[4]);
    atomicAdd(&e[13], w * L[5]);
    atomicAdd(&e[14], w * L[5] * L[5]);
    atomicAdd(&e[15], w * L[7]);
}
// the block's nonempty groups into the global table
__device__ inline void lab_table_flush(const double *tab, int ng, double *out) {
    for (int k = threadIdx.x; k < LAB_GROUP_VALUES * ng; k += blockDim.x) {
        const int g = k / LAB_GROUP_VALUES, v = k % LAB_GROUP_VALUES;
        if (tab[LAB_GROUP_VALUES * g] == 0.0) continue;
        if (v == 3)
            atomicMin(&out[k], tab[k]);
        else if (v == 4)
            atomicMax(&out[k], tab[k]);
        else
            atomicAdd(&out[k], tab[k]);
    }
}

__host__ __device__ inline int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Ring plane of logical window plane l (0 <= l < nz).
__host__ __device__ inline int ring_plane(int l, int k0r, int nz) {
    int p = l + k0r;
    return p >= nz ? p - nz : p;
}

__host__ __device__ inline int64_t cell_index(const Params &P, int i, int j, int p) {
    return (int64_t)wrapi(i, P.nx) + (int64_t)P.nx * ((int64_t)wrapi(j, P.ny) + (int64_t)P.ny * p);
}

// Quadratic B-spline S(d) = 3/4 - d^2 (|d| <= 1/2), (3/2 - |d|)^2 / 2 (1/2 < |d| < 3/2).
template <typename T> __device__ inline T spline2(T d) {
    T a = d < T(0) ? -d : d;
    if (a <= T(0.5)) return T(0.75) - d * d;
    if (a < T(1.5)) {
        T t = T(1.5) - a;
        return T(0.5) * t * t;
    }
    return T(0);
}

template <typename T> __device__ inline T dspline2(T d) {
    T a = d < T(0) ? -d : d;
    if (a <= T(0.5)) return T(-2) * d;
    if (a < T(1.5)) return d >= T(0) ? -(T(1.5) - d) : (T(1.5) + d);
    return T(0);
}

// Three weights of the nearest node n and its neighbours for offset d = x - n, |d| <= 1/2.
template <typename T> __device__ inline void weights3(T d, T w[3]) {
    T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * b * b;
}

// ---------------------------------------------------------------- external field
// Lab field B = B0 env (cos phi, sin phi, 0) (helical) / (0, sin phi, 0) (planar),
// phi = k_u a with a = z_lab - z_start; boosted: B' = gR B_perp, E' = gR bR (zhat x B).
__device__ inline void und_env(const Params &P, double a, double &env, double &denv) {
    env = 0.0;
    denv = 0.0;
    if (a < 0.0 || a > P.Lu) return;
    if (P.Ru <= 0.0) {
        env = 1.0;
        return;
    }
    double up = a / P.Ru, dn = (P.Lu - a) / P.Ru;
    if (up < 1.0 && up <= dn) {
        env = up;
        denv = 1.0 / P.Ru;
    } else if (dn < 1.0) {
        env = dn;
        denv = -1.0 / P.Ru;
    } else
        env = 1.0;
}

// Field at boosted (z, t) plus its z derivative (FP64).
__device__ inline void ext_field64(const Params &P, double z, double t, double E[3], double B[3], double dE[3],
                                   double dB[3]) {
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
    dE[0] = dE[1] = dE[2] = dB[0] = dB[1] = dB[2] = 0.0;
    if (P.und_kind == 0) return;
    double a = P.gR * (z - P.zoff + P.bR * t) - P.z0u;
    double env, denv;
    und_env(P, a, env, denv);
    if (env == 0.0 && denv == 0.0) return;
    double sn, cs;
    sincos(P.ku * a, &sn, &cs);
    double bx, by, dbx, dby;
    if (P.und_kind == 1) {
        bx = P.B0 * env * cs;
        by = P.B0 * env * sn;
        dbx = P.B0 * (denv * cs - env * P.ku * sn);
        dby = P.B0 * (denv * sn + env * P.ku * cs);
    } else {
        bx = 0.0;
        dbx = 0.0;
        by = P.B0 * env * sn;
        dby = P.B0 * (denv * sn + env * P.ku * cs);
    }
    double ge = P.gR * P.bR;
    E[0] = -ge * by;
    E[1] = ge * bx;
    B[0] = P.gR * bx;
    B[1] = P.gR * by;
    dE[0] = -ge * P.gR * dby;
    dE[1] = ge * P.gR * dbx;
    dB[0] = P.gR * P.gR * dbx;
    dB[1] = P.gR * P.gR * dby;
}

// ---------------------------------------------------------------- pushers
// a = (q/m) dt / 2: -dt/2 for electrons, +dt / (2 M) for mobile ions of mass M
template <typename T> __device__ inline T dot3(const T a[3], const T b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <typename T> __device__ inline void cross3(const T a[3], const T b[3], T o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Boris: half kick, rotation, half kick.
template <typename T> __device__ inline void push_boris(T a, const T u[3], const T E[3], const T B[3], T out[3]) {
    T um[3], Tv[3], S[3], up[3], c[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + a * E[d];
    const T igm = T(1) / sqrt(T(1) + dot3(um, um));  // one division per push, then products
    for (int d = 0; d < 3; ++d) Tv[d] = a * B[d] * igm;
    const T sc = T(2) / (T(1) + dot3(Tv, Tv));
    for (int d = 0; d < 3; ++d) S[d] = sc * Tv[d];
    cross3(um, Tv, c);
    for (int d = 0; d < 3; ++d) up[d] = um[d] + c[d];
    cross3(up, S, c);
    for (int d = 0; d < 3; ++d) out[d] = um[d] + c[d] + a * E[d];
}

// Vay: velocity average in the magnetic term, closed-form Lorentz factor.
template <typename T> __device__ inline void push_vay(T a, const T u[3], const T E[3], const T B[3], T out[3]) {
    const T ig0 = T(1) / sqrt(T(1) + dot3(u, u));
    T v0[3], c[3], u1[3], tau[3], t[3];
    for (int d = 0; d < 3; ++d) v0[d] = u[d] * ig0;
    cross3(v0, B, c);
    for (int d = 0; d < 3; ++d) u1[d] = u[d] + T(2) * a * E[d] + a * c[d];
    for (int d = 0; d < 3; ++d) tau[d] = a * B[d];
    T us = dot3(u1, tau), tau2 = dot3(tau, tau);
    T sig = T(1) + dot3(u1, u1) - tau2;
    T D = sqrt(sig * sig + T(4) * (tau2 + us * us));
    const T ign = T(1) / sqrt(T(0.5) * (sig + D));
    for (int d = 0; d < 3; ++d) t[d] = tau[d] * ign;
    T sf = T(1) / (T(1) + dot3(t, t));
    T ut = dot3(u1, t);
    cross3(u1, t, c);
    for (int d = 0; d < 3; ++d) out[d] = sf * (u1[d] + ut * t[d] + c[d]);
}

template <typename T> __device__ inline void push(int pusher, T a, const T u[3], const T E[3], const T B[3], T out[3]) {
    if (pusher == 1)
        push_vay(a, u, E, B, out);
    else
        push_boris(a, u, E, B, out);
}

// plasma lab profile in [0, 1] (linear up-ramp, flat, zero outside; Lp <= 0: uniform)
__host__ __device__ inline double plasma_profile(double Lp, double z0p, double Rp, double zl) {
    if (Lp <= 0.0) return 1.0;
    double a = zl - z0p;
    if (a < 0.0 || a >= Lp) return 0.0;
    if (Rp > 0.0 && a < Rp) return a / Rp;
    return 1.0;
}

// boosted position of lattice sheet l at time t: ((l + 1/2) / ppz) - bR t
__host__ __device__ inline double sheet_z(int64_t l, int ppz, double bR, double t) {
    return ((double)l + 0.5) / ppz - bR * t;
}

// particles of one lattice sheet: nx ny ppx ppy electrons, then as many mobile
// ions at the same places (stored with the plasma, marked by a negative weight)
__host__ __device__ inline int64_t sheet_particles(const Params &P) {
    return (int64_t)P.plane * P.ppx * P.ppy * (P.mobile ? 2 : 1);
}

// per-particle weight of sheet l (boosted density gR n(z_lab), Eq. Nnormi)
__host__ __device__ inline double sheet_weight(const Params &P, int64_t l) {
    double zl = P.gR * (sheet_z(l, P.ppz, P.bR, 0.0) - P.zoff);
    return P.wsheet * plasma_profile(P.Lp, P.z0p, P.Rp, zl);
}

}  // namespace pic
