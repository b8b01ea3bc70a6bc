// k_diag.hip -- diagnostics: beam moments and normalised emittances, bunching
// factor, energies and the Gauss-law residual div E - rho.
//
// The paper bases its analysis on quantities that do not depend on the
// frame change (transverse dynamics, charge; section 2) and reports the beam
// modulation at the boosted undulator period and half of it (section 3); the
// bunching factor |sum w exp(i k z')| / sum w is taken at fixed t' in the
// boosted frame.  All sums are FP64 with per-block partials, reduced on the
// device in a fixed order (k_reduce_partials), so a diagnostic of a given
// particle order is reproducible bit for bit.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "pic_internal.h"

namespace pic {

void split_rho(Ctx &c, double *rho, int mask);                 // k_split32.hip
int split_plasma_kinetic_partials(Ctx &c, double *red);        // k_split32.hip
int64_t split_beam_to64(Ctx &c, double *dst6);                 // k_split32.hip

constexpr int DT = 256;

template <int NV> __device__ inline void block_sum(double (*s)[DT], double v[NV], double *out) {
    for (int k = 0; k < NV; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = DT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < NV; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) out[(int64_t)blockIdx.x * NV + k] = s[k][0];
}

// pass 1: count, w, w x, w y, w z, w ux, w uy, w uz, w cos kz, w sin kz, w cos 2kz, w sin 2kz, w (gamma - 1)
__global__ void __launch_bounds__(DT) k_mom1(Part64 p, int64_t n, double wconst, double kb, double *out) {
    __shared__ double s[13][DT];
    double v[13] = {0};
    int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q < n && (!p.alive || p.alive[q])) {
        double w = p.w ? p.w[q] : wconst;
        double z = p.z[q], ux = p.ux[q], uy = p.uy[q], uz = p.uz[q];
        double s1, c1, s2, c2;
        sincos(kb * z, &s1, &c1);
        sincos(2.0 * kb * z, &s2, &c2);
        v[0] = 1.0;
        v[1] = w;
        v[2] = w * p.x[q];
        v[3] = w * p.y[q];
        v[4] = w * z;
        v[5] = w * ux;
        v[6] = w * uy;
        v[7] = w * uz;
        v[8] = w * c1;
        v[9] = w * s1;
        v[10] = w * c2;
        v[11] = w * s2;
        v[12] = w * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
    }
    block_sum<13>(s, v, out);
}

// pass 2: central second moments about the pass-1 means
__global__ void __launch_bounds__(DT) k_mom2(Part64 p, int64_t n, double wconst, double mx, double my, double mz,
                                             double mux, double muy, double muz, double *out) {
    __shared__ double s[8][DT];
    double v[8] = {0};
    int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q < n && (!p.alive || p.alive[q])) {
        double w = p.w ? p.w[q] : wconst;
        double dx = p.x[q] - mx, dy = p.y[q] - my, dz = p.z[q] - mz;
        double a = p.ux[q] - mux, b = p.uy[q] - muy, cz = p.uz[q] - muz;
        v[0] = w * dx * dx;
        v[1] = w * dy * dy;
        v[2] = w * dz * dz;
        v[3] = w * a * a;
        v[4] = w * b * b;
        v[5] = w * cz * cz;
        v[6] = w * dx * a;
        v[7] = w * dy * b;
    }
    block_sum<8>(s, v, out);
}

// count and kinetic energy m w (gamma - 1) of the plasma slots (mobile ions: w < 0, mass mi)
__global__ void __launch_bounds__(DT) k_kin(Part64 p, int64_t n, double mi, double *out) {
    __shared__ double s[2][DT];
    double v[2] = {0, 0};
    int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q < n && p.alive[q]) {
        double ux = p.ux[q], uy = p.uy[q], uz = p.uz[q];
        v[0] = 1.0;
        const double w = p.w[q];
        v[1] = (w < 0.0 ? -mi * w : w) * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
    }
    block_sum<2>(s, v, out);
}

template <typename T> __global__ void __launch_bounds__(DT) k_fenergy(FieldsT<T> f, int64_t nc, double *out) {
    __shared__ double s[1][DT];
    double v[1] = {0};
    for (int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x; q < nc; q += (int64_t)gridDim.x * DT)
        for (int c = 0; c < 3; ++c) {
            double e = f.E[c][q], b = f.B[c][q];
            v[0] += e * e + b * b;
        }
    block_sum<1>(s, v, out);
}

// charge -w of FP64 particles on the nodes (mobile ions carry w < 0), FP64 atomics into rho (ring order)
__global__ void __launch_bounds__(DT) k_rho64(Params P, int64_t k0, int k0r, Part64 p, int64_t n, double *rho) {
    int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q >= n || !p.alive[q]) return;
    double X[3] = {p.x[q], p.y[q], p.z[q]};
    double w[3][3];
    int64_t lo[3];
    for (int d = 0; d < 3; ++d) {
        double nn = floor(X[d] + 0.5);
        weights3<double>(X[d] - nn, w[d]);
        lo[d] = (int64_t)nn - 1;
    }
    double qw = -p.w[q];
    for (int c = 0; c < 3; ++c) {
        int pl = ring_plane((int)(lo[2] + c - k0), k0r, P.nz);
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a)
                atomicAdd(&rho[cell_index(P, (int)(lo[0] + a), (int)(lo[1] + b), pl)], qw * w[0][a] * w[1][b] * w[2][c]);
    }
}

// ion charge profile (logical planes): sum over sheets of w ppx ppy S(k - z_l)
// w32: the FP32 mode's ions carry their electrons' FP32-rounded weight
__global__ void k_rho_ion(Params P, int64_t sh_lo, int64_t ns, double t, int64_t k0, double *prof, int w32) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    int64_t l = sh_lo + q;
    double w = sheet_weight(P, l);
    if (w32) w = (double)(float)w;
    w *= (double)(P.ppx * P.ppy);
    if (w == 0.0) return;
    double z = sheet_z(l, P.ppz, P.bR, t);
    double nn = floor(z + 0.5), ws[3];
    weights3<double>(z - nn, ws);
    for (int c = 0; c < 3; ++c) {
        int lp = (int)((int64_t)nn - 1 + c - k0);
        if (lp >= 0 && lp < P.nz) atomicAdd(&prof[lp], w * ws[c]);
    }
}

// r = div E - rho on nodes of the band [band, nz - band); max |r|, max |rho|,
// max |r - r_prev| where the previous residual covers the same absolute plane.
template <typename T>
__global__ void __launch_bounds__(DT) k_gauss(Params P, int k0r, FieldsT<T> f, const double *rho, const double *ion,
                                              double *rprev, int64_t dk, int have, int band, double *out) {
    __shared__ double s[3][DT];
    double v[3] = {0, 0, 0};
    int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q < P.nc) {
        int i = (int)(q % P.nx);
        int64_t r = q / P.nx;
        int j = (int)(r % P.ny);
        int l = (int)(r / P.ny);
        double rv = 0.0;
        if (l >= band && l < P.nz - band) {
            int p = ring_plane(l, k0r, P.nz), pm = ring_plane(l - 1, k0r, P.nz);
            int64_t o = cell_index(P, i, j, p);
            double dv = ((double)f.E[0][o] - (double)f.E[0][cell_index(P, i - 1, j, p)]) +
                        ((double)f.E[1][o] - (double)f.E[1][cell_index(P, i, j - 1, p)]) +
                        ((double)f.E[2][o] - (double)f.E[2][cell_index(P, i, j, pm)]);
            double rh = rho[o] + ion[l];
            rv = dv - rh;
            v[0] = fabs(rv);
            v[1] = fabs(rh);
            int64_t lp = (int64_t)l + dk;  // same absolute plane in the previous call
            if (have && lp >= band && lp < P.nz - band)
                v[2] = fabs(rv - rprev[(int64_t)i + (int64_t)P.nx * (j + (int64_t)P.ny * lp)]);
        }
    }
    for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = DT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = fmax(s[k][threadIdx.x], s[k][threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[3 * (int64_t)blockIdx.x + k] = s[k][0];
}

template <typename T>
__global__ void __launch_bounds__(DT) k_store_r(Params P, int k0r, FieldsT<T> f, const double *rho, const double *ion,
                                                double *rnew, int band) {
    int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q >= P.nc) return;
    int i = (int)(q % P.nx);
    int64_t r = q / P.nx;
    int j = (int)(r % P.ny);
    int l = (int)(r / P.ny);
    double rv = 0.0;
    if (l >= band && l < P.nz - band) {
        int p = ring_plane(l, k0r, P.nz), pm = ring_plane(l - 1, k0r, P.nz);
        int64_t o = cell_index(P, i, j, p);
        double dv = ((double)f.E[0][o] - (double)f.E[0][cell_index(P, i - 1, j, p)]) +
                    ((double)f.E[1][o] - (double)f.E[1][cell_index(P, i, j - 1, p)]) +
                    ((double)f.E[2][o] - (double)f.E[2][cell_index(P, i, j, pm)]);
        rv = dv - (rho[o] + ion[l]);
    }
    rnew[q] = rv;
}

// The nv values of nblk per-block partials (red[b nv + k]) reduced in a fixed
// order by one block: thread t takes the blocks [t m, (t + 1) m) in order, then
// a fixed tree; the results overwrite red[0 .. nv).  OP 0 sums, OP 1 takes the
// maximum with 0.
constexpr int RED_MAX_NV = 16;
template <int OP> __global__ void __launch_bounds__(DT) k_reduce_partials(double *red, int64_t nblk, int nv) {
    __shared__ double s[DT];
    const int64_t m = (nblk + DT - 1) / DT, b0 = (int64_t)threadIdx.x * m, b1 = min(b0 + m, nblk);
    double acc[RED_MAX_NV];
#pragma unroll
    for (int k = 0; k < RED_MAX_NV; ++k) acc[k] = 0.0;
    for (int64_t b = b0; b < b1; ++b)
#pragma unroll
        for (int k = 0; k < RED_MAX_NV; ++k)
            if (k < nv) {
                const double v = red[b * nv + k];
                acc[k] = OP == 0 ? acc[k] + v : (acc[k] < v ? v : acc[k]);
            }
    __syncthreads();  // every partial read before red[0 .. nv) is overwritten
    for (int k = 0; k < nv; ++k) {
        s[threadIdx.x] = acc[k < RED_MAX_NV ? k : 0];
        __syncthreads();
        for (int h = DT / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) {
                const double v = s[threadIdx.x + h];
                s[threadIdx.x] = OP == 0 ? s[threadIdx.x] + v : (s[threadIdx.x] < v ? v : s[threadIdx.x]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) red[k] = s[0];
        __syncthreads();
    }
}

// reduce nblk partials of nv values in red and copy the nv results to acc (host)
static void reduce_partials(Ctx &c, double *red, int64_t nblk, int nv, int op, double *acc) {
    if (op == 0)
        hipLaunchKernelGGL(k_reduce_partials<0>, dim3(1), dim3(DT), 0, c.st, red, nblk, nv);
    else
        hipLaunchKernelGGL(k_reduce_partials<1>, dim3(1), dim3(DT), 0, c.st, red, nblk, nv);
    hipMemcpyAsync(acc, red, 8 * (uint64_t)nv, hipMemcpyDeviceToHost, c.st);
    hipStreamSynchronize(c.st);
}

// lab-frame probe over the live FP64 beam slots: each block's five sums added to acc
__global__ void __launch_bounds__(DT) k_probe64(Params P, Part64 p, int64_t n, double t1, double T, double k,
                                                double *acc) {
    __shared__ double s[5][DT];
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x; q < n; q += (int64_t)gridDim.x * DT)
        if (p.alive[q]) probe_particle(P, p.z[q], p.ux[q], p.uy[q], p.uz[q], p.w[q], t1, T, k, v);
    for (int j = 0; j < 5; ++j) s[j][threadIdx.x] = v[j];
    __syncthreads();
    for (int h = DT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int j = 0; j < 5; ++j) s[j][threadIdx.x] += s[j][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int j = 0; j < 5; ++j) atomicAdd(&acc[j], s[j][0]);
}

// ---------------------------------------------------------------- lab frame (section 2)
__global__ void __launch_bounds__(DT) k_lab64(Params P, Part64 p, int64_t n, double t, double *out) {
    const int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q >= n) return;
    double L[8];
    lab_of(P, t, p.x[q], p.y[q], p.z[q], p.ux[q], p.uy[q], p.uz[q], L);
    for (int k = 0; k < 8; ++k) out[(uint64_t)k * n + q] = L[k];
}

// FP32 mode: in place over the absolute FP64 phase space split_read wrote (rows x y z ux uy uz w)
__global__ void __launch_bounds__(DT) k_lab_inplace(Params P, double *a, int64_t n, double t) {
    const int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x;
    if (q >= n) return;
    double L[8];
    lab_of(P, t, a[q], a[n + q], a[2 * n + q], a[3 * n + q], a[4 * n + q], a[5 * n + q], L);
    for (int k = 0; k < 8; ++k) a[(uint64_t)k * n + q] = L[k];
}

__global__ void k_lab_groups_init(double *out, int ng) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= LAB_GROUP_VALUES * ng) return;
    const int v = k % LAB_GROUP_VALUES;
    out[k] = v == 3 ? INFINITY : (v == 4 ? -INFINITY : 0.0);
}

__global__ void __launch_bounds__(DT) k_lab_groups64(Params P, LabGroupSpec G, Part64 p, int64_t n, double t,
                                                     double *out) {
    __shared__ double tab[LAB_GROUP_VALUES * LAB_GROUPS_MAX];
    const int ng = G.nz * G.nu;
    lab_table_clear(tab, ng);
    __syncthreads();
    for (int64_t q = (int64_t)blockIdx.x * DT + threadIdx.x; q < n; q += (int64_t)gridDim.x * DT)
        if (p.alive[q]) lab_group_add(tab, G, P, t, p.x[q], p.y[q], p.z[q], p.ux[q], p.uy[q], p.uz[q], p.w[q]);
    __syncthreads();
    lab_table_flush(tab, ng, out);
}

pic_status lab_groups(Ctx &c, const LabGroupSpec &G, double *out) {
    const int ng = G.nz * G.nu;
    const double t = (double)c.step * c.P.dt;
    hipLaunchKernelGGL(k_lab_groups_init, dim3(nblocks(LAB_GROUP_VALUES * ng, DT)), dim3(DT), 0, c.st, out, ng);
    if (c.precision == PIC_FP64_PLAIN) {
        if (c.nb_slots)
            hipLaunchKernelGGL(k_lab_groups64, dim3(std::min(nblocks(c.nb_slots, DT), 1024)), dim3(DT), 0, c.st, c.P,
                               G, c.b64, c.nb_slots, t, out);
    } else {
        split_lab_groups(c, G, t, out);
    }
    PIC_HIP(c, hipStreamSynchronize(c.st));
    return PIC_OK;
}

pic_status lab_beam(Ctx &c, double *out, int64_t *n) {
    const double t = (double)c.step * c.P.dt;
    if (c.precision == PIC_FP64_PLAIN) {
        *n = c.nb_slots;
        if (out && c.nb_slots)
            hipLaunchKernelGGL(k_lab64, dim3(nblocks(c.nb_slots, DT)), dim3(DT), 0, c.st, c.P, c.b64, c.nb_slots, t,
                               out);
    } else {
        split_read(c, 0, nullptr, nullptr, n);
        if (out && *n) {
            split_read(c, 0, out, nullptr, n);
            hipLaunchKernelGGL(k_lab_inplace, dim3(nblocks(*n, DT)), dim3(DT), 0, c.st, c.P, out, *n, t);
        }
    }
    PIC_HIP(c, hipStreamSynchronize(c.st));
    return PIC_OK;
}

// after a step (c.step, c.k0 already advanced): sample the beam particles whose lab time passed the probe's
void probe_step(Ctx &c) {
    const double t1 = (double)c.step * c.P.dt;
    if (c.precision == PIC_FP64_PLAIN) {
        if (c.nb_slots > 0) {
            const int nblk = (int)std::min<int64_t>(nblocks(c.nb_slots, DT), 1024);
            hipLaunchKernelGGL(k_probe64, dim3(nblk), dim3(DT), 0, c.st, c.P, c.b64, c.nb_slots, t1, c.probe_t,
                               c.probe_k, c.probe_acc);
        }
    } else {
        split_probe(c, c.probe_acc);
    }
}

// beam charge on the nodes (ring order), added into rho
void beam_rho(Ctx &c, double *rho) {
    const Params &P = c.P;
    if (c.precision == PIC_FP64_PLAIN) {
        if (c.nb_slots)
            hipLaunchKernelGGL(k_rho64, dim3(nblocks(c.nb_slots, DT)), dim3(DT), 0, c.st, P, c.k0,
                               (int)(c.k0 % P.nz), c.b64, c.nb_slots, rho);
    } else {
        split_rho(c, rho, 1);
    }
}

// partial sums run_diag needs in red (doubles)
int64_t diag_partials(const Ctx &c, uint32_t mask) {
    const Params &P = c.P;
    const int64_t nb = c.precision == PIC_FP64_PLAIN ? c.nb_slots : c.beam.n_macro;
    int64_t need = 13 * (int64_t)nblocks(std::max<int64_t>(nb, 1), DT);
    if (mask & PIC_DIAG_ENERGY) need = std::max<int64_t>(need, 1024);
    if (P.has_plasma)
        need = std::max<int64_t>(need, 2 * (c.precision == PIC_FP64_PLAIN
                                                ? (int64_t)nblocks(std::max<int64_t>(c.np_slots, 1), DT)
                                                : (int64_t)P.nbins + 1));
    if (mask & PIC_DIAG_GAUSS) need = std::max<int64_t>(need, 3 * (int64_t)nblocks(P.nc, DT));
    return need;
}

pic_status run_diag(Ctx &c, uint32_t mask, double kb, pic_diag_out *o, double *red, int64_t red_cap) {
    memset(o, 0, sizeof *o);
    const Params &P = c.P;
    if (diag_partials(c, mask) > red_cap) {
        c.err = "diagnostics: more partial sums than the reduction buffer holds";
        return PIC_ERANGE;
    }
    o->t = (double)c.step * P.dt;
    o->step = (double)c.step;
    o->k0 = (double)c.k0;
    o->window_beta = c.bw;
    o->window_x = c.win_x0 + c.bw * ((double)c.step * P.dt - c.win_t0);
    o->frac_bits = P.frac_bits;
    int k0r = (int)(c.k0 % P.nz);
    // beam as FP64 arrays
    Part64 bp;
    int64_t nb;
    double wconst = P.wbeam;
    if (c.precision == PIC_FP64_PLAIN) {
        bp = c.b64;
        nb = c.nb_slots;
    } else {
        nb = split_beam_to64(c, c.stage);
        uint64_t cap = (uint64_t)std::max<int64_t>(c.beam.n_macro, 1);
        bp.x = c.stage;
        bp.y = c.stage + cap;
        bp.z = c.stage + 2 * cap;
        bp.ux = c.stage + 3 * cap;
        bp.uy = c.stage + 4 * cap;
        bp.uz = c.stage + 5 * cap;
        bp.w = nullptr;
        bp.alive = nullptr;
    }
    double m1[13] = {0};
    if (nb > 0) {
        int nblk = nblocks(nb, DT);
        hipLaunchKernelGGL(k_mom1, dim3(nblk), dim3(DT), 0, c.st, bp, nb, wconst, kb, red);
        reduce_partials(c, red, nblk, 13, 0, m1);
    }
    o->n_beam = m1[0];
    o->beam_lost = (double)c.beam.n_macro - m1[0];
    o->wsum = m1[1];
    double W = m1[1];
    if (W > 0) {
        double mean[6];
        for (int k = 0; k < 6; ++k) mean[k] = m1[2 + k] / W;
        for (int k = 0; k < 3; ++k) {
            o->mean[k] = mean[k];
            o->umean[k] = mean[3 + k];
        }
        o->b1_re = m1[8] / W;
        o->b1_im = m1[9] / W;
        o->b2_re = m1[10] / W;
        o->b2_im = m1[11] / W;
        o->b1_abs = sqrt(m1[8] * m1[8] + m1[9] * m1[9]) / W;
        o->b2_abs = sqrt(m1[10] * m1[10] + m1[11] * m1[11]) / W;
        o->kin_beam = m1[12];
        if (mask & PIC_DIAG_MOMENTS) {
            int nblk = nblocks(nb, DT);
            hipLaunchKernelGGL(k_mom2, dim3(nblk), dim3(DT), 0, c.st, bp, nb, wconst, mean[0], mean[1], mean[2],
                               mean[3], mean[4], mean[5], red);
            double m2[8];
            reduce_partials(c, red, nblk, 8, 0, m2);
            for (int k = 0; k < 3; ++k) {
                o->sigma[k] = sqrt(m2[k] / W);
                o->usigma[k] = sqrt(m2[3 + k] / W);
            }
            for (int k = 0; k < 2; ++k) {
                double a = m2[k] / W, b = m2[3 + k] / W, x = m2[6 + k] / W;
                o->emit[k] = sqrt(std::max(0.0, a * b - x * x));
            }
        }
    }
    if (mask & PIC_DIAG_ENERGY) {
        int nblk = 1024;
        double fe[1];
        if (c.precision == PIC_FP64_PLAIN) {
            FieldsT<double> f;
            for (int k = 0; k < 3; ++k) {
                f.E[k] = c.E64[k];
                f.B[k] = c.B64[k];
            }
            hipLaunchKernelGGL(k_fenergy<double>, dim3(nblk), dim3(DT), 0, c.st, f, P.nc, red);
        } else {
            FieldsT<float> f;
            for (int k = 0; k < 3; ++k) {
                f.E[k] = c.E32[k];
                f.B[k] = c.B32[k];
            }
            hipLaunchKernelGGL(k_fenergy<float>, dim3(nblk), dim3(DT), 0, c.st, f, P.nc, red);
        }
        reduce_partials(c, red, nblk, 1, 0, fe);
        o->field_energy = 0.5 * fe[0];
    }
    // plasma counts and kinetic energy
    if (P.has_plasma) {
        if (c.precision == PIC_FP64_PLAIN) {
            if (c.np_slots > 0) {
                int nblk = nblocks(c.np_slots, DT);
                hipLaunchKernelGGL(k_kin, dim3(nblk), dim3(DT), 0, c.st, c.p64, c.np_slots, c.P.mi, red);
                double kp[2];
                reduce_partials(c, red, nblk, 2, 0, kp);
                o->n_plasma = kp[0];
                o->kin_plasma = kp[1];
            }
        } else {
            double kp[2];
            const int nblk = split_plasma_kinetic_partials(c, red);
            reduce_partials(c, red, nblk, 2, 0, kp);
            o->n_plasma = kp[0];
            o->kin_plasma = kp[1];
        }
    }
    if (mask & PIC_DIAG_GAUSS) {
        const int band = 8;
        // scratch: rho in J_x (zero between steps), ion profile in the ion-current buffer
        double *rho = c.precision == PIC_FP64_PLAIN ? c.J64[0] : (double *)c.Ji[0];
        double *ion = c.precision == PIC_FP64_PLAIN ? c.jion64 : (double *)c.jioni;
        if (c.precision == PIC_FP64_PLAIN) {
            if (c.nb_slots) hipLaunchKernelGGL(k_rho64, dim3(nblocks(c.nb_slots, DT)), dim3(DT), 0, c.st, P, c.k0, k0r, c.b64, c.nb_slots, rho);
            if (c.np_slots) hipLaunchKernelGGL(k_rho64, dim3(nblocks(c.np_slots, DT)), dim3(DT), 0, c.st, P, c.k0, k0r, c.p64, c.np_slots, rho);
        } else {
            split_rho(c, rho, 3);
        }
        if (P.ions && c.sh_hi > c.sh_lo)
            hipLaunchKernelGGL(k_rho_ion, dim3(nblocks(c.sh_hi - c.sh_lo, 128)), dim3(128), 0, c.st, P, c.sh_lo,
                               c.sh_hi - c.sh_lo, o->t, c.k0, ion, c.precision != PIC_FP64_PLAIN);
        launch_neutraliser_rho(c, rho);
        int nblk = nblocks(P.nc, DT);
        int64_t dk = c.k0 - c.rprev_k0;
        if (c.precision == PIC_FP64_PLAIN) {
            FieldsT<double> f;
            for (int k = 0; k < 3; ++k) {
                f.E[k] = c.E64[k];
                f.B[k] = c.B64[k];
            }
            hipLaunchKernelGGL(k_gauss<double>, dim3(nblk), dim3(DT), 0, c.st, P, k0r, f, rho, ion, c.rprev, dk,
                               c.have_rprev, band, red);
            hipLaunchKernelGGL(k_store_r<double>, dim3(nblk), dim3(DT), 0, c.st, P, k0r, f, rho, ion, c.rprev, band);
        } else {
            FieldsT<float> f;
            for (int k = 0; k < 3; ++k) {
                f.E[k] = c.E32[k];
                f.B[k] = c.B32[k];
            }
            hipLaunchKernelGGL(k_gauss<float>, dim3(nblk), dim3(DT), 0, c.st, P, k0r, f, rho, ion, c.rprev, dk,
                               c.have_rprev, band, red);
            hipLaunchKernelGGL(k_store_r<float>, dim3(nblk), dim3(DT), 0, c.st, P, k0r, f, rho, ion, c.rprev, band);
        }
        hipMemsetAsync(rho, 0, 8 * P.nc, c.st);
        hipMemsetAsync(ion, 0, 8 * P.nz, c.st);
        double g[3];
        reduce_partials(c, red, nblk, 3, 1, g);
        o->gauss_max = g[0];
        o->rho_max = g[1];
        o->gauss_drift = c.have_rprev ? g[2] : -1.0;
        c.have_rprev = 1;
        c.rprev_k0 = c.k0;
    }
    int32_t fl = 0;
    hipMemcpyAsync(&fl, c.dflags, 4, hipMemcpyDeviceToHost, c.st);
    hipError_t e = hipStreamSynchronize(c.st);
    if (e != hipSuccess) return hip_check(c, e, "diag");
    o->error_flags = fl;
    return PIC_OK;
}

// ---------------------------------------------------------------- allocation-free diagnostics
// The reduction buffer of pic_diag_static: a file-scope device array, one per
// GPU the library runs on, held until the process ends.  Host code reaches it
// only through the address hipGetSymbolAddress returns for each device.
static __device__ __align__(256) double scratch[DIAG_STATIC_DOUBLES];
static std::mutex g_scratch_mu;
static double *g_scratch[64];

pic_status static_scratch_setup(Ctx &c) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c.device < 0 || c.device >= 64) {
        c.err = "static scratch: device ordinal beyond 63";
        return PIC_EDEVICE;
    }
    if (g_scratch[c.device]) return PIC_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_check(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch");
    g_scratch[c.device] = (double *)p;
    return PIC_OK;
}

double *static_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < 64 ? g_scratch[device] : nullptr;
}

}  // namespace pic
