// k_initfield.hip -- initial self-field of the beam in the boosted frame (FP64).
//
// Section 1 carries fields between frames.  The beam's rest-frame field is
// electrostatic; moved into the boosted frame, where the beam drifts at
// beta_b along z, it solves
//     (d_xx + d_yy + d_zz / gamma_b^2) phi = -rho,
//     E_perp = -grad_perp phi,  E_z = -d_z phi / gamma_b^2,  B = beta_b z x E.
// On the Yee grid of the step: rho and phi on nodes, second differences,
// periodic x and y (as the field solver), phi = 0 one plane beyond each z face,
// so that the discrete divergence of E equals rho node by node.  The stored B
// is the one at t' = -dt/2 (the state between steps is (E^n, B^(n-1/2))): the
// pattern moves at beta_b, so B is beta_b z x E displaced by beta_b dt / 2
// along z, interpolated linearly between planes.
//
// Solver: a DFT along x and along y (the periodic operator is diagonal there;
// one workgroup per grid line, the line and its twiddles in LDS), a
// tridiagonal solve along z per transverse mode (one thread per mode), and the
// inverse DFTs.  It runs once, at t' = 0 (window origin 0), on scratch that the
// current arrays provide: they are zero between steps and are cleared again
// afterwards.
#include <math.h>

#include <type_traits>

#include "pic_internal.h"

namespace pic {

constexpr int IT = 256;

// in-place DFT of n-point lines of the split complex array (re, im): line L
// starts at (L % na) * sa + (L / na) * sb, its elements se apart;
// X[m] = scale * sum_t x[t] exp(sign 2 pi i m t / n)
__global__ void __launch_bounds__(IT) k_dft_lines(double *re, double *im, int n, int64_t se, int na, int64_t sa,
                                                  int64_t sb, double sign, double scale) {
    extern __shared__ double sm[];
    double *xr = sm, *xi = sm + n, *cs = sm + 2 * n, *sn = sm + 3 * n;
    const int64_t L = blockIdx.x;
    const int64_t base = (L % na) * sa + (L / na) * sb;
    for (int t = threadIdx.x; t < n; t += IT) {
        xr[t] = re[base + t * se];
        xi[t] = im[base + t * se];
        double s, c;
        sincospi(2.0 * t / n, &s, &c);
        cs[t] = c;
        sn[t] = sign * s;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < n; m += IT) {
        double ar = 0.0, ai = 0.0;
        int k = 0;  // m t mod n
        for (int t = 0; t < n; ++t) {
            const double c = cs[k], s = sn[k];
            ar += xr[t] * c - xi[t] * s;
            ai += xr[t] * s + xi[t] * c;
            k += m;
            if (k >= n) k -= n;
        }
        re[base + m * se] = ar * scale;
        im[base + m * se] = ai * scale;
    }
}

// one transverse mode (kx, ky) per thread: g2 phi[l-1] + (lam - 2 g2) phi[l] + g2 phi[l+1] = -rho[l],
// phi[-1] = 0, and above the top face phi[nz] = 0 or, with an open top, phi[nz] = phi[nz-1] (no
// field through it); forward elimination (coefficients kept in cp), then back substitution
__global__ void __launch_bounds__(IT) k_tri_z(Params P, double *re, double *im, double *cp, double g2, int open_top) {
    const int64_t q = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (q >= P.plane) return;
    const int kx = (int)(q % P.nx), ky = (int)(q / P.nx);
    const double sx = sinpi((double)kx / P.nx), sy = sinpi((double)ky / P.ny);
    const double diag = -4.0 * sx * sx - 4.0 * sy * sy - 2.0 * g2;
    const int64_t pl = P.plane;
    double c = g2 / diag;
    double dr = -re[q] / diag, di = -im[q] / diag;
    cp[q] = c;
    re[q] = dr;
    im[q] = di;
    for (int l = 1; l < P.nz; ++l) {
        const int64_t o = q + (int64_t)l * pl;
        const double m = (open_top && l == P.nz - 1 ? diag + g2 : diag) - g2 * c;
        c = g2 / m;
        dr = (-re[o] - g2 * dr) / m;
        di = (-im[o] - g2 * di) / m;
        cp[o] = c;
        re[o] = dr;
        im[o] = di;
    }
    for (int l = P.nz - 2; l >= 0; --l) {
        const int64_t o = q + (int64_t)l * pl;
        dr = re[o] - cp[o] * dr;
        di = im[o] - cp[o] * di;
        re[o] = dr;
        im[o] = di;
    }
}

// E on the edges from phi, B = beta z x E at t' = -dt/2 (w: weight of the plane above)
// (open_top: phi above the top face equals the top plane's, and the top plane's E_x, E_y are left
// out -- the neutralising charge's field, see below)
template <typename T>
__global__ void __launch_bounds__(IT) k_field_from_phi(Params P, const double *phi, double g2, double beta, double w,
                                                      int open_top, FieldsT<T> f) {
    const int64_t o = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (o >= P.nc) return;
    const int i = (int)(o % P.nx);
    const int64_t r = o / P.nx;
    const int j = (int)(r % P.ny);
    const int l = (int)(r / P.ny);
    const int ip = i + 1 == P.nx ? 0 : i + 1, jp = j + 1 == P.ny ? 0 : j + 1;
    auto at = [&](int ii, int jj, int ll) -> double {  // beyond the top face: 0, or the top plane's (open)
        return ll < P.nz ? phi[cell_index(P, ii, jj, ll)] : (open_top ? phi[cell_index(P, ii, jj, P.nz - 1)] : 0.0);
    };
    const double p = phi[o], pu = at(i, j, l + 1);
    const bool keep_t = !(open_top && l == P.nz - 1);
    const double ex = keep_t ? -(at(ip, j, l) - p) : 0.0, ey = keep_t ? -(at(i, jp, l) - p) : 0.0,
                 ez = -(pu - p) * g2;
    const double exu = -(at(ip, j, l + 1) - pu), eyu = -(at(i, jp, l + 1) - pu);
    f.E[0][o] = (T)ex;
    f.E[1][o] = (T)ey;
    f.E[2][o] = (T)ez;
    f.B[0][o] = (T)(-beta * ((1.0 - w) * ey + w * eyu));
    f.B[1][o] = (T)(beta * ((1.0 - w) * ex + w * exu));
    f.B[2][o] = (T)0;
}

// the solver's scratch: the three current arrays (8 bytes per cell each, zero between steps)
static void solver_scratch(Ctx &c, double *&re, double *&im, double *&cp) {
    if (c.precision == PIC_FP64_PLAIN) {
        re = c.J64[0];
        im = c.J64[1];
        cp = c.J64[2];
    } else {
        re = (double *)c.Ji[0];
        im = (double *)c.Ji[1];
        cp = (double *)c.Ji[2];
    }
}

// the beam's node charge at t' = 0 into re (im cleared), then phi of
// (d_xx + d_yy + g2 d_zz) phi = -rho in re
static pic_status solve_beam_potential(Ctx &c, double g2, int open_top, double *re, double *im, double *cp) {
    const Params &P = c.P;
    if (c.k0 != 0 || c.step != 0) {
        c.err = "initial fields: only at t' = 0";
        return PIC_ESTATE;
    }
    if (P.nx > 2048 || P.ny > 2048) {
        c.err = "init_fields: transverse grid edges above 2048 are not supported";
        return PIC_EINVAL;
    }
    const uint64_t bytes = 8 * (uint64_t)P.nc;
    PIC_HIP(c, hipMemsetAsync(re, 0, bytes, c.st));
    PIC_HIP(c, hipMemsetAsync(im, 0, bytes, c.st));
    beam_rho(c, re);
    const int64_t pl = P.plane;
    // forward DFT along x (lines over j, l), then along y (lines over i, l)
    hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(P.ny * (int64_t)P.nz)), dim3(IT), 32 * P.nx, c.st, re, im, P.nx,
                       (int64_t)1, P.ny, (int64_t)P.nx, pl, -1.0, 1.0);
    hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(P.nx * (int64_t)P.nz)), dim3(IT), 32 * P.ny, c.st, re, im, P.ny,
                       (int64_t)P.nx, P.nx, (int64_t)1, pl, -1.0, 1.0);
    hipLaunchKernelGGL(k_tri_z, dim3((unsigned)nblocks(pl, IT)), dim3(IT), 0, c.st, P, re, im, cp, g2, open_top);
    hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(P.nx * (int64_t)P.nz)), dim3(IT), 32 * P.ny, c.st, re, im, P.ny,
                       (int64_t)P.nx, P.nx, (int64_t)1, pl, 1.0, 1.0 / P.ny);
    hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(P.ny * (int64_t)P.nz)), dim3(IT), 32 * P.nx, c.st, re, im, P.nx,
                       (int64_t)1, P.ny, (int64_t)P.nx, pl, 1.0, 1.0 / P.nx);
    return PIC_OK;
}

static pic_status clear_scratch(Ctx &c, double *re, double *im, double *cp) {
    const uint64_t bytes = 8 * (uint64_t)c.P.nc;
    PIC_HIP(c, hipMemsetAsync(re, 0, bytes, c.st));
    PIC_HIP(c, hipMemsetAsync(im, 0, bytes, c.st));
    PIC_HIP(c, hipMemsetAsync(cp, 0, bytes, c.st));
    PIC_HIP(c, hipStreamSynchronize(c.st));
    return PIC_OK;
}

pic_status init_beam_fields(Ctx &c) {
    const Params &P = c.P;
    const double beta = c.beam_beta0;
    if (!(beta > -1.0 && beta < 1.0)) {
        c.err = "init_fields: no beam velocity";
        return PIC_EINVAL;
    }
    const double g2 = (1.0 - beta) * (1.0 + beta);  // 1 / gamma_b^2
    double *re, *im, *cp;
    solver_scratch(c, re, im, cp);
    pic_status st = solve_beam_potential(c, g2, 0, re, im, cp);
    if (st != PIC_OK) return st;
    const double w = 0.5 + 0.5 * beta * P.dt;
    const unsigned nb = (unsigned)nblocks(P.nc, IT);
    if (c.precision == PIC_FP64_PLAIN) {
        FieldsT<double> f;
        for (int k = 0; k < 3; ++k) {
            f.E[k] = c.E64[k];
            f.B[k] = c.B64[k];
        }
        hipLaunchKernelGGL(k_field_from_phi<double>, dim3(nb), dim3(IT), 0, c.st, P, re, g2, beta, w, 0, f);
    } else {
        FieldsT<float> f;
        for (int k = 0; k < 3; ++k) {
            f.E[k] = c.E32[k];
            f.B[k] = c.B32[k];
        }
        hipLaunchKernelGGL(k_field_from_phi<float>, dim3(nb), dim3(IT), 0, c.st, P, re, g2, beta, w, 0, f);
    }
    return clear_scratch(c, re, im, cp);
}

// ---------------------------------------------------------------- neutralising charge (section 3)
// A charge equal and opposite to the beam's at t' = 0, at rest in the boosted
// frame, whose fraction left falls linearly from 1 to 0 over fc_T.  Over a
// step it drops by fc_rho (f(t) - f(t1)); the current -E_b (f(t) - f(t1)) / dt,
// E_b the charge's electrostatic field (div E_b = fc_rho node by node), carries
// exactly that away, so Gauss's law keeps its residual.  Both are stored for
// the planes of the window at origin 0 and stay where they are as it moves.
// E_b is the field of the beam's charge with no field through the top face and
// without the top plane's E_x, E_y (the front face holds those at zero, so
// none of E_b may sit there), and the charge is its discrete divergence: the
// beam's own, except on the top plane, where it differs by the left-out
// components' divergence (about 1e-3 of the peak charge in the workloads).
// The net flux of the transversely periodic box leaves through the back face,
// the first to leave the window.
// node charge div E (x, y periodic; E_z below plane 0 left out, as the Gauss
// diagnostic does)
__global__ void __launch_bounds__(IT) k_div_e(Params P, const double *Ex, const double *Ey, const double *Ez,
                                              double *rho) {
    const int64_t o = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (o >= P.nc) return;
    const int i = (int)(o % P.nx);
    const int64_t r = o / P.nx;
    const int j = (int)(r % P.ny);
    const int l = (int)(r / P.ny);
    const int im = i == 0 ? P.nx - 1 : i - 1, jm = j == 0 ? P.ny - 1 : j - 1;
    double d = (Ex[o] - Ex[cell_index(P, im, j, l)]) + (Ey[o] - Ey[cell_index(P, i, jm, l)]) + Ez[o];
    if (l > 0) d -= Ez[cell_index(P, i, j, l - 1)];
    rho[o] = d;
}

pic_status init_neutraliser(Ctx &c) {
    const Params &P = c.P;
    double *re, *im, *cp;
    solver_scratch(c, re, im, cp);
    pic_status st = solve_beam_potential(c, 1.0, 1, re, im, cp);
    if (st != PIC_OK) return st;
    FieldsT<double> f;  // E_b into fc_E; B of a charge at rest is zero (written to the scratch im)
    for (int k = 0; k < 3; ++k) {
        f.E[k] = c.fc_E[k];
        f.B[k] = im;
    }
    hipLaunchKernelGGL(k_field_from_phi<double>, dim3((unsigned)nblocks(P.nc, IT)), dim3(IT), 0, c.st, P, re, 1.0,
                       0.0, 0.5, 1, f);
    hipLaunchKernelGGL(k_div_e, dim3((unsigned)nblocks(P.nc, IT)), dim3(IT), 0, c.st, P, c.fc_E[0], c.fc_E[1],
                       c.fc_E[2], c.fc_rho);
    return clear_scratch(c, re, im, cp);
}

double neutraliser_left(const Ctx &c, double t) {
    if (!(c.fc_T > 0.0)) return 0.0;
    const double f = 1.0 - t / c.fc_T;
    return f > 0.0 ? f : 0.0;
}

// ring plane p of the window holds logical plane l = (p - k0) mod nz, i.e. the plane k0 + l of
// the window at origin 0, where the neutralising charge's arrays hold it when k0 + l < nz
template <typename JT>
__global__ void __launch_bounds__(IT) k_neutraliser_current(Params P, int64_t k0, int k0r, const double *E0,
                                                            const double *E1, const double *E2, double a, double fs,
                                                            JT *J0, JT *J1, JT *J2) {
    const int64_t o = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (o >= P.nc) return;
    const int p = (int)(o / P.plane);
    const int64_t inplane = o - (int64_t)p * P.plane;
    const int l = p >= k0r ? p - k0r : p - k0r + P.nz;
    const int64_t k = k0 + l;
    if (k >= P.nz) return;
    const int64_t src = k * P.plane + inplane;
    const double v[3] = {-a * E0[src], -a * E1[src], -a * E2[src]};
    JT *J[3] = {J0, J1, J2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if constexpr (std::is_integral<JT>::value)  // 64-bit fixed point
            J[d][o] += (JT)__double2ll_rn(v[d] * fs);
        else
            J[d][o] += (JT)v[d];
    }
}

void launch_neutraliser_current(Ctx &c, const StepCtx &S) {
    if (!(c.fc_T > 0.0) || !c.fc_rho) return;
    const double a = (neutraliser_left(c, S.t) - neutraliser_left(c, S.t1)) / c.P.dt;
    if (a == 0.0) return;
    const Params &P = c.P;
    const unsigned nb = (unsigned)nblocks(P.nc, IT);
    if (c.precision == PIC_FP64_PLAIN)
        hipLaunchKernelGGL(k_neutraliser_current<double>, dim3(nb), dim3(IT), 0, c.st, P, S.k0, S.k0r, c.fc_E[0],
                           c.fc_E[1], c.fc_E[2], a, 1.0, c.J64[0], c.J64[1], c.J64[2]);
    else
        hipLaunchKernelGGL(k_neutraliser_current<long long>, dim3(nb), dim3(IT), 0, c.st, P, S.k0, S.k0r, c.fc_E[0],
                           c.fc_E[1], c.fc_E[2], a, P.fscale, c.Ji[0], c.Ji[1], c.Ji[2]);
}

__global__ void __launch_bounds__(IT) k_neutraliser_rho(Params P, int64_t k0, int k0r, const double *rho0, double f,
                                                        double *rho) {
    const int64_t o = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (o >= P.nc) return;
    const int p = (int)(o / P.plane);
    const int l = p >= k0r ? p - k0r : p - k0r + P.nz;
    const int64_t k = k0 + l;
    if (k < P.nz) rho[o] -= f * rho0[k * P.plane + (o - (int64_t)p * P.plane)];
}

void launch_neutraliser_rho(Ctx &c, double *rho) {
    if (!c.fc_rho) return;
    const double f = neutraliser_left(c, (double)c.step * c.P.dt);
    if (f == 0.0) return;
    hipLaunchKernelGGL(k_neutraliser_rho, dim3((unsigned)nblocks(c.P.nc, IT)), dim3(IT), 0, c.st, c.P, c.k0,
                       (int)(c.k0 % c.P.nz), c.fc_rho, f, rho);
}

}  // namespace pic
