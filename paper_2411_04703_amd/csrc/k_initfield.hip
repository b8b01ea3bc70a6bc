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
// phi[-1] = phi[nz] = 0; forward elimination (coefficients kept in cp), then back substitution
__global__ void __launch_bounds__(IT) k_tri_z(Params P, double *re, double *im, double *cp, double g2) {
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
        const double m = diag - g2 * c;
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
template <typename T>
__global__ void __launch_bounds__(IT) k_field_from_phi(Params P, const double *phi, double g2, double beta, double w,
                                                      FieldsT<T> f) {
    const int64_t o = (int64_t)blockIdx.x * IT + threadIdx.x;
    if (o >= P.nc) return;
    const int i = (int)(o % P.nx);
    const int64_t r = o / P.nx;
    const int j = (int)(r % P.ny);
    const int l = (int)(r / P.ny);
    const int ip = i + 1 == P.nx ? 0 : i + 1, jp = j + 1 == P.ny ? 0 : j + 1;
    auto at = [&](int ii, int jj, int ll) -> double {
        return ll < P.nz ? phi[cell_index(P, ii, jj, ll)] : 0.0;  // phi = 0 beyond the top face
    };
    const double p = phi[o], pu = at(i, j, l + 1);
    const double ex = -(at(ip, j, l) - p), ey = -(at(i, jp, l) - p), ez = -(pu - p) * g2;
    const double exu = -(at(ip, j, l + 1) - pu), eyu = -(at(i, jp, l + 1) - pu);
    f.E[0][o] = (T)ex;
    f.E[1][o] = (T)ey;
    f.E[2][o] = (T)ez;
    f.B[0][o] = (T)(-beta * ((1.0 - w) * ey + w * eyu));
    f.B[1][o] = (T)(beta * ((1.0 - w) * ex + w * exu));
    f.B[2][o] = (T)0;
}

pic_status init_beam_fields(Ctx &c) {
    const Params &P = c.P;
    if (c.k0 != 0 || c.step != 0) {
        c.err = "init_beam_fields: only at t' = 0";
        return PIC_ESTATE;
    }
    if (P.nx > 2048 || P.ny > 2048) {
        c.err = "init_fields: transverse grid edges above 2048 are not supported";
        return PIC_EINVAL;
    }
    const double beta = c.beam_beta0;
    if (!(beta > -1.0 && beta < 1.0)) {
        c.err = "init_fields: no beam velocity";
        return PIC_EINVAL;
    }
    const double g2 = (1.0 - beta) * (1.0 + beta);  // 1 / gamma_b^2
    // scratch: the three current arrays (8 bytes per cell each, zero between steps)
    double *re, *im, *cp;
    if (c.precision == PIC_FP64_PLAIN) {
        re = c.J64[0];
        im = c.J64[1];
        cp = c.J64[2];
    } else {
        re = (double *)c.Ji[0];
        im = (double *)c.Ji[1];
        cp = (double *)c.Ji[2];
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
    hipLaunchKernelGGL(k_tri_z, dim3((unsigned)nblocks(pl, IT)), dim3(IT), 0, c.st, P, re, im, cp, g2);
    hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(P.nx * (int64_t)P.nz)), dim3(IT), 32 * P.ny, c.st, re, im, P.ny,
                       (int64_t)P.nx, P.nx, (int64_t)1, pl, 1.0, 1.0 / P.ny);
    hipLaunchKernelGGL(k_dft_lines, dim3((unsigned)(P.ny * (int64_t)P.nz)), dim3(IT), 32 * P.nx, c.st, re, im, P.nx,
                       (int64_t)1, P.ny, (int64_t)P.nx, pl, 1.0, 1.0 / P.nx);
    const double w = 0.5 + 0.5 * beta * P.dt;
    const unsigned nb = (unsigned)nblocks(P.nc, IT);
    if (c.precision == PIC_FP64_PLAIN) {
        FieldsT<double> f;
        for (int k = 0; k < 3; ++k) {
            f.E[k] = c.E64[k];
            f.B[k] = c.B64[k];
        }
        hipLaunchKernelGGL(k_field_from_phi<double>, dim3(nb), dim3(IT), 0, c.st, P, re, g2, beta, w, f);
    } else {
        FieldsT<float> f;
        for (int k = 0; k < 3; ++k) {
            f.E[k] = c.E32[k];
            f.B[k] = c.B32[k];
        }
        hipLaunchKernelGGL(k_field_from_phi<float>, dim3(nb), dim3(IT), 0, c.st, P, re, g2, beta, w, f);
    }
    PIC_HIP(c, hipMemsetAsync(re, 0, bytes, c.st));
    PIC_HIP(c, hipMemsetAsync(im, 0, bytes, c.st));
    PIC_HIP(c, hipMemsetAsync(cp, 0, bytes, c.st));
    PIC_HIP(c, hipStreamSynchronize(c.st));
    return PIC_OK;
}

}  // namespace pic
