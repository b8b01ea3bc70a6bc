// k_adjoint.hip -- exact discrete adjoint of one FP64 step, for gradients of
// the final bunching factor with respect to the undulator K and the plasma
// density.  The step is reversed one sub-operation at a time:
//   window shift -> E update with Mur faces -> second B half step ->
//   deposit (ion current) -> move -> push -> gather (+ external field) ->
//   first B half step.
// Discrete events (window shift, removal, injection) are those the forward
// step takes from state n; the forward state is recomputed, never stored.
// The external field is linear in K and every plasma weight is linear in n0,
// so K dL/dK = sum <lam_field_at_particle, external field> and
// n0 dL/dn0 = sum <lam_J, J_plasma + J_ions>.
// Adjoint fields are kept in the ring order of the forward fields.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pic_internal.h"

namespace pic {

constexpr int AT = 256;

struct Lam {  // views into the caller's adjoint vector
    double *x[3], *u[3];
};

static Lam lam_view(double *lam, int64_t off, int64_t cap) {
    Lam L;
    uint64_t c = (uint64_t)std::max<int64_t>(cap, 1);
    for (int d = 0; d < 3; ++d) {
        L.x[d] = lam + off + d * c;
        L.u[d] = lam + off + (3 + d) * c;
    }
    return L;
}

// ---------------------------------------------------------------- fields
__device__ inline int plane_of(const Params &P, int64_t o, int k0r, int &i, int &j, int &p) {
    i = (int)(o % P.nx);
    int64_t r = o / P.nx;
    j = (int)(r % P.ny);
    p = (int)(r / P.ny);
    int l = p - k0r;
    return l < 0 ? l + P.nz : l;
}

// adjoint of the E^{n+1} values produced by the interior update (Mur terms folded in)
__device__ inline double lam_eff(const Params &P, const double *lE, int c, int i, int j, int l, int k0r, int shift,
                                 int fm, double cm) {
    if (l < 0 || l >= P.nz) return 0.0;
    int p = ring_plane(l, k0r, P.nz);
    int64_t o = cell_index(P, i, j, p);
    if (c == 2) return l == P.nz - 1 ? 0.0 : lE[o];
    if (l == 0 || l == P.nz - 1) return 0.0;
    double v = lE[o];
    if (l == 1 && !shift) v += cm * lE[cell_index(P, i, j, ring_plane(0, k0r, P.nz))];
    if (l == P.nz - 2 && fm) v += cm * lE[cell_index(P, i, j, ring_plane(P.nz - 1, k0r, P.nz))];
    return v;
}

// fm: the forward applied the Mur condition at the front face (window at rest)
__global__ void __launch_bounds__(AT) k_adj_e(Params P, int k0r, int shift, int fm, double cm, const double *lEx,
                                              const double *lEy, const double *lEz, double *nEx, double *nEy,
                                              double *nEz, double *lBx, double *lBy, double *lBz, double *Jx,
                                              double *Jy, double *Jz) {
    int64_t o = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (o >= P.nc) return;
    int i, j, p;
    int l = plane_of(P, o, k0r, i, j, p);
    const double *lE[3] = {lEx, lEy, lEz};
    double *nE[3] = {nEx, nEy, nEz}, *J[3] = {Jx, Jy, Jz};
    double dt = P.dt;
    double e[3];
    for (int c = 0; c < 3; ++c) {
        e[c] = lam_eff(P, lE[c], c, i, j, l, k0r, shift, fm, cm);
        double n = e[c];
        if (c < 2) {
            if (l == 0 && !shift) n += -cm * lE[c][o];
            if (l == 1 && !shift) n += lE[c][cell_index(P, i, j, ring_plane(0, k0r, P.nz))];
            if (l == P.nz - 1) n += fm ? -cm * lE[c][o] : lE[c][o];  // Mur, or the face kept
            if (l == P.nz - 2 && fm) n += lE[c][cell_index(P, i, j, ring_plane(P.nz - 1, k0r, P.nz))];
        } else if (l == P.nz - 1)
            n += lE[2][o];  // untouched outside half plane
        nE[c][o] = n;
        J[c][o] = -dt * e[c];
    }
    // lam_B += dt * (transpose of the curl of B in the E update)
    double ex_l1 = lam_eff(P, lEx, 0, i, j, l + 1, k0r, shift, fm, cm);
    double ey_l1 = lam_eff(P, lEy, 1, i, j, l + 1, k0r, shift, fm, cm);
    double ez_j1 = lam_eff(P, lEz, 2, i, j + 1, l, k0r, shift, fm, cm);
    double ez_i1 = lam_eff(P, lEz, 2, i + 1, j, l, k0r, shift, fm, cm);
    double ex_j1 = lam_eff(P, lEx, 0, i, j + 1, l, k0r, shift, fm, cm);
    double ey_i1 = lam_eff(P, lEy, 1, i + 1, j, l, k0r, shift, fm, cm);
    lBx[o] += dt * (e[1] - ey_l1 - e[2] + ez_j1);
    lBy[o] += dt * (-e[0] + ex_l1 + e[2] - ez_i1);
    lBz[o] += dt * (e[0] - ex_j1 - e[1] + ey_i1);
}

// lam_E += transpose of (B <- B - h curl E) applied to lam_B
__global__ void __launch_bounds__(AT) k_adj_bhalf(Params P, int k0r, double h, const double *lBx, const double *lBy,
                                                  const double *lBz, double *nEx, double *nEy, double *nEz) {
    int64_t o = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (o >= P.nc) return;
    int i, j, p;
    int l = plane_of(P, o, k0r, i, j, p);
    // lam of Bx, By at (i, j, l') with l' = nz-1 does not feed E (those half planes are not updated)
    auto bxy = [&](const double *a, int ii, int jj, int ll) -> double {
        if (ll < 0 || ll >= P.nz - 1) return 0.0;
        return a[cell_index(P, ii, jj, ring_plane(ll, k0r, P.nz))];
    };
    auto bz = [&](int ii, int jj, int ll) -> double { return lBz[cell_index(P, ii, jj, ring_plane(ll, k0r, P.nz))]; };
    nEx[o] += h * (bxy(lBy, i, j, l) - bxy(lBy, i, j, l - 1) - bz(i, j, l) + bz(i, j - 1, l));
    nEy[o] += h * (bz(i, j, l) - bz(i - 1, j, l) - bxy(lBx, i, j, l) + bxy(lBx, i, j, l - 1));
    nEz[o] += h * (bxy(lBx, i, j, l) - bxy(lBx, i, j - 1, l) - bxy(lBy, i, j, l) + bxy(lBy, i - 1, j, l));
}

__global__ void k_zero_plane(int64_t plane, int p, double *a0, double *a1, double *a2, double *b0, double *b1,
                             double *b2) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= plane) return;
    int64_t o = (int64_t)p * plane + s;
    a0[o] = a1[o] = a2[o] = 0.0;
    b0[o] = b1[o] = b2[o] = 0.0;
}

// <lam_Jz, J_ion>: sum over cells of lam_Jz times the ion profile of the cell's plane
__global__ void __launch_bounds__(AT) k_ion_dot(Params P, int k0r, const double *lJz, const double *jion, double *out) {
    __shared__ double s[AT];
    double v = 0.0;
    for (int64_t o = (int64_t)blockIdx.x * AT + threadIdx.x; o < P.nc; o += (int64_t)gridDim.x * AT) {
        int p = (int)(o / P.plane);
        int l = p - k0r;
        if (l < 0) l += P.nz;
        if (l != P.nz - 1) v += lJz[o] * jion[l];
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = AT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

// ---------------------------------------------------------------- particle reverse
__device__ inline void weights_d(double x, double off, double w[3], double dw[3], int64_t &lo) {
    double n = floor(x - off + 0.5);
    lo = (int64_t)n - 1;
    for (int a = 0; a < 3; ++a) {
        double d = x - off - (double)(lo + a);
        w[a] = spline2<double>(d);
        dw[a] = dspline2<double>(d);
    }
}

// value of one component and the scatter of lam * shape into the adjoint field; returns d(lam*value)/dX
__device__ inline void gather_adj(const Params &P, const StepCtx &S, const double *F, double *lF, const double X[3],
                                  int sx, int sy, int sz, double lam, double gX[3]) {
    double w[3][3], dw[3][3];
    int64_t lo[3];
    weights_d(X[0], sx ? 0.5 : 0.0, w[0], dw[0], lo[0]);
    weights_d(X[1], sy ? 0.5 : 0.0, w[1], dw[1], lo[1]);
    weights_d(X[2], sz ? 0.5 : 0.0, w[2], dw[2], lo[2]);
    for (int c = 0; c < 3; ++c) {
        int p = ring_plane((int)(lo[2] + c - S.k0), S.k0r, P.nz);
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                int64_t o = cell_index(P, (int)(lo[0] + a), (int)(lo[1] + b), p);
                if (lam != 0.0) atomicAdd(&lF[o], lam * w[0][a] * w[1][b] * w[2][c]);
                double f = F[o] * lam;
                gX[0] += f * dw[0][a] * w[1][b] * w[2][c];
                gX[1] += f * w[0][a] * dw[1][b] * w[2][c];
                gX[2] += f * w[0][a] * w[1][b] * dw[2][c];
            }
    }
}

// adjoint of the tight-window Esirkepov deposit: returns <lamJ, J_p>
__device__ inline double deposit_adj(const Params &P, const StepCtx &S, double *const lJ[3], const double X0[3],
                                     const double X1[3], double w, double gX0[3], double gX1[3]) {
    double S0[3][4], DS[3][4], d0[3][4], d1[3][4];
    int64_t base[3];
    for (int d = 0; d < 3; ++d) {
        int64_t n0 = (int64_t)floor(X0[d] + 0.5), n1 = (int64_t)floor(X1[d] + 0.5);
        base[d] = (n0 < n1 ? n0 : n1) - 1;
        for (int m = 0; m < 4; ++m) {
            double node = (double)(base[d] + m);
            S0[d][m] = spline2<double>(X0[d] - node);
            DS[d][m] = spline2<double>(X1[d] - node) - S0[d][m];
            d0[d][m] = dspline2<double>(X0[d] - node);
            d1[d][m] = dspline2<double>(X1[d] - node);
        }
    }
    double f = w / P.dt;
    double gS0[3][4] = {{0}}, gDS[3][4] = {{0}};
    double val = 0.0;
    for (int c = 0; c < 3; ++c) {
        int ca = (c + 1) % 3, cb = (c + 2) % 3;
        for (int ma = 0; ma < 4; ++ma)
            for (int mb = 0; mb < 4; ++mb) {
                double lam[3], suf = 0.0;
                for (int m = 2; m >= 0; --m) {
                    int64_t id[3];
                    id[c] = base[c] + m;
                    id[ca] = base[ca] + ma;
                    id[cb] = base[cb] + mb;
                    int p = ring_plane((int)(id[2] - S.k0), S.k0r, P.nz);
                    suf += lJ[c][cell_index(P, (int)id[0], (int)id[1], p)];
                    lam[m] = f * suf;
                }
                double A = S0[ca][ma] * S0[cb][mb] + 0.5 * DS[ca][ma] * S0[cb][mb] + 0.5 * S0[ca][ma] * DS[cb][mb] +
                           DS[ca][ma] * DS[cb][mb] * (1.0 / 3.0);
                double gA = 0.0;
                for (int m = 0; m < 3; ++m) {
                    val += DS[c][m] * A * lam[m];
                    gDS[c][m] += A * lam[m];
                    gA += DS[c][m] * lam[m];
                }
                gS0[ca][ma] += gA * (S0[cb][mb] + 0.5 * DS[cb][mb]);
                gDS[ca][ma] += gA * (0.5 * S0[cb][mb] + DS[cb][mb] * (1.0 / 3.0));
                gS0[cb][mb] += gA * (S0[ca][ma] + 0.5 * DS[ca][ma]);
                gDS[cb][mb] += gA * (0.5 * S0[ca][ma] + DS[ca][ma] * (1.0 / 3.0));
            }
    }
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < 4; ++m) {
            gX0[d] += (gS0[d][m] - gDS[d][m]) * d0[d][m];
            gX1[d] += gDS[d][m] * d1[d][m];
        }
    return val;
}

__device__ inline void push_boris_adj(double dt, const double u[3], const double E[3], const double B[3],
                                      const double lo[3], double lu[3], double lE[3], double lB[3]) {
    double a = -0.5 * dt;
    double um[3], T[3], Sv[3], up[3], c[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + a * E[d];
    double gm = sqrt(1.0 + dot3(um, um));
    for (int d = 0; d < 3; ++d) T[d] = a * B[d] / gm;
    double tt = dot3(T, T);
    for (int d = 0; d < 3; ++d) Sv[d] = 2.0 * T[d] / (1.0 + tt);
    cross3(um, T, c);
    for (int d = 0; d < 3; ++d) up[d] = um[d] + c[d];
    double lum[3], lup[3], lS[3], lT[3], tmp[3];
    for (int d = 0; d < 3; ++d) {
        lE[d] = a * lo[d];
        lum[d] = lo[d];
    }
    cross3(Sv, lo, lup);
    cross3(lo, up, lS);
    cross3(T, lup, tmp);
    for (int d = 0; d < 3; ++d) lum[d] += lup[d] + tmp[d];
    cross3(lup, um, lT);
    double TS = dot3(T, lS), den = 1.0 + tt;
    for (int d = 0; d < 3; ++d) lT[d] += 2.0 * lS[d] / den - 4.0 * T[d] * TS / (den * den);
    double lgm = -a * dot3(B, lT) / (gm * gm);
    for (int d = 0; d < 3; ++d) lB[d] = a * lT[d] / gm;
    for (int d = 0; d < 3; ++d) lum[d] += lgm * um[d] / gm;
    for (int d = 0; d < 3; ++d) {
        lu[d] = lum[d];
        lE[d] += a * lum[d];
    }
}

__device__ inline void push_vay_adj(double dt, const double u[3], const double E[3], const double B[3],
                                    const double lo[3], double lu[3], double lE[3], double lB[3]) {
    double a = -0.5 * dt;
    double g0 = sqrt(1.0 + dot3(u, u));
    double v0[3], c[3], u1[3], tau[3], t[3], w[3];
    for (int d = 0; d < 3; ++d) v0[d] = u[d] / g0;
    cross3(v0, B, c);
    for (int d = 0; d < 3; ++d) u1[d] = u[d] + 2.0 * a * E[d] + a * c[d];
    for (int d = 0; d < 3; ++d) tau[d] = a * B[d];
    double us = dot3(u1, tau), tau2 = dot3(tau, tau);
    double sig = 1.0 + dot3(u1, u1) - tau2;
    double D = sqrt(sig * sig + 4.0 * (tau2 + us * us));
    double gn = sqrt(0.5 * (sig + D));
    for (int d = 0; d < 3; ++d) t[d] = tau[d] / gn;
    double sf = 1.0 / (1.0 + dot3(t, t));
    double ut = dot3(u1, t);
    cross3(u1, t, c);
    for (int d = 0; d < 3; ++d) w[d] = u1[d] + ut * t[d] + c[d];
    double lsf = dot3(lo, w), lw[3], lu1[3], lt[3], ltau[3], tmp[3];
    for (int d = 0; d < 3; ++d) lw[d] = sf * lo[d];
    double tlw = dot3(t, lw);
    cross3(t, lw, tmp);
    for (int d = 0; d < 3; ++d) lu1[d] = lw[d] + tlw * t[d] + tmp[d];
    cross3(lw, u1, tmp);
    for (int d = 0; d < 3; ++d) lt[d] = tlw * u1[d] + ut * lw[d] + tmp[d];
    for (int d = 0; d < 3; ++d) lt[d] += -2.0 * lsf * sf * sf * t[d];
    double lgn = -dot3(tau, lt) / (gn * gn);
    for (int d = 0; d < 3; ++d) ltau[d] = lt[d] / gn;
    double lsig = lgn / (4.0 * gn), lD = lgn / (4.0 * gn);
    lsig += lD * sig / D;
    double ltau2 = lD * 2.0 / D, lus = lD * 4.0 * us / D;
    ltau2 += -lsig;
    for (int d = 0; d < 3; ++d) lu1[d] += 2.0 * lsig * u1[d];
    for (int d = 0; d < 3; ++d) {
        ltau[d] += 2.0 * ltau2 * tau[d] + lus * u1[d];
        lu1[d] += lus * tau[d];
    }
    for (int d = 0; d < 3; ++d) lB[d] = a * ltau[d];
    double lv0[3];
    cross3(B, lu1, lv0);
    cross3(lu1, v0, tmp);
    for (int d = 0; d < 3; ++d) {
        lv0[d] *= a;
        lB[d] += a * tmp[d];
        lE[d] = 2.0 * a * lu1[d];
        lu[d] = lu1[d];
    }
    double uv = dot3(u, lv0);
    for (int d = 0; d < 3; ++d) lu[d] += lv0[d] / g0 - u[d] * uv / (g0 * g0 * g0);
}

__global__ void __launch_bounds__(AT) k_adj_particles(Params P, StepCtx S, Part64 p, int64_t n, Lam L,
                                                      FieldsT<double> fE, const double *Bnx, const double *Bny,
                                                      const double *Bnz, double *nEx, double *nEy, double *nEz,
                                                      double *lBx, double *lBy, double *lBz, double *lJx,
                                                      double *lJy, double *lJz, int plasma, double *part) {
    __shared__ double sh[2][AT];
    double gK = 0.0, gn = 0.0;
    int64_t q = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (q < n) {
        if (!p.alive[q]) {
            for (int d = 0; d < 3; ++d) {
                L.x[d][q] = 0.0;
                L.u[d][q] = 0.0;
            }
        } else {
            double X[3] = {p.x[q], p.y[q], p.z[q]}, U[3] = {p.ux[q], p.uy[q], p.uz[q]};
            const double *Bn[3] = {Bnx, Bny, Bnz};
            double E[3], B[3], Ee[3], Be[3], dEe[3], dBe[3];
            // forward recompute: gather (values only), push, move
            const int stE[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, stB[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
            for (int c = 0; c < 3; ++c) {
                E[c] = 0.0;
                B[c] = 0.0;
                double wv[3][3], dv[3][3];
                int64_t lo[3];
                for (int d = 0; d < 3; ++d) weights_d(X[d], stE[c][d] ? 0.5 : 0.0, wv[d], dv[d], lo[d]);
                for (int cc = 0; cc < 3; ++cc) {
                    int pl = ring_plane((int)(lo[2] + cc - S.k0), S.k0r, P.nz);
                    for (int b = 0; b < 3; ++b)
                        for (int a = 0; a < 3; ++a)
                            E[c] += wv[0][a] * wv[1][b] * wv[2][cc] *
                                    fE.E[c][cell_index(P, (int)(lo[0] + a), (int)(lo[1] + b), pl)];
                }
                for (int d = 0; d < 3; ++d) weights_d(X[d], stB[c][d] ? 0.5 : 0.0, wv[d], dv[d], lo[d]);
                for (int cc = 0; cc < 3; ++cc) {
                    int pl = ring_plane((int)(lo[2] + cc - S.k0), S.k0r, P.nz);
                    for (int b = 0; b < 3; ++b)
                        for (int a = 0; a < 3; ++a)
                            B[c] += wv[0][a] * wv[1][b] * wv[2][cc] *
                                    Bn[c][cell_index(P, (int)(lo[0] + a), (int)(lo[1] + b), pl)];
                }
            }
            ext_field64(P, X[2], S.t, Ee, Be, dEe, dBe);
            for (int d = 0; d < 3; ++d) {
                E[d] += Ee[d];
                B[d] += Be[d];
            }
            double Un[3];
            push<double>(P.pusher, -0.5 * P.dt, U, E, B, Un);
            double g = sqrt(1.0 + dot3(Un, Un));
            double X1[3];
            for (int d = 0; d < 3; ++d) X1[d] = X[d] + P.dt * Un[d] / g;
            if (!(isfinite(X1[0]) && isfinite(X1[1]) && isfinite(X1[2]))) {
                // the forward step dropped this particle without a deposit
                for (int d = 0; d < 3; ++d) {
                    L.x[d][q] = 0.0;
                    L.u[d][q] = 0.0;
                }
            } else {
                int alive1 = !(X1[2] < (double)(S.k0n + 3) || X1[2] >= (double)(S.k0n + P.nz - 4));
                double gX1[3], lun[3];
                for (int d = 0; d < 3; ++d) {
                    gX1[d] = alive1 ? L.x[d][q] : 0.0;
                    lun[d] = alive1 ? L.u[d][q] : 0.0;
                }
                double gX[3] = {0, 0, 0};
                double *lJ[3] = {lJx, lJy, lJz};
                double val = deposit_adj(P, S, lJ, X, X1, p.w[q], gX, gX1);
                if (plasma) gn += val;
                double ug = dot3(Un, gX1);
                for (int d = 0; d < 3; ++d) {
                    gX[d] += gX1[d];
                    lun[d] += P.dt * (gX1[d] / g - Un[d] * ug / (g * g * g));
                }
                double lu[3], lEp[3], lBp[3];
                if (P.pusher == 1)
                    push_vay_adj(P.dt, U, E, B, lun, lu, lEp, lBp);
                else
                    push_boris_adj(P.dt, U, E, B, lun, lu, lEp, lBp);
                gK += dot3(lEp, Ee) + dot3(lBp, Be);
                gX[2] += dot3(lEp, dEe) + dot3(lBp, dBe);
                double *nE[3] = {nEx, nEy, nEz}, *lB[3] = {lBx, lBy, lBz};
                for (int c = 0; c < 3; ++c) {
                    gather_adj(P, S, fE.E[c], nE[c], X, stE[c][0], stE[c][1], stE[c][2], lEp[c], gX);
                    gather_adj(P, S, Bn[c], lB[c], X, stB[c][0], stB[c][1], stB[c][2], lBp[c], gX);
                }
                for (int d = 0; d < 3; ++d) {
                    L.x[d][q] = gX[d];
                    L.u[d][q] = lu[d];
                }
            }
        }
    }
    sh[0][threadIdx.x] = gK;
    sh[1][threadIdx.x] = gn;
    __syncthreads();
    for (int h = AT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

__global__ void k_zero_slots(Lam L, int64_t a, int64_t b) {
    int64_t q = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= b) return;
    for (int d = 0; d < 3; ++d) {
        L.x[d][q] = 0.0;
        L.u[d][q] = 0.0;
    }
}

// ---------------------------------------------------------------- seed
__global__ void __launch_bounds__(AT) k_bunch_sums(Part64 p, int64_t n, double kb, double *out) {
    __shared__ double s[3][AT];
    double v[3] = {0, 0, 0};
    int64_t q = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (q < n && p.alive[q]) {
        double sn, cs;
        sincos(kb * p.z[q], &sn, &cs);
        v[0] = p.w[q];
        v[1] = p.w[q] * cs;
        v[2] = p.w[q] * sn;
    }
    for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = AT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[3 * blockIdx.x + k] = s[k][0];
}

__global__ void k_bunch_seed(Part64 p, int64_t n, double kb, double C, double Sn, double A, double W, double *lz) {
    int64_t q = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (q >= n || !p.alive[q]) return;
    double sn, cs;
    sincos(kb * p.z[q], &sn, &cs);
    lz[q] = p.w[q] * kb * (-C * sn + Sn * cs) / (A * W);
}

pic_status adjoint_seed(Ctx &c, double kb, double *lam, double *loss) {
    int64_t len = 6 * (std::max<int64_t>(c.cap_b, 1) + std::max<int64_t>(c.cap_p, 1)) + 6 * c.P.nc;
    PIC_HIP(c, hipMemsetAsync(lam, 0, 8 * (uint64_t)len, c.st));
    int64_t n = c.nb_slots;
    double C = 0, Sn = 0, W = 0;
    if (n > 0) {
        int nblk = nblocks(n, AT);
        hipLaunchKernelGGL(k_bunch_sums, dim3(nblk), dim3(AT), 0, c.st, c.b64, n, kb, c.red);
        std::vector<double> h(3 * (size_t)nblk);
        PIC_HIP(c, hipMemcpyAsync(h.data(), c.red, 24 * (uint64_t)nblk, hipMemcpyDeviceToHost, c.st));
        PIC_HIP(c, hipStreamSynchronize(c.st));
        for (int b = 0; b < nblk; ++b) {
            W += h[3 * b];
            C += h[3 * b + 1];
            Sn += h[3 * b + 2];
        }
    }
    if (W <= 0) {
        c.err = "adjoint seed: no beam particles";
        return PIC_ESTATE;
    }
    double A = sqrt(C * C + Sn * Sn);
    *loss = A / W;
    Lam L = lam_view(lam, 0, c.cap_b);
    hipLaunchKernelGGL(k_bunch_seed, dim3(nblocks(n, AT)), dim3(AT), 0, c.st, c.b64, n, kb, C, Sn, A, W, L.x[2]);
    PIC_HIP(c, hipStreamSynchronize(c.st));
    return PIC_OK;
}

// slots of plasma after the forward step's injection (host replay of the sheet logic)
static int64_t plasma_slots_after(const Ctx &c, const StepCtx &S) {
    if (!c.P.has_plasma) return c.np_slots;
    int64_t sheet = sheet_particles(c.P);
    double hi = (double)(S.k0n + c.P.nz - 4);
    int64_t l = c.sh_hi, n = c.np_slots;
    while (sheet_z(l, c.P.ppz, c.P.bR, S.t1) < hi) {
        if (sheet_weight(c.P, l) != 0.0) n += sheet;
        ++l;
    }
    return n;
}

pic_status adjoint_step(Ctx &c, double *lam, double grad[2]) {
    const Params &P = c.P;
    StepCtx S = make_step_ctx(c);
    uint64_t cb = (uint64_t)std::max<int64_t>(c.cap_b, 1), cp = (uint64_t)std::max<int64_t>(c.cap_p, 1);
    Lam Lb = lam_view(lam, 0, c.cap_b), Lp = lam_view(lam, 6 * cb, c.cap_p);
    double *lE[3], *lB[3], *nE[3], *Bn[3];
    for (int k = 0; k < 3; ++k) {
        lE[k] = lam + 6 * (cb + cp) + k * P.nc;
        lB[k] = lam + 6 * (cb + cp) + (3 + k) * P.nc;
        nE[k] = c.adj + k * P.nc;
        Bn[k] = c.adj + (3 + k) * P.nc;
    }
    // slots injected during step n carry no adjoint into state n
    int64_t np1 = std::min<int64_t>(plasma_slots_after(c, S), c.cap_p);
    if (np1 > c.np_slots)
        hipLaunchKernelGGL(k_zero_slots, dim3(nblocks(np1 - c.np_slots, AT)), dim3(AT), 0, c.st, Lp, c.np_slots, np1);
    // B^n = B^{n-1/2} - (dt/2) curl E^n
    for (int k = 0; k < 3; ++k)
        PIC_HIP(c, hipMemcpyAsync(Bn[k], c.B64[k], 8 * P.nc, hipMemcpyDeviceToDevice, c.st));
    FieldsT<double> fn;
    for (int k = 0; k < 3; ++k) {
        fn.E[k] = c.E64[k];
        fn.B[k] = Bn[k];
    }
    launch_bhalf<double>(P, S.k0r, fn, 0.5 * P.dt, nullptr, c.st);
    // window shift: the back plane became the empty front plane
    if (S.shift)
        hipLaunchKernelGGL(k_zero_plane, dim3(nblocks(P.plane, 256)), dim3(256), 0, c.st, (int64_t)P.plane, S.k0r,
                           lE[0], lE[1], lE[2], lB[0], lB[1], lB[2]);
    // E update with Mur faces
    double cm = (P.dt - 1.0) / (P.dt + 1.0);
    int nb = nblocks(P.nc, AT);
    hipLaunchKernelGGL(k_adj_e, dim3(nb), dim3(AT), 0, c.st, P, S.k0r, S.shift, (int)(c.bw <= 0.0), cm, lE[0], lE[1],
                       lE[2], nE[0], nE[1],
                       nE[2], lB[0], lB[1], lB[2], c.J64[0], c.J64[1], c.J64[2]);
    // second half step
    hipLaunchKernelGGL(k_adj_bhalf, dim3(nb), dim3(AT), 0, c.st, P, S.k0r, 0.5 * P.dt, lB[0], lB[1], lB[2], nE[0],
                       nE[1], nE[2]);
    // ion current: n0 dL/dn0 += <lam_Jz, J_ion>
    double gn = 0.0, gK = 0.0;
    if (P.ions && c.sh_hi > c.sh_lo) {
        launch_ion64(P, c.sh_lo, c.sh_hi - c.sh_lo, S.t, S.t1, S.k0, c.jion64, c.st);
        hipLaunchKernelGGL(k_ion_dot, dim3(256), dim3(AT), 0, c.st, P, S.k0r, c.J64[2], c.jion64, c.red);
        std::vector<double> h(256);
        PIC_HIP(c, hipMemcpyAsync(h.data(), c.red, 8 * 256, hipMemcpyDeviceToHost, c.st));
        PIC_HIP(c, hipMemsetAsync(c.jion64, 0, 8 * P.nz, c.st));
        PIC_HIP(c, hipStreamSynchronize(c.st));
        for (int b = 0; b < 256; ++b) gn += h[b];
    }
    // particles
    for (int sp = 0; sp < 2; ++sp) {
        int64_t n = sp ? c.np_slots : c.nb_slots;
        if (n <= 0) continue;
        int nblk = nblocks(n, AT);
        hipLaunchKernelGGL(k_adj_particles, dim3(nblk), dim3(AT), 0, c.st, P, S, sp ? c.p64 : c.b64, n, sp ? Lp : Lb,
                           fn, Bn[0], Bn[1], Bn[2], nE[0], nE[1], nE[2], lB[0], lB[1], lB[2], c.J64[0], c.J64[1],
                           c.J64[2], sp, c.red);
        std::vector<double> h(2 * (size_t)nblk);
        PIC_HIP(c, hipMemcpyAsync(h.data(), c.red, 16 * (uint64_t)nblk, hipMemcpyDeviceToHost, c.st));
        PIC_HIP(c, hipStreamSynchronize(c.st));
        for (int b = 0; b < nblk; ++b) {
            gK += h[2 * b];
            gn += h[2 * b + 1];
        }
    }
    // first half step, then the new lam_E
    hipLaunchKernelGGL(k_adj_bhalf, dim3(nb), dim3(AT), 0, c.st, P, S.k0r, 0.5 * P.dt, lB[0], lB[1], lB[2], nE[0],
                       nE[1], nE[2]);
    for (int k = 0; k < 3; ++k) {
        PIC_HIP(c, hipMemcpyAsync(lE[k], nE[k], 8 * P.nc, hipMemcpyDeviceToDevice, c.st));
        PIC_HIP(c, hipMemsetAsync(c.J64[k], 0, 8 * P.nc, c.st));
    }
    PIC_HIP(c, hipStreamSynchronize(c.st));
    grad[0] += gK;
    grad[1] += gn;
    return PIC_OK;
}

}  // namespace pic
