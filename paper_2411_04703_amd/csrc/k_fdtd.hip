// k_fdtd.hip -- Yee FDTD in normalised units on the ring-buffered moving window.
//
// Maxwell's curl equations with electron and ion currents (section 1,
// Eq. Max1, Max2 of the paper; Gaussian factors absorbed by the units):
//   B <- B - (dt/2) curl E      (twice per step, around the particle push)
//   E <- E + dt (curl B - J)
// Yee staggering: Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2), Bx(i,j+1/2,k+1/2)
// By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k).  x, y periodic.  z: nz logical planes
// stored as a ring (logical plane l lives in ring plane (l + k0) mod nz).  The
// z boundaries absorb (section 1): first-order Mur on the tangential E at the
// back face, and at the front face while the window is at rest; a moving
// window's front face keeps its tangential E, and the half planes beyond it
// stay zero.
// One thread per cell, x fastest: every array access is coalesced along x.  The
// grid is (cells of a plane, ring planes): the ring plane is the block's y
// index and (i, j) come from 32-bit arithmetic on the in-plane index.
#include "pic_internal.h"

namespace pic {

template <typename JT> __device__ inline double jvalue(JT v, double finv);
template <> __device__ inline double jvalue<double>(double v, double) { return v; }
template <> __device__ inline double jvalue<long long>(long long v, double finv) { return (double)v * finv; }

// in-plane index s = i + nx j of the calling thread, false past the plane's end
__device__ inline bool plane_cell(const Params &P, int &i, int &j) {
    const int s = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
    if (s >= P.plane) return false;
    j = s / P.nx;
    i = s - j * P.nx;
    return true;
}

template <typename T>
__global__ void __launch_bounds__(256) k_bhalf(Params P, int k0r, FieldsT<T> f, T h, T *murbuf) {
    int i, j;
    if (!plane_cell(P, i, j)) return;
    const int p = (int)blockIdx.y;
    const int64_t o = (int64_t)p * P.plane + i + (int64_t)P.nx * j;
    int l = p - k0r;
    if (l < 0) l += P.nz;
    int64_t oi = o + ((i + 1 == P.nx) ? 1 - P.nx : 1);
    int64_t oj = o + ((j + 1 == P.ny) ? (int64_t)(1 - P.ny) * P.nx : P.nx);
    const T *Ex = f.E[0], *Ey = f.E[1], *Ez = f.E[2];
    T ex = Ex[o], ey = Ey[o], ez = Ez[o];
    if (l != P.nz - 1) {
        int64_t ol = o + ((p + 1 == P.nz) ? -(int64_t)(P.nz - 1) * P.plane : (int64_t)P.plane);
        f.B[0][o] -= h * ((Ez[oj] - ez) - (Ey[ol] - ey));
        f.B[1][o] -= h * ((Ex[ol] - ex) - (Ez[oi] - ez));
    }
    f.B[2][o] -= h * ((Ey[oi] - ey) - (Ex[oj] - ex));
    if (murbuf) {
        int q = l == 0 ? 0 : l == 1 ? 1 : l == P.nz - 2 ? 2 : l == P.nz - 1 ? 3 : -1;
        if (q >= 0) {
            int64_t s = (int64_t)i + (int64_t)P.nx * j;
            murbuf[(2 * q + 0) * (int64_t)P.plane + s] = ex;
            murbuf[(2 * q + 1) * (int64_t)P.plane + s] = ey;
        }
    }
}

template <typename T, typename JT>
__global__ void __launch_bounds__(256) k_eupdate(Params P, int k0r, FieldsT<T> f, JT *Jx, JT *Jy, JT *Jz,
                                                 const JT *jion, T dt) {
    int i, j;
    if (!plane_cell(P, i, j)) return;
    const int p = (int)blockIdx.y;
    const int64_t o = (int64_t)p * P.plane + i + (int64_t)P.nx * j;
    int l = p - k0r;
    if (l < 0) l += P.nz;
    int64_t oi = o - ((i == 0) ? 1 - P.nx : 1);
    int64_t oj = o - ((j == 0) ? (int64_t)(1 - P.ny) * P.nx : P.nx);
    int64_t ol = o - ((p == 0) ? -(int64_t)(P.nz - 1) * P.plane : (int64_t)P.plane);
    const T *Bx = f.B[0], *By = f.B[1], *Bz = f.B[2];
    T bx = Bx[o], by = By[o], bz = Bz[o];
    double jx = jvalue<JT>(Jx[o], P.finv), jy = jvalue<JT>(Jy[o], P.finv), jz = jvalue<JT>(Jz[o], P.finv);
    Jx[o] = JT(0);
    Jy[o] = JT(0);
    Jz[o] = JT(0);
    if (l != 0 && l != P.nz - 1) {
        f.E[0][o] += dt * ((bz - Bz[oj]) - (by - By[ol]) - (T)jx);
        f.E[1][o] += dt * ((bx - Bx[ol]) - (bz - Bz[oi]) - (T)jy);
    }
    if (l != P.nz - 1) {
        double jt = jz + jvalue<JT>(jion[l], P.finv);
        f.E[2][o] += dt * ((by - By[oi]) - (bx - Bx[oj]) - (T)jt);
    }
}

// Mur faces (tangential E on logical planes 0 and nz-1) from the saved
// pre-update planes -- the front face only while the window is at rest: a
// moving window's front keeps its tangential E (zero; the planes enter empty),
// since a static-face Mur condition at a face that jumps forward every step or
// two is unstable with plasma streaming in.  When the window shifts after this
// step, the back plane becomes the new (empty) front plane instead: E and B
// there are zeroed.  Also clears the ion current profile for the next step.
template <typename T, typename JT>
__global__ void k_mur_shift(Params P, int k0r, int shift, int front_mur, FieldsT<T> f, const T *murbuf, JT *jion,
                            T cm) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < P.nz) jion[s] = JT(0);
    if (s >= P.plane) return;
    int64_t pl = P.plane;
    int p0 = k0r, p1 = ring_plane(1, k0r, P.nz), pm = ring_plane(P.nz - 2, k0r, P.nz),
        pt = ring_plane(P.nz - 1, k0r, P.nz);
    for (int c = 0; c < 2; ++c) {
        const T *o0 = murbuf + (0 + c) * pl, *o1 = murbuf + (2 + c) * pl;
        const T *o2 = murbuf + (4 + c) * pl, *o3 = murbuf + (6 + c) * pl;
        T *F = f.E[c];
        if (!shift) F[p0 * pl + s] = o1[s] + cm * (F[p1 * pl + s] - o0[s]);
        if (front_mur) F[pt * pl + s] = o2[s] + cm * (F[pm * pl + s] - o3[s]);
    }
    if (shift) {
        for (int c = 0; c < 3; ++c) {
            f.E[c][p0 * pl + s] = T(0);
            f.B[c][p0 * pl + s] = T(0);
        }
    }
}

template <typename T>
void launch_bhalf(const Params &P, int k0r, FieldsT<T> f, T h, T *murbuf, hipStream_t st) {
    hipLaunchKernelGGL(k_bhalf<T>, dim3(nblocks(P.plane, 256), P.nz), dim3(256), 0, st, P, k0r, f, h, murbuf);
}

template <typename T, typename JT>
void launch_eupdate(const Params &P, int k0r, FieldsT<T> f, JT *J[3], const JT *jion, T dt, hipStream_t st) {
    hipLaunchKernelGGL((k_eupdate<T, JT>), dim3(nblocks(P.plane, 256), P.nz), dim3(256), 0, st, P, k0r, f, J[0], J[1],
                       J[2], jion, dt);
}

template <typename T, typename JT>
void launch_mur_shift(const Params &P, int k0r, int shift, int front_mur, FieldsT<T> f, const T *murbuf, JT *jion,
                      T dt, hipStream_t st) {
    int64_t n = P.plane > P.nz ? P.plane : P.nz;
    T cm = (dt - T(1)) / (dt + T(1));
    hipLaunchKernelGGL((k_mur_shift<T, JT>), dim3(nblocks(n, 256)), dim3(256), 0, st, P, k0r, shift, front_mur, f,
                       murbuf, jion, cm);
}

template void launch_bhalf<double>(const Params &, int, FieldsT<double>, double, double *, hipStream_t);
template void launch_bhalf<float>(const Params &, int, FieldsT<float>, float, float *, hipStream_t);
template void launch_eupdate<double, double>(const Params &, int, FieldsT<double>, double *[3], const double *,
                                             double, hipStream_t);
template void launch_eupdate<float, long long>(const Params &, int, FieldsT<float>, long long *[3],
                                               const long long *, float, hipStream_t);
template void launch_mur_shift<double, double>(const Params &, int, int, int, FieldsT<double>, const double *, double *,
                                               double, hipStream_t);
template void launch_mur_shift<float, long long>(const Params &, int, int, int, FieldsT<float>, const float *,
                                                 long long *, float, hipStream_t);

// ---------------------------------------------------------------- ion current
// Immobile lab ions: the plasma lattice drifting rigidly at -beta_R.  Summed
// over a transversely uniform lattice, their Esirkepov current is J_z(z) only:
// per sheet the running sum of -q w ppx ppy (S(z1 - k) - S(z0 - k)) / dt.
// One thread per sheet, contributions added into a logical-plane profile.
// w32: the FP32 mode's ions, which carry the FP32-rounded weight of their sheet's electrons
// (the weight the electrons are stored with), so that the cold lattice is exactly neutral
// and current-free in either mode
__device__ inline void ion_sheet_terms(const Params &P, int64_t l, double t0, double t1, int64_t k0, double out[4],
                                       int &lbase, bool w32) {
    double w = sheet_weight(P, l);
    if (w32) w = (double)(float)w;
    double z0 = sheet_z(l, P.ppz, P.bR, t0), z1 = sheet_z(l, P.ppz, P.bR, t1);
    int64_t b = (int64_t)floor(z0 + 0.5) - 2;
    double acc = 0.0, f = -w * (double)(P.ppx * P.ppy) / P.dt;
    for (int m = 0; m < 4; ++m) {
        acc += spline2<double>(z1 - (double)(b + m)) - spline2<double>(z0 - (double)(b + m));
        out[m] = f * acc;
    }
    lbase = (int)(b - k0);
}

__global__ void k_ion64(Params P, int64_t sh_lo, int64_t ns, double t0, double t1, int64_t k0, double *jion) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    double v[4];
    int lb;
    ion_sheet_terms(P, sh_lo + q, t0, t1, k0, v, lb, false);
    for (int m = 0; m < 4; ++m)
        if (v[m] != 0.0 && lb + m >= 0 && lb + m < P.nz) atomicAdd(&jion[lb + m], v[m]);
}

__global__ void k_ion_fixed(Params P, int64_t sh_lo, int64_t ns, double t0, double t1, int64_t k0, long long *jion,
                            int32_t *flags) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ns) return;
    double v[4];
    int lb;
    ion_sheet_terms(P, sh_lo + q, t0, t1, k0, v, lb, true);
    for (int m = 0; m < 4; ++m) {
        double s = v[m] * P.fscale;
        if (fabs(s) > 4.0e18) atomicOr(flags, DFLAG_FIXED_OVERFLOW);
        long long iv = (long long)rint(s);
        if (iv != 0 && lb + m >= 0 && lb + m < P.nz)
            atomicAdd((unsigned long long *)&jion[lb + m], (unsigned long long)iv);
    }
}

void launch_ion64(const Params &P, int64_t sh_lo, int64_t ns, double t0, double t1, int64_t k0, double *jion,
                  hipStream_t st) {
    if (ns <= 0) return;
    hipLaunchKernelGGL(k_ion64, dim3(nblocks(ns, 128)), dim3(128), 0, st, P, sh_lo, ns, t0, t1, k0, jion);
}

void launch_ion_fixed(const Params &P, int64_t sh_lo, int64_t ns, double t0, double t1, int64_t k0,
                      long long *jion, int32_t *flags, hipStream_t st) {
    if (ns <= 0) return;
    hipLaunchKernelGGL(k_ion_fixed, dim3(nblocks(ns, 128)), dim3(128), 0, st, P, sh_lo, ns, t0, t1, k0, jion, flags);
}

}  // namespace pic
