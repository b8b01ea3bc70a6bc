// k_plain64.hip -- FP64 plain particle path: absolute FP64 positions, one
// thread per particle, fields read from global memory, current added with
// FP64 atomics.  This is the reference-precision GPU path the FP32 split path
// is measured against.
#include "pic_internal.h"

namespace pic {

// ---------------------------------------------------------------- beam init
// Lab-frame Gaussian at lab time 0 around the box axis (section 3: beam defined
// in the lab), per-particle Lorentz transform of the event and the momentum
// (Eq. Lor1, Lor2), then a straight drift to t' = 0 (the event of particle j
// happens at t'_j = -gR bR z_j).  FP64 throughout.
__global__ void k_beam_init64(Params P, const double *g, int64_t n, double sx, double sy, double szl, double sux,
                              double suy, double gB, double es, Part64 p, double *part) {
    __shared__ double red[2][256];
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double cnt = 0.0, vzs = 0.0;
    if (q < n) {
        double x = 0.5 * P.nx + sx * g[q];
        double y = 0.5 * P.ny + sy * g[n + q];
        double zl = szl * g[2 * n + q];
        double ux = sux * g[3 * n + q], uy = suy * g[4 * n + q];
        double gam = gB * (1.0 + es * g[5 * n + q]);
        double uz = sqrt(gam * gam - 1.0 - ux * ux - uy * uy);
        double glab = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        double zb = P.gR * zl;
        double tb = -P.gR * P.bR * zl;
        double uzb = P.gR * (uz - P.bR * glab);
        double gb = sqrt(1.0 + ux * ux + uy * uy + uzb * uzb);
        double drift = -tb;
        x = x + ux / gb * drift;
        y = y + uy / gb * drift;
        double z = zb + uzb / gb * drift + P.zoff;
        x = fmod(x, (double)P.nx);
        if (x < 0) x += P.nx;
        y = fmod(y, (double)P.ny);
        if (y < 0) y += P.ny;
        p.x[q] = x;
        p.y[q] = y;
        p.z[q] = z;
        p.ux[q] = ux;
        p.uy[q] = uy;
        p.uz[q] = uzb;
        p.w[q] = P.wbeam;
        int al = (z >= 3.0 && z < (double)(P.nz - 4));
        p.alive[q] = al;
        if (al) {
            cnt = 1.0;
            vzs = uzb / gb;
        }
    }
    red[0][threadIdx.x] = cnt;
    red[1][threadIdx.x] = vzs;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

void launch_beam_init64(const Params &P, const double *normals, int64_t n, const double sig[5], double gB, double es,
                        Part64 p, double *partials, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_beam_init64, dim3(nblk), dim3(256), 0, st, P, normals, n, sig[0], sig[1], sig[2], sig[3],
                       sig[4], gB, es, p, partials);
}

// ---------------------------------------------------------------- plasma sheets
// Cold lattice electrons at rest in the lab: boosted u = -gR bR zhat, boosted
// density gR n (Eq. Nnormi).  Sheet l holds nx ny ppx ppy particles in the
// order (j, b, i, a), x = i + (a + 1/2)/ppx, y = j + (b + 1/2)/ppy; with
// mobile ions, as many ions follow in the same order, with the same velocity
// and the weight negated (the charge sign: the deposit and the charge density
// take -w, and the push selects q/m = +1/M by it).
__global__ void k_inject64(Params P, int64_t l0, int64_t total, double t, Part64 p, int64_t slot0) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int64_t per = sheet_particles(P), pe = (int64_t)P.plane * P.ppx * P.ppy;
    int64_t l = l0 + q / per;
    int64_t r = q % per;
    const bool ion = r >= pe;
    if (ion) r -= pe;
    int a = (int)(r % P.ppx);
    r /= P.ppx;
    int i = (int)(r % P.nx);
    r /= P.nx;
    int b = (int)(r % P.ppy);
    int j = (int)(r / P.ppy);
    int64_t s = slot0 + q;
    p.x[s] = i + (a + 0.5) / P.ppx;
    p.y[s] = j + (b + 0.5) / P.ppy;
    p.z[s] = sheet_z(l, P.ppz, P.bR, t);
    p.ux[s] = 0.0;
    p.uy[s] = 0.0;
    p.uz[s] = -P.uR;
    p.w[s] = ion ? -sheet_weight(P, l) : sheet_weight(P, l);
    p.alive[s] = 1;
}

void launch_inject64(const Params &P, int64_t l0, int64_t nsheets, double t, Part64 p, int64_t slot0,
                     hipStream_t st) {
    int64_t total = nsheets * sheet_particles(P);
    if (total <= 0) return;
    hipLaunchKernelGGL(k_inject64, dim3(nblocks(total, 256)), dim3(256), 0, st, P, l0, total, t, p, slot0);
}

// ---------------------------------------------------------------- the step
// Field value of one Yee component at absolute position X, quadratic shape at
// the component's own staggered sites (sx, sy, sz in {0, 1/2}).
__device__ inline double gather64(const Params &P, const StepCtx &S, const double *F, const double X[3], int sx,
                                  int sy, int sz) {
    double wx[3], wy[3], wz[3];
    int64_t lo[3];
    const int st[3] = {sx, sy, sz};
    double *ws[3] = {wx, wy, wz};
    for (int d = 0; d < 3; ++d) {
        double off = st[d] ? 0.5 : 0.0;
        double n = floor(X[d] - off + 0.5);
        weights3<double>(X[d] - off - n, ws[d]);
        lo[d] = (int64_t)n - 1;
    }
    double acc = 0.0;
    for (int c = 0; c < 3; ++c) {
        int p = ring_plane((int)(lo[2] + c - S.k0), S.k0r, P.nz);
        for (int b = 0; b < 3; ++b) {
            double wyz = wy[b] * wz[c];
            for (int a = 0; a < 3; ++a)
                acc += wx[a] * wyz * F[cell_index(P, (int)(lo[0] + a), (int)(lo[1] + b), p)];
        }
    }
    return acc;
}

// Esirkepov (2001) current of the move X0 -> X1 (|dX| < 1 per axis) with
// quadratic shapes, on the tight four-node window of each axis:
//   W_c = DS_c (S0_a S0_b + DS_a S0_b / 2 + S0_a DS_b / 2 + DS_a DS_b / 3),
//   J_c(m + 1/2) = J_c(m - 1/2) - q w W_c(m) / dt (running sum from below),
// the fourth running sum vanishing identically.  q w = -w: electrons carry
// w > 0, mobile ions w < 0.
__device__ inline void deposit64(const Params &P, const StepCtx &S, double *J[3], const double X0[3],
                                 const double X1[3], double w) {
    double S0[3][4], DS[3][4];
    int64_t base[3];
    for (int d = 0; d < 3; ++d) {
        int64_t n0 = (int64_t)floor(X0[d] + 0.5), n1 = (int64_t)floor(X1[d] + 0.5);
        base[d] = (n0 < n1 ? n0 : n1) - 1;
        for (int m = 0; m < 4; ++m) {
            double node = (double)(base[d] + m);
            S0[d][m] = spline2<double>(X0[d] - node);
            DS[d][m] = spline2<double>(X1[d] - node) - S0[d][m];
        }
    }
    double f = w / P.dt;  // -q w / dt
    for (int c = 0; c < 3; ++c) {
        int ca = (c + 1) % 3, cb = (c + 2) % 3;
        for (int ma = 0; ma < 4; ++ma)
            for (int mb = 0; mb < 4; ++mb) {
                double A = S0[ca][ma] * S0[cb][mb] + 0.5 * DS[ca][ma] * S0[cb][mb] + 0.5 * S0[ca][ma] * DS[cb][mb] +
                           DS[ca][ma] * DS[cb][mb] * (1.0 / 3.0);
                if (A == 0.0) continue;
                double run = 0.0;
                for (int m = 0; m < 3; ++m) {
                    run += DS[c][m] * A;
                    if (run == 0.0) continue;
                    int64_t id[3];
                    id[c] = base[c] + m;
                    id[ca] = base[ca] + ma;
                    id[cb] = base[cb] + mb;
                    int p = ring_plane((int)(id[2] - S.k0), S.k0r, P.nz);
                    atomicAdd(&J[c][cell_index(P, (int)id[0], (int)id[1], p)], f * run);
                }
            }
    }
}

__global__ void __launch_bounds__(256) k_step64(Params P, StepCtx S, Part64 p, int64_t n, FieldsT<double> f,
                                                double *Jx, double *Jy, double *Jz, int32_t *flags) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n || !p.alive[q]) return;
    double X[3] = {p.x[q], p.y[q], p.z[q]};
    double U[3] = {p.ux[q], p.uy[q], p.uz[q]};
    double E[3], B[3], Ee[3], Be[3], dEe[3], dBe[3];
    E[0] = gather64(P, S, f.E[0], X, 1, 0, 0);
    E[1] = gather64(P, S, f.E[1], X, 0, 1, 0);
    E[2] = gather64(P, S, f.E[2], X, 0, 0, 1);
    B[0] = gather64(P, S, f.B[0], X, 0, 1, 1);
    B[1] = gather64(P, S, f.B[1], X, 1, 0, 1);
    B[2] = gather64(P, S, f.B[2], X, 1, 1, 0);
    ext_field64(P, X[2], S.t, Ee, Be, dEe, dBe);
    for (int d = 0; d < 3; ++d) {
        E[d] += Ee[d];
        B[d] += Be[d];
    }
    double Un[3];
    push<double>(P.pusher, p.w[q] < 0.0 ? P.ahi : -0.5 * P.dt, U, E, B, Un);
    double g = sqrt(1.0 + dot3(Un, Un));
    double X1[3];
    for (int d = 0; d < 3; ++d) X1[d] = X[d] + P.dt * Un[d] / g;
    if (!(isfinite(X1[0]) && isfinite(X1[1]) && isfinite(X1[2]) && isfinite(g))) {
        // never let a non-finite position reach the index arithmetic: drop the particle
        atomicOr(flags, DFLAG_NONFINITE);
        p.alive[q] = 0;
        return;
    }
    double *J[3] = {Jx, Jy, Jz};
    deposit64(P, S, J, X, X1, p.w[q]);
    if (X1[0] < 0) X1[0] += P.nx;
    if (X1[0] >= P.nx) X1[0] -= P.nx;
    if (X1[1] < 0) X1[1] += P.ny;
    if (X1[1] >= P.ny) X1[1] -= P.ny;
    p.x[q] = X1[0];
    p.y[q] = X1[1];
    p.z[q] = X1[2];
    p.ux[q] = Un[0];
    p.uy[q] = Un[1];
    p.uz[q] = Un[2];
    // window after this step's shift: active band [k0n + 3, k0n + nz - 4)
    if (X1[2] < (double)(S.k0n + 3) || X1[2] >= (double)(S.k0n + P.nz - 4)) p.alive[q] = 0;
}

void launch_step64(const Params &P, const StepCtx &S, Part64 p, int64_t n, FieldsT<double> f, double *J[3],
                   int32_t *flags, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_step64, dim3(nblocks(n, 256)), dim3(256), 0, st, P, S, p, n, f, J[0], J[1], J[2], flags);
}

// ---------------------------------------------------------------- compaction
// Stable removal of dead slots (forward mode only): block-local ranks plus a
// host-side exclusive scan of the block counts, then a scatter.
__global__ void k_count_alive(const int32_t *alive, int64_t n, int32_t *bc) {
    __shared__ int32_t s[256];
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    s[threadIdx.x] = (q < n && alive[q]) ? 1 : 0;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) bc[blockIdx.x] = s[0];
}

__global__ void k_scatter_alive(Part64 src, Part64 dst, int64_t n, const int64_t *boff) {
    __shared__ int32_t s[256];
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int al = (q < n && src.alive[q]) ? 1 : 0;
    s[threadIdx.x] = al;
    __syncthreads();
    // inclusive scan (Hillis-Steele) inside the block
    for (int k = 1; k < 256; k <<= 1) {
        int v = (int)threadIdx.x >= k ? s[threadIdx.x - k] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (!al) return;
    int64_t o = boff[blockIdx.x] + s[threadIdx.x] - 1;
    dst.x[o] = src.x[q];
    dst.y[o] = src.y[q];
    dst.z[o] = src.z[q];
    dst.ux[o] = src.ux[q];
    dst.uy[o] = src.uy[q];
    dst.uz[o] = src.uz[q];
    dst.w[o] = src.w[q];
    dst.alive[o] = 1;
}

int64_t compact64(Ctx &c, Part64 src, Part64 dst, int64_t n) {
    if (n <= 0) return 0;
    int nb = nblocks(n, 256);
    int32_t *bc = (int32_t *)c.i64scratch;  // reuse: nb int32 then nb+1 int64 offsets
    int64_t *boff = c.i64scratch + (nb + 1) / 2 + 1;
    hipLaunchKernelGGL(k_count_alive, dim3(nb), dim3(256), 0, c.st, src.alive, n, bc);
    std::string tmp;
    int32_t *h = (int32_t *)malloc(sizeof(int32_t) * nb);
    int64_t *ho = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
    (void)hipMemcpyAsync(h, bc, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, c.st);
    (void)hipStreamSynchronize(c.st);
    ho[0] = 0;
    for (int b = 0; b < nb; ++b) ho[b + 1] = ho[b] + h[b];
    (void)hipMemcpyAsync(boff, ho, sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, c.st);
    hipLaunchKernelGGL(k_scatter_alive, dim3(nb), dim3(256), 0, c.st, src, dst, n, boff);
    (void)hipStreamSynchronize(c.st);
    int64_t tot = ho[nb];
    free(h);
    free(ho);
    return tot;
}

}  // namespace pic
