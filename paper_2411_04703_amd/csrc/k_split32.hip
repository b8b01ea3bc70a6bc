// k_split32.hip -- FP32 split-precision path.
//
// Particles: int32 logical cell index (i + nx (j + ny l), l = window plane)
// plus FP32 offsets from the cell's centre in [-1/2, 1/2) (position = cell +
// 1/2 + offset), FP32 momenta and weight: 32 bytes each, SoA.  Offsets from
// the centre keep the representation mirror-symmetric: a carry into either
// neighbour is exact, a particle at rest at the centre has offset 0, and the
// coarsest offset step is 2^-25 of a cell.
// They are kept binned by cell tile ("bins") in two buffers; every step reads
// the current buffer and appends each surviving particle to its destination
// bin in the other buffer (wave-aggregated slot reservation), so the bins are
// exact after every step without a separate sort.  A full bin sends its
// particles to an overflow tail, processed the next step by the untiled path;
// the bins are re-laid out from the counts when the periodic host check finds
// overflow or a bin close to its capacity.
//
// Work: one (bin, chunk) item at a time per workgroup, items taken from an
// atomic counter by a persistent grid.  Per item: stage the tile's E, B (+
// halo) in LDS, gather with quadratic shapes, push (FP32; FP64 above a
// Lorentz-factor threshold), move, and deposit Esirkepov currents as 64-bit
// fixed-point integers into an LDS tile that is flushed with global 64-bit
// integer atomics.  Integer sums do not depend on their order: the current,
// and all that follows from it, is bitwise reproducible.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pic_internal.h"

namespace pic {

constexpr int ST = 512;    // threads per workgroup of the auxiliary kernels
constexpr int SST = 768;   // threads per workgroup of the step kernel (3 waves per SIMD)
constexpr int CH = 12 * SST;  // particles per work item (bins larger than this are split; measured best of 3-24 x SST)
constexpr int WT = 512;    // threads of the work-list kernels
constexpr int QPAD = 64;   // int32 stride of the slab queue counters: one 256-byte block each, apart from
                           // everything else (a counter sharing a cache line with the read-only queue
                           // bounds, or with another counter, slowed the step kernel by ~25 %)

struct Store {
    Part32 buf[2];
    int32_t *id[2];        // record mode: per-buffer particle ids (slots in the FP64 record layout), else null
    int64_t *off[2];       // nbins + 1 slot offsets of each buffer
    int32_t *cnt[2];       // per-buffer bin counts (may exceed the capacity: the excess is in the overflow tail)
    int32_t *ovf[2];       // per-buffer overflow counts
    int64_t bin_slots;     // slots of the bin region
    int64_t ovf_cap;
    int64_t n_flat;        // init only
};

struct SpeciesIO;

struct SplitState {
    Store s[2];            // 0 beam, 1 plasma
    int4 *items;
    int32_t *nitems, *next;
    int64_t items_cap;
    int64_t *scan_part;
    int32_t *tmpcnt;       // 2 x nbins
    int64_t *tmpoff;       // 2 x (nbins + 2)
    int grid;              // persistent grid of the step kernel
    void (*kern)(Params, StepCtx, const int4 *, const int32_t *, int32_t *, int, struct IOPair, FieldsT<float>,
                 long long *, long long *, long long *, int32_t *, const double *, const float *,
                 const float *);  // its instantiation (tile, deposit variant)
    int lds_bytes;
    SpeciesIO *ios;        // device descriptors: [cur 0][2], [cur 1][2], [flat init][2]
    struct IdIO *iids;     // their record-mode id arrays, same order
    double *tabA;          // undulator phase table of the step, entry l + 1 for logical plane l (nz + 2)
    float *tabC, *tabS;
    int nslab;             // work queues: slabs of whole bin layers (one per XCD when they divide evenly)
    int32_t *qnext, *qstart;  // per-slab item counters (stride QPAD); slab q's items are [qstart[q], qstart[q + 1])
    // host copies of a store's bin counts, offsets and prefix (sized once: later reads allocate nothing)
    std::vector<int32_t> hcnt;
    std::vector<int64_t> hoff, hpref;
};

static SplitState &SS(Ctx &c) { return *static_cast<SplitState *>(c.split); }

// LDS of one step-kernel workgroup: E box (T+4)^3 and B box (T+3)^3 in FP32,
// the three int64 current boxes, the undulator phase table
int split_lds_bytes(int tx, int ty, int tz) {
    int nF = (tx + 4) * (ty + 4) * (tz + 4), nE = (tx + 3) * (ty + 3) * (tz + 3);
    int nJ = (tx + 4) * (ty + 5) * (tz + 5) + (tx + 5) * (ty + 4) * (tz + 5) + (tx + 5) * (ty + 5) * (tz + 4);
    return ((3 * nF * 4 + 3 * nE * 4 + 15) & ~15) + 8 * nJ + 16 * (tz + 3);
}

static int lds_bytes_of(const Params &P) { return split_lds_bytes(P.tx, P.ty, P.tz); }

// ---------------------------------------------------------------- helpers
// The particle and bin arrays are device (global) memory: accessed through
// these casts the compiler uses global instructions with scalar bases even for
// pointers it loaded from memory.
template <typename T> __device__ inline __attribute__((address_space(1))) T *gbl(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Hides v's value from the optimiser: what is computed from it is neither folded into
// constants nor hoisted out of the work-item loop (and kept live, or spilled, across it).
__device__ inline void opaque(int &v) { asm volatile("" : "+v"(v)); }

// Reserve one slot per active lane in bin `key` of cnt; lanes with equal keys
// share one atomic.  Returns the rank within the bin (-1 for inactive lanes).
// Called by every lane of the wave.
__device__ inline int reserve_slot(bool active, int key, int32_t *cnt) {
    int lane = __lane_id();
    bool pending = active;
    int slot = -1;
    unsigned long long todo = __ballot(pending);
    while (todo) {
        int leader = __ffsll((unsigned long long)todo) - 1;
        int lkey = __shfl(key, leader);
        bool grp = pending && key == lkey;
        unsigned long long gm = __ballot(grp);
        int base = 0;
        if (lane == leader) base = atomicAdd(&cnt[lkey], __popcll(gm));
        base = __shfl(base, leader);
        if (grp) {
            slot = base + __popcll(gm & ((1ull << lane) - 1ull));
            pending = false;
        }
        todo &= ~gm;
    }
    return slot;
}

// The same reservation in two phases, so that its atomic's round trip can
// overlap other work: reserve_issue groups the lanes by key and lets each
// group's first lane add the group size (one atomic instruction for all
// groups); reserve_slot_of, called later, hands every lane its slot.
struct SlotTicket {
    int lr;    // group leader lane | rank within the group << 8
    int base;  // the group's first slot (in the leader lane)
};

__device__ inline SlotTicket reserve_issue(bool active, int key, int32_t *cnt) {
    const int lane = __lane_id();
    SlotTicket t{lane, 0};
    bool pending = active, lead = false;
    int size = 0;
    unsigned long long todo = __ballot(pending);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int lkey = __shfl(key, leader);
        const bool grp = pending && key == lkey;
        const unsigned long long gm = __ballot(grp);
        if (grp) {
            t.lr = leader | __popcll(gm & ((1ull << lane) - 1ull)) << 8;
            pending = false;
        }
        if (lane == leader) {
            lead = true;
            size = __popcll(gm);
        }
        todo &= ~gm;
    }
    if (lead) t.base = atomicAdd(&cnt[key], size);
    return t;
}

__device__ inline int reserve_slot_of(bool active, const SlotTicket &t) {
    const int base = __shfl(t.base, t.lr & 63);
    return active ? base + (t.lr >> 8) : -1;
}

struct OutStore {
    Part32 buf;
    const int64_t *off;
    int32_t *cnt;
    int32_t *ovf;
    int64_t bin_slots, ovf_cap;
};

struct SpeciesIO {
    Part32 in;
    const int64_t *in_off;
    const int32_t *in_cnt;
    const int32_t *in_ovf;
    int64_t in_ovf_start, in_ovf_cap;
    OutStore out;
};

// record mode: the id arrays of a species' input and output buffers
struct IdIO {
    const int32_t *in;
    int32_t *out;
};

// both species' descriptors as one kernel argument; the ids come after both
// SpeciesIO so that the descriptor fields the hot loop reads keep their
// argument offsets (putting them inside made the step kernel ~25 % slower)
struct IOPair {
    SpeciesIO s[2];
    IdIO id[2];
};

// append (active lanes) to bin `bin` of the output store; overflow tail when the bin is full
// (id_out: record mode, the particle id moves with it; null otherwise)
__device__ inline void store_in_bin(const OutStore &O, bool active, int r, int bin, int cell, const float o[3],
                                    const float u[3], float w, int32_t *flags, int32_t *id_out, int id);

__device__ inline void append(const OutStore &O, bool active, int bin, int cell, const float o[3], const float u[3],
                              float w, int32_t *flags, int32_t *id_out, int id) {
    const int r = reserve_slot(active, active ? bin : 0, O.cnt);
    store_in_bin(O, active, r, bin, cell, o, u, w, flags, id_out, id);
}

// particle to rank r of bin `bin` (its reserved place), or to the overflow tail when the bin is full
__device__ inline void store_in_bin(const OutStore &O, bool active, int r, int bin, int cell, const float o[3],
                                    const float u[3], float w, int32_t *flags, int32_t *id_out, int id) {
    if (!active) return;
    int64_t b0 = gbl(O.off)[bin], cap = gbl(O.off)[bin + 1] - b0;
    int64_t s;
    if (r < cap) {
        s = b0 + r;
    } else {
        int k = atomicAdd(O.ovf, 1);
        if (k >= O.ovf_cap) {
            atomicOr(flags, DFLAG_BIN_LOST);
            return;
        }
        s = O.bin_slots + k;
    }
    const Part32 &b = O.buf;
    gbl(b.cell)[s] = cell;
    gbl(b.ox)[s] = o[0];
    gbl(b.oy)[s] = o[1];
    gbl(b.oz)[s] = o[2];
    gbl(b.ux)[s] = u[0];
    gbl(b.uy)[s] = u[1];
    gbl(b.uz)[s] = u[2];
    gbl(b.w)[s] = w;
    if (id_out) gbl(id_out)[s] = id;
}

// store_in_bin with the bin's first slot b0 and capacity cap already loaded
__device__ inline void store_at(const OutStore &O, bool active, int r, int64_t b0, int64_t cap, int cell,
                                const float o[3], const float u[3], float w, int32_t *flags, int32_t *id_out, int id) {
    if (!active) return;
    int64_t s;
    if (r < cap) {
        s = b0 + r;
    } else {
        int k = atomicAdd(O.ovf, 1);
        if (k >= O.ovf_cap) {
            atomicOr(flags, DFLAG_BIN_LOST);
            return;
        }
        s = O.bin_slots + k;
    }
    const Part32 &b = O.buf;
    gbl(b.cell)[s] = cell;
    gbl(b.ox)[s] = o[0];
    gbl(b.oy)[s] = o[1];
    gbl(b.oz)[s] = o[2];
    gbl(b.ux)[s] = u[0];
    gbl(b.uy)[s] = u[1];
    gbl(b.uz)[s] = u[2];
    gbl(b.w)[s] = w;
    if (id_out) gbl(id_out)[s] = id;
}

__device__ inline int bin_of(const Params &P, int i, int j, int l) {
    return (i >> P.lgx) + P.ntx * ((j >> P.lgy) + P.nty * (l >> P.lgz));
}

// packed particle cell: i | j << cbx | l << (cbx + cby) (shifts, no divisions)
__device__ inline int pack_cell(const Params &P, int i, int j, int l) {
    return i | (j << P.cbx) | (l << (P.cbx + P.cby));
}
__device__ inline void unpack_cell(const Params &P, int cell, int &i, int &j, int &l) {
    i = cell & ((1 << P.cbx) - 1);
    j = (cell >> P.cbx) & ((1 << P.cby) - 1);
    l = cell >> (P.cbx + P.cby);
}

// periodic wrap of an index at most one period outside [0, n)
__device__ inline int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// linear index of cell (i, j, ring plane p), i and j at most one period outside the grid;
// NY1: a two-dimensional x-z grid (ny = 1, tile edge 1 in y), where every j is row 0
template <bool NY1 = false> __device__ inline int64_t near_cell(const Params &P, int i, int j, int p) {
    return (int64_t)wrap1(i, P.nx) + (int64_t)P.nx * ((NY1 ? (int64_t)0 : (int64_t)wrap1(j, P.ny)) + (int64_t)P.ny * p);
}
// the same in 32 bits: an FP32-mode grid has at most 2^31 cells (its cell index packs into 31 bits)
template <bool NY1 = false> __device__ inline uint32_t near_cell32(const Params &P, int i, int j, int p) {
    return (uint32_t)wrap1(i, P.nx) +
           (uint32_t)P.nx * ((NY1 ? 0u : (uint32_t)wrap1(j, P.ny)) + (uint32_t)P.ny * (uint32_t)p);
}


// number of valid particles of bin b in a store
__device__ inline int bin_count(const int64_t *off, const int32_t *cnt, int b) {
    int64_t cap = off[b + 1] - off[b];
    int c = cnt[b];
    return (int64_t)c < cap ? c : (int)cap;
}

// fixed-point value rint(x y) of one current contribution, rounded to nearest
// even: the FMA forms x y exactly and rounds it once together with the added
// 1.5 * 2^52, which leaves the integer in the low mantissa bits whenever
// |x y| < 2^51, which fixed_ok() has established for the whole particle
__device__ inline long long to_fixed(double x, double y) {
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    return __double_as_longlong(fma(x, y, magic)) - __double_as_longlong(magic);
}

// the same integer v with the 1.5 * 2^52 left in: the bit pattern 0x4338000000000000 + v.  The
// bias has its low 48 bits zero, so a sum of such patterns (wrapping modulo 2^64) differs from the
// sum of the v in bits 48 and up only: sign-extending its low 48 bits gives the sum of the v
// whenever that lies in [-2^47, 2^47) (the LDS current boxes, whose sums the fixed-point scale of
// the FP32 mode keeps below 2^47; see unbias48)
template <bool BIASED> __device__ inline long long to_fixed_as(double x, double y) {
    if (!BIASED) return to_fixed(x, y);
    return __double_as_longlong(fma(x, y, 6755399441055744.0));
}
__device__ inline long long unbias48(long long sum) { return (long long)((unsigned long long)sum << 16) >> 16; }

// Every Esirkepov contribution of a particle is f P_c[m] A_c[a][b] with
// |P_c| <= 1 and 0 <= A_c <= 9/16, so |f| bounds them all: one range check per
// particle (false also for a non-finite f)
__device__ inline bool fixed_ok(double f, double fscale) {
    return fabs(f) * fscale < 2251799813685248.0;  // 2^51
}

// ---------------------------------------------------------------- particle math
struct PState {
    int i, j, l;
    float o[3], u[3], w;
    int id;  // record mode only
};

__device__ inline void load_particle(const Part32 &in, int64_t s, const Params &P, PState &q, const int32_t *id_in) {
    unpack_cell(P, gbl(in.cell)[s], q.i, q.j, q.l);
    q.o[0] = gbl(in.ox)[s];
    q.o[1] = gbl(in.oy)[s];
    q.o[2] = gbl(in.oz)[s];
    q.u[0] = gbl(in.ux)[s];
    q.u[1] = gbl(in.uy)[s];
    q.u[2] = gbl(in.uz)[s];
    q.w = gbl(in.w)[s];
    q.id = id_in ? gbl(id_in)[s] : 0;
}

// undulator field at the centre of logical plane l's cells: the phase and envelope
// argument there in FP64, the in-cell phase advance k_u gR oz (oz the centred
// offset) in FP32 by angle addition
__device__ inline void ext_plane(const Params &P, int64_t k0, int l, double t, double &a_l, float &c, float &s) {
    a_l = P.gR * ((double)(k0 + l) + 0.5 - P.zoff + P.bR * t) - P.z0u;
    double sn, cs;
    sincos(P.ku * a_l, &sn, &cs);
    c = (float)cs;
    s = (float)sn;
}

// per step: ext_plane of every logical plane -1 .. nz (entry l + 1)
__global__ void k_ext_table(Params P, StepCtx S, double *tabA, float *tabC, float *tabS) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P.nz + 2) ext_plane(P, S.k0, e - 1, S.t, tabA[e], tabC[e], tabS[e]);
}

__device__ inline void ext32(const Params &P, double a_l, float cphi, float sphi, float oz, float E[3], float B[3]) {
    double a = a_l + P.gR * (double)oz;
    double env, denv;
    und_env(P, a, env, denv);
    if (env == 0.0) return;
    float sd, cd;
    sincosf((float)(P.ku * P.gR) * oz, &sd, &cd);
    float c = cphi * cd - sphi * sd, s = sphi * cd + cphi * sd;
    float b0 = (float)(P.B0 * env);
    float bx = P.und_kind == 1 ? b0 * c : 0.0f, by = b0 * s;
    float ge = (float)(P.gR * P.bR), g = (float)P.gR;
    E[0] += -ge * by;
    E[1] += ge * bx;
    B[0] += g * bx;
    B[1] += g * by;
}

// push in FP32, or FP64 above the Lorentz-factor threshold; false when non-finite.
// ion: a mobile ion (q/m = +1/M), else an electron (q/m = -1)
__device__ inline bool push32(const Params &P, bool ion, const float E[3], const float B[3], float u[3]) {
    float g2 = 1.0f + u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    float un[3];
    if (g2 > (float)(P.gthr * P.gthr)) {
        double ud[3] = {u[0], u[1], u[2]}, Ed[3] = {E[0], E[1], E[2]}, Bd[3] = {B[0], B[1], B[2]}, o[3];
        push<double>(P.pusher, ion ? P.ahi : -0.5 * P.dt, ud, Ed, Bd, o);
        for (int d = 0; d < 3; ++d) un[d] = (float)o[d];
    } else {
        push<float>(P.pusher, ion ? (float)P.ahi : -0.5f * (float)P.dt, u, E, B, un);
    }
    for (int d = 0; d < 3; ++d) u[d] = un[d];
    return isfinite(un[0]) && isfinite(un[1]) && isfinite(un[2]);
}

// Esirkepov weights of a move X0 -> X1 (coordinates relative to the particle's cell).
// The four-node window along d starts one node below the lower of the nearest
// nodes n0, n1 of X0, X1; its last node carries weight only when n0 != n1
// (bit d of cross).
struct Esk {
    int base[3], cross;
    float S0[3][4], DS[3][4];
};

__device__ inline void esk_setup(const float X0[3], const float X1[3], Esk &e) {
    e.cross = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int n0 = X0[d] >= 0.0f ? 1 : 0;
        const int n1 = (int)floorf(X1[d] + 1.0f);
        const int lo = n0 < n1 ? n0 : n1;
        e.base[d] = lo - 1;
        e.cross |= n0 != n1 ? 1 << d : 0;
        // the three nonzero weights around each nearest node, placed in the window
        float w0[3], w1[3];
        weights3<float>(X0[d] - ((float)n0 - 0.5f), w0);  // offset from the node, one rounding
        weights3<float>(X1[d] - ((float)n1 - 0.5f), w1);
        const bool h0 = n0 > lo, h1 = n1 > lo;  // window shifted by one node for this position
        float S1[4];
        e.S0[d][0] = h0 ? 0.0f : w0[0];
        e.S0[d][1] = h0 ? w0[0] : w0[1];
        e.S0[d][2] = h0 ? w0[1] : w0[2];
        e.S0[d][3] = h0 ? w0[2] : 0.0f;
        S1[0] = h1 ? 0.0f : w1[0];
        S1[1] = h1 ? w1[0] : w1[1];
        S1[2] = h1 ? w1[1] : w1[2];
        S1[3] = h1 ? w1[2] : 0.0f;
#pragma unroll
        for (int m = 0; m < 4; ++m) e.DS[d][m] = S1[m] - e.S0[d][m];
    }
}

// Esirkepov contributions: fn(c, m, a, b, J) with J the 64-bit fixed-point
// value of the contribution at node offsets base_c + m along c and base_a + a,
// base_b + b along the other two axes a, b in cyclic order (m, a, b are
// compile-time constants once the loops are unrolled, so the callers' LDS
// addresses are one per-particle base plus an immediate offset).
// Per component c the current factorises:
//   J_c(m, a, b) = f P_c[m] A_c[a][b],  P_c[m] = sum_{m' <= m} DS_c[m'],
//   A_c[a][b] = S0_a (S0_b + DS_b / 2) + DS_a (S0_b / 2 + DS_b / 3)
//             = (S0_a + DS_a / 2) S0_b + (S0_a / 2 + DS_a / 3) DS_b,
// and P_c[2] = -DS_c[3] (the DS sum to zero), exactly zero without a crossing.
// A_c is evaluated as the mean of its two factorised forms, so that it is the
// same FP32 number with the axes a and b exchanged: the transverse currents J_x
// (a, b = y, z) and J_y (a, b = z, x) then round alike, and an FP32 run keeps
// the x-y mirror symmetry of the FP64 scheme (with one form only, J_x rounded
// differently from J_y and the beam's sigma_x drifted from sigma_y by 1e-3 over
// a 1000-step plasma run).  f = w / dt is formed in FP64; f P_c[m] 2^fs is one
// FP64 product, and each value converted is that product times A_c rounded
// once to the fixed point (BIASED: left biased, see to_fixed_as).
// DEP 0 visits nonzero contributions only (one branch each); DEP 1 visits all
// 48 of a component that moves along its axis; DEP 2 leaves out the window's
// last node along an axis (m = 2, a = 3 or b = 3) when no lane of the wave
// crosses there (wave-uniform branches).  The values visited differ only by
// zeros, so the integer current sums are the same.
template <int C, int DEP, bool BIASED, typename F>
__device__ inline void esk_component(const Esk &e, double f, double fscale, F &&fn) {
    constexpr int CA = C == 2 ? 0 : C + 1, CB = C == 0 ? 2 : C - 1;
    float Pm[3];
    Pm[0] = e.DS[C][0];
    Pm[1] = Pm[0] + e.DS[C][1];
    Pm[2] = -e.DS[C][3];
    if (DEP != 0 && Pm[0] == 0.0f && Pm[1] == 0.0f && Pm[2] == 0.0f) return;
    const double fs = fscale * f;
    double Pd[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) Pd[m] = (double)Pm[m] * fs;
    // u_d = S0_d + DS_d / 2, v_d = S0_d / 2 + DS_d / 3 along both cross axes
    float ub[4], vb[4], ua[4], va[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        ub[b] = fmaf(0.5f, e.DS[CB][b], e.S0[CB][b]);
        vb[b] = fmaf(1.0f / 3.0f, e.DS[CB][b], 0.5f * e.S0[CB][b]);
        ua[b] = fmaf(0.5f, e.DS[CA][b], e.S0[CA][b]);
        va[b] = fmaf(1.0f / 3.0f, e.DS[CA][b], 0.5f * e.S0[CA][b]);
    }
    // exchanging a and b swaps the two fmaf terms, whose sum is then the same number
    auto Aab = [&](int a, int b) {
        return 0.5f * (fmaf(e.S0[CA][a], ub[b], e.DS[CA][a] * vb[b]) + fmaf(ua[a], e.S0[CB][b], va[a] * e.DS[CB][b]));
    };
    if (DEP == 2) {
        const bool m2 = __any(e.cross & (1 << C)), a3 = __any(e.cross & (1 << CA)), b3 = __any(e.cross & (1 << CB));
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if (a == 3 && !a3) break;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (b == 3 && !b3) break;
                const double A = (double)Aab(a, b);
                fn(C, 0, a, b, to_fixed_as<BIASED>(A, Pd[0]));
                fn(C, 1, a, b, to_fixed_as<BIASED>(A, Pd[1]));
                if (m2) fn(C, 2, a, b, to_fixed_as<BIASED>(A, Pd[2]));
            }
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float A = Aab(a, b);
            if (DEP == 0 && A == 0.0f) continue;
            const double Ad = (double)A;
#pragma unroll
            for (int m = 0; m < 3; ++m)
                if (DEP != 0 || Pm[m] != 0.0f) fn(C, m, a, b, to_fixed_as<BIASED>(Ad, Pd[m]));
        }
}

template <int DEP, bool BIASED = false, typename F>
__device__ inline void esk_visit(const Esk &e, double f, double fscale, F &&fn) {
    esk_component<0, DEP, BIASED>(e, f, fscale, fn);
    __builtin_amdgcn_sched_barrier(0);
    esk_component<1, DEP, BIASED>(e, f, fscale, fn);
    __builtin_amdgcn_sched_barrier(0);
    esk_component<2, DEP, BIASED>(e, f, fscale, fn);
}

// carry new offsets into the cell, apply the window shift; false if the particle left the band.
// Offsets are taken from the cell's centre, in [-1/2, 1/2); a move is less than a cell, so a
// new offset lies in [-3/2, 3/2) and the carry o -+ 1 is exact either way (Sterbenz).
__device__ inline bool renormalise(const Params &P, const StepCtx &S, PState &q) {
    int dc[3];
    for (int d = 0; d < 3; ++d) {
        dc[d] = 0;
        if (q.o[d] >= 0.5f) {
            q.o[d] -= 1.0f;
            dc[d] = 1;
        } else if (q.o[d] < -0.5f) {
            q.o[d] += 1.0f;
            dc[d] = -1;
        }
    }
    q.i += dc[0];
    if (q.i < 0) q.i += P.nx;
    if (q.i >= P.nx) q.i -= P.nx;
    q.j += dc[1];
    if (q.j < 0) q.j += P.ny;
    if (q.j >= P.ny) q.j -= P.ny;
    q.l += dc[2] - S.shift;
    return q.l >= 3 && q.l < P.nz - 4;
}

// ---------------------------------------------------------------- shared per-particle arithmetic
// This file is compiled without floating-point contraction: the tiled (LDS)
// and the untiled (global) path run the very same operations in the same
// order, so a particle's update does not depend on which path handled it --
// which in turn depends on bin occupancy and atomic order.  FMAs are written
// out explicitly where wanted.

// field value accessors: staged LDS box (tiled) or ring-buffered global arrays (untiled)
// The B update of one node from E at the node and its +x, +y, +z neighbours
// (strides sx, sy, sz): dB = -h curl E, Bx and By untouched on the last
// logical plane.  The tiled and the untiled path both call this, so B^n is the
// same wherever a particle is handled.
__device__ inline void half_curl_b(const float *ex, const float *ey, const float *ez, int64_t sx, int64_t sy,
                                   int64_t sz, bool last_plane, float h, float dB[3]) {
    const float x0 = ex[0], y0 = ey[0], z0 = ez[0];
    dB[0] = last_plane ? 0.0f : -(h * ((ez[sy] - z0) - (ey[sz] - y0)));
    dB[1] = last_plane ? 0.0f : -(h * ((ex[sz] - x0) - (ez[sx] - z0)));
    dB[2] = -(h * ((ey[sx] - y0) - (ex[sy] - x0)));
}

struct GlobalField {
    const Params *P;
    const float *const *F;  // E0 E1 E2 B0 B1 B2 (B at n - 1/2)
    int i0, j0, l0, k0r;    // cell of the particle (indices relative to it)
    float hb;               // dt / 2
    __device__ float e(int comp, int i, int j, int l) const {
        return F[comp][cell_index(*P, i, j, ring_plane(l, k0r, P->nz))];
    }
    __device__ float at(int comp, int x, int y, int z) const {
        const int i = i0 + x, j = j0 + y, l = l0 + z;
        if (comp < 3) return e(comp, i, j, l);
        // B^n from B^(n-1/2) and E^n, exactly as the tiled staging forms it
        float ex[2][2][2], ey[2][2][2], ez[2][2][2];  // [dz][dy][dx], only the needed corners filled
        ex[0][0][0] = e(0, i, j, l);
        ey[0][0][0] = e(1, i, j, l);
        ez[0][0][0] = e(2, i, j, l);
        ex[1][0][0] = e(0, i, j, l + 1);
        ex[0][1][0] = e(0, i, j + 1, l);
        ey[1][0][0] = e(1, i, j, l + 1);
        ey[0][0][1] = e(1, i + 1, j, l);
        ez[0][1][0] = e(2, i, j + 1, l);
        ez[0][0][1] = e(2, i + 1, j, l);
        float dB[3];
        half_curl_b(&ex[0][0][0], &ey[0][0][0], &ez[0][0][0], 1, 2, 4, l == P->nz - 1, hb, dB);
        return e(comp, i, j, l) + dB[comp - 3];
    }
    struct Plane {
        const GlobalField *g;
        int comp, x, y, z;
        __device__ float operator()(int a, int b) const { return g->at(comp, x + a, y + b, z); }
    };
    struct Node {
        const GlobalField *g;
        int comp, x, y, z;
        __device__ Plane plane(int c) const { return Plane{g, comp, x, y, z + c}; }
    };
    __device__ Node node(int comp, int x, int y, int z) const { return Node{this, comp, x, y, z}; }
};

// six Yee components with quadratic shapes; (x0, y0, z0) = cell relative to the accessor's origin.
// Per component the 27-node sum is taken as nested one-dimensional sums: along x for each of the
// nine rows, along y for each of the three planes, then along z.  Both accessors (the LDS box of
// the tiled path and the global arrays of the untiled one) see the same operations in the same order.
template <class FA> __device__ inline void gather6(const FA &fa, const float o[3], int x0, int y0, int z0, float EB[6]) {
    float wI[3][3], wH[3][3];
    int bI[3], bH[3];
    const int rel[3] = {x0, y0, z0};
    for (int d = 0; d < 3; ++d) {
        int nn = o[d] >= 0.0f ? 1 : 0;                        // nearest integer node: cell + nn
        weights3<float>(o[d] - ((float)nn - 0.5f), wI[d]);      // offset from it, one rounding
        weights3<float>(o[d], wH[d]);                           // the cell's centre is a half node
        bI[d] = rel[d] + nn - 1;  // first integer node
        bH[d] = rel[d] - 1;       // first half node
    }
#pragma unroll
    for (int comp = 0; comp < 6; ++comp) {
        const int sx = comp == 0 || comp == 4 || comp == 5, sy = comp == 1 || comp == 3 || comp == 5,
                  sz = comp == 2 || comp == 3 || comp == 4;
        const float *wx = sx ? wH[0] : wI[0], *wy = sy ? wH[1] : wI[1], *wz = sz ? wH[2] : wI[2];
        const int bx = sx ? bH[0] : bI[0], by = sy ? bH[1] : bI[1], bz = sz ? bH[2] : bI[2];
        const auto box = fa.node(comp, bx, by, bz);  // plane c's values are box.plane(c)(a, b), a, b in 0..2
        float pz[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const auto pl = box.plane(c);
            float py[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) py[b] = fmaf(wx[2], pl(2, b), fmaf(wx[1], pl(1, b), wx[0] * pl(0, b)));
            pz[c] = fmaf(wy[2], py[2], fmaf(wy[1], py[1], wy[0] * py[0]));
        }
        EB[comp] = fmaf(wz[2], pz[2], fmaf(wz[1], pz[1], wz[0] * pz[0]));
        __builtin_amdgcn_sched_barrier(0);  // components do not interleave (register pressure)
    }
}

// external field, push, new (unwrapped) offsets X1; false when non-finite
__device__ inline bool advance(const Params &P, float EB[6], bool ext, double a_l, float cphi, float sphi, PState &q,
                               float X1[3]) {
    float E[3] = {EB[0], EB[1], EB[2]}, B[3] = {EB[3], EB[4], EB[5]};
    if (ext) ext32(P, a_l, cphi, sphi, q.o[2], E, B);
    if (!push32(P, q.w < 0.0f, E, B, q.u)) return false;
    // 1 / gamma with the hardware reciprocal square root (1 ulp)
    const float ig = __builtin_amdgcn_rsqf(1.0f + q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]);
    const float dt = (float)P.dt;
    for (int d = 0; d < 3; ++d) X1[d] = q.o[d] + dt * (q.u[d] * ig);
    return true;
}

// ---------------------------------------------------------------- untiled (global memory) update
__device__ inline bool particle_global(const Params &P, const StepCtx &S, const float *const *F6, long long *Jx,
                                       long long *Jy, long long *Jz, PState &q, int32_t *flags) {
    if (!(q.o[0] >= -0.5f && q.o[0] < 0.5f && q.o[1] >= -0.5f && q.o[1] < 0.5f && q.o[2] >= -0.5f &&
          q.o[2] < 0.5f && q.l >= 3 && q.l < P.nz - 4)) {
        atomicOr(flags, DFLAG_NONFINITE);
        return false;
    }
    GlobalField gf{&P, F6, q.i, q.j, q.l, S.k0r, (float)(0.5 * P.dt)};
    float EB[6];
    gather6(gf, q.o, 0, 0, 0, EB);
    double a_l = 0.0;
    float cphi = 0.0f, sphi = 0.0f;
    if (P.und_kind) ext_plane(P, S.k0, q.l, S.t, a_l, cphi, sphi);
    float X1[3];
    if (!advance(P, EB, P.und_kind != 0, a_l, cphi, sphi, q, X1)) {
        atomicOr(flags, DFLAG_NONFINITE);
        return false;
    }
    Esk e;
    esk_setup(q.o, X1, e);
    long long *J[3] = {Jx, Jy, Jz};
    const double fq = (double)q.w / P.dt;
    if (!fixed_ok(fq, P.fscale)) {
        atomicOr(flags, DFLAG_FIXED_OVERFLOW);
        return false;
    }
    esk_visit<0>(e, fq, P.fscale, [&](int c, int m, int a, int b, long long iv) {
        const int ca = c == 2 ? 0 : c + 1, cb = c == 0 ? 2 : c - 1;
        int r[3];
        r[c] = e.base[c] + m;
        r[ca] = e.base[ca] + a;
        r[cb] = e.base[cb] + b;
        int p = ring_plane(q.l + r[2], S.k0r, P.nz);
        atomicAdd((unsigned long long *)&J[c][cell_index(P, q.i + r[0], q.j + r[1], p)], (unsigned long long)iv);
    });
    for (int d = 0; d < 3; ++d) q.o[d] = X1[d];
    return renormalise(P, S, q);
}

// ---------------------------------------------------------------- the step kernel
// Tile TX x TY x TZ cells (compile time, so that every LDS access of the gather
// and the deposit is one per-particle base address plus an immediate offset),
// ST threads, 2 waves per SIMD.  DEP selects the deposit variant (esk_component).
template <int TX, int TY, int TZ> struct TileGeom {
    static constexpr int EX = TX + 3, EY = TY + 3, EZ = TZ + 3, NE = EX * EY * EZ;  // B box (t0 - 1 ...)
    static constexpr int FX = TX + 4, FY = TY + 4, FZ = TZ + 4, NF = FX * FY * FZ;  // E box (t0 - 1 ...), one more
                                                                                    // node for the curl at B sites
    // current boxes (origin t0 - 2): along their own axis TX + 4, across TX + 5
    static constexpr int XX = TX + 4, XY = TY + 5, XZ = TZ + 5;
    static constexpr int YX = TX + 5, YY = TY + 4, YZ = TZ + 5;
    static constexpr int ZX = TX + 5, ZY = TY + 5, ZZ = TZ + 4;
    static constexpr int NJX = XX * XY * XZ, NJY = YX * YY * YZ, NJZ = ZX * ZY * ZZ, NJ = NJX + NJY + NJZ;
    static constexpr int NTAB = TZ + 3;
    static constexpr int EBYTES = (3 * NF * 4 + 3 * NE * 4 + 15) & ~15;
    static constexpr int LDS = EBYTES + 8 * NJ + 16 * NTAB;
};

template <class G> struct LdsBoxT {
    const float *F;  // 3 E boxes of G::NF floats, then 3 B boxes of G::NE; box index of (half-)node k
                     // (relative to t0) is k + 1
    // the 27 nodes from (x, y, z) on of one component, plane by plane: one LDS address per plane
    // (kept in its own register, so that the nine reads of a plane, paired or not, take their
    // node offsets as immediates), sy and sz compile-time once inlined (the component is)
    using LdsPtr = const __attribute__((address_space(3))) float *;
    struct Plane {
        LdsPtr p;
        int sy;
        __device__ float operator()(int a, int b) const { return p[a + sy * b]; }
    };
    struct Node {
        LdsPtr L;
        int idx, sy, sz;
        __device__ Plane plane(int c) const {
            int k = idx + sz * c;
            opaque(k);
            return Plane{L + k, sy};
        }
    };
    __device__ Node node(int comp, int x, int y, int z) const {
        const LdsPtr L = (LdsPtr)F;
        return comp < 3 ? Node{L, comp * G::NF + (x + 1) + G::FX * ((y + 1) + G::FY * (z + 1)), G::FX, G::FX * G::FY}
                        : Node{L, 3 * G::NF + (comp - 3) * G::NE + (x + 1) + G::EX * ((y + 1) + G::EY * (z + 1)),
                               G::EX, G::EX * G::EY};
    }
};

// A particle record as loaded; it is unpacked when its round starts, so that
// the loads of the next round are in flight while the current round computes.
struct PRaw {
    int cell;
    float o[3], u[3], w;
    int id;
};

__device__ inline void load_raw(const Part32 &in, int64_t s, PRaw &r, const int32_t *id_in) {
    r.cell = gbl(in.cell)[s];
    r.o[0] = gbl(in.ox)[s];
    r.o[1] = gbl(in.oy)[s];
    r.o[2] = gbl(in.oz)[s];
    r.u[0] = gbl(in.ux)[s];
    r.u[1] = gbl(in.uy)[s];
    r.u[2] = gbl(in.uz)[s];
    r.w = gbl(in.w)[s];
    r.id = id_in ? gbl(id_in)[s] : 0;
}

__device__ inline void unpack_raw(const Params &P, const PRaw &r, PState &q) {
    unpack_cell(P, r.cell, q.i, q.j, q.l);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        q.o[d] = r.o[d];
        q.u[d] = r.u[d];
    }
    q.w = r.w;
    q.id = r.id;
}

// One float from global memory straight into LDS (no register on the way):
// lane L of the wave writes dst_wave[L]; dst_wave is the same for the whole wave.
__device__ inline void lds_load(const float *src, float *dst_wave) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                     (__attribute__((address_space(3))) void *)dst_wave, 4, 0, 0);
}

// one work item as the step kernel sees it (wave-uniform values)
struct ItemT {
    int sp, bin, start, end, t0x, t0y, t0z;
    int64_t b0;
};

template <int TX, int TY, int TZ, int DEP, bool REC>
__global__ void __launch_bounds__(SST, 3) k_split_step(Params P, StepCtx S, const int4 *items, const int32_t *qstart,
                                                      int32_t *qnext, int nslab, IOPair iop, FieldsT<float> f,
                                                      long long *Jx, long long *Jy, long long *Jz, int32_t *flags,
                                                      const double *gtabA, const float *gtabC, const float *gtabS) {
    using G = TileGeom<TX, TY, TZ>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item, s_qstart[9];
    const int tid = threadIdx.x;
    if (tid <= nslab) s_qstart[tid] = qstart[tid];  // constant during the launch
    float *Fs = (float *)smem;
    float *Bs = Fs + 3 * G::NF;
    long long *Js = (long long *)(smem + G::EBYTES);
    double *tabA = (double *)(Js + G::NJ);
    float *tabC = (float *)(tabA + G::NTAB), *tabS = tabC + G::NTAB;
    const float *F6[6] = {f.E[0], f.E[1], f.E[2], f.B[0], f.B[1], f.B[2]};
    const float hb = (float)(0.5 * P.dt);
    for (int k = tid; k < G::NJ; k += SST) Js[k] = 0;  // cleared once; every flush clears what it reads
    __syncthreads();

    // Work queues: one per z slab of bins; this workgroup's XCD's slab first, then the others'
    // (work stealing).  Thread 0 keeps one claim on queue q in flight: the counter value for
    // the item after the current one, claimed when the current one starts and resolved when it
    // ends, so the atomic's round trip is hidden behind the item's work.
    int q = (int)(blockIdx.x % (unsigned)nslab), hops = 0, claim = 0;
    auto resolve = [&]() -> int {  // thread 0: the claimed item, or the next queue's, or -1
        int k = s_qstart[q] + claim;
        while (k >= s_qstart[q + 1]) {
            q = q + 1 == nslab ? 0 : q + 1;
            if (++hops >= nslab) return -1;
            k = s_qstart[q] + atomicAdd(&qnext[q * QPAD], 1);
        }
        return k;
    };
    auto decode = [&](int item) -> ItemT {
        ItemT I;
        const int4 it = items[item];
        I.sp = __builtin_amdgcn_readfirstlane(it.x);
        I.bin = __builtin_amdgcn_readfirstlane(it.y);
        I.start = __builtin_amdgcn_readfirstlane(it.z);
        const int cnt = __builtin_amdgcn_readfirstlane(it.w);
        I.end = min(cnt, I.start + CH);
        const int bin = I.bin < 0 ? 0 : I.bin;
        I.t0x = (bin % P.ntx) * TX;
        I.t0y = ((bin / P.ntx) % P.nty) * TY;
        I.t0z = (bin / (P.ntx * P.nty)) * TZ;
        I.b0 = I.bin < 0 ? 0 : gbl(iop.s[I.sp].in_off)[bin];
        return I;
    };
    // E^n and B^(n-1/2) of an item's tile (box node (a, b, c) <-> absolute node
    // (t0x - 1 + a, t0y - 1 + b, t0z - 1 + c)) and its undulator phase table, loaded straight
    // into LDS; nothing waits for them until the next barrier at the top of the item loop
    auto stage = [&](const ItemT &I) {
        // thread t owns one (x, y) column of the E box or of the B box: its global offset is
        // formed once, each plane adds a wave-uniform plane base.  The E columns take the
        // first threads, the B columns the waves after them and, for what is left, the first
        // threads again, so that in every wave the lanes that load are a prefix and lane L of
        // the wave that starts at column c0 writes column c0 + L of a plane
        constexpr int NCE = G::FX * G::FY, NCB = G::EX * G::EY, WE = (NCE + 63) & ~63;
        constexpr int NB1 = NCB < SST - WE ? NCB : SST - WE, NB2 = NCB - NB1;
        static_assert(NCE <= SST && NB2 <= SST, "one pass of columns per box");
        const int w64 = __builtin_amdgcn_readfirstlane(tid & ~63);
        const uint32_t pl = (uint32_t)P.nx * (uint32_t)P.ny;
        auto plane_of = [&](int c) {
            int l = I.t0z - 1 + c;
            l = l < 0 ? 0 : (l >= P.nz ? P.nz - 1 : l);  // outside the window: never gathered
            return pl * (uint32_t)ring_plane(l, S.k0r, P.nz);
        };
        if (tid < NCE) {
            const int b = tid / G::FX, a = tid - b * G::FX;
            const uint32_t col = near_cell32<TY == 1>(P, I.t0x - 1 + a, I.t0y - 1 + b, 0);
#pragma unroll
            for (int c = 0; c < G::FZ; ++c) {
                const uint32_t o = col + plane_of(c);
#pragma unroll
                for (int qq = 0; qq < 3; ++qq) lds_load(F6[qq] + o, Fs + qq * G::NF + c * NCE + w64);
            }
        }
        auto stage_b = [&](int u, int c0) {  // B column u; the wave's first lane has column c0
            const int b = u / G::EX, a = u - b * G::EX;
            const uint32_t col = near_cell32<TY == 1>(P, I.t0x - 1 + a, I.t0y - 1 + b, 0);
#pragma unroll
            for (int c = 0; c < G::EZ; ++c) {
                const uint32_t o = col + plane_of(c);
#pragma unroll
                for (int qq = 0; qq < 3; ++qq) lds_load(F6[3 + qq] + o, Bs + qq * G::NE + c * NCB + c0);
            }
        };
        if (tid >= WE && tid - WE < NB1) stage_b(tid - WE, w64 - WE);
        if (NB2 > 0 && tid < NB2) stage_b(NB1 + tid, NB1 + w64);
        static_assert(G::NTAB <= SST, "one table entry per thread");
        if (P.und_kind && tid < G::NTAB) {  // planes t0z - 1 ...: table entries t0z ...
            int k = tid;
            opaque(k);
            tabA[k] = gtabA[I.t0z + k];
            tabC[k] = gtabC[I.t0z + k];
            tabS[k] = gtabS[I.t0z + k];
        }
    };

    if (tid == 0) {
        claim = atomicAdd(&qnext[q * QPAD], 1);
        const int first = resolve();
        s_item = first;
    }
    __syncthreads();
    int cur = __builtin_amdgcn_readfirstlane(s_item);
    ItemT I{};
    PRaw nx;  // this thread's particle of the next round
    if (cur >= 0) {
        I = decode(cur);
        if (I.bin >= 0) {
            stage(I);
            if (I.start + tid < I.end) load_raw(iop.s[I.sp].in, I.b0 + I.start + tid, nx, REC ? iop.id[I.sp].in : nullptr);
        }
    }

    while (cur >= 0) {
        // the staged boxes have landed, and the previous item's flush has cleared the current boxes
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const SpeciesIO &IO = iop.s[I.sp];
        if (I.bin >= 0) {  // overflow tails (bin < 0) are k_split_overflow's
            // B^n = B^(n-1/2) - (dt/2) curl E^n on the B box (the first half of the Yee B update)
            for (int k = tid; k < G::NE; k += SST) {
                const int bc = k / G::EX, a = k - bc * G::EX, c = bc / G::EY, b = bc - c * G::EY;
                const float *ex = Fs + a + G::FX * (b + G::FY * c), *ey = ex + G::NF, *ez = ey + G::NF;
                float B3[3];
                half_curl_b(ex, ey, ez, 1, G::FX, G::FX * G::FY, I.t0z - 1 + c == P.nz - 1, hb, B3);
                Bs[k] += B3[0];
                Bs[G::NE + k] += B3[1];
                Bs[2 * G::NE + k] += B3[2];
            }
        }
        __syncthreads();  // (also publishes s_item)
        // the item after this one, resolved by thread 0 at the top of this one: its descriptor
        // loads are in flight during the rounds
        if (I.bin >= 0) {
            const LdsBoxT<G> box{Fs};
            for (int base = I.start; base < I.end; base += SST) {
                // pushed: advanced (deposits its current); act: still in the band (appended)
                bool act = base + tid < I.end, pushed = false;
                PState q;
                float X0[3] = {0.0f, 0.0f, 0.0f}, X1[3] = {0.0f, 0.0f, 0.0f};
                double fq = 0.0;
                int li = 0, lj = 0, lk = 0;
                if (act) {
                    unpack_raw(P, nx, q);
                    li = q.i - I.t0x;
                    lj = q.j - I.t0y;
                    lk = q.l - I.t0z;
                    const bool inside = li >= 0 && li < TX && lj >= 0 && lj < TY && lk >= 0 && lk < TZ &&
                                        q.o[0] >= -0.5f && q.o[0] < 0.5f && q.o[1] >= -0.5f &&
                                        q.o[1] < 0.5f && q.o[2] >= -0.5f && q.o[2] < 0.5f;
                    if (!inside) {
                        // cannot happen: every binned particle was appended to the bin of its cell
                        atomicOr(flags, DFLAG_BIN_LOST);
                        act = false;
                    } else {
                        float EB[6];
                        gather6(box, q.o, li, lj, lk, EB);
                        if (!advance(P, EB, P.und_kind != 0, tabA[lk + 1], tabC[lk + 1], tabS[lk + 1], q, X1)) {
                            atomicOr(flags, DFLAG_NONFINITE);
                            act = false;
                        } else {
                            fq = (double)q.w / P.dt;
                            if (!fixed_ok(fq, P.fscale)) {
                                atomicOr(flags, DFLAG_FIXED_OVERFLOW);
                                fq = 0.0;
                            }
                            for (int d = 0; d < 3; ++d) {
                                X0[d] = q.o[d];
                                q.o[d] = X1[d];
                            }
                            pushed = true;
                            act = renormalise(P, S, q);
                        }
                    }
                }
                // destination slot: the reservation's atomic is in flight during the deposit,
                // and so are the loads of the next round's particles
                const int bin = act ? bin_of(P, q.i, q.j, q.l) : 0;
                const SlotTicket tk = reserve_issue(act, bin, IO.out.cnt);
                const int64_t ob0 = gbl(IO.out.off)[bin], ocap = gbl(IO.out.off)[bin + 1] - ob0;
                {  // every lane loads (a clamped index past the item's end), so the waits stay static
                    const int nb = min(base + SST + tid, I.end - 1);
                    load_raw(IO.in, I.b0 + nb, nx, REC ? iop.id[I.sp].in : nullptr);
                }
                if (pushed) {
                    Esk e;
                    esk_setup(X0, X1, e);
                    // LDS current boxes, origin t0 - 2: box index of offset r is l + r + 2;
                    // one base index per component, the node offsets are immediates; the values
                    // are added biased (to_fixed_as) and unbiased when the flush reads the sums
                    const int bx = li + e.base[0] + 2, by = lj + e.base[1] + 2, bz = lk + e.base[2] + 2;
                    const int jb[3] = {bx + G::XX * (by + G::XY * bz), G::NJX + bx + G::YX * (by + G::YY * bz),
                                       G::NJX + G::NJY + bx + G::ZX * (by + G::ZY * bz)};
                    esk_visit<DEP, true>(e, fq, P.fscale, [&](int c, int m, int a, int b, long long iv) {
                        int off;
                        if (c == 0)  // (m, a, b) along (x, y, z)
                            off = m + G::XX * (a + G::XY * b);
                        else if (c == 1)  // (y, z, x)
                            off = b + G::YX * (m + G::YY * a);
                        else  // (z, x, y)
                            off = a + G::ZX * (b + G::ZY * m);
                        atomicAdd((unsigned long long *)&Js[jb[c] + off], (unsigned long long)iv);
                    });
                }
                store_at(IO.out, act, reserve_slot_of(act, tk), ob0, ocap, act ? pack_cell(P, q.i, q.j, q.l) : 0,
                         q.o, q.u, q.w, flags, REC ? iop.id[I.sp].out : nullptr, q.id);
            }
        }
        if (tid == 0) {
            claim = atomicAdd(&qnext[q * QPAD], 1);
            s_item = resolve();
        }
        // every deposit of this item is in the current boxes
        __syncthreads();
        const int next = __builtin_amdgcn_readfirstlane(s_item);
        ItemT N{};
        if (next >= 0) N = decode(next);
        const ItemT C = I;
        // the next item's fields and first particles are on their way during this item's flush
        if (next >= 0) {
            I = N;
            if (I.bin >= 0) {
                stage(I);
                if (I.start + tid < I.end)
                    load_raw(iop.s[I.sp].in, I.b0 + I.start + tid, nx, REC ? iop.id[I.sp].in : nullptr);
            }
        }
        // flush nonzero LDS currents (unbiased) with global 64-bit integer atomics, clearing the boxes.
        // Thread t takes columns t and t + SST of the three boxes' (x, y) footprints and walks
        // their planes: a column's global offset is formed once, a plane's is wave-uniform.
        if (C.bin >= 0) {
            constexpr int CX = G::XX * G::XY, CY = G::YX * G::YY, CZ = G::ZX * G::ZY, NCOL = CX + CY + CZ;
            constexpr int NPMAX = G::XZ > G::ZZ ? G::XZ : G::ZZ;
            static_assert(NCOL <= 2 * SST && G::XZ == G::YZ, "two columns per thread");
            const uint32_t pl = (uint32_t)P.nx * (uint32_t)P.ny;
#pragma unroll 1
            for (int r = 0; r < 2; ++r) {
                const int g = tid + r * SST;
                if (g < NCOL) {
                    int x, y, np, stride, lb;
                    long long *J;
                    if (g < CX) {
                        y = g / G::XX;
                        x = g - y * G::XX;
                        np = G::XZ, stride = CX, lb = g, J = Jx;
                    } else if (g < CX + CY) {
                        const int h = g - CX;
                        y = h / G::YX;
                        x = h - y * G::YX;
                        np = G::YZ, stride = CY, lb = G::NJX + h, J = Jy;
                    } else {
                        const int h = g - CX - CY;
                        y = h / G::ZX;
                        x = h - y * G::ZX;
                        np = G::ZZ, stride = CZ, lb = G::NJX + G::NJY + h, J = Jz;
                    }
                    const uint32_t col = near_cell32<TY == 1>(P, C.t0x - 2 + x, C.t0y - 2 + y, 0);
#pragma unroll 1
                    for (int z = 0; z < NPMAX; ++z) {
                        if (z >= np) continue;
                        const long long sum = Js[lb + z * stride];
                        if (sum == 0) continue;
                        Js[lb + z * stride] = 0;
                        const long long v = unbias48(sum);
                        if (v == 0) continue;
                        const int l = C.t0z - 2 + z;
                        if (l < 0 || l >= P.nz) continue;  // cannot hold a contribution: particles stay in [3, nz-4)
                        const uint32_t o = col + pl * (uint32_t)ring_plane(l, S.k0r, P.nz);
                        atomicAdd((unsigned long long *)&J[o], (unsigned long long)v);
                    }
                }
            }
        }
        cur = next;
    }
}

// the tiles the step kernel is instantiated for
#define PIC_SPLIT_TILES(X) X(8, 8, 4) X(8, 8, 8) X(8, 8, 16) X(16, 8, 4) X(16, 16, 4) X(16, 8, 8) X(16, 1, 16)

using StepKernel = void (*)(Params, StepCtx, const int4 *, const int32_t *, int32_t *, int, IOPair,
                            FieldsT<float>, long long *, long long *, long long *, int32_t *, const double *,
                            const float *, const float *);

// record mode has one instantiation per tile (the wave-pruned deposit: every
// variant gives the same integer currents)
static StepKernel step_kernel(int tx, int ty, int tz, int dep, bool rec) {
#define PIC_PICK(a, b, c)                                                                              \
    if (tx == a && ty == b && tz == c)                                                                 \
        return rec ? k_split_step<a, b, c, 2, true>                                                    \
                   : (dep == 0 ? k_split_step<a, b, c, 0, false>                                       \
                               : (dep == 1 ? k_split_step<a, b, c, 1, false> : k_split_step<a, b, c, 2, false>));
    PIC_SPLIT_TILES(PIC_PICK)
#undef PIC_PICK
    return nullptr;
}

bool split_tile_supported(int tx, int ty, int tz) { return step_kernel(tx, ty, tz, 0, false) != nullptr; }

// overflow tails of the previous step: untiled path, one particle per thread,
// persistent grid over the tail lengths read on the device
__global__ void __launch_bounds__(256) k_split_overflow(Params P, StepCtx S, const SpeciesIO *ios, const IdIO *iids,
                                                        FieldsT<float> f, long long *Jx, long long *Jy, long long *Jz,
                                                        int32_t *flags) {
    const float *F6[6] = {f.E[0], f.E[1], f.E[2], f.B[0], f.B[1], f.B[2]};
    for (int sp = 0; sp < 2; ++sp) {
        const SpeciesIO &IO = ios[sp];
        const int n = (int)min((int64_t)*IO.in_ovf, IO.in_ovf_cap);
        for (int base = blockIdx.x * 256; base < n; base += gridDim.x * 256) {
            int k = base + threadIdx.x;
            bool act = k < n;
            PState q;
            if (act) {
                load_particle(IO.in, IO.in_ovf_start + k, P, q, iids[sp].in);
                act = particle_global(P, S, F6, Jx, Jy, Jz, q, flags);
            }
            append(IO.out, act, act ? bin_of(P, q.i, q.j, q.l) : 0, act ? pack_cell(P, q.i, q.j, q.l) : 0, q.o,
                   q.u, q.w, flags, iids[sp].out, q.id);
        }
    }
}

// ---------------------------------------------------------------- rebin (no physics)
__global__ void __launch_bounds__(ST) k_rebin(Params P, const int4 *items, const int32_t *nitems, int32_t *next,
                                              const SpeciesIO *ios, const IdIO *iids, int32_t *flags) {
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int total = *nitems;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(next, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int4 it = items[item];
        const SpeciesIO &IO = ios[it.x];
        const int bin = it.y, start = it.z, cnt = it.w;
        const int64_t b0 = bin < 0 ? IO.in_ovf_start : IO.in_off[bin];
        const int end = min(cnt, start + CH);
        for (int base = start; base < end; base += ST) {
            int k = base + tid;
            bool act = k < end;
            PState q;
            if (act) load_particle(IO.in, b0 + k, P, q, iids[it.x].in);
            append(IO.out, act, act ? bin_of(P, q.i, q.j, q.l) : 0, act ? pack_cell(P, q.i, q.j, q.l) : 0, q.o,
                   q.u, q.w, flags, iids[it.x].out, q.id);
        }
    }
}

// ---------------------------------------------------------------- work list
// items (species, bin, first particle, bin count) for every CH-chunk of every
// non-empty bin of the input buffer, then the overflow tails (bin = -1).
// Three kernels: per-block item counts, single-thread scan of the block
// totals, per-block writes.  They also clear the output counters.
__device__ inline int items_of(int n) { return (n + CH - 1) / CH; }

// Work-list entry e (0 <= e < 2 nbins) in slab-major order: the bins form
// nslab slabs of whole z layers (bins are numbered z-major), and within a slab
// the beam's bins come before the plasma's.
__device__ inline void entry_of(int e, int nbins, int nslab, int &sp, int &bin) {
    const int bps = nbins / nslab, s = e / (2 * bps), r = e - s * 2 * bps;
    sp = r >= bps ? 1 : 0;
    bin = s * bps + (r - sp * bps);
}

__global__ void k_wl_count(const int64_t *off0, const int32_t *cnt0, const int64_t *off1, const int32_t *cnt1,
                           int nbins, int nslab, int64_t *part) {
    __shared__ int64_t s[WT];
    int e = blockIdx.x * WT + threadIdx.x;
    int v = 0;
    if (e < 2 * nbins) {
        int sp, bin;
        entry_of(e, nbins, nslab, sp, bin);
        v = items_of(sp ? bin_count(off1, cnt1, bin) : bin_count(off0, cnt0, bin));
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = WT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_wl_scan(int64_t *part, int nblk, const int32_t *ovf0, int64_t ocap0, const int32_t *ovf1,
                          int64_t ocap1, int32_t *nitems, int32_t *next, int4 *items, int64_t items_cap,
                          int32_t *clr0, int32_t *clr1, int32_t *qnext, int32_t *qstart, int nslab) {
    if (threadIdx.x != 0) return;
    int64_t acc = 0;
    for (int b = 0; b < nblk; ++b) {
        int64_t v = part[b];
        part[b] = acc;
        acc += v;
    }
    for (int q = 0; q < nslab; ++q) qnext[q * QPAD] = 0;
    qstart[nslab] = (int32_t)min(acc, items_cap);  // the slab queues end before the overflow items
    int o0 = (int)min((int64_t)*ovf0, ocap0), o1 = (int)min((int64_t)*ovf1, ocap1);
    for (int k = 0; k < items_of(o0) && acc < items_cap; ++k) items[acc++] = make_int4(0, -1, k * CH, o0);
    for (int k = 0; k < items_of(o1) && acc < items_cap; ++k) items[acc++] = make_int4(1, -1, k * CH, o1);
    *nitems = (int32_t)min(acc, items_cap);
    *next = 0;
    *clr0 = 0;
    *clr1 = 0;
}

__global__ void k_wl_write(const int64_t *off0, const int32_t *cnt0, const int64_t *off1, const int32_t *cnt1,
                           int nbins, int nslab, const int64_t *part, int4 *items, int64_t items_cap, int32_t *zero0,
                           int32_t *zero1, int32_t *qstart) {
    __shared__ int64_t s[WT];
    int e = blockIdx.x * WT + threadIdx.x;
    int v = 0, c = 0, sp = 0, bin = 0;
    if (e < 2 * nbins) {
        entry_of(e, nbins, nslab, sp, bin);
        c = sp ? bin_count(off1, cnt1, bin) : bin_count(off0, cnt0, bin);
    }
    v = items_of(c);
    s[threadIdx.x] = v;
    __syncthreads();
    for (int k = 1; k < WT; k <<= 1) {  // inclusive scan in the block
        int64_t t = (int)threadIdx.x >= k ? s[threadIdx.x - k] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t o = part[blockIdx.x] + s[threadIdx.x] - v;
    for (int k = 0; k < v; ++k)
        if (o + k < items_cap) items[o + k] = make_int4(sp, bin, k * CH, c);
    if (e < 2 * nbins) {
        if (sp) zero1[bin] = 0;
        else zero0[bin] = 0;
        const int bps = nbins / nslab;
        if (e % (2 * bps) == 0) qstart[e / (2 * bps)] = (int32_t)min(o, items_cap);  // first entry of a slab
    }
}

// in_cap0/1: how many overflow-tail particles the input buffer can hold
static void build_worklist(Ctx &c, int cur, int64_t in_cap0, int64_t in_cap1) {
    SplitState &X = SS(c);
    int nb = c.P.nbins;
    int nblk = nblocks(2 * (int64_t)nb, WT);
    int o = cur ^ 1;
    Store &b = X.s[0], &p = X.s[1];
    hipLaunchKernelGGL(k_wl_count, dim3(nblk), dim3(WT), 0, c.st, b.off[cur], b.cnt[cur], p.off[cur], p.cnt[cur], nb,
                       X.nslab, X.scan_part);
    hipLaunchKernelGGL(k_wl_scan, dim3(1), dim3(64), 0, c.st, X.scan_part, nblk, b.ovf[cur], in_cap0, p.ovf[cur],
                       in_cap1, X.nitems, X.next, X.items, X.items_cap, b.ovf[o], p.ovf[o], X.qnext, X.qstart, X.nslab);
    hipLaunchKernelGGL(k_wl_write, dim3(nblk), dim3(WT), 0, c.st, b.off[cur], b.cnt[cur], p.off[cur], p.cnt[cur], nb,
                       X.nslab, X.scan_part, X.items, X.items_cap, b.cnt[o], p.cnt[o], X.qstart);
}

static IdIO species_ids(Ctx &c, int sp, int cur) {
    Store &s = SS(c).s[sp];
    return IdIO{s.id[cur], s.id[cur ^ 1]};
}

static SpeciesIO species_io(Ctx &c, int sp, int cur, int64_t in_ovf_start) {
    Store &s = SS(c).s[sp];
    int o = cur ^ 1;
    SpeciesIO io;
    io.in = s.buf[cur];
    io.in_off = s.off[cur];
    io.in_cnt = s.cnt[cur];
    io.in_ovf = s.ovf[cur];
    io.in_ovf_start = in_ovf_start;
    io.in_ovf_cap = in_ovf_start == 0 ? s.bin_slots + s.ovf_cap : s.ovf_cap;
    io.out.buf = s.buf[o];
    io.out.off = s.off[o];
    io.out.cnt = s.cnt[o];
    io.out.ovf = s.ovf[o];
    io.out.bin_slots = s.bin_slots;
    io.out.ovf_cap = s.ovf_cap;
    return io;
}

// ---------------------------------------------------------------- setup
// one particle buffer: 8 arrays of 4 B per slot, plus the id array in record mode
static uint64_t slot_bytes(const Ctx &c) { return c.record ? 36 : 32; }

static Part32 carve32(char *base, int64_t slots) {
    Part32 p;
    uint64_t n = (uint64_t)slots;
    p.cell = (int32_t *)base;
    float *f = (float *)(base + 4 * n);
    p.ox = f;
    p.oy = f + n;
    p.oz = f + 2 * n;
    p.ux = f + 3 * n;
    p.uy = f + 4 * n;
    p.uz = f + 5 * n;
    p.w = f + 6 * n;
    return p;
}

void split_setup(Ctx &c) {
    SplitState *X = new SplitState();
    c.split = X;
    X->hcnt.resize(c.P.nbins);
    X->hoff.resize(c.P.nbins + 1);
    X->hpref.resize(c.P.nbins + 2);
    const Params &P = c.P;
    char *A = c.arena;
    int64_t nb = P.nbins;
    for (int sp = 0; sp < 2; ++sp) {
        Store &s = X->s[sp];
        s.bin_slots = sp ? c.split_slots_p : c.split_slots_b;
        s.ovf_cap = sp ? c.ovf_cap_p : c.ovf_cap_b;
        int64_t slots = s.bin_slots + s.ovf_cap;
        char *b = A + (sp ? c.split_off_p : c.split_off_b);
        for (int k = 0; k < 2; ++k) {
            char *bk = b + k * slot_bytes(c) * (uint64_t)slots;
            s.buf[k] = carve32(bk, slots);
            s.id[k] = c.record ? (int32_t *)(bk + 32 * (uint64_t)slots) : nullptr;
        }
    }
    char *bins = A + c.split_off_bins;
    int64_t *offs = (int64_t *)bins;
    int32_t *cnts = (int32_t *)(offs + 4 * (nb + 1));
    int32_t *ovfs = cnts + 4 * nb;
    for (int sp = 0; sp < 2; ++sp)
        for (int k = 0; k < 2; ++k) {
            X->s[sp].off[k] = offs + (2 * sp + k) * (nb + 1);
            X->s[sp].cnt[k] = cnts + (2 * sp + k) * nb;
            X->s[sp].ovf[k] = ovfs + (2 * sp + k);
        }
    X->nitems = ovfs + 4;
    X->next = ovfs + 5;
    char *wl = A + c.split_off_wl;
    X->items_cap = c.split_items_cap;
    X->items = (int4 *)wl;
    X->scan_part = (int64_t *)(wl + 16 * (uint64_t)X->items_cap);
    X->tmpcnt = (int32_t *)(X->scan_part + nblocks(2 * nb, WT) + 8);
    X->tmpoff = (int64_t *)(X->tmpcnt + 2 * nb + 8);
    X->ios = (SpeciesIO *)(((uintptr_t)(X->tmpoff + nb + 8) + 15) & ~(uintptr_t)15);
    X->iids = (IdIO *)(X->ios + 6);
    X->tabA = (double *)(((uintptr_t)(X->iids + 6) + 15) & ~(uintptr_t)15);
    X->tabC = (float *)(X->tabA + P.nz + 2);
    X->tabS = X->tabC + P.nz + 2;
    X->qnext = (int32_t *)(((uintptr_t)(X->tabS + P.nz + 2) + 255) & ~(uintptr_t)255);
    X->qstart = X->qnext + 8 * QPAD;  // its own 256-byte block
    X->nslab = P.ntz % 8 == 0 ? 8 : 1;  // workgroups are dispatched round-robin over the 8 XCDs
    X->lds_bytes = lds_bytes_of(P);
    // deposit: option 0 = wave-pruned windows, 1 = whole components, 2 = zero-skipping
    X->kern = step_kernel(P.tx, P.ty, P.tz, c.opt.variant == 0 ? 2 : (c.opt.variant == 1 ? 1 : 0), c.record != 0);
    const void *kern = (const void *)X->kern;
    (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, X->lds_bytes);
    // persistent grid: resident workgroups per CU as registers and LDS allow, or as requested
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, SST, X->lds_bytes) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (c.opt.wg_per_cu > 0) per_cu = std::min(per_cu, c.opt.wg_per_cu);
    int dev = 0, ncu = 256;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) ncu = prop.multiProcessorCount;
    X->grid = ncu * per_cu;
    (void)hipMemsetAsync(bins, 0, c.split_bins_bytes, c.st);
    // species descriptors (pointers only; their targets change, they do not)
    SpeciesIO h[6] = {species_io(c, 0, 0, X->s[0].bin_slots), species_io(c, 1, 0, X->s[1].bin_slots),
                      species_io(c, 0, 1, X->s[0].bin_slots), species_io(c, 1, 1, X->s[1].bin_slots),
                      species_io(c, 0, 1, 0), species_io(c, 1, 1, 0)};
    (void)hipMemcpyAsync(X->ios, h, sizeof h, hipMemcpyHostToDevice, c.st);
    IdIO hi[6] = {species_ids(c, 0, 0), species_ids(c, 1, 0), species_ids(c, 0, 1),
                  species_ids(c, 1, 1), species_ids(c, 0, 1), species_ids(c, 1, 1)};
    (void)hipMemcpyAsync(X->iids, hi, sizeof hi, hipMemcpyHostToDevice, c.st);
    (void)hipStreamSynchronize(c.st);
}

void split_free(Ctx &c) {
    delete static_cast<SplitState *>(c.split);
    c.split = nullptr;
}

// ---------------------------------------------------------------- flat -> bins (init)
// beam: lab Gaussian -> boosted frame (FP64, as in the FP64 path) -> split
// position, appended to a flat list at the start of buffer 1
__global__ void k_beam_init32(Params P, const double *g, int64_t n, double sx, double sy, double szl, double sux,
                              double suy, double gB, double es, Part32 flat, int32_t *flat_id, int32_t *nflat,
                              double *part) {
    __shared__ double red[2][ST];
    int64_t q = (int64_t)blockIdx.x * ST + threadIdx.x;
    double cnt = 0.0, vzs = 0.0;
    bool act = false;
    PState s;
    if (q < n) {
        double x = 0.5 * P.nx + sx * g[q];
        double y = 0.5 * P.ny + sy * g[n + q];
        double zl = szl * g[2 * n + q];
        double ux = sux * g[3 * n + q], uy = suy * g[4 * n + q];
        double gam = gB * (1.0 + es * g[5 * n + q]);
        double uz = sqrt(gam * gam - 1.0 - ux * ux - uy * uy);
        double glab = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        double zb = P.gR * zl, tb = -P.gR * P.bR * zl;
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
        if (z >= 3.0 && z < (double)(P.nz - 4)) {
            act = true;
            double fx = floor(x), fy = floor(y), fz = floor(z);
            s.i = min((int)fx, P.nx - 1);
            s.j = min((int)fy, P.ny - 1);
            s.l = (int)fz;
            s.o[0] = (float)(x - fx - 0.5);  // from the cell's centre (x - fx and the 0.5 exact in FP64)
            s.o[1] = (float)(y - fy - 0.5);
            s.o[2] = (float)(z - fz - 0.5);
            for (int d = 0; d < 3; ++d)
                if (s.o[d] >= 0.5f) s.o[d] = 0.49999997f;  // FP32 rounding up to the cell's edge
            s.u[0] = (float)ux;
            s.u[1] = (float)uy;
            s.u[2] = (float)uzb;
            s.w = (float)P.wbeam;
            cnt = 1.0;
            vzs = uzb / gb;
        }
    }
    int r = reserve_slot(act, 0, nflat);
    if (act) {
        flat.cell[r] = pack_cell(P, s.i, s.j, s.l);
        flat.ox[r] = s.o[0];
        flat.oy[r] = s.o[1];
        flat.oz[r] = s.o[2];
        flat.ux[r] = s.u[0];
        flat.uy[r] = s.u[1];
        flat.uz[r] = s.u[2];
        flat.w[r] = s.w;
        if (flat_id) flat_id[r] = (int)q;  // beam slot = beam index
    }
    red[0][threadIdx.x] = cnt;
    red[1][threadIdx.x] = vzs;
    __syncthreads();
    for (int h = ST / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

// plasma sheets [l0, l0 + nsheets) at time t, window origin k0: appended to bins
// of `out` (bins == true) or to a flat list counted by out.ovf (bins == false)
__global__ void k_inject32(Params P, int64_t l0, int64_t total, double t, int64_t k0, OutStore out, int bins,
                           int32_t *flags, int32_t *out_id, int64_t id0) {
    int64_t q = (int64_t)blockIdx.x * ST + threadIdx.x;
    bool act = q < total;
    PState s;
    int key = 0;
    if (act) {
        const int64_t per = sheet_particles(P), pe = (int64_t)P.plane * P.ppx * P.ppy;
        int64_t l = l0 + q / per;
        int64_t r = q % per;
        const bool ion = r >= pe;  // mobile ions follow the sheet's electrons, weight negated
        if (ion) r -= pe;
        int a = (int)(r % P.ppx);
        r /= P.ppx;
        s.i = (int)(r % P.nx);
        r /= P.nx;
        int b = (int)(r % P.ppy);
        s.j = (int)(r / P.ppy);
        double w = sheet_weight(P, l);
        double z = sheet_z(l, P.ppz, P.bR, t) - (double)k0;  // logical
        double fz = floor(z);
        s.l = (int)fz;
        s.o[0] = (float)((a + 0.5) / P.ppx - 0.5);  // from the cell's centre
        s.o[1] = (float)((b + 0.5) / P.ppy - 0.5);
        s.o[2] = (float)(z - fz - 0.5);
        if (s.o[2] >= 0.5f) s.o[2] = 0.49999997f;
        s.u[0] = 0.0f;
        s.u[1] = 0.0f;
        s.u[2] = (float)(-P.uR);
        s.w = ion ? (float)-w : (float)w;
        s.id = (int)(id0 + q);  // the lattice particle's FP64 record slot
        act = w != 0.0 && s.l >= 3 && s.l < P.nz - 4;
        key = act ? bin_of(P, s.i, s.j, s.l) : 0;
    }
    if (bins) {
        append(out, act, key, act ? pack_cell(P, s.i, s.j, s.l) : 0, s.o, s.u, s.w, flags, out_id, s.id);
    } else {
        int r = reserve_slot(act, 0, out.ovf);
        if (act) {
            out.buf.cell[r] = pack_cell(P, s.i, s.j, s.l);
            out.buf.ox[r] = s.o[0];
            out.buf.oy[r] = s.o[1];
            out.buf.oz[r] = s.o[2];
            out.buf.ux[r] = s.u[0];
            out.buf.uy[r] = s.u[1];
            out.buf.uz[r] = s.u[2];
            out.buf.w[r] = s.w;
            if (out_id) out_id[r] = s.id;
        }
    }
}

__global__ void k_count_bins(Params P, Part32 flat, int64_t n, int32_t *cnt) {
    int64_t q = (int64_t)blockIdx.x * ST + threadIdx.x;
    if (q >= n) return;
    int i, j, l;
    unpack_cell(P, flat.cell[q], i, j, l);
    atomicAdd(&cnt[bin_of(P, i, j, l)], 1);
}

// bin capacities from counts with slack; host side
static bool layout_from_counts(Ctx &c, int sp, const std::vector<int32_t> &cnt, std::vector<int64_t> &off) {
    Store &s = SS(c).s[sp];
    int64_t nb = c.P.nbins;
    off.assign(nb + 1, 0);
    int64_t total = 0;
    for (int64_t b = 0; b < nb; ++b) total += cnt[b];
    int64_t spare = s.bin_slots - total;
    if (spare < 0) return false;
    // every bin: count + headroom (1/2 of its count for the beam, which pinches and drifts between
    // re-layouts; 1/8 for the plasma) + an even share of the remaining room
    const int64_t hd = sp == 0 ? 2 : 8;
    int64_t extra = 0;
    for (int64_t b = 0; b < nb; ++b) extra += cnt[b] / hd;
    int64_t share = std::max<int64_t>(0, (spare - extra) / std::max<int64_t>(1, nb));
    for (int64_t b = 0; b < nb; ++b) {
        int64_t cap = cnt[b] + (extra <= spare ? cnt[b] / hd : 0) + share;
        off[b + 1] = off[b] + cap;
    }
    return off[nb] <= s.bin_slots;
}

static pic_status upload_layout(Ctx &c, int sp, const std::vector<int64_t> &off, int which) {
    Store &s = SS(c).s[sp];
    PIC_HIP(c, hipMemcpyAsync(s.off[which], off.data(), 8 * off.size(), hipMemcpyHostToDevice, c.st));
    return PIC_OK;
}

// layout both buffers from the flat lists held in buffer 1 (counts in ovf[1]),
// then move them into the bins of buffer 0
static pic_status bins_from_flat(Ctx &c) {
    SplitState &X = SS(c);
    const Params &P = c.P;
    int64_t nb = P.nbins;
    std::vector<int32_t> nflat(2);
    for (int sp = 0; sp < 2; ++sp)
        PIC_HIP(c, hipMemcpyAsync(&nflat[sp], X.s[sp].ovf[1], 4, hipMemcpyDeviceToHost, c.st));
    PIC_HIP(c, hipMemsetAsync(X.tmpcnt, 0, 8 * nb, c.st));
    PIC_HIP(c, hipStreamSynchronize(c.st));
    for (int sp = 0; sp < 2; ++sp)
        if (nflat[sp] > 0)
            hipLaunchKernelGGL(k_count_bins, dim3(nblocks(nflat[sp], ST)), dim3(ST), 0, c.st, P, X.s[sp].buf[1],
                               (int64_t)nflat[sp], X.tmpcnt + sp * nb);
    std::vector<int32_t> h(2 * nb);
    PIC_HIP(c, hipMemcpyAsync(h.data(), X.tmpcnt, 8 * nb, hipMemcpyDeviceToHost, c.st));
    PIC_HIP(c, hipStreamSynchronize(c.st));
    for (int sp = 0; sp < 2; ++sp) {
        std::vector<int32_t> cs(h.begin() + sp * nb, h.begin() + (sp + 1) * nb);
        std::vector<int64_t> off;
        if (!layout_from_counts(c, sp, cs, off)) {
            c.err = "split layout: particle capacity exceeded";
            return PIC_ENOMEM;
        }
        pic_status s = upload_layout(c, sp, off, 0);
        if (s == PIC_OK) s = upload_layout(c, sp, off, 1);
        if (s != PIC_OK) return s;
        // the flat list is the "overflow" of buffer 1: no bin entries
        PIC_HIP(c, hipMemsetAsync(X.s[sp].cnt[1], 0, 4 * nb, c.st));
        X.s[sp].n_flat = nflat[sp];
    }
    // the flat lists are read as overflow tails that start at slot 0 and may fill the whole buffer
    build_worklist(c, 1, X.s[0].bin_slots + X.s[0].ovf_cap, X.s[1].bin_slots + X.s[1].ovf_cap);
    hipLaunchKernelGGL(k_rebin, dim3(X.grid), dim3(ST), 0, c.st, P, X.items, X.nitems, X.next, X.ios + 4, X.iids + 4,
                       c.dflags);
    for (int sp = 0; sp < 2; ++sp) PIC_HIP(c, hipMemsetAsync(X.s[sp].ovf[1], 0, 4, c.st));
    c.cur32 = 0;
    PIC_HIP(c, hipStreamSynchronize(c.st));
    return PIC_OK;
}

void split_beam_init(Ctx &c, const double *normals_dev) {
    SplitState &X = SS(c);
    const Params &P = c.P;
    int64_t n = c.beam.n_macro;
    double D = c.grid.dx_m;
    double F = c.beam.gamma_lab / (c.beam.gamma_lab * P.gR - sqrt(c.beam.gamma_lab * c.beam.gamma_lab - 1.0) *
                                                                   sqrt(P.gR * P.gR - 1.0));
    int nblk = nblocks(n, ST);
    hipLaunchKernelGGL(k_beam_init32, dim3(nblk), dim3(ST), 0, c.st, P, normals_dev, n, c.beam.sigma_cells[0],
                       c.beam.sigma_cells[1], c.beam.sigma_cells[2] / F, c.beam.emit_n_m[0] / (c.beam.sigma_cells[0] * D),
                       c.beam.emit_n_m[1] / (c.beam.sigma_cells[1] * D), c.beam.gamma_lab, c.beam.rel_energy_spread_rms,
                       X.s[0].buf[1], X.s[0].id[1], X.s[0].ovf[1], c.red);
    std::vector<double> h(2 * (size_t)nblk);
    (void)hipMemcpyAsync(h.data(), c.red, 16 * (uint64_t)nblk, hipMemcpyDeviceToHost, c.st);
    (void)hipStreamSynchronize(c.st);
    double cnt = 0, vz = 0;
    for (int k = 0; k < nblk; ++k) {
        cnt += h[2 * k];
        vz += h[2 * k + 1];
    }
    c.bw = cnt > 0 ? vz / cnt : 0.0;
}

// inject the nonzero-weight sheets of [l0, l1) at time t: one launch per run of
// consecutive nonzero-weight sheets, whose particles take the next ids (the
// slots the FP64 record layout gives them, in the same order)
static pic_status inject_runs32(Ctx &c, int64_t l0, int64_t l1, double t, int64_t k0, const OutStore &o,
                                int32_t *o_id, int bins) {
    const Params &P = c.P;
    const int64_t per = sheet_particles(P);
    int64_t l = l0;
    while (l < l1) {
        while (l < l1 && sheet_weight(P, l) == 0.0) ++l;
        const int64_t a = l;
        while (l < l1 && sheet_weight(P, l) != 0.0) ++l;
        const int64_t total = (l - a) * per;
        if (total > 0) {
            if (c.record && c.np_slots + total > 2147483647) {
                c.err = "record mode: more than 2^31 plasma particles over the run";
                return PIC_ERANGE;
            }
            hipLaunchKernelGGL(k_inject32, dim3(nblocks(total, ST)), dim3(ST), 0, c.st, P, a, total, t, k0, o, bins,
                               c.dflags, o_id, c.np_slots);
            c.np_slots += total;
        }
    }
    return PIC_OK;
}

pic_status split_plasma_fill(Ctx &c) {
    SplitState &X = SS(c);
    const Params &P = c.P;
    if (P.has_plasma) {
        OutStore o;
        o.buf = X.s[1].buf[1];
        o.off = X.s[1].off[1];
        o.cnt = X.s[1].cnt[1];
        o.ovf = X.s[1].ovf[1];
        o.bin_slots = X.s[1].bin_slots;
        o.ovf_cap = X.s[1].ovf_cap;
        pic_status st = inject_runs32(c, c.sh_lo, c.sh_hi, 0.0, 0, o, X.s[1].id[1], 0);
        if (st != PIC_OK) return st;
    }
    return bins_from_flat(c);
}

// ---------------------------------------------------------------- the step
void split_step(Ctx &c, const StepCtx &S) {
    SplitState &X = SS(c);
    const Params &P = c.P;
    FieldsT<float> f;
    for (int k = 0; k < 3; ++k) {
        f.E[k] = c.E32[k];
        f.B[k] = c.B32[k];
    }
    int cur = c.cur32;
    // the first B half step is formed inside the particle kernel (B^n in LDS); the field state between
    // steps stays (E^n, B^(n-1/2)), and after the push one full B step replaces the two halves
    hipEvent_t t1 = timing_begin(c);
    build_worklist(c, cur, 0, 0);  // overflow tails go to k_split_overflow
    if (P.und_kind)
        hipLaunchKernelGGL(k_ext_table, dim3(nblocks(P.nz + 2, 256)), dim3(256), 0, c.st, P, S, X.tabA, X.tabC,
                           X.tabS);
    timing_end(c, 2, t1);
    hipEvent_t t2 = timing_begin(c);
    hipLaunchKernelGGL(X.kern, dim3(X.grid), dim3(SST), X.lds_bytes, c.st, P, S, X.items, X.qstart, X.qnext, X.nslab,
                       IOPair{{species_io(c, 0, cur, X.s[0].bin_slots), species_io(c, 1, cur, X.s[1].bin_slots)},
                              {species_ids(c, 0, cur), species_ids(c, 1, cur)}},
                       f,
                       c.Ji[0], c.Ji[1], c.Ji[2], c.dflags, X.tabA, X.tabC, X.tabS);
    hipLaunchKernelGGL(k_split_overflow, dim3(256), dim3(256), 0, c.st, P, S, X.ios + 2 * cur, X.iids + 2 * cur, f,
                       c.Ji[0], c.Ji[1],
                       c.Ji[2], c.dflags);
    timing_end(c, 0, t2);
    hipEvent_t t3 = timing_begin(c);
    if (P.ions) launch_ion_fixed(P, c.sh_lo, c.sh_hi - c.sh_lo, S.t, S.t1, S.k0, c.jioni, c.dflags, c.st);
    launch_neutraliser_current(c, S);
    timing_end(c, 2, t3);
    hipEvent_t t4 = timing_begin(c);
    launch_bhalf<float>(P, S.k0r, f, (float)P.dt, (float *)c.murbuf, c.st);  // B^(n-1/2) -> B^(n+1/2)
    launch_eupdate<float, long long>(P, S.k0r, f, c.Ji, c.jioni, (float)P.dt, c.st);
    launch_mur_shift<float, long long>(P, S.k0r, S.shift, c.bw <= 0.0, f, (const float *)c.murbuf, c.jioni,
                                       (float)P.dt, c.st);
    timing_end(c, 1, t4);
}

// inject sheets [l0, l1) at time t into the output buffer (after split_step), then swap
pic_status split_inject_and_swap(Ctx &c, int64_t l0, int64_t l1, double t, int64_t k0n) {
    SplitState &X = SS(c);
    const Params &P = c.P;
    int o = c.cur32 ^ 1;
    if (P.has_plasma && l1 > l0) {
        OutStore out;
        out.buf = X.s[1].buf[o];
        out.off = X.s[1].off[o];
        out.cnt = X.s[1].cnt[o];
        out.ovf = X.s[1].ovf[o];
        out.bin_slots = X.s[1].bin_slots;
        out.ovf_cap = X.s[1].ovf_cap;
        pic_status st = inject_runs32(c, l0, l1, t, k0n, out, X.s[1].id[o], 1);
        if (st != PIC_OK) return st;
    }
    c.cur32 = o;
    return PIC_OK;
}

// ---------------------------------------------------------------- record mode export
// every particle of the current buffer to its FP64 record slot (its id):
// absolute boosted position, momentum, weight, alive; one block per bin, the
// last block takes the overflow tail
__global__ void k_split_export(Params P, int64_t k0, Part32 in, const int32_t *in_id, const int64_t *off,
                               const int32_t *cnt, int64_t ovf_start, const int32_t *ovf, int64_t ovf_cap, Part64 dst) {
    const int b = blockIdx.x;
    int64_t s0, n;
    if (b < P.nbins) {
        s0 = off[b];
        n = min((int64_t)cnt[b], off[b + 1] - off[b]);
    } else {
        s0 = ovf_start;
        n = min((int64_t)*ovf, ovf_cap);
    }
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
        const int64_t s = s0 + k, d = in_id[s];
        int i, j, l;
        unpack_cell(P, in.cell[s], i, j, l);
        dst.x[d] = (i + 0.5) + (double)in.ox[s];
        dst.y[d] = (j + 0.5) + (double)in.oy[s];
        dst.z[d] = ((double)(k0 + l) + 0.5) + (double)in.oz[s];
        dst.ux[d] = in.ux[s];
        dst.uy[d] = in.uy[s];
        dst.uz[d] = in.uz[s];
        dst.w[d] = in.w[s];
        dst.alive[d] = 1;
    }
}

void split_export64(const Ctx &c, Part64 beam, Part64 plasma, hipStream_t st) {
    const SplitState &X = *static_cast<const SplitState *>(c.split);
    for (int sp = 0; sp < 2; ++sp) {
        const Store &S = X.s[sp];
        hipLaunchKernelGGL(k_split_export, dim3(c.P.nbins + 1), dim3(256), 0, st, c.P, c.k0, S.buf[c.cur32],
                           S.id[c.cur32], S.off[c.cur32], S.cnt[c.cur32], S.bin_slots, S.ovf[c.cur32], S.ovf_cap,
                           sp ? plasma : beam);
    }
}

// ---------------------------------------------------------------- snapshots
// FP32 state after a step: the fields (the current is zero between steps), the
// bin layout and counts of both buffers, and the current particle buffer of
// each species (the other buffer is rewritten by the next step).
static uint64_t a256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

uint64_t split_state_payload(int64_t nc, int64_t slots_b, int64_t slots_p, uint64_t bins_bytes, int record) {
    const uint64_t sb = record ? 36 : 32;
    return 6 * a256(4 * (uint64_t)nc) + a256(sb * (uint64_t)slots_b) + a256(sb * (uint64_t)slots_p) + a256(bins_bytes);
}

pic_status split_copy_state(Ctx &c, char *dev, bool save) {
    SplitState &X = SS(c);
    uint64_t o = 0;
    auto mv = [&](void *mine, uint64_t bytes) -> pic_status {
        PIC_HIP(c, hipMemcpyAsync(save ? dev + o : mine, save ? (const void *)mine : (const void *)(dev + o), bytes,
                                  hipMemcpyDeviceToDevice, c.st));
        o += a256(bytes);
        return PIC_OK;
    };
    pic_status st;
    for (int k = 0; k < 3; ++k)
        if ((st = mv(c.E32[k], 4 * (uint64_t)c.P.nc)) != PIC_OK) return st;
    for (int k = 0; k < 3; ++k)
        if ((st = mv(c.B32[k], 4 * (uint64_t)c.P.nc)) != PIC_OK) return st;
    for (int sp = 0; sp < 2; ++sp) {
        Store &S = X.s[sp];
        if ((st = mv(S.buf[c.cur32].cell, slot_bytes(c) * (uint64_t)(S.bin_slots + S.ovf_cap))) != PIC_OK) return st;
    }
    return mv(c.arena + c.split_off_bins, c.split_bins_bytes);
}

// periodic host check: re-lay out the bins when any overflowed or is nearly full
pic_status split_check(Ctx &c) {
    SplitState &X = SS(c);
    const Params &P = c.P;
    int64_t nb = P.nbins;
    int cur = c.cur32;
    std::vector<int32_t> h(2 * nb);
    std::vector<int64_t> off(2 * (nb + 1));
    int32_t ov[2];
    for (int sp = 0; sp < 2; ++sp) {
        PIC_HIP(c, hipMemcpyAsync(h.data() + sp * nb, X.s[sp].cnt[cur], 4 * nb, hipMemcpyDeviceToHost, c.st));
        PIC_HIP(c, hipMemcpyAsync(off.data() + sp * (nb + 1), X.s[sp].off[cur], 8 * (nb + 1), hipMemcpyDeviceToHost, c.st));
        PIC_HIP(c, hipMemcpyAsync(&ov[sp], X.s[sp].ovf[cur], 4, hipMemcpyDeviceToHost, c.st));
    }
    PIC_HIP(c, hipStreamSynchronize(c.st));
    bool need = false;
    for (int sp = 0; sp < 2; ++sp) {
        if (ov[sp] > 0) need = true;
        for (int64_t b = 0; b < nb && !need; ++b) {
            int64_t cap = off[sp * (nb + 1) + b + 1] - off[sp * (nb + 1) + b];
            if ((int64_t)h[sp * nb + b] * 16 > cap * 15 && cap > 0) need = true;
        }
    }
    if (!need) return PIC_OK;
    // new layout from the true counts (bin counts clipped to capacity + overflow re-binned below)
    // count per destination bin including overflow particles: count kernel over the overflow tails
    PIC_HIP(c, hipMemsetAsync(X.tmpcnt, 0, 8 * nb, c.st));
    for (int sp = 0; sp < 2; ++sp) {
        int n = std::min<int64_t>(ov[sp], X.s[sp].ovf_cap);
        if (n > 0) {
            Part32 t = X.s[sp].buf[cur];
            Part32 v;
            int64_t s0 = X.s[sp].bin_slots;
            v.cell = t.cell + s0;
            v.ox = t.ox + s0;
            v.oy = t.oy + s0;
            v.oz = t.oz + s0;
            v.ux = t.ux + s0;
            v.uy = t.uy + s0;
            v.uz = t.uz + s0;
            v.w = t.w + s0;
            hipLaunchKernelGGL(k_count_bins, dim3(nblocks(n, ST)), dim3(ST), 0, c.st, P, v, (int64_t)n,
                               X.tmpcnt + sp * nb);
        }
    }
    std::vector<int32_t> extra(2 * nb);
    PIC_HIP(c, hipMemcpyAsync(extra.data(), X.tmpcnt, 8 * nb, hipMemcpyDeviceToHost, c.st));
    PIC_HIP(c, hipStreamSynchronize(c.st));
    int o = cur ^ 1;
    std::vector<std::vector<int64_t>> lay(2);
    for (int sp = 0; sp < 2; ++sp) {
        std::vector<int32_t> cs(nb);
        for (int64_t b = 0; b < nb; ++b) {
            int64_t cap = off[sp * (nb + 1) + b + 1] - off[sp * (nb + 1) + b];
            cs[b] = (int32_t)std::min<int64_t>(h[sp * nb + b], cap) + extra[sp * nb + b];
        }
        if (!layout_from_counts(c, sp, cs, lay[sp])) {
            c.err = "split re-layout: particle capacity exceeded";
            return PIC_ENOMEM;
        }
        pic_status s = upload_layout(c, sp, lay[sp], o);
        if (s != PIC_OK) return s;
    }
    build_worklist(c, cur, X.s[0].ovf_cap, X.s[1].ovf_cap);
    hipLaunchKernelGGL(k_rebin, dim3(X.grid), dim3(ST), 0, c.st, P, X.items, X.nitems, X.next, X.ios + 2 * cur,
                       X.iids + 2 * cur, c.dflags);
    for (int sp = 0; sp < 2; ++sp) {
        pic_status s = upload_layout(c, sp, lay[sp], cur);
        if (s != PIC_OK) return s;
    }
    c.cur32 = o;
    PIC_HIP(c, hipStreamSynchronize(c.st));
    return PIC_OK;
}

// ---------------------------------------------------------------- read-back
// one block per bin (plus one for the overflow tail): FP64 absolute coordinates
__global__ void k_split_out(Params P, int64_t k0, Part32 in, const int64_t *off, const int32_t *cnt, int64_t ovf_start,
                            int32_t ovf_n, const int64_t *pref, int nbins, double *dst, int64_t stride, int nout,
                            int32_t *alive) {
    int b = blockIdx.x;
    int64_t s0, n;
    if (b < nbins) {
        s0 = off[b];
        int64_t cap = off[b + 1] - off[b];
        n = cnt[b] < cap ? cnt[b] : cap;
    } else {
        s0 = ovf_start;
        n = ovf_n;
    }
    int64_t d0 = pref[b];
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
        int64_t s = s0 + k, d = d0 + k;
        if (alive) {
            alive[d] = 1;
            continue;
        }
        int i, j, l;
        unpack_cell(P, in.cell[s], i, j, l);
        double v[7] = {(i + 0.5) + (double)in.ox[s], (j + 0.5) + (double)in.oy[s],
                       ((double)(k0 + l) + 0.5) + (double)in.oz[s],
                       (double)in.ux[s], (double)in.uy[s], (double)in.uz[s], (double)in.w[s]};
        for (int q = 0; q < nout; ++q) dst[q * stride + d] = v[q];
    }
}

// charge -w of split particles on the nodes (mobile ions carry w < 0), FP64 atomics into rho (ring order)
__global__ void k_split_rho(Params P, int64_t k0, int k0r, Part32 in, const int64_t *off, const int32_t *cnt,
                            int64_t ovf_start, int32_t ovf_n, int nbins, double *rho) {
    int b = blockIdx.x;
    int64_t s0, n;
    if (b < nbins) {
        s0 = off[b];
        int64_t cap = off[b + 1] - off[b];
        n = cnt[b] < cap ? cnt[b] : cap;
    } else {
        s0 = ovf_start;
        n = ovf_n;
    }
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
        int64_t s = s0 + k;
        int i, j, l;
        unpack_cell(P, in.cell[s], i, j, l);
        float o[3] = {in.ox[s], in.oy[s], in.oz[s]};
        double w[3][3];
        int lo[3];
        const int base[3] = {i, j, l};
        for (int d = 0; d < 3; ++d) {
            int nn = o[d] >= 0.0f ? 1 : 0;
            weights3<double>((double)o[d] + 0.5 - nn, w[d]);
            lo[d] = base[d] + nn - 1;
        }
        double qw = -(double)in.w[s];
        for (int c = 0; c < 3; ++c) {
            int p = ring_plane(lo[2] + c, k0r, P.nz);
            for (int bb = 0; bb < 3; ++bb)
                for (int a = 0; a < 3; ++a)
                    atomicAdd(&rho[cell_index(P, lo[0] + a, lo[1] + bb, p)], qw * w[0][a] * w[1][bb] * w[2][c]);
        }
    }
}

__global__ void k_split_kin(Params P, Part32 in, const int64_t *off, const int32_t *cnt, int64_t ovf_start,
                            int32_t ovf_n, int nbins, double *part) {
    __shared__ double s[2][256];
    int b = blockIdx.x;
    int64_t s0, n;
    if (b < nbins) {
        s0 = off[b];
        int64_t cap = off[b + 1] - off[b];
        n = cnt[b] < cap ? cnt[b] : cap;
    } else {
        s0 = ovf_start;
        n = ovf_n;
    }
    double v0 = 0, v1 = 0;
    for (int64_t k = threadIdx.x; k < n; k += 256) {
        int64_t q = s0 + k;
        double ux = in.ux[q], uy = in.uy[q], uz = in.uz[q];
        v0 += 1.0;
        const double w = (double)in.w[q];
        v1 += (w < 0.0 ? -P.mi * w : w) * (sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
    }
    s[0][threadIdx.x] = v0;
    s[1][threadIdx.x] = v1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s[0][threadIdx.x] += s[0][threadIdx.x + h];
            s[1][threadIdx.x] += s[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * b] = s[0][0];
        part[2 * b + 1] = s[1][0];
    }
}

// prefix offsets (host) of the valid particles of each bin (+ overflow) of species sp
static int64_t split_prefix(Ctx &c, int sp, int32_t &ovf_n) {
    SplitState &X = SS(c);
    int64_t nb = c.P.nbins;
    Store &s = X.s[sp];
    int cur = c.cur32;
    std::vector<int32_t> &h = X.hcnt;
    std::vector<int64_t> &off = X.hoff, &pref = X.hpref;
    (void)hipMemcpyAsync(h.data(), s.cnt[cur], 4 * nb, hipMemcpyDeviceToHost, c.st);
    (void)hipMemcpyAsync(off.data(), s.off[cur], 8 * (nb + 1), hipMemcpyDeviceToHost, c.st);
    (void)hipMemcpyAsync(&ovf_n, s.ovf[cur], 4, hipMemcpyDeviceToHost, c.st);
    (void)hipStreamSynchronize(c.st);
    ovf_n = (int32_t)std::min<int64_t>(ovf_n, s.ovf_cap);
    pref[0] = 0;
    for (int64_t b = 0; b < nb; ++b) pref[b + 1] = pref[b] + std::min<int64_t>(h[b], off[b + 1] - off[b]);
    pref[nb + 1] = pref[nb] + ovf_n;
    (void)hipMemcpyAsync(X.tmpoff, pref.data(), 8 * (nb + 2), hipMemcpyHostToDevice, c.st);
    return pref[nb + 1];
}

void split_read(Ctx &c, int sp, double *dst7, int32_t *alive, int64_t *n) {
    SplitState &X = SS(c);
    int32_t ovf_n = 0;
    int64_t tot = split_prefix(c, sp, ovf_n);
    *n = tot;
    if ((!dst7 && !alive) || tot == 0) return;
    Store &s = X.s[sp];
    int cur = c.cur32;
    hipLaunchKernelGGL(k_split_out, dim3(c.P.nbins + 1), dim3(256), 0, c.st, c.P, c.k0, s.buf[cur], s.off[cur],
                       s.cnt[cur], s.bin_slots, ovf_n, X.tmpoff, c.P.nbins, dst7, tot, 7, alive);
}

int64_t split_beam_to64(Ctx &c, double *dst6) {
    SplitState &X = SS(c);
    int32_t ovf_n = 0;
    int64_t tot = split_prefix(c, 0, ovf_n);
    if (tot == 0) return 0;
    Store &s = X.s[0];
    int cur = c.cur32;
    int64_t stride = std::max<int64_t>(c.beam.n_macro, 1);
    if (tot > stride) tot = stride;  // cannot happen: beam particles are never created
    hipLaunchKernelGGL(k_split_out, dim3(c.P.nbins + 1), dim3(256), 0, c.st, c.P, c.k0, s.buf[cur], s.off[cur],
                       s.cnt[cur], s.bin_slots, ovf_n, X.tmpoff, c.P.nbins, dst6, stride, 6, (int32_t *)nullptr);
    return tot;
}

void split_rho(Ctx &c, double *rho, int mask) {
    SplitState &X = SS(c);
    int cur = c.cur32;
    for (int sp = 0; sp < 2; ++sp) {
        if (!(mask & (1 << sp))) continue;
        Store &s = X.s[sp];
        int32_t ovf_n = 0;
        (void)hipMemcpyAsync(&ovf_n, s.ovf[cur], 4, hipMemcpyDeviceToHost, c.st);
        (void)hipStreamSynchronize(c.st);
        ovf_n = (int32_t)std::min<int64_t>(ovf_n, s.ovf_cap);
        hipLaunchKernelGGL(k_split_rho, dim3(c.P.nbins + 1), dim3(256), 0, c.st, c.P, c.k0, (int)(c.k0 % c.P.nz),
                           s.buf[cur], s.off[cur], s.cnt[cur], s.bin_slots, ovf_n, c.P.nbins, rho);
    }
}

// lab-frame probe over the binned beam (one block per bin, the last one takes the overflow tail)
__global__ void k_split_probe(Params P, int64_t k0, Part32 in, const int64_t *off, const int32_t *cnt,
                              int64_t ovf_start, const int32_t *ovf, int64_t ovf_cap, double t1, double T, double k,
                              double *acc) {
    __shared__ double s[5][256];
    const int b = blockIdx.x;
    int64_t s0, n;
    if (b < P.nbins) {
        s0 = off[b];
        n = min((int64_t)cnt[b], off[b + 1] - off[b]);
    } else {
        s0 = ovf_start;
        n = min((int64_t)*ovf, ovf_cap);
    }
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const int64_t q = s0 + j;
        int i, jj, l;
        unpack_cell(P, in.cell[q], i, jj, l);
        probe_particle(P, ((double)(k0 + l) + 0.5) + (double)in.oz[q], in.ux[q], in.uy[q], in.uz[q], in.w[q], t1, T,
                       k, v);
    }
    for (int j = 0; j < 5; ++j) s[j][threadIdx.x] = v[j];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int j = 0; j < 5; ++j) s[j][threadIdx.x] += s[j][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int j = 0; j < 5; ++j) atomicAdd(&acc[j], s[j][0]);
}

// lab-frame groups of the binned beam: blocks stride over the bins (and the overflow tail, "bin" nbins)
__global__ void __launch_bounds__(256) k_split_lab_groups(Params P, LabGroupSpec G, int64_t k0, Part32 in,
                                                          const int64_t *off, const int32_t *cnt, int64_t ovf_start,
                                                          const int32_t *ovf, int64_t ovf_cap, double t, double *out) {
    __shared__ double tab[LAB_GROUP_VALUES * LAB_GROUPS_MAX];
    const int ng = G.nz * G.nu;
    lab_table_clear(tab, ng);
    __syncthreads();
    for (int b = blockIdx.x; b <= P.nbins; b += gridDim.x) {
        int64_t s0, n;
        if (b < P.nbins) {
            s0 = off[b];
            n = min((int64_t)cnt[b], off[b + 1] - off[b]);
        } else {
            s0 = ovf_start;
            n = min((int64_t)*ovf, ovf_cap);
        }
        for (int64_t j = threadIdx.x; j < n; j += 256) {
            const int64_t q = s0 + j;
            int i, jj, l;
            unpack_cell(P, in.cell[q], i, jj, l);
            lab_group_add(tab, G, P, t, (i + 0.5) + (double)in.ox[q], (jj + 0.5) + (double)in.oy[q],
                          ((double)(k0 + l) + 0.5) + (double)in.oz[q], in.ux[q], in.uy[q], in.uz[q], in.w[q]);
        }
    }
    __syncthreads();
    lab_table_flush(tab, ng, out);
}

void split_lab_groups(Ctx &c, const LabGroupSpec &G, double t, double *out) {
    SplitState &X = SS(c);
    const Store &S = X.s[0];
    const int cur = c.cur32;
    hipLaunchKernelGGL(k_split_lab_groups, dim3(std::min(c.P.nbins + 1, 1024)), dim3(256), 0, c.st, c.P, G, c.k0,
                       S.buf[cur], S.off[cur], S.cnt[cur], S.bin_slots, S.ovf[cur], S.ovf_cap, t, out);
}

void split_probe(Ctx &c, double *acc) {
    SplitState &X = SS(c);
    const Store &S = X.s[0];
    const int cur = c.cur32;
    hipLaunchKernelGGL(k_split_probe, dim3(c.P.nbins + 1), dim3(256), 0, c.st, c.P, c.k0, S.buf[cur], S.off[cur],
                       S.cnt[cur], S.bin_slots, S.ovf[cur], S.ovf_cap, (double)c.step * c.P.dt, c.probe_t, c.probe_k,
                       acc);
}

// plasma count and kinetic energy: one pair of partials per bin (and the overflow tail) into red
int split_plasma_kinetic_partials(Ctx &c, double *red) {
    SplitState &X = SS(c);
    int cur = c.cur32;
    Store &s = X.s[1];
    int32_t ovf_n = 0;
    (void)hipMemcpyAsync(&ovf_n, s.ovf[cur], 4, hipMemcpyDeviceToHost, c.st);
    (void)hipStreamSynchronize(c.st);
    ovf_n = (int32_t)std::min<int64_t>(ovf_n, s.ovf_cap);
    int nblk = c.P.nbins + 1;
    hipLaunchKernelGGL(k_split_kin, dim3(nblk), dim3(256), 0, c.st, c.P, s.buf[cur], s.off[cur], s.cnt[cur],
                       s.bin_slots, ovf_n, c.P.nbins, red);
    return nblk;
}

}  // namespace pic
