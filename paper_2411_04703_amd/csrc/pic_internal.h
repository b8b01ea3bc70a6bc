// pic_internal.h -- context layout and kernel launchers (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/pic.h"
#include "dev_common.h"

namespace pic {

// FP64 particle SoA (absolute boosted-frame positions in cells).
struct Part64 {
    double *x, *y, *z, *ux, *uy, *uz, *w;
    int32_t *alive;
};

// FP32 split particle SoA: logical cell index (i + nx (j + ny l), l = window plane)
// plus FP32 offsets in [0, 1), FP32 momenta and weight.
struct Part32 {
    int32_t *cell;
    float *ox, *oy, *oz, *ux, *uy, *uz, *w;
};

template <typename T> struct FieldsT {
    T *E[3], *B[3];
};

enum { DFLAG_FIXED_OVERFLOW = 1, DFLAG_NONFINITE = 2, DFLAG_BIN_LOST = 4 };

struct Ctx {
    Params P;
    int precision = 0, record = 0, device = 0, check_every = 64;
    hipStream_t st = nullptr;
    pic_grid grid;
    pic_frame frame;
    pic_beam beam;
    pic_plasma plasma;
    pic_undulator und;
    pic_options opt;
    double bw = 0, k_bunch_default = 0;
    // window position (cells) at time t: win_x0 + bw (t - win_t0); k0 = its floor, at most one shift per step
    double win_x0 = 0, win_t0 = 0;
    // neutralising charge faded over fc_T (normalised time; 0 = none): its node charge and
    // electrostatic field at t' = 0 (FP64, planes of the window at origin 0)
    double fc_T = 0;
    double *fc_rho = nullptr, *fc_E[3] = {};
    double beam_beta0 = 0;  // mean boosted beta_z of the beam at t' = 0
    int probe_on = 0;       // lab-frame probe armed
    double probe_t = 0, probe_k = 0;
    double *probe_acc = nullptr;  // its five sums (device)

    // host-side dynamic state (deterministic, no device read needed)
    int64_t step = 0, k0 = 0, sh_lo = 0, sh_hi = 0;
    int64_t cap_b = 0, cap_p = 0, nb_slots = 0, np_slots = 0;

    // arena
    char *arena = nullptr;
    uint64_t arena_bytes = 0, state_bytes = 0;

    // fields: FP64 mode uses E64/B64/J64, FP32 mode E32/B32 and J as int64 fixed point
    double *E64[3] = {}, *B64[3] = {}, *J64[3] = {};
    float *E32[3] = {}, *B32[3] = {};
    long long *Ji[3] = {};
    double *jion64 = nullptr;
    long long *jioni = nullptr;
    void *murbuf = nullptr;

    // particles
    Part64 b64{}, p64{}, p64alt{};
    Part32 b32[2]{}, p32[2]{};
    int cur32 = 0;  // which of the double buffers is current
    int64_t ovf_cap_b = 0, ovf_cap_p = 0;
    // FP32 split mode: host-side state of the binned stores (k_split32.hip)
    void *split = nullptr;
    int64_t split_slots_b = 0, split_slots_p = 0, split_items_cap = 0;
    uint64_t split_off_b = 0, split_off_p = 0, split_off_bins = 0, split_bins_bytes = 0, split_off_wl = 0;

    // scratch
    double *red = nullptr;       // reduction partials
    int64_t red_cap = 0;
    double *rprev = nullptr;     // previous Gauss residual (logical order)
    int64_t rprev_k0 = 0;
    int have_rprev = 0;
    double *adj = nullptr;       // adjoint scratch: lEn[3], Bn[3]
    double *stage = nullptr;     // normals staging (init)
    int32_t *dflags = nullptr;   // device error flags
    int64_t *i64scratch = nullptr;

    // kernel timing (HIP events on the context stream)
    int timing = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;

    std::string err;
};

// start / stop a timed region of class cls (no-op unless timing is on)
hipEvent_t timing_begin(Ctx &c);
void timing_end(Ctx &c, int cls, hipEvent_t start);

// ---------------------------------------------------------------- launchers
// FDTD (k_fdtd.hip)
template <typename T>
void launch_bhalf(const Params &P, int k0r, FieldsT<T> f, T h, T *murbuf, hipStream_t st);
template <typename T, typename JT>
void launch_eupdate(const Params &P, int k0r, FieldsT<T> f, JT *J[3], const JT *jion, T dt, hipStream_t st);
template <typename T, typename JT>
void launch_mur_shift(const Params &P, int k0r, int shift, int front_mur, FieldsT<T> f, const T *murbuf, JT *jion,
                      T dt, hipStream_t st);
void launch_ion64(const Params &P, int64_t sh_lo, int64_t nsheets, double t0, double t1, int64_t k0, double *jion,
                  hipStream_t st);
void launch_ion_fixed(const Params &P, int64_t sh_lo, int64_t nsheets, double t0, double t1, int64_t k0,
                      long long *jion, int32_t *flags, hipStream_t st);

// FP64 plain particles (k_plain64.hip)
void launch_beam_init64(const Params &P, const double *normals, int64_t n, const double sig[5], double gB,
                        double es, Part64 p, double *partials, int nblk, hipStream_t st);
void launch_inject64(const Params &P, int64_t l0, int64_t nsheets, double t, Part64 p, int64_t slot0,
                     hipStream_t st);
void launch_step64(const Params &P, const StepCtx &S, Part64 p, int64_t n, FieldsT<double> f, double *J[3],
                   int32_t *flags, hipStream_t st);
int64_t compact64(Ctx &c, Part64 src, Part64 dst, int64_t n);  // returns survivors (synchronising)

// FP32 split particles (k_split32.hip)
void split_setup(Ctx &c);
bool split_tile_supported(int tx, int ty, int tz);  // tiles the FP32 step kernel is built for
int split_lds_bytes(int tx, int ty, int tz);         // LDS of one FP32 step-kernel workgroup
uint64_t split_state_payload(int64_t nc, int64_t slots_b, int64_t slots_p, uint64_t bins_bytes, int record);
void split_export64(const Ctx &c, Part64 beam, Part64 plasma, hipStream_t st);  // record mode: particles to slots
pic_status split_copy_state(Ctx &c, char *dev, bool save);  // snapshot <-> context (device buffer)
void split_free(Ctx &c);
void split_beam_init(Ctx &c, const double *normals_dev);
pic_status split_plasma_fill(Ctx &c);  // also builds the initial bins of both species
void split_step(Ctx &c, const StepCtx &S);
pic_status split_inject_and_swap(Ctx &c, int64_t l0, int64_t l1, double t, int64_t k0n);
pic_status split_check(Ctx &c);  // bin capacity check + re-layout (synchronising)
void split_read(Ctx &c, int species, double *dst7, int32_t *alive, int64_t *n);
void split_probe(Ctx &c, double *acc);  // lab-frame probe over the binned beam
void split_lab_groups(Ctx &c, const LabGroupSpec &G, double t, double *out);  // lab-frame groups of the binned beam

// diagnostics (k_diag.hip)
int64_t diag_partials(const Ctx &c, uint32_t mask);  // partial sums run_diag needs for this mask
pic_status run_diag(Ctx &c, uint32_t mask, double kb, pic_diag_out *out, double *red, int64_t red_cap);
// allocation-free diagnostics: a static device array of DIAG_STATIC_DOUBLES per GPU
enum : int64_t { DIAG_STATIC_DOUBLES = (int64_t)1 << 19 };  // 4 MiB
pic_status static_scratch_setup(Ctx &c);  // once per device, with the device current (pic_init)
double *static_scratch(int device);       // its device address, or NULL before the set-up
void beam_rho(Ctx &c, double *rho);  // beam charge on the nodes (ring order), added into rho
void probe_step(Ctx &c);             // lab-frame probe: sample the beam particles that crossed its lab time
pic_status lab_beam(Ctx &c, double *out, int64_t *n);                   // the beam's lab phase space (8 rows)
pic_status lab_groups(Ctx &c, const LabGroupSpec &G, double *out);      // its groups (16 values each)

// initial beam self-field and the faded neutralising charge (k_initfield.hip)
pic_status init_beam_fields(Ctx &c);
pic_status init_neutraliser(Ctx &c);
double neutraliser_left(const Ctx &c, double t);  // fraction of the neutralising charge left at time t
void launch_neutraliser_current(Ctx &c, const StepCtx &S);  // adds its current of the step into J
void launch_neutraliser_rho(Ctx &c, double *rho);           // adds its charge now into rho (ring order)

// adjoint (k_adjoint.hip)
pic_status adjoint_seed(Ctx &c, double kb, double *lam, double *loss);
pic_status adjoint_step(Ctx &c, double *lam, double grad[2]);

// helpers (pic_api.cpp)
StepCtx make_step_ctx(const Ctx &c);
pic_status hip_check(Ctx &c, hipError_t e, const char *what);

inline int nblocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace pic

#define PIC_HIP(c, call)                                                    \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) return ::pic::hip_check((c), e_, #call);     \
    } while (0)
