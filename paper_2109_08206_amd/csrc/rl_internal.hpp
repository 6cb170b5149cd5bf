// Internal declarations of the rodlcp HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rodlcp.h"

namespace rl {

constexpr int kBlock = 256;              // threads per workgroup for the flat kernels
constexpr int kWaves = kBlock / 64;      // wave64
constexpr int kImgZero = 0x888;          // packed zero periodic shift
constexpr double kEpsPar = 1e-14;        // below this 1 - (di.dj)^2 the axes are parallel
constexpr double kBandPar = 1e-10;       // flag band for near-parallel axes
constexpr double kDegenDist = 1e-12;     // axis distance below which the normal is di x dj
constexpr double kCutoffBand = 1e-9;     // flag band around the pair threshold

// Solver modes of the rod / constraint kernels.
enum Mode : int {
    kModeInit = 0,    // gamma' = max(0, gamma): w0 = Mc gamma0 + q
    kModeAlpha0 = 1,  // gamma' = projected gradient: alpha0 = gh.gh / gh.Mc gh
    kModeLoop = 2,    // gamma' = max(0, gamma - alpha g): one BBPGD iteration
    kModeApply = 3,   // gamma' = gamma (no projection): w = Mc gamma (+ q)
    kModeRefresh = 4, // mixed precision: FP64 g = Mc gamma + q, residual, FP32 state reset
};

// Device-resident solver state.  The loop kernels never write fields that
// other workgroups of the same launch read: alpha and the stop latch are
// published by workgroup 0 of the rod kernel and read by later launches.
struct SolverState {
    double alpha;          // step of iteration 0 (alpha0)
    double alpha0, amin, amax;
    double tol;
    long long max_iter;
    // results for the host, written once when the stop is decided
    double res, ss, sy, yy;
    long long iter;
    int done, status;
    // mixed precision: inner rounds run until the FP32 residual is below
    // inner_tol; then an FP64 refresh recomputes g and the certified residual
    double inner_tol, rho64;
    long long refreshes;
    int refresh;  // set by the rod kernel when the inner round ends
    int pad;
};

// Per-rod mobility: a_par, a_perp (translation along / normal to the axis),
// r_perp (rotation about a normal axis).  Axial rotation uses r_perp as well.
struct Mob {
    double apar, aperp, rperp;
};

// Host-side view of the mobility constants of a uniform-length system.
Mob mobility_host(double L, double diam, double eta);

// rod kernel: kRodLanes lanes per rod, kRodBlock / kRodLanes rods per workgroup
#ifndef RL_ROD_BLOCK
#define RL_ROD_BLOCK 1024
#endif
#ifndef RL_ROD_LANES
#define RL_ROD_LANES 4
#endif
constexpr int kRodBlock = RL_ROD_BLOCK;
constexpr int kRodLanes = RL_ROD_LANES;
#ifndef RL_ROD_LOOP_BLOCK
#define RL_ROD_LOOP_BLOCK 256
#endif
constexpr int kRodLoopBlock = RL_ROD_LOOP_BLOCK;  // workgroup of the single-solve rod kernel
#ifndef RL_CON_BLOCK
#define RL_CON_BLOCK 512
#endif
#ifndef RL_CON_GRIDMAX
#define RL_CON_GRIDMAX 512
#endif
#ifndef RL_CON_CPL
#define RL_CON_CPL 2
#endif
constexpr int kConBlock = RL_CON_BLOCK;     // constraint kernel workgroup
constexpr int kConGridMax = RL_CON_GRIDMAX; // constraint kernel grid cap (grid-stride beyond)
constexpr int kConGridMixed = 256;  // the same cap for the mixed-precision solve
#ifndef RL_CON_PER_GROUP
#define RL_CON_PER_GROUP 2048
#endif
constexpr int kConPerGroup = RL_CON_PER_GROUP;  // target constraints per constraint workgroup
constexpr int kConCpl = RL_CON_CPL;         // constraints per lane per round, loaded together

// Arguments shared by the solver kernels (passed by value).
struct SolveArgs {
    int64_t n, nc;
    const double *dir;      // [n][3]
    const double *coef;     // [n][3] per-rod mobility, or nullptr when uniform
    Mob mob;                // uniform mobility
    const int2 *pp;         // [nc] (pi, pj)
    const int32_t *pptr;    // [n+1] first constraint with pi >= r
    const int32_t *qptr;    // [n+1] Q-side incidence offsets
    const int32_t *qidx;    // [nc] constraints with pj == r, ascending
    const int32_t *qpos;    // [nc] position of constraint c in the Q-side list
    const double *geo;      // [nc][4] (ex, ey, ez, s_i): what the rod kernel reads
    const double2 *geo2;    // [nc] (s_j, q): the rest of the constraint record
    const double *qgeo;     // [nc][4] Q-side list order: (ex, ey, ez, s_j)
    double2 *st;            // [nc] (gamma, g) of the current iterate
    double2 *stq;           // [nc] the same in Q-side list order
    double *V;              // [n][6] per rod: M_t F_c and Omega_c x dir (adjoint kernels)
    const double *qv;       // [nc] q alone, for the constraint kernel
    double *uP;             // [nc] e.(V_i + s_i W_i): velocity of the contact point on pi along e
    double *uQ;             // [nc] e.(V_j + s_j W_j) in Q-side list order
    double *partial;        // [2][gcon][4] workgroup partials, by iteration parity
    double *alpha_buf;      // [2] step length of iteration k at k & 1
    int gcon;               // workgroups of the constraint kernel
    SolverState *state;
    double *out;            // kModeApply output
    // mixed precision (RL_FP32_MIXED): gamma = gamma64 + delta with delta >= b = -gamma64
    float4 *st32;           // [nc] (delta, h, b, h0): h approximates g, h0 = g at the last refresh
    float4 *stq32;          // [nc] (delta, h, b, 0) in Q-side list order
    const float4 *geo32;    // [nc] (ex, ey, ez, s_i)
    const float4 *qgeo32;   // [nc] Q-side list order: (ex, ey, ez, s_j)
    float *uP32;            // [nc] contact velocities of the correction, P side
    float *uQ32;            // [nc] the same, Q side in list order
    // general constraint sets (bilateral links, fixed bodies): constraints
    // sorted by (pi, kind), Q lists by (kind, index)
    bool gen;               // the set holds bilateral or one-sided constraints
    const int32_t *psplit;  // [n] first bilateral constraint of rod r's P range
    const int32_t *qsplit;  // [n] first bilateral position in rod r's Q list
    const double *cmpv;     // [nc] compliance 1/(kappa h) (bilateral) or -1 (unilateral)
    // host-visible progress word of the FP64 loop: workgroup 0 of the rod
    // kernel of iteration k stores 2 k + (1 once the stop is decided), so the
    // host follows the loop without copies in the stream (may be null)
    unsigned long long *progress;
};

// --- kernels launchers (implemented in the .hip files) ----------------------
hipError_t launch_directors(hipStream_t st, int64_t n, const double *quat, double *dir);
hipError_t launch_mobility_coeffs(hipStream_t st, int64_t n, const double *len, double diam, double eta,
                                  double *coef);

// the walls of one call, by value in kernel arguments
struct WallSet {
    int n;
    int kind[RL_MAX_WALLS];
    double p[RL_MAX_WALLS][3], a[RL_MAX_WALLS][3], r[RL_MAX_WALLS];
};

struct PairGrid {
    int nc[3];
    double cell[3];
    int S[3];
    double box[3];
    int64_t ncell;
};

}  // namespace rl

// Opaque handle.
struct rl_ctx {
    rl_params prm;
    hipStream_t stream = nullptr;
    int device = 0;
    // grow-only workspace slots
    static constexpr int kSlots = 128;
    void *buf[kSlots] = {};
    size_t cap[kSlots] = {};
    rl::SolverState *state = nullptr;       // device
    rl::SolverState *state_host = nullptr;  // pinned
    int *flag_dev = nullptr;                // device error flags
    int64_t *host_scratch = nullptr;        // pinned, for small readbacks
    unsigned long long *progress_host = nullptr;  // pinned coherent word written by the loop (SolveArgs::progress)
    unsigned long long *progress_dev = nullptr;   // its device address
    // event sampling of the loop kernels
    static constexpr int kMaxEv = 64;
    int prof_every = 0;
    hipEvent_t ev[kMaxEv][4] = {};  // start/stop of the rod and the constraint kernel
    long long ev_iter[kMaxEv] = {};
    double prof_ms[2] = {0.0, 0.0};
    double prof_cnt[2] = {0.0, 0.0};
    hipEvent_t chk_ev = nullptr;  // marks the state copy of a stop-flag check
    // batched solves: a stream of our own (graph capture), workgroup sizes
    hipStream_t own_stream = nullptr;
    int batch_rb = 0, batch_cb = 0;            // fixed by the caller; 0 = tune
    int batch_rb_used = 0, batch_cb_used = 0;  // the last solve's choice
    int tune_loaded = 0;
    int tune_rb[64] = {}, tune_cb[64] = {};    // per log2(constraints) bucket
    void *host_buf = nullptr;                  // pinned staging for tables
    size_t host_cap = 0;
    // allocation-free calls: while arena_on, ws_get hands out consecutive
    // pieces of the device's scratch array instead of allocating
    char *scratch = nullptr;                   // this device's scratch array
    size_t arena_used = 0;
    bool arena_on = false;
    // warm start: sorted constraint keys and forces of the last warm step
    int64_t warm_count = -1;                   // -1: none kept
    int64_t warm_n = 0;                        // its rod count
};

namespace rl {

enum Slot : int {
    kWsDir = 0, kWsCoef, kWsV, kWsUnc, kWsPptr, kWsQptr, kWsQidx, kWsQcnt, kWsG, kWsPartial,
    kWsCellOf, kWsCellCnt, kWsCellStart, kWsCellCur, kWsSorted, kWsXs, kWsDs, kWsLs, kWsPcnt, kWsPoff,
    kWsStepPi, kWsStepPj, kWsStepImg, kWsStepFlags, kWsStepPhi, kWsStepE, kWsStepArm, kWsStepQ, kWsStepGamma,
    kWsStepU, kWsScan, kWsLenMax, kWsPP, kWsGeo, kWsSt, kWsAlpha, kWsQpos, kWsQgeo, kWsStq, kWsSortIdx, kWsSortTmp, kWsCellKey, kWsFs,
    kWsSt32, kWsStq32, kWsGeo32, kWsUP32, kWsQgeo32, kWsUQ32,
    kWsBatchTab, kWsBatchOff, kWsBatchState, kWsBatchAlpha, kWsBatchCtr, kWsBatchPartial,
    kWsBatchPartial2, kWsBatchDone, kWsBatchMap, kWsGeo2, kWsPairCache, kWsScanTmp, kWsEmitCount, kWsEmitKeys, kWsEmitFlags,
    kWsAdjG, kWsAdjUbar, kWsAdjQbd, kWsAdjCs, kWsAdjCr, kWsAdjCq, kWsAdjSc, kWsAdjPQ, kWsAdjDmob,
    kWsAdjEbar, kWsAdjArmbar, kWsAdjQbar, kWsAdjDbar, kWsAdjGbar, kWsAdjFs, kWsQv, kWsUP, kWsUQ,
    kWsGenKey, kWsGenKeyOut, kWsGenOrd, kWsGenPi, kWsGenPj, kWsGenE, kWsGenArm, kWsGenQ, kWsGenCmp, kWsGenGamma,
    kWsGenPsplit, kWsGenQsplit, kWsLinkLen, kWsLinkFlags, kWsInvPerm, kWsWallCnt, kWsWallOff,
    kWsCatPi, kWsCatPj, kWsCatE, kWsCatArm, kWsCatQ, kWsCatKind, kWsCatCmp, kWsCatLen, kWsStepUnc,
    kWsFtot, kWsWarmKeys, kWsWarmGam, kWsWarmKeysNew, kWsWarmGamNew, kWsStress,
    kWsKmcCount, kWsKmcFlag, kWsKmcOff, kWsKmcKey, kWsKmcKeyOut, kWsKmcPerm,
    kWsCount  // number of slots; must not exceed rl_ctx::kSlots
};
static_assert(kWsCount <= rl_ctx::kSlots, "workspace slot table too small");

// Returns a device buffer of at least `bytes` in slot `s` (grow-only).
void *ws_get(rl_ctx *h, int s, size_t bytes, int *err);
// Pinned host staging buffer of at least `bytes` (grow-only).
void *ws_get_host(rl_ctx *h, size_t bytes, int *err);

void set_error(const char *fmt, ...);

// Internal building blocks used by the C-ABI layer.
int build_pairs_impl(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                     int64_t capacity, int32_t *pi, int32_t *pj, int32_t *img, uint8_t *flags, int64_t *n_pairs);
hipError_t launch_gather6(hipStream_t st, int64_t n, const int *perm, const double *src, double *dst);
int stable_sort_by_key(rl_ctx *h, int64_t n, const int *keys, int bits, int *keys_out, int *perm);

// Filaments binned by centre into periodic cells of edge >= L_max/2 +
// radius, for queries of the filaments whose axis passes within `radius` of
// a point (the nearest image of each centre; RL_ERR_ARG when L_max/2 +
// radius exceeds half the box).  Rods in cell order, stable by index.
struct RodCells {
    int nc[3];
    double cell[3], box[3];
    const int *start;             // [ncell + 1]
    const int *order;             // cell position -> caller's index
    const double *xs, *ds, *ls;   // centres, directors, lengths in cell order
};
int rod_cells(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
              double radius, RodCells *out);
// out[0..m] = exclusive prefix sums of in[0..m-1] (out[m] = the total, also
// written to *total when given), on the handle's stream.  tmp (may be null:
// taken from the workspace) holds scan_tmp_bytes(m) bytes.
int device_scan(rl_ctx *h, const int *in, int64_t m, int *out, int64_t *total, void *tmp = nullptr);
int scan_tmp_bytes(int64_t m, size_t *bytes);
// bytes of the allocation-free scratch array on each device
constexpr size_t kScratchBytes = (size_t)RL_NOALLOC_SCRATCH_BYTES;
// sorts m (key, value) pairs by key (the warm start's constraint keys)
int sort_key_values(rl_ctx *h, int64_t m, const unsigned long long *keys, const double *vals,
                    unsigned long long *keys_out, double *vals_out);
// Pair list in the solver's own rod order (cell order).  On return *perm
// (device, n) maps solver rod -> caller rod and xs/ds/ls hold the rods'
// centres, directors and lengths in solver order (handle workspace).
int build_pairs_sorted(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                       int64_t *n_pairs, const int **perm, const double **xs, const double **ds, const double **ls);
int assemble_impl(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                  int64_t nc, const int32_t *pi, const int32_t *pj, const int32_t *img, const double *F,
                  double *phi, double *e, double *arm, double *q);
// trusted: the pair list was built by the library itself (rl_step), so the
// index checks and their host sync are skipped
int prepare_solve(rl_ctx *h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                  const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                  double *gamma, SolveArgs *a, bool trusted = false);
int apply_impl(rl_ctx *h, SolveArgs &a, double *w);
int solve_impl(rl_ctx *h, SolveArgs &a, const double *F, double *U, double *gamma_out, rl_solve_info *info,
               const int *perm = nullptr);
// xu (may be null): unwrapped centres, += h U_t without wrapping
int integrate_impl(rl_ctx *h, int64_t n, const double *U, double *x, double *quat, double *xu = nullptr);
// mixed precision: FP32 copies of the geometry, then the refinement loop
int prepare_mixed(rl_ctx *h, SolveArgs &a);
int solve_mixed_impl(rl_ctx *h, SolveArgs &a, long long *refreshes);
// FP64 refresh for the mixed solver: gamma64 += delta (if accum), g64 = Mc gamma64 + q,
// certified residual, FP32 state reset
hipError_t launch_refresh64(rl_ctx *h, const SolveArgs &a, bool accum);
hipError_t launch_alpha0_64(rl_ctx *h, const SolveArgs &a);
hipError_t launch_velocity64(rl_ctx *h, const SolveArgs &a, const double *F, const int *perm, double *U);
hipError_t launch_velocity_on(hipStream_t st, const SolveArgs &a, const double *F, const int *perm, double *U);
hipError_t launch_unpack_gamma(hipStream_t st, const SolveArgs &a, double *gamma);
__global__ void k_state_init(SolverState *st, double tol, long long max_iter);
__global__ void k_restore_start(int64_t nc, const double *gamma_in, const int32_t *qpos, double2 *st,
                                double2 *stq);
// adjoint (rl_adjoint.hip): lambda on the active set by CG, then the
// per-rod and per-constraint adjoints.  `a` is a prepared solve whose st
// holds gamma; Ubar is in solver rod order; F and F_bar in the caller's
// (perm maps solver -> caller, may be null).  step: q includes D^T M F
// (rl_step_adjoint) rather than being an input of its own.
struct AdjOut {
    double *F_bar;     // [n][6] caller order
    double *q_bar;     // [nc]
    double *e_bar;     // [nc][3]
    double *arm_bar;   // [nc][2]
    double *d_bar;     // [nc][6] lever-arm parts of dir_bar (rod i, rod j)
    double *dmob;      // [n][3] mobility part of dir_bar, solver order
};
int adjoint_core(rl_ctx *h, SolveArgs &a, bool step, const double *Ubar, const double *F, const int *perm,
                 double cg_tol, const AdjOut &o, rl_adjoint_info *info);
// dir_bar = dmob + sum of the lever-arm parts over each rod's constraints
hipError_t launch_dir_bar(hipStream_t st, const SolveArgs &a, const double *dmob, const double *d_bar,
                          double *dir_bar);
// step: adjoint of the Euler update (solver order out), and the final
// per-rod sums into x_bar / quat_bar (caller order, in place)
hipError_t launch_integrate_adj(hipStream_t st, int64_t n, const int *perm, const double *x_bar,
                                const double *quat_bar, const double *quat, const double *U, double dt,
                                double *Ubar, double *qbd);
hipError_t launch_step_bar(hipStream_t st, const SolveArgs &a, const int *perm, const double *gbar,
                           const double *dmob, const double *qbd, const double *quat, double *x_bar,
                           double *quat_bar);
// closest-point adjoint (rl_geometry.hip): per constraint (r0_bar, dir_i_bar,
// dir_j_bar) from (phi_bar = q_bar / h, e_bar, arm_bar) plus the lever-arm
// parts d_bar
hipError_t launch_geo_adjoint(hipStream_t st, int64_t nc, const double *x, const double *dir, const double *len,
                              double len0, const double box[3], const int32_t *pi, const int32_t *pj,
                              const int32_t *img, double dt, const double *q_bar, const double *e_bar,
                              const double *arm_bar, const double *d_bar, double *gbar);
// general constraint sets (rl_general.hip): validation (unless trusted),
// the merged order by (pi, kind) (*order: merged position -> input index),
// and the solver's records
int prepare_general(rl_ctx *h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                    const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                    const uint8_t *kind, const double *cmp, const double *gamma, bool trusted, SolveArgs *out,
                    const int **order);
hipError_t launch_scatter_gamma(hipStream_t st, const SolveArgs &a, const int *order, double *gamma);
// Multi-step pieces of a step (rl_general.hip).  A step's constraint list in
// input order: [0, np) contacts (pi, pj in the solver's rod order, img),
// [np, np + nl) links, then wall contacts.  perm: solver -> caller rod.
struct StepList {
    int64_t n, np, nl, nc;
    const int *perm;
    const int32_t *pi, *pj, *img;
    const double *dir;                 // solver order
    const double *e, *arm, *phi;       // input order (phi: contacts)
    const double *link_len;            // [nl]
    const int64_t *link_key;           // [nl] warm-start keys (null: the index)
};
// Brownian force: Ftot = F + sqrt(2 kT/h) M^(-1/2) noise (caller order)
hipError_t launch_brownian(hipStream_t st, int64_t n, const double *dir, const double *len, double len0, double diam,
                           double eta, double dt, double kT, const double *noise, const double *F, double *Ftot);
// gamma0 (input order) from the last warm step's keys (0 where none matches)
int warm_lookup(rl_ctx *h, const StepList &L, double *gamma0);
// keeps this step's keys and forces (gamma in input order)
int warm_store(rl_ctx *h, const StepList &L, const double *gamma);
// the 18 stress components (host) from the forces in input order
int step_stress(rl_ctx *h, const StepList &L, const double *gamma, double *out);
// wall contacts of rods (x, dir, len in one order; Unc = M F in the same)
int walls_impl(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
               const double *Unc, const WallSet &W, int64_t capacity, int32_t *rod, double *e, double *arm,
               double *phi, double *q, uint8_t *flags, int64_t *count);
// checks and copies the caller's walls
int wall_set(int n_walls, const rl_wall *walls, WallSet *W);
hipError_t launch_unc(hipStream_t st, int64_t n, const double *dir, const double *len, double len0, double diam,
                      double eta, const double *F, double *Unc);
hipError_t launch_links(hipStream_t st, int64_t nl, int64_t n, const double *x, const double *dir, const int *inv,
                        const rl_links *lk, const double box[3], double dt, const double *Unc, int32_t *pi,
                        int32_t *pj, double *len, double *e, double *arm, double *q, double *cmp, uint8_t *flags,
                        int *err);
int solve_batched_impl(rl_ctx *h, int S, const int64_t *rod_off, const int64_t *pair_off, SolveArgs &a,
                       const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                       const double *gamma_in, const double *F, double *gamma_out, double *U, rl_solve_info *infos);

}  // namespace rl

#define RL_HIP(call)                                                                               \
    do {                                                                                           \
        hipError_t _e = (call);                                                                    \
        if (_e != hipSuccess) {                                                                    \
            rl::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, __LINE__); \
            return RL_ERR_HIP;                                                                     \
        }                                                                                          \
    } while (0)
