/*
 * rodlcp — steric-constraint step for rigid spherocylinder filaments on one
 * AMD MI355X (gfx950) GPU.
 *
 * The method is the constraint-based collision handling of Yan et al.,
 * "Towards the cellular-scale simulation of motor-driven cytoskeletal
 * assemblies" (arXiv 2109.08206), unilateral (collision) constraints only:
 *
 *   * each rod has a centre x and a unit quaternion theta; velocities and
 *     forces are 6-vectors per rod, U = M F with a block-diagonal mobility
 *     (Section 3 "Filament dynamics"; Appendix "Filament dynamics");
 *   * near-contact pairs are the rod pairs whose surface gap phi is below a
 *     threshold (Appendix "Implementation");
 *   * the force on a pair acts along the unit normal e at the closest points,
 *     F_u = D_u gamma_u (eq. dmap, the column D_PQ of Appendix "Symmetry of
 *     the geometrically constrained optimization problem");
 *   * one linearised implicit Euler step (eq. constrainedeom_euler,
 *     eq. linearconstraints) reduces to the complementarity problem
 *     gamma >= 0, w = Mc gamma + q >= 0, gamma.w = 0, with Mc = D^T M D and
 *     q = phi/h + D^T M F_ext (eq. blockdef, blocks A and B; eq. cqpdef),
 *     solved by Barzilai-Borwein projected gradient descent (Section
 *     "Instantiation in a massively parallel computing environment").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: um, s, pN.  All arrays are DEVICE pointers in the caller's
 * allocation (e.g. torch tensors), row-major, double precision unless noted;
 * the library never frees them and never keeps them past the call.  The
 * library owns only its handle's workspace.  Work is enqueued on the
 * handle's stream (rl_set_stream); entry points that return host values
 * (counts, rl_solve_info) synchronise that stream before returning.
 *
 *   x[n][3]      rod centres, each coordinate inside [0, box)
 *   quat[n][4]   unit quaternions [s, px, py, pz]; the rod axis is body z
 *   dir[n][3]    unit directors R(theta) e_z
 *   len[n]       rod lengths; or len == NULL and every rod has length len0
 *   F[n][6]      external force (3) and torque (3) per rod
 *   U[n][6]      translational (3) and angular (3) velocity per rod
 *   pi, pj[nc]   int32 rod indices of each constraint, pi <= pj, sorted so
 *                that pi is non-decreasing (canonical order below)
 *   img[nc]      int32 packed periodic shift n of rod pj: rod pj is taken at
 *                x_pj + n*box; img = ((nx+8)<<8) | ((ny+8)<<4) | (nz+8),
 *                |n| <= 7, zero shift = 0x888; packed values order like
 *                (nx, ny, nz) lexicographically
 *   flags[nc]    uint8 bit 0: |phi - cutoff| <= 1e-9; bit 1: axes within
 *                1e-10 of parallel (1 - (di.dj)^2 <= 1e-10); bit 2: axes
 *                closer than 1e-12 (normal taken from di x dj)
 *   phi[nc]      surface gap = axis distance - diam
 *   e[nc][3]     unit normal at the closest points, pointing from rod pj
 *                (imaged) to rod pi; gamma > 0 pushes them apart
 *   arm[nc][2]   (s_i, s_j): arclength of the closest point on each axis
 *                from its centre, |s| <= L/2; lever arm y = s * dir
 *   q[nc]        phi/h + D^T M F
 *   gamma[nc]    constraint force magnitudes (pN)
 *
 * Canonical pair order: ascending (pi, pj, img); a rod may pair with its own
 * periodic image (pi == pj) only with a lexicographically positive shift.
 *
 * Return codes: 0 OK; > 0 warnings (outputs valid, solve not converged);
 * < 0 errors (outputs undefined).  rl_status_str() names them and
 * rl_last_error() gives the message of the last error on the calling thread.
 */
#ifndef RODLCP_H
#define RODLCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RL_OK 0
#define RL_NOT_CONVERGED 1  /* max_iter reached; gamma, U are the last iterate */
#define RL_STAGNATED 2      /* BB step made no progress (gamma unchanged) above tol */
#define RL_ERR_ARG (-1)     /* bad argument: NULL pointer, size, layout or value */
#define RL_ERR_CAPACITY (-2)/* pair capacity too small; required count written */
#define RL_ERR_NONFINITE (-3) /* NaN/Inf met in inputs or iterates */
#define RL_ERR_HIP (-4)     /* a HIP runtime call failed */
#define RL_ERR_NOMEM (-5)   /* workspace allocation failed */

#define RL_FP64 0           /* all solver arithmetic in double precision */
#define RL_FP32_MIXED 1     /* BBPGD in single precision on a correction delta to an
                               FP64 iterate (gamma = gamma64 + delta); the BB dot
                               products and residuals accumulate in FP64 and an
                               FP64 product re-anchors gamma64 and g whenever the
                               FP32 residual has dropped by 1e-4 (or stalls); the
                               stop test and the returned residual are FP64 */

typedef struct rl_ctx *rl_handle;

typedef struct {
    double box[3];      /* periodic box edges, > 0 (every system is periodic) */
    double diam;        /* rod diameter, > 0 */
    double cutoff;      /* keep pairs with phi < cutoff (strict), >= 0 */
    double eta;         /* fluid viscosity, > 0 (pN s / um^2) */
    double dt;          /* time step h, > 0 */
    double tol;         /* BBPGD stops when max_c |min(gamma_c, w_c)| <= tol */
    int64_t max_iter;   /* BBPGD iteration cap, >= 0 */
    int32_t precision;  /* RL_FP64 or RL_FP32_MIXED */
    int32_t check_every;/* 0 = default (32).  FP64 loop: the host follows a progress word that the
                           loop stores into pinned host memory and keeps min(check_every, 7)
                           iterations queued past the running one.  FP32-mixed, batched and
                           adjoint loops: iterations between host checks of the stop flag, with
                           up to 8 more queued behind each check.  Iterations queued past the
                           stop return at once without touching the result */
} rl_params;

typedef struct {
    int64_t iterations; /* BBPGD iterations taken (products Mc*gamma in the loop) */
    double residual;    /* max_c |min(gamma_c, w_c)| at exit, evaluated in FP64 */
    double alpha0;      /* initial step length */
    int32_t status;     /* RL_OK, RL_NOT_CONVERGED or RL_STAGNATED */
    int32_t fp64_refreshes; /* RL_FP32_MIXED: FP64 products that re-anchored the
                               FP32 iteration (0 in RL_FP64) */
} rl_solve_info;

/* Handle lifecycle.  rl_create copies *prm (validated: RL_ERR_ARG on a bad
 * value) and binds the device that is current on the calling thread.  The
 * default stream is the null stream. */
int rl_create(rl_handle *h, const rl_params *prm);
int rl_destroy(rl_handle h);
int rl_set_params(rl_handle h, const rl_params *prm);
int rl_get_params(rl_handle h, rl_params *prm);
/* hip_stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream). */
int rl_set_stream(rl_handle h, void *hip_stream);
/* Pre-size the workspace for up to max_rods rods and max_pairs constraints
 * so that later calls of that size allocate nothing. */
int rl_reserve(rl_handle h, int64_t max_rods, int64_t max_pairs);
const char *rl_status_str(int status);
const char *rl_last_error(void);

/* Directors dir = R(theta) e_z (Appendix "Filament dynamics": rotation
 * matrix of the unit quaternion; the rod axis is body z). */
int rl_directors(rl_handle h, int64_t n, const double *quat, double *dir);

/* Near-contact pairs (Appendix "Implementation": only pairs whose minimal
 * distance is below the threshold enter the solver; here phi < cutoff on
 * the surface gap).  Writes the canonical list into pi, pj, img, flags
 * (each of length capacity) and the count into *n_pairs (host).  If the
 * count exceeds capacity nothing is written to the lists, *n_pairs holds
 * the required count and RL_ERR_CAPACITY is returned.  RL_ERR_ARG if a
 * centre lies outside [0, box) or box < (reach of two rods)/7 in any
 * direction; RL_ERR_NONFINITE on NaN/Inf in x or dir.  Synchronises. */
int rl_build_pairs(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                   int64_t capacity, int32_t *pi, int32_t *pj, int32_t *img, uint8_t *flags, int64_t *n_pairs);

/* Constraint geometry and right-hand side for a pair list (eq. blockdef,
 * block A: q = phi/h + D^T M F; the column of D for pair (P, Q) =
 * (pi, pj) is [e; y_P x e; -e; -(y_Q x e)], Appendix "Symmetry ...").
 * Writes phi, e, arm, q.  F may be NULL (no external load).  RL_ERR_ARG if
 * a pair index is outside [0, n).  Synchronises (index validation). */
int rl_assemble_D(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                  int64_t nc, const int32_t *pi, const int32_t *pj, const int32_t *img, const double *F,
                  double *phi, double *e, double *arm, double *q);

/* w = Mc gamma + q with Mc = D^T M D applied matrix-free (the gradient of
 * the QP of eq. cqpdef).  q may be NULL (then w = Mc gamma).  gamma is
 * used as given (no projection).  RL_ERR_ARG if pi is not sorted or an
 * index is out of range.  Synchronises (index validation). */
int rl_apply_M(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
               const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
               const double *gamma, double *w);

/* Solve the complementarity problem of eq. cqpdef (unilateral block) by
 * BBPGD and return the velocities U = M (D gamma + F) (eq.
 * constrainedeom_euler).  gamma is the start on entry (negative entries are
 * clipped to 0; zeros = cold start) and the solution on exit.  F may be NULL
 * (zero external load).  *info (host) receives iterations, residual and
 * status.  Returns info->status (>= 0) or an error.  Synchronises. */
int rl_solve_lcp(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                 const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                 const double *F, double *gamma, double *U, rl_solve_info *info);

/* ---------------------------------------------------------------------------
 * Bilateral constraints and general constraint sets
 * ---------------------------------------------------------------------------
 * Hookean links (crosslinkers, joints) are bilateral constraints: the
 * spring law K (Phi_b - Phi_b^0) = -gamma_b (eq. bilateralconstraint),
 * linearised over the step, adds the rows of eq. linearconstraints (b) to the
 * problem: the quadratic program of eq. suppcqpdef with gamma_u >= 0 and
 * gamma_b free, its matrix D^T M D plus K^-1/h on the bilateral diagonal
 * (eq. blockdef, blocks C-F).  The same BBPGD solves it; bilateral entries
 * are not projected and their residual is |w_b|.
 *
 * A link joins the point at arclength arm[k][0] on rod p[k]'s axis to the
 * point at arm[k][1] on rod q[k]'s axis (points fixed on the bodies), or,
 * with q[k] < 0, to the fixed point anchor[k] (a tether to the lab frame:
 * only rod p's side enters D, Appendix "Equation of motion with geometric
 * constraints", last paragraph).  Its vector r = (x_p + s_p d_p) - (x_q +
 * s_q d_q) takes each component of the difference to its nearest periodic
 * image; length |r|, e = r / |r| (from q to p; gamma > 0 pushes apart,
 * gamma < 0 pulls).  kappa > 0 (pN/um; INFINITY: a rigid joint), rest >= 0
 * (um). */
typedef struct {
    int64_t n_links;
    const int32_t *p, *q;   /* [n_links] rod indices (device); q < 0: fixed point */
    const double *arm;      /* [n_links][2] arclengths on the two axes (device) */
    const double *kappa;    /* [n_links] stiffness (device) */
    const double *rest;     /* [n_links] rest length (device) */
    const double *anchor;   /* [n_links][3] fixed points (device; may be NULL if no q < 0) */
    const int64_t *key;     /* [n_links] warm-start keys, distinct, 0 <= key < 2^62 (device; may be NULL:
                               a link's key is its index).  Keys are not checked: a repeated key or one
                               outside the range only gives a link another link's start (the solution is
                               the same) */
} rl_links;

/* Link geometry and rows: writes length[n_links], e[n_links][3], q[n_links]
 * = (length - rest)/h + D^T M F (F may be NULL), cmp[n_links] = 1/(kappa h)
 * and flags[n_links] (may be NULL; bit 2: zero length, e normal to both
 * axes).  RL_ERR_ARG on an index outside the rods, p == q, kappa <= 0, a
 * bad rest length or a missing anchor.  Synchronises. */
int rl_assemble_links(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                      const rl_links *links, const double *F, double *length, double *e, double *q, double *cmp,
                      uint8_t *flags);

/* The mixed problem over a general constraint list of nc entries in any
 * order: kind[c] = 0 for a unilateral constraint (contact, wall), 1 for a
 * bilateral one with compliance cmp[c] >= 0 (cmp may be NULL when no entry
 * is bilateral); pi[c] in [0, n) is the rod on the P side, pj[c] the rod on
 * the Q side or -1 for a fixed body (a wall or an anchor; pj may equal pi
 * for a periodic self-contact); e, arm and q as for rl_solve_lcp.  gamma
 * (start on entry: unilateral entries clipped to >= 0; solution on exit) and
 * U = M (D gamma + F) as in rl_solve_lcp; info->residual is the largest of
 * |min(gamma_u, w_u)| and |w_b|.  RL_FP64 only.  The constraints are reordered
 * internally (by P rod, unilateral first); every result is returned in the
 * caller's order.  RL_ERR_ARG on a bad index, kind or compliance.
 * Synchronises. */
int rl_solve_general(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                     const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                     const uint8_t *kind, const double *cmp, const double *F, double *gamma, double *U,
                     rl_solve_info *info);

/* Walls: confinement by fixed bodies (Appendix "Equation of motion with
 * geometric constraints", last paragraph: a flat substrate or a spherical
 * shell; only the rod's side enters D).
 *   RL_WALL_PLANE        the allowed side is a.(x - p) >= 0 (a: unit normal)
 *   RL_WALL_SPHERE_IN    inside the sphere |x - p| <= r
 *   RL_WALL_CYLINDER_IN  inside the cylinder of axis p + t a (a unit), radius r
 * Each region is convex, so a rod's axis stays inside exactly when both of
 * its ends do.  For each rod, end s = -L/2 then +L/2, and each wall in order,
 * the end's gap phi = (its distance to the wall) - diam/2; an end with
 * phi < cutoff gives a unilateral constraint against the wall: e is the
 * wall's unit normal at its nearest point, pointing into the allowed region,
 * the lever arm is s, q = phi/h + D^T M F.  Walls are host structs, at most
 * RL_MAX_WALLS per call; the caller keeps the confinement inside the
 * periodic box (the centres are used as given). */
#define RL_WALL_PLANE 0
#define RL_WALL_SPHERE_IN 1
#define RL_WALL_CYLINDER_IN 2
#define RL_MAX_WALLS 8
typedef struct {
    int32_t kind;
    double p[3];   /* a point of the plane / the centre / a point of the axis */
    double a[3];   /* unit normal (plane) or unit axis (cylinder) */
    double r;      /* radius (sphere, cylinder) */
} rl_wall;

/* Wall contacts in that order: rod[m] (int32), e[m][3], arm[m][2] = (s, 0),
 * phi[m], q[m] (F may be NULL), flags[m] (may be NULL; bit 0: |phi - cutoff|
 * <= 1e-9), each of length capacity; *n_contacts (host) gets the count.  If
 * it exceeds capacity nothing is written and RL_ERR_CAPACITY is returned.
 * For rl_solve_general they are kind 0 with pj = -1.  RL_ERR_ARG on a bad
 * wall (unknown kind, zero normal or axis, radius <= 0, more than
 * RL_MAX_WALLS).  Synchronises. */
int rl_assemble_walls(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                      const double *F, int32_t n_walls, const rl_wall *walls, int64_t capacity, int32_t *rod,
                      double *e, double *arm, double *phi, double *q, uint8_t *flags, int64_t *n_contacts);

/* rl_solve_lcp without allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): the same problem, kernels and result as rl_solve_lcp
 * (bitwise), with every workspace piece taken from a scratch array of
 * RL_NOALLOC_SCRATCH_BYTES that the library keeps on each device for the
 * life of the process.  The call makes no hipMalloc, hipFree or other
 * allocating call; the handle (rl_create) must already exist.  RL_FP64 only;
 * kernel-event sampling (rl_profile_enable) is ignored.
 * Workspace: 152 bytes per constraint and 12 bytes per rod (36 with per-rod
 * lengths) plus a few KB (e.g. 100,000 rods with 468,687 constraints take
 * 73 MB); a larger problem returns RL_ERR_ARG with nothing enqueued.
 * Every call on one GPU uses that GPU's one array: calls that overlap in time
 * on the same GPU (other threads, other handles, other streams) race and must
 * be serialised by the caller.  Synchronises, like rl_solve_lcp. */
#define RL_NOALLOC_SCRATCH_BYTES (96ull << 20)
int rl_solve_lcp_noalloc(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                         const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                         const double *F, double *gamma, double *U, rl_solve_info *info);

/* One whole timestep: directors, pairs, geometry, solve, then the
 * linearised Euler update x += h U_t (wrapped into the box) and
 * theta += h Psi(theta) Omega, renormalised (eq. constrainedeom_euler,
 * first line; Psi of Appendix "Filament dynamics").  x and quat are updated
 * in place; U (may be NULL) receives the velocities; *n_pairs (host, may be
 * NULL) the constraint count.  Pair and constraint storage is the handle's.
 * The step synchronises its stream: the pair count sizes the constraint
 * arrays and the BBPGD loop's length is decided by its stop test, both read
 * on the host (a whole step is therefore not capturable in a graph).
 *
 * Tape (for differentiating rollouts): the step's constraint forces gamma,
 * in the step's own constraint order (the canonical pair order of the rods
 * renumbered in cell order; opaque to the caller, but a pure function of
 * (x, quat, len)).  gamma_tape is a device array of tape_len doubles.
 *   RL_TAPE_NONE    gamma_tape unused (may be NULL); cold start gamma = 0.
 *   RL_TAPE_RECORD  cold start; the solution is written to gamma_tape.  If
 *                   the constraint count exceeds tape_len, nothing is
 *                   changed, *n_pairs holds the count and RL_ERR_CAPACITY
 *                   is returned.
 *   RL_TAPE_REPLAY  gamma_tape holds the tape recorded for the same
 *                   (x, quat, len) and tape_len must equal its count
 *                   (RL_ERR_ARG otherwise); the solve starts from it, so an
 *                   identical state stops at once with the identical
 *                   solution (written back to gamma_tape).
 * Synchronises. */
#define RL_TAPE_NONE 0
#define RL_TAPE_RECORD 1
#define RL_TAPE_REPLAY 2
/* Optional parts of a step (extra may be NULL: none of them; NULL or 0
 * fields are absent).
 *   x_unwrapped[n][3]  device, in/out: the centres without periodic
 *                      wrapping; the step adds h U_t to them (the same
 *                      increment as x, eq. constrainedeom_euler, first line).
 *   links              bilateral links (rl_links, rod indices in the caller's
 *                      numbering) solved together with the contacts
 *                      (eq. linearconstraints a and b).
 *   gamma_links        [n_links] device out: the links' forces (pN; > 0 pushes
 *                      the ends apart).
 *   n_walls, walls     host walls (rl_wall) confining the rods.
 *   n_wall_contacts    host out: the step's wall constraints.
 *   noise[n][6], kT    device N(0,1) draws (caller's rod order) and the
 *                      thermal energy (pN um): the Brownian force
 *                      F_B = sqrt(2 kT/h) M^(-1/2) noise joins F in F_nc
 *                      (velocity noise of covariance 2 kT M / h over the
 *                      step; the caller draws the numbers).
 *   warm_start         1: start the solve from the forces of the previous
 *                      step on this handle that also had warm_start set,
 *                      matched by constraint (a contact by its two rods and
 *                      periodic shift in the caller's numbering, a link by
 *                      its key, rl_links.key, or by its index when that is
 *                      NULL; wall contacts start at 0), and keep this
 *                      step's forces for the next one.  The result is the
 *                      same problem's solution; only the start differs.
 *   stress[18]         host out: the virial of the constraint forces between
 *                      rods, (1/V) sum_c gamma_c (x_P - x_Q') e_c^T over the
 *                      contacts (stress[0..8], row-major) and over the links
 *                      between two rods (stress[9..17]); V = box volume,
 *                      pN/um^2; positive trace for repulsion (pressure =
 *                      trace / 3).
 * With links or walls the step solves the general problem (RL_FP64 only, no
 * gamma tape). */
typedef struct {
    double *x_unwrapped;
    const rl_links *links;
    double *gamma_links;
    int32_t n_walls;
    const rl_wall *walls;
    int64_t *n_wall_contacts;
    const double *noise;
    double kT;
    int32_t warm_start;
    double *stress;
} rl_step_extra;
int rl_step(rl_handle h, int64_t n, double *x, double *quat, const double *len, double len0, const double *F,
            double *U, rl_solve_info *info, int64_t *n_pairs, double *gamma_tape, int64_t tape_len,
            int32_t tape_mode, const rl_step_extra *extra);

/* Batching form: S independent periodic systems solved together (one set
 * of launches per BBPGD phase for all of them, iterations replayed from a
 * captured HIP graph, workgroup sizes picked by timing; the problem of each
 * system is that of rl_solve_lcp).  The systems are concatenated: system s
 * owns rods [rod_off[s], rod_off[s+1]) and constraints
 * [pair_off[s], pair_off[s+1]) of the device arrays, which have the layouts
 * above; pi and pj are indices into the concatenated rods and each
 * constraint must join two rods of its own system.  rod_off and pair_off are
 * HOST arrays of S + 1 entries starting at 0.  Each system has its own step
 * length, stop test and iteration count; infos (host, S entries) receives
 * them.  Returns the most severe status over the systems.  RL_FP64 only.
 * Synchronises; work runs on a stream the handle owns, after the handle's
 * stream has drained. */
int rl_solve_lcp_batched(rl_handle h, int32_t S, const int64_t *rod_off, const int64_t *pair_off, const double *dir,
                         const double *len, double len0, const int32_t *pi, const int32_t *pj, const double *e,
                         const double *arm, const double *q, const double *F, double *gamma, double *U,
                         rl_solve_info *infos);
/* Workgroup sizes of the batched kernels: rod_block in {256, 1024} and
 * con_block in {256, 512}, or both 0 to time the candidates on the first
 * solve of each problem size (the default; (256, 256) is kept unless another
 * pair is at least 3% faster; cached in the handle and appended to the file
 * named by the environment variable RODLCP_TUNE_CACHE if set).
 * chosen (host, may be NULL) receives the sizes the last solve used. */
int rl_batch_tuning(rl_handle h, int rod_block, int con_block, int *chosen);

/* Differentiation form.  Where the step is differentiable, the constraint
 * rows of the active set A hold as equalities (eq. linearconstraints): on A,
 * Mc_AA gamma_A + q_A = 0, and gamma = 0 off A.  Here c is in A when
 * gamma_c > w_c for the solution gamma and w = Mc gamma + q.  The adjoint
 * then solves Mc_AA lambda = D_A^T M U_bar by conjugate gradients (the
 * Chronopoulos-Gear form, one fused reduction per iteration).  It starts
 * from 0, which gives the minimum-norm lambda when Mc_AA is singular, and
 * stops when ||r||_2 <= cg_tol * ||D_A^T M U_bar||_2 (cg_tol <= 0: 1e-10)
 * or after prm.max_iter iterations.  All arithmetic is FP64 and every sum
 * runs in a fixed order, so results are bitwise repeatable. */
typedef struct {
    int64_t cg_iterations;   /* CG iterations (products Mc_AA p) */
    double cg_residual;      /* ||r||_2 / ||b||_2 at exit (0 when b = 0) */
    int64_t n_active;        /* |A| */
    int32_t status;          /* RL_OK, RL_NOT_CONVERGED (iteration cap) or
                                RL_STAGNATED (CG breakdown, curvature <= 0) */
    int32_t solve_status;    /* rl_step_adjoint: status of its forward solve */
    int64_t solve_iterations;/* rl_step_adjoint: BBPGD iterations of it */
    double solve_residual;   /* rl_step_adjoint: its residual */
} rl_adjoint_info;

/* Adjoint of rl_solve_lcp taken as the map (dir, e, arm, q, F) -> U, with
 * gamma its solution.  q is an input in its own right here (its own
 * dependence on D and F belongs to rl_step_adjoint).  Given U_bar[n][6],
 * it writes the gradients of U_bar . U:
 *   q_bar[nc]      = -lambda (0 off A)
 *   e_bar[nc][3], arm_bar[nc][2]   through the columns of D
 *   F_bar[n][6]    = M U_bar
 *   dir_bar[n][3]  through the mobility blocks and the lever arms s * dir
 * Inputs have the layouts of rl_solve_lcp (pi sorted, pi <= pj); gamma is
 * the solution returned by rl_solve_lcp on the same inputs.  F may be NULL.
 * Outputs are device arrays owned by the caller and are overwritten.
 * Returns info->status, or an error (RL_ERR_ARG on a NULL array, an
 * unsorted or out-of-range index, a bad size).  Synchronises. */
int rl_solve_lcp_adjoint(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                         const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                         const double *F, const double *gamma, const double *U_bar, double cg_tol, double *q_bar,
                         double *e_bar, double *arm_bar, double *F_bar, double *dir_bar, rl_adjoint_info *info);

/* Adjoint of one rl_step.  The step is the map (x, theta, F) -> (x', theta')
 * with x' = x + h U_t (wrapping shifts by whole box lengths and has
 * derivative 1) and theta' = normalise(theta + h Psi(theta) Omega).  The
 * entry point re-runs the forward step from (x, quat, F): pair search,
 * geometry, BBPGD from gamma = 0.  It is the same computation as rl_step on
 * those inputs, and x, quat are not changed.  Then it differentiates the
 * step at that point, with the pair list and A held fixed:
 *   x_bar[n][3]    in: adjoint of x'; out: adjoint of x
 *   quat_bar[n][4] in: adjoint of theta'; out: adjoint of theta, with its
 *                  component along theta removed (the gradient on the unit
 *                  sphere; theta is renormalised each step)
 *   F_bar[n][6]    out: adjoint of F (F may be NULL: zero load)
 * The closest points are differentiated through the clamped normal
 * equations.  Where an arclength sits on a rod end it is held there.  For
 * parallel axes (1 - (di.dj)^2 <= 1e-14) the closest points are held fixed.
 * For intersecting axes (distance < 1e-12) the normal is held fixed.
 * gamma_tape (may be NULL) is the tape rl_step recorded for the same
 * (x, quat, len) with tape_len its count.  The forward solve then starts
 * from it and stops at once.  Without it, the solve runs from gamma = 0 to
 * the same bitwise result.  RL_ERR_ARG if tape_len does not match.
 * Returns the CG status (>= 0; a forward solve that did not converge is
 * reported in info->solve_status), or an error.  Synchronises. */
int rl_step_adjoint(rl_handle h, int64_t n, const double *x, const double *quat, const double *len, double len0,
                    const double *F, const double *gamma_tape, int64_t tape_len, double *x_bar, double *quat_bar,
                    double *F_bar, double cg_tol, rl_adjoint_info *info);

/* ---------------------------------------------------------------------------
 * Crosslinker kinetics (kinetic Monte Carlo of binding and unbinding)
 * ---------------------------------------------------------------------------
 * Section "2. Crosslinker binding and unbinding" (Table tab:rates) and the
 * appendix "Kinetic Monte-Carlo" (Table tab:supprates).  A crosslinker is a
 * Hookean tether between heads A and B, in one of four states: RL_XL_U (both
 * unbound), RL_XL_SA / RL_XL_SB (one head bound), RL_XL_D (both bound).  In a
 * step of length h (the handle's dt) every crosslinker makes at most one
 * transition, with probability 1 - exp(-R h) for the total rate R of its
 * possible transitions (eq. P_bind), chosen in proportion to the rates:
 *   U -> S_h : R = k_oS[h] K_a[h] eps 3/(4 pi r_cs^3) sum_i L_in,i, L_in,i the
 *              length of filament i's axis inside the sphere of radius r_cs
 *              about the crosslinker (eq. KMC01exp); the head lands
 *              uniformly on the captured length (filaments in index order).
 *   S_h -> U : R = k_oS[h]; the crosslinker reappears uniformly in the
 *              sphere of radius r_cs about the head.
 *   S_h -> D : the free head g binds a site of another filament within r_cd
 *              of the bound head: R = k_oD[g] K_e[g] / V_bd sum_sites
 *              exp(-(kappa/kT)((1 - lambda)/2 Delta^2 - x_c Delta)), Delta =
 *              l - l_o - D the tether's stretch (eq. Ucl); the site is chosen
 *              over the filaments in index order, their sites in order.
 *   D -> S   : head h releases at R = k_oD[h] exp((kappa/kT)(lambda/2
 *              Delta^2 + x_c Delta)) (eq. KMC_DS_Edep, eq. KMC_SD_fdep).
 * Sites: floor(eps L) per filament (at least one) at the centres of equal
 * arclength intervals.  V_bd = 4 pi int_0^r_cd exp(-kappa (r - l_o - D)^2 /
 * (2 kT)) r^2 dr (eq. double_bind_volume_gen).  Before the transitions the
 * unbound crosslinkers diffuse, x += sqrt(2 d_U h) xi (Section "1.
 * Crosslinking motor diffusion and stepping").  Filaments are taken at the
 * periodic image of their centre nearest to the query point, so L_max/2 +
 * max(r_cs, r_cd) must not exceed half the box (RL_ERR_ARG).  Association
 * constants are volumes (um^3; K in 1/uM is K / 602.214 um^3).  Random
 * numbers are inputs: per crosslinker and step u[m][4] uniform in [0, 1)
 * (event, which transition, target, reappearance radius) and xi[m][3]
 * N(0, 1) (diffusion, reappearance direction). */
#define RL_XL_U 0
#define RL_XL_SA 1
#define RL_XL_SB 2
#define RL_XL_D 3
#define RL_EV_NONE 0
#define RL_EV_BIND 1     /* U -> S */
#define RL_EV_UNBIND 2   /* S -> U */
#define RL_EV_CROSS 3    /* S -> D */
#define RL_EV_RELEASE 4  /* D -> S */
typedef struct {
    double eps;     /* binding sites per um of filament */
    double Ka[2];   /* U <-> S association constants of heads A, B (um^3) */
    double koS[2];  /* S -> U rates (1/s) */
    double Ke[2];   /* S <-> D association constants (um^3) */
    double koD[2];  /* D -> S rates without load (1/s) */
    double kappa;   /* tether stiffness (pN/um) */
    double rest;    /* tether free length l_o (um) */
    double lambda;  /* energy factor of the release rate, in [0, 1] */
    double xc;      /* characteristic length of the force dependence (um) */
    double kT;      /* thermal energy (pN um), > 0 */
    double rcs;     /* capture radius of U -> S (um), > 0 */
    double rcd;     /* cutoff of the S -> D site sum (um), > 0 */
    double dU;      /* diffusion constant of unbound crosslinkers (um^2/s) */
} rl_kmc_params;

/* The crosslinkers, device arrays owned by the caller, updated in place:
 * state[m]; rod[m][2] and arc[m][2] the filament (-1: unbound) and arclength
 * of heads A and B; x[m][3] the position (the crosslinker's when unbound,
 * the bound head's in S, head A's in D; in the box). */
typedef struct {
    int64_t m;
    int32_t *state;
    int32_t *rod;
    double *arc;
    double *x;
} rl_crosslinkers;

/* V_bd of kp with the handle's diameter (host out).  RL_ERR_ARG on bad
 * parameters. */
int rl_kmc_effective_volume(rl_handle h, const rl_kmc_params *kp, double *vbd);

/* One step of the kinetics for all crosslinkers against the filaments (x,
 * dir, len as for rl_build_pairs; not changed).  u, xi: the step's random
 * numbers (device).  event[m] (device, may be NULL): RL_EV_* per crosslinker.
 * counts[5] (host, may be NULL): crosslinkers per event.  RL_ERR_ARG on bad
 * parameters, a bad state or head, or a box below the reach (nothing is
 * changed then), and when the axes of more than 128 filaments pass within
 * the query radius of one crosslinker (a few pass at the paper's densities):
 * that crosslinker is left unchanged while the others have stepped.
 * Synchronises. */
int rl_kmc_step(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                const rl_kmc_params *kp, const rl_crosslinkers *xl, const double *u, const double *xi,
                int32_t *event, int64_t *counts);

/* The doubly bound crosslinkers as bilateral links (rl_links) for the
 * filament step: p = head A's filament, q = head B's, arm = their
 * arclengths, kappa = kp->kappa, rest = kp->rest + diam (the tether's rest
 * length between the axes, eq. Ucl), in crosslinker order; key (may be
 * NULL) = the crosslinker's index, a warm-start key (rl_links.key) that
 * stays with the crosslinker while it is bound, whatever binds or unbinds
 * elsewhere.  Each array has room for capacity links.  *n_links (host) gets
 * the count; if it exceeds capacity nothing is written and RL_ERR_CAPACITY
 * is returned.  Synchronises. */
int rl_kmc_links(rl_handle h, const rl_kmc_params *kp, const rl_crosslinkers *xl, int64_t capacity, int32_t *p,
                 int32_t *q, double *arm, double *kappa, double *rest, int64_t *key, int64_t *n_links);

/* Kernel timing with HIP events on the handle's stream, for measurement.
 * With every > 0, every every-th BBPGD iteration of later solves records
 * events around its rod kernel and its constraint kernel (iterations after
 * convergence are not counted); every = 0 turns it off.  rl_profile_read
 * writes {rod_ms_total, rod_launches, constraint_ms_total,
 * constraint_launches} to out[4] (host) and resets the totals. */
int rl_profile_enable(rl_handle h, int every);
int rl_profile_read(rl_handle h, double *out);


#ifdef __cplusplus
}
#endif

#endif /* RODLCP_H */
