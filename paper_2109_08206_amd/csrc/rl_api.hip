// C-ABI entry points of librodlcp: argument checks, handle and workspace
// management, and the order of kernel launches of each call.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <new>

#include "rl_internal.hpp"

namespace rl {

static thread_local char g_last_error[512] = "";

// The scratch array of the allocation-free entry point (rl_solve_lcp_noalloc).
// Every device the library runs on holds one copy of it, at its own address,
// for the life of the process.  In host code `scratch` names a host-side
// stand-in, never the device memory: the device address comes from
// hipGetSymbolAddress, taken once per device (scratch_of) with that device
// current, and is the only one host code passes on.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};

// the device address of the current device's scratch array (dev is current)
static int scratch_of(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the scratch table", dev);
        return RL_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
            return RL_ERR_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = (char *)g_scratch_dev[dev];
    return RL_OK;
}

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void *ws_get(rl_ctx *h, int s, size_t bytes, int *err)
{
    if (s < 0 || s >= kWsCount) {
        set_error("internal: workspace slot %d out of range", s);
        *err = RL_ERR_ARG;
        return nullptr;
    }
    if (bytes == 0) bytes = 8;
    if (h->arena_on) {
        // allocation-free call: the next 256-byte aligned piece of the scratch array
        const size_t off = (h->arena_used + 255) & ~(size_t)255;
        if (off > kScratchBytes || bytes > kScratchBytes - off) {
            set_error("the problem needs more than the %zu bytes of the allocation-free scratch array",
                      kScratchBytes);
            *err = RL_ERR_ARG;
            return nullptr;
        }
        h->arena_used = off + bytes;
        return h->scratch + off;
    }
    if (h->cap[s] >= bytes) return h->buf[s];
    if (h->buf[s]) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->buf[s]);
        h->buf[s] = nullptr;
        h->cap[s] = 0;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 255) & ~(size_t)255;
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        set_error("workspace allocation of %zu bytes failed", want);
        *err = RL_ERR_NOMEM;
        return nullptr;
    }
    h->buf[s] = p;
    h->cap[s] = want;
    return p;
}

void *ws_get_host(rl_ctx *h, size_t bytes, int *err)
{
    if (bytes == 0) bytes = 8;
    if (h->host_cap >= bytes) return h->host_buf;
    if (h->host_buf) {
        (void)hipStreamSynchronize(h->stream);
        if (h->own_stream) (void)hipStreamSynchronize(h->own_stream);
        (void)hipHostFree(h->host_buf);
        h->host_buf = nullptr;
        h->host_cap = 0;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("pinned host allocation of %zu bytes failed", bytes);
        *err = RL_ERR_NOMEM;
        return nullptr;
    }
    h->host_buf = p;
    h->host_cap = bytes;
    return p;
}

static int check_params(const rl_params *p)
{
    if (!p) {
        set_error("params is NULL");
        return RL_ERR_ARG;
    }
    for (int a = 0; a < 3; ++a)
        if (!(p->box[a] > 0.0) || !std::isfinite(p->box[a])) {
            set_error("box edges must be finite and > 0");
            return RL_ERR_ARG;
        }
    if (!(p->diam > 0.0) || !(p->cutoff >= 0.0) || !(p->eta > 0.0) || !(p->dt > 0.0) || !(p->tol >= 0.0) ||
        !std::isfinite(p->diam) || !std::isfinite(p->cutoff) || !std::isfinite(p->eta) || !std::isfinite(p->dt)) {
        set_error("need diam > 0, cutoff >= 0, eta > 0, dt > 0, tol >= 0");
        return RL_ERR_ARG;
    }
    if (p->max_iter < 0 || p->check_every < 0) {
        set_error("max_iter and check_every must be >= 0");
        return RL_ERR_ARG;
    }
    if (p->precision != RL_FP64 && p->precision != RL_FP32_MIXED) {
        set_error("unknown precision %d", p->precision);
        return RL_ERR_ARG;
    }
    return RL_OK;
}

__global__ void k_invert_perm(int64_t n, const int *__restrict__ perm, int *__restrict__ inv)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < n) inv[perm[t]] = (int)t;
}

// One step with links and/or walls: the contacts, the links and the wall
// constraints of the rods in cell order, concatenated in that order, solved
// as one general problem.
static int step_general(rl_ctx *h, int64_t n, double *x, double *quat, const double *len, double len0,
                        const double *F, double *U, rl_solve_info *info, int64_t *n_pairs, const rl_step_extra *ex)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    if (p.precision != RL_FP64) {
        set_error("rl_step: links and walls need RL_FP64");
        return RL_ERR_ARG;
    }
    WallSet W;
    int rc = wall_set(ex->n_walls, ex->walls, &W);
    if (rc) return rc;
    const rl_links *lk = ex->links;
    const int64_t nl = lk ? lk->n_links : 0;
    if (nl < 0 || nl >= 0x7fffffff || (nl > 0 && (!lk->p || !lk->q || !lk->arm || !lk->kappa || !lk->rest))) {
        set_error("rl_step: bad links");
        return RL_ERR_ARG;
    }
    int err = 0;
    double *dir = (double *)ws_get(h, kWsDir, sizeof(double) * 3 * n, &err);
    if (err) return err;
    RL_HIP(launch_directors(st, n, quat, dir));
    if (ex->noise && ex->kT > 0.0) {
        // F_nc = F + the Brownian force, caller order
        double *Ftot = (double *)ws_get(h, kWsFtot, sizeof(double) * 6 * n, &err);
        if (err) return err;
        RL_HIP(launch_brownian(st, n, dir, len, len0, p.diam, p.eta, p.dt, ex->kT, ex->noise, F, Ftot));
        F = Ftot;
    }
    int64_t np = 0;
    const int *perm = nullptr;
    const double *xs = nullptr, *ds = nullptr, *ls = nullptr;
    rc = build_pairs_sorted(h, n, x, dir, len, len0, &np, &perm, &xs, &ds, &ls);
    if (rc) return rc;
    if (n_pairs) *n_pairs = np;
    const double *lsv = len ? ls : nullptr;
    double *Fs = F ? (double *)ws_get(h, kWsFs, sizeof(double) * 6 * n, &err) : nullptr;
    double *Unc = (double *)ws_get(h, kWsStepUnc, sizeof(double) * 6 * n, &err);
    int *inv = (int *)ws_get(h, kWsInvPerm, sizeof(int) * n, &err);
    double *Uw = U ? U : (double *)ws_get(h, kWsStepU, sizeof(double) * 6 * n, &err);
    if (err) return err;
    if (F) {
        RL_HIP(launch_gather6(st, n, perm, F, Fs));
        RL_HIP(launch_unc(st, n, ds, lsv, len0, p.diam, p.eta, Fs, Unc));
    } else {
        RL_HIP(hipMemsetAsync(Unc, 0, sizeof(double) * 6 * n, st));
    }
    // wall contacts: count first (sizes the concatenated list)
    int64_t nw = 0;
    rc = walls_impl(h, n, xs, ds, lsv, len0, Unc, W, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &nw);
    if (rc && rc != RL_ERR_CAPACITY) return rc;
    if (ex->n_wall_contacts) *ex->n_wall_contacts = nw;
    const int64_t nc = np + nl + nw;
    if (nc >= 0x7fffffff) {
        set_error("rl_step: too many constraints");
        return RL_ERR_CAPACITY;
    }
    const int64_t nb = nc > 0 ? nc : 1;
    int32_t *cpi = (int32_t *)ws_get(h, kWsCatPi, sizeof(int32_t) * nb, &err);
    int32_t *cpj = (int32_t *)ws_get(h, kWsCatPj, sizeof(int32_t) * nb, &err);
    double *ce = (double *)ws_get(h, kWsCatE, sizeof(double) * 3 * nb, &err);
    double *carm = (double *)ws_get(h, kWsCatArm, sizeof(double) * 2 * nb, &err);
    double *cq = (double *)ws_get(h, kWsCatQ, sizeof(double) * nb, &err);
    uint8_t *ckind = (uint8_t *)ws_get(h, kWsCatKind, (size_t)nb, &err);
    double *ccmp = (double *)ws_get(h, kWsCatCmp, sizeof(double) * nb, &err);
    double *cgam = (double *)ws_get(h, kWsStepGamma, sizeof(double) * nb, &err);
    double *phi = (double *)ws_get(h, kWsStepPhi, sizeof(double) * (np > 0 ? np : 1), &err);
    double *llen = (double *)ws_get(h, kWsLinkLen, sizeof(double) * (nl > 0 ? nl : 1), &err);
    if (err) return err;
    if (np > 0) {
        RL_HIP(hipMemcpyAsync(cpi, h->buf[kWsStepPi], sizeof(int32_t) * np, hipMemcpyDeviceToDevice, st));
        RL_HIP(hipMemcpyAsync(cpj, h->buf[kWsStepPj], sizeof(int32_t) * np, hipMemcpyDeviceToDevice, st));
        rc = assemble_impl(h, n, xs, ds, lsv, len0, np, (const int32_t *)h->buf[kWsStepPi],
                           (const int32_t *)h->buf[kWsStepPj], (const int32_t *)h->buf[kWsStepImg], Fs, phi, ce, carm,
                           cq);
        if (rc) return rc;
        RL_HIP(hipMemsetAsync(ckind, 0, (size_t)np, st));
    }
    if (nl > 0) {
        hipLaunchKernelGGL(k_invert_perm, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, perm,
                           inv);
        RL_HIP(hipGetLastError());
        RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int), st));
        RL_HIP(launch_links(st, nl, n, xs, ds, inv, lk, p.box, p.dt, Unc, cpi + np, cpj + np, llen, ce + 3 * np,
                            carm + 2 * np, cq + np, ccmp + np, nullptr, h->flag_dev));
        RL_HIP(hipMemcpyAsync(h->host_scratch, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
        RL_HIP(hipStreamSynchronize(st));
        if (((int *)h->host_scratch)[0]) {
            set_error("rl_step: a link has a rod index outside [0, n), p == q, kappa <= 0, a bad rest length or no "
                      "anchor");
            return RL_ERR_ARG;
        }
        RL_HIP(hipMemsetAsync(ckind + np, 1, (size_t)nl, st));
    }
    if (nw > 0) {
        int64_t nw2 = 0;
        rc = walls_impl(h, n, xs, ds, lsv, len0, Unc, W, nw, cpi + np + nl, ce + 3 * (np + nl), carm + 2 * (np + nl),
                        nullptr, cq + np + nl, nullptr, &nw2);
        if (rc) return rc;
        RL_HIP(hipMemsetAsync(cpj + np + nl, 0xff, sizeof(int32_t) * nw, st));  // -1: no Q side
        RL_HIP(hipMemsetAsync(ckind + np + nl, 0, (size_t)nw, st));
    }
    const StepList L{n, np, nl, nc, perm, cpi, cpj, (const int32_t *)h->buf[kWsStepImg], ds, ce, carm, phi, llen,
                     lk ? lk->key : nullptr};
    if (ex->warm_start) {
        rc = warm_lookup(h, L, cgam);
        if (rc) return rc;
    } else {
        RL_HIP(hipMemsetAsync(cgam, 0, sizeof(double) * nb, st));
    }
    SolveArgs a;
    const int *ord = nullptr;
    rc = prepare_general(h, n, ds, lsv, len0, nc, cpi, cpj, ce, carm, cq, ckind, ccmp, cgam, true, &a, &ord);
    if (rc) return rc;
    rc = solve_impl(h, a, F, Uw, nullptr, info, perm);
    if (rc < 0) return rc;
    // the forces back in input order: contacts, links, walls
    RL_HIP(launch_scatter_gamma(st, a, ord, cgam));
    if (ex->gamma_links && nl > 0)
        RL_HIP(hipMemcpyAsync(ex->gamma_links, cgam + np, sizeof(double) * nl, hipMemcpyDeviceToDevice, st));
    if (ex->warm_start) {
        const int rcw = warm_store(h, L, cgam);
        if (rcw) return rcw;
    }
    if (ex->stress) {
        const int rcs = step_stress(h, L, cgam, ex->stress);
        if (rcs) return rcs;
    }
    const int rc2 = integrate_impl(h, n, Uw, x, quat, ex->x_unwrapped);
    if (rc2) return rc2;
    RL_HIP(hipStreamSynchronize(st));
    return rc;
}

}  // namespace rl

using namespace rl;

#define RL_CHECK_HANDLE(h)                      \
    do {                                        \
        if (!(h)) {                             \
            set_error("handle is NULL");        \
            return RL_ERR_ARG;                  \
        }                                       \
        RL_HIP(hipSetDevice((h)->device));      \
    } while (0)

#define RL_REQUIRE(cond, msg)     \
    do {                          \
        if (!(cond)) {            \
            set_error("%s", msg); \
            return RL_ERR_ARG;    \
        }                         \
    } while (0)

extern "C" {

const char *rl_status_str(int status)
{
    switch (status) {
    case RL_OK: return "ok";
    case RL_NOT_CONVERGED: return "not converged (iteration cap reached)";
    case RL_STAGNATED: return "stagnated (no progress above tolerance)";
    case RL_ERR_ARG: return "invalid argument";
    case RL_ERR_CAPACITY: return "pair capacity too small";
    case RL_ERR_NONFINITE: return "non-finite value";
    case RL_ERR_HIP: return "HIP runtime error";
    case RL_ERR_NOMEM: return "out of device memory";
    default: return "unknown status";
    }
}

const char *rl_last_error(void) { return g_last_error; }

int rl_create(rl_handle *out, const rl_params *prm)
{
    if (!out) {
        set_error("rl_create: out is NULL");
        return RL_ERR_ARG;
    }
    *out = nullptr;
    int rc = check_params(prm);
    if (rc) return rc;
    rl_ctx *h = new (std::nothrow) rl_ctx();
    if (!h) return RL_ERR_NOMEM;
    h->prm = *prm;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_error("rl_create: no HIP device");
        return RL_ERR_HIP;
    }
    if (hipMalloc(&h->state, sizeof(SolverState)) != hipSuccess ||
        hipMalloc(&h->flag_dev, sizeof(int) * 4) != hipSuccess ||
        hipHostMalloc(&h->state_host, sizeof(SolverState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&h->host_scratch, sizeof(int64_t) * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&h->progress_host, 64, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&h->progress_dev, h->progress_host, 0) != hipSuccess ||
        hipEventCreateWithFlags(&h->chk_ev, hipEventDisableTiming) != hipSuccess) {
        set_error("rl_create: allocation failed");
        rl_destroy(h);
        return RL_ERR_NOMEM;
    }
    rc = scratch_of(h->device, &h->scratch);
    if (rc) {
        const std::string msg = rl_last_error();
        rl_destroy(h);
        set_error("%s", msg.c_str());
        return rc;
    }
    memset(h->state_host, 0, sizeof(SolverState));
    *out = h;
    return RL_OK;
}

int rl_destroy(rl_handle h)
{
    if (!h) return RL_OK;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (int v = 0; v < rl_ctx::kMaxEv; ++v)
        for (int k = 0; k < 4; ++k)
            if (h->ev[v][k]) (void)hipEventDestroy(h->ev[v][k]);
    if (h->chk_ev) (void)hipEventDestroy(h->chk_ev);
    for (int s = 0; s < rl_ctx::kSlots; ++s)
        if (h->buf[s]) (void)hipFree(h->buf[s]);
    if (h->state) (void)hipFree(h->state);
    if (h->flag_dev) (void)hipFree(h->flag_dev);
    if (h->state_host) (void)hipHostFree(h->state_host);
    if (h->host_scratch) (void)hipHostFree(h->host_scratch);
    if (h->progress_host) (void)hipHostFree(h->progress_host);
    if (h->host_buf) (void)hipHostFree(h->host_buf);
    if (h->own_stream) {
        (void)hipStreamSynchronize(h->own_stream);
        (void)hipStreamDestroy(h->own_stream);
    }
    delete h;
    return RL_OK;
}

int rl_set_params(rl_handle h, const rl_params *prm)
{
    if (!h) return RL_ERR_ARG;
    int rc = check_params(prm);
    if (rc) return rc;
    h->prm = *prm;
    return RL_OK;
}

int rl_get_params(rl_handle h, rl_params *prm)
{
    if (!h || !prm) return RL_ERR_ARG;
    *prm = h->prm;
    return RL_OK;
}

int rl_set_stream(rl_handle h, void *stream)
{
    if (!h) return RL_ERR_ARG;
    h->stream = (hipStream_t)stream;
    return RL_OK;
}

int rl_reserve(rl_handle h, int64_t max_rods, int64_t max_pairs)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(max_rods >= 0 && max_pairs >= 0 && max_pairs < 0x7fffffff, "rl_reserve: bad sizes");
    int err = 0;
    const int64_t n = max_rods > 0 ? max_rods : 1, nc = max_pairs > 0 ? max_pairs : 1;
    const size_t sz[][2] = {
        {kWsDir, sizeof(double) * 3 * n},  {kWsCoef, sizeof(double) * 3 * n},  {kWsV, sizeof(double) * 6 * n},
        {kWsUnc, sizeof(double) * 6 * n},  {kWsPptr, sizeof(int) * (n + 1)},   {kWsQptr, sizeof(int) * (n + 1)},
        {kWsQidx, sizeof(int) * nc},       {kWsQcnt, sizeof(int) * n},         {kWsG, sizeof(double) * nc},
        {kWsPartial, sizeof(double) * 8 * kConGridMax},
        {kWsCellOf, sizeof(int) * n},      {kWsSorted, sizeof(int) * n},       {kWsXs, sizeof(double) * 3 * n},
        {kWsDs, sizeof(double) * 3 * n},   {kWsLs, sizeof(double) * n},        {kWsPcnt, sizeof(int) * n},
        {kWsPoff, sizeof(int) * (n + 1)},  {kWsStepPi, sizeof(int) * nc},      {kWsStepPj, sizeof(int) * nc},
        {kWsStepImg, sizeof(int) * nc},    {kWsStepFlags, (size_t)nc},                 {kWsStepPhi, sizeof(double) * nc},
        {kWsStepE, sizeof(double) * 3 * nc}, {kWsStepArm, sizeof(double) * 2 * nc},
        {kWsStepQ, sizeof(double) * nc},   {kWsStepGamma, sizeof(double) * nc}, {kWsStepU, sizeof(double) * 6 * n},
        {kWsPP, sizeof(int) * 2 * nc},     {kWsGeo, sizeof(double) * 4 * nc}, {kWsGeo2, sizeof(double) * 2 * nc},  {kWsSt, sizeof(double) * 2 * nc},
        {kWsAlpha, sizeof(double) * 2},    {kWsQpos, sizeof(int) * nc},        {kWsQgeo, sizeof(double) * 4 * nc},
        {kWsStq, sizeof(double) * 2 * nc},
    };
    for (auto &e : sz) {
        ws_get(h, (int)e[0], e[1], &err);
        if (err) return err;
    }
    return RL_OK;
}

int rl_directors(rl_handle h, int64_t n, const double *quat, double *dir)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0, "rl_directors: n < 0");
    RL_REQUIRE(n == 0 || (quat && dir), "rl_directors: NULL array");
    RL_HIP(launch_directors(h->stream, n, quat, dir));
    return RL_OK;
}

int rl_build_pairs(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                   int64_t capacity, int32_t *pi, int32_t *pj, int32_t *img, uint8_t *flags, int64_t *n_pairs)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff, "rl_build_pairs: bad n");
    RL_REQUIRE(capacity >= 0, "rl_build_pairs: capacity < 0");
    RL_REQUIRE(n == 0 || (x && dir), "rl_build_pairs: NULL x or dir");
    RL_REQUIRE(capacity == 0 || (pi && pj && img && flags), "rl_build_pairs: NULL output list");
    return build_pairs_impl(h, n, x, dir, len, len0, capacity, pi, pj, img, flags, n_pairs);
}

int rl_assemble_D(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                  int64_t nc, const int32_t *pi, const int32_t *pj, const int32_t *img, const double *F,
                  double *phi, double *e, double *arm, double *q)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff && nc >= 0 && nc < 0x7fffffff, "rl_assemble_D: bad sizes");
    RL_REQUIRE(nc == 0 || (x && dir && pi && pj && img && phi && e && arm && q), "rl_assemble_D: NULL array");
    RL_REQUIRE(len || len0 > 0.0, "rl_assemble_D: len0 must be > 0 when len is NULL");
    return assemble_impl(h, n, x, dir, len, len0, nc, pi, pj, img, F, phi, e, arm, q);
}

int rl_apply_M(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
               const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
               const double *gamma, double *w)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff && nc >= 0 && nc < 0x7fffffff, "rl_apply_M: bad sizes");
    RL_REQUIRE(nc == 0 || (dir && pi && pj && e && arm && gamma && w), "rl_apply_M: NULL array");
    RL_REQUIRE(len || len0 > 0.0, "rl_apply_M: len0 must be > 0 when len is NULL");
    SolveArgs a;
    int rc = prepare_solve(h, n, dir, len, len0, nc, pi, pj, e, arm, q, const_cast<double *>(gamma), &a);
    if (rc) return rc;
    rc = apply_impl(h, a, w);
    if (rc) return rc;
    RL_HIP(hipStreamSynchronize(h->stream));
    return RL_OK;
}

int rl_solve_lcp(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                 const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                 const double *F, double *gamma, double *U, rl_solve_info *info)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff && nc >= 0 && nc < 0x7fffffff, "rl_solve_lcp: bad sizes");
    RL_REQUIRE(nc == 0 || (dir && pi && pj && e && arm && q && gamma), "rl_solve_lcp: NULL array");
    RL_REQUIRE(n == 0 || dir || !U, "rl_solve_lcp: NULL dir");
    RL_REQUIRE(len || len0 > 0.0, "rl_solve_lcp: len0 must be > 0 when len is NULL");
    SolveArgs a;
    int rc = prepare_solve(h, n, dir, len, len0, nc, pi, pj, e, arm, q, gamma, &a);
    if (rc) return rc;
    return solve_impl(h, a, F, U, gamma, info);
}

int rl_solve_lcp_noalloc(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                         const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                         const double *F, double *gamma, double *U, rl_solve_info *info)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff && nc >= 0 && nc < 0x7fffffff, "rl_solve_lcp_noalloc: bad sizes");
    RL_REQUIRE(nc == 0 || (dir && pi && pj && e && arm && q && gamma), "rl_solve_lcp_noalloc: NULL array");
    RL_REQUIRE(n == 0 || dir || !U, "rl_solve_lcp_noalloc: NULL dir");
    RL_REQUIRE(len || len0 > 0.0, "rl_solve_lcp_noalloc: len0 must be > 0 when len is NULL");
    RL_REQUIRE(h->prm.precision == RL_FP64, "rl_solve_lcp_noalloc: RL_FP64 only");
    RL_REQUIRE(h->scratch != nullptr, "rl_solve_lcp_noalloc: no scratch array on this device");
    // every workspace piece comes from the scratch array (prepare_solve takes
    // them all before it launches anything, so an oversized problem fails
    // with nothing enqueued)
    struct Arena {
        rl_ctx *h;
        explicit Arena(rl_ctx *c) : h(c) { h->arena_on = true; h->arena_used = 0; }
        ~Arena() { h->arena_on = false; }
    } arena(h);
    SolveArgs a;
    int rc = prepare_solve(h, n, dir, len, len0, nc, pi, pj, e, arm, q, gamma, &a);
    if (rc) return rc;
    return solve_impl(h, a, F, U, gamma, info);
}

int rl_step(rl_handle h, int64_t n, double *x, double *quat, const double *len, double len0, const double *F,
            double *U, rl_solve_info *info, int64_t *n_pairs, double *gamma_tape, int64_t tape_len,
            int32_t tape_mode, const rl_step_extra *extra)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff, "rl_step: bad n");
    RL_REQUIRE(n == 0 || (x && quat), "rl_step: NULL x or quat");
    RL_REQUIRE(len || len0 > 0.0, "rl_step: len0 must be > 0 when len is NULL");
    RL_REQUIRE(tape_mode == RL_TAPE_NONE || tape_mode == RL_TAPE_RECORD || tape_mode == RL_TAPE_REPLAY,
               "rl_step: bad tape_mode");
    RL_REQUIRE(tape_mode == RL_TAPE_NONE || tape_len >= 0, "rl_step: tape_len < 0");
    if (n == 0) {
        if (n_pairs) *n_pairs = 0;
        if (info) *info = rl_solve_info{0, 0.0, 0.0, RL_OK, 0};
        if (extra && extra->n_wall_contacts) *extra->n_wall_contacts = 0;
        return RL_OK;
    }
    if (extra && ((extra->links && extra->links->n_links > 0) || extra->n_walls > 0)) {
        RL_REQUIRE(tape_mode == RL_TAPE_NONE, "rl_step: no gamma tape with links or walls");
        return step_general(h, n, x, quat, len, len0, F, U, info, n_pairs, extra);
    }
    if (extra && extra->n_wall_contacts) *extra->n_wall_contacts = 0;
    const bool warm = extra && extra->warm_start;
    RL_REQUIRE(!warm || tape_mode == RL_TAPE_NONE, "rl_step: warm start and gamma tape exclude each other");
    int err = 0;
    double *dir = (double *)ws_get(h, kWsDir, sizeof(double) * 3 * n, &err);
    if (err) return err;
    RL_HIP(launch_directors(h->stream, n, quat, dir));
    if (extra && extra->noise && extra->kT > 0.0) {
        // F_nc = F + the Brownian force, caller order
        double *Ftot = (double *)ws_get(h, kWsFtot, sizeof(double) * 6 * n, &err);
        if (err) return err;
        RL_HIP(launch_brownian(h->stream, n, dir, len, len0, h->prm.diam, h->prm.eta, h->prm.dt, extra->kT,
                               extra->noise, F, Ftot));
        F = Ftot;
    }
    // pairs with the rods renumbered in cell order: the solver then reads
    // neighbouring rods and constraints from neighbouring memory
    int64_t np = 0;
    const int *perm = nullptr;
    const double *xs = nullptr, *ds = nullptr, *ls = nullptr;
    int rc = build_pairs_sorted(h, n, x, dir, len, len0, &np, &perm, &xs, &ds, &ls);
    if (rc) return rc;
    if (n_pairs) *n_pairs = np;
    if (tape_mode == RL_TAPE_RECORD && np > tape_len) {
        set_error("rl_step: tape holds %lld values, the step has %lld constraints", (long long)tape_len,
                  (long long)np);
        return RL_ERR_CAPACITY;
    }
    if (tape_mode == RL_TAPE_REPLAY && np != tape_len) {
        set_error("rl_step: tape of %lld values replayed on a step with %lld constraints", (long long)tape_len,
                  (long long)np);
        return RL_ERR_ARG;
    }
    RL_REQUIRE(tape_mode == RL_TAPE_NONE || np == 0 || gamma_tape, "rl_step: NULL gamma_tape");
    const int64_t nb = np > 0 ? np : 1;
    double *phi = (double *)ws_get(h, kWsStepPhi, sizeof(double) * nb, &err);
    double *e = (double *)ws_get(h, kWsStepE, sizeof(double) * 3 * nb, &err);
    double *arm = (double *)ws_get(h, kWsStepArm, sizeof(double) * 2 * nb, &err);
    double *q = (double *)ws_get(h, kWsStepQ, sizeof(double) * nb, &err);
    double *gamma = (double *)ws_get(h, kWsStepGamma, sizeof(double) * nb, &err);
    double *Fs = F ? (double *)ws_get(h, kWsFs, sizeof(double) * 6 * n, &err) : nullptr;
    double *Uw = U ? U : (double *)ws_get(h, kWsStepU, sizeof(double) * 6 * n, &err);
    if (err) return err;
    if (F) RL_HIP(launch_gather6(h->stream, n, perm, F, Fs));
    const double *lsv = len ? ls : nullptr;
    const int32_t *pi = (const int32_t *)h->buf[kWsStepPi], *pj = (const int32_t *)h->buf[kWsStepPj];
    const int32_t *img = (const int32_t *)h->buf[kWsStepImg];
    rc = assemble_impl(h, n, xs, ds, lsv, len0, np, pi, pj, img, Fs, phi, e, arm, q);
    if (rc) return rc;
    const StepList L{n, np, 0, np, perm, pi, pj, img, ds, e, arm, phi, nullptr, nullptr};
    if (tape_mode == RL_TAPE_REPLAY && np > 0) {
        RL_HIP(hipMemcpyAsync(gamma, gamma_tape, sizeof(double) * np, hipMemcpyDeviceToDevice, h->stream));
    } else if (warm) {
        rc = warm_lookup(h, L, gamma);
        if (rc) return rc;
    } else {
        RL_HIP(hipMemsetAsync(gamma, 0, sizeof(double) * nb, h->stream));
    }
    SolveArgs a;
    rc = prepare_solve(h, n, ds, lsv, len0, np, pi, pj, e, arm, q, gamma, &a, true);
    if (rc) return rc;
    rc = solve_impl(h, a, F, Uw, tape_mode != RL_TAPE_NONE && np > 0 ? gamma_tape : gamma, info, perm);
    if (rc < 0) return rc;
    // gamma (or the tape) holds the forces in the step's constraint order
    const double *gsol = tape_mode != RL_TAPE_NONE && np > 0 ? gamma_tape : gamma;
    if (warm) {
        const int rcw = warm_store(h, L, gsol);
        if (rcw) return rcw;
    }
    if (extra && extra->stress) {
        const int rcs = step_stress(h, L, gsol, extra->stress);
        if (rcs) return rcs;
    }
    const int rc2 = integrate_impl(h, n, Uw, x, quat, extra ? extra->x_unwrapped : nullptr);
    if (rc2) return rc2;
    RL_HIP(hipStreamSynchronize(h->stream));
    return rc;
}

int rl_solve_lcp_adjoint(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                         const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                         const double *F, const double *gamma, const double *U_bar, double cg_tol, double *q_bar,
                         double *e_bar, double *arm_bar, double *F_bar, double *dir_bar, rl_adjoint_info *info)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff && nc >= 0 && nc < 0x7fffffff, "rl_solve_lcp_adjoint: bad sizes");
    RL_REQUIRE(nc == 0 || (pi && pj && e && arm && q && gamma && q_bar && e_bar && arm_bar),
               "rl_solve_lcp_adjoint: NULL constraint array");
    RL_REQUIRE(n == 0 || (dir && U_bar && F_bar && dir_bar), "rl_solve_lcp_adjoint: NULL rod array");
    RL_REQUIRE(len || len0 > 0.0, "rl_solve_lcp_adjoint: len0 must be > 0 when len is NULL");
    if (info) *info = rl_adjoint_info{0, 0.0, 0, RL_OK, RL_OK, 0, 0.0};
    if (n == 0) return RL_OK;
    SolveArgs a;
    int rc = prepare_solve(h, n, dir, len, len0, nc, pi, pj, e, arm, q, const_cast<double *>(gamma), &a);
    if (rc) return rc;
    int err = 0;
    double *dmob = (double *)ws_get(h, kWsAdjDmob, sizeof(double) * 3 * n, &err);
    double *d_bar = (double *)ws_get(h, kWsAdjDbar, sizeof(double) * 6 * (nc > 0 ? nc : 1), &err);
    if (err) return err;
    AdjOut o{F_bar, q_bar, e_bar, arm_bar, d_bar, dmob};
    rl_adjoint_info ai{0, 0.0, 0, RL_OK, RL_OK, 0, 0.0};
    rc = adjoint_core(h, a, false, U_bar, F, nullptr, cg_tol, o, &ai);
    if (rc < 0) return rc;
    RL_HIP(launch_dir_bar(h->stream, a, dmob, d_bar, dir_bar));
    RL_HIP(hipStreamSynchronize(h->stream));
    if (info) *info = ai;
    return rc;
}

int rl_step_adjoint(rl_handle h, int64_t n, const double *x, const double *quat, const double *len, double len0,
                    const double *F, const double *gamma_tape, int64_t tape_len, double *x_bar, double *quat_bar,
                    double *F_bar, double cg_tol, rl_adjoint_info *info)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(n >= 0 && n < 0x7fffffff, "rl_step_adjoint: bad n");
    RL_REQUIRE(n == 0 || (x && quat && x_bar && quat_bar && F_bar), "rl_step_adjoint: NULL array");
    RL_REQUIRE(len || len0 > 0.0, "rl_step_adjoint: len0 must be > 0 when len is NULL");
    if (info) *info = rl_adjoint_info{0, 0.0, 0, RL_OK, RL_OK, 0, 0.0};
    if (n == 0) return RL_OK;
    hipStream_t st = h->stream;
    int err = 0;
    double *dir = (double *)ws_get(h, kWsDir, sizeof(double) * 3 * n, &err);
    if (err) return err;
    RL_HIP(launch_directors(st, n, quat, dir));
    // the forward step, as rl_step takes it (rods in cell order)
    int64_t np = 0;
    const int *perm = nullptr;
    const double *xs = nullptr, *ds = nullptr, *ls = nullptr;
    int rc = build_pairs_sorted(h, n, x, dir, len, len0, &np, &perm, &xs, &ds, &ls);
    if (rc) return rc;
    if (gamma_tape && tape_len != np) {
        set_error("rl_step_adjoint: tape of %lld values for a step with %lld constraints", (long long)tape_len,
                  (long long)np);
        return RL_ERR_ARG;
    }
    const int64_t nb = np > 0 ? np : 1;
    double *phi = (double *)ws_get(h, kWsStepPhi, sizeof(double) * nb, &err);
    double *e = (double *)ws_get(h, kWsStepE, sizeof(double) * 3 * nb, &err);
    double *arm = (double *)ws_get(h, kWsStepArm, sizeof(double) * 2 * nb, &err);
    double *q = (double *)ws_get(h, kWsStepQ, sizeof(double) * nb, &err);
    double *gamma = (double *)ws_get(h, kWsStepGamma, sizeof(double) * nb, &err);
    double *Fs = F ? (double *)ws_get(h, kWsFs, sizeof(double) * 6 * n, &err) : nullptr;
    double *Uc = (double *)ws_get(h, kWsStepU, sizeof(double) * 6 * n, &err);
    double *Ubar = (double *)ws_get(h, kWsAdjUbar, sizeof(double) * 6 * n, &err);
    double *qbd = (double *)ws_get(h, kWsAdjQbd, sizeof(double) * 4 * n, &err);
    double *dmob = (double *)ws_get(h, kWsAdjDmob, sizeof(double) * 3 * n, &err);
    double *qbar = (double *)ws_get(h, kWsAdjQbar, sizeof(double) * nb, &err);
    double *ebar = (double *)ws_get(h, kWsAdjEbar, sizeof(double) * 3 * nb, &err);
    double *armbar = (double *)ws_get(h, kWsAdjArmbar, sizeof(double) * 2 * nb, &err);
    double *dbar = (double *)ws_get(h, kWsAdjDbar, sizeof(double) * 6 * nb, &err);
    double *gbar = (double *)ws_get(h, kWsAdjGbar, sizeof(double) * 9 * nb, &err);
    if (err) return err;
    if (F) RL_HIP(launch_gather6(st, n, perm, F, Fs));
    const double *lsv = len ? ls : nullptr;
    const int32_t *pi = (const int32_t *)h->buf[kWsStepPi], *pj = (const int32_t *)h->buf[kWsStepPj];
    const int32_t *img = (const int32_t *)h->buf[kWsStepImg];
    rc = assemble_impl(h, n, xs, ds, lsv, len0, np, pi, pj, img, Fs, phi, e, arm, q);
    if (rc) return rc;
    if (gamma_tape && np > 0)
        RL_HIP(hipMemcpyAsync(gamma, gamma_tape, sizeof(double) * np, hipMemcpyDeviceToDevice, st));
    else
        RL_HIP(hipMemsetAsync(gamma, 0, sizeof(double) * nb, st));
    SolveArgs a;
    rc = prepare_solve(h, n, ds, lsv, len0, np, pi, pj, e, arm, q, gamma, &a, true);
    if (rc) return rc;
    rl_solve_info si{0, 0.0, 0.0, RL_OK, 0};
    const int src = solve_impl(h, a, F, Uc, nullptr, &si, perm);
    if (src < 0) return src;
    // adjoint: Euler update, then the solve, then the geometry
    RL_HIP(launch_integrate_adj(st, n, perm, x_bar, quat_bar, quat, Uc, h->prm.dt, Ubar, qbd));
    AdjOut o{F_bar, qbar, ebar, armbar, dbar, dmob};
    rl_adjoint_info ai{0, 0.0, 0, RL_OK, RL_OK, 0, 0.0};
    rc = adjoint_core(h, a, true, Ubar, F, perm, cg_tol, o, &ai);
    if (rc < 0) return rc;
    RL_HIP(launch_geo_adjoint(st, np, xs, ds, lsv, len0, h->prm.box, pi, pj, img, h->prm.dt, qbar, ebar, armbar, dbar,
                              gbar));
    RL_HIP(launch_step_bar(st, a, perm, gbar, dmob, qbd, quat, x_bar, quat_bar));
    RL_HIP(hipStreamSynchronize(st));
    ai.solve_status = si.status;
    ai.solve_iterations = si.iterations;
    ai.solve_residual = si.residual;
    if (info) *info = ai;
    return rc;
}

int rl_solve_lcp_batched(rl_handle h, int32_t S, const int64_t *rod_off, const int64_t *pair_off, const double *dir,
                         const double *len, double len0, const int32_t *pi, const int32_t *pj, const double *e,
                         const double *arm, const double *q, const double *F, double *gamma, double *U,
                         rl_solve_info *infos)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(S >= 1 && rod_off && pair_off, "rl_solve_lcp_batched: need S >= 1 and host offsets");
    RL_REQUIRE(rod_off[0] == 0 && pair_off[0] == 0, "rl_solve_lcp_batched: offsets must start at 0");
    for (int s = 0; s < S; ++s)
        RL_REQUIRE(rod_off[s + 1] >= rod_off[s] && pair_off[s + 1] >= pair_off[s],
                   "rl_solve_lcp_batched: offsets must be non-decreasing");
    const int64_t n = rod_off[S], nc = pair_off[S];
    RL_REQUIRE(n < 0x7fffffff && nc < 0x7fffffff, "rl_solve_lcp_batched: sizes overflow int32");
    RL_REQUIRE(nc == 0 || (dir && pi && pj && e && arm && q && gamma), "rl_solve_lcp_batched: NULL array");
    RL_REQUIRE(n == 0 || dir || !U, "rl_solve_lcp_batched: NULL dir");
    RL_REQUIRE(len || len0 > 0.0, "rl_solve_lcp_batched: len0 must be > 0 when len is NULL");
    RL_REQUIRE(h->prm.precision == RL_FP64, "rl_solve_lcp_batched: the batched solve runs in RL_FP64");
    SolveArgs a;
    int rc = prepare_solve(h, n, dir, len, len0, nc, pi, pj, e, arm, q, gamma, &a);
    if (rc) return rc;
    return solve_batched_impl(h, S, rod_off, pair_off, a, pi, pj, e, arm, q, gamma, F, gamma, U, infos);
}

int rl_batch_tuning(rl_handle h, int rod_block, int con_block, int *chosen)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE((rod_block == 0 && con_block == 0) ||
                   ((rod_block == 256 || rod_block == 1024) && (con_block == 256 || con_block == 512)),
               "rl_batch_tuning: rod_block in {256, 1024} and con_block in {256, 512}, or both 0");
    h->batch_rb = rod_block;
    h->batch_cb = con_block;
    if (chosen) {
        chosen[0] = h->batch_rb_used;
        chosen[1] = h->batch_cb_used;
    }
    return RL_OK;
}

int rl_profile_enable(rl_handle h, int every)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(every >= 0, "rl_profile_enable: every < 0");
    h->prof_every = every;
    return RL_OK;
}

int rl_profile_read(rl_handle h, double *out)
{
    RL_CHECK_HANDLE(h);
    RL_REQUIRE(out != nullptr, "rl_profile_read: NULL out");
    out[0] = h->prof_ms[0];
    out[1] = h->prof_cnt[0];
    out[2] = h->prof_ms[1];
    out[3] = h->prof_cnt[1];
    h->prof_ms[0] = h->prof_ms[1] = 0.0;
    h->prof_cnt[0] = h->prof_cnt[1] = 0.0;
    return RL_OK;
}

}  // extern "C"
