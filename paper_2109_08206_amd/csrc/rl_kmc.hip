// Crosslinker kinetics: kinetic Monte Carlo of binding and unbinding
// (Section "2. Crosslinker binding and unbinding", Table tab:rates; appendix
// "Kinetic Monte-Carlo", Table tab:supprates).
//
// Every crosslinker is independent of the others within a step (steric
// interactions between motors are neglected).  The crosslinkers are first
// ordered by (state class, cell of the query point).  A crosslinker with at
// most one head bound gets a wave: its lanes share the filaments of the 27
// cells around the query point (the crosslinker, or its bound head), keep
// those whose axis passes within the query radius, and sum the sites of the
// kept ones; one lane then decides with the crosslinker's uniform numbers
// and, for a binding, walks the kept filaments in index order (inverse
// transform).  A doubly bound crosslinker needs only its two heads: one lane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "rl_vec.hpp"

// the rounding of the rate arithmetic follows the written order
#pragma clang fp contract(off)

namespace rl {

constexpr int kKmcBlock = 64;   // crosslinkers per workgroup of the check

static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct KmcArgs {
    int64_t m, n;
    int32_t *state;
    int32_t *rod;
    double *arc;
    double *xl;
    const double *u, *xi;
    int32_t *event;
    const double *x, *dir, *len;
    double len0;
    int nc[3];
    double cell[3], box[3];
    const int *start, *order;
    const double *xs, *ds, *ls;
    rl_kmc_params P;
    double diam, dt, vbd;
    unsigned long long *counts;  // [5]
};

__device__ __forceinline__ double wrap1(double v, double b)
{
    v -= b * floor(v / b);
    if (v >= b) v -= b;
    return v;
}

__device__ __forceinline__ double rlen(const KmcArgs &A, int64_t i) { return A.len ? A.len[i] : A.len0; }

// the point at arclength s on filament i, wrapped into the box
__device__ __forceinline__ void axis_point(const KmcArgs &A, int64_t i, double s, double p[3])
{
    for (int a = 0; a < 3; ++a) p[a] = wrap1(A.x[3 * i + a] + s * A.dir[3 * i + a], A.box[a]);
}

// centre c (nearest image relative to p) and director d of a filament
__device__ __forceinline__ void centre_rel(const double *xc, const double *box, const double p[3], double c[3])
{
    for (int a = 0; a < 3; ++a) {
        double d = xc[a] - p[a];
        d -= box[a] * floor(d / box[a] + 0.5);
        c[a] = d;
    }
}

// arclength interval of the axis inside the sphere of radius r about p
__device__ __forceinline__ void inside_interval(const double *xc, const double *d, double L, const double *box,
                                                const double p[3], double r, double &lo, double &hi)
{
    double c[3];
    centre_rel(xc, box, p, c);
    const double b = c[0] * d[0] + c[1] * d[1] + c[2] * d[2];
    const double w0 = c[0] - b * d[0], w1 = c[1] - b * d[1], w2 = c[2] - b * d[2];
    const double h2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double half_len = 0.5 * L;
    lo = 0.0;
    hi = 0.0;
    if (h2 >= r * r) return;
    const double half = sqrt(r * r - h2);
    double a0 = -b - half, a1 = -b + half;
    if (a0 < -half_len) a0 = -half_len;
    if (a1 > half_len) a1 = half_len;
    lo = a0;
    hi = a1;
}

__device__ __forceinline__ double stretch_of(const KmcArgs &A, double l) { return l - A.P.rest - A.diam; }

__device__ __forceinline__ double cross_weight(const KmcArgs &A, double l)
{
    const double dl = stretch_of(A, l);
    return exp(-(A.P.kappa / A.P.kT) * (0.5 * (1.0 - A.P.lambda) * dl * dl - A.P.xc * dl));
}

__device__ __forceinline__ double release_rate(const KmcArgs &A, double k0, double l)
{
    const double dl = stretch_of(A, l);
    return k0 * exp((A.P.kappa / A.P.kT) * (0.5 * A.P.lambda * dl * dl + A.P.xc * dl));
}

__device__ __forceinline__ int64_t sites_of(const KmcArgs &A, double L)
{
    const int64_t m = (int64_t)floor(A.P.eps * L);
    return m < 1 ? 1 : m;
}

__device__ __forceinline__ double site_arc(double L, int64_t m, int64_t k) { return -0.5 * L + (k + 0.5) * (L / m); }

// S -> D weight of filament j's sites within r_cd of p, in site order (the
// sites of the axis interval within a slightly larger sphere, each tested
// by its own distance); with pick >= 0 it stops where the running sum first
// exceeds pick and returns that site in *site (else the last counted one).
__device__ double site_sum(const KmcArgs &A, int64_t j, const double p[3], double pick, int64_t *site)
{
    const double L = rlen(A, j);
    const int64_t m = sites_of(A, L);
    const double *xc = A.x + 3 * j, *d = A.dir + 3 * j;
    double lo, hi;
    // the margin keeps every site the distance test accepts inside the range
    inside_interval(xc, d, L, A.box, p, A.P.rcd * (1.0 + 1e-9), lo, hi);
    if (site) *site = -1;
    if (!(hi > lo)) return 0.0;
    const double step = L / m;
    int64_t k0 = (int64_t)floor((lo + 0.5 * L) / step - 0.5) - 1;
    int64_t k1 = (int64_t)ceil((hi + 0.5 * L) / step - 0.5) + 1;
    if (k0 < 0) k0 = 0;
    if (k1 > m - 1) k1 = m - 1;
    double c[3];
    centre_rel(xc, A.box, p, c);
    double sum = 0.0;
    int64_t last = -1;
    for (int64_t k = k0; k <= k1; ++k) {
        const double s = site_arc(L, m, k);
        const double v0 = c[0] + s * d[0], v1 = c[1] + s * d[1], v2 = c[2] + s * d[2];
        const double l = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        if (!(l <= A.P.rcd)) continue;
        sum += cross_weight(A, l);
        last = k;
        if (pick >= 0.0 && sum > pick) break;
    }
    if (site) *site = last;
    return sum;
}

__global__ void __launch_bounds__(kKmcBlock) k_kmc_check(KmcArgs A, int *__restrict__ flag)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= A.m) return;
    const int s = A.state[c];
    const int ra = A.rod[2 * c], rb = A.rod[2 * c + 1];
    const bool a_ok = ra >= 0 && ra < A.n, b_ok = rb >= 0 && rb < A.n;
    bool ok;
    switch (s) {
    case RL_XL_U: ok = ra == -1 && rb == -1; break;
    case RL_XL_SA: ok = a_ok && rb == -1; break;
    case RL_XL_SB: ok = ra == -1 && b_ok; break;
    case RL_XL_D: ok = a_ok && b_ok && ra != rb; break;
    default: ok = false;
    }
    if (!ok) atomicOr(flag, 1);
}

// Processing order: crosslinkers with one head bound first, then unbound,
// then doubly bound (the three cost very differently), each class by the
// cell of its query point.  heavy[0] counts the first two classes.
__global__ void k_kmc_keys(KmcArgs A, int *__restrict__ key, int *__restrict__ heavy)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= A.m) return;
    const int s = A.state[c];
    int cls = 2;
    double p[3] = {0.0, 0.0, 0.0};
    if (s == RL_XL_SA || s == RL_XL_SB) {
        const int hd = s == RL_XL_SA ? 0 : 1;
        axis_point(A, A.rod[2 * c + hd], A.arc[2 * c + hd], p);
        cls = 0;
    } else if (s == RL_XL_U) {
        for (int a = 0; a < 3; ++a) p[a] = wrap1(A.xl[3 * c + a], A.box[a]);
        cls = 1;
    }
    int id = 0;
    if (cls < 2) {
        int k[3];
        for (int a = 0; a < 3; ++a) {
            int v = (int)floor(p[a] / A.cell[a]);
            k[a] = v < 0 ? 0 : (v >= A.nc[a] ? A.nc[a] - 1 : v);
        }
        id = (k[0] * A.nc[1] + k[1]) * A.nc[2] + k[2];
        atomicAdd(heavy, 1);
    }
    key[c] = (cls << 26) | id;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Crosslinkers without both heads bound: one wave each (a 64-thread
// workgroup), its lanes sharing the candidate filaments of the 27 cells
// around the query point.  A candidate is kept when its axis passes within
// the query radius; the kept ones go to an LDS list, sorted by filament
// index, over which the rate is summed and the binding walks, in the order
// the method defines.  The S -> D weight of a kept filament is summed over
// its sites by all lanes.
constexpr int kNearCap = 128;

__global__ void __launch_bounds__(64) k_kmc_heavy(KmcArgs A, const int *__restrict__ perm, int nheavy,
                                                  int *__restrict__ err)
{
    __shared__ int cstart[27], cpre[28];
    __shared__ int nnear;
    __shared__ int nidx[kNearCap], sidx[kNearCap];
    __shared__ double nw[kNearCap], sw[kNearCap];
    const int lane = threadIdx.x;
    if ((int)blockIdx.x >= nheavy) return;
    const int64_t c = perm[blockIdx.x];
    const rl_kmc_params &P = A.P;
    const double *uc = A.u + 4 * c, *xc = A.xi + 3 * c;
    const int s = A.state[c];
    const bool unb = s == RL_XL_U;
    const int hd = s == RL_XL_SB ? 1 : 0, g = 1 - hd;
    const int own = unb ? -1 : A.rod[2 * c + hd];
    // query point: the diffused crosslinker, or the bound head
    double p[3];
    if (unb) {
        const double hop = sqrt(2.0 * P.dU * A.dt);
        for (int a = 0; a < 3; ++a) p[a] = wrap1(A.xl[3 * c + a] + hop * xc[a], A.box[a]);
    } else {
        axis_point(A, own, A.arc[2 * c + hd], p);
    }
    const double r = unb ? P.rcs : P.rcd;
    // the distinct cells around p (fewer than 27 when a direction has < 3)
    int lo[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
        int v = (int)floor(p[a] / A.cell[a]);
        v = v < 0 ? 0 : (v >= A.nc[a] ? A.nc[a] - 1 : v);
        lo[a] = A.nc[a] >= 3 ? v - 1 : 0;
        cnt[a] = A.nc[a] >= 3 ? 3 : A.nc[a];
    }
    const int ncl = cnt[0] * cnt[1] * cnt[2];
    if (lane < ncl) {
        const int ix = lane / (cnt[1] * cnt[2]), iy = (lane / cnt[2]) % cnt[1], iz = lane % cnt[2];
        const int wx = (lo[0] + ix + A.nc[0]) % A.nc[0], wy = (lo[1] + iy + A.nc[1]) % A.nc[1],
                  wz = (lo[2] + iz + A.nc[2]) % A.nc[2];
        const int w = (wx * A.nc[1] + wy) * A.nc[2] + wz;
        cstart[lane] = A.start[w];
        cpre[lane + 1] = A.start[w + 1] - A.start[w];
    }
    if (lane == 0) nnear = 0;
    __syncthreads();
    if (lane == 0) {
        cpre[0] = 0;
        for (int k = 0; k < ncl; ++k) cpre[k + 1] += cpre[k];
    }
    __syncthreads();
    const int T = cpre[ncl];
    // candidate pass: a cheap centre-distance test (nearest image, reach
    // L/2 + r with a margin), then the exact captured interval
    const double inv[3] = {1.0 / A.box[0], 1.0 / A.box[1], 1.0 / A.box[2]};
    for (int t = lane; t < T; t += 64) {
        int k = 0;
        while (cpre[k + 1] <= t) ++k;
        const int q = cstart[k] + (t - cpre[k]);
        const double *xq = A.xs + 3 * (int64_t)q, *dq = A.ds + 3 * (int64_t)q;
        const double Lq = A.ls[q];
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double d = xq[a] - p[a];
            d -= A.box[a] * rint(d * inv[a]);
            d2 += d * d;
        }
        const double reach = 0.5 * Lq + r;
        if (d2 > reach * reach * (1.0 + 1e-9) + 1e-24) continue;
        const int j = A.order[q];
        if (j == own) continue;
        double a0, a1;
        inside_interval(xq, dq, Lq, A.box, p, unb ? r : r * (1.0 + 1e-9), a0, a1);
        if (!(a1 > a0)) continue;
        const int slot = atomicAdd(&nnear, 1);
        if (slot < kNearCap) {
            nidx[slot] = j;
            nw[slot] = a1 - a0;
        }
    }
    __syncthreads();
    const int K = nnear;
    if (K > kNearCap) {
        if (lane == 0) atomicOr(err, 2);
        return;
    }
    // sort the kept filaments by index (ranks; the indices are distinct)
    for (int k = lane; k < K; k += 64) {
        const int me = nidx[k];
        int rank = 0;
        for (int o = 0; o < K; ++o) rank += nidx[o] < me;
        sidx[rank] = me;
        sw[rank] = nw[k];
    }
    __syncthreads();
    // S -> D weights of the kept filaments, sites spread over the lanes
    if (!unb) {
        for (int k = 0; k < K; ++k) {
            const int j = sidx[k];
            const double L = rlen(A, j);
            const int64_t m = sites_of(A, L);
            const double *xj = A.x + 3 * (int64_t)j, *dj = A.dir + 3 * (int64_t)j;
            double a0, a1;
            inside_interval(xj, dj, L, A.box, p, P.rcd * (1.0 + 1e-9), a0, a1);
            const double step = L / m;
            int64_t k0 = (int64_t)floor((a0 + 0.5 * L) / step - 0.5) - 1;
            int64_t k1 = (int64_t)ceil((a1 + 0.5 * L) / step - 0.5) + 1;
            if (k0 < 0) k0 = 0;
            if (k1 > m - 1) k1 = m - 1;
            double cc[3];
            centre_rel(xj, A.box, p, cc);
            double part = 0.0;
            for (int64_t ks = k0 + lane; ks <= k1; ks += 64) {
                const double sa = site_arc(L, m, ks);
                const double v0 = cc[0] + sa * dj[0], v1 = cc[1] + sa * dj[1], v2 = cc[2] + sa * dj[2];
                const double l = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
                if (l <= P.rcd) part += cross_weight(A, l);
            }
            const double wj = wave_sum(part);
            if (lane == 0) sw[k] = wj;
        }
        __syncthreads();
    }
    if (lane != 0) return;
    // the total over the kept filaments in index order
    double tot = 0.0;
    for (int k = 0; k < K; ++k) tot += sw[k];
    int ev = RL_EV_NONE;
    if (unb) {
        for (int a = 0; a < 3; ++a) A.xl[3 * c + a] = p[a];
        const double cap = 3.0 * P.eps / (4.0 * 3.14159265358979323846 * P.rcs * P.rcs * P.rcs);
        const double RA = P.koS[0] * P.Ka[0] * cap * tot, RB = P.koS[1] * P.Ka[1] * cap * tot;
        const double R = RA + RB;
        if (R > 0.0 && uc[0] < 1.0 - exp(-R * A.dt) && K > 0) {
            const int h = uc[1] * R < RA ? 0 : 1;
            const double t = uc[2] * tot;
            double cum = 0.0, before = 0.0;
            int pick = -1;
            for (int k = 0; k < K; ++k) {
                pick = sidx[k];
                before = cum;
                cum += sw[k];
                if (cum > t) break;
            }
            double a0, a1;
            inside_interval(A.x + 3 * (int64_t)pick, A.dir + 3 * (int64_t)pick, rlen(A, pick), A.box, p, P.rcs, a0,
                            a1);
            double sa = a0 + (t - before);
            if (sa > a1) sa = a1;
            if (sa < a0) sa = a0;
            A.state[c] = h == 0 ? RL_XL_SA : RL_XL_SB;
            A.rod[2 * c + h] = pick;
            A.arc[2 * c + h] = sa;
            double q[3];
            axis_point(A, pick, sa, q);
            for (int a = 0; a < 3; ++a) A.xl[3 * c + a] = q[a];
            ev = RL_EV_BIND;
        }
    } else {
        const double Ron = P.koD[g] * P.Ke[g] / A.vbd * tot;
        const double Roff = P.koS[hd];
        const double R = Ron + Roff;
        for (int a = 0; a < 3; ++a) A.xl[3 * c + a] = p[a];
        if (R > 0.0 && uc[0] < 1.0 - exp(-R * A.dt)) {
            if (uc[1] * R < Roff) {
                const double nx = sqrt(xc[0] * xc[0] + xc[1] * xc[1] + xc[2] * xc[2]);
                const double rad = P.rcs * cbrt(uc[3]);
                for (int a = 0; a < 3; ++a) {
                    const double dn = nx > 0.0 ? xc[a] / nx : (a == 2 ? 1.0 : 0.0);
                    A.xl[3 * c + a] = wrap1(p[a] + rad * dn, A.box[a]);
                }
                A.state[c] = RL_XL_U;
                A.rod[2 * c + hd] = -1;
                A.arc[2 * c + hd] = 0.0;
                ev = RL_EV_UNBIND;
            } else if (K > 0) {
                const double t = uc[2] * tot;
                double cum = 0.0;
                int pick = -1;
                int64_t site = -1;
                for (int k = 0; k < K; ++k) {
                    if (!(sw[k] > 0.0)) continue;
                    pick = sidx[k];
                    if (cum + sw[k] > t) {
                        site_sum(A, pick, p, t - cum, &site);
                        break;
                    }
                    cum += sw[k];
                }
                // rounding left t at or past the total: the last site
                if (pick >= 0 && site < 0) site_sum(A, pick, p, -1.0, &site);
                if (pick >= 0 && site >= 0) {
                    const double L = rlen(A, pick);
                    A.state[c] = RL_XL_D;
                    A.rod[2 * c + g] = pick;
                    A.arc[2 * c + g] = site_arc(L, sites_of(A, L), site);
                    if (g == 0) {
                        double q[3];
                        axis_point(A, pick, A.arc[2 * c], q);
                        for (int a = 0; a < 3; ++a) A.xl[3 * c + a] = q[a];
                    }
                    ev = RL_EV_CROSS;
                }
            }
        }
    }
    if (A.event) A.event[c] = ev;
    if (ev != RL_EV_NONE) atomicAdd(A.counts + ev, 1ull);
}

// Doubly bound crosslinkers: one lane each (two axis points, two rates).
__global__ void __launch_bounds__(256) k_kmc_light(KmcArgs A, const int *__restrict__ perm, int nheavy)
{
    __shared__ unsigned nrel;
    if (threadIdx.x == 0) nrel = 0;
    __syncthreads();
    const int64_t t = nheavy + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < A.m) {
        const int64_t c = perm[t];
        const double *uc = A.u + 4 * c;
        const rl_kmc_params &P = A.P;
        int ev = RL_EV_NONE;
        double pa[3], pb[3];
        axis_point(A, A.rod[2 * c], A.arc[2 * c], pa);
        axis_point(A, A.rod[2 * c + 1], A.arc[2 * c + 1], pb);
        double l2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double d = pa[a] - pb[a];
            d -= A.box[a] * floor(d / A.box[a] + 0.5);
            l2 += d * d;
        }
        const double l = sqrt(l2);
        const double RA = release_rate(A, P.koD[0], l), RB = release_rate(A, P.koD[1], l);
        const double R = RA + RB;
        for (int a = 0; a < 3; ++a) A.xl[3 * c + a] = pa[a];
        if (R > 0.0 && uc[0] < 1.0 - exp(-R * A.dt)) {
            const int hd = uc[1] * R < RA ? 0 : 1;
            A.state[c] = hd == 0 ? RL_XL_SB : RL_XL_SA;
            A.rod[2 * c + hd] = -1;
            A.arc[2 * c + hd] = 0.0;
            if (hd == 0)
                for (int a = 0; a < 3; ++a) A.xl[3 * c + a] = pb[a];
            ev = RL_EV_RELEASE;
            atomicAdd(&nrel, 1u);
        }
        if (A.event) A.event[c] = ev;
    }
    __syncthreads();
    if (threadIdx.x == 0 && nrel) atomicAdd(A.counts + RL_EV_RELEASE, (unsigned long long)nrel);
}

// doubly bound crosslinkers: flags, then their links in crosslinker order
__global__ void k_kmc_dflag(int64_t m, const int32_t *__restrict__ state, int *__restrict__ f)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c < m) f[c] = state[c] == RL_XL_D ? 1 : 0;
}

__global__ void k_kmc_links(int64_t m, const int32_t *__restrict__ state, const int32_t *__restrict__ rod,
                            const double *__restrict__ arc, const int *__restrict__ off, double kappa, double rest,
                            int32_t *__restrict__ p, int32_t *__restrict__ q, double *__restrict__ arm,
                            double *__restrict__ kap, double *__restrict__ rst, int64_t *__restrict__ key)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= m || state[c] != RL_XL_D) return;
    const int64_t k = off[c];
    p[k] = rod[2 * c];
    q[k] = rod[2 * c + 1];
    arm[2 * k] = arc[2 * c];
    arm[2 * k + 1] = arc[2 * c + 1];
    kap[k] = kappa;
    rst[k] = rest;
    if (key) key[k] = c;
}

// V_bd by Gauss-Legendre quadrature (8 nodes per panel, 256 panels; the
// integrand is smooth and its peak is resolved by the panels)
static double effective_volume(const rl_kmc_params &P, double diam)
{
    static const double xg[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    static const double wg[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const int panels = 256;
    const double h = P.rcd / panels;
    const double a = P.kappa / P.kT, c0 = P.rest + diam;
    double acc = 0.0;
    for (int k = 0; k < panels; ++k) {
        const double mid = (k + 0.5) * h, half = 0.5 * h;
        for (int g = 0; g < 4; ++g)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double r = mid + sgn * half * xg[g];
                const double dl = r - c0;
                acc += wg[g] * half * std::exp(-0.5 * a * dl * dl) * r * r;
            }
    }
    return 4.0 * 3.14159265358979323846 * acc;
}

static int check_kmc(const rl_kmc_params *kp)
{
    if (!kp) {
        set_error("kmc: params are NULL");
        return RL_ERR_ARG;
    }
    const rl_kmc_params &P = *kp;
    bool ok = P.eps > 0.0 && std::isfinite(P.eps) && P.kappa > 0.0 && std::isfinite(P.kappa) && P.rest >= 0.0 &&
              P.lambda >= 0.0 && P.lambda <= 1.0 && std::isfinite(P.xc) && P.kT > 0.0 && P.rcs > 0.0 &&
              P.rcd > 0.0 && P.dU >= 0.0 && std::isfinite(P.rcs) && std::isfinite(P.rcd) && std::isfinite(P.dU);
    for (int h = 0; h < 2; ++h)
        ok = ok && P.Ka[h] >= 0.0 && P.koS[h] >= 0.0 && P.Ke[h] >= 0.0 && P.koD[h] >= 0.0 && std::isfinite(P.Ka[h]) &&
             std::isfinite(P.koS[h]) && std::isfinite(P.Ke[h]) && std::isfinite(P.koD[h]);
    if (!ok) {
        set_error("kmc: bad parameters (all rates and constants >= 0 and finite; eps, kappa, kT, r_cs, r_cd > 0; "
                  "0 <= lambda <= 1)");
        return RL_ERR_ARG;
    }
    return RL_OK;
}

}  // namespace rl

using namespace rl;

extern "C" {

int rl_kmc_effective_volume(rl_handle h, const rl_kmc_params *kp, double *vbd)
{
    if (!h || !vbd) {
        set_error("rl_kmc_effective_volume: NULL argument");
        return RL_ERR_ARG;
    }
    const int rc = check_kmc(kp);
    if (rc) return rc;
    *vbd = effective_volume(*kp, h->prm.diam);
    return RL_OK;
}

int rl_kmc_step(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                const rl_kmc_params *kp, const rl_crosslinkers *xl, const double *u, const double *xi,
                int32_t *event, int64_t *counts)
{
    if (!h) {
        set_error("handle is NULL");
        return RL_ERR_ARG;
    }
    RL_HIP(hipSetDevice(h->device));
    int rc = check_kmc(kp);
    if (rc) return rc;
    if (!xl || xl->m < 0 || xl->m >= 0x7fffffff || n < 0 || n >= 0x7fffffff || (n > 0 && (!x || !dir)) ||
        (!len && !(len0 > 0.0)) || (xl->m > 0 && (!xl->state || !xl->rod || !xl->arc || !xl->x || !u || !xi))) {
        set_error("rl_kmc_step: bad sizes or NULL array");
        return RL_ERR_ARG;
    }
    if (counts)
        for (int k = 0; k < 5; ++k) counts[k] = 0;
    const int64_t m = xl->m;
    if (m == 0) return RL_OK;
    hipStream_t st = h->stream;
    int werr = 0;
    auto *cnt = (unsigned long long *)ws_get(h, kWsKmcCount, sizeof(unsigned long long) * 8, &werr);
    int *flag = (int *)ws_get(h, kWsKmcFlag, sizeof(int) * 4, &werr);
    if (werr) return werr;
    KmcArgs A{};
    A.m = m;
    A.n = n;
    A.state = xl->state;
    A.rod = xl->rod;
    A.arc = xl->arc;
    A.xl = xl->x;
    A.u = u;
    A.xi = xi;
    A.event = event;
    A.x = x;
    A.dir = dir;
    A.len = len;
    A.len0 = len0;
    A.P = *kp;
    A.diam = h->prm.diam;
    A.dt = h->prm.dt;
    A.vbd = effective_volume(*kp, h->prm.diam);
    A.counts = cnt;
    // the state is checked before anything changes
    RL_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, st));
    hipLaunchKernelGGL(k_kmc_check, dim3(grid_of(m, kKmcBlock)), dim3(kKmcBlock), 0, st, A, flag);
    RL_HIP(hipGetLastError());
    RL_HIP(hipMemcpyAsync(h->host_scratch + 4, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    RodCells cells;
    rc = rod_cells(h, n, x, dir, len, len0, std::max(kp->rcs, kp->rcd), &cells);
    if (rc) return rc;  // rod_cells synchronises: the flag copy has landed
    if (((int *)(h->host_scratch + 4))[0]) {
        set_error("rl_kmc_step: a crosslinker has a bad state or head (a bound head needs a filament in [0, n), "
                  "an unbound one -1, the two heads different filaments)");
        return RL_ERR_ARG;
    }
    for (int a = 0; a < 3; ++a) {
        A.nc[a] = cells.nc[a];
        A.cell[a] = cells.cell[a];
        A.box[a] = cells.box[a];
    }
    A.start = cells.start;
    A.order = cells.order;
    A.xs = cells.xs;
    A.ds = cells.ds;
    A.ls = cells.ls;
    int *key = (int *)ws_get(h, kWsKmcKey, sizeof(int) * m, &werr);
    int *key_out = (int *)ws_get(h, kWsKmcKeyOut, sizeof(int) * m, &werr);
    int *perm = (int *)ws_get(h, kWsKmcPerm, sizeof(int) * m, &werr);
    if (werr) return werr;
    RL_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, st));
    hipLaunchKernelGGL(k_kmc_keys, dim3(grid_of(m, 256)), dim3(256), 0, st, A, key, flag + 1);
    RL_HIP(hipGetLastError());
    rc = stable_sort_by_key(h, m, key, 28, key_out, perm);
    if (rc) return rc;
    RL_HIP(hipMemcpyAsync(h->host_scratch + 4, flag + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    const int nheavy = ((int *)(h->host_scratch + 4))[0];
    RL_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * 8, st));
    if (nheavy > 0)
        hipLaunchKernelGGL(k_kmc_heavy, dim3((unsigned)nheavy), dim3(64), 0, st, A, (const int *)perm, nheavy, flag);
    RL_HIP(hipGetLastError());
    if (m > nheavy)
        hipLaunchKernelGGL(k_kmc_light, dim3(grid_of(m - nheavy, 256)), dim3(256), 0, st, A, (const int *)perm,
                           nheavy);
    RL_HIP(hipGetLastError());
    RL_HIP(hipMemcpyAsync(h->host_scratch, cnt, sizeof(unsigned long long) * 5, hipMemcpyDeviceToHost, st));
    RL_HIP(hipMemcpyAsync(h->host_scratch + 5, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    if (((int *)(h->host_scratch + 5))[0] & 2) {
        set_error("rl_kmc_step: more than %d filaments pass within the query radius of one crosslinker", kNearCap);
        return RL_ERR_ARG;
    }
    if (counts) {
        int64_t ev = 0;
        for (int k = 1; k < 5; ++k) {
            counts[k] = h->host_scratch[k];
            ev += counts[k];
        }
        counts[0] = m - ev;
    }
    return RL_OK;
}

int rl_kmc_links(rl_handle h, const rl_kmc_params *kp, const rl_crosslinkers *xl, int64_t capacity, int32_t *p,
                 int32_t *q, double *arm, double *kappa, double *rest, int64_t *key, int64_t *n_links)
{
    if (!h) {
        set_error("handle is NULL");
        return RL_ERR_ARG;
    }
    RL_HIP(hipSetDevice(h->device));
    int rc = check_kmc(kp);
    if (rc) return rc;
    if (!xl || xl->m < 0 || xl->m >= 0x7fffffff || capacity < 0 || (xl->m > 0 && (!xl->state || !xl->rod || !xl->arc)) ||
        (capacity > 0 && (!p || !q || !arm || !kappa || !rest))) {
        set_error("rl_kmc_links: bad sizes or NULL array");
        return RL_ERR_ARG;
    }
    if (n_links) *n_links = 0;
    const int64_t m = xl->m;
    if (m == 0) return RL_OK;
    hipStream_t st = h->stream;
    int werr = 0;
    int *f = (int *)ws_get(h, kWsKmcFlag, sizeof(int) * (m + 1), &werr);
    int *off = (int *)ws_get(h, kWsKmcOff, sizeof(int) * (m + 1), &werr);
    int64_t *tot = (int64_t *)ws_get(h, kWsScan, sizeof(int64_t) * 2, &werr);
    if (werr) return werr;
    hipLaunchKernelGGL(k_kmc_dflag, dim3(grid_of(m, 256)), dim3(256), 0, st, m, (const int32_t *)xl->state, f);
    RL_HIP(hipGetLastError());
    rc = device_scan(h, f, m, off, tot);
    if (rc) return rc;
    RL_HIP(hipMemcpyAsync(h->host_scratch, tot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    const int64_t nl = h->host_scratch[0];
    if (n_links) *n_links = nl;
    if (nl > capacity) {
        set_error("rl_kmc_links: %lld links exceed capacity %lld", (long long)nl, (long long)capacity);
        return RL_ERR_CAPACITY;
    }
    if (nl == 0) return RL_OK;
    hipLaunchKernelGGL(k_kmc_links, dim3(grid_of(m, 256)), dim3(256), 0, st, m, (const int32_t *)xl->state,
                       (const int32_t *)xl->rod, (const double *)xl->arc, (const int *)off, kp->kappa,
                       kp->rest + h->prm.diam, p, q, arm, kappa, rest, key);
    RL_HIP(hipGetLastError());
    RL_HIP(hipStreamSynchronize(st));
    return RL_OK;
}

}  // extern "C"
