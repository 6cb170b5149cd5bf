// Crosslinker kinetics: kinetic Monte Carlo of binding and unbinding
// (Section "2. Crosslinker binding and unbinding", Table tab:rates; appendix
// "Kinetic Monte-Carlo", Table tab:supprates).
//
// Every crosslinker is independent of the others within a step (steric
// interactions between motors are neglected), so the step is one lane per
// crosslinker.  A lane finds the filaments near its query point (the
// crosslinker, or its bound head) through a periodic cell list of filament
// centres, accumulates the rate of each possible transition, decides with
// its own uniform numbers, and for a binding walks the candidates in
// filament-index order (inverse transform): their weights are kept in a
// small per-lane list in LDS, sorted by index before the walk; a lane with
// more candidates than the list holds walks by repeated search instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "rl_vec.hpp"

// the rounding of the rate arithmetic follows the written order
#pragma clang fp contract(off)

namespace rl {

constexpr int kKmcBlock = 64;   // crosslinkers per workgroup (one wave)
constexpr int kKmcList = 32;    // candidates a lane keeps in LDS

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

// the filaments whose centres lie in the cells around p (each once): f(j)
template <class Fn>
__device__ __forceinline__ void for_candidates(const KmcArgs &A, const double p[3], Fn f)
{
    int lo[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
        int c = (int)floor(p[a] / A.cell[a]);
        c = c < 0 ? 0 : (c >= A.nc[a] ? A.nc[a] - 1 : c);
        if (A.nc[a] >= 3) {
            lo[a] = c - 1;
            cnt[a] = 3;
        } else {
            lo[a] = 0;
            cnt[a] = A.nc[a];
        }
    }
    for (int ix = 0; ix < cnt[0]; ++ix) {
        const int wx = (lo[0] + ix + A.nc[0]) % A.nc[0];
        for (int iy = 0; iy < cnt[1]; ++iy) {
            const int wy = (lo[1] + iy + A.nc[1]) % A.nc[1];
            for (int iz = 0; iz < cnt[2]; ++iz) {
                const int wz = (lo[2] + iz + A.nc[2]) % A.nc[2];
                const int w = (wx * A.nc[1] + wy) * A.nc[2] + wz;
                for (int q = A.start[w]; q < A.start[w + 1]; ++q) f(q, A.order[q]);
            }
        }
    }
}

// the lane's candidate list: index and weight, [slot][lane]
struct KmcList {
    int idx[kKmcList][kKmcBlock];
    double w[kKmcList][kKmcBlock];
};

__device__ __forceinline__ void list_sort(KmcList &S, int lane, int K)
{
    for (int a = 1; a < K; ++a) {
        const int ki = S.idx[a][lane];
        const double kw = S.w[a][lane];
        int b = a - 1;
        while (b >= 0 && S.idx[b][lane] > ki) {
            S.idx[b + 1][lane] = S.idx[b][lane];
            S.w[b + 1][lane] = S.w[b][lane];
            --b;
        }
        S.idx[b + 1][lane] = ki;
        S.w[b + 1][lane] = kw;
    }
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
// cell of its query point, so that the lanes of a wave scan the same cells
// together and their loads of a filament's record coincide.
__global__ void k_kmc_keys(KmcArgs A, int *__restrict__ key)
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
    }
    key[c] = (cls << 26) | id;
}

__global__ void __launch_bounds__(kKmcBlock) k_kmc(KmcArgs A, const int *__restrict__ perm)
{
    __shared__ KmcList S;
    __shared__ unsigned cnt[5];
    const int lane = threadIdx.x;
    if (lane < 5) cnt[lane] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x * (int64_t)kKmcBlock + lane;
    if (t < A.m) {
        const int64_t c = perm[t];
        const rl_kmc_params &P = A.P;
        const double *uc = A.u + 4 * c, *xc = A.xi + 3 * c;
        int ev = RL_EV_NONE;
        const int s = A.state[c];
        if (s == RL_XL_U) {
            const double hop = sqrt(2.0 * P.dU * A.dt);
            double p[3];
            for (int a = 0; a < 3; ++a) {
                p[a] = wrap1(A.xl[3 * c + a] + hop * xc[a], A.box[a]);
                A.xl[3 * c + a] = p[a];
            }
            double Lt = 0.0;
            int K = 0;
            for_candidates(A, p, [&](int q, int j) {
                double lo, hi;
                inside_interval(A.xs + 3 * (int64_t)q, A.ds + 3 * (int64_t)q, A.ls[q], A.box, p, P.rcs, lo, hi);
                if (!(hi > lo)) return;
                Lt += hi - lo;
                if (K < kKmcList) {
                    S.idx[K][lane] = j;
                    S.w[K][lane] = hi - lo;
                }
                ++K;
            });
            const double cap = 3.0 * P.eps / (4.0 * 3.14159265358979323846 * P.rcs * P.rcs * P.rcs);
            const double RA = P.koS[0] * P.Ka[0] * cap * Lt, RB = P.koS[1] * P.Ka[1] * cap * Lt;
            const double R = RA + RB;
            if (R > 0.0 && uc[0] < 1.0 - exp(-R * A.dt)) {
                const int hd = uc[1] * R < RA ? 0 : 1;
                const double t = uc[2] * Lt;
                double cum = 0.0, before = 0.0;
                int pick = -1;
                if (K <= kKmcList) {
                    list_sort(S, lane, K);
                    for (int k = 0; k < K; ++k) {
                        pick = S.idx[k][lane];
                        before = cum;
                        cum += S.w[k][lane];
                        if (cum > t) break;
                    }
                } else {
                    // more candidates than the list holds: take them in index
                    // order by repeated search
                    int cur = -1;
                    for (;;) {
                        int next = 0x7fffffff;
                        double wn = 0.0;
                        for_candidates(A, p, [&](int q, int j) {
                            if (j <= cur || j >= next) return;
                            double lo, hi;
                            inside_interval(A.xs + 3 * (int64_t)q, A.ds + 3 * (int64_t)q, A.ls[q], A.box, p, P.rcs,
                                            lo, hi);
                            if (!(hi > lo)) return;
                            next = j;
                            wn = hi - lo;
                        });
                        if (next == 0x7fffffff) break;
                        pick = next;
                        before = cum;
                        cum += wn;
                        if (cum > t) break;
                        cur = next;
                    }
                }
                if (pick >= 0) {
                    double lo, hi;
                    inside_interval(A.x + 3 * (int64_t)pick, A.dir + 3 * (int64_t)pick, rlen(A, pick), A.box, p,
                                    P.rcs, lo, hi);
                    double sa = lo + (t - before);
                    if (sa > hi) sa = hi;
                    if (sa < lo) sa = lo;
                    A.state[c] = hd == 0 ? RL_XL_SA : RL_XL_SB;
                    A.rod[2 * c + hd] = pick;
                    A.arc[2 * c + hd] = sa;
                    double q[3];
                    axis_point(A, pick, sa, q);
                    for (int a = 0; a < 3; ++a) A.xl[3 * c + a] = q[a];
                    ev = RL_EV_BIND;
                }
            }
        } else if (s == RL_XL_SA || s == RL_XL_SB) {
            const int hd = s == RL_XL_SA ? 0 : 1, g = 1 - hd;
            const int i = A.rod[2 * c + hd];
            double p[3];
            axis_point(A, i, A.arc[2 * c + hd], p);
            double W = 0.0;
            int K = 0;
            for_candidates(A, p, [&](int, int j) {
                if (j == i) return;
                const double wj = site_sum(A, j, p, -1.0, nullptr);
                if (!(wj > 0.0)) return;
                W += wj;
                if (K < kKmcList) {
                    S.idx[K][lane] = j;
                    S.w[K][lane] = wj;
                }
                ++K;
            });
            const double Ron = P.koD[g] * P.Ke[g] / A.vbd * W;
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
                } else {
                    const double t = uc[2] * W;
                    double cum = 0.0;
                    int pick = -1;
                    int64_t site = -1;
                    bool found = false;
                    if (K <= kKmcList) {
                        list_sort(S, lane, K);
                        for (int k = 0; k < K; ++k) {
                            const int j = S.idx[k][lane];
                            const double wj = S.w[k][lane];
                            pick = j;
                            if (cum + wj > t) {
                                site_sum(A, j, p, t - cum, &site);
                                found = true;
                                break;
                            }
                            cum += wj;
                        }
                    } else {
                        int cur = -1;
                        for (;;) {
                            int next = 0x7fffffff;
                            for_candidates(A, p, [&](int, int j) {
                                if (j == i || j <= cur || j >= next) return;
                                if (site_sum(A, j, p, -1.0, nullptr) > 0.0) next = j;
                            });
                            if (next == 0x7fffffff) break;
                            const double wj = site_sum(A, next, p, -1.0, nullptr);
                            pick = next;
                            if (cum + wj > t) {
                                site_sum(A, next, p, t - cum, &site);
                                found = true;
                                break;
                            }
                            cum += wj;
                            cur = next;
                        }
                    }
                    // rounding left t at or past the total: the last site
                    if (!found && pick >= 0) site_sum(A, pick, p, -1.0, &site);
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
        } else if (s == RL_XL_D) {
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
            }
        }
        if (A.event) A.event[c] = ev;
        atomicAdd(&cnt[ev], 1u);
    }
    __syncthreads();
    if (lane < 5 && cnt[lane]) atomicAdd(A.counts + lane, (unsigned long long)cnt[lane]);
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
                            double *__restrict__ kap, double *__restrict__ rst)
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
    hipLaunchKernelGGL(k_kmc_keys, dim3(grid_of(m, 256)), dim3(256), 0, st, A, key);
    RL_HIP(hipGetLastError());
    rc = stable_sort_by_key(h, m, key, 28, key_out, perm);
    if (rc) return rc;
    RL_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * 8, st));
    hipLaunchKernelGGL(k_kmc, dim3(grid_of(m, kKmcBlock)), dim3(kKmcBlock), 0, st, A, (const int *)perm);
    RL_HIP(hipGetLastError());
    RL_HIP(hipMemcpyAsync(h->host_scratch, cnt, sizeof(unsigned long long) * 5, hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    if (counts)
        for (int k = 0; k < 5; ++k) counts[k] = h->host_scratch[k];
    return RL_OK;
}

int rl_kmc_links(rl_handle h, const rl_kmc_params *kp, const rl_crosslinkers *xl, int64_t capacity, int32_t *p,
                 int32_t *q, double *arm, double *kappa, double *rest, int64_t *n_links)
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
                       kp->rest + h->prm.diam, p, q, arm, kappa, rest);
    RL_HIP(hipGetLastError());
    RL_HIP(hipStreamSynchronize(st));
    return RL_OK;
}

}  // extern "C"
