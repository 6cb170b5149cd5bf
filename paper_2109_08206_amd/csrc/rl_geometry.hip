// Rod geometry on gfx950: directors, per-rod mobility, closest points of rod
// axes, the uniform-grid pair search and the constraint geometry.
//
// Method: Yan et al., arXiv 2109.08206.  Directors come from the unit
// quaternion of each rod (Appendix "Filament dynamics"); pairs are the rods
// whose surface gap is below the threshold (Appendix "Implementation");
// the constraint column of a pair uses the closest points and the unit
// normal between them (Appendix "Symmetry of the geometrically constrained
// optimization problem", D_PQ and r = x_P + y_P - x_Q - y_Q); q follows
// eq. (blockdef), block A.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "rl_vec.hpp"

namespace rl {


// ---------------------------------------------------------------------------
// directors: third column of R(theta) = (s^2 - p.p) I + 2 p p^T + 2 s [p]x
// ---------------------------------------------------------------------------
__global__ void k_directors(int64_t n, const double *__restrict__ quat, double *__restrict__ dir)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 a = *reinterpret_cast<const double2 *>(quat + 4 * i);
    const double2 b = *reinterpret_cast<const double2 *>(quat + 4 * i + 2);
    const double s = a.x, px = a.y, py = b.x, pz = b.y;
    dir[3 * i + 0] = 2.0 * (px * pz + s * py);
    dir[3 * i + 1] = 2.0 * (py * pz - s * px);
    dir[3 * i + 2] = s * s - px * px - py * py + pz * pz;
}

hipError_t launch_directors(hipStream_t st, int64_t n, const double *quat, double *dir)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_directors, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, quat, dir);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// slender-body mobility of a rod of length L (perpendicular drag
// 4 pi eta L / log(2L/d) as in Section 3; parallel drag half of it;
// rotational drag pi eta L^3 / (3 log(2L/d)))
// ---------------------------------------------------------------------------
__host__ __device__ inline Mob mobility_of(double L, double diam, double eta)
{
    const double lg = log(2.0 * L / diam);
    Mob m;
    m.aperp = lg / (4.0 * M_PI * eta * L);
    m.apar = 2.0 * m.aperp;
    m.rperp = 3.0 * lg / (M_PI * eta * L * L * L);
    return m;
}

Mob mobility_host(double L, double diam, double eta) { return mobility_of(L, diam, eta); }

__global__ void k_mobility_coeffs(int64_t n, const double *__restrict__ len, double diam, double eta,
                                  double *__restrict__ coef)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Mob m = mobility_of(len[i], diam, eta);
    coef[3 * i + 0] = m.apar;
    coef[3 * i + 1] = m.aperp;
    coef[3 * i + 2] = m.rperp;
}

hipError_t launch_mobility_coeffs(hipStream_t st, int64_t n, const double *len, double diam, double eta, double *coef)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mobility_coeffs, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, len,
                       diam, eta, coef);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Closest points of two rod axes xi + s di (|s| <= hi) and xj + t dj
// (|t| <= hj), xj already imaged.  The squared distance is a convex
// quadratic in (s, t): take the stationary s with t free and clamp it, the
// best t for that s, and if t leaves its range clamp it and take the best s
// again (clamped normal equations for segment pairs, Lumelsky 1985).  For
// parallel axes (1 - b^2 <= 1e-14) the contact is the midpoint of the
// overlap of the two parameter ranges, else the best end-point candidate.
// ---------------------------------------------------------------------------
struct Contact {
    double s, t, dist;
    V3 e;
    unsigned flags;
};

__device__ Contact closest_point(V3 xi, V3 di, double hi, V3 xj, V3 dj, double hj)
{
    const V3 r0 = xi - xj;
    const double b = dot(di, dj);
    const double c = dot(di, r0);
    const double f = dot(dj, r0);
    const double den = 1.0 - b * b;
    Contact out;
    out.flags = den <= kBandPar ? 2u : 0u;
    double s, t;
    if (den > kEpsPar) {
        s = clampd((b * f - c) / den, -hi, hi);
        t = b * s + f;
        if (t < -hj) {
            t = -hj;
            s = clampd(b * t - c, -hi, hi);
        } else if (t > hj) {
            t = hj;
            s = clampd(b * t - c, -hi, hi);
        }
    } else {
        const double sg = b >= 0.0 ? 1.0 : -1.0;
        double lo = (-hj - f) * sg, up = (hj - f) * sg;
        if (lo > up) {
            const double tmp = lo;
            lo = up;
            up = tmp;
        }
        lo = lo > -hi ? lo : -hi;
        up = up < hi ? up : hi;
        if (lo <= up) {
            s = 0.5 * (lo + up);
            t = clampd(b * s + f, -hj, hj);
        } else {
            double best = INFINITY;
            s = 0.0;
            t = 0.0;
            for (int k = 0; k < 4; ++k) {
                double sk, tk;
                if (k < 2) {
                    sk = k == 0 ? -hi : hi;
                    tk = clampd(b * sk + f, -hj, hj);
                } else {
                    tk = k == 2 ? -hj : hj;
                    sk = clampd(b * tk - c, -hi, hi);
                }
                const V3 rk = r0 + sk * di - tk * dj;
                const double d2 = dot(rk, rk);
                if (d2 < best) {
                    best = d2;
                    s = sk;
                    t = tk;
                }
            }
        }
    }
    const V3 r = r0 + s * di - t * dj;
    const double dist = sqrt(dot(r, r));
    out.s = s;
    out.t = t;
    out.dist = dist;
    if (dist >= kDegenDist) {
        out.e = v3(r.x / dist, r.y / dist, r.z / dist);
    } else {
        out.flags |= 4u;
        V3 nrm = cross(di, dj);
        double nn = sqrt(dot(nrm, nrm));
        if (nn < 1e-12) {
            // collinear axes: normal to di and the coordinate axis least aligned with it
            const double ax = fabs(di.x), ay = fabs(di.y), az = fabs(di.z);
            int k = 0;
            double best = ax;
            if (ay < best) {
                k = 1;
                best = ay;
            }
            if (az < best) k = 2;
            const V3 ek = v3(k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0);
            nrm = cross(di, ek);
            nn = sqrt(dot(nrm, nrm));
        }
        const double sg = dot(nrm, r0) >= 0.0 ? 1.0 : -1.0;
        out.e = v3(sg * nrm.x / nn, sg * nrm.y / nn, sg * nrm.z / nn);
    }
    return out;
}

// ---------------------------------------------------------------------------
// Pair search.  Cells of edge >= reach (max length + diam + cutoff) on a
// periodic grid; rods are binned by centre and copied in cell order so that
// the lanes of a wave, which hold rods of the same cell, read the same
// neighbour-cell entries together.  The stencil offset u of a cell maps to
// the wrapped cell u mod nc and the shift floor(u / nc) of the neighbour.
// ---------------------------------------------------------------------------
struct GridDev {
    int nc[3];
    int S[3];
    double cell[3];
    double box[3];
};

__device__ __forceinline__ int cell_coord(double x, double cell, int nc)
{
    int k = (int)floor(x / cell);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

// Spread the low three bits of v to bits 0, 3 and 6.
__device__ __forceinline__ unsigned spread3(unsigned v)
{
    return (v & 1u) | ((v & 2u) << 2) | ((v & 4u) << 4);
}

// cell_of[i] = the rod's cell, followed by `fb` bits (0, 3, 6 or 9) of the
// Morton code of its sub-cell (fb / 3 bits per direction) when the rods are
// to be ordered by position inside their cells as well.
__global__ void k_bin(int64_t n, const double *__restrict__ x, const double *__restrict__ dir, GridDev g, int fb,
                      int *__restrict__ cell_of, int *__restrict__ cell_cnt, int *__restrict__ err)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const V3 xi = load3(x + 3 * i), di = load3(dir + 3 * i);
    const double xs[3] = {xi.x, xi.y, xi.z};
    bool finite = isfinite(xi.x) && isfinite(xi.y) && isfinite(xi.z) && isfinite(di.x) && isfinite(di.y) &&
                  isfinite(di.z);
    if (!finite) {
        // keep the cell counts consistent with the scatter that follows
        atomicOr(err, 1);
        cell_of[i] = 0;
        atomicAdd(cell_cnt, 1);
        return;
    }
    int kc[3];
    unsigned sub = 0;
    const int per = fb / 3, side = 1 << per;
    bool inside = true;
    for (int a = 0; a < 3; ++a) {
        inside = inside && xs[a] >= 0.0 && xs[a] < g.box[a];
        kc[a] = cell_coord(xs[a], g.cell[a], g.nc[a]);
        if (per > 0) {
            int f = (int)floor((xs[a] / g.cell[a] - kc[a]) * side);
            f = f < 0 ? 0 : (f >= side ? side - 1 : f);
            sub |= spread3((unsigned)f << (3 - per)) << a;
        }
    }
    if (!inside) atomicOr(err, 2);
    const int id = (kc[0] * g.nc[1] + kc[1]) * g.nc[2] + kc[2];
    cell_of[i] = (int)(((unsigned)id << fb) | (sub >> (9 - fb)));
    atomicAdd(cell_cnt + id, 1);
}


__global__ void k_scatter(int64_t n, const double *__restrict__ x, const double *__restrict__ dir,
                          const double *__restrict__ len, double len0, const int *__restrict__ cell_of,
                          const int *__restrict__ cell_start, int *__restrict__ cell_cur, int *__restrict__ sorted,
                          double *__restrict__ xs, double *__restrict__ ds, double *__restrict__ ls)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int slot = cell_start[c] + atomicAdd(cell_cur + c, 1);
    sorted[slot] = (int)i;
    store3(xs + 3 * (int64_t)slot, load3(x + 3 * i));
    store3(ds + 3 * (int64_t)slot, load3(dir + 3 * i));
    ls[slot] = len ? len[i] : len0;
}

__device__ __forceinline__ bool lex_positive(int a, int b, int c)
{
    return a > 0 || (a == 0 && (b > 0 || (b == 0 && c > 0)));
}

// One lane per rod (in cell order t).  INTERNAL: rods are numbered by their
// cell-order slot; otherwise by the caller's index sorted[t].  A pair is
// listed by its smaller rod number (self-images: positive shifts only).
// Pair search, one workgroup per home cell.  The home cell's rods and then,
// one stencil cell at a time, the neighbour cell's rods (shifted by the
// periodic image) are staged in LDS; every (home, neighbour) combination is
// tested from LDS in parallel with the cheap necessary conditions (centre
// distance within reach; axis lines closer than the threshold).  Survivors
// go to an LDS queue and get the exact closest-point test together, on full
// waves.  Counting pass: per-rod counts.  Filling pass: each pair takes the
// next slot of its rod (LDS atomic); the order within a rod is then fixed by
// the per-rod sort that follows.
constexpr int kPairBlock = 256;
constexpr int kCellChunk = 256;  // rods of one cell staged at a time
constexpr int kQueue = 4096;     // candidate (home, neighbour) pairs per flush
#ifndef RL_PAIR_SPLIT
#define RL_PAIR_SPLIT 9
#endif

// The staged copies are FP32, with the centres relative to the home cell's
// corner (so they stay within a few cells of 0 and round finely): the cheap
// tests run on them with margins that cover FP32 rounding, so that they
// never drop a pair the FP64 tests would keep; the exact test of a survivor
// reads the FP64 values from the cell-order arrays.
struct CellStage {
    float p[7][kCellChunk];  // x, y, z (shifted by image - corner), dx, dy, dz, length
    int idx[kCellChunk];     // rod index (the caller's or the cell order's)
};

template <bool INTERNAL>
__device__ __forceinline__ void stage_cell(CellStage &S, int q0, int m, V3 shift, const int *sorted,
                                           const double *xs, const double *ds, const double *ls)
{
    for (int u = threadIdx.x; u < m; u += kPairBlock) {
        const int64_t q = q0 + u;
        S.p[0][u] = (float)(xs[3 * q] + shift.x);
        S.p[1][u] = (float)(xs[3 * q + 1] + shift.y);
        S.p[2][u] = (float)(xs[3 * q + 2] + shift.z);
        S.p[3][u] = (float)ds[3 * q];
        S.p[4][u] = (float)ds[3 * q + 1];
        S.p[5][u] = (float)ds[3 * q + 2];
        S.p[6][u] = (float)ls[q];
        S.idx[u] = INTERNAL ? (int)q : sorted[q];
    }
}

// Pass modes: count pairs per rod, fill the per-rod slots, or emit every
// pair once as a key (pi, pj, shift) with its flags at a slot reserved per
// flush (the list is put in canonical order afterwards: bucketed by pi, then
// sorted per rod).
enum PairPass : int { kPairCount = 0, kPairFill = 1, kPairEmit = 2 };

// exclusive prefix of v over the workgroup; tot = the sum (lds: 5 ints)
__device__ __forceinline__ void block_excl_scan(int v, int &excl, int &tot, int *lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) lds[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < kPairBlock / 64; ++k) {
            const int t = lds[k];
            lds[k] = run;
            run += t;
        }
        lds[kPairBlock / 64] = run;
    }
    __syncthreads();
    excl = lds[w] + incl - v;
    tot = lds[kPairBlock / 64];
}

template <int PASS, bool INTERNAL>
__global__ void __launch_bounds__(kPairBlock) k_pairs(GridDev g, double diam, double cutoff,
                                                      const int *__restrict__ sorted, const double *__restrict__ xs,
                                                      const double *__restrict__ ds, const double *__restrict__ ls,
                                                      const int *__restrict__ cell_start, int *__restrict__ pcnt,
                                                      const int *__restrict__ poff, int32_t *__restrict__ pi,
                                                      int32_t *__restrict__ pj, int32_t *__restrict__ img,
                                                      uint8_t *__restrict__ flags, unsigned long long *ecount,
                                                      unsigned long long *__restrict__ ekeys,
                                                      uint8_t *__restrict__ eflags, int64_t ecap, int kshift,
                                                      int split)
{
    constexpr bool FILL = PASS == kPairFill;
    __shared__ CellStage H, Nb;
    __shared__ int hcnt[kCellChunk], hoff[kCellChunk];
    __shared__ int queue[kQueue];
    __shared__ int qn;
    __shared__ int scan_lds[kPairBlock / 64 + 1];
    __shared__ unsigned long long ebase;
    // the emitting pass may split a home cell's stencil over `split`
    // workgroups (each takes every split-th neighbour cell)
    const int h = blockIdx.x / split, part = blockIdx.x % split;
    const int hz = h % g.nc[2], hy = (h / g.nc[2]) % g.nc[1], hx = h / (g.nc[2] * g.nc[1]);
    const int hb = cell_start[h], he = cell_start[h + 1];
    // FP32 margins.  Staged centres lie within S + 1 cells of the corner (S <=
    // 7), so a component of r0 carries at most 1e-6 x cell of rounding, and
    // directions 6e-8 per component.  The reach test gets 1e-3 + 1e-5 x reach
    // more.  The axis-line test runs only where |d_i x d_j|^2 > 1e-5 (|n| >
    // 3.1e-3) and gets 1e-2 x (1 + reach) on the gap: the rounding of r0 . n,
    // below 2.2e-6 x reach (cell <= reach), is then under a tenth of
    // margin x |n|.
    const float greach = (float)(diam + cutoff), fgap0 = (float)(diam + cutoff) + 1e-2f;
    const V3 corner = v3(hx * g.cell[0], hy * g.cell[1], hz * g.cell[2]);
    const int NY = 2 * g.S[1] + 1, NZ = 2 * g.S[2] + 1, NS = (2 * g.S[0] + 1) * NY * NZ;
    for (int a0 = hb; a0 < he; a0 += kCellChunk) {
        const int na = he - a0 < kCellChunk ? he - a0 : kCellChunk;
        stage_cell<INTERNAL>(H, a0, na, v3(-corner.x, -corner.y, -corner.z), sorted, xs, ds, ls);
        for (int u = threadIdx.x; u < na; u += kPairBlock) {
            hcnt[u] = 0;
            if (PASS == kPairFill) hoff[u] = poff[INTERNAL ? a0 + u : sorted[a0 + u]];
        }
        __syncthreads();
        for (int sc = part; sc < NS; sc += split) {
            const int ux = hx + sc / (NY * NZ) - g.S[0];
            const int uy = hy + (sc / NZ) % NY - g.S[1];
            const int uz = hz + sc % NZ - g.S[2];
            const int wx = ((ux % g.nc[0]) + g.nc[0]) % g.nc[0];
            const int wy = ((uy % g.nc[1]) + g.nc[1]) % g.nc[1];
            const int wz = ((uz % g.nc[2]) + g.nc[2]) % g.nc[2];
            const int sx = (ux - wx) / g.nc[0], sy = (uy - wy) / g.nc[1], sz = (uz - wz) / g.nc[2];
            const bool selfok = lex_positive(sx, sy, sz);
            const int packed = ((sx + 8) << 8) | ((sy + 8) << 4) | (sz + 8);
            const V3 shift = v3(sx * g.box[0], sy * g.box[1], sz * g.box[2]);
            const int w = (wx * g.nc[1] + wy) * g.nc[2] + wz;
            const int nb = cell_start[w], ne = cell_start[w + 1];
            for (int b0 = nb; b0 < ne; b0 += kCellChunk) {
                const int nn = ne - b0 < kCellChunk ? ne - b0 : kCellChunk;
                // rods in cell order: a neighbour chunk entirely below the home
                // chunk holds no j >= i
                if (INTERNAL && b0 + nn <= a0) continue;
                __syncthreads();
                stage_cell<INTERNAL>(Nb, b0, nn, v3(shift.x - corner.x, shift.y - corner.y, shift.z - corner.z),
                                     sorted, xs, ds, ls);
                __syncthreads();
                const int total = na * nn;
                // (a, b) of entry e = a nn + b, advanced by kPairBlock entries
                // per step without a division
                const int step_a = kPairBlock / nn, step_b = kPairBlock % nn;
                for (int base = 0; base < total; base += kQueue) {
                    if (threadIdx.x == 0) qn = 0;
                    __syncthreads();
                    const int lim = total - base < kQueue ? total - base : kQueue;
                    int a = (base + (int)threadIdx.x) / nn, b = (base + (int)threadIdx.x) - a * nn;
                    for (int e = threadIdx.x; e < lim; e += kPairBlock) {
                        const int ca = a, cb = b;
                        a += step_a;
                        b += step_b;
                        if (b >= nn) {
                            b -= nn;
                            ++a;
                        }
                        const int i = H.idx[ca], j = Nb.idx[cb];
                        if (j < i || (j == i && !selfok)) continue;
                        const float rx = H.p[0][ca] - Nb.p[0][cb], ry = H.p[1][ca] - Nb.p[1][cb],
                                    rz = H.p[2][ca] - Nb.p[2][cb];
                        const float reach0 = 0.5f * (H.p[6][ca] + Nb.p[6][cb]) + greach;
                        const float reach = reach0 * (1.0f + 1e-5f) + 1e-3f;
                        if (rx * rx + ry * ry + rz * rz >= reach * reach) continue;
                        // two segments are never closer than their axis lines
                        // (near-parallel lines go through)
                        const float ax = H.p[3][ca], ay = H.p[4][ca], az = H.p[5][ca];
                        const float bx = Nb.p[3][cb], by = Nb.p[4][cb], bz = Nb.p[5][cb];
                        const float nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
                        const float nn2 = nx * nx + ny * ny + nz * nz, rn = rx * nx + ry * ny + rz * nz;
                        const float fgap = fgap0 + 1e-2f * reach0;
                        if (nn2 > 1e-5f && rn * rn > fgap * fgap * nn2) continue;
                        queue[atomicAdd(&qn, 1)] = (ca << 16) | cb;
                    }
                    __syncthreads();
                    const int nq = qn;
                    int mine = 0;
                    for (int u = threadIdx.x; u < nq; u += kPairBlock) {
                        const int a = (queue[u] >> 16) & 0xff, b = queue[u] & 0xff;
                        const int64_t qa = a0 + a, qb = b0 + b;
                        const V3 xi = load3(xs + 3 * qa), di = load3(ds + 3 * qa);
                        const V3 xq = load3(xs + 3 * qb), dj = load3(ds + 3 * qb);
                        const V3 xj = v3(xq.x + shift.x, xq.y + shift.y, xq.z + shift.z);
                        const Contact c = closest_point(xi, di, 0.5 * ls[qa], xj, dj, 0.5 * ls[qb]);
                        const double phi = c.dist - diam;
                        if (!(phi < cutoff)) continue;
                        const unsigned fl = c.flags | (fabs(phi - cutoff) <= kCutoffBand ? 1u : 0u);
                        if (PASS == kPairEmit) {
                            // mark the entry: bit 31 = pair, bits 24..27 = flags
                            queue[u] = (int)(0x80000000u | (fl << 24) | (unsigned)queue[u]);
                            ++mine;
                            continue;
                        }
                        const int slot = atomicAdd(&hcnt[a], 1);
                        if (FILL) {
                            const int o = hoff[a] + slot;
                            pi[o] = H.idx[a];
                            pj[o] = Nb.idx[b];
                            img[o] = packed;
                            flags[o] = (uint8_t)fl;
                        }
                    }
                    if (PASS == kPairEmit) {
                        int excl = 0, tot = 0;
                        block_excl_scan(mine, excl, tot, scan_lds);
                        if (threadIdx.x == 0) ebase = tot > 0 ? atomicAdd(ecount, (unsigned long long)tot) : 0ull;
                        __syncthreads();
                        unsigned long long o = ebase + (unsigned long long)excl;
                        for (int u = threadIdx.x; u < nq; u += kPairBlock) {
                            const unsigned v = (unsigned)queue[u];
                            if (!(v >> 31)) continue;
                            if (o < (unsigned long long)ecap) {
                                const int a = (v >> 16) & 0xff, b = v & 0xff;
                                ekeys[o] = ((unsigned long long)(unsigned)H.idx[a] << kshift) |
                                           ((unsigned long long)(unsigned)Nb.idx[b] << 12) | (unsigned long long)packed;
                                eflags[o] = (uint8_t)((v >> 24) & 15u);
                            }
                            ++o;
                        }
                    }
                    __syncthreads();
                }
            }
        }
        if (PASS == kPairCount)
            for (int u = threadIdx.x; u < na; u += kPairBlock) pcnt[H.idx[u]] = hcnt[u];
        __syncthreads();
    }
}

// Emitted pair keys (pi, pj, shift) into the canonical order: bucketed by
// pi (a histogram, its scan, a scatter), then each rod's short list sorted
// by (pj, shift).  The keys are distinct, so the result is the order of the
// keys whatever order the scatter's atomics took.
__global__ void k_pair_hist(int64_t m, const unsigned long long *__restrict__ keys, int shift, int *__restrict__ cnt)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= m) return;
    atomicAdd(cnt + (int)(keys[t] >> shift), 1);
}

__global__ void k_pair_scatter(int64_t m, const unsigned long long *__restrict__ keys,
                               const uint8_t *__restrict__ kflags, int ibits, const int *__restrict__ off,
                               int *__restrict__ cur, int32_t *__restrict__ pi, int32_t *__restrict__ pj,
                               int32_t *__restrict__ img, uint8_t *__restrict__ flags)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= m) return;
    const unsigned long long k = keys[t];
    const int a = (int)(k >> (ibits + 12));
    const int slot = off[a] + atomicAdd(cur + a, 1);
    pi[slot] = a;
    pj[slot] = (int32_t)((k >> 12) & ((1ull << ibits) - 1ull));
    img[slot] = (int32_t)(k & 0xfffull);
    flags[slot] = kflags[t];
}

// copies of centres, directors, lengths (and forces) in cell order
__global__ void k_gather_rods(int64_t n, const int *__restrict__ perm, const double *__restrict__ x,
                              const double *__restrict__ dir, const double *__restrict__ len, double len0,
                              double *__restrict__ xs, double *__restrict__ ds, double *__restrict__ ls)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t i = perm[t];
    store3(xs + 3 * t, load3(x + 3 * i));
    store3(ds + 3 * t, load3(dir + 3 * i));
    ls[t] = len ? len[i] : len0;
}

// order each rod's pairs by (pj, img).  Up to 32 pairs (every rod at the paper's densities)
// are sorted in registers by an odd-even transposition network over keys
// (pj, img, flags) packed into 64 bits, so the loads go out together and the
// stores once; longer lists take an insertion sort in memory.
constexpr int kSortRegs = 32;

// (256-thread groups, so that the 32 keys stay in registers)
__global__ void __launch_bounds__(256)
    k_sort_pairs(int64_t n, const int *__restrict__ poff, int32_t *__restrict__ pj, int32_t *__restrict__ img,
                 uint8_t *__restrict__ flags)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = poff[i], e = poff[i + 1];
    const int cnt = e - b;
    if (cnt <= 1) return;
    if (cnt <= kSortRegs) {
        unsigned long long key[kSortRegs];
#pragma unroll
        for (int k = 0; k < kSortRegs; ++k)
            key[k] = k < cnt ? ((unsigned long long)(unsigned)pj[b + k] << 16) |
                                   ((unsigned long long)(unsigned)img[b + k] << 4) | (unsigned long long)flags[b + k]
                             : ~0ull;
#pragma unroll
        for (int r = 0; r < kSortRegs; ++r)
#pragma unroll
            for (int k = r & 1; k + 1 < kSortRegs; k += 2) {
                const unsigned long long lo = key[k] < key[k + 1] ? key[k] : key[k + 1];
                const unsigned long long hi = key[k] < key[k + 1] ? key[k + 1] : key[k];
                key[k] = lo;
                key[k + 1] = hi;
            }
#pragma unroll
        for (int k = 0; k < kSortRegs; ++k)
            if (k < cnt) {
                pj[b + k] = (int32_t)(key[k] >> 16);
                img[b + k] = (int32_t)((key[k] >> 4) & 0xfffull);
                flags[b + k] = (uint8_t)(key[k] & 15ull);
            }
        return;
    }
    for (int k = b + 1; k < e; ++k) {
        const int32_t kj = pj[k], ki = img[k];
        const uint8_t kf = flags[k];
        const long long key = ((long long)kj << 12) | ki;
        int m = k - 1;
        while (m >= b && (((long long)pj[m] << 12) | img[m]) > key) {
            pj[m + 1] = pj[m];
            img[m + 1] = img[m];
            flags[m + 1] = flags[m];
            --m;
        }
        pj[m + 1] = kj;
        img[m + 1] = ki;
        flags[m + 1] = kf;
    }
}

__global__ void k_len_max(int64_t n, const double *__restrict__ len, unsigned long long *__restrict__ out,
                          int *__restrict__ err)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double L = len[i];
    if (!(L > 0.0) || !isfinite(L)) {
        atomicOr(err, 4);
        return;
    }
    // positive doubles order like their bit patterns
    atomicMax(out, (unsigned long long)__double_as_longlong(L));
}

static inline unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__global__ void k_gather6(int64_t n, const int *__restrict__ perm, const double *__restrict__ src,
                          double *__restrict__ dst)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t i = perm[t];
    for (int a = 0; a < 6; ++a) dst[6 * t + a] = src[6 * i + a];
}

hipError_t launch_gather6(hipStream_t st, int64_t n, const int *perm, const double *src, double *dst)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather6, dim3(grid_of(n)), dim3(kBlock), 0, st, n, perm, src, dst);
    return hipGetLastError();
}

// Shared body of the two pair searches.  internal = false: canonical list
// in the caller's rod numbering; internal = true: rods renumbered in cell
// order (stable by caller index), h's workspace keeps the order and copies.
static int pairs_core(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                      bool internal, int64_t capacity, int32_t *pi, int32_t *pj, int32_t *img, uint8_t *flags,
                      int64_t *n_pairs)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    int werr = 0;
    if (n_pairs) *n_pairs = 0;
    if (n == 0) return RL_OK;
    // longest rod
    double Lmax = len0;
    RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int) * 4, st));
    if (len) {
        auto *lm = (unsigned long long *)ws_get(h, kWsLenMax, sizeof(unsigned long long), &werr);
        if (werr) return werr;
        RL_HIP(hipMemsetAsync(lm, 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_len_max, dim3(grid_of(n)), dim3(kBlock), 0, st, n, len, lm, h->flag_dev);
        RL_HIP(hipGetLastError());
        RL_HIP(hipMemcpyAsync(h->host_scratch, lm, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        RL_HIP(hipMemcpyAsync(h->host_scratch + 1, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
        RL_HIP(hipStreamSynchronize(st));
        if (((int *)(h->host_scratch + 1))[0] & 4) {
            set_error("pair search: rod lengths must be finite and > 0");
            return RL_ERR_ARG;
        }
        unsigned long long bits = (unsigned long long)h->host_scratch[0];
        std::memcpy(&Lmax, &bits, sizeof(double));
    } else if (!(len0 > 0.0)) {
        set_error("pair search: len0 must be > 0");
        return RL_ERR_ARG;
    }
    const double reach = Lmax + p.diam + p.cutoff;
    GridDev g;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int nca = (int)floor(p.box[a] / reach);
        if (nca < 1) nca = 1;
        if (nca > 1024) nca = 1024;
        g.nc[a] = nca;
        g.cell[a] = p.box[a] / nca;
        g.S[a] = (int)ceil(reach / g.cell[a]);
        g.box[a] = p.box[a];
        if (g.S[a] > 7) {
            set_error("pair search: box edge %g too small for rod reach %g (needs box >= reach/7)", p.box[a], reach);
            return RL_ERR_ARG;
        }
        ncell *= nca;
    }
    if (ncell > (1 << 26)) {
        set_error("pair search: too many cells (%lld)", (long long)ncell);
        return RL_ERR_ARG;
    }
    int *cell_of = (int *)ws_get(h, kWsCellOf, sizeof(int) * n, &werr);
    int *cell_cnt = (int *)ws_get(h, kWsCellCnt, sizeof(int) * ncell, &werr);
    int *cell_start = (int *)ws_get(h, kWsCellStart, sizeof(int) * (ncell + 1), &werr);
    int *cell_cur = (int *)ws_get(h, kWsCellCur, sizeof(int) * ncell, &werr);
    int *sorted = (int *)ws_get(h, kWsSorted, sizeof(int) * n, &werr);
    int *cell_key = internal ? (int *)ws_get(h, kWsCellKey, sizeof(int) * n, &werr) : nullptr;
    double *xs = (double *)ws_get(h, kWsXs, sizeof(double) * 3 * n, &werr);
    double *ds = (double *)ws_get(h, kWsDs, sizeof(double) * 3 * n, &werr);
    double *ls = (double *)ws_get(h, kWsLs, sizeof(double) * n, &werr);
    int *pcnt = (int *)ws_get(h, kWsPcnt, sizeof(int) * n, &werr);
    int *poff = (int *)ws_get(h, kWsPoff, sizeof(int) * (n + 1), &werr);
    int64_t *tot = (int64_t *)ws_get(h, kWsScan, sizeof(int64_t) * 2, &werr);
    if (werr) return werr;

    // internal order: by cell, then along a Morton curve of 8^3 sub-cells
    // inside the cell (fewer when the cell ids leave no room in 31 bits), so
    // that rods with consecutive numbers are close in space and so are their
    // partners' records in the solver's Q-side arrays
    int cbits = 1;
    while ((1LL << cbits) < ncell) ++cbits;
    const int fb = internal ? std::min(9, (31 - cbits) / 3 * 3) : 0;
    RL_HIP(hipMemsetAsync(cell_cnt, 0, sizeof(int) * ncell, st));
    hipLaunchKernelGGL(k_bin, dim3(grid_of(n)), dim3(kBlock), 0, st, n, x, dir, g, fb, cell_of, cell_cnt,
                       h->flag_dev);
    RL_HIP(hipGetLastError());
    {
        const int rc = device_scan(h, cell_cnt, ncell, cell_start, nullptr);
        if (rc) return rc;
    }
    if (internal) {
        int rc = stable_sort_by_key(h, n, cell_of, cbits + fb, cell_key, sorted);
        if (rc) return rc;
        hipLaunchKernelGGL(k_gather_rods, dim3(grid_of(n)), dim3(kBlock), 0, st, n, (const int *)sorted, x, dir, len,
                           len0, xs, ds, ls);
    } else {
        RL_HIP(hipMemsetAsync(cell_cur, 0, sizeof(int) * ncell, st));
        hipLaunchKernelGGL(k_scatter, dim3(grid_of(n)), dim3(kBlock), 0, st, n, x, dir, len, len0, cell_of,
                           cell_start, cell_cur, sorted, xs, ds, ls);
    }
    RL_HIP(hipGetLastError());
    // one pass emitting keys (pi, pj, shift), then buckets by pi and a per-rod
    // sort into the canonical order; rod counts above 2^26 do not fit the
    // 64-bit key and take the counting and filling passes instead
    int ibits = 1;
    while ((1LL << ibits) < n) ++ibits;
    const bool emit = 2 * ibits + 12 <= 64;
    const dim3 pgrid((unsigned)ncell), pblock(kPairBlock);
    // with few cells, one workgroup per home cell leaves the chip short of
    // waves: the emitting pass splits each stencil over several workgroups,
    // up to RL_PAIR_SPLIT of them, for about 4,096 workgroups in all
    // (100k rods, 729 cells: 838 us with one per cell, 423 with three, 376
    // with six)
    const int split = (int)std::max<int64_t>(1, std::min<int64_t>(RL_PAIR_SPLIT, 4096 / ncell));
    const dim3 egrid((unsigned)(ncell * split));
    auto *none_u64 = (unsigned long long *)nullptr;
    auto *none_u8 = (uint8_t *)nullptr;
    if (emit) {
        const int64_t ecap = capacity > 0 ? capacity : 0;
        auto *ecount = (unsigned long long *)ws_get(h, kWsEmitCount, sizeof(unsigned long long), &werr);
        auto *ekeys = (unsigned long long *)ws_get(h, kWsEmitKeys, sizeof(unsigned long long) * (ecap > 0 ? ecap : 1), &werr);
        auto *eflags = (uint8_t *)ws_get(h, kWsEmitFlags, (size_t)(ecap > 0 ? ecap : 1), &werr);
        if (werr) return werr;
        RL_HIP(hipMemsetAsync(ecount, 0, sizeof(unsigned long long), st));
        const int kshift = ibits + 12;
        if (internal)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs<kPairEmit, true>), egrid, pblock, 0, st, g, p.diam, p.cutoff,
                               sorted, xs, ds, ls, cell_start, pcnt, (const int *)nullptr, (int32_t *)nullptr,
                               (int32_t *)nullptr, (int32_t *)nullptr, none_u8, ecount, ekeys, eflags, ecap, kshift,
                               split);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs<kPairEmit, false>), egrid, pblock, 0, st, g, p.diam, p.cutoff,
                               sorted, xs, ds, ls, cell_start, pcnt, (const int *)nullptr, (int32_t *)nullptr,
                               (int32_t *)nullptr, (int32_t *)nullptr, none_u8, ecount, ekeys, eflags, ecap, kshift,
                               split);
        RL_HIP(hipGetLastError());
        RL_HIP(hipMemcpyAsync(h->host_scratch, ecount, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    } else {
        if (internal)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs<kPairCount, true>), pgrid, pblock, 0, st, g, p.diam, p.cutoff,
                               sorted, xs, ds, ls, cell_start, pcnt, (const int *)nullptr, (int32_t *)nullptr,
                               (int32_t *)nullptr, (int32_t *)nullptr, none_u8, none_u64, none_u64, none_u8,
                               (int64_t)0, 0, 1);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs<kPairCount, false>), pgrid, pblock, 0, st, g, p.diam, p.cutoff,
                               sorted, xs, ds, ls, cell_start, pcnt, (const int *)nullptr, (int32_t *)nullptr,
                               (int32_t *)nullptr, (int32_t *)nullptr, none_u8, none_u64, none_u64, none_u8,
                               (int64_t)0, 0, 1);
        RL_HIP(hipGetLastError());
        const int rc = device_scan(h, pcnt, n, poff, tot);
        if (rc) return rc;
        RL_HIP(hipMemcpyAsync(h->host_scratch, tot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    }
    RL_HIP(hipMemcpyAsync(h->host_scratch + 1, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    const int64_t total = h->host_scratch[0];
    const int ferr = ((int *)(h->host_scratch + 1))[0];
    if (ferr & 1) {
        set_error("pair search: non-finite centre or director");
        return RL_ERR_NONFINITE;
    }
    if (ferr & 2) {
        set_error("pair search: a centre lies outside [0, box)");
        return RL_ERR_ARG;
    }
    if (n_pairs) *n_pairs = total;
    if (total > capacity) {
        set_error("pair search: %lld pairs exceed capacity %lld", (long long)total, (long long)capacity);
        return RL_ERR_CAPACITY;
    }
    if (total > 0x7fffffffLL) {
        set_error("pair search: pair count overflows int32");
        return RL_ERR_CAPACITY;
    }
    if (total == 0) return RL_OK;
    if (emit) {
        auto *ekeys = (unsigned long long *)h->buf[kWsEmitKeys];
        auto *eflags = (uint8_t *)h->buf[kWsEmitFlags];
        RL_HIP(hipMemsetAsync(pcnt, 0, sizeof(int) * n, st));
        hipLaunchKernelGGL(k_pair_hist, dim3(grid_of(total)), dim3(kBlock), 0, st, total,
                           (const unsigned long long *)ekeys, ibits + 12, pcnt);
        RL_HIP(hipGetLastError());
        const int rc = device_scan(h, pcnt, n, poff, nullptr);
        if (rc) return rc;
        RL_HIP(hipMemsetAsync(pcnt, 0, sizeof(int) * n, st));
        hipLaunchKernelGGL(k_pair_scatter, dim3(grid_of(total)), dim3(kBlock), 0, st, total,
                           (const unsigned long long *)ekeys, (const uint8_t *)eflags, ibits, (const int *)poff, pcnt,
                           pi, pj, img, flags);
        RL_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sort_pairs, dim3(grid_of(n)), dim3(kBlock), 0, st, n, (const int *)poff, pj, img, flags);
        RL_HIP(hipGetLastError());
        return RL_OK;
    }
    if (internal)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs<kPairFill, true>), pgrid, pblock, 0, st, g, p.diam, p.cutoff, sorted,
                           xs, ds, ls, cell_start, pcnt, (const int *)poff, pi, pj, img, flags, none_u64, none_u64,
                           none_u8, (int64_t)0, 0, 1);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs<kPairFill, false>), pgrid, pblock, 0, st, g, p.diam, p.cutoff,
                           sorted, xs, ds, ls, cell_start, pcnt, (const int *)poff, pi, pj, img, flags, none_u64,
                           none_u64, none_u8, (int64_t)0, 0, 1);
    RL_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sort_pairs, dim3(grid_of(n)), dim3(kBlock), 0, st, n, (const int *)poff, pj, img, flags);
    RL_HIP(hipGetLastError());
    return RL_OK;
}

int rod_cells(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
              double radius, RodCells *out)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    int werr = 0;
    double Lmax = len0;
    RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int) * 4, st));
    if (len && n > 0) {
        auto *lm = (unsigned long long *)ws_get(h, kWsLenMax, sizeof(unsigned long long), &werr);
        if (werr) return werr;
        RL_HIP(hipMemsetAsync(lm, 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_len_max, dim3(grid_of(n)), dim3(kBlock), 0, st, n, len, lm, h->flag_dev);
        RL_HIP(hipGetLastError());
        RL_HIP(hipMemcpyAsync(h->host_scratch, lm, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        RL_HIP(hipMemcpyAsync(h->host_scratch + 1, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
        RL_HIP(hipStreamSynchronize(st));
        if (((int *)(h->host_scratch + 1))[0] & 4) {
            set_error("rod cells: rod lengths must be finite and > 0");
            return RL_ERR_ARG;
        }
        unsigned long long bits = (unsigned long long)h->host_scratch[0];
        std::memcpy(&Lmax, &bits, sizeof(double));
    } else if (!(len0 > 0.0)) {
        set_error("rod cells: len0 must be > 0");
        return RL_ERR_ARG;
    }
    const double reach = 0.5 * Lmax + radius;
    GridDev g;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(2.0 * reach <= p.box[a])) {
            set_error("rod cells: half the longest rod plus the radius %g exceeds half the box edge %g", reach,
                      0.5 * p.box[a]);
            return RL_ERR_ARG;
        }
        int nca = (int)floor(p.box[a] / reach);
        if (nca < 1) nca = 1;
        if (nca > 1024) nca = 1024;
        g.nc[a] = nca;
        g.cell[a] = p.box[a] / nca;
        g.S[a] = 1;
        g.box[a] = p.box[a];
        ncell *= nca;
    }
    if (ncell > (1 << 26)) {
        set_error("rod cells: too many cells (%lld)", (long long)ncell);
        return RL_ERR_ARG;
    }
    const int64_t nb = n > 0 ? n : 1;
    int *cell_of = (int *)ws_get(h, kWsCellOf, sizeof(int) * nb, &werr);
    int *cell_cnt = (int *)ws_get(h, kWsCellCnt, sizeof(int) * ncell, &werr);
    int *cell_start = (int *)ws_get(h, kWsCellStart, sizeof(int) * (ncell + 1), &werr);
    int *sorted = (int *)ws_get(h, kWsSorted, sizeof(int) * nb, &werr);
    int *cell_key = (int *)ws_get(h, kWsCellKey, sizeof(int) * nb, &werr);
    double *xs = (double *)ws_get(h, kWsXs, sizeof(double) * 3 * nb, &werr);
    double *ds = (double *)ws_get(h, kWsDs, sizeof(double) * 3 * nb, &werr);
    double *ls = (double *)ws_get(h, kWsLs, sizeof(double) * nb, &werr);
    if (werr) return werr;
    RL_HIP(hipMemsetAsync(cell_cnt, 0, sizeof(int) * ncell, st));
    if (n > 0) {
        hipLaunchKernelGGL(k_bin, dim3(grid_of(n)), dim3(kBlock), 0, st, n, x, dir, g, 0, cell_of, cell_cnt,
                           h->flag_dev);
        RL_HIP(hipGetLastError());
    }
    {
        const int rc = device_scan(h, cell_cnt, ncell, cell_start, nullptr);
        if (rc) return rc;
    }
    if (n > 0) {
        int cbits = 1;
        while ((1LL << cbits) < ncell) ++cbits;
        const int rc = stable_sort_by_key(h, n, cell_of, cbits, cell_key, sorted);
        if (rc) return rc;
        hipLaunchKernelGGL(k_gather_rods, dim3(grid_of(n)), dim3(kBlock), 0, st, n, (const int *)sorted, x, dir, len,
                           len0, xs, ds, ls);
        RL_HIP(hipGetLastError());
    }
    RL_HIP(hipMemcpyAsync(h->host_scratch + 1, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    const int ferr = ((int *)(h->host_scratch + 1))[0];
    if (ferr & 1) {
        set_error("rod cells: non-finite centre or director");
        return RL_ERR_NONFINITE;
    }
    if (ferr & 2) {
        set_error("rod cells: a centre lies outside [0, box)");
        return RL_ERR_ARG;
    }
    for (int a = 0; a < 3; ++a) {
        out->nc[a] = g.nc[a];
        out->cell[a] = g.cell[a];
        out->box[a] = g.box[a];
    }
    out->start = cell_start;
    out->order = sorted;
    out->xs = xs;
    out->ds = ds;
    out->ls = ls;
    return RL_OK;
}

int build_pairs_impl(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                     int64_t capacity, int32_t *pi, int32_t *pj, int32_t *img, uint8_t *flags, int64_t *n_pairs)
{
    return pairs_core(h, n, x, dir, len, len0, false, capacity, pi, pj, img, flags, n_pairs);
}

int build_pairs_sorted(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                       int64_t *n_pairs, const int **perm, const double **xs, const double **ds, const double **ls)
{
    int err = 0;
    int64_t cap = (int64_t)(h->cap[kWsStepPi] / sizeof(int32_t));
    int64_t np = 0;
    int rc = RL_ERR_CAPACITY;
    for (int attempt = 0; attempt < 2 && rc == RL_ERR_CAPACITY; ++attempt) {
        if (cap > 0 && (h->cap[kWsStepPj] < sizeof(int32_t) * cap || h->cap[kWsStepImg] < sizeof(int32_t) * cap ||
                        h->cap[kWsStepFlags] < (size_t)cap))
            cap = 0;
        rc = pairs_core(h, n, x, dir, len, len0, true, cap, (int32_t *)h->buf[kWsStepPi],
                        (int32_t *)h->buf[kWsStepPj], (int32_t *)h->buf[kWsStepImg], (uint8_t *)h->buf[kWsStepFlags],
                        &np);
        if (rc == RL_ERR_CAPACITY && np <= 0x7fffffffLL) {
            cap = np + np / 4 + 64;
            ws_get(h, kWsStepPi, sizeof(int32_t) * cap, &err);
            ws_get(h, kWsStepPj, sizeof(int32_t) * cap, &err);
            ws_get(h, kWsStepImg, sizeof(int32_t) * cap, &err);
            ws_get(h, kWsStepFlags, (size_t)cap, &err);
            if (err) return err;
            cap = (int64_t)(h->cap[kWsStepPi] / sizeof(int32_t));
        }
    }
    if (rc) return rc;
    *n_pairs = np;
    *perm = (const int *)h->buf[kWsSorted];
    *xs = (const double *)h->buf[kWsXs];
    *ds = (const double *)h->buf[kWsDs];
    *ls = (const double *)h->buf[kWsLs];
    return RL_OK;
}

// ---------------------------------------------------------------------------
// Constraint geometry: phi, e, arm and q = phi/h + D^T M F per pair.
// ---------------------------------------------------------------------------
template <bool UNI>
__global__ void k_unc(int64_t n, const double *__restrict__ dir, const double *__restrict__ len, Mob mob, double diam,
                      double eta, const double *__restrict__ F, double *__restrict__ Unc)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Mob m = UNI ? mob : mobility_of(len[i], diam, eta);
    const V3 d = load3(dir + 3 * i);
    V3 f = v3(0, 0, 0), tq = v3(0, 0, 0);
    if (F) {
        f = load3(F + 6 * i);
        tq = load3(F + 6 * i + 3);
    }
    const V3 u = m.aperp * f + ((m.apar - m.aperp) * dot(d, f)) * d;
    const V3 w = m.rperp * tq;  // axial rotational mobility equals the normal one
    store3(Unc + 6 * i, u);
    store3(Unc + 6 * i + 3, w);
}

__global__ void k_assemble(int64_t nc, const double *__restrict__ x, const double *__restrict__ dir,
                           const double *__restrict__ len, double len0, GridDev g, double diam, double dt,
                           const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                           const int32_t *__restrict__ img, const double *__restrict__ Unc, double *__restrict__ phi,
                           double *__restrict__ e, double *__restrict__ arm, double *__restrict__ q, int64_t n,
                           int *__restrict__ err)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int i = pi[c], j = pj[c], im = img[c];
    if (i < 0 || j < 0 || i >= n || j >= n) {
        atomicOr(err, 8);
        phi[c] = q[c] = arm[2 * c] = arm[2 * c + 1] = NAN;
        store3(e + 3 * c, v3(NAN, NAN, NAN));
        return;
    }
    const double sx = ((im >> 8) & 15) - 8, sy = ((im >> 4) & 15) - 8, sz = (im & 15) - 8;
    const V3 xi = load3(x + 3 * (int64_t)i), di = load3(dir + 3 * (int64_t)i);
    const V3 xj = load3(x + 3 * (int64_t)j) + v3(sx * g.box[0], sy * g.box[1], sz * g.box[2]);
    const V3 dj = load3(dir + 3 * (int64_t)j);
    const double Li = len ? len[i] : len0, Lj = len ? len[j] : len0;
    const Contact ct = closest_point(xi, di, 0.5 * Li, xj, dj, 0.5 * Lj);
    const double ph = ct.dist - diam;
    phi[c] = ph;
    store3(e + 3 * c, ct.e);
    arm[2 * c] = ct.s;
    arm[2 * c + 1] = ct.t;
    // D^T U_nc: e.U_i + (s_i d_i x e).Omega_i - e.U_j - (t d_j x e).Omega_j
    const V3 ui = load3(Unc + 6 * (int64_t)i), wi = load3(Unc + 6 * (int64_t)i + 3);
    const V3 uj = load3(Unc + 6 * (int64_t)j), wj = load3(Unc + 6 * (int64_t)j + 3);
    const double rate = dot(ct.e, ui) + dot(cross(ct.s * di, ct.e), wi) - dot(ct.e, uj) -
                        dot(cross(ct.t * dj, ct.e), wj);
    q[c] = ph / dt + rate;
}

hipError_t launch_unc(hipStream_t st, int64_t n, const double *dir, const double *len, double len0, double diam,
                      double eta, const double *F, double *Unc)
{
    if (n <= 0) return hipSuccess;
    const Mob mob = mobility_of(len ? 1.0 : len0, diam, eta);
    if (len)
        hipLaunchKernelGGL(k_unc<false>, dim3(grid_of(n)), dim3(kBlock), 0, st, n, dir, len, mob, diam, eta, F, Unc);
    else
        hipLaunchKernelGGL(k_unc<true>, dim3(grid_of(n)), dim3(kBlock), 0, st, n, dir, len, mob, diam, eta, F, Unc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bilateral links (eq. linearconstraints b): a Hookean link between the point
// at arclength sP on rod P's axis and the point at sQ on rod Q's axis, or a
// fixed point (Q < 0).  r = (x_P + sP d_P) - (x_Q + sQ d_Q) with each
// component of the difference taken to its nearest periodic image; the
// link's length is |r|, its direction e = r/|r| (from Q to P), its column of
// D is that of a contact with lever arms sP d_P and sQ d_Q (Appendix
// "Symmetry ...": the two points are arbitrary for bilateral constraints).
// Row (eq. blockdef D and F): q = (|r| - rest)/h + D^T M F, compliance
// 1/(kappa h), 0 for kappa = +inf.  A link of zero length takes e normal to
// both axes (d_P x d_Q, or d_P x the coordinate axis least aligned with d_P
// for parallel axes, d_Q = e_z for a fixed point) and flag bit 2.
// inv (may be null) maps the caller's rod index to the rods' order in x.
// ---------------------------------------------------------------------------
__device__ V3 normal_to(V3 dp, V3 dq)
{
    V3 c = cross(dp, dq);
    double nn = sqrt(dot(c, c));
    if (nn < 1e-12) {
        const double ax = fabs(dp.x), ay = fabs(dp.y), az = fabs(dp.z);
        int k = 0;
        double best = ax;
        if (ay < best) {
            k = 1;
            best = ay;
        }
        if (az < best) k = 2;
        c = cross(dp, v3(k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0));
        nn = sqrt(dot(c, c));
    }
    return v3(c.x / nn, c.y / nn, c.z / nn);
}

__global__ void k_links(int64_t nl, int64_t n, const double *__restrict__ x, const double *__restrict__ dir,
                        const int *__restrict__ inv, const int32_t *__restrict__ lp, const int32_t *__restrict__ lq,
                        const double *__restrict__ larm, const double *__restrict__ kappa,
                        const double *__restrict__ rest, const double *__restrict__ anchor, GridDev g, double dt,
                        const double *__restrict__ Unc, int32_t *__restrict__ pi_out, int32_t *__restrict__ pj_out,
                        double *__restrict__ len_out, double *__restrict__ e_out, double *__restrict__ arm_out,
                        double *__restrict__ q_out, double *__restrict__ cmp_out, uint8_t *__restrict__ fl_out,
                        int *__restrict__ err)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nl) return;
    const int32_t P0 = lp[k], Q0 = lq[k];
    const double kap = kappa[k], r0 = rest[k];
    if (P0 < 0 || P0 >= n || Q0 >= n || Q0 < -1 || P0 == Q0 || (Q0 < 0 && !anchor) || !(kap > 0.0) ||
        !(r0 >= 0.0) || !isfinite(r0)) {
        atomicOr(err, 16);
        return;
    }
    const int P = inv ? inv[P0] : P0, Q = Q0 < 0 ? -1 : (inv ? inv[Q0] : Q0);
    const double sP = larm[2 * k], sQ = larm[2 * k + 1];
    const V3 xP = load3(x + 3 * (int64_t)P), dP = load3(dir + 3 * (int64_t)P);
    const V3 aP = xP + sP * dP;
    V3 dQ = v3(0.0, 0.0, 1.0), aQ;
    if (Q >= 0) {
        dQ = load3(dir + 3 * (int64_t)Q);
        aQ = load3(x + 3 * (int64_t)Q) + sQ * dQ;
    } else {
        aQ = load3(anchor + 3 * k);
    }
    double r[3] = {aP.x - aQ.x, aP.y - aQ.y, aP.z - aQ.z};
    for (int a = 0; a < 3; ++a) r[a] -= g.box[a] * floor(r[a] / g.box[a] + 0.5);
    const V3 rv = v3(r[0], r[1], r[2]);
    const double L = sqrt(dot(rv, rv));
    V3 e;
    uint8_t fl = 0;
    if (L < kDegenDist) {
        e = normal_to(dP, dQ);
        fl = 4;
    } else {
        e = v3(rv.x / L, rv.y / L, rv.z / L);
    }
    // D^T U_nc: e.U_P + (sP d_P x e).W_P - e.U_Q - (sQ d_Q x e).W_Q
    double rate = dot(e, load3(Unc + 6 * (int64_t)P)) + dot(cross(sP * dP, e), load3(Unc + 6 * (int64_t)P + 3));
    if (Q >= 0)
        rate -= dot(e, load3(Unc + 6 * (int64_t)Q)) + dot(cross(sQ * dQ, e), load3(Unc + 6 * (int64_t)Q + 3));
    pi_out[k] = P;
    pj_out[k] = Q;
    len_out[k] = L;
    store3(e_out + 3 * k, e);
    arm_out[2 * k] = sP;
    arm_out[2 * k + 1] = Q >= 0 ? sQ : 0.0;
    q_out[k] = (L - r0) / dt + rate;
    cmp_out[k] = isinf(kap) ? 0.0 : 1.0 / (kap * dt);
    if (fl_out) fl_out[k] = fl;
}

hipError_t launch_links(hipStream_t st, int64_t nl, int64_t n, const double *x, const double *dir, const int *inv,
                        const rl_links *lk, const double box[3], double dt, const double *Unc, int32_t *pi,
                        int32_t *pj, double *len, double *e, double *arm, double *q, double *cmp, uint8_t *flags,
                        int *err)
{
    if (nl <= 0) return hipSuccess;
    GridDev g{};
    for (int a = 0; a < 3; ++a) g.box[a] = box[a];
    hipLaunchKernelGGL(k_links, dim3(grid_of(nl)), dim3(kBlock), 0, st, nl, n, x, dir, inv, lk->p, lk->q, lk->arm,
                       lk->kappa, lk->rest, lk->anchor, g, dt, Unc, pi, pj, len, e, arm, q, cmp, flags, err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Walls (confinement): constraints between a rod and a fixed body, only the
// rod's side in D (Appendix "Equation of motion with geometric constraints",
// last paragraph).  The allowed regions are convex (a half-space, the inside
// of a sphere or of a cylinder), so each end of a rod is a candidate contact
// point: for ends s = -L/2, +L/2 and each wall in order, phi = (distance of
// the end to the wall) - diam/2, and an end with phi < cutoff gives a
// unilateral constraint with e the wall's inward unit normal at its nearest
// point, lever arm s and q = phi/h + D^T M F.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wall_gap(const WallSet &W, int w, V3 pt, double diam, V3 &e)
{
    const int kind = W.kind[w];
    const V3 p0 = v3(W.p[w][0], W.p[w][1], W.p[w][2]), a = v3(W.a[w][0], W.a[w][1], W.a[w][2]);
    V3 v = pt - p0;
    if (kind == RL_WALL_PLANE) {
        e = a;
        return dot(a, v) - 0.5 * diam;
    }
    if (kind == RL_WALL_CYLINDER_IN) v = v - dot(v, a) * a;
    const double dist = sqrt(dot(v, v));
    e = dist > 0.0 ? v3(-v.x / dist, -v.y / dist, -v.z / dist) : v3(0.0, 0.0, 0.0);
    return W.r[w] - dist - 0.5 * diam;
}

// FILL = false: per-rod counts; FILL = true: the list at the rod's offset
template <bool FILL>
__global__ void k_walls(int64_t n, const double *__restrict__ x, const double *__restrict__ dir,
                        const double *__restrict__ len, double len0, double diam, double cutoff, double dt, WallSet W,
                        const double *__restrict__ Unc, int *__restrict__ cnt, const int *__restrict__ off,
                        int32_t *__restrict__ rod, double *__restrict__ e_out, double *__restrict__ arm,
                        double *__restrict__ phi, double *__restrict__ q, uint8_t *__restrict__ flags)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const V3 xi = load3(x + 3 * i), di = load3(dir + 3 * i);
    const double L = len ? len[i] : len0;
    int m = FILL ? off[i] : 0;
    for (int end = 0; end < 2; ++end) {
        const double s = end == 0 ? -0.5 * L : 0.5 * L;
        const V3 pt = xi + s * di;
        for (int w = 0; w < W.n; ++w) {
            V3 e;
            const double ph = wall_gap(W, w, pt, diam, e);
            if (!(ph < cutoff)) continue;
            if (FILL) {
                const double rate = dot(e, load3(Unc + 6 * i)) + dot(cross(s * di, e), load3(Unc + 6 * i + 3));
                rod[m] = (int32_t)i;
                store3(e_out + 3 * (int64_t)m, e);
                arm[2 * (int64_t)m] = s;
                arm[2 * (int64_t)m + 1] = 0.0;
                if (phi) phi[m] = ph;
                q[m] = ph / dt + rate;
                if (flags) flags[m] = fabs(ph - cutoff) <= kCutoffBand ? 1u : 0u;
            }
            ++m;
        }
    }
    if (!FILL) cnt[i] = m;
}

int walls_impl(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
               const double *Unc, const WallSet &W, int64_t capacity, int32_t *rod, double *e, double *arm,
               double *phi, double *q, uint8_t *flags, int64_t *count)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    int werr = 0;
    *count = 0;
    if (n <= 0 || W.n <= 0) return RL_OK;
    int *cnt = (int *)ws_get(h, kWsWallCnt, sizeof(int) * n, &werr);
    int *off = (int *)ws_get(h, kWsWallOff, sizeof(int) * (n + 1), &werr);
    int64_t *tot = (int64_t *)ws_get(h, kWsScan, sizeof(int64_t) * 2, &werr);
    if (werr) return werr;
    hipLaunchKernelGGL(k_walls<false>, dim3(grid_of(n)), dim3(kBlock), 0, st, n, x, dir, len, len0, p.diam, p.cutoff,
                       p.dt, W, Unc, cnt, (const int *)nullptr, (int32_t *)nullptr, (double *)nullptr,
                       (double *)nullptr, (double *)nullptr, (double *)nullptr, (uint8_t *)nullptr);
    RL_HIP(hipGetLastError());
    int rc = device_scan(h, cnt, n, off, tot);
    if (rc) return rc;
    RL_HIP(hipMemcpyAsync(h->host_scratch, tot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    const int64_t total = h->host_scratch[0];
    *count = total;
    if (total > capacity) {
        set_error("walls: %lld contacts exceed capacity %lld", (long long)total, (long long)capacity);
        return RL_ERR_CAPACITY;
    }
    if (total == 0) return RL_OK;
    hipLaunchKernelGGL(k_walls<true>, dim3(grid_of(n)), dim3(kBlock), 0, st, n, x, dir, len, len0, p.diam, p.cutoff,
                       p.dt, W, Unc, cnt, (const int *)off, rod, e, arm, phi, q, flags);
    RL_HIP(hipGetLastError());
    return RL_OK;
}

int assemble_impl(rl_ctx *h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                  int64_t nc, const int32_t *pi, const int32_t *pj, const int32_t *img, const double *F,
                  double *phi, double *e, double *arm, double *q)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    int werr = 0;
    if (nc == 0) return RL_OK;
    double *Unc = (double *)ws_get(h, kWsUnc, sizeof(double) * 6 * (n > 0 ? n : 1), &werr);
    if (werr) return werr;
    const Mob mob = mobility_of(len ? 1.0 : len0, p.diam, p.eta);
    if (len)
        hipLaunchKernelGGL(k_unc<false>, dim3(grid_of(n)), dim3(kBlock), 0, st, n, dir, len, mob, p.diam, p.eta, F,
                           Unc);
    else
        hipLaunchKernelGGL(k_unc<true>, dim3(grid_of(n)), dim3(kBlock), 0, st, n, dir, len, mob, p.diam, p.eta, F,
                           Unc);
    RL_HIP(hipGetLastError());
    GridDev g{};
    for (int a = 0; a < 3; ++a) g.box[a] = p.box[a];
    RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_assemble, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, x, dir, len, len0, g, p.diam, p.dt,
                       pi, pj, img, (const double *)Unc, phi, e, arm, q, n, h->flag_dev);
    RL_HIP(hipGetLastError());
    RL_HIP(hipMemcpyAsync(h->host_scratch, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    if (((int *)h->host_scratch)[0] & 8) {
        set_error("rl_assemble_D: a pair index is outside [0, n)");
        return RL_ERR_ARG;
    }
    return RL_OK;
}

// ---------------------------------------------------------------------------
// adjoint of the constraint geometry (differentiation form)
// ---------------------------------------------------------------------------
// Per constraint, from phi_bar = q_bar / h, e_bar and the arclength
// adjoints (s_bar, t_bar), the adjoints of r0 = x_i - x_j' and of the two
// directors; d_bar (the lever-arm parts) is added to the director terms.
// r = r0 + s di - t dj, phi = |r| - diam, e = r / |r|.  The arclengths are
// stationary points of |r|^2 over the free ones: r.di = 0 when s is inside
// (-L_i/2, L_i/2), r.dj = 0 when t is inside (-L_j/2, L_j/2); an arclength
// on a rod end stays there.  Their derivatives follow from differentiating
// those conditions (implicit function; unit directors, so the 2x2 system
// has the matrix [[1, -b], [b, -1]], b = di.dj).  Parallel axes keep their
// closest points fixed and intersecting axes their normal (the midpoint and
// cross-product rules have no derivative that the step uses).
__global__ void k_geo_adjoint(int64_t nc, const double *__restrict__ x, const double *__restrict__ dir,
                              const double *__restrict__ len, double len0, GridDev g,
                              const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                              const int32_t *__restrict__ img, double dt, const double *__restrict__ qbar,
                              const double *__restrict__ ebar, const double *__restrict__ armbar,
                              const double *__restrict__ dbar, double *__restrict__ gbar)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int i = pi[c], j = pj[c], im = img[c];
    const double sx = ((im >> 8) & 15) - 8, sy = ((im >> 4) & 15) - 8, sz = (im & 15) - 8;
    const V3 xi = load3(x + 3 * (int64_t)i), di = load3(dir + 3 * (int64_t)i);
    const V3 xj = load3(x + 3 * (int64_t)j) + v3(sx * g.box[0], sy * g.box[1], sz * g.box[2]);
    const V3 dj = load3(dir + 3 * (int64_t)j);
    const double hi = 0.5 * (len ? len[i] : len0), hj = 0.5 * (len ? len[j] : len0);
    const Contact ct = closest_point(xi, di, hi, xj, dj, hj);
    const double b = dot(di, dj), den = 1.0 - b * b;
    const V3 r = (xi - xj) + ct.s * di - ct.t * dj;
    const double phib = qbar[c] / dt;
    const V3 eb = load3(ebar + 3 * c);
    V3 rb = phib * ct.e;
    if (!(ct.flags & 4u)) rb = rb + (1.0 / ct.dist) * (eb - dot(ct.e, eb) * ct.e);
    const double sb = armbar[2 * c] + dot(rb, di);
    const double tb = armbar[2 * c + 1] - dot(rb, dj);
    V3 r0b = rb;
    V3 dib = ct.s * rb + load3(dbar + 6 * c);
    V3 djb = (-ct.t) * rb + load3(dbar + 6 * c + 3);
    if (den > kEpsPar) {
        const bool s_in = fabs(ct.s) < hi, t_in = fabs(ct.t) < hj;
        // dF1 = dr0.di + (r + s di).ddi - t di.ddj (+ ds - b dt)
        // dF2 = dr0.dj + s dj.ddi + (r - t dj).ddj (+ b ds - dt)
        if (s_in && t_in) {
            const double mu2 = -(tb + b * sb) / den, mu1 = sb - b * mu2;
            r0b = r0b - (mu1 * di + mu2 * dj);
            dib = dib - (mu1 * (r + ct.s * di) + (mu2 * ct.s) * dj);
            djb = djb - ((-mu1 * ct.t) * di + mu2 * (r - ct.t * dj));
        } else if (t_in) {
            r0b = r0b + tb * dj;
            dib = dib + (tb * ct.s) * dj;
            djb = djb + tb * (r - ct.t * dj);
        } else if (s_in) {
            r0b = r0b - sb * di;
            dib = dib - sb * (r + ct.s * di);
            djb = djb + (sb * ct.t) * di;
        }
    }
    store3(gbar + 9 * c, r0b);
    store3(gbar + 9 * c + 3, dib);
    store3(gbar + 9 * c + 6, djb);
}

hipError_t launch_geo_adjoint(hipStream_t st, int64_t nc, const double *x, const double *dir, const double *len,
                              double len0, const double box[3], const int32_t *pi, const int32_t *pj,
                              const int32_t *img, double dt, const double *q_bar, const double *e_bar,
                              const double *arm_bar, const double *d_bar, double *gbar)
{
    if (nc <= 0) return hipSuccess;
    GridDev g{};
    for (int a = 0; a < 3; ++a) g.box[a] = box[a];
    hipLaunchKernelGGL(k_geo_adjoint, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, x, dir, len, len0, g, pi, pj, img,
                       dt, q_bar, e_bar, arm_bar, d_bar, gbar);
    return hipGetLastError();
}

}  // namespace rl
