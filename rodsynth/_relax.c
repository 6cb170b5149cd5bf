/*
 * Overlap removal for synthetic rod suspensions (input preparation only).
 *
 * Dense random placements of spherocylinders overlap; the paper resolves the
 * overlaps of its initial configurations before the timed runs (Results,
 * "Polarity sorting in a spherical shell").  This routine does the same for
 * the synthetic inputs by plain geometry: overlapping rods are pushed apart
 * (centres translated, axes turned) until every pair of rods, including
 * periodic images, is separated by at least `gap` beyond contact.  No
 * mobility, force or time step is involved: it only moves inputs, and its
 * results are checked by the tests against the oracle's own distances.
 *
 * Separation of two segments: the squared distance is a convex function on
 * the rectangle of the two arclength ranges, so its minimum is either the
 * stationary point of the infinite lines (when it falls inside both ranges)
 * or lies on an edge of the rectangle, where one arclength sits at a rod end
 * and the distance is a point-to-segment distance.  The routine evaluates
 * those five candidates and keeps the smallest.
 *
 * Sweeps are Gauss-Seidel steps over the candidate pairs (each push moves
 * the pair's two rods at once, over-relaxed), swept brick by brick in a fixed
 * colouring so that bricks of one colour touch disjoint rods and run in
 * parallel: the result does not depend on the thread count.
 */
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

typedef struct {
    double d, s, t; /* separation of the axes and the two arclengths */
} sep_t;

/* over-relaxation of the pushes (1 = move an overlapping pair exactly to the
 * target separation; 1.9 clears dense jams in a few tens of sweeps where 1
 * needs hundreds) */
static const double kOmega = 1.9;

/* threads of the parallel loops of the calling thread's rs_relax */
static _Thread_local int g_threads = 1;

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* distance from point p to segment c + u d, |u| <= h; returns u in *u */
static double point_seg(const double p[3], const double c[3], const double d[3], double h, double *u)
{
    const double w[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
    const double uu = clampd(w[0] * d[0] + w[1] * d[1] + w[2] * d[2], -h, h);
    const double r[3] = {w[0] - uu * d[0], w[1] - uu * d[1], w[2] - uu * d[2]};
    *u = uu;
    return sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

static sep_t separation(const double xi[3], const double di[3], double hi, const double xj[3], const double dj[3],
                        double hj)
{
    sep_t best = {INFINITY, 0.0, 0.0};
    const double r0[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
    const double b = di[0] * dj[0] + di[1] * dj[1] + di[2] * dj[2];
    const double den = 1.0 - b * b;
    if (den > 1e-12) {
        const double c = di[0] * r0[0] + di[1] * r0[1] + di[2] * r0[2];
        const double f = dj[0] * r0[0] + dj[1] * r0[1] + dj[2] * r0[2];
        const double s = (b * f - c) / den, t = (f - b * c) / den;
        if (fabs(s) <= hi && fabs(t) <= hj) {
            const double r[3] = {r0[0] + s * di[0] - t * dj[0], r0[1] + s * di[1] - t * dj[1],
                                 r0[2] + s * di[2] - t * dj[2]};
            best.d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            best.s = s;
            best.t = t;
        }
    }
    for (int k = 0; k < 2; ++k) {
        const double sg = k ? 1.0 : -1.0;
        double u;
        const double pi[3] = {xi[0] + sg * hi * di[0], xi[1] + sg * hi * di[1], xi[2] + sg * hi * di[2]};
        double dd = point_seg(pi, xj, dj, hj, &u);
        if (dd < best.d) {
            best.d = dd;
            best.s = sg * hi;
            best.t = u;
        }
        const double pj[3] = {xj[0] + sg * hj * dj[0], xj[1] + sg * hj * dj[1], xj[2] + sg * hj * dj[2]};
        dd = point_seg(pj, xi, di, hi, &u);
        if (dd < best.d) {
            best.d = dd;
            best.s = u;
            best.t = sg * hj;
        }
    }
    return best;
}

static void normalize3(double v[3])
{
    const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n;
    v[1] /= n;
    v[2] /= n;
}

/* a unit vector normal to d */
static void any_normal(const double d[3], double out[3])
{
    const double ax = fabs(d[0]), ay = fabs(d[1]), az = fabs(d[2]);
    double e[3] = {0.0, 0.0, 0.0};
    if (ax <= ay && ax <= az) e[0] = 1.0;
    else if (ay <= az) e[1] = 1.0;
    else e[2] = 1.0;
    out[0] = d[1] * e[2] - d[2] * e[1];
    out[1] = d[2] * e[0] - d[0] * e[2];
    out[2] = d[0] * e[1] - d[1] * e[0];
    normalize3(out);
}

typedef struct {
    int nc[3], S[3];
    double cell[3], box[3];
    int *start, *idx;
} grid_t;

static int cell_of(double v, double cell, int nc)
{
    int k = (int)floor(v / cell);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

static int grid_build(grid_t *g, int64_t n, const double *x, const double box[3], double reach)
{
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int m = (int)floor(box[a] / (0.5 * reach));
        if (m < 1) m = 1;
        if (m > 512) m = 512;
        g->nc[a] = m;
        g->cell[a] = box[a] / m;
        g->S[a] = (int)ceil(reach / g->cell[a]);
        g->box[a] = box[a];
        ncell *= m;
    }
    g->start = (int *)calloc((size_t)ncell + 1, sizeof(int));
    g->idx = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *key = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!g->start || !g->idx || !key) {
        free(key);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) {
        const int k = (cell_of(x[3 * i], g->cell[0], g->nc[0]) * g->nc[1] + cell_of(x[3 * i + 1], g->cell[1], g->nc[1])) *
                          g->nc[2] +
                      cell_of(x[3 * i + 2], g->cell[2], g->nc[2]);
        key[i] = k;
        g->start[k + 1] += 1;
    }
    for (int64_t k = 0; k < ncell; ++k) g->start[k + 1] += g->start[k];
    int *fill = (int *)calloc((size_t)ncell, sizeof(int));
    if (!fill) {
        free(key);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) g->idx[g->start[key[i]] + fill[key[i]]++] = (int)i;
    free(fill);
    free(key);
    return 0;
}

static void grid_free(grid_t *g)
{
    free(g->start);
    free(g->idx);
}

/* Candidate pairs (i, j, shift) whose separation minus diam is below
 * `within`, each listed once (i < j, or i == j with a lexicographically
 * positive shift), in ascending (i, j, shift) order. */
typedef struct {
    int i, j;
    double sh[3];
} cand_t;

typedef struct {
    cand_t *v;
    int64_t n, cap;
} cands_t;

static int lex_pos(int a, int b, int c) { return a > 0 || (a == 0 && (b > 0 || (b == 0 && c > 0))); }

/* appends the candidates of rod i (j >= i) to out in stencil order; returns
 * -1 on allocation failure */
static int rod_cands(int64_t i, const grid_t *g, const double *x, const double *dir, const double *len,
                     const double box[3], double diam, double within, cands_t *out)
{
    const double *xi = x + 3 * i, *di = dir + 3 * i;
    const double hi = 0.5 * len[i];
    const double lim = diam + within;
    const int k0 = cell_of(xi[0], g->cell[0], g->nc[0]), k1 = cell_of(xi[1], g->cell[1], g->nc[1]),
              k2 = cell_of(xi[2], g->cell[2], g->nc[2]);
    for (int o0 = -g->S[0]; o0 <= g->S[0]; ++o0)
        for (int o1 = -g->S[1]; o1 <= g->S[1]; ++o1)
            for (int o2 = -g->S[2]; o2 <= g->S[2]; ++o2) {
                const int u0 = k0 + o0, u1 = k1 + o1, u2 = k2 + o2;
                const int w0 = ((u0 % g->nc[0]) + g->nc[0]) % g->nc[0];
                const int w1 = ((u1 % g->nc[1]) + g->nc[1]) % g->nc[1];
                const int w2 = ((u2 % g->nc[2]) + g->nc[2]) % g->nc[2];
                const int s0 = (u0 - w0) / g->nc[0], s1 = (u1 - w1) / g->nc[1], s2 = (u2 - w2) / g->nc[2];
                const double sh[3] = {s0 * box[0], s1 * box[1], s2 * box[2]};
                const int w = (w0 * g->nc[1] + w1) * g->nc[2] + w2;
                for (int q = g->start[w]; q < g->start[w + 1]; ++q) {
                    const int j = g->idx[q];
                    if (j < i || (j == i && !lex_pos(s0, s1, s2))) continue;
                    const double xj[3] = {x[3 * j] + sh[0], x[3 * j + 1] + sh[1], x[3 * j + 2] + sh[2]};
                    const double hj = 0.5 * len[j];
                    const double r0[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
                    const double rc = hi + hj + lim;
                    if (r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2] >= rc * rc) continue;
                    const double *dj = dir + 3 * j;
                    /* two segments are never closer than their infinite lines */
                    const double nx = di[1] * dj[2] - di[2] * dj[1], ny = di[2] * dj[0] - di[0] * dj[2],
                                 nz = di[0] * dj[1] - di[1] * dj[0];
                    const double nn = nx * nx + ny * ny + nz * nz, rn = r0[0] * nx + r0[1] * ny + r0[2] * nz;
                    if (nn > 1e-8 && rn * rn > lim * lim * nn * 1.0000001) continue;
                    const sep_t sp = separation(xi, di, hi, xj, dj, hj);
                    if (sp.d - diam >= within) continue;
                    if (out->n == out->cap) {
                        const int64_t nc = out->cap ? 2 * out->cap : 4096;
                        cand_t *v = (cand_t *)realloc(out->v, sizeof(cand_t) * (size_t)nc);
                        if (!v) return -1;
                        out->v = v;
                        out->cap = nc;
                    }
                    out->v[out->n].i = (int)i;
                    out->v[out->n].j = j;
                    memcpy(out->v[out->n].sh, sh, sizeof(sh));
                    out->n += 1;
                }
            }
    return 0;
}

/* Candidate pairs (i, j, shift) whose separation minus diam is below
 * `within`, each listed once (i < j, or i == j with a lexicographically
 * positive shift), grouped by i in ascending order.  Rods are taken in
 * chunks, each chunk fills a buffer of its own in parallel, and the buffers
 * are joined in chunk order: the list does not depend on the thread count. */
#define RS_CHUNK 256
static int build_cands(cands_t *out, int64_t n, const double *x, const double *dir, const double *len,
                       const double box[3], double diam, double within, double Lmax)
{
    grid_t g;
    const double reach = Lmax + diam + within;
    out->n = 0;
    if (grid_build(&g, n, x, box, reach)) {
        grid_free(&g);
        return -1;
    }
    const int64_t nchunk = (n + RS_CHUNK - 1) / RS_CHUNK;
    cands_t *part = (cands_t *)calloc((size_t)(nchunk > 0 ? nchunk : 1), sizeof(cands_t));
    if (!part) {
        grid_free(&g);
        return -1;
    }
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail) num_threads(g_threads)
    for (int64_t ch = 0; ch < nchunk; ++ch) {
        cands_t *pc = part + ch;
        const int64_t lo = ch * RS_CHUNK, hi = lo + RS_CHUNK < n ? lo + RS_CHUNK : n;
        for (int64_t i = lo; i < hi && !fail; ++i)
            if (rod_cands(i, &g, x, dir, len, box, diam, within, pc)) fail = 1;
    }
    int64_t total = 0;
    for (int64_t ch = 0; ch < nchunk; ++ch) total += part[ch].n;
    if (!fail && total > out->cap) {
        cand_t *v = (cand_t *)realloc(out->v, sizeof(cand_t) * (size_t)(total + 1));
        if (!v) fail = 1;
        else {
            out->v = v;
            out->cap = total + 1;
        }
    }
    if (!fail) {
        int64_t o = 0;
        for (int64_t ch = 0; ch < nchunk; ++ch) {
            if (part[ch].n) memcpy(out->v + o, part[ch].v, sizeof(cand_t) * (size_t)part[ch].n);
            o += part[ch].n;
        }
        out->n = total;
    }
    for (int64_t ch = 0; ch < nchunk; ++ch) free(part[ch].v);
    free(part);
    grid_free(&g);
    return fail ? -1 : 0;
}

/* turns unit vector d so that its point at arclength s moves by `mv` along
 * the part of u normal to d */
static void turn(double d[3], double s, double mv, const double u[3])
{
    const double ud = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
    const double f = mv / s;
    for (int a = 0; a < 3; ++a) d[a] += f * (u[a] - ud * d[a]);
    normalize3(d);
}

/* Pushes the two rods of candidate k apart if they are closer than
 * diam + gap; returns their separation minus diam. */
static double push_pair(const cand_t *cd, double *x, double *dir, const double *len, double diam, double gap,
                        int *over)
{
    const int i = cd->i, j = cd->j;
    double *xi = x + 3 * i, *di = dir + 3 * i, *xjr = x + 3 * j, *dj = dir + 3 * j;
    const double hi = 0.5 * len[i], hj = 0.5 * len[j];
    const double xj[3] = {xjr[0] + cd->sh[0], xjr[1] + cd->sh[1], xjr[2] + cd->sh[2]};
    const sep_t sp = separation(xi, di, hi, xj, dj, hj);
    const double excess = sp.d - diam;
    if (excess >= gap) return excess;
    ++*over;
    double u[3];
    if (sp.d > 1e-9) {
        for (int a = 0; a < 3; ++a) u[a] = (xi[a] + sp.s * di[a] - xj[a] - sp.t * dj[a]) / sp.d;
    } else {
        u[0] = di[1] * dj[2] - di[2] * dj[1];
        u[1] = di[2] * dj[0] - di[0] * dj[2];
        u[2] = di[0] * dj[1] - di[1] * dj[0];
        if (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] < 1e-18) any_normal(di, u);
        normalize3(u);
    }
    const double need = kOmega * (gap - excess);
    if (i == j) {
        /* a rod and its own image: only turning separates them */
        const double ds = sp.s - sp.t;
        if (fabs(ds) > 1e-6) turn(di, ds, need, u);
        return excess;
    }
    const double li = hi > 0.0 ? sp.s / hi : 0.0, lj = hj > 0.0 ? sp.t / hj : 0.0;
    const double wi = 1.0 + 3.0 * li * li, wj = 1.0 + 3.0 * lj * lj;
    /* shares of the shortfall: the contact point of rod i moves by
     * need wi / (wi + wj), that of rod j by need wj / (wi + wj) */
    const double mi = need * wi / (wi + wj), mj = need * wj / (wi + wj);
    for (int a = 0; a < 3; ++a) {
        xi[a] += mi / wi * u[a];
        xjr[a] -= mj / wj * u[a];
    }
    if (fabs(sp.s) > 1e-6) turn(di, sp.s, mi * (wi - 1.0) / wi, u);
    if (fabs(sp.t) > 1e-6) {
        const double mu[3] = {-u[0], -u[1], -u[2]};
        turn(dj, sp.t, mj * (wj - 1.0) / wj, mu);
    }
    return excess;
}

static void wrap_all(int64_t n, double *x, const double *box)
{
    for (int64_t i = 0; i < 3 * n; ++i) {
        const double b = box[i % 3];
        double v = x[i] - b * floor(x[i] / b);
        if (v >= b || v < 0.0) v = 0.0;
        x[i] = v;
    }
}

/*
 * Relaxes x[n][3] (inside [0, box)) and dir[n][3] (unit) in place until every
 * separation of two rods (or a rod and an image) exceeds diam + gap_min.
 *
 * A sweep visits the candidate pairs and moves the two rods of an overlapping
 * pair at once (Gauss-Seidel with over-relaxation kOmega), apart along the
 * normal at their closest points towards a separation of diam + gap: partly
 * by translating both centres and partly by turning both axes about their
 * centres, in the proportion 1 : 3 (s/h)^2 that the contact point at
 * arclength s of a rod of half-length h gets from a push (a rod's own image
 * is separated only by turning).  Candidates are the pairs closer than
 * diam + gap + skin, rebuilt once some point of some rod has moved by half
 * the skin.
 *
 * Parallel sweeps with a result independent of the thread count: space is
 * cut into bricks at least one pair reach wide, a multiple of three per
 * direction (or one), and a pair belongs to the brick of its first rod's
 * centre.  Bricks whose indices agree modulo 3 in every direction touch
 * disjoint sets of rods, so they are swept in parallel, one colour after the
 * other, each brick in candidate order.
 *
 * Returns the number of sweeps (>= 0), -1 when max_sweeps pass without
 * success, -2 on allocation failure; *worst_out receives the smallest
 * separation minus diam.
 */
static int relax_core(int64_t n, double *x, double *dir, const double *len, const double *box, double diam,
                      double gap, double gap_min, int max_sweeps, double *worst_out)
{
    double Lmax = 0.0;
    for (int64_t i = 0; i < n; ++i) Lmax = len[i] > Lmax ? len[i] : Lmax;
    const double skin = 6.0 * diam;
    /* a candidate's centres are within Lmax + diam + gap + skin when built and
     * each moves by at most skin / 2 before the next build */
    const double wmin = Lmax + diam + gap + 2.0 * skin;
    int nb[3];
    for (int a = 0; a < 3; ++a) {
        const int m = (int)floor(box[a] / (3.0 * wmin));
        nb[a] = m >= 1 ? 3 * m : 1;
    }
    const int nbrick = nb[0] * nb[1] * nb[2];
    double *x0 = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    double *d0 = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int *brick = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int64_t *bstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nbrick + 1));
    int64_t *bfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nbrick);
    int *border = (int *)malloc(sizeof(int) * (size_t)nbrick);
    int corder[28];
    cands_t c = {NULL, 0, 0};
    cand_t *cb = NULL;
    int64_t cbcap = 0;
    if (!x0 || !d0 || !brick || !bstart || !bfill || !border) {
        free(x0);
        free(d0);
        free(brick);
        free(bstart);
        free(bfill);
        free(border);
        return -2;
    }
    /* bricks grouped by colour: corder[col] .. corder[col + 1] in border */
    {
        int k = 0;
        for (int col = 0; col < 27; ++col) {
            corder[col] = k;
            for (int b = 0; b < nbrick; ++b) {
                const int bz = b % nb[2], by = (b / nb[2]) % nb[1], bx = b / (nb[2] * nb[1]);
                if ((bx % 3) * 9 + (by % 3) * 3 + (bz % 3) == col) border[k++] = b;
            }
        }
        corder[27] = k;
    }
    int result = -1, rebuild = 1, builds = 0;
    const int trace = getenv("RODSYNTH_TRACE") != NULL;
    for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
        if (rebuild) {
            wrap_all(n, x, box);
            const double tb = now_s();
            if (build_cands(&c, n, x, dir, len, box, diam, gap + skin, Lmax)) {
                result = -2;
                break;
            }
            /* bucket the candidates by the brick of their first rod, keeping
             * their order within a brick */
            for (int64_t i = 0; i < n; ++i) {
                int k[3];
                for (int a = 0; a < 3; ++a) {
                    k[a] = (int)floor(x[3 * i + a] / (box[a] / nb[a]));
                    k[a] = k[a] < 0 ? 0 : (k[a] >= nb[a] ? nb[a] - 1 : k[a]);
                }
                brick[i] = (k[0] * nb[1] + k[1]) * nb[2] + k[2];
            }
            memset(bstart, 0, sizeof(int64_t) * (size_t)(nbrick + 1));
            for (int64_t k = 0; k < c.n; ++k) bstart[brick[c.v[k].i] + 1] += 1;
            for (int b = 0; b < nbrick; ++b) bstart[b + 1] += bstart[b];
            if (c.n > cbcap) {
                free(cb);
                cbcap = c.n;
                cb = (cand_t *)malloc(sizeof(cand_t) * (size_t)(cbcap > 0 ? cbcap : 1));
                if (!cb) {
                    result = -2;
                    break;
                }
            }
            memcpy(bfill, bstart, sizeof(int64_t) * (size_t)nbrick);
            for (int64_t k = 0; k < c.n; ++k) cb[bfill[brick[c.v[k].i]]++] = c.v[k];
            memcpy(x0, x, sizeof(double) * 3 * (size_t)n);
            memcpy(d0, dir, sizeof(double) * 3 * (size_t)n);
            rebuild = 0;
            ++builds;
            if (trace) fprintf(stderr, "build %d: %lld candidates in %.3f s\n", builds, (long long)c.n, now_s() - tb);
        }
        double worst = INFINITY;
        int64_t over = 0;
        for (int col = 0; col < 27; ++col) {
#pragma omp parallel for schedule(dynamic, 1) reduction(min : worst) reduction(+ : over) num_threads(g_threads)
            for (int q = corder[col]; q < corder[col + 1]; ++q) {
                const int b = border[q];
                int ov = 0;
                for (int64_t k = bstart[b]; k < bstart[b + 1]; ++k) {
                    const double e = push_pair(cb + k, x, dir, len, diam, gap, &ov);
                    if (e < worst) worst = e;
                }
                over += ov;
            }
        }
        if (trace && sweep % 10 == 0)
            fprintf(stderr, "sweep %d candidates %lld overlaps %lld worst %g builds %d\n", sweep, (long long)c.n,
                    (long long)over, worst, builds);
        *worst_out = worst;
        if (worst >= gap_min) {
            result = sweep;
            break;
        }
        double maxmv = 0.0;
#pragma omp parallel for reduction(max : maxmv) num_threads(g_threads)
        for (int64_t i = 0; i < n; ++i) {
            const double *a = x + 3 * i, *a0 = x0 + 3 * i, *e = dir + 3 * i, *e0 = d0 + 3 * i;
            const double mx = sqrt((a[0] - a0[0]) * (a[0] - a0[0]) + (a[1] - a0[1]) * (a[1] - a0[1]) +
                                   (a[2] - a0[2]) * (a[2] - a0[2]));
            const double md = sqrt((e[0] - e0[0]) * (e[0] - e0[0]) + (e[1] - e0[1]) * (e[1] - e0[1]) +
                                   (e[2] - e0[2]) * (e[2] - e0[2]));
            const double mv = mx + 0.5 * len[i] * md;
            if (mv > maxmv) maxmv = mv;
        }
        if (maxmv > 0.5 * skin) rebuild = 1;
    }
    wrap_all(n, x, box);
    free(c.v);
    free(cb);
    free(x0);
    free(d0);
    free(brick);
    free(bstart);
    free(bfill);
    free(border);
    return result;
}

/* rs_relax on the rods renumbered in cell order (neighbours close in memory);
 * the results go back to the caller's order */
int rs_relax(int64_t n, double *x, double *dir, const double *len, const double *box, double diam, double gap,
             double gap_min, int max_sweeps, int threads, double *worst_out)
{
    g_threads = threads > 0 ? threads : 1;
    if (n <= 0) {
        *worst_out = INFINITY;
        return 0;
    }
    int nc[3];
    for (int a = 0; a < 3; ++a) {
        int m = (int)floor(box[a] / 0.5);
        nc[a] = m < 1 ? 1 : (m > 1024 ? 1024 : m);
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *cnt = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *xs = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *ds = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *ls = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = -2;
    if (cnt && key && perm && xs && ds && ls) {
        for (int64_t i = 0; i < n; ++i) {
            int k[3];
            for (int a = 0; a < 3; ++a) k[a] = cell_of(x[3 * i + a], box[a] / nc[a], nc[a]);
            key[i] = ((int64_t)k[0] * nc[1] + k[1]) * nc[2] + k[2];
            cnt[key[i] + 1] += 1;
        }
        for (int64_t k = 0; k < ncell; ++k) cnt[k + 1] += cnt[k];
        for (int64_t i = 0; i < n; ++i) perm[cnt[key[i]]++] = i; /* stable: ascending i within a cell */
        for (int64_t t = 0; t < n; ++t) {
            const int64_t i = perm[t];
            memcpy(xs + 3 * t, x + 3 * i, sizeof(double) * 3);
            memcpy(ds + 3 * t, dir + 3 * i, sizeof(double) * 3);
            ls[t] = len[i];
        }
        rc = relax_core(n, xs, ds, ls, box, diam, gap, gap_min, max_sweeps, worst_out);
        for (int64_t t = 0; t < n; ++t) {
            const int64_t i = perm[t];
            memcpy(x + 3 * i, xs + 3 * t, sizeof(double) * 3);
            memcpy(dir + 3 * i, ds + 3 * t, sizeof(double) * 3);
        }
    }
    free(cnt);
    free(key);
    free(perm);
    free(xs);
    free(ds);
    free(ls);
    return rc;
}
