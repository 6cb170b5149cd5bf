/*
 * Plain FP64 CPU oracle for one timestep of the constraint-based steric
 * solver for rigid filaments of Yan et al., "Towards the cellular-scale
 * simulation of motor-driven cytoskeletal assemblies" (arXiv 2109.08206).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this code; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the HIP library.
 *
 * Everything is double precision, sequential and unblocked: every loop runs
 * in the order of the definition it restates, so that a reader can check it
 * against the paper by eye.  Speed is not a goal.
 *
 * Host layout, row-major:
 *   x[n][3] centres, quat[n][4] = [s, px, py, pz], dir[n][3] unit directors,
 *   len[n] lengths (or NULL and a uniform length len0),
 *   F[n][6] = [force, torque], U[n][6] = [velocity, angular velocity],
 *   pairs: pi[nc], pj[nc], img[nc] (packed periodic shift of rod pj),
 *   e[nc][3] unit normal from rod pj to rod pi, arm[nc][2] = (s_i, s_j)
 *   arclength positions of the contact points on the two axes, phi[nc], q[nc].
 *
 * Image packing: img = ((nx+8) << 8) | ((ny+8) << 4) | (nz+8) with
 * |n| <= 7; the shift moves rod pj by n * box.  Packed values order
 * lexicographically by (nx, ny, nz); the zero shift is 0x888.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_IMG_ZERO 0x888
#define ORA_FLAG_CUTOFF 1u     /* |phi - cutoff| <= 1e-9                    */
#define ORA_FLAG_PARALLEL 2u   /* 1 - (di.dj)^2 <= 1e-10                    */
#define ORA_FLAG_DEGENERATE 4u /* axis distance < 1e-12                     */

#define ORA_EPS_PAR 1e-14
#define ORA_BAND_PAR 1e-10
#define ORA_DEGEN_DIST 1e-12
#define ORA_CUTOFF_BAND 1e-9

/* solver status codes (same meaning as the library's public ones) */
#define ORA_OK 0
#define ORA_NOT_CONVERGED 1
#define ORA_STAGNATED 2

static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }
static inline double rod_len(const double *len, double len0, int64_t i) { return len ? len[i] : len0; }

int ora_img_pack(int nx, int ny, int nz) { return ((nx + 8) << 8) | ((ny + 8) << 4) | (nz + 8); }
void ora_img_unpack(int img, int *n3)
{
    n3[0] = ((img >> 8) & 15) - 8;
    n3[1] = ((img >> 4) & 15) - 8;
    n3[2] = (img & 15) - 8;
}

/* ------------------------------------------------------------------------ */
/* Orientation.  The configuration of a rod is its centre and a unit        */
/* quaternion theta = [s, p]; the lab-frame image of a body vector Y is     */
/* R(theta) Y (Appendix "Filament dynamics": "Constraint quadratic          */
/* programming" and "Symmetry of the geometrically constrained optimization */
/* problem").  R = (s^2 - p.p) I + 2 p p^T + 2 s [p]x.  The rod axis is the */
/* body z axis, so the director is the third column of R.                   */
/* ------------------------------------------------------------------------ */
void ora_rotation(const double *q, double *R /* [3][3] row-major */)
{
    const double s = q[0], p[3] = {q[1], q[2], q[3]};
    const double pp = dot3(p, p);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) R[3 * a + b] = (a == b ? s * s - pp : 0.0) + 2.0 * p[a] * p[b];
    /* + 2 s [p]x, where ([p]x)_{ab} v_b = (p x v)_a */
    R[0 * 3 + 1] += -2.0 * s * p[2];
    R[0 * 3 + 2] += 2.0 * s * p[1];
    R[1 * 3 + 0] += 2.0 * s * p[2];
    R[1 * 3 + 2] += -2.0 * s * p[0];
    R[2 * 3 + 0] += -2.0 * s * p[1];
    R[2 * 3 + 1] += 2.0 * s * p[0];
}

void ora_directors(int64_t n, const double *quat, double *dir)
{
    double R[9];
    for (int64_t i = 0; i < n; ++i) {
        ora_rotation(quat + 4 * i, R);
        dir[3 * i + 0] = R[0 * 3 + 2];
        dir[3 * i + 1] = R[1 * 3 + 2];
        dir[3 * i + 2] = R[2 * 3 + 2];
    }
}

/* Psi(theta) Omega: the quaternion rate of a body spinning at lab-frame    */
/* angular velocity Omega.  Psi = 1/2 [ -p^T ; s I - P ], P_ij = eps_ikj p_k */
/* (Appendix "Filament dynamics", geometric matrix G).                       */
void ora_psi_times(const double *q, const double *w, double *qdot)
{
    const double s = q[0];
    double P[9];
    /* P_ij = eps_{ikj} p_k */
    const double *p = q + 1;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) {
                int eps;
                /* Levi-Civita eps_{i k j} */
                if (i == k || k == j || i == j) eps = 0;
                else eps = ((i == 0 && k == 1 && j == 2) || (i == 1 && k == 2 && j == 0) || (i == 2 && k == 0 && j == 1)) ? 1 : -1;
                v += eps * p[k];
            }
            P[3 * i + j] = v;
        }
    qdot[0] = -0.5 * dot3(p, w);
    for (int i = 0; i < 3; ++i) qdot[1 + i] = 0.5 * (s * w[i] - (P[3 * i + 0] * w[0] + P[3 * i + 1] * w[1] + P[3 * i + 2] * w[2]));
}

/* ------------------------------------------------------------------------ */
/* Mobility.  U = M F with M block diagonal, one 6x6 block per rod           */
/* (Appendix "Filament dynamics", Stokes mobility).  The paper states the   */
/* perpendicular slender-body drag 4 pi eta L / log(2L/d) (Section 3,       */
/* "Filament dynamics"); the parallel drag is half of it and the rotational */
/* drag about an axis normal to the rod is pi eta L^3 / (3 log(2L/d)), the  */
/* leading-order slender-body values.  The axial rotational mobility equals */
/* the normal one (contact torques are always normal to the axis).          */
/* coef = {a_par, a_perp, r_perp, r_par}, all mobilities (inverse drags).   */
/* ------------------------------------------------------------------------ */
void ora_mobility_coeffs(double L, double diam, double eta, double *coef)
{
    const double lg = log(2.0 * L / diam);
    const double drag_perp = 4.0 * M_PI * eta * L / lg;
    const double drag_par = 0.5 * drag_perp;
    const double drag_rot = M_PI * eta * L * L * L / (3.0 * lg);
    coef[0] = 1.0 / drag_par;
    coef[1] = 1.0 / drag_perp;
    coef[2] = 1.0 / drag_rot;
    coef[3] = coef[2];
}

/* The 6x6 mobility block of one rod, row-major. */
void ora_mobility_block(const double *d, double L, double diam, double eta, double *M6)
{
    double c[4];
    ora_mobility_coeffs(L, diam, eta, c);
    memset(M6, 0, 36 * sizeof(double));
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double ddt = d[a] * d[b];
            M6[6 * a + b] = (a == b ? c[1] : 0.0) + (c[0] - c[1]) * ddt;
            M6[6 * (a + 3) + (b + 3)] = (a == b ? c[2] : 0.0) + (c[3] - c[2]) * ddt;
        }
}

void ora_apply_mobility(int64_t n, const double *dir, const double *len, double len0, double diam, double eta,
                        const double *F, double *U)
{
    double M6[36];
    for (int64_t i = 0; i < n; ++i) {
        ora_mobility_block(dir + 3 * i, rod_len(len, len0, i), diam, eta, M6);
        for (int a = 0; a < 6; ++a) {
            double v = 0.0;
            for (int b = 0; b < 6; ++b) v += M6[6 * a + b] * F[6 * i + b];
            U[6 * i + a] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Minimal distance between two rods.  The separation of a pair is the      */
/* minimal distance between the filaments, zero at contact (Section 3,      */
/* "Filament dynamics"); the constraint geometry uses the two closest       */
/* points, r = x_P + y_P - x_Q - y_Q (Appendix figure "pairwise geometry"). */
/* For spherocylinders of diameter d the surface gap is the axis distance   */
/* minus d.                                                                 */
/*                                                                          */
/* Axis i: x_i + s dir_i, |s| <= L_i/2.  Axis j (already imaged):           */
/* xj + t dir_j, |t| <= L_j/2.  The squared distance is a convex quadratic  */
/* in (s, t); we take the clamped normal-equation method for segment pairs  */
/* (Lumelsky 1985; Ericson, Real-Time Collision Detection, 2005, 5.1.9):    */
/* minimise over s with t free, clamp; take the best t for that s; if that  */
/* t leaves its range, clamp it and re-take the best s.  Near-parallel axes */
/* use the midpoint of the overlap of the two parameter ranges.             */
/* ------------------------------------------------------------------------ */
typedef struct {
    double s, t, dist;
    double r[3]; /* closest point on i minus closest point on j */
    double e[3]; /* unit normal from j to i */
    unsigned flags;
} ora_contact;

static double seg_dist2(const double *r0, const double *di, const double *dj, double s, double t, double *r)
{
    for (int a = 0; a < 3; ++a) r[a] = r0[a] + s * di[a] - t * dj[a];
    return dot3(r, r);
}

void ora_closest(const double *xi, const double *di, double Li, const double *xj, const double *dj, double Lj,
                 ora_contact *out)
{
    const double hi = 0.5 * Li, hj = 0.5 * Lj;
    double r0[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
    const double b = dot3(di, dj);
    const double c = dot3(di, r0);
    const double f = dot3(dj, r0);
    const double den = 1.0 - b * b;
    double s, t;
    unsigned flags = 0;
    if (den <= ORA_BAND_PAR) flags |= ORA_FLAG_PARALLEL;
    if (den > ORA_EPS_PAR) {
        /* stationary point of |r0 + s di - t dj|^2: s - b t = -c, b s - t = -f */
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
        /* parallel: the s for which the foot point b s + f lies on axis j */
        const double bs = (b >= 0.0) ? 1.0 : -1.0; /* b is +-1 up to rounding */
        double lo = (-hj - f) * bs, up = (hj - f) * bs;
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
            /* disjoint along the axis: best of the end-point candidates */
            double best = INFINITY, rr[3];
            const double cs[4][2] = {{-hi, 0}, {hi, 0}, {0, -hj}, {0, hj}};
            s = 0.0;
            t = 0.0;
            for (int k = 0; k < 4; ++k) {
                double sk, tk;
                if (k < 2) {
                    sk = cs[k][0];
                    tk = clampd(b * sk + f, -hj, hj);
                } else {
                    tk = cs[k][1];
                    sk = clampd(b * tk - c, -hi, hi);
                }
                const double d2 = seg_dist2(r0, di, dj, sk, tk, rr);
                if (d2 < best) {
                    best = d2;
                    s = sk;
                    t = tk;
                }
            }
        }
    }
    seg_dist2(r0, di, dj, s, t, out->r);
    const double dist = sqrt(dot3(out->r, out->r));
    out->s = s;
    out->t = t;
    out->dist = dist;
    if (dist >= ORA_DEGEN_DIST) {
        for (int a = 0; a < 3; ++a) out->e[a] = out->r[a] / dist;
    } else {
        /* axes intersect: normal to both axes, oriented along r0 */
        double n3[3];
        flags |= ORA_FLAG_DEGENERATE;
        cross3(di, dj, n3);
        double nn = sqrt(dot3(n3, n3));
        if (nn < 1e-12) {
            /* collinear: normal to di and the coordinate axis least aligned with it */
            int k = 0;
            for (int a = 1; a < 3; ++a)
                if (fabs(di[a]) < fabs(di[k])) k = a;
            double ek[3] = {0, 0, 0};
            ek[k] = 1.0;
            cross3(di, ek, n3);
            nn = sqrt(dot3(n3, n3));
        }
        double sg = (dot3(n3, r0) >= 0.0) ? 1.0 : -1.0;
        for (int a = 0; a < 3; ++a) out->e[a] = sg * n3[a] / nn;
    }
    out->flags = flags;
}

/* Convenience wrapper for the test suite: out7 = {s, t, dist, e0, e1, e2, flags}. */
void ora_closest_flat(const double *xi, const double *di, double Li, const double *xj, const double *dj, double Lj,
                      double *out7)
{
    ora_contact c;
    ora_closest(xi, di, Li, xj, dj, Lj, &c);
    out7[0] = c.s;
    out7[1] = c.t;
    out7[2] = c.dist;
    out7[3] = c.e[0];
    out7[4] = c.e[1];
    out7[5] = c.e[2];
    out7[6] = (double)c.flags;
}

/* ------------------------------------------------------------------------ */
/* Near-contact pairs.  Only pairs whose minimal distance is below the      */
/* threshold enter the solver (Appendix "Implementation").  Here the        */
/* threshold applies to the surface gap phi, strictly.  The set is          */
/* { (i, j, n) : phi(i, j + n box) < cutoff }, listed once per unordered    */
/* contact: i < j with any shift n, or i == j with n lexicographically      */
/* positive (a rod touching its own periodic image).                        */
/* ------------------------------------------------------------------------ */

/* one candidate: closest point with rod j shifted by n * box */
static int pair_test(const double *x, const double *dir, const double *len, double len0, const double *box, int64_t i,
                     int64_t j, const int *n3, double diam, double cutoff, ora_contact *c)
{
    const double Li = rod_len(len, len0, i), Lj = rod_len(len, len0, j);
    double xj[3];
    for (int a = 0; a < 3; ++a) xj[a] = x[3 * j + a] + n3[a] * box[a];
    /* exact reject: the axes are at least |xi - xj| - (Li + Lj)/2 apart */
    double r0[3] = {x[3 * i] - xj[0], x[3 * i + 1] - xj[1], x[3 * i + 2] - xj[2]};
    const double reach = 0.5 * (Li + Lj) + diam + cutoff;
    if (dot3(r0, r0) >= reach * reach) return 0;
    ora_closest(x + 3 * i, dir + 3 * i, Li, xj, dir + 3 * j, Lj, c);
    const double phi = c->dist - diam;
    if (!(phi < cutoff)) return 0;
    if (fabs(phi - cutoff) <= ORA_CUTOFF_BAND) c->flags |= ORA_FLAG_CUTOFF;
    return 1;
}

static int lex_positive(const int *n3)
{
    for (int a = 0; a < 3; ++a) {
        if (n3[a] > 0) return 1;
        if (n3[a] < 0) return 0;
    }
    return 0;
}

static double max_len(int64_t n, const double *len, double len0)
{
    if (!len) return len0;
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = len[i] > m ? len[i] : m;
    return m;
}

/* Brute force over all (i, j, n): the definition.  Returns the number of   */
/* pairs; writes at most cap of them, in canonical order (i, j, img).       */
int64_t ora_pairs_brute(int64_t n, const double *x, const double *dir, const double *len, double len0, const double *box,
                        double diam, double cutoff, int64_t cap, int32_t *pi, int32_t *pj, int32_t *img, uint8_t *flags)
{
    const double rcut = max_len(n, len, len0) + diam + cutoff;
    int m[3];
    for (int a = 0; a < 3; ++a) m[a] = (int)ceil(rcut / box[a]);
    int64_t cnt = 0;
    ora_contact c;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i; j < n; ++j)
            for (int nx = -m[0]; nx <= m[0]; ++nx)
                for (int ny = -m[1]; ny <= m[1]; ++ny)
                    for (int nz = -m[2]; nz <= m[2]; ++nz) {
                        const int n3[3] = {nx, ny, nz};
                        if (j == i && !lex_positive(n3)) continue;
                        if (!pair_test(x, dir, len, len0, box, i, j, n3, diam, cutoff, &c)) continue;
                        if (cnt < cap) {
                            pi[cnt] = (int32_t)i;
                            pj[cnt] = (int32_t)j;
                            img[cnt] = ora_img_pack(nx, ny, nz);
                            flags[cnt] = (uint8_t)c.flags;
                        }
                        ++cnt;
                    }
    return cnt;
}

/* A plain uniform-grid cell list, independent of the brute force: bin by   */
/* centre into cells no smaller than the interaction reach, visit the       */
/* stencil of cells around each rod's cell (with periodic wrap recorded as  */
/* an image shift), then sort each rod's list by (j, img).                  */
typedef struct {
    int32_t j, img;
    uint8_t fl;
} ora_cand;

static int cand_cmp(const void *a, const void *b)
{
    const ora_cand *u = (const ora_cand *)a, *v = (const ora_cand *)b;
    if (u->j != v->j) return u->j < v->j ? -1 : 1;
    if (u->img != v->img) return u->img < v->img ? -1 : 1;
    return 0;
}

int64_t ora_pairs_cells(int64_t n, const double *x, const double *dir, const double *len, double len0, const double *box,
                        double diam, double cutoff, int64_t cap, int32_t *pi, int32_t *pj, int32_t *img, uint8_t *flags)
{
    const double rcut = max_len(n, len, len0) + diam + cutoff;
    int nc[3], S[3];
    double cell[3];
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int)floor(box[a] / rcut);
        if (nc[a] < 1) nc[a] = 1;
        cell[a] = box[a] / nc[a];
        S[a] = (int)ceil(rcut / cell[a]);
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (ncell + 1));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int (*cc)[3] = malloc(sizeof(int[3]) * (n > 0 ? n : 1));
    for (int64_t k = 0; k <= ncell; ++k) head[k] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            int k = (int)floor(x[3 * i + a] / cell[a]);
            if (k < 0) k = 0;
            if (k >= nc[a]) k = nc[a] - 1;
            cc[i][a] = k;
        }
        cid[i] = ((int64_t)cc[i][0] * nc[1] + cc[i][1]) * nc[2] + cc[i][2];
        head[cid[i] + 1]++;
    }
    for (int64_t k = 0; k < ncell; ++k) head[k + 1] += head[k];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (ncell + 1));
        memcpy(fill, head, sizeof(int64_t) * (ncell + 1));
        for (int64_t i = 0; i < n; ++i) order[fill[cid[i]]++] = i;
        free(fill);
    }
    int64_t cnt = 0, lcap = 64;
    ora_cand *list = (ora_cand *)malloc(sizeof(ora_cand) * lcap);
    ora_contact c;
    for (int64_t i = 0; i < n; ++i) {
        int64_t nl = 0;
        for (int ox = -S[0]; ox <= S[0]; ++ox)
            for (int oy = -S[1]; oy <= S[1]; ++oy)
                for (int oz = -S[2]; oz <= S[2]; ++oz) {
                    const int o[3] = {ox, oy, oz};
                    int w[3], sh[3];
                    for (int a = 0; a < 3; ++a) {
                        const int u = cc[i][a] + o[a];
                        w[a] = ((u % nc[a]) + nc[a]) % nc[a];
                        sh[a] = (u - w[a]) / nc[a]; /* rod j is moved by sh * box */
                    }
                    const int64_t k = ((int64_t)w[0] * nc[1] + w[1]) * nc[2] + w[2];
                    for (int64_t q = head[k]; q < head[k + 1]; ++q) {
                        const int64_t j = order[q];
                        if (j < i || (j == i && !lex_positive(sh))) continue;
                        if (!pair_test(x, dir, len, len0, box, i, j, sh, diam, cutoff, &c)) continue;
                        if (nl == lcap) {
                            lcap *= 2;
                            list = (ora_cand *)realloc(list, sizeof(ora_cand) * lcap);
                        }
                        list[nl].j = (int32_t)j;
                        list[nl].img = ora_img_pack(sh[0], sh[1], sh[2]);
                        list[nl].fl = (uint8_t)c.flags;
                        ++nl;
                    }
                }
        qsort(list, (size_t)nl, sizeof(ora_cand), cand_cmp);
        for (int64_t k = 0; k < nl; ++k) {
            if (cnt < cap) {
                pi[cnt] = (int32_t)i;
                pj[cnt] = list[k].j;
                img[cnt] = list[k].img;
                flags[cnt] = list[k].fl;
            }
            ++cnt;
        }
    }
    free(list);
    free(head);
    free(order);
    free(cid);
    free(cc);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Constraint geometry.  For pair c = (P, Q) = (pi, pj) the column of the   */
/* constraint matrix is D_c = [e; y_P x e; -e; -(y_Q x e)] with             */
/* e = r/|r| pointing from Q to P and y the lever arms from the centres to  */
/* the closest points (Appendix "Equation of motion with geometric          */
/* constraints", force map F_u = D_u gamma_u, and "Symmetry ...": D_PQ).    */
/* phi = |r| - diam.  q = phi/h + D^T M F_nc (eq. blockdef, block A).       */
/* ------------------------------------------------------------------------ */
static void pair_geometry(const double *x, const double *dir, const double *len, double len0, const double *box,
                          int32_t i, int32_t j, int32_t im, ora_contact *c)
{
    int n3[3];
    ora_img_unpack(im, n3);
    double xj[3];
    for (int a = 0; a < 3; ++a) xj[a] = x[3 * j + a] + n3[a] * box[a];
    ora_closest(x + 3 * i, dir + 3 * i, rod_len(len, len0, i), xj, dir + 3 * j, rod_len(len, len0, j), c);
}

/* Full 12-entry column of D for constraint c: [F_P(3), T_P(3), F_Q(3), T_Q(3)] per unit gamma. */
/* A constraint against a fixed body (j < 0: a wall, or a tether to a fixed */
/* point) has no Q side: only e_P and y_P enter D (Appendix "Equation of    */
/* motion with geometric constraints", last paragraph).                     */
static void d_column(const double *dir, int32_t i, int32_t j, const double *e, double si, double sj, double *col)
{
    double yP[3], yQ[3], t[3];
    for (int a = 0; a < 3; ++a) {
        yP[a] = si * dir[3 * i + a];
        yQ[a] = j >= 0 ? sj * dir[3 * j + a] : 0.0;
    }
    for (int a = 0; a < 3; ++a) col[a] = e[a];
    cross3(yP, e, t);
    for (int a = 0; a < 3; ++a) col[3 + a] = t[a];
    if (j < 0) {
        for (int a = 6; a < 12; ++a) col[a] = 0.0;
        return;
    }
    double me[3] = {-e[0], -e[1], -e[2]};
    for (int a = 0; a < 3; ++a) col[6 + a] = me[a];
    cross3(yQ, me, t);
    for (int a = 0; a < 3; ++a) col[9 + a] = t[a];
}

void ora_assemble(int64_t n, const double *x, const double *dir, const double *len, double len0, const double *box,
                  double diam, double eta, double dt, int64_t nc, const int32_t *pi, const int32_t *pj,
                  const int32_t *img, const double *F, double *phi, double *e, double *arm, double *q)
{
    double *Unc = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    ora_apply_mobility(n, dir, len, len0, diam, eta, F, Unc);
    ora_contact c;
    double col[12];
    for (int64_t k = 0; k < nc; ++k) {
        pair_geometry(x, dir, len, len0, box, pi[k], pj[k], img[k], &c);
        phi[k] = c.dist - diam;
        for (int a = 0; a < 3; ++a) e[3 * k + a] = c.e[a];
        arm[2 * k + 0] = c.s;
        arm[2 * k + 1] = c.t;
        d_column(dir, pi[k], pj[k], c.e, c.s, c.t, col);
        double dtu = 0.0;
        for (int a = 0; a < 6; ++a) dtu += col[a] * Unc[6 * pi[k] + a] + col[6 + a] * Unc[6 * pj[k] + a];
        q[k] = phi[k] / dt + dtu;
    }
    free(Unc);
}

/* Dense D (6n x nc, row-major) for small systems, for the dense cross-checks. */
void ora_dense_D(int64_t n, const double *dir, int64_t nc, const int32_t *pi, const int32_t *pj, const double *e,
                 const double *arm, double *D)
{
    memset(D, 0, sizeof(double) * 6 * n * nc);
    double col[12];
    for (int64_t k = 0; k < nc; ++k) {
        d_column(dir, pi[k], pj[k], e + 3 * k, arm[2 * k], arm[2 * k + 1], col);
        for (int a = 0; a < 6; ++a) {
            D[(6 * (int64_t)pi[k] + a) * nc + k] += col[a];
            if (pj[k] >= 0) D[(6 * (int64_t)pj[k] + a) * nc + k] += col[6 + a];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Matrix-free constraint-space operator: w = Mc gamma + q with             */
/* Mc = D^T M D (eq. blockdef, block B; eq. suppcqpdef).  D gamma is a      */
/* scatter over constraints, M is applied per rod, D^T U is a gather.       */
/* Fc[n][6] receives D gamma and Uc[n][6] receives M D gamma.               */
/* ------------------------------------------------------------------------ */
/* General constraint set (used by the bilateral and wall extensions):      */
/* kind[c] = 0 for a unilateral constraint (gamma_c >= 0, complementarity), */
/* 1 for a bilateral one (gamma_c free; eq. linearconstraints b), whose row */
/* of Mc carries the compliance cmp[c] = 1/(kappa_c h) on the diagonal       */
/* (eq. blockdef, block F: D_b^T M D_b + K^-1 / h).  kind == NULL: all      */
/* unilateral.  pj[c] < 0: a constraint against a fixed body.               */
typedef struct {
    int64_t n, nc;
    const double *dir, *len;
    double len0, diam, eta;
    const int32_t *pi, *pj;
    const double *e, *arm, *q;
    const uint8_t *kind;
    const double *cmp;
} ora_sys;

static int is_bilateral(const ora_sys *S, int64_t k) { return S->kind && S->kind[k]; }

static void sys_D_gamma(const ora_sys *S, const double *gamma, double *Fc)
{
    double col[12];
    memset(Fc, 0, sizeof(double) * 6 * S->n);
    for (int64_t k = 0; k < S->nc; ++k) {
        d_column(S->dir, S->pi[k], S->pj[k], S->e + 3 * k, S->arm[2 * k], S->arm[2 * k + 1], col);
        for (int a = 0; a < 6; ++a) {
            Fc[6 * S->pi[k] + a] += col[a] * gamma[k];
            if (S->pj[k] >= 0) Fc[6 * S->pj[k] + a] += col[6 + a] * gamma[k];
        }
    }
}

static void sys_DT_U(const ora_sys *S, const double *U, double *w)
{
    double col[12];
    for (int64_t k = 0; k < S->nc; ++k) {
        d_column(S->dir, S->pi[k], S->pj[k], S->e + 3 * k, S->arm[2 * k], S->arm[2 * k + 1], col);
        double v = 0.0;
        for (int a = 0; a < 6; ++a) {
            v += col[a] * U[6 * S->pi[k] + a];
            if (S->pj[k] >= 0) v += col[6 + a] * U[6 * S->pj[k] + a];
        }
        w[k] = v;
    }
}

/* w = Mc gamma (+ q if add_q); Mc includes the bilateral compliances */
static void sys_apply(const ora_sys *S, const double *gamma, int add_q, double *Fc, double *Uc, double *w)
{
    sys_D_gamma(S, gamma, Fc);
    ora_apply_mobility(S->n, S->dir, S->len, S->len0, S->diam, S->eta, Fc, Uc);
    sys_DT_U(S, Uc, w);
    for (int64_t k = 0; k < S->nc; ++k)
        if (is_bilateral(S, k)) w[k] += S->cmp[k] * gamma[k];
    if (add_q)
        for (int64_t k = 0; k < S->nc; ++k) w[k] += S->q[k];
}

void ora_apply_Mc(int64_t n, const double *dir, const double *len, double len0, double diam, double eta, int64_t nc,
                  const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                  const double *gamma, double *w)
{
    ora_sys S = {n, nc, dir, len, len0, diam, eta, pi, pj, e, arm, q, NULL, NULL};
    double *Fc = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    double *Uc = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    sys_apply(&S, gamma, q != NULL, Fc, Uc, w);
    free(Fc);
    free(Uc);
}

/* U = M (D gamma + F): the rod velocities once gamma is known (eq.        */
/* constrainedeom_euler, second line).                                      */
void ora_velocity(int64_t n, const double *dir, const double *len, double len0, double diam, double eta, int64_t nc,
                  const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *gamma,
                  const double *F, double *U)
{
    ora_sys S = {n, nc, dir, len, len0, diam, eta, pi, pj, e, arm, NULL, NULL, NULL};
    double *Ft = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    sys_D_gamma(&S, gamma, Ft);
    for (int64_t k = 0; k < 6 * n; ++k) Ft[k] += F[k];
    ora_apply_mobility(n, dir, len, len0, diam, eta, Ft, U);
    free(Ft);
}

/* ------------------------------------------------------------------------ */
/* Barzilai-Borwein projected gradient descent on                           */
/*   min 1/2 g^T Mc g + q^T g  s.t. g >= 0   (eq. cqpdef / suppcqpdef),      */
/* whose gradient Mc gamma + q is one sparse product (Section               */
/* "Instantiation in a massively parallel computing environment").  The     */
/* paper names the method and defers its details to earlier work; this is   */
/* the projected BB iteration (Barzilai & Borwein 1988; Dai & Fletcher      */
/* 2005) with the choices below.                                            */
/*                                                                          */
/* residual(gamma, g) = max_c |min(gamma_c, g_c)|, the natural residual of  */
/* the complementarity conditions gamma >= 0, g >= 0, gamma.g = 0.          */
/*                                                                          */
/* start: gamma0 given (>= 0), g0 = Mc gamma0 + q; stop if residual <= tol. */
/* alpha0 = gh.gh / gh.Mc gh with gh the projected gradient (gh_c = 0 where */
/* gamma_c = 0 and g_c > 0); stop if gh = 0; alpha0 = 1 if gh.Mc gh <= 0.   */
/* iteration k = 0, 1, ...:                                                 */
/*   gamma' = max(0, gamma - alpha g); g' = Mc gamma' + q;                  */
/*   stop if residual(gamma', g') <= tol;                                   */
/*   s = gamma' - gamma, y = g' - g; s.s == 0 -> stagnated;                 */
/*   if s.y > 0: alpha = s.s/s.y (k even) or s.y/y.y (k odd), clamped to    */
/*   [1e-12 alpha0, 1e12 alpha0]; otherwise alpha is kept.                  */
/* info = {iterations, residual, status}.                                   */
/* ------------------------------------------------------------------------ */
static double natural_residual(const ora_sys *S, const double *gamma, const double *g)
{
    double r = 0.0;
    for (int64_t k = 0; k < S->nc; ++k) {
        /* bilateral rows: the residual of the equation itself, |w| */
        const double m = is_bilateral(S, k) ? fabs(g[k]) : fabs(gamma[k] < g[k] ? gamma[k] : g[k]);
        r = m > r ? m : r;
    }
    return r;
}

static int bbpgd_core(const ora_sys *S, double tol, int64_t max_iter, double *gamma, double *g_out, double *info)
{
    const int64_t n = S->n, nc = S->nc;
    const int64_t nb = nc > 0 ? nc : 1, rb = n > 0 ? n : 1;
    double *g = (double *)malloc(sizeof(double) * nb), *gn = (double *)malloc(sizeof(double) * nb);
    double *gam_n = (double *)malloc(sizeof(double) * nb), *gh = (double *)malloc(sizeof(double) * nb);
    double *Fc = (double *)malloc(sizeof(double) * 6 * rb), *Uc = (double *)malloc(sizeof(double) * 6 * rb);
    int status = ORA_OK;
    int64_t it = 0;
    double res, alpha = 1.0, alpha0 = 1.0;

    /* projection onto the feasible set: gamma_u >= 0, gamma_b free */
    for (int64_t k = 0; k < nc; ++k)
        if (!is_bilateral(S, k)) gamma[k] = gamma[k] > 0.0 ? gamma[k] : 0.0;
    sys_apply(S, gamma, 1, Fc, Uc, g);
    res = natural_residual(S, gamma, g);
    if (res > tol) {
        double ghgh = 0.0, ghMgh = 0.0;
        for (int64_t k = 0; k < nc; ++k) {
            gh[k] = (!is_bilateral(S, k) && gamma[k] <= 0.0 && g[k] > 0.0) ? 0.0 : g[k];
            ghgh += gh[k] * gh[k];
        }
        if (ghgh == 0.0) goto done;
        sys_apply(S, gh, 0, Fc, Uc, gn);
        for (int64_t k = 0; k < nc; ++k) ghMgh += gh[k] * gn[k];
        alpha0 = ghMgh > 0.0 ? ghgh / ghMgh : 1.0;
        alpha = alpha0;
        status = ORA_NOT_CONVERGED;
        for (int64_t k = 0; k < max_iter; ++k) {
            for (int64_t c = 0; c < nc; ++c) {
                const double v = gamma[c] - alpha * g[c];
                gam_n[c] = (is_bilateral(S, c) || v > 0.0) ? v : 0.0;
            }
            sys_apply(S, gam_n, 1, Fc, Uc, gn);
            it = k + 1;
            res = natural_residual(S, gam_n, gn);
            double ss = 0.0, sy = 0.0, yy = 0.0;
            for (int64_t c = 0; c < nc; ++c) {
                const double sc = gam_n[c] - gamma[c], yc = gn[c] - g[c];
                ss += sc * sc;
                sy += sc * yc;
                yy += yc * yc;
            }
            memcpy(gamma, gam_n, sizeof(double) * nc);
            memcpy(g, gn, sizeof(double) * nc);
            if (res <= tol) {
                status = ORA_OK;
                break;
            }
            if (ss == 0.0) {
                status = ORA_STAGNATED;
                break;
            }
            if (sy > 0.0) {
                alpha = (k % 2 == 0) ? ss / sy : sy / yy;
                alpha = clampd(alpha, 1e-12 * alpha0, 1e12 * alpha0);
            }
        }
    }
done:
    if (g_out) memcpy(g_out, g, sizeof(double) * nc);
    if (info) {
        info[0] = (double)it;
        info[1] = res;
        info[2] = alpha0;
    }
    free(g);
    free(gn);
    free(gam_n);
    free(gh);
    free(Fc);
    free(Uc);
    return status;
}

int ora_bbpgd(int64_t n, const double *dir, const double *len, double len0, double diam, double eta, int64_t nc,
              const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q, double tol,
              int64_t max_iter, double *gamma /* in: start, out: solution */, double *g_out /* may be NULL */,
              double *info /* [3]: iterations, residual, alpha0 */)
{
    ora_sys S = {n, nc, dir, len, len0, diam, eta, pi, pj, e, arm, q, NULL, NULL};
    return bbpgd_core(&S, tol, max_iter, gamma, g_out, info);
}

/* ------------------------------------------------------------------------ */
/* Mixed problem of eq. linearconstraints: unilateral constraints           */
/* (kind 0) and bilateral ones (kind 1, compliance cmp), in any order, some */
/* possibly against fixed bodies (pj < 0).  The quadratic program of eq.    */
/* suppcqpdef with gamma_u >= 0 and gamma_b free, by the same BBPGD: the    */
/* projection and the projected gradient leave bilateral entries alone,     */
/* and the stop test uses |w_b| for them.                                    */
/* ------------------------------------------------------------------------ */
int ora_bbpgd_gen(int64_t n, const double *dir, const double *len, double len0, double diam, double eta, int64_t nc,
                  const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                  const uint8_t *kind, const double *cmp, double tol, int64_t max_iter, double *gamma,
                  double *g_out, double *info)
{
    ora_sys S = {n, nc, dir, len, len0, diam, eta, pi, pj, e, arm, q, kind, cmp};
    return bbpgd_core(&S, tol, max_iter, gamma, g_out, info);
}

void ora_apply_Mc_gen(int64_t n, const double *dir, const double *len, double len0, double diam, double eta,
                      int64_t nc, const int32_t *pi, const int32_t *pj, const double *e, const double *arm,
                      const double *q, const uint8_t *kind, const double *cmp, const double *gamma, double *w)
{
    ora_sys S = {n, nc, dir, len, len0, diam, eta, pi, pj, e, arm, q, kind, cmp};
    double *Fc = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    double *Uc = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    sys_apply(&S, gamma, q != NULL, Fc, Uc, w);
    free(Fc);
    free(Uc);
}

/* ------------------------------------------------------------------------ */
/* Bilateral (spring) constraints: a Hookean link between the point at      */
/* arclength sP on rod P's axis and the point at sQ on rod Q's axis         */
/* (points fixed on the bodies; Appendix "Equation of motion with geometric */
/* constraints": Phi_b is the distance between two fixed points, the link's */
/* length).  r = x_P + sP d_P - (x_Q + sQ d_Q), each component of the       */
/* centre difference taken to its nearest periodic image; length = |r|,     */
/* e = r / |r| (from Q to P, gamma > 0 pushes the ends apart), the column   */
/* of D is [e; y_P x e; -e; -(y_Q x e)] as for a contact (Appendix          */
/* "Symmetry ...": the points are arbitrary for bilateral constraints).     */
/* The Hookean law K (Phi_b - Phi_b^0) = -gamma_b (eq. bilateralconstraint) */
/* linearised over the step gives the row (eq. linearconstraints b; eq.     */
/* blockdef D and F): q_b = (length - rest)/h + D_b^T M F, and the diagonal */
/* compliance cmp = 1/(kappa h) (kappa = +inf: a rigid joint, cmp = 0).     */
/* A link of zero length has no direction: e is then taken normal to both   */
/* axes, d_P x d_Q normalised, or d_P x (the coordinate axis least aligned  */
/* with d_P) when the axes are parallel; its flag is set.  Q < 0 anchors    */
/* the link at the fixed point (sQ unused) given in anchor[3*k].            */
/* ------------------------------------------------------------------------ */
static void unit_normal_of(const double *dP, const double *dQ, double *e)
{
    double c[3];
    cross3(dP, dQ, c);
    double nn = sqrt(dot3(c, c));
    if (nn < 1e-12) {
        const double ax = fabs(dP[0]), ay = fabs(dP[1]), az = fabs(dP[2]);
        double ek[3] = {0.0, 0.0, 0.0};
        int k = 0;
        double best = ax;
        if (ay < best) {
            k = 1;
            best = ay;
        }
        if (az < best) k = 2;
        ek[k] = 1.0;
        cross3(dP, ek, c);
        nn = sqrt(dot3(c, c));
    }
    for (int a = 0; a < 3; ++a) e[a] = c[a] / nn;
}

void ora_links(int64_t n, const double *x, const double *dir, const double *len, double len0, const double *box,
               double diam, double eta, double dt, int64_t nl, const int32_t *lp, const int32_t *lq,
               const double *sarm, const double *kappa, const double *rest, const double *anchor, const double *F,
               double *length, double *e, double *q, double *cmp, uint8_t *flags)
{
    double *Unc = (double *)calloc((size_t)(6 * (n > 0 ? n : 1)), sizeof(double));
    if (F) ora_apply_mobility(n, dir, len, len0, diam, eta, F, Unc);
    for (int64_t k = 0; k < nl; ++k) {
        const int32_t P = lp[k], Q = lq[k];
        const double sP = sarm[2 * k], sQ = sarm[2 * k + 1];
        double r[3];
        for (int a = 0; a < 3; ++a) {
            const double aP = x[3 * P + a] + sP * dir[3 * P + a];
            const double aQ = Q >= 0 ? x[3 * Q + a] + sQ * dir[3 * Q + a] : anchor[3 * k + a];
            double d = aP - aQ;
            d -= box[a] * floor(d / box[a] + 0.5);
            r[a] = d;
        }
        const double L = sqrt(dot3(r, r));
        flags[k] = 0;
        if (L < ORA_DEGEN_DIST) {
            const double ez[3] = {0.0, 0.0, 1.0};
            unit_normal_of(dir + 3 * P, Q >= 0 ? dir + 3 * Q : ez, e + 3 * k);
            flags[k] = ORA_FLAG_DEGENERATE;
        } else {
            for (int a = 0; a < 3; ++a) e[3 * k + a] = r[a] / L;
        }
        length[k] = L;
        double col[12];
        d_column(dir, P, Q, e + 3 * k, sP, sQ, col);
        double dtu = 0.0;
        for (int a = 0; a < 6; ++a) {
            dtu += col[a] * Unc[6 * P + a];
            if (Q >= 0) dtu += col[6 + a] * Unc[6 * Q + a];
        }
        q[k] = (L - rest[k]) / dt + dtu;
        cmp[k] = isinf(kappa[k]) ? 0.0 : 1.0 / (kappa[k] * dt);
    }
    free(Unc);
}

/* ------------------------------------------------------------------------ */
/* Brownian force (F_nc = Brownian + external, Appendix "Filament dynamics" */
/* and eq. mobilitydef).  The paper does not print the noise amplitude; the */
/* overdamped Langevin equation with the fluctuation-dissipation relation    */
/* gives a velocity noise of covariance 2 kT M / h over one Euler step,      */
/* i.e. U_B = sqrt(2 kT / h) M^(1/2) xi with xi ~ N(0, I_6) per rod, or as a  */
/* force F_B = sqrt(2 kT / h) M^(-1/2) xi (so that M F_B = U_B).  M^(1/2) of */
/* the block a_perp I + (a_par - a_perp) d d^T is sqrt(a_perp) I +           */
/* (sqrt(a_par) - sqrt(a_perp)) d d^T (same eigenvectors); the rotational    */
/* block is r I (axial = normal).  xi is passed in: the oracle draws        */
/* nothing.                                                                 */
/* ------------------------------------------------------------------------ */
void ora_mobility_pow_block(const double *d, double L, double diam, double eta, double power, double *M6)
{
    double c[4];
    ora_mobility_coeffs(L, diam, eta, c);
    const double ap = pow(c[0], power), an = pow(c[1], power), rn = pow(c[2], power), rp = pow(c[3], power);
    memset(M6, 0, 36 * sizeof(double));
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double ddt = d[a] * d[b];
            M6[6 * a + b] = (a == b ? an : 0.0) + (ap - an) * ddt;
            M6[6 * (a + 3) + (b + 3)] = (a == b ? rn : 0.0) + (rp - rn) * ddt;
        }
}

void ora_brownian_force(int64_t n, const double *dir, const double *len, double len0, double diam, double eta,
                        double dt, double kT, const double *xi, double *FB)
{
    const double amp = sqrt(2.0 * kT / dt);
    double M6[36];
    for (int64_t i = 0; i < n; ++i) {
        ora_mobility_pow_block(dir + 3 * i, rod_len(len, len0, i), diam, eta, -0.5, M6);
        for (int a = 0; a < 6; ++a) {
            double v = 0.0;
            for (int b = 0; b < 6; ++b) v += M6[6 * a + b] * xi[6 * i + b];
            FB[6 * i + a] = amp * v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Walls (confinement): constraints between a rod and a fixed body, with    */
/* only the rod's side in D (Appendix "Equation of motion with geometric    */
/* constraints", last paragraph: a flat substrate or a spherical shell).    */
/* Wall kinds, as 8 doubles {kind, p[3], a[3], r}:                          */
/*   0 plane: the allowed side is a.x >= a.p (a unit normal, pointing in);  */
/*   1 sphere, rods inside: |x - p| <= r;                                   */
/*   2 cylinder, rods inside: |(x - p) - ((x - p).a) a| <= r (a unit axis). */
/* Each region is convex, so a rod's axis stays inside exactly when both of */
/* its end points do: each end is a candidate contact point.  For end       */
/* s = -L/2 and +L/2 (in that order) of each rod, and each wall in order,   */
/* the gap phi = (distance from the end point to the wall) - diam/2; ends   */
/* with phi < cutoff become unilateral constraints with e the unit normal   */
/* of the wall at its nearest point, pointing into the allowed region, the  */
/* lever arm s, and q = phi/h + D^T M F as for a contact (eq. blockdef,     */
/* block A).  Returns the count (lists written only up to cap).             */
/* ------------------------------------------------------------------------ */
static int wall_gap(const double *w, const double *pt, double diam, double *phi, double *e)
{
    const int kind = (int)w[0];
    const double *p0 = w + 1, *a = w + 4, r = w[7];
    if (kind == 0) {
        double d = 0.0;
        for (int k = 0; k < 3; ++k) d += a[k] * (pt[k] - p0[k]);
        *phi = d - 0.5 * diam;
        for (int k = 0; k < 3; ++k) e[k] = a[k];
        return 0;
    }
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = pt[k] - p0[k];
    if (kind == 2) {
        const double va = dot3(v, a);
        for (int k = 0; k < 3; ++k) v[k] -= va * a[k];
    }
    const double dist = sqrt(dot3(v, v));
    *phi = r - dist - 0.5 * diam;
    if (dist > 0.0)
        for (int k = 0; k < 3; ++k) e[k] = -v[k] / dist;
    else
        for (int k = 0; k < 3; ++k) e[k] = 0.0; /* at the centre: far from the wall */
    return 0;
}

int64_t ora_walls(int64_t n, const double *x, const double *dir, const double *len, double len0, double diam,
                  double eta, double dt, double cutoff, int64_t nw, const double *walls, const double *F, int64_t cap,
                  int32_t *rod, double *e, double *arm, double *phi, double *q)
{
    double *Unc = (double *)calloc((size_t)(6 * (n > 0 ? n : 1)), sizeof(double));
    if (F) ora_apply_mobility(n, dir, len, len0, diam, eta, F, Unc);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double L = rod_len(len, len0, i);
        for (int end = 0; end < 2; ++end) {
            const double s = end == 0 ? -0.5 * L : 0.5 * L;
            double pt[3];
            for (int k = 0; k < 3; ++k) pt[k] = x[3 * i + k] + s * dir[3 * i + k];
            for (int64_t w = 0; w < nw; ++w) {
                double ph, ee[3];
                wall_gap(walls + 8 * w, pt, diam, &ph, ee);
                if (!(ph < cutoff)) continue;
                if (m < cap) {
                    double col[12];
                    d_column(dir, (int32_t)i, -1, ee, s, 0.0, col);
                    double dtu = 0.0;
                    for (int k = 0; k < 6; ++k) dtu += col[k] * Unc[6 * i + k];
                    rod[m] = (int32_t)i;
                    for (int k = 0; k < 3; ++k) e[3 * m + k] = ee[k];
                    arm[2 * m] = s;
                    arm[2 * m + 1] = 0.0;
                    phi[m] = ph;
                    q[m] = ph / dt + dtu;
                }
                ++m;
            }
        }
    }
    free(Unc);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Time integration.  Linearised implicit Euler on the configuration:       */
/* C^{k+1} = C^k + h G U (eq. constrainedeom_euler, first line), i.e.       */
/* x += h U_t and theta += h Psi(theta) Omega, then theta is renormalised   */
/* (the paper keeps theta a unit quaternion).  Centres are wrapped into     */
/* the periodic box; xu (may be NULL) accumulates unwrapped centres.        */
/* ------------------------------------------------------------------------ */
void ora_integrate(int64_t n, const double *box, double dt, const double *U, double *x, double *xu, double *quat)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            const double dx = dt * U[6 * i + a];
            double v = x[3 * i + a] + dx;
            v -= box[a] * floor(v / box[a]);
            if (v >= box[a]) v -= box[a];
            x[3 * i + a] = v;
            if (xu) xu[3 * i + a] += dx;
        }
        double qd[4];
        ora_psi_times(quat + 4 * i, U + 6 * i + 3, qd);
        double nrm = 0.0;
        for (int a = 0; a < 4; ++a) {
            quat[4 * i + a] += dt * qd[a];
            nrm += quat[4 * i + a] * quat[4 * i + a];
        }
        nrm = sqrt(nrm);
        for (int a = 0; a < 4; ++a) quat[4 * i + a] /= nrm;
    }
}
