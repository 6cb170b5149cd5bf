/*
 * CPU oracle of the crosslinker binding kinetics (kinetic Monte Carlo):
 * TEST INFRASTRUCTURE ONLY, like the rest of this folder.  Plain sequential C,
 * double precision, every crosslinker against every filament (no neighbour
 * search), shares no code with the HIP library.
 *
 * What is computed (Section "2. Crosslinker binding and unbinding", Table
 * tab:rates; Appendix "Kinetic Monte-Carlo", Table tab:supprates):
 *   A crosslinker is a Hookean tether between two heads A and B and is in one
 *   of four states: unbound (U), one head bound (S_A or S_B), both bound (D).
 *   Within a step of length h each crosslinker makes at most one transition
 *   (the tight-binding assumption of the appendix), with the probability
 *   1 - exp(-R h) of eq. P_bind for the total rate R of its possible
 *   transitions; the transition is then chosen in proportion to the rates.
 *     U -> S_h : R = k_oS[h] K_a[h] eps 3 / (4 pi r_cs^3) * sum_i L_in,i,
 *                L_in,i the length of filament i's axis inside the capture
 *                sphere of radius r_cs about the crosslinker (eq. KMC01exp);
 *                the head lands uniformly on the captured axis length
 *                (inverse transform over the filaments in index order).
 *     S_h -> U : R = k_oS[h]; the crosslinker reappears uniformly in the
 *                sphere of radius r_cs about the head (appendix, after eq.
 *                KMC_SU).
 *     S_h -> D : the free head g binds a site of another filament (never the
 *                bound head's own filament) within r_cd of the bound head:
 *                R = k_oD[g] K_e[g] / V_bd * sum_sites exp(-beta kappa
 *                ((1 - lambda)/2 Delta^2 - x_c Delta)), Delta = l - l_o - D
 *                the tether's stretch (eq. Ucl; Table tab:supprates), the
 *                site chosen by inverse transform over the filaments in index
 *                order and their sites in order.
 *     D -> S   : head h unbinds at R = k_oD[h] exp(beta kappa (lambda/2
 *                Delta^2 + x_c Delta)) (eq. KMC_DS_Edep with eq.
 *                KMC_SD_fdep); the other head stays.
 *   V_bd = 4 pi int_0^r_cd exp(-beta U(r)) r^2 dr, U = kappa/2 (r - l_o - D)^2
 *   (eq. double_bind_volume_gen).  Binding sites: floor(eps L) of them per
 *   filament (at least one), at the centres of equal arclength intervals
 *   (eps is the linear site density, so eps ds counts sites).
 *   Before the transitions, unbound crosslinkers diffuse: x += sqrt(2 d_U h)
 *   xi (Section "1. Crosslinking motor diffusion and stepping").
 * Geometry: periodic box; each filament is taken at the image of its centre
 * nearest to the query point (the caller keeps L/2 + the query radius below
 * half the box).  Random numbers are inputs: per crosslinker and step four
 * uniforms u (event, which transition, target, radius of the reappearance)
 * and three normals xi (diffusion, direction of the reappearance).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double eps;     /* binding sites per um of filament */
    double Ka[2];   /* U <-> S association constants of heads A, B (um^3) */
    double koS[2];  /* S -> U rates (1/s) */
    double Ke[2];   /* S <-> D association constants (um^3) */
    double koD[2];  /* D -> S rates without load (1/s) */
    double kappa;   /* tether stiffness (pN/um) */
    double rest;    /* tether free length l_o (um) */
    double lambda;  /* energy factor of the unbinding rate */
    double xc;      /* characteristic length of the force dependence (um) */
    double kT;      /* thermal energy (pN um) */
    double rcs;     /* capture radius of U -> S (um) */
    double rcd;     /* cutoff of the S -> D site sum (um) */
    double dU;      /* diffusion constant of unbound crosslinkers (um^2/s) */
    double diam;    /* filament diameter D (um) */
    double dt;      /* time step h (s) */
} ora_kmc_params;

enum { KMC_U = 0, KMC_SA = 1, KMC_SB = 2, KMC_D = 3 };
enum { EV_NONE = 0, EV_BIND = 1, EV_UNBIND = 2, EV_CROSS = 3, EV_RELEASE = 4 };

static const double kPi = 3.14159265358979323846;

static double rlen(const double *len, double len0, int64_t i) { return len ? len[i] : len0; }

/* the point at arclength s on filament i, in the box (wrapped) */
static void axis_point(const double *x, const double *dir, const double *box, int64_t i, double s, double *p)
{
    for (int a = 0; a < 3; ++a) {
        double v = x[3 * i + a] + s * dir[3 * i + a];
        v -= box[a] * floor(v / box[a]);
        if (v >= box[a]) v -= box[a];
        p[a] = v;
    }
}

/* centre of filament i relative to point p, nearest image */
static void centre_rel(const double *x, const double *box, int64_t i, const double *p, double *c)
{
    for (int a = 0; a < 3; ++a) {
        double d = x[3 * i + a] - p[a];
        d -= box[a] * floor(d / box[a] + 0.5);
        c[a] = d;
    }
}

/* The arclength interval [lo, hi] of filament i's axis inside the sphere of
 * radius r about p (empty: hi <= lo). */
static void inside_interval(const double *x, const double *dir, const double *len, double len0, const double *box,
                            int64_t i, const double *p, double r, double *lo, double *hi)
{
    double c[3];
    centre_rel(x, box, i, p, c);
    const double *d = dir + 3 * i;
    const double b = c[0] * d[0] + c[1] * d[1] + c[2] * d[2];
    const double w[3] = {c[0] - b * d[0], c[1] - b * d[1], c[2] - b * d[2]};
    const double h2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double half_len = 0.5 * rlen(len, len0, i);
    *lo = 0.0;
    *hi = 0.0;
    if (h2 >= r * r) return;
    const double half = sqrt(r * r - h2);
    /* the axis point at arclength s is c + s d: closest to p at s = -b */
    double a0 = -b - half, a1 = -b + half;
    if (a0 < -half_len) a0 = -half_len;
    if (a1 > half_len) a1 = half_len;
    *lo = a0;
    *hi = a1;
}

static double stretch_of(const ora_kmc_params *P, double l) { return l - P->rest - P->diam; }

/* weight of one site at tether length l for the S -> D binding */
static double cross_weight(const ora_kmc_params *P, double l)
{
    const double dl = stretch_of(P, l);
    return exp(-(P->kappa / P->kT) * (0.5 * (1.0 - P->lambda) * dl * dl - P->xc * dl));
}

/* D -> S rate of a head with zero-load rate k0 */
static double release_rate(const ora_kmc_params *P, double k0, double l)
{
    const double dl = stretch_of(P, l);
    return k0 * exp((P->kappa / P->kT) * (0.5 * P->lambda * dl * dl + P->xc * dl));
}

static int64_t sites_of(const ora_kmc_params *P, double L)
{
    int64_t m = (int64_t)floor(P->eps * L);
    return m < 1 ? 1 : m;
}

static double site_arc(double L, int64_t m, int64_t k) { return -0.5 * L + (k + 0.5) * (L / m); }

/* distance from p to the site at arclength s of filament j (nearest image of
 * the filament's centre) */
static double site_dist(const double *x, const double *dir, const double *box, int64_t j, const double *p, double s)
{
    double c[3];
    centre_rel(x, box, j, p, c);
    const double *d = dir + 3 * j;
    const double v[3] = {c[0] + s * d[0], c[1] + s * d[1], c[2] + s * d[2]};
    return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

/* Sum of the S -> D weights of filament j's sites within r_cd of p, in site
 * order; with pick >= 0 the walk stops at the site where the running sum
 * first exceeds pick (its index in *site; the last counted site otherwise). */
static double site_sum(const ora_kmc_params *P, const double *x, const double *dir, const double *len, double len0,
                       const double *box, int64_t j, const double *p, double pick, int64_t *site)
{
    const double L = rlen(len, len0, j);
    const int64_t m = sites_of(P, L);
    double sum = 0.0;
    int64_t last = -1;
    if (site) *site = -1;
    /* every site lies on the axis segment: none is within r_cd when the
     * segment's nearest point is farther (a margin covers rounding) */
    {
        double c[3];
        centre_rel(x, box, j, p, c);
        const double *d = dir + 3 * j;
        double t = -(c[0] * d[0] + c[1] * d[1] + c[2] * d[2]);
        if (t < -0.5 * L) t = -0.5 * L;
        if (t > 0.5 * L) t = 0.5 * L;
        const double v[3] = {c[0] + t * d[0], c[1] + t * d[1], c[2] + t * d[2]};
        if (sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) > P->rcd * (1.0 + 1e-9)) return 0.0;
    }
    for (int64_t k = 0; k < m; ++k) {
        const double l = site_dist(x, dir, box, j, p, site_arc(L, m, k));
        if (!(l <= P->rcd)) continue;
        sum += cross_weight(P, l);
        last = k;
        if (pick >= 0.0 && sum > pick) break;
    }
    if (site) *site = last;
    return sum;
}

double ora_kmc_effective_volume(const ora_kmc_params *P)
{
    /* composite Simpson rule, 2^16 intervals on [0, r_cd] (the integrand is
     * smooth; the tests check the result against the closed form of the
     * untruncated Gaussian integral) */
    const int64_t m = 1 << 16;
    const double hstep = P->rcd / m;
    double acc = 0.0;
    for (int64_t k = 0; k <= m; ++k) {
        const double r = k * hstep;
        const double dl = stretch_of(P, r);
        const double f = exp(-(P->kappa / P->kT) * 0.5 * dl * dl) * r * r;
        const double wgt = (k == 0 || k == m) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
        acc += wgt * f;
    }
    return 4.0 * kPi * acc * hstep / 3.0;
}

/* Length of filament i's axis inside the sphere of radius r about p. */
double ora_kmc_inside_length(int64_t n, const double *x, const double *dir, const double *len, double len0,
                             const double *box, int64_t i, const double *p, double r)
{
    (void)n;
    double lo, hi;
    inside_interval(x, dir, len, len0, box, i, p, r, &lo, &hi);
    return hi > lo ? hi - lo : 0.0;
}

/* Total S -> D weight about point p excluding filament `skip` (for tests). */
double ora_kmc_cross_sum(int64_t n, const double *x, const double *dir, const double *len, double len0,
                         const double *box, const ora_kmc_params *P, const double *p, int64_t skip)
{
    double W = 0.0;
    for (int64_t j = 0; j < n; ++j)
        if (j != skip) W += site_sum(P, x, dir, len, len0, box, j, p, -1.0, NULL);
    return W;
}

/* One step for crosslinkers [0, m): state[m], rod[m][2] (filament of head A,
 * B; -1 unbound), arc[m][2] (their arclengths), xl[m][3] (position: the
 * crosslinker's when unbound, the bound head's in S, head A's in D).
 * u[m][4], xi[m][3]: the step's random numbers.  event[m] (may be NULL):
 * 0 none, 1 U->S, 2 S->U, 3 S->D, 4 D->S.  Vbd: the effective volume. */
void ora_kmc_step(int64_t n, const double *x, const double *dir, const double *len, double len0, const double *box,
                  const ora_kmc_params *P, double Vbd, int64_t m, int32_t *state, int32_t *rod, double *arc,
                  double *xl, const double *u, const double *xi, int32_t *event)
{
    const double cap = 3.0 * P->eps / (4.0 * kPi * P->rcs * P->rcs * P->rcs);
    const double hop = sqrt(2.0 * P->dU * P->dt);
    for (int64_t c = 0; c < m; ++c) {
        const double *uc = u + 4 * c, *xc = xi + 3 * c;
        int32_t ev = EV_NONE;
        const int32_t s = state[c];
        if (s == KMC_U) {
            double p[3];
            for (int a = 0; a < 3; ++a) {
                double v = xl[3 * c + a] + hop * xc[a];
                v -= box[a] * floor(v / box[a]);
                if (v >= box[a]) v -= box[a];
                p[a] = v;
                xl[3 * c + a] = v;
            }
            double Lt = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double lo, hi;
                inside_interval(x, dir, len, len0, box, i, p, P->rcs, &lo, &hi);
                if (hi > lo) Lt += hi - lo;
            }
            const double RA = P->koS[0] * P->Ka[0] * cap * Lt, RB = P->koS[1] * P->Ka[1] * cap * Lt;
            const double R = RA + RB;
            if (R > 0.0 && uc[0] < 1.0 - exp(-R * P->dt)) {
                const int hd = uc[1] * R < RA ? 0 : 1;
                const double t = uc[2] * Lt;
                double cum = 0.0;
                int64_t pick = -1;
                double plo = 0.0, phi = 0.0, before = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    double lo, hi;
                    inside_interval(x, dir, len, len0, box, i, p, P->rcs, &lo, &hi);
                    if (!(hi > lo)) continue;
                    pick = i;
                    plo = lo;
                    phi = hi;
                    before = cum;
                    cum += hi - lo;
                    if (cum > t) break;
                }
                if (pick < 0) goto done; /* no captured length: cannot happen with R > 0 */
                double sa = plo + (t - before);
                if (sa > phi) sa = phi;
                if (sa < plo) sa = plo;
                state[c] = hd == 0 ? KMC_SA : KMC_SB;
                rod[2 * c + hd] = (int32_t)pick;
                arc[2 * c + hd] = sa;
                axis_point(x, dir, box, pick, sa, xl + 3 * c);
                ev = EV_BIND;
            }
        } else if (s == KMC_SA || s == KMC_SB) {
            const int hd = s == KMC_SA ? 0 : 1, g = 1 - hd;
            const int64_t i = rod[2 * c + hd];
            double p[3];
            axis_point(x, dir, box, i, arc[2 * c + hd], p);
            double W = 0.0;
            for (int64_t j = 0; j < n; ++j)
                if (j != i) W += site_sum(P, x, dir, len, len0, box, j, p, -1.0, NULL);
            const double Ron = P->koD[g] * P->Ke[g] / Vbd * W;
            const double Roff = P->koS[hd];
            const double R = Ron + Roff;
            for (int a = 0; a < 3; ++a) xl[3 * c + a] = p[a];
            if (R > 0.0 && uc[0] < 1.0 - exp(-R * P->dt)) {
                if (uc[1] * R < Roff) {
                    /* the crosslinker leaves into the capture sphere */
                    const double nx = sqrt(xc[0] * xc[0] + xc[1] * xc[1] + xc[2] * xc[2]);
                    const double rad = P->rcs * cbrt(uc[3]);
                    for (int a = 0; a < 3; ++a) {
                        const double dirn = nx > 0.0 ? xc[a] / nx : (a == 2 ? 1.0 : 0.0);
                        double v = p[a] + rad * dirn;
                        v -= box[a] * floor(v / box[a]);
                        if (v >= box[a]) v -= box[a];
                        xl[3 * c + a] = v;
                    }
                    state[c] = KMC_U;
                    rod[2 * c + hd] = -1;
                    arc[2 * c + hd] = 0.0;
                    ev = EV_UNBIND;
                } else {
                    const double t = uc[2] * W;
                    double cum = 0.0;
                    int64_t pick = -1, site = -1;
                    for (int64_t j = 0; j < n; ++j) {
                        if (j == i) continue;
                        const double wj = site_sum(P, x, dir, len, len0, box, j, p, -1.0, NULL);
                        if (!(wj > 0.0)) continue;
                        pick = j;
                        if (cum + wj > t) {
                            site_sum(P, x, dir, len, len0, box, j, p, t - cum, &site);
                            break;
                        }
                        cum += wj;
                        site_sum(P, x, dir, len, len0, box, j, p, -1.0, &site);
                    }
                    if (pick < 0 || site < 0) goto done; /* no weight: cannot happen with R_on > 0 */
                    const double L = rlen(len, len0, pick);
                    state[c] = KMC_D;
                    rod[2 * c + g] = (int32_t)pick;
                    arc[2 * c + g] = site_arc(L, sites_of(P, L), site);
                    if (g == 0) axis_point(x, dir, box, pick, arc[2 * c], xl + 3 * c);
                    ev = EV_CROSS;
                }
            }
        } else if (s == KMC_D) {
            double pa[3], pb[3];
            axis_point(x, dir, box, rod[2 * c], arc[2 * c], pa);
            axis_point(x, dir, box, rod[2 * c + 1], arc[2 * c + 1], pb);
            double l2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double d = pa[a] - pb[a];
                d -= box[a] * floor(d / box[a] + 0.5);
                l2 += d * d;
            }
            const double l = sqrt(l2);
            const double RA = release_rate(P, P->koD[0], l), RB = release_rate(P, P->koD[1], l);
            const double R = RA + RB;
            for (int a = 0; a < 3; ++a) xl[3 * c + a] = pa[a];
            if (R > 0.0 && uc[0] < 1.0 - exp(-R * P->dt)) {
                const int hd = uc[1] * R < RA ? 0 : 1;
                state[c] = hd == 0 ? KMC_SB : KMC_SA;
                rod[2 * c + hd] = -1;
                arc[2 * c + hd] = 0.0;
                if (hd == 0) for (int a = 0; a < 3; ++a) xl[3 * c + a] = pb[a];
                ev = EV_RELEASE;
            }
        }
    done:
        if (event) event[c] = ev;
    }
}
