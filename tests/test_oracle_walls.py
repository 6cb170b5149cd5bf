"""Pins of the oracle's wall (confinement) constraints (CPU).

A wall is a fixed body: its constraints have only the rod's side in D
(Appendix "Equation of motion with geometric constraints", last paragraph).
The allowed regions (a half-space above a substrate, the inside of a
spherical shell or of a cylinder) are convex, so a rod's axis stays inside
exactly when both of its ends do.  Pins:
  * sampled segments: no interior point of a rod is closer to the wall than
    its nearer end (the distance to the boundary is concave along a line);
  * each gap and normal put the wall point p - (phi + d/2) e on the wall,
    with e normal to the wall there;
  * closed forms: a rod standing on a substrate or pointing out through a
    shell and pushed into the wall stops with its end exactly at contact
    (Mc = a_par, gamma = -(phi/h + a_par F.e)/a_par); pulled away, it moves
    freely (gamma = 0);
  * a rod lying flat on a substrate under a uniform load: both ends carry
    half the load and the rod does not turn.
"""
import numpy as np
import pytest

import oracle

DIAM, ETA, DT, CUT = 0.025, 0.01, 1e-4, 0.05


def _quat_z_to(d):
    z = np.array([0.0, 0.0, 1.0])
    d = np.asarray(d, float) / np.linalg.norm(d)
    w = 1.0 + z @ d
    if w < 1e-12:
        return np.array([0.0, 1.0, 0.0, 0.0])
    q = np.array([w, *np.cross(z, d)])
    return q / np.linalg.norm(q)


def _wall_dist(w, pts):
    """Distance of points to the wall, from the wall's own description."""
    kind, p0, a, r = int(w[0]), w[1:4], w[4:7], w[7]
    v = pts - p0
    if kind == oracle.WALL_PLANE:
        return v @ a
    if kind == oracle.WALL_CYLINDER_IN:
        v = v - np.outer(v @ a, a)
    return r - np.linalg.norm(v, axis=1)


WALLS = [oracle.wall(oracle.WALL_PLANE, (0.0, 0.0, 1.0), (0.0, 0.6, 0.8)),
         oracle.wall(oracle.WALL_SPHERE_IN, (2.0, 2.0, 2.0), r=1.6),
         oracle.wall(oracle.WALL_CYLINDER_IN, (2.0, 2.0, 0.0), (0.6, 0.0, 0.8), r=1.2)]


@pytest.mark.parametrize("k", range(len(WALLS)))
def test_wall_gaps_against_sampled_rods(k):
    rng = np.random.default_rng(k)
    w = WALLS[k]
    n = 400
    x = rng.uniform(0.4, 3.6, (n, 3))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    L = rng.uniform(0.5, 1.5, n)
    wc = oracle.walls(x, d, L, DIAM, ETA, DT, 10.0, [w])   # cutoff 10: every end listed
    assert wc.n == 2 * n
    t = np.linspace(-0.5, 0.5, 1001)
    for m in range(wc.n):
        i, s = wc.rod[m], wc.arm[m, 0]
        assert abs(abs(s) - 0.5 * L[i]) == 0.0
        pts = x[i] + np.outer(t * L[i], d[i])
        dist = _wall_dist(w, pts)
        # the ends are the nearest points: no sample closer than both ends
        ends = wc.phi[2 * (m // 2):2 * (m // 2) + 2] + 0.5 * DIAM
        assert dist.min() >= ends.min() - 1e-12
        end_pt = x[i] + s * d[i]
        assert abs(_wall_dist(w, end_pt[None])[0] - (wc.phi[m] + 0.5 * DIAM)) < 1e-12
        # e is the inward unit normal at the nearest wall point
        foot = end_pt - (wc.phi[m] + 0.5 * DIAM) * wc.e[m]
        assert abs(np.linalg.norm(wc.e[m]) - 1.0) < 1e-14
        assert abs(_wall_dist(w, foot[None])[0]) < 1e-12
        eps = 1e-6
        assert abs(_wall_dist(w, (foot + eps * wc.e[m])[None])[0] - eps) < 1e-9


def _solve_walls(x, quat, L, wl, F):
    d = oracle.directors(quat)
    wc = oracle.walls(x, d, L, DIAM, ETA, DT, CUT, wl, F)
    gc = oracle.general_all(wc=wc)
    r = oracle.bbpgd_gen(d, L, DIAM, ETA, gc, tol=1e-12, max_iter=10_000)
    assert r.status == oracle.OK
    U = oracle.velocity_gen(d, L, DIAM, ETA, gc, r.gamma, F)
    return d, wc, r, U


@pytest.mark.parametrize("push", [-3.0, 3.0])
def test_rod_standing_on_a_substrate(push):
    a = np.array([0.0, 0.0, 1.0])
    wl = [oracle.wall(oracle.WALL_PLANE, (0.0, 0.0, 1.0), a)]
    gap = 0.004
    x = np.array([[2.0, 2.0, 1.0 + 0.5 + 0.5 * DIAM + gap]])
    F = np.zeros((1, 6))
    F[0, 2] = push
    d, wc, r, U = _solve_walls(x, np.array([[1.0, 0, 0, 0]]), 1.0, wl, F)
    assert wc.n == 1 and wc.arm[0, 0] == -0.5 and abs(wc.phi[0] - gap) < 1e-15
    apar = oracle.mobility_coeffs(1.0, DIAM, ETA)[0]
    if push < 0 and apar * -push * DT > gap:
        assert np.isclose(r.gamma[0], -(gap / DT + apar * push) / apar, rtol=1e-12)
        assert abs(gap + DT * U[0, 2]) < 1e-15           # lands exactly on the wall
    else:
        assert r.gamma[0] == 0.0 and np.isclose(U[0, 2], apar * push, rtol=1e-14)
    assert np.abs(U[0, 3:]).max() < 1e-12


def test_rod_pushed_out_through_a_shell():
    c, R = np.array([2.0, 2.0, 2.0]), 1.5
    wl = [oracle.wall(oracle.WALL_SPHERE_IN, c, r=R)]
    u = np.array([0.48, -0.6, 0.64])
    gap = 0.003
    x = (c + (R - 0.5 * DIAM - gap - 0.5) * u)[None]
    F = np.zeros((1, 6))
    F[0, :3] = 4.0 * u
    d, wc, r, U = _solve_walls(x, _quat_z_to(u)[None], 1.0, wl, F)
    assert wc.n == 1 and np.allclose(wc.e[0], -u) and wc.arm[0, 0] == 0.5
    assert abs(gap - DT * (U[0, :3] @ u)) < 1e-14   # the outer end reaches the shell


def test_rod_lying_on_a_substrate_shares_the_load():
    wl = [oracle.wall(oracle.WALL_PLANE, (0.0, 0.0, 1.0), (0.0, 0.0, 1.0))]
    x = np.array([[2.0, 2.0, 1.0 + 0.5 * DIAM + 0.001]])
    quat = _quat_z_to([1.0, 0.0, 0.0])[None]
    F = np.zeros((1, 6))
    F[0, 2] = -50.0
    d, wc, r, U = _solve_walls(x, quat, 1.0, wl, F)
    assert wc.n == 2
    assert np.isclose(r.gamma[0], r.gamma[1], rtol=1e-9)
    assert np.abs(U[0, 3:]).max() < 1e-9
    assert abs(0.001 + DT * U[0, 2]) < 1e-14
