"""Pins of the oracle's bilateral (Hookean link) constraints (CPU).

Links join points fixed on two rod axes (or a rod and a fixed point).  Their
row of the linearised step is eq. linearconstraints (b) with the blocks D and
F of eq. blockdef: q_b = (Phi_b - Phi_b^0)/h + D_b^T M F and the compliance
K^-1/h on the diagonal; gamma_b is free.  Pins:
  * the column of D is the gradient of the link length under rigid motions
    (eq. symmetrydmap b), by central differences;
  * a rod held by N parallel links to fixed points relaxes their stretch as
    the implicit Euler step of l' = -lambda (l - l0) with the rate
    lambda = N kappa / (4 pi eta L / log(2L/D)) that Section 3 prints, and
    the printed 1/lambda of about 3e-6 s for N = 10, kappa = 100 pN/um in
    water; two free rods relax at twice that rate (relative mobility 2/drag);
  * kappa -> infinity (K^-1 -> 0): the linearised length returns to the rest
    length in one step, the stiff-joint limit the appendix discusses;
  * a links-only problem has the unique solution (Mc + K^-1/h) gamma = -q,
    checked against a dense linear solve; a mixed problem satisfies the KKT
    conditions of both kinds and its active rows reproduce gamma.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _quat_z_to(d):
    """A unit quaternion turning body z to unit vector d."""
    z = np.array([0.0, 0.0, 1.0])
    d = np.asarray(d, float) / np.linalg.norm(d)
    c = np.cross(z, d)
    w = 1.0 + z @ d
    if w < 1e-12:
        return np.array([0.0, 1.0, 0.0, 0.0])
    q = np.array([w, *c])
    return q / np.linalg.norm(q)


def _links(p, q, arm, kappa, rest, anchor=None):
    return oracle.Links(np.asarray(p, np.int32), np.asarray(q, np.int32), np.asarray(arm, float).reshape(-1, 2),
                        np.asarray(kappa, float), np.asarray(rest, float),
                        None if anchor is None else np.asarray(anchor, float).reshape(-1, 3))


def _step_links(x, quat, L, box, lk, eta, dt, diam=0.025, F=None):
    n = x.shape[0]
    F = np.zeros((n, 6)) if F is None else F
    d = oracle.directors(quat)
    lg = oracle.links_geometry(x, d, L, box, diam, eta, dt, lk, F)
    gc = oracle.general(lk=lk, lg=lg)
    r = oracle.bbpgd_gen(d, L, diam, eta, gc, tol=1e-12, max_iter=100_000)
    assert r.status == oracle.OK
    U = oracle.velocity_gen(d, L, diam, eta, gc, r.gamma, F)
    return d, lg, gc, r, U


def test_link_column_is_the_gradient_of_its_length():
    rng = np.random.default_rng(3)
    n, box, h = 6, 8.0, 1e-6
    x = rng.uniform(2.0, 6.0, (n, 3))
    quat = rng.standard_normal((n, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    L = rng.uniform(0.6, 1.4, n)
    lk = _links([0, 1, 2, 3, 5], [1, 4, 5, -1, -1], rng.uniform(-0.3, 0.3, (5, 2)), [50.0] * 5, [0.1] * 5,
                anchor=rng.uniform(2.0, 6.0, (5, 3)))
    d = oracle.directors(quat)
    lg = oracle.links_geometry(x, d, L, box, 0.025, 0.01, 1e-4, lk)
    gc = oracle.general(lk=lk, lg=lg)
    D = oracle.dense_D(d, oracle.Pairs(gc.pi, gc.pj, np.zeros(gc.n, np.int32), gc.kind),
                       oracle.Constraints(lg.length, gc.e, gc.arm, gc.q))
    for rod in range(n):
        for k6 in range(6):
            v = np.zeros(3)
            v[k6 % 3] = 1.0
            vals = []
            for sgn in (1.0, -1.0):
                xx, qq = x.copy(), quat.copy()
                if k6 < 3:
                    xx[rod] += sgn * h * v
                else:
                    # rotation about lab axis v by angle sgn*h: q <- exp(sgn h v / 2) q
                    a = 0.5 * sgn * h
                    r = np.array([math.cos(a), *(math.sin(a) * v)])
                    s1, v1, s2, v2 = r[0], r[1:], qq[rod, 0], qq[rod, 1:]
                    qq[rod] = np.r_[s1 * s2 - v1 @ v2, s1 * v2 + s2 * v1 + np.cross(v1, v2)]
                lg2 = oracle.links_geometry(xx, oracle.directors(qq), L, box, 0.025, 0.01, 1e-4, lk)
                vals.append(lg2.length)
            fd = (vals[0] - vals[1]) / (2 * h)
            assert np.allclose(fd, D[6 * rod + k6], atol=1e-7), (rod, k6)


def _paper_rate(N, kappa, eta, L, diam):
    """Section 3: lambda = N kappa / (4 pi eta L / log(2L/D))."""
    return N * kappa / (4.0 * math.pi * eta * L / math.log(2.0 * L / diam))


@pytest.mark.parametrize("N", [1, 3, 10])
def test_anchored_rod_relaxes_at_the_papers_rate(N):
    eta, dt, L, kappa, l0, stretch = 0.01, 1e-5, 1.0, 100.0, 0.02, 0.01
    x = np.array([[5.0, 5.0, 5.0]])
    quat = np.array([[1.0, 0.0, 0.0, 0.0]])          # axis along z
    s = np.linspace(-0.4, 0.4, N) if N > 1 else np.zeros(1)
    anchors = np.stack([np.full(N, 5.0 + l0 + stretch), np.full(N, 5.0), 5.0 + s], axis=1)
    lk = _links([0] * N, [-1] * N, np.stack([s, np.zeros(N)], axis=1), [kappa] * N, [l0] * N, anchors)
    d, lg, gc, r, U = _step_links(x, quat, L, 10.0, lk, eta, dt)
    assert np.allclose(lg.length, l0 + stretch)
    lam = _paper_rate(N, kappa, eta, L, 0.025)
    x1 = x + dt * U[:, :3]
    new_len = np.linalg.norm(x1[0] + s[:, None] * d[0] - anchors, axis=1)
    expect = l0 + stretch / (1.0 + lam * dt)
    assert np.allclose(new_len, expect, rtol=0, atol=1e-12)
    assert np.abs(U[0, 3:]).max() < 1e-9   # symmetric links: no turning


def test_papers_printed_relaxation_time():
    """N = 10 tethers of 100 pN/um on a 1 um filament in water: the printed
    1/lambda of about 3e-6 s (one significant digit) against the rate at
    which the oracle's step relaxes the stretch."""
    g = json.load(open(os.path.join(GOLD, "paper_slender_body.json")))
    N, kappa, eta, L = g["N_crosslinkers"], g["k_tether_pN_per_um"], g["eta_water_pN_s_per_um2"], g["L_um"]
    dt, l0, stretch = 1e-9, 0.02, 0.01
    s = np.linspace(-0.4, 0.4, N)
    anchors = np.stack([np.full(N, 5.0 + l0 + stretch), np.full(N, 5.0), 5.0 + s], axis=1)
    lk = _links([0] * N, [-1] * N, np.stack([s, np.zeros(N)], axis=1), [kappa] * N, [l0] * N, anchors)
    d, lg, gc, r, U = _step_links(np.array([[5.0, 5.0, 5.0]]), np.array([[1.0, 0, 0, 0]]), L, 10.0, lk, eta, dt,
                                  diam=g["D_fil_um"])
    rate = -(U[0, 0] * -1.0) / stretch        # d(stretch)/dt = U . e with e = -x
    inv = 1.0 / rate
    assert abs(inv - g["inv_lambda_s"]) <= g["printed_precision_rel"] * g["inv_lambda_s"]


@pytest.mark.parametrize("N", [1, 4])
def test_two_free_rods_relax_at_twice_the_rate(N):
    eta, dt, L, kappa, l0, stretch = 0.01, 1e-5, 1.0, 100.0, 0.03, -0.008
    x = np.array([[5.0, 5.0, 5.0], [5.0 + l0 + stretch, 5.0, 5.0]])
    quat = np.array([[1.0, 0.0, 0.0, 0.0]] * 2)
    s = np.linspace(-0.3, 0.3, N) if N > 1 else np.zeros(1)
    lk = _links([0] * N, [1] * N, np.stack([s, s], axis=1), [kappa] * N, [l0] * N)
    d, lg, gc, r, U = _step_links(x, quat, L, 10.0, lk, eta, dt)
    lam = 2.0 * _paper_rate(N, kappa, eta, L, 0.025)
    x1 = x + dt * U[:, :3]
    new_len = np.linalg.norm((x1[0] + s[:, None] * d[0]) - (x1[1] + s[:, None] * d[1]), axis=1)
    assert np.allclose(new_len, l0 + stretch / (1.0 + lam * dt), rtol=0, atol=1e-12)
    assert np.all(r.gamma > 0)                 # compressed springs push apart


def test_rigid_joint_limit():
    """kappa = inf: cmp = 0, and one linearised step restores the rest length
    for links that only translate the rods (e normal to both axes)."""
    x = np.array([[5.0, 5.0, 5.0], [5.04, 5.0, 5.0]])
    quat = np.array([[1.0, 0.0, 0.0, 0.0]] * 2)
    s = np.array([-0.2, 0.2])
    lk = _links([0, 0], [1, 1], np.stack([s, s], axis=1), [np.inf, np.inf], [0.03, 0.03])
    d, lg, gc, r, U = _step_links(x, quat, 1.0, 10.0, lk, 0.01, 1e-4)
    assert np.all(lg.cmp == 0.0)
    x1 = x + 1e-4 * U[:, :3]
    new_len = np.linalg.norm((x1[0] + s[:, None] * d[0]) - (x1[1] + s[:, None] * d[1]), axis=1)
    assert np.allclose(new_len, 0.03, rtol=0, atol=1e-13)


def _dense_Mc(d, L, gc, diam=0.025, eta=0.01):
    n = d.shape[0]
    D = oracle.dense_D(d, oracle.Pairs(gc.pi, gc.pj, np.zeros(gc.n, np.int32), gc.kind),
                       oracle.Constraints(np.zeros(gc.n), gc.e, gc.arm, gc.q))
    M = np.zeros((6 * n, 6 * n))
    for i in range(n):
        M[6 * i:6 * i + 6, 6 * i:6 * i + 6] = oracle.mobility_block(d[i], L if np.isscalar(L) else L[i], diam, eta)
    return D, M, D.T @ M @ D


def test_links_only_match_a_dense_solve():
    rng = np.random.default_rng(11)
    n = 8
    x = rng.uniform(3.0, 5.0, (n, 3))
    quat = rng.standard_normal((n, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    F = rng.standard_normal((n, 6))
    p = [0, 0, 1, 2, 3, 4, 5, 6, 7]
    q = [1, 2, 3, 3, 4, -1, 7, -1, 0]
    lk = _links(p, q, rng.uniform(-0.4, 0.4, (9, 2)), rng.uniform(10.0, 500.0, 9), rng.uniform(0.0, 0.3, 9),
                anchor=rng.uniform(3.0, 5.0, (9, 3)))
    d = oracle.directors(quat)
    lg = oracle.links_geometry(x, d, 1.0, 10.0, 0.025, 0.01, 1e-4, lk, F)
    gc = oracle.general(lk=lk, lg=lg)
    r = oracle.bbpgd_gen(d, 1.0, 0.025, 0.01, gc, tol=1e-10, max_iter=200_000)
    assert r.status == oracle.OK
    D, M, Mc = _dense_Mc(d, 1.0, gc)
    g_dense = np.linalg.solve(Mc + np.diag(lg.cmp), -lg.q)
    assert np.allclose(r.gamma, g_dense, rtol=1e-7, atol=1e-7 * np.abs(g_dense).max())
    U = oracle.velocity_gen(d, 1.0, 0.025, 0.01, gc, r.gamma, F)
    assert np.allclose(U.reshape(-1), M @ (D @ g_dense + F.reshape(-1)), rtol=1e-8, atol=1e-8)
    # the operator itself: w = (Mc + C) gamma + q
    w = oracle.apply_Mc_gen(d, 1.0, 0.025, 0.01, gc, r.gamma)
    assert np.allclose(w, (Mc + np.diag(lg.cmp)) @ r.gamma + lg.q, atol=1e-9)


def test_mixed_contacts_and_links_kkt():
    import rodsynth
    s = rodsynth.make_system(150, seed=4, box=2.2)
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
    rng = np.random.default_rng(2)
    nl = 40
    p = rng.integers(0, s.n, nl)
    q = (p + 1 + rng.integers(0, s.n - 1, nl)) % s.n
    lk = _links(p, q, rng.uniform(-0.5, 0.5, (nl, 2)), rng.uniform(20.0, 200.0, nl), rng.uniform(0.0, 0.5, nl))
    lg = oracle.links_geometry(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, lk, s.force)
    gc = oracle.general(pr, cs, lk, lg)
    r = oracle.bbpgd_gen(d, 1.0, s.diam, s.eta, gc, tol=1e-9, max_iter=200_000)
    assert r.status == oracle.OK
    w = oracle.apply_Mc_gen(d, 1.0, s.diam, s.eta, gc, r.gamma)
    u = gc.kind == 0
    assert r.gamma[u].min() >= 0.0 and w[u].min() >= -1e-9
    assert np.abs(np.minimum(r.gamma[u], w[u])).max() <= 1e-9
    assert np.abs(w[~u]).max() <= 1e-9
    # the equality rows of the active set reproduce U (gamma may be non-unique)
    D, M, Mc = _dense_Mc(d, 1.0, gc)
    A = (~u) | (r.gamma > w)
    C = np.diag(gc.cmp)
    sol = np.linalg.lstsq((Mc + C)[np.ix_(A, A)], -gc.q[A], rcond=None)[0]
    g2 = np.zeros(gc.n)
    g2[A] = sol
    U1 = oracle.velocity_gen(d, 1.0, s.diam, s.eta, gc, r.gamma, s.force)
    U2 = (M @ (D @ g2 + s.force.reshape(-1))).reshape(-1, 6)
    assert np.linalg.norm(U1 - U2) <= 1e-6 * np.linalg.norm(U2)
