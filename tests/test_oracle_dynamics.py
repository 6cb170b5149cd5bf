"""Pins of the oracle's multi-step pieces: Brownian force and stress (CPU).

Brownian force (F_nc = Brownian + external; the paper does not print the
noise amplitude): F_B = sqrt(2 kT/h) M^(-1/2) xi.  Pins:
  * M^(1/2) M^(1/2) = M and M^(-1/2) M^(1/2) = I for the rod block;
  * fluctuation-dissipation: the velocity noise M F_B has covariance 2 kT M / h
    (sampled);
  * the paper's "with thermal motion filaments may diffuse about 1 um in
    1 s" (Results, aster formation; 300 K, the solvent of Section Results,
    the asters' 0.5 um filaments): free rods stepped with the oracle for 1 s
    spread by sqrt(<|dx|^2>) = sqrt(6 D t), D = kT (a_par + 2 a_perp) / 3.
Stress (the virial of the constraint forces; the paper defines the pressure
as Tr(sigma)/3 and calls collision stress positive, crosslinker stress
negative):
  * the pair sum (1/V) sum_c gamma_c (x_P - x_Q') e_c equals the body sum
    (1/V) sum_i x_i (outer) f_i of the constraint forces on each rod when no
    pair crosses the periodic boundary (Clausius form);
  * repulsive contacts give a positive trace, stretched links a negative one.
"""
import math

import numpy as np

import oracle
import rodsynth

DIAM, ETA = 0.025, 0.01


def test_mobility_square_roots():
    rng = np.random.default_rng(0)
    for _ in range(5):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        L = rng.uniform(0.5, 1.5)
        M = oracle.mobility_block(d, L, DIAM, ETA)
        H = oracle.mobility_pow_block(d, L, DIAM, ETA, 0.5)
        Hi = oracle.mobility_pow_block(d, L, DIAM, ETA, -0.5)
        assert np.allclose(H @ H, M, rtol=1e-13, atol=1e-12 * np.abs(M).max())
        assert np.allclose(Hi @ H, np.eye(6), atol=1e-13)


def test_brownian_velocity_covariance():
    rng = np.random.default_rng(1)
    n, dt, kT = 200_000, 1e-4, oracle.KT_300K
    d = np.tile(np.array([0.6, 0.0, 0.8]), (n, 1))
    xi = rng.standard_normal((n, 6))
    FB = oracle.brownian_force(d, 1.0, DIAM, ETA, dt, kT, xi)
    U = oracle.apply_mobility(d, 1.0, DIAM, ETA, FB)
    C = U.T @ U / n
    M = oracle.mobility_block(d[0], 1.0, DIAM, ETA)
    # each entry within 4 standard errors of 2 kT M / h
    target = 2.0 * kT / dt * M
    se = np.sqrt((np.outer(np.diag(target), np.diag(target)) + target ** 2) / n)
    assert np.all(np.abs(C - target) <= 4.0 * se + 1e-12)


def test_free_rods_diffuse_about_a_micron_per_second():
    rng = np.random.default_rng(2)
    n, L, T, steps = 4000, 0.5, 1.0, 100
    dt = T / steps
    kT = oracle.KT_300K
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    x = np.full((n, 3), 50.0)
    x0 = x.copy()
    xu = x.copy()
    for _ in range(steps):
        d = oracle.directors(q)
        FB = oracle.brownian_force(d, L, DIAM, ETA, dt, kT, rng.standard_normal((n, 6)))
        U = oracle.apply_mobility(d, L, DIAM, ETA, FB)
        oracle.integrate(100.0, dt, U, x, q, xu)
    msd = np.mean(np.sum((xu - x0) ** 2, axis=1))
    c = oracle.mobility_coeffs(L, DIAM, ETA)
    D = kT * (c[0] + 2.0 * c[1]) / 3.0
    assert abs(msd - 6.0 * D * T) <= 4.0 * 6.0 * D * T * math.sqrt(2.0 / (3 * n))
    rms = math.sqrt(msd)
    assert 0.5 <= rms <= 1.5          # "about 1 um in 1 s", one printed digit


def _stress_by_bodies(x, d, n, pr, cs, gamma, V):
    D = oracle.dense_D(d, pr, cs)
    Fc = (D @ gamma).reshape(n, 6)
    return np.einsum("ia,ib->ab", x, Fc[:, :3]) / V


def test_pair_stress_is_the_clausius_virial():
    s = rodsynth.make_system(300, seed=5, box=4.0)
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff)
    keep = pr.img == oracle.IMG_ZERO       # pairs inside the box only
    pr = oracle.Pairs(pr.pi[keep], pr.pj[keep], pr.img[keep], pr.flags[keep])
    cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
    r = oracle.bbpgd(d, 1.0, s.diam, s.eta, pr, cs, tol=1e-10)
    assert r.status == oracle.OK and (r.gamma > 0).sum() > 10
    sc, _ = oracle.stress(s.x, d, 1.0, s.box, pr, cs, r.gamma)
    ref = _stress_by_bodies(s.x, d, s.n, pr, cs, r.gamma, s.box ** 3)
    assert np.allclose(sc, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert np.trace(sc) > 0.0              # collisions push: positive


def test_link_stress_sign():
    x = np.array([[5.0, 5.0, 5.0], [5.06, 5.0, 5.0]])
    quat = np.array([[1.0, 0.0, 0.0, 0.0]] * 2)
    d = oracle.directors(quat)
    lk = oracle.Links(np.array([0], np.int32), np.array([1], np.int32), np.zeros((1, 2)), np.array([100.0]),
                      np.array([0.03]))
    lg = oracle.links_geometry(x, d, 1.0, 10.0, DIAM, ETA, 1e-4, lk)
    gc = oracle.general(lk=lk, lg=lg)
    r = oracle.bbpgd_gen(d, 1.0, DIAM, ETA, gc, tol=1e-12)
    assert r.gamma[0] < 0.0                # stretched: pulls the rods together
    empty = oracle.Pairs(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8))
    _, sl = oracle.stress(x, d, 1.0, 10.0, empty, None, np.zeros(0), lk, lg, r.gamma)
    assert np.trace(sl) < 0.0              # crosslinkers contract: negative
    assert np.isclose(sl[0, 0], r.gamma[0] * (-0.06) * (-1.0) / 1000.0, rtol=1e-12)
