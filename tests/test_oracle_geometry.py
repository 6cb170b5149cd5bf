"""Pins of the oracle's orientation, mobility and closest-point code against
values fixed by the paper and by elementary geometry (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_quat(rng, n=None):
    q = rng.standard_normal(4 if n is None else (n, 4))
    return q / np.linalg.norm(q, axis=-1, keepdims=True)


def _unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v)


# --- orientation ---------------------------------------------------------------

def test_rotation_quarter_turn_about_x():
    # a right-handed quarter turn about +x takes +z to -y and +y to +z
    q = np.array([math.cos(math.pi / 4), math.sin(math.pi / 4), 0.0, 0.0])
    R = oracle.rotation(q)
    assert np.allclose(R @ [0, 0, 1], [0, -1, 0], atol=1e-15)
    assert np.allclose(R @ [0, 1, 0], [0, 0, 1], atol=1e-15)
    assert np.allclose(oracle.directors(q[None])[0], [0, -1, 0], atol=1e-15)


def test_rotation_matches_rodrigues():
    rng = np.random.default_rng(1)
    for _ in range(20):
        axis = _unit(rng.standard_normal(3))
        ang = rng.uniform(-math.pi, math.pi)
        q = np.r_[math.cos(ang / 2), math.sin(ang / 2) * axis]
        K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
        Rr = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
        assert np.allclose(oracle.rotation(q), Rr, atol=1e-14)
        assert np.allclose(oracle.rotation(-q), Rr, atol=1e-14)


def test_psi_is_lab_frame_angular_velocity():
    """Appendix 'Symmetry ...': a body point y = R Y moves as omega x y when
    theta' = Psi(theta) omega.  Central difference of R(theta + eps Psi w) Y."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        q = _rand_quat(rng)
        w = rng.standard_normal(3)
        Y = rng.standard_normal(3)
        qd = oracle.psi_times(q, w)
        eps = 1e-6
        yp = oracle.rotation(q + eps * qd) @ Y
        ym = oracle.rotation(q - eps * qd) @ Y
        fd = (yp - ym) / (2 * eps)
        assert np.allclose(fd, np.cross(w, oracle.rotation(q) @ Y), atol=1e-8)
        # the rate is tangent to the unit sphere: |theta| is preserved to first order
        assert abs(np.dot(q, qd)) < 1e-14


# --- mobility ------------------------------------------------------------------

def test_perpendicular_drag_matches_paper_value():
    g = json.load(open(os.path.join(GOLD, "paper_slender_body.json")))
    c = oracle.mobility_coeffs(g["L_um"], g["D_fil_um"], g["eta_water_pN_s_per_um2"])
    drag_perp = 1.0 / c[1]
    assert abs(drag_perp - g["drag_perp_pN_s_per_um"]) <= g["printed_precision_rel"] * g["drag_perp_pN_s_per_um"]
    inv_lambda = drag_perp / (g["N_crosslinkers"] * g["k_tether_pN_per_um"])
    assert abs(inv_lambda - g["inv_lambda_s"]) <= g["printed_precision_rel"] * g["inv_lambda_s"]


def test_mobility_coefficients_closed_form():
    # slender-body values with log(2L/d): parallel drag is half the normal one
    L, d, eta = 1.0, 0.025, 0.01
    lg = math.log(2 * L / d)
    c = oracle.mobility_coeffs(L, d, eta)
    assert c[1] == pytest.approx(lg / (4 * math.pi * eta * L), rel=1e-15)
    assert c[0] == pytest.approx(2 * c[1], rel=1e-15)
    assert c[2] == pytest.approx(3 * lg / (math.pi * eta * L ** 3), rel=1e-15)
    # the figures quoted for the benchmark rods (um/(pN s), 1/(pN um s))
    assert c[0] == pytest.approx(69.74, abs=0.01)
    assert c[1] == pytest.approx(34.87, abs=0.01)
    assert c[2] == pytest.approx(418.4, abs=0.1)


@pytest.mark.parametrize("L", [0.5, 1.0, 1.37, 4.0])
def test_rotational_drag_is_the_second_moment_of_the_normal_drag(L):
    """Resistive-force picture: a rod turning at rate w about a normal axis
    through its centre moves its point at arclength s at w s, normal to the
    axis, against the normal drag density zeta_perp / L; the torque of that
    drag, integrated along the rod by quadrature, must be the torque that
    gives w through the oracle's rotational mobility."""
    from scipy.integrate import quad
    d, eta = 0.025, 0.01
    c = oracle.mobility_coeffs(L, d, eta)
    zeta_perp = 1.0 / c[1]
    torque = 2.7
    w = c[2] * torque
    drag_torque, _ = quad(lambda s: s * (zeta_perp / L) * (w * s), -0.5 * L, 0.5 * L, epsabs=0.0, epsrel=1e-13)
    assert drag_torque == pytest.approx(torque, rel=1e-12)


def test_mobility_block_eigenstructure():
    rng = np.random.default_rng(3)
    d = _unit(rng.standard_normal(3))
    M = oracle.mobility_block(d, 1.3, 0.025, 0.01)
    c = oracle.mobility_coeffs(1.3, 0.025, 0.01)
    perp = _unit(np.cross(d, rng.standard_normal(3)))
    assert np.allclose(M[:3, :3] @ d, c[0] * d, rtol=1e-14)
    assert np.allclose(M[:3, :3] @ perp, c[1] * perp, rtol=1e-13)
    assert np.allclose(M[3:, 3:] @ perp, c[2] * perp, rtol=1e-13)
    assert np.allclose(M[:3, 3:], 0) and np.allclose(M[3:, :3], 0)
    assert np.allclose(M, M.T, atol=0)
    assert np.linalg.eigvalsh(M).min() > 0


# --- closest points ------------------------------------------------------------

def _sampled_min(xi, di, Li, xj, dj, Lj, m=2001):
    s = np.linspace(-Li / 2, Li / 2, m)
    t = np.linspace(-Lj / 2, Lj / 2, m)
    P = xi[None, :] + s[:, None] * di[None, :]
    Q = xj[None, :] + t[:, None] * dj[None, :]
    best = np.inf
    for k in range(0, m, 256):
        dd = np.linalg.norm(P[k:k + 256, None, :] - Q[None, :, :], axis=-1)
        best = min(best, dd.min())
    return best, Li / (m - 1), Lj / (m - 1)


def test_closest_against_sampling():
    rng = np.random.default_rng(4)
    for k in range(40):
        Li, Lj = rng.uniform(0.3, 1.5, 2)
        xi = rng.uniform(-0.2, 0.2, 3)
        xj = rng.uniform(-0.6, 0.6, 3)
        di, dj = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
        if k % 4 == 0:   # nearly parallel pairs as well
            dj = _unit(di + 1e-3 * rng.standard_normal(3))
        s, t, dist, e, _ = oracle.closest(xi, di, Li, xj, dj, Lj)
        smin, ds, dt = _sampled_min(xi, di, Li, xj, dj, Lj)
        assert dist <= smin + 1e-14
        assert dist >= smin - 0.5 * (ds + dt) - 1e-14
        # the reported parameters realise the reported distance
        r = xi + s * di - xj - t * dj
        assert np.linalg.norm(r) == pytest.approx(dist, rel=1e-12, abs=1e-15)
        assert abs(s) <= Li / 2 and abs(t) <= Lj / 2
        assert np.allclose(e, r / dist, atol=1e-14)


def test_closest_crossing_perpendicular():
    h = 0.3
    s, t, dist, e, fl = oracle.closest([0, 0, h], [1, 0, 0], 1.0, [0, 0, 0], [0, 1, 0], 1.0)
    assert dist == pytest.approx(h, abs=1e-15) and s == 0 and t == 0
    assert np.allclose(e, [0, 0, 1])
    assert fl == 0


def test_closest_parallel_side_by_side_midpoint():
    # rod j shifted along the common axis by 0.2: overlap of parameters is [-0.3, 0.5]
    s, t, dist, e, fl = oracle.closest([0.0, 0.05, 0], [1, 0, 0], 1.0, [0.2, 0.0, 0], [1, 0, 0], 1.0)
    assert dist == pytest.approx(0.05, abs=1e-15)
    assert s == pytest.approx(0.1, abs=1e-15) and t == pytest.approx(-0.1, abs=1e-15)
    assert np.allclose(e, [0, 1, 0])
    assert fl & oracle.FLAG_PARALLEL


def test_closest_antiparallel():
    s, t, dist, e, fl = oracle.closest([0.0, 0.05, 0], [1, 0, 0], 1.0, [0.2, 0.0, 0], [-1, 0, 0], 1.0)
    assert dist == pytest.approx(0.05, abs=1e-15)
    assert s == pytest.approx(0.1, abs=1e-15) and t == pytest.approx(0.1, abs=1e-15)


def test_closest_collinear_end_to_end():
    s, t, dist, e, fl = oracle.closest([0, 0, 0], [0, 0, 1], 1.0, [0, 0, 1.3], [0, 0, 1], 1.0)
    assert dist == pytest.approx(0.3, abs=1e-15)
    assert s == 0.5 and t == -0.5
    assert np.allclose(e, [0, 0, -1])


def test_closest_t_contact_end_on_middle():
    # the end of rod j touches the middle of rod i from above
    s, t, dist, e, fl = oracle.closest([0, 0, 0], [1, 0, 0], 1.0, [0, 0, 0.52], [0, 0, 1], 1.0)
    assert dist == pytest.approx(0.02, abs=1e-15)
    assert s == 0 and t == -0.5
    assert np.allclose(e, [0, 0, -1])


def test_closest_skew_lines_interior():
    rng = np.random.default_rng(5)
    for _ in range(20):
        di, dj = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
        n = _unit(np.cross(di, dj))
        h = rng.uniform(0.01, 0.2)
        a, b = rng.uniform(-0.3, 0.3, 2)
        xi = np.zeros(3)
        xj = xi + a * di - b * dj - h * n   # closest points at s = a, t = b
        s, t, dist, e, _ = oracle.closest(xi, di, 2.0, xj, dj, 2.0)
        line = abs(np.dot(xi - xj, np.cross(di, dj))) / np.linalg.norm(np.cross(di, dj))
        assert dist == pytest.approx(line, rel=1e-12)
        assert dist == pytest.approx(h, rel=1e-12)
        assert s == pytest.approx(a, abs=1e-12) and t == pytest.approx(b, abs=1e-12)


def test_closest_invariances():
    rng = np.random.default_rng(6)
    for _ in range(30):
        Li, Lj = rng.uniform(0.5, 1.5, 2)
        xi, xj = rng.uniform(-0.4, 0.4, 3), rng.uniform(-0.4, 0.4, 3)
        di, dj = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
        s, t, dist, e, _ = oracle.closest(xi, di, Li, xj, dj, Lj)
        # swap i and j
        s2, t2, d2, e2, _ = oracle.closest(xj, dj, Lj, xi, di, Li)
        assert d2 == pytest.approx(dist, rel=1e-12)
        assert np.allclose(e2, -e, atol=1e-10)
        # flip a director: the same points with negated arclength
        s3, t3, d3, e3, _ = oracle.closest(xi, -di, Li, xj, dj, Lj)
        assert d3 == pytest.approx(dist, rel=1e-12)
        assert np.allclose(xi + s * di, xi + s3 * (-di), atol=1e-10)
        # rigid motion
        q = _rand_quat(rng)
        R = oracle.rotation(q)
        sh = rng.standard_normal(3)
        s4, t4, d4, e4, _ = oracle.closest(R @ xi + sh, R @ di, Li, R @ xj + sh, R @ dj, Lj)
        assert d4 == pytest.approx(dist, rel=1e-11)
        assert np.allclose(e4, R @ e, atol=1e-9)


def test_closest_degenerate_crossing_axes():
    # the axes intersect: the normal falls back to di x dj, oriented along x_i - x_j
    s, t, dist, e, fl = oracle.closest([0, 0, 0], [1, 0, 0], 1.0, [0, 0, 0], [0, 1, 0], 1.0)
    assert dist == 0 and fl & oracle.FLAG_DEGENERATE
    assert np.allclose(np.abs(e), [0, 0, 1])
