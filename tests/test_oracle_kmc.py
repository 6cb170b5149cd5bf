"""Pins of the oracle's crosslinker kinetics (kinetic Monte Carlo; CPU).

The kinetics follow Section "2. Crosslinker binding and unbinding" (Table
tab:rates) and the appendix "Kinetic Monte-Carlo" (Table tab:supprates).  The
rates are chosen so that binding and unbinding obey detailed balance; the
pins check the oracle against what that fixes, never against its own
formulas:
  * the captured axis length L_in against brute-force sampling of the
    segment, and its closed forms (chord of a line through a sphere);
  * V_bd against the closed form of the untruncated Gaussian integral;
  * U <-> S equilibrium: the mean-field steady state of the appendix's
    reservoir equations, N_S = N a / (1 + a) with a = eps (K_A + K_B) L / V,
    and the head ratio N_SA / N_SB = K_A / K_B;
  * S <-> D equilibrium: the doubly bound fraction and the distribution of
    the second head over the sites follow the Boltzmann factor exp(-beta U)
    of the tether, the same for every lambda (lambda only sets how fast);
  * a head lands uniformly on the captured axis length;
  * the two heads never bind the same filament;
  * unbound crosslinkers diffuse with mean square displacement 6 d_U t;
  * the printed capture radii of the crosslinker table are (l_o + D) / 2.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import erf

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "kmc_crosslinker_parameters.json")))
DIAM = 0.025
KT = oracle.KT_300K


def _rods(centres, dirs, box):
    x = np.ascontiguousarray(centres, float)
    d = np.asarray(dirs, float)
    d = np.ascontiguousarray(d / np.linalg.norm(d, axis=1, keepdims=True))
    return x, d


def _params(**kw):
    base = dict(eps=27.0, Ka=0.1, koS=5.0, Ke=0.0, koD=0.0, kappa=100.0, rest=0.05, lam=0.5, kT=KT, rcs=0.04,
                rcd=0.12, dU=1.0, diam=DIAM, dt=1e-4)
    base.update(kw)
    return oracle.kmc_params(**base)


def _xl(m, box, rng, state=oracle.KMC_U):
    return oracle.Crosslinkers(np.full(m, state, np.int32), np.full((m, 2), -1, np.int32), np.zeros((m, 2)),
                               np.ascontiguousarray(rng.random((m, 3)) * box))


def _draws(rng, m):
    return rng.random((m, 4)), rng.standard_normal((m, 3))


# --- geometry ------------------------------------------------------------------

def test_inside_length_closed_forms():
    box = 5.0
    x, d = _rods([[2.5, 2.5, 2.5]], [[1.0, 0.0, 0.0]], box)
    r = 0.3
    # line through the centre: the diameter
    assert oracle.kmc_inside_length(x, d, 1.0, box, 0, [2.6, 2.5, 2.5], r) == pytest.approx(2 * r, rel=1e-15)
    # offset h: the chord 2 sqrt(r^2 - h^2)
    h = 0.17
    assert oracle.kmc_inside_length(x, d, 1.0, box, 0, [2.4, 2.5 + h, 2.5], r) == \
        pytest.approx(2 * math.sqrt(r * r - h * h), rel=1e-14)
    # sphere about the rod's end: half the diameter is on the rod
    assert oracle.kmc_inside_length(x, d, 1.0, box, 0, [3.0, 2.5, 2.5], r) == pytest.approx(r, rel=1e-15)
    # no contact
    assert oracle.kmc_inside_length(x, d, 1.0, box, 0, [2.5, 2.9, 2.5], r) == 0.0


def test_inside_length_against_sampled_segments():
    rng = np.random.default_rng(0)
    box = 3.0
    n = 40
    x = rng.random((n, 3)) * box
    d = rng.standard_normal((n, 3))
    L = rng.uniform(0.5, 1.5, n)
    x, d = _rods(x, d, box)
    t = (np.arange(200_000) + 0.5) / 200_000 - 0.5
    for k in range(200):
        i = int(rng.integers(n))
        r = rng.uniform(0.05, 0.6)
        # points near the rod (some across the periodic boundary)
        p = (x[i] + rng.uniform(-0.5, 0.5) * L[i] * d[i] + rng.normal(0, 0.2, 3)) % box
        got = oracle.kmc_inside_length(x, d, L, box, i, p, r)
        c = x[i] - p
        c -= box * np.floor(c / box + 0.5)
        pts = c[None, :] + np.outer(t * L[i], d[i])
        want = L[i] * np.mean(np.einsum("ij,ij->i", pts, pts) <= r * r)
        assert abs(got - want) <= 2.0 * L[i] / t.size + 1e-12


def test_effective_volume_closed_form():
    # untruncated: 4 pi int_0^inf r^2 exp(-a (r - c)^2) dr
    #            = 4 pi [(c^2 + 1/(2a)) G + c exp(-a c^2) / (2a)],
    #   G = int_{-c}^inf exp(-a t^2) dt = sqrt(pi/a) (1 + erf(c sqrt a)) / 2
    for kappa, rest in ((300.0, 0.053), (100.0, 0.040), (10.0, 0.05)):
        a = kappa / (2.0 * KT)
        c = rest + DIAM
        G = 0.5 * math.sqrt(math.pi / a) * (1.0 + erf(c * math.sqrt(a)))
        want = 4.0 * math.pi * ((c * c + 0.5 / a) * G + c * math.exp(-a * c * c) / (2.0 * a))
        P = _params(kappa=kappa, rest=rest, rcd=c + 12.0 / math.sqrt(a))
        assert oracle.kmc_effective_volume(P) == pytest.approx(want, rel=1e-10)


def test_printed_capture_radii_are_half_the_tether_plus_diameter():
    D = GOLD["filament_diameter_um"]
    for name, m in GOLD["motors"].items():
        assert round((m["l0_um"] + D) / 2.0, 3) == pytest.approx(m["rc_um"], abs=0.0011), name


# --- kinetics ------------------------------------------------------------------

def _bound_counts(st):
    return np.sum(st == oracle.KMC_SA), np.sum(st == oracle.KMC_SB), np.sum(st == oracle.KMC_D)


def test_unbound_singly_bound_mean_field_equilibrium():
    """Three 1 um filaments in a 2 um box (the setting of Fig. bind_rad) and
    4,000 passive crosslinkers.  The reservoir equations of the appendix give
    at steady state chi = eps k_on C / k_off per length for each head, so
    N_S = eps (K_A + K_B) L C and N = N_S + C V.  A capture radius of 0.4 um
    keeps R h small (the rate is piecewise large near a filament; the steady
    state does not depend on the radius when R h << 1); a fast diffusion
    (20 um^2/s) and fast rates (k_oS of 50 and 80 /s at h = 2e-5 s) bring it
    to equilibrium within about 3,000 steps (the approach is limited by the
    diffusion into the capture zones)."""
    rng = np.random.default_rng(1)
    box, n, m = 2.0, 3, 4000
    x, d = _rods(rng.random((n, 3)) * box, rng.standard_normal((n, 3)), box)
    KA, KB = 0.12, 0.05
    P = _params(Ka=(KA, KB), koS=(50.0, 80.0), rcs=0.4, eps=27.0, dU=20.0, dt=2e-5)
    xl = _xl(m, box, rng)
    a = 27.0 * (KA + KB) * n * 1.0 / box ** 3
    frac = []
    ratio = []
    for step in range(6000):
        u, xi = _draws(rng, m)
        oracle.kmc_step(x, d, 1.0, box, P, 1.0, xl, u, xi)
        if step >= 3000 and step % 40 == 0:
            sa, sb, dd = _bound_counts(xl.state)
            assert dd == 0
            frac.append((sa + sb) / m)
            ratio.append(sa / max(sb, 1))
    assert np.mean(frac) == pytest.approx(a / (1.0 + a), rel=0.02)
    assert np.mean(ratio) == pytest.approx(KA / KB, rel=0.05)
    # bound heads sit on their filaments, unbound ones anywhere
    b = xl.state != oracle.KMC_U
    assert np.all((xl.rod[b, 0] >= 0) ^ (xl.rod[b, 1] >= 0))


def _parallel_pair(h, box=4.0):
    c = box / 2
    return _rods([[c, c, c], [c, c + h, c]], [[1.0, 0, 0], [1.0, 0, 0]], box)


@pytest.mark.parametrize("lam", [0.2, 0.6])
def test_singly_doubly_bound_boltzmann_equilibrium(lam):
    """Head A held on filament 0 (no S -> U, and head A never releases);
    head B binds the sites of the parallel filament 1 and releases.  At
    equilibrium the doubly bound fraction is p_D / p_S = (K_e / V_bd)
    sum_k exp(-beta U(l_k)) and the second head's sites are weighted by
    exp(-beta U): the tether's Boltzmann factor, whatever lambda is."""
    rng = np.random.default_rng(2)
    box, h = 4.0, 0.075
    x, d = _parallel_pair(h, box)
    kappa, rest, eps = 10.0, 0.05, 27.0
    c = rest + DIAM
    rcd = 0.145
    Pv = _params(kappa=kappa, rest=rest, rcd=rcd, eps=eps, Ke=(0.0, 1.0), koD=(0.0, 200.0), koS=(0.0, 0.0),
                 lam=lam, dt=2e-5)
    Vbd = oracle.kmc_effective_volume(Pv)
    Ke = 0.3 * Vbd
    P = _params(kappa=kappa, rest=rest, rcd=rcd, eps=eps, Ke=(0.0, Ke), koD=(0.0, 200.0), koS=(0.0, 0.0), lam=lam,
                dt=2e-5)
    m = 2000
    sA = rng.uniform(-0.3, 0.3, m)
    xl = oracle.Crosslinkers(np.full(m, oracle.KMC_SA, np.int32), np.stack([np.zeros(m, np.int32),
                             -np.ones(m, np.int32)], axis=1).astype(np.int32).copy(),
                             np.ascontiguousarray(np.stack([sA, np.zeros(m)], axis=1)), np.zeros((m, 3)))
    # sites of filament 1 (length 1): floor(eps L) of them at interval centres
    ns = int(math.floor(eps * 1.0))
    sites = -0.5 + (np.arange(ns) + 0.5) / ns
    ell = np.sqrt(h * h + (sites[None, :] - sA[:, None]) ** 2)
    boltz = np.where(ell <= rcd, np.exp(-(kappa / KT) * 0.5 * (ell - c) ** 2), 0.0)
    ratio_pred = Ke / Vbd * boltz.sum(axis=1)                 # p_D / p_S per crosslinker
    pD_pred = np.mean(ratio_pred / (1.0 + ratio_pred))
    site_pred = np.sum(boltz / boltz.sum(axis=1, keepdims=True) * (ratio_pred / (1 + ratio_pred))[:, None], axis=0)
    counts = np.zeros(ns)
    pD = []
    for step in range(4000):
        u, xi = _draws(rng, m)
        oracle.kmc_step(x, d, 1.0, box, P, Vbd, xl, u, xi)
        if step >= 1000 and step % 10 == 0:
            dd = xl.state == oracle.KMC_D
            assert np.all(xl.rod[:, 0] == 0) and np.all(xl.rod[dd, 1] == 1)
            pD.append(dd.mean())
            k = np.rint((xl.arc[dd, 1] + 0.5) * ns - 0.5).astype(int)
            np.add.at(counts, k, 1.0)
    assert np.mean(pD) == pytest.approx(pD_pred, rel=0.03)
    # the sites' shares against the Boltzmann prediction (chi-square over the
    # sites that carry at least 1% of the weight)
    exp_share = site_pred / site_pred.sum()
    obs_share = counts / counts.sum()
    keep = exp_share > 0.01
    assert np.abs(obs_share[keep] - exp_share[keep]).max() <= 0.1 * exp_share[keep].max()


def test_head_lands_uniformly_on_the_captured_length():
    rng = np.random.default_rng(3)
    box = 4.0
    x, d = _rods([[2.0, 2.0, 2.0]], [[1.0, 0.0, 0.0]], box)
    m = 20000
    p0 = np.array([2.1, 2.0 + 0.2, 2.0])
    r = 0.3
    P = _params(rcs=r, Ka=(1.0, 3.0), koS=(1e6, 1e6), dU=0.0, dt=1.0)     # every crosslinker binds
    xl = oracle.Crosslinkers(np.zeros(m, np.int32), np.full((m, 2), -1, np.int32), np.zeros((m, 2)),
                             np.ascontiguousarray(np.tile(p0, (m, 1))))
    u, xi = _draws(rng, m)
    ev = oracle.kmc_step(x, d, 1.0, box, P, 1.0, xl, u, xi)
    assert np.all(ev == oracle.EV_BIND)
    half = math.sqrt(r * r - 0.04)
    lo, hi = 0.1 - half, 0.1 + half
    s = np.where(xl.state == oracle.KMC_SA, xl.arc[:, 0], xl.arc[:, 1])
    assert s.min() >= lo - 1e-12 and s.max() <= hi + 1e-12
    # uniform: Kolmogorov-Smirnov distance
    srt = np.sort((s - lo) / (hi - lo))
    ks = np.max(np.abs(srt - (np.arange(m) + 0.5) / m))
    assert ks < 1.63 / math.sqrt(m)
    # heads in proportion to K_A k_A : K_B k_B
    assert np.mean(xl.state == oracle.KMC_SB) == pytest.approx(0.75, abs=0.015)


def test_heads_never_share_a_filament():
    rng = np.random.default_rng(4)
    box = 4.0
    x, d = _rods([[2.0, 2.0, 2.0]], [[1.0, 0.0, 0.0]], box)
    m = 500
    P = _params(Ke=1.0, koD=1e4, koS=0.0, dt=1e-3)
    xl = oracle.Crosslinkers(np.full(m, oracle.KMC_SA, np.int32),
                             np.ascontiguousarray(np.stack([np.zeros(m), -np.ones(m)], 1).astype(np.int32)),
                             np.ascontiguousarray(np.stack([rng.uniform(-0.4, 0.4, m), np.zeros(m)], 1)),
                             np.zeros((m, 3)))
    for _ in range(20):
        u, xi = _draws(rng, m)
        ev = oracle.kmc_step(x, d, 1.0, box, P, 1.0, xl, u, xi)
        assert np.all(ev == oracle.EV_NONE) and np.all(xl.state == oracle.KMC_SA)


def test_unbound_crosslinkers_diffuse():
    rng = np.random.default_rng(5)
    box, m, steps, dt, dU = 50.0, 20000, 50, 1e-3, 0.7
    x, d = _rods([[1.0, 1.0, 1.0]], [[1.0, 0.0, 0.0]], box)
    P = _params(dU=dU, dt=dt, Ka=0.0)
    xl = _xl(m, box, rng)
    xl.x[:] = 25.0
    x0 = xl.x.copy()
    for _ in range(steps):
        u, xi = _draws(rng, m)
        oracle.kmc_step(x, d, 1.0, box, P, 1.0, xl, u, xi)
    msd = np.mean(np.sum((xl.x - x0) ** 2, axis=1))
    T = steps * dt
    assert msd == pytest.approx(6 * dU * T, rel=4 * math.sqrt(2.0 / (3 * m)))
