"""Crosslinker kinetics on the GPU against the oracle (rl_kmc_step,
rl_kmc_links, rl_kmc_effective_volume).

Each crosslinker's step is a pure function of the filaments, its state and
its own random numbers, so the comparison is crosslinker by crosslinker:
states, filaments and events bit-exact, arclengths and positions to 1e-12
(the two sides sum the candidates' rates in different orders; a decision can
only differ when a uniform number falls within rounding of its threshold,
which no case here comes near).  Systems: the small test suspension, varied
lengths in a 2 um box (every filament near several images of the query
point), the paper-scale nematic suspension with the kinesin-5 parameters of
the crosslinker table on sampled crosslinkers, and a run of several steps.
"""
import json
import os

import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "kmc_crosslinker_parameters.json")))
UM3 = oracle.AVOGADRO_UM3_PER_UM


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _kinesin5(rate=1.0, **kw):
    m = GOLD["motors"]["kinesin5"]
    base = dict(eps=m["eps_per_um"], Ka=[v / UM3 for v in m["Ka_per_uM"]], koS=[rate * v for v in m["koS_per_s"]],
                Ke=[v / UM3 for v in m["Ke_per_uM"]], koD=[rate * v for v in m["koD_per_s"]],
                kappa=m["kappa_pN_per_um"], rest=m["l0_um"], lam=m["lambda"], kT=oracle.KT_300K, rcs=m["rc_um"],
                rcd=0.11, dU=1.0)
    base.update(kw)
    return base


def _params(gpu_lib, dt, diam, **kw):
    ko = oracle.kmc_params(diam=diam, dt=dt, **kw)
    kg = gpu_lib.kmc_params(**kw)
    return ko, kg


def _populate(s, d, L, ko, vbd, m, steps, seed):
    """Crosslinkers in mixed states: m unbound ones run through the oracle."""
    xl = oracle.Crosslinkers(np.zeros(m, np.int32), np.full((m, 2), -1, np.int32), np.zeros((m, 2)),
                             rodsynth.crosslinker_positions(m, s.box, seed))
    for k in range(steps):
        u, xi = rodsynth.kmc_draws(m, seed, 1000 + k)
        oracle.kmc_step(s.x, d, L, s.box, ko, vbd, xl, u, xi)
    return xl


def _gpu_step(gpu_lib, slv, s, d, L, kg, xl, u, xi):
    st, rod, arc, xx = _t(xl.state, torch.int32), _t(xl.rod, torch.int32), _t(xl.arc), _t(xl.x)
    ev = torch.empty(xl.state.shape[0], dtype=torch.int32, device="cuda")
    counts = slv.kmc_step(_t(s.x), _t(d), L if np.isscalar(L) else _t(L), kg, st, rod, arc, xx, _t(u), _t(xi), ev)
    return (oracle.Crosslinkers(st.cpu().numpy(), rod.cpu().numpy(), arc.cpu().numpy(), xx.cpu().numpy()),
            ev.cpu().numpy(), counts)


def _compare(got, gev, want, wev):
    assert np.array_equal(got.state, want.state)
    assert np.array_equal(got.rod, want.rod)
    assert np.array_equal(gev, wev)
    assert np.abs(got.arc - want.arc).max(initial=0.0) <= 1e-12
    dx = np.abs(got.x - want.x)
    assert dx.max(initial=0.0) <= 1e-12


def _solver(gpu_lib, s, dt=1e-4):
    return gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=dt)


@pytest.mark.parametrize("which", ["kinesin5", "dynein"])
def test_effective_volume_matches_oracle(gpu_lib, which):
    m = GOLD["motors"][which]
    kw = _kinesin5(kappa=m["kappa_pN_per_um"], rest=m["l0_um"], lam=m["lambda"])
    ko, kg = _params(gpu_lib, 1e-4, 0.025, **kw)
    s = rodsynth.cfg_small(0)
    with _solver(gpu_lib, s) as slv:
        v = slv.kmc_effective_volume(kg)
    assert v == pytest.approx(oracle.kmc_effective_volume(ko), rel=1e-11)


@pytest.mark.parametrize("which,rate", [("small", 1.0), ("small", 100.0), ("lengths", 10.0)])
def test_kmc_step_matches_oracle(gpu_lib, which, rate):
    if which == "small":
        s = rodsynth.cfg_small(1)
    else:
        s = rodsynth.make_system(300, seed=9, box=2.0, length=(0.5, 1.5))
    L = s.uniform_length if s.uniform_length is not None else s.length
    d = oracle.directors(s.quat)
    kw = _kinesin5(rate)
    ko, kg = _params(gpu_lib, s.dt, s.diam, **kw)
    vbd = oracle.kmc_effective_volume(ko)
    pop = oracle.kmc_params(diam=s.diam, dt=s.dt, **_kinesin5(300.0))
    xl = _populate(s, d, L, pop, oracle.kmc_effective_volume(pop), 3000, 6, seed=len(which))
    states = np.bincount(xl.state, minlength=4)
    assert np.all(states > 50), states
    with _solver(gpu_lib, s) as slv:
        for step in range(3):
            u, xi = rodsynth.kmc_draws(3000, 7, step)
            want = xl.copy()
            wev = oracle.kmc_step(s.x, d, L, s.box, ko, vbd, want, u, xi)
            got, gev, counts = _gpu_step(gpu_lib, slv, s, d, L, kg, xl, u, xi)
            _compare(got, gev, want, wev)
            assert counts == np.bincount(wev, minlength=5).tolist()
            xl = want
    assert np.bincount(wev, minlength=5)[1:].sum() > 0


def test_kmc_paper_scale_sampled(gpu_lib):
    """The 100,000-filament nematic suspension with the kinesin-5 parameters:
    400,000 crosslinkers in mixed states stepped on the GPU; 300 sampled
    crosslinkers of each state stepped by the oracle (every crosslinker is
    independent of the others) and compared."""
    s = rodsynth.cfg_paper_scale(0)
    d = oracle.directors(s.quat)
    kw = _kinesin5(30.0)
    ko, kg = _params(gpu_lib, s.dt, s.diam, **kw)
    vbd = oracle.kmc_effective_volume(ko)
    m = 400_000
    rng = np.random.default_rng(11)
    # mixed states: unbound crosslinkers, heads bound at random sites, and
    # doubly bound ones on the contact pairs of the suspension
    pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff, method="cells")
    cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
    state = rng.integers(0, 4, m).astype(np.int32)
    rod = np.full((m, 2), -1, np.int32)
    arc = np.zeros((m, 2))
    sa = state == oracle.KMC_SA
    sb = state == oracle.KMC_SB
    dd = state == oracle.KMC_D
    rod[sa, 0] = rng.integers(0, s.n, sa.sum())
    arc[sa, 0] = rng.uniform(-0.5, 0.5, sa.sum())
    rod[sb, 1] = rng.integers(0, s.n, sb.sum())
    arc[sb, 1] = rng.uniform(-0.5, 0.5, sb.sum())
    k = rng.integers(0, pr.n, dd.sum())
    keep = pr.pi[k] != pr.pj[k]
    idx = np.flatnonzero(dd)
    rod[idx[keep], 0], rod[idx[keep], 1] = pr.pi[k[keep]], pr.pj[k[keep]]
    arc[idx[keep], 0], arc[idx[keep], 1] = cs.arm[k[keep], 0], cs.arm[k[keep], 1]
    state[idx[~keep]] = oracle.KMC_U
    x = rodsynth.crosslinker_positions(m, s.box, 3)
    xl = oracle.Crosslinkers(state, rod, np.ascontiguousarray(arc), x)
    u, xi = rodsynth.kmc_draws(m, 5, 0)
    with _solver(gpu_lib, s) as slv:
        got, gev, counts = _gpu_step(gpu_lib, slv, s, d, 1.0, kg, xl, u, xi)
    assert sum(counts) == m and all(c > 0 for c in counts)
    pick = np.concatenate([rng.choice(np.flatnonzero(state == k), 300, replace=False) for k in range(4)])
    sub = oracle.Crosslinkers(state[pick].copy(), rod[pick].copy(), np.ascontiguousarray(arc[pick]),
                              np.ascontiguousarray(x[pick]))
    wev = oracle.kmc_step(s.x, d, 1.0, s.box, ko, vbd, sub, np.ascontiguousarray(u[pick]),
                          np.ascontiguousarray(xi[pick]))
    _compare(oracle.Crosslinkers(got.state[pick], got.rod[pick], got.arc[pick], got.x[pick]), gev[pick], sub, wev)
    assert np.bincount(wev, minlength=5)[1:].sum() > 50


def test_kmc_links_are_the_doubly_bound(gpu_lib):
    s = rodsynth.cfg_small(2)
    d = oracle.directors(s.quat)
    kw = _kinesin5(300.0)
    ko, kg = _params(gpu_lib, s.dt, s.diam, **kw)
    xl = _populate(s, d, 1.0, ko, oracle.kmc_effective_volume(ko), 2000, 6, seed=4)
    with _solver(gpu_lib, s) as slv:
        p, q, arm, kap, rest = slv.kmc_links(kg, _t(xl.state, torch.int32), _t(xl.rod, torch.int32), _t(xl.arc))
    dd = xl.state == oracle.KMC_D
    assert dd.sum() > 10
    assert np.array_equal(p.cpu().numpy(), xl.rod[dd, 0]) and np.array_equal(q.cpu().numpy(), xl.rod[dd, 1])
    assert np.array_equal(arm.cpu().numpy(), xl.arc[dd])
    assert np.all(kap.cpu().numpy() == kw["kappa"]) and np.all(rest.cpu().numpy() == kw["rest"] + s.diam)


def test_kmc_errors(gpu_lib):
    s = rodsynth.cfg_small(0)
    d = oracle.directors(s.quat)
    ko, kg = _params(gpu_lib, s.dt, s.diam, **_kinesin5())
    m = 4
    u, xi = rodsynth.kmc_draws(m, 0, 0)
    with _solver(gpu_lib, s) as slv:
        bad = [(np.array([1, 0, 0, 0]), np.array([[-1, -1]] * 4)),          # S_A without a filament
               (np.array([3, 0, 0, 0]), np.array([[5, 5], [-1, -1], [-1, -1], [-1, -1]])),  # both heads on one
               (np.array([0, 0, 7, 0]), np.array([[-1, -1]] * 4)),          # unknown state
               (np.array([2, 0, 0, 0]), np.array([[-1, 1000], [-1, -1], [-1, -1], [-1, -1]]))]  # index >= n
        for st, rod in bad:
            with pytest.raises(gpu_lib.RodLCPError) as ei:
                slv.kmc_step(_t(s.x), _t(d), 1.0, kg, _t(st, torch.int32), _t(rod, torch.int32),
                             _t(np.zeros((m, 2))), _t(np.full((m, 3), 1.0)), _t(u), _t(xi))
            assert ei.value.status == gpu_lib.ERR_ARG
    # a capture reach beyond half the box
    small = rodsynth.make_system(10, seed=0, box=1.1)
    with _solver(gpu_lib, small) as slv:
        with pytest.raises(gpu_lib.RodLCPError) as ei:
            slv.kmc_step(_t(small.x), _t(oracle.directors(small.quat)), 1.0, kg,
                         _t(np.zeros(m), torch.int32), _t(np.full((m, 2), -1), torch.int32), _t(np.zeros((m, 2))),
                         _t(np.full((m, 3), 0.5)), _t(u), _t(xi))
        assert ei.value.status == gpu_lib.ERR_ARG
