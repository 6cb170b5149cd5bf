"""Multi-step pieces of the step on the GPU against the oracle: the Brownian
force, warm starts and the virial stress.

* Brownian: one step with N(0,1) draws and kT must give the oracle's
  velocities with F_nc = F + sqrt(2 kT/h) M^(-1/2) xi.
* Warm start: a step repeated on the same state starts at its own solution
  (0 iterations): the keys (two rods and shift in the caller's numbering,
  link key or index) find every constraint again although the pairs are
  built in the solver's own rod order, and links handed in another order
  with the same keys find theirs.  A short warm-started run with fresh random
  loads follows the oracle's cold-started run step by step (U is unique, so
  the start does not change it).
* Stress: the contact and link virials against the oracle's, on systems
  whose forces are unique (dilute contacts; links, definite by compliance).
"""
import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _solver(gpu_lib, s, **kw):
    return gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8, max_iter=200_000,
                          **kw)


def _oracle_U(s, L, F):
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, L, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, L, s.box, s.diam, s.eta, s.dt, pr, F)
    r = oracle.bbpgd(d, L, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=200_000)
    assert r.status == oracle.OK
    return d, pr, cs, r, oracle.velocity(d, L, s.diam, s.eta, pr, cs, r.gamma, F)


@pytest.mark.parametrize("which", ["small", "lengths"])
def test_brownian_step_matches_oracle(gpu_lib, which):
    s = rodsynth.cfg_small(3) if which == "small" else rodsynth.make_system(800, seed=6, phi=0.04,
                                                                               length=(0.5, 1.5))
    L = s.uniform_length if s.uniform_length is not None else s.length
    xi = np.random.default_rng(7).standard_normal((s.n, 6))
    kT = oracle.KT_300K
    d = oracle.directors(s.quat)
    Fnc = s.force + oracle.brownian_force(d, L, s.diam, s.eta, s.dt, kT, xi)
    _, pr, _, _, Uo = _oracle_U(s, L, Fnc)
    x, quat = _t(s.x), _t(s.quat)
    with _solver(gpu_lib, s) as slv:
        U, info, npairs = slv.step(x, quat, L if np.isscalar(L) else _t(L), F=_t(s.force), noise=_t(xi), kT=kT)
    assert info.status == gpu_lib.OK and npairs == pr.n
    U = U.cpu().numpy()
    assert np.linalg.norm(U - Uo) <= 1e-6 * np.linalg.norm(Uo)
    # the noise (forces of about 1.5 pN at 300 K over 1e-4 s) moves the
    # velocities well away from those of the external forces alone
    U_ext = _oracle_U(s, L, s.force)[4]
    assert np.linalg.norm(Uo - U_ext) > 0.1 * np.linalg.norm(Uo)


def test_warm_start_finds_every_constraint_again(gpu_lib):
    s = rodsynth.relaxed_system(3000, seed=2, phi=0.08, length=(0.5, 1.5))
    x0, q0 = _t(s.x), _t(s.quat)
    L, F = _t(s.length), _t(s.force)
    with _solver(gpu_lib, s) as slv:
        x, q = x0.clone(), q0.clone()
        U1, i1, n1 = slv.step(x, q, L, F=F, warm_start=True)
        assert i1.status == gpu_lib.OK and i1.iterations > 50
        x, q = x0.clone(), q0.clone()
        U2, i2, n2 = slv.step(x, q, L, F=F, warm_start=True)
    assert n2 == n1 and i2.status == gpu_lib.OK
    assert i2.iterations == 0 and i2.residual <= 1e-8
    assert torch.allclose(U1, U2, rtol=0, atol=1e-12 * float(U1.abs().max()))


def test_warm_start_follows_links_by_key(gpu_lib):
    """Links handed in another order with the same keys (as the crosslinker
    kinetics does, whose link list shifts whenever a crosslinker binds or
    unbinds) still find their previous forces: the repeated step starts at
    its solution.  Without keys (matched by index) the permuted links start
    from the wrong forces."""
    s = rodsynth.relaxed_system(2000, seed=5, phi=0.05)
    rng = np.random.default_rng(9)
    nl = 600
    a = rng.integers(0, s.n, nl)
    b = (a + 1 + rng.integers(0, s.n - 1, nl)) % s.n
    arm = rng.uniform(-0.5, 0.5, (nl, 2))
    d = oracle.directors(s.quat)
    pa = s.x[a] + arm[:, :1] * d[a]
    pb = s.x[b] + arm[:, 1:] * d[b]
    sep = pb - pa
    sep -= s.box * np.round(sep / s.box)
    rest = np.linalg.norm(sep, axis=1) * rng.uniform(0.8, 1.2, nl)
    kap = np.full(nl, 300.0)
    keys = rng.permutation(10 * nl)[:nl].astype(np.int64)
    perm = rng.permutation(nl)
    x0, q0, F = _t(s.x), _t(s.quat), _t(s.force)

    def links(order, with_keys):
        out = (_t(a[order], torch.int32), _t(b[order], torch.int32), _t(arm[order]), _t(kap[order]),
               _t(rest[order]), None)
        return out + (_t(keys[order], torch.int64),) if with_keys else out

    with _solver(gpu_lib, s) as slv:
        ident = np.arange(nl)
        g1 = torch.empty(nl, dtype=torch.float64, device="cuda")
        U1, i1, _ = slv.step(x0.clone(), q0.clone(), 1.0, F=F, links=links(ident, True), gamma_links=g1,
                             warm_start=True)
        assert i1.status == gpu_lib.OK and i1.iterations > 0
        g2 = torch.empty(nl, dtype=torch.float64, device="cuda")
        U2, i2, _ = slv.step(x0.clone(), q0.clone(), 1.0, F=F, links=links(perm, True), gamma_links=g2,
                             warm_start=True)
        assert i2.status == gpu_lib.OK and i2.iterations == 0
        assert torch.allclose(U1, U2, rtol=0, atol=1e-12 * float(U1.abs().max()))
        assert torch.allclose(g1[torch.as_tensor(perm, device="cuda")], g2, rtol=0,
                              atol=1e-12 * float(g1.abs().max()))
        # matched by index instead: the permuted links start from other links' forces
        slv.step(x0.clone(), q0.clone(), 1.0, F=F, links=links(ident, False), warm_start=True)
        _, i3, _ = slv.step(x0.clone(), q0.clone(), 1.0, F=F, links=links(perm, False), warm_start=True)
        assert i3.status == gpu_lib.OK and i3.iterations > 0


def test_kmc_link_keys_are_crosslinker_indices(gpu_lib):
    s = rodsynth.cfg_small(2)
    d = oracle.directors(s.quat)
    um3 = oracle.AVOGADRO_UM3_PER_UM
    kw = dict(eps=1625.0, Ka=[90.9 / um3] * 2, koS=[33.0] * 2, Ke=[90.9 / um3] * 2, koD=[33.0] * 2, kappa=300.0,
              rest=0.053, lam=0.258, kT=oracle.KT_300K, rcs=0.039, rcd=0.11, dU=1.0)
    ko = oracle.kmc_params(diam=s.diam, dt=s.dt, **kw)
    vbd = oracle.kmc_effective_volume(ko)
    m = 2000
    xl = oracle.Crosslinkers(np.zeros(m, np.int32), np.full((m, 2), -1, np.int32), np.zeros((m, 2)),
                             rodsynth.crosslinker_positions(m, s.box, 4))
    for k in range(6):
        u, xi = rodsynth.kmc_draws(m, 4, k)
        oracle.kmc_step(s.x, d, 1.0, s.box, ko, vbd, xl, u, xi)
    with _solver(gpu_lib, s) as slv:
        kp = gpu_lib.kmc_params(**kw)
        p, q, arm, kap, rest, key = slv.kmc_links(kp, _t(xl.state, torch.int32), _t(xl.rod, torch.int32),
                                                  _t(xl.arc), keys=True)
    dd = np.flatnonzero(xl.state == oracle.KMC_D)
    assert dd.size > 10
    assert np.array_equal(key.cpu().numpy(), dd)
    assert np.array_equal(p.cpu().numpy(), xl.rod[dd, 0]) and np.array_equal(q.cpu().numpy(), xl.rod[dd, 1])


def test_warm_started_run_follows_the_oracle(gpu_lib):
    s = rodsynth.cfg_small(4)
    rng = np.random.default_rng(3)
    forces = [s.force] + [rng.standard_normal((s.n, 6)) for _ in range(4)]
    xo, qo = s.x.copy(), s.quat.copy()
    x, q = _t(s.x), _t(s.quat)
    cold_iters, warm_iters = [], []
    with _solver(gpu_lib, s) as slv, _solver(gpu_lib, s) as cold:
        for t, F in enumerate(forces):
            so = rodsynth.RodSystem(x=xo, quat=qo, length=s.length, force=F, box=s.box)
            _, pr, _, r, Uo = _oracle_U(so, 1.0, F)
            xc, qc = x.clone(), q.clone()
            _, ic, _ = cold.step(xc, qc, 1.0, F=_t(F))
            U, info, npairs = slv.step(x, q, 1.0, F=_t(F), warm_start=True)
            assert info.status == gpu_lib.OK and npairs == pr.n
            assert np.linalg.norm(U.cpu().numpy() - Uo) <= 1e-6 * np.linalg.norm(Uo), t
            oracle.integrate(s.box, s.dt, Uo, xo, qo)
            cold_iters.append(ic.iterations)
            warm_iters.append(info.iterations)
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-9
    # fresh random loads every step: the previous forces are no better a
    # start than zero here (the counts are printed, not asserted)
    print(f"\nwarm-start iterations {warm_iters}, cold {cold_iters}")


def test_stress_matches_oracle(gpu_lib):
    s = rodsynth.cfg_small(5)
    d, pr, cs, r, Uo = _oracle_U(s, 1.0, s.force)
    rng = np.random.default_rng(4)
    k = rng.choice(pr.n, size=300, replace=False)
    links = oracle.Links(pr.pi[k].astype(np.int32), pr.pj[k].astype(np.int32), cs.arm[k].copy(),
                         rng.uniform(20.0, 200.0, 300), np.zeros(300))
    lg = oracle.links_geometry(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, links)
    links.rest = np.maximum(lg.length + rng.normal(0.0, 0.01, 300), 0.0)
    lg = oracle.links_geometry(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, links, s.force)
    gc = oracle.general(pr, cs, links, lg)
    rg = oracle.bbpgd_gen(d, 1.0, s.diam, s.eta, gc, tol=1e-10, max_iter=200_000)
    assert rg.status == oracle.OK
    sc, sl = oracle.stress(s.x, d, 1.0, s.box, pr, cs, rg.gamma[:pr.n], links, lg, rg.gamma[pr.n:])
    lk = (_t(links.p, torch.int32), _t(links.q, torch.int32), _t(links.arm), _t(links.kappa), _t(links.rest), None)
    with _solver(gpu_lib, s, ) as slv:
        slv.set_params(tol=1e-10)
        _, info, _ = slv.step(_t(s.x), _t(s.quat), 1.0, F=_t(s.force), links=lk, stress=True)
        st = slv.last_stress
        # contacts alone, through the plain step
        _, info2, _ = slv.step(_t(s.x), _t(s.quat), 1.0, F=_t(s.force), stress=True)
        st2 = slv.last_stress
    assert info.status == gpu_lib.OK and info2.status == gpu_lib.OK
    assert np.allclose(st[0], sc, rtol=0, atol=1e-6 * np.abs(sc).max())
    assert np.allclose(st[1], sl, rtol=0, atol=1e-6 * np.abs(sl).max())
    sc0, _ = oracle.stress(s.x, d, 1.0, s.box, pr, cs, r.gamma)
    assert np.allclose(st2[0], sc0, rtol=0, atol=1e-5 * np.abs(sc0).max())
    assert np.all(st2[1] == 0.0) and np.trace(st2[0]) > 0.0
