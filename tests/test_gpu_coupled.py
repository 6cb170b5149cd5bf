"""The method's whole coupled step on the GPU against the oracle, step by
step: crosslinker kinetics, the doubly bound crosslinkers as links (keyed by
crosslinker for the warm start), and the filament step with contacts, links
and a confining shell as one constraint set under Brownian forces; then the
Euler update.  Each step starts both sides from the oracle's state, so the
comparison covers a realistic trajectory without letting rounding decide a
later kinetic event: states, filaments and events bit-exact, arclengths and
crosslinker positions to 1e-12, U to 1e-6 of its norm, centres to the same
bar times h."""
import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_coupled_steps_follow_the_oracle(gpu_lib):
    # the paper's confined suspension: 3,200 rods of length 1 in a shell of radius 3
    n, m, radius = 3200, 8000, 3.0
    s = rodsynth.confined_system(n, seed=1, radius=radius)
    wl = [rodsynth.shell_wall(s, radius)]
    ow = [oracle.wall(k, p, a, r) for (k, p, a, r) in wl]
    um3 = oracle.AVOGADRO_UM3_PER_UM
    kT = oracle.KT_300K
    kw = dict(eps=1625.0, Ka=[90.9 / um3] * 2, koS=[30.0] * 2, Ke=[90.9 / um3] * 2, koD=[30.0] * 2, kappa=300.0,
              rest=0.053, lam=0.258, kT=kT, rcs=0.039, rcd=0.11, dU=1.0)
    ko = oracle.kmc_params(diam=s.diam, dt=s.dt, **kw)
    vbd = oracle.kmc_effective_volume(ko)
    c = 0.5 * s.box
    xl = oracle.Crosslinkers(np.zeros(m, np.int32), np.full((m, 2), -1, np.int32), np.zeros((m, 2)),
                             rodsynth.crosslinker_positions_ball(m, (c, c, c), radius, 5))
    d0 = oracle.directors(s.quat)
    for k in range(8):
        u, xi = rodsynth.kmc_draws(m, 5, 100 + k)
        oracle.kmc_step(s.x, d0, 1.0, s.box, ko, vbd, xl, u, xi)
    rng = np.random.default_rng(11)
    xo, qo = s.x.copy(), s.quat.copy()
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                        max_iter=200_000) as slv:
        kp = gpu_lib.kmc_params(**{k: v for k, v in kw.items()})
        for step in range(3):
            d = oracle.directors(qo)
            u, xi = rodsynth.kmc_draws(m, 5, step)
            # kinetics
            st, rod, arc, xx = _t(xl.state, torch.int32), _t(xl.rod, torch.int32), _t(xl.arc), _t(xl.x)
            ev = torch.empty(m, dtype=torch.int32, device="cuda")
            slv.kmc_step(_t(xo), _t(d), 1.0, kp, st, rod, arc, xx, _t(u), _t(xi), ev)
            wev = oracle.kmc_step(xo, d, 1.0, s.box, ko, vbd, xl, u, xi)
            assert np.array_equal(st.cpu().numpy(), xl.state) and np.array_equal(rod.cpu().numpy(), xl.rod)
            assert np.array_equal(ev.cpu().numpy(), wev)
            assert np.abs(arc.cpu().numpy() - xl.arc).max(initial=0.0) <= 1e-12
            assert np.abs(xx.cpu().numpy() - xl.x).max(initial=0.0) <= 1e-12
            # links of the doubly bound, keyed by crosslinker
            p, q, arm, kap, rest, key = slv.kmc_links(kp, st, rod, arc, keys=True)
            dd = np.flatnonzero(xl.state == oracle.KMC_D)
            assert dd.size > 100 and np.array_equal(key.cpu().numpy(), dd)
            links = oracle.Links(xl.rod[dd, 0].copy(), xl.rod[dd, 1].copy(), np.ascontiguousarray(xl.arc[dd]),
                                 np.full(dd.size, kw["kappa"]), np.full(dd.size, kw["rest"] + s.diam))
            # the filament step, both sides from the oracle's state
            noise = rng.standard_normal((n, 6))
            Fnc = s.force + oracle.brownian_force(d, 1.0, s.diam, s.eta, s.dt, kT, noise)
            pr = oracle.pairs(xo, d, 1.0, s.box, s.diam, s.cutoff)
            cs = oracle.assemble(xo, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, Fnc)
            lg = oracle.links_geometry(xo, d, 1.0, s.box, s.diam, s.eta, s.dt, links, Fnc)
            wc = oracle.walls(xo, d, 1.0, s.diam, s.eta, s.dt, s.cutoff, ow, Fnc)
            gc = oracle.general_all(pr, cs, links, lg, wc)
            r = oracle.bbpgd_gen(d, 1.0, s.diam, s.eta, gc, tol=1e-8, max_iter=200_000)
            assert r.status == oracle.OK
            Uo = oracle.velocity_gen(d, 1.0, s.diam, s.eta, gc, r.gamma, Fnc)
            x, quat = _t(xo), _t(qo)
            U = torch.empty((n, 6), dtype=torch.float64, device="cuda")
            _, info, npairs = slv.step(x, quat, 1.0, F=_t(s.force), U=U, links=(p, q, arm, kap, rest, None, key),
                                       walls=wl, noise=_t(noise), kT=kT, warm_start=True)
            assert info.status == gpu_lib.OK and info.residual <= 1e-8
            assert npairs == pr.n and slv.last_wall_contacts == wc.n
            U = U.cpu().numpy()
            assert np.linalg.norm(U - Uo) <= 1e-6 * np.linalg.norm(Uo), step
            oracle.integrate(s.box, s.dt, Uo, xo, qo)
            assert np.abs(x.cpu().numpy() - xo).max() <= 1e-6 * s.dt * np.linalg.norm(Uo) + 1e-13, step
