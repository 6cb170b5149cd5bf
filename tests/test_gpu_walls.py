"""Walls and whole steps with links and walls on the GPU against the oracle.

rl_assemble_walls against the oracle's wall contacts (same list, same
order); the paper's confined suspension (3,200 rods of 1 um in a spherical
shell of radius 3 um) stepped with its shell; and a step with contacts,
crosslinker-like links and walls together, where the velocities and the
links' forces (unique: the compliance makes their part definite) must match
the oracle's."""
import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _ora_walls(wl):
    return [oracle.wall(k, p, a, r) for (k, p, a, r) in wl]


def test_assemble_walls_matches_oracle(gpu_lib):
    s = rodsynth.make_system(2000, seed=4, box=6.0, length=(0.5, 1.5))
    wl = [(gpu_lib.WALL_PLANE, (0.0, 0.0, 0.8), (0.0, 0.6, 0.8), 0.0),
          (gpu_lib.WALL_SPHERE_IN, (3.0, 3.0, 3.0), (0.0, 0.0, 1.0), 2.2),
          (gpu_lib.WALL_CYLINDER_IN, (3.0, 3.0, 0.0), (0.6, 0.0, 0.8), 2.0)]
    d = oracle.directors(s.quat)
    ref = oracle.walls(s.x, d, s.length, s.diam, s.eta, s.dt, s.cutoff, _ora_walls(wl), s.force)
    assert ref.n > 500
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt) as slv:
        rod, e, arm, phi, q, fl = slv.assemble_walls(_t(s.x), _t(d), _t(s.length), wl, F=_t(s.force))
    rod, e, arm, phi, q, fl = (v.cpu().numpy() for v in (rod, e, arm, phi, q, fl))
    assert not fl.any()
    assert np.array_equal(rod, ref.rod) and np.array_equal(arm, ref.arm)
    assert np.allclose(phi, ref.phi, rtol=0, atol=1e-13)
    assert np.allclose(e, ref.e, rtol=0, atol=1e-13)
    assert np.allclose(q, ref.q, rtol=1e-12, atol=1e-12 * np.abs(ref.q).max())


def _oracle_step(s, L, links=None, wl=None):
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, L, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, L, s.box, s.diam, s.eta, s.dt, pr, s.force)
    lg = oracle.links_geometry(s.x, d, L, s.box, s.diam, s.eta, s.dt, links, s.force) if links else None
    wc = oracle.walls(s.x, d, L, s.diam, s.eta, s.dt, s.cutoff, _ora_walls(wl), s.force) if wl else None
    gc = oracle.general_all(pr, cs, links, lg, wc)
    r = oracle.bbpgd_gen(d, L, s.diam, s.eta, gc, tol=1e-8, max_iter=200_000)
    assert r.status == oracle.OK
    U = oracle.velocity_gen(d, L, s.diam, s.eta, gc, r.gamma, s.force)
    gl = r.gamma[pr.n:pr.n + (links.n if links else 0)]
    return pr, wc, U, gl


def _gpu_step(gpu_lib, s, L, links=None, wl=None):
    x, quat = _t(s.x), _t(s.quat)
    U = torch.empty((s.n, 6), dtype=torch.float64, device="cuda")
    lk = None if links is None else (_t(links.p, torch.int32), _t(links.q, torch.int32), _t(links.arm),
                                     _t(links.kappa), _t(links.rest),
                                     _t(links.anchor) if links.anchor is not None else None)
    gl = torch.empty(links.n if links else 0, dtype=torch.float64, device="cuda")
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                        max_iter=200_000) as slv:
        _, info, npairs = slv.step(x, quat, L if np.isscalar(L) else _t(L), F=_t(s.force), U=U, links=lk,
                                   gamma_links=gl if links else None, walls=wl)
        nw = slv.last_wall_contacts
    return x.cpu().numpy(), quat.cpu().numpy(), U.cpu().numpy(), gl.cpu().numpy(), info, npairs, nw


def test_confined_suspension_step(gpu_lib):
    s = rodsynth.confined_system(3200, seed=1)
    wl = [rodsynth.shell_wall(s)]
    # push the rods outwards so that many of them meet the shell within the step
    c = 0.5 * s.box
    out = s.x - c
    s.force[:, :3] += 40.0 * out / np.linalg.norm(out, axis=1, keepdims=True)
    pr, wc, Uo, _ = _oracle_step(s, 1.0, wl=wl)
    x, quat, U, _, info, npairs, nw = _gpu_step(gpu_lib, s, 1.0, wl=wl)
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    assert npairs == pr.n and nw == wc.n
    assert np.linalg.norm(U - Uo) <= 1e-6 * np.linalg.norm(Uo)
    xo, qo = s.x.copy(), s.quat.copy()
    oracle.integrate(s.box, s.dt, Uo, xo, qo)
    assert np.abs(x - xo).max() <= 1e-6 * s.dt * np.linalg.norm(Uo) + 1e-14


def test_step_with_contacts_links_and_walls(gpu_lib):
    s = rodsynth.make_system(1500, seed=3, box=5.0, length=(0.5, 1.5))
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, s.length, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, s.length, s.box, s.diam, s.eta, s.dt, pr, s.force)
    rng = np.random.default_rng(2)
    k = rng.choice(pr.n, size=600, replace=False)
    p, q = pr.pi[k], pr.pj[k]
    arm = np.stack([np.clip(cs.arm[k, 0] + rng.uniform(-0.05, 0.05, 600), -0.5 * s.length[p], 0.5 * s.length[p]),
                    np.clip(cs.arm[k, 1] + rng.uniform(-0.05, 0.05, 600), -0.5 * s.length[q], 0.5 * s.length[q])],
                   axis=1)
    links = oracle.Links(p.astype(np.int32), q.astype(np.int32), arm, rng.uniform(20.0, 200.0, 600), np.zeros(600))
    lg = oracle.links_geometry(s.x, d, s.length, s.box, s.diam, s.eta, s.dt, links)
    links.rest = np.maximum(lg.length + rng.normal(0.0, 0.01, 600), 0.0)
    anch = rng.random(600) < 0.15
    links.anchor = s.x[p] + arm[:, :1] * d[p] + rng.normal(0.0, 0.02, (600, 3))
    links.q = np.where(anch, -1, links.q).astype(np.int32)
    wl = [(1, (2.5, 2.5, 2.5), (0.0, 0.0, 1.0), 2.6), (0, (0.0, 0.0, 0.3), (0.0, 0.0, 1.0), 0.0)]
    pr2, wc, Uo, glo = _oracle_step(s, s.length, links, wl)
    assert wc.n > 50
    x, quat, U, gl, info, npairs, nw = _gpu_step(gpu_lib, s, s.length, links, wl)
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    assert npairs == pr2.n and nw == wc.n
    assert np.linalg.norm(U - Uo) <= 1e-6 * np.linalg.norm(Uo)
    assert np.linalg.norm(gl - glo) <= 1e-6 * np.linalg.norm(glo)
