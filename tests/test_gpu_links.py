"""Bilateral links and general constraint sets on the GPU against the oracle.

rl_assemble_links against the oracle's link geometry; rl_solve_general on
links alone (a unique solution: the compliance makes the matrix definite),
on contacts and links together, with tethers to fixed points, in shuffled
input orders; the anchored-rod relaxation at the rate Section 3 prints; and
the errors the entry points report."""
import math

import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _random_links(rng, n, nl, box, frac_anchor=0.2):
    p = rng.integers(0, n, nl)
    q = (p + 1 + rng.integers(0, n - 1, nl)) % n
    q = np.where(rng.random(nl) < frac_anchor, -1, q)
    arm = rng.uniform(-0.45, 0.45, (nl, 2))
    kappa = rng.uniform(10.0, 400.0, nl)
    rest = rng.uniform(0.0, 0.4, nl)
    anchor = rng.uniform(0.0, box, (nl, 3))
    return oracle.Links(p.astype(np.int32), q.astype(np.int32), arm, kappa, rest, anchor)


def _crosslinks(rng, s, d, L, pr, cs, nl, frac_anchor=0.1):
    """Links like doubly bound crosslinkers: between rods that are near each
    other (pairs of the contact list), near their closest points, with rest
    lengths near the current separation; some tether a rod to a point next
    to it."""
    k = rng.choice(pr.n, size=min(nl, pr.n), replace=False)
    p, q = pr.pi[k].astype(np.int32), pr.pj[k].astype(np.int32)
    Lp = L if np.isscalar(L) else L[p]
    Lq = L if np.isscalar(L) else L[q]
    arm = np.stack([np.clip(cs.arm[k, 0] + rng.uniform(-0.05, 0.05, k.size), -0.5 * Lp, 0.5 * Lp),
                    np.clip(cs.arm[k, 1] + rng.uniform(-0.05, 0.05, k.size), -0.5 * Lq, 0.5 * Lq)], axis=1)
    lk = oracle.Links(p, q, arm, rng.uniform(20.0, 200.0, k.size), np.zeros(k.size), None)
    lg = oracle.links_geometry(s.x, d, L, s.box, s.diam, s.eta, s.dt, lk)
    lk.rest = np.maximum(lg.length + rng.normal(0.0, 0.005, k.size), 0.0)
    anch = rng.random(k.size) < frac_anchor
    lk.anchor = s.x[p] + arm[:, :1] * d[p] + rng.normal(0.0, 0.02, (k.size, 3))
    lk.q = np.where(anch, -1, q).astype(np.int32)
    return lk


def _gpu_links(lk):
    return (_t(lk.p, torch.int32), _t(lk.q, torch.int32), _t(lk.arm), _t(lk.kappa), _t(lk.rest),
            _t(lk.anchor) if lk.anchor is not None else None)


def test_assemble_links_matches_oracle(gpu_lib):
    s = rodsynth.make_system(300, seed=3, box=3.0, length=(0.5, 1.5))
    rng = np.random.default_rng(5)
    lk = _random_links(rng, s.n, 500, s.box)
    lk.kappa[:10] = np.inf                       # rigid joints
    # a zero-length link: two rods whose link points coincide
    lk.p[10], lk.q[10], lk.arm[10] = 0, 1, (0.0, 0.0)
    x = s.x.copy()
    x[1] = x[0]
    d = oracle.directors(s.quat)
    ref = oracle.links_geometry(x, d, s.length, s.box, s.diam, s.eta, s.dt, lk, s.force)
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt) as slv:
        L, e, q, cmp, fl = slv.assemble_links(_t(x), _t(d), _t(s.length), *_gpu_links(lk), F=_t(s.force))
    L, e, q, cmp, fl = (v.cpu().numpy() for v in (L, e, q, cmp, fl))
    assert np.allclose(L, ref.length, rtol=1e-14, atol=1e-14)
    assert np.allclose(e, ref.e, rtol=0, atol=1e-12)
    assert np.allclose(q, ref.q, rtol=1e-12, atol=1e-12 * np.abs(ref.q).max())
    assert np.array_equal(cmp, ref.cmp) or np.allclose(cmp, ref.cmp, rtol=1e-15, atol=0)
    assert np.array_equal(fl, ref.flags) and fl[10] == 4 and np.all(cmp[:10] == 0.0)


def _general_inputs(s, d, L, pr, cs, lk, lg, order=None):
    gc = oracle.general(pr, cs, lk, lg)
    o = np.arange(gc.n) if order is None else order
    args = (_t(d), _t(L) if not np.isscalar(L) else L, _t(gc.pi[o], torch.int32), _t(gc.pj[o], torch.int32),
            _t(gc.e[o]), _t(gc.arm[o]), _t(gc.q[o]), _t(gc.kind[o], torch.uint8), _t(gc.cmp[o]))
    return gc, args


def _check(gpu_lib, s, d, L, gc, g, U, info, tol=1e-8):
    assert info.status == gpu_lib.OK and info.residual <= tol, info
    w = oracle.apply_Mc_gen(d, L, s.diam, s.eta, gc, g)
    u = gc.kind == 0
    scale = 1e-12 * max(1.0, np.abs(gc.q).max(initial=1.0))
    assert g[u].min(initial=0.0) >= 0.0
    assert np.abs(np.minimum(g[u], w[u])).max(initial=0.0) <= tol + scale
    assert np.abs(w[~u]).max(initial=0.0) <= tol + scale
    ref = oracle.bbpgd_gen(d, L, s.diam, s.eta, gc, tol=tol, max_iter=200_000)
    assert ref.status == oracle.OK
    Uo = oracle.velocity_gen(d, L, s.diam, s.eta, gc, ref.gamma, s.force)
    assert np.linalg.norm(U - Uo) <= 1e-6 * np.linalg.norm(Uo)
    return ref


def test_links_only_unique_solution(gpu_lib):
    s = rodsynth.make_system(200, seed=8, box=3.0)
    rng = np.random.default_rng(9)
    lk = _random_links(rng, s.n, 300, s.box)
    d = oracle.directors(s.quat)
    lg = oracle.links_geometry(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, lk, s.force)
    gc, args = _general_inputs(s, d, 1.0, None, None, lk, lg)
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                        max_iter=200_000) as slv:
        g, U, info = slv.solve_general(*args, F=_t(s.force))
    g, U = g.cpu().numpy(), U.cpu().numpy()
    ref = _check(gpu_lib, s, d, 1.0, gc, g, U, info)
    # the compliance makes Mc + C definite: gamma itself is unique
    assert np.linalg.norm(g - ref.gamma) <= 1e-6 * np.linalg.norm(ref.gamma)


@pytest.mark.parametrize("which", ["small", "lengths", "dense"])
def test_contacts_and_links(gpu_lib, which):
    if which == "small":
        s = rodsynth.cfg_small(2)
    elif which == "lengths":
        s = rodsynth.make_system(800, seed=6, phi=0.04, length=(0.5, 1.5))
    else:
        s = rodsynth.relaxed_system(3000, seed=4, phi=0.08, length=(0.5, 1.5))
    L = s.uniform_length if s.uniform_length is not None else s.length
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, L, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, L, s.box, s.diam, s.eta, s.dt, pr, s.force)
    rng = np.random.default_rng(len(which))
    lk = _crosslinks(rng, s, d, L, pr, cs, s.n // 2)
    lg = oracle.links_geometry(s.x, d, L, s.box, s.diam, s.eta, s.dt, lk, s.force)
    gc, args = _general_inputs(s, d, L, pr, cs, lk, lg)
    with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                        max_iter=200_000) as slv:
        g, U, info = slv.solve_general(*args, F=_t(s.force))
        g, U = g.cpu().numpy(), U.cpu().numpy()
        _check(gpu_lib, s, d, L, gc, g, U, info)
        # any input order: the same problem, the same velocities
        perm = rng.permutation(gc.n)
        _, args2 = _general_inputs(s, d, L, pr, cs, lk, lg, perm)
        g2, U2, info2 = slv.solve_general(*args2, F=_t(s.force))
    assert info2.status == gpu_lib.OK
    U2 = U2.cpu().numpy()
    assert np.linalg.norm(U2 - U) <= 1e-6 * np.linalg.norm(U)


def test_anchored_rod_relaxes_at_the_papers_rate(gpu_lib):
    N, eta, dt, kappa, l0, stretch = 5, 0.01, 1e-5, 100.0, 0.02, 0.01
    s_arm = np.linspace(-0.4, 0.4, N)
    anchors = np.stack([np.full(N, 5.0 + l0 + stretch), np.full(N, 5.0), 5.0 + s_arm], axis=1)
    lk = oracle.Links(np.zeros(N, np.int32), -np.ones(N, np.int32), np.stack([s_arm, np.zeros(N)], axis=1),
                      np.full(N, kappa), np.full(N, l0), anchors)
    x = np.array([[5.0, 5.0, 5.0]])
    d = np.array([[0.0, 0.0, 1.0]])
    with gpu_lib.Solver(box=10.0, eta=eta, dt=dt, tol=1e-12, max_iter=100_000) as slv:
        Lg, e, q, cmp, fl = slv.assemble_links(_t(x), _t(d), 1.0, *_gpu_links(lk))
        kind = torch.ones(N, dtype=torch.uint8, device="cuda")
        g, U, info = slv.solve_general(_t(d), 1.0, _t(lk.p, torch.int32), _t(lk.q, torch.int32), e, _t(lk.arm), q,
                                       kind, cmp)
    assert info.status == gpu_lib.OK
    U = U.cpu().numpy()
    lam = N * kappa / (4.0 * math.pi * eta * 1.0 / math.log(2.0 / 0.025))
    x1 = x[0] + dt * U[0, :3]
    new_len = np.linalg.norm(x1 + s_arm[:, None] * d[0] - anchors, axis=1)
    assert np.allclose(new_len, l0 + stretch / (1.0 + lam * dt), rtol=0, atol=1e-11)


def test_general_errors(gpu_lib):
    d = _t(np.array([[0.0, 0.0, 1.0]] * 2))
    e = _t(np.array([[1.0, 0.0, 0.0]]))
    arm = _t(np.zeros((1, 2)))
    q = _t(np.ones(1))
    with gpu_lib.Solver(box=10.0) as slv:
        for pi, pj, kind, cmp in ((0, 2, 0, 0.0), (0, -2, 0, 0.0), (0, 1, 2, 0.0), (0, 1, 1, -1.0)):
            with pytest.raises(gpu_lib.RodLCPError) as ei:
                slv.solve_general(d, 1.0, _t([pi], torch.int32), _t([pj], torch.int32), e, arm, q,
                                  _t([kind], torch.uint8), _t([cmp]))
            assert ei.value.status == gpu_lib.ERR_ARG
        with pytest.raises(gpu_lib.RodLCPError) as ei:
            slv.assemble_links(_t(np.zeros((2, 3))), d, 1.0, _t([0], torch.int32), _t([0], torch.int32), arm,
                               _t([1.0]), _t([0.1]))
        assert ei.value.status == gpu_lib.ERR_ARG
