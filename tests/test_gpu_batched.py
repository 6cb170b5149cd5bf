"""Batching form: many independent systems solved in one batched solve.
Each system must match the oracle on its own (oracle-certified residual <=
1e-8, U within 1e-6), finished systems must not be disturbed by the ones
still iterating, and every workgroup-size choice must give a valid answer."""
import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _batch(systems):
    """Oracle inputs per system and the concatenated inputs (per-rod lengths)."""
    per, rods, pairs = [], [0], [0]
    cat = {k: [] for k in ("dir", "len", "pi", "pj", "e", "arm", "q", "F")}
    for s in systems:
        d = oracle.directors(s.quat)
        pr = oracle.pairs(s.x, d, s.length, s.box, s.diam, s.cutoff)
        cs = oracle.assemble(s.x, d, s.length, s.box, s.diam, s.eta, s.dt, pr, s.force)
        per.append((s, d, pr, cs))
        cat["dir"].append(d)
        cat["len"].append(s.length)
        cat["pi"].append(pr.pi + rods[-1])
        cat["pj"].append(pr.pj + rods[-1])
        cat["e"].append(cs.e)
        cat["arm"].append(cs.arm)
        cat["q"].append(cs.q)
        cat["F"].append(s.force)
        rods.append(rods[-1] + s.n)
        pairs.append(pairs[-1] + pr.n)
    arrays = {k: np.concatenate(v) for k, v in cat.items()}
    return per, np.array(rods), np.array(pairs), arrays


def _run(rl, systems, arrays, rods, pairs, rb=0, cb=0, max_iter=100_000):
    lens = arrays["len"]
    length = float(lens[0]) if lens.size and np.all(lens == lens[0]) else _t(lens)
    with rl.Solver(box=1.0, tol=1e-8, max_iter=max_iter) as slv:
        slv.batch_tuning(rb, cb)
        g, U, infos = slv.solve_lcp_batched(
            rods, pairs, _t(arrays["dir"]), length, _t(arrays["pi"], torch.int32), _t(arrays["pj"], torch.int32),
            _t(arrays["e"]), _t(arrays["arm"]), _t(arrays["q"]), F=_t(arrays["F"]))
        used = slv.batch_tuning(rb, cb)
    return g.cpu().numpy(), U.cpu().numpy(), infos, used


@pytest.fixture(scope="module")
def batch():
    # relaxed starts, volume fractions in [0.02, 0.1] as in the full batch
    systems = rodsynth.cfg_batched(3, systems=10, n_lo=100, n_hi=1500)
    systems.append(rodsynth.make_system(150, seed=9, box=40.0))            # no contacts at all
    systems.append(rodsynth.make_system(120, seed=2, phi=0.03))
    return systems, _batch(systems)


def test_batched_matches_oracle_per_system(gpu_lib, batch):
    systems, (per, rods, pairs, arrays) = batch
    g, U, infos, used = _run(gpu_lib, systems, arrays, rods, pairs)
    assert used[0] in (256, 1024) and used[1] in (256, 512)
    for k, (s, d, pr, cs) in enumerate(per):
        info = infos[k]
        assert info.status == gpu_lib.OK and info.residual <= 1e-8, (k, info)
        gk = g[pairs[k]:pairs[k + 1]]
        Uk = U[rods[k]:rods[k + 1]]
        w = oracle.apply_Mc(d, s.length, s.diam, s.eta, pr, cs, gk)
        assert np.abs(np.minimum(gk, w)).max(initial=0.0) <= 1e-8 + 1e-12 * np.abs(cs.q).max(initial=1.0)
        ref = oracle.bbpgd(d, s.length, s.diam, s.eta, pr, cs, tol=1e-8)
        Uref = oracle.velocity(d, s.length, s.diam, s.eta, pr, cs, ref.gamma, s.force)
        assert np.linalg.norm(Uk - Uref) <= 1e-6 * np.linalg.norm(Uref), k
    assert infos[10].iterations == 0 and pairs[11] == pairs[10]


@pytest.mark.parametrize("rb,cb", [(256, 256), (256, 512), (1024, 256), (1024, 512)])
def test_batched_every_workgroup_size(gpu_lib, batch, rb, cb):
    systems, (per, rods, pairs, arrays) = batch
    g, U, infos, used = _run(gpu_lib, systems, arrays, rods, pairs, rb, cb)
    assert used == (rb, cb)
    assert all(i.status == gpu_lib.OK and i.residual <= 1e-8 for i in infos)
    g2, U2, infos2, _ = _run(gpu_lib, systems, arrays, rods, pairs, rb, cb)
    assert np.array_equal(U, U2) and [i.iterations for i in infos] == [i.iterations for i in infos2]


def test_batched_infeasible_system_does_not_disturb_others(gpu_lib):
    """The middle system is the unrelaxed 300-rod system at volume fraction
    0.08 for which the CPU tests hold an infeasibility certificate (a
    non-negative z with D z = 0 and phi.z < 0): no solver can reach the
    tolerance on it.  It must be reported, and its neighbours must still
    match the oracle."""
    systems = [rodsynth.relaxed_system(400, seed=5, phi=0.05),
               rodsynth.make_system(300, seed=0, phi=0.08, length=(0.5, 1.5), orientation="isotropic"),
               rodsynth.relaxed_system(300, seed=6, phi=0.04)]
    per, rods, pairs, arrays = _batch(systems)
    g, U, infos, _ = _run(gpu_lib, systems, arrays, rods, pairs, max_iter=2000)
    assert infos[0].status == gpu_lib.OK and infos[2].status == gpu_lib.OK
    assert infos[1].status in (gpu_lib.NOT_CONVERGED, gpu_lib.STAGNATED) and infos[1].residual > 1e-8
    if infos[1].status == gpu_lib.NOT_CONVERGED:
        assert infos[1].iterations == 2000
    for k in (0, 2):
        s, d, pr, cs = per[k]
        ref = oracle.bbpgd(d, s.length, s.diam, s.eta, pr, cs, tol=1e-8)
        Uref = oracle.velocity(d, s.length, s.diam, s.eta, pr, cs, ref.gamma, s.force)
        assert np.linalg.norm(U[rods[k]:rods[k + 1]] - Uref) <= 1e-6 * np.linalg.norm(Uref)


def test_batched_system_is_bitwise_the_same_alone(gpu_lib, batch):
    """A system's tiles, partial sums and step lengths depend on that system
    alone (with the workgroup sizes fixed), so its answer in the batch is
    bitwise the answer of a batch holding only it.  (Against rl_solve_lcp it
    agrees to the certificate, not bitwise: the single solve splits the
    step-length sums into other workgroup partials, and BB steps amplify the
    last-bit differences into other iterate paths.)"""
    systems, (per, rods, pairs, arrays) = batch
    g, U, infos, _ = _run(gpu_lib, systems, arrays, rods, pairs, 256, 256)
    for k in (1, 4, 7):
        s1 = [systems[k]]
        p1, r1, q1, a1 = _batch(s1)
        g1, U1, i1, _ = _run(gpu_lib, s1, a1, r1, q1, 256, 256)
        assert np.array_equal(g1, g[pairs[k]:pairs[k + 1]]), k
        assert np.array_equal(U1, U[rods[k]:rods[k + 1]]), k
        assert i1[0].iterations == infos[k].iterations


def test_batched_rejects_cross_system_pairs(gpu_lib, batch):
    systems, (per, rods, pairs, arrays) = batch
    bad = dict(arrays)
    bad["pj"] = arrays["pj"].copy()
    bad["pj"][pairs[1]] = rods[3]     # a constraint of system 1 pointing into system 3
    with pytest.raises(gpu_lib.RodLCPError) as ei:
        _run(gpu_lib, systems, bad, rods, pairs, 256, 256)
    assert ei.value.status == gpu_lib.ERR_ARG


def test_batched_varied_lengths(gpu_lib):
    """Per-rod lengths (the kernels' per-rod mobility path), with the hub
    system (one rod 4 long with 18 incidences on each side) among rods of
    lengths in [0.5, 1.5]: each system matches the oracle."""
    systems = [rodsynth.make_system(300, seed=1, phi=0.04, length=(0.5, 1.5)), rodsynth.cfg_hub(1),
               rodsynth.make_system(500, seed=5, phi=0.05, length=(0.5, 1.5))]
    per, rods, pairs = [], [0], [0]
    cat = {k: [] for k in ("dir", "len", "pi", "pj", "e", "arm", "q", "F")}
    for s in systems:
        d = oracle.directors(s.quat)
        pr = oracle.pairs(s.x, d, s.length, s.box, s.diam, s.cutoff)
        cs = oracle.assemble(s.x, d, s.length, s.box, s.diam, s.eta, s.dt, pr, s.force)
        per.append((s, d, pr, cs))
        for k, v in (("dir", d), ("len", s.length), ("pi", pr.pi + rods[-1]), ("pj", pr.pj + rods[-1]),
                     ("e", cs.e), ("arm", cs.arm), ("q", cs.q), ("F", s.force)):
            cat[k].append(v)
        rods.append(rods[-1] + s.n)
        pairs.append(pairs[-1] + pr.n)
    arr = {k: np.concatenate(v) for k, v in cat.items()}
    with gpu_lib.Solver(box=1.0, tol=1e-8, max_iter=100_000) as slv:
        g, U, infos = slv.solve_lcp_batched(
            np.array(rods), np.array(pairs), _t(arr["dir"]), _t(arr["len"]), _t(arr["pi"], torch.int32),
            _t(arr["pj"], torch.int32), _t(arr["e"]), _t(arr["arm"]), _t(arr["q"]), F=_t(arr["F"]))
    g, U = g.cpu().numpy(), U.cpu().numpy()
    for k, (s, d, pr, cs) in enumerate(per):
        assert infos[k].status == gpu_lib.OK and infos[k].residual <= 1e-8, (k, infos[k])
        gk, Uk = g[pairs[k]:pairs[k + 1]], U[rods[k]:rods[k + 1]]
        w = oracle.apply_Mc(d, s.length, s.diam, s.eta, pr, cs, gk)
        assert np.abs(np.minimum(gk, w)).max(initial=0.0) <= 1e-8 + 1e-12 * np.abs(cs.q).max(initial=1.0)
        ref = oracle.bbpgd(d, s.length, s.diam, s.eta, pr, cs, tol=1e-8)
        Uref = oracle.velocity(d, s.length, s.diam, s.eta, pr, cs, ref.gamma, s.force)
        assert np.linalg.norm(Uk - Uref) <= 1e-6 * np.linalg.norm(Uref), k
