"""Parity of the precision and batching forms at the sizes bench.py times:
the 400,000-rod precision workload and the 256-system batch (1.26M rods).

The oracle cannot run BBPGD on these within a test, but it can certify an
answer with its own operator: gamma >= 0, |min(gamma, Mc gamma + q)| <= tol
(the natural residual of the complementarity problem), and U recomputed by
the oracle from that gamma.  A certified gamma solves the convex QP, and U
is unique for it, so the certificate pins U without a stored reference.  The
constraint geometry is the oracle's own, so the GPU solver sees exactly the
problem the oracle certifies."""
import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _certify(d, length, s, pr, cs, g, U, tag):
    """Oracle certificate of one solution; returns the residual and U error."""
    w = oracle.apply_Mc(d, length, s.diam, s.eta, pr, cs, g)
    cert = float(np.abs(np.minimum(g, w)).max(initial=0.0))
    Uo = oracle.velocity(d, length, s.diam, s.eta, pr, cs, g, s.force)
    uerr = float(np.linalg.norm(U - Uo) / max(np.linalg.norm(Uo), 1e-300))
    assert g.min(initial=0.0) >= 0.0, tag
    # the two sides round differently: 1e-12 relative to |q| on top of tol
    assert cert <= 1e-8 + 1e-12 * np.abs(cs.q).max(initial=1.0), (tag, cert)
    assert uerr <= 1e-12, (tag, uerr)
    return cert, uerr


def test_precision_workload_fullsize(gpu_lib):
    """400k rods, lengths in [0.5, 1.5]: the FP32-mixed and the FP64 solve are
    each certified by the oracle, and their velocities agree to 1e-6."""
    s = rodsynth.cfg_precision(0)
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, s.length, s.box, s.diam, s.cutoff, method="cells")
    cs = oracle.assemble(s.x, d, s.length, s.box, s.diam, s.eta, s.dt, pr, s.force)
    out = {}
    for prec in (gpu_lib.FP64, gpu_lib.FP32_MIXED):
        with gpu_lib.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                            max_iter=200_000, precision=prec) as slv:
            g, U, info = slv.solve_lcp(_t(d), _t(s.length), _t(pr.pi, torch.int32), _t(pr.pj, torch.int32),
                                       _t(cs.e), _t(cs.arm), _t(cs.q), F=_t(s.force))
        assert info.status == gpu_lib.OK and info.residual <= 1e-8, (prec, info)
        g, U = g.cpu().numpy(), U.cpu().numpy()
        cert, uerr = _certify(d, s.length, s, pr, cs, g, U, prec)
        print(f"\nprecision {prec}: {pr.n} constraints, {info.iterations} iterations, "
              f"{info.fp64_refreshes} FP64 refreshes, oracle residual {cert:.2e}, U vs oracle(gamma) {uerr:.2e}")
        out[prec] = U
    a, b = out[gpu_lib.FP64], out[gpu_lib.FP32_MIXED]
    assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)


def test_batched_workload_fullsize(gpu_lib):
    """The 256-system batch in one batched solve, with the tuner choosing the
    workgroups as bench.py lets it: every system certified by the oracle."""
    systems = rodsynth.cfg_batched(0)
    per, rods, pairs = [], [0], [0]
    cat = {k: [] for k in ("dir", "pi", "pj", "e", "arm", "q", "F")}
    for s in systems:
        d = oracle.directors(s.quat)
        pr = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff, method="cells")
        cs = oracle.assemble(s.x, d, 1.0, s.box, s.diam, s.eta, s.dt, pr, s.force)
        per.append((s, d, pr, cs))
        for k, v in (("dir", d), ("pi", pr.pi + rods[-1]), ("pj", pr.pj + rods[-1]), ("e", cs.e),
                     ("arm", cs.arm), ("q", cs.q), ("F", s.force)):
            cat[k].append(v)
        rods.append(rods[-1] + s.n)
        pairs.append(pairs[-1] + pr.n)
    arr = {k: np.concatenate(v) for k, v in cat.items()}
    with gpu_lib.Solver(box=1.0, tol=1e-8, max_iter=400_000) as slv:
        g, U, infos = slv.solve_lcp_batched(
            np.array(rods), np.array(pairs), _t(arr["dir"]), 1.0, _t(arr["pi"], torch.int32),
            _t(arr["pj"], torch.int32), _t(arr["e"]), _t(arr["arm"]), _t(arr["q"]), F=_t(arr["F"]))
    g, U = g.cpu().numpy(), U.cpu().numpy()
    worst = 0.0
    for k, (s, d, pr, cs) in enumerate(per):
        info = infos[k]
        assert info.status == gpu_lib.OK and info.residual <= 1e-8, (k, info)
        cert, _ = _certify(d, 1.0, s, pr, cs, g[pairs[k]:pairs[k + 1]], U[rods[k]:rods[k + 1]], k)
        worst = max(worst, cert)
    print(f"\nbatch: {len(systems)} systems, {rods[-1]} rods, {pairs[-1]} constraints, most iterations "
          f"{max(i.iterations for i in infos)}, worst oracle residual {worst:.2e}")
