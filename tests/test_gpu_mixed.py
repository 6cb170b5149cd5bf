"""Parity of the mixed-precision solve (RL_FP32_MIXED: single-precision BB
iteration on a correction to an FP64 iterate, FP64 dot products, residual and
refresh products) with the FP64 oracle.  The bar is the FP64 one: residual
<= 1e-8 certified by the oracle's own operator, and U within 1e-6 of the
oracle's U.  The error of each result against the oracle is printed."""
import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _length(s):
    return s.uniform_length if s.uniform_length is not None else s.length


def _gpu_length(s):
    return s.uniform_length if s.uniform_length is not None else _t(s.length)


def _setup(s):
    d = oracle.directors(s.quat)
    pr = oracle.pairs(s.x, d, _length(s), s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, _length(s), s.box, s.diam, s.eta, s.dt, pr, s.force)
    return d, pr, cs


def _solve(rl, s, d, pr, cs, precision, **kw):
    with rl.Solver(box=s.box, diam=s.diam, cutoff=s.cutoff, eta=s.eta, dt=s.dt, tol=1e-8,
                   precision=precision, **kw) as slv:
        g, U, info = slv.solve_lcp(_t(d), _gpu_length(s), _t(pr.pi, torch.int32), _t(pr.pj, torch.int32),
                                   _t(cs.e), _t(cs.arm), _t(cs.q), F=_t(s.force))
    return g.cpu().numpy(), U.cpu().numpy(), info


@pytest.mark.parametrize("which", ["small", "lengths", "dense10k", "hub", "phi08"])
def test_mixed_matches_oracle(gpu_lib, which):
    """"phi08": a relaxed isotropic suspension at 12 constraints per rod
    (the FP32 rod kernel's dense form, eight lanes per rod with three rounds
    of records each, and rods with more than the 24 records a side that
    they hold)."""
    s = {"small": lambda: rodsynth.cfg_small(0), "hub": lambda: rodsynth.cfg_hub(1),
         "lengths": lambda: rodsynth.make_system(1000, seed=1, phi=0.04, length=(0.5, 1.5)),
         "dense10k": lambda: rodsynth.cfg_paper_scale(0, n=10_000),
         "phi08": lambda: rodsynth.relaxed_system(1500, seed=3, phi=0.08, length=(0.5, 1.5))}[which]()
    d, pr, cs = _setup(s)
    if which == "phi08":
        assert pr.n > 8 * s.n and np.bincount(pr.pi, minlength=s.n).max() > 24
    ref = oracle.bbpgd(d, _length(s), s.diam, s.eta, pr, cs, tol=1e-8)
    Uref = oracle.velocity(d, _length(s), s.diam, s.eta, pr, cs, ref.gamma, s.force)
    g, U, info = _solve(gpu_lib, s, d, pr, cs, gpu_lib.FP32_MIXED)
    assert info.status == gpu_lib.OK and info.residual <= 1e-8
    w = oracle.apply_Mc(d, _length(s), s.diam, s.eta, pr, cs, g)
    cert = float(np.abs(np.minimum(g, w)).max())
    uerr = float(np.linalg.norm(U - Uref) / np.linalg.norm(Uref))
    print(f"\nmixed[{which}]: iterations {info.iterations} (oracle {ref.iterations}), FP64 refreshes "
          f"{info.fp64_refreshes}, oracle-certified residual {cert:.2e}, U rel err vs oracle {uerr:.2e}, "
          f"max |gamma - gamma_oracle| {np.abs(g - ref.gamma).max():.2e}")
    assert g.min() >= 0 and cert <= 1e-8 + 1e-12 * np.abs(cs.q).max()
    assert uerr <= 1e-6
    assert info.fp64_refreshes >= 2


def test_mixed_step_and_status(gpu_lib):
    s = rodsynth.cfg_small(4)
    r = oracle.step_solve(s)
    x, q = _t(s.x), _t(s.quat)
    with gpu_lib.Solver(box=s.box, tol=1e-8, precision=gpu_lib.FP32_MIXED) as slv:
        U, info, npairs = slv.step(x, q, 1.0, F=_t(s.force))
    assert npairs == r.pairs.n and info.status == gpu_lib.OK and info.residual <= 1e-8
    U = U.cpu().numpy()
    assert np.linalg.norm(U - r.U) <= 1e-6 * np.linalg.norm(r.U)
    d, pr, cs = _setup(s)
    g, U2, info2 = _solve(gpu_lib, s, d, pr, cs, gpu_lib.FP32_MIXED, max_iter=3)
    assert info2.status == gpu_lib.NOT_CONVERGED and info2.iterations == 3 and info2.residual > 1e-8


def test_mixed_reports_infeasible(gpu_lib):
    s = rodsynth.make_system(900, seed=4, phi=0.08, length=(0.5, 1.5))
    d, pr, cs = _setup(s)
    g, U, info = _solve(gpu_lib, s, d, pr, cs, gpu_lib.FP32_MIXED, max_iter=3000)
    assert info.status == gpu_lib.NOT_CONVERGED and info.residual > 1.0
