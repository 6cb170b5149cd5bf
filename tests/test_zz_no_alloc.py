"""The allocation-free solve (rl_solve_lcp_noalloc) against rl_solve_lcp.

Same kernels, same problem: the result must be bitwise that of
rl_solve_lcp, over two calls in a row on one handle (the second smaller, so
it reuses the scratch array's start with the first call's contents still in
it), and both must match the oracle.  A problem beyond the scratch array is
refused with an error."""
import numpy as np
import pytest

import oracle
import rodsynth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _problem(s):
    d = oracle.directors(s.quat)
    L = s.uniform_length if s.uniform_length is not None else s.length
    pr = oracle.pairs(s.x, d, L, s.box, s.diam, s.cutoff)
    cs = oracle.assemble(s.x, d, L, s.box, s.diam, s.eta, s.dt, pr, s.force)
    return d, L, pr, cs


def _args(s, d, L, pr, cs):
    length = L if np.isscalar(L) else _t(L)
    return (_t(d), length, _t(pr.pi, torch.int32), _t(pr.pj, torch.int32), _t(cs.e), _t(cs.arm), _t(cs.q))


def test_noalloc_matches_solve_lcp_twice(gpu_lib):
    big = rodsynth.relaxed_system(500, seed=2, phi=0.06, length=(0.5, 1.5))
    small = rodsynth.make_system(300, seed=4, box=3.0)
    probs = [(s, *_problem(s)) for s in (big, small)]
    assert probs[1][0].n < probs[0][0].n and probs[1][3].n < probs[0][3].n
    with gpu_lib.Solver(box=big.box, tol=1e-8) as na, gpu_lib.Solver(box=big.box, tol=1e-8) as ref:
        for s, d, L, pr, cs in probs:
            na.set_params(box=s.box)
            ref.set_params(box=s.box)
            args = _args(s, d, L, pr, cs)
            F = _t(s.force)
            g1 = torch.zeros(pr.n, dtype=torch.float64, device="cuda")
            U1 = torch.empty((s.n, 6), dtype=torch.float64, device="cuda")
            g1, U1, i1 = na.solve_lcp_noalloc(*args, g1, U1, F=F)
            g2, U2, i2 = ref.solve_lcp(*args, F=F)
            assert i1.status == gpu_lib.OK and i1.residual <= 1e-8
            assert i1.iterations == i2.iterations
            assert torch.equal(g1, g2) and torch.equal(U1, U2)
            r = oracle.bbpgd(d, L, s.diam, s.eta, pr, cs, tol=1e-8)
            Uo = oracle.velocity(d, L, s.diam, s.eta, pr, cs, r.gamma, s.force)
            Un = U1.cpu().numpy()
            assert np.linalg.norm(Un - Uo) <= 1e-6 * np.linalg.norm(Uo)


def test_noalloc_refuses_a_problem_beyond_the_scratch_array(gpu_lib):
    nc = 700_000   # 152 bytes each: more than the 96 MiB array
    n = 2
    dev = "cuda"
    d = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    d[:, 2] = 1.0
    pi = torch.zeros(nc, dtype=torch.int32, device=dev)
    pj = torch.ones(nc, dtype=torch.int32, device=dev)
    e = torch.zeros((nc, 3), dtype=torch.float64, device=dev)
    e[:, 0] = 1.0
    arm = torch.zeros((nc, 2), dtype=torch.float64, device=dev)
    q = torch.ones(nc, dtype=torch.float64, device=dev)
    g = torch.zeros(nc, dtype=torch.float64, device=dev)
    U = torch.empty((n, 6), dtype=torch.float64, device=dev)
    with gpu_lib.Solver(box=10.0, tol=1e-8) as na:
        with pytest.raises(gpu_lib.RodLCPError) as ei:
            na.solve_lcp_noalloc(d, 1.0, pi, pj, e, arm, q, g, U)
        assert ei.value.status == gpu_lib.ERR_ARG
        assert "scratch" in str(ei.value)
    assert torch.count_nonzero(g) == 0
