"""Relaxed (overlap-free) starts of the dense workloads (CPU).

The precision workload (volume fraction 0.08, lengths in [0.5, 1.5]) and the
batch (fractions up to 0.1) start from placements whose overlaps have been
removed, as the paper does before its timed runs.  These tests check the
generator's output with the oracle's own geometry: every gap (all pairs and
periodic images, by brute force where the box is small) is non-negative, so
the linearised step always has a solution, and the oracle's BBPGD finds it.
"""
import numpy as np
import pytest

import oracle
import rodsynth


def _gaps(s, method="auto"):
    d = oracle.directors(s.quat)
    L = s.uniform_length if s.uniform_length is not None else s.length
    pr = oracle.pairs(s.x, d, L, s.box, s.diam, s.cutoff, method=method)
    cs = oracle.assemble(s.x, d, L, s.box, s.diam, s.eta, s.dt, pr, s.force)
    return d, L, pr, cs


def _nematic_order(d):
    Q = 1.5 * (d.T @ d) / d.shape[0] - 0.5 * np.eye(3)
    return float(np.linalg.eigvalsh(Q).max())


@pytest.fixture(scope="module")
def dense():
    return rodsynth.relaxed_system(3000, seed=0, phi=0.08, length=(0.5, 1.5))


def test_relaxed_precision_copy_is_overlap_free_and_solvable(dense):
    s = dense
    vol = rodsynth.spherocylinder_volume(s.length, s.diam).sum()
    assert abs(vol / s.box ** 3 - 0.08) < 1e-12
    assert np.all((s.x >= 0.0) & (s.x < s.box))
    assert np.allclose(np.linalg.norm(s.quat, axis=1), 1.0, atol=1e-14)
    d, L, pr, cs = _gaps(s)
    assert pr.n > 10 * s.n          # dense: about 12 near contacts per rod
    assert cs.phi.min() >= 1e-4 - 1e-12
    r = oracle.bbpgd(d, L, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=100_000)
    assert r.status == oracle.OK and r.residual <= 1e-8
    # the relaxation leaves the orientations isotropic
    assert _nematic_order(d) < 0.05


def test_relaxation_is_deterministic(dense):
    again = rodsynth.relaxed_system(3000, seed=0, phi=0.08, length=(0.5, 1.5), threads=1)
    assert np.array_equal(again.x, dense.x) and np.array_equal(again.quat, dense.quat)


@pytest.mark.parametrize("n,seed", [(200, 0), (200, 5), (700, 1)])
def test_relaxed_small_dense_boxes(n, seed):
    """Batch systems at volume fraction 0.1 down to 200 rods (box about 1.0,
    shorter than the rods: many periodic images, including a rod's own)."""
    s = rodsynth.relaxed_system(n, seed=seed, phi=0.1)
    d, L, pr, cs = _gaps(s, method="brute")
    assert cs.phi.min() >= 1e-4 - 1e-12
    r = oracle.bbpgd(d, L, s.diam, s.eta, pr, cs, tol=1e-8, max_iter=200_000)
    assert r.status == oracle.OK and r.residual <= 1e-8


def test_batch_plan_spans_the_stated_ranges():
    counts, phis = rodsynth.batch_plan(0)
    assert counts.shape == (256,) and counts.min() >= 200 and counts.max() <= 20_000
    assert phis.min() >= 0.02 and phis.max() <= 0.1 and phis.max() > 0.095
