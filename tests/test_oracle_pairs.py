"""Pins of the oracle's near-contact pair search (no GPU): the brute-force
enumeration is the definition; the cell list must reproduce it exactly; small
hand-built periodic cases fix the image convention."""
import numpy as np
import pytest

import oracle
import rodsynth


def _both(sysm, L=None):
    d = oracle.directors(sysm.quat)
    L = sysm.uniform_length if L is None else L
    L = sysm.length if L is None else L
    a = oracle.pairs(sysm.x, d, L, sysm.box, sysm.diam, sysm.cutoff, method="brute")
    b = oracle.pairs(sysm.x, d, L, sysm.box, sysm.diam, sysm.cutoff, method="cells")
    return d, a, b


def _same(a, b):
    return (np.array_equal(a.pi, b.pi) and np.array_equal(a.pj, b.pj)
            and np.array_equal(a.img, b.img) and np.array_equal(a.flags, b.flags))


@pytest.mark.parametrize("seed", [0, 1])
def test_cells_equal_brute_small_config(seed):
    s = rodsynth.cfg_small(seed)
    d, a, b = _both(s)
    assert a.n > 500 and _same(a, b)


def test_cells_equal_brute_varied_lengths_dense():
    s = rodsynth.make_system(600, seed=3, phi=0.08, length=(0.5, 1.5))
    d, a, b = _both(s)
    assert a.n > 0 and _same(a, b)


@pytest.mark.parametrize("n,phi", [(200, 0.1), (120, 0.02), (60, 0.1)])
def test_cells_equal_brute_small_boxes(n, phi):
    # boxes comparable to or smaller than the rod length: several images of one
    # neighbour, and rods touching their own images
    s = rodsynth.make_system(n, seed=11, phi=phi)
    d, a, b = _both(s)
    assert _same(a, b)
    if s.box < 1.075:
        assert np.any(a.pi == a.pj)


def test_pairs_are_canonical_and_below_cutoff():
    s = rodsynth.cfg_small(2)
    d, a, _ = _both(s)
    key = a.pi.astype(np.int64) * (1 << 40) + a.pj.astype(np.int64) * (1 << 12) + a.img
    assert np.all(np.diff(key) > 0)
    assert np.all(a.pi <= a.pj)
    imgs = oracle.img_unpack(a.img)
    self_ = a.pi == a.pj
    # self contacts only with a lexicographically positive shift
    for n3 in imgs[self_]:
        nz = n3[np.nonzero(n3)[0][0]]
        assert nz > 0
    for k in range(0, a.n, 37):
        i, j = a.pi[k], a.pj[k]
        xj = s.x[j] + imgs[k] * s.box
        _, _, dist, _, _ = oracle.closest(s.x[i], d[i], 1.0, xj, d[j], 1.0)
        assert dist - s.diam < s.cutoff


def test_completeness_against_all_images_numpy():
    """Every pair with gap < cutoff under any shift appears (independent scan
    with the closest-point routine over a generous image range)."""
    s = rodsynth.make_system(40, seed=5, phi=0.1)
    d = oracle.directors(s.quat)
    got = oracle.pairs(s.x, d, 1.0, s.box, s.diam, s.cutoff, method="brute")
    gotset = set(zip(got.pi.tolist(), got.pj.tolist(), got.img.tolist()))
    want = set()
    m = 4
    for i in range(s.n):
        for j in range(i, s.n):
            for nx in range(-m, m + 1):
                for ny in range(-m, m + 1):
                    for nz in range(-m, m + 1):
                        n3 = (nx, ny, nz)
                        if i == j and not (n3 > (0, 0, 0)):
                            continue
                        xj = s.x[j] + np.array(n3) * s.box
                        if np.linalg.norm(s.x[i] - xj) > 1.2:
                            continue
                        _, _, dist, _, _ = oracle.closest(s.x[i], d[i], 1.0, xj, d[j], 1.0)
                        if dist - s.diam < s.cutoff:
                            want.add((i, j, oracle.img_pack(*n3)))
    assert gotset == want


def _quat_for(dvec):
    dvec = np.asarray(dvec, float) / np.linalg.norm(dvec)
    z = np.array([0.0, 0.0, 1.0])
    v = np.cross(z, dvec)
    q = np.r_[1.0 + dvec[2], v]
    return q / np.linalg.norm(q)


def test_pair_across_periodic_boundary():
    box = 4.0
    x = np.array([[0.02, 2.0, 2.0], [3.99, 2.0, 2.03]])
    quat = np.stack([_quat_for([0, 1, 0]), _quat_for([0, 0, 1])])
    d = oracle.directors(quat)
    assert np.allclose(d, [[0, 1, 0], [0, 0, 1]], atol=1e-15)
    p = oracle.pairs(x, d, 1.0, box, 0.025, 0.05, method="brute")
    assert p.n == 1 and p.pi[0] == 0 and p.pj[0] == 1
    # rod 1 is moved by -box along x to reach rod 0
    assert tuple(oracle.img_unpack(p.img)[0]) == (-1, 0, 0)
    pc = oracle.pairs(x, d, 1.0, box, 0.025, 0.05, method="cells")
    assert _same(p, pc)


def test_self_image_contact():
    # a rod of length 1 lying along x in a box of side 1.04 touches its own image
    box = 1.04
    x = np.array([[0.5, 0.5, 0.5]])
    quat = _quat_for([1, 0, 0])[None]
    d = oracle.directors(quat)
    p = oracle.pairs(x, d, 1.0, box, 0.025, 0.05, method="brute")
    assert p.n == 1 and p.pi[0] == 0 and p.pj[0] == 0
    assert tuple(oracle.img_unpack(p.img)[0]) == (1, 0, 0)
    assert p.flags[0] & oracle.FLAG_PARALLEL


@pytest.mark.parametrize("seed", [0, 1])
def test_hub_pairs(seed):
    """A rod of length 4 crossed by 36 rods of length 1 (axes 0.005-0.06
    apart, closer than diam + cutoff = 0.075): every crosser touches the long
    rod, the cell list (two cells per side of the box of 10) finds the same
    pairs as the brute force, and the long rod's lists hold 18 contacts on
    each side.  The surface gap of each hub pair is within the tilt's reach of
    the axis offset minus the diameter."""
    s = rodsynth.cfg_hub(seed)
    d, a, b = _both(s)
    assert _same(a, b)
    hub = 18
    assert np.sum(a.pi == hub) == 18 and np.sum(a.pj == hub) == 18
    cs = oracle.assemble(s.x, d, s.length, s.box, s.diam, s.eta, s.dt, a, s.force)
    for c in np.flatnonzero((a.pi == hub) | (a.pj == hub)):
        other = a.pj[c] if a.pi[c] == hub else a.pi[c]
        off = s.x[other, 2] - s.x[hub, 2]
        # the crosser's axis is tilted by at most 0.05 rad over half a length
        # of 0.5, but it passes the long rod near its own centre
        assert off - s.diam - 0.03 <= cs.phi[c] <= off - s.diam + 1e-12
