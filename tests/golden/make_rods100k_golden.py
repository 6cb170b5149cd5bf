"""Writes rods100k_seed0.json: oracle results for the 100,000-rod nematic
suspension (volume fraction 0.05, vMF kappa 20, seed 0) used by the
full-size GPU parity test.  Calls only the CPU oracle; takes about a minute.

Stored: the pair count, the number of pairs flagged near the threshold, a
SHA-256 of the canonical pair list (pi, pj, img as little-endian int32), the
oracle's BBPGD iterations and residual at tol 1e-8, and U = M(D gamma + F)
for 500 rods drawn with numpy seed 1234, with the 2-norm of U over all rods.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import rodsynth  # noqa: E402


def pair_hash(pi, pj, img):
    h = hashlib.sha256()
    for a in (pi, pj, img):
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def main():
    s = rodsynth.cfg_paper_scale(0)
    t0 = time.time()
    r = oracle.step_solve(s, tol=1e-8, max_iter=200_000, pair_method="cells")
    sample = np.sort(np.random.default_rng(1234).choice(s.n, 500, replace=False))
    out = {
        "system": "rodsynth.cfg_paper_scale(0): 100000 rods, L=1, d=0.025, phi=0.05, vMF kappa=20, seed 0",
        "n_pairs": int(r.pairs.n),
        "n_flagged_cutoff": int(np.count_nonzero(r.pairs.flags & oracle.FLAG_CUTOFF)),
        "pair_sha256": pair_hash(r.pairs.pi, r.pairs.pj, r.pairs.img),
        "oracle_iterations": int(r.solve.iterations),
        "oracle_residual": float(r.solve.residual),
        "oracle_status": int(r.solve.status),
        "U_norm": float(np.linalg.norm(r.U)),
        "sample_rods": sample.tolist(),
        "U_sample": r.U[sample].tolist(),
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "rods100k_seed0.json"), "w") as f:
        json.dump(out, f, indent=0)
    print({k: v for k, v in out.items() if k not in ("sample_rods", "U_sample")})


if __name__ == "__main__":
    main()
