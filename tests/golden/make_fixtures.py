"""Write sampled FP64-oracle results of the full-size workloads for the GPU parity tests.

    python tests/golden/make_fixtures.py c2     # 128x128x16 x 24, 100 iterations
    python tests/golden/make_fixtures.py c3     # 192x192x32 x 30 x 8 coils, 30 iterations

Calls only oracle/ (and the seeded generators in synth/).  The full arrays are too large to
store, so each fixture keeps the oracle's value at a fixed pseudo-random sample of voxels
for L, S and M, the full-array norms, the final singular values and statistics.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

ITERS = {"c2": (2, 100), "c3": (3, 30)}
NSAMP = 4096


def sample_index(shape, n, seed=5150):
    rng = np.random.default_rng(seed)
    total = int(np.prod(shape))
    return np.sort(rng.choice(total, size=min(n, total), replace=False))


def main(name):
    cfg, iters = ITERS[name]
    t0 = time.time()
    p = synth.config(cfg)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=2,
                     iters=iters)
    idx = sample_index(p.shape, NSAMP)
    out = dict(config=cfg, iters=iters, idx=idx,
               L=r["L"].reshape(-1)[idx], S=r["S"].reshape(-1)[idx], M=r["M"].reshape(-1)[idx],
               norm_L=np.linalg.norm(r["L"]), norm_S=np.linalg.norm(r["S"]),
               norm_M=np.linalg.norm(r["M"]), norm_X=np.linalg.norm(r["X"]),
               sigma=r["sigma"][-1], resid=r["resid"][-1], nuclear=r["nuclear"][-1],
               rel_change=r["rel_change"][-1])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle_samples.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    for a in sys.argv[1:] or ["c2"]:
        main(a)
