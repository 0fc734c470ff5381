"""The stopping rule of Section 3 (relative change of the solution below tol) on the GPU
against the FP64 oracle: the iteration at which a tol > 0 solve stops, and the iterate it
stops with.

The library tests the rule at the end of every chunk of check_every iterations, the oracle
after every iteration.  So the expected stop is the first multiple m of check_every with
rel_change(m) < tol in the oracle's history (or max_iter).  tol is placed between two
consecutive checked values of that history with a margin far above the FP32 path's error in
the relative change, so both sides take the same decision.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

MAX_IT = 30


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def problem():
    return synth.small(nx=32, ny=48, nz=8, nt=12, nc=3, accel=4, rank=3, nblobs=4, seed=4242,
                       levels=2)


@pytest.fixture(scope="module")
def history():
    p = problem()
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=2,
                     iters=MAX_IT)
    return p, r["rel_change"]


def pick_tol(rc, ce, target):
    """A tol that the checked history crosses first at the check iteration nearest `target`,
    with every earlier checked value at least 2% above it and the crossing value at least 2%
    below; None if the history has no such crossing."""
    checks = list(range(ce, MAX_IT + 1, ce))
    order = sorted(checks, key=lambda m: abs(m - target))
    for m in order:
        earlier = [rc[k - 1] for k in checks if k < m]
        hi = min(earlier) if earlier else math.inf
        lo = rc[m - 1]
        if hi > 1.05 * lo:
            tol = math.sqrt(hi * lo) if earlier else 1.5 * lo
            if hi > 1.02 * tol and lo < tol / 1.02:
                return tol, m
    return None


@pytest.mark.parametrize("ce,target", [(1, 8), (3, 12), (4, 9)])
def test_stopping_iteration_matches_oracle(history, ce, target):
    p, rc = history
    got = pick_tol(rc, ce, target)
    assert got is not None, "no clean crossing in the oracle's history"
    tol, m = got
    t = pls.to_device(p)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2) as h:
        out, st = h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], lambda_L=p.lambda_L,
                          lambda_S=p.lambda_S, max_iter=MAX_IT, tol=tol, check_every=ce)
    assert st["iters"] == m, (st["iters"], m, tol)
    assert st["converged"] == 1
    assert st["rel_change"] < tol
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=2,
                     iters=m)
    if ce == 1:
        # the oracle's own stopping rule stops at the same iteration
        ro = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S,
                          levels=2, iters=MAX_IT, tol=tol)
        assert ro["iters"] == m
    for k in ("L", "S", "X", "M"):
        e = rel(out[k].cpu().numpy().astype(np.complex128), r[k])
        assert e < 1e-4, (k, e)
    assert st["rel_change"] == pytest.approx(rc[m - 1], rel=1e-3)
    assert st["objective"] == pytest.approx(r["objective"][-1], rel=1e-4)


def test_no_stop_above_tolerance(history):
    # a tol below every value of the history: the solve runs max_iter iterations, in chunks
    # whose last one is shorter than check_every
    p, rc = history
    tol = 0.5 * float(np.min(rc))
    t = pls.to_device(p)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2) as h:
        out, st = h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], lambda_L=p.lambda_L,
                          lambda_S=p.lambda_S, max_iter=MAX_IT - 1, tol=tol, check_every=4)
    assert st["iters"] == MAX_IT - 1
    assert st["converged"] == 0
    assert st["rel_change"] == pytest.approx(rc[MAX_IT - 2], rel=1e-3)
