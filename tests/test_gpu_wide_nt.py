"""GPU parity for windows of 33..64 frames: the wide Gram (tiles split over the waves of a
block, all three precision modes), the 64-frame eigensolver (one LDS copy of the matrix,
register-staged set-up) and the 128 x 128 back-projection operand, against the FP64 oracle.
Odd and even frame counts at both ends of the class, the single steps (1)-(2), full solves
with the Haar and Daubechies transforms, and a batch of two window lengths of the class."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

MODE_TOL = {"fp64": (1e-5, 1e-4), "fp32": (1e-4, 1e-4), "bf16x3": (1e-3, 1e-3)}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.complex64)).cuda()


def _rel(g, want):
    g = g.detach().cpu().numpy().astype(np.complex128) if hasattr(g, "cpu") else np.asarray(g)
    return float(np.linalg.norm(g - want) / max(np.linalg.norm(want), 1e-300))


def _load(h, p, **kw):
    t = pls.to_device(p)
    args = dict(lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=0)
    args.update(kw)
    return h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], **args)


@pytest.mark.parametrize("nt", [33, 48, 64])
@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x3"])
def test_op_svt_wide(nt, mode):
    tol_op, _ = MODE_TOL[mode]
    p = synth.small(nx=16, ny=16, nz=4, nt=nt, nc=1, accel=3, rank=4, nblobs=3, seed=100 + nt,
                    levels=2)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, gram_mode=mode) as h:
        _load(h, p)
        Cm = oracle.EH(p.kspace, p.mask, p.sens).astype(np.complex64).astype(np.complex128)
        Lg, sig = h.op_svt(_dev(Cm))
    Lw, sw, _, _ = oracle.svt(oracle.cas(Cm), p.lambda_L)
    e = _rel(Lg, oracle.uncas(Lw, p.shape))
    print(f"nt={nt} {mode}: op_svt rel L2 {e:.2e}")
    assert e < tol_op, e
    assert len(sig) == nt
    np.testing.assert_allclose(sig, sw, rtol=tol_op, atol=tol_op * sw[0])


@pytest.mark.parametrize("nt,mode", [(40, "fp64"), (64, "fp32"), (48, "bf16x3")])
def test_solve_wide(nt, mode):
    _, tol = MODE_TOL[mode]
    p = synth.small(nx=16, ny=32, nz=4, nt=nt, nc=2, accel=3, rank=4, nblobs=3, seed=110 + nt,
                    levels=2)
    K = 6
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, gram_mode=mode) as h:
        out, st = _load(h, p, max_iter=K, check_every=3)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=2,
                     iters=K)
    for k in ("L", "S", "X", "M"):
        e = _rel(out[k], r[k])
        print(f"nt={nt} {mode} {k}: rel L2 {e:.2e}")
        assert e < tol, (k, e)
    assert st["iters"] == K
    assert len(st["sigma"]) == nt
    np.testing.assert_allclose(st["sigma"], r["sigma"][-1], rtol=tol,
                               atol=tol * r["sigma"][-1][0])
    assert st["nuclear_norm"] == pytest.approx(r["nuclear"][-1], rel=tol)


def test_solve_wide_daubechies():
    p = synth.small(nx=16, ny=16, nz=8, nt=36, nc=1, accel=3, rank=3, nblobs=3, seed=120,
                    prior=False, lambda_S=0.02)
    K = 5
    t = pls.to_device(p)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, transform="db4") as h:
        out, _ = h.solve(t["kspace"], t["mask"], t["sens"], None, lambda_L=p.lambda_L,
                         lambda_S=p.lambda_S, max_iter=K, check_every=5)
    r = oracle.solve(p.kspace, p.mask, p.sens, None, p.lambda_L, p.lambda_S, levels=2, iters=K,
                     transform="db4")
    for k in ("L", "S", "M"):
        e = _rel(out[k], r[k])
        assert e < 1e-4, (k, e)


def test_batch_of_wide_windows_matches_each_alone():
    ps = [synth.small(nx=16, ny=16, nz=4, nt=nt, nc=nc, accel=3, rank=3, nblobs=3, seed=130 + nt,
                      levels=2) for nt, nc in ((40, 1), (57, 2))]
    prm = dict(max_iter=4, check_every=2)
    alone = []
    for p in ps:
        with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2) as h:
            o, _ = _load(h, p, **prm)
            alone.append(o)
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2) for p in ps]
    try:
        with pls.Batch(hs) as b:
            outs, _ = b.solve([pls.to_device(p) for p in ps],
                              [pls.make_params(lambda_L=p.lambda_L, lambda_S=p.lambda_S, **prm)
                               for p in ps])
    finally:
        for h in hs:
            h.close()
    for i, (o, a) in enumerate(zip(outs, alone)):
        for k in ("L", "S", "X", "M"):
            assert torch.equal(o[k], a[k]), (i, k)
