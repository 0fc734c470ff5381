"""prior_ls_svt_noalloc, the allocation-free form of steps (1)-(2) (the singular-value soft
threshold and the singular-value prior of Algorithm 1), against the handle entry point
prior_ls_op_svt on the same Casorati matrices and against the FP64 oracle: two calls in a
row on one GPU, the second with fewer voxels and frames, so the second reuses the static
scratch the first left behind."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

TOL_OP = 1e-5

# (geometry, Gram mode, lambda_p): the first call is the larger one
CALLS = [(dict(nx=32, ny=48, nz=8, nt=24, nc=2, seed=71), "fp32", 0.5),
         (dict(nx=16, ny=16, nz=4, nt=6, nc=1, seed=72), "fp32", 0.0)]


def rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def reference(geom, mode, lam_p):
    """The handle path: prior_ls_op_svt after a zero-iteration solve with the same lambdas."""
    g = dict(geom)
    seed = g.pop("seed")
    p = synth.small(**g, accel=3, rank=2, nblobs=3, seed=seed, levels=1)
    rng = np.random.default_rng(seed)
    prev = np.sort(rng.uniform(0.5, 3.0, p.nt))[::-1].copy()
    Cm = oracle.EH(p.kspace, p.mask, p.sens).astype(np.complex64)
    Cd = torch.from_numpy(Cm).cuda()
    t = pls.to_device(p)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1, gram_mode=mode) as h:
        h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], lambda_L=p.lambda_L,
                lambda_S=p.lambda_S, lambda_p=lam_p, sigma_prev=prev if lam_p > 0 else None,
                max_iter=0, outputs=())
        L1, s1 = h.op_svt(Cd)
    torch.cuda.synchronize()
    return p, prev, Cm, Cd, L1, np.asarray(s1)


def test_noalloc_equals_op_svt_on_two_calls_in_a_row():
    refs = [reference(*c) for c in CALLS]
    for (geom, mode, lam_p), (p, prev, Cm, Cd, L1, s1) in zip(CALLS, refs):
        prev_d = torch.from_numpy(prev).cuda() if lam_p > 0 else None
        L2, s2 = pls.svt_noalloc(Cd, lambda_L=p.lambda_L, lambda_p=lam_p, sigma_prev=prev_d,
                                 gram_mode=mode)
        torch.cuda.synchronize()
        e = rel(L2.cpu().numpy(), L1.cpu().numpy())
        assert e < TOL_OP, (geom, e)
        np.testing.assert_allclose(s2.cpu().numpy(), s1, rtol=1e-6, atol=1e-7 * s1[0])
        # and the FP64 oracle's SVD route
        Lw, sw, _, _ = oracle.svt(oracle.cas(Cm.astype(np.complex128)), p.lambda_L, True, lam_p,
                                  prev if lam_p > 0 else None)
        e = rel(L2.cpu().numpy(), oracle.uncas(Lw, p.shape))
        assert e < TOL_OP, (geom, e)
        np.testing.assert_allclose(s2.cpu().numpy(), sw, rtol=1e-5, atol=1e-6 * sw[0])


def test_noalloc_rejects_bad_sizes():
    C = torch.zeros((33, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(pls.PriorLSError) as e:
        pls.svt_noalloc(C)
    assert e.value.status == pls.ESHAPE and "32" in str(e.value)
    C = torch.zeros((4, 96), dtype=torch.complex64, device="cuda")    # not a multiple of 64
    with pytest.raises(pls.PriorLSError) as e:
        pls.svt_noalloc(C)
    assert e.value.status == pls.ESHAPE
    C = torch.zeros((4, 128), dtype=torch.complex64, device="cuda")
    with pytest.raises(pls.PriorLSError) as e:
        pls.svt_noalloc(C.cpu(), out=C)                                # host input
    assert e.value.status == pls.EINVAL
    with pytest.raises(pls.PriorLSError) as e:
        pls.svt_noalloc(C, lambda_p=0.5)                               # no sigma_prev
    assert e.value.status == pls.EINVAL
    with pytest.raises(pls.PriorLSError) as e:
        pls.svt_noalloc(C, out=C)                                      # L overlaps C
    assert e.value.status == pls.EINVAL
