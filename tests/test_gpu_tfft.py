"""GPU parity of the temporal-Fourier sparsifying transform (PRIOR_LS_T_TFFT): the fused
forward-DFT / shrink / inverse-DFT kernels against the FP64 oracle.  Window lengths whose
DFT factors into radices 2, 3, 4, 5 and 7 take an in-register FFT per voxel; the others take
the dense product on MFMA (both operand sizes: nt <= 16 and 16 < nt <= 32).  With and
without prior weights, as one step, as a full solve and through the sliding-window
recursion."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

TOL, TOL_OP = 1e-4, 1e-5
CASES = {
    "3d_16x16x4_nt6_nc2": dict(nx=16, ny=16, nz=4, nt=6, nc=2, seed=51),
    "3d_24x32x8_nt17_nc3": dict(nx=24, ny=32, nz=8, nt=17, nc=3, seed=52),
    "2d_32x32_nt30_nc1": dict(nx=32, ny=32, nz=1, nt=30, nc=1, seed=53),
    "3d_16x48x4_nt16_nc2": dict(nx=16, ny=48, nz=4, nt=16, nc=2, seed=54),
}


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _rel(g, want):
    g = g.cpu().numpy().astype(np.complex128)
    return float(np.linalg.norm(g - want) / max(np.linalg.norm(want), 1e-300))


def _problem(kw, weights):
    p = synth.small(**kw, prior=False, lambda_S=0.02)
    w = None
    if weights:
        rng = np.random.default_rng(kw["seed"] + 1000)
        w = np.where(rng.random((p.nt, p.nz, p.ny, p.nx)) < 0.2, 255, 0).astype(np.uint8)
    return p, w


def _args(p, w):
    sens = None if p.sens is None else _dev(p.sens, torch.complex64)
    return (_dev(p.kspace, torch.complex64), _dev(p.mask, torch.uint8), sens,
            None if w is None else _dev(w, torch.uint8))


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("weights", [False, True])
def test_tfft_sparse_step(name, weights):
    p, w = _problem(CASES[name], weights)
    rng = np.random.default_rng(7)
    shp = (p.nt, p.nz, p.ny, p.nx)
    Xm = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.05
    Lp = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.02
    want, _ = oracle.sparse_step(Xm, Lp, w, p.lambda_S, 0, transform="tfft")
    k, m, s, wd = _args(p, w)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, transform="tfft") as h:
        h.solve(k, m, s, wd, lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=0, outputs=())
        S = h.op_sparse(_dev(Xm, torch.complex64), _dev(Lp, torch.complex64))
    e = _rel(S, want)
    print(f"{name} weights={weights}: op_sparse rel L2 {e:.2e}")
    assert e < TOL_OP


# frame counts of the in-register FFT (radices 2, 3, 4, 5, 7 and their products up to 32)
# and of the MFMA fallback (prime factors 11, 13, 31)
NTS = [2, 5, 7, 9, 12, 14, 21, 25, 27, 28, 32, 11, 26, 31]


@pytest.mark.parametrize("nt", NTS)
def test_tfft_sparse_step_frame_counts(nt):
    p, w = _problem(dict(nx=16, ny=16, nz=1, nt=nt, nc=1, seed=60 + nt), True)
    rng = np.random.default_rng(nt)
    shp = (p.nt, p.nz, p.ny, p.nx)
    Xm = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.05
    Lp = (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.02
    want, _ = oracle.sparse_step(Xm, Lp, w, p.lambda_S, 0, transform="tfft")
    k, m, s, wd = _args(p, w)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, transform="tfft") as h:
        h.solve(k, m, s, wd, lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=0, outputs=())
        S = h.op_sparse(_dev(Xm, torch.complex64), _dev(Lp, torch.complex64))
    e = _rel(S, want)
    print(f"nt={nt}: op_sparse rel L2 {e:.2e}")
    assert e < TOL_OP


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("weights", [False, True])
def test_tfft_solve(name, weights):
    p, w = _problem(CASES[name], weights)
    K = 10
    ref = oracle.solve(p.kspace, p.mask, p.sens, w, p.lambda_L, p.lambda_S, levels=0, iters=K,
                       transform="tfft")
    k, m, s, wd = _args(p, w)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, transform="tfft") as h:
        out, st = h.solve(k, m, s, wd, lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=K,
                          check_every=5)
    for key in ("L", "S", "M"):
        e = _rel(out[key], ref[key])
        print(f"{name} weights={weights} {key}: rel L2 {e:.2e}")
        assert e < TOL, (key, e)
    assert st["l1_weighted"] == pytest.approx(float(ref["l1w"][-1]), rel=1e-3)


def test_tfft_append_chain():
    q = synth.sequence(nx=16, ny=16, nz=4, nt=6, nc=2, accel=3, n_append=2, seed=55,
                       lambda_S=0.02)
    d, m = q.first_window()
    ref = oracle.solve(d, m, q.sens, None, q.lambda_L, q.lambda_S, levels=0, iters=6,
                       transform="tfft")
    refs = [ref]
    for j in range(q.n_append):
        dn, mn = q.frame(j)
        ref, d, m = oracle.append_frame(ref, d, m, q.sens, dn, mn, q.lambda_L, q.lambda_S,
                                        lambda_p=0.3, levels=0, iters=5, transform="tfft")
        refs.append(ref)
    sens = _dev(q.sens, torch.complex64)
    with pls.PriorLS(q.nx, q.ny, q.nz, q.nt, q.nc, transform="tfft") as h:
        d0, m0 = q.first_window()
        outs = [h.solve(_dev(d0, torch.complex64), _dev(m0, torch.uint8), sens,
                        lambda_L=q.lambda_L, lambda_S=q.lambda_S, max_iter=6)[0]]
        for j in range(q.n_append):
            dn, mn = q.frame(j)
            outs.append(h.append(_dev(dn, torch.complex64), _dev(mn, torch.uint8),
                                 lambda_L=q.lambda_L, lambda_S=q.lambda_S, lambda_p=0.3,
                                 max_iter=5)[0])
    for wnd, (o, r) in enumerate(zip(outs, refs)):
        for key in ("L", "S", "M"):
            assert _rel(o[key], r[key]) < TOL, (wnd, key)
