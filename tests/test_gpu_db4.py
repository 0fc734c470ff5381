"""GPU parity of the Daubechies-4 sparsifying transform (PRIOR_LS_T_DB4): the three-pass
update (x lines, (y, z) planes with the weighted shrink, x lines) against the FP64 oracle,
as one step for every depth J and several planes (2D and 3D, ragged line tiles, radix-3
lengths), as a full solve with and without prior weights, through the sliding-window
recursion (the support map of the standard decomposition carried to the next window), and
in a batch of problems of different window length and coil count (bit for bit as alone)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

TOL, TOL_OP = 1e-4, 1e-5
# (nx, ny, nz, nt, nc, J): P = ny nz not a multiple of the 32-line tile (16 x 1), radix-3
# lengths (24, 48, 96), every depth, nz = 1 (2D), the largest line (nx = 256) and plane, and
# the 192 x 192 x 32 benchmark volume's plane (6144 points) and line (192)
STEP_CASES = [
    (16, 16, 1, 3, 1, 1), (32, 16, 4, 4, 2, 2), (24, 48, 8, 3, 2, 3), (48, 32, 8, 5, 1, 2),
    (16, 96, 16, 2, 2, 1), (256, 16, 8, 2, 1, 3), (16, 256, 32, 2, 1, 2), (64, 24, 4, 3, 1, 2),
    (32, 32, 14, 3, 1, 1), (16, 192, 32, 2, 1, 2), (192, 16, 8, 2, 1, 3),
]


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _rel(g, want):
    g = g.cpu().numpy().astype(np.complex128) if hasattr(g, "cpu") else np.asarray(g)
    return float(np.linalg.norm(g - want) / max(np.linalg.norm(want), 1e-300))


def _weights(p, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random((p.nt, p.nz, p.ny, p.nx)) < 0.2, 255, 0).astype(np.uint8)


def _args(p, w):
    sens = None if p.sens is None else _dev(p.sens, torch.complex64)
    return (_dev(p.kspace, torch.complex64), _dev(p.mask, torch.uint8), sens,
            None if w is None else _dev(w, torch.uint8))


@pytest.mark.parametrize("case", STEP_CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}_nt{c[3]}_J{c[5]}"
                                                   for c in STEP_CASES])
@pytest.mark.parametrize("weights", [False, True])
def test_db4_sparse_step(case, weights):
    nx, ny, nz, nt, nc, J = case
    p = synth.small(nx=nx, ny=ny, nz=nz, nt=nt, nc=nc, seed=70 + nx + ny + nz, prior=False,
                    lambda_S=0.02)
    w = _weights(p, nx * ny + nz) if weights else None
    rng = np.random.default_rng(nx + 3 * ny + 7 * nz)
    shp = (p.nt, p.nz, p.ny, p.nx)
    Xm = ((rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.05).astype(np.complex64)
    Lp = ((rng.standard_normal(shp) + 1j * rng.standard_normal(shp)) * 0.02).astype(np.complex64)
    want, _ = oracle.sparse_step(Xm.astype(np.complex128), Lp.astype(np.complex128), w,
                                 p.lambda_S, J, transform="db4")
    k, m, s, wd = _args(p, w)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, transform="db4") as h:
        h.solve(k, m, s, wd, lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=0, outputs=())
        S = h.op_sparse(_dev(Xm, torch.complex64), _dev(Lp, torch.complex64))
    e = _rel(S, want)
    print(f"{case} weights={weights}: op_sparse rel L2 {e:.2e}")
    assert e < TOL_OP


SOLVE_CASES = {
    "3d_16x16x4_nt6_nc2_J2": (dict(nx=16, ny=16, nz=4, nt=6, nc=2, seed=81), 2),
    "3d_32x48x8_nt12_nc3_J2": (dict(nx=32, ny=48, nz=8, nt=12, nc=3, seed=82), 2),
    "2d_32x32_nt10_nc1_J3": (dict(nx=32, ny=32, nz=1, nt=10, nc=1, seed=83), 3),
}


@pytest.mark.parametrize("name", sorted(SOLVE_CASES))
@pytest.mark.parametrize("weights", [False, True])
def test_db4_solve(name, weights):
    kw, J = SOLVE_CASES[name]
    p = synth.small(**kw, prior=False, lambda_S=0.02)
    w = _weights(p, kw["seed"] + 1000) if weights else None
    K = 8
    ref = oracle.solve(p.kspace, p.mask, p.sens, w, p.lambda_L, p.lambda_S, levels=J, iters=K,
                       transform="db4")
    k, m, s, wd = _args(p, w)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, transform="db4") as h:
        out, st = h.solve(k, m, s, wd, lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=K,
                          check_every=4)
    for key in ("L", "S", "X", "M"):
        e = _rel(out[key], ref[key])
        print(f"{name} weights={weights} {key}: rel L2 {e:.2e}")
        assert e < TOL, (key, e)
    assert st["iters"] == K
    assert st["resid_norm"] == pytest.approx(float(ref["resid"][-1]), rel=1e-4)
    assert st["l1_weighted"] == pytest.approx(float(ref["l1w"][-1]), rel=1e-3)


def test_db4_append_chain():
    q = synth.sequence(nx=16, ny=32, nz=4, nt=6, nc=2, accel=3, n_append=2, seed=85,
                       lambda_S=0.02)
    J = 2
    d, m = q.first_window()
    ref = oracle.solve(d, m, q.sens, None, q.lambda_L, q.lambda_S, levels=J, iters=6,
                       transform="db4")
    refs = [ref]
    for j in range(q.n_append):
        dn, mn = q.frame(j)
        ref, d, m = oracle.append_frame(ref, d, m, q.sens, dn, mn, q.lambda_L, q.lambda_S,
                                        lambda_p=0.3, levels=J, iters=5, transform="db4")
        refs.append(ref)
    sens = _dev(q.sens, torch.complex64)
    with pls.PriorLS(q.nx, q.ny, q.nz, q.nt, q.nc, wavelet_levels=J, transform="db4") as h:
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
            e = _rel(o[key], r[key])
            print(f"window {wnd} {key}: rel L2 {e:.2e}")
            assert e < TOL, (wnd, key, e)


def test_db4_batch_matches_each_problem_alone():
    # one plane (32 x 8), J = 2; window length, readout length and coil count differ
    kws = [dict(nx=16, ny=32, nz=8, nt=6, nc=2, seed=91), dict(nx=32, ny=32, nz=8, nt=9, nc=1, seed=92),
           dict(nx=24, ny=32, nz=8, nt=6, nc=3, seed=93)]
    ps = [synth.small(**kw, prior=False, lambda_S=0.02) for kw in kws]
    prm = dict(max_iter=6, check_every=3)
    alone = []
    for p in ps:
        with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, transform="db4") as h:
            o, _ = h.solve(*_args(p, None), lambda_L=p.lambda_L, lambda_S=p.lambda_S, **prm)
            alone.append(o)
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, transform="db4")
          for p in ps]
    try:
        with pls.Batch(hs) as b:
            outs, _ = b.solve([pls.to_device(p) for p in ps],
                              [pls.make_params(lambda_L=p.lambda_L, lambda_S=p.lambda_S, **prm)
                               for p in ps])
    finally:
        for h in hs:
            h.close()
    for i, (o, a) in enumerate(zip(outs, alone)):
        for key in ("L", "S", "X", "M"):
            assert torch.equal(o[key], a[key]), (i, key)
