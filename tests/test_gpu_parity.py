"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerance: relative L2 <= 1e-4 per result after K iterations (FP32 FFT / threshold
path, FP64 Gram and eigensolve); the single-step operators are held to 1e-5.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

TOL = 1e-4
TOL_OP = 1e-5

# (name, problem kwargs, levels): several tiles, ragged plane batches, radix-3 lengths,
# 2D and 3D, single and multi coil
CASES = [
    ("3d_16x16x4_nt6_nc2", dict(nx=16, ny=16, nz=4, nt=6, nc=2, accel=3, rank=2, nblobs=3, seed=11), 2),
    ("3d_24x24x4_nt5_nc1", dict(nx=24, ny=24, nz=4, nt=5, nc=1, accel=2, rank=2, nblobs=2, seed=12), 1),
    ("3d_32x48x8_nt12_nc3", dict(nx=32, ny=48, nz=8, nt=12, nc=3, accel=4, rank=3, nblobs=4, seed=13), 2),
    ("2d_32x32_nt8_nc1", dict(nx=32, ny=32, nz=1, nt=8, nc=1, accel=3, rank=2, nblobs=3, seed=14), 2),
    ("3d_48x96x16_nt17_nc2", dict(nx=48, ny=96, nz=16, nt=17, nc=2, accel=6, rank=3, nblobs=6, seed=15), 3),
    # nz = 14 (the cardiac geometry's slice count): radix 14 = 2 x 7 along z
    ("3d_16x32x14_nt6_nc2", dict(nx=16, ny=32, nz=14, nt=6, nc=2, accel=3, rank=2, nblobs=3, seed=16), 1),
    ("3d_32x16x14_nt5_nc1", dict(nx=32, ny=16, nz=14, nt=5, nc=1, accel=2, rank=2, nblobs=2, seed=17), 1),
    ("3d_16x256x14_nt4_nc1", dict(nx=16, ny=256, nz=14, nt=4, nc=1, accel=4, rank=2, nblobs=3, seed=18), 1),
]


def rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.complex64)).cuda()


def make(case):
    name, kw, J = case
    p = synth.small(**kw, levels=J)
    return p, J


def handle(p, J, **kw):
    return pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, **kw)


def load(h, p, **kw):
    t = pls.to_device(p)
    args = dict(lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=0)
    args.update(kw)
    return h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], **args)


@pytest.fixture(params=CASES, ids=[c[0] for c in CASES])
def case(request):
    return make(request.param)


def test_step0_adjoint_of_data(case):
    p, J = case
    with handle(p, J) as h:
        out, st = load(h, p)
        want = oracle.EH(p.kspace, p.mask, p.sens)
        e1, e2 = rel(host(out["M"]), want), rel(host(out["L"]), want)
        assert e1 < TOL_OP and e2 < TOL_OP, (e1, e2)
        assert np.abs(host(out["S"])).max() == 0


def test_op_dc_matches_oracle(case):
    p, J = case
    rng = np.random.default_rng(3)
    Y = p.X_true + 0.1 * (rng.standard_normal(p.X_true.shape) + 1j * rng.standard_normal(p.X_true.shape))
    Y = Y.astype(np.complex64).astype(np.complex128)
    with handle(p, J) as h:
        load(h, p)
        M, r = h.op_dc(dev(Y))
    want, R = oracle.dc_step(Y, p.kspace, p.mask, p.sens)
    e = rel(host(M), want)
    assert e < TOL_OP, e
    assert r == pytest.approx(np.linalg.norm(R), rel=1e-5)


def test_normal_operator_is_hermitian(case):
    """<N x, y> = <x, N y> for N = E^H E = op_dc(0) - op_dc(Y) + Y (adjoint identity)."""
    p, J = case
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape)).astype(np.complex64)
    y = (rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape)).astype(np.complex64)
    with handle(p, J) as h:
        load(h, p)
        m0, _ = h.op_dc(torch.zeros(p.shape, dtype=torch.complex64, device="cuda"))
        mx, _ = h.op_dc(dev(x))
        my, _ = h.op_dc(dev(y))
    Nx = host(m0) - host(mx) + x
    Ny = host(m0) - host(my) + y
    lhs = np.vdot(y, Nx)
    rhs = np.vdot(Ny, x)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    e = rel(Nx, oracle.EH(oracle.E(x, p.mask, p.sens), p.mask, p.sens))
    assert e < TOL_OP, e


def test_op_svt_matches_oracle(case):
    p, J = case
    with handle(p, J) as h:
        load(h, p)
        Cm = oracle.EH(p.kspace, p.mask, p.sens).astype(np.complex64).astype(np.complex128)
        Lg, sig = h.op_svt(dev(Cm))
    Lw, sw, _, _ = oracle.svt(oracle.cas(Cm), p.lambda_L)
    e = rel(host(Lg), oracle.uncas(Lw, p.shape))
    assert e < TOL_OP, e
    np.testing.assert_allclose(sig, sw, rtol=1e-5, atol=1e-6 * sw[0])


def test_op_svt_sigma_prior(case):
    p, J = case
    rng = np.random.default_rng(8)
    prev = np.sort(rng.uniform(0, 2, p.nt))[::-1]
    with handle(p, J) as h:
        load(h, p, lambda_p=0.5, sigma_prev=prev)
        Cm = oracle.EH(p.kspace, p.mask, p.sens).astype(np.complex64).astype(np.complex128)
        Lg, _ = h.op_svt(dev(Cm))
    Lw, _, _, _ = oracle.svt(oracle.cas(Cm), p.lambda_L, True, 0.5, prev)
    e = rel(host(Lg), oracle.uncas(Lw, p.shape))
    assert e < TOL_OP, e


def test_op_sparse_matches_oracle(case):
    p, J = case
    M0 = oracle.EH(p.kspace, p.mask, p.sens)
    Lp = (0.5 * M0).astype(np.complex64).astype(np.complex128)
    M0 = M0.astype(np.complex64).astype(np.complex128)
    with handle(p, J) as h:
        load(h, p, lambda_S=0.02)
        Sg = h.op_sparse(dev(M0), dev(Lp))
    Sw, _ = oracle.sparse_step(M0, Lp, p.prior_w, 0.02, J)
    e = rel(host(Sg), Sw)
    assert e < TOL_OP, e


@pytest.mark.parametrize("iters", [1, 7])
def test_solve_matches_oracle(case, iters):
    p, J = case
    with handle(p, J) as h:
        out, st = load(h, p, max_iter=iters, check_every=3)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=J,
                     iters=iters)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)
    assert st["iters"] == iters
    assert st["resid_norm"] == pytest.approx(r["resid"][-1], rel=1e-4)
    assert st["nuclear_norm"] == pytest.approx(r["nuclear"][-1], rel=1e-4)
    assert st["rel_change"] == pytest.approx(r["rel_change"][-1], rel=1e-3)
    np.testing.assert_allclose(st["sigma"], r["sigma"][-1], rtol=1e-4, atol=1e-5 * r["sigma"][-1][0])
    # the reported objective 0.5 ||r||^2 + tau_L ||L||_* + lambda_S ||(1 - w) T(S)||_1 and its
    # parts
    assert st["tau_L"] == pytest.approx(r["tau_L"][-1], rel=1e-4)
    assert st["l1_weighted"] == pytest.approx(r["l1w"][-1], rel=1e-4)
    assert st["objective"] == pytest.approx(r["objective"][-1], rel=1e-4)


def test_solve_with_sigma_prior_and_warm_start(case):
    p, J = case
    rng = np.random.default_rng(9)
    prev = np.sort(rng.uniform(0, 3, p.nt))[::-1]
    L0 = (0.9 * p.L_true).astype(np.complex64).astype(np.complex128)
    S0 = (0.8 * p.S_true).astype(np.complex64).astype(np.complex128)
    with handle(p, J) as h:
        out, st = load(h, p, max_iter=5, lambda_p=0.5, sigma_prev=prev, L0=dev(L0), S0=dev(S0))
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, lambda_p=0.5,
                     sigma_prev=prev, levels=J, iters=5, L0=L0, S0=S0)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)


def test_sigma_prev_in_device_memory(case):
    # sigma_prev may be host or device memory: the same bits either way (in any order)
    p, J = case
    rng = np.random.default_rng(10)
    prev = rng.uniform(0, 3, p.nt)
    with handle(p, J) as h:
        a, _ = load(h, p, max_iter=4, lambda_p=0.5, sigma_prev=list(prev))
        b, _ = load(h, p, max_iter=4, lambda_p=0.5,
                    sigma_prev=torch.from_numpy(prev[::-1].copy()).cuda())
    for k in ("L", "S", "X", "M"):
        assert torch.equal(a[k], b[k]), k


def test_determinism_resume_and_graphs(case):
    p, J = case
    with handle(p, J) as h:
        a, _ = load(h, p, max_iter=6, check_every=4)
        b, _ = load(h, p, max_iter=6, check_every=2, use_graph=False)
        c0, _ = load(h, p, max_iter=4, check_every=4)
        c, _ = h.step(2)
    for k in ("L", "S", "M"):
        assert torch.equal(a[k], b[k]), k
        assert torch.equal(a[k], c[k]), k


def test_config1_full(request):
    p = synth.config(1)
    with handle(p, 2) as h:
        out, st = load(h, p, max_iter=p.iters, check_every=10)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=2,
                     iters=p.iters)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)


# Gram precision modes: FP64 MFMA (default, exact products), FP32 MFMA, split BF16 (hi+lo,
# three products, FP32 accumulate).  The split-BF16 path is held to 1e-3.
MODE_TOL = {"fp64": (1e-5, 1e-4), "fp32": (1e-4, 1e-4), "bf16x3": (1e-3, 1e-3)}


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_gram_modes_svt_and_solve(case, mode):
    p, J = case
    tol_op, tol = MODE_TOL[mode]
    with handle(p, J, gram_mode=mode) as h:
        load(h, p)
        Cm = oracle.EH(p.kspace, p.mask, p.sens).astype(np.complex64).astype(np.complex128)
        Lg, sig = h.op_svt(dev(Cm))
        out, st = load(h, p, max_iter=7, check_every=7)
    Lw, sw, _, _ = oracle.svt(oracle.cas(Cm), p.lambda_L)
    e = rel(host(Lg), oracle.uncas(Lw, p.shape))
    assert e < tol_op, (mode, e)
    np.testing.assert_allclose(sig, sw, rtol=tol_op, atol=tol_op * sw[0])
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=J, iters=7)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < tol, (mode, k, e)


@pytest.mark.parametrize("geom", [dict(nx=16, ny=16, nz=4, nt=6, nc=2),
                                  dict(nx=24, ny=48, nz=8, nt=5, nc=1)],
                         ids=["3d_16x16x4_nt6_nc2", "3d_24x48x8_nt5_nc1"])
def test_empty_and_fully_sampled_frames(geom):
    # degenerate masks: frame 0 has no samples (no lines in the compact data, an empty
    # residual) and frame 2 is fully sampled (every entry is replaced by data)
    p = synth.small(**geom, accel=3, rank=2, nblobs=3, seed=21, levels=1, snr_db=None)
    m = p.mask.copy()
    m[0] = 0
    m[2] = 1
    p.mask = m
    p.kspace = synth.sample(p.L_true + p.S_true, m, p.sens)
    rng = np.random.default_rng(5)
    X = p.L_true + p.S_true
    Y = X + 0.1 * (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape))
    Y = Y.astype(np.complex64).astype(np.complex128)
    with handle(p, 1) as h:
        out, st = load(h, p, max_iter=7, check_every=7)
        M, r0 = h.op_dc(dev(Y))
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=1,
                     iters=7)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)
    assert st["resid_norm"] == pytest.approx(r["resid"][-1], rel=1e-4)
    Mo, R = oracle.dc_step(Y, p.kspace, p.mask, p.sens)
    assert rel(host(M), Mo) < TOL_OP
    assert r0 == pytest.approx(np.linalg.norm(R), rel=1e-5)


# the largest planes: 256 x 32 (8192 points, 512-thread blocks), 128 x 32 and 96 x 32
# (radix 3 along y), each with more than one coil
MAX_PLANES = [dict(nx=16, ny=256, nz=32, nt=3, nc=2), dict(nx=16, ny=128, nz=32, nt=4, nc=3),
              dict(nx=16, ny=96, nz=32, nt=3, nc=2)]


@pytest.mark.parametrize("geom", MAX_PLANES, ids=["256x32", "128x32", "96x32"])
def test_largest_planes_match_oracle(geom):
    p = synth.small(**geom, accel=4, rank=2, nblobs=3, seed=23, levels=1)
    rng = np.random.default_rng(6)
    Y = p.X_true + 0.1 * (rng.standard_normal(p.X_true.shape)
                          + 1j * rng.standard_normal(p.X_true.shape))
    Y = Y.astype(np.complex64).astype(np.complex128)
    with handle(p, 1) as h:
        out, st = load(h, p, max_iter=4, check_every=2)
        M, r0 = h.op_dc(dev(Y))
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=1,
                     iters=4)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)
    Mo, R = oracle.dc_step(Y, p.kspace, p.mask, p.sens)
    assert rel(host(M), Mo) < TOL_OP
    assert r0 == pytest.approx(np.linalg.norm(R), rel=1e-5)
