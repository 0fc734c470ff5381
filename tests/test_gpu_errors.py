"""Error paths of the solve-level entry points on the GPU: every status the input checks and
the statistics kernel return, and that a handle stays usable after each of them.

Statuses (include/prior_ls.h): EINVAL for a host pointer where device memory is required,
lambda_L or lambda_S < 0, lambda_p outside [0, 1], L0 without S0 (or S0 without L0),
lambda_p > 0 without sigma_prev, step before solve, a negative iteration count; ENONFINITE when
NaN or Inf reaches the iterate (Algorithm 1 run on data with a NaN).
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402


@pytest.fixture(scope="module")
def prob():
    p = synth.small(nx=16, ny=16, nz=4, nt=6, nc=2, accel=3, rank=2, nblobs=3, seed=31, levels=1)
    return p, pls.to_device(p)


def solve(h, t, p, **kw):
    args = dict(lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=3, check_every=3)
    args.update(kw)
    ins = dict(kspace=t["kspace"], mask=t["mask"], sens=t["sens"], prior_w=t["prior_w"])
    for k in ("kspace", "mask", "sens", "prior_w"):
        if k in args:
            ins[k] = args.pop(k)
    return h.solve(ins["kspace"], ins["mask"], ins["sens"], ins["prior_w"], **args)


def status_of(fn):
    with pytest.raises(pls.PriorLSError) as e:
        fn()
    return e.value.status


def still_usable(h, t, p):
    out, st = solve(h, t, p)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=1,
                     iters=3)
    g = out["X"].cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(g - r["X"]) / np.linalg.norm(r["X"]) < 1e-4
    assert st["nonfinite"] == 0


@pytest.mark.parametrize("which", ["kspace", "mask", "sens", "prior_w"])
def test_host_pointer_is_einval(prob, which):
    p, t = prob
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        bad = {which: t[which].cpu()}
        assert status_of(lambda: solve(h, t, p, **bad)) == pls.EINVAL
        assert "device" in pls.lib().prior_ls_last_error(h._h).decode()
        still_usable(h, t, p)


def test_host_pointer_warm_start_is_einval(prob):
    p, t = prob
    L0 = torch.zeros(p.shape, dtype=torch.complex64)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        assert status_of(lambda: solve(h, t, p, L0=L0, S0=L0.cuda())) == pls.EINVAL
        assert status_of(lambda: solve(h, t, p, L0=L0.cuda(), S0=L0)) == pls.EINVAL


def test_host_output_is_einval(prob):
    p, t = prob
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        Xh = torch.zeros(p.shape, dtype=torch.complex64)
        o = pls.Outputs(None, None, C.c_void_p(Xh.data_ptr()), None)
        ins = pls.Inputs(pls._ptr(t["kspace"]), pls._ptr(t["mask"]), pls._ptr(t["sens"]),
                         pls._ptr(t["prior_w"]), None, None, None)
        prm = pls.make_params(max_iter=1)
        rc = pls.lib().prior_ls_solve(h._h, C.byref(ins), C.byref(prm), C.byref(o), None)
        assert rc == pls.EINVAL


@pytest.mark.parametrize("kw", [dict(lambda_L=-0.01), dict(lambda_S=-1e-3), dict(lambda_p=1.5),
                                dict(lambda_p=-0.1), dict(tol=-1.0), dict(max_iter=-1),
                                dict(check_every=0)],
                         ids=["lambda_L<0", "lambda_S<0", "lambda_p>1", "lambda_p<0", "tol<0",
                              "max_iter<0", "check_every=0"])
def test_bad_parameters_are_einval(prob, kw):
    p, t = prob
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        extra = dict(sigma_prev=np.ones(p.nt)) if "lambda_p" in kw else {}
        assert status_of(lambda: solve(h, t, p, **kw, **extra)) == pls.EINVAL
        still_usable(h, t, p)


def test_warm_start_needs_both(prob):
    p, t = prob
    Z = torch.zeros(p.shape, dtype=torch.complex64, device="cuda")
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        assert status_of(lambda: solve(h, t, p, L0=Z)) == pls.EINVAL
        assert status_of(lambda: solve(h, t, p, S0=Z)) == pls.EINVAL
        still_usable(h, t, p)


def test_sigma_prior_needs_sigma_prev(prob):
    p, t = prob
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        assert status_of(lambda: solve(h, t, p, lambda_p=0.5)) == pls.EINVAL


def test_missing_required_arrays(prob):
    p, t = prob
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        assert status_of(lambda: solve(h, t, p, sens=None)) == pls.EINVAL   # nc = 2
        ins = pls.Inputs(None, pls._ptr(t["mask"]), pls._ptr(t["sens"]), None, None, None, None)
        prm = pls.make_params(max_iter=1)
        assert pls.lib().prior_ls_solve(h._h, C.byref(ins), C.byref(prm), None, None) == pls.EINVAL


def test_step_before_solve_and_negative_count(prob):
    p, t = prob
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        assert status_of(lambda: h.step(1)) == pls.EINVAL
        solve(h, t, p)
        assert status_of(lambda: h.step(-1)) == pls.EINVAL
        out, st = h.step(1)
        assert st["iters"] == 4


@pytest.mark.parametrize("bad", [float("nan"), float("inf")], ids=["nan", "inf"])
def test_nonfinite_data_is_enonfinite(prob, bad):
    p, t = prob
    k = t["kspace"].clone()
    # a sampled entry of frame 2, coil 1
    z, y = np.argwhere(p.mask[2] != 0)[0]
    k[1, 2, z, y, 3] = complex(bad, 0.0)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=1) as h:
        with pytest.raises(pls.PriorLSError) as e:
            solve(h, t, p, kspace=k)
        assert e.value.status == pls.ENONFINITE
        assert "non-finite" in pls.lib().prior_ls_last_error(h._h).decode()
        # the same handle then solves clean data
        still_usable(h, t, p)
