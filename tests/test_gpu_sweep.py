"""GPU parity over every kernel instance the library advertises, against the FP64 oracle.

The header's shape set compiles one data-consistency kernel per (ny, nz) phase-encode plane
(Algorithm 1 step (4); the 2D (y, z) FFTs of the acquisition operator of Section 2) and one
kx inverse DFT per readout length nx (step (0), the adjoint applied to the data).  Each
instance is compared element by element with the oracle at small nx, nt and nc:

  * data consistency M = Y - A^H(A Y - d) on a perturbed image (1e-5 relative L2), with the
    residual norm;
  * two full iterations with T the identity (wavelet_levels J = 0), so the sparse update's
    J = 0 instance runs too (1e-4 relative L2 for L, S, X = L + S and M);
  * the adjoint of the data, X_0 = A^H d, for every readout length (1e-5).

The instance list is the header's; tests/test_abi_cpu.py checks that the library accepts
exactly this set.
"""
import numpy as np
import pytest

import oracle
import synth
from instances import PLANES, READOUT_NX

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

TOL = 1e-4
TOL_OP = 1e-5


def rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.complex64)).cuda()


def perturbed(p, seed):
    rng = np.random.default_rng(seed)
    X = p.X_true
    Y = X + 0.1 * (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape))
    return Y.astype(np.complex64).astype(np.complex128)


def load(h, p, **kw):
    t = pls.to_device(p)
    args = dict(lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=0)
    args.update(kw)
    return h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], **args)


@pytest.mark.parametrize("ny,nz", PLANES, ids=[f"{ny}x{nz}" for ny, nz in PLANES])
def test_plane_instance_matches_oracle(ny, nz):
    # the 192 x 32 plane runs the 24-points-per-thread configuration of the 8-coil workload
    nc = 3 if (ny, nz) == (192, 32) else 2
    p = synth.small(nx=16, ny=ny, nz=nz, nt=3, nc=nc, accel=3, rank=2, nblobs=2,
                    seed=1000 + 37 * ny + nz, levels=0)
    Y = perturbed(p, ny + nz)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=0) as h:
        out, st = load(h, p, max_iter=2, check_every=2)
        M, r0 = h.op_dc(dev(Y))
    Mo, R = oracle.dc_step(Y, p.kspace, p.mask, p.sens)
    e = rel(host(M), Mo)
    assert e < TOL_OP, ("dc", e)
    assert r0 == pytest.approx(np.linalg.norm(R), rel=TOL_OP)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=0,
                     iters=2)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)
    assert st["resid_norm"] == pytest.approx(r["resid"][-1], rel=TOL)


@pytest.mark.parametrize("nx", READOUT_NX)
def test_readout_instance_adjoint_of_data(nx):
    p = synth.small(nx=nx, ny=16, nz=4, nt=2, nc=2, accel=3, rank=2, nblobs=2,
                    seed=2000 + nx, levels=0)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=0) as h:
        out, _ = load(h, p)
    want = oracle.EH(p.kspace, p.mask, p.sens)
    for k in ("M", "L"):
        e = rel(host(out[k]), want)
        assert e < TOL_OP, (k, e)


def test_c3_plane_with_haar_levels():
    # the 8-coil workload's plane and Haar depth (J = 2) over several iterations
    p = synth.small(nx=16, ny=192, nz=32, nt=3, nc=3, accel=10, rank=2, nblobs=3, seed=3001,
                    levels=2)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, gram_mode="fp32") as h:
        out, st = load(h, p, max_iter=5, check_every=5)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=2,
                     iters=5)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)


@pytest.mark.parametrize("lam", [0.02, 0.05])
@pytest.mark.parametrize("geom", [dict(nx=24, ny=48, nz=8, nt=7, nc=2),
                                  dict(nx=32, ny=32, nz=1, nt=9, nc=1)],
                         ids=["3d_24x48x8", "2d_32x32"])
def test_identity_transform_with_prior_weights(geom, lam):
    # J = 0: T is the identity, so the weights act voxel by voxel.  The voxels of the prior
    # support (w = 1) pass unshrunk and add exactly nothing to the weighted l1 norm; with
    # lambda_S = 0.02 about a hundred voxels off the support survive the threshold, with 0.05
    # none does and the norm is 0
    p = synth.small(**geom, accel=3, rank=2, nblobs=3, seed=3100 + geom["nx"], levels=0)
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=0) as h:
        out, st = load(h, p, max_iter=6, check_every=3, lambda_S=lam)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, lam, levels=0, iters=6)
    for k in ("L", "S", "X", "M"):
        e = rel(host(out[k]), r[k])
        assert e < TOL, (k, e)
    assert st["l1_weighted"] == pytest.approx(r["l1w"][-1], rel=TOL, abs=1e-7)
