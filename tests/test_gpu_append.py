"""GPU parity of the sliding-window recursion (prior_ls_append) against the FP64 oracle's
append_frame chain: the first window by plain L+S, then frames appended one at a time,
each window compared element by element (relative L2 of L, S and M)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

TOL = 1e-4

CASES = {
    "3d_16x16x4_nt5_nc2": dict(nx=16, ny=16, nz=4, nt=5, nc=2, accel=3, n_append=3, seed=11),
    "3d_24x32x8_nt7_nc3": dict(nx=24, ny=32, nz=8, nt=7, nc=3, accel=4, n_append=2, seed=12),
    "2d_32x32_nt6_nc1": dict(nx=32, ny=32, nz=1, nt=6, nc=1, accel=4, n_append=2, seed=13),
}


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _rel(g, want):
    g = g.cpu().numpy().astype(np.complex128)
    return float(np.linalg.norm(g - want) / max(np.linalg.norm(want), 1e-300))


def run_chain(q, k0, k1, lam_p, gram_mode="fp64"):
    d, m = q.first_window()
    ref = oracle.solve(d, m, q.sens, None, q.lambda_L, q.lambda_S, levels=2, iters=k0)
    refs = [ref]
    for j in range(q.n_append):
        dn, mn = q.frame(j)
        ref, d, m = oracle.append_frame(ref, d, m, q.sens, dn, mn, q.lambda_L, q.lambda_S,
                                        lambda_p=lam_p, iters=k1)
        refs.append(ref)
    sens = None if q.sens is None else _dev(q.sens, torch.complex64)
    got = []
    with pls.PriorLS(q.nx, q.ny, q.nz, q.nt, q.nc, wavelet_levels=2, gram_mode=gram_mode) as h:
        d0, m0 = q.first_window()
        out, st = h.solve(_dev(d0, torch.complex64), _dev(m0, torch.uint8), sens,
                          lambda_L=q.lambda_L, lambda_S=q.lambda_S, max_iter=k0, check_every=4)
        got.append((out, st))
        for j in range(q.n_append):
            dn, mn = q.frame(j)
            out, st = h.append(_dev(dn, torch.complex64), _dev(mn, torch.uint8),
                               lambda_L=q.lambda_L, lambda_S=q.lambda_S, lambda_p=lam_p,
                               max_iter=k1, check_every=4)
            assert st["iters"] == k1
            got.append((out, st))
    return refs, got


@pytest.mark.parametrize("name", sorted(CASES))
def test_append_chain_matches_oracle(name):
    q = synth.sequence(**CASES[name])
    refs, got = run_chain(q, k0=8, k1=6, lam_p=0.3)
    for w, (ref, (out, st)) in enumerate(zip(refs, got)):
        for k in ("L", "S", "M"):
            e = _rel(out[k], ref[k])
            print(f"{name} window {w} {k}: rel L2 vs FP64 oracle {e:.3e}")
            assert e < TOL, (name, w, k, e)
        assert st["resid_norm"] == pytest.approx(float(ref["resid"][-1]), rel=TOL)
        np.testing.assert_allclose(np.array(st["sigma"][: q.nt]), ref["sigma"][-1],
                                   rtol=TOL, atol=TOL * ref["sigma"][-1][0])


def test_append_grows_the_sample_store():
    # the appended frames are fully sampled while the first window is 4x undersampled:
    # each new frame needs more room than any frame slot holds
    q = synth.sequence(nx=16, ny=16, nz=4, nt=5, nc=2, accel=1, accel_first=4,
                       n_append=2, seed=21)
    refs, got = run_chain(q, k0=5, k1=4, lam_p=0.0)
    for w, (ref, (out, _)) in enumerate(zip(refs, got)):
        for k in ("L", "S", "M"):
            assert _rel(out[k], ref[k]) < TOL, (w, k)


def test_append_full_noiseless_recovers_frames():
    # E^H E = I under full sampling: M of every window is the true images of its frames
    q = synth.sequence(nx=16, ny=16, nz=4, nt=4, nc=2, accel=1, accel_first=1, snr_db=None,
                       n_append=2, seed=22)
    _, got = run_chain(q, k0=3, k1=3, lam_p=0.2)
    for w, (out, _) in enumerate(got):
        want = q.X_true[w:w + q.nt]
        assert _rel(out["M"], want) < 1e-5, w
