"""Pins of the oracle's sliding-window recursion (Section 3, Fig. 2) and of the a-priori
knowledge solve() hands to the next time instance.  CPU only."""
import numpy as np
import pytest

import oracle
import synth


def _seq(**kw):
    args = dict(nx=16, ny=16, nz=4, nt=5, n_append=2, nc=2, accel=3, seed=7)
    args.update(kw)
    return synth.sequence(**args)


def _first(q, iters=6, **kw):
    d, m = q.first_window()
    return oracle.solve(d, m, q.sens, None, q.lambda_L, q.lambda_S, levels=2, iters=iters, **kw)


def test_sigma_L_are_the_singular_values_of_L():
    # sigma_L must be what an independent SVD of the returned L gives (L = U diag(s~) V^H)
    q = _seq()
    r = _first(q)
    sv = np.linalg.svd(oracle.cas(r["L"]), compute_uv=False)
    np.testing.assert_allclose(sv, r["sigma_L"], rtol=0, atol=1e-10 * sv[0])
    assert np.all(np.diff(r["sigma_L"]) <= 0)


def test_support_is_the_nonzero_set_of_T_of_S():
    # supp must equal where the forward transform of the returned S is nonzero (T is
    # orthonormal, so T(S) reproduces the shrunk coefficients to FP64 rounding)
    q = _seq()
    r = _first(q)
    c = np.abs(oracle.haar_fwd(r["S"], 2))
    nz = c > 1e-9 * c.max()
    assert r["supp"].dtype == np.uint8 and set(np.unique(r["supp"])) <= {0, 255}
    assert np.array_equal(nz, r["supp"] == 255)
    assert 0 < nz.sum() < nz.size


def test_no_iteration_gives_empty_priors():
    q = _seq()
    r = _first(q, iters=0)
    assert not r["supp"].any() and not r["sigma_L"].any()


def test_append_on_full_noiseless_data_recovers_the_new_window():
    # fully sampled, noiseless: E^H E = I (coils normalised to sum of squares 1), so the
    # data-consistent iterate M of any window is exactly the true images of its frames,
    # whatever the priors; this pins which frames the shifted window holds
    q = _seq(accel=1, accel_first=1, snr_db=None, nt=4, n_append=2)
    r = _first(q, iters=3)
    np.testing.assert_allclose(r["M"], q.X_true[:4], atol=1e-12)
    d, m = q.first_window()
    for j in range(2):
        dn, mn = q.frame(j)
        r, d, m = oracle.append_frame(r, d, m, q.sens, dn, mn, q.lambda_L, q.lambda_S,
                                      lambda_p=0.3, iters=3)
        np.testing.assert_allclose(r["M"], q.X_true[j + 1:j + 5], atol=1e-12)


def test_append_is_a_warm_solve_of_the_shifted_window():
    # the recursion built by hand from index lists: frames [1..nt-1] + new, warm start and
    # support from the previous frames [1..nt-1] + [nt-1], sigma prior from sigma_L
    q = _seq()
    nt = q.nt
    r0 = _first(q)
    d0, m0 = q.first_window()
    dn, mn = q.frame(0)
    r1, d1, m1 = oracle.append_frame(r0, d0, m0, q.sens, dn, mn, q.lambda_L, q.lambda_S,
                                     lambda_p=0.25, iters=4)
    keep = list(range(1, nt)) + [nt - 1]
    frames = list(range(1, nt + 1))
    np.testing.assert_array_equal(d1, q.kspace[:, frames])
    np.testing.assert_array_equal(m1, q.mask[frames])
    want = oracle.solve(q.kspace[:, frames], q.mask[frames], q.sens, r0["supp"][keep],
                        q.lambda_L, q.lambda_S, lambda_p=0.25, sigma_prev=r0["sigma_L"],
                        levels=2, iters=4, L0=r0["L"][keep], S0=r0["S"][keep])
    for k in ("L", "S", "M"):
        np.testing.assert_array_equal(r1[k], want[k])


def test_support_prior_protects_coefficients():
    # with the previous support everywhere (w = 1), nothing is shrunk: S = X - L_prev
    # exactly after one iteration (step (3) with a zero threshold)
    q = _seq()
    d, m = q.first_window()
    w = np.full((q.nt, q.nz, q.ny, q.nx), 255, np.uint8)
    r = oracle.solve(d, m, q.sens, w, q.lambda_L, 1.0, levels=2, iters=1)
    M0 = oracle.EH(d, m, q.sens)
    np.testing.assert_allclose(r["S"], M0 - M0, atol=1e-14)     # X_0 - L_0 = 0
    r2 = oracle.solve(d, m, q.sens, w, q.lambda_L, 1.0, levels=2, iters=2)
    np.testing.assert_allclose(r2["S"], r["M"] - r["L"], atol=1e-12)
