"""Pins of the FP64 oracle against closed forms, invariants and brute force.

The paper prints no worked numeric example, so every pin here is a closed form, a
mathematical invariant, a special case that reduces to a textbook routine, or a
brute-force dense-matrix evaluation on a tiny input.  Each test names the pin it
implements and the passage it follows.
"""
import math

import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(20141120)


def cg(shape, rng=RNG):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def rand_unitary(n, rng=RNG):
    q, r = np.linalg.qr(cg((n, n), rng))
    return q * (np.diag(r) / np.abs(np.diag(r)))


# ---------------------------------------------------------------- P1 soft threshold (Sec. 2)
def test_p1_soft_closed_form():
    # 3+4i has modulus 5: shrinking by 1 keeps the phase and leaves modulus 4
    assert oracle.soft(3 + 4j, 1.0) == pytest.approx(2.4 + 3.2j, abs=1e-15)
    assert oracle.soft(3 + 4j, 5.0) == 0
    assert oracle.soft(3 + 4j, 7.0) == 0
    assert oracle.soft(-2.0, 0.5) == pytest.approx(-1.5, abs=1e-15)
    assert oracle.soft(0.0, 1.0) == 0
    assert oracle.soft(1j, 0.25) == pytest.approx(0.75j, abs=1e-15)
    z = cg(1000)
    np.testing.assert_array_equal(oracle.soft(z, 0.0), z)
    tau = RNG.uniform(0, 1, 1000)
    out = oracle.soft(z, tau)
    np.testing.assert_allclose(np.abs(out), np.maximum(np.abs(z) - tau, 0), atol=1e-15)
    keep = np.abs(out) > 0
    np.testing.assert_allclose(np.angle(out[keep]), np.angle(z[keep]), atol=1e-13)


# ---------------------------------------------------------------- P2 / P3 SVT (steps 1-2)
def _prescribed(N, nt, sigma, rng=RNG):
    U, _ = np.linalg.qr(cg((N, nt), rng))
    V = rand_unitary(nt, rng)
    return U, V, (U * sigma) @ V.conj().T


def test_p2_svt_prescribed_singular_values():
    sigma = np.array([10.0, 5.0, 2.0, 0.9, 0.31, 0.05])
    U, V, C = _prescribed(200, 6, sigma)
    lam = 0.04                                  # tau = 0.4 (relative to sigma_1 = 10)
    L, s, st, tau = oracle.svt(C, lam, relative=True)
    assert tau == pytest.approx(0.4)
    np.testing.assert_allclose(s, sigma, rtol=1e-12)
    expect = (U * np.array([9.6, 4.6, 1.6, 0.5, 0.0, 0.0])) @ V.conj().T
    np.testing.assert_allclose(L, expect, atol=1e-12)
    # absolute threshold
    L2, _, st2, tau2 = oracle.svt(C, 1.0, relative=False)
    assert tau2 == 1.0
    np.testing.assert_allclose(st2, [9.0, 4.0, 1.0, 0.0, 0.0, 0.0], atol=1e-12)


def test_p3_sigma_prior_closed_form():
    sigma = np.array([8.0, 4.0, 2.0, 1.0])
    prev = np.array([7.0, 4.5, 1.0, 0.5])
    U, V, C = _prescribed(64, 4, sigma)
    for lp in (0.0, 0.5, 1.0):
        L, _, st, _ = oracle.svt(C, 0.5, relative=False, lambda_p=lp, sigma_prev=prev)
        hat = np.maximum(sigma - 0.5, 0)
        want = (1 - lp) * hat + lp * prev
        np.testing.assert_allclose(st, want, atol=1e-12)
        np.testing.assert_allclose(L, (U * want) @ V.conj().T, atol=1e-12)
    # lambda_p = 1 returns exactly the previous singular values
    _, _, st, _ = oracle.svt(C, 0.5, relative=False, lambda_p=1.0, sigma_prev=prev[::-1])
    np.testing.assert_array_equal(st, prev)


def test_p3_sigma_prior_zero_pads_and_pairs_descending():
    sigma = np.array([4.0, 3.0, 2.0])
    U, V, C = _prescribed(30, 3, sigma)
    _, _, st, _ = oracle.svt(C, 0.0, relative=False, lambda_p=0.5, sigma_prev=np.array([1.0, 5.0]))
    np.testing.assert_allclose(st, [4.5, 2.0, 1.0], atol=1e-12)


# ---------------------------------------------------------------- P4 / P5 the operator E
def _tiny(nz=2, ny=4, nx=4, nt=3, nc=2, rng=RNG, full=False):
    mask = (rng.uniform(size=(nt, nz, ny)) < 0.5).astype(np.uint8)
    if full:
        mask[:] = 1
    sens = cg((nc, nz, ny, nx), rng)
    sens /= np.sqrt(np.sum(np.abs(sens) ** 2, axis=0, keepdims=True))
    return mask, sens


def test_p4_adjoint_identity():
    for nc in (1, 3):
        mask, sens = _tiny(nz=4, ny=6, nx=8, nt=5, nc=nc)
        sens = None if nc == 1 else sens
        x = cg((5, 4, 6, 8))
        y = cg((nc, 5, 4, 6, 8))
        lhs = np.vdot(oracle.E(x, mask, sens), y)
        rhs = np.vdot(x, oracle.EH(y, mask, sens))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _dft(n):
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


@pytest.mark.parametrize("workers", [None, 4], ids=["numpy", "scipy_threads"])
def test_p5_fft_matches_explicit_dft_matrix(workers):
    # both library calls the oracle can use (numpy.fft; scipy.fft on threads, for timing)
    x = cg((3, 2, 4, 6))
    Fz, Fy, Fx = _dft(2), _dft(4), _dft(6)
    want = np.einsum("az,by,cx,tzyx->tabc", Fz, Fy, Fx, x)
    try:
        oracle.set_fft_workers(workers)
        np.testing.assert_allclose(oracle.fft3(x), want, atol=1e-14)
        np.testing.assert_allclose(oracle.ifft3(want), x, atol=1e-14)
        y = cg((2, 8, 12, 10))
        np.testing.assert_allclose(oracle.ifft3(oracle.fft3(y)), y, atol=1e-13)
    finally:
        oracle.set_fft_workers(None)


def test_threaded_fft_gives_the_same_iterate():
    # the timing configuration of the oracle computes the same iteration
    p = synth.small(nx=16, ny=16, nz=4, nt=5, nc=2, accel=3, rank=2, nblobs=2, seed=44)
    a = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, 0.01, 0.01, levels=2, iters=3)
    try:
        oracle.set_fft_workers(4)
        seen = []
        b = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, 0.01, 0.01, levels=2, iters=3,
                         on_iteration=seen.append)
    finally:
        oracle.set_fft_workers(None)
    assert seen == [0, 1, 2, 3]
    for k in ("L", "S", "M"):
        np.testing.assert_allclose(b[k], a[k], atol=1e-13)


def test_p5_normal_operator_is_identity_when_fully_sampled():
    mask, sens = _tiny(nz=4, ny=8, nx=6, nt=3, nc=4, full=True)
    x = cg((3, 4, 8, 6))
    np.testing.assert_allclose(oracle.EH(oracle.E(x, mask, sens), mask, sens), x, atol=1e-13)
    assert np.linalg.norm(oracle.E(x, mask, sens)) == pytest.approx(np.linalg.norm(x), rel=1e-13)


def test_p5_E_as_dense_matrix():
    """Brute force: assemble E column by column from its definition with explicit DFT
    matrices and compare both E and E^H (conjugate transpose)."""
    nt, nz, ny, nx, nc = 2, 2, 2, 4, 2
    mask, sens = _tiny(nz, ny, nx, nt, nc)
    F = np.kron(np.kron(_dft(nz), _dft(ny)), _dft(nx))
    n = nz * ny * nx
    blocks = np.zeros((nc * nt * n, nt * n), complex)
    for c in range(nc):
        for t in range(nt):
            m = np.repeat(mask[t].reshape(-1), nx).astype(float)
            blocks[(c * nt + t) * n:(c * nt + t + 1) * n, t * n:(t + 1) * n] = \
                (m[:, None] * F) @ np.diag(sens[c].reshape(-1))
    x = cg((nt, nz, ny, nx))
    np.testing.assert_allclose(oracle.E(x, mask, sens).reshape(-1), blocks @ x.reshape(-1), atol=1e-14)
    y = cg((nc, nt, nz, ny, nx))
    np.testing.assert_allclose(oracle.EH(y, mask, sens).reshape(-1),
                               blocks.conj().T @ y.reshape(-1), atol=1e-14)


# ---------------------------------------------------------------- P6 Haar transform T
def test_p6_haar_1d_explicit():
    s = 1 / math.sqrt(2)
    # canonical layout for n = 4, J = 2: [aa, ad, d0, d1]
    H = np.array([[0.5, 0.5, 0.5, 0.5],
                  [0.5, 0.5, -0.5, -0.5],
                  [s, -s, 0, 0],
                  [0, 0, s, -s]])
    for k in range(4):
        e = np.zeros((1, 1, 4))
        e[0, 0, k] = 1
        np.testing.assert_allclose(oracle.haar_fwd(e, 2)[0, 0], H[:, k], atol=1e-15)


def test_p6_haar_2d_nonstandard_pyramid():
    x = cg((1, 4, 4))
    c = oracle.haar_fwd(x, 2)
    s = 1 / math.sqrt(2)
    X = x[0]
    # level-1 detail in x, low in y, at block (0,0): NOT decomposed further
    a_y = (X[0, :] + X[1, :]) * s                       # low along y, rows 0-1
    want_01 = (a_y[0] - a_y[1]) * s                     # detail along x, cols 0-1
    assert c[0, 0, 2] == pytest.approx(want_01, abs=1e-14)
    # level-1 diagonal detail at block (1,1) (rows 2-3, cols 2-3)
    B = X[2:4, 2:4]
    assert c[0, 3, 3] == pytest.approx((B[0, 0] - B[0, 1] - B[1, 0] + B[1, 1]) / 2, abs=1e-14)
    # coarsest coefficient = sum / 4 (mean * sqrt(16))
    assert c[0, 0, 0] == pytest.approx(X.sum() / 4, abs=1e-14)
    # level-2 detail along y of the all-low band: (rows 0-1 minus rows 2-3) / 4
    assert c[0, 1, 0] == pytest.approx((X[0:2].sum() - X[2:4].sum()) / 4, abs=1e-14)


@pytest.mark.parametrize("shape,J", [((1, 8, 8), 2), ((4, 8, 16), 2), ((8, 8, 8), 3),
                                     ((1, 1, 16), 4), ((4, 4, 4), 0)])
def test_p6_haar_orthonormal(shape, J):
    x = cg((3,) + shape)
    c = oracle.haar_fwd(x, J)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-14)
    np.testing.assert_allclose(oracle.haar_inv(c, J), x, atol=1e-14)
    # T^H T = I as a dense matrix on the smallest shapes
    n = int(np.prod(shape))
    if n <= 64:
        T = np.stack([oracle.haar_fwd(np.eye(n)[k].reshape(shape), J).reshape(-1) for k in range(n)], 1)
        np.testing.assert_allclose(T.T @ T, np.eye(n), atol=1e-14)


def test_p6_haar_constant_input():
    x = np.full((1, 4, 8, 8), 3.0 + 1.0j)
    c = oracle.haar_fwd(x, 2)
    coarse = c[0, :1, :2, :2]
    np.testing.assert_allclose(coarse, (3 + 1j) * 8.0, atol=1e-13)   # mean * sqrt(4*4*4)
    rest = c.copy()
    rest[0, :1, :2, :2] = 0
    assert np.abs(rest).max() < 1e-13


# ---------------------------------------------------------------- P7 / P8 fixed points
def _full_problem(nt=6, nz=4, ny=8, nx=8, nc=2, rank=2, nblobs=2, seed=3):
    p = synth.small(nx=nx, ny=ny, nz=nz, nt=nt, nc=nc, accel=1, snr_db=None,
                    rank=rank, nblobs=nblobs, seed=seed)
    assert p.mask.all()
    return p


def test_p7_fully_sampled_noiseless_is_data_consistent():
    p = _full_problem()
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, 0.01, 0.01, levels=2, iters=3)
    np.testing.assert_allclose(r["M"], p.X_true, atol=1e-13)


def test_p8_exact_rank_plus_sparse_is_a_fixed_point():
    p = _full_problem()
    T = oracle.haar_fwd(p.S_true, 2)
    supp = np.abs(T) > 1e-12 * np.abs(T).max()
    w = np.where(supp, 255, 0).astype(np.uint8)
    r = oracle.solve(p.kspace, p.mask, p.sens, w, lambda_L=0.05, lambda_S=0.05, lambda_p=1.0,
                     sigma_prev=p.sigma_true, levels=2, iters=1, L0=p.L_true, S0=p.S_true)
    np.testing.assert_allclose(r["L"], p.L_true, atol=1e-12)
    np.testing.assert_allclose(r["S"], p.S_true, atol=1e-12)
    # and with no prior the same start is NOT a fixed point (the pin has teeth)
    r0 = oracle.solve(p.kspace, p.mask, p.sens, None, 0.05, 0.05, levels=2, iters=1,
                      L0=p.L_true, S0=p.S_true)
    assert oracle.rel_l2(r0["L"], p.L_true) > 1e-3


# ---------------------------------------------------------------- P9 zero prior == plain L+S
def test_p9_zero_prior_reduces_to_plain_ls():
    p = synth.small(nx=16, ny=16, nz=4, nt=6, nc=2, accel=3, seed=5)
    a = oracle.solve(p.kspace, p.mask, p.sens, np.zeros_like(p.prior_w), 0.02, 0.01,
                     lambda_p=0.0, sigma_prev=None, levels=2, iters=8)
    b = oracle.plain_ls(p.kspace, p.mask, p.sens, 0.02, 0.01, levels=2, iters=8)
    for k in ("L", "S", "M"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-13)
    # and the prior actually changes the result
    c = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, 0.02, 0.01, levels=2, iters=8)
    assert oracle.rel_l2(c["S"], a["S"]) > 1e-3


# ---------------------------------------------------------------- P10 nt = 1
def test_p10_single_frame_svt_is_vector_shrink():
    c = cg((50, 1))
    nrm = np.linalg.norm(c)
    for tau in (0.3 * nrm, 2 * nrm):
        L, _, _, _ = oracle.svt(c, tau, relative=False)
        np.testing.assert_allclose(L, c * max(1 - tau / nrm, 0), atol=1e-14)


def test_p10_zero_thresholds_full_sampling():
    p = _full_problem(nt=1, rank=1)
    r = oracle.solve(p.kspace, p.mask, p.sens, None, 0.0, 0.0, levels=1, iters=1)
    np.testing.assert_allclose(r["M"], p.X_true, atol=1e-13)
    # first sparse update sees X_0 - L_0 = 0
    assert np.abs(r["S"]).max() == 0
    r2 = oracle.solve(p.kspace, p.mask, p.sens, None, 0.0, 0.0, levels=1, iters=2)
    np.testing.assert_allclose(r2["S"], r["M"] - r["L"], atol=1e-13)


# ---------------------------------------------------------------- P11 Gram route == SVD route
def test_p11_gram_eigh_route_matches_svd_route():
    sigma = np.array([5.0, 3.0, 2.5, 1.0, 0.5, 0.2, 0.1, 0.05])
    U, V, C = _prescribed(500, 8, sigma)
    for lp, prev in ((0.0, None), (0.5, np.linspace(4, 0.1, 8))):
        a = oracle.svt(C, 0.1, True, lp, prev)
        b = oracle.svt_gram(C, 0.1, True, lp, prev)
        np.testing.assert_allclose(b[0], a[0], atol=1e-10)
        np.testing.assert_allclose(b[1], a[1], rtol=1e-10)


# ---------------------------------------------------------------- P12 invariants
def test_p12_invariants():
    p = synth.small(nx=16, ny=16, nz=4, nt=8, nc=2, accel=3, seed=9)
    M = oracle.EH(p.kspace, p.mask, p.sens)
    L_prev = 0.7 * M
    S, Zs = oracle.sparse_step(M, L_prev, p.prior_w, 0.02, 2)
    Z = oracle.haar_fwd(M - L_prev, 2)
    tau = 0.02 * (1 - p.prior_w / 255.0)
    assert np.all(Zs[np.abs(Z) <= tau] == 0)
    np.testing.assert_allclose(oracle.haar_fwd(S, 2), Zs, atol=1e-14)
    C = oracle.cas(M)
    L, sigma, st, tau_L = oracle.svt(C, 0.05)
    assert np.linalg.matrix_rank(L, tol=1e-10 * sigma[0]) <= int(np.sum(sigma > tau_L))
    G = C.conj().T @ C
    lam, V = np.linalg.eigh(G)
    s = np.sqrt(np.maximum(lam, 0))
    st2, _ = oracle.sv_targets(s[::-1], 0.05, True, 0.0, None)
    phi = np.divide(st2[::-1], s, out=np.zeros_like(s), where=s > 0)
    W = (V * phi) @ V.conj().T
    np.testing.assert_allclose(W, W.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(W).min() > -1e-12


# ---------------------------------------------------------------- brute-force iteration
def _haar1(n):
    s = 1 / math.sqrt(2)
    H = np.zeros((n, n))
    for m in range(n // 2):
        H[m, 2 * m], H[m, 2 * m + 1] = s, s
        H[n // 2 + m, 2 * m], H[n // 2 + m, 2 * m + 1] = s, -s
    return H


def test_brute_force_three_iterations_dense():
    """Algorithm 1 written with dense matrices on a 1 x 4 x 4 x 3-frame problem with two
    coils: explicit DFT and Haar (J = 1) matrices, LAPACK SVD, elementwise shrink."""
    rng = np.random.default_rng(77)
    nt, nz, ny, nx, nc = 3, 1, 4, 4, 2
    mask = (rng.uniform(size=(nt, nz, ny)) < 0.6).astype(np.uint8)
    mask[:, :, 0] = 1
    sens = cg((nc, nz, ny, nx), rng)
    sens /= np.sqrt(np.sum(np.abs(sens) ** 2, axis=0, keepdims=True))
    d = cg((nc, nt, nz, ny, nx), rng) * mask[None, :, :, :, None]
    w = (rng.uniform(size=(nt, nz, ny, nx)) < 0.3).astype(np.uint8) * 255
    lamL, lamS, lamp = 0.1, 0.05, 0.3
    sprev = np.array([3.0, 1.0, 0.2])
    n = ny * nx
    F = np.kron(_dft(ny), _dft(nx))
    T = np.kron(_haar1(ny), _haar1(nx))
    Es = []
    for c in range(nc):
        for t in range(nt):
            m = np.repeat(mask[t, 0], nx).astype(float)
            Es.append((c, t, (m[:, None] * F) @ np.diag(sens[c, 0].reshape(-1))))

    def Eop(Y):  # Y: n x nt
        return {(c, t): A @ Y[:, t] for c, t, A in Es}

    def EHop(R):
        out = np.zeros((n, nt), complex)
        for c, t, A in Es:
            out[:, t] += A.conj().T @ R[(c, t)]
        return out

    dd = {(c, t): d[c, t, 0].reshape(-1) for c in range(nc) for t in range(nt)}
    X = EHop(dd)
    Lp = X.copy()
    S = np.zeros_like(X)
    for _ in range(3):
        U, sv, Vh = np.linalg.svd(X - S, full_matrices=False)
        hat = np.maximum(sv - lamL * sv[0], 0)
        tgt = hat - lamp * (hat - sprev)
        tgt[sv <= 1e-3 * sv[0]] = 0
        Ln = (U * tgt) @ Vh
        Z = T @ (X - Lp)
        thr = lamS * (1 - w[:, 0].reshape(nt, n).T / 255.0)
        mag = np.abs(Z)
        Zs = np.where(mag > thr, Z * (1 - thr / np.where(mag > 0, mag, 1)), 0)
        S = T.T @ Zs
        Y = Ln + S
        R = {k: v - dd[k] for k, v in Eop(Y).items()}
        X = Y - EHop(R)
        Lp = Ln
    r = oracle.solve(d, mask, sens, w, lamL, lamS, lambda_p=lamp, sigma_prev=sprev,
                     levels=1, iters=3)
    np.testing.assert_allclose(oracle.cas(r["L"]), Lp, atol=1e-13)
    np.testing.assert_allclose(oracle.cas(r["S"]), S, atol=1e-13)
    np.testing.assert_allclose(oracle.cas(r["M"]), X, atol=1e-13)


# ---------------------------------------------------------------- convergence sanity
def test_recovery_improves_on_zero_filled():
    """Reported, not pinned: on a small noisy problem the reconstruction beats the
    zero-filled adjoint in PSNR."""
    p = synth.small(nx=32, ny=32, nz=1, nt=10, nc=1, accel=3, seed=4, rank=2, nblobs=4)
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, 0.01, 0.01, levels=2, iters=30)
    zf = oracle.EH(p.kspace, p.mask, p.sens)
    assert oracle.psnr(r["X"], p.X_true) > oracle.psnr(zf, p.X_true) + 1.0


# ---- the temporal Fourier sparsifying transform (tfft) ------------------------------------
def test_tfft_is_the_unitary_dft_along_frames():
    # against the DFT matrix written out from its definition, and unitarity
    rng = np.random.default_rng(41)
    nt = 5
    x = rng.standard_normal((nt, 2, 3, 4)) + 1j * rng.standard_normal((nt, 2, 3, 4))
    f = np.arange(nt)
    Fm = np.exp(-2j * np.pi * np.outer(f, f) / nt) / np.sqrt(nt)
    want = np.einsum("ft,tzyx->fzyx", Fm, x)
    np.testing.assert_allclose(oracle.tfft_fwd(x), want, atol=1e-13)
    np.testing.assert_allclose(oracle.tfft_inv(want), x, atol=1e-13)
    assert np.linalg.norm(oracle.tfft_fwd(x)) == pytest.approx(np.linalg.norm(x), rel=1e-13)


def test_tfft_sparse_step_keeps_a_single_temporal_frequency():
    # a voxel series that is one complex exponential has one nonzero coefficient, of
    # magnitude sqrt(nt) |a|; the soft threshold shrinks it by tau and leaves the frequency
    nt = 8
    t = np.arange(nt)[:, None, None, None]
    a, k = 0.7 - 0.2j, 3
    X = a * np.exp(2j * np.pi * k * t / nt) * np.ones((1, 1, 2, 2))
    S, Zs = oracle.sparse_step(X, np.zeros_like(X), None, 0.1, 0, transform="tfft")
    mag = np.sqrt(nt) * abs(a)
    assert np.count_nonzero(np.abs(Zs) > 1e-12) == 4
    np.testing.assert_allclose(np.abs(Zs[k]), mag - 0.1, atol=1e-12)
    np.testing.assert_allclose(S, X * (mag - 0.1) / mag, atol=1e-12)


def test_tfft_full_weight_prior_passes_everything():
    rng = np.random.default_rng(42)
    X = rng.standard_normal((6, 1, 4, 4)) + 1j * rng.standard_normal((6, 1, 4, 4))
    w = np.full(X.shape, 255, np.uint8)
    S, _ = oracle.sparse_step(X, 0 * X, w, 5.0, 0, transform="tfft")
    np.testing.assert_allclose(S, X, atol=1e-12)


# ---- the Daubechies-4 wavelet (db4), standard decomposition, periodic ----------------------
def test_db4_filter_taps_and_identities():
    # the published four-tap Daubechies scaling filter, and the identities that make the
    # two-channel bank orthonormal with two vanishing moments
    np.testing.assert_allclose(oracle.DB4_H, [0.48296291314453416, 0.83651630373780794,
                                              0.22414386804201339, -0.12940952255126037],
                               atol=1e-15)
    h, g = oracle.DB4_H, oracle.DB4_G
    assert h.sum() == pytest.approx(np.sqrt(2.0), abs=1e-15)
    assert (h * h).sum() == pytest.approx(1.0, abs=1e-15)
    assert h[0] * h[2] + h[1] * h[3] == pytest.approx(0.0, abs=1e-16)   # even shifts orthogonal
    assert (g * g).sum() == pytest.approx(1.0, abs=1e-15)
    assert (h * g).sum() == pytest.approx(0.0, abs=1e-16)
    assert h[0] * g[2] + h[1] * g[3] == pytest.approx(0.0, abs=1e-16)
    m = np.arange(4)
    assert g.sum() == pytest.approx(0.0, abs=1e-15)                     # vanishing moment 0
    assert (m * g).sum() == pytest.approx(0.0, abs=1e-15)               # vanishing moment 1
    assert (m * m * g).sum() != pytest.approx(0.0, abs=1e-3)            # but not moment 2


@pytest.mark.parametrize("shape,J", [((1, 1, 8), 1), ((1, 1, 16), 2), ((1, 4, 8), 1),
                                     ((4, 8, 8), 2), ((2, 8, 16), 1)])
def test_db4_orthonormal(shape, J):
    # the transform matrix built column by column is unitary (real orthogonal), so the
    # inverse is its adjoint and energy is kept
    rng = np.random.default_rng(44 + J)
    n = int(np.prod(shape))
    T = np.stack([oracle.db4_fwd(np.eye(n)[k].reshape(shape), J).reshape(-1)
                  for k in range(n)], 1)
    np.testing.assert_allclose(T.conj().T @ T, np.eye(n), atol=1e-13)
    x = rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)
    c = oracle.db4_fwd(x, J)
    np.testing.assert_allclose(oracle.db4_inv(c, J), x, atol=1e-13)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-13)


def test_db4_vanishing_moments_on_a_ramp():
    # a linear ramp along x: every detail coefficient whose four-tap window does not wrap
    # around the periodic boundary is zero; a constant has no detail at all and its
    # approximation is sqrt(2) times the constant
    n = 16
    xs = np.arange(n, dtype=float)
    ramp = (0.3 - 0.2j) + (0.05 + 0.01j) * xs
    c = oracle.db4_fwd(ramp.reshape(1, 1, 1, n), 1)[0, 0, 0]
    d = c[n // 2:]
    np.testing.assert_allclose(d[: n // 2 - 1], 0.0, atol=1e-14)
    assert abs(d[-1]) > 1e-3                                           # the wrapped window
    k = np.full((1, 1, 1, n), 2.5 - 1.0j)
    c = oracle.db4_fwd(k, 1)[0, 0, 0]
    np.testing.assert_allclose(c[n // 2:], 0.0, atol=1e-14)
    np.testing.assert_allclose(c[: n // 2], np.sqrt(2.0) * (2.5 - 1.0j), atol=1e-14)


def test_db4_one_level_matches_the_filter_bank_definition():
    # one level along a periodic axis of length 8, written out as the analysis matrix:
    # row k of the low half holds h_m at column (2k + m) mod 8, of the high half g_m
    n = 8
    A = np.zeros((n, n))
    for k in range(n // 2):
        for m in range(4):
            A[k, (2 * k + m) % n] += oracle.DB4_H[m]
            A[n // 2 + k, (2 * k + m) % n] += oracle.DB4_G[m]
    rng = np.random.default_rng(45)
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    np.testing.assert_allclose(oracle.db4_fwd(u.reshape(1, 1, 1, n), 1)[0, 0, 0], A @ u,
                               atol=1e-14)


def test_db4_standard_decomposition_is_separable():
    # a separable volume f(z) g(y) h(x) transforms to the outer product of the three 1D
    # transforms (each axis decomposed fully, independently of the others)
    rng = np.random.default_rng(46)
    nz, ny, nx, J = 8, 16, 8, 2
    f = rng.standard_normal(nz) + 1j * rng.standard_normal(nz)
    g = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    h = rng.standard_normal(nx) + 1j * rng.standard_normal(nx)
    vol = f[:, None, None] * g[None, :, None] * h[None, None, :]
    c = oracle.db4_fwd(vol[None], J)[0]
    F = oracle.db4_fwd(f.reshape(1, 1, 1, nz), J)[0, 0, 0]
    G = oracle.db4_fwd(g.reshape(1, 1, 1, ny), J)[0, 0, 0]
    H = oracle.db4_fwd(h.reshape(1, 1, 1, nx), J)[0, 0, 0]
    np.testing.assert_allclose(c, F[:, None, None] * G[None, :, None] * H[None, None, :],
                               atol=1e-13)


def test_db4_sparse_step_limits():
    # lambda_S = 0 keeps X - L_prev; a threshold above every coefficient gives S = 0; a
    # full-weight prior passes everything through
    rng = np.random.default_rng(47)
    X = rng.standard_normal((3, 4, 8, 8)) + 1j * rng.standard_normal((3, 4, 8, 8))
    L = 0.3 * X
    S, _ = oracle.sparse_step(X, L, None, 0.0, 2, transform="db4")
    np.testing.assert_allclose(S, X - L, atol=1e-13)
    S, Zs = oracle.sparse_step(X, L, None, 1e6, 2, transform="db4")
    assert np.abs(S).max() == 0.0 and np.abs(Zs).max() == 0.0
    w = np.full(X.shape, 255, np.uint8)
    S, _ = oracle.sparse_step(X, L, w, 5.0, 2, transform="db4")
    np.testing.assert_allclose(S, X - L, atol=1e-13)


# ---- PSNR (Section 4's quality measure, magnitude images) ---------------------------------
def test_psnr_closed_forms():
    rng = np.random.default_rng(43)
    ref = rng.standard_normal((3, 2, 5, 7)) + 1j * rng.standard_normal((3, 2, 5, 7))
    peak = np.abs(ref).max()
    n = ref.size
    # every magnitude raised by delta (phase kept): MSE = delta^2
    delta = 0.0125
    x = ref * (1.0 + delta / np.abs(ref))
    assert oracle.psnr(x, ref) == pytest.approx(20 * np.log10(peak / delta), rel=1e-12)
    # magnitude images: a change of phase alone costs nothing, so it leaves the value
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, ref.shape))
    assert oracle.psnr(x * ph, ref) == pytest.approx(20 * np.log10(peak / delta), rel=1e-12)
    # one voxel off by e in magnitude: MSE = e^2 / n; the peak is the reference's, so a
    # change at the reference's brightest voxel keeps it
    k = int(np.argmax(np.abs(ref)))
    e = 0.3
    y = ref.copy().ravel()
    y[k] *= (1.0 + e / abs(y[k]))
    y = y.reshape(ref.shape)
    assert oracle.psnr(y, ref) == pytest.approx(10 * np.log10(peak ** 2 * n / e ** 2), rel=1e-12)
    # half the magnitudes everywhere: MSE = mean(|ref|^2) / 4
    want = 10 * np.log10(peak ** 2 / (np.mean(np.abs(ref) ** 2) / 4))
    assert oracle.psnr(0.5 * ref, ref) == pytest.approx(want, rel=1e-12)
