"""FP64 CPU oracle for the Priori L+S reconstruction (Zonoobi, Faghih Roohi, Kassim,
"Low-Rank and Sparse Matrix Decomposition with a-priori knowledge for Dynamic 3D
MRI reconstruction", arXiv 1411.6206).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously-correct
reference the GPU library is checked against.  Only the test-suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the library never
calls it, and it shares no code with the library.

Everything is complex128 / float64, numpy + LAPACK.  Every function names the
passage it follows.  Readings of points the paper leaves open are marked
"Reading:" and are listed, with their reasons, in the design notes.

Conventions (user layout, x fastest):
  X, L, S, M        complex [nt][nz][ny][nx]
  d (k-space)       complex [nc][nt][nz][ny][nx], entries off the mask ignored
  mask              uint8   [nt][nz][ny]   (phase-encode lines, broadcast over kx)
  sens              complex [nc][nz][ny][nx] or None (single unit coil)
  prior_w           uint8   [nt][nz][ny][nx] in T's canonical coefficient layout, w = q/255,
                    or None
"""
from __future__ import annotations

import numpy as np

SQRT_HALF = np.sqrt(0.5)


# --------------------------------------------------------------------------------------
# Section 2: the acquisition operator A (here E) and its adjoint (the paper writes the
# adjoint as A^{-1}, Notations paragraph).
# --------------------------------------------------------------------------------------
# The library call that evaluates the DFT: numpy.fft by default; set_fft_workers(n) with
# n > 1 evaluates the same unitary DFT with scipy.fft on n threads (for timing the oracle on
# many cores; the tests keep the default).
_FFT_WORKERS = None


def set_fft_workers(n):
    global _FFT_WORKERS
    _FFT_WORKERS = int(n) if n and int(n) > 1 else None


def fft3(x):
    """Unitary, unshifted 3D DFT over the last three axes (z, y, x); index 0 is DC."""
    if _FFT_WORKERS:
        import scipy.fft
        return scipy.fft.fftn(x, axes=(-3, -2, -1), norm="ortho", workers=_FFT_WORKERS)
    return np.fft.fftn(x, axes=(-3, -2, -1), norm="ortho")


def ifft3(x):
    """Inverse of fft3 (its adjoint, since it is unitary)."""
    if _FFT_WORKERS:
        import scipy.fft
        return scipy.fft.ifftn(x, axes=(-3, -2, -1), norm="ortho", workers=_FFT_WORKERS)
    return np.fft.ifftn(x, axes=(-3, -2, -1), norm="ortho")


def _mask5(mask):
    return mask.astype(bool)[None, :, :, :, None]


def E(X, mask, sens):
    """Frame-by-frame undersampled acquisition (Section 2): for coil c and frame t,
    E(X)[c, t] = m_t * F(C_c * X_t), with the phase-encode mask broadcast over kx."""
    X = np.asarray(X, np.complex128)
    coil_imgs = X[None] if sens is None else X[None] * sens[:, None]
    return fft3(coil_imgs) * _mask5(mask)


def EH(R, mask, sens):
    """Adjoint of E (Notations: A^{-1} denotes the adjoint):
    E^H(R)[t] = sum_c conj(C_c) * F^{-1}(m_t * R[c, t])."""
    imgs = ifft3(np.asarray(R, np.complex128) * _mask5(mask))
    if sens is None:
        return imgs[0]
    return np.sum(np.conj(sens)[:, None] * imgs, axis=0)


# --------------------------------------------------------------------------------------
# Section 2: the soft-thresholding operator S{x, lambda} = x/|x| max(|x| - lambda, 0),
# complex-aware, applied elementwise.  Reading: S{0, lambda} = 0.
# --------------------------------------------------------------------------------------
def soft(z, tau):
    z = np.asarray(z, np.complex128)
    mag = np.abs(z)
    shrunk = np.maximum(mag - tau, 0.0)
    scale = np.divide(shrunk, mag, out=np.zeros_like(mag), where=mag > 0)
    return z * scale


# --------------------------------------------------------------------------------------
# Sparsifying transform T (Section 2: "such as Wavelets"; Section 4: the sparse domain
# is the wavelet domain).  Reading: orthonormal Haar, nonstandard pyramid (one level
# along every spatial axis of size > 1, then recurse on the all-low band), J levels,
# applied per frame, coefficients in canonical Mallat layout.
# --------------------------------------------------------------------------------------
def _active_axes(shape3):
    return [ax for ax, n in zip((-3, -2, -1), shape3) if n > 1]


def haar_fwd(x, levels):
    """T: image [..., nz, ny, nx] -> Haar coefficients (same shape, canonical layout)."""
    c = np.array(x, np.complex128, copy=True)
    shape3 = c.shape[-3:]
    axes = _active_axes(shape3)
    for j in range(levels):
        ext = [n >> j if n > 1 else 1 for n in shape3]
        sl = (Ellipsis, slice(0, ext[0]), slice(0, ext[1]), slice(0, ext[2]))
        band = c[sl]
        for ax in axes:
            n = band.shape[ax]
            even = np.take(band, np.arange(0, n, 2), axis=ax)
            odd = np.take(band, np.arange(1, n, 2), axis=ax)
            band = np.concatenate([(even + odd) * SQRT_HALF, (even - odd) * SQRT_HALF], axis=ax)
        c[sl] = band
    return c


def haar_inv(c, levels):
    """T^{-1} = T^H (orthonormal): coefficients -> image."""
    x = np.array(c, np.complex128, copy=True)
    shape3 = x.shape[-3:]
    axes = _active_axes(shape3)
    for j in reversed(range(levels)):
        ext = [n >> j if n > 1 else 1 for n in shape3]
        sl = (Ellipsis, slice(0, ext[0]), slice(0, ext[1]), slice(0, ext[2]))
        band = x[sl]
        for ax in reversed(axes):
            n = band.shape[ax]
            lo = np.take(band, np.arange(0, n // 2), axis=ax)
            hi = np.take(band, np.arange(n // 2, n), axis=ax)
            out = np.empty_like(band)
            idx_e = [slice(None)] * band.ndim
            idx_o = [slice(None)] * band.ndim
            idx_e[ax] = slice(0, n, 2)
            idx_o[ax] = slice(1, n, 2)
            out[tuple(idx_e)] = (lo + hi) * SQRT_HALF
            out[tuple(idx_o)] = (lo - hi) * SQRT_HALF
            band = out
        x[sl] = band
    return x


# --------------------------------------------------------------------------------------
# A second sparsifying transform (Section 2 leaves T generic; the L+S method the paper builds
# on uses the temporal Fourier transform for cardiac series): the unitary DFT along the
# frames of every voxel.  Coefficient (f, z, y, x) is temporal frequency f of voxel (z,y,x).
# --------------------------------------------------------------------------------------
def tfft_fwd(x):
    return np.fft.fft(np.asarray(x, np.complex128), axis=0, norm="ortho")


def tfft_inv(c):
    return np.fft.ifft(np.asarray(c, np.complex128), axis=0, norm="ortho")


# --------------------------------------------------------------------------------------
# A third sparsifying transform: another wavelet family (Section 2, "such as Wavelets";
# Section 5 names other transforms as future work).  Reading: the orthonormal Daubechies
# wavelet with four taps (two vanishing moments), periodic extension, in the standard
# (tensor-product) decomposition: the full J-level 1D transform along x, then along y, then
# along z, every spatial axis of size > 1; coefficients in canonical Mallat order along each
# axis, [a_J | d_J | d_{J-1} | ... | d_1].
# Analysis: a_k = sum_m h_m u[(2k + m) mod n], d_k = sum_m g_m u[(2k + m) mod n], with
# g_m = (-1)^m h_{3-m}; synthesis is the adjoint (the filter bank is orthonormal).
# --------------------------------------------------------------------------------------
_S3 = np.sqrt(3.0)
DB4_H = np.array([1 + _S3, 3 + _S3, 3 - _S3, 1 - _S3]) / (4 * np.sqrt(2.0))
DB4_G = np.array([(-1) ** m * DB4_H[3 - m] for m in range(4)])


def _db4_step(u, axis):
    """One analysis level along `axis` (length n, even): returns [a | d] along that axis."""
    u = np.moveaxis(np.asarray(u, np.complex128), axis, -1)
    n = u.shape[-1]
    a = np.zeros(u.shape[:-1] + (n // 2,), np.complex128)
    d = np.zeros_like(a)
    for k in range(n // 2):
        for m in range(4):
            v = u[..., (2 * k + m) % n]
            a[..., k] += DB4_H[m] * v
            d[..., k] += DB4_G[m] * v
    return np.moveaxis(np.concatenate([a, d], axis=-1), -1, axis)


def _db4_step_inv(c, axis):
    """Adjoint of _db4_step: u[(2k + m) mod n] += h_m a_k + g_m d_k."""
    c = np.moveaxis(np.asarray(c, np.complex128), axis, -1)
    n = c.shape[-1]
    a, d = c[..., : n // 2], c[..., n // 2:]
    u = np.zeros_like(c)
    for k in range(n // 2):
        for m in range(4):
            u[..., (2 * k + m) % n] += DB4_H[m] * a[..., k] + DB4_G[m] * d[..., k]
    return np.moveaxis(u, -1, axis)


def db4_fwd(x, levels):
    """T: image [..., nz, ny, nx] -> coefficients (same shape), J levels along each axis."""
    c = np.array(x, np.complex128, copy=True)
    for ax in _active_axes(c.shape[-3:]):
        n = c.shape[ax]
        for j in range(levels):
            m = n >> j
            idx = [slice(None)] * c.ndim
            idx[ax] = slice(0, m)
            c[tuple(idx)] = _db4_step(c[tuple(idx)], ax)
    return c


def db4_inv(c, levels):
    """T^{-1} = T^H (orthonormal): coefficients -> image."""
    x = np.array(c, np.complex128, copy=True)
    for ax in reversed(_active_axes(x.shape[-3:])):
        n = x.shape[ax]
        for j in reversed(range(levels)):
            m = n >> j
            idx = [slice(None)] * x.ndim
            idx[ax] = slice(0, m)
            x[tuple(idx)] = _db4_step_inv(x[tuple(idx)], ax)
    return x


TRANSFORMS = ("haar", "tfft", "db4")


def T_fwd(x, levels, transform="haar"):
    if transform == "haar":
        return haar_fwd(x, levels)
    if transform == "db4":
        return db4_fwd(x, levels)
    return tfft_fwd(x)


def T_inv(c, levels, transform="haar"):
    if transform == "haar":
        return haar_inv(c, levels)
    if transform == "db4":
        return db4_inv(c, levels)
    return tfft_inv(c)


# --------------------------------------------------------------------------------------
# Casorati matrix.  Reading: rows = voxels of one volume, columns = the nt time frames
# (the L+S convention the paper builds on), so cas(X) is N x nt.
# --------------------------------------------------------------------------------------
def cas(X):
    nt = X.shape[0]
    return X.reshape(nt, -1).T


def uncas(C, shape):
    return np.ascontiguousarray(C.T.reshape(shape))


# --------------------------------------------------------------------------------------
# Algorithm 1, steps (1) and (2): singular-value soft-thresholding of X - S, then the
# gradient step that pulls the singular values toward those of L^(t-1).
# --------------------------------------------------------------------------------------
NULL_REL = 1e-3   # Reading: singular values <= 1e-3 sigma_1 are numerically null


def sv_targets(sigma, lambda_L, relative, lambda_p, sigma_prev):
    """Singular values after step (1) and step (2), paired in descending order.

    step (1): sigma_hat = S{sigma, tau_L}, tau_L = lambda_L * sigma_1 (relative) or lambda_L
    step (2): D = sigma_hat - sigma_prev; sigma_tilde = sigma_hat - lambda_p * D
    Reading: sigma_prev is zero-padded to the number of frames; components whose
    sigma <= 1e-3 sigma_1 are null (sigma_tilde = 0)."""
    sigma = np.asarray(sigma, np.float64)
    n = sigma.size
    s1 = sigma[0] if n else 0.0
    tau = lambda_L * s1 if relative else lambda_L
    sig_hat = np.maximum(sigma - tau, 0.0)
    prev = np.zeros(n)
    if sigma_prev is not None and lambda_p != 0.0:
        sp = np.sort(np.asarray(sigma_prev, np.float64))[::-1][:n]
        prev[:sp.size] = sp
    D = sig_hat - prev
    sig_t = sig_hat - lambda_p * D
    sig_t = np.where(sigma <= NULL_REL * s1, 0.0, sig_t)
    return sig_t, tau


def svt(C, lambda_L, relative=True, lambda_p=0.0, sigma_prev=None):
    """Steps (1)-(2) on a Casorati matrix C (N x nt) with a LAPACK thin SVD.
    Returns (L, sigma, sigma_tilde, tau_L)."""
    U, sigma, Vh = np.linalg.svd(C, full_matrices=False)
    sig_t, tau = sv_targets(sigma, lambda_L, relative, lambda_p, sigma_prev)
    return (U * sig_t) @ Vh, sigma, sig_t, tau


def svt_gram(C, lambda_L, relative=True, lambda_p=0.0, sigma_prev=None):
    """The same steps through the Gram matrix G = C^H C = V diag(sigma^2) V^H:
    L = C W with W = V diag(sigma_tilde / sigma) V^H (FP64 eigh).  Mathematically equal
    to svt() whenever the singular values are distinct from the threshold."""
    G = C.conj().T @ C
    lam, V = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    sigma = np.sqrt(np.maximum(lam, 0.0))
    sig_t, tau = sv_targets(sigma, lambda_L, relative, lambda_p, sigma_prev)
    phi = np.divide(sig_t, sigma, out=np.zeros_like(sigma), where=sigma > 0)
    W = (V * phi) @ V.conj().T
    return C @ W, sigma, sig_t, tau


# --------------------------------------------------------------------------------------
# Algorithm 1, step (3): shrink the sparsifying-transform coefficients that lie outside
# the a-priori support T^(t-1); coefficients on it pass through unshrunk.
# Reading: the argument is X_{it-1} - L_{it-1} (the L+S sparse update the paper follows;
# the literal T(S_{it-1}) would never see the data), and the support indicator is
# generalised to a weight w in [0, 1] giving the threshold lambda_S (1 - w).
# --------------------------------------------------------------------------------------
def sparse_step(M_prev, L_prev, prior_w, lambda_S, levels, transform="haar"):
    Z = T_fwd(M_prev - L_prev, levels, transform)
    w = 0.0 if prior_w is None else prior_w.astype(np.float64) / 255.0
    tau = lambda_S * (1.0 - w)
    Zs = soft(Z, tau)
    return T_inv(Zs, levels, transform), Zs


# --------------------------------------------------------------------------------------
# Algorithm 1, step (4): data consistency, X = L + S - A^{-1}(A(L + S) - d).
# --------------------------------------------------------------------------------------
def dc_step(Y, d, mask, sens):
    R = E(Y, mask, sens) - np.asarray(d, np.complex128) * _mask5(mask)
    return Y - EH(R, mask, sens), R


def solve(d, mask, sens, prior_w, lambda_L, lambda_S, lambda_p=0.0, sigma_prev=None,
          levels=2, iters=50, tol=0.0, L0=None, S0=None, lambda_L_relative=True,
          svt_fn=None, transform="haar", on_iteration=None):
    """Algorithm 1 (Priori L+S), step by step, for `iters` iterations or until the
    relative change of the solution drops below tol (Section 3, stopping rule).

    Initialisation, step (0): X_0 = A^{-1}(d), S_0 = 0.  Reading: L_0 = X_0, so the
    first sparse update sees X_0 - L_0 = 0.  A warm start (L0, S0) instead takes
    X_0 = Y - A^{-1}(A(Y) - d) with Y = L0 + S0 (one data-consistency step).

    Returns a dict with L, S, X = L + S, M (the data-consistent iterate X_it),
    per-iteration statistics, and what the next time instance takes as a-priori
    knowledge (Section 3): supp, 255 on the support of T(S) (the coefficients that survive
    the last shrinkage, canonical layout; all 0 when no iteration ran) and sigma_L, the
    singular values of the returned L (descending; zeros when no iteration ran).
    on_iteration (optional) is called with 0 once the set-up is done and with k after
    iteration k (timing only; it sees nothing of the state)."""
    svt_fn = svt if svt_fn is None else svt_fn
    d = np.asarray(d, np.complex128)
    shape = d.shape[1:]
    if L0 is None:
        M = EH(d * _mask5(mask), mask, sens)
        L = M.copy()
        S = np.zeros(shape, np.complex128)
    else:
        L = np.asarray(L0, np.complex128).copy()
        S = np.asarray(S0, np.complex128).copy()
        M, _ = dc_step(L + S, d, mask, sens)
    w = None if prior_w is None else prior_w.astype(np.float64) / 255.0
    hist = dict(rel_change=[], resid=[], nuclear=[], l1w=[], objective=[], sigma=[], tau_L=[])
    supp = np.zeros(shape, np.uint8)
    sigma_L = np.zeros(shape[0])
    it = 0
    if on_iteration is not None:
        on_iteration(0)
    for it in range(1, iters + 1):
        Y_prev = L + S
        # step (1) + (2)
        Lc, sigma, sig_t, tau_L = svt_fn(cas(M - S), lambda_L, lambda_L_relative,
                                         lambda_p, sigma_prev)
        L_new = uncas(Lc, shape)
        # step (3)
        S_new, Zs = sparse_step(M, L, prior_w, lambda_S, levels, transform)
        L, S = L_new, S_new
        supp = np.where(Zs != 0, 255, 0).astype(np.uint8)
        sigma_L = sig_t
        # step (4)
        Y = L + S
        M, R = dc_step(Y, d, mask, sens)
        # statistics
        den = np.linalg.norm(Y_prev)
        rel = np.linalg.norm(Y - Y_prev) / den if den > 0 else np.inf
        resid = np.linalg.norm(R)
        nuc = float(np.sum(sig_t))
        l1w = float(np.sum(np.abs(Zs) * (1.0 if w is None else (1.0 - w))))
        hist["rel_change"].append(rel)
        hist["resid"].append(resid)
        hist["nuclear"].append(nuc)
        hist["l1w"].append(l1w)
        hist["objective"].append(0.5 * resid ** 2 + tau_L * nuc + lambda_S * l1w)
        hist["sigma"].append(sigma)
        hist["tau_L"].append(tau_L)
        if on_iteration is not None:
            on_iteration(it)
        if tol > 0 and rel < tol:
            break
    return dict(L=L, S=S, X=L + S, M=M, iters=it, supp=supp, sigma_L=np.asarray(sigma_L),
                **{k: np.array(v) for k, v in hist.items()})


# --------------------------------------------------------------------------------------
# The priori L+S scheme over a time sequence (Section 3, Fig. 2): each time instance is
# reconstructed by Algorithm 1 with the previous instance's L and S as a-priori knowledge;
# the first instance uses plain L+S (solve() with no weights and lambda_p = 0).
# Reading: a time instance is a window of nt frames that slides by one frame, so the new
# window shares nt - 1 frames with the previous one, and
#   * data and masks drop the oldest frame and take the new one last;
#   * the support prior T^(t-1) and the singular values Sigma(L^(t-1)) are those of the
#     previous window's result, its support map shifted with the frames and the new frame
#     given the previous last frame's support (adjacent frames share their support);
#   * the iteration is warm-started from the previous L and S, shifted the same way (the
#     new frame starts from the previous last frame).
# --------------------------------------------------------------------------------------
def shift_window(a, new):
    """Frames 1..nt-1 of a (axis 0) followed by `new` (one frame)."""
    return np.concatenate([np.asarray(a)[1:], np.asarray(new)[None]], axis=0)


def append_frame(prev, d, mask, sens, d_new, mask_new, lambda_L, lambda_S, lambda_p=0.0,
                 levels=2, iters=20, tol=0.0, lambda_L_relative=True, transform="haar"):
    """One step of the sequence: prev is the result of solve() (or append_frame) for the
    window (d, mask); d_new [nc][nz][ny][nx] and mask_new [nz][ny] are the new frame.
    Returns (result of the new window, its data, its mask).
    Reading: with the temporal Fourier transform a coefficient is a temporal frequency of
    the whole window, not a frame, and sliding the window by one frame changes the phase of
    the spectrum, not its magnitude; its support prior is taken over unshifted."""
    d_next = np.concatenate([np.asarray(d)[:, 1:], np.asarray(d_new)[:, None]], axis=1)
    mask_next = shift_window(mask, mask_new)
    L0 = shift_window(prev["L"], prev["L"][-1])
    S0 = shift_window(prev["S"], prev["S"][-1])
    if transform in ("haar", "db4"):
        w = shift_window(prev["supp"], prev["supp"][-1])
    else:
        w = np.array(prev["supp"], copy=True)
    r = solve(d_next, mask_next, sens, w, lambda_L, lambda_S, lambda_p=lambda_p,
              sigma_prev=prev["sigma_L"], levels=levels, iters=iters, tol=tol, L0=L0, S0=S0,
              lambda_L_relative=lambda_L_relative, transform=transform)
    return r, d_next, mask_next


def plain_ls(d, mask, sens, lambda_L, lambda_S, levels=2, iters=50):
    """The L+S method without priors (the paper's starting point and its t = 1 case):
    written separately from solve() so that solve() with zero prior weights and
    lambda_p = 0 can be checked against it."""
    d = np.asarray(d, np.complex128) * _mask5(mask)
    nt = d.shape[1]
    X = EH(d, mask, sens)
    Lpre = X.copy()
    S = np.zeros_like(X)
    for _ in range(iters):
        U, sv, Vh = np.linalg.svd(X.reshape(nt, -1).T - S.reshape(nt, -1).T,
                                  full_matrices=False)
        thr = lambda_L * sv[0]
        keep = np.where(sv > 1e-3 * sv[0], np.maximum(sv - thr, 0.0), 0.0)
        Lmat = (U * keep) @ Vh
        Lnew = np.ascontiguousarray(Lmat.T.reshape(X.shape))
        coef = haar_fwd(X - Lpre, levels)
        mag = np.abs(coef)
        coef = np.where(mag > lambda_S, coef * (1.0 - lambda_S / np.where(mag > 0, mag, 1.0)), 0)
        S = haar_inv(coef, levels)
        Y = Lnew + S
        resk = E(Y, mask, sens) - d
        X = Y - EH(resk, mask, sens)
        Lpre = Lnew
    return dict(L=Lpre, S=S, X=Lpre + S, M=X)


def psnr(x, ref):
    """Peak signal-to-noise ratio (Section 4) of magnitude images, in dB."""
    mse = np.mean(np.abs(np.abs(x) - np.abs(ref)) ** 2)
    peak = np.max(np.abs(ref))
    return 10.0 * np.log10(peak ** 2 / mse)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
