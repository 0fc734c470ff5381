"""Seeded synthetic inputs for the Priori L+S reconstruction.

This module is a simulated scanner plus phantom generator.  It is shared by the
tests, the benchmark and the smoke check; it contains none of the
reconstruction's arithmetic (no soft-thresholding, no SVD, no wavelet transform,
no adjoint operator).  The only transform it applies is the scanner's forward
sampling of the phantom's k-space (a unitary 3D DFT of each coil image, masked),
which is how measured data come into being (Section 2 of the paper: the
measurement is the undersampled k-space of each volume plus complex Gaussian
noise of finite energy).

Layouts (user layout, x fastest):
  image arrays       [nt][nz][ny][nx]
  k-space            [nc][nt][nz][ny][nx]   (kz, ky, kx; unshifted, index 0 = DC)
  mask               [nt][nz][ny]           uint8, 1 = phase-encode line sampled for all kx
  coil sensitivities [nc][nz][ny][nx]       None when nc == 1 (unit coil)
  prior weights      [nt][nz][ny][nx]       uint8 q, weight q/255, canonical
                                            (Mallat) Haar coefficient layout

Workload recipe (the paper's real cardiac data are not available; these seeded
phantoms stand in for them):
  * background: rank-r, L = U diag(a) V^H with smooth orthonormal spatial maps U,
    orthonormal temporal bases V and a_i = 2^-(i-1)
  * dynamics: compact blobs (Gaussian in 2D, ellipsoidal Gaussian in 3D),
    truncated to zero beyond 3 sigma, moving on sinusoidal paths with sinusoidal
    intensity and a constant random phase
  * variable-density Cartesian phase-encode masks, fully sampled centre, density
    proportional to (1 - r)^2 on the normalised elliptical radius, kx fully read
  * coils: smooth complex Gaussians on a ring, normalised to sum-of-squares 1
  * prior support: Haar coefficients whose footprint meets the previous frame's
    true sparse support, with 5% of members removed and as many non-members added
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

MASTER_SEED = 14116206


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    nt: int
    nc: int
    levels: int                 # Haar levels J used for the prior-support footprint
    kspace: np.ndarray          # complex128 [nc][nt][nz][ny][nx], zero off the mask
    mask: np.ndarray            # uint8 [nt][nz][ny]
    sens: Optional[np.ndarray]  # complex128 [nc][nz][ny][nx] or None
    prior_w: Optional[np.ndarray]  # uint8 [nt][nz][ny][nx] (canonical Haar layout) or None
    L_true: np.ndarray          # complex128 [nt][nz][ny][nx]
    S_true: np.ndarray          # complex128 [nt][nz][ny][nx]
    sigma_true: np.ndarray      # float64 [rank] singular values of L_true (voxels x frames)
    lambda_L: float = 0.01
    lambda_S: float = 0.01
    lambda_p: float = 0.0
    iters: int = 50
    name: str = ""

    @property
    def X_true(self) -> np.ndarray:
        return self.L_true + self.S_true

    @property
    def shape(self):
        return (self.nt, self.nz, self.ny, self.nx)


def _rngs(seed: int, n: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def _cgauss(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def _signed_freq(n):
    """Frequency index k in [-n/2, n/2) of each unshifted DFT bin."""
    return np.fft.fftfreq(n) * n


def _lowpass(vol, sig):
    """Gaussian low-pass of complex volumes [..., nz, ny, nx] with per-axis sigma in px."""
    axes = (-3, -2, -1)
    spec = np.fft.fftn(vol, axes=axes)
    for ax, s in zip(axes, sig):
        n = vol.shape[ax]
        f = np.fft.fftfreq(n)
        g = np.exp(-2.0 * (math.pi * s * f) ** 2) if n > 1 else np.ones(1)
        shape = [1] * vol.ndim
        shape[ax] = n
        spec = spec * g.reshape(shape)
    return np.fft.ifftn(spec, axes=axes)


def background(rng, nx, ny, nz, nt, rank):
    """Rank-r background as an [nt][nz][ny][nx] array with known singular values."""
    N = nx * ny * nz
    maps = _cgauss(rng, (rank, nz, ny, nx))
    maps = _lowpass(maps, (nz / 16.0, ny / 16.0, nx / 16.0))
    U, _ = np.linalg.qr(maps.reshape(rank, N).T)          # N x r orthonormal
    V, _ = np.linalg.qr(_cgauss(rng, (nt, rank)))          # nt x r orthonormal
    a = 2.0 ** -np.arange(rank)
    cas = (U * a) @ V.conj().T                             # N x nt
    return np.ascontiguousarray(cas.T.reshape(nt, nz, ny, nx)), a


@dataclasses.dataclass
class _Blob:
    p0: np.ndarray      # (z, y, x) centre
    amp: np.ndarray     # motion amplitude (y, x)
    freq: float
    phase: float
    sig: np.ndarray     # (z, y, x) widths in px
    alpha: float
    g: float
    psi: float
    cphase: float


def _make_blobs(rng, nx, ny, nz, nt, nblobs, ellipsoid, peak_ref):
    # widths and motion amplitudes shrink with the field of view for small test shapes
    smax = max(1.0, min(ny, nx) / 12.0)
    blobs = []
    for _ in range(nblobs):
        if ellipsoid:
            sig = rng.uniform(2.0, 4.0, size=3)
        else:
            sig = np.array([2.0, 2.0, 2.0])
        sig = np.minimum(sig, smax)
        if nz == 1:
            sig[0] = 1.0
        else:
            sig[0] = min(sig[0], max(1.0, nz / 8.0))
        amp = np.minimum(rng.uniform(1.0, 4.0, size=2), smax)
        margin = 3.0 * sig[1:] + amp + 1.0
        p0 = np.empty(3)
        zlo, zhi = 3.0 * sig[0], nz - 1 - 3.0 * sig[0]
        p0[0] = rng.uniform(zlo, zhi) if (nz > 1 and zhi > zlo) else (nz - 1) / 2.0
        for k, n in ((1, ny), (2, nx)):
            lo, hi = margin[k - 1], n - 1 - margin[k - 1]
            p0[k] = rng.uniform(lo, hi) if hi > lo else (n - 1) / 2.0
        blobs.append(_Blob(p0=p0, amp=amp, freq=float(rng.integers(1, 3)),
                           phase=rng.uniform(0, 2 * math.pi), sig=sig,
                           alpha=rng.uniform(0.3, 0.5) * peak_ref,
                           g=float(rng.integers(1, 3)), psi=rng.uniform(0, 2 * math.pi),
                           cphase=rng.uniform(0, 2 * math.pi)))
    return blobs


def _render_blobs(blobs, t, nt, nx, ny, nz):
    """Sparse component of frame t (t may be -1 for the frame before the window)."""
    out = np.zeros((nz, ny, nx), np.complex128)
    for b in blobs:
        ang = 2 * math.pi * b.freq * t / nt + b.phase
        c = b.p0 + np.array([0.0, b.amp[0] * math.sin(ang), b.amp[1] * math.cos(ang)])
        inten = b.alpha * (1.0 + 0.5 * math.sin(2 * math.pi * b.g * t / nt + b.psi))
        lo = np.maximum(np.floor(c - 3 * b.sig).astype(int), 0)
        hi = np.minimum(np.ceil(c + 3 * b.sig).astype(int) + 1, [nz, ny, nx])
        if nz == 1:
            lo[0], hi[0] = 0, 1
        zz, yy, xx = np.meshgrid(np.arange(lo[0], hi[0]), np.arange(lo[1], hi[1]),
                                 np.arange(lo[2], hi[2]), indexing="ij")
        r2 = ((yy - c[1]) / b.sig[1]) ** 2 + ((xx - c[2]) / b.sig[2]) ** 2
        if nz > 1:
            r2 = r2 + ((zz - c[0]) / b.sig[0]) ** 2
        val = np.where(r2 <= 9.0, np.exp(-0.5 * r2), 0.0) * inten * np.exp(1j * b.cphase)
        out[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += val
    return out


def coils(rng, nx, ny, nz, nc):
    """Smooth complex Gaussian coil maps on a ring, normalised to sum |C_c|^2 = 1."""
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    fov = max(nx, ny)
    maps = np.empty((nc, nz, ny, nx), np.complex128)
    for c in range(nc):
        th = 2 * math.pi * c / nc + rng.uniform(-0.1, 0.1)
        cy = ny / 2 + 0.35 * fov * math.sin(th)
        cx = nx / 2 + 0.35 * fov * math.cos(th)
        cz = (nz - 1) / 2
        w = 0.3 * fov
        mag = np.exp(-(((y - cy) ** 2 + (x - cx) ** 2 + ((z - cz) * fov / max(nz, 1)) ** 2)
                       / (2 * w * w)))
        ky, kx = rng.uniform(-1.5, 1.5, size=2) * 2 * math.pi / fov
        ph = rng.uniform(0, 2 * math.pi) + ky * y + kx * x
        maps[c] = mag * np.exp(1j * ph)
    maps /= np.sqrt(np.sum(np.abs(maps) ** 2, axis=0, keepdims=True))
    return maps


def masks(rng, ny, nz, nt, accel, centre=None):
    """Variable-density Cartesian phase-encode masks [nt][nz][ny], uint8.

    The centre (low |k|) is fully sampled: `centre` = (cz, cy) box size, default
    (nz/8, ny/16) in 3D and 8 ky lines in 2D.  The remaining lines are drawn
    without replacement with probability proportional to (1 - r)^2 of the
    normalised elliptical radius, to a total of round(P / accel) per frame.
    """
    P = ny * nz
    target = int(round(P / accel))
    kz = _signed_freq(nz)[:, None]
    ky = _signed_freq(ny)[None, :]
    if centre is None:
        centre = (max(1, nz // 8), max(1, ny // 16)) if nz > 1 else (1, 8)
    cz, cy = centre
    in_centre = ((kz >= -(cz // 2)) & (kz < cz - cz // 2) &
                 (ky >= -(cy // 2)) & (ky < cy - cy // 2))
    r = np.sqrt((ky / (ny / 2.0)) ** 2 + ((kz / (nz / 2.0)) ** 2 if nz > 1 else 0 * kz))
    # a small floor keeps every line reachable (corners beyond r = 1 included)
    dens = np.clip(1.0 - r, 0.0, None) ** 2 + 1e-4
    out = np.zeros((nt, nz, ny), np.uint8)
    for t in range(nt):
        if target >= P:
            out[t] = 1
            continue
        m = in_centre.copy()
        need = target - int(m.sum())
        if need > 0:
            p = np.where(m, 0.0, dens).ravel()
            p = p / p.sum()
            pick = rng.choice(P, size=need, replace=False, p=p)
            m.ravel()[pick] = True
        out[t] = m
    return out


def footprint_support(S, levels):
    """Boolean support, in canonical (Mallat) Haar layout, of the coefficients whose
    footprint meets supp(S) for an image-domain array S of shape [nz][ny][nx].

    Pure index logic: at level j the footprint grid is the support any-pooled over
    2^j blocks on every transformed axis (axes of size > 1)."""
    nz, ny, nx = S.shape
    ax_n = [nz, ny, nx]
    active = [n > 1 for n in ax_n]
    supp = np.abs(S) > 0
    out = np.zeros(S.shape, bool)
    if levels == 0:
        return supp

    def pool(a, f):
        sh = []
        for n, act in zip(a.shape, active):
            sh += [n // f, f] if act else [n, 1]
        return a.reshape(sh).any(axis=(1, 3, 5))

    for j in range(1, levels + 1):
        f = 2 ** j
        grid = pool(supp, f)                 # footprint grid of level-j coefficients
        for band in range(1, 8):
            bits = [(band >> 2) & 1, (band >> 1) & 1, band & 1]   # (z, y, x): 1 = detail
            if any(b and not a for b, a in zip(bits, active)):
                continue
            sl = []
            for b, n, act in zip(bits, ax_n, active):
                if not act:
                    sl.append(slice(0, 1))
                else:
                    m = n // f
                    sl.append(slice(m, 2 * m) if b else slice(0, m))
            out[tuple(sl)] |= grid
    f = 2 ** levels
    sl = tuple(slice(0, n // f) if act else slice(0, 1) for n, act in zip(ax_n, active))
    out[sl] |= pool(supp, f)
    return out


def flip_support(rng, supp, frac=0.05):
    """Remove round(frac*|T|) members of the support and add as many non-members."""
    s = supp.ravel().copy()
    on = np.flatnonzero(s)
    off = np.flatnonzero(~s)
    k = int(round(frac * on.size))
    if k > 0:
        s[rng.choice(on, size=min(k, on.size), replace=False)] = False
        s[rng.choice(off, size=min(k, off.size), replace=False)] = True
    return s.reshape(supp.shape)


def sample(X, mask, sens):
    """Scanner simulation: masked unitary 3D DFT of every coil image, [nc][nt][nz][ny][nx]."""
    try:
        import scipy.fft as sfft
        import os
        workers = len(os.sched_getaffinity(0))
        fftn = lambda a: sfft.fftn(a, axes=(-3, -2, -1), norm="ortho", workers=workers)
    except Exception:  # pragma: no cover
        fftn = lambda a: np.fft.fftn(a, axes=(-3, -2, -1), norm="ortho")
    nt = X.shape[0]
    nc = 1 if sens is None else sens.shape[0]
    out = np.empty((nc,) + X.shape, np.complex128)
    for c in range(nc):
        img = X if sens is None else X * sens[c][None]
        out[c] = fftn(img) * mask[:, :, :, None]
    return out


def make_problem(nx, ny, nz, nt, nc, accel, snr_db, rank, nblobs, seed,
                 levels=2, ellipsoid=None, prior=True, lambda_L=0.01, lambda_S=0.01,
                 lambda_p=0.0, iters=50, name="", centre=None):
    """Build one seeded problem instance.  All arrays complex128 / uint8."""
    r_bg, r_blob, r_mask, r_coil, r_noise, r_flip = _rngs(seed, 6)
    if ellipsoid is None:
        ellipsoid = nz > 1
    L, a = background(r_bg, nx, ny, nz, nt, rank)
    peak = float(np.abs(L).max())
    blobs = _make_blobs(r_blob, nx, ny, nz, nt, nblobs, ellipsoid, peak)
    S = np.stack([_render_blobs(blobs, t, nt, nx, ny, nz) for t in range(nt)])
    scale = 1.0 / float(np.abs(L + S).max())
    L *= scale
    S *= scale
    sigma = a * scale
    m = masks(r_mask, ny, nz, nt, accel, centre)
    sens = coils(r_coil, nx, ny, nz, nc) if nc > 1 else None
    d = sample(L + S, m, sens)
    if snr_db is not None:
        sig_norm = np.linalg.norm(d)
        nsamp = int(m.sum()) * nx * nc
        noise = _cgauss(r_noise, d.shape) * m[None, :, :, :, None]
        noise *= sig_norm / (np.linalg.norm(noise) * 10 ** (snr_db / 20.0))
        d = d + noise
        del noise, nsamp
    w = None
    if prior:
        S_prev = _render_blobs(blobs, -1, nt, nx, ny, nz) * scale
        w = np.zeros((nt, nz, ny, nx), np.uint8)
        for t in range(nt):
            src = S_prev if t == 0 else S[t - 1]
            w[t] = np.where(flip_support(r_flip, footprint_support(src, levels)), 255, 0)
    return Problem(nx=nx, ny=ny, nz=nz, nt=nt, nc=nc, levels=levels, kspace=d, mask=m,
                   sens=sens, prior_w=w, L_true=L, S_true=S, sigma_true=sigma,
                   lambda_L=lambda_L, lambda_S=lambda_S, lambda_p=lambda_p,
                   iters=iters, name=name)


# The four single-solve workloads.  Shapes follow the workload descriptions:
#   c1  64x64 (2D) x 16 frames, 1 coil, 4x, rank 3 + 12 Gaussian blobs, 40 dB, 50 iterations
#   c2  128x128x16 x 24 frames, 1 coil, 8x, rank 5 + 40 ellipsoids, 35 dB, 100 iterations
#   c3  192x192x32 x 30 frames, 8 coils, 10x, rank 6 + 60 ellipsoids, 35 dB
#   c4  = c3 (solved with the split-precision Gram)
CONFIGS = {
    1: dict(nx=64, ny=64, nz=1, nt=16, nc=1, accel=4, snr_db=40.0, rank=3, nblobs=12,
            iters=50, name="c1 64x64 x16 1coil R4"),
    2: dict(nx=128, ny=128, nz=16, nt=24, nc=1, accel=8, snr_db=35.0, rank=5, nblobs=40,
            iters=100, name="c2 128x128x16 x24 1coil R8"),
    3: dict(nx=192, ny=192, nz=32, nt=30, nc=8, accel=10, snr_db=35.0, rank=6, nblobs=60,
            iters=30, name="c3 192x192x32 x30 8coil R10"),
    4: dict(nx=192, ny=192, nz=32, nt=30, nc=8, accel=10, snr_db=35.0, rank=6, nblobs=60,
            iters=30, name="c4 192x192x32 x30 8coil R10 bf16x3 Gram"),
}


def config(i: int, seed: Optional[int] = None, **over) -> Problem:
    kw = dict(CONFIGS[i])
    kw.update(over)
    s = MASTER_SEED * 10 + i if seed is None else seed
    return make_problem(seed=s, **kw)


def small(nx=16, ny=16, nz=4, nt=6, nc=2, accel=3, snr_db=40.0, rank=2, nblobs=3,
          seed=1, **kw) -> Problem:
    """A small instance for tests (a few tiles, ragged where the shape allows)."""
    return make_problem(nx=nx, ny=ny, nz=nz, nt=nt, nc=nc, accel=accel, snr_db=snr_db,
                        rank=rank, nblobs=nblobs, seed=seed, **kw)


@dataclasses.dataclass
class Sequence:
    """A recursive real-time acquisition: a first window of nt frames followed by
    n_append frames that arrive one at a time (all arrays complex128 / uint8)."""
    nx: int
    ny: int
    nz: int
    nt: int
    nc: int
    n_append: int
    kspace: np.ndarray          # [nc][nt + n_append][nz][ny][nx], zero off the mask
    mask: np.ndarray            # [nt + n_append][nz][ny]
    sens: Optional[np.ndarray]  # [nc][nz][ny][nx] or None
    L_true: np.ndarray          # [nt + n_append][nz][ny][nx]
    S_true: np.ndarray
    lambda_L: float = 0.01
    lambda_S: float = 0.01
    lambda_p: float = 0.0

    @property
    def X_true(self) -> np.ndarray:
        return self.L_true + self.S_true

    def first_window(self):
        """(kspace [nc][nt]..., mask [nt]...) of frames 0..nt-1."""
        return (np.ascontiguousarray(self.kspace[:, :self.nt]),
                np.ascontiguousarray(self.mask[:self.nt]))

    def frame(self, j):
        """(kspace [nc][nz][ny][nx], mask [nz][ny]) of appended frame j (0-based)."""
        f = self.nt + j
        return (np.ascontiguousarray(self.kspace[:, f]), np.ascontiguousarray(self.mask[f]))


def sequence(nx, ny, nz, nt, n_append, nc, accel, seed, accel_first=2.0, snr_db=40.0,
             rank=2, nblobs=3, lambda_L=0.01, lambda_S=0.01, lambda_p=0.0, centre=None):
    """A seeded sequence for the sliding-window recursion.  The first window is sampled
    at accel_first (the first time instance is densely sampled, 50% by default) and every
    appended frame at accel.  snr_db None gives noiseless data."""
    r_bg, r_blob, r_mask, r_coil, r_noise, r_first = _rngs(seed, 6)
    nf = nt + n_append
    L, a = background(r_bg, nx, ny, nz, nf, rank)
    peak = float(np.abs(L).max())
    blobs = _make_blobs(r_blob, nx, ny, nz, nf, nblobs, nz > 1, peak)
    S = np.stack([_render_blobs(blobs, t, nf, nx, ny, nz) for t in range(nf)])
    scale = 1.0 / float(np.abs(L + S).max())
    L *= scale
    S *= scale
    m = masks(r_mask, ny, nz, nf, accel, centre)
    m[:nt] = masks(r_first, ny, nz, nt, accel_first, centre)
    sens = coils(r_coil, nx, ny, nz, nc) if nc > 1 else None
    d = sample(L + S, m, sens)
    if snr_db is not None:
        noise = _cgauss(r_noise, d.shape) * m[None, :, :, :, None]
        noise *= np.linalg.norm(d) / (np.linalg.norm(noise) * 10 ** (snr_db / 20.0))
        d = d + noise
    return Sequence(nx=nx, ny=ny, nz=nz, nt=nt, nc=nc, n_append=n_append, kspace=d, mask=m,
                    sens=sens, L_true=L, S_true=S, lambda_L=lambda_L, lambda_S=lambda_S,
                    lambda_p=lambda_p)


def phantom(nx, ny, nz, nt, rank, nblobs, seed):
    """The phantom alone (L, S), complex128 [nt][nz][ny][nx], scaled to max |L + S| = 1:
    for workloads whose k-space is formed elsewhere (the serving stream)."""
    r_bg, r_blob = _rngs(seed, 2)
    L, _ = background(r_bg, nx, ny, nz, nt, rank)
    blobs = _make_blobs(r_blob, nx, ny, nz, nt, nblobs, nz > 1, float(np.abs(L).max()))
    S = np.stack([_render_blobs(blobs, t, nt, nx, ny, nz) for t in range(nt)])
    scale = 1.0 / float(np.abs(L + S).max())
    return L * scale, S * scale


# The serving stream: 64 recursive reconstruction requests, Poisson arrivals at 20 per
# second, sizes uniform over three volumes x three window lengths x three coil counts,
# acceleration uniform in [8, 12] for the appended frames, the first window at 50%;
# 8 appended frames per request.  Phantom per volume: rank / blobs as the single-solve
# workloads of that size.
SERVING = dict(n_requests=64, rate_per_s=20.0, n_append=8, accel_first=2.0, accel=(8.0, 12.0),
               volumes=((64, 64, 8), (128, 128, 16), (192, 192, 32)), nts=(16, 24, 30),
               ncs=(1, 4, 8), rank={64: 3, 128: 5, 192: 6}, nblobs={64: 12, 128: 40, 192: 60},
               snr_db=35.0, first_iters=50, append_iters=20)


def serving_requests(seed=MASTER_SEED * 10 + 5):
    """The request list of the serving stream: (arrival s, (nx, ny, nz), nt, nc, accel,
    first-window masks [nt][nz][ny], appended-frame masks [n_append][nz][ny])."""
    c = SERVING
    rng = np.random.default_rng(seed)
    n = c["n_requests"]
    gaps = rng.exponential(1.0 / c["rate_per_s"], size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        vol = c["volumes"][rng.integers(len(c["volumes"]))]
        nt = int(c["nts"][rng.integers(len(c["nts"]))])
        nc = int(c["ncs"][rng.integers(len(c["ncs"]))])
        accel = float(rng.uniform(*c["accel"]))
        nx, ny, nz = vol
        m0 = masks(rng, ny, nz, nt, c["accel_first"])
        mf = masks(rng, ny, nz, c["n_append"], accel)
        out.append((float(arrivals[i]), vol, nt, nc, accel, m0, mf))
    return out
