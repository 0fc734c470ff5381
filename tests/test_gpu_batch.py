"""Batches (prior_ls_batch_*): several problems of one geometry advanced with one launch per
kernel.  Each problem of a batch must produce bit for bit what it produces alone (the same
kernels on its own arrays, the same reduction orders), stop where it stops alone, and match
the FP64 oracle to the tolerance of the single-problem parity tests."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

TOL = 1e-4
KEYS = ("L", "S", "X", "M")

# (name, geometry, Haar levels, transform): 2D single coil, 3D multi-coil, ragged plane
# batches, the temporal transform
GEOMS = [
    ("2d_32x32_nt8_nc1", dict(nx=32, ny=32, nz=1, nt=8, nc=1), 2, "haar"),
    ("3d_32x48x8_nt12_nc3", dict(nx=32, ny=48, nz=8, nt=12, nc=3), 2, "haar"),
    ("3d_24x24x4_nt20_nc2_tfft", dict(nx=24, ny=24, nz=4, nt=20, nc=2), 1, "tfft"),
    ("3d_16x32x14_nt6_nc2", dict(nx=16, ny=32, nz=14, nt=6, nc=2), 1, "haar"),
]


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problems(geom, J, count, seed0, tf="haar"):
    # the temporal transform runs without Haar-footprint priors (as its own parity tests)
    extra = dict(prior=False, lambda_S=0.02) if tf == "tfft" else dict(levels=J)
    return [synth.small(**geom, accel=3, rank=2, nblobs=3, seed=seed0 + k, **extra)
            for k in range(count)]


def params_for(p, **kw):
    a = dict(lambda_L=p.lambda_L, lambda_S=p.lambda_S, max_iter=6, check_every=3)
    a.update(kw)
    return a


def solo(p, J, tf, **kw):
    with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, transform=tf) as h:
        t = pls.to_device(p)
        return h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], **params_for(p, **kw))


def batch_solve(ps, J, tf, kws):
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, transform=tf) for p in ps]
    try:
        with pls.Batch(hs) as b:
            prm = [pls.make_params(**params_for(p, **kw)) for p, kw in zip(ps, kws)]
            outs, sts = b.solve([pls.to_device(p) for p in ps], prm)
    finally:
        for h in hs:
            h.close()
    return outs, sts


@pytest.mark.parametrize("geom", GEOMS, ids=[g[0] for g in GEOMS])
def test_batch_equals_each_problem_alone_and_the_oracle(geom):
    name, g, J, tf = geom
    ps = problems(g, J, 3, 40, tf)
    kws = [dict(), dict(max_iter=4, check_every=2), dict(max_iter=7, check_every=7)]
    outs, sts = batch_solve(ps, J, tf, kws)
    for k, (p, kw) in enumerate(zip(ps, kws)):
        o1, s1 = solo(p, J, tf, **kw)
        for key in KEYS:
            assert torch.equal(outs[k][key], o1[key]), (k, key)
        assert sts[k]["iters"] == s1["iters"] == params_for(p, **kw)["max_iter"]
        assert sts[k]["resid_norm"] == s1["resid_norm"]
        assert sts[k]["nuclear_norm"] == s1["nuclear_norm"]
    # the first problem against the FP64 oracle
    p = ps[0]
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=J,
                     iters=6, transform=tf)
    for key in KEYS:
        e = rel(host(outs[0][key]), r[key])
        assert e < TOL, (key, e)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_batch_gram_modes_equal_each_problem_alone(mode):
    name, g, J, tf = GEOMS[1]
    ps = problems(g, J, 2, 140)
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, gram_mode=mode) for p in ps]
    try:
        with pls.Batch(hs) as b:
            prm = [pls.make_params(**params_for(p)) for p in ps]
            outs, sts = b.solve([pls.to_device(p) for p in ps], prm)
    finally:
        for h in hs:
            h.close()
    for k, p in enumerate(ps):
        with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, gram_mode=mode) as h:
            t = pls.to_device(p)
            o1, s1 = h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], **params_for(p))
        for key in KEYS:
            assert torch.equal(outs[k][key], o1[key]), (mode, k, key)


def test_batch_stops_each_problem_where_it_stops_alone():
    name, g, J, tf = GEOMS[1]
    ps = problems(g, J, 3, 60)
    # a tolerance that the first problem meets early (its relative change after 8
    # iterations): find where it stops alone, then batch it beside problems that run to
    # their iteration limits with other check intervals
    _, s8 = solo(ps[0], J, tf, max_iter=8, check_every=4)
    tol = s8["rel_change"] * 1.001
    o0, s0 = solo(ps[0], J, tf, max_iter=40, check_every=4, tol=tol)
    assert s0["converged"] == 1 and s0["iters"] <= 8
    kws = [dict(max_iter=40, check_every=4, tol=tol), dict(max_iter=9, check_every=5),
           dict(max_iter=13, check_every=13)]
    outs, sts = batch_solve(ps, J, tf, kws)
    assert sts[0]["converged"] == 1 and sts[0]["iters"] == s0["iters"]
    for key in KEYS:
        assert torch.equal(outs[0][key], o0[key]), key
    assert sts[1]["iters"] == 9 and sts[2]["iters"] == 13
    for k in (1, 2):
        o1, s1 = solo(ps[k], J, tf, **kws[k])
        for key in KEYS:
            assert torch.equal(outs[k][key], o1[key]), (k, key)


def test_batch_step_resumes_like_solve():
    name, g, J, tf = GEOMS[0]
    ps = problems(g, J, 4, 80)
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, transform=tf) for p in ps]
    try:
        with pls.Batch(hs) as b:
            prm = [pls.make_params(**params_for(p, max_iter=4, check_every=2)) for p in ps]
            b.solve([pls.to_device(p) for p in ps], prm, outputs=())
            outs, sts = b.step(5)
    finally:
        for h in hs:
            h.close()
    for k, p in enumerate(ps):
        o1, s1 = solo(p, J, tf, max_iter=9, check_every=2)
        assert sts[k]["iters"] == 9
        for key in KEYS:
            # 4 + 5 iterations chunked (2, 2 | 2, 2, 1) against (2, 2, 2, 2, 1): the same
            # iterations, so the same bits
            assert torch.equal(outs[k][key], o1[key]), (k, key)


def test_batch_step_from_different_iteration_counts():
    # problems solved for 4 and 5 iterations hold their iterates at different indices; a
    # batched step takes each from its own and equals solving for the total alone
    name, g, J, tf = GEOMS[1]
    ps = problems(g, J, 3, 120)
    counts = [4, 5, 7]
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, transform=tf) for p in ps]
    try:
        for h, p, k in zip(hs, ps, counts):
            t = pls.to_device(p)
            h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], outputs=(),
                    **params_for(p, max_iter=k, check_every=2))
        with pls.Batch(hs) as b:
            outs, sts = b.step(3)
    finally:
        for h in hs:
            h.close()
    for k, (p, c) in enumerate(zip(ps, counts)):
        o1, s1 = solo(p, J, tf, max_iter=c + 3, check_every=2)
        assert sts[k]["iters"] == c + 3
        for key in KEYS:
            assert torch.equal(outs[k][key], o1[key]), (k, key)


def test_batch_rejects_incompatible_problems_and_reused_handles():
    # another plane, another Gram tile class (nt 8 against 20), another Haar depth: each
    # needs other kernel instances
    a = pls.PriorLS(32, 32, 1, 8, 1, wavelet_levels=2)
    others = [pls.PriorLS(32, 48, 1, 8, 1, wavelet_levels=2),
              pls.PriorLS(32, 32, 1, 20, 1, wavelet_levels=2),
              pls.PriorLS(32, 32, 1, 8, 1, wavelet_levels=1)]
    try:
        for o in others:
            with pytest.raises(pls.PriorLSError) as e:
                pls.Batch([a, o])
            assert e.value.status == pls.EINVAL
        with pytest.raises(pls.PriorLSError):
            pls.Batch([a, a])
    finally:
        a.close()
        for o in others:
            o.close()


# Problems of different geometry in one batch: one plane shape, transform and Gram tile class,
# different nx, nt and nc (each kernel is launched with the largest problem's grid)
MIXED = [
    ("haar_nt_le16", [dict(nx=32, ny=48, nz=8, nt=12, nc=3), dict(nx=16, ny=48, nz=8, nt=9, nc=1),
                      dict(nx=48, ny=48, nz=8, nt=16, nc=2)], 2, "haar"),
    ("haar_nt_17_32", [dict(nx=16, ny=32, nz=4, nt=30, nc=2), dict(nx=32, ny=32, nz=4, nt=17, nc=1),
                       dict(nx=24, ny=32, nz=4, nt=24, nc=4)], 1, "haar"),
    ("2d", [dict(nx=32, ny=64, nz=1, nt=8, nc=1), dict(nx=64, ny=64, nz=1, nt=16, nc=2)], 2, "haar"),
    ("tfft_one_nt", [dict(nx=24, ny=24, nz=4, nt=20, nc=2), dict(nx=48, ny=24, nz=4, nt=20, nc=1)],
     1, "tfft"),
]


@pytest.mark.parametrize("mix", MIXED, ids=[m[0] for m in MIXED])
def test_mixed_geometry_batch_equals_each_problem_alone(mix):
    name, geoms, J, tf = mix
    extra = dict(prior=False, lambda_S=0.02) if tf == "tfft" else dict(levels=J)
    ps = [synth.small(**g, accel=3, rank=2, nblobs=3, seed=300 + k, **extra)
          for k, g in enumerate(geoms)]
    kws = [dict(), dict(max_iter=4, check_every=2), dict(max_iter=7, check_every=7)][:len(ps)]
    outs, sts = batch_solve(ps, J, tf, kws)
    for k, (p, kw) in enumerate(zip(ps, kws)):
        o1, s1 = solo(p, J, tf, **kw)
        for key in KEYS:
            assert torch.equal(outs[k][key], o1[key]), (k, key)
        assert sts[k]["iters"] == s1["iters"] == params_for(p, **kw)["max_iter"]
        assert sts[k]["resid_norm"] == s1["resid_norm"]
        assert sts[k]["l1_weighted"] == s1["l1_weighted"]
    # the largest problem against the FP64 oracle
    k = max(range(len(ps)), key=lambda i: ps[i].nx * ps[i].nt * ps[i].nc)
    p = ps[k]
    r = oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=J,
                     iters=params_for(p, **kws[k])["max_iter"], transform=tf)
    for key in KEYS:
        e = rel(host(outs[k][key]), r[key])
        assert e < TOL, (key, e)


def test_mixed_geometry_batched_step_from_different_iteration_counts():
    name, geoms, J, tf = MIXED[0]
    ps = [synth.small(**g, accel=3, rank=2, nblobs=3, seed=320 + k, levels=J)
          for k, g in enumerate(geoms)]
    counts = [3, 6, 5]
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J) for p in ps]
    try:
        for h, p, c in zip(hs, ps, counts):
            t = pls.to_device(p)
            h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], outputs=(),
                    **params_for(p, max_iter=c, check_every=2))
        with pls.Batch(hs) as b:
            outs, sts = b.step(4)
    finally:
        for h in hs:
            h.close()
    for k, (p, c) in enumerate(zip(ps, counts)):
        o1, s1 = solo(p, J, tf, max_iter=c + 4, check_every=2)
        assert sts[k]["iters"] == c + 4
        for key in KEYS:
            assert torch.equal(outs[k][key], o1[key]), (k, key)


@pytest.mark.skip(reason="the batch autotuner was withdrawn: the process aborted (exit 134, no "
                         "GPU fault) in the destroy of a new handle after this test's tuned "
                         "batch, with no cause found; prior_ls_batch_tune is not exported")
def test_batch_tune_leaves_the_problems_loaded_and_the_bits_unchanged():
    # the batch autotuner changes only the sparse fork point and grid, neither of which
    # changes an iterate: after tuning, a batched step of 6 equals each problem solved alone
    name, g, J, tf = GEOMS[1]
    ps = problems(g, J, 3, 160)
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, transform=tf) for p in ps]
    try:
        with pls.Batch(hs) as b:
            prm = [pls.make_params(**params_for(p)) for p in ps]
            choice = b.tune([pls.to_device(p) for p in ps], prm)
            assert choice["sparse_fork"] in (0, 1) and choice["ms_per_iteration"] > 0
            outs, sts = b.step(6)
    finally:
        for h in hs:
            h.close()
    for k, p in enumerate(ps):
        o1, s1 = solo(p, J, tf)
        assert sts[k]["iters"] == 6
        for key in KEYS:
            assert torch.equal(outs[k][key], o1[key]), (k, key)
