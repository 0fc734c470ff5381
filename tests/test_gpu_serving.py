"""GPU tests of the serving runtime (prior_ls_server_*): a sequence served matches the FP64
oracle's recursion; every sequence gives the same result alone and in a mix of concurrent
sequences of other shapes; admission never holds more than the HBM budget."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1411_6206_amd as pls  # noqa: E402

GEOMS = [dict(nx=16, ny=16, nz=4, nt=5, nc=2, accel=3),
         dict(nx=24, ny=32, nz=8, nt=7, nc=3, accel=4),
         dict(nx=32, ny=32, nz=1, nt=6, nc=1, accel=4)]
K0, K1, LAM_P = 8, 6, 0.3


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def make_request(i, n_append):
    g = dict(GEOMS[i % len(GEOMS)])
    q = synth.sequence(n_append=n_append, seed=100 + i, **g)
    d0, m0 = q.first_window()
    frames = [q.frame(j) for j in range(n_append)]
    args = dict(kspace0=_dev(d0, torch.complex64), mask0=_dev(m0, torch.uint8),
                kspace_frames=_dev(np.stack([f[0] for f in frames]), torch.complex64),
                mask_frames=_dev(np.stack([f[1] for f in frames]), torch.uint8),
                sens=None if q.sens is None else _dev(q.sens, torch.complex64))
    dims = pls.make_dims(q.nx, q.ny, q.nz, q.nt, q.nc, 2, "fp64")
    return q, dims, args


def submit(srv, dims, args):
    return srv.submit(dims, first=pls.make_params(max_iter=K0, check_every=4),
                      append_params=pls.make_params(lambda_p=LAM_P, max_iter=K1, check_every=4),
                      **args)


def test_served_sequence_matches_oracle():
    q, dims, args = make_request(0, n_append=3)
    with pls.Server(max_active=2) as srv:
        outs, res = srv.wait(submit(srv, dims, args))
    assert res["status"] == pls.OK, res["message"]
    assert len(res["latency_ms"]) == 4 and all(x > 0 for x in res["latency_ms"])
    d, m = q.first_window()
    ref = oracle.solve(d, m, q.sens, None, q.lambda_L, q.lambda_S, levels=2, iters=K0)
    for j in range(3):
        dn, mn = q.frame(j)
        ref, d, m = oracle.append_frame(ref, d, m, q.sens, dn, mn, q.lambda_L, q.lambda_S,
                                        lambda_p=LAM_P, iters=K1)
    for k in ("L", "S", "M"):
        g = outs[k].cpu().numpy().astype(np.complex128)
        e = np.linalg.norm(g - ref[k]) / np.linalg.norm(ref[k])
        print(f"served {k}: rel L2 vs FP64 oracle {e:.3e}")
        assert e < 1e-4, (k, e)
    assert [w["iters"] for w in res["windows"]] == [K0] + [K1] * 3


def test_same_alone_and_in_the_mix():
    # (sequences are no longer driven independently on streams of their own; with
    # max_active = 4 the server runs groups of one geometry as batches)
    reqs = [make_request(i, n_append=2 + i % 3) for i in range(6)]
    alone = []
    with pls.Server(max_active=1) as srv:
        for q, dims, args in reqs:
            outs, res = srv.wait(submit(srv, dims, args))
            assert res["status"] == pls.OK, res["message"]
            alone.append(outs)
    # all at once: groups of up to four of one geometry, with a budget that forces some
    # to queue
    needs = sorted(pls.plan_bytes(q.nx, q.ny, q.nz, q.nt, q.nc) for q, _, _ in reqs)
    budget = int(sum(needs[-2:]) * 1.5)
    with pls.Server(max_active=4, hbm_budget=budget) as srv:
        tickets = [submit(srv, dims, args) for _, dims, args in reqs]
        mixed = [srv.wait(t) for t in tickets]
        info = srv.info()
    print("server:", info)
    assert info["peak_used"] <= budget and info["completed"] == len(reqs)
    assert info["peak_active"] >= 2
    for i, ((outs, res), ref) in enumerate(zip(mixed, alone)):
        assert res["status"] == pls.OK, res["message"]
        for k in ("L", "S", "X", "M"):
            assert torch.equal(outs[k], ref[k]), (i, k)


def test_same_alone_and_in_a_queued_mix():
    # sequences of three geometries (0, 0, 1, 2, 2, 0) submitted at once under a budget
    # that holds the largest plan and little beside it: they queue, reuse the resident
    # handle of their geometry (whose state the previous sequence left behind) or evict idle
    # ones, one sequence in flight at a time; each result must equal, bit for bit, the
    # result of the sequence served on its own
    reqs = [make_request(i, n_append=1 + i % 3) for i in (0, 3, 1, 2, 5, 6)]
    alone = []
    for q, dims, args in reqs:
        with pls.Server(max_active=1) as srv:
            outs, res = srv.wait(submit(srv, dims, args))
            assert res["status"] == pls.OK, res["message"]
            alone.append(outs)
    budget = int(max(pls.plan_bytes(q.nx, q.ny, q.nz, q.nt, q.nc) for q, _, _ in reqs) * 1.2)
    with pls.Server(max_active=1, hbm_budget=budget) as srv:
        tickets = [submit(srv, dims, args) for _, dims, args in reqs]
        mixed = [srv.wait(t) for t in tickets]
        info = srv.info()
    print("server:", info)
    assert info["completed"] == len(reqs) and info["peak_used"] <= budget
    assert info["reused"] >= 1 and info["evicted"] >= 1
    for i, ((outs, res), ref) in enumerate(zip(mixed, alone)):
        assert res["status"] == pls.OK, res["message"]
        for k in ("L", "S", "X", "M"):
            assert torch.equal(outs[k], ref[k]), (i, k)


def test_same_alone_and_in_a_batched_group():
    # requests of two geometries (0, 0, 1, 0, 1, 0, 0) submitted at once with room for all:
    # those of one geometry run together as a batched group, joining at window boundaries;
    # each result must equal, bit for bit, the sequence served on its own
    picks = [0, 3, 1, 6, 4, 9, 12]                  # GEOMS[i % 3]: 0, 0, 1, 0, 1, 0, 0
    reqs = [make_request(i, n_append=1 + i % 3) for i in picks]
    alone = []
    for q, dims, args in reqs:
        with pls.Server(max_active=1) as srv:
            outs, res = srv.wait(submit(srv, dims, args))
            assert res["status"] == pls.OK, res["message"]
            alone.append((outs, res))
    with pls.Server(max_active=4) as srv:
        tickets = [submit(srv, dims, args) for _, dims, args in reqs]
        grouped = [srv.wait(t) for t in tickets]
        info = srv.info()
    print("server:", info)
    assert info["completed"] == len(reqs) and info["peak_active"] >= 2
    for i, ((outs, res), (ref, rres)) in enumerate(zip(grouped, alone)):
        assert res["status"] == pls.OK, res["message"]
        for k in ("L", "S", "X", "M"):
            assert torch.equal(outs[k], ref[k]), (i, k)
        assert [w["iters"] for w in res["windows"]] == [w["iters"] for w in rres["windows"]]
        assert [w["resid_norm"] for w in res["windows"]] == [w["resid_norm"] for w in rres["windows"]]


def test_admission_respects_budget_and_reuses_plans():
    reqs = [make_request(1, n_append=1) for _ in range(4)]     # one geometry
    need = pls.plan_bytes(24, 32, 8, 7, 3)
    with pls.Server(max_active=4, hbm_budget=int(need * 1.2)) as srv:
        tickets = [submit(srv, dims, args) for _, dims, args in reqs]
        results = [srv.wait(t)[1] for t in tickets]
        info = srv.info()
    assert all(r["status"] == pls.OK for r in results)
    assert info["peak_active"] == 1 and info["peak_used"] <= int(need * 1.2)
    assert info["reused"] == 3 and sum(r["reused_plan"] for r in results) == 3
    assert max(r["queue_ms"] for r in results) > 0


def test_submit_from_another_thread():
    # requests arrive on a thread of their own while the caller waits
    import queue
    import threading
    reqs = [make_request(i, n_append=1) for i in range(3)]
    q = queue.Queue()
    with pls.Server(max_active=2) as srv:
        def submitter():
            try:
                for _, dims, args in reqs:
                    q.put(submit(srv, dims, args))
            except Exception as e:
                q.put(e)
        th = threading.Thread(target=submitter)
        th.start()
        for _ in reqs:
            t = q.get(timeout=120)
            assert not isinstance(t, Exception), t
            _, res = srv.wait(t)
            assert res["status"] == pls.OK, res["message"]
        th.join()
