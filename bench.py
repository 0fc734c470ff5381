"""Benchmark: Priori L+S iterations/s at 192^2 x 32 x 30 frames x 8 coils on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--gram-mode fp32|fp64|bf16x3]

A step is one iteration of Algorithm 1 over the whole volume (Gram, eigensolve,
sparse update, back-projection, data consistency, statistics), everything in FP32 except
the FP64 eigensolve and statistics; the Gram runs on FP32 MFMA unless --gram-mode says
otherwise, and all three Gram modes are also timed and checked against the FP64-oracle
fixture of the workload at the end.  Inputs are the seeded
synthetic phantom of the 192x192x32x30x8 workload, resident in HBM before timing.
The timed region runs K iterations through prior_ls_step_timed, which records a
hipEvent around every kernel on the stream it runs on; the dominant kernel's average
launch duration comes from those events.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Priori L+S iterations/s at 192²×32×30×8coil; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_VALU_TFLOPS = 157.3     # MI355X FP32 vector peak
FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
FP64_MFMA_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
GRAM_NAMES = {"fp64": "FP64 MFMA", "fp32": "FP32 MFMA", "bf16x3": "split-BF16 (hi+lo x3) MFMA"}
KERNEL_SOURCES = {
    "data_consistency": ["pls_dc_impl.hpp", "pls_fft.hpp", "pls_common.hpp"],
    "gram": ["pls_gram.hip", "pls_common.hpp"],
    "backproject": ["pls_ls.hip"],
    "sparse": ["pls_ls.hip"],
}


def algorithmic(name, p, nsamp):
    """(bytes, flops, bound-unit peak) per launch of a kernel, from the problem size alone.
    bytes: each array the kernel must read or write once; flops: the operation's count."""
    N = p.nx * p.ny * p.nz
    I = N * p.nt * 8                      # one complex64 image array
    P = p.ny * p.nz
    if name == "data_consistency":
        dh = p.nx * p.nc * nsamp * 8      # compact hybrid k-space, sampled entries only
        sens = p.nc * N * 8 if p.nc > 1 else 0
        b = 3 * I + dh + sens + p.nt * P * 2
        # two 2D FFTs per coil and frame (5 n log2 n each) and the two coil multiplies
        # (6 flops each: C_c Y before the forward transform, conj(C_c) (.) after the inverse)
        f = p.nc * p.nt * p.nx * 2 * 5 * P * math.log2(P) + p.nc * p.nt * N * 12
        return b, f
    if name == "gram":
        return I, 8 * N * p.nt ** 2
    if name == "backproject":
        return 2 * I, 8 * N * p.nt ** 2
    if name == "sparse":
        return 4 * I + N * p.nt, 0
    if name == "change":
        return 4 * I, 0
    return 0, 0


def launches(name, steps):
    """Launches of a kernel in one prior_ls_step_timed call of `steps` iterations: the
    statistics and the change of the iterate run on the last iteration only."""
    return 1 if name in ("stats", "change") else steps


def source_hash(name):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(name, []):
        with open(os.path.join(ROOT, "paper_1411_6206_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(name, workload):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (committed under
    profiles/), or None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(f"{workload}:{name}")
    if not rec or rec.get("source_hash") != source_hash(name):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(p, iters):
    """The FP64 oracle, untuned, on the benchmark's own workload: `iters` full iterations of
    Algorithm 1 (all frames, coils and voxels) after its set-up step (0).  The value is one
    over the median seconds per iteration.  The DFTs run through scipy.fft on every core the
    process may use (the same unitary DFT as numpy.fft, pinned in the oracle's tests), LAPACK
    with its default threads; the oracle's other numpy work runs on one core."""
    import resource
    import oracle
    cores = len(os.sched_getaffinity(0))
    try:
        with open("/proc/meminfo") as fh:
            ram_gib = int(fh.readline().split()[1]) / (1 << 20)
    except OSError:
        ram_gib = float("nan")
    stamps = []
    oracle.set_fft_workers(cores)
    try:
        oracle.solve(p.kspace, p.mask, p.sens, p.prior_w, p.lambda_L, p.lambda_S, levels=2,
                     iters=iters, on_iteration=lambda k: stamps.append(time.perf_counter()))
    finally:
        oracle.set_fft_workers(None)
    per = sorted(b - a for a, b in zip(stamps[:-1], stamps[1:]))
    med = per[len(per) // 2] if len(per) % 2 else 0.5 * (per[len(per) // 2 - 1] + per[len(per) // 2])
    rss = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / (1 << 20)
    return {"value": 1.0 / med, "unit": "iterations/s", "cores": cores, "kind": "oracle",
            "sample": f"{iters} full FP64 oracle iterations of the same {p.nx}x{p.ny}x{p.nz} x "
                      f"{p.nt}-frame x {p.nc}-coil problem after its set-up step, median "
                      f"{med:.1f} s per iteration (all: {', '.join(f'{x:.1f}' for x in per)} s); "
                      f"DFTs on {cores} threads (scipy.fft), LAPACK threaded, other numpy work "
                      f"on one core; host RAM {ram_gib:.0f} GiB, peak RSS {rss:.1f} GiB",
            "seconds_per_iteration": per}


def serving_bench(budget_gib, forms):
    """The serving stream (64 recursive reconstructions, Poisson arrivals) through the
    library's server, once per form (max_active, gram_mode).  The k-space of every
    (volume, frames, coils) class is formed once on the device from the class phantom and
    coils (off-mask entries are ignored by the library, so requests of a class share it and
    differ in their masks).  Returns the per-form throughput and latency percentiles."""
    import queue
    import threading

    import numpy as np
    import torch
    import synth
    import paper_1411_6206_amd as pls

    cfg = synth.SERVING
    reqs = synth.serving_requests()
    napp = cfg["n_append"]
    t0 = time.perf_counter()
    nf_max = max(cfg["nts"]) + napp
    X = {}
    for vol in sorted({r[1] for r in reqs}):
        nx, ny, nz = vol
        L, S = synth.phantom(nx, ny, nz, nf_max, cfg["rank"][nx], cfg["nblobs"][nx],
                             seed=synth.MASTER_SEED * 100 + nx)
        X[vol] = torch.from_numpy((L + S).astype(np.complex64)).cuda()
    data, sens = {}, {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.MASTER_SEED)
    for _, vol, nt, nc, _, _, _ in reqs:
        if (vol, nt, nc) in data:
            continue
        nx, ny, nz = vol
        if (vol, nc) not in sens:
            sens[(vol, nc)] = None if nc == 1 else torch.from_numpy(
                synth.coils(np.random.default_rng(nx * 100 + nc), nx, ny, nz, nc)
                .astype(np.complex64)).cuda()
        sc = sens[(vol, nc)]
        x = X[vol][:nt + napp]
        k = torch.empty((nc, nt + napp, nz, ny, nx), dtype=torch.complex64, device="cuda")
        for c in range(nc):
            k[c] = torch.fft.fftn(x if sc is None else x * sc[c], dim=(-3, -2, -1), norm="ortho")
        noise = torch.randn(k.shape, dtype=torch.complex64, device="cuda", generator=gen)
        k += noise * (torch.linalg.vector_norm(k) /
                      (torch.linalg.vector_norm(noise) * 10 ** (cfg["snr_db"] / 20.0)))
        del noise
        data[(vol, nt, nc)] = (k[:, :nt].contiguous(), k[:, nt:].transpose(0, 1).contiguous(), sc)
        del k
    m0 = [torch.from_numpy(r[5]).cuda() for r in reqs]
    mf = [torch.from_numpy(r[6]).cuda() for r in reqs]
    # the reconstructed images X of every request, allocated up front: the submitting
    # thread then makes no GPU call, the server's dispatcher is the only HIP caller
    outx = [torch.empty((nt, v[2], v[1], v[0]), dtype=torch.complex64, device="cuda")
            for _, v, nt, _, _, _, _ in reqs]
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    first = pls.make_params(max_iter=cfg["first_iters"], check_every=cfg["first_iters"] // 2)
    nxt = pls.make_params(lambda_p=0.1, max_iter=cfg["append_iters"],
                          check_every=cfg["append_iters"])
    iters = cfg["first_iters"] + napp * cfg["append_iters"]
    work = sum(v[0] * v[1] * v[2] * nt * nc * iters for _, v, nt, nc, _, _, _ in reqs)
    out = {"workload": (f"{len(reqs)} recursive reconstructions, Poisson arrivals at "
                        f"{cfg['rate_per_s']:g}/s, volumes {'/'.join('x'.join(map(str, v)) for v in cfg['volumes'])}"
                        f" x {'/'.join(map(str, cfg['nts']))} frames x {'/'.join(map(str, cfg['ncs']))} coils, "
                        f"first window 50% sampled + {napp} appended frames at 8-12x; "
                        f"{cfg['first_iters']} + {napp} x {cfg['append_iters']} iterations each"),
           "hbm_budget_bytes": int(budget_gib * (1 << 30)), "input_gen_s": gen_s, "forms": {}}
    for max_active, mode in forms:
        q = queue.Queue()
        with pls.Server(hbm_budget=int(budget_gib * (1 << 30)), max_active=max_active) as srv:
            start = time.perf_counter()

            def submitter():
                try:
                    for i, (arr, vol, nt, nc, _, _, _) in enumerate(reqs):
                        delay = start + arr - time.perf_counter()
                        if delay > 0:
                            time.sleep(delay)
                        k0, kf, sc = data[(vol, nt, nc)]
                        dims = pls.make_dims(*vol, nt, nc, 2, mode)
                        sub = time.perf_counter()
                        q.put((i, srv.submit(dims, k0, m0[i], kf, mf[i], sc, first=first,
                                             append_params=nxt, out={"X": outx[i]},
                                             sync=False), sub))
                except Exception as e:          # handed to the waiting thread
                    q.put((None, e, None))

            th = threading.Thread(target=submitter)
            th.start()
            lat_app, lat_first, total, queued, ends, bad = [], [], [], [], [], 0
            for n_done in range(len(reqs)):
                i, tk, sub = q.get(timeout=300)
                if i is None:
                    th.join()
                    raise tk
                outs, res = srv.wait(tk)
                if (n_done + 1) % 16 == 0:
                    print(f"[bench] serving {mode} x{max_active}: {n_done + 1} of {len(reqs)} done",
                          file=sys.stderr, flush=True)
                del outs
                bad += res["status"] != pls.OK
                lat_first.append(res["latency_ms"][0])
                lat_app.extend(res["latency_ms"][1:])
                total.append(res["total_ms"])
                queued.append(res["queue_ms"])
                ends.append(sub - start + res["total_ms"] * 1e-3)
            th.join()
            info = srv.info()
        span = max(ends)
        pct = lambda a, p: float(np.percentile(np.array(a), p))
        out["forms"][f"{mode}_x{max_active}"] = {
            "max_active": max_active, "gram_mode": mode, "failed": bad,
            "makespan_s": span, "iterations_per_s": len(reqs) * iters / span,
            "voxel_frame_coil_iterations_per_s": work / span,
            "append_p50_ms": pct(lat_app, 50), "append_p99_ms": pct(lat_app, 99),
            "first_window_p50_ms": pct(lat_first, 50), "first_window_p99_ms": pct(lat_first, 99),
            "request_p50_ms": pct(total, 50), "request_p99_ms": pct(total, 99),
            "queue_p50_ms": pct(queued, 50), "queue_p99_ms": pct(queued, 99),
            "peak_resident_gib": info["peak_used"] / (1 << 30), "peak_active": info["peak_active"],
            "plans_reused": info["reused"], "plans_evicted": info["evicted"]}
        print(f"[bench] serving {mode} x{max_active}: {len(reqs) * iters / span:.0f} it/s, "
              f"append p50 {pct(lat_app, 50):.1f} ms", file=sys.stderr, flush=True)
    del data, X, sens, outx
    torch.cuda.empty_cache()
    return out


def batching_bench(steps, warmup, gram_mode):
    """Batched iterations (prior_ls_batch_*) of the small configurations: B problems of one
    geometry advanced with one launch per kernel, against one problem alone (tuned by its
    autotuner first), all with the given Gram mode."""
    import torch
    import synth
    import paper_1411_6206_amd as pls
    res = {}
    for cfg, sizes in ((1, (1, 8, 32)), (2, (1, 4, 8))):
        p = synth.config(cfg)
        t = pls.to_device(p)
        J = 2
        kw = dict(lambda_L=p.lambda_L, lambda_S=p.lambda_S)
        # one problem on its own handle (hipGraph chunks of 10 iterations)
        with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, gram_mode=gram_mode) as h:
            single = h.tune(t["kspace"], t["mask"], t["sens"], t["prior_w"], check_every=10, **kw)
            h.step(warmup, outputs=())
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            h.step(steps, outputs=())
            torch.cuda.synchronize()
            alone = steps / (time.perf_counter() - a0)
        rec = {"workload": f"{p.nx}x{p.ny}x{p.nz} voxels x {p.nt} frames x {p.nc} coil(s), "
                           f"{gram_mode.upper()} Gram",
               "alone_iterations_per_s": alone, "batches": {}}
        def run_batch(B, tb, n):
            """B copies of the problem as one batch with launch shapes tb: batched
            iterations/s over n iterations after the warm-up."""
            hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=J, gram_mode=gram_mode)
                  for _ in range(B)]
            for hh in hs:
                hh.set_tuning(tb["gram_blocks"], tb["bp_grid"], tb["sparse_fork"],
                              tb["sparse_grid"])
            try:
                with pls.Batch(hs) as b:
                    b.solve([t] * B, pls.make_params(max_iter=warmup, **kw), outputs=())
                    torch.cuda.synchronize()
                    a0 = time.perf_counter()
                    b.step(n, outputs=())
                    torch.cuda.synchronize()
                    el = time.perf_counter() - a0
            finally:
                for hh in hs:
                    hh.close()
            return B * n / el

        for B in sizes:
            # launch shapes of the batch (taken from its first handle): one problem keeps the
            # autotuner's choice; several take the fastest of a few sparse-update schedules
            # (fork after or before the Gram, about 512 workgroups in all, 256 per problem,
            # or one per tile), each timed over 20 iterations of a batch of its own
            if B == 1:
                tb = dict(single)
            else:
                cands = [(1, max(64, 512 // B)), (0, max(64, 512 // B)), (0, 256), (1, 256),
                         (1, 0)]
                trial = {c: run_batch(B, dict(single, sparse_fork=c[0], sparse_grid=c[1]),
                                      min(steps, 20)) for c in cands}
                fork, grid = max(trial, key=trial.get)
                tb = dict(single, sparse_fork=fork, sparse_grid=grid)
            rate = run_batch(B, tb, steps)
            rec["batches"][str(B)] = {"iterations_per_s": rate,
                                      "speedup_vs_alone": rate / alone,
                                      "tuning": {k: tb[k] for k in ("sparse_fork", "sparse_grid")}}
        res[f"c{cfg}"] = rec
        del t, p
        torch.cuda.empty_cache()
        print(f"[bench] batching c{cfg}: {rec}", file=sys.stderr, flush=True)
    res["mixed"] = mixed_batch_bench(steps, warmup)
    return res


def mixed_batch_bench(steps, warmup):
    """Problems of different geometry in one batch: the serving stream's 128x128x16 volume with
    window lengths 24 and 30 and 1, 4 or 8 coils (one plane shape and Gram tile class, so one
    set of kernel instances), against the same problems run one after another alone."""
    import torch
    import synth
    import paper_1411_6206_amd as pls
    shapes = [(24, 1), (24, 4), (24, 8), (30, 1), (30, 4), (30, 8)]
    ps = [synth.make_problem(nx=128, ny=128, nz=16, nt=nt, nc=nc, accel=10.0, snr_db=35.0,
                             rank=5, nblobs=40, seed=synth.MASTER_SEED * 10 + 40 + k, levels=2)
          for k, (nt, nc) in enumerate(shapes)]
    ts = [pls.to_device(p) for p in ps]
    kw = dict(lambda_L=0.01, lambda_S=0.01)
    hs = [pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, gram_mode="fp32")
          for p in ps]
    try:
        # alone: each problem in turn, hipGraph chunks of 10 iterations
        for h, t in zip(hs, ts):
            h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], max_iter=warmup, outputs=(),
                    check_every=10, **kw)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for h in hs:
            h.step(steps, outputs=())
        torch.cuda.synchronize()
        alone_s = time.perf_counter() - a0
        with pls.Batch(hs) as b:
            prm = pls.make_params(max_iter=warmup, check_every=10, **kw)
            b.solve(ts, prm, outputs=())
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            b.step(steps, outputs=())
            torch.cuda.synchronize()
            batch_s = time.perf_counter() - a0
    finally:
        for h in hs:
            h.close()
    work = sum(p.nx * p.ny * p.nz * p.nt * p.nc for p in ps) * steps
    rec = {"workload": "128x128x16 voxels, window lengths 24 and 30 x 1, 4 and 8 coils (6 "
                       "problems, one of each), 10x sampling, FP32 Gram, J=2",
           "alone_problem_iterations_per_s": len(ps) * steps / alone_s,
           "batch_problem_iterations_per_s": len(ps) * steps / batch_s,
           "alone_voxel_frame_coil_iterations_per_s": work / alone_s,
           "batch_voxel_frame_coil_iterations_per_s": work / batch_s,
           "speedup_vs_alone": alone_s / batch_s}
    print(f"[bench] batching mixed: {rec}", file=sys.stderr, flush=True)
    del ts
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--latency-reps", type=int, default=20)
    ap.add_argument("--latency-iters", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3,
                    help="full oracle iterations timed for the CPU baseline")
    ap.add_argument("--gram-mode", default="fp32", choices=("fp64", "fp32", "bf16x3"))
    ap.add_argument("--no-gram-modes", action="store_true",
                    help="skip the per-Gram-mode comparison (short profiling runs)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes, no autotuning")
    ap.add_argument("--no-transforms", action="store_true",
                    help="skip the temporal-Fourier transform measurement")
    ap.add_argument("--serving-budget-gib", type=float, default=48.0)
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batched small-configuration measurements")
    ap.add_argument("--no-alone", action="store_true",
                    help="skip the per-kernel timing with every kernel alone")
    ap.add_argument("--alone-steps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the iteration shards by x-plane with one Gram all-reduce per iteration; not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1411_6206_amd as pls

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    pls.lib()                                   # fails loudly when the library is missing
    t0 = time.perf_counter()
    p = synth.config(args.config)
    gen_s = time.perf_counter() - t0
    print(f"[bench] inputs generated in {gen_s:.1f} s", file=sys.stderr, flush=True)
    nsamp = int(p.mask.sum())
    t = pls.to_device(p)
    h = pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, gram_mode=args.gram_mode)
    solve_kw = dict(lambda_L=p.lambda_L, lambda_S=p.lambda_S)

    def solve(n, **kw):
        return h.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], max_iter=n,
                       outputs=(), **solve_kw, **kw)

    # a plain copy of known size (1 GiB read + 1 GiB written by one elementwise kernel): the
    # reference dispatch that scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes
    cal = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    torch.neg(cal.fill_(1.0), out=torch.empty_like(cal))
    del cal
    if args.no_tune:
        solve(0)                                # load: compact k-space, coils, weights, X_0
        tuning = None
    else:
        # the library's autotuner: times the sparse fork point, the Gram split and the
        # back-projection grid on this problem and keeps the fastest; leaves X_0 loaded
        tuning = h.tune(t["kspace"], t["mask"], t["sens"], t["prior_w"], check_every=10,
                        **solve_kw)
        print(f"[bench] tuned: {tuning}", file=sys.stderr, flush=True)
    h.step(args.warmup) if args.warmup > 0 else None
    torch.cuda.synchronize()
    ts = time.perf_counter()
    kms, st = h.step_timed(args.steps)
    torch.cuda.synchronize()
    te = time.perf_counter()
    ms_per_step = (te - ts) * 1e3 / args.steps
    value = args.steps / (te - ts)

    # the same iterations replayed as hipGraph chunks (production path)
    torch.cuda.synchronize()
    tg = time.perf_counter()
    h.step(args.steps)
    torch.cuda.synchronize()
    graph_its = args.steps / (time.perf_counter() - tg)

    # solve latency (load + step (0) + latency_iters iterations + outputs)
    lat = []
    for _ in range(args.latency_reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        solve(args.latency_iters, check_every=args.latency_iters)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)
    print(f"[bench] timed {args.steps} iterations: {value:.1f} it/s; solve latency done",
          file=sys.stderr, flush=True)

    # every kernel alone: the same iterations with the sparse update on the main stream and
    # one workgroup per tile (outside the timed region; the tuned schedule is restored)
    alone = {}
    if not args.no_alone:
        tuned = h.get_tuning()
        h.set_tuning(tuned["gram_blocks"], tuned["bp_grid"], 2, 0)
        h.step(2)
        ka, _ = h.step_timed(args.alone_steps)
        h.set_tuning(tuned["gram_blocks"], tuned["bp_grid"], tuned["sparse_fork"],
                     tuned["sparse_grid"])
        for name, tot in ka.items():
            per = tot / launches(name, args.alone_steps)
            b, f = algorithmic(name, p, nsamp)
            alone[name] = {"ms_per_launch": per,
                           "GB_s": (b / (per * 1e-3) / 1e9) if b and per > 0 else None,
                           "hbm_frac": (b / (per * 1e-3) / 1e9 / HBM_PEAK_GBS) if b and per > 0
                           else None,
                           "TFLOP_s": (f / (per * 1e-3) / 1e12) if f and per > 0 else None}

    workload = f"c{args.config}"
    kernels = {}
    for name, tot in kms.items():
        per = tot / launches(name, args.steps)
        b, f = algorithmic(name, p, nsamp)
        gb_s = (b / (per * 1e-3) / 1e9) if b and per > 0 else None
        kernels[name] = {"ms_per_launch": per, "GB_s": gb_s,
                         "hbm_frac": gb_s / HBM_PEAK_GBS if gb_s else None,
                         "algorithmic_bytes": b or None, "traffic_bytes": traffic_for(name, workload),
                         "TFLOP_s": (f / (per * 1e-3) / 1e12) if f and per > 0 else None}
    dom = max(kms, key=kms.get)
    per = kms[dom] / args.steps
    b, f = algorithmic(dom, p, nsamp)
    gbs = b / (per * 1e-3) / 1e9 if b else 0.0
    if dom == "data_consistency":
        tfl = f / (per * 1e-3) / 1e12
        if tfl / FP32_VALU_TFLOPS >= gbs / HBM_PEAK_GBS:
            roof = {"bound": "alu", "achieved": tfl, "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif dom == "gram" and args.gram_mode in ("fp64", "fp32"):
        tfl = f / (per * 1e-3) / 1e12
        pk = FP64_MFMA_TFLOPS if args.gram_mode == "fp64" else FP32_MFMA_TFLOPS
        if tfl / pk >= gbs / HBM_PEAK_GBS:
            roof = {"bound": "mfma", "achieved": tfl, "peak": pk, "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    roof["traffic"] = traffic_for(dom, workload)
    roof["algorithmic_bytes_per_launch"] = b
    roof["algorithmic_flops_per_launch"] = f

    out = {
        "metric": METRIC, "value": value, "unit": "iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{p.nx}x{p.ny}x{p.nz} voxels x {p.nt} frames x {p.nc} coils, "
                               f"{nsamp} of {p.nt * p.ny * p.nz} phase-encode lines (10x), "
                               f"rank-6 + 60 blobs seeded phantom, J=2 Haar, "
                               f"{GRAM_NAMES[args.gram_mode]} Gram",
                   "nx": p.nx, "ny": p.ny, "nz": p.nz, "nt": p.nt, "nc": p.nc,
                   "gram_mode": args.gram_mode},
        "roofline": roof,
        "p50_solve_ms": float(np.percentile(lat, 50)),
        "p99_solve_ms": float(np.percentile(lat, 99)),
        "solve_iters": args.latency_iters,
        "graph_iterations_per_s": graph_its,
        "kernels": kernels,
        "kernels_alone": alone,
        "resid_norm": st["resid_norm"],
        "eig_sweeps_last": st["eig_sweeps"],
        "tuning": tuning,
        "input_gen_s": gen_s,
    }
    h.close()

    # Gram precision modes on the same problem: throughput, Gram time and, where the sampled
    # FP64-oracle fixture of this workload (30 iterations) is present, the relative L2 error
    # of L, S and X = L + S at its sample voxels
    fx_path = os.path.join(ROOT, "tests", "golden", f"c{args.config}_oracle_samples.npz")
    fx = np.load(fx_path) if os.path.exists(fx_path) else None
    modes = {}
    for mode in (() if args.no_gram_modes else ("fp64", "fp32", "bf16x3")):
        hm = pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2, gram_mode=mode)
        iters = int(fx["iters"]) if fx is not None else 0
        outm, _ = hm.solve(t["kspace"], t["mask"], t["sens"], t["prior_w"], max_iter=iters,
                           check_every=max(iters, 1), outputs=("L", "S", "X"), **solve_kw)
        rec = {}
        if fx is not None:
            idx = torch.from_numpy(fx["idx"]).cuda()
            want = {"L": fx["L"], "S": fx["S"], "X": fx["L"] + fx["S"]}
            for k in ("L", "S", "X"):
                g = outm[k].reshape(-1)[idx].cpu().numpy().astype(np.complex128)
                rec[f"rel_l2_{k}_vs_fp64_oracle"] = float(np.linalg.norm(g - want[k]) /
                                                          np.linalg.norm(want[k]))
        del outm
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        km, _ = hm.step_timed(args.steps)
        torch.cuda.synchronize()
        rec["iterations_per_s"] = args.steps / (time.perf_counter() - a0)
        rec["gram_ms"] = km["gram"] / args.steps
        modes[mode] = rec
        hm.close()
    out["gram_modes"] = modes or None
    out["gram_modes_sample"] = (f"{iters} iterations, {len(fx['idx'])} sampled voxels of the "
                                f"committed FP64-oracle fixture") if fx is not None and modes else None
    # the temporal-Fourier sparsifying transform on the same problem (no prior weights:
    # the workload's weights are Haar-domain): throughput and its sparse-update kernel
    if not args.no_transforms:
        with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, gram_mode=args.gram_mode,
                         transform="tfft") as ht:
            ht.solve(t["kspace"], t["mask"], t["sens"], None, max_iter=args.warmup, outputs=(),
                     **solve_kw)
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            kmt, _ = ht.step_timed(args.steps)
            torch.cuda.synchronize()
            its = args.steps / (time.perf_counter() - a0)
            per = kmt["sparse"] / args.steps
            b = 4 * p.nx * p.ny * p.nz * p.nt * 8 + p.nx * p.ny * p.nz * p.nt
            # the sparse kernel alone (serial schedule), outside the timed region
            ht.set_tuning(0, 0, 2, 0)
            kma, _ = ht.step_timed(args.steps)
            pa = kma["sparse"] / args.steps
            out["transforms"] = {"tfft": {
                "iterations_per_s": its,
                "sparse_ms": per, "sparse_GB_s": b / (per * 1e-3) / 1e9,
                "sparse_hbm_frac": b / (per * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "sparse_alone_ms": pa, "sparse_alone_GB_s": b / (pa * 1e-3) / 1e9,
                "sparse_alone_hbm_frac": b / (pa * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "note": "unitary DFT along frames on FP32 MFMA, forward and inverse fused "
                        "with the shrink in one kernel"}}
        # the Daubechies-4 wavelet (J = 2, no prior weights) on the same problem: three passes
        # (x lines, (y, z) planes with the shrink, x lines): 3 + 1 + 1 reads and 1 + 1 + 1
        # writes of an image array, plus the support map
        with pls.PriorLS(p.nx, p.ny, p.nz, p.nt, p.nc, wavelet_levels=2,
                         gram_mode=args.gram_mode, transform="db4") as hd:
            hd.solve(t["kspace"], t["mask"], t["sens"], None, max_iter=args.warmup, outputs=(),
                     **solve_kw)
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            kmd, _ = hd.step_timed(args.steps)
            torch.cuda.synchronize()
            its = args.steps / (time.perf_counter() - a0)
            per = kmd["sparse"] / args.steps
            nvox = p.nx * p.ny * p.nz * p.nt
            b = 8 * nvox * 8 + nvox
            hd.set_tuning(0, 0, 2, 0)
            kma, _ = hd.step_timed(args.steps)
            pa = kma["sparse"] / args.steps
            out["transforms"]["db4"] = {
                "iterations_per_s": its,
                "sparse_ms": per, "sparse_GB_s": b / (per * 1e-3) / 1e9,
                "sparse_alone_ms": pa, "sparse_alone_GB_s": b / (pa * 1e-3) / 1e9,
                "sparse_alone_hbm_frac": b / (pa * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "note": "periodic four-tap Daubechies wavelet, J = 2 along every axis (standard "
                        "decomposition): x-line, plane and x-line passes"}
        # the paper's own geometry: 256x256x14 volumes x 20 frames (one coil, sampling 1/7,
        # Haar J = 1 since 14 = 2 x 7), radix 7 along z
        g0 = time.perf_counter()
        pg = synth.make_problem(nx=256, ny=256, nz=14, nt=20, nc=1, accel=7.0, snr_db=35.0,
                                rank=5, nblobs=40, seed=synth.MASTER_SEED * 10 + 6, levels=1)
        tg = pls.to_device(pg)
        with pls.PriorLS(256, 256, 14, 20, 1, wavelet_levels=1, gram_mode=args.gram_mode) as hg:
            g1 = time.perf_counter()
            tun = hg.tune(tg["kspace"], tg["mask"], tg["sens"], tg["prior_w"], check_every=10,
                          lambda_L=pg.lambda_L, lambda_S=pg.lambda_S)
            hg.step(args.warmup) if args.warmup > 0 else None
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            kmg, _ = hg.step_timed(args.steps)
            torch.cuda.synchronize()
            out["transforms"]["geometry_256x256x14x20"] = {
                "iterations_per_s": args.steps / (time.perf_counter() - a0),
                "data_consistency_ms": kmg["data_consistency"] / args.steps,
                "kernels_ms": {k: v / launches(k, args.steps) for k, v in kmg.items()},
                "tuning": tun,
                "input_gen_s": g1 - g0,
                "note": "the cardiac geometry of the paper's experiments, synthetic phantom"}
        del tg, pg
    del t
    torch.cuda.empty_cache()
    if not args.no_batching:
        out["batching"] = batching_bench(args.steps, args.warmup, args.gram_mode)
    if not args.no_serving:
        # one sequence at a time against groups of up to 8 sequences of one geometry
        # advanced as batches, and the split-BF16 Gram form grouped
        out["serving"] = serving_bench(args.serving_budget_gib,
                                       forms=((1, "fp32"), (8, "fp32"), (8, "bf16x3")))
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_iters)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
