"""Benchmark of the offline random-sampling stage on one MI355X.

One step = the whole hot path over the workload: coefficient gather and
block factorization of every buffered patch, device-drawn boundary samples,
lifting, multi-RHS sweeps with FP64 iterative refinement, restriction, and the
range finder.  Prints one JSON line (see the fields below).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The throughput form replays several handles' graphs on streams of their own:
# give them hardware queues of their own (HIP's default is 4 per process; set
# before the runtime starts).  MSRS_BENCH_HW_QUEUES overrides the count.
os.environ["GPU_MAX_HW_QUEUES"] = os.environ.get("MSRS_BENCH_HW_QUEUES", "16")

METRIC = "patch×sample local solves/s; online solve p50/p99 ms at rel err ≤1e-6"
PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "fp32_valu": 157.3e12, "fp64_valu": 78.6e12, "hbm": 8.0e12}
K_FACTOR, K_SWEEP, K_RESIDUAL, K_RANGE = 3, 4, 5, 7


def patch_sizes(cfg):
    """(b, nl, N_int, nK, s) per patch from the workload geometry."""
    N, M = cfg["N"], cfg["M"]
    nH = N // M
    out = []
    for m2 in range(M):
        for m1 in range(M):
            d = int(cfg["overlap"][m2 * M + m1])
            cx = min(N, (m1 + 1) * nH + d) - max(0, m1 * nH - d)
            cy = min(N, (m2 + 1) * nH + d) - max(0, m2 * nH - d)
            b, nl = min(cx, cy) - 1, max(cx, cy) - 1
            out.append((b, nl, b * nl, (nH + 1) ** 2, cfg["s"]))
    return out


def algorithmic(cfg):
    """Algorithmic flops of one launch of each kernel class (banded-direct count).

    factor: sum_p N_p (b_p+1)^2 (banded Cholesky of A_II); one sweep launch
    (forward + back for all s columns): sum_p 4 N_p (b_p+1) s; range finder
    (CholQR2 count): sum_p 6 nK s^2.
    """
    ps = patch_sizes(cfg)
    return {K_FACTOR: sum(n * (b + 1) ** 2 for b, nl, n, nk, s in ps),
            K_SWEEP: sum(4 * n * (b + 1) * s for b, nl, n, nk, s in ps),
            K_RANGE: sum(6 * nk * s * s for b, nl, n, nk, s in ps)}


def measured_traffic(kernel_class, workload):
    """HBM bytes per launch of a kernel class on a workload from the committed
    counter summary (profiles/traffic_*.json), or None when there is none or the
    kernel source has changed since the counters were taken (the record carries
    the source's SHA-1)."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel_class") != kernel_class or rec.get("workload") != workload:
            continue
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != rec["source_sha1"]:
                return None
        return rec["hbm_read_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"]
    return None


def host_info():
    """CPU model, the threads the process may use, and numpy's LAPACK."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import numpy as np
        lp = np.__config__.CONFIG["Build Dependencies"]["lapack"]
        lapack = f"{lp.get('name')} {lp.get('version')}"
    except Exception:
        lapack = "unknown"
    return dict(cpu_model=model, cores=len(os.sched_getaffinity(0)), lapack=lapack)


def cpu_baseline(cfg, max_seconds=20.0):
    """The oracle's offline stage on every host core the process may use, over
    a bounded sample of patches (one process per core, one BLAS thread each)."""
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    from oracle import elliptic as E
    info = host_info()
    workers = info["cores"]
    geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
    # probe one interior patch to size the sample
    t0 = time.perf_counter()
    _oracle_patch((cfg, geo[len(geo) // 2 + cfg["M"] // 2]))
    t1 = time.perf_counter() - t0
    n = int(min(len(geo), max(workers, max_seconds * workers / max(t1, 1e-3))))
    n = max(1, min(len(geo), (n // workers) * workers or workers))
    pick = np.linspace(0, len(geo) - 1, n).astype(int)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, initializer=_one_thread) as ex:
        list(ex.map(_oracle_patch, [(cfg, geo[i]) for i in pick]))
    T = time.perf_counter() - t0
    return {"value": n * cfg["s"] / T, "unit": "patch×sample local solves/s", "cores": workers, "kind": "oracle",
            "sample": f"{n} of {len(geo)} patches of {cfg['name']} (offline stage: banded Cholesky, "
                      f"{cfg['s']} solves, restriction, QR+SVD), {workers} worker processes x 1 BLAS thread, "
                      f"{T:.1f} s", "cpu_model": info["cpu_model"], "lapack": info["lapack"]}


def cpu_online(names=("elliptic_lognormal_512", "elliptic_lognormal_1024"), n_req=100):
    """The oracle's online stage per request: the least-squares coefficients
    from the precomputed Householder QR of P~ (Q^T d, a triangular solve) and
    the partition-of-unity reconstruction; median of n_req requests per domain.
    The offline bases and the QR are computed first, untimed (the offline
    patches over every host core)."""
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    import synth
    from synth import configs
    from oracle import elliptic as E
    workers = len(os.sched_getaffinity(0))
    out = {}
    for name in names:
        cfg = configs.WORKLOADS[name]()
        geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=workers, initializer=_one_thread) as ex:
            ref = list(ex.map(_oracle_patch_basis, [(cfg, g) for g in geo]))
        P, n_cont, drows, off = E.coarse_rows(cfg["N"], cfg["M"], ref, cfg["coef"])
        Qf, Rf = E.coarse_factor(P)
        t_setup = time.perf_counter() - t0
        reqs = synth.fourier_boundary(cfg["N"], range(n_req))
        ts = []
        for r in range(n_req):
            t0 = time.perf_counter()
            c = E.coarse_solve(Qf, Rf, n_cont, drows, reqs[r])
            E.reconstruct(cfg["N"], cfg["M"], ref, off, c)
            ts.append(time.perf_counter() - t0)
        out[cfg["name"]] = {"p50_ms": float(np.median(ts) * 1e3), "p99_ms": float(np.percentile(ts, 99) * 1e3),
                            "requests": n_req, "setup_s": t_setup, "ls_rows": int(P.shape[0]),
                            "coarse_dim": int(P.shape[1])}
        print(f"[bench] cpu online {cfg['name']}: p50 {out[cfg['name']]['p50_ms']:.1f} ms "
              f"(set-up {t_setup:.0f} s)", file=sys.stderr, flush=True)
    return out


def _one_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _oracle_patch(args):
    cfg, g = args
    from oracle import elliptic as E
    from oracle.rangefinder import range_finder
    Y = E.sample_patch(cfg["coef"], cfg["N"], g, E.patch_omega(cfg["seed"], g, cfg["s"]))
    range_finder(Y, cfg["k"])
    return 0


def _oracle_patch_basis(args):
    cfg, g = args
    from oracle import elliptic as E
    from oracle.rangefinder import range_finder
    Y = E.sample_patch(cfg["coef"], cfg["N"], g, E.patch_omega(cfg["seed"], g, cfg["s"]))
    Q, sv = range_finder(Y, cfg["k"])
    return dict(geo=g, Q=Q, sv=sv)


def _desc(cfg, precision, flags, seed, ir_stop=0.0):
    from paper_1807_08848_amd import msrs
    kin = cfg["kind"] == "kinetic"
    return msrs.make_desc(msrs.KIND_KINETIC_DO if kin else msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"],
                          list(cfg["overlap"]), cfg["s"], cfg["k"], precision=precision, seed=seed,
                          n_vel=cfg.get("n_vel", 0), eps=cfg.get("eps", 1.0), hg=cfg.get("hg", 0.0),
                          flags=flags | (msrs.FLAG_FULL_BASIS_ENDS if kin else 0), ir_stop=ir_stop)


def run_pipelined(cfg, precision, pr, a, steps, warmup, max_handles, tune, factor_share=2, ir_stop=0.0):
    """Throughput form of the offline stage: several handles, each an independent
    sampling pass over the same medium (its own Omega seed), replay their captured
    steps on their own streams, round-robin, so that one pass's latency-bound
    phases (the factor's chain of lines, the per-patch eigensolver) overlap
    another's wide ones.  The handle count is chosen by timing 1..max_handles;
    pr (seed cfg["seed"]) is the first handle.  Every handle's factor is
    compiled for factor_share resident workgroups per compute unit (its graph
    captured again with that shape)."""
    import torch
    from paper_1807_08848_amd import msrs, tuning
    hs = [pr]
    pr.set_tuning(msrs.TUNE_FACTOR_SHARE, factor_share)
    pr.offline_graph_capture(a)
    try:
        for h in range(1, max_handles):
            sh = torch.cuda.Stream()
            with torch.cuda.stream(sh):
                ph = msrs.Problem(_desc(cfg, precision, 0, cfg["seed"] + h, ir_stop), stream=sh)
                hs.append(ph)
                if tune:
                    tuning.tune(ph, msrs.TUNE_STAGE_OFFLINE)
                ph.set_tuning(msrs.TUNE_FACTOR_SHARE, factor_share)
                ph.assemble_patch(a)
                ph.sample_local_solutions(None, None)
                ph.range_finder(None, None)
                ph.offline_graph_capture(a)
        torch.cuda.synchronize()

        def timed(P, n):
            for i in range(max(warmup, 1) * P):
                hs[i % P].offline_graph_launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                hs[i % P].offline_graph_launch()
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        n_try = max(steps, 12)
        trials = {P: timed(P, n_try) / n_try for P in range(1, max_handles + 1)}
        best = min(trials, key=trials.get)
        for ph in hs:
            ph.reset_stats()
        T = timed(best, steps)
        stats = [ph.stats() for ph in hs[:best]]
        ok = all(st.error_latched == 0 and st.max_rel_residual <= 1e-10 for st in stats)
        return dict(T=T, handles=best, ok=ok, max_rel_residual=max(st.max_rel_residual for st in stats),
                    trials_ms={P: t * 1e3 for P, t in trials.items()}, factor_share=factor_share)
    finally:
        for ph in hs[1:]:
            ph.close()


def run_gpu(cfg, precision, steps, warmup, flags=0, tune=False, graph=False, pipeline=0, timing=True, ir_stop=0.0):
    """Time `steps` offline steps (assemble + sample + range finder) after `warmup`.

    Eager: the three calls per step, with per-kernel-class HIP event timing.
    graph=True additionally times replays of the captured step (the
    production form: no host synchronisation between refinement iterations);
    pipeline=P > 0 then times the throughput form with up to P handles.
    timing=False leaves out the per-kernel-class events (wall clock only).
    ir_stop > 0: FP32 refinement stops once a patch's largest relative
    residual is at most ir_stop (0: the library's default, 1e-13).
    """
    import torch
    from paper_1807_08848_amd import msrs, tuning
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    d = _desc(cfg, precision, flags | (msrs.FLAG_TIMING if timing else 0), cfg["seed"], ir_stop)
    with torch.cuda.stream(stream):
        pr = msrs.Problem(d, stream=stream)
        a = torch.tensor(cfg["coef"], device=dev)

        def step():
            pr.assemble_patch(a)
            pr.sample_local_solutions(None, None)
            pr.range_finder(None, None)

        tuned = None
        if tune:
            pr.assemble_patch(a)
            tuned = tuning.tune(pr, msrs.TUNE_STAGE_OFFLINE)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        pr.reset_stats()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        st = pr.stats()
        L = pr.layout()
        # local solves per step: s per sampled patch, one per basis column of a full-basis patch
        n_solves = sum(pr.patch(p).n_samples for p in range(L.n_patches))
        res = dict(T=T, stats=st, n_solves=n_solves, tuned=tuned)
        if graph:
            t0 = time.perf_counter()
            pr.offline_graph_capture(a)
            t_cap = time.perf_counter() - t0
            for _ in range(warmup):
                pr.offline_graph_launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                pr.offline_graph_launch()
            torch.cuda.synchronize()
            res["T_graph"] = time.perf_counter() - t0
            res["graph_capture_s"] = t_cap
            sg = pr.stats()
            res["graph_ok"] = sg.error_latched == 0 and sg.max_rel_residual <= 1e-10
            res["graph_max_rel_residual"] = sg.max_rel_residual
            if pipeline:
                res["pipe"] = run_pipelined(cfg, precision, pr, a, steps, warmup, pipeline, tune, ir_stop=ir_stop)
        pr.close()
    return res


def build_model(cfg, precision=1):
    """A handle of the workload with its bases and coarse factor resident (online shapes tuned)."""
    import torch
    from paper_1807_08848_amd import msrs, tuning
    d = msrs.make_desc(msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"],
                       precision=precision, seed=cfg["seed"])
    pr = msrs.Problem(d)
    pr.assemble_patch(torch.tensor(cfg["coef"], device="cuda:0"))
    pr.sample_local_solutions()
    pr.range_finder()
    pr.set_max_batch(4096)
    t0 = time.perf_counter()
    pr.assemble_coarse()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    pr.tuned = tuning.tune(pr, msrs.TUNE_STAGE_ONLINE)
    pr.cond = pr.coarse_condition()
    return pr, ts


def run_constrained(reps=50):
    """The two online formulations on the h=1/64 workload with full bases on
    the boundary patches (4x4 patches, buffers of 8 cells, k=8 sampled on the
    interior): plain least squares against the constrained variant (Dirichlet
    rows exact).  Set-up time (msrs_assemble_coarse), device time of one
    batched solve of 1 and of 32 requests (events on the handle's stream,
    mean over reps), and the largest boundary mismatch |u - phi| on dOmega."""
    import numpy as np
    import torch
    import synth
    from paper_1807_08848_amd import msrs
    N, M, k = 64, 4, 8
    a = torch.tensor(synth.periodic_coefficient(N, 1.0 / 8.0), device="cuda:0")
    phis = torch.tensor(synth.fourier_boundary(N, range(32)), device="cuda:0")
    b = np.array([(i, 0) for i in range(N)] + [(N, j) for j in range(N)] + [(i, N) for i in range(N, 0, -1)]
                 + [(0, j) for j in range(N, 0, -1)])
    bidx = torch.tensor(b[:, 1] * (N + 1) + b[:, 0], device="cuda:0")
    out = {"workload": f"elliptic_periodic_N{N}_M{M}_k{k}, full bases on the boundary patches"}
    for name, extra in (("least_squares", 0), ("constrained", msrs.FLAG_CONSTRAINED_BC)):
        d = msrs.make_desc(msrs.KIND_ELLIPTIC_Q1, N, M, [8] * (M * M), k, k, precision=msrs.PREC_FP32_IR, seed=2,
                           flags=msrs.FLAG_FULL_BASIS_BOUNDARY | extra)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream), msrs.Problem(d, stream=stream) as pr:
            pr.assemble_patch(a)
            pr.sample_local_solutions()
            pr.range_finder()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pr.assemble_coarse()
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            u = torch.empty((32, (N + 1) ** 2), device="cuda:0", dtype=torch.float64)
            res = {"setup_ms": ts * 1e3}
            for nb in (1, 32):
                pr.solve_global(phis[:nb], u[:nb])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    pr.solve_global(phis[:nb], u[:nb])
                e1.record(stream)
                e1.synchronize()
                res[f"solve_ms_batch{nb}"] = e0.elapsed_time(e1) / reps
            res["max_boundary_mismatch"] = float((u[:, bidx] - phis).abs().max())
            out[name] = res
    return out


def _fixtures():
    import importlib.util
    spec = importlib.util.spec_from_file_location("online_fixtures",
                                                  os.path.join(ROOT, "tests", "golden", "make_online_fixtures.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def served_accuracy(srv, cfgs, pool):
    """Relative L2 error of served solutions against the oracle's (its own
    bases, Householder-QR least squares and reconstruction), stored at every
    32nd node in each direction for serving requests 0..3 of both domains;
    submitted as one interleaved mix through the server."""
    import numpy as np
    fx = _fixtures()
    ref = [fx.load(_fixture_name(c)) for c in cfgs]
    tickets = []
    for r in range(fx.N_REQUESTS):
        for m in range(len(cfgs)):
            tickets.append((m, r, srv.submit(m, pool[m][r])))
    worst = {}
    for m, r, t in tickets:
        nodes, U, _ = ref[m]
        u = np.empty(srv.problems[m].layout().n_nodes)
        srv.fetch(t, u)
        e = float(np.linalg.norm(u[nodes] - U[:, 1 + r]) / np.linalg.norm(U[:, 1 + r]))
        worst[cfgs[m]["name"]] = max(worst.get(cfgs[m]["name"], 0.0), e)
    return worst


def _fixture_name(cfg):
    return {"elliptic_lognormal_N512_M8_s32_k12": "elliptic_lognormal_512",
            "elliptic_lognormal_N1024_M16_s64_k16": "elliptic_lognormal_1024"}[cfg["name"]]


def run_serving(lams=(200, 500, 1000, 2000), seconds=2.0, seed_arrival=5):
    """Online stage over two resident models (h = 1/512 and h = 1/1024 domains).

    Open-loop Poisson arrivals at each rate (50/50 model mix, pre-drawn arrival
    times, boundary data of 16 Fourier modes): latency = solution resident in
    HBM minus scheduled arrival.  Also the saturation throughput of the server
    (all requests queued at once) and of the plain FP64 path (one request at
    a time: P~^T d and two band triangular solves, then the reconstruction).
    """
    import numpy as np
    import torch
    import synth
    from synth import configs
    from paper_1807_08848_amd import msrs
    cfgs = [configs.elliptic_lognormal_512(), configs.elliptic_lognormal_1024()]
    models, setup = [], []
    for c in cfgs:
        pr, ts = build_model(c)
        models.append(pr)
        setup.append(ts)
    nn = [m.layout().n_nodes for m in models]
    pool = [synth.fourier_boundary(c["N"], range(64)) for c in cfgs]   # request bodies, reused cyclically
    # accuracy of the batched solve against the banded direct solve on the same bases
    acc = []
    for pr, P in zip(models, pool):
        f = torch.tensor(P[:8], device="cuda:0")
        ub = torch.empty((8, pr.layout().n_nodes), device="cuda:0", dtype=torch.float64)
        ud = torch.empty_like(ub)
        pr.solve_global(f, ub)
        pr.solve_global_banded(f, ud)
        torch.cuda.synchronize()
        acc.append(float((ub - ud).abs().max() / ud.abs().max()))
    # plain FP64 path, one request at a time
    plain = {}
    for c, pr, P in zip(cfgs, models, pool):
        f = torch.tensor(P[:1], device="cuda:0")
        u = torch.empty((1, pr.layout().n_nodes), device="cuda:0", dtype=torch.float64)
        pr.solve_global_banded(f, u)
        torch.cuda.synchronize()
        n = 10
        t0 = time.perf_counter()
        for i in range(n):
            pr.solve_global_banded(f, u)
            torch.cuda.synchronize()
        plain[c["name"]] = (time.perf_counter() - t0) / n * 1e3
    plain_rate = 2.0 / sum(plain.values()) * 1e3      # 50/50 mix, requests/s

    def summary(infos, t_first):
        lat = np.array([i.t_done - i.t_arrival for i in infos]) * 1e3
        mdl = np.array([i.model for i in infos])
        span = max(i.t_done for i in infos) - t_first
        out = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "requests": len(infos), "solves_per_s": len(infos) / span,
               "mean_batch": float(np.mean([i.batch_size for i in infos])),
               "mean_ms": {"wait_admit": float(np.mean([i.t_admit - i.t_arrival for i in infos]) * 1e3),
                           "wait_launch": float(np.mean([i.t_launch - i.t_admit for i in infos]) * 1e3),
                           "device": float(np.mean([i.t_done - i.t_launch for i in infos]) * 1e3)}}
        for m, c in enumerate(cfgs):
            if np.any(mdl == m):
                out["p50_ms_" + c["name"]] = float(np.percentile(lat[mdl == m], 50))
                out["p99_ms_" + c["name"]] = float(np.percentile(lat[mdl == m], 99))
        return out

    rng = np.random.default_rng(seed_arrival)
    res = {}
    # the worker polls through idle gaps of up to 0.2 s (a host core for arrival latency: at 200 req/s one
    # gap in 7 exceeds the default 10 ms, after which a wake-up would add the scheduler's latency)
    with msrs.Server(models, n_streams=4, max_batch=32, slot_bytes=2 << 30, idle_spin_us=200000) as srv:
        accuracy = served_accuracy(srv, cfgs, pool)
        mdl = rng.integers(0, 2, 200)
        srv.replay(mdl, [pool[m][i % 64] for i, m in enumerate(mdl)])          # warm-up
        for lam in lams:
            n = int(max(400, lam * seconds))
            mdl = rng.integers(0, 2, n)
            arr = msrs.server_clock() + 0.02 + np.cumsum(rng.exponential(1.0 / lam, n))
            infos = srv.replay(mdl, [pool[m][i % 64] for i, m in enumerate(mdl)], arr)
            res[str(lam)] = summary(infos, arr[0])
            print(f"[bench] serving lambda={lam}: p50 {res[str(lam)]['p50_ms']:.3f} ms, "
                  f"p99 {res[str(lam)]['p99_ms']:.3f} ms", file=sys.stderr, flush=True)
        # saturation: the whole trace queued at once (back-pressure from the
        # slot and staging budgets), completion rate of the device
        n = 8000
        mdl = rng.integers(0, 2, n)
        t0 = msrs.server_clock()
        infos = srv.replay(mdl, [pool[m][i % 64] for i, m in enumerate(mdl)])
        sat_s = summary(infos, t0)
        sat = sat_s["solves_per_s"]
        sat_batch = sat_s["mean_batch"]
        st = srv.stats()
    out = {
        "workload": "serving over elliptic_lognormal_512 + elliptic_lognormal_1024 (50/50, Poisson arrivals)",
        "n_nodes": nn, "coarse_dim": [int(m.layout().coarse_dim) for m in models], "setup_s": setup,
        "autotune": [m.tuned for m in models],
        "rel_err_batched_vs_banded": acc, "rel_err_vs_oracle": accuracy,
        "coarse_condition": [{"kappa1_normal_equations": m.cond[0], "kappa_least_squares": m.cond[1]} for m in models],
        "open_loop": res,
        "saturation_solves_per_s": sat, "saturation_mean_batch": sat_batch, "saturation": sat_s,
        "plain_fp64_ms_per_request": plain,
        "plain_fp64_solves_per_s": plain_rate, "speedup_vs_plain": sat / plain_rate,
        "server": {"streams": 4, "max_batch": 32, "idle_spin_us": 200000, "mean_batch": st.mean_batch, "max_in_flight": st.max_in_flight,
                   "admission_waits": st.admission_waits, "peak_slot_bytes": st.peak_slot_bytes},
    }
    for m in models:
        m.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="elliptic_lognormal_1024")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu-online", action="store_true")
    ap.add_argument("--handles", type=int, default=8,
                    help="largest number of concurrent handles tried for the throughput form (1: one handle)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    from synth import configs
    cfg = configs.WORKLOADS[args.workload]()
    from paper_1807_08848_amd import msrs
    print(f"[bench] workload {cfg['name']}: FP32 factor/sweeps + FP64 refinement, {args.warmup} warmup + "
          f"{args.steps} timed steps", file=sys.stderr, flush=True)
    r = run_gpu(cfg, msrs.PREC_FP32_IR, args.steps, args.warmup, tune=True, graph=True, pipeline=args.handles)
    st = r["stats"]
    if not r["graph_ok"]:
        raise RuntimeError("graph replay latched an error or missed the residual tolerance")
    T = r["T_graph"]
    pipe = r.get("pipe")
    if pipe:
        if not pipe["ok"]:
            raise RuntimeError("a pipelined graph replay latched an error or missed the residual tolerance")
        T = pipe["T"]
    value = r["n_solves"] * args.steps / T
    # dominant kernel and its roofline (the banded-direct counts are those of the elliptic geometry)
    kinetic = cfg["kind"] == "kinetic"
    alg = algorithmic(cfg) if not kinetic else {K_FACTOR: 0, K_SWEEP: 0, K_RANGE: 0}
    ms = {k: st.kernel_ms[k] for k in range(11)}
    n = {k: st.kernel_launches[k] for k in range(11)}
    dom = max((K_FACTOR, K_SWEEP, K_RANGE), key=lambda k: ms[k])
    avg_ms = ms[dom] / max(n[dom], 1)
    achieved = alg[dom] / (avg_ms * 1e-3)
    kind = {K_FACTOR: ("alu", "fp32_valu", "factor (Gauss-Jordan block inverses, FP32 VALU)"),
            K_SWEEP: ("mfma", "fp32_mfma", "sweep (E_l y products on FP32 MFMA)"),
            K_RANGE: ("alu", "fp64_valu", "range finder (FP64)")}[dom]
    peak = PEAK[kind[1]]
    out = {
        "metric": METRIC, "value": value, "unit": "patch×sample local solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic (seeded lognormal medium, device Philox boundary samples)",
        "config": {"workload": cfg["name"], "N": cfg["N"], "M": cfg["M"], "samples": cfg["s"], "rank": cfg["k"],
                   "patches": cfg["M"] if kinetic else cfg["M"] ** 2,
                   "precision": "fp32 factor+sweeps, fp64 refinement/range finder"},
        "roofline": {"bound": kind[0], "kernel": kind[2], "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic({K_FACTOR: "factor", K_SWEEP: "sweep", K_RANGE: "range"}[dom], cfg["name"]),
                     "avg_launch_ms": avg_ms, "launches": n[dom]},
        "kernel_ms_per_step": {msrs.K_CLASSES[k]: ms[k] / args.steps for k in range(11) if n[k]},
        "ir_iters": st.ir_iters, "max_rel_residual": st.max_rel_residual, "autotune": r["tuned"],
        "timed_form": (f"hipGraph replays of the captured step by {pipe['handles']} independent handles "
                       "(one Omega seed each) on their own streams, round-robin" if pipe else
                       "hipGraph replay of the captured step"),
        "graph": {"capture_s": r["graph_capture_s"], "max_rel_residual": r["graph_max_rel_residual"],
                  "eager_ms_per_step": r["T"] / args.steps * 1e3,
                  "one_handle_ms_per_step": r["T_graph"] / args.steps * 1e3},
    }
    if pipe:
        out["pipeline"] = {"handles": pipe["handles"], "ms_per_step_by_handles": pipe["trials_ms"],
                           "max_rel_residual": pipe["max_rel_residual"], "factor_share": pipe["factor_share"]}
    if kinetic:
        out["roofline"] = None     # no banded-direct count is defined for the transport operator here
    if not args.no_plain:
        # the plain FP64 method: FP64 factor and sweeps, no refinement, one
        # launch per patch per stage, eager, no events
        print("[bench] plain FP64 reference (one launch per patch per stage)", file=sys.stderr, flush=True)
        n_plain = max(1, min(3, args.steps))
        rp = run_gpu(cfg, msrs.PREC_FP64, n_plain, 1, flags=msrs.FLAG_PER_PATCH_LAUNCH, timing=False)
        vp = rp["n_solves"] * n_plain / rp["T"]
        out["plain_fp64"] = {"value": vp, "speedup": value / vp,
                             "form": "eager, one launch per patch per stage, FP64 factor and sweeps"}
        # the same FP64 method in the timed form (batched launches, graph
        # replay, concurrent handles): the precision pattern's own gain
        print("[bench] batched FP64 in the timed form", file=sys.stderr, flush=True)
        rb = run_gpu(cfg, msrs.PREC_FP64, args.steps, args.warmup, graph=True, pipeline=args.handles, timing=False)
        Tb = rb["pipe"]["T"] if rb.get("pipe") else rb["T_graph"]
        vb = rb["n_solves"] * args.steps / Tb
        out["batched_fp64"] = {"value": vb, "speedup": value / vb,
                               "handles": rb["pipe"]["handles"] if rb.get("pipe") else 1,
                               "form": "batched launches, graph replay by concurrent handles, FP64 factor and sweeps"}
        # the FP32 path refined only to the 1e-10 relative residual of the
        # local-solve parity bar (the headline refines to stagnation, ~1e-13)
        print("[bench] FP32 refinement to 1e-10 in the timed form", file=sys.stderr, flush=True)
        rt = run_gpu(cfg, msrs.PREC_FP32_IR, args.steps, args.warmup, graph=True, pipeline=args.handles, timing=False,
                     ir_stop=1e-10)
        Tt = rt["pipe"]["T"] if rt.get("pipe") else rt["T_graph"]
        vt = rt["n_solves"] * args.steps / Tt
        out["fp32_ir_to_1e-10"] = {"value": vt, "speedup_vs_batched_fp64": vt / vb,
                                   "handles": rt["pipe"]["handles"] if rt.get("pipe") else 1,
                                   "refinement_passes": rt["stats"].ir_iters,
                                   "max_rel_residual": rt["pipe"]["max_rel_residual"] if rt.get("pipe") else rt["graph_max_rel_residual"],
                                   "form": "as the headline, refinement stopped at relative residual <= 1e-10"}
    if not args.no_serve:
        print("[bench] online serving (two resident models)", file=sys.stderr, flush=True)
        out["online"] = run_serving()
        print("[bench] online formulations: least squares vs constrained", file=sys.stderr, flush=True)
        out["online_constrained"] = run_constrained()
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
        if not args.no_cpu_online:
            out["cpu_baseline"]["online"] = cpu_online()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
