"""GPU: the online stage and the request server through the C ABI.

Bars: global solutions against the FP64 oracle to relative L2 <= 1e-6; the
batched solve (c = K f) against the banded direct solve to 1e-10 relative;
a request served inside a mixed stream of requests against the same request
solved alone: bit-identical (the per-request arithmetic does not depend on
the batch), which implies the stated tolerance 1e-12 relative.
"""
import time

import numpy as np
import pytest

import synth
from synth import configs
from oracle import elliptic as E
from oracle import kinetic as K

from gpu_cases import resident

pytestmark = pytest.mark.gpu

FP64, FP32_IR = 0, 1


def _kin_cfg():
    return dict(name="kin_small", kind="kinetic", N=512, M=8, overlap=np.full(8, 32, np.int32), s=40, k=8,
                n_vel=32, eps=2.0 ** -6, coef=synth.kinetic_sigma(512, 0.05), seed=3)


def _kin_requests(ids):
    v, _ = K.ordinates(32)
    out = []
    for r in ids:
        g = np.random.default_rng([4, int(r)])
        a, b = g.standard_normal(2)
        out.append(np.concatenate([3 + a * np.sin(2 * np.pi * v[v > 0]), 2 + b * np.cos(2 * np.pi * v[v < 0])]))
    return np.array(out)


def _solve(pr, f, banded=False):
    import torch
    L = pr.layout()
    ft = torch.tensor(np.atleast_2d(f), device="cuda:0")
    u = torch.empty((ft.shape[0], L.n_nodes), device="cuda:0", dtype=torch.float64)
    (pr.solve_global_banded if banded else pr.solve_global)(ft, u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.fixture(scope="module")
def models(lib):
    """Two elliptic grids (h = 1/64 and 1/128) and one kinetic slab, resident."""
    cfg_a = configs.small_elliptic(N=64, M=4, delta=4, s=12, k=8)
    cfg_b = configs.elliptic_periodic_128()
    cfg_k = _kin_cfg()
    prs = [resident(cfg_a, FP32_IR, max_batch=256), resident(cfg_b, FP32_IR, max_batch=256),
           resident(cfg_k, FP32_IR, max_batch=256)]
    yield [cfg_a, cfg_b, cfg_k], prs
    for p in prs:
        p.close()


def _requests(cfg, ids):
    if cfg["kind"] == "kinetic":
        return _kin_requests(ids)
    return synth.fourier_boundary(cfg["N"], ids)


def test_batched_and_banded_agree_with_the_oracle(models):
    cfgs, prs = models
    for cfg, pr in zip(cfgs, prs):
        f = _requests(cfg, range(6))
        ub = _solve(pr, f)
        ud = _solve(pr, f, banded=True)
        assert np.abs(ub - ud).max() <= 1e-10 * np.abs(ud).max(), cfg["name"]
        if cfg["kind"] == "kinetic":
            ref = K.offline(cfg["coef"], cfg["eps"], cfg["N"], cfg["M"], cfg["overlap"], 32, cfg["s"], cfg["k"],
                            seed=cfg["seed"])
            uo = K.online(cfg["M"], 32, ref, f.T)
        else:
            ref = E.offline(cfg["coef"], cfg["N"], cfg["M"], cfg["overlap"], cfg["s"], cfg["k"], seed=cfg["seed"])
            uo = E.online(cfg["N"], cfg["M"], ref, cfg["coef"], f.T)
        for r in range(f.shape[0]):
            assert np.linalg.norm(ub[r] - uo[:, r]) <= 1e-6 * np.linalg.norm(uo[:, r]), (cfg["name"], r)


def test_batch_of_more_than_one_launch(models):
    """Batches above one reconstruction launch (32 requests) give the per-request results."""
    cfgs, prs = models
    f = _requests(cfgs[0], range(70))
    u_all = _solve(prs[0], f)
    for r in (0, 31, 32, 69):
        assert np.array_equal(u_all[r], _solve(prs[0], f[r])[0])


def test_server_results_equal_alone_and_in_a_mix(models):
    """Continuous batching over three resident models with a slot budget of a few
    solutions: every result equals the same request solved alone."""
    from paper_1807_08848_amd import msrs
    cfgs, prs = models
    rng = np.random.default_rng(5)
    n = 120
    mdl = rng.integers(0, 3, n)
    reqs = [_requests(cfgs[m], [1000 + i])[0] for i, m in enumerate(mdl)]
    big = max(p.layout().n_nodes for p in prs) * 8
    with msrs.Server(prs, n_streams=3, max_batch=5, slot_bytes=6 * big) as srv:
        tickets = []
        for i in range(n // 2):
            tickets.append(srv.submit(int(mdl[i]), reqs[i]))
            if i % 17 == 0:
                time.sleep(0.002)          # let batches start while requests keep arriving
        while len(tickets) < n:            # the rest in bulk, as far as staging allows
            tickets += srv.submit_many(mdl[len(tickets):], reqs[len(tickets):])
        outs, infos = [], []
        for i, t in enumerate(tickets):
            u = np.empty(prs[mdl[i]].layout().n_nodes)
            infos.append(srv.fetch(t, u))
            outs.append(u)
        st = srv.stats()
    assert st.submitted == n and st.completed == n
    assert st.peak_slot_bytes <= st.slot_capacity
    assert st.admission_waits > 0                      # the budget forced requests to wait
    assert max(i.batch_size for i in infos) > 1        # requests were batched
    assert len({i.stream for i in infos}) > 1          # on several streams
    for i in range(n):
        inf = infos[i]
        assert inf.status == 0 and inf.model == mdl[i]
        assert inf.t_arrival <= inf.t_admit <= inf.t_launch <= inf.t_done
        alone = _solve(prs[mdl[i]], reqs[i])[0]
        assert np.array_equal(outs[i], alone), i


def test_server_open_loop_poisson(models):
    """Open-loop Poisson arrivals replayed natively (mixed models): every request
    completes, latencies are ordered and sane, slots are released at completion."""
    from paper_1807_08848_amd import msrs
    cfgs, prs = models
    rng = np.random.default_rng(7)
    n, lam = 300, 2000.0
    mdl = rng.integers(0, 2, n)
    reqs = [_requests(cfgs[m], [i])[0] for i, m in enumerate(mdl)]
    with msrs.Server(prs[:2]) as srv:
        arr = msrs.server_clock() + 0.01 + np.cumsum(rng.exponential(1.0 / lam, n))
        infos = srv.replay(mdl, reqs, arr)
        st = srv.stats()
        burst = srv.replay(mdl[:100], reqs[:100])           # all at once: batches form
    assert st.completed == n and st.peak_slot_bytes <= st.slot_capacity
    for i, inf in enumerate(infos):
        assert inf.status == 0 and inf.model == mdl[i]
        assert abs(inf.t_arrival - arr[i]) < 1e-9
        assert inf.t_arrival <= inf.t_admit <= inf.t_launch <= inf.t_done
    lat = np.array([i.t_done - i.t_arrival for i in infos])
    assert np.percentile(lat, 50) < 0.5
    assert max(i.batch_size for i in burst) > 1


def test_server_argument_and_state_errors(models):
    from paper_1807_08848_amd import msrs
    cfgs, prs = models
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Server(prs[:1], slot_bytes=1024)
    assert e.value.status == msrs.ERR_OOM
    with msrs.Server(prs[:1]) as srv:
        with pytest.raises(msrs.MsrsError) as e:
            srv.submit(3, np.zeros(4 * 64))
        assert e.value.status == msrs.ERR_ARG
        with pytest.raises(msrs.MsrsError) as e:
            prs[0].assemble_coarse()            # a served handle refuses set-up calls
        assert e.value.status == msrs.ERR_STATE
        with pytest.raises(msrs.MsrsError) as e:
            srv.fetch(123456)
        assert e.value.status == msrs.ERR_ARG
    # the handle is usable again once the server is gone
    f = _requests(cfgs[0], [3])
    assert np.isfinite(_solve(prs[0], f)).all()


def test_tuning_keeps_results_bitwise(models):
    """Every launch shape of the online product and reconstruction gives the same bits;
    the autotuner reports all 9 candidates and keeps one of them."""
    from paper_1807_08848_amd import msrs
    cfgs, prs = models
    pr = prs[1]
    f = _requests(cfgs[1], range(21))
    ref = None
    for rb in (1, 2, 4, 8, 16):
        for ab in (4, 8, 16):
            pr.set_tuning(msrs.TUNE_RECON_BATCH, rb)
            pr.set_tuning(msrs.TUNE_APPLY_BATCH, ab)
            u = _solve(pr, f)
            if ref is None:
                ref = u
            assert np.array_equal(u, ref), (rb, ab)
    trials = pr.autotune(msrs.TUNE_STAGE_ONLINE, reps=2)
    assert len(trials) == 9 and all(t[2] > 0 for t in trials)
    best = min(trials, key=lambda t: t[2])[1]
    assert pr.get_tuning(msrs.TUNE_RECON_BATCH) * 100 + pr.get_tuning(msrs.TUNE_APPLY_BATCH) == best
    assert np.array_equal(_solve(pr, f), ref)
    with pytest.raises(msrs.MsrsError) as e:
        pr.set_tuning(msrs.TUNE_APPLY_BATCH, 5)
    assert e.value.status == msrs.ERR_ARG
