"""Independent handles whose captured offline steps replay concurrently on
their own streams (the throughput form of the offline stage): every handle's
bases and singular values equal those of its replays alone, bit for bit, and
the first handle's bases match the oracle's."""
import numpy as np
import pytest

from synth import configs
from oracle import elliptic as E
from oracle.rangefinder import sin_max_angle

FP32_IR = 1


@pytest.mark.gpu
def test_concurrent_graph_replays_equal_solo_replays(lib):
    import torch
    from gpu_cases import _unpack
    cfg = configs.small_elliptic(N=64, M=4, delta=4, s=12, k=8)
    dev = torch.device("cuda:0")
    a = torch.tensor(cfg["coef"], device=dev)
    hs = []
    try:
        for h in range(3):
            st = torch.cuda.Stream()
            d = lib.make_desc(lib.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"],
                              precision=FP32_IR, seed=cfg["seed"] + h)
            pr = lib.Problem(d, stream=st)
            hs.append(pr)
            pr.assemble_patch(a)
            pr.sample_local_solutions()
            pr.range_finder()
            pr.offline_graph_capture(a)
        L = hs[0].layout()

        def results(pr):
            Q = torch.empty(L.Q_total, device=dev, dtype=torch.float64)
            sv = torch.empty(L.sv_total, device=dev, dtype=torch.float64)
            pr.copy_results(None, Q, sv)
            torch.cuda.synchronize()
            return Q.cpu().numpy(), sv.cpu().numpy()

        solo = []
        for pr in hs:
            pr.offline_graph_launch()
            torch.cuda.synchronize()
            solo.append(results(pr))
        for rnd in range(4):
            for pr in hs:
                pr.offline_graph_launch()
            torch.cuda.synchronize()
            for h, pr in enumerate(hs):
                Q, sv = results(pr)
                assert np.array_equal(Q, solo[h][0]) and np.array_equal(sv, solo[h][1]), (rnd, h)
                s = pr.stats()
                assert s.error_latched == 0 and s.max_rel_residual <= 1e-10
        assert not np.array_equal(solo[0][0], solo[1][0])       # distinct seeds, distinct samples
        ref = E.offline(cfg["coef"], cfg["N"], cfg["M"], cfg["overlap"], cfg["s"], cfg["k"], seed=cfg["seed"])
        infos = [hs[0].patch(p) for p in range(L.n_patches)]
        for p, (r, inf) in enumerate(zip(ref, infos)):
            Qg = _unpack(solo[0][0], inf.Q_off, inf.n_rows, inf.n_cols)
            assert sin_max_angle(r["Q"], Qg) < 1e-6, p
    finally:
        for pr in hs:
            pr.close()
