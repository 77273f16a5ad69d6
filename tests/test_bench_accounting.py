"""The benchmark's bookkeeping on the CPU: the algorithmic flop count its
roofline divides by, worked out by hand for the benchmarked h=1/512 geometry,
and its refusal of more than one GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    saved = os.environ.get("GPU_MAX_HW_QUEUES")
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        # importing bench sets the queue count for its own runs; keep this process as it was
        if saved is None:
            os.environ.pop("GPU_MAX_HW_QUEUES", None)
        else:
            os.environ["GPU_MAX_HW_QUEUES"] = saved
    return bench


def test_factor_flops_of_the_benchmarked_workload():
    """h=1/512, 8x8 patches of 64 cells, buffers of 16 cells clipped at the
    domain: 36 interior patches of 96x96 cells (b = nl = 95), 24 edge patches of
    80x96 (b = 79, nl = 95), 4 corners of 80x80 (b = nl = 79).  Banded count
    N (b+1)^2 with N = b nl interior unknowns."""
    bench = _bench()
    from synth import configs
    cfg = configs.elliptic_lognormal_512()
    sizes = sorted({(b, nl) for b, nl, n, nk, s in bench.patch_sizes(cfg)})
    assert sizes == [(79, 79), (79, 95), (95, 95)]
    expect = 36 * (95 * 95) * 96 ** 2 + 24 * (79 * 95) * 80 ** 2 + 4 * (79 * 79) * 80 ** 2
    assert expect == 4_306_816_000
    alg = bench.algorithmic(cfg)
    assert alg[bench.K_FACTOR] == expect
    # one sweep launch: 4 N (b+1) s; range finder: 6 nK s^2 with nK = 65^2
    assert alg[bench.K_SWEEP] == 4 * 32 * (36 * 95 * 95 * 96 + 24 * 79 * 95 * 80 + 4 * 79 * 79 * 80)
    assert alg[bench.K_RANGE] == 64 * 6 * 65 ** 2 * 32 ** 2


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
