"""Write the oracle's global solutions of the two benchmarked elliptic domains
at sampled nodes (tests/golden/online_<workload>.txt).

The oracle's least-squares gluing at h = 1/1024 (a dense Householder QR of a
65821 x 4096 system, after 256 local offline solves) takes minutes on a CPU,
too long to repeat inside the GPU tests and the benchmark, so its results are
stored here.  Calls only oracle/ and synth/ (no HIP path).

For each workload: the offline stage of the oracle (Philox boundary samples,
banded Cholesky local solves, Householder QR + SVD range finder), the
least-squares coefficients of eq. elliptic_cond_reduced by Householder QR,
and the partition-of-unity reconstruction u = sum_m w_m G_m c_m, for the
workload's own Dirichlet data and for serving requests 0..3 (16 Fourier modes,
request seed 4).  Stored: u at the nodes (i, j) with i, j multiples of N/32.

    python tests/golden/make_online_fixtures.py [workload ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from synth import configs  # noqa: E402
from oracle import elliptic as E  # noqa: E402

N_REQUESTS = 4
STRIDE_DIV = 32


def sample_nodes(N: int) -> np.ndarray:
    st = N // STRIDE_DIV
    jj, ii = np.meshgrid(np.arange(0, N + 1, st), np.arange(0, N + 1, st), indexing="ij")
    return (jj * (N + 1) + ii).ravel()


def path(name: str) -> str:
    return os.path.join(HERE, f"online_{name}.txt")


def make(name: str) -> str:
    cfg = configs.WORKLOADS[name]()
    N, M = cfg["N"], cfg["M"]
    t0 = time.time()
    ref = E.offline(cfg["coef"], N, M, cfg["overlap"], cfg["s"], cfg["k"], seed=cfg["seed"])
    P, n_cont, drows, off = E.coarse_rows(N, M, ref, cfg["coef"])
    Qf, Rf = E.coarse_factor(P)
    phis = np.column_stack([cfg["phi"]] + [synth.fourier_boundary(N, [r])[0] for r in range(N_REQUESTS)])
    c = E.coarse_solve(Qf, Rf, n_cont, drows, phis)
    u = E.reconstruct(N, M, ref, off, c)
    nodes = sample_nodes(N)
    out = path(name)
    with open(out, "w") as f:
        f.write(f"# oracle global solutions of {cfg['name']} (offline stage, least squares of eq. "
                f"elliptic_cond_reduced by Householder QR, partition-of-unity reconstruction)\n")
        f.write(f"# written by tests/golden/make_online_fixtures.py {name}; {time.time() - t0:.0f} s\n")
        f.write(f"# columns: node index j*(N+1)+i at i, j multiples of N/{STRIDE_DIV}; u for the workload's "
                f"Dirichlet data; u for serving requests 0..{N_REQUESTS - 1} (synth.fourier_boundary, seed 4)\n")
        f.write(f"# N {N} rows {nodes.size} norm2_full " +
                " ".join(f"{np.linalg.norm(u[:, r]):.14e}" for r in range(u.shape[1])) + "\n")
        for k, n in enumerate(nodes):
            f.write(f"{n} " + " ".join(f"{v:.14e}" for v in u[n]) + "\n")
    return out


def load(name: str):
    """(nodes, U, full_norms) of a fixture: U[:, 0] the workload's data, U[:, 1 + r] request r."""
    with open(path(name)) as f:
        lines = f.read().splitlines()
    head = [l for l in lines if l.startswith("# N ")][0].split()
    norms = np.array([float(x) for x in head[head.index("norm2_full") + 1:]])
    rows = np.array([[float(x) for x in l.split()] for l in lines if not l.startswith("#")])
    return rows[:, 0].astype(np.int64), rows[:, 1:], norms


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["elliptic_lognormal_512", "elliptic_lognormal_1024"]):
        print(make(nm), flush=True)
