"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
unpack its concatenated outputs per patch (imported by tests only)."""
from __future__ import annotations

import numpy as np


def _unpack(flat, off, rows, cols):
    return flat[off:off + rows * cols].reshape(cols, rows).T


def run(cfg, precision, omegas=None, flags=0, phi=None, n_req=None, max_batch=None, stats=True, tuning=None):
    """Run assemble -> sample -> range finder (-> coarse + solve) on cuda:0.

    cfg: a workload dict of synth.configs; omegas: optional list of per-patch
    boundary-sample matrices (n_bdry x s) passed explicitly; phi: optional
    global boundary data (n_bdry,) or (B, n_bdry) for the online stage.
    """
    import torch
    from paper_1807_08848_amd import msrs

    kin = cfg["kind"] == "kinetic"
    d = msrs.make_desc(msrs.KIND_KINETIC_DO if kin else msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"],
                       list(cfg["overlap"]), cfg["s"], cfg["k"], precision=precision, seed=cfg["seed"],
                       n_vel=cfg.get("n_vel", 0), eps=cfg.get("eps", 1.0), hg=cfg.get("hg", 0.0),
                       rank_tol=cfg.get("rank_tol", 0.0), flags=flags | (msrs.FLAG_FULL_BASIS_ENDS if kin else 0))
    pr = msrs.Problem(d)
    try:
        for key, value in (tuning or {}).items():
            pr.set_tuning(key, value)
        L = pr.layout()
        infos = [pr.patch(p) for p in range(L.n_patches)]
        dev = torch.device("cuda:0")
        a = torch.tensor(np.asarray(cfg["coef"]), device=dev, dtype=torch.float64)
        pr.assemble_patch(a)
        om = None
        if omegas is not None:
            flat = np.zeros(L.omega_total)
            for p, inf in enumerate(infos):
                if omegas[p] is not None:
                    flat[inf.omega_off:inf.omega_off + inf.n_bdry * inf.n_samples] = np.asarray(omegas[p]).T.ravel()
            om = torch.tensor(flat, device=dev)
        Y = torch.empty(L.Y_total, device=dev, dtype=torch.float64)
        pr.sample_local_solutions(om, Y)
        Q = torch.empty(L.Q_total, device=dev, dtype=torch.float64)
        sv = torch.empty(L.sv_total, device=dev, dtype=torch.float64)
        pr.range_finder(Q, sv)
        infos = [pr.patch(p) for p in range(L.n_patches)]     # ranks chosen at a tolerance, if any
        L = pr.layout()
        Om = torch.empty(L.omega_total, device=dev, dtype=torch.float64)
        pr.copy_omega(Om)
        st = pr.stats() if stats else None
        Yh, Qh, svh, Omh = (t.cpu().numpy() for t in (Y, Q, sv, Om))
        out = dict(layout=L, infos=infos, stats=st, Q_flat=Qh,
                   Y=[_unpack(Yh, i.Y_off, i.n_rows, i.n_samples) for i in infos],
                   Q=[_unpack(Qh, i.Q_off, i.n_rows, i.n_cols) for i in infos],
                   sv=[svh[i.sv_off:i.sv_off + i.n_samples] for i in infos],
                   omega=[_unpack(Omh, i.omega_off, i.n_bdry, i.n_samples) for i in infos])
        if phi is not None:
            phi = np.atleast_2d(np.asarray(phi, dtype=np.float64))
            if max_batch:
                pr.set_max_batch(max_batch)
            pr.assemble_coarse()
            f = torch.tensor(phi, device=dev)
            u = torch.empty((phi.shape[0], L.n_nodes), device=dev, dtype=torch.float64)
            pr.solve_global(f, u)
            out["u"] = u.cpu().numpy()
        torch.cuda.synchronize()
        return out
    finally:
        pr.close()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def resident(cfg, precision, max_batch=None, flags=0):
    """A handle with bases and coarse factor resident (caller closes it)."""
    import torch
    from paper_1807_08848_amd import msrs

    kin = cfg["kind"] == "kinetic"
    d = msrs.make_desc(msrs.KIND_KINETIC_DO if kin else msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"],
                       list(cfg["overlap"]), cfg["s"], cfg["k"], precision=precision, seed=cfg["seed"],
                       n_vel=cfg.get("n_vel", 0), eps=cfg.get("eps", 1.0), hg=cfg.get("hg", 0.0),
                       rank_tol=cfg.get("rank_tol", 0.0), flags=flags | (msrs.FLAG_FULL_BASIS_ENDS if kin else 0))
    pr = msrs.Problem(d)
    try:
        a = torch.tensor(np.asarray(cfg["coef"]), device="cuda:0", dtype=torch.float64)
        pr.assemble_patch(a)
        pr.sample_local_solutions()
        pr.range_finder()
        if max_batch:
            pr.set_max_batch(max_batch)
        pr.assemble_coarse()
        torch.cuda.synchronize()
        return pr
    except Exception:
        pr.close()
        raise


def bases(pr):
    """Per-patch Q of a resident handle (host), in the oracle's patch dicts' shape."""
    import torch
    L = pr.layout()
    infos = [pr.patch(p) for p in range(L.n_patches)]
    Q = torch.empty(L.Q_total, device="cuda:0", dtype=torch.float64)
    pr.range_finder(Q)
    Qh = Q.cpu().numpy()
    return [_unpack(Qh, i.Q_off, i.n_rows, i.n_cols) for i in infos]
