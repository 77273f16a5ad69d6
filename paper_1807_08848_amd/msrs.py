"""Thin Python binding of the msrs C ABI (include/msrs.h).

Argument marshalling only: every computation runs in libmsrs.so's HIP
kernels.  Device arrays are torch CUDA tensors (float64, contiguous); the
stream is torch's current stream unless one is given.  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsrs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1807_08848_amd.build`")

# torch first: its HIP runtime then satisfies libmsrs.so's runtime dependency,
# so that one runtime instance serves both (torch streams are valid handles
# and stream order spans torch's work and the library's kernels).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

(OK, ERR_ARG, ERR_STATE, ERR_OOM, ERR_HIP, ERR_NO_DEVICE, ERR_NOT_SPD, ERR_NOCONV, ERR_RANK, ERR_BUSY, ERR_IO,
 ERR_NONFINITE) = range(12)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_STATE", 3: "ERR_OOM", 4: "ERR_HIP", 5: "ERR_NO_DEVICE",
                6: "ERR_NOT_SPD", 7: "ERR_NOCONV", 8: "ERR_RANK", 9: "ERR_BUSY", 10: "ERR_IO", 11: "ERR_NONFINITE"}
KIND_ELLIPTIC_Q1, KIND_KINETIC_DO = 0, 1
PREC_FP64, PREC_FP32_IR = 0, 1
FLAG_FULL_BASIS_ENDS, FLAG_PER_PATCH_LAUNCH, FLAG_TIMING, FLAG_FULL_BASIS_BOUNDARY = 1, 2, 4, 8
FLAG_CONSTRAINED_BC = 16
FLAG_FULL_BASIS = 32
FLAG_TWO_PASS = 64
FLAG_LS_NORMAL, FLAG_LS_CORRECTED = 128, 256
TUNE_SWEEP_COLS, TUNE_RECON_BATCH, TUNE_APPLY_BATCH, TUNE_FACTOR_SHARE = 0, 1, 2, 3
TUNE_STAGE_OFFLINE, TUNE_STAGE_ONLINE = 0, 1
TUNE_NAMES = {TUNE_SWEEP_COLS: "sweep_cols", TUNE_RECON_BATCH: "recon_batch", TUNE_APPLY_BATCH: "apply_batch",
              TUNE_FACTOR_SHARE: "factor_share"}
K_CLASSES = ["assemble", "omega", "lift", "factor", "sweep", "residual", "restrict", "range",
             "coarse", "csolve", "recon", "graph"]


class ProblemDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_cells", C.c_int32), ("M", C.c_int32), ("n_samples", C.c_int32),
                ("rank", C.c_int32), ("precision", C.c_int32), ("ir_max_iters", C.c_int32), ("n_vel", C.c_int32),
                ("seed", C.c_uint64), ("ir_tol", C.c_double), ("eps", C.c_double),
                ("overlap", C.POINTER(C.c_int32)), ("flags", C.c_uint32), ("reserved", C.c_int32),
                ("hg_g", C.c_double), ("rank_tol", C.c_double), ("ir_stop", C.c_double)]


class Layout(C.Structure):
    _fields_ = [("n_patches", C.c_int32), ("n_samples", C.c_int32), ("rank", C.c_int32), ("n_bdry", C.c_int32),
                ("n_nodes", C.c_int64), ("omega_total", C.c_int64), ("Y_total", C.c_int64), ("Q_total", C.c_int64),
                ("sv_total", C.c_int64), ("coarse_dim", C.c_int64), ("device_bytes", C.c_int64)]


class PatchInfo(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("cx", C.c_int32), ("cy", C.c_int32),
                ("kx0", C.c_int32), ("ky0", C.c_int32), ("nH", C.c_int32), ("n_bdry", C.c_int32),
                ("n_rows", C.c_int32), ("n_cols", C.c_int32), ("full_basis", C.c_int32), ("line_len", C.c_int32),
                ("n_lines", C.c_int32), ("n_samples", C.c_int32),
                ("omega_off", C.c_int64), ("Y_off", C.c_int64), ("Q_off", C.c_int64), ("sv_off", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("ir_iters", C.c_int32), ("error_latched", C.c_int32), ("max_rel_residual", C.c_double),
                ("min_rel_gap", C.c_double), ("kernel_ms", C.c_double * 12), ("kernel_launches", C.c_int64 * 12)]


class ServerConfig(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("max_batch", C.c_int32), ("max_pending", C.c_int32),
                ("idle_spin_us", C.c_int32), ("slot_bytes", C.c_size_t), ("staging_bytes", C.c_size_t)]


class RequestInfo(C.Structure):
    _fields_ = [("model", C.c_int32), ("status", C.c_int32), ("batch_size", C.c_int32), ("stream", C.c_int32),
                ("t_arrival", C.c_double), ("t_admit", C.c_double), ("t_launch", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("max_in_flight", C.c_int64), ("peak_slot_bytes", C.c_int64), ("slot_capacity", C.c_int64),
                ("admission_waits", C.c_int64), ("mean_batch", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("n_trials", C.c_int32), ("key", C.c_int32 * 32), ("value", C.c_int32 * 32), ("ms", C.c_double * 32)]


_H = C.c_void_p
_P = C.c_void_p
_sig = {
    "msrs_version": (C.c_int32, []),
    "msrs_device_count": (C.c_int32, []),
    "msrs_create": (C.c_int32, [C.POINTER(_H), C.POINTER(ProblemDesc), _P, C.c_size_t]),
    "msrs_assemble_patch": (C.c_int32, [_H, _P]),
    "msrs_sample_local_solutions": (C.c_int32, [_H, _P, _P]),
    "msrs_range_finder": (C.c_int32, [_H, _P, _P]),
    "msrs_assemble_coarse": (C.c_int32, [_H]),
    "msrs_solve_global": (C.c_int32, [_H, C.c_int32, _P, _P, _P]),
    "msrs_solve_global_banded": (C.c_int32, [_H, C.c_int32, _P, _P, _P]),
    "msrs_coarse_condition": (C.c_int32, [_H, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "msrs_coarse_corrected": (C.c_int32, [_H, C.POINTER(C.c_int32)]),
    "msrs_solve_global_noalloc": (C.c_int32, [_H, C.c_int32, _P, _P, _P]),
    "msrs_server_clock": (C.c_double, []),
    "msrs_server_last_error": (C.c_char_p, []),
    "msrs_server_create": (C.c_int32, [C.POINTER(_H), C.POINTER(_H), C.c_int32, C.POINTER(ServerConfig)]),
    "msrs_server_submit": (C.c_int32, [_H, C.c_int32, _P, C.c_double, C.POINTER(C.c_int64)]),
    "msrs_server_submit_many": (C.c_int32, [_H, C.c_int32, _P, _P, _P, _P, C.POINTER(C.c_int32)]),
    "msrs_server_replay": (C.c_int32, [_H, C.c_int32, _P, _P, _P, C.POINTER(RequestInfo)]),
    "msrs_server_wait": (C.c_int32, [_H, C.c_int64, C.c_double]),
    "msrs_server_fetch": (C.c_int32, [_H, C.c_int64, _P, C.POINTER(RequestInfo)]),
    "msrs_server_get_stats": (C.c_int32, [_H, C.POINTER(ServerStats)]),
    "msrs_server_destroy": (None, [_H]),
    "msrs_set_max_batch": (C.c_int32, [_H, C.c_int32]),
    "msrs_copy_omega": (C.c_int32, [_H, _P]),
    "msrs_draw_boundary_samples": (C.c_int32, [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P]),
    "msrs_save": (C.c_int32, [_H, C.c_char_p]),
    "msrs_load": (C.c_int32, [C.POINTER(_H), C.c_char_p, _P]),
    "msrs_copy_results": (C.c_int32, [_H, _P, _P, _P]),
    "msrs_offline_graph_capture": (C.c_int32, [_H, _P]),
    "msrs_offline_graph_launch": (C.c_int32, [_H]),
    "msrs_query_layout": (C.c_int32, [_H, C.POINTER(Layout)]),
    "msrs_set_tuning": (C.c_int32, [_H, C.c_int32, C.c_int32]),
    "msrs_get_tuning": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_int32)]),
    "msrs_autotune": (C.c_int32, [_H, C.c_int32, C.c_int32, C.POINTER(TuneReport)]),
    "msrs_query_patch": (C.c_int32, [_H, C.c_int32, C.POINTER(PatchInfo)]),
    "msrs_get_stats": (C.c_int32, [_H, C.POINTER(Stats)]),
    "msrs_reset_stats": (C.c_int32, [_H]),
    "msrs_last_error": (C.c_char_p, [_H]),
    "msrs_destroy": (None, [_H]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

lib = _lib


class MsrsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def version() -> int:
    return _lib.msrs_version()


def device_count() -> int:
    return _lib.msrs_device_count()


def _ptr(t):
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def make_desc(kind, n_cells, M, overlap, n_samples, rank, precision=PREC_FP64, seed=2, ir_tol=1e-10,
              ir_max_iters=30, n_vel=0, eps=1.0, flags=0, hg=0.0, rank_tol=0.0, ir_stop=0.0):
    ov = (C.c_int32 * len(overlap))(*[int(x) for x in overlap])
    d = ProblemDesc(kind=kind, n_cells=n_cells, M=M, n_samples=n_samples, rank=rank, precision=precision,
                    ir_max_iters=ir_max_iters, n_vel=n_vel, seed=seed, ir_tol=ir_tol, eps=eps,
                    overlap=C.cast(ov, C.POINTER(C.c_int32)), flags=flags, reserved=0, hg_g=hg, rank_tol=rank_tol,
                    ir_stop=ir_stop)
    d._keep = ov
    return d


class Problem:
    """One handle of the library (msrs_create ... msrs_destroy)."""

    def __init__(self, desc: ProblemDesc, stream=None, hbm_budget_bytes: int = 0):
        h = _H()
        st = _lib.msrs_create(C.byref(h), C.byref(desc), _stream(stream), C.c_size_t(hbm_budget_bytes))
        if st != OK:
            raise MsrsError(st, _lib.msrs_last_error(None).decode())
        self.h = h
        self.desc = desc

    def _check(self, st):
        if st != OK:
            raise MsrsError(st, _lib.msrs_last_error(self.h).decode())

    def save(self, path):
        """Write the offline product (bases, singular values, coefficients) to a basis file."""
        self._check(_lib.msrs_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, path, stream=None):
        """A handle made from a basis file, ready for assemble_coarse / solve_global."""
        h = _H()
        st = _lib.msrs_load(C.byref(h), os.fsencode(path), _stream(stream))
        if st != OK:
            raise MsrsError(st, _lib.msrs_last_error(None).decode())
        obj = cls.__new__(cls)
        obj.h = h
        obj.desc = None
        return obj

    def assemble_patch(self, coef):
        self._check(_lib.msrs_assemble_patch(self.h, _ptr(coef)))

    def sample_local_solutions(self, omega=None, Y_out=None):
        self._check(_lib.msrs_sample_local_solutions(self.h, _ptr(omega), _ptr(Y_out)))

    def range_finder(self, Q_out=None, sv_out=None):
        self._check(_lib.msrs_range_finder(self.h, _ptr(Q_out), _ptr(sv_out)))

    def copy_omega(self, out):
        self._check(_lib.msrs_copy_omega(self.h, _ptr(out)))

    def copy_results(self, Y_out=None, Q_out=None, sv_out=None):
        self._check(_lib.msrs_copy_results(self.h, _ptr(Y_out), _ptr(Q_out), _ptr(sv_out)))

    def offline_graph_capture(self, coef):
        self._check(_lib.msrs_offline_graph_capture(self.h, _ptr(coef)))

    def offline_graph_launch(self):
        self._check(_lib.msrs_offline_graph_launch(self.h))

    def assemble_coarse(self):
        self._check(_lib.msrs_assemble_coarse(self.h))

    def coarse_condition(self):
        """(1-norm condition estimate of P~^T P~, its square root) from msrs_assemble_coarse."""
        kn, kl = C.c_double(), C.c_double()
        self._check(_lib.msrs_coarse_condition(self.h, C.byref(kn), C.byref(kl)))
        return kn.value, kl.value

    def coarse_corrected(self):
        """True if the online solves take the corrected semi-normal step."""
        v = C.c_int32()
        self._check(_lib.msrs_coarse_corrected(self.h, C.byref(v)))
        return bool(v.value)

    def set_max_batch(self, n):
        self._check(_lib.msrs_set_max_batch(self.h, int(n)))

    def solve_global(self, f, u, stream=None):
        n_req = f.shape[0] if f.dim() == 2 else 1
        s = None if stream is None else _stream(stream)
        self._check(_lib.msrs_solve_global(self.h, int(n_req), _ptr(f), _ptr(u), s))

    def solve_global_noalloc(self, f, u, stream=None):
        """msrs_solve_global with the workspace in the library's fixed device array (no allocation)."""
        n_req = f.shape[0] if f.dim() == 2 else 1
        s = None if stream is None else _stream(stream)
        self._check(_lib.msrs_solve_global_noalloc(self.h, int(n_req), _ptr(f), _ptr(u), s))

    def solve_global_banded(self, f, u, stream=None):
        n_req = f.shape[0] if f.dim() == 2 else 1
        s = None if stream is None else _stream(stream)
        self._check(_lib.msrs_solve_global_banded(self.h, int(n_req), _ptr(f), _ptr(u), s))

    def set_tuning(self, key: int, value: int):
        self._check(_lib.msrs_set_tuning(self.h, int(key), int(value)))

    def get_tuning(self, key: int) -> int:
        v = C.c_int32()
        self._check(_lib.msrs_get_tuning(self.h, int(key), C.byref(v)))
        return v.value

    def autotune(self, stage: int, reps: int = 3):
        """Native autotuner (msrs_autotune): returns [(key, value, ms), ...]; the fastest is kept."""
        out = TuneReport()
        self._check(_lib.msrs_autotune(self.h, int(stage), int(reps), C.byref(out)))
        return [(out.key[i], out.value[i], out.ms[i]) for i in range(out.n_trials)]

    def layout(self) -> Layout:
        out = Layout()
        self._check(_lib.msrs_query_layout(self.h, C.byref(out)))
        return out

    def patch(self, p: int) -> PatchInfo:
        out = PatchInfo()
        self._check(_lib.msrs_query_patch(self.h, int(p), C.byref(out)))
        return out

    def stats(self, check: bool = True) -> Stats:
        out = Stats()
        st = _lib.msrs_get_stats(self.h, C.byref(out))
        if check:
            self._check(st)
        return out

    def reset_stats(self):
        self._check(_lib.msrs_reset_stats(self.h))

    def close(self):
        if getattr(self, "h", None):
            _lib.msrs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def draw_boundary_samples(seed: int, patch: int, n_node: int, n_sample: int, words=None, normals=None, stream=None):
    """The device generator of the boundary samples (msrs_draw_boundary_samples):
    words (int32 CUDA tensor of 4 n_node n_sample, the Philox output words as
    stored bits) and normals (float64 CUDA tensor of n_node n_sample), each
    optional, in Omega's column-major order."""
    def p(t, dtype):
        if t is None:
            return None
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
            raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
        return C.c_void_p(t.data_ptr())
    import torch
    st = _lib.msrs_draw_boundary_samples(C.c_uint64(seed), int(patch), int(n_node), int(n_sample),
                                         p(words, torch.int32), p(normals, torch.float64), _stream(stream))
    if st != OK:
        raise MsrsError(st, _lib.msrs_last_error(None).decode())


def server_clock() -> float:
    return _lib.msrs_server_clock()


class Server:
    """A request server over resident problems (msrs_server_create ... destroy).

    submit() takes boundary data in host memory (a float64 numpy array);
    fetch() copies the solution into a host numpy array or a CUDA tensor and
    returns the request's RequestInfo.
    """

    def __init__(self, problems, n_streams=0, max_batch=0, max_pending=0, slot_bytes=0, staging_bytes=0,
                 idle_spin_us=0):
        hs = (_H * len(problems))(*[p.h for p in problems])
        cfg = ServerConfig(n_streams=n_streams, max_batch=max_batch, max_pending=max_pending,
                           idle_spin_us=idle_spin_us, slot_bytes=slot_bytes, staging_bytes=staging_bytes)
        h = _H()
        st = _lib.msrs_server_create(C.byref(h), hs, len(problems), C.byref(cfg))
        if st != OK:
            raise MsrsError(st, _lib.msrs_server_last_error().decode())
        self.h = h
        self.problems = list(problems)

    def _check(self, st):
        if st != OK:
            raise MsrsError(st, _lib.msrs_server_last_error().decode())

    def submit(self, model: int, f, t_arrival: float = 0.0) -> int:
        import numpy as np
        f = np.ascontiguousarray(f, dtype=np.float64)
        t = C.c_int64()
        self._check(_lib.msrs_server_submit(self.h, int(model), f.ctypes.data_as(C.c_void_p), float(t_arrival), C.byref(t)))
        return t.value

    def try_submit(self, model: int, f, t_arrival: float = 0.0):
        """submit() that returns None instead of raising on ERR_BUSY (back-pressure)."""
        try:
            return self.submit(model, f, t_arrival)
        except MsrsError as e:
            if e.status == ERR_BUSY:
                return None
            raise

    def submit_many(self, models, fs, t_arrival=None):
        """Queue requests in order; returns the tickets of those queued (stops at ERR_BUSY)."""
        import numpy as np
        n = len(models)
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in fs]
        m = np.ascontiguousarray(models, dtype=np.int32)
        ptrs = (C.c_void_p * n)(*[f.ctypes.data for f in fs])
        ta = None if t_arrival is None else np.ascontiguousarray(t_arrival, dtype=np.float64)
        tk = np.zeros(n, dtype=np.int64)
        done = C.c_int32()
        st = _lib.msrs_server_submit_many(self.h, n, m.ctypes.data_as(C.c_void_p), ptrs,
                                          None if ta is None else ta.ctypes.data_as(C.c_void_p),
                                          tk.ctypes.data_as(C.c_void_p), C.byref(done))
        if st not in (OK, ERR_BUSY):
            self._check(st)
        return list(tk[:done.value])

    def replay(self, models, fs, t_arrival=None):
        """Replay an arrival trace natively (msrs_server_replay); returns the RequestInfo records."""
        import numpy as np
        n = len(models)
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in fs]
        m = np.ascontiguousarray(models, dtype=np.int32)
        ptrs = (C.c_void_p * n)(*[f.ctypes.data for f in fs])
        ta = None if t_arrival is None else np.ascontiguousarray(t_arrival, dtype=np.float64)
        infos = (RequestInfo * n)()
        self._check(_lib.msrs_server_replay(self.h, n, m.ctypes.data_as(C.c_void_p), ptrs,
                                            None if ta is None else ta.ctypes.data_as(C.c_void_p), infos))
        return list(infos)

    def wait(self, ticket: int, timeout: float = -1.0) -> bool:
        st = _lib.msrs_server_wait(self.h, int(ticket), float(timeout))
        if st == ERR_BUSY:
            return False
        self._check(st)
        return True

    def fetch(self, ticket: int, out=None) -> RequestInfo:
        info = RequestInfo()
        if out is None:
            p = None
        elif hasattr(out, "data_ptr"):
            p = _ptr(out)
        else:
            import numpy as np
            if not (out.dtype == np.float64 and out.flags["C_CONTIGUOUS"]):
                raise ValueError("expected a contiguous float64 array")
            p = out.ctypes.data_as(C.c_void_p)
        self._check(_lib.msrs_server_fetch(self.h, int(ticket), p, C.byref(info)))
        return info

    def stats(self) -> ServerStats:
        out = ServerStats()
        self._check(_lib.msrs_server_get_stats(self.h, C.byref(out)))
        return out

    def close(self):
        if getattr(self, "h", None):
            _lib.msrs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
