"""Python binding of libdt (include/dt.h): argument marshalling only.

Every step of the triangulation runs in the HIP library; this module only
converts numpy arrays / torch tensors to pointers and back.  Device inputs
are torch tensors on a ROCm device (torch is used for device memory and
streams); host inputs are numpy arrays.  If libdt.so has not been built the
calls raise -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdt.so")
_lib = None

DT_OK, DT_E_INVALID_ARG, DT_E_NONFINITE, DT_E_DUPLICATE, DT_E_DEGENERATE = 0, -1, -2, -3, -4
DT_E_NOMEM, DT_E_DEVICE, DT_E_INTERNAL, DT_E_NOT_READY = -5, -6, -7, -8
DIVIDE = {"sample": 0, "kd": 1, "auto": 2}
WEIGHT = {"log": 0, "const": 1, "inverse": 2, "linear": 3}
PRECISION = {"fp64": 0, "fp32": 1}
BORDER = {"region": 0, "grid": 1, "bbox": 2, "exact": 3, "refined": 4}
STAGES = ["validate", "sample", "sample_dt", "partition", "assign", "scatter", "local_dt",
          "border", "border_dt", "merge", "output", "total"]
KERNELS = ["k4_pick", "k4_cavity", "k4_insert", "assign", "bucket", "border", "merge",
           "k4_select"]
ARR = {"sample": 0, "sample_dt": 1, "part": 2, "pid": 3, "order": 4, "border_v": 5,
       "local": 6, "border_dt": 7, "nearest": 8, "graph": 9, "weights": 10}
EXPORTS = ["dt_default_options", "dt_strerror", "dt_triangulate", "dt_result_count",
           "dt_result_dim", "dt_result_copy", "dt_result_stats", "dt_result_free",
           "dt_result_stage", "dt_batch_triangulate", "dt_result_set_offsets",
           "dt_server_create", "dt_server_submit", "dt_server_poll", "dt_server_wait",
           "dt_server_times", "dt_server_destroy", "dt_batch_autotune", "dt_result_neighbors",
           "dt_release_cached_memory", "dt_predicates", "dt_triangulate_noalloc"]
NOALLOC_MAX_POINTS = {2: 131072, 3: 49152}


class Options(ctypes.Structure):
    _fields_ = [("divide", ctypes.c_int), ("weight", ctypes.c_int), ("precision", ctypes.c_int),
                ("sort_output", ctypes.c_int), ("eps", ctypes.c_double),
                ("grid_cell", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("refine_iters", ctypes.c_int), ("keep_stages", ctypes.c_int),
                ("border", ctypes.c_int), ("profile", ctypes.c_int),
                ("start_active", ctypes.c_int), ("grow_div", ctypes.c_int),
                ("cand_blocks", ctypes.c_int), ("grow_num", ctypes.c_int),
                ("recursive", ctypes.c_int), ("gift_wrap", ctypes.c_int),
                ("refine_swaps", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("eta", ctypes.c_int64), ("num_simplices", ctypes.c_int64),
                ("border_simplices", ctypes.c_int64), ("border_vertices", ctypes.c_int64),
                ("tb_simplices", ctypes.c_int64), ("local_simplices", ctypes.c_int64),
                ("k", ctypes.c_int32), ("D", ctypes.c_int32), ("cv", ctypes.c_double),
                ("max_dev", ctypes.c_double), ("o_dt", ctypes.c_double),
                ("cut_weight", ctypes.c_double), ("max_part", ctypes.c_int64),
                ("min_part", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("pred", (ctypes.c_int64 * 4) * 4), ("fail", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("stage_ms", ctypes.c_double * 12),
                ("probe_hist", ctypes.c_int64 * 16), ("kern_ms", ctypes.c_double * 8),
                ("kern_launches", ctypes.c_int64 * 8), ("cavity_cells", ctypes.c_int64),
                ("candidates", ctypes.c_int64),
                ("divide_used", ctypes.c_int64), ("divide_stat", ctypes.c_double),
                ("large_cavities", ctypes.c_int64), ("wrap_levels", ctypes.c_int64),
                ("seeded_sets", ctypes.c_int64)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_
             if f not in ("pred", "stage_ms", "probe_hist", "pad", "kern_ms", "kern_launches")}
        names = ["orient2d", "orient3d", "insphere2d", "insphere3d"]
        d["pred"] = {names[i]: {"calls": self.pred[i][0], "fp32": self.pred[i][1],
                                "fp64": self.pred[i][2], "exact": self.pred[i][3]}
                     for i in range(4)}
        d["stage_ms"] = {STAGES[i]: self.stage_ms[i] for i in range(12)}
        d["probe_hist"] = list(self.probe_hist)
        d["kern"] = {KERNELS[i]: {"ms": self.kern_ms[i], "launches": self.kern_launches[i]}
                     for i in range(len(KERNELS))}
        return d


class DTError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"libdt status {status}: {strerror(status)} {msg}".strip())
        self.status = status


def load():
    """Load libdt.so (built by paper_1902_07554_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1902_07554_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, VP = ctypes.POINTER, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.dt_default_options.argtypes = [P(Options)]
    lib.dt_default_options.restype = None
    lib.dt_strerror.argtypes = [I]
    lib.dt_strerror.restype = ctypes.c_char_p
    lib.dt_triangulate.argtypes = [VP, I64, I, I, D, P(Options), I, VP, P(VP)]
    lib.dt_triangulate.restype = I
    lib.dt_result_count.argtypes = [VP]
    lib.dt_result_count.restype = I64
    lib.dt_result_dim.argtypes = [VP]
    lib.dt_result_dim.restype = I
    lib.dt_result_copy.argtypes = [VP, VP, I64, I, VP]
    lib.dt_result_copy.restype = I
    lib.dt_result_neighbors.argtypes = [VP, VP, I64, I, VP]
    lib.dt_result_neighbors.restype = I
    lib.dt_result_stats.argtypes = [VP, P(Stats)]
    lib.dt_result_stats.restype = I
    lib.dt_result_free.argtypes = [VP]
    lib.dt_result_free.restype = None
    lib.dt_result_stage.argtypes = [VP, I, VP, I64, P(I64)]
    lib.dt_result_stage.restype = I
    lib.dt_batch_triangulate.argtypes = [VP, VP, VP, I64, I, P(Options), I, VP, P(VP)]
    lib.dt_batch_triangulate.restype = I
    lib.dt_result_set_offsets.argtypes = [VP, VP, I64]
    lib.dt_result_set_offsets.restype = I
    lib.dt_batch_autotune.argtypes = [VP, VP, I64, I, P(Options), I, VP, I64, P(Options)]
    lib.dt_batch_autotune.restype = I
    lib.dt_server_create.argtypes = [ctypes.c_size_t, P(Options), P(VP)]
    lib.dt_server_create.restype = I
    lib.dt_server_submit.argtypes = [VP, VP, I64, I, I, D, I, P(ctypes.c_uint64)]
    lib.dt_server_submit.restype = I
    lib.dt_server_poll.argtypes = [VP, ctypes.c_uint64, P(VP)]
    lib.dt_server_poll.restype = I
    lib.dt_server_wait.argtypes = [VP, ctypes.c_uint64, P(VP)]
    lib.dt_server_wait.restype = I
    lib.dt_server_times.argtypes = [VP, ctypes.c_uint64, P(D)]
    lib.dt_server_times.restype = I
    lib.dt_server_destroy.argtypes = [VP]
    lib.dt_server_destroy.restype = None
    lib.dt_triangulate_noalloc.argtypes = [VP, I64, I, P(Options), VP, I64, P(I64), VP]
    lib.dt_triangulate_noalloc.restype = I
    lib.dt_predicates.argtypes = [I, I, I, VP, VP, I64, VP, VP, VP]
    lib.dt_predicates.restype = I
    lib.dt_release_cached_memory.argtypes = []
    lib.dt_release_cached_memory.restype = I
    _lib = lib
    return lib


def release_cached_memory() -> None:
    """Free the device blocks the library keeps between calls."""
    st = load().dt_release_cached_memory()
    if st != DT_OK:
        raise DTError(st)


def strerror(status: int) -> str:
    try:
        return load().dt_strerror(status).decode()
    except Exception:
        return "?"


def options(**kw) -> Options:
    o = Options()
    load().dt_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "divide":
            v = DIVIDE[v] if isinstance(v, str) else v
        elif k == "weight":
            v = WEIGHT[v] if isinstance(v, str) else v
        elif k == "precision":
            v = PRECISION[v] if isinstance(v, str) else v
        elif k == "border":
            v = BORDER[v] if isinstance(v, str) else v
        setattr(o, k, v)
    return o


def _pointer(points):
    """(pointer, n, D, on_device, keepalive, stream) for numpy or torch input."""
    try:
        import torch
        if isinstance(points, torch.Tensor):
            if points.dtype != torch.float64 or points.dim() != 2:
                raise ValueError("points must be a float64 (n, D) tensor")
            t = points.contiguous()
            if t.is_cuda:
                return t.data_ptr(), t.shape[0], t.shape[1], 1, t, torch.cuda.current_stream(
                    t.device).cuda_stream
            a = t.numpy()
            return a.ctypes.data, a.shape[0], a.shape[1], 0, a, None
    except ImportError:
        pass
    a = np.ascontiguousarray(points, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("points must be (n, D)")
    return a.ctypes.data, a.shape[0], a.shape[1], 0, a, None


class Result:
    """Owns a dt_result handle."""

    def __init__(self, handle):
        self.h = handle

    def __del__(self):
        try:
            if self.h:
                load().dt_result_free(self.h)
        except Exception:
            pass

    @property
    def count(self) -> int:
        return int(load().dt_result_count(self.h))

    @property
    def dim(self) -> int:
        return int(load().dt_result_dim(self.h))

    def rows(self) -> np.ndarray:
        m, d = self.count, self.dim
        out = np.empty((m, d + 1), dtype=np.int32)
        st = load().dt_result_copy(self.h, out.ctypes.data, m, 0, None)
        if st != DT_OK:
            raise DTError(st)
        return out

    def neighbors(self) -> np.ndarray:
        """dt_result_neighbors: row of the simplex across the facet opposite
        each vertex, -1 on the hull."""
        m, d = self.count, self.dim
        out = np.empty((m, d + 1), dtype=np.int32)
        st = load().dt_result_neighbors(self.h, out.ctypes.data, m, 0, None)
        if st != DT_OK:
            raise DTError(st)
        return out

    def rows_device(self, device=None):
        import torch
        m, d = self.count, self.dim
        out = torch.empty((m, d + 1), dtype=torch.int32, device=device or "cuda")
        st = load().dt_result_copy(self.h, ctypes.c_void_p(out.data_ptr()), m, 1,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        if st != DT_OK:
            raise DTError(st)
        return out

    def stats(self) -> dict:
        s = Stats()
        st = load().dt_result_stats(self.h, ctypes.byref(s))
        if st != DT_OK:
            raise DTError(st)
        return s.as_dict()

    def stage(self, name: str) -> np.ndarray:
        which = ARR[name]
        cnt = ctypes.c_int64(0)
        lib = load()
        st = lib.dt_result_stage(self.h, which, None, 0, ctypes.byref(cnt))
        if st != DT_OK:
            raise DTError(st)
        dt = {"sample": np.int64, "weights": np.float64}.get(name, np.int32)
        out = np.empty(cnt.value, dtype=dt)
        if cnt.value:
            st = lib.dt_result_stage(self.h, which, out.ctypes.data, cnt.value, ctypes.byref(cnt))
            if st != DT_OK:
                raise DTError(st)
        d = self.dim
        if name in ("sample_dt", "border_dt"):
            return out.reshape(-1, d + 1)
        if name == "local":
            return out.reshape(-1, d + 2)
        if name == "graph":
            return out.reshape(-1, 2)
        return out

    def set_offsets(self, num_sets: int) -> np.ndarray:
        out = np.empty(num_sets + 1, dtype=np.int64)
        st = load().dt_result_set_offsets(self.h, out.ctypes.data, num_sets + 1)
        if st != DT_OK:
            raise DTError(st)
        return out


def predicates(kind: str, tuples, keys=None, precision: str = "fp64"):
    """dt_predicates: signs (and deciding stages) of orientation
    ("orient") or in-sphere ("insphere") tests on (q, np, D) point tuples.
    Inputs are moved to the GPU with torch; returns two numpy int8 arrays
    (sign, stage: 0 FP32 filter, 1 FP64 filter, 2 exact)."""
    import torch
    lib = load()
    t = torch.as_tensor(np.ascontiguousarray(tuples, dtype=np.float64)).cuda()
    nq, npts, d = t.shape
    kt = None
    if keys is not None:
        kt = torch.as_tensor(np.ascontiguousarray(keys, dtype=np.int64)).cuda()
        if tuple(kt.shape) != (nq, npts):
            raise ValueError("keys must be (q, np)")
    sign = torch.empty(nq, dtype=torch.int8, device=t.device)
    stage = torch.empty(nq, dtype=torch.int8, device=t.device)
    st = lib.dt_predicates({"orient": 0, "insphere": 1}[kind], d, PRECISION[precision],
                           ctypes.c_void_p(t.data_ptr()),
                           ctypes.c_void_p(kt.data_ptr()) if kt is not None else None, nq,
                           ctypes.c_void_p(sign.data_ptr()), ctypes.c_void_p(stage.data_ptr()),
                           ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream))
    if st != DT_OK:
        raise DTError(st)
    return sign.cpu().numpy(), stage.cpu().numpy()


def triangulate_noalloc(points, out=None, **opts):
    """dt_triangulate_noalloc: DT(points) with k = 1 and no allocation by
    the library.  points: a float64 (n, D) torch tensor on the GPU.  out:
    an int32 (cap, D+1) device tensor for the rows (allocated here by torch
    when None, with room for 8n rows).  Returns the rows as a device tensor
    view of `out`."""
    import torch
    lib = load()
    if not (isinstance(points, torch.Tensor) and points.is_cuda):
        raise ValueError("points must be a CUDA tensor")
    ptr, n, d, _, keep, stream = _pointer(points)
    if out is None:
        out = torch.empty((max(8 * n, 1), d + 1), dtype=torch.int32, device=points.device)
    o = options(**opts)
    cnt = ctypes.c_int64(0)
    st = lib.dt_triangulate_noalloc(ctypes.c_void_p(ptr), n, d, ctypes.byref(o),
                                    ctypes.c_void_p(out.data_ptr()), out.shape[0],
                                    ctypes.byref(cnt), ctypes.c_void_p(stream))
    del keep
    if st != DT_OK:
        raise DTError(st, f"(count {cnt.value})")
    return out[:cnt.value]


def triangulate(points, k: int = 1, sample_rate: float = 0.0, **opts) -> Result:
    """dt_triangulate: DT(points) with k partitions."""
    lib = load()
    ptr, n, d, on_dev, keep, stream = _pointer(points)
    o = options(**opts)
    h = ctypes.c_void_p()
    st = lib.dt_triangulate(ctypes.c_void_p(ptr), n, d, k, sample_rate, ctypes.byref(o), on_dev,
                            ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
    del keep
    if st != DT_OK:
        raise DTError(st)
    return Result(h)


def batch_triangulate(points, offsets, ids=None, **opts) -> Result:
    """dt_batch_triangulate: DT of every set offsets[s]..offsets[s+1]-1."""
    lib = load()
    ptr, n, d, on_dev, keep, stream = _pointer(points)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        idp = ids.ctypes.data
    o = options(**opts)
    h = ctypes.c_void_p()
    st = lib.dt_batch_triangulate(ctypes.c_void_p(ptr), idp, off.ctypes.data, len(off) - 1, d,
                                  ctypes.byref(o), on_dev,
                                  ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
    del keep
    if st != DT_OK:
        raise DTError(st)
    return Result(h)


def batch_autotune(points, offsets, sample_points: int = 0, **opts) -> dict:
    """dt_batch_autotune: the fastest launch tunables for batches like this
    one, as a dict of option values to pass to batch_triangulate."""
    lib = load()
    ptr, n, d, on_dev, keep, stream = _pointer(points)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    o = options(**opts)
    out = Options()
    st = lib.dt_batch_autotune(ctypes.c_void_p(ptr), off.ctypes.data, len(off) - 1, d,
                               ctypes.byref(o), on_dev, ctypes.c_void_p(stream) if stream else None,
                               int(sample_points), ctypes.byref(out))
    del keep
    if st != DT_OK:
        raise DTError(st)
    return {"start_active": out.start_active, "grow_div": out.grow_div,
            "cand_blocks": out.cand_blocks, "grow_num": out.grow_num}


class Server:
    """dt_server_*: continuous-batching triangulation server."""

    def __init__(self, hbm_budget_bytes: int, **opts):
        self.lib = load()
        o = options(**opts)
        self.h = ctypes.c_void_p()
        st = self.lib.dt_server_create(hbm_budget_bytes, ctypes.byref(o), ctypes.byref(self.h))
        if st != DT_OK:
            raise DTError(st)

    def submit(self, points, k: int = 1, sample_rate: float = 0.0) -> int:
        ptr, n, d, on_dev, keep, _ = _pointer(points)
        t = ctypes.c_uint64(0)
        st = self.lib.dt_server_submit(self.h, ctypes.c_void_p(ptr), n, d, k, sample_rate, on_dev,
                                       ctypes.byref(t))
        del keep
        if st != DT_OK:
            raise DTError(st)
        return t.value

    def poll(self, ticket: int):
        h = ctypes.c_void_p()
        st = self.lib.dt_server_poll(self.h, ticket, ctypes.byref(h))
        if st == DT_E_NOT_READY:
            return None
        if st != DT_OK:
            raise DTError(st)
        if not h:
            raise DTError(DT_E_INVALID_ARG, "result already taken")
        return Result(h)

    def wait(self, ticket: int) -> Result:
        h = ctypes.c_void_p()
        st = self.lib.dt_server_wait(self.h, ticket, ctypes.byref(h))
        if st != DT_OK:
            raise DTError(st)
        if not h:
            raise DTError(DT_E_INVALID_ARG, "result already taken")
        return Result(h)

    def times(self, ticket: int):
        t = (ctypes.c_double * 3)()
        st = self.lib.dt_server_times(self.h, ticket, t)
        if st != DT_OK:
            raise DTError(st)
        return tuple(t)

    def close(self):
        if self.h:
            self.lib.dt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
