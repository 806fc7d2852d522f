"""CPU oracle for the sample-based divide-and-conquer Delaunay triangulation.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  Nothing here
imports or calls the GPU library, and the GPU library shares no code with it.

Two layers:
  * dt_oracle.c (plain C, loaded with ctypes): exact predicates and a plain
    Bowyer-Watson Delaunay triangulation -- the plain definition of what the
    whole method must reproduce (paper, Section "Delaunay Triangulations":
    no input point strictly inside any simplex's circumsphere; unique under
    the symbolic perturbation described in dt_oracle.c).
  * numpy functions below: the deterministic per-stage steps of the method,
    each written from its passage in the paper, step by step:
      - sample_ids          Algorithm 2, the random sample of eta(n) points
      - graph_edges/weights Algorithm 2 + Table "weights", DT edges as graph
      - nearest_sample      Algorithm 2, nearest sample point of every point
      - buckets             Algorithm 2, the partitions P_1..P_k
      - kd_divide           Section "Recursive Bisection": cyclic median split
      - merge               Algorithm 1, "Merging"
      - partition metrics   Section "Partitioning Quality" (deviation, c_v,
                            o_DT, cut weight)
      - certify             Section "Delaunay Triangulations": a certificate
                            that a claimed simplex set is DT(P), for sizes
                            beyond the plain triangulation's reach
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, INVALID, NONFINITE, DUPLICATE, DEGENERATE, NOMEM, INTERNAL = 0, -1, -2, -3, -4, -5, -7


def build(force: bool = False) -> str:
    """Compile dt_oracle.c with gcc.  Contraction of a*b+c into fused
    multiply-adds is disabled: the filters' error bounds assume every
    product and sum rounds separately."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_dt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                               ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                               ctypes.POINTER(ctypes.c_int64)]
        lib.orc_dt.restype = ctypes.c_int
        lib.orc_orient.argtypes = [ctypes.c_int, ctypes.c_void_p]
        lib.orc_orient.restype = ctypes.c_int
        lib.orc_insphere.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_insphere.restype = ctypes.c_int
        lib.orc_free.argtypes = [ctypes.c_void_p]
        lib.orc_certify.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(_Cert),
                                    ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                    ctypes.POINTER(ctypes.c_int64)]
        lib.orc_certify.restype = ctypes.c_int
        _lib = lib
    return _lib


class _Cert(ctypes.Structure):
    _fields_ = [("bad_rows", ctypes.c_int64), ("flat", ctypes.c_int64),
                ("over_shared", ctypes.c_int64), ("interior", ctypes.c_int64),
                ("hull", ctypes.c_int64), ("same_side", ctypes.c_int64),
                ("not_local", ctypes.c_int64), ("unused", ctypes.c_int64),
                ("edges", ctypes.c_int64), ("volume", ctypes.c_double)]


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status}")
        self.status = status


def neighbors(rows: np.ndarray) -> np.ndarray:
    """Algorithm 1, neighbourhood update, by its definition: two simplices
    are neighbours when they share a facet (D of their D+1 vertices).
    Entry (i, j) is the row sharing the facet of row i opposite its j-th
    vertex, -1 when no other row has that facet (a convex-hull facet)."""
    rows = np.asarray(rows, dtype=np.int64)
    m, w = rows.shape
    out = np.full((m, w), -1, dtype=np.int64)
    seen = {}
    for i in range(m):
        for j in range(w):
            f = tuple(sorted(int(rows[i, r]) for r in range(w) if r != j))
            if f in seen:
                i2, j2 = seen.pop(f)
                out[i, j] = i2
                out[i2, j2] = i
            else:
                seen[f] = (i, j)
    return out


def canonical(simplices: np.ndarray) -> np.ndarray:
    """Sort ids inside each row, then rows lexicographically."""
    s = np.sort(np.asarray(simplices, dtype=np.int64), axis=1)
    if len(s) == 0:
        return s
    order = np.lexsort(s.T[::-1])
    return s[order]


def delaunay(points: np.ndarray, ids: np.ndarray | None = None) -> np.ndarray:
    """Finite simplices of DT(points) as canonical rows of ids.

    ids: global ids of the points (perturbation order and output labels);
    default 0..n-1."""
    lib = _load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, dim = pts.shape
    if ids is None:
        ids = np.arange(n, dtype=np.int64)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = ctypes.POINTER(ctypes.c_int32)()
    m = ctypes.c_int64(0)
    st = lib.orc_dt(pts.ctypes.data, ids.ctypes.data, n, dim, ctypes.byref(out), ctypes.byref(m))
    if st != OK:
        raise OracleError(st)
    try:
        arr = np.ctypeslib.as_array(out, shape=(m.value * (dim + 1),)).copy() if m.value else \
            np.zeros(0, np.int32)
    finally:
        lib.orc_free(out)
    loc = arr.reshape(-1, dim + 1).astype(np.int64)
    return canonical(ids[loc])


def certify(points: np.ndarray, rows: np.ndarray, ids: np.ndarray | None = None) -> dict:
    """Certificate that `rows` (m x (D+1) point indices) is DT(points)
    under the perturbation of `delaunay` (Section "Delaunay
    Triangulations"), computed in dt_oracle.c: counts of invalid rows, flat
    simplices, facets in more than two simplices, interior facets whose
    simplices lie on one side, interior facets that are not locally
    Delaunay, unused points; the number of edges, interior and hull facets;
    the summed volume; and the hull facets as sorted rows of D indices.
    The caller compares the hull facets and the volume with the convex
    hull.  ids: perturbation order (default: the index)."""
    lib = _load()
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, dim = pts.shape
    r = np.ascontiguousarray(rows, dtype=np.int32)
    if r.ndim != 2 or r.shape[1] != dim + 1:
        raise ValueError("rows must be m x (D+1)")
    k = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
    c = _Cert()
    hp = ctypes.POINTER(ctypes.c_int32)()
    nh = ctypes.c_int64(0)
    st = lib.orc_certify(pts.ctypes.data, None if k is None else k.ctypes.data, n, dim,
                         r.ctypes.data, len(r), ctypes.byref(c), ctypes.byref(hp), ctypes.byref(nh))
    if st != OK:
        raise OracleError(st)
    try:
        hull = np.ctypeslib.as_array(hp, shape=(nh.value * dim,)).copy() if nh.value else \
            np.zeros(0, np.int32)
    finally:
        lib.orc_free(hp)
    out = {f: getattr(c, f) for f, _ in _Cert._fields_}
    out["hull_facets"] = hull.reshape(-1, dim).astype(np.int64)
    out["n"], out["m"], out["dim"] = n, len(r), dim
    return out


def certificate_ok(cert: dict, hull_facets: np.ndarray, hull_volume: float,
                   rtol: float = 1e-9) -> list[str]:
    """The conditions under which a certified row set is DT(P): no
    violation counts, the hull facets equal the convex hull's (sorted rows),
    the volume equals the hull's, and the Euler characteristic of a
    triangulated D-ball (V - E + F - T = 1 in 3D, V - E + F = 1 in 2D).
    Returns the failed conditions (empty when all hold)."""
    bad = [f for f in ("bad_rows", "flat", "over_shared", "same_side", "not_local", "unused")
           if cert[f]]
    mine = np.unique(np.sort(np.asarray(cert["hull_facets"]), axis=1), axis=0)
    want = np.unique(np.sort(np.asarray(hull_facets, dtype=np.int64), axis=1), axis=0)
    if mine.shape != want.shape or not np.array_equal(mine, want):
        bad.append("hull_facets")
    if not abs(cert["volume"] - hull_volume) <= rtol * abs(hull_volume):
        bad.append("volume")
    v = cert["n"] - cert["unused"]
    if cert["dim"] == 3:
        chi = v - cert["edges"] + (cert["interior"] + cert["hull"]) - cert["m"]
    else:
        chi = v - cert["edges"] + cert["m"]
    if chi != 1:
        bad.append("euler")
    return bad


def orient(pts: np.ndarray) -> int:
    """Exact sign of Orient1(p_0..p_D) = det[p_i 1]."""
    p = np.ascontiguousarray(pts, dtype=np.float64)
    return _load().orc_orient(p.shape[1], p.ctypes.data)


def insphere(pts: np.ndarray, keys: np.ndarray | None = None) -> int:
    """Exact sign of In(p_0..p_D, q) = det[p_i |p_i|^2 1; q |q|^2 1]; with
    keys, the sign under the perturbed lifting (smaller key = larger
    perturbation)."""
    p = np.ascontiguousarray(pts, dtype=np.float64)
    k = None if keys is None else np.ascontiguousarray(keys, dtype=np.int64)
    return _load().orc_insphere(p.shape[1], p.ctypes.data, None if k is None else k.ctypes.data)


# ---------------------------------------------------------------------------
# Per-stage references (numpy).
# ---------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014), elementwise, uint64."""
    z = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def sample_size(n: int, rate: float, dim: int) -> int:
    """eta = round-half-up(rate * n), at least dim + 2, at most n; rate 0
    selects the paper's default sqrt(n) (Section "Sample Size")."""
    if rate == 0:
        eta = int(np.floor(np.sqrt(n) + 0.5))
    else:
        eta = int(np.floor(rate * n + 0.5))
    return int(min(n, max(eta, dim + 2)))


def sample_keys(n: int, seed: int) -> np.ndarray:
    """Random key of every point: splitmix64(seed xor id*golden)."""
    with np.errstate(over="ignore"):
        ids = np.arange(n, dtype=np.uint64)
        x = np.uint64(seed) ^ (ids * np.uint64(0x9E3779B97F4A7C15))
        return splitmix64(x)


def sample_ids(n: int, eta: int, seed: int) -> np.ndarray:
    """Algorithm 2: choose eta(n) points uniformly at random without
    replacement -- here the eta points with the smallest random keys (ties by
    id), returned in ascending id order."""
    keys = sample_keys(n, seed)
    order = np.lexsort((np.arange(n), keys))
    return np.sort(order[:eta]).astype(np.int64)


def graph_edges(simplices: np.ndarray) -> np.ndarray:
    """Algorithm 2: E = the edges of the sample triangulation, as unique
    sorted pairs (u < v) of the ids appearing in `simplices`."""
    s = np.asarray(simplices, dtype=np.int64)
    k = s.shape[1]
    pairs = [s[:, [i, j]] for i in range(k) for j in range(i + 1, k)]
    e = np.sort(np.concatenate(pairs, axis=0), axis=1)
    return np.unique(e, axis=0)


def edge_weights(points: np.ndarray, edges: np.ndarray, kind: str = "log",
                 dstar: float | None = None) -> np.ndarray:
    """Table "weights": d = |v-w| / d*, d* = length of the maximum diagonal
    (of the input's bounding box).  log: -ln d; const: 1; inverse: 1/d;
    linear: 1 - d."""
    p = np.asarray(points, dtype=np.float64)
    if dstar is None:
        dstar = float(np.linalg.norm(p.max(axis=0) - p.min(axis=0)))
    d = np.linalg.norm(p[edges[:, 0]] - p[edges[:, 1]], axis=1) / dstar
    if kind == "log":
        return -np.log(d)
    if kind == "const":
        return np.ones_like(d)
    if kind == "inverse":
        return 1.0 / d
    if kind == "linear":
        return 1.0 - d
    raise ValueError(kind)


def nearest_sample(points: np.ndarray, sample_pts: np.ndarray,
                   sample_id: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """Algorithm 2: the nearest sample point of every point.  The distance
    key is (fl(d^2), sample id), d^2 = ((dx*dx) + (dy*dy)) + (dz*dz) with
    each operation rounded separately; the minimum key wins.  Returns the
    index into sample_pts."""
    p = np.asarray(points, dtype=np.float64)
    s = np.asarray(sample_pts, dtype=np.float64)
    sid = np.asarray(sample_id, dtype=np.int64)
    out = np.empty(len(p), dtype=np.int64)
    for a in range(0, len(p), chunk):
        q = p[a:a + chunk]
        d2 = None
        for k in range(p.shape[1]):
            dk = q[:, None, k] - s[None, :, k]
            t = dk * dk
            d2 = t if d2 is None else d2 + t
        best = d2.min(axis=1)
        cand = d2 == best[:, None]
        ids = np.where(cand, sid[None, :], np.iinfo(np.int64).max)
        out[a:a + chunk] = np.argmin(ids, axis=1)
    return out


def buckets(pid: np.ndarray, k: int) -> list[np.ndarray]:
    """Algorithm 2: the partitions P_1..P_k -- P_i holds the points whose
    nearest sample lies in block i.  Returned as ascending index arrays in
    block order; the method fixes no order of the points inside a block."""
    pid = np.asarray(pid, dtype=np.int64)
    return [np.nonzero(pid == i)[0] for i in range(k)]


def kd_divide(points: np.ndarray, k: int) -> np.ndarray:
    """Section "Recursive Bisection": recursive median split with cyclic
    split dimension (x, y, z, x, ...) starting with x; the lower half of a
    block of m points is the floor(m/2) points with the smallest
    (coordinate, id) keys.  k must be a power of two; returns pid with the
    box index (leaves numbered left to right)."""
    p = np.asarray(points, dtype=np.float64)
    n, dim = p.shape
    levels = int(round(np.log2(k)))
    if 1 << levels != k:
        raise ValueError("k must be a power of two")
    pid = np.zeros(n, dtype=np.int64)
    blocks = [np.arange(n)]
    for lev in range(levels):
        ax = lev % dim
        nb = []
        for b in blocks:
            order = b[np.lexsort((b, p[b, ax]))]
            h = len(b) // 2
            nb.append(order[:h])
            nb.append(order[h:])
        blocks = nb
    for i, b in enumerate(blocks):
        pid[b] = i
    return pid


def merge(parts: list[np.ndarray], flags: list[np.ndarray], border: np.ndarray,
          pid_of: np.ndarray) -> np.ndarray:
    """Algorithm 1, "Merging": T = (union T_i) minus B, plus every border
    simplex that spans several partitions or equals a simplex of B.
    parts[i]: canonical rows of T_i; flags[i]: bool per row (in B);
    border: canonical rows of T_B; pid_of: partition of every global id."""
    keep = [t[~f] for t, f in zip(parts, flags)]
    bset = set()
    for t, f in zip(parts, flags):
        for row in t[f]:
            bset.add(tuple(int(x) for x in row))
    extra = []
    for row in border:
        ps = pid_of[row]
        if (ps != ps[0]).any() or tuple(int(x) for x in row) in bset:
            extra.append(row)
    allr = keep + ([np.asarray(extra, dtype=np.int64)] if extra else [])
    dim1 = border.shape[1] if border.ndim == 2 else parts[0].shape[1]
    allr = [a.reshape(-1, dim1) for a in allr]
    return canonical(np.concatenate(allr, axis=0) if allr else np.zeros((0, dim1), np.int64))


def deviation(sizes: np.ndarray) -> np.ndarray:
    """Section "Partitioning Quality": p_i / (N/k) - 1."""
    s = np.asarray(sizes, dtype=np.float64)
    return s / (s.sum() / len(s)) - 1.0


def coeff_variation(sizes: np.ndarray) -> float:
    """Section "Partitioning Quality": c_v = sigma/mu with the k-1
    denominator in sigma."""
    s = np.asarray(sizes, dtype=np.float64)
    k = len(s)
    mu = s.sum() / k
    return float(np.sqrt(((s - mu) ** 2).sum() / (k - 1)) / mu)


def overtriangulation(n: int, eta: int, border_vertices: int) -> float:
    """Section "Partitioning Quality": o_DT = (|P| + |P_S| + |vertices(B)|)/|P|
    for one sample and one border triangulation."""
    return (n + eta + border_vertices) / n


def cut_weight(edges: np.ndarray, weights: np.ndarray, part: np.ndarray) -> float:
    """Section "Partitioning Quality": sum of the weights of edges whose
    endpoints lie in different blocks.  `part` is indexed by edge endpoint."""
    e = np.asarray(edges)
    return float(np.asarray(weights)[part[e[:, 0]] != part[e[:, 1]]].sum())


def balanced(part: np.ndarray, k: int, eps: float) -> bool:
    """Section "Sample-based Partitioning": |V_i| <= (1+eps) ceil(|V|/k)."""
    cnt = np.bincount(np.asarray(part), minlength=k)
    return bool(cnt.max() <= (1.0 + eps) * np.ceil(len(part) / k))
