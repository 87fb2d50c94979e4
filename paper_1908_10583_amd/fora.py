"""Python binding of the FORA HIP library (``libfora.so``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. PyTorch provides device memory and streams. The functions keep
the C ABI's names (``fora_build_csr``, ``fora_ssppr``, ``fora_ssppr_batch``,
...). If the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfora.so")

FORA_OK, FORA_E_ARG, FORA_E_GRAPH, FORA_E_NOMEM, FORA_E_HIP, FORA_E_OVERFLOW = 0, -1, -2, -3, -4, -5
FORA_MAX_K = 4096
FORA_MAX_BATCH = 4096


class FORAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"FORA error {code}: {msg}")
        self.code = code


class fora_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("term_violations", ctypes.c_int32),
                ("pushes", ctypes.c_int64), ("edge_ops", ctypes.c_int64),
                ("plan_entries", ctypes.c_int64), ("walks", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("r_sum", ctypes.c_double),
                ("rmax", ctypes.c_double), ("omega_unit", ctypes.c_double),
                ("t_alpha", ctypes.c_uint32), ("ms_push", ctypes.c_float),
                ("ms_plan", ctypes.c_float), ("ms_walk", ctypes.c_float),
                ("ms_topk", ctypes.c_float), ("pull_rounds", ctypes.c_uint32),
                ("balance_stopped", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class fora_query(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("k", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("eps", ctypes.c_double), ("delta", ctypes.c_double), ("pf", ctypes.c_double),
                ("rmax", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("walk_cost", ctypes.c_double)]


class fora_tuning(ctypes.Structure):
    _fields_ = [("walk_blocks_per_cu", ctypes.c_int32), ("walk_chunk", ctypes.c_int32),
                ("push_blocks_per_cu", ctypes.c_int32), ("graph_rounds", ctypes.c_int32),
                ("pull_ratio", ctypes.c_int32), ("walk_agg", ctypes.c_int32),
                ("record_ids", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class fora_views(ctypes.Structure):
    _fields_ = [("residue_fx", ctypes.c_void_p), ("reserve", ctypes.c_void_p),
                ("walk_count", ctypes.c_void_p), ("walk_weight_fx", ctypes.c_void_p),
                ("pi_hat", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, U64, F64, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                      ctypes.c_size_t)
    sig = {
        "fora_last_error": ([], ctypes.c_char_p),
        "fora_build_csr": ([I32, I64, P, P, P, ctypes.POINTER(P)], ctypes.c_int),
        "fora_free_graph": ([P], ctypes.c_int),
        "fora_graph_info": ([P, ctypes.POINTER(I32), ctypes.POINTER(I64), ctypes.POINTER(I32)],
                            ctypes.c_int),
        "fora_get_tuning": ([P, ctypes.POINTER(fora_tuning)], ctypes.c_int),
        "fora_set_tuning": ([P, ctypes.POINTER(fora_tuning)], ctypes.c_int),
        "fora_workspace_size": ([P, I32, ctypes.POINTER(SZ)], ctypes.c_int),
        "fora_workspace_views": ([P, I32, P, ctypes.POINTER(fora_views)], ctypes.c_int),
        "fora_ssppr": ([P, I32, F64, F64, F64, F64, I32, F64, U64, P, SZ, P, P,
                        ctypes.POINTER(fora_stats), P], ctypes.c_int),
        "fora_ssppr_static": ([P, I32, F64, F64, F64, F64, I32, F64, U64, P, P,
                               ctypes.POINTER(fora_stats), P], ctypes.c_int),
        "fora_ssppr_batch": ([P, I32, ctypes.POINTER(fora_query), I32, P, SZ, P, P,
                              ctypes.POINTER(fora_stats), P], ctypes.c_int),
        "fora_dist_batch": ([P, I32, ctypes.POINTER(fora_query), P, I32, P, SZ, P, P,
                             ctypes.POINTER(fora_stats), P], ctypes.c_int),
        "fora_build_index": ([P, F64, F64, ctypes.c_uint32, ctypes.c_uint32, P], ctypes.c_int),
        "fora_index_info": ([P, ctypes.POINTER(I64), ctypes.POINTER(F64), ctypes.POINTER(F64),
                             ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)],
                            ctypes.c_int),
        "fora_index_export": ([P, P, P, P], ctypes.c_int),
        "fora_topk_workspace_size": ([P, I32, I32, ctypes.POINTER(SZ)], ctypes.c_int),
        "fora_topk_batch": ([P, I32, ctypes.POINTER(fora_query), I32, P, SZ, P, P,
                             ctypes.POINTER(fora_stats), P, P, P], ctypes.c_int),
        "fora_push_only": ([P, I32, F64, F64, P, P, SZ, I32, P, P, I64,
                            ctypes.POINTER(fora_stats), P], ctypes.c_int),
        "fora_walk_only": ([P, I64, P, P, P, U32, U32, F64, P, SZ, ctypes.POINTER(U64), P],
                           ctypes.c_int),
        "fora_philox": ([I64, P, U32, U32, P, P], ctypes.c_int),
        "fora_graph_rank": ([P, P, P], ctypes.c_int),
        "fora_features": ([P, I32, P, F64, F64, F64, F64, P, P], ctypes.c_int),
        "fora_mlp_forward": ([I32, P, P, P, P, P], ctypes.c_int),
        "fora_mlp_backward": ([I32, P, P, P, P, P, P, P, P, P], ctypes.c_int),
        "fora_adam_step": ([P, P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, I32, P], ctypes.c_int),
        "fora_mlp_to_bf16": ([P, P, P], ctypes.c_int),
        "fora_mlp_forward_bf16": ([I32, P, P, P, P], ctypes.c_int),
        "fora_predict_rmax": ([P, I32, P, F64, F64, F64, F64, P, F64, F64, P, P,
                               ctypes.POINTER(I32), P], ctypes.c_int),
        "fora_push_sweep": ([P, I32, ctypes.POINTER(fora_query), I32, P, P, SZ, P, P, P],
                            ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()

EXPORTED = ["fora_last_error", "fora_build_csr", "fora_free_graph", "fora_graph_info",
            "fora_get_tuning", "fora_set_tuning",
            "fora_workspace_size", "fora_workspace_views", "fora_ssppr", "fora_ssppr_static",
            "fora_ssppr_batch",
            "fora_dist_batch",
            "fora_push_only", "fora_walk_only", "fora_philox", "fora_graph_rank", "fora_features",
            "fora_mlp_forward", "fora_mlp_backward", "fora_adam_step", "fora_mlp_to_bf16",
            "fora_mlp_forward_bf16", "fora_predict_rmax", "fora_push_sweep",
            "fora_topk_workspace_size", "fora_topk_batch", "fora_build_index",
            "fora_index_info", "fora_index_export"]

FORA_PRUNE_ZERO_HOP = 1
FORA_BALANCE = 2
FORA_USE_INDEX = 4
FORA_WALK_COUNTS = 8
FORA_MLP_FEATURES = 7
FORA_MLP_PARAMS = 4751
FORA_MLP_ACTS = 128


def FORA_MLP_SCRATCH(count: int) -> int:
    return count * 129 + (count + 255) // 256


def FORA_PREDICT_SCRATCH(count: int) -> int:
    return count * 8 + 1


def _check(rc: int):
    if rc != FORA_OK:
        raise FORAError(rc, _lib.fora_last_error().decode())


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Graph:
    """A validated CSR graph on the device (``fora_build_csr``). Keeps the CSR
    tensors alive for as long as the handle lives."""

    def __init__(self, rowptr: torch.Tensor, colidx: torch.Tensor, stream=None):
        if rowptr.dtype != torch.int32 or colidx.dtype != torch.int32:
            raise TypeError("rowptr and colidx must be int32")
        if not (rowptr.is_cuda and colidx.is_cuda):
            raise TypeError("rowptr and colidx must be device tensors")
        self.rowptr = rowptr.contiguous()
        self.colidx = colidx.contiguous()
        self.n = int(self.rowptr.numel() - 1)
        self.m = int(self.colidx.numel())
        self.device = self.rowptr.device
        h = ctypes.c_void_p()
        _check(_lib.fora_build_csr(self.n, self.m, _ptr(self.rowptr), _ptr(self.colidx),
                                   ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int32()
        m = ctypes.c_int64()
        md = ctypes.c_int32()
        _check(_lib.fora_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m),
                                    ctypes.byref(md)))
        self.max_degree = md.value

    @classmethod
    def from_numpy(cls, rowptr: np.ndarray, colidx: np.ndarray, device="cuda"):
        return cls(torch.from_numpy(np.ascontiguousarray(rowptr, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(colidx, np.int32)).to(device))

    def get_tuning(self) -> dict:
        t = fora_tuning()
        _check(_lib.fora_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = fora_tuning()
        _check(_lib.fora_get_tuning(self.handle, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(_lib.fora_set_tuning(self.handle, ctypes.byref(t)))

    def close(self):
        if getattr(self, "handle", None) is not None:
            _lib.fora_free_graph(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fora_workspace_size(g: Graph, batch: int) -> int:
    out = ctypes.c_size_t()
    _check(_lib.fora_workspace_size(g.handle, batch, ctypes.byref(out)))
    return out.value


def workspace(g: Graph, batch: int = 1) -> torch.Tensor:
    """A device byte tensor large enough for ``batch`` queries."""
    return torch.empty(fora_workspace_size(g, batch), dtype=torch.uint8, device=g.device)


def fora_workspace_views(g: Graph, batch: int, ws: torch.Tensor) -> dict:
    """Tensors aliasing the dense per-query arrays inside ``ws`` (rows of n),
    plus ``residue``: a float64 copy of the fixed-point residues (exact where
    the residue has at most 53 significant bits, else rounded to nearest)."""
    v = fora_views()
    _check(_lib.fora_workspace_views(g.handle, batch, _ptr(ws), ctypes.byref(v)))
    base = ws.data_ptr()
    cap = batch * g.n

    def view(p, dtype, itemsize):
        off = p - base
        return ws[off:off + cap * itemsize].view(dtype).view(batch, g.n)

    residue_fx = view(v.residue_fx, torch.int64, 8)  # uint64 bits, values below 2^63
    return dict(residue_fx=residue_fx,
                residue=residue_fx.double() * 2.0**-62,
                reserve=view(v.reserve, torch.float32, 4),
                walk_count=view(v.walk_count, torch.int64, 8),        # uint64 bits
                walk_weight_fx=view(v.walk_weight_fx, torch.int64, 8),  # uint64 bits
                pi_hat=view(v.pi_hat, torch.float32, 4))


@dataclass
class Result:
    ids: torch.Tensor
    vals: torch.Tensor
    stats: list | dict | None


def fora_ssppr(g: Graph, src: int, alpha: float = 0.2, eps: float = 0.5,
               delta: float | None = None, pf: float | None = None, k: int = 500,
               rmax: float | None = None, seed: int = 0, ws: torch.Tensor | None = None,
               stats: bool = False, out: tuple | None = None, stream=None,
               flags: int = 0) -> Result:
    """One query. ``flags`` (the FORA_* query flags) need the batch entry
    point, so a call with flags runs as a batch of one."""
    delta = 1.0 / g.n if delta is None else delta
    pf = 1.0 / g.n if pf is None else pf
    ws = workspace(g, 1) if ws is None else ws
    if flags:
        qs = make_queries([src], alpha=alpha, eps=eps, delta=delta, pf=pf, k=k, rmax=rmax,
                          seed=seed, n=g.n, flags=flags)
        bout = None if out is None else (out[0].view(1, k), out[1].view(1, k))
        r = fora_ssppr_batch(g, qs, kmax=k, ws=ws, stats=stats, out=bout, stream=stream)
        return Result(r.ids[0], r.vals[0], r.stats[0] if stats else None)
    if out is None:
        ids = torch.empty(k, dtype=torch.int32, device=g.device)
        vals = torch.empty(k, dtype=torch.float32, device=g.device)
    else:
        ids, vals = out
    st = fora_stats() if stats else None
    _check(_lib.fora_ssppr(g.handle, int(src), alpha, eps, delta, pf, int(k),
                           0.0 if rmax is None else float(rmax), int(seed) & (2**64 - 1),
                           _ptr(ws), ws.numel(), _ptr(ids), _ptr(vals),
                           ctypes.byref(st) if st is not None else None,
                           ctypes.c_void_p(_stream(stream))))
    return Result(ids, vals, st.as_dict() if st is not None else None)


FORA_STATIC_SCRATCH_BYTES = 128 << 20


def fora_ssppr_static(g: Graph, src: int, alpha: float = 0.2, eps: float = 0.5,
                      delta: float | None = None, pf: float | None = None, k: int = 500,
                      rmax: float | None = None, seed: int = 0, stats: bool = False,
                      out: tuple | None = None, stream=None) -> Result:
    """One query with the library's static device workspace: the call itself
    allocates no device memory (the outputs are allocated here unless
    ``out`` is given)."""
    delta = 1.0 / g.n if delta is None else delta
    pf = 1.0 / g.n if pf is None else pf
    if out is None:
        ids = torch.empty(k, dtype=torch.int32, device=g.device)
        vals = torch.empty(k, dtype=torch.float32, device=g.device)
    else:
        ids, vals = out
    st = fora_stats() if stats else None
    _check(_lib.fora_ssppr_static(g.handle, int(src), alpha, eps, delta, pf, int(k),
                                  0.0 if rmax is None else float(rmax),
                                  int(seed) & (2**64 - 1), _ptr(ids), _ptr(vals),
                                  ctypes.byref(st) if st is not None else None,
                                  ctypes.c_void_p(_stream(stream))))
    return Result(ids, vals, st.as_dict() if st is not None else None)


def make_queries(srcs, alpha=0.2, eps=0.5, delta=None, pf=None, k=500, rmax=None, seed=0,
                 n: int | None = None, flags=0, walk_cost=0.0):
    """An array of ``fora_query`` (scalars broadcast; lists give per-query values).
    flags: FORA_PRUNE_ZERO_HOP | FORA_BALANCE (Algorithm 3); walk_cost: one
    walk's cost in residue increments for FORA_BALANCE."""
    srcs = list(np.asarray(srcs).reshape(-1))
    B = len(srcs)

    def per(x, default=None):
        if x is None:
            return [default] * B
        if np.ndim(x) == 0:
            return [x] * B
        x = list(np.asarray(x).reshape(-1))
        assert len(x) == B
        return x

    delta = per(delta, None if n is None else 1.0 / n)
    pf = per(pf, None if n is None else 1.0 / n)
    arr = (fora_query * B)()
    for i, (s, a, e, d, p, kk, r, sd, fl, wc) in enumerate(
            zip(srcs, per(alpha), per(eps), delta, pf, per(k), per(rmax, 0.0), per(seed),
                per(flags), per(walk_cost))):
        arr[i].src, arr[i].k = int(s), int(kk)
        arr[i].flags, arr[i].walk_cost = int(fl), float(wc)
        arr[i].alpha, arr[i].eps = float(a), float(e)
        arr[i].delta, arr[i].pf = float(d), float(p)
        arr[i].rmax = 0.0 if r is None else float(r)
        arr[i].seed = int(sd) & (2**64 - 1)
    return arr


def fora_ssppr_batch(g: Graph, queries, kmax: int | None = None,
                     ws: torch.Tensor | None = None, stats: bool = False,
                     out: tuple | None = None, stream=None) -> Result:
    B = len(queries)
    kmax = max(q.k for q in queries) if kmax is None else kmax
    ws = workspace(g, B) if ws is None else ws
    if out is None:
        ids = torch.empty((B, kmax), dtype=torch.int32, device=g.device)
        vals = torch.empty((B, kmax), dtype=torch.float32, device=g.device)
    else:
        ids, vals = out
    st = (fora_stats * B)() if stats else None
    _check(_lib.fora_ssppr_batch(g.handle, B, queries, kmax, _ptr(ws), ws.numel(), _ptr(ids),
                                 _ptr(vals), st, ctypes.c_void_p(_stream(stream))))
    return Result(ids, vals, [s.as_dict() for s in st] if st is not None else None)


def fora_dist_batch(g: Graph, queries, sigma: torch.Tensor, kmax: int | None = None,
                    ws: torch.Tensor | None = None, stats: bool = False,
                    out: tuple | None = None, stream=None) -> Result:
    """FORA for source distributions: query b starts from r = sigma[b]
    (float64 [batch, n] on the graph's device); the queries' src fields are
    not used."""
    B = len(queries)
    sigma = sigma.to(device=g.device, dtype=torch.float64).contiguous()
    if tuple(sigma.shape) != (B, g.n):
        raise ValueError(f"sigma must have shape ({B}, {g.n})")
    kmax = max(q.k for q in queries) if kmax is None else kmax
    ws = workspace(g, B) if ws is None else ws
    if out is None:
        ids = torch.empty((B, kmax), dtype=torch.int32, device=g.device)
        vals = torch.empty((B, kmax), dtype=torch.float32, device=g.device)
    else:
        ids, vals = out
    st = (fora_stats * B)() if stats else None
    _check(_lib.fora_dist_batch(g.handle, B, queries, _ptr(sigma), kmax, _ptr(ws), ws.numel(),
                                _ptr(ids), _ptr(vals), st, ctypes.c_void_p(_stream(stream))))
    return Result(ids, vals, [s.as_dict() for s in st] if st is not None else None)


def pagerank(g: Graph, alpha: float = 0.2, eps: float = 0.5, delta: float | None = None,
             pf: float | None = None, k: int = 500, seed: int = 0, flags: int = 0,
             ws: torch.Tensor | None = None, stats: bool = False) -> Result:
    """Global PageRank with FORA: the source distribution (1/n, ..., 1/n)."""
    qs = make_queries([0], alpha=alpha, eps=eps, delta=delta, pf=pf, k=k, seed=seed, n=g.n,
                      flags=flags)
    sigma = torch.full((1, g.n), 1.0 / g.n, dtype=torch.float64, device=g.device)
    r = fora_dist_batch(g, qs, sigma, kmax=k, ws=ws, stats=stats)
    return Result(r.ids[0], r.vals[0], r.stats[0] if stats else None)


def fora_build_index(g: Graph, alpha: float, walks_per_degree: float, key0: int, key1: int,
                     stream=None):
    """Builds the graph's FORA+ walk-destination index (section 3.3)."""
    _check(_lib.fora_build_index(g.handle, alpha, walks_per_degree, key0 & 0xFFFFFFFF,
                                 key1 & 0xFFFFFFFF, ctypes.c_void_p(_stream(stream))))


def fora_index_info(g: Graph) -> dict:
    t, a, w = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    k0, k1 = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_lib.fora_index_info(g.handle, ctypes.byref(t), ctypes.byref(a), ctypes.byref(w),
                                ctypes.byref(k0), ctypes.byref(k1)))
    return dict(total=t.value, alpha=a.value, walks_per_degree=w.value, key=(k0.value, k1.value))


def fora_index_export(g: Graph, stream=None):
    """Copies of the index: offsets (int64 tensor holding uint64, n + 1) and
    end points (int32 tensor)."""
    total = fora_index_info(g)["total"]
    off = torch.empty(g.n + 1, dtype=torch.int64, device=g.device)
    dest = torch.empty(max(total, 1), dtype=torch.int32, device=g.device)
    _check(_lib.fora_index_export(g.handle, _ptr(off), _ptr(dest),
                                  ctypes.c_void_p(_stream(stream))))
    return off, dest[:total]


def fora_topk_workspace_size(g: Graph, batch: int, kmax: int) -> int:
    out = ctypes.c_size_t()
    _check(_lib.fora_topk_workspace_size(g.handle, batch, kmax, ctypes.byref(out)))
    return out.value


def fora_topk_batch(g: Graph, queries, kmax: int | None = None, ws: torch.Tensor | None = None,
                    stats: bool = False, out: tuple | None = None, stream=None):
    """Top-k FORA (Algorithm 5) for every query; returns (Result, iterations,
    final delta) with the last two as numpy arrays."""
    B = len(queries)
    kmax = max(q.k for q in queries) if kmax is None else kmax
    if ws is None:
        ws = torch.empty(fora_topk_workspace_size(g, B, kmax), dtype=torch.uint8,
                         device=g.device)
    if out is None:
        ids = torch.empty((B, kmax), dtype=torch.int32, device=g.device)
        vals = torch.empty((B, kmax), dtype=torch.float32, device=g.device)
    else:
        ids, vals = out
    st = (fora_stats * B)() if stats else None
    iters = np.zeros(B, np.int32)
    delta = np.zeros(B, np.float64)
    _check(_lib.fora_topk_batch(g.handle, B, queries, kmax, _ptr(ws), ws.numel(), _ptr(ids),
                                _ptr(vals), st, iters.ctypes.data_as(ctypes.c_void_p),
                                delta.ctypes.data_as(ctypes.c_void_p),
                                ctypes.c_void_p(_stream(stream))))
    return (Result(ids, vals, [s.as_dict() for s in st] if st is not None else None), iters,
            delta)


def fora_push_only(g: Graph, src: int, alpha: float, rmax: float,
                   ws: torch.Tensor | None = None, max_rounds: int = 4096,
                   log_frontiers: bool = False, frontier_cap: int | None = None, stream=None,
                   sigma: torch.Tensor | None = None):
    """The push phase alone; with ``sigma`` (float64 [n] on the device) the
    push of that source distribution (``src`` is then not used)."""
    ws = workspace(g, 1) if ws is None else ws
    if sigma is not None:
        sigma = sigma.to(device=g.device, dtype=torch.float64).contiguous().view(-1)
        if sigma.numel() != g.n:
            raise ValueError(f"sigma must have {g.n} entries")
    sizes = np.zeros(max_rounds, np.int32)
    cap = frontier_cap if frontier_cap is not None else 64 * g.n
    flog = torch.empty(cap, dtype=torch.int32, device=g.device) if log_frontiers else None
    st = fora_stats()
    _check(_lib.fora_push_only(g.handle, int(src), alpha, rmax, _ptr(sigma), _ptr(ws), ws.numel(),
                               max_rounds, sizes.ctypes.data_as(ctypes.c_void_p), _ptr(flog),
                               cap if log_frontiers else 0, ctypes.byref(st),
                               ctypes.c_void_p(_stream(stream))))
    v = fora_workspace_views(g, 1, ws)
    out = dict(r=v["residue"][0], r_fx=v["residue_fx"][0], q=v["reserve"][0], stats=st.as_dict(),
               round_sizes=sizes[:st.rounds].copy())
    if log_frontiers:
        offs = np.concatenate([[0], np.cumsum(out["round_sizes"])])
        host = flog[:int(offs[-1])].cpu().numpy()
        out["frontiers"] = [np.sort(host[offs[i]:offs[i + 1]]) for i in range(st.rounds)]
    return out


def fora_walk_only(g: Graph, plan_v, plan_omega, plan_w, key0: int, key1: int,
                   alpha: float, ws: torch.Tensor | None = None, stream=None):
    ws = workspace(g, 1) if ws is None else ws
    dv = torch.as_tensor(np.ascontiguousarray(plan_v, np.int32)).to(g.device)
    do = torch.as_tensor(np.ascontiguousarray(plan_omega, np.uint64).view(np.int64)).to(g.device)
    dw = torch.as_tensor(np.ascontiguousarray(plan_w, np.float64)).to(g.device)
    steps = ctypes.c_uint64()
    _check(_lib.fora_walk_only(g.handle, int(dv.numel()), _ptr(dv), _ptr(do), _ptr(dw),
                               key0 & 0xFFFFFFFF, key1 & 0xFFFFFFFF, alpha, _ptr(ws),
                               ws.numel(), ctypes.byref(steps), ctypes.c_void_p(_stream(stream))))
    v = fora_workspace_views(g, 1, ws)
    return dict(cnt=v["walk_count"][0], acc_fx=v["walk_weight_fx"][0], steps=steps.value)


def fora_graph_rank(g: Graph, stream=None) -> torch.Tensor:
    """The graph's degree rank (int32 [n]): out-degree descending, ties by id."""
    out = torch.empty(g.n, dtype=torch.int32, device=g.device)
    _check(_lib.fora_graph_rank(g.handle, _ptr(out), ctypes.c_void_p(_stream(stream))))
    return out


def fora_philox(ctr: np.ndarray, key, device="cuda", stream=None) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    dc = torch.as_tensor(c.view(np.int32)).to(device)
    out = torch.empty_like(dc)
    _check(_lib.fora_philox(c.shape[0], _ptr(dc), int(key[0]) & 0xFFFFFFFF,
                            int(key[1]) & 0xFFFFFFFF, _ptr(out), ctypes.c_void_p(_stream(stream))))
    return out.cpu().numpy().view(np.uint32)


# ---- learned r_max --------------------------------------------------------------
def _s(stream):
    return ctypes.c_void_p(_stream(stream))


def fora_features(g: Graph, srcs: torch.Tensor, alpha: float, eps: float, delta: float,
                  pf: float, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    srcs = srcs.to(device=g.device, dtype=torch.int32).contiguous()
    out = torch.empty((srcs.numel(), FORA_MLP_FEATURES), dtype=torch.float32,
                      device=g.device) if out is None else out
    _check(_lib.fora_features(g.handle, srcs.numel(), _ptr(srcs), alpha, eps, delta, pf,
                              _ptr(out), _s(stream)))
    return out


def fora_mlp_forward(x: torch.Tensor, params: torch.Tensor, acts: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(_lib.fora_mlp_forward(x.shape[0], _ptr(x), _ptr(params), _ptr(y), _ptr(acts),
                                 _s(stream)))
    return y


def fora_mlp_backward(x, params, acts, y, target, grad, loss, scratch, stream=None):
    _check(_lib.fora_mlp_backward(x.shape[0], _ptr(x), _ptr(params), _ptr(acts), _ptr(y),
                                  _ptr(target), _ptr(grad), _ptr(loss), _ptr(scratch),
                                  _s(stream)))


def fora_adam_step(params, grad, m, v, lr, beta1, beta2, eps, step, stream=None):
    _check(_lib.fora_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), lr, beta1, beta2,
                               eps, step, _s(stream)))


def fora_mlp_to_bf16(params: torch.Tensor, stream=None) -> torch.Tensor:
    out = torch.empty(FORA_MLP_PARAMS, dtype=torch.int16, device=params.device)
    _check(_lib.fora_mlp_to_bf16(_ptr(params), _ptr(out), _s(stream)))
    return out


def fora_mlp_forward_bf16(x: torch.Tensor, params_bf16: torch.Tensor, stream=None):
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(_lib.fora_mlp_forward_bf16(x.shape[0], _ptr(x), _ptr(params_bf16), _ptr(y),
                                      _s(stream)))
    return y


def fora_predict_rmax(g: Graph, srcs: torch.Tensor, params_bf16: torch.Tensor, alpha: float,
                      eps: float, delta: float, pf: float, log_lo: float, log_hi: float,
                      stream=None):
    srcs = srcs.to(device=g.device, dtype=torch.int32).contiguous()
    n = srcs.numel()
    scratch = torch.empty(FORA_PREDICT_SCRATCH(n), dtype=torch.float32, device=g.device)
    rmax = torch.empty(n, dtype=torch.float64, device=g.device)
    fb = ctypes.c_int32()
    _check(_lib.fora_predict_rmax(g.handle, n, _ptr(srcs), alpha, eps, delta, pf,
                                  _ptr(params_bf16), log_lo, log_hi, _ptr(scratch), _ptr(rmax),
                                  ctypes.byref(fb), _s(stream)))
    return rmax, fb.value


def fora_push_sweep(g: Graph, queries, mults, ws: torch.Tensor | None = None, stream=None):
    B = len(queries)
    mults = np.ascontiguousarray(mults, np.float64)
    ws = workspace(g, B) if ws is None else ws
    e = np.zeros((B, mults.size), np.int64)
    w = np.zeros((B, mults.size), np.uint64)
    _check(_lib.fora_push_sweep(g.handle, B, queries, mults.size,
                                mults.ctypes.data_as(ctypes.c_void_p), _ptr(ws), ws.numel(),
                                e.ctypes.data_as(ctypes.c_void_p),
                                w.ctypes.data_as(ctypes.c_void_p), _s(stream)))
    return e, w
