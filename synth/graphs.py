"""Seeded synthetic inputs: graphs in CSR form and source lists.

This module only draws inputs. It holds none of the PPR method's arithmetic,
so both the CPU oracle and the HIP path can take their inputs from it.

Graph model (paper §2.1): a directed graph, one out-adjacency list per node,
stored as CSR with int32 ``rowptr[n+1]`` and ``colidx[m]``; each row is sorted
by target id. The random-walk-with-restart semantics are undefined at a node
with no out-edge, so every generator here returns graphs where every node has
out-degree >= 1.

* ``uniform_out_graph``: every node gets exactly ``d`` distinct, non-self,
  uniformly random targets (the n=1,000 correctness graph).
* ``rmat_graph``: R-MAT (Chakrabarti, Zhan, Faloutsos, SDM'04) with
  16*n samples by default and (a, b, c, d) = (.57, .19, .19, .05); duplicate
  edges and self-loops removed; node ids relabelled by a seeded random
  permutation so that hubs are not clustered at low ids; then every node left
  with out-degree 0 gets one uniformly random non-self out-edge. The paper
  uses R-MAT graphs for its scalability study (§8) but does not give their
  parameters; these are the ones the workloads here name.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    """A CSR graph plus the facts about how it was drawn."""

    rowptr: np.ndarray  # int32[n+1]
    colidx: np.ndarray  # int32[m]
    name: str = ""
    # out-degree before the dangling-node fix-up (R-MAT only); used to draw
    # sources "from nodes with out-degree >= 1" in the R-MAT sense.
    deg_before_fixup: np.ndarray | None = None
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.colidx.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))


def _csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray):
    """Sort edges by (src, dst) and build int32 CSR."""
    key = src.astype(np.int64) * n + dst.astype(np.int64)
    key.sort(kind="stable")
    s = key // n
    t = key - s * n
    counts = np.bincount(s, minlength=n)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("graph has 2^31 or more edges; CSR is int32")
    return rowptr.astype(np.int32), t.astype(np.int32)


def uniform_out_graph(n: int = 1000, d: int = 10, seed: int = 0) -> Graph:
    """Every node has exactly ``d`` distinct non-self uniform out-neighbours."""
    if d > n - 1:
        raise ValueError("d must be at most n-1")
    rng = np.random.Generator(np.random.PCG64(seed))
    src = np.repeat(np.arange(n, dtype=np.int64), d)
    dst = np.empty(n * d, np.int64)
    for v in range(n):
        t = rng.choice(n - 1, size=d, replace=False)
        t = t + (t >= v)  # skip the node itself
        dst[v * d:(v + 1) * d] = t
    rowptr, colidx = _csr_from_edges(n, src, dst)
    return Graph(rowptr, colidx, name=f"uniform-n{n}-d{d}-s{seed}",
                 params=dict(kind="uniform", n=n, d=d, seed=seed))


def hub_graph(n: int = 8000, extra: int = 3, seed: int = 0) -> Graph:
    """Node 0 points to every other node (out-degree n-1), every other node
    points to node 1 (in-degree n-1 or so) and to ``extra`` random non-self
    targets: a small graph whose frontiers hold very high-degree entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    src = [np.zeros(n - 1, np.int64)]
    dst = [np.arange(1, n, dtype=np.int64)]
    others = np.arange(2, n, dtype=np.int64)
    src.append(others)
    dst.append(np.ones(n - 2, np.int64))
    for _ in range(extra):
        t = rng.integers(0, n - 1, size=n - 1)
        v = np.arange(1, n, dtype=np.int64)
        t = t + (t >= v)
        src.append(v)
        dst.append(t)
    s_ = np.concatenate(src)
    d_ = np.concatenate(dst)
    key = np.unique(s_ * n + d_)
    rowptr, colidx = _csr_from_edges(n, key // n, key % n)
    return Graph(rowptr, colidx, name=f"hub-n{n}-s{seed}",
                 params=dict(kind="hub", n=n, extra=extra, seed=seed))


def _rmat_samples(scale: int, count: int, a: float, b: float, c: float,
                  rng: np.random.Generator):
    """Draw ``count`` R-MAT (src, dst) pairs on 2^scale nodes."""
    # quadrant thresholds on a uniform 32-bit draw
    t_a = np.uint32(min(round(a * 2**32), 2**32 - 1))
    t_ab = np.uint32(min(round((a + b) * 2**32), 2**32 - 1))
    t_abc = np.uint32(min(round((a + b + c) * 2**32), 2**32 - 1))
    src = np.zeros(count, np.uint32)
    dst = np.zeros(count, np.uint32)
    for level in range(scale):
        u = rng.integers(0, 2**32, size=count, dtype=np.uint32)
        sh = np.uint32(scale - 1 - level)
        ge_a = u >= t_a
        down = u >= t_ab                      # quadrants c, d: src bit set
        right = ge_a ^ down ^ (u >= t_abc)    # quadrants b, d: dst bit set
        src |= down.astype(np.uint32) << sh
        dst |= right.astype(np.uint32) << sh
    return src.astype(np.int64), dst.astype(np.int64)


_RMAT_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat.c")
_RMAT_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librmat.so")
_rmat_lib = None


def build_sampler(force: bool = False) -> str:
    """Compile the multithreaded R-MAT sampler (gcc, OpenMP)."""
    if force or not os.path.exists(_RMAT_LIB) or \
            os.path.getmtime(_RMAT_LIB) < os.path.getmtime(_RMAT_SRC):
        import subprocess
        tmp = _RMAT_LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _RMAT_SRC],
                       check=True)
        os.replace(tmp, _RMAT_LIB)
    return _RMAT_LIB


def _load_sampler():
    global _rmat_lib
    if _rmat_lib is None:
        import ctypes
        lib = ctypes.CDLL(build_sampler())
        P = ctypes.c_void_p
        lib.synth_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                   P, P, P, ctypes.c_int64, P]
        lib.synth_rmat.restype = ctypes.c_int
        _rmat_lib = lib
    return _rmat_lib


def _rmat_graph_c(scale, samples, a, b, c, seed):
    import ctypes
    n = 1 << scale
    rowptr = np.empty(n + 1, np.int32)
    deg0 = np.empty(n, np.int32)
    cap = samples + n
    col = np.empty(cap, np.int32)
    m = np.zeros(1, np.int64)
    rc = _load_sampler().synth_rmat(scale, samples, a, b, c, seed & (2**64 - 1),
                                    rowptr.ctypes.data, deg0.ctypes.data, col.ctypes.data,
                                    cap, m.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"R-MAT sampler failed ({rc})")
    return rowptr, col[:int(m[0])], deg0


def rmat_graph(scale: int, edge_factor: int = 16, a: float = 0.57,
               b: float = 0.19, c: float = 0.19, seed: int = 0,
               chunk: int = 1 << 24, cache: bool = True,
               sampler: str | None = None) -> Graph:
    """R-MAT graph on n = 2^scale nodes from ``edge_factor * n`` samples.

    Two samplers draw from the same model with different random streams:
    ``"numpy"`` (PCG64, level by level; the default up to scale 23) and
    ``"c"`` (SplitMix64 at counters, multithreaded; the default from scale 24,
    where numpy takes minutes)."""
    n = 1 << scale
    samples = edge_factor * n
    sampler = sampler or ("numpy" if scale <= 23 else "c")
    tag = f"rmat-s{scale}-ef{edge_factor}-a{a}-b{b}-c{c}-seed{seed}"
    if sampler == "c":
        tag += "-c"
        rowptr, colidx, deg0 = _rmat_graph_c(scale, samples, a, b, c, seed)
        return Graph(rowptr, colidx, name=tag, deg_before_fixup=deg0,
                     params=dict(kind="rmat", scale=scale, edge_factor=edge_factor,
                                 a=a, b=b, c=c, seed=seed, sampler="c"))
    path = os.path.join(_cache_dir(), tag + ".npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Graph(z["rowptr"], z["colidx"], name=tag,
                     deg_before_fixup=z["deg0"],
                     params=dict(kind="rmat", scale=scale, edge_factor=edge_factor,
                                 a=a, b=b, c=c, seed=seed))
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = []
    for start in range(0, samples, chunk):
        cnt = min(chunk, samples - start)
        s, t = _rmat_samples(scale, cnt, a, b, c, rng)
        keep = s != t  # drop self-loops
        k = (s[keep] << np.int64(scale)) | t[keep]
        keys.append(np.unique(k))
    key = np.unique(np.concatenate(keys)) if len(keys) > 1 else keys[0]
    del keys
    s = key >> np.int64(scale)
    t = key & np.int64(n - 1)
    del key
    perm = rng.permutation(n).astype(np.int64)
    s = perm[s]
    t = perm[t]
    deg0 = np.bincount(s, minlength=n).astype(np.int32)
    dangling = np.flatnonzero(deg0 == 0)
    if dangling.size:
        extra = rng.integers(0, n - 1, size=dangling.size)
        extra = extra + (extra >= dangling)
        s = np.concatenate([s, dangling.astype(np.int64)])
        t = np.concatenate([t, extra.astype(np.int64)])
    rowptr, colidx = _csr_from_edges(n, s, t)
    g = Graph(rowptr, colidx, name=tag, deg_before_fixup=deg0,
              params=dict(kind="rmat", scale=scale, edge_factor=edge_factor,
                          a=a, b=b, c=c, seed=seed))
    if path:
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, rowptr=rowptr, colidx=colidx, deg0=deg0)
        os.replace(tmp, path)
    return g


def _cache_dir() -> str:
    d = os.environ.get("FORA_SYNTH_CACHE", os.path.join("/tmp", "fora_synth_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def sources_uniform(g: Graph, count: int, seed: int, exclude=None) -> np.ndarray:
    """``count`` distinct sources uniform over nodes whose R-MAT out-degree
    (before the dangling fix-up) is at least 1; all nodes for other graphs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = g.deg_before_fixup if g.deg_before_fixup is not None else g.degrees()
    pool = np.flatnonzero(deg >= 1)
    if exclude is not None:
        pool = np.setdiff1d(pool, np.asarray(exclude))
    return np.sort(rng.choice(pool, size=count, replace=False)).astype(np.int32)


def sources_by_degree(g: Graph, count: int, seed: int, exclude=None) -> np.ndarray:
    """``count`` sources drawn with replacement, probability proportional to
    out-degree (duplicates kept, in draw order); nodes in ``exclude`` are
    never drawn."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = g.degrees().astype(np.float64)
    if exclude is not None:
        deg[np.asarray(exclude, np.int64)] = 0.0
    return rng.choice(g.n, size=count, replace=True, p=deg / deg.sum()).astype(np.int32)


def random_walk_plan(g: Graph, entries: int, max_walks: int, seed: int):
    """A seeded synthetic walk plan: ``entries`` distinct start nodes (ascending),
    a walk count in [1, max_walks] and a positive weight for each. Used to
    exercise the walk phase on its own."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = np.sort(rng.choice(g.n, size=entries, replace=False)).astype(np.int32)
    omega = rng.integers(1, max_walks + 1, size=entries).astype(np.uint64)
    w = rng.random(entries) * 1e-6 + 1e-9
    return v, omega, w


def poisson_requests(count: int, qps: float, sources: np.ndarray, seed: int,
                     eps_choices=(0.1, 0.5), k_choices=(50, 500)):
    """A seeded request trace: arrival times of a Poisson process of rate
    ``qps`` (exponential gaps), a source drawn uniformly from ``sources``, and
    eps and k each drawn uniformly from their choices. Returns a list of dicts
    (id, t, src, eps, k, seed)."""
    if count <= 0:
        return []
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps) - gaps[0]
    src = rng.choice(np.asarray(sources), size=count, replace=True)
    eps = rng.choice(np.asarray(eps_choices, np.float64), size=count)
    k = rng.choice(np.asarray(k_choices, np.int64), size=count)
    seeds = rng.integers(0, 2**31, size=count)
    return [dict(id=i, t=float(t[i]), src=int(src[i]), eps=float(eps[i]), k=int(k[i]),
                 seed=int(seeds[i])) for i in range(count)]


def workload(name: str) -> tuple[Graph, np.ndarray]:
    """The named workloads: graph and source list."""
    if name == "uniform1k":
        g = uniform_out_graph(1000, 10, seed=1)
        return g, np.array([0], np.int32)
    if name == "rmat20":
        g = rmat_graph(20, seed=20)
        return g, sources_uniform(g, 100, seed=2020)
    if name == "rmat20L":
        # training sources for a learned r_max on the rmat20 graph, then the
        # 100 rmat20 sources (held out: disjoint from the training ones)
        g = rmat_graph(20, seed=20)
        bench = sources_uniform(g, 100, seed=2020)
        train = sources_uniform(g, 4096, seed=2021, exclude=bench)
        return g, np.concatenate([train, bench])
    if name == "rmat23":
        # the multithreaded sampler builds this graph in seconds (numpy: a minute)
        g = rmat_graph(23, seed=23, sampler="c")
        return g, sources_by_degree(g, 1024, seed=2323)
    if name == "rmat23L":
        # training sources for a learned r_max on the rmat23 graph (drawn the
        # same way, never one of the 1,024 workload sources), then those
        # 1,024 (held out)
        g = rmat_graph(23, seed=23, sampler="c")
        bench = sources_by_degree(g, 1024, seed=2323)
        train = sources_by_degree(g, 4096, seed=2324, exclude=np.unique(bench))
        return g, np.concatenate([train, bench])
    if name == "rmat22":
        g = rmat_graph(22, seed=22)
        return g, sources_uniform(g, 22048, seed=2222)
    if name == "rmat26":
        g = rmat_graph(26, seed=26)
        return g, sources_uniform(g, 4096, seed=2626)
    raise KeyError(name)
