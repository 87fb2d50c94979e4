"""The synthetic inputs (CPU only): the multithreaded R-MAT sampler in C,
used from 2^24 nodes, builds a valid CSR with the dangling-node fix-up, is
deterministic whatever the thread count, and draws the same model as the
numpy sampler (same edge count, degree skew and share of dangling nodes,
within sampling noise)."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check_csr(g):
    n, rp, ci = g.n, g.rowptr.astype(np.int64), g.colidx.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == g.m == len(ci) and np.all(np.diff(rp) >= 1)
    assert ci.min() >= 0 and ci.max() < n
    src = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(src != ci)  # no self-loops
    key = src * n + ci
    assert np.all(np.diff(key) > 0)  # rows sorted, no duplicate edges
    extra = np.diff(rp) - g.deg_before_fixup
    assert set(np.unique(extra).tolist()) <= {0, 1}
    assert np.all((extra == 1) == (g.deg_before_fixup == 0))


def test_c_sampler_builds_a_valid_graph():
    g = synth.rmat_graph(12, seed=5, sampler="c")
    assert g.n == 4096 and g.m > 0.7 * 16 * 4096
    _check_csr(g)


def _digest(seed):
    code = ("import sys, hashlib; sys.path.insert(0, %r); import synth; "
            "g = synth.rmat_graph(13, seed=%d, sampler='c'); "
            "print(hashlib.sha256(g.rowptr.tobytes() + g.colidx.tobytes()).hexdigest())"
            % (ROOT, seed))
    return code


@pytest.mark.parametrize("threads", ["1", "3", "8"])
def test_c_sampler_does_not_depend_on_the_thread_count(threads):
    g = synth.rmat_graph(13, seed=9, sampler="c")
    here = hashlib.sha256(g.rowptr.tobytes() + g.colidx.tobytes()).hexdigest()
    env = dict(os.environ, OMP_NUM_THREADS=threads)
    out = subprocess.run([sys.executable, "-c", _digest(9)], env=env, capture_output=True,
                         text=True, check=True, timeout=120)
    assert out.stdout.strip() == here
    # and a different seed gives a different graph
    other = synth.rmat_graph(13, seed=10, sampler="c")
    assert not (other.m == g.m and np.array_equal(other.colidx, g.colidx))


@pytest.mark.parametrize("seed", [1, 2])
def test_c_and_numpy_samplers_draw_the_same_model(seed):
    a = synth.rmat_graph(14, seed=seed, sampler="c")
    b = synth.rmat_graph(14, seed=seed, sampler="numpy", cache=False)
    _check_csr(b)
    assert abs(a.m - b.m) < 0.01 * b.m

    def stats(g):
        d0 = g.deg_before_fixup
        d = np.sort(d0)[::-1]
        return (d0 == 0).mean(), d[:100].sum() / d.sum(), d[0]

    za, sa, ma = stats(a)
    zb, sb, mb = stats(b)
    assert abs(za - zb) < 0.01       # share of nodes R-MAT left without out-edges
    assert abs(sa - sb) < 0.005      # share of edges at the 100 largest out-degrees
    assert abs(ma - mb) < 0.1 * mb   # largest out-degree
