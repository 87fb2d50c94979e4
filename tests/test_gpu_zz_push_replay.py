"""GPU push rounds against the oracle's replay of the GPU's own frontiers,
where a residue sits on its threshold.

The device sums residues exactly in fixed point (62 fraction bits) and the
oracle in FP64, so where a residue's FP64 value rounds to its threshold the
two may decide the push test differently: Algorithm 1 allows either (any
push order keeps eqn:layerppr), and a free-running comparison cannot be
element-wise. Replaying the frontiers the device logged rebuilds in FP64 the
state the device should reach: every listed node must pass the push test
within 1e-5 relative, no unlisted node may be over its threshold by more,
and r and q must then agree element by element (1e-5 relative).

Two families of cases, each through push rounds and through pull rounds:
* exact FP64 ties after round 0 (a node holding exactly r_max d(u)): both
  sides decide them alike;
* constructed flips: a node u receives two increments in round 1 whose FP64
  sum rounds down below their exact sum, with r_max chosen so that the FP64
  threshold equals that rounded sum. The oracle's test fails (equal, not
  above) while the device's exact sum passes: the device must push u in
  round 2 and the oracle must not, and the replay must still reconcile the
  two states."""
from fractions import Fraction

import numpy as np
import pytest

import exactcmp
import oracle
import synth
from synth.graphs import Graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora  # noqa: E402

ALPHA, TAU = 0.2, 1e-5


@pytest.mark.parametrize("pull_ratio", [0, 1 << 30])
def test_replayed_frontiers_reconcile_threshold_ties(pull_ratio):
    g = synth.rmat_graph(10, seed=3, cache=False)
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    G.set_tuning(pull_ratio=pull_ratio)
    deg = g.degrees()
    cases = 0
    for s in (0, 5, 17):
        for u in g.colidx[g.rowptr[s]:g.rowptr[s + 1]][:3]:
            # after round 0, u holds (1 - alpha) / d(s): exactly its threshold
            rmax = ((1.0 - ALPHA) / deg[s]) / deg[u]
            got = fora.fora_push_only(G, s, ALPHA, rmax, log_frontiers=True)
            rep = exactcmp.check_push(g, s, ALPHA, rmax, got["frontiers"],
                                      got["r"].cpu().numpy(), got["q"].cpu().numpy())
            assert got["stats"]["rounds"] == rep["rounds"]
            cases += 1
    assert cases == 7  # vertex 0 has one out-neighbour, 5 and 17 three or more
    G.close()


def _flip_cases(limit=6):
    """(d1, d2, du, rmax): s -> {v1, v2}; v1 and v2 of out-degrees d1, d2
    both point to u (out-degree du). After round 1, u holds inc1 + inc2,
    whose FP64 sum (the oracle's) is below the exact sum (the device's: both
    increments are exact in the fixed point), and r_max du == that FP64 sum
    exactly; v1, v2 and s pass their tests."""
    out = []
    a = ((1.0 - ALPHA) * 1.0) / 2
    for d1 in range(2, 30):
        for d2 in range(d1, 30):
            i1 = ((1.0 - ALPHA) * a) / d1
            i2 = ((1.0 - ALPHA) * a) / d2
            fl = i1 + i2
            exact_fx = Fraction(i1) * 2**62 + Fraction(i2) * 2**62
            if not (exact_fx.denominator == 1 and exact_fx > Fraction(fl) * 2**62):
                continue
            for du in range(2, 200):
                rmax = fl / du
                if rmax * du == fl and a > rmax * max(d1, d2) and 1.0 > rmax * 2:
                    out.append((d1, d2, du, rmax))
                    break
            if len(out) == limit:
                return out
    return out


def _flip_graph(d1, d2, du):
    # 0 = s, 1 = v1, 2 = v2, 3 = u; fillers after them point back to s
    edges = [(0, 1), (0, 2), (1, 3), (2, 3)]
    nxt = 4
    for v, d in ((1, d1), (2, d2), (3, du)):
        for _ in range(d - 1 if v != 3 else d):
            edges.append((v, nxt))
            edges.append((nxt, 0))
            nxt += 1
    e = np.array(sorted(edges), np.int64)
    rowptr = np.zeros(nxt + 1, np.int64)
    np.add.at(rowptr, e[:, 0] + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return Graph(rowptr, e[:, 1].astype(np.int32), name=f"flip-{d1}-{d2}-{du}")


@pytest.mark.parametrize("pull_ratio", [0, 1 << 30])
def test_device_pushes_a_node_the_oracle_leaves_and_the_replay_reconciles(pull_ratio):
    cases = _flip_cases()
    assert len(cases) >= 4
    for d1, d2, du, rmax in cases:
        g = _flip_graph(d1, d2, du)
        assert g.degrees()[3] == du and g.degrees()[1] == d1 and g.degrees()[2] == d2
        G = fora.Graph.from_numpy(g.rowptr, g.colidx)
        G.set_tuning(pull_ratio=pull_ratio)
        got = fora.fora_push_only(G, 0, ALPHA, rmax, log_frontiers=True)
        ref = oracle.push(g, 0, ALPHA, rmax, log_frontiers=True)
        # round 0: s; round 1: v1 and v2 (and no one else has residue yet)
        assert list(got["frontiers"][1]) == [1, 2] and list(ref["frontiers"][1]) == [1, 2]
        # round 2: u on the device, not in the oracle's free run (which may
        # end after round 1)
        ref_f2 = ref["frontiers"][2] if len(ref["frontiers"]) > 2 else []
        assert len(got["frontiers"]) > 2 and 3 in got["frontiers"][2] and 3 not in ref_f2
        exactcmp.check_push(g, 0, ALPHA, rmax, got["frontiers"], got["r"].cpu().numpy(),
                            got["q"].cpu().numpy())
        G.close()
