"""FORA+ on the GPU (section 3.3): the walk-destination index bit-exact
against the oracle's, and queries that read it equal to the oracle's queries
with walks keyed by the index key (walks past omega_max(v) run live)."""
import numpy as np
import pytest

import oracle
import synth
import exactcmp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora  # noqa: E402

ALPHA = 0.2
KEY = (123456, 789)


def close(g, o, rtol=1e-5, atol=1e-12):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return np.abs(g - o) <= rtol * np.abs(o) + atol


@pytest.fixture(scope="module")
def g1k():
    return synth.uniform_out_graph(1000, 10, seed=1)


@pytest.fixture(scope="module")
def G1k(g1k):
    G = fora.Graph.from_numpy(g1k.rowptr, g1k.colidx)
    c = oracle.constants(g1k.m, ALPHA, 0.5, 1e-3, 1e-3)
    fora.fora_build_index(G, ALPHA, c["rmax"] * c["omega_unit"], *KEY)
    yield G
    G.close()


@pytest.mark.parametrize("scale,wpd", [(12, 3.0), (10, 0.7)])
def test_index_matches_oracle(scale, wpd):
    g = synth.rmat_graph(scale, seed=scale, cache=False)
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    fora.fora_build_index(G, ALPHA, wpd, *KEY)
    info = fora.fora_index_info(G)
    ref = oracle.build_index(g, ALPHA, wpd, KEY)
    assert info["total"] == int(ref["off"][-1]) and info["key"] == KEY
    off, dest = fora.fora_index_export(G)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref["off"])
    assert np.array_equal(dest.cpu().numpy(), ref["dest"])
    G.close()


@pytest.mark.parametrize("delta", [1e-3, 2e-4])
def test_index_queries_match_oracle(g1k, G1k, delta):
    # delta = 2e-4 plans 5x more walks than the index holds: the tail runs live
    srcs = [0, 17, 999]
    qs = fora.make_queries(srcs, k=50, seed=[5, 6, 7], n=g1k.n, delta=delta, pf=1e-3,
                           flags=fora.FORA_USE_INDEX | fora.FORA_WALK_COUNTS)
    ws = fora.workspace(G1k, len(srcs))
    res = fora.fora_ssppr_batch(G1k, qs, ws=ws, stats=True)
    views = fora.fora_workspace_views(G1k, 3, ws)
    for i, s in enumerate(srcs):
        st_ = res.stats[i]
        # the index holds the end points of walks keyed by the index key, so
        # the oracle walking the device's plan live with that key reproduces
        # every end point (moves are not compared: indexed walks make none
        # on the device)
        exactcmp.check_query(g1k, G1k, s, ALPHA, st_["rmax"], exactcmp.row_of(views, i), st_,
                             key0=KEY[0], key1=KEY[1], steps=False)
        ref = oracle.fora(g1k, s, k=50, seed=5 + i, delta=delta, pf=1e-3, walk_key=KEY)
        assert st_["rounds"] == ref["rounds"]
        if ref["min_margin"] > 1e-5:
            assert np.array_equal(views["walk_count"][i].cpu().numpy().view(np.uint64),
                                  ref["cnt"])
        if delta == 1e-3:
            assert st_["steps"] == 0  # every walk came from the index
        else:
            assert st_["steps"] > 0   # the tail beyond omega_max ran live


def test_index_and_plain_queries_in_one_batch(g1k, G1k):
    qs = fora.make_queries([0, 0], k=50, seed=[1, 1], n=g1k.n, delta=1e-3, pf=1e-3,
                           flags=[fora.FORA_USE_INDEX | fora.FORA_WALK_COUNTS,
                                  fora.FORA_WALK_COUNTS])
    ws = fora.workspace(G1k, 2)
    res = fora.fora_ssppr_batch(G1k, qs, ws=ws, stats=True)
    views = fora.fora_workspace_views(G1k, 2, ws)
    for i, key in enumerate((KEY, (0, 1))):
        exactcmp.check_query(g1k, G1k, 0, ALPHA, res.stats[i]["rmax"], exactcmp.row_of(views, i),
                             res.stats[i], key0=key[0], key1=key[1], steps=i == 1)
    # one push, two walk keys: the residues are the same, the walks are not
    assert torch.equal(views["residue_fx"][0], views["residue_fx"][1])
    assert res.stats[0]["steps"] == 0 and res.stats[1]["steps"] > 0


def test_index_errors(g1k, G1k):
    G = fora.Graph.from_numpy(g1k.rowptr, g1k.colidx)
    cases = [(G, dict(flags=fora.FORA_USE_INDEX)),                       # no index
             (G1k, dict(flags=fora.FORA_USE_INDEX, alpha=0.3)),          # other alpha
             (G1k, dict(flags=fora.FORA_USE_INDEX | fora.FORA_PRUNE_ZERO_HOP))]
    for graph, kw in cases:
        qs = fora.make_queries([0], k=10, n=g1k.n, **kw)
        with pytest.raises(fora.FORAError) as ei:
            fora.fora_ssppr_batch(graph, qs)
        assert ei.value.code == fora.FORA_E_ARG
    with pytest.raises(fora.FORAError):
        fora.fora_build_index(G, ALPHA, -1.0, 0, 0)
    G.close()
