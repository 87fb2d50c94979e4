"""The serving loop on the GPU: a Poisson trace of mixed-eps, mixed-k
queries through several slots under a memory budget; every result equals the
same query run alone, bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora, serve  # noqa: E402


@pytest.fixture(scope="module")
def graph():
    g = synth.rmat_graph(12, seed=12, cache=False)
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    yield g, G
    G.close()


def test_results_alone_equal_results_in_the_mix(graph):
    g, G = graph
    srcs = synth.sources_uniform(g, 64, seed=77)
    trace = synth.poisson_requests(24, 3000.0, srcs, seed=9)
    # repeat one request so that a duplicate runs in the mix as well
    trace.append(dict(trace[3], id=24, t=trace[-1]["t"]))
    budget = 2 * fora.fora_workspace_size(G, 4) + fora.fora_workspace_size(G, 2)
    srv = serve.Server(G, slots=3, max_batch=4, mem_budget=budget, keep_rows=True, stats=True,
                       query_flags=fora.FORA_WALK_COUNTS)
    reqs = serve.run_trace(srv, trace)
    assert all(r.error is None for r in reqs), [r.error for r in reqs if r.error]
    assert srv.peak <= budget and srv.max_running >= 2
    assert {r.eps for r in reqs} == {0.1, 0.5} and {r.k for r in reqs} == {50, 500}
    ws1 = fora.workspace(G, 1)
    for r in reqs:
        alone = fora.fora_ssppr(G, r.src, 0.2, r.eps, 1 / g.n, 1 / g.n, r.k, seed=r.seed,
                                ws=ws1, stats=True, flags=fora.FORA_WALK_COUNTS)
        v = {k: t[0].cpu().numpy() for k, t in fora.fora_workspace_views(G, 1, ws1).items()}
        assert r.stats["omega_unit"] == alone.stats["omega_unit"]
        assert r.stats["rmax"] == alone.stats["rmax"]
        for key in ("residue_fx", "reserve", "walk_count", "walk_weight_fx", "pi_hat"):
            assert np.array_equal(r.rows[key], v[key]), key
        assert np.array_equal(r.ids, alone.ids.cpu().numpy()[:r.k])
        assert np.array_equal(r.vals, alone.vals.cpu().numpy()[:r.k])
        for key in ("rounds", "edge_ops", "walks", "steps"):
            assert r.stats[key] == alone.stats[key], key
        # the top-k is the order of the query's own estimate
        order = np.lexsort((np.arange(g.n), -r.rows["pi_hat"]))[:r.k]
        assert np.array_equal(r.ids, order)
    dup = [r for r in reqs if r.id in (3, 24)]
    assert dup[0].rows is not None and dup[1].rows is not None


def test_memory_budget_of_one_query(graph):
    g, G = graph
    srcs = synth.sources_uniform(g, 16, seed=78)
    trace = synth.poisson_requests(6, 5000.0, srcs, seed=10, eps_choices=(0.5,), k_choices=(50,))
    srv = serve.Server(G, slots=3, max_batch=4, mem_budget=fora.fora_workspace_size(G, 1))
    reqs = serve.run_trace(srv, trace)
    assert all(r.error is None for r in reqs)
    assert srv.max_running == 1 and all(r.batch == 1 for r in reqs)
    s = serve.summarize(reqs, srv)
    assert s["requests"] == 6 and s["latency_ms"]["p50"] > 0
