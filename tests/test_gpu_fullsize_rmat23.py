"""Parity at the batched workload's full size: R-MAT 2^23 nodes (about 136M
edges), sources drawn in proportion to out-degree (hubs included), one wave
of 256 queries in one batched call with the launch shape the autotuner picks
for it on MI355X; eps = 0.5, delta = p_f = 1/n, k = 500.

The graph comes from the multithreaded C sampler (the same R-MAT model as the
numpy sampler, checked on the CPU), which builds it in seconds. As at 2^20,
the checks are sampled outputs the oracle computes one by one and properties
that hold at any size:
* every query: mass conservation, the estimate's total, the walk count as a
  function of the residues, and the selection against a stable sort of the
  estimate (computed on the device, one row at a time);
* the largest-degree and the median-degree source of the wave element by
  element: the batch row's push equals the same query's push alone and the
  oracle's replay of its frontiers (r and q to 1e-5, every push decision
  within 1e-5 of its threshold); the median-degree query's walk end-point
  counts and moves exactly equal to the oracle's walks on the device's
  residues (all of its walks, in pieces over worker processes);
* walk counts bit-exact on a sampled part of the oracle's walk plan, run on
  the full graph;
* sampled queries in the batch equal to the same queries run alone, bit for
  bit;
* the learned r_max (the committed model for this workload, trained on
  other degree-weighted sources): FORA at the predicted thresholds of 64
  sources of the wave in one batch keeps the per-query invariants, and the
  query with the median prediction goes element by element through the
  replay with its walks exact on the device's residues."""
import os

import numpy as np
import pytest

import exactcmp
import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora, learned  # noqa: E402

ALPHA, EPS, K, SEED, B = 0.2, 0.5, 500, 0, 256
MODEL = os.path.join(os.path.dirname(learned.__file__), "models", "rmat23_rmax_mlp.json")
# the launch shape the autotuner picks for 256-query waves of this workload
WAVE_TUNING = dict(walk_blocks_per_cu=16, walk_chunk=1024, push_blocks_per_cu=32,
                   graph_rounds=0, pull_ratio=64, record_ids=1, walk_agg=0)


@pytest.fixture(scope="module")
def workload():
    g = synth.rmat_graph(23, seed=23, sampler="c", cache=False)
    srcs = synth.sources_by_degree(g, B, seed=2323)
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    G.set_tuning(**WAVE_TUNING)
    deg = g.degrees()
    sampled = (int(np.argmax(deg[srcs])), int(np.argsort(deg[srcs])[B // 2]))
    yield g, srcs, G, sampled
    G.close()


@pytest.fixture(scope="module")
def refs(workload):
    """The oracle's push for each sampled query (seconds each at this size)."""
    g, srcs, G, sampled = workload
    c = oracle.constants(g.m, ALPHA, EPS, 1.0 / g.n, 1.0 / g.n)
    return c, {i: oracle.push(g, int(srcs[i]), ALPHA, c["rmax"]) for i in sampled}


@pytest.fixture(scope="module")
def batch(workload):
    g, srcs, G, sampled = workload
    qs = fora.make_queries(srcs, alpha=ALPHA, eps=EPS, k=K, seed=SEED, n=g.n,
                           flags=fora.FORA_WALK_COUNTS)
    ws = fora.workspace(G, B)
    res = fora.fora_ssppr_batch(G, qs, kmax=K, ws=ws, stats=True)
    v = fora.fora_workspace_views(G, B, ws)
    omega_unit = res.stats[0]["omega_unit"]
    per_query = []
    for i in range(B):
        r, q, pi = v["residue"][i], v["reserve"][i], v["pi_hat"][i]
        order = torch.argsort(-pi, stable=True)[:K]
        per_query.append(dict(
            r_sum=r.sum(dtype=torch.float64).item(),
            q_sum=q.sum(dtype=torch.float64).item(),
            pi_sum=pi.sum(dtype=torch.float64).item(),
            walks=int(torch.ceil(r.double() * omega_unit).sum().item()),
            order_ok=bool(torch.equal(order.to(torch.int32), res.ids[i]))))
    rows = {i: exactcmp.row_of(v, i) for i in sampled}
    out = dict(stats=res.stats, per_query=per_query, rows=rows, ids=res.ids.cpu().numpy(),
               vals=res.vals.cpu().numpy())
    del v, ws, res
    torch.cuda.empty_cache()
    return out


def test_every_query_keeps_the_invariants(workload, batch):
    g, srcs, G, _ = workload
    for i in range(B):
        st_, pq = batch["stats"][i], batch["per_query"][i]
        # push moves mass from r to q and to neighbours' r: sum q + sum r = 1
        assert abs(pq["q_sum"] + pq["r_sum"] - 1.0) < 1e-4
        # each walk adds r(v) / omega_v: the walk mass equals sum r
        assert abs(pq["pi_sum"] - 1.0) < 1e-4
        assert st_["walks"] == pq["walks"]
        assert pq["order_ok"]
        assert st_["term_violations"] == 0
        assert np.all(np.diff(batch["vals"][i].astype(np.float64)) <= 0)


def test_sampled_pushes_match_oracle(workload, batch, refs):
    g, srcs, G, sampled = workload
    c, pushes = refs
    for i in sampled:
        got = batch["rows"][i]
        st_ = batch["stats"][i]
        assert st_["rmax"] == c["rmax"] and st_["omega_unit"] == c["omega_unit"]
        p = fora.fora_push_only(G, int(srcs[i]), ALPHA, c["rmax"], log_frontiers=True)
        assert np.array_equal(p["r_fx"].cpu().numpy(), got["residue_fx"])
        assert np.array_equal(p["q"].cpu().numpy(), got["reserve"])
        exactcmp.check_push(g, int(srcs[i]), ALPHA, c["rmax"], p["frontiers"],
                            got["residue"], got["reserve"])
        del p
        # the oracle's free-running push: the same rounds and states where no
        # residue of it comes within 1e-5 of its threshold
        ref = pushes[i]
        if ref["min_margin"] > 1e-5:
            assert st_["rounds"] == ref["rounds"]
            assert np.all(exactcmp.close(got["residue"], ref["r"]))


def test_median_query_walks_exactly_as_the_oracle(workload, batch, refs):
    g, srcs, G, sampled = workload
    i = sampled[1]
    st_ = batch["stats"][i]
    ref = exactcmp.oracle_walks_on(g, batch["rows"][i]["residue"], st_["omega_unit"],
                                   int(srcs[i]), SEED, st_["t_alpha"], workers=16)
    assert ref["walks"] == st_["walks"]
    exactcmp.check_walks(ref, batch["rows"][i]["walk_count"], st_["steps"],
                         batch["rows"][i]["walk_weight_fx"])


def test_sampled_walks_are_bit_exact_on_the_full_graph(workload, refs):
    g, srcs, G, sampled = workload
    i = sampled[0]
    c, pushes = refs
    pv, po, pw = oracle.plan(pushes[i]["r"], c["omega_unit"])
    rng = np.random.default_rng(23)
    pick = np.union1d(rng.choice(len(pv), min(2000, len(pv)), replace=False),
                      np.argsort(po)[-5:])
    pv, po, pw = pv[pick], po[pick], pw[pick]
    key0, key1 = int(srcs[i]), SEED
    ref = oracle.walks(g, key0, key1, c["t_alpha"], pv, po, pw)
    got = fora.fora_walk_only(G, pv, po, pw, key0, key1, ALPHA)
    assert np.array_equal(got["cnt"].cpu().numpy().view(np.uint64), ref["cnt"])
    assert got["steps"] == ref["steps"]
    acc = got["acc_fx"].cpu().numpy().view(np.uint64).astype(np.float64) / 2.0**62
    tol = ref["cnt"] * 2.0**-62 + 1e-15 * ref["acc"]
    assert np.all(np.abs(acc - ref["acc"]) <= tol)


def test_query_in_the_batch_equals_it_alone(workload, batch):
    g, srcs, G, sampled = workload
    ws = fora.workspace(G, 1)
    for i in sampled:
        one = fora.fora_ssppr(G, int(srcs[i]), ALPHA, EPS, k=K, seed=SEED, ws=ws, stats=True,
                              flags=fora.FORA_WALK_COUNTS)
        alone = exactcmp.row_of(fora.fora_workspace_views(G, 1, ws), 0)
        for key in ("residue_fx", "reserve", "walk_count", "walk_weight_fx", "pi_hat"):
            assert np.array_equal(alone[key], batch["rows"][i][key]), key
        assert np.array_equal(one.ids.cpu().numpy(), batch["ids"][i])
        assert np.array_equal(one.vals.cpu().numpy(), batch["vals"][i])
        for key in ("rounds", "edge_ops", "walks", "steps", "r_sum"):
            assert one.stats[key] == batch["stats"][i][key], key


def test_learned_rmax_at_the_batched_workload(workload):
    g, srcs, G, _ = workload
    model = learned.Model.load(MODEL)
    sub = srcs[:64]
    rm, fb = model.predict_rmax(G, sub, ALPHA, EPS)
    rm = rm.cpu().numpy()
    rstar = oracle.constants(g.m, ALPHA, EPS, 1.0 / g.n, 1.0 / g.n)["rmax"]
    assert fb == 0 and np.all(rm < rstar)  # the model lowers r_max for every source
    Bl = len(sub)
    qs = fora.make_queries(sub, alpha=ALPHA, eps=EPS, k=K, seed=SEED, n=g.n, rmax=rm,
                           flags=fora.FORA_WALK_COUNTS)
    ws = fora.workspace(G, Bl)
    res = fora.fora_ssppr_batch(G, qs, kmax=K, ws=ws, stats=True)
    v = fora.fora_workspace_views(G, Bl, ws)
    for i in range(Bl):
        st_ = res.stats[i]
        r, q, pi = v["residue"][i], v["reserve"][i], v["pi_hat"][i]
        assert st_["rmax"] == rm[i] and st_["term_violations"] == 0
        assert abs(r.sum(dtype=torch.float64).item() + q.sum(dtype=torch.float64).item()
                   - 1.0) < 1e-4
        assert abs(pi.sum(dtype=torch.float64).item() - 1.0) < 1e-4
        assert st_["walks"] == int(torch.ceil(r.double() * st_["omega_unit"]).sum().item())
        order = torch.argsort(-pi, stable=True)[:K].to(torch.int32)
        assert torch.equal(order, res.ids[i])
    i = int(np.argsort(rm)[Bl // 2])
    row = exactcmp.row_of(v, i)
    st_ = res.stats[i]
    del v, ws
    torch.cuda.empty_cache()
    exactcmp.check_query(g, G, int(sub[i]), ALPHA, float(rm[i]), row, st_, key1=SEED,
                         workers=16)
