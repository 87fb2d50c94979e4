"""Parity at the learned-r_max workload's full size: R-MAT 2^22 nodes (about
67M edges; the C sampler's graph of the same model), its 2,048 held-out
sources and the committed model trained for this workload.

* the features the device computes equal the oracle's (64 sampled held-out
  sources and the largest-degree node);
* the BF16 inference on the device agrees with the oracle's BF16 forward
  pass, and the predicted r_max is r_max* exp(y) inside the model's output
  range and r_max* (eqn:rmax) outside it, for all 2,048 held-out sources;
* FORA at the predicted r_max (64 held-out sources in one batch) keeps the
  per-query invariants, and the push of sampled queries at their predicted
  r_max equals the oracle's replay of their frontiers, element by element;
* what the network gains: on 128 held-out sources, the cost a E + b W of the
  whole query (E residue increments, W walks, counted exactly by the device;
  a and b the per-unit costs the model was trained with) at the learned
  r_max is at least 30% below the cost at eqn:rmax, and within 2% of the
  best single multiplier of r_max* (the labels on these uniform sources are
  nearly constant, so the network cannot do better than that constant)."""
import json
import os

import numpy as np
import pytest

import exactcmp
import oracle
import synth
from oracle import mlp

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora, learned  # noqa: E402

ALPHA, EPS, K, SEED = 0.2, 0.5, 500, 0
MODEL = os.path.join(os.path.dirname(learned.__file__), "models", "rmat22_rmax_mlp.json")


@pytest.fixture(scope="module")
def workload():
    g = synth.rmat_graph(22, seed=22, sampler="c", cache=False)
    heldout = synth.sources_uniform(g, 22048, seed=2222)[-2048:]
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    model = learned.Model.load(MODEL)
    rstar = oracle.constants(g.m, ALPHA, EPS, 1.0 / g.n, 1.0 / g.n)["rmax"]
    yield g, heldout, G, model, rstar
    G.close()


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def test_features_match_oracle(workload):
    g, heldout, G, model, rstar = workload
    srcs = np.concatenate([[int(np.argmax(g.degrees()))], heldout[::32]]).astype(np.int32)
    n = g.n
    got = fora.fora_features(G, _dev(srcs, torch.int32), ALPHA, EPS, 1 / n, 1 / n).cpu().numpy()
    want = mlp.features(g, srcs, ALPHA, EPS, rstar)
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-7)


def test_predicted_rmax_follows_the_model(workload):
    g, heldout, G, model, rstar = workload
    n = g.n
    srcs = _dev(heldout, torch.int32)
    X = fora.fora_features(G, srcs, ALPHA, EPS, 1 / n, 1 / n)
    pb = model.bf16()
    y = fora.fora_mlp_forward_bf16(X, pb).cpu().numpy().astype(np.float64)
    p = model.params.cpu().numpy()
    pick = np.arange(0, len(heldout), 16)
    y_ref = mlp.forward_bf16(p, X.cpu().numpy()[pick])
    np.testing.assert_allclose(y[pick], y_ref, rtol=2e-2, atol=2e-2)
    rm, fb = model.predict_rmax(G, srcs, ALPHA, EPS)
    rm = rm.cpu().numpy()
    lo, hi = model.log_range
    inside = np.isfinite(y) & (y >= lo) & (y <= hi)
    assert fb == np.count_nonzero(~inside)
    np.testing.assert_allclose(rm[inside], rstar * np.exp(y[inside]), rtol=1e-12)
    assert np.all(rm[~inside] == rstar)


def test_fora_at_the_predicted_rmax(workload):
    g, heldout, G, model, rstar = workload
    srcs = heldout[:64]
    rm, _ = model.predict_rmax(G, srcs, ALPHA, EPS)
    rm = rm.cpu().numpy()
    B = len(srcs)
    qs = fora.make_queries(srcs, alpha=ALPHA, eps=EPS, k=K, seed=SEED, n=g.n, rmax=rm)
    ws = fora.workspace(G, B)
    res = fora.fora_ssppr_batch(G, qs, kmax=K, ws=ws, stats=True)
    v = fora.fora_workspace_views(G, B, ws)
    for i in range(B):
        st_ = res.stats[i]
        r, q, pi = v["residue"][i], v["reserve"][i], v["pi_hat"][i]
        assert st_["rmax"] == rm[i]
        assert abs(r.sum(dtype=torch.float64).item() + q.sum(dtype=torch.float64).item()
                   - 1.0) < 1e-4
        assert abs(pi.sum(dtype=torch.float64).item() - 1.0) < 1e-4
        assert st_["walks"] == int(torch.ceil(r.double() * st_["omega_unit"]).sum().item())
        assert st_["term_violations"] == 0
        order = torch.argsort(-pi, stable=True)[:K].to(torch.int32)
        assert torch.equal(order, res.ids[i])
    # the query at its predicted threshold, element by element: the batch
    # row equals its push alone and the oracle's replay of those frontiers
    for i in (0, int(np.argmin(rm)), int(np.argmax(rm))):
        p = fora.fora_push_only(G, int(srcs[i]), ALPHA, float(rm[i]), log_frontiers=True)
        assert np.array_equal(p["r_fx"].cpu().numpy(), v["residue_fx"][i].cpu().numpy())
        assert np.array_equal(p["q"].cpu().numpy(), v["reserve"][i].cpu().numpy())
        assert p["stats"]["rounds"] == res.stats[i]["rounds"]
        exactcmp.check_push(g, int(srcs[i]), ALPHA, float(rm[i]), p["frontiers"],
                            v["residue"][i].cpu().numpy(), v["reserve"][i].cpu().numpy())
        del p


def test_learned_rmax_gain_over_the_fixed_rule(workload):
    g, heldout, G, model, rstar = workload
    rep = json.load(open(MODEL.replace(".json", ".report.json")))
    a = rep["unit_costs"]["ms_per_edge_op"]
    b = rep["unit_costs"]["ms_per_walk"]
    mult = rep["modelled_cost_ms"]["best_global_mult"]
    srcs = heldout[::16]
    rm, fb = model.predict_rmax(G, srcs, ALPHA, EPS)
    assert fb == 0
    ws = fora.workspace(G, len(srcs))

    def cost(rmax):
        qs = fora.make_queries(srcs, alpha=ALPHA, eps=EPS, k=K, seed=SEED, n=g.n, rmax=rmax)
        res = fora.fora_ssppr_batch(G, qs, kmax=K, ws=ws, stats=True)
        return np.array([a * x["edge_ops"] + b * x["walks"] for x in res.stats])

    fixed = cost(None)
    learnt = cost(rm.cpu().numpy())
    const = cost(np.full(len(srcs), rstar * mult))
    gain = 1.0 - learnt.mean() / fixed.mean()
    vs_const = learnt.mean() / const.mean() - 1.0
    print(f"learned r_max: modelled cost {learnt.mean():.3f} ms against {fixed.mean():.3f} ms "
          f"at eqn:rmax ({gain:.1%} lower) and {const.mean():.3f} ms at the best single "
          f"multiplier {mult:.4f} ({vs_const:+.2%})")
    assert gain >= 0.30
    assert vs_const <= 0.02
