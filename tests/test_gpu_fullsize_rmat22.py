"""Parity at the learned-r_max workload's full size: R-MAT 2^22 nodes (about
67M edges; the C sampler's graph of the same model), its 2,048 held-out
sources and the committed model trained for this workload.

* the features the device computes equal the oracle's (64 sampled held-out
  sources and the largest-degree node);
* the BF16 inference on the device agrees with the oracle's BF16 forward
  pass, and the predicted r_max is r_max* exp(y) inside the model's output
  range and r_max* (eqn:rmax) outside it, for all 2,048 held-out sources;
* FORA at the predicted r_max (64 held-out sources in one batch) keeps the
  per-query invariants, and the push of a sampled query at its predicted
  r_max agrees with the oracle's push at that threshold."""
import os

import numpy as np
import pytest

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
    i = 0
    ref = oracle.push(g, int(srcs[i]), ALPHA, float(rm[i]))
    r = v["residue"][i].cpu().numpy().astype(np.float64)
    q = v["reserve"][i].cpu().numpy().astype(np.float64)
    if ref["min_margin"] > 1e-5:
        assert res.stats[i]["rounds"] == ref["rounds"]
        np.testing.assert_allclose(q, ref["q"], rtol=1e-5, atol=1e-12)
        np.testing.assert_allclose(r, ref["r"], rtol=1e-5, atol=1e-12)
    else:
        # a residue within FP32 rounding of its threshold may be pushed one
        # round apart on the two sides: the states still agree closely
        assert abs(res.stats[i]["rounds"] - ref["rounds"]) <= 1
        assert np.abs(q - ref["q"]).sum() < 1e-3
        assert np.abs(r - ref["r"]).sum() < 1e-3
