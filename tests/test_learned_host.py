"""Host-side logic of the learned r_max (CPU only): the cost labels."""
import numpy as np
import pytest

pytest.importorskip("torch")
learned = pytest.importorskip("paper_1908_10583_amd.learned")


def test_labels_find_the_minimum_of_a_balanced_cost():
    # E ~ A / mult and W ~ B mult: cost a A / mult + b B mult has its minimum at
    # mult = sqrt(a A / (b B)); the parabola through the grid argmin and its
    # neighbours (uniform in ln mult) lands close to it
    x = np.log(learned.MULTS)
    A = np.array([1e6, 2e6, 5e5, 1e7])
    B = np.array([1e5, 3e5, 2e6, 1e4])
    E = np.rint(np.exp(-x)[None, :] * A[:, None]).astype(np.int64)
    W = np.rint(np.exp(x)[None, :] * B[:, None]).astype(np.uint64)
    cost = dict(ms_per_edge_op=1e-8, ms_per_walk=4e-8)
    y, total = learned.labels(E, W, cost)
    want = 0.5 * np.log(1e-8 * A / (4e-8 * B))
    inside = (want > x[-1]) & (want < x[0])
    np.testing.assert_allclose(y[inside], want[inside], atol=0.02)
    # minima beyond the grid stay on its edge
    assert np.all((y >= x[-1] - 1e-12) & (y <= x[0] + 1e-12))
    assert np.all(y[~inside] == np.where(want[~inside] > x[0], x[0], x[-1]))
    assert total.shape == E.shape


def test_model_file_keeps_its_output_range(tmp_path):
    import json
    import torch
    from paper_1908_10583_amd import fora
    path = str(tmp_path / "m.json")
    m = learned.Model(torch.zeros(fora.FORA_MLP_PARAMS), log_range=(-1.0, 2.0))
    m.save(path)
    assert learned.Model.load(path, device="cpu").log_range == (-1.0, 2.0)
    # a file without the field holds a model of the earlier grid, [0.25, 8] r_max*
    d = json.load(open(path))
    del d["log_range"]
    json.dump(d, open(path, "w"))
    assert learned.Model.load(path, device="cpu").log_range == learned.LEGACY_LOG_RANGE
    assert abs(learned.MULTS[0] - 8.0) < 1e-12 and abs(learned.MULTS[-1] - 1 / 32) < 1e-15
