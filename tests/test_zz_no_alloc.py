"""The allocation-free entry point (fora_ssppr_static, through the C ABI)
against fora_ssppr: the same results bit for bit, on two calls in a row
whose second has a smaller graph (the static workspace keeps the first
call's contents, which must not leak into the second), and a clear error
for a graph whose workspace exceeds the static array."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1908_10583_amd import fora  # noqa: E402


def _both(g, src, k, seed):
    G = fora.Graph.from_numpy(g.rowptr, g.colidx)
    ref = fora.fora_ssppr(G, src, k=k, seed=seed, stats=True)
    got = fora.fora_ssppr_static(G, src, k=k, seed=seed, stats=True)
    torch.cuda.synchronize()
    assert torch.equal(got.ids, ref.ids)
    assert torch.equal(got.vals, ref.vals)
    for key in ("rounds", "pushes", "edge_ops", "plan_entries", "walks", "steps", "r_sum",
                "rmax", "omega_unit", "t_alpha", "pull_rounds"):
        assert got.stats[key] == ref.stats[key], key
    assert got.stats["ms_walk"] == 0.0  # no events in the allocation-free path
    G.close()
    return ref


def test_static_entry_point_equals_fora_ssppr_twice_second_smaller():
    big = synth.rmat_graph(14, seed=14, cache=False)       # 16384 nodes
    small = synth.uniform_out_graph(1000, 10, seed=1)      # 1000 nodes
    a = _both(big, int(np.argmax(big.degrees())), 500, 3)
    b = _both(small, 0, 50, 1)
    assert a.stats["walks"] > 0 and b.stats["walks"] > 0
    # and back to the larger graph: nothing of the smaller call's state leaks
    _both(big, 7, 100, 4)


def test_static_entry_point_rejects_graphs_beyond_its_array():
    n = 3_000_000  # a cycle: about 52 bytes of workspace per node > 128 MiB
    rowptr = np.arange(n + 1, dtype=np.int32)
    colidx = ((np.arange(n) + 1) % n).astype(np.int32)
    G = fora.Graph.from_numpy(rowptr, colidx)
    assert fora.fora_workspace_size(G, 1) > fora.FORA_STATIC_SCRATCH_BYTES
    with pytest.raises(fora.FORAError) as ei:
        fora.fora_ssppr_static(G, 0, k=10)
    assert ei.value.code == fora.FORA_E_NOMEM
    assert "static scratch" in str(ei.value)
    G.close()
