"""The oracle's Philox4x32-10 block function (Salmon et al., SC'11; the walk
randomness of Algorithm 2 draws one block per step) against an independent
implementation of the same function: rocRAND's, compiled for the host from
its headers by `philox_rocrand.cpp`. CPU only.

Every output word must agree, on the all-zero and all-one blocks, on blocks
shaped like the walks' (counter = (start node, walk index, step, 0), key =
(source, seed) and the distribution key), and on random counters and keys."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_block(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(HEADER)):
        pytest.skip("hipcc or rocRAND's headers are not installed")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O1",
                    os.path.join(HERE, "philox_rocrand.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=300)

    def run(ctrs, keys):
        ctrs = np.asarray(ctrs, np.uint32).reshape(-1, 4)
        keys = np.asarray(keys, np.uint32).reshape(-1, 2)
        rows = np.concatenate([ctrs, keys], axis=1)
        text = "".join(" ".join("%x" % w for w in r) + "\n" for r in rows)
        out = subprocess.run([exe], input=text, capture_output=True, text=True,
                             check=True, timeout=120).stdout.split()
        return np.array([int(w, 16) for w in out], np.uint32).reshape(-1, 4)

    return run


def _oracle(ctrs, keys):
    ctrs = np.asarray(ctrs, np.uint32).reshape(-1, 4)
    keys = np.asarray(keys, np.uint32).reshape(-1, 2)
    out = np.empty_like(ctrs)
    for key in np.unique(keys, axis=0):
        sel = np.all(keys == key, axis=1)
        out[sel] = oracle.philox(ctrs[sel], key)
    return out


def test_extreme_blocks(rocrand_block):
    ctrs = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 0, 1]]
    keys = [[0, 0], [0xFFFFFFFF] * 2, [0, 0], [0, 1]]
    np.testing.assert_array_equal(_oracle(ctrs, keys), rocrand_block(ctrs, keys))


def test_walk_shaped_blocks(rocrand_block):
    rng = np.random.default_rng(3)
    v = rng.integers(0, 1 << 26, 400)
    j = rng.integers(0, 1 << 20, 400)
    b = rng.integers(0, 64, 400)
    ctrs = np.stack([v, j, b, np.zeros_like(v)], axis=1)
    for key0 in (0, 12345, (1 << 26) - 1, oracle.DIST_KEY0):
        keys = np.tile([key0, 7], (len(ctrs), 1))
        np.testing.assert_array_equal(_oracle(ctrs, keys), rocrand_block(ctrs, keys))


def test_random_blocks(rocrand_block):
    rng = np.random.default_rng(11)
    ctrs = rng.integers(0, 1 << 32, (4000, 4), dtype=np.uint64)
    keys = np.repeat(rng.integers(0, 1 << 32, (40, 2), dtype=np.uint64), 100, axis=0)
    np.testing.assert_array_equal(_oracle(ctrs, keys), rocrand_block(ctrs, keys))
