"""The oracle's C core under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a copy of the oracle package is built with
-fsanitize=address,undefined (every report fatal) and the core pins run
against it in a fresh interpreter with the sanitizer runtime preloaded. Any
out-of-bounds access, use after free, signed overflow, misaligned or invalid
shift in the push, the replay, the plan, the walks, Philox or the top-k
aborts the run."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = [
    "tests/test_oracle_pins.py",
    "tests/test_replay_oracle.py",
    "tests/test_alg3_oracle.py",
    "tests/test_dist_oracle.py",
    "tests/test_index_oracle.py",
    "tests/test_philox_library.py::test_extreme_blocks",
]


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run_sanitized(tmp_path, pins, plant=None):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    pkg = tmp_path / "oracle"
    shutil.copytree(ORACLE, pkg, ignore=shutil.ignore_patterns("__pycache__", "*.so*"))
    if plant is not None:
        src = pkg / "fora_oracle.c"
        text = src.read_text()
        assert text.count(plant[0]) == 1
        src.write_text(text.replace(plant[0], plant[1]))
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", str(pkg / "liboracle.so"), str(pkg / "fora_oracle.c"), "-lm"],
                   check=True, capture_output=True, timeout=120)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = ("import sys; sys.path.insert(0, %r); import oracle; "
            "assert oracle.__file__.startswith(%r); sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main(['-q', '-s', '-p', 'no:cacheprovider', '-m', 'not gpu', *%r]))"
            % (str(tmp_path), str(pkg), ROOT, pins))
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                          timeout=1200, env=env)


@pytest.mark.slow
def test_core_pins_pass_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    out = _run_sanitized(tmp_path, PINS)
    assert out.returncode == 0, (out.stdout[-3000:], out.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in out.stderr
    assert "runtime error" not in out.stderr


@pytest.mark.slow
def test_the_sanitized_build_catches_a_planted_overrun(tmp_path):
    # one edge past each node's row: the last node reads beyond colidx
    out = _run_sanitized(
        tmp_path, ["tests/test_oracle_pins.py::test_push_invariant_uniform"],
        ("for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) r[colidx[e]] += inc;",
         "for (int32_t e = rowptr[v]; e <= rowptr[v + 1]; ++e) r[colidx[e]] += inc;"))
    assert out.returncode != 0
    assert "AddressSanitizer" in out.stderr
