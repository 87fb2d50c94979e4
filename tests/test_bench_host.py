"""The benchmark's host logic (CPU only): it refuses more than one GPU with a
one-line JSON message, and it takes HBM traffic from a committed counter
record only while the kernel's code is the code the counters were taken on
(comments do not count)."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    lines = out.stdout.strip().splitlines()
    assert len(lines) == 1 and "error" in json.loads(lines[0])


V1 = "// the kernel\nint f(int x) {\n  return x + 1;  /* one */\n}\n"


def _tree(tmp_path, monkeypatch, text):
    """A one-source tree whose counter record was taken on V1."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "k.hip"
    src.write_text(V1)
    (tmp_path / "profiles").mkdir()
    rec = dict(sources=["k.hip"], traffic_bytes_per_launch=1234,
               code_sha256=bench.code_digest(["k.hip"]))
    (tmp_path / "profiles" / "k_walks_w_b1_traffic.json").write_text(json.dumps(rec))
    src.write_text(text)
    return src


def test_traffic_record_is_used_while_the_code_matches(tmp_path, monkeypatch):
    _tree(tmp_path, monkeypatch, V1)
    assert bench.recorded_traffic("k_walks", "w_b1") == (
        1234, os.path.join("profiles", "k_walks_w_b1_traffic.json"))
    assert bench.recorded_traffic("k_walks", "other_b1") == (None, None)


def test_comment_and_layout_edits_keep_the_record(tmp_path, monkeypatch):
    _tree(tmp_path, monkeypatch,
          "// the kernel, reworded\n/* a new\n   block comment */\nint f(int x)\n{\n"
          "    return x + 1;\n}\n")
    assert bench.recorded_traffic("k_walks", "w_b1")[0] == 1234


@pytest.mark.parametrize("code", ["int f(int x) { return x + 2; }",
                                  "int f(int x) { return x - 1; }",
                                  "int f(long x) { return x + 1; }"])
def test_traffic_record_is_dropped_once_the_code_changes(tmp_path, monkeypatch, code):
    src = _tree(tmp_path, monkeypatch, code)
    assert bench.recorded_traffic("k_walks", "w_b1") == (None, None)
    src.unlink()  # a missing source counts as changed
    assert bench.recorded_traffic("k_walks", "w_b1") == (None, None)


@pytest.mark.parametrize("path", sorted(
    p for p in os.listdir(os.path.join(ROOT, "profiles")) if p.endswith("_traffic.json")))
def test_committed_traffic_records_are_well_formed(path):
    rec = json.load(open(os.path.join(ROOT, "profiles", path)))
    assert rec["traffic_bytes_per_launch"] > 0
    assert len(rec["code_sha256"]) == 64
    for src in rec["sources"]:
        assert os.path.exists(os.path.join(ROOT, src)), src


@pytest.mark.parametrize("path", sorted(
    p for p in os.listdir(os.path.join(ROOT, "profiles")) if p.endswith(".md")))
def test_profile_summaries_name_commands_over_committed_files(path):
    text = open(os.path.join(ROOT, "profiles", path)).read()
    cmds = [line.strip() for line in text.splitlines()
            if line.strip().startswith("rocprofv3") and " -- " in line]
    assert cmds, "a summary gives the command that made it"
    for cmd in cmds:
        prog = cmd.split(" -- ", 1)[1].split()
        assert prog[0] in ("python3", "python") and prog[1].endswith(".py"), cmd
        assert os.path.exists(os.path.join(ROOT, prog[1])), cmd
        assert not prog[1].startswith("_work"), cmd
