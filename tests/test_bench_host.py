"""Host logic of bench.py (no GPU): the algorithmic byte model of the
iteration kernels, the guard that ties committed counter readings to the
kernel code they were taken on, and the single-GPU refusal of --gpus N."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("word,b", [(8, 2), (8, 4), (4, 2)])
def test_kernel_bytes_model(word, b):
    # each array once: stencil reads s, d_old and the FP64 operator (24 B per
    # cell) and writes d, q; the Z^T pass reads r, q, d, x, D^-1 and writes
    # r', x, t; the Z pass reads t, r' and writes s; every nonzero of Z is read
    # once per pass as a value and an index
    n, E = 1000, 7777
    kb = bench.kernel_bytes(n, E, word, b)
    assert kb["stencil"] == 4 * word * n + 24 * n
    assert kb["axpy_zt"] == 8 * word * n + (word + b) * E
    assert kb["z_dot"] == 3 * word * n + (word + b) * E
    if word == 8:
        assert sum(kb.values()) == 144 * n + 2 * (8 + b) * E


def test_kernel_names_carry_formats():
    k = bench.kernel_names(8, (3, 7))
    assert k == {"stencil": "k_stencil<double, false, double, 0>", "axpy_zt": "k_zt<double, true, 3>",
                 "z_dot": "k_z<double, true, false, 7>"}
    assert bench.kernel_names(4, (1, 1))["z_dot"] == "k_z<float, true, false, 1>"


def _hash_of(monkeypatch, tmp_path, texts):
    files = []
    for i, t in enumerate(texts):
        f = tmp_path / f"src{i}.h"
        f.write_text(t)
        files.append(str(f))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", files)
    return bench.kernel_source_hash()


def test_source_hash_ignores_comments_not_code(monkeypatch, tmp_path):
    base = _hash_of(monkeypatch, tmp_path, ["int f(int a) {\n    return a + 1;\n}\n"])
    commented = _hash_of(monkeypatch, tmp_path, [
        "// the successor\n/* of a,\n   in int */\nint f(int a) {   // one more\n\n    return a + 1;\n}\n"])
    changed = _hash_of(monkeypatch, tmp_path, ["int f(int a) {\n    return a + 2;\n}\n"])
    assert commented == base
    assert changed != base


def test_measured_traffic_only_for_matching_code(monkeypatch, tmp_path):
    h = _hash_of(monkeypatch, tmp_path, ["int g;\n"])
    rec = {"source_sha256": h, "profile": "profiles/x.md",
           "kernels": {"k_zt<double, true, 3>": {"hbm_bytes_per_launch": 123456}}}
    cf = tmp_path / "counters.json"
    cf.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "COUNTER_FILE", str(cf))
    assert bench.measured_traffic("k_zt<double, true, 3>") == (123456, "profiles/x.md")
    assert bench.measured_traffic("k_z<double, true, false, 7>")[0] is None
    rec["source_sha256"] = "0" * 64
    cf.write_text(json.dumps(rec))
    val, why = bench.measured_traffic("k_zt<double, true, 3>")
    assert val is None and "changed" in why
    monkeypatch.setattr(bench, "COUNTER_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("k_zt<double, true, 3>")[0] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_cpu_baseline_helpers_small():
    """The CPU-baseline legs run the oracle on bounded samples: Jacobi PCG on
    a small grid and whole ensemble solves; rates are positive and the
    ensemble aggregate is the per-core rate times the host threads."""
    from gen import orca
    p = orca.orca_problem(37, 23, 5)
    j = bench.cpu_jacobi(p, 0.05)
    assert j["value"] > 0 and j["unit"] == "iter/s"
    e = bench.cpu_ensemble(0.01, members=2, nrhs=1)
    assert e["solves_per_s_per_core"] > 0
    threads = os.cpu_count() or 1
    assert abs(e["solves_per_s_all_threads"] - e["solves_per_s_per_core"] * threads) <= 0.1 * threads
    assert bench.host_cpu_model() is None or isinstance(bench.host_cpu_model(), str)


def test_deferred_x_update_names_and_bytes():
    """With the x update moved into the stencil (format bit 16), the kernels
    carry the stencil's x mode and the Z^T kernel's launched format, and one
    vector pass moves from the Z^T kernel's count to nowhere (8 n less)."""
    k = bench.kernel_names(8, (11 | 16, 7))
    assert k == {"stencil": "k_stencil<double, false, double, 2>",
                 "axpy_zt": "k_zt<double, true, 19>", "z_dot": "k_z<double, true, false, 7>"}
    assert bench.kernel_names(8, (3 | 16, 7))["stencil"] == "k_stencil<double, false, double, 1>"
    n, E = 1000, 5000
    a = bench.kernel_bytes(n, E, 8, 2, x_in_stencil=False)
    b = bench.kernel_bytes(n, E, 8, 2, x_in_stencil=True)
    assert sum(a.values()) - sum(b.values()) == 8 * n
    assert b["stencil"] - a["stencil"] == 16 * n and a["axpy_zt"] - b["axpy_zt"] == 24 * n
    sa, sb = bench.survey_bytes(n, E), bench.survey_bytes(n, E, x_in_stencil=True)
    assert sa["iteration"] == sb["iteration"] == 152 * n + 24 * E
    assert sb["stencil"] + sb["axpy_zt"] == sa["stencil"] + sa["axpy_zt"]
