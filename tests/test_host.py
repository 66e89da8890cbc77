"""Host-side behaviour that needs no GPU: the library refuses to run without
its HIP build (no fallback), the benchmark refuses more than one GPU, and the
seeded inputs are deterministic and shaped like the named workloads."""
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_fails_loudly(tmp_path):
    from paper_1503_07037_amd import _lib
    with pytest.raises(RuntimeError, match="not found"):
        _lib.load(str(tmp_path / "libdmpt.so"))


def test_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1503_07037_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            text = open(os.path.join(pkg, name)).read()
            assert "import oracle" not in text and "from oracle" not in text, name


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workloads_are_seeded_and_shaped():
    a = workloads.config("cubic2048")
    b = workloads.config("cubic2048")
    assert a["H0"].shape == (2048, 2048)
    assert np.array_equal(a["H0"], b["H0"])
    assert np.array_equal(a["H0"], a["H0"].T)
    c = workloads.config("banded8192", n_override=512)
    assert c["H0"].shape == (512, 512) and c["Ne"] == 256.0 and len(c["H1"]) == 3
    band = np.abs(c["H0"][np.abs(np.subtract.outer(np.arange(512), np.arange(512))) > 256])
    assert band.size == 0 or band.max() == 0.0
    sy = workloads.batched_systems(4, count=64)
    assert len(sy) == 64 and all(256 <= s["N"] <= 3072 * 1.1 for s in sy)
    assert all(5.0 <= s["beta"] <= 40.0 and s["Ne"] == s["N"] / 2.0 for s in sy)
    assert sy == workloads.batched_systems(4, count=64)
