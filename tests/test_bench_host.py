"""bench.py host logic (CPU): the one-GPU guard, and the rule that a committed
counter summary is used only while the kernel source it was taken with is
unchanged."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("storage", ["tiled", "tiled32", "pooled", "expanded"])
def test_counter_traffic_follows_the_kernel_source(storage, monkeypatch):
    import bench
    t = bench.counter_traffic(storage)
    assert t is None or t > 0
    # any change of the kernel code makes the summary stale
    real = bench.kernel_source
    monkeypatch.setattr(bench, "kernel_source", lambda k: real(k) + "int changed;\n")
    assert bench.counter_traffic(storage) is None


def test_kernel_source_ignores_comments(tmp_path, monkeypatch):
    """The key is the code: comments, trailing blanks and empty lines do not
    change it; a changed statement does."""
    import bench
    src = open(os.path.join(ROOT, "paper_2412_12506_amd", "csrc", "kernels.hip")).read()
    root = tmp_path / "repo"
    (root / "paper_2412_12506_amd" / "csrc").mkdir(parents=True)
    f = root / "paper_2412_12506_amd" / "csrc" / "kernels.hip"
    monkeypatch.setattr(bench, "ROOT", str(root))
    f.write_text(src)
    base = {k: bench.kernel_source(k) for k in ("tiled", "fwd")}
    at = src.index("__global__", src.index("// tiled forward BSR kernel"))
    f.write_text(src[:at] + "// a new comment line\n\n" + src[at:].replace("{\n", "{   // trailing note\n", 1))
    assert {k: bench.kernel_source(k) for k in ("tiled", "fwd")} == base
    f.write_text(src[:at] + "static int changed;\n" + src[at:])
    assert bench.kernel_source("tiled") != base["tiled"]


def test_committed_counter_summaries_are_consistent():
    """Each summary's traffic is its scaled FETCH_SIZE + WRITE_SIZE."""
    prof = os.path.join(ROOT, "profiles")
    names = [n for n in os.listdir(prof) if n.endswith("_counters.json")]
    assert names
    for n in names:
        rec = json.load(open(os.path.join(prof, n)))
        t = (rec["fetch_size_kib_mean"] * 1024 * rec["fetch_scale"] +
             rec["write_size_kib_mean"] * 1024 * rec["write_scale"])
        assert abs(t - rec["traffic_bytes_per_launch"]) <= 1e-6 * t, n
        assert rec["algorithmic_bytes_per_launch"] > 0
        assert os.path.exists(os.path.join(prof, n.replace(".json", ".md"))), n
