"""Host-only checks of the benchmark script: it refuses more than one GPU
before touching any device, it reports HBM traffic only while the kernel
sources match the counter run, and every committed profile summary names the
command that produced it."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run_bench(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                          capture_output=True, text=True, timeout=120, env=env, cwd=ROOT)


@pytest.mark.parametrize("args,env", [
    (["--gpus", "2"], None),
    (["--gpus", "8", "--steps", "1"], None),
    (["--gpus", "1"], {"WORLD_SIZE": "2"}),
])
def test_more_than_one_gpu_refused(args, env):
    p = _run_bench(args, env)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""          # no JSON line for a refused run


def _traffic_file():
    return os.path.join(ROOT, "profiles", "hbm_traffic_d64_n1e4_k64.txt")


def _committed_digest_and_kernel():
    digest, kernel = None, None
    with open(_traffic_file()) as f:
        for line in f:
            line = line.strip()
            if line.startswith("source_sha256:"):
                digest = line.split(":", 1)[1].strip()
            elif line.startswith("kernel ") and kernel is None:
                kernel = dict(p.split("=", 1) for p in line.split()[1:])["name"]
    return digest, kernel


@pytest.mark.skipif(not os.path.exists(_traffic_file()), reason="no committed traffic summary")
def test_traffic_only_while_sources_match(monkeypatch):
    digest, kernel = _committed_digest_and_kernel()
    assert digest and kernel
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: digest)
    v = bench.measured_traffic(kernel)
    assert v is not None and v > 0
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 64)
    assert bench.measured_traffic(kernel) is None


def test_source_digest_covers_every_kernel_source(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1708_03340_amd", "csrc")
    dst = tmp_path / "paper_1708_03340_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_source_digest()
    assert d0 == bench.kernel_source_digest()
    names = sorted(n for n in os.listdir(dst) if n.endswith((".hip", ".h")))
    assert any(n.endswith(".hip") for n in names)
    for n in names:                      # a one-byte edit of any source changes it
        f = dst / n
        orig = f.read_bytes()
        f.write_bytes(orig + b" ")
        assert bench.kernel_source_digest() != d0, n
        f.write_bytes(orig)
    assert bench.kernel_source_digest() == d0


def test_profile_summaries_name_their_command():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))
    assert files
    for path in files:
        with open(path) as f:
            text = f.read()
        assert "rocprofv3 " in text, path
        assert "bench.py" in text, path
        assert len(text) < 64 * 1024, path     # short summaries, not raw traces
