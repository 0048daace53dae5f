"""The benchmark's command-line contract and the binding's refusal to run
without the HIP library (CPU only, no GPU call)."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""          # no JSON line for a configuration it does not run


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libcgks.so cannot be imported: there is no
    CPU fallback to run instead."""
    pkg = tmp_path / "paper_2509_06347_amd"
    pkg.mkdir()
    for f in ("__init__.py", "cgks.py"):
        shutil.copy(os.path.join(ROOT, "paper_2509_06347_amd", f), pkg / f)
    env = dict(os.environ, PYTHONPATH=str(tmp_path))
    r = subprocess.run([sys.executable, "-c", "import paper_2509_06347_amd.cgks"],
                       cwd=tmp_path, capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "no CPU fallback" in r.stderr
