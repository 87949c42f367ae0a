"""Host logic of bench.py that needs no GPU: the HBM traffic figure of a kernel is read
from a committed rocprofv3 summary only while the kernel's source files still hash to
the value recorded next to it (otherwise the figure is reported as unknown)."""
import hashlib
import os

import bench


def _write_profile(root, sha, nbytes=1234567):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "k_traffic_pmc.txt"), "w") as f:
        f.write("# rocprofv3 PMC summary\n")
        f.write(f"# traffic: stage=eigh_lds config=2 precision=mixed bytes_per_launch={nbytes} "
                f"source=src/a.hip,src/b.h sha256={sha}\n")


def test_traffic_figure_follows_the_source_hash(tmp_path, monkeypatch):
    root = str(tmp_path)
    os.makedirs(os.path.join(root, "src"))
    for name, text in (("a.hip", "kernel a\n"), ("b.h", "header b\n")):
        with open(os.path.join(root, "src", name), "w") as f:
            f.write(text)
    h = hashlib.sha256()
    for name in ("a.hip", "b.h"):  # hashed in the listed order
        h.update(open(os.path.join(root, "src", name), "rb").read())
    _write_profile(root, h.hexdigest()[:16])
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic("eigh_lds", 2, "mixed") == 1234567.0
    # another workload, precision or stage has no figure
    assert bench.measured_traffic("eigh_lds", 3, "mixed") is None
    assert bench.measured_traffic("eigh_lds", 2, "fp64") is None
    assert bench.measured_traffic("gemm_P", 2, "mixed") is None
    # a changed source makes the recorded figure stale
    with open(os.path.join(root, "src", "b.h"), "a") as f:
        f.write("changed\n")
    assert bench.measured_traffic("eigh_lds", 2, "mixed") is None
    # a missing source likewise
    os.remove(os.path.join(root, "src", "b.h"))
    assert bench.measured_traffic("eigh_lds", 2, "mixed") is None


def test_more_than_one_gpu_is_refused():
    """The path runs on one GPU: --gpus N with N > 1 exits with status 2 and says so,
    before any device or oracle work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.abspath(bench.__file__))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""
