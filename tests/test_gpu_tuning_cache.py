"""The GEMM tuning cache of etdm_create (gemm_tuning = 0).

The kernel choice of a stage is timed once per stage signature in a process and, with
ETDM_TUNE_CACHE naming a file, read from and appended to that file.  The workload
here has shapes no other test uses, so its first handle is a cache miss.
"""
import copy

import numpy as np
import pytest

from oracle import etdm as O
from workloads import tiny_real

from gpu_helpers import energy_grad, make_handle

pytestmark = pytest.mark.gpu

VARIANTS = ["tile64", "packed64", "packed128x64", "packed64x128", "packed128"]


def _workload():
    # two instances of M = 333, N = 131 (stages of at least 128 x 128, so the tuning
    # has five kernels to choose from), mixed precision keeps them FP64
    return tiny_real(333, 131, seed=61, scale=0.2, n_inst=2)


def _gemm_stages(h):
    return [k for k in h.stage_kernels() if k["kernel"]]


def test_tuning_cache_reuses_and_persists_choices(tmp_path, monkeypatch):
    wl = _workload()
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("ETDM_TUNE_CACHE", str(path))
    print("[case] tuning cache: first handle (timed)", flush=True)
    h1, _ = make_handle(wl, "mixed", gemm_tuning=0)
    k1 = _gemm_stages(h1)
    h1.close()
    assert k1
    lines = path.read_text().split("\n")[:-1]
    assert lines, "no tuning entries were written"
    for line in lines:
        f = line.split()
        assert len(f) == 2 + len(VARIANTS), line
        assert f[0].startswith("gfx") and 0 <= int(f[1]) < len(VARIANTS)

    # a second handle with the same stages takes the cached choice: the same kernels and
    # the very same stored times (timing again would not reproduce them)
    print("[case] tuning cache: second handle (cached)", flush=True)
    h2, _ = make_handle(wl, "mixed", gemm_tuning=0)
    k2 = _gemm_stages(h2)
    h2.close()
    assert [k["kernel"] for k in k2] == [k["kernel"] for k in k1]
    assert [k["tuned_ms"] for k in k2] == [k["tuned_ms"] for k in k1]
    assert path.read_text().split("\n")[:-1] == lines  # nothing appended on a hit

    # entries from a file are honoured: every stage pinned to the 64 x 64 packed kernel
    pinned = tmp_path / "pinned.txt"
    pinned.write_text("".join(" ".join([l.split()[0], "1"] + l.split()[2:]) + "\n" for l in lines))
    monkeypatch.setenv("ETDM_TUNE_CACHE", str(pinned))
    print("[case] tuning cache: choices read from a file", flush=True)
    h3, _ = make_handle(wl, "mixed", gemm_tuning=0)
    k3 = _gemm_stages(h3)
    params = O.parity_params(wl)
    E, g = energy_grad(h3, wl, params)
    h3.close()
    assert all(k["kernel"].endswith("packed64") for k in k3), [k["kernel"] for k in k3]
    for k, inst in enumerate(wl.instances):
        sub = copy.copy(wl)
        sub.instances = [inst]
        E_ref, (g_ref,) = O.energy_grad(sub, [params[k]])
        assert abs(E[k] - E_ref) / inst.f.sum() < 1e-8
        assert np.linalg.norm(g[k] - g_ref) / np.linalg.norm(g_ref) < 1e-6
