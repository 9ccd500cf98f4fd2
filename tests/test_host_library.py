"""Host-side checks of the C-ABI library: it loads, exports every declared
entry point, validates its launch plans for every workload size without a
GPU, and reports missing devices as an error."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lrcc.h")).read()
    return sorted(set(re.findall(r"\b(lrcc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2508_01266_amd import lrcc
    L = ctypes.CDLL(lrcc.LIB_PATH)
    names = _declared()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("name,nrhs", [("c1", 9), ("c2", 9), ("c3", 48), ("c4", 2), ("c4s", 2)])
def test_plans_in_bounds_for_workloads(name, nrhs):
    from paper_2508_01266_amd import plan_check
    w = synth.WORKLOADS[name]
    plan_check(w.nk, w.nocc, w.nvir, w.naux, nrhs)


@pytest.mark.parametrize("nk,o,v,naux,nrhs", [(1, 1, 1, 1, 1), (2, 3, 5, 7, 3), (4, 2, 3, 5, 2), (9, 12, 80, 276, 1)])
def test_plans_in_bounds_edge_sizes(nk, o, v, naux, nrhs):
    from paper_2508_01266_amd import plan_check
    plan_check(nk, o, v, naux, nrhs)


@pytest.mark.parametrize("mesh,o,v,naux,nrhs", [((2, 2, 1), 2, 3, 5, 3), ((2, 2, 2), 1, 3, 4, 2),
                                                 ((3, 2, 1), 2, 4, 6, 2), ((2, 2, 2), 8, 40, 144, 12),
                                                 ((1, 1, 4), 3, 5, 7, 24)])
def test_plans_in_bounds_on_3d_meshes(mesh, o, v, naux, nrhs):
    from paper_2508_01266_amd import plan_check
    plan_check(mesh, o, v, naux, nrhs)


def test_plan_check_rejects_bad_sizes():
    from paper_2508_01266_amd import LrccError, plan_check
    with pytest.raises(LrccError):
        plan_check(0, 1, 1, 1, 1)
    with pytest.raises(LrccError):
        plan_check((2, 0, 1), 1, 1, 1, 1)


def test_create_without_device_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2508_01266_amd import Context, LrccError
    with pytest.raises(LrccError):
        Context(0)


def test_measure_peaks_without_device_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2508_01266_amd import LrccError, measure_peaks
    with pytest.raises(LrccError):
        measure_peaks(0)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
