"""The C ABI library loads and exports every entry point include/fmm.h declares;
argument validation works on the host (no GPU work is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2003_13218_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2003_13218_amd import build
        build.build()
    return binding.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("fmm_plan", "fmm_energy_forces", "fmm_solute_solvent_energy", "fmm_last_error", "fmm_destroy"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    from paper_2003_13218_amd import binding
    assert set(binding.EXPORTED) == set(declared_functions())


def test_version_and_null_handling():
    lib = _lib()
    assert b"gfx950" in lib.fmm_version()
    lib.fmm_destroy(None)  # ignored
    assert lib.fmm_last_error(None) is not None


@pytest.mark.parametrize("box,levels,p", [(0.0, 3, 4), (-1.0, 3, 4), (float("nan"), 3, 4), (float("inf"), 3, 4),
                                          (10.0, 0, 4), (10.0, 11, 4), (10.0, 3, -1), (10.0, 3, 21)])
def test_plan_rejects_bad_arguments(box, levels, p):
    lib = _lib()
    h = ctypes.c_void_p(123)
    st = lib.fmm_plan(box, levels, p, ctypes.byref(h))
    assert st == -1  # FMM_ERR_INVALID, before any device call
    assert h.value is None
    assert lib.fmm_last_error(None).decode().startswith("fmm_plan:")


def test_calls_on_null_plan_are_rejected():
    lib = _lib()
    e = ctypes.c_double()
    assert lib.fmm_energy_forces(None, 0, None, None, ctypes.byref(e), None, None) == -1
    assert lib.fmm_solute_solvent_energy(None, None, ctypes.byref(e)) == -1
    assert lib.fmm_plan_config(None, 0, 0.0, None) == -1
    assert lib.fmm_profile(None, 1) == -1
    hit = ctypes.c_int(7)
    assert lib.fmm_batch_set_tuning(None, None, None) == -1
    assert lib.fmm_autotune_batch_cached(None, None, None, None, None, b"x", ctypes.byref(hit)) == -1
    assert hit.value == 0


def test_plan_without_gpu_reports_device_error():
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    lib = _lib()
    h = ctypes.c_void_p()
    st = lib.fmm_plan(10.0, 3, 4, ctypes.byref(h))
    assert st == -3  # FMM_ERR_DEVICE
    assert "device" in lib.fmm_last_error(None).decode()


def test_bench_cli_single_gpu_only():
    # bench.py imports and parses on a machine without a GPU, and refuses a
    # multi-GPU run with a message (this build runs on one GPU)
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and "--uv-scheme" in r.stdout
