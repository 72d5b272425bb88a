"""CPU-side checks of the boundary: the HIP library builds for gfx950, loads, and
exports every function declared in include/sgn.h.  No compute call is made."""

import ctypes
import os

import pytest

from paper_2601_02540_amd import binding


def test_header_declares_core_api():
    syms = binding.header_symbols()
    for name in ("sgn_create", "sgn_destroy", "sgn_set_bathymetry", "sgn_init_aux", "sgn_rhs", "sgn_step",
                 "sgn_mass", "sgn_energy", "sgn_rates", "sgn_cfl_dt", "sgn_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2601_02540_amd import build
        build.build()
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [s for s in binding.header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_library_targets_gfx950_only():
    """The offload bundle inside the library carries gfx950 code objects."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    data = open(binding.LIB_PATH, "rb").read()
    assert b"gfx950" in data
    assert b"gfx942" not in data and b"gfx90a" not in data


def test_status_strings_without_gpu():
    lib = binding.load_library()
    assert lib.sgn_status_string(0) == b"SGN_OK"
    assert lib.sgn_status_string(-5) == b"SGN_E_NONPOS_DEPTH"


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2601_02540_amd import workloads as W
    with pytest.raises(RuntimeError):
        binding.Solver(W.Grid(8, 8, 0.0, 1.0, 0.0, 1.0))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message before
    touching a device."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["requested_gpus"] == 2 and "one GPU" in msg["error"]


def test_product_fails_loudly_without_library_or_gpu(monkeypatch):
    """No fallback: a missing library raises, and so does a solver on a host
    without a ROCm GPU (this container has none)."""
    import torch
    from paper_2601_02540_amd import workloads as W
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", os.path.join(os.path.dirname(binding.LIB_PATH), "missing_libsgn.so"))
    with pytest.raises(RuntimeError, match="missing"):
        binding.load_library()
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError, match="ROCm GPU"):
            binding.Solver(W.Grid(8, 8, 0.0, 1.0, 0.0, 1.0))
