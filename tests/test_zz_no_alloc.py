"""sgn_mass_energy_noalloc (totals with no context and no allocation) against
sgn_mass_energy on the same inputs: bit-identical (same kernels, same order),
on two calls in a row, the second on a smaller grid (the static partial-sum
array keeps the first call's contents), in FP64 and FP32, periodic and
reflecting; and the argument errors.  Through the C ABI."""

import numpy as np
import pytest
import torch

from paper_2601_02540_amd import workloads as W
from paper_2601_02540_amd.binding import SgnError, Solver, mass_energy_noalloc

pytestmark = pytest.mark.gpu


def state(n, ny, bc, dtype, seed):
    g = W.Grid(n, ny, -1.0, 2.0, 0.5, 2.0, bc, bc, 9.81, 500.0)
    q, b = W.random_state(g, seed, b_scale=0.05)
    return g, torch.from_numpy(q).to(dtype).cuda().contiguous(), torch.from_numpy(b).to(dtype).cuda().contiguous()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", [W.PERIODIC, W.REFLECTING])
def test_noalloc_totals_match_context_totals(bc, dtype):
    # a grid with more rows than reduction blocks, then a small ragged one
    for n, ny, seed in ((700, 1300, 1), (37, 9, 2)):
        g, q, b = state(n, ny, bc, dtype, seed)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        mass_energy_noalloc(g, q, b, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        s = Solver(g, dtype)
        s.set_bathymetry(b)
        m, e = s.mass_energy(q)
        s.close()
        assert got[0] == m and got[1] == e, (n, ny, got, m, e)
        assert np.isfinite(got).all()


def test_noalloc_totals_on_a_side_stream():
    g, q, b = state(300, 200, W.PERIODIC, torch.float64, 3)
    side = torch.cuda.Stream()
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        mass_energy_noalloc(g, q, b, out, stream=side)
    side.synchronize()
    s = Solver(g, torch.float64)
    s.set_bathymetry(b)
    m, e = s.mass_energy(q)
    assert out[0].item() == m and out[1].item() == e


def test_noalloc_argument_errors():
    from paper_2601_02540_amd.binding import SgnParams, load_library
    import ctypes
    lib = load_library()
    g, q, b = state(16, 16, W.PERIODIC, torch.float64, 4)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    p = SgnParams(3, 16, 0.0, 1.0, 0.0, 1.0, 0, 0, 9.81, 500.0, 0, 0)   # fewer than 4 nodes
    st = lib.sgn_mass_energy_noalloc(ctypes.byref(p), ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                     None, ctypes.cast(ctypes.c_void_p(out.data_ptr()), ctypes.POINTER(ctypes.c_double)))
    assert st == -2 and b"4 nodes" in lib.sgn_last_error(None)
    p = SgnParams(16, 16, 0.0, 1.0, 0.0, 1.0, 0, 0, 9.81, 500.0, 0, 0)
    st = lib.sgn_mass_energy_noalloc(ctypes.byref(p), None, ctypes.c_void_p(b.data_ptr()), None,
                                     ctypes.cast(ctypes.c_void_p(out.data_ptr()), ctypes.POINTER(ctypes.c_double)))
    assert st == -1
    with pytest.raises(ValueError):
        mass_energy_noalloc(g, q, b.float(), out)
    with pytest.raises(SgnError):
        bad = W.Grid(16, 16, 1.0, 0.0, 0.0, 1.0, 0, 0, 9.81, 500.0)   # xmax < xmin
        mass_energy_noalloc(bad, q, b, out)
