"""cgks_compute_dt_noalloc, the time-step entry point that allocates nothing (its block partials live
in the library's static device scratch), against cgks_compute_dt of a context holding the same state:
the same time step bit for bit, on two calls in a row, the second with a smaller grid; a non-physical
cell is reported in the flag output."""
import ctypes

import numpy as np
import pytest

from paper_2508_19911_amd import inputs

pytestmark = pytest.mark.gpu


def _noalloc(lib, case, q_dev, out_dev, cfl, stream):
    from paper_2508_19911_amd import cgks
    p = cgks.params_from_case(case)
    return lib.cgks_compute_dt_noalloc(ctypes.byref(p), ctypes.c_void_p(q_dev.data_ptr()),
                                       ctypes.c_void_p(stream.cuda_stream), float(cfl),
                                       ctypes.c_void_p(out_dev.data_ptr()))


def test_noalloc_time_step_matches_context_time_step():
    import torch
    from paper_2508_19911_amd import cgks
    lib = cgks.load()
    stream = torch.cuda.current_stream()
    # 96^3 needs more blocks than the scratch holds (each thread then folds several cells); the second
    # call is a small ragged grid with the inviscid limit only
    cases = [inputs.tgv_case(96, ma=0.3).with_(recon=1),
             inputs.vortex_case(8).with_(nx=10, ny=8, nz=6, lz=2.0)]
    for k, case in enumerate(cases):
        q, g = inputs.seeded_smooth_state(case, seed=31 + k, amp=0.2)
        s = cgks.Solver(case)
        s.set_state(q, g)
        ref = s.compute_dt(case.cfl)
        s.close()
        q_dev = torch.tensor(q, dtype=torch.float64, device="cuda").contiguous()
        out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
        assert _noalloc(lib, case, q_dev, out, case.cfl, stream) == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got[0] == ref and got[1] == 0.0, (k, got, ref)
    # a non-physical cell sets the flag; a bad argument is rejected before any device work
    q[4, 5] = -1.0
    q_dev = torch.tensor(q, dtype=torch.float64, device="cuda").contiguous()
    assert _noalloc(lib, cases[1], q_dev, out, 0.5, stream) == 0
    torch.cuda.synchronize()
    assert out.cpu().numpy()[1] == 1.0
    assert _noalloc(lib, cases[1], q_dev, out, -0.5, stream) == -1
    p = cgks.params_from_case(cases[1].with_(nx=0))
    assert lib.cgks_compute_dt_noalloc(ctypes.byref(p), ctypes.c_void_p(q_dev.data_ptr()), None, 0.5,
                                       ctypes.c_void_p(out.data_ptr())) == -1
