"""The allocation-free entry point (lbm13_advance_noalloc), through the C ABI,
against the context path it is a variant of: set_state, step(n), get_state on
a context with the same launch configuration (three steps per launch, the
interior-tile kernel off).  Same kernels, so the results are bit-identical;
two calls in a row, the second on a smaller domain, reuse the static scratch."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from paper_1401_0188_amd import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print("[case] " + msg, flush=True)


def _context_run(lbm13, nx, ny, precision, f_in, n, sides, kw):
    lat = lbm13.Lattice(nx, ny, precision)
    lat.set_steps_per_launch(3)
    lat.set_interior_kernel(0)
    lat.set_params(sides=sides, **kw)
    lat.set_state(f_in)
    lat.step(n)
    out = lat.get_state().cpu().numpy()
    lat.destroy()
    return out


def _noalloc_run(lbm13, nx, ny, precision, f_in, n, sides, kw):
    import torch
    f = torch.as_tensor(f_in, dtype=torch.float64, device="cuda").contiguous()
    out = torch.full_like(f, float("nan"))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    st = lbm13.lib().lbm13_advance_noalloc(nx, ny, precision, ctypes.byref(lbm13.make_params(**kw)), sides,
                                           ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                                           ctypes.c_void_p(stream.cuda_stream))
    assert st == lbm13.OK, lbm13.lib().lbm13_last_error(None)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# (nx, ny, steps, sides (kinds, u_t, T_w), parameters): a walled cavity with
# buoyancy, then a smaller periodic-x channel with a moving wall and a force
CASES = [
    (96, 80, 31, ((2, 2, 1, 1), (0.01, 0.0, 0.0, 0.0), (-1.995, -2.005, 0.0, 0.0)), dict(g=(0.0, -0.02))),
    (40, 24, 17, ((0, 0, 2, 2), (0.0, 0.0, 0.02, 0.0), (0.0, 0.0, -1.99, -2.01)), dict(F0=(1e-5, 0.0))),
]


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_context_two_calls(precision):
    from paper_1401_0188_amd import lbm13
    for nx, ny, n, sd, kw in CASES:
        say("noalloc precision %d, %dx%d, %d steps" % (precision, nx, ny, n))
        sides = lbm13.make_sides(*sd)
        po = oracle.params(**{k: v for k, v in dict(gx=kw.get("g", (0, 0))[0], gy=kw.get("g", (0, 0))[1],
                                                     F0x=kw.get("F0", (0, 0))[0],
                                                     F0y=kw.get("F0", (0, 0))[1]).items()})
        # input: the oracle's post-collision populations of a seeded cavity state
        f0 = oracle.collide(oracle.init(*workloads.cavity_fields(nx, ny=ny, seed=7, dT=0.01), po), po)
        ref = _context_run(lbm13, nx, ny, precision, f0, n, sides, kw)
        got = _noalloc_run(lbm13, nx, ny, precision, f0, n, sides, kw)
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref), float(np.abs(got - ref).max())


def test_noalloc_rejects_before_device_work():
    from paper_1401_0188_amd import lbm13
    L = lbm13.lib()
    sides = lbm13.make_sides()
    p = ctypes.byref(lbm13.make_params())
    dummy = ctypes.c_void_p(256)  # never dereferenced: every case fails its host checks
    assert L.lbm13_advance_noalloc(4096, 4096, lbm13.FP32_DEV, p, sides, dummy, dummy, 3, None) == lbm13.EINVAL
    assert b"static scratch" in L.lbm13_last_error(None)
    assert L.lbm13_advance_noalloc(557, 557, lbm13.FP64, p, sides, dummy, dummy, 3, None) == lbm13.EINVAL
    assert L.lbm13_advance_noalloc(64, 64, lbm13.FP64, p, sides, dummy, dummy, -1, None) == lbm13.EINVAL
    assert L.lbm13_advance_noalloc(64, 64, lbm13.FP64, p, sides, None, dummy, 3, None) == lbm13.EINVAL
    bad = ctypes.byref(lbm13.make_params(s_XX=2.5))
    assert L.lbm13_advance_noalloc(64, 64, lbm13.FP64, bad, sides, dummy, dummy, 3, None) == lbm13.EUNSTABLE_PARAMS
