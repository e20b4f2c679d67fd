"""C-ABI checks that need no GPU: the library loads, exports every function
include/lbm13.h declares, and its host-side logic (parameter derivation,
workspace sizing, argument validation) behaves as documented."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import oracle
from paper_1401_0188_amd import lbm13

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm13.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+(lbm13_[A-Za-z0-9_]+)\s*\(", text, re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lbm13_create", "lbm13_set_params", "lbm13_step", "lbm13_moments", "lbm13_diagnostics",
                 "lbm13_init_moments", "lbm13_destroy", "lbm13_batch_create", "lbm13_batch_step"):
        assert must in names
    assert len(names) >= 30


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(lbm13.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert missing == []


def test_binding_covers_every_declared_symbol():
    lbm13.lib()
    for n in declared_functions():
        assert getattr(lbm13.lib(), n).argtypes is not None, n


@pytest.mark.parametrize("kw", [dict(), dict(s_XX=1.2, Pr=1.0), dict(s_XX=1.9, Pr=7.0, c1=-2.5, E0=-1.0, k2=-1.0),
                                dict(c_epsE=-1.0, c_varpi_rho=-3.0, c_varpi_E=-0.2)])
def test_library_derivation_matches_oracle(kw):
    """Two independent codes (library C++, oracle C) agree on the constrained
    coefficients of eqs (d2q13-diffusion), (d2q13-sigma-qx)."""
    st_l, dl = lbm13.derive(**kw)
    okw = {k: v for k, v in kw.items()}
    st_o, do = oracle.derive(oracle.params(**okw))
    assert (st_l == lbm13.OK) == (st_o == 0)
    for k in do:
        assert dl[k] == pytest.approx(do[k], rel=1e-13, abs=1e-15), k


def test_derive_rejects_out_of_range_rates():
    assert lbm13.derive(s_XX=2.0)[0] == lbm13.EUNSTABLE_PARAMS
    assert lbm13.derive(s_rx=0.0)[0] == lbm13.EUNSTABLE_PARAMS
    assert lbm13.derive(Pr=0.0)[0] == lbm13.EUNSTABLE_PARAMS
    assert lbm13.derive()[0] == lbm13.OK


@pytest.mark.parametrize("kw", [dict(c1=-8.0, E0=0.0, c_epsE=-30.0),     # A = -9, every rate in (0, 2)
                                dict(c1=-7.0, E0=-2.0, c_epsE=-2.5),     # A = 0
                                dict(c1=-3.0, E0=-28.5, c_epsE=-2.5)])   # A = -1 through E0
def test_derive_rejects_nonpositive_sound_speed(kw):
    """A = 13 c1 + 95 + 2 E0 <= 0 leaves no positive sound speed (cs2 = A/52)
    nor viscosity (nu = sigma_XX A/104): both codes return the unstable code,
    even where the given and derived rates all lie in (0, 2)."""
    st_l, dl = lbm13.derive(**kw)
    st_o, do = oracle.derive(oracle.params(**kw))
    assert dl["A"] <= 0.0 and do["A"] <= 0.0
    assert st_l == lbm13.EUNSTABLE_PARAMS
    assert st_o != 0
    if kw["c_epsE"] == -30.0:
        assert 0.0 < dl["s_q"] < 2.0  # only the sign of A rules this set out


def test_workspace_sizes():
    L = lbm13.lib()
    a = L.lbm13_workspace_bytes(4096, 4096, lbm13.FP32_DEV)
    b = L.lbm13_workspace_bytes(4096, 4096, lbm13.FP64)
    # two population buffers dominate: 2 * 13 * nodes * bytes
    assert 2 * 13 * 4096 * 4096 * 4 < a < 1.02 * 2 * 13 * 4096 * 4096 * 4
    assert 2 * 13 * 4096 * 4096 * 8 < b < 1.02 * 2 * 13 * 4096 * 4096 * 8
    assert L.lbm13_workspace_bytes(1, 8, lbm13.FP64) == 0
    assert L.lbm13_workspace_bytes(8, 8, 7) == 0
    nx = (ctypes.c_int * 3)(64, 100, 37)
    ny = (ctypes.c_int * 3)(64, 50, 300)
    assert L.lbm13_batch_workspace_bytes(3, nx, ny, lbm13.FP32_DEV) > 2 * 13 * 4 * (64 * 64 + 100 * 50 + 37 * 300)


def test_create_rejects_bad_arguments_without_touching_the_device():
    L = lbm13.lib()
    h = ctypes.c_void_p()
    assert L.lbm13_create(64, 64, lbm13.FP64, None, 1 << 30, None, ctypes.byref(h)) == lbm13.EINVAL
    assert L.lbm13_create(1, 64, lbm13.FP64, ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h)) == lbm13.EINVAL
    assert L.lbm13_create(64, 64, lbm13.FP64, ctypes.c_void_p(256), 16, None, ctypes.byref(h)) == lbm13.ENOMEM
    assert L.lbm13_create(64, 64, lbm13.FP64, ctypes.c_void_p(257), 1 << 30, None, ctypes.byref(h)) == lbm13.EINVAL
    assert h.value is None
    assert L.lbm13_step(None, 1) == lbm13.EINVAL
    assert L.lbm13_destroy(None) == lbm13.EINVAL
    assert L.lbm13_last_error(None) == b"null context"


def test_c_api_example_builds_without_torch(tmp_path):
    """include/lbm13.h is a self-sufficient C ABI: a C++ program that uses only
    HIP and the library's calls compiles and links against liblbm13.so."""
    from paper_1401_0188_amd import build
    out = build.build_example(out=str(tmp_path / "c_api_example"))
    assert os.path.getsize(out) > 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry point raises: there is no CPU path."""
    monkeypatch.setattr(lbm13, "LIB_PATH", str(tmp_path / "liblbm13.so"))
    monkeypatch.setattr(lbm13, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        lbm13.lib()
    with pytest.raises(Exception):
        lbm13.Lattice(8, 8, lbm13.FP64)
    with pytest.raises(Exception):
        lbm13.Batch([(8, 8)], lbm13.FP32_DEV)


def test_no_device_fails_loudly():
    """On a host without a GPU the binding raises instead of computing on the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(Exception):
        lbm13.Lattice(8, 8, lbm13.FP64)
    with pytest.raises(Exception):
        lbm13.Batch([(8, 8), (5, 3)], lbm13.FP32_DEV)


def test_checkpoint_blob_checked_on_host():
    """load() validates the checkpoint tensor before any copy is issued."""
    import torch
    with pytest.raises(lbm13.LBM13Error, match="device tensor"):
        lbm13._checkpoint_blob(torch.zeros(64, dtype=torch.uint8), torch, 64)
    with pytest.raises(lbm13.LBM13Error, match="device tensor"):
        lbm13._checkpoint_blob(b"\0" * 64, torch, 64)
