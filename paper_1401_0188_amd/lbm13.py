"""Thin ctypes binding of liblbm13.so (C ABI in include/lbm13.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch provides the device workspace and the stream.  There is
no CPU fallback: if the library is missing or no GPU is present the calls
raise.

Two layers:
  * ``lib()``: the raw ctypes handle with the C names (``lbm13_create`` ...).
  * ``Lattice`` / ``Batch``: owners of a context whose methods carry the same
    names without the ``lbm13_`` / ``lbm13_batch_`` prefix.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm13.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE_PARAMS, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_DEV = 0, 1
PERIODIC, WALL_ADIABATIC, WALL_DIRICHLET_T = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
DIAG_NAMES = ("sum_rho", "sum_jx", "sum_jy", "sum_E", "heat_flux", "Nu_mean", "u_max", "asym_abs",
              "asym_rel", "nonfinite", "rho_min", "Nu_west", "Nu_east", "wall_energy_in", "wall_mass_in")
FOURIER_FIELDS = ("rho", "ux", "uy", "E")
TILE_SHAPES = ((64, 4), (64, 8), (64, 16), (32, 8), (32, 16))
_FUSED = ((64, 16), (64, 12), (64, 8), (64, 4), (32, 32), (32, 16), (32, 8), (32, 4))
FUSED_TILE_SHAPES = {FP32_DEV: _FUSED, FP64: _FUSED}
# tiles of three steps per launch
STEP3_TILE_SHAPES = {FP32_DEV: ((64, 16), (32, 32), (64, 8), (32, 16), (32, 8)), FP64: ((64, 8), (32, 16), (32, 8))}


class LBM13Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbm13 error %d: %s" % (code, msg))
        self.code = code


class Side(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("u_tangential", ctypes.c_double), ("T_wall", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("s_XX", ctypes.c_double), ("s_rx", ctypes.c_double), ("s_eps", ctypes.c_double),
                ("s_varpi", ctypes.c_double), ("s_XXe", ctypes.c_double),
                ("Pr", ctypes.c_double), ("E0", ctypes.c_double), ("c1", ctypes.c_double),
                ("k2", ctypes.c_double), ("c_epsE", ctypes.c_double), ("c_varpi_rho", ctypes.c_double),
                ("c_varpi_E", ctypes.c_double),
                ("F0", ctypes.c_double * 2), ("g", ctypes.c_double * 2), ("rho0", ctypes.c_double),
                ("collide", ctypes.c_int), ("Q_E", ctypes.c_double)]


class Derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "A", "Y", "h1", "k1", "h2", "c2", "c_eps_rho", "sigma_XX", "sigma_q", "s_q",
        "nu", "kappa", "cs2", "B", "kappa_E")]


# Free-parameter set used by default (the paper prints none; chosen by a
# linear-stability scan of the dispersion relation, as the paper describes).
DEFAULT_PARAMS = dict(s_XX=1.6, s_rx=1.05, s_eps=1.0, s_varpi=1.0, s_XXe=1.5, Pr=0.71, E0=-2.0, c1=-3.0,
                      k2=-2.5, c_epsE=-2.5, c_varpi_rho=-6.0, c_varpi_E=-0.5, F0=(0.0, 0.0), g=(0.0, 0.0),
                      rho0=1.0, collide=1, Q_E=0.0)

_lib = None


def lib():
    """Load liblbm13.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbm13.so is not built: run `python -m paper_1401_0188_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
    sz, i32, i64 = ctypes.c_size_t, ctypes.c_int, ctypes.c_longlong
    P, S, D = ctypes.POINTER(Params), ctypes.POINTER(Side), ctypes.POINTER(Derived)
    sig = {
        "lbm13_derive": (i32, [P, D]),
        "lbm13_workspace_bytes": (sz, [i32, i32, i32]),
        "lbm13_create": (i32, [i32, i32, i32, vp, sz, vp, ctypes.POINTER(vp)]),
        "lbm13_set_params": (i32, [vp, P, S, D]),
        "lbm13_init_moments": (i32, [vp, dp, dp, dp, dp]),
        "lbm13_step": (i32, [vp, i64]),
        "lbm13_moments": (i32, [vp, dp, dp, dp, dp]),
        "lbm13_diagnostics": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
        "lbm13_fourier": (i32, [vp, i32, i32, ctypes.POINTER(ctypes.c_double)]),
        "lbm13_get_state": (i32, [vp, dp]),
        "lbm13_set_state": (i32, [vp, dp]),
        "lbm13_steps_done": (i64, [vp]),
        "lbm13_state_bytes": (sz, [vp]),
        "lbm13_save": (i32, [vp, vp, sz]),
        "lbm13_load": (i32, [vp, vp, sz]),
        "lbm13_set_tile": (i32, [vp, i32, i32]),
        "lbm13_autotune": (i32, [vp, i32, ip, ip]),
        "lbm13_autotune_cached": (i32, [vp, i32, ctypes.c_char_p, ip]),
        "lbm13_use_graph": (i32, [vp, i32]),
        "lbm13_set_steps_per_launch": (i32, [vp, i32]),
        "lbm13_set_fused_tile": (i32, [vp, i32, i32]),
        "lbm13_set_interior_kernel": (i32, [vp, i32]),
        "lbm13_launch_config": (i32, [vp, ip]),
        "lbm13_destroy": (i32, [vp]),
        "lbm13_last_error": (ctypes.c_char_p, [vp]),
        "lbm13_advance_noalloc": (i32, [i32, i32, i32, P, S, dp, dp, i64, vp]),
        "lbm13_batch_workspace_bytes": (sz, [i32, ip, ip, i32]),
        "lbm13_batch_create": (i32, [i32, ip, ip, i32, vp, sz, vp, ctypes.POINTER(vp)]),
        "lbm13_batch_set_params": (i32, [vp, i32, P, S, D]),
        "lbm13_batch_init_moments": (i32, [vp, i32, dp, dp, dp, dp]),
        "lbm13_batch_step": (i32, [vp, i64]),
        "lbm13_batch_moments": (i32, [vp, i32, dp, dp, dp, dp]),
        "lbm13_batch_diagnostics": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
        "lbm13_batch_fourier": (i32, [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_double)]),
        "lbm13_batch_get_state": (i32, [vp, i32, dp]),
        "lbm13_batch_set_state": (i32, [vp, i32, dp]),
        "lbm13_batch_state_bytes": (sz, [vp, i32]),
        "lbm13_batch_save": (i32, [vp, i32, vp, sz]),
        "lbm13_batch_load": (i32, [vp, i32, vp, sz]),
        "lbm13_batch_set_tile": (i32, [vp, i32, i32]),
        "lbm13_batch_autotune": (i32, [vp, i32, ip, ip]),
        "lbm13_batch_autotune_cached": (i32, [vp, i32, ctypes.c_char_p, ip]),
        "lbm13_batch_use_graph": (i32, [vp, i32]),
        "lbm13_batch_set_steps_per_launch": (i32, [vp, i32]),
        "lbm13_batch_set_fused_tile": (i32, [vp, i32, i32]),
        "lbm13_batch_set_interior_kernel": (i32, [vp, i32]),
        "lbm13_batch_launch_config": (i32, [vp, ip]),
        "lbm13_batch_nodes": (i64, [vp]),
        "lbm13_batch_destroy": (i32, [vp]),
        "lbm13_batch_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def make_params(**kw) -> Params:
    d = dict(DEFAULT_PARAMS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError("unknown parameter %r" % k)
        d[k] = v
    p = Params()
    for k, v in d.items():
        if k in ("F0", "g"):
            getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
        elif k == "collide":
            p.collide = int(v)
        else:
            setattr(p, k, float(v))
    return p


def make_sides(kinds=(PERIODIC,) * 4, u_t=(0.0,) * 4, T_w=(0.0,) * 4):
    arr = (Side * 4)()
    for w in range(4):
        arr[w].kind = int(kinds[w])
        arr[w].u_tangential = float(u_t[w])
        arr[w].T_wall = float(T_w[w])
    return arr


def advance_noalloc(nx: int, ny: int, precision: int, f_in, n: int, sides=None, f_out=None, stream=None, **kw):
    """lbm13_advance_noalloc: n steps of one domain from the absolute FP64
    post-collision populations f_in (device tensor [13][ny][nx]) into f_out
    (a new tensor unless given; may be f_in), with no context, no workspace
    and no device allocation inside the library (buffers in its static
    scratch).  Calls that overlap on one device race.  Returns f_out."""
    torch = _torch()
    f_in = _dev_f64(f_in, torch, 13 * int(nx) * int(ny))
    if f_out is None:
        f_out = torch.empty_like(f_in)
    elif not (f_out.is_cuda and f_out.is_contiguous() and f_out.dtype == torch.float64
              and f_out.numel() == f_in.numel()):
        raise LBM13Error(EINVAL, "f_out must be a contiguous float64 device tensor of 13*nx*ny values")
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib().lbm13_advance_noalloc(int(nx), int(ny), int(precision), ctypes.byref(make_params(**kw)),
                                     sides if sides is not None else make_sides(), ctypes.c_void_p(f_in.data_ptr()),
                                     ctypes.c_void_p(f_out.data_ptr()), int(n), ctypes.c_void_p(s.cuda_stream))
    if st != OK:
        raise LBM13Error(st, (lib().lbm13_last_error(None) or b"").decode())
    f_in.record_stream(s)
    f_out.record_stream(s)
    return f_out


def derive(**kw):
    """Host-side derived coefficients; returns (status, dict)."""
    d = Derived()
    st = lib().lbm13_derive(ctypes.byref(make_params(**kw)), ctypes.byref(d))
    return st, {n: getattr(d, n) for n, _ in Derived._fields_}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("lbm13 needs a GPU: torch.cuda.is_available() is False")
    return torch


def _checkpoint_blob(blob, torch, nbytes):
    """A checkpoint handed to load(): a contiguous device tensor of exactly the
    context's checkpoint size.  Checked on the host, so no copy is issued from
    a wrong buffer."""
    if not isinstance(blob, torch.Tensor) or not blob.is_cuda:
        raise LBM13Error(EINVAL, "checkpoint must be a device tensor")
    if not blob.is_contiguous():
        raise LBM13Error(EINVAL, "checkpoint tensor must be contiguous")
    if blob.numel() * blob.element_size() != nbytes:
        raise LBM13Error(EINVAL, "checkpoint has %d bytes, this domain's has %d"
                         % (blob.numel() * blob.element_size(), nbytes))
    return blob


def _dev_f64(a, torch, n):
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64) if not isinstance(a, torch.Tensor) else a,
                        dtype=torch.float64, device="cuda").contiguous()
    if t.numel() != n:
        raise ValueError("field has %d values, expected %d" % (t.numel(), n))
    return t


class _Base:
    _prefix = ""

    def launch_config(self) -> dict:
        """{steps_per_launch, tile (single-step), fused_tile (two- and three-step),
        interior_kernel: 0 every multi-step tile on the general kernel, 1 interior
        tiles on their own kernel beside it, 2 (three steps) both in one launch}."""
        cfg = (ctypes.c_int * 6)()
        self._check(getattr(lib(), self._prefix + "launch_config")(self._h, cfg))
        return dict(steps_per_launch=cfg[0], tile=(cfg[1], cfg[2]), fused_tile=(cfg[3], cfg[4]),
                    interior_kernel=int(cfg[5]))

    def set_interior_kernel(self, mode):
        """0 (False), 1 (True) or 2: see lbm13_set_interior_kernel."""
        self._check(getattr(lib(), self._prefix + "set_interior_kernel")(self._h, int(mode)))

    # The library works on the context's stream; tensors cross between it and
    # the caller's current stream here.  Both helpers do nothing when the two
    # streams are the same (the default).
    def _use(self, tensors):
        """Tensors the library reads or writes on the context's stream: that
        stream first waits for the work queued on the caller's stream (the
        tensors' contents, or earlier uses of their memory), and the allocator
        keeps their memory until the context's stream is done with it."""
        torch = _torch()
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)
            for t in tensors:
                t.record_stream(self.stream)

    def _hand_over(self, tensors):
        """Tensors the library wrote on the context's stream, returned to the
        caller: the caller's stream waits for them."""
        torch = _torch()
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            cur.wait_stream(self.stream)
        return tensors

    def _check(self, st):
        if st != OK:
            msg = getattr(lib(), self._prefix + "last_error")(self._h)
            raise LBM13Error(st, (msg or b"").decode())
        return st


class Lattice(_Base):
    """One nx x ny domain (owns its workspace tensor and context)."""

    _prefix = "lbm13_"

    def __init__(self, nx: int, ny: int, precision: int = FP64, stream=None):
        torch = _torch()
        L = lib()
        self.nx, self.ny, self.precision = int(nx), int(ny), int(precision)
        nbytes = L.lbm13_workspace_bytes(self.nx, self.ny, self.precision)
        if nbytes == 0:
            raise LBM13Error(EINVAL, "invalid size or precision")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._use([self.workspace])
        h = ctypes.c_void_p()
        st = L.lbm13_create(self.nx, self.ny, self.precision, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise LBM13Error(st, "lbm13_create failed: " + (L.lbm13_last_error(None) or b"").decode())
        self._h = h
        self.derived = None
        self._keep = []

    def set_params(self, sides=None, **kw):
        d = Derived()
        self._check(lib().lbm13_set_params(self._h, ctypes.byref(make_params(**kw)),
                                           sides if sides is not None else make_sides(), ctypes.byref(d)))
        self.derived = {n: getattr(d, n) for n, _ in Derived._fields_}
        return self.derived

    def init_moments(self, rho, ux, uy, T):
        torch = _torch()
        n = self.nx * self.ny
        f = [_dev_f64(a, torch, n) for a in (rho, ux, uy, T)]
        self._keep = f  # kept alive until the next init (the kernel is async)
        self._use(f)
        self._check(lib().lbm13_init_moments(self._h, *[ctypes.c_void_p(t.data_ptr()) for t in f]))

    def step(self, n: int = 1):
        self._check(lib().lbm13_step(self._h, int(n)))

    def moments(self):
        torch = _torch()
        out = [torch.empty((self.ny, self.nx), dtype=torch.float64, device="cuda") for _ in range(4)]
        self._use(out)
        self._check(lib().lbm13_moments(self._h, *[ctypes.c_void_p(t.data_ptr()) for t in out]))
        return tuple(self._hand_over(out))

    def diagnostics(self, check: bool = True):
        out = (ctypes.c_double * 16)()
        st = lib().lbm13_diagnostics(self._h, out)
        if check:
            self._check(st)
        return dict(zip(DIAG_NAMES, list(out)[:len(DIAG_NAMES)]))

    def fourier(self, kx: int, ky: int) -> dict:
        """sum q exp(-2 pi i (kx x/nx + ky y/ny)) for q in FOURIER_FIELDS (complex)."""
        out = (ctypes.c_double * 8)()
        self._check(lib().lbm13_fourier(self._h, int(kx), int(ky), out))
        return {q: complex(out[2 * k], out[2 * k + 1]) for k, q in enumerate(FOURIER_FIELDS)}

    def get_state(self):
        torch = _torch()
        out = torch.empty((13, self.ny, self.nx), dtype=torch.float64, device="cuda")
        self._use([out])
        self._check(lib().lbm13_get_state(self._h, ctypes.c_void_p(out.data_ptr())))
        return self._hand_over([out])[0]

    def set_state(self, src):
        torch = _torch()
        t = _dev_f64(src, torch, 13 * self.nx * self.ny)
        self._keep = [t]
        self._use([t])
        self._check(lib().lbm13_set_state(self._h, ctypes.c_void_p(t.data_ptr())))

    def save(self):
        """Raw checkpoint (device uint8 tensor): header (size, precision, steps)
        and the stored working-precision state."""
        torch = _torch()
        nbytes = int(lib().lbm13_state_bytes(self._h))
        out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._use([out])
        self._check(lib().lbm13_save(self._h, ctypes.c_void_p(out.data_ptr()), nbytes))
        return self._hand_over([out])[0]

    def load(self, blob):
        """Restore a checkpoint of this context's size and precision (and its
        step counter); anything else raises LBM13Error(EINVAL)."""
        torch = _torch()
        nbytes = int(lib().lbm13_state_bytes(self._h))
        blob = _checkpoint_blob(blob, torch, nbytes)
        self._keep = [blob]
        self._use([blob])
        self._check(lib().lbm13_load(self._h, ctypes.c_void_p(blob.data_ptr()), nbytes))

    def steps_done(self) -> int:
        return int(lib().lbm13_steps_done(self._h))

    def set_tile(self, tile_x: int, tile_y: int):
        self._check(lib().lbm13_set_tile(self._h, int(tile_x), int(tile_y)))

    def autotune(self, steps: int = 20):
        tx, ty = ctypes.c_int(), ctypes.c_int()
        self._check(lib().lbm13_autotune(self._h, int(steps), ctypes.byref(tx), ctypes.byref(ty)))
        return tx.value, ty.value

    def autotune_cached(self, cache_path: str, steps: int = 20) -> bool:
        """Autotune through the cache file; True when the cached choice was applied."""
        hit = ctypes.c_int()
        self._check(lib().lbm13_autotune_cached(self._h, int(steps), os.fsencode(cache_path), ctypes.byref(hit)))
        return bool(hit.value)

    def use_graph(self, k: int):
        self._check(lib().lbm13_use_graph(self._h, int(k)))

    def set_steps_per_launch(self, k: int):
        self._check(lib().lbm13_set_steps_per_launch(self._h, int(k)))

    def set_fused_tile(self, tile_x: int, tile_y: int):
        self._check(lib().lbm13_set_fused_tile(self._h, int(tile_x), int(tile_y)))

    def destroy(self):
        if getattr(self, "_h", None):
            lib().lbm13_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch(_Base):
    """Many independent domains advanced by one launch per step."""

    _prefix = "lbm13_batch_"

    def __init__(self, sizes, precision: int = FP32_DEV, stream=None):
        torch = _torch()
        L = lib()
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        self.count = len(self.sizes)
        self.precision = int(precision)
        nx = (ctypes.c_int * self.count)(*[s[0] for s in self.sizes])
        ny = (ctypes.c_int * self.count)(*[s[1] for s in self.sizes])
        nbytes = L.lbm13_batch_workspace_bytes(self.count, nx, ny, self.precision)
        if nbytes == 0:
            raise LBM13Error(EINVAL, "invalid sizes or precision")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._use([self.workspace])
        h = ctypes.c_void_p()
        st = L.lbm13_batch_create(self.count, nx, ny, self.precision, ctypes.c_void_p(self.workspace.data_ptr()),
                                  nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise LBM13Error(st, "lbm13_batch_create failed: " + (L.lbm13_batch_last_error(None) or b"").decode())
        self._h = h
        self.derived = [None] * self.count
        self._keep = {}

    def set_params(self, i: int, sides=None, **kw):
        d = Derived()
        self._check(lib().lbm13_batch_set_params(self._h, int(i), ctypes.byref(make_params(**kw)),
                                                 sides if sides is not None else make_sides(), ctypes.byref(d)))
        self.derived[i] = {n: getattr(d, n) for n, _ in Derived._fields_}
        return self.derived[i]

    def init_moments(self, i: int, rho, ux, uy, T):
        torch = _torch()
        nx, ny = self.sizes[i]
        f = [_dev_f64(a, torch, nx * ny) for a in (rho, ux, uy, T)]
        self._keep[i] = f
        self._use(f)
        self._check(lib().lbm13_batch_init_moments(self._h, int(i), *[ctypes.c_void_p(t.data_ptr()) for t in f]))

    def step(self, n: int = 1):
        self._check(lib().lbm13_batch_step(self._h, int(n)))

    def moments(self, i: int):
        torch = _torch()
        nx, ny = self.sizes[i]
        out = [torch.empty((ny, nx), dtype=torch.float64, device="cuda") for _ in range(4)]
        self._use(out)
        self._check(lib().lbm13_batch_moments(self._h, int(i), *[ctypes.c_void_p(t.data_ptr()) for t in out]))
        return tuple(self._hand_over(out))

    def diagnostics(self, check: bool = True):
        out = (ctypes.c_double * (16 * self.count))()
        st = lib().lbm13_batch_diagnostics(self._h, out)
        if check:
            self._check(st)
        vals = np.array(list(out)).reshape(self.count, 16)
        return [dict(zip(DIAG_NAMES, row[:len(DIAG_NAMES)])) for row in vals]

    def fourier(self, i: int, kx: int, ky: int) -> dict:
        out = (ctypes.c_double * 8)()
        self._check(lib().lbm13_batch_fourier(self._h, int(i), int(kx), int(ky), out))
        return {q: complex(out[2 * k], out[2 * k + 1]) for k, q in enumerate(FOURIER_FIELDS)}

    def get_state(self, i: int):
        torch = _torch()
        nx, ny = self.sizes[i]
        out = torch.empty((13, ny, nx), dtype=torch.float64, device="cuda")
        self._use([out])
        self._check(lib().lbm13_batch_get_state(self._h, int(i), ctypes.c_void_p(out.data_ptr())))
        return self._hand_over([out])[0]

    def set_state(self, i: int, src):
        torch = _torch()
        nx, ny = self.sizes[i]
        t = _dev_f64(src, torch, 13 * nx * ny)
        self._keep[("state", i)] = t
        self._use([t])
        self._check(lib().lbm13_batch_set_state(self._h, int(i), ctypes.c_void_p(t.data_ptr())))

    def save(self, i: int):
        torch = _torch()
        nbytes = int(lib().lbm13_batch_state_bytes(self._h, int(i)))
        out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._use([out])
        self._check(lib().lbm13_batch_save(self._h, int(i), ctypes.c_void_p(out.data_ptr()), nbytes))
        return self._hand_over([out])[0]

    def load(self, i: int, blob):
        torch = _torch()
        nbytes = int(lib().lbm13_batch_state_bytes(self._h, int(i)))
        blob = _checkpoint_blob(blob, torch, nbytes)
        self._keep[("blob", i)] = blob
        self._use([blob])
        self._check(lib().lbm13_batch_load(self._h, int(i), ctypes.c_void_p(blob.data_ptr()), nbytes))

    def set_tile(self, tile_x: int, tile_y: int):
        self._check(lib().lbm13_batch_set_tile(self._h, int(tile_x), int(tile_y)))

    def autotune(self, steps: int = 20):
        tx, ty = ctypes.c_int(), ctypes.c_int()
        self._check(lib().lbm13_batch_autotune(self._h, int(steps), ctypes.byref(tx), ctypes.byref(ty)))
        return tx.value, ty.value

    def autotune_cached(self, cache_path: str, steps: int = 20) -> bool:
        """Autotune through the cache file; True when the cached choice was applied."""
        hit = ctypes.c_int()
        self._check(lib().lbm13_batch_autotune_cached(self._h, int(steps), os.fsencode(cache_path),
                                                       ctypes.byref(hit)))
        return bool(hit.value)

    def use_graph(self, k: int):
        self._check(lib().lbm13_batch_use_graph(self._h, int(k)))

    def set_steps_per_launch(self, k: int):
        self._check(lib().lbm13_batch_set_steps_per_launch(self._h, int(k)))

    def set_fused_tile(self, tile_x: int, tile_y: int):
        self._check(lib().lbm13_batch_set_fused_tile(self._h, int(tile_x), int(tile_y)))

    def nodes(self) -> int:
        return int(lib().lbm13_batch_nodes(self._h))

    def destroy(self):
        if getattr(self, "_h", None):
            lib().lbm13_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
