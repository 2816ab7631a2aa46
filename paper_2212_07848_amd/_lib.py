"""ctypes binding of ``libfsc.so`` (include/fsc.h): argument marshalling only.

Every computation runs in the library's HIP kernels; this module converts
numpy arrays and Python scalars to the C ABI and raises on error codes.  The
library must have been built (``__graft_entry__.build()``); importing the
binding without it raises, so there is no silent fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FSC_LIB selects another build of the library (a debug build, say); by
# default the one built in the package directory
LIBPATH = os.environ.get("FSC_LIB") or os.path.join(_HERE, "libfsc.so")

FSC_E4, FSC_E8 = 4, 8
FSC_FP32_SHIFTED, FSC_FP64 = 0, 1
FSC_SK_AXIS, FSC_SK_RADIAL = 0, 1

ERRORS = {0: "ok", -1: "invalid argument", -2: "HIP runtime error", -3: "out of memory",
          -4: "diverged", -5: "invalid state", -6: "not supported", -7: "file error",
          -8: "input exceeds the fixed-size scratch"}

# Every symbol include/fsc.h declares.
EXPORTS = [
    "fsc_create", "fsc_create_external", "fsc_destroy", "fsc_last_error", "fsc_strerror",
    "fsc_get_params", "fsc_init_uniform", "fsc_set_populations", "fsc_get_populations",
    "fsc_step", "fsc_run", "fsc_get_step", "fsc_save", "fsc_load", "fsc_density",
    "fsc_read_density", "fsc_stats", "fsc_conserved", "fsc_sk_reset",
    "fsc_measure_sk", "fsc_sk_nbins", "fsc_read_sk", "fsc_series_enable", "fsc_read_series",
    "fsc_ens_create", "fsc_ens_destroy", "fsc_ens_last_error", "fsc_ens_init_uniform",
    "fsc_ens_run", "fsc_ens_get_step", "fsc_ens_get_populations", "fsc_ens_set_populations",
    "fsc_ens_stats", "fsc_ens_density", "fsc_ens_sk_nbins", "fsc_ens_read_sk", "fsc_ens_sk_reset",
    "fsc_ens_save", "fsc_ens_load", "fsc_modes_enable", "fsc_read_modes", "fsc_ens_modes_enable",
    "fsc_ens_read_modes", "fsc_ens_series_enable", "fsc_ens_read_series",
    "fsc_autotune", "fsc_ens_autotune", "fsc_get_tiling", "fsc_ens_get_tiling",
    "fsc_tile_shapes", "fsc_set_tiling", "fsc_ens_set_tiling",
    "fsc_copy", "fsc_philox", "fsc_normals", "fsc_linear_sk", "fsc_linear_sk_radial",
    "fsc_linear_corr",
    "fsc_sur_create", "fsc_sur_destroy", "fsc_sur_last_error", "fsc_sur_nparams",
    "fsc_sur_set_params", "fsc_sur_get_params", "fsc_sur_set_norm", "fsc_sur_forward",
    "fsc_sur_grad", "fsc_sur_train_step", "fsc_sur_rollout", "fsc_sur_set_fusion", "fsc_sur_gather",
    "fsc_stack_scales", "fsc_coarsen", "fsc_ens_coarsen", "fsc_field_nbins",
    "fsc_field_sk", "fsc_field_sk_noalloc", "fsc_mfma_probe",
]


class FscError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{ERRORS.get(code, code)} ({code}){': ' + msg if msg else ''}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("D", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("stencil", C.c_int32), ("precision", C.c_int32),
                ("T_hat", C.c_double), ("G", C.c_double), ("rho0", C.c_double),
                ("lambda_bulk", C.c_double), ("lambda_shear", C.c_double),
                ("lambda_ghost", C.c_double), ("kBT", C.c_double),
                ("seed", C.c_uint64), ("replica", C.c_uint32), ("reserved", C.c_uint32)]


assert C.sizeof(Params) == 96


def make_params(*, D=2, nx=64, ny=64, nz=1, stencil=4, precision="fp32", T_hat=0.9,
                G=math.nan, rho0=0.5, lam=(1.0, 1.0, 1.0), kBT=0.0, seed=0, replica=0) -> Params:
    prec = {"fp32": FSC_FP32_SHIFTED, "fp64": FSC_FP64}.get(precision, precision)
    return Params(D, nx, ny, 1 if D == 2 else nz, stencil, prec, T_hat, G, rho0,
                  lam[0], lam[1], lam[2], kBT, seed, replica, 0)


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is not built; run __graft_entry__.build() first")
    # PyTorch ships its own HIP runtime (same soname, another file name).  With
    # torch loaded first, this library binds to that runtime; loaded first, it
    # would bring in the system one, and torch would start a second runtime in
    # the same process that finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIBPATH)
    vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
    fp = C.POINTER(C.c_float)
    pp = C.POINTER(Params)
    u32p = C.POINTER(C.c_uint32)
    sig = {
        "fsc_create": ([pp, vp, C.POINTER(vp)], C.c_int),
        "fsc_create_external": ([pp, vp, vp, vp, C.POINTER(vp)], C.c_int),
        "fsc_destroy": ([vp], C.c_int),
        "fsc_last_error": ([vp], C.c_char_p),
        "fsc_strerror": ([C.c_int], C.c_char_p),
        "fsc_get_params": ([vp, pp], C.c_int),
        "fsc_init_uniform": ([vp], C.c_int),
        "fsc_set_populations": ([vp, dp, C.c_int64], C.c_int),
        "fsc_get_populations": ([vp, dp, i64p], C.c_int),
        "fsc_step": ([vp, C.c_int64], C.c_int),
        "fsc_run": ([vp, C.c_int64, C.c_int64], C.c_int),
        "fsc_get_step": ([vp, i64p], C.c_int),
        "fsc_save": ([vp, C.c_char_p], C.c_int),
        "fsc_load": ([vp, C.c_char_p], C.c_int),
        "fsc_ens_save": ([vp, C.c_char_p], C.c_int),
        "fsc_ens_load": ([vp, C.c_char_p], C.c_int),
        "fsc_density": ([vp, dp], C.c_int),
        "fsc_stats": ([vp, dp], C.c_int),
        "fsc_read_density": ([vp, dp], C.c_int),
        "fsc_conserved": ([vp, dp, dp], C.c_int),
        "fsc_sk_reset": ([vp], C.c_int),
        "fsc_measure_sk": ([vp], C.c_int),
        "fsc_sk_nbins": ([vp, C.c_int, C.POINTER(C.c_int)], C.c_int),
        "fsc_read_sk": ([vp, C.c_int, dp, dp, i64p, C.c_int], C.c_int),
        "fsc_series_enable": ([vp, C.c_int], C.c_int),
        "fsc_read_series": ([vp, dp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "fsc_ens_series_enable": ([vp, C.c_int], C.c_int),
        "fsc_ens_read_series": ([vp, C.c_int, dp, C.c_int, C.POINTER(C.c_int),
                                 C.POINTER(C.c_int)], C.c_int),
        "fsc_ens_create": ([pp, C.c_int, vp, C.POINTER(vp)], C.c_int),
        "fsc_ens_destroy": ([vp], C.c_int),
        "fsc_ens_last_error": ([vp], C.c_char_p),
        "fsc_ens_init_uniform": ([vp], C.c_int),
        "fsc_ens_run": ([vp, C.c_int64, C.c_int64], C.c_int),
        "fsc_ens_get_step": ([vp, i64p], C.c_int),
        "fsc_ens_get_populations": ([vp, C.c_int, dp], C.c_int),
        "fsc_ens_set_populations": ([vp, C.c_int, dp], C.c_int),
        "fsc_ens_stats": ([vp, C.c_int, dp], C.c_int),
        "fsc_ens_sk_nbins": ([vp, C.c_int, C.c_int, C.POINTER(C.c_int)], C.c_int),
        "fsc_ens_read_sk": ([vp, C.c_int, C.c_int, dp, dp, i64p, C.c_int], C.c_int),
        "fsc_ens_sk_reset": ([vp], C.c_int),
        "fsc_ens_density": ([vp, C.c_int, dp], C.c_int),
        "fsc_linear_sk": ([pp, dp, C.c_int64, dp, vp], C.c_int),
        "fsc_linear_corr": ([pp, dp, C.c_int64, C.POINTER(C.c_int), C.c_int, dp, vp], C.c_int),
        "fsc_modes_enable": ([vp, C.c_int, C.c_int], C.c_int),
        "fsc_read_modes": ([vp, dp, C.c_int, C.POINTER(C.c_int)], C.c_int),
        "fsc_ens_modes_enable": ([vp, C.c_int, C.c_int], C.c_int),
        "fsc_ens_read_modes": ([vp, C.c_int, dp, C.c_int, C.POINTER(C.c_int)], C.c_int),
        "fsc_linear_sk_radial": ([pp, dp, i64p, C.c_int, vp], C.c_int),
        "fsc_autotune": ([vp], C.c_int),
        "fsc_ens_autotune": ([vp], C.c_int),
        "fsc_get_tiling": ([vp, C.POINTER(C.c_int)], C.c_int),
        "fsc_ens_get_tiling": ([vp, C.POINTER(C.c_int)], C.c_int),
        "fsc_tile_shapes": ([C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.c_int], C.c_int),
        "fsc_set_tiling": ([vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64], C.c_int),
        "fsc_ens_set_tiling": ([vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64], C.c_int),
        "fsc_copy": ([vp, vp, C.c_int64, vp], C.c_int),
        "fsc_philox": ([u32p, u32p, u32p, C.c_int64], C.c_int),
        "fsc_sur_create": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, vp,
                            C.POINTER(vp)],
                           C.c_int),
        "fsc_sur_destroy": ([vp], C.c_int),
        "fsc_sur_last_error": ([vp], C.c_char_p),
        "fsc_sur_nparams": ([vp, i64p], C.c_int),
        "fsc_sur_set_params": ([vp, fp, C.c_int64], C.c_int),
        "fsc_sur_get_params": ([vp, fp, C.c_int64], C.c_int),
        "fsc_sur_set_norm": ([vp, C.c_float, C.c_float, C.c_float], C.c_int),
        "fsc_sur_forward": ([vp, vp, vp, vp, C.c_int], C.c_int),
        "fsc_sur_grad": ([vp, vp, vp, vp, C.c_int, fp, dp], C.c_int),
        "fsc_sur_train_step": ([vp, vp, vp, vp, C.c_int, C.c_float, dp], C.c_int),
        "fsc_sur_rollout": ([vp, vp, vp, C.c_int, C.c_int], C.c_int),
        "fsc_sur_set_fusion": ([vp, C.c_int], C.c_int),
        "fsc_sur_gather": ([vp, vp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                            C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp], C.c_int),
        "fsc_stack_scales": ([vp, C.c_int, C.c_int64, C.c_int, C.c_double, dp, dp, vp], C.c_int),
        "fsc_coarsen": ([vp, C.c_int, vp], C.c_int),
        "fsc_ens_coarsen": ([vp, C.c_int, C.c_int, vp], C.c_int),
        "fsc_field_nbins": ([C.c_int, C.POINTER(C.c_int)], C.c_int),
        "fsc_field_sk": ([vp, C.c_int, C.c_int, C.c_int, vp, dp, dp, C.c_int], C.c_int),
        "fsc_field_sk_noalloc": ([vp, C.c_int, C.c_int, C.c_int, vp, dp, dp, C.c_int], C.c_int),
        "fsc_mfma_probe": ([fp, fp, fp], C.c_int),
        "fsc_normals": ([C.c_int, C.c_int, C.c_uint64, C.c_uint32, i64p, i64p, C.c_int64, dp],
                        C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, errfn=None, handle=None):
    if rc != 0:
        msg = ""
        if errfn is not None:
            m = errfn(handle)
            msg = m.decode() if m else ""
        raise FscError(rc, msg)


def _torch_stream_or(stream):
    """`stream`, or torch's current stream when none is given and torch is in
    use: calls on torch tensors are then ordered with torch's own work."""
    if stream is not None:
        return stream
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_available():
        return torch.cuda.current_stream()
    return None


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):  # torch.cuda.Stream
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _q(D):
    return 9 if D == 2 else 19


class Lattice:
    """One periodic lattice (fsc_ctx)."""

    def __init__(self, p: Params, stream=None, buffers=None):
        L = lib()
        self._h = C.c_void_p()
        if buffers is None:
            rc = L.fsc_create(C.byref(p), _stream_handle(stream), C.byref(self._h))
        else:
            a, b = buffers
            rc = L.fsc_create_external(C.byref(p), _stream_handle(stream), C.c_void_p(a.data_ptr()),
                                       C.c_void_p(b.data_ptr()), C.byref(self._h))
            self._keep = buffers
        _check(rc, L.fsc_last_error, None)
        self.p = Params()
        _check(L.fsc_get_params(self._h, C.byref(self.p)))
        self.D, self.Q = p.D, _q(p.D)
        self.shape = (p.ny, p.nx) if p.D == 2 else (p.nz, p.ny, p.nx)

    def _c(self, rc):
        _check(rc, lib().fsc_last_error, self._h)

    def close(self):
        if self._h:
            lib().fsc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def G(self):
        return self.p.G

    def init_uniform(self):
        self._c(lib().fsc_init_uniform(self._h))

    def autotune(self):
        self._c(lib().fsc_autotune(self._h))

    @property
    def tiling(self):
        out = (C.c_int * 5)()
        self._c(lib().fsc_get_tiling(self._h, out))
        return dict(tx=out[0], ty=out[1], pf=out[2], blocks=out[3], steps=out[4])

    def set_tiling(self, tx: int, ty: int, pf: int, steps: int = 1, target_blocks: int = 2048):
        self._c(lib().fsc_set_tiling(self._h, int(tx), int(ty), int(pf), int(steps), int(target_blocks)))

    def set_populations(self, f: np.ndarray, step: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (self.Q,) + self.shape
        self._c(lib().fsc_set_populations(self._h, _dp(f), int(step)))

    def get_populations(self):
        f = np.empty((self.Q,) + self.shape)
        st = C.c_int64()
        self._c(lib().fsc_get_populations(self._h, _dp(f), C.byref(st)))
        return f

    @property
    def t(self) -> int:
        st = C.c_int64()
        self._c(lib().fsc_get_step(self._h, C.byref(st)))
        return st.value

    def step(self, n: int):
        self._c(lib().fsc_step(self._h, int(n)))

    def run(self, n: int, sk_every: int = 0):
        self._c(lib().fsc_run(self._h, int(n), int(sk_every)))

    def density(self):
        n = np.empty(self.shape)
        self._c(lib().fsc_density(self._h, _dp(n)))
        return n

    def conserved(self, allow_diverged: bool = False):
        """(mass, momentum[D]) of the current state (fsc_conserved)."""
        mass = C.c_double()
        mom = np.zeros(3)
        rc = lib().fsc_conserved(self._h, C.byref(mass), _dp(mom))
        if rc != 0 and not (allow_diverged and rc == -4):
            self._c(rc)
        return mass.value, mom[:self.D].copy()

    def stats(self, allow_diverged: bool = False):
        out = np.empty(8)
        rc = lib().fsc_stats(self._h, _dp(out))
        if rc != 0 and not (allow_diverged and rc == -4):
            self._c(rc)
        return dict(mass=out[0], mom=out[1:1 + self.D].copy(), rho_min=out[4], rho_max=out[5],
                    bad=int(out[6]), nodes=int(out[7]))

    def sk_reset(self):
        self._c(lib().fsc_sk_reset(self._h))

    def modes_enable(self, nm: int, capacity: int):
        """Record the axis-mode amplitudes m = 1..nm at every S(k) sample."""
        self._c(lib().fsc_modes_enable(self._h, int(nm), int(capacity)))
        self._modes_nm = int(nm)

    def read_modes(self):
        """Recorded amplitudes as complex [rows][D][nm]."""
        n = C.c_int()
        self._c(lib().fsc_read_modes(self._h, None, 0, C.byref(n)))
        out = np.zeros((max(n.value, 1), self.D, self._modes_nm, 2))
        self._c(lib().fsc_read_modes(self._h, _dp(out), n.value, C.byref(n)))
        return (out[..., 0] + 1j * out[..., 1])[:n.value]

    def save(self, path: str):
        """Checkpoint: step, populations as stored, S(k) accumulators."""
        self._c(lib().fsc_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        self._c(lib().fsc_load(self._h, os.fsencode(path)))

    def measure_sk(self):
        self._c(lib().fsc_measure_sk(self._h))

    def series_enable(self, capacity: int):
        self._c(lib().fsc_series_enable(self._h, int(capacity)))

    def read_series(self):
        rc, rows = _read_series(lib().fsc_read_series, self._h)
        self._c(rc)
        return _series_dict(rows)

    def coarsen(self, factor: int, out_tensor):
        """Block means into a device float tensor of shape (ny/factor, nx/factor)."""
        self._c(lib().fsc_coarsen(self._h, int(factor), C.c_void_p(out_tensor.data_ptr())))

    def read_sk(self, kind=FSC_SK_AXIS):
        nb = C.c_int()
        self._c(lib().fsc_sk_nbins(self._h, kind, C.byref(nb)))
        s, q = np.zeros(nb.value), np.zeros(nb.value)
        c = np.zeros(nb.value, dtype=np.int64)
        self._c(lib().fsc_read_sk(self._h, kind, _dp(s), _dp(q),
                                  c.ctypes.data_as(C.POINTER(C.c_int64)), nb.value))
        if kind == FSC_SK_AXIS:
            s, q, c = (v.reshape(self.D, -1) for v in (s, q, c))
        return s, q, c


def _read_series(fn, *args):
    n, ln = C.c_int(), C.c_int()
    rc = fn(*args, None, 0, C.byref(n), C.byref(ln))
    if rc != 0:
        return rc, None
    out = np.zeros((max(n.value, 0), ln.value))
    if n.value:
        rc = fn(*args, _dp(out), n.value, C.byref(n), C.byref(ln))
    return rc, out


def _series_dict(rows):
    return dict(step=rows[:, 0].astype(np.int64), L=rows[:, 1], S=rows[:, 2:])


class Ensemble:
    """Many replicas advanced by one launch per step (fsc_ens)."""

    def __init__(self, plist, stream=None):
        L = lib()
        arr = (Params * len(plist))(*plist)
        self._h = C.c_void_p()
        _check(L.fsc_ens_create(arr, len(plist), _stream_handle(stream), C.byref(self._h)),
               L.fsc_ens_last_error, None)
        self.plist = list(plist)
        self.n = len(plist)

    def _c(self, rc):
        _check(rc, lib().fsc_ens_last_error, self._h)

    def close(self):
        if self._h:
            lib().fsc_ens_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self, r):
        p = self.plist[r]
        return (_q(p.D),) + ((p.ny, p.nx) if p.D == 2 else (p.nz, p.ny, p.nx))

    def init_uniform(self):
        self._c(lib().fsc_ens_init_uniform(self._h))

    def autotune(self):
        self._c(lib().fsc_ens_autotune(self._h))

    @property
    def tiling(self):
        out = (C.c_int * 5)()
        self._c(lib().fsc_ens_get_tiling(self._h, out))
        return dict(tx=out[0], ty=out[1], pf=out[2], blocks=out[3], steps=out[4])

    def set_tiling(self, tx: int, ty: int, pf: int, steps: int = 1, target_blocks: int = 2048):
        self._c(lib().fsc_ens_set_tiling(self._h, int(tx), int(ty), int(pf), int(steps),
                                         int(target_blocks)))

    def run(self, n: int, sk_every: int = 0):
        self._c(lib().fsc_ens_run(self._h, int(n), int(sk_every)))

    @property
    def t(self) -> int:
        st = C.c_int64()
        self._c(lib().fsc_ens_get_step(self._h, C.byref(st)))
        return st.value

    def get_populations(self, r: int):
        f = np.empty(self._shape(r))
        self._c(lib().fsc_ens_get_populations(self._h, r, _dp(f)))
        return f

    def set_populations(self, r: int, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == self._shape(r)
        self._c(lib().fsc_ens_set_populations(self._h, r, _dp(f)))

    def stats(self, r: int, allow_diverged: bool = False):
        out = np.empty(8)
        rc = lib().fsc_ens_stats(self._h, r, _dp(out))
        if rc != 0 and not (allow_diverged and rc == -4):
            self._c(rc)
        return dict(mass=out[0], mom=out[1:4].copy(), rho_min=out[4], rho_max=out[5],
                    bad=int(out[6]), nodes=int(out[7]))

    def sk_reset(self):
        self._c(lib().fsc_ens_sk_reset(self._h))

    def density(self, r: int):
        p = self.plist[r]
        shape = (p.ny, p.nx) if p.D == 2 else (p.nz, p.ny, p.nx)
        out = np.empty(shape)
        self._c(lib().fsc_ens_density(self._h, r, _dp(out)))
        return out

    def modes_enable(self, nm: int, capacity: int):
        """Record the axis-mode amplitudes m = 1..nm of every replica at every sample."""
        self._c(lib().fsc_ens_modes_enable(self._h, int(nm), int(capacity)))
        self._modes_nm = int(nm)

    def read_modes(self, r: int):
        """Recorded amplitudes of replica r as complex [rows][D][nm]."""
        n = C.c_int()
        self._c(lib().fsc_ens_read_modes(self._h, r, None, 0, C.byref(n)))
        D = self.plist[r].D
        out = np.zeros((max(n.value, 1), D, self._modes_nm, 2))
        self._c(lib().fsc_ens_read_modes(self._h, r, _dp(out), n.value, C.byref(n)))
        return (out[..., 0] + 1j * out[..., 1])[:n.value]

    def save(self, path: str):
        """Checkpoint of every replica (see fsc_ens_save)."""
        self._c(lib().fsc_ens_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        self._c(lib().fsc_ens_load(self._h, os.fsencode(path)))

    def series_enable(self, capacity: int):
        self._c(lib().fsc_ens_series_enable(self._h, int(capacity)))

    def read_series(self, r: int):
        rc, rows = _read_series(lib().fsc_ens_read_series, self._h, r)
        self._c(rc)
        return _series_dict(rows)

    def coarsen(self, r: int, factor: int, out_tensor):
        self._c(lib().fsc_ens_coarsen(self._h, r, int(factor), C.c_void_p(out_tensor.data_ptr())))

    def read_sk(self, r: int, kind=FSC_SK_AXIS):
        nb = C.c_int()
        self._c(lib().fsc_ens_sk_nbins(self._h, r, kind, C.byref(nb)))
        s, q = np.zeros(nb.value), np.zeros(nb.value)
        c = np.zeros(nb.value, dtype=np.int64)
        self._c(lib().fsc_ens_read_sk(self._h, r, kind, _dp(s), _dp(q),
                                      c.ctypes.data_as(C.POINTER(C.c_int64)), nb.value))
        if kind == FSC_SK_AXIS:
            D = self.plist[r].D
            s, q, c = (v.reshape(D, -1) for v in (s, q, c))
        return s, q, c


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Surrogate:
    """The learned coarse-grained surrogate (fsc_sur).  Device fields are
    passed as objects with data_ptr() (torch tensors) or raw pointers; `prev`
    (the field one stride earlier) is used by two-channel networks only.  The
    calls run on `stream`, by default torch's current stream at creation."""

    def __init__(self, layers: int, H: int, W: int, max_batch: int, seed: int = 0, stream=None,
                 in_ch: int = 2):
        L = lib()
        self._h = C.c_void_p()
        _check(L.fsc_sur_create(layers, in_ch, H, W, max_batch, C.c_uint64(seed),
                                _stream_handle(_torch_stream_or(stream)), C.byref(self._h)),
               L.fsc_sur_last_error, None)
        n = C.c_int64()
        self._c(L.fsc_sur_nparams(self._h, C.byref(n)))
        self.nparams = n.value
        self.layers, self.in_ch, self.H, self.W = layers, in_ch, H, W

    def _c(self, rc):
        _check(rc, lib().fsc_sur_last_error, self._h)

    def close(self):
        if self._h:
            lib().fsc_sur_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptr(x):
        if x is None:
            return None
        return C.c_void_p(x.data_ptr() if hasattr(x, "data_ptr") else int(x))

    def get_params(self):
        out = np.zeros(self.nparams, dtype=np.float32)
        self._c(lib().fsc_sur_get_params(self._h, _fp(out), self.nparams))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        self._c(lib().fsc_sur_set_params(self._h, _fp(p), self.nparams))

    def set_norm(self, mean: float, in_scale: float, out_scale: float):
        self._c(lib().fsc_sur_set_norm(self._h, mean, in_scale, out_scale))

    def set_fusion(self, mode: int):
        """Pairs of 32 -> 32 layers in one launch at inference: 0 never, 1
        always, 2 small batches (the default); bit-identical either way (see
        fsc_sur_set_fusion)."""
        self._c(lib().fsc_sur_set_fusion(self._h, int(mode)))

    def forward(self, prev, x, out, batch: int):
        self._c(lib().fsc_sur_forward(self._h, self._ptr(prev), self._ptr(x), self._ptr(out),
                                      int(batch)))

    def grad(self, prev, x, target, batch: int):
        g = np.zeros(self.nparams, dtype=np.float32)
        loss = C.c_double()
        self._c(lib().fsc_sur_grad(self._h, self._ptr(prev), self._ptr(x), self._ptr(target),
                                   int(batch), _fp(g), C.byref(loss)))
        return loss.value, g

    def train_step(self, prev, x, target, batch: int, lr: float, want_loss: bool = True):
        loss = C.c_double()
        self._c(lib().fsc_sur_train_step(self._h, self._ptr(prev), self._ptr(x), self._ptr(target),
                                         int(batch), float(lr),
                                         C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def rollout(self, prev, traj, batch: int, passes: int):
        """`passes` forward passes replayed from a captured graph: traj
        [passes + 1][batch][H][W] with traj[0] the start (see fsc_sur_rollout)."""
        self._c(lib().fsc_sur_rollout(self._h, self._ptr(prev), self._ptr(traj), int(batch),
                                      int(passes)))

    def gather(self, snaps, t_idx, r_idx, dt: int, shift, transpose: bool, out):
        """Batch of snapshot images with a periodic shift and an optional
        transpose (see fsc_sur_gather); snaps is a device tensor [K][R][H][W]."""
        t = np.ascontiguousarray(t_idx, dtype=np.int32)
        r = np.ascontiguousarray(r_idx, dtype=np.int32)
        K, R = int(snaps.shape[0]), int(snaps.shape[1])
        ip = C.POINTER(C.c_int)
        self._c(lib().fsc_sur_gather(self._h, self._ptr(snaps), K, R, t.ctypes.data_as(ip),
                                     r.ctypes.data_as(ip), int(t.size), int(dt), int(shift[0]),
                                     int(shift[1]), int(bool(transpose)), self._ptr(out)))


def stack_scales(snaps, t_first: int, centre: float = 1.0, stream=None):
    """(input std, increment std) of a device snapshot stack [K][...] in FP64
    (see fsc_stack_scales)."""
    K = int(snaps.shape[0])
    per = int(np.prod(snaps.shape[1:]))
    a, b = C.c_double(), C.c_double()
    ptr = C.c_void_p(snaps.data_ptr())
    _check(lib().fsc_stack_scales(ptr, K, per, int(t_first), float(centre), C.byref(a), C.byref(b),
                                  _stream_handle(_torch_stream_or(stream))))
    return a.value, b.value


def field_sk(fields, batch: int, n: int, stream=None, noalloc: bool = False):
    """Radial shell means of S(k) and L for device float fields [batch][n][n].

    noalloc=True calls fsc_field_sk_noalloc (fixed-size library scratch, no
    device allocation; sides up to 1024)."""
    nb = C.c_int()
    _check(lib().fsc_field_nbins(n, C.byref(nb)))
    shells = np.zeros((batch, nb.value))
    L = np.zeros(batch)
    ptr = C.c_void_p(fields.data_ptr() if hasattr(fields, "data_ptr") else int(fields))
    fn = lib().fsc_field_sk_noalloc if noalloc else lib().fsc_field_sk
    _check(fn(ptr, batch, n, n, _stream_handle(_torch_stream_or(stream)), _dp(shells), _dp(L),
              nb.value))
    return shells, L


def tile_shapes(D: int, stencil: int, precision: str = "fp32"):
    """Compiled (tile x, tile y, prefetch depth, steps per launch) tilings of a
    lattice kind; the first is the default."""
    prec = {"fp32": FSC_FP32_SHIFTED, "fp64": FSC_FP64}[precision] if isinstance(precision, str) \
        else int(precision)
    out = (C.c_int * 128)()
    n = lib().fsc_tile_shapes(int(D), int(stencil), prec, out, 32)
    if n < 0:
        raise FscError(n, "unsupported lattice kind")
    return [tuple(out[4 * i:4 * i + 4]) for i in range(min(n, 32))]


def linear_sk(p: Params, kvecs) -> np.ndarray:
    """Exact stationary S(k) of the linearised step at wave vectors [nk][D]."""
    k = np.ascontiguousarray(kvecs, dtype=np.float64).reshape(-1, p.D)
    out = np.zeros(k.shape[0])
    _check(lib().fsc_linear_sk(C.byref(p), _dp(k), k.shape[0], _dp(out), None))
    return out


def linear_sk_radial(p: Params, nbins: int):
    """Shell means of the exact linear S(k) over the lattice's wave vectors,
    binned like the radial structure-factor bins; returns (mean, modes)."""
    mean = np.zeros(nbins)
    cnt = np.zeros(nbins, dtype=np.int64)
    _check(lib().fsc_linear_sk_radial(C.byref(p), _dp(mean), cnt.ctypes.data_as(C.POINTER(C.c_int64)),
                                      nbins, None))
    return mean, cnt


def linear_corr(p: Params, kvecs, lags) -> np.ndarray:
    """Exact C(k, tau) of the linearised step, complex [nk][nlag]."""
    k = np.ascontiguousarray(kvecs, dtype=np.float64).reshape(-1, p.D)
    lg = np.ascontiguousarray(lags, dtype=np.int32)
    out = np.zeros((k.shape[0], len(lg), 2))
    _check(lib().fsc_linear_corr(C.byref(p), _dp(k), k.shape[0],
                                 lg.ctypes.data_as(C.POINTER(C.c_int)), len(lg), _dp(out), None))
    return out[..., 0] + 1j * out[..., 1]


def mfma_probe(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    Cm = np.zeros((16, 16), dtype=np.float32)
    _check(lib().fsc_mfma_probe(_fp(A), _fp(B), _fp(Cm)))
    return Cm


def device_copy(src_ptr: int, dst_ptr: int, nbytes: int, stream=None):
    """Plain device copy (diagnostic; asynchronous on `stream`)."""
    _check(lib().fsc_copy(C.c_void_p(src_ptr), C.c_void_p(dst_ptr), int(nbytes),
                          _stream_handle(stream)))


def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    n = ctr.shape[0]
    out = np.zeros((n, 4), dtype=np.uint32)
    u32p = C.POINTER(C.c_uint32)
    _check(lib().fsc_philox(ctr.ctypes.data_as(u32p), key.ctypes.data_as(u32p),
                            out.ctypes.data_as(u32p), n))
    return out


def normals(D: int, precision: str, seed: int, replica: int, nodes, steps) -> np.ndarray:
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    steps = np.ascontiguousarray(steps, dtype=np.int64)
    n = nodes.size
    nn = 6 if D == 2 else 15
    out = np.zeros((n, nn))
    prec = {"fp32": 0, "fp64": 1}[precision]
    i64p = C.POINTER(C.c_int64)
    _check(lib().fsc_normals(D, prec, C.c_uint64(seed), C.c_uint32(replica),
                             nodes.ctypes.data_as(i64p), steps.ctypes.data_as(i64p), n, _dp(out)))
    return out
