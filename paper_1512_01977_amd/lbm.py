"""Python binding of liblbm_axi.so (the C ABI in include/lbm_axi.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  The functions keep the C names; `LbmAxi` wraps a handle.  PyTorch is
used for device memory (the distribution buffers are a torch allocation handed
to the library as a workspace) and for the caller's current stream.

There is no fallback: if the library is missing or no GPU is present, the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_axi.so")

LBM_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "allocation failed", -3: "HIP runtime error",
          -4: "EOS domain left", -5: "non-finite value", -6: "unsupported"}
EOS_IDEAL, EOS_VDW, EOS_CS = 0, 1, 2
TOP_FREE_SLIP, TOP_NO_SLIP = 0, 1
PREC_FP64, PREC_FP32 = 0, 1
FORCING_EDM, FORCING_GUO = 0, 1

# Exported names, in the order include/lbm_axi.h declares them.
EXPORTS = [
    "lbm_axi_status_string", "lbm_axi_eos_critical", "lbm_axi_eos_coexistence", "lbm_axi_init",
    "lbm_axi_batch_init", "lbm_axi_workspace_bytes", "lbm_axi_batch_init_ws", "lbm_axi_destroy",
    "lbm_axi_step", "lbm_axi_step_timed", "lbm_axi_sync", "lbm_axi_errors",
    "lbm_axi_set_graph_chunk",
    "lbm_axi_moments", "lbm_axi_mass", "lbm_axi_mass_async", "lbm_axi_laplace", "lbm_axi_axis_interface",
    "lbm_axi_get_f", "lbm_axi_set_f",
    "lbm_axi_get_launch", "lbm_axi_set_launch", "lbm_axi_autotune", "lbm_axi_stream_copy",
    "lbm_axi_sizes",
]


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: status {code} ({STATUS.get(code, 'unknown')})")
        self.code = code


class lbm_axi_params(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32), ("nr", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("eos", ctypes.c_int32),
        ("T", ctypes.c_double),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double), ("eos_R", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("A", ctypes.c_double),
        ("axisym", ctypes.c_int32),
        ("faxis_sound", ctypes.c_int32),
        ("bc_top", ctypes.c_int32),
        ("gz", ctypes.c_double),
        ("forcing", ctypes.c_int32),
        ("source_mid", ctypes.c_int32),
    ]


class lbm_axi_launch(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("seg_rows", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("xcd_swizzle", ctypes.c_int32), ("regf", ctypes.c_int32),
                ("streams", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


@dataclass
class Params:
    """One instance (fields as in lbm_axi_params)."""
    nz: int
    nr: int
    tau: float = 1.0
    eos: int = EOS_CS
    T: float = 0.0
    eos_a: float = 1.0
    eos_b: float = 4.0
    eos_R: float = 1.0
    lam: float = 1.0
    A: float = 0.0
    axisym: int = 1
    faxis_sound: int = 0
    bc_top: int = TOP_FREE_SLIP
    gz: float = 0.0
    forcing: int = 0
    source_mid: int = 0

    def c(self) -> lbm_axi_params:
        return lbm_axi_params(self.nz, self.nr, self.tau, self.eos, self.T, self.eos_a, self.eos_b,
                              self.eos_R, self.lam, self.A, self.axisym, self.faxis_sound,
                              self.bc_top, self.gz, self.forcing, self.source_mid)


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_H = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime: load it first so that the library binds to the
        # same runtime instead of pulling a second copy into the process.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1512_01977_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(lbm_axi_params)
        LP = ctypes.POINTER(lbm_axi_launch)
        L.lbm_axi_status_string.restype = ctypes.c_char_p
        L.lbm_axi_status_string.argtypes = [ctypes.c_int32]
        L.lbm_axi_eos_critical.argtypes = [P, _dp, _dp, _dp]
        L.lbm_axi_eos_coexistence.argtypes = [P, _dp, _dp, _dp]
        L.lbm_axi_init.argtypes = [P, ctypes.c_int32, _dp, _dp, _dp, ctypes.c_void_p,
                                   ctypes.POINTER(_H)]
        L.lbm_axi_batch_init.argtypes = [ctypes.c_int32, P, ctypes.c_int32,
                                         ctypes.POINTER(_dp), ctypes.c_void_p, ctypes.POINTER(_H)]
        L.lbm_axi_workspace_bytes.argtypes = [ctypes.c_int32, P, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_size_t)]
        L.lbm_axi_batch_init_ws.argtypes = [ctypes.c_int32, P, ctypes.c_int32, ctypes.POINTER(_dp),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.POINTER(_H)]
        L.lbm_axi_destroy.argtypes = [_H]
        L.lbm_axi_destroy.restype = None
        L.lbm_axi_step.argtypes = [_H, ctypes.c_int64]
        L.lbm_axi_step_timed.argtypes = [_H, ctypes.c_int64, _dp]
        L.lbm_axi_sync.argtypes = [_H]
        L.lbm_axi_errors.argtypes = [_H, ctypes.POINTER(ctypes.c_int32)]
        L.lbm_axi_set_graph_chunk.argtypes = [_H, ctypes.c_int32]
        L.lbm_axi_moments.argtypes = [_H, ctypes.c_int32, _dp, _dp, _dp]
        L.lbm_axi_mass.argtypes = [_H, _dp]
        L.lbm_axi_mass_async.argtypes = [_H, ctypes.c_void_p]
        L.lbm_axi_laplace.argtypes = [_H, _dp, _dp, _dp, _dp]
        L.lbm_axi_axis_interface.argtypes = [_H, _dp, _dp, _dp]
        L.lbm_axi_get_f.argtypes = [_H, ctypes.c_int32, _dp]
        L.lbm_axi_set_f.argtypes = [_H, ctypes.c_int32, _dp]
        L.lbm_axi_get_launch.argtypes = [_H, LP]
        L.lbm_axi_set_launch.argtypes = [_H, LP]
        L.lbm_axi_autotune.argtypes = [_H, ctypes.c_int32, LP, _dp]
        L.lbm_axi_stream_copy.argtypes = [ctypes.c_int64, ctypes.c_int32, _dp]
        L.lbm_axi_sizes.argtypes = [_H, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        for name in EXPORTS:
            if name not in ("lbm_axi_status_string", "lbm_axi_destroy"):
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(code: int, where: str):
    if code != LBM_OK:
        raise LbmError(code, where)


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def lbm_axi_eos_critical(p: Params):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lbm_axi_eos_critical(ctypes.byref(p.c()), ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(c)), "lbm_axi_eos_critical")
    return a.value, b.value, c.value


def lbm_axi_eos_coexistence(p: Params):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lbm_axi_eos_coexistence(ctypes.byref(p.c()), ctypes.byref(a), ctypes.byref(b),
                                         ctypes.byref(c)), "lbm_axi_eos_coexistence")
    return a.value, b.value, c.value


def lbm_axi_stream_copy(nbytes: int, iters: int = 10) -> float:
    """Device-to-device copy rate in GB/s (read + write) of a plain streaming kernel."""
    g = ctypes.c_double()
    _check(lib().lbm_axi_stream_copy(int(nbytes), int(iters), ctypes.byref(g)), "lbm_axi_stream_copy")
    return g.value


def _current_stream():
    import torch
    s = torch.cuda.current_stream().cuda_stream
    return s if s else None


class LbmAxi:
    """A handle of n instances advanced together (n = 1 for a single domain)."""

    def __init__(self, params, rho0, precision: int = PREC_FP64, uz0=None, ur0=None,
                 stream=None, torch_workspace: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs an MI355X")
        single = isinstance(params, Params)
        plist = [params] if single else list(params)
        rlist = [rho0] if single else list(rho0)
        if len(plist) != len(rlist):
            raise ValueError("one rho0 per instance")
        self.params = plist
        self.precision = precision
        n = len(plist)
        carr = (lbm_axi_params * n)(*[p.c() for p in plist])
        self._rho0 = [_f64(r) for r in rlist]
        for p, r in zip(plist, self._rho0):
            if r.shape != (p.nr, p.nz):
                raise ValueError(f"rho0 must have shape (nr, nz) = {(p.nr, p.nz)}, got {r.shape}")
        ptrs = (_dp * n)(*[_ptr(r) for r in self._rho0])
        h = _H()
        st = stream if stream is not None else _current_stream()
        self._ws = None
        L = lib()
        if single and (uz0 is not None or ur0 is not None):
            uz, ur = _f64(uz0), _f64(ur0)
            _check(L.lbm_axi_init(ctypes.byref(carr[0]), precision, ptrs[0], _ptr(uz), _ptr(ur),
                                  st, ctypes.byref(h)), "lbm_axi_init")
        elif torch_workspace:
            nb = ctypes.c_size_t()
            _check(L.lbm_axi_workspace_bytes(n, carr, precision, ctypes.byref(nb)),
                   "lbm_axi_workspace_bytes")
            self._ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            _check(L.lbm_axi_batch_init_ws(n, carr, precision, ptrs, st, self._ws.data_ptr(),
                                           nb.value, ctypes.byref(h)), "lbm_axi_batch_init_ws")
        else:
            _check(L.lbm_axi_batch_init(n, carr, precision, ptrs, st, ctypes.byref(h)),
                   "lbm_axi_batch_init")
        self.h = h
        self.n = n

    # -- lifetime
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().lbm_axi_destroy(self.h)
            self.h = _H()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- stepping
    def step(self, nsteps: int):
        _check(lib().lbm_axi_step(self.h, int(nsteps)), "lbm_axi_step")

    def step_timed(self, nsteps: int) -> float:
        ms = ctypes.c_double()
        _check(lib().lbm_axi_step_timed(self.h, int(nsteps), ctypes.byref(ms)), "lbm_axi_step_timed")
        return ms.value

    def sync(self):
        _check(lib().lbm_axi_sync(self.h), "lbm_axi_sync")

    def errors(self) -> np.ndarray:
        """Per-instance device error bits (1: EOS domain left, 2: non-finite; 0: clean)."""
        out = np.zeros(self.n, dtype=np.int32)
        _check(lib().lbm_axi_errors(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
               "lbm_axi_errors")
        return out

    def set_graph_chunk(self, chunk: int):
        _check(lib().lbm_axi_set_graph_chunk(self.h, int(chunk)), "lbm_axi_set_graph_chunk")

    # -- observables
    def moments(self, k: int = 0):
        p = self.params[k]
        rho, uz, ur = (np.empty((p.nr, p.nz)) for _ in range(3))
        _check(lib().lbm_axi_moments(self.h, k, _ptr(rho), _ptr(uz), _ptr(ur)), "lbm_axi_moments")
        return rho, uz, ur

    def mass(self) -> np.ndarray:
        m = np.empty(self.n)
        _check(lib().lbm_axi_mass(self.h, _ptr(m)), "lbm_axi_mass")
        return m

    def mass_async(self, out) -> None:
        """lbm_axi_mass_async: the masses into `out`, a float64 CUDA tensor of n elements on the
        handle's device; enqueued on the handle's stream, nothing allocated, no synchronisation."""
        import torch
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
                and out.numel() >= self.n and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 CUDA tensor of n elements")
        _check(lib().lbm_axi_mass_async(self.h, ctypes.c_void_p(out.data_ptr())), "lbm_axi_mass_async")

    def laplace(self, zc, r_in, r_out) -> np.ndarray:
        zc, r_in, r_out = (np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64),
                                                                (self.n,))) for v in (zc, r_in, r_out))
        dp = np.empty(self.n)
        _check(lib().lbm_axi_laplace(self.h, _ptr(zc), _ptr(r_in), _ptr(r_out), _ptr(dp)),
               "lbm_axi_laplace")
        return dp

    def axis_interface(self, zc, thr) -> np.ndarray:
        """Per instance, where rho on the axis row first falls to thr going +z from
        floor(zc) (the drop's interface on the symmetry axis, Sec. 3.2)."""
        zc, thr = (np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (self.n,)))
                   for v in (zc, thr))
        z = np.empty(self.n)
        _check(lib().lbm_axi_axis_interface(self.h, _ptr(zc), _ptr(thr), _ptr(z)), "lbm_axi_axis_interface")
        return z

    def get_f(self, k: int = 0) -> np.ndarray:
        p = self.params[k]
        f = np.empty((9, p.nr, p.nz))
        _check(lib().lbm_axi_get_f(self.h, k, _ptr(f)), "lbm_axi_get_f")
        return f

    def set_f(self, f, k: int = 0):
        p = self.params[k]
        f = _f64(f)
        if f.shape != (9, p.nr, p.nz):
            raise ValueError("f must have shape (9, nr, nz)")
        _check(lib().lbm_axi_set_f(self.h, k, _ptr(f)), "lbm_axi_set_f")

    # -- launch shape
    def get_launch(self) -> dict:
        c = lbm_axi_launch()
        _check(lib().lbm_axi_get_launch(self.h, ctypes.byref(c)), "lbm_axi_get_launch")
        return c.as_dict()

    def set_launch(self, **kw):
        c = lbm_axi_launch()
        _check(lib().lbm_axi_get_launch(self.h, ctypes.byref(c)), "lbm_axi_get_launch")
        for k, v in kw.items():
            setattr(c, k, int(v))
        _check(lib().lbm_axi_set_launch(self.h, ctypes.byref(c)), "lbm_axi_set_launch")

    def autotune(self, steps_per_trial: int = 3):
        c = lbm_axi_launch()
        ms = ctypes.c_double()
        _check(lib().lbm_axi_autotune(self.h, int(steps_per_trial), ctypes.byref(c),
                                      ctypes.byref(ms)), "lbm_axi_autotune")
        return c.as_dict(), ms.value

    def sizes(self):
        n, nodes, fb = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lbm_axi_sizes(self.h, ctypes.byref(n), ctypes.byref(nodes), ctypes.byref(fb)),
               "lbm_axi_sizes")
        return n.value, nodes.value, fb.value
