"""CPU oracle of the axisymmetric multiphase LBM step (arXiv:1512.01977).

TEST INFRASTRUCTURE ONLY.  A plain FP64 C implementation (lbm_oracle.c)
behind ctypes.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the HIP library never does, and this
package never imports the HIP library.

Grid and direction conventions are those of lbm_oracle.h: node fields are
numpy arrays of shape (nr, nz), the distribution has shape (9, nr, nz).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")

EOS_IDEAL, EOS_VDW, EOS_CS = 0, 1, 2
TOP_FREE_SLIP, TOP_NO_SLIP = 0, 1
FORCING_EDM, FORCING_GUO = 0, 1

# D2Q9 set as numbered in lbm_oracle.h (c_z, c_r), Sec. 2.1.
CZ = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CR = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WEIGHTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        names = {-1: "bad argument", -4: "EOS domain left (psi not real)", -5: "non-finite value"}
        super().__init__(f"{where}: oracle status {code} ({names.get(code, 'unknown')})")
        self.code = code


class _Params(ctypes.Structure):
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
        ("hr_printed_sign", ctypes.c_int32),
        ("gz", ctypes.c_double),
        ("forcing", ctypes.c_int32),
        ("source_mid", ctypes.c_int32),
    ]


@dataclass
class Params:
    """Parameters of one oracle run (see lbm_oracle.h)."""
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
    hr_printed_sign: int = 0
    gz: float = 0.0
    forcing: int = 0
    source_mid: int = 0

    def c(self) -> _Params:
        return _Params(self.nz, self.nr, self.tau, self.eos, self.T, self.eos_a, self.eos_b,
                       self.eos_R, self.lam, self.A, self.axisym, self.faxis_sound, self.bc_top,
                       self.hr_printed_sign, self.gz, self.forcing, self.source_mid)


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Params)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbm_oracle_eos.argtypes = [P, ctypes.c_double, dp, dp, dp]
        L.lbm_oracle_critical.argtypes = [P, dp, dp, dp]
        L.lbm_oracle_coexistence.argtypes = [P, dp, dp, dp]
        L.lbm_oracle_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
        L.lbm_oracle_equilibrium.restype = None
        L.lbm_oracle_derivative.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_double, dp]
        L.lbm_oracle_force_psi.argtypes = [P, dp, dp, dp, dp]
        L.lbm_oracle_source.argtypes = [P] + [ctypes.c_double] * 7 + [dp]
        L.lbm_oracle_source.restype = None
        L.lbm_oracle_source_field.argtypes = [P, dp, dp, dp, dp]
        L.lbm_oracle_guo_source.argtypes = [ctypes.c_double] * 5 + [dp]
        L.lbm_oracle_guo_source.restype = None
        L.lbm_oracle_threads.argtypes = []
        L.lbm_oracle_set_threads.argtypes = [ctypes.c_int]
        L.lbm_oracle_set_threads.restype = None
        L.lbm_oracle_init.argtypes = [P, dp, dp, dp, dp]
        L.lbm_oracle_step.argtypes = [P, dp, ctypes.c_int64]
        L.lbm_oracle_moments.argtypes = [P, dp, dp, dp, dp]
        L.lbm_oracle_mass.argtypes = [P, dp, dp]
        L.lbm_oracle_laplace.argtypes = [P, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, dp]
        L.lbm_oracle_axis_interface.argtypes = [P, dp, ctypes.c_double, ctypes.c_double, dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(code: int, where: str):
    if code != 0:
        raise OracleError(code, where)


def eos(p: Params, rho: float):
    """(P_k, kappa = dP_k/drho, psi) at density rho."""
    P, k, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lbm_oracle_eos(ctypes.byref(p.c()), rho, ctypes.byref(P), ctypes.byref(k),
                                ctypes.byref(s)), "eos")
    return P.value, k.value, s.value


def critical(p: Params):
    """(rho_c, T_c, P_c) of the EOS in p."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lbm_oracle_critical(ctypes.byref(p.c()), ctypes.byref(a), ctypes.byref(b),
                                     ctypes.byref(c)), "critical")
    return a.value, b.value, c.value


def coexistence(p: Params):
    """Maxwell (rho_v, rho_l, P_sat) at p.T."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().lbm_oracle_coexistence(ctypes.byref(p.c()), ctypes.byref(a), ctypes.byref(b),
                                        ctypes.byref(c)), "coexistence")
    return a.value, b.value, c.value


def equilibrium(rho: float, uz: float, ur: float) -> np.ndarray:
    out = np.zeros(9)
    lib().lbm_oracle_equilibrium(rho, uz, ur, _ptr(out))
    return out


def derivative(g: np.ndarray, axis: int, par_axis: float = 1.0, par_top: float = 1.0):
    g = np.ascontiguousarray(g, dtype=np.float64)
    nr, nz = g.shape
    out = np.zeros_like(g)
    _check(lib().lbm_oracle_derivative(_ptr(g), nz, nr, axis, par_axis, par_top, _ptr(out)),
           "derivative")
    return out


def force_psi(p: Params, psi: np.ndarray, kappa: np.ndarray | None = None):
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    kap = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    Fz, Fr = np.zeros_like(psi), np.zeros_like(psi)
    _check(lib().lbm_oracle_force_psi(ctypes.byref(p.c()), _ptr(psi), _ptr(kap), _ptr(Fz),
                                      _ptr(Fr)), "force_psi")
    return Fz, Fr


def source(p: Params, r, rho, uz, ur, dr_uz, dz_ur, dr_ur) -> np.ndarray:
    h = np.zeros(9)
    lib().lbm_oracle_source(ctypes.byref(p.c()), r, rho, uz, ur, dr_uz, dz_ur, dr_ur, _ptr(h))
    return h


def source_field(p: Params, rho: np.ndarray, uz: np.ndarray, ur: np.ndarray) -> np.ndarray:
    """h_i of every node as (9, nr, nz) from node fields rho, u (physical velocity): at the
    node, or with p.source_mid = 1 the mean over each link's two ends (Sec. 2.2)."""
    rho, uz, ur = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, uz, ur))
    assert rho.shape == uz.shape == ur.shape == (p.nr, p.nz)
    h = np.zeros((9, p.nr, p.nz))
    _check(lib().lbm_oracle_source_field(ctypes.byref(p.c()), _ptr(rho), _ptr(uz), _ptr(ur), _ptr(h)),
           "source_field")
    return h


def threads() -> int:
    """Host threads of the oracle's parallel loops."""
    return int(lib().lbm_oracle_threads())


def set_threads(n: int) -> None:
    """Host threads for the oracle's parallel loops from now on."""
    lib().lbm_oracle_set_threads(int(n))


def guo_source(tau, uz, ur, Fz, Fr) -> np.ndarray:
    """Guo's S_i of Sec. 2.1 at one node."""
    S = np.zeros(9)
    lib().lbm_oracle_guo_source(tau, uz, ur, Fz, Fr, _ptr(S))
    return S


def init(p: Params, rho0: np.ndarray, uz0=None, ur0=None) -> np.ndarray:
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    assert rho0.shape == (p.nr, p.nz)
    uz0 = None if uz0 is None else np.ascontiguousarray(uz0, dtype=np.float64)
    ur0 = None if ur0 is None else np.ascontiguousarray(ur0, dtype=np.float64)
    f = np.zeros((9, p.nr, p.nz))
    _check(lib().lbm_oracle_init(ctypes.byref(p.c()), _ptr(rho0), _ptr(uz0), _ptr(ur0), _ptr(f)),
           "init")
    return f


def step(p: Params, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance f (shape (9, nr, nz)) in place by nsteps; returns f."""
    assert f.shape == (9, p.nr, p.nz) and f.dtype == np.float64 and f.flags.c_contiguous
    _check(lib().lbm_oracle_step(ctypes.byref(p.c()), _ptr(f), nsteps), "step")
    return f


def moments(p: Params, f: np.ndarray):
    """(rho, u_z, u_r) with the physical velocity u = (j + F/2)/rho."""
    rho, uz, ur = (np.zeros((p.nr, p.nz)) for _ in range(3))
    _check(lib().lbm_oracle_moments(ctypes.byref(p.c()), _ptr(f), _ptr(rho), _ptr(uz), _ptr(ur)),
           "moments")
    return rho, uz, ur


def mass(p: Params, f: np.ndarray) -> float:
    m = ctypes.c_double()
    _check(lib().lbm_oracle_mass(ctypes.byref(p.c()), _ptr(f), ctypes.byref(m)), "mass")
    return m.value


def laplace(p: Params, f: np.ndarray, zc: float, r_in: float, r_out: float) -> float:
    d = ctypes.c_double()
    _check(lib().lbm_oracle_laplace(ctypes.byref(p.c()), _ptr(f), zc, r_in, r_out,
                                    ctypes.byref(d)), "laplace")
    return d.value


def axis_interface(p: Params, f: np.ndarray, zc: float, thr: float) -> float:
    """Where rho on the axis row first falls to thr going +z from floor(zc) (Sec. 3.2)."""
    z = ctypes.c_double()
    _check(lib().lbm_oracle_axis_interface(ctypes.byref(p.c()), _ptr(f), zc, thr, ctypes.byref(z)),
           "axis_interface")
    return z.value
