"""Shared test workloads: parameter dictionaries turned into oracle or HIP-path
parameter objects, and the seeded initial densities (from the input module).
Holds none of the method's arithmetic."""
from __future__ import annotations

import os

import numpy as np

import oracle as O
from paper_1512_01977_amd import inputs

_TC = {}


def cs_tc(a=1.0, b=4.0, R=1.0):
    key = (a, b, R)
    if key not in _TC:
        _TC[key] = O.critical(O.Params(nz=4, nr=4, eos=O.EOS_CS, eos_a=a, eos_b=b, eos_R=R))[1]
    return _TC[key]


def base(nz, nr, **kw):
    d = dict(nz=nz, nr=nr, tau=1.0, eos=O.EOS_CS, T=0.8 * cs_tc(), eos_a=1.0, eos_b=4.0,
             eos_R=1.0, lam=1.0, A=0.0, axisym=1, faxis_sound=0, bc_top=0, gz=0.0, forcing=0)
    d.update(kw)
    return d


def oracle_params(d) -> O.Params:
    return O.Params(**d)


def gpu_params(d):
    from paper_1512_01977_amd import lbm
    return lbm.Params(**d)


def oparams(p) -> O.Params:
    """The oracle's parameter object for a binding Params (the same fields)."""
    return O.Params(nz=p.nz, nr=p.nr, tau=p.tau, eos=p.eos, T=p.T, eos_a=p.eos_a, eos_b=p.eos_b,
                    eos_R=p.eos_R, lam=p.lam, A=p.A, axisym=p.axisym, faxis_sound=p.faxis_sound,
                    bc_top=p.bc_top, gz=p.gz, forcing=p.forcing, source_mid=p.source_mid)


class OracleEOS:
    """Critical point and Maxwell densities from the oracle: the EOS helper of the named
    workloads in tests that compare with the oracle, so that none of its inputs comes from
    the library."""

    @staticmethod
    def critical(p):
        return O.critical(oparams(p))

    @staticmethod
    def coexistence(p):
        return O.coexistence(oparams(p))


def droplet_rho(d, radius, eps=0.0, noise=1e-4, seed=1, width=5.0, zc=None):
    if d["eos"] == O.EOS_IDEAL:
        r = inputs.radial_wave(d["nz"], d["nr"], 1.0, amplitude=0.05, wavelength=d["nr"] / 1.5,
                               noise=noise, seed=seed)
        return r
    rv, rl, _ = O.coexistence(oracle_params(d))
    return inputs.droplet(d["nz"], d["nr"], rv, rl, radius, zc=zc, width=width, eps=eps,
                          noise=noise, seed=seed)


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_table1():
    """Table 1 (Sec. 3.1) as printed: {(T, A): (sigma_2D, sigma_axis)}."""
    out = {}
    with open(os.path.join(GOLDEN, "table1_surface_tension.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                T, A, s2, sa = map(float, line)
                out[(T, A)] = (s2, sa)
    return out
