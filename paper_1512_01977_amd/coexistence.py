"""Coexistence densities of the scheme and calibration of the mixing parameter A
(Sec. 2.3; the flat-interface set-up of Fig. 2).

A planar liquid layer across the periodic z direction (uniform in r, so that F_axis
and the source h_i vanish) relaxes to the scheme's own coexistence densities.  With
the exact-difference force these depend on Kupershtokh's A (eq. kupershtokhforcing):
A = 0 puts the vapour branch below the Maxwell construction, and a suitable negative
A brings it back (the paper's -0.152 for the reduced van der Waals EOS).  `measure`
runs any set of cases as one batched launch of the HIP path and returns the bulk
densities; `fit_a` scans A over a temperature range and returns the A at which the
vapour branch sits on the Maxwell densities.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

from . import inputs
from .lbm import PREC_FP64, LbmAxi, LbmError, Params, lbm_axi_eos_coexistence, lbm_axi_eos_critical


@dataclass
class Coexistence:
    """Bulk densities of one flat-interface run next to the Maxwell values."""
    params: Params
    rho_v: float          # measured vapour density (nan if the run left the EOS domain)
    rho_l: float          # measured liquid density
    rho_v_maxwell: float
    rho_l_maxwell: float

    @property
    def dev_v(self) -> float:
        return self.rho_v / self.rho_v_maxwell - 1.0

    @property
    def dev_l(self) -> float:
        return self.rho_l / self.rho_l_maxwell - 1.0


def with_temperature(p: Params, t_reduced: float, A: float) -> Params:
    """Copy of p at T = t_reduced T_c (the EOS's own critical temperature) and the given A."""
    q = dataclasses.replace(p, A=float(A))
    _, tc, _ = lbm_axi_eos_critical(q)
    q.T = t_reduced * tc
    return q


def measure(cases: list[Params], steps: int = 20000, width: float = 5.0, graph_chunk: int = 100,
            precision: int = PREC_FP64) -> list[Coexistence]:
    """Relax a liquid layer (the middle half of z, tanh interfaces of the given width, the
    Maxwell densities as the start) for every case, all in one batched launch, and return
    the bulk densities: liquid over the ten columns at the layer's centre, vapour over the
    five columns at either end of the domain.  Every case needs nz >= 40."""
    rhos, mx = [], []
    for p in cases:
        if p.nz < 40:
            raise ValueError("flat-interface cases need nz >= 40")
        rv, rl, _ = lbm_axi_eos_coexistence(p)
        mx.append((rv, rl))
        rhos.append(inputs.slab(p.nz, p.nr, rv, rl, 0.25 * p.nz, 0.75 * p.nz, width=width))
    out = []
    with LbmAxi(cases, rhos, precision=precision) as sim:
        if graph_chunk:
            sim.set_graph_chunk(graph_chunk)
        sim.step(steps)
        try:
            sim.sync()
        except LbmError:
            pass  # members that left the EOS domain are flagged below
        bad = sim.errors()
        for k, (p, (rv, rl)) in enumerate(zip(cases, mx)):
            if bad[k]:
                out.append(Coexistence(p, float("nan"), float("nan"), rv, rl))
                continue
            rho = sim.moments(k)[0]
            c = p.nz // 2
            liq = rho[:, c - 5:c + 5].mean()
            vap = np.concatenate([rho[:, :5], rho[:, -5:]], axis=1).mean()
            out.append(Coexistence(p, float(vap), float(liq), rv, rl))
    return out


def zero_crossing(a, d) -> float:
    """First zero of d(a) on the grid a, by linear interpolation between the two grid
    points that bracket it (non-finite entries skipped); nan if no pair brackets one."""
    a = np.asarray(a, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    for j in range(len(a) - 1):
        if np.isfinite(d[j]) and np.isfinite(d[j + 1]) and d[j] * d[j + 1] <= 0.0 and d[j] != d[j + 1]:
            return float(a[j] - d[j] * (a[j + 1] - a[j]) / (d[j + 1] - d[j]))
    return float("nan")


def fit_a(base: Params, t_reduced: list[float], a_grid: list[float], **kw):
    """Scan A over a_grid at every T/T_c in t_reduced (one batched launch) and return
    (A_fit, A_star, table): A_star[i] is the zero of the vapour deviation at t_reduced[i]
    (`zero_crossing`), A_fit their mean, and table[i][j] the Coexistence of
    (t_reduced[i], a_grid[j]).  The domain must hold bulk vapour and liquid at the
    highest temperature: near T_c the interfaces widen (for Carnahan-Starling with
    lambda = 0.05, nz = 300 is enough at T/T_c = 0.9, nz = 150 is not)."""
    cases = [with_temperature(base, t, a) for t in t_reduced for a in a_grid]
    res = measure(cases, **kw)
    na = len(a_grid)
    table = [res[i * na:(i + 1) * na] for i in range(len(t_reduced))]
    star = np.array([zero_crossing(a_grid, [c.dev_v for c in row]) for row in table])
    fit = float(np.nanmean(star)) if np.isfinite(star).any() else float("nan")
    return fit, star, table
