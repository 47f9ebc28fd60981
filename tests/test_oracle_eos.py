"""Pins of the oracle's equation-of-state layer (Sec. 2.3) against closed forms
and the defining conditions of the critical point and of the Maxwell
construction.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O


def cs(T=0.0, lam=1.0):
    return O.Params(nz=8, nr=8, eos=O.EOS_CS, T=T, eos_a=1.0, eos_b=4.0, eos_R=1.0, lam=lam)


def vdw(T=0.0, lam=0.01):
    return O.Params(nz=8, nr=8, eos=O.EOS_VDW, T=T, lam=lam)


def P_of(p, rho):
    return O.eos(p, rho)[0]


def test_vdw_reduced_critical_point():
    # The dimensionless vdW EOS of eq. (kupershtokvdwpressure) is written in reduced
    # variables, so its critical point is rho = T = 1 with P_k = lambda.
    rc, Tc, Pc = O.critical(vdw())
    assert rc == pytest.approx(1.0, rel=1e-6)
    assert Tc == pytest.approx(1.0, rel=1e-12)
    assert Pc == pytest.approx(0.01, rel=1e-12)


def test_cs_critical_point_conditions():
    # At the critical point dP/drho = d2P/drho2 = 0 (checked by central differences of P_k),
    # and the Carnahan-Starling-van der Waals critical compressibility factor is 0.3590.
    rc, Tc, Pc = O.critical(cs())
    p = cs(T=Tc)
    h = 1e-3 * rc
    d1 = (P_of(p, rc + h) - P_of(p, rc - h)) / (2 * h)
    d2 = (P_of(p, rc + h) - 2 * P_of(p, rc) + P_of(p, rc - h)) / h ** 2
    scale = Pc / rc
    # truncation of the differences is O(h^2) of the third derivative
    assert abs(d1) < 1e-5 * scale
    assert abs(d2) < 1e-4 * scale / rc
    # a point off the critical point fails the same test
    off = (P_of(p, 1.1 * rc + h) - P_of(p, 1.1 * rc - h)) / (2 * h)
    assert abs(off) > 1e-3 * scale
    assert Pc / (rc * Tc) == pytest.approx(0.3590, abs=2e-4)
    assert P_of(p, rc) == pytest.approx(Pc, rel=1e-12)


@pytest.mark.parametrize("kind", ["cs", "vdw"])
def test_kappa_is_dP_drho(kind):
    p = cs(T=0.08) if kind == "cs" else vdw(T=0.85)
    for rho in ([0.01, 0.1, 0.2, 0.3, 0.45] if kind == "cs" else [0.2, 0.8, 1.5, 2.2]):
        h = 1e-6 * rho
        fd = (P_of(p, rho + h) - P_of(p, rho - h)) / (2 * h)
        assert O.eos(p, rho)[1] == pytest.approx(fd, rel=1e-7, abs=1e-12)


def test_vdw_sound_speed_matches_paper():
    # eq. (kupershtokhspeedofsound): c_k^2 = lambda (24 T/(rho-3)^2 - 6 rho)
    p = vdw(T=0.8)
    for rho in [0.3, 1.0, 1.9]:
        ck2 = 0.01 * (24 * 0.8 / (rho - 3) ** 2 - 6 * rho)
        assert O.eos(p, rho)[1] == pytest.approx(ck2, rel=1e-13)


def test_psi_definition_and_domain():
    # psi = sqrt(rho/3 - P_k) (Sec. 2.3); outside the real range the oracle reports -4.
    rc, Tc, _ = O.critical(cs())
    p = cs(T=0.485 * Tc)
    P, _, psi = O.eos(p, 0.3)
    assert psi * psi == pytest.approx(0.3 / 3 - P, rel=1e-14)
    with pytest.raises(O.OracleError) as e:
        O.eos(p, 0.6)        # above the psi-real limit (about 0.557) at this T
    assert e.value.code == -4
    with pytest.raises(O.OracleError):
        O.eos(p, -1e-3)
    ideal = O.Params(nz=8, nr=8, eos=O.EOS_IDEAL)
    assert O.eos(ideal, 0.7) == (pytest.approx(0.7 / 3), pytest.approx(1 / 3), 0.0)


@pytest.mark.parametrize("kind,t", [("cs", 0.9), ("cs", 0.8), ("cs", 0.7), ("cs", 0.5),
                                    ("cs", 0.485), ("vdw", 0.9), ("vdw", 0.8), ("vdw", 0.7)])
def test_maxwell_equal_area(kind, t):
    # Coexistence: equal pressures and the equal-area rule int_{v_l}^{v_v} (P - P_sat) dv = 0.
    if kind == "cs":
        _, Tc, _ = O.critical(cs())
        p = cs(T=t * Tc)
    else:
        p = vdw(T=t)
    rv, rl, ps = O.coexistence(p)
    assert rv < rl
    assert P_of(p, rv) == pytest.approx(ps, rel=1e-9)
    assert P_of(p, rl) == pytest.approx(ps, rel=1e-9)
    f = lambda v: P_of(p, 1.0 / v) - ps
    area, _ = integrate.quad(f, 1.0 / rl, 1.0 / rv, limit=400, epsabs=0, epsrel=1e-10)
    scale = ps * (1.0 / rv - 1.0 / rl)
    assert abs(area) < 1e-7 * scale
    # Both coexisting states are mechanically stable (outside the spinodal region).
    assert O.eos(p, rv)[1] > 0 and O.eos(p, rl)[1] > 0


def test_cs_ratio_1000_temperature():
    # The density ratio reaches 1e3 near T/T_c = 0.485 (used by the high-ratio workloads).
    _, Tc, _ = O.critical(cs())
    rv, rl, _ = O.coexistence(cs(T=0.485 * Tc))
    assert 950 < rl / rv < 1050
