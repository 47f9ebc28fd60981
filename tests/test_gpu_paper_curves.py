"""The paper's other two validations, run with the HIP path in FP64: the coexistence
curve of the exact-difference Kupershtokh model (Fig. 2 set-up) and the propagating
density wave of Sec. 3.3 against the cylindrical wave equation's Bessel-series solution
(eq. analyticdensityprop)."""
import numpy as np
import pytest

from cases import paper_table1
from scipy import special

import oracle as O

pytestmark = pytest.mark.gpu


# --------------------------------------------------------------------------- coexistence curve

def test_flat_interface_coexistence_curve():
    # Fig. 2 set-up: 150 x 100, tau = 1, lambda = 0.01, reduced vdW, A = 0 and A = -0.152.
    # A planar liquid layer across the domain (uniform in r, so F_axis and h_i vanish)
    # relaxes to the scheme's coexistence densities; all instances run as one batch.
    # With A = -0.152 they sit on the Maxwell construction (the paper's reason for that
    # value), down to a density ratio above 10^3 at T = 0.35; with A = 0 the vapour branch
    # falls below it, increasingly so as T drops.
    from paper_1512_01977_amd import inputs, lbm
    cases = [(-0.152, T) for T in (0.35, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9)] + \
            [(0.0, T) for T in (0.5, 0.6, 0.7, 0.8, 0.9)]
    ps, rhos, maxwell = [], [], []
    for A, T in cases:
        p = lbm.Params(nz=150, nr=100, tau=1.0, eos=lbm.EOS_VDW, T=T, lam=0.01, A=A)
        rv, rl, _ = lbm.lbm_axi_eos_coexistence(p)
        ps.append(p)
        rhos.append(inputs.slab(150, 100, rv, rl, 37.5, 112.5, width=5.0))
        maxwell.append((rv, rl))
    dev = {}
    with lbm.LbmAxi(ps, rhos) as sim:
        sim.set_graph_chunk(100)
        sim.step(20000)
        assert not sim.errors().any()
        for k, ((A, T), (rv, rl)) in enumerate(zip(cases, maxwell)):
            rho = sim.moments(k)[0]
            liq = rho[:, 70:80].mean()
            vap = np.concatenate([rho[:, :5], rho[:, 145:]], axis=1).mean()
            dev[(A, T)] = (liq / rl - 1, vap / rv - 1, liq / vap)
            print(f"A {A:+.3f} T {T:.2f}: rho_l {liq:.5f} ({liq / rl - 1:+.2e} vs Maxwell), "
                  f"rho_v {vap:.6f} ({vap / rv - 1:+.2e}), ratio {liq / vap:.0f}", flush=True)
    for (A, T), (dl, dv, ratio) in dev.items():
        if A != 0.0:
            assert abs(dl) <= 1e-3 and abs(dv) <= (2e-2 if T < 0.4 else 5e-3), (A, T)
        else:
            assert dv < -5e-3 and abs(dv) > 3 * abs(dev[(-0.152, T)][1]), (A, T)
    assert dev[(-0.152, 0.35)][2] > 1000


# --------------------------------------------------------------------------- density wave

def bessel_series(r, init, R, c, t, zeros, norm, mean, nquad=20001):
    """sum_n a_n J0(k_n r / R) cos(c k_n t / R) (+ the mean for the rigid-wall modes),
    a_n = 2 / (R^2 norm(k_n)^2) int_0^R init(r') J0(k_n r' / R) r' dr'."""
    rr = np.linspace(0.0, R, nquad)
    w = init(rr) * rr
    out = np.full_like(r, 2.0 / R**2 * np.trapezoid(w, rr) if mean else 0.0)
    for kn in np.array_split(zeros, 10):
        a = 2.0 / (R**2 * norm(kn) ** 2) * np.trapezoid(special.j0(np.outer(kn, rr) / R) * w, rr, axis=1)
        out += (a[:, None] * special.j0(np.outer(kn, r) / R) * np.cos(c * kn[:, None] * t / R)).sum(0)
    return out


def test_density_wave_against_bessel_series():
    # Sec. 3.3 set-up: 1 x 2000, tau = 0.6, vdW T = 0.8, rho_0 = 1.8, A = 0, lambda = 0.01,
    # no-slip wall.  The paper gives neither the disturbance's shape, width nor amplitude:
    # here a Gaussian ring of width w_d = 40 and amplitude 1e-3 at r = 1000.  The linear
    # inviscid solution is the Bessel series with c_k^2 = dP_k/drho(rho_0); the paper prints
    # it with the zeros of J0 (a node at r = R), while a rigid wall gives the zeros of J1
    # plus the mean.  Until the wave reaches the wall (t_w <= 3.98 here) the two are the same
    # field, which is checked, and the simulation is compared with it.
    from paper_1512_01977_amd import inputs, lbm
    R, r0, wd, amp, rho0 = 2000.0, 1000.0, 40.0, 1e-3, 1.8
    p = lbm.Params(nz=1, nr=2000, tau=0.6, eos=lbm.EOS_VDW, T=0.8, lam=0.01, A=0.0,
                   bc_top=lbm.TOP_NO_SLIP)
    _, kap, _ = O.eos(O.Params(nz=1, nr=4, eos=O.EOS_VDW, T=0.8, lam=0.01), rho0)
    c = np.sqrt(kap)
    r = np.arange(2000) + 0.5
    init = lambda x: amp * np.exp(-((x - r0) / wd) ** 2)
    with lbm.LbmAxi(p, inputs.gaussian_pulse(1, 2000, rho0, amp, r0, wd)) as sim:
        m0 = sim.mass()[0]
        done = 0
        for tw in (1.0, 2.0, 3.98):
            t = int(round(tw * wd / c))
            sim.step(t - done)
            done = t
            rho1 = sim.moments()[0][:, 0] - rho0
            rigid = bessel_series(r, init, R, c, t, special.jn_zeros(1, 600), special.j0, True)
            printed = bessel_series(r, init, R, c, t, special.jn_zeros(0, 600), special.j1, False)
            err = np.abs(rho1 - rigid).max() / amp
            drift = sim.mass()[0] / m0 - 1
            print(f"t_w {tw}: {t} steps, max |sim - series| / amplitude {err:.4f}, "
                  f"peak {rho1.max() / amp:.4f} vs {rigid.max() / amp:.4f}, mass drift {drift:+.1e}",
                  flush=True)
            assert np.abs(printed - rigid).max() / amp <= 1e-10
            assert err <= 0.04
            assert abs(drift) <= 1e-12


# --------------------------------------------------------------------------- Guo vs exact difference

def test_guo_forcing_against_exact_difference():
    # The two force applications of the paper side by side (both in one batched launch):
    # Sec. 2.1 prints Guo's term, Sec. 2.3 relies on the exact-difference method.
    # (a) Table 1 set-up (vdW, lambda 0.01, 500 x 200, tau 1.5, R_0 = 150, T 0.8, A 0 and
    #     -0.152, 2-D and axisymmetric): Guo's sigma = dp R / lambda lands on the printed
    #     values (within 6 %), the exact-difference one is 1.6x them; the axisymmetric/2-D
    #     agreement the paper reports holds for both.
    # (b) flat-interface coexistence (150 x 100, tau 1): only the exact-difference method
    #     with A = -0.152 sits on the Maxwell curve; Guo leaves it by tens of per cent.
    from paper_1512_01977_amd import inputs, lbm
    table1 = {k: v for k, v in paper_table1().items() if k[0] == 0.8}
    cases = [(fo, A, ax) for fo in (0, 1) for A in (0.0, -0.152) for ax in (0, 1)]
    ps, rhos = [], []
    for fo, A, ax in cases:
        p = lbm.Params(nz=500, nr=200, tau=1.5, eos=lbm.EOS_VDW, T=0.8, lam=0.01, A=A, axisym=ax, forcing=fo)
        rv, rl, _ = lbm.lbm_axi_eos_coexistence(p)
        ps.append(p)
        rhos.append(inputs.droplet(500, 200, rv, rl, 150.0, zc=250.0, width=5.0, noise=1e-4, seed=1))
    sig = {c: [] for c in cases}
    with lbm.LbmAxi(ps, rhos) as sim:
        sim.set_graph_chunk(100)
        sim.step(35000)
        for _ in range(6):
            sim.step(5000)
            dps = sim.laplace([250.0] * len(cases), [75.0] * len(cases), [170.0] * len(cases))
            for k, c in enumerate(cases):
                R = r_volume(sim.moments(k)[0], 250.0, 150.0, c[2])
                sig[c].append(dps[k] * R / 0.01)
        assert not sim.errors().any()
    for fo in (0, 1):
        for A in (0.0, -0.152):
            s2, s3 = np.mean(sig[(fo, A, 0)]), np.mean(sig[(fo, A, 1)])
            p2, p3 = table1[(0.8, A)]
            print(f"forcing {'Guo' if fo else 'EDM'} A {A:+.3f}: sigma_2D {s2:.3f} (paper {p2}), "
                  f"sigma_axis {s3:.3f} (paper {p3})", flush=True)
            assert s3 == pytest.approx(s2, rel=0.05)
            if fo:
                assert s2 == pytest.approx(p2, rel=0.06) and s3 == pytest.approx(p3, rel=0.06)
            else:
                assert s2 > 1.5 * p2
    coex = {}
    cases = [(fo, A) for fo in (0, 1) for A in (0.0, -0.152)]
    ps, rhos, mx = [], [], []
    for fo, A in cases:
        p = lbm.Params(nz=150, nr=100, tau=1.0, eos=lbm.EOS_VDW, T=0.8, lam=0.01, A=A, forcing=fo)
        rv, rl, _ = lbm.lbm_axi_eos_coexistence(p)
        ps.append(p)
        rhos.append(inputs.slab(150, 100, rv, rl, 37.5, 112.5, width=5.0))
        mx.append(rv)
    with lbm.LbmAxi(ps, rhos) as sim:
        sim.set_graph_chunk(100)
        sim.step(20000)
        for k, c in enumerate(cases):
            rho = sim.moments(k)[0]
            coex[c] = np.concatenate([rho[:, :5], rho[:, 145:]], axis=1).mean() / mx[k] - 1
            print(f"forcing {'Guo' if c[0] else 'EDM'} A {c[1]:+.3f}: rho_v {coex[c]:+.2e} vs Maxwell", flush=True)
    assert abs(coex[(0, -0.152)]) < 5e-3
    assert min(abs(coex[(1, 0.0)]), abs(coex[(1, -0.152)])) > 0.1


def r_volume(rho, zc, R0, axisym, margin=20):
    """Equivalent radius from the liquid volume (sphere in the axisymmetric case)."""
    nr, nz = rho.shape
    Z, Rr = np.meshgrid(np.arange(nz) - zc, np.arange(nr) + 0.5)
    d = np.hypot(Z, Rr)
    rin, rout = rho[d < R0 / 2].mean(), rho[d > R0 + margin].mean()
    frac = (rho - rout) / (rin - rout)
    if axisym:
        return (3 * (2 * np.pi * Rr * frac).sum() / (4 * np.pi)) ** (1 / 3)
    return np.sqrt(2 * frac.sum() / np.pi)


# --------------------------------------------------------------------------- A calibration

def test_mixing_parameter_calibration():
    # Flat-interface coexistence scanned over Kupershtokh's A (Sec. 2.3).  (a) For the
    # reduced vdW EOS with lambda = 0.01 the A that puts the vapour branch on the Maxwell
    # curve is the paper's -0.152 (within 0.005 at every T from 0.5 to 0.9).  (b) The same
    # calibration for Carnahan-Starling with lambda = 0.05 (the scale of the ratio-1e3
    # workloads) gives a T-independent A as well (-0.164); at that A the vapour density is
    # within 0.5 % of Maxwell from T/T_c = 0.6 to 0.9, where A = 0 misses it by 5-98 %.
    from paper_1512_01977_amd import coexistence as C, lbm
    grid = [round(-0.24 + 0.02 * j, 2) for j in range(13)]
    vdw = lbm.Params(nz=300, nr=8, tau=1.0, eos=lbm.EOS_VDW, lam=0.01)
    fit, star, _ = C.fit_a(vdw, [0.5, 0.7, 0.9], grid, steps=40000)
    print(f"vdW lambda 0.01: A_fit {fit:+.4f}, A*(T) {np.round(star, 4)} (paper -0.152)", flush=True)
    assert np.all(np.abs(star + 0.152) <= 5e-3)
    cs = lbm.Params(nz=300, nr=8, tau=1.0, eos=lbm.EOS_CS, eos_a=1.0, eos_b=4.0, eos_R=1.0, lam=0.05)
    ts = [0.6, 0.7, 0.8, 0.9]
    fit_cs, star_cs, table = C.fit_a(cs, ts, grid, steps=40000)
    print(f"CS lambda 0.05: A_fit {fit_cs:+.4f}, A*(T) {np.round(star_cs, 4)}", flush=True)
    assert np.all(np.isfinite(star_cs)) and np.ptp(star_cs) <= 5e-3
    check = C.measure([C.with_temperature(cs, t, a) for a in (fit_cs, 0.0) for t in ts], steps=40000)
    at_fit, at_zero = check[:len(ts)], check[len(ts):]
    for t, c1, c0 in zip(ts, at_fit, at_zero):
        print(f"  T/T_c {t}: vapour vs Maxwell at A_fit {c1.dev_v:+.4f}, at A = 0 {c0.dev_v:+.4f}; "
              f"liquid {c1.dev_l:+.5f}", flush=True)
        assert abs(c1.dev_v) <= 5e-3 and abs(c1.dev_l) <= 2e-3
        assert abs(c0.dev_v) >= 0.03
