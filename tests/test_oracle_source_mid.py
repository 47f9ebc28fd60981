"""Pins of the oracle's link-midpoint source (Sec. 2.2: h_i evaluated half-way along the
link, at x + c_i/2), flag source_mid = 1: the mean of h_i over the link's two ends.

What fixes it without retyping it:
* Totals.  Over the whole grid the mean over links only moves source between neighbours:
  with z periodic and mirrored sources beyond the axis and the wall (mirror direction,
  -rho u_r/r and H_z even, H_r odd), sum_x sum_i h_i and sum_x sum_i c_iz h_i are the
  same as for the node source, exactly.  So one step changes the plain sum of rho by
  -sum rho u_r / r (eq. masscylinderical) in either variant.
* Order of accuracy.  For smooth fields the link mean is within O(k^2) of the continuum
  h_i at the midpoint x + c_i/2 (the node value is only within O(k)), with the continuum
  value taken from the node source at that point with exact derivatives.
Each pin is also run against copies of the oracle with one plausible slip planted.
CPU only."""
import ctypes
import os
import tempfile

import numpy as np
import pytest

import oracle as O
from oracle import build as obuild
from paper_1512_01977_amd import inputs


def cs_params(nz, nr, **kw):
    tc = O.critical(O.Params(nz=4, nr=4, eos=O.EOS_CS))[1]
    kw.setdefault("tau", 0.9)
    return O.Params(nz=nz, nr=nr, eos=O.EOS_CS, T=0.8 * tc, **kw)


def random_fields(nz, nr, seed):
    rng = np.random.default_rng(seed)
    rho = 0.2 + 0.05 * rng.random((nr, nz))
    uz = 0.02 * rng.standard_normal((nr, nz))
    ur = 0.02 * rng.standard_normal((nr, nz))
    return rho, uz, ur


def smooth_fields(k, z, r):
    """Analytic rho, u_z, u_r (u_r odd in r) and the three derivatives the source needs."""
    rho = 1.0 + 0.05 * np.cos(k * z + 0.3) * (1.0 + 0.1 * np.cos(k * r))
    uz = 0.01 * np.cos(k * z) * np.cos(k * r)
    ur = 0.01 * np.sin(k * r) * np.cos(k * z + 0.5)
    dr_uz = -0.01 * k * np.cos(k * z) * np.sin(k * r)
    dz_ur = -0.01 * k * np.sin(k * r) * np.sin(k * z + 0.5)
    dr_ur = 0.01 * k * np.cos(k * r) * np.cos(k * z + 0.5)
    return rho, uz, ur, dr_uz, dz_ur, dr_ur


class _Shipped:
    source_field = staticmethod(O.source_field)
    step = staticmethod(O.step)


class _Lib:
    def __init__(self, path):
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(O._Params)
        dp = ctypes.POINTER(ctypes.c_double)
        L.lbm_oracle_source_field.argtypes = [P, dp, dp, dp, dp]
        L.lbm_oracle_step.argtypes = [P, dp, ctypes.c_int64]
        self.L = L

    def source_field(self, p, rho, uz, ur):
        rho, uz, ur = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, uz, ur))
        h = np.zeros((9, p.nr, p.nz))
        assert self.L.lbm_oracle_source_field(ctypes.byref(p.c()), O._ptr(rho), O._ptr(uz), O._ptr(ur),
                                              O._ptr(h)) == 0
        return h

    def step(self, p, f, n):
        assert self.L.lbm_oracle_step(ctypes.byref(p.c()), O._ptr(f), n) == 0
        return f


# --------------------------------------------------------------------------- pins

def totals_fail(impl, bc_top):
    p0 = cs_params(21, 11, bc_top=bc_top)
    p1 = cs_params(21, 11, bc_top=bc_top, source_mid=1)
    rho, uz, ur = random_fields(21, 11, seed=7 + bc_top)
    h0 = O.source_field(p0, rho, uz, ur)          # node source of the shipped oracle
    h1 = impl.source_field(p1, rho, uz, ur)
    scale = np.abs(h0).sum()
    out = []
    if not np.abs(h1 - h0).max() > 1e-3 * np.abs(h0).max():
        out.append("no local change")
    if abs(h1.sum() - h0.sum()) > 1e-13 * scale:
        out.append("zeroth total")
    if abs((O.CZ[:, None, None] * h1).sum() - (O.CZ[:, None, None] * h0).sum()) > 1e-13 * scale:
        out.append("z total")
    return out


def accuracy_fail(impl):
    """Max error of the link mean and of the node value against the continuum h_i at
    x + c_i/2, over interior nodes of the same physical region, at k, k/2, k/4."""
    err_mid, err_node = [], []
    for s in (1, 2, 4):
        nz = nr = 32 * s
        k = 2 * np.pi * 2 / nz
        p1 = O.Params(nz=nz, nr=nr, eos=O.EOS_IDEAL, tau=0.8, source_mid=1)
        Z, R = np.meshgrid(np.arange(nz, dtype=float), np.arange(nr) + 0.5)
        rho, uz, ur, *_ = smooth_fields(k, Z, R)
        hm = impl.source_field(p1, rho, uz, ur)
        rows = slice(nr // 4, 3 * nr // 4)   # away from the axis and the wall
        Zi, Ri = Z[rows], R[rows]
        em = en = hmax = 0.0
        for i in range(9):
            zc, rc = Zi + 0.5 * O.CZ[i], Ri + 0.5 * O.CR[i]
            ex = np.vectorize(lambda *a: O.source(p1, *a)[i])(rc, *smooth_fields(k, zc, rc))
            hn = np.vectorize(lambda *a: O.source(p1, *a)[i])(Ri, *smooth_fields(k, Zi, Ri))
            em = max(em, np.abs(hm[i][rows] - ex).max())
            en = max(en, np.abs(hn - ex).max())
            hmax = max(hmax, np.abs(ex).max())
        err_mid.append(em / hmax)
        err_node.append(en / hmax)
    out = []
    rm = err_mid[0] / err_mid[1], err_mid[1] / err_mid[2]
    if not (min(rm) > 3.3):
        out.append(f"not second order: {err_mid}")
    if not err_mid[-1] < 0.2 * err_node[-1]:
        out.append(f"no better than the node value: {err_mid} vs {err_node}")
    return out


def step_mass_fail(impl):
    # Collision and the force conserve mass and streaming permutes populations, so the
    # plain sum of rho changes by the total source, -sum rho u_r / r, in either variant.
    p = cs_params(40, 20, A=-0.152, source_mid=1)
    rv, rl, _ = O.coexistence(p)
    f = O.init(p, inputs.droplet(40, 20, rv, rl, 8.0, eps=0.15, noise=1e-4, seed=2))
    impl.step(p, f, 30)
    rho, uz, ur = O.moments(p, f)
    src = -(rho * ur / (np.arange(20) + 0.5)[:, None]).sum()
    s0 = f.sum()
    impl.step(p, f, 1)
    return [] if abs((f.sum() - s0) - src) <= 1e-9 * abs(src) + 1e-14 * s0 else ["mass per step"]


@pytest.mark.parametrize("bc_top", [O.TOP_FREE_SLIP, O.TOP_NO_SLIP])
def test_link_mean_totals(bc_top):
    assert totals_fail(_Shipped, bc_top) == []


def test_link_mean_is_second_order_at_the_midpoint():
    assert accuracy_fail(_Shipped) == []


def test_step_mass_change_is_the_total_source():
    assert step_mass_fail(_Shipped) == []


def test_two_d_mode_has_no_source():
    p = cs_params(12, 7, axisym=0, source_mid=1)
    assert not np.any(O.source_field(p, *random_fields(12, 7, 1)))


def test_variants_differ_but_keep_symmetry():
    # A z-mirror-symmetric drop stays symmetric with the link-midpoint source, and its state
    # after a few hundred steps differs from the node-source run.
    out = {}
    for mid in (0, 1):
        p = cs_params(48, 24, A=-0.152, source_mid=mid)
        rv, rl, _ = O.coexistence(p)
        rho0 = inputs.droplet(48, 24, rv, rl, 9.0, eps=0.2, noise=0.0, seed=1)
        f = O.init(p, rho0)
        O.step(p, f, 300)
        out[mid] = O.moments(p, f)[0]
    rho = out[1]
    # node k mirrors to node 48 - k (the drop is centred at z = 24)
    assert np.abs(rho[:, 1:] - rho[:, 1:][:, ::-1]).max() <= 1e-12 * rho.max()
    assert np.abs(out[1] - out[0]).max() > 1e-7


# --------------------------------------------------------------------------- planted slips

SLIPS = {
    "sum, not mean": ("0.5 * (source_ext(hn, nz, nr, i, k, j) + source_ext",
                      "1.0 * (source_ext(hn, nz, nr, i, k, j) + source_ext"),
    "far end at x - c_i": ("source_ext(hn, nz, nr, i, k + CZ[i], j + CR[i])",
                           "source_ext(hn, nz, nr, i, k - CZ[i], j - CR[i])"),
    "ghost not mirrored in direction": (
        "if (j < 0) return hn[(size_t)mirror_dir(i) * n + at(nz, k, -1 - j)];",
        "if (j < 0) return hn[(size_t)i * n + at(nz, k, -1 - j)];"),
    "ghost at the wall not mirrored in direction": (
        "if (j >= nr) return hn[(size_t)mirror_dir(i) * n + at(nz, k, 2 * nr - 1 - j)];",
        "if (j >= nr) return hn[(size_t)i * n + at(nz, k, 2 * nr - 1 - j)];"),
}


def _planted(tmp, name):
    old, new = SLIPS[name]
    with open(obuild.SRC) as fh:
        src = fh.read()
    assert src.count(old) == 1, name
    path = os.path.join(tmp, "mut.c")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    lib = os.path.join(tmp, "mut.so")
    obuild.compile_source(path, lib)
    return _Lib(lib)


@pytest.mark.parametrize("name", sorted(SLIPS))
def test_pins_catch_planted_slip(name):
    with tempfile.TemporaryDirectory() as tmp:
        impl = _planted(tmp, name)
        failed = totals_fail(impl, O.TOP_FREE_SLIP) + totals_fail(impl, O.TOP_NO_SLIP)
        if not failed:
            failed = step_mass_fail(impl)
        if not failed:
            failed = accuracy_fail(impl)
        assert failed, name
