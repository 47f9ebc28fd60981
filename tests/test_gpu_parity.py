"""HIP path against the CPU oracle, through the C ABI, on MI355X.

FP64: every field within 1e-10 relative (max norm) of the oracle; the same bar the
static-droplet workload is held to after 1000 steps.  Bitwise checks for the
properties that must not depend on launch shape: batch vs single instance,
graph replay vs eager launches, checkpoint round trip, repeat runs.
"""
import numpy as np
import pytest

import oracle as O
from cases import base, droplet_rho, gpu_params, oracle_params, rel_inf

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def lbm():
    from paper_1512_01977_amd import lbm as L
    return L


def run_pair(d, rho0, steps, precision=0, launch=None, uz0=None):
    L = lbm()
    po = oracle_params(d)
    f = O.init(po, rho0, uz0=uz0)
    O.step(po, f, steps)
    ro, uzo, uro = O.moments(po, f)
    with L.LbmAxi(gpu_params(d), rho0, precision=precision, uz0=uz0) as sim:
        if launch:
            sim.set_launch(**launch)
        sim.step(steps)
        rg, uzg, urg = sim.moments()
        fg = sim.get_f()
    return (ro, uzo, uro, f), (rg, uzg, urg, fg)


def assert_fp64_parity(o, g, tol=TOL64):
    """Max-norm errors relative to each field's scale; both velocity components are
    measured against the velocity scale max(|u_z|, |u_r|) of the oracle."""
    ro, uzo, uro, fo = o
    rg, uzg, urg, fg = g
    uscale = max(np.abs(uzo).max(), np.abs(uro).max(), 1e-300)
    errs = {"rho": rel_inf(rg, ro), "f": rel_inf(fg, fo),
            "uz": float(np.abs(uzg - uzo).max() / uscale),
            "ur": float(np.abs(urg - uro).max() / uscale)}
    print("parity", errs, flush=True)
    assert max(errs.values()) <= tol, errs


def test_initial_state_matches_oracle():
    d = base(40, 24)
    rho0 = droplet_rho(d, 8.0, eps=0.1)
    assert_fp64_parity(*run_pair(d, rho0, 0), tol=1e-15)


def test_static_droplet_1000_steps_fp64():
    # 128 x 64 static droplet, CS at T/Tc = 0.8, tau = 1, R = 20, noise 1e-4 (seed 1).
    d = base(128, 64)
    rho0 = droplet_rho(d, 20.0, noise=1e-4, seed=1)
    print("case static droplet 128x64 fp64 1000 steps", flush=True)
    assert_fp64_parity(*run_pair(d, rho0, 1000))


LAUNCHES = [
    dict(width=64, seg_rows=8, persistent=0, xcd_swizzle=0, regf=0),
    dict(width=64, seg_rows=16, persistent=1, xcd_swizzle=1, regf=1),
    dict(width=128, seg_rows=0, persistent=0, xcd_swizzle=1, regf=1),
    dict(width=128, seg_rows=9, persistent=1, xcd_swizzle=0, regf=0),
    dict(width=256, seg_rows=13, persistent=1, xcd_swizzle=1, regf=0),
    dict(width=256, seg_rows=20, persistent=0, xcd_swizzle=1, regf=1),
    dict(width=128, seg_rows=24, persistent=0, xcd_swizzle=2, regf=1),
    dict(width=64, seg_rows=11, persistent=0, xcd_swizzle=2, regf=0),
]


@pytest.mark.parametrize("launch", LAUNCHES,
                         ids=lambda c: f"w{c['width']}s{c['seg_rows']}p{c['persistent']}"
                                       f"x{c['xcd_swizzle']}r{c['regf']}")
def test_launch_shapes_agree_with_oracle(launch):
    # strips with ragged tails (nz = 150 is no multiple of width - 12) and row segments
    d = base(150, 37, A=-0.152, tau=0.9)
    rho0 = droplet_rho(d, 11.0, eps=0.2, zc=70.0)
    print("case", launch, flush=True)
    assert_fp64_parity(*run_pair(d, rho0, 120, launch=launch))


@pytest.mark.parametrize("width", [128, 256])
def test_several_strips_per_row_agree_with_oracle(width):
    # nz = 800 spans several strips (256 lanes: 224 x 3 + 128 columns, the last strip's upper
    # wave ends at once), segments of 12 rows, one workgroup per item
    # with the populations in registers and the persistent queue gathering them again
    d = base(800, 30, A=-0.152, tau=0.85)
    rho0 = droplet_rho(d, 10.0, eps=0.2, zc=400.0, seed=7)
    for regf, pers in ((1, 0), (0, 1)):
        launch = dict(width=width, seg_rows=12, persistent=pers, xcd_swizzle=2 if not pers else 0, regf=regf)
        print("case nz 800", launch, flush=True)
        assert_fp64_parity(*run_pair(d, rho0, 60, launch=launch))


def test_fp32_form_launch_shapes_agree_bitwise():
    # The FP32 form in every launch shape of the list above on the same case: the
    # decomposition into strips (whole 128-byte lines: 32 floats) and segments does not
    # change what a node computes, so all shapes agree bitwise; and the result is within
    # FP32 rounding of the FP64 oracle.
    d = base(150, 37, A=-0.152, tau=0.9)
    rho0 = droplet_rho(d, 11.0, eps=0.2, zc=70.0)
    o, first = None, None
    for launch in LAUNCHES:
        print("case", launch, flush=True)
        o, g = run_pair(d, rho0, 120, precision=1, launch=launch) if o is None else (o, run_pair_gpu(d, rho0, 120, 1, launch))
        if first is None:
            first = g
            ro, uzo, uro, _ = o
            uscale = max(np.abs(uzo).max(), np.abs(uro).max())
            er = rel_inf(g[0], ro)
            eu = max(np.abs(g[1] - uzo).max(), np.abs(g[2] - uro).max()) / uscale
            print(f"FP32 vs oracle: rho {er:.2e}, u {eu:.2e}", flush=True)
            assert er <= 1e-5 and eu <= 1e-4
        else:
            for a, b in zip(g, first):
                assert np.array_equal(a, b), launch


def test_fp64_form_launch_shapes_agree_bitwise():
    # FP64: the populations carried in registers (F_K then travels through the LDS rings and
    # kappa and 1/r are computed again, the same expressions) or gathered again for the
    # collision, persistent or not, any strip width and segment length: the same arithmetic
    # on every node, so bitwise the same state; the first shape is also checked against the
    # oracle.
    d = base(150, 37, A=-0.152, tau=0.9)
    rho0 = droplet_rho(d, 11.0, eps=0.2, zc=70.0)
    o, first = run_pair(d, rho0, 120, precision=0, launch=LAUNCHES[0])
    assert_fp64_parity(o, first)
    for launch in LAUNCHES[1:]:
        print("case", launch, flush=True)
        g = run_pair_gpu(d, rho0, 120, 0, launch)
        for a, b in zip(g, first):
            assert np.array_equal(a, b), launch


def run_pair_gpu(d, rho0, steps, precision, launch):
    L = lbm()
    with L.LbmAxi(gpu_params(d), rho0, precision=precision) as sim:
        sim.set_launch(**launch)
        sim.step(steps)
        rg, uzg, urg = sim.moments()
        return rg, uzg, urg, sim.get_f()


VARIANTS = {
    "no_slip_top": dict(bc_top=1),
    "two_d": dict(axisym=0),
    "lattice_cs4": dict(faxis_sound=1, A=-0.152),
    "vdw": dict(eos=O.EOS_VDW, lam=0.01, T=0.8, tau=0.7),
    "body_force": dict(gz=2e-6),
    "A_positive": dict(A=0.1),
    "guo": dict(forcing=1, A=-0.152, gz=2e-6),
    "guo_two_d_no_slip": dict(forcing=1, axisym=0, bc_top=1),
}


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_variants_agree_with_oracle(name):
    d = base(48, 30, **VARIANTS[name])
    rho0 = droplet_rho(d, 9.0, eps=0.15, zc=20.0)
    print("case", name, flush=True)
    assert_fp64_parity(*run_pair(d, rho0, 150))


def test_ideal_gas_with_velocity():
    d = base(33, 20, eos=O.EOS_IDEAL, tau=0.75, bc_top=1, gz=1e-6)
    rng = np.random.default_rng(5)
    rho0 = 1.0 + 0.01 * rng.standard_normal((20, 33))
    uz0 = 0.01 * rng.standard_normal((20, 33))
    assert_fp64_parity(*run_pair(d, rho0, 100, uz0=uz0))


@pytest.mark.parametrize("nz", [1, 2, 5])
def test_narrow_domains(nz):
    # nz = 1 is the paper's wave-propagation geometry (Sec. 3.3): every lane wraps to one column.
    d = base(nz, 40, T=0.9 * base(1, 1)["T"] / 0.8, tau=0.7, bc_top=1)
    from paper_1512_01977_amd import inputs
    rv, _, _ = O.coexistence(oracle_params(d))
    rho0 = inputs.radial_wave(nz, 40, rv, amplitude=1e-2, wavelength=16.0, noise=1e-6, seed=3)
    assert_fp64_parity(*run_pair(d, rho0, 200))


def test_minimum_rows():
    d = base(20, 4, eos=O.EOS_IDEAL, tau=0.8)
    rho0 = 1.0 + 0.02 * np.random.default_rng(1).standard_normal((4, 20))
    assert_fp64_parity(*run_pair(d, rho0, 50))


def test_mass_and_laplace_match_oracle():
    L = lbm()
    d = base(96, 48)
    rho0 = droplet_rho(d, 16.0)
    po = oracle_params(d)
    f = O.init(po, rho0)
    O.step(po, f, 300)
    with L.LbmAxi(gpu_params(d), rho0) as sim:
        sim.step(300)
        m = sim.mass()[0]
        dp = sim.laplace(48.0, 8.0, 28.0)[0]
        m2 = sim.mass()[0]
    assert m == m2                                   # deterministic reduction
    assert m == pytest.approx(O.mass(po, f), rel=1e-12)
    assert dp == pytest.approx(O.laplace(po, f, 48.0, 8.0, 28.0), rel=1e-9)


def test_axis_interface_matches_oracle():
    # The drop's interface on the axis (Sec. 3.2) in a batch: a P2-stretched drop in FP64
    # (against the oracle on the same populations), the same drop in FP32 (against the
    # FP64 value, to FP32 rounding of the densities), and a threshold below the vapour
    # density (no crossing: NaN on both sides).  zc outside the domain is refused.
    L = lbm()
    d = base(96, 48, A=-0.152)
    rho0 = droplet_rho(d, 16.0, eps=0.2, zc=48.0)
    rv, rl, _ = O.coexistence(oracle_params(d))
    thr = 0.5 * (rv + rl)
    po = oracle_params(d)
    f = O.init(po, rho0)
    O.step(po, f, 200)
    z_o = O.axis_interface(po, f, 48.0, thr)
    assert np.isnan(O.axis_interface(po, f, 48.0, 0.5 * rv))
    got = {}
    for prec in (0, 1):
        with L.LbmAxi([gpu_params(d), gpu_params(d)], [rho0, rho0], precision=prec) as sim:
            sim.step(200)
            z = sim.axis_interface([48.0, 48.0], [thr, 0.5 * rv])
            with pytest.raises(L.LbmError):
                sim.axis_interface([48.0, 96.0], [thr, thr])
        assert np.isnan(z[1])
        got[prec] = z[0]
    print(f"axis interface: oracle {z_o:.12f}, FP64 {got[0]:.12f}, FP32 {got[1]:.9f}", flush=True)
    assert 48.0 + 12.0 < z_o < 48.0 + 24.0
    assert got[0] == pytest.approx(z_o, rel=1e-10)
    assert got[1] == pytest.approx(z_o, abs=1e-3)


def test_checkpoint_round_trip_bitwise():
    L = lbm()
    d = base(64, 32, A=-0.152)
    rho0 = droplet_rho(d, 10.0, eps=0.1)
    for prec in (0, 1):
        with L.LbmAxi(gpu_params(d), rho0, precision=prec) as a:
            a.step(40)
            ref = a.get_f()
            a.step(40)
            full = a.get_f()
        with L.LbmAxi(gpu_params(d), rho0, precision=prec) as b:
            b.set_f(ref)
            assert np.array_equal(b.get_f(), ref)
            b.step(40)
            assert np.array_equal(b.get_f(), full)


def test_batch_members_equal_single_runs_bitwise():
    L = lbm()
    ds = [base(64, 32), base(40, 24, tau=0.7, A=-0.1), base(100, 50, axisym=0, bc_top=1),
          base(24, 12, T=0.9 * base(1, 1)["T"] / 0.8)]
    rhos = [droplet_rho(d, 0.3 * d["nr"], eps=0.1 * (k % 2), seed=10 + k) for k, d in enumerate(ds)]
    for prec in (0, 1):
        with L.LbmAxi([gpu_params(d) for d in ds], rhos, precision=prec) as bat:
            assert bat.get_launch()["persistent"] == 1
            bat.step(60)
            fb = [bat.get_f(k) for k in range(len(ds))]
            mb = bat.mass()
        for k, d in enumerate(ds):
            with L.LbmAxi(gpu_params(d), rhos[k], precision=prec) as one:
                one.step(60)
                assert np.array_equal(one.get_f(), fb[k]), (prec, k)
                assert one.mass()[0] == mb[k]
        # one workgroup per item in each of the three item orders (XCD runs, longest first,
        # longest first with row bands kept on one XCD): the same result bitwise
        for xs in (0, 1, 2):
            with L.LbmAxi([gpu_params(d) for d in ds], rhos, precision=prec) as bat:
                bat.set_launch(width=64, seg_rows=10, persistent=0, grid=0, xcd_swizzle=xs, regf=xs & 1)
                bat.step(60)
                for k in range(len(ds)):
                    assert np.array_equal(bat.get_f(k), fb[k]), (prec, xs, k)
        # the members split over two to four stream groups, stepped eagerly and through
        # graph replays (an odd eager remainder between replays), persistent or not
        for ns, pers, chunk in ((2, 0, 0), (3, 1, 0), (4, 0, 10), (2, 1, 10)):
            with L.LbmAxi([gpu_params(d) for d in ds], rhos, precision=prec) as bat:
                bat.set_launch(width=128, seg_rows=16, persistent=pers, grid=0, xcd_swizzle=2, regf=1,
                               streams=ns)
                assert bat.get_launch()["streams"] == ns
                bat.set_graph_chunk(chunk)
                for n in (25, 1, 20, 14):
                    bat.step(n)
                bat.sync()
                assert bat.mass().tolist() == mb.tolist(), (prec, ns)
                for k in range(len(ds)):
                    assert np.array_equal(bat.get_f(k), fb[k]), (prec, ns, pers, chunk, k)


def test_mixed_forcing_batch_equals_single_runs_bitwise():
    # A batch with exact-difference and Guo members runs the kernel that branches per
    # instance; every member must equal its own single run (the exact-difference one on the
    # kernel compiled without Guo's branch).
    L = lbm()
    ds = [base(64, 32, A=-0.152), base(48, 30, forcing=1, A=-0.152), base(40, 24, forcing=1, axisym=0)]
    rhos = [droplet_rho(d, 0.3 * d["nr"], eps=0.1, seed=20 + k) for k, d in enumerate(ds)]
    for prec in (0, 1):
        with L.LbmAxi([gpu_params(d) for d in ds], rhos, precision=prec) as bat:
            bat.step(50)
            fb = [bat.get_f(k) for k in range(len(ds))]
        for k, d in enumerate(ds):
            with L.LbmAxi(gpu_params(d), rhos[k], precision=prec) as one:
                one.step(50)
                assert np.array_equal(one.get_f(), fb[k]), (prec, k)


def test_autotune_restores_the_state():
    # The tuner times every candidate shape (stream groups included) on the handle's own
    # state and restores it after each: after tuning, the state is bitwise the one before,
    # the error words are clean, and further steps in the chosen shape give bitwise what an
    # untuned handle gives.
    L = lbm()
    ds = [base(64, 32), base(40, 24, tau=0.7, A=-0.1), base(24, 12)]
    rhos = [droplet_rho(d, 0.3 * d["nr"], eps=0.1, seed=30 + k) for k, d in enumerate(ds)]
    with L.LbmAxi([gpu_params(d) for d in ds], rhos, precision=1) as ref:
        ref.step(31)
        want = [ref.get_f(k) for k in range(len(ds))]
    with L.LbmAxi([gpu_params(d) for d in ds], rhos, precision=1) as sim:
        sim.step(11)
        before = [sim.get_f(k) for k in range(len(ds))]
        launch, ms = sim.autotune(1)
        print("tuned", launch, ms, flush=True)
        assert ms > 0 and sim.get_launch() == launch
        assert all(np.array_equal(sim.get_f(k), b) for k, b in enumerate(before))
        assert not sim.errors().any()
        sim.set_graph_chunk(4)
        sim.step(20)
        assert all(np.array_equal(sim.get_f(k), w) for k, w in enumerate(want))


def test_graph_replays_after_an_odd_number_of_steps():
    # A captured chunk reads and writes fixed buffers; after an odd eager remainder the state
    # sits in the other buffer, so the replays must use the chunk captured from there.
    L = lbm()
    d = base(80, 40)
    rho0 = droplet_rho(d, 12.0, eps=0.1)
    with L.LbmAxi(gpu_params(d), rho0) as a:
        a.step(57)
        ref = a.get_f()
    with L.LbmAxi(gpu_params(d), rho0) as b:
        b.set_graph_chunk(10)
        b.step(13)                  # 1 replay + 3 eager: state in the other buffer
        b.step(20)                  # 2 replays of the chunk captured from that buffer
        b.step(11)                  # 1 replay + 1 eager: back to the first buffer
        b.step(13)
        assert np.array_equal(b.get_f(), ref)


def test_graph_replay_equals_eager_and_repeats():
    L = lbm()
    d = base(80, 40)
    rho0 = droplet_rho(d, 12.0, eps=0.1)
    with L.LbmAxi(gpu_params(d), rho0) as a:
        a.step(100)
        ref = a.get_f()
    with L.LbmAxi(gpu_params(d), rho0) as b:
        b.set_graph_chunk(10)
        b.step(30)                  # 3 replays of one captured graph
        b.sync()
        b.step(64)                  # 6 replays + 4 eager steps
        b.step(6)
        assert np.array_equal(b.get_f(), ref)


def test_fp32_form_static_droplet_laplace():
    # FP32 storage and arithmetic (EOS and psi in FP64, FP64 reductions) on the static droplet
    # for its full 2000 steps: the Laplace pressure jump within 1 % of the FP64 oracle; field
    # and mass errors reported.
    L = lbm()
    d = base(128, 64)
    rho0 = droplet_rho(d, 20.0, noise=1e-4, seed=1)
    po = oracle_params(d)
    f = O.init(po, rho0)
    m0 = O.mass(po, f)
    O.step(po, f, 2000)
    with L.LbmAxi(gpu_params(d), rho0, precision=1) as sim:
        sim.step(2000)
        m32 = sim.mass()[0]
        dp32 = sim.laplace(64.0, 10.0, 32.0)[0]
        rg, uzg, urg = sim.moments()
    dp64 = O.laplace(po, f, 64.0, 10.0, 32.0)
    ro, uzo, uro = O.moments(po, f)
    uscale = max(np.abs(uzo).max(), np.abs(uro).max())
    print("fp32 static droplet: rho", rel_inf(rg, ro), "u", np.abs(uzg - uzo).max() / uscale,
          np.abs(urg - uro).max() / uscale, "dp", dp32 / dp64 - 1, "mass",
          (m32 - O.mass(po, f)) / m0, flush=True)
    assert dp32 == pytest.approx(dp64, rel=1e-2)
    assert rel_inf(rg, ro) < 1e-3
    # the droplet's axisymmetric mass is not conserved (the FP64 run itself drifts ~1e-4):
    # FP32 round-off moves it along a slightly different trajectory
    assert abs(m32 - O.mass(po, f)) / m0 < 1e-4


def test_fp32_form_density_wave_mass_trace():
    # Radial density wave in the vapour (T/Tc = 0.9, tau = 0.7, no-slip wall, Sec. 3.3):
    # |M_fp32(t) - M_fp64(t)| / M(0) <= 1e-6 along the run.
    L = lbm()
    from paper_1512_01977_amd import inputs
    d = base(8, 256, T=0.9 * base(1, 1)["T"] / 0.8, tau=0.7, bc_top=1)
    rv, _, _ = O.coexistence(oracle_params(d))
    rho0 = inputs.radial_wave(8, 256, rv, amplitude=1e-2, wavelength=64.0, noise=1e-6, seed=3)
    po = oracle_params(d)
    f = O.init(po, rho0)
    m0 = O.mass(po, f)
    worst = 0.0
    with L.LbmAxi(gpu_params(d), rho0, precision=1) as sim:
        for _ in range(4):
            O.step(po, f, 250)
            sim.step(250)
            worst = max(worst, abs(sim.mass()[0] - O.mass(po, f)) / m0)
    print("fp32 wave mass trace error", worst, "oracle drift", O.mass(po, f) / m0 - 1, flush=True)
    assert worst <= 1e-6


def test_device_reports_eos_domain_error():
    # CS at T/Tc = 0.485 with a five-node interface leaves the psi-real range within a few
    # steps (the oracle raises the same error); the device flags it, no fault.
    L = lbm()
    d = base(64, 32, T=0.485 * base(1, 1)["T"] / 0.8, tau=0.8)
    rho0 = droplet_rho(d, 10.0)
    po = oracle_params(d)
    f = O.init(po, rho0)
    with pytest.raises(O.OracleError):
        O.step(po, f, 200)
    with L.LbmAxi(gpu_params(d), rho0) as sim:
        sim.step(200)
        with pytest.raises(L.LbmError) as e:
            sim.sync()
        assert e.value.code in (-4, -5)


def test_autotune_keeps_a_raised_error():
    # The state of the case above leaves the EOS domain; autotuning the handle afterwards
    # must neither clear the sticky error nor touch the state or the launch shape.
    L = lbm()
    d = base(64, 32, T=0.485 * base(1, 1)["T"] / 0.8, tau=0.8)
    with L.LbmAxi(gpu_params(d), droplet_rho(d, 10.0)) as sim:
        sim.step(200)
        with pytest.raises(L.LbmError) as e0:
            sim.sync()
        keep = sim.get_launch()
        flags0 = sim.errors()
        with pytest.raises(L.LbmError) as e:
            sim.autotune(1)
        assert e.value.code == e0.value.code
        with pytest.raises(L.LbmError) as e:
            sim.sync()
        assert e.value.code == e0.value.code
        assert np.array_equal(sim.errors(), flags0)
        assert sim.get_launch() == keep


@pytest.mark.parametrize("streams", [1, 2])
def test_error_in_one_member_leaves_the_others_readable(streams):
    # A batch of a failing member (as above) and a sound one: the handle-wide sync reports
    # the error, the flags name the failing member only, and the sound member still reads
    # back bitwise equal to its single-instance run; also with the two members stepped on
    # two streams, whose launches share the error words.
    L = lbm()
    bad = base(64, 32, T=0.485 * base(1, 1)["T"] / 0.8, tau=0.8)
    good = base(64, 32)
    rb, rg = droplet_rho(bad, 10.0), droplet_rho(good, 10.0, seed=3)
    with L.LbmAxi([gpu_params(bad), gpu_params(good)], [rb, rg]) as sim:
        if streams > 1:
            sim.set_launch(width=128, seg_rows=16, persistent=0, grid=0, xcd_swizzle=2, regf=1,
                           streams=streams)
            sim.set_graph_chunk(20)
        sim.step(200)
        with pytest.raises(L.LbmError):
            sim.sync()
        flags = sim.errors()
        assert flags[0] != 0 and flags[1] == 0
        with pytest.raises(L.LbmError):
            sim.moments(0)
        mg = sim.moments(1)
        fg = sim.get_f(1)
    with L.LbmAxi(gpu_params(good), rg) as one:
        one.step(200)
        assert np.array_equal(one.get_f(), fg)
        assert all(np.array_equal(a, b) for a, b in zip(one.moments(), mg))


def test_host_rejects_bad_input():
    L = lbm()
    d = base(16, 8, T=0.485 * base(1, 1)["T"] / 0.8)
    with pytest.raises(L.LbmError) as e:
        L.LbmAxi(gpu_params(d), np.full((8, 16), 0.6))
    assert e.value.code == -4
    with pytest.raises(L.LbmError) as e:
        L.LbmAxi(gpu_params(base(16, 8, tau=0.4)), np.full((8, 16), 0.1))
    assert e.value.code == -1
    with pytest.raises(L.LbmError) as e:   # an empty batch
        L.LbmAxi([], [])
    assert e.value.code == -1
    with L.LbmAxi(gpu_params(base(16, 8)), np.full((8, 16), 0.1)) as sim:
        f0 = sim.get_f()
        sim.step(0)                        # zero steps: nothing runs, the state is unchanged
        sim.sync()
        assert np.array_equal(sim.get_f(), f0)
        with pytest.raises(L.LbmError) as e:
            sim.step(-1)
        assert e.value.code == -1
        keep = sim.get_launch()
        for bad_launch in (dict(xcd_swizzle=3), dict(xcd_swizzle=-1), dict(regf=2), dict(seg_rows=5),
                           dict(streams=2), dict(streams=-1)):
            with pytest.raises(L.LbmError) as e:
                sim.set_launch(**{**keep, **bad_launch})
            assert e.value.code == -1, bad_launch
        assert sim.get_launch() == keep
    two = [gpu_params(base(16, 8)), gpu_params(base(24, 8))]
    with L.LbmAxi(two, [np.full((8, 16), 0.1), np.full((8, 24), 0.1)]) as sim:
        keep = sim.get_launch()
        for bad in (3, 5):          # more groups than instances; more than four
            with pytest.raises(L.LbmError) as e:
                sim.set_launch(**{**keep, "streams": bad})
            assert e.value.code == -1, bad
        sim.set_launch(**{**keep, "streams": 2})
        assert sim.get_launch()["streams"] == 2
