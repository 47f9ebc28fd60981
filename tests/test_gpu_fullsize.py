"""The benchmark workloads at full size, in the launch shapes bench.py times (the shape the
committed byte counters were taken in, else the tuner's pick), against the oracle on the
same seeded inputs (their temperatures and densities set through the oracle's EOS helpers,
which agree with the library's to rounding).

FP64 is held to the 1e-10 bar of the small-grid parity tests.  The FP32 form's field
errors against the FP64 oracle are printed and bounded at about ten times what FP32
rounding gives here (unit roundoff 6e-8, a few times 1e-8 per step in rho; measured
1.1e-6 in rho and 7e-6 of the velocity scale after 20 steps); its tolerances on the
physics (Laplace pressure, oscillation frequency, mass) are tested elsewhere.
"""
import numpy as np
import pytest

import bench
import oracle as O
from cases import OracleEOS, oparams

pytestmark = pytest.mark.gpu

ENSEMBLE_STEPS = 20
LARGE_STEPS = 2




def oracle_moments(p, rho0, steps):
    q = oparams(p)
    f = O.init(q, rho0)
    O.step(q, f, steps)
    return O.moments(q, f)


def field_errors(g, o):
    rg, uzg, urg = g
    ro, uzo, uro = o
    uscale = max(np.abs(uzo).max(), np.abs(uro).max(), 1e-300)
    return (float(np.abs(rg - ro).max() / np.abs(ro).max()),
            float(max(np.abs(uzg - uzo).max(), np.abs(urg - uro).max()) / uscale))


def run_gpu(wl, steps, chunk):
    from paper_1512_01977_amd import lbm, tuning
    single = len(wl.params) == 1
    with lbm.LbmAxi(wl.params[0] if single else wl.params, wl.rho0[0] if single else wl.rho0,
                    precision=wl.precision) as sim:
        rec = bench.traffic_record(wl.name, "f32" if wl.precision == lbm.PREC_FP32 else "f64")
        if rec and rec.get("launch"):
            sim.set_launch(**rec["launch"])
            launch = sim.get_launch()
        else:
            launch = tuning.choose_launch(sim, wl, tune=True, log=lambda *a: print(*a, flush=True))
        print("launch", launch, flush=True)
        if chunk:
            sim.set_graph_chunk(chunk)
        sim.step(steps)
        assert not sim.errors().any()
        return [sim.moments(k) for k in range(len(wl.params))]


@pytest.fixture(scope="module")
def ensemble_oracle():
    from paper_1512_01977_amd import workloads
    wl = workloads.ensemble(precision=0, eos=OracleEOS)
    return [oracle_moments(p, r, ENSEMBLE_STEPS) for p, r in zip(wl.params, wl.rho0)]


@pytest.mark.parametrize("precision", [0, 1])
def test_ensemble_full_size_bench_launch(precision, ensemble_oracle):
    # All 256 members (12 889 106 nodes, nr 32..256, ragged strips) after 20 steps run as
    # two 10-step graph replays, in the shape bench.py times for this precision.
    from paper_1512_01977_amd import workloads
    wl = workloads.ensemble(precision=precision, eos=OracleEOS)
    got = run_gpu(wl, ENSEMBLE_STEPS, 10)
    errs = np.array([field_errors(g, o) for g, o in zip(got, ensemble_oracle)])
    print(f"ensemble precision {precision}: max rho err {errs[:, 0].max():.3e}, "
          f"max u err {errs[:, 1].max():.3e} (of the member's velocity scale)", flush=True)
    if precision == 0:
        assert errs.max() <= 1e-10
    else:
        assert errs[:, 0].max() <= 1e-5 and errs[:, 1].max() <= 1e-4


@pytest.fixture(scope="module")
def large_oracle():
    from paper_1512_01977_amd import workloads
    wl = workloads.large_droplet(precision=0, eos=OracleEOS)
    return oracle_moments(wl.params[0], wl.rho0[0], LARGE_STEPS)


@pytest.mark.parametrize("precision", [0, 1])
def test_large_domain_full_size_bench_launch(precision, large_oracle):
    # The 16384 x 8192 droplet (134 217 728 nodes) after two steps, every node.
    from paper_1512_01977_amd import workloads
    wl = workloads.large_droplet(precision=precision, eos=OracleEOS)
    (g,) = run_gpu(wl, LARGE_STEPS, 0)
    er, eu = field_errors(g, large_oracle)
    print(f"large precision {precision}: rho err {er:.3e}, u err {eu:.3e}", flush=True)
    if precision == 0:
        assert max(er, eu) <= 1e-10
    else:
        assert er <= 5e-6 and eu <= 5e-5


SINGLE_STEPS = {"mode2": 20, "wave": 4}


@pytest.fixture(scope="module")
def single_oracle():
    from paper_1512_01977_amd import workloads
    out = {}
    for name, steps in SINGLE_STEPS.items():
        wl = workloads.REGISTRY[name](precision=0, eos=OracleEOS)
        out[name] = oracle_moments(wl.params[0], wl.rho0[0], steps)
    return out


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", sorted(SINGLE_STEPS))
def test_single_domain_workloads_full_size(name, precision, single_oracle):
    # The mode-2 droplet at density ratio ~1e3 (1024 x 512, 524 288 nodes) after 20 steps and
    # the density wave (4096 x 2048 with a no-slip wall, 8 388 608 nodes) after 4 steps, every
    # node against the oracle, in the tuner's launch shape for the workload.
    # The FP32 velocity is bounded in lattice units: the momentum is a sum of FP32 populations
    # of size ~w_i rho, so u carries an absolute rounding error of order the FP32 unit
    # roundoff whatever its own size (the wave starts at rest: after 4 steps its velocity scale
    # is small enough for that to be 2e-4 of it).
    from paper_1512_01977_amd import workloads
    wl = workloads.REGISTRY[name](precision=precision, eos=OracleEOS)
    (g,) = run_gpu(wl, SINGLE_STEPS[name], 0)
    er, eu = field_errors(g, single_oracle[name])
    ua = max(float(np.abs(g[1] - single_oracle[name][1]).max()), float(np.abs(g[2] - single_oracle[name][2]).max()))
    print(f"{wl.name} precision {precision}: rho err {er:.3e}, u err {eu:.3e} of its scale, "
          f"{ua:.3e} absolute", flush=True)
    if precision == 0:
        assert max(er, eu) <= 1e-10
    else:
        assert er <= 5e-6 and ua <= 1e-6


def test_fp64_domain_beyond_four_gib_per_three_planes():
    # 16384 x 12288 in FP64 (201M nodes, 14.5 GB per distribution buffer): three direction
    # planes span 4.8 GB, more than 32-bit offsets reach from one base; the step kernel
    # rebases its descriptors per work item.  Whole-column segments (the segment cap then
    # splits each column), two steps, every node against the oracle.
    from paper_1512_01977_amd import lbm, workloads
    wl = workloads.large_droplet(precision=0, nz=16384, nr=12288, radius=2500.0, eos=OracleEOS)
    p, rho0 = wl.params[0], wl.rho0[0]
    with lbm.LbmAxi(p, rho0, precision=0) as sim:
        sim.set_launch(width=256, seg_rows=0, persistent=0, grid=0, xcd_swizzle=1, regf=0)
        sim.step(LARGE_STEPS)
        assert not sim.errors().any()
        g = sim.moments(0)
    er, eu = field_errors(g, oracle_moments(p, rho0, LARGE_STEPS))
    print(f"16384 x 12288 FP64: rho err {er:.3e}, u err {eu:.3e}", flush=True)
    assert max(er, eu) <= 1e-10
