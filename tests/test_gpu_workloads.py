"""The shipped benchmark workloads stay inside the EOS domain (psi real, finite) on the GPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_ensemble_runs_clean(precision):
    from paper_1512_01977_amd import lbm, workloads
    wl = workloads.ensemble(precision=precision)
    with lbm.LbmAxi(wl.params, wl.rho0, precision=precision) as sim:
        m0 = sim.mass()
        sim.set_graph_chunk(100)
        sim.step(2000)
        assert not sim.errors().any(), np.nonzero(sim.errors())
        m1 = sim.mass()
    assert np.all(np.isfinite(m1))
    # each member keeps its axisymmetric mass to well under a per cent
    assert np.abs(m1 / m0 - 1).max() < 1e-2


@pytest.mark.parametrize("name,steps", [("mode2", 2000), ("large", 300), ("wave", 300)])
def test_single_domain_workloads_run_clean(name, steps):
    from paper_1512_01977_amd import lbm, workloads
    wl = workloads.REGISTRY[name](precision=lbm.PREC_FP32)
    print("workload", wl.name, wl.nodes, flush=True)
    with lbm.LbmAxi(wl.params[0], wl.rho0[0], precision=wl.precision) as sim:
        m0 = sim.mass()[0]
        sim.set_graph_chunk(100)
        sim.step(steps)
        assert not sim.errors().any()
        m1 = sim.mass()[0]
    assert abs(m1 / m0 - 1) < 1e-2
