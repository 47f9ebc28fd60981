"""The allocation-free entry point lbm_axi_mass_async (partials in the library's static
device scratch) against lbm_axi_mass on the same states: bitwise equal, on two calls in a
row with the second on a smaller input, and a handle with more rows than the scratch holds
is refused.  Through the C ABI."""
import numpy as np
import pytest

from cases import base, droplet_rho, gpu_params

pytestmark = pytest.mark.gpu


def lbm():
    from paper_1512_01977_amd import lbm as L
    return L


def masses(sim, torch):
    out = torch.full((sim.n,), float("nan"), dtype=torch.float64, device="cuda")
    sim.mass_async(out)
    sim.sync()   # orders the handle's stream before the copy back
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_mass_async_equals_mass_on_two_calls(precision):
    import torch
    L = lbm()
    big = [base(96, 48), base(64, 32, A=-0.152), base(128, 64, bc_top=1), base(40, 24, source_mid=1)]
    small = [base(24, 12)]
    for ds, steps in ((big, 40), (small, 15)):     # the second call has fewer rows
        rhos = [droplet_rho(d, 0.3 * d["nr"], eps=0.1, seed=50 + k) for k, d in enumerate(ds)]
        with L.LbmAxi([gpu_params(d) for d in ds], rhos, precision=precision) as sim:
            sim.step(steps)
            want = sim.mass()
            got = masses(sim, torch)
            print("mass_async", precision, len(ds), got, flush=True)
            assert got.shape == want.shape and np.array_equal(got, want)
            sim.step(3)                             # and again after more steps
            assert np.array_equal(masses(sim, torch), sim.mass())


def test_mass_async_refuses_more_rows_than_the_scratch_holds():
    import torch
    L = lbm()
    nr = 131072 + 8          # one FP64 partial per row: just beyond 1 MiB
    d = base(1, nr, eos=0, tau=0.8)
    rho0 = np.full((nr, 1), 1.0)
    with L.LbmAxi(gpu_params(d), rho0, precision=1) as sim:
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(L.LbmError) as e:
            sim.mass_async(out)
        assert e.value.code == -6
        assert sim.mass()[0] == pytest.approx(np.pi * nr * nr, rel=1e-12)   # the plain entry point still works
