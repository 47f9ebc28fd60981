"""The FP32 form (FP32 populations and arithmetic, FP64 EOS and reductions) against the
FP64 oracle directly, for the full step count of each benchmark configuration on an
analogue the oracle can run inside a test:

* the batched ensemble: members of the 256-member ensemble itself (those of at most 20 000
  nodes, small and large temperatures and relaxation times alike), 2000 steps, per-member
  Laplace pressure difference (tolerance 1 %);
* the density wave: the wave's full radial profile (2048 rows, a no-slip wall at r = nr)
  on 8 columns, 10 000 steps, the axisymmetric mass sum(2 pi r rho) every 1000 steps
  (tolerance 1e-6 of the initial mass);
* the mode-2 drop at density ratio ~1e3: the same EOS, lambda, A and tau on 256 x 128 with
  R = 30 (P2 amplitude 0.05), 20 000 steps, the drop's interface on the axis every 200 steps
  (tolerance 1 % of its excursion).  At this radius viscosity damps the mode within about a
  period (rate 5 nu / R^2 against a period of several thousand steps), which leaves a fitted
  frequency ill-conditioned, so the traces themselves are compared; the 1 % frequency
  criterion is checked at full size against the FP64 form (test_gpu_validation.py).

The oracle runs on the host threads next to the GPU; FP32-versus-FP64-GPU comparisons at
full size are in test_gpu_validation.py."""
import numpy as np
import pytest

import oracle as O
from cases import OracleEOS, oparams

pytestmark = pytest.mark.gpu


def lbm():
    from paper_1512_01977_amd import lbm as L
    return L


def test_ensemble_members_laplace_2000_steps():
    L = lbm()
    from paper_1512_01977_amd import workloads
    wl = workloads.ensemble(precision=L.PREC_FP32, eos=OracleEOS)
    pick = [k for k, p in enumerate(wl.params) if p.nz * p.nr <= 20000][:6]
    assert len(pick) == 6
    meta = [wl.meta["members"][k] for k in pick]
    zc, rin, rout = ([m["zc"] for m in meta], [m["R"] / 2 for m in meta], [m["R"] + 12 for m in meta])
    with L.LbmAxi([wl.params[k] for k in pick], [wl.rho0[k] for k in pick], precision=L.PREC_FP32) as s:
        s.set_graph_chunk(100)
        s.step(2000)
        dp32 = s.laplace(zc, rin, rout)
    rel = []
    for j, k in enumerate(pick):
        q = oparams(wl.params[k])
        f = O.init(q, wl.rho0[k])
        O.step(q, f, 2000)
        dp64 = O.laplace(q, f, zc[j], rin[j], rout[j])
        rel.append(abs(dp32[j] / dp64 - 1))
        print(f"member {k} ({q.nz}x{q.nr}, T/Tc {wl.params[k].T / 0.0943287031:.3f}, tau {q.tau:.3f}): "
              f"dp FP32 {dp32[j]:.6e}, oracle {dp64:.6e}, rel {rel[-1]:.2e}", flush=True)
    assert max(rel) <= 1e-2


def test_density_wave_mass_trace_10000_steps():
    L = lbm()
    from paper_1512_01977_amd import workloads
    wl = workloads.density_wave(precision=L.PREC_FP64, nz=8, nr=2048, eos=OracleEOS)
    p, rho0 = wl.params[0], wl.rho0[0]
    q = oparams(p)
    f = O.init(q, rho0)
    m0 = O.mass(q, f)
    worst = drift = 0.0
    with L.LbmAxi(p, rho0, precision=L.PREC_FP32) as s:
        s.set_graph_chunk(100)
        for _ in range(10):
            s.step(1000)
            O.step(q, f, 1000)
            m64 = O.mass(q, f)
            worst = max(worst, abs(s.mass()[0] - m64) / m0)
            drift = m64 / m0 - 1
    print(f"wave 8x2048, 10 000 steps: |M_FP32 - M_oracle| / M0 <= {worst:.2e}; "
          f"oracle drift {drift:+.2e}", flush=True)
    assert worst <= 1e-6


def test_mode2_ratio_1000_frequency_20000_steps():
    L = lbm()
    from paper_1512_01977_amd import inputs, workloads
    p = workloads.cs_params(256, 128, 0.485, 0.8, lam=0.05, A=-0.152, eos=OracleEOS)
    rv, rl = workloads.coexistence(p, OracleEOS)
    rho0 = inputs.droplet(256, 128, rv, rl, 30.0, zc=128.0, width=10.0, eps=0.05, noise=1e-4, seed=2)
    thr = 0.5 * (rv + rl)
    q = oparams(p)
    f = O.init(q, rho0)
    every = 200
    t, z32, z64 = [], [], []
    with L.LbmAxi(p, rho0, precision=L.PREC_FP32) as s:
        s.set_graph_chunk(every)
        for n in range(20000 // every):
            s.step(every)
            O.step(q, f, every)
            t.append((n + 1) * every)
            z32.append(s.axis_interface(128.0, thr)[0])
            z64.append(O.axis_interface(q, f, 128.0, thr))
    t, z32, z64 = map(np.asarray, (t, z32, z64))
    m = t >= 1000
    span = np.ptp(z64[m])
    diff = np.abs(z32 - z64).max()
    print(f"mode 2 ratio 1e3, 256x128 R 30: interface excursion {span:.3f} lu, FP32 - oracle max "
          f"{diff:.2e} lu ({diff / span:.2e} of it)", flush=True)
    assert span > 0.1 and diff <= 1e-2 * span
