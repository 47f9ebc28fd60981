"""CPU checks of the HIP library's host side: it loads, exports every entry point its
header declares, and its host EOS helpers agree with the independent oracle ones.
No kernel is launched here."""
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(lbm_axi_\w+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_1512_01977_amd import lbm
    L = lbm.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lbm.EXPORTS)


def header_structs():
    """Field lists (C type, name) of the typedef'd structs the header declares."""
    text = open(os.path.join(ROOT, "include", "lbm_axi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef\s+struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            ctype, names = decl.split(None, 1)
            fields += [(ctype, n.strip()) for n in names.split(",")]
        out[name] = fields
    return out


def test_binding_structs_mirror_the_header():
    # The ctypes structures passed by pointer through the ABI have the header's fields, in
    # its order and with its types (a missing or reordered field would shift every later one).
    import ctypes
    from paper_1512_01977_amd import lbm
    ctype_of = {"int32_t": ctypes.c_int32, "double": ctypes.c_double}
    structs = header_structs()
    for name in ("lbm_axi_params", "lbm_axi_launch"):
        want = [(n, ctype_of[t]) for t, n in structs[name]]
        got = [("lambda" if n == "lambda_" else n, t) for n, t in getattr(lbm, name)._fields_]
        assert got == want, name


def test_status_strings():
    from paper_1512_01977_amd import lbm
    L = lbm.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.lbm_axi_status_string(code)
    assert L.lbm_axi_status_string(-4).startswith(b"equation-of-state")


@pytest.mark.parametrize("t", [0.9, 0.8, 0.7, 0.55, 0.485])
def test_host_cs_coexistence_matches_oracle(t):
    from paper_1512_01977_amd import lbm
    pl = lbm.Params(nz=4, nr=4, eos=lbm.EOS_CS)
    rc, Tc, Pc = lbm.lbm_axi_eos_critical(pl)
    orc, oTc, oPc = O.critical(O.Params(nz=4, nr=4, eos=O.EOS_CS))
    assert Tc == pytest.approx(oTc, rel=1e-12)
    assert rc == pytest.approx(orc, rel=1e-7)
    pl.T = t * Tc
    rv, rl, ps = lbm.lbm_axi_eos_coexistence(pl)
    orv, orl, ops = O.coexistence(O.Params(nz=4, nr=4, eos=O.EOS_CS, T=t * oTc))
    assert rv == pytest.approx(orv, rel=1e-9)
    assert rl == pytest.approx(orl, rel=1e-12)
    assert ps == pytest.approx(ops, rel=1e-9)


@pytest.mark.parametrize("T", [0.9, 0.8, 0.7])
def test_host_vdw_coexistence_matches_oracle(T):
    from paper_1512_01977_amd import lbm
    rv, rl, ps = lbm.lbm_axi_eos_coexistence(lbm.Params(nz=4, nr=4, eos=lbm.EOS_VDW, lam=0.01, T=T))
    orv, orl, ops = O.coexistence(O.Params(nz=4, nr=4, eos=O.EOS_VDW, lam=0.01, T=T))
    assert (rv, rl, ps) == (pytest.approx(orv, rel=1e-9), pytest.approx(orl, rel=1e-9),
                            pytest.approx(ops, rel=1e-9))


def test_host_helpers_reject_bad_input():
    from paper_1512_01977_amd import lbm
    with pytest.raises(lbm.LbmError):
        lbm.lbm_axi_eos_coexistence(lbm.Params(nz=4, nr=4, eos=lbm.EOS_CS, T=1.0))  # above T_c
    with pytest.raises(lbm.LbmError):
        lbm.lbm_axi_eos_critical(lbm.Params(nz=4, nr=4, eos=lbm.EOS_IDEAL))


def test_ensemble_workload_shape():
    # The seeded ensemble: 256 members, nz = 2 nr, 12 889 106 nodes for seed 151201977.
    from paper_1512_01977_amd import inputs
    ens = inputs.ensemble()
    assert len(ens) == 256
    assert all(i.nz == 2 * i.nr and 32 <= i.nr <= 256 for i in ens)
    assert sum(i.nz * i.nr for i in ens) == 12_889_106
    assert all(0.55 <= i.t_reduced <= 0.9 for i in ens)


def test_tuning_size_class_keys():
    from paper_1512_01977_amd import lbm, tuning
    a = tuning.size_class([lbm.Params(nz=16384, nr=8192)], 1)
    b = tuning.size_class([lbm.Params(nz=16384, nr=8192)], 0)
    c = tuning.size_class([lbm.Params(nz=64, nr=32)] * 256, 1)
    assert a != b and a.startswith("gfx950:f32:single") and c.startswith("gfx950:f32:batch256")


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    from paper_1512_01977_amd import tuning
    monkeypatch.setenv("LBM_AXI_TUNING_CACHE", str(tmp_path / "sub" / "tuning.json"))
    key = "gfx950:f32:batch256:n23:z9"
    if tuning.lookup(key) is not None:  # a shipped entry takes precedence
        pytest.skip("a shipped tuning file holds this key")
    launch = dict(width=256, seg_rows=64, persistent=0, grid=0, xcd_swizzle=2, regf=1, streams=2)
    tuning.store(key, launch, 0.25)
    assert tuning.lookup(key) == {"launch": launch, "ms_per_step": 0.25}
    tuning.store("other", dict(launch, streams=1), 0.3)
    assert tuning.lookup(key)["launch"]["streams"] == 2 and tuning.lookup("other")["launch"]["streams"] == 1
    (tmp_path / "sub" / "tuning.json").write_text("not json")
    assert tuning.lookup(key) is None  # a damaged cache reads as empty


def test_workspace_sizing_and_offset_limit():
    # Two buffers; per instance nr row blocks of the nine planes, rows padded to 128 bytes,
    # the instance padded to 64 elements.  A work item's rows are addressed with 32-bit
    # offsets from one descriptor, so rows so wide that a 22-row item spans 2 GiB are
    # refused up front.
    import ctypes
    from paper_1512_01977_amd import lbm
    L = lbm.lib()

    def ws(nz, nr, prec):
        p = (lbm.lbm_axi_params * 1)(lbm.Params(nz=nz, nr=nr, eos=lbm.EOS_CS, T=0.05).c())
        nb = ctypes.c_size_t()
        return L.lbm_axi_workspace_bytes(1, p, prec, ctypes.byref(nb)), nb.value

    st, nb = ws(16384, 8192, lbm.PREC_FP64)             # a 128 KiB pitch gets one more line
    assert st == 0 and nb == 2 * 9 * 8 * 16400 * 8192
    st, nb = ws(100, 7, lbm.PREC_FP32)                  # rows of 128 floats: 9 * 128 * 7 = 8064
    assert st == 0 and nb == 2 * 4 * 8064
    st, nb = ws(100, 7, lbm.PREC_FP64)                  # rows of 112 doubles: 7056 -> 7104
    assert st == 0 and nb == 2 * 8 * 7104
    assert ws(16384, 11000, lbm.PREC_FP64)[0] == 0
    assert ws(1 << 21, 4, lbm.PREC_FP64)[0] == -6      # 22 row blocks of 151 MB exceed 2 GiB
    assert ws(1 << 21, 4, lbm.PREC_FP32)[0] == 0
    assert ws(16384, 3, lbm.PREC_FP32)[0] == -1         # nr < 4
    assert ws(0, 8, lbm.PREC_FP32)[0] == -1             # nz < 1
    assert ws(16, 8, 2)[0] == -1                        # unknown precision
    nb = ctypes.c_size_t()
    p = (lbm.lbm_axi_params * 1)(lbm.Params(nz=16, nr=8, eos=lbm.EOS_CS, T=0.05).c())
    assert L.lbm_axi_workspace_bytes(0, p, lbm.PREC_FP32, ctypes.byref(nb)) == -1   # empty batch
    assert L.lbm_axi_workspace_bytes(1, None, lbm.PREC_FP32, ctypes.byref(nb)) == -1
    bad_tau = (lbm.lbm_axi_params * 1)(lbm.Params(nz=16, nr=8, tau=0.5, eos=lbm.EOS_CS, T=0.05).c())
    assert L.lbm_axi_workspace_bytes(1, bad_tau, lbm.PREC_FP32, ctypes.byref(nb)) == -1


def test_coexistence_zero_crossing():
    # the A-calibration's root finder: linear interpolation between the bracketing grid
    # points, non-finite entries (members that left the EOS domain) skipped
    import numpy as np
    from paper_1512_01977_amd import coexistence as C
    assert C.zero_crossing([-0.3, -0.2, -0.1, 0.0], [0.3, 0.1, -0.1, -0.3]) == pytest.approx(-0.15)
    assert C.zero_crossing([-0.3, -0.2, -0.1], [0.4, 0.1, -0.2]) == pytest.approx(-0.2 + 0.1 / 3)
    assert C.zero_crossing([0.0, 1.0, 2.0], [np.nan, 1.0, -1.0]) == pytest.approx(1.5)
    assert np.isnan(C.zero_crossing([0.0, 1.0, 2.0], [2.0, np.nan, -1.0]))  # a gap is not bridged
    assert np.isnan(C.zero_crossing([0.0, 1.0], [1.0, 2.0]))
    assert C.zero_crossing([0.0, 1.0], [0.0, 2.0]) == 0.0


def test_bench_traffic_belongs_to_its_kernel_and_shape(monkeypatch):
    # The committed byte counts are used only for the kernel source they were taken on and
    # only in the launch shape recorded with them (a missing stream count reads as one).
    import bench
    rec = bench.traffic_record("droplet_ensemble_256", "f32")
    assert rec is not None and rec["bytes_per_launch"] > 0 and rec["launch"]
    shape = dict(rec["launch"])
    assert bench.same_launch(shape, shape)
    assert bench.same_launch({k: v for k, v in shape.items() if k != "streams"}, {**shape, "streams": 1})
    assert bench.same_launch(shape, {**shape, "streams": 1}) == (shape.get("streams", 1) == 1)
    assert not bench.same_launch(shape, {**shape, "seg_rows": shape["seg_rows"] + 8})
    assert not bench.same_launch(None, shape)
    assert bench.traffic_record("no_such_workload", "f32") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.traffic_record("droplet_ensemble_256", "f32") is None


def test_kernel_hash_ignores_comments_and_layout():
    import bench
    code = "int f(int x) {  // doubles\n  return 2 * x; /* the value */\n}\n"
    assert bench.code_text(code) == bench.code_text("int f(int x) {\n\n\treturn 2 * x;\n}")
    assert bench.code_text(code) != bench.code_text("int f(int x) { return 3 * x; }")


def test_bench_refuses_more_than_one_gpu():
    # The method's kernel is measured on one GPU; asking for several exits with a message
    # before anything touches a device.
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_bench_needs_a_gpu():
    # No CPU fallback: without a visible GPU the benchmark refuses to run.
    import subprocess
    import sys
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "needs a GPU" in r.stderr and r.stdout == ""


def test_binding_fails_loudly_without_its_library_or_a_gpu(monkeypatch, tmp_path):
    # No fallback path: a missing library is an error, and so is a handle without a GPU.
    import numpy as np
    from paper_1512_01977_amd import lbm
    monkeypatch.setattr(lbm, "_lib", None)
    monkeypatch.setattr(lbm, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="missing"):
        lbm.lib()
    monkeypatch.undo()
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError, match="no GPU"):
            lbm.LbmAxi(lbm.Params(nz=16, nr=8, eos=lbm.EOS_CS, T=0.05), np.full((8, 16), 0.1))


def test_committed_traffic_figures_are_consistent():
    # profiles/traffic.json: the scale factors come from the copy kernel of known size, each
    # workload's bytes from its counters and those factors, and its algorithmic bytes from
    # its node count (9 populations read and written, S bytes each).
    import json
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    cal = d["calibration"]
    kib = cal["copy_bytes"] / 1024
    assert abs(cal["fetch_scale"] - kib / cal["FETCH_SIZE_kib"]) < 1e-12
    assert abs(cal["write_scale"] - kib / cal["WRITE_SIZE_kib"]) < 1e-12
    nodes = {"droplet_ensemble_256": 12_889_106, "large_droplet_16384x8192": 16384 * 8192}
    for key, rec in d.items():
        if ":" not in key:
            continue
        workload, dtype = key.split(":")
        S = 4 if dtype == "f32" else 8
        assert rec["algorithmic_bytes_per_launch"] == 2 * 9 * S * nodes[workload]
        assert abs(rec["read_bytes"] - rec["FETCH_SIZE_kib"] * cal["fetch_scale"] * 1024) < 1.0
        assert abs(rec["write_bytes"] - rec["WRITE_SIZE_kib"] * cal["write_scale"] * 1024) < 1.0
        assert abs(rec["bytes_per_launch"] - rec["read_bytes"] - rec["write_bytes"]) < 1.0
        assert rec["dispatches_per_step"] == rec["launch"].get("streams", 1)
        # no form reads or writes less than the populations it must move
        assert rec["read_over_algorithmic"] >= 1.0 and rec["write_over_algorithmic"] >= 1.0
