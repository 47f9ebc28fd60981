"""CPU checks of the step kernel's work lists as the library builds them (the host code in
paper_1512_01977_amd/csrc/work_items.h, compiled into a small test program): the items of a
launch cover every node of every instance exactly once, strips are whole 128-byte lines,
segments respect the 2 GiB descriptor cap, each item order keeps its promise, and a batch
split into stream groups gives every instance to one group with balanced node counts."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
XCDS = 8


@pytest.fixture(scope="module")
def lister(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("work_items") / "check")
    cmd = ["hipcc", "-std=c++17", "-O1", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_1512_01977_amd", "csrc"),
           os.path.join(ROOT, "tests", "work_items_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def work_list(lister, esize, width, seg, persistent, xcd, streams, members):
    spec = f"{esize} {width} {seg} {persistent} {xcd} {streams} {len(members)}\n" + \
           "".join(f"{nz} {nr}\n" for nz, nr in members)
    out = subprocess.run([lister], input=spec, capture_output=True, text=True, check=True).stdout.split("\n")
    groups = [tuple(map(int, out[g].split())) for g in range(streams)]
    items = np.array([list(map(int, l.split())) for l in out[streams:] if l.strip()], dtype=np.int64)
    return groups, items.reshape(-1, 5)


def cost(it):  # rows swept by an item, pipeline rows included (the order key)
    return (it[:, 4] - it[:, 3]) + np.minimum(6, it[:, 3]) + 6


def check_list(lister, esize, width, seg, persistent, xcd, streams, members):
    groups, items = work_list(lister, esize, width, seg, persistent, xcd, streams, members)
    line = 128 // esize
    wout = (width - 12) // line * line
    # seven halo lanes on either side (the link-midpoint source's pipeline) fit as well
    assert wout + 14 <= width and wout == (width - 14) // line * line
    # stream groups: contiguous ranges covering the list, each instance in exactly one
    assert groups[0][1] == 0 and sum(g[2] for g in groups) == len(items)
    for a, b in zip(groups, groups[1:]):
        assert b[1] == a[1] + a[2]
    owner = {}
    for g, first, count in groups:
        assert count > 0
        for inst in set(items[first:first + count, 0].tolist()):
            assert inst not in owner
            owner[inst] = g
    assert sorted(owner) == list(range(len(members)))
    if streams > 1:  # greedy largest-first split: loads differ by at most the largest member
        load = np.zeros(streams)
        for inst, g in owner.items():
            load[g] += members[inst][0] * members[inst][1]
        assert load.max() - load.min() <= max(nz * nr for nz, nr in members)
    # strips of whole lines, segments within the cap, every node exactly once
    for inst, (nz, nr) in enumerate(members):
        mine = items[items[:, 0] == inst]
        pitch = -(-nz // line) * line
        pitch += line if pitch * esize % 2048 == 0 else 0   # no power-of-two plane stride
        cap = (1 << 31) // (9 * pitch * esize) - 16
        seg_eff = min(seg if seg > 0 else nr, cap)
        assert np.all(mine[:, 1] % line == 0)
        assert np.all(mine[:, 2] == np.minimum(wout, nz - mine[:, 1]))
        assert np.all(mine[:, 3] % seg_eff == 0) and np.all(mine[:, 4] - mine[:, 3] <= seg_eff)
        assert np.all(mine[:, 4] == np.minimum(nr, mine[:, 3] + seg_eff))
        cover = np.zeros((nr, nz), dtype=np.int32)
        for _, k0, nc, s, e in mine:
            cover[s:e, k0:k0 + nc] += 1
        assert np.all(cover == 1), (inst, nz, nr)
    # orders
    for g, first, count in groups:
        part = items[first:first + count]
        if not persistent and xcd == 1:  # as built: instance, segment, strip
            key = part[:, 0] * (1 << 40) + part[:, 3] * (1 << 20) + part[:, 1]
            assert np.all(np.diff(key) > 0)
        elif persistent or xcd == 0:  # longest first
            assert np.all(np.diff(cost(part)) <= 0)
        else:  # XCD x runs positions x, x + 8, ... longest first; bands split <= once per XCD
            for x in range(XCDS):
                assert np.all(np.diff(cost(part[x::XCDS])) <= 0)
            bands = {}
            for p, (inst, _, _, s, _) in enumerate(part):
                bands.setdefault((inst, s), set()).add(p % XCDS)
            assert sum(len(v) - 1 for v in bands.values()) <= XCDS
    return groups, items


CASES = [
    # esize, width, seg, persistent, xcd_swizzle, streams, members
    (4, 128, 16, 0, 2, 2, [(64, 32), (40, 24), (100, 50), (24, 12)]),
    (8, 64, 8, 1, 0, 1, [(150, 37)]),
    (4, 256, 0, 0, 1, 1, [(150, 37)]),
    (8, 128, 9, 0, 0, 3, [(64, 32), (40, 24), (100, 50), (24, 12), (7, 5)]),
    (4, 64, 13, 0, 2, 4, [(64, 32), (40, 24), (100, 50), (24, 12), (1, 4), (2, 9)]),
    (8, 256, 96, 0, 2, 1, [(1000, 300)]),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"s{c[0]}w{c[1]}g{c[2]}p{c[3]}x{c[4]}n{c[5]}")
def test_work_list_properties(lister, case):
    check_list(lister, *case)


def test_benchmark_ensemble_work_list(lister):
    # the 256-member ensemble in the benchmark's shape (two stream groups, row bands on one
    # XCD) and in one launch longest first
    from paper_1512_01977_amd import inputs
    members = [(m.nz, m.nr) for m in inputs.ensemble(n=256, seed=151201977, tau_lo=0.7)]
    assert sum(nz * nr for nz, nr in members) == 12_889_106
    _, items = check_list(lister, 4, 256, 64, 0, 2, 2, members)
    check_list(lister, 4, 128, 112, 0, 0, 1, members)
    assert len(items) > 1000


def test_segment_cap_for_wide_fp64_rows(lister):
    # 16384-wide FP64 rows (pitch 16400 with the padding line): a row block is 1.18 MB, so a
    # work item may span at most 2^31 / (9 * 16400 * 8) - 16 = 1802 rows; whole-column segments
    # are split there.
    _, items = check_list(lister, 8, 256, 0, 0, 1, 1, [(16384, 4000)])
    assert (items[:, 4] - items[:, 3]).max() == 1802
