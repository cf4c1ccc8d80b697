"""Host side of the residency probe: the interval reduction, and that each
probe kernel's gfx950 code object declares exactly the register count it
stands for (so a measured residency is the residency at that count)."""
import os
import re
import subprocess

import numpy as np

from paper_1701_08547_amd import build, probe


def test_max_overlap_by_brute_force():
    g = np.random.default_rng(3)
    for _ in range(200):
        n = int(g.integers(0, 30))
        s = g.integers(0, 50, n)
        e = s + g.integers(1, 20, n)
        brute = max([int(((s <= t) & (t < e)).sum()) for t in range(0, 80)] + [0])
        assert probe.max_overlap(s, e) == brute
    # touching intervals do not overlap
    assert probe.max_overlap(np.array([0, 10, 20]), np.array([10, 20, 30])) == 1
    assert probe.max_overlap(np.array([0, 0, 5]), np.array([10, 10, 6])) == 3


def test_concurrency_keys_by_compute_unit():
    # two CUs on XCC 0 and 1 with the same HW_ID: kept apart by the XCC id
    hw = (3 << 8) | 5
    rec = np.array([[0, 10, hw, 0], [1, 10, hw, 0], [2, 9, hw, 0],
                    [0, 10, hw, 1], [12, 20, hw, 1]], np.int64)
    c = probe.concurrency(rec)
    assert c["cus"] == 2 and c["max"] == 3 and c["min"] == 1
    # the wave and SIMD fields of HW_ID (bits 0..7) do not split a CU
    rec2 = rec.copy()
    rec2[1, 2] = hw | 0x3F
    assert probe.concurrency(rec2)["max"] == 3


def test_probe_kernels_declare_their_register_counts(tmp_path):
    out = str(tmp_path / "sa_probe.s")
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    subprocess.run([build.hipcc(), *flags, "-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC,
                    "--cuda-device-only", "-S", os.path.join(build.CSRC, "sa_probe.hip"), "-o", out], check=True)
    txt = open(out).read()
    meta = txt[txt.index("amdhsa.kernels:"):]
    found = {}
    # one metadata entry per kernel, each opening with its agpr count
    for entry in re.split(r"\n  - (?=\.agpr_count)", meta)[1:]:
        m = re.search(r"\.name:\s+\S*sa_residency_kernelILi(\d+)ELi(\d+)E", entry)
        if not m:
            continue
        vg = int(re.search(r"\.vgpr_count:\s+(\d+)", entry).group(1))
        ag = int(re.search(r"\.agpr_count:\s+(\d+)", entry).group(1))
        lds = int(re.search(r"\.group_segment_fixed_size:\s+(\d+)", entry).group(1))
        found[(int(m.group(1)), int(m.group(2)))] = (vg, ag, lds)
    want = {(lb, r) for lb, rs in probe.PROBES.items() for r in rs}
    assert set(found) == want
    for (lb, r), (vg, ag, lds) in found.items():
        assert vg == r, (lb, r, vg)
        assert ag == (256 if r == 512 else 0), (lb, r, ag)
        assert lds == 0
