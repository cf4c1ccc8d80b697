"""The static-vs-dynamic instruction-mix comparison (Sec. IV-B's error rates of
the instruction-mix metrics, the analog of its Table II check) recomputed on
the host: the static side from the library's own gfx950 assembly of the
measured kernel families, the dynamic side from the committed per-dispatch SQ
counter table of one rocprofv3 run; the error table in the profile summary
must be what these two give."""
import os
import re

import pytest

from paper_1701_08547_amd import imix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "profiles", "imix_runtime_families_counters.txt")
SUMMARY = os.path.join(ROOT, "profiles", "imix_runtime_families.md")
CLASSES = ("valu", "salu", "smem", "vmem_rd", "vmem_wr", "lds")


@pytest.fixture(scope="module")
def report():
    dyn = imix.read_table(TABLE)
    assert len(dyn) == len(imix.cases()) == 81
    return imix.compare(imix.predicted(imix.cases(), 256), dyn)


def test_summary_table_is_what_the_counters_give(report):
    rows = {}
    for line in open(SUMMARY):
        m = re.match(r"\| (matvec|stencil|reduce) \|(.*)\|\s*$", line)
        if m:
            cells = [c.strip() for c in m.group(2).split("|")]
            rows[m.group(1)] = cells
    assert set(rows) == {"matvec", "stencil", "reduce"}
    for fam, cells in rows.items():
        s = report["summary"][fam]
        for cls, cell in zip(CLASSES, cells):
            mean, mx = (float(x) for x in re.findall(r"[0-9.]+", cell))
            assert round(s[cls]["mean_abs_error"], 3) == mean, (fam, cls)
            assert round(s[cls]["max_abs_error"], 3) == mx, (fam, cls)
        assert cells[-1] == "exact" and s["waves_exact"]


def test_static_mix_properties(report):
    """Where the static count is exact by construction it is exact on the
    device: every family's wave count, the stencil within 0.4 %, the matvec's
    LDS (none); the reduction's one atomic per block is over-counted by the
    block's other waves (W_B - 1 per block)."""
    s = report["summary"]
    assert s["stencil"]["valu"]["max_abs_error"] < 0.005
    assert s["matvec"]["lds"]["max_abs_error"] == 0.0
    for r in report["cases"]:
        if r["family"] == "reduce":
            wb = -(-r["T"] // 64)
            assert r["vmem_wr"]["static"] - r["vmem_wr"]["dynamic"] == (wb - 1) * r["vmem_wr"]["dynamic"]
