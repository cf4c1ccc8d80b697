"""Static instruction mix of this library's own gfx950 kernels, read from the
assembly the build writes (``sa_runtime_gfx950.s``).

The paper derives its model inputs by statically analysing each kernel
variant's machine code: instruction counts by category, registers and shared
memory per thread block (Sec. III, Sec. IV-C).  Here the same is done for the
measured kernel families, on AMD code objects built in this tree:

  * n_fp   vector floating-point arithmetic (f16/bf16/f32/f64 operations,
           transcendentals, float compares), conversions excluded
  * n_int  other vector ALU operations: integer, bitwise, compares,
           selects, conversions
  * n_ld   vector memory loads: global / buffer / flat, LDS reads
  * n_st   vector memory stores and atomics, LDS writes
  * n_br   scalar branches (s_cbranch_*, s_branch, s_setpc)
  * n_bar  workgroup barriers (s_barrier)
  * n_reg  register moves (v_mov*, v_accvgpr_*) and scratch accesses
Scalar ALU and scalar-memory instructions execute once per wave, not per
thread, and are not counted (except the branches and barriers above).

Counts are per basic-block group: instructions outside every loop, and per
loop (loops as the compiler annotates them, in program order).  A thread's
dynamic count is the outside count plus each loop's count times its trip
count.  Divergence d is the trip-weighted share of vector instructions in
loops that run under an exec mask opened inside a loop (a branch of the
loop body), the static stand-in for the fraction of the issue stream that
executes both sides of a branch.
"""
from __future__ import annotations

import os
import re
from dataclasses import dataclass, field

import yaml

CATEGORIES = ("n_fp", "n_int", "n_ld", "n_st", "n_br", "n_bar", "n_reg")
# issue classes of the hardware's per-wave instruction counters
HW_CLASSES = ("valu", "salu", "smem", "vmem_rd", "vmem_wr", "lds", "branch")

_FLOAT_TYPES = ("_f16", "_bf16", "_f32", "_f64")
_LABEL = re.compile(r"^(\.LBB\d+_\d+|; %bb\.\d+):?")
_HEADER = re.compile(r"Loop Header: Depth=(\d+)")
_IN_LOOP = re.compile(r"in Loop: Header=(BB\d+_\d+) Depth=(\d+)")


def category(mnemonic: str) -> str | None:
    """Category of one instruction mnemonic, None when not counted."""
    m = mnemonic.lower()
    if m.startswith("s_"):
        if m.startswith("s_cbranch") or m in ("s_branch", "s_setpc_b64"):
            return "n_br"
        if m == "s_barrier":
            return "n_bar"
        return None
    if m.startswith("scratch_") or m.startswith("v_mov") or m.startswith("v_accvgpr"):
        return "n_reg"
    if m.startswith(("global_load", "buffer_load", "flat_load", "ds_read", "ds_load")):
        return "n_ld"
    if m.startswith(("global_store", "buffer_store", "flat_store", "ds_write", "ds_store", "global_atomic",
                     "buffer_atomic", "flat_atomic", "ds_add", "ds_sub", "ds_max", "ds_min", "ds_and", "ds_or",
                     "ds_xor", "ds_inc", "ds_dec", "ds_cmpst", "ds_wrxchg")):
        return "n_st"
    if m.startswith("v_"):
        if m.startswith("v_cvt"):
            return "n_int"
        base = m.split("_e32")[0].split("_e64")[0].split("_dpp")[0].split("_sdwa")[0]
        if any(t in base for t in _FLOAT_TYPES) or base.startswith(("v_rcp", "v_rsq", "v_sqrt", "v_exp", "v_log",
                                                                     "v_sin", "v_cos", "v_mfma")):
            return "n_fp"
        return "n_int"
    return None


def hw_class(mnemonic: str) -> str | None:
    """Issue class of one instruction as the per-wave hardware counters see
    it (vector ALU including moves and MFMA, scalar ALU, scalar memory,
    vector memory reads / writes, LDS, branches); None for the rest (waits,
    barriers, no-ops, end of program)."""
    m = mnemonic.lower()
    if m.startswith("v_"):
        return "valu"
    if m.startswith("ds_"):
        return "lds"
    if m.startswith(("global_load", "buffer_load", "flat_load", "scratch_load")):
        return "vmem_rd"
    if m.startswith(("global_store", "buffer_store", "flat_store", "scratch_store", "global_atomic", "buffer_atomic",
                     "flat_atomic")):
        return "vmem_wr"
    if m.startswith(("s_load", "s_buffer_load", "s_scratch_load", "s_dcache", "s_memtime", "s_memrealtime")):
        return "smem"
    if m.startswith("s_cbranch") or m in ("s_branch", "s_setpc_b64", "s_swappc_b64"):
        return "branch"
    if m.startswith(("s_waitcnt", "s_barrier", "s_nop", "s_endpgm", "s_sleep", "s_setprio", "s_sendmsg", "s_trap",
                     "s_icache", "s_ttrace", "s_sethalt", "s_set_gpr_idx")):
        return None
    if m.startswith("s_"):
        return "salu"
    return None


@dataclass
class KernelMix:
    name: str
    outside: dict = field(default_factory=lambda: dict.fromkeys(CATEGORIES, 0))
    loops: list = field(default_factory=list)        # per loop: category counts
    loop_vec: list = field(default_factory=list)     # per loop: vector instructions
    loop_div: list = field(default_factory=list)     # per loop: of which under an in-loop exec mask
    vgpr: int = 0
    agpr: int = 0
    lds: int = 0
    hw_outside: dict = field(default_factory=lambda: dict.fromkeys(HW_CLASSES, 0))
    hw_loops: list = field(default_factory=list)     # per loop: issue-class counts

    @property
    def regs(self) -> int:
        """Unified registers per thread: VGPRs (rounded to 4) plus AGPRs."""
        return ((self.vgpr + 3) // 4) * 4 + self.agpr

    def counts(self, trips) -> dict:
        """Per-thread dynamic counts for the given trip count of each loop."""
        if len(trips) != len(self.loops):
            raise ValueError("%s has %d loops, %d trip counts given" % (self.name, len(self.loops), len(trips)))
        out = dict(self.outside)
        for t, c in zip(trips, self.loops):
            for k in CATEGORIES:
                out[k] += int(t) * c[k]
        return out

    def hw_counts(self, trips) -> dict:
        """Per-wave dynamic counts by issue class for the given trip counts
        (every lane of the wave taking the same path)."""
        if len(trips) != len(self.hw_loops):
            raise ValueError("%s has %d loops, %d trip counts given" % (self.name, len(self.hw_loops), len(trips)))
        out = dict(self.hw_outside)
        for t, c in zip(trips, self.hw_loops):
            for k in HW_CLASSES:
                out[k] += int(t) * c[k]
        return out

    def divergence(self, trips) -> float:
        vec = sum(int(t) * v for t, v in zip(trips, self.loop_vec))
        div = sum(int(t) * d for t, d in zip(trips, self.loop_div))
        return div / vec if vec else 0.0


def _is_vector(mn: str) -> bool:
    return mn.startswith(("v_", "global_", "buffer_", "flat_", "ds_", "scratch_"))


def parse(text: str) -> dict:
    """Kernel name -> KernelMix for every kernel in an AMDGPU assembly file."""
    kernels: dict[str, KernelMix] = {}
    cur: KernelMix | None = None
    loop_ids: dict[str, int] = {}
    block_loop = None        # loop index of the current block, None outside loops
    block_in_loop = False
    mask_stack: list[bool] = []  # exec-mask regions: opened inside a loop?
    for raw in text.splitlines():
        line = raw.rstrip()
        if not line:
            continue
        if not line[0].isspace() and not line.startswith((".", ";")) and ":" in line:
            sym = line.split(":", 1)[0]
            if sym.startswith("_Z") or sym.isidentifier():
                cur = KernelMix(sym)
                kernels[sym] = cur
                loop_ids, block_loop, block_in_loop, mask_stack = {}, None, False, []
                continue
        if cur is None:
            continue
        lab = _LABEL.match(line)
        if lab:
            block_loop, block_in_loop = None, False
            h = _HEADER.search(line)
            il = _IN_LOOP.search(line)
            if h or il:
                depth = int((h or il).group(1) if h else il.group(2))
                if depth != 1:
                    raise ValueError("%s: nested loops are not supported" % cur.name)
                hid = lab.group(1).lstrip(".").replace("LBB", "BB") if h else il.group(1)
                if hid not in loop_ids:
                    loop_ids[hid] = len(cur.loops)
                    cur.loops.append(dict.fromkeys(CATEGORIES, 0))
                    cur.hw_loops.append(dict.fromkeys(HW_CLASSES, 0))
                    cur.loop_vec.append(0)
                    cur.loop_div.append(0)
                block_loop, block_in_loop = loop_ids[hid], True
            continue
        s = line.strip()
        if s.startswith((".", ";")) or s.endswith(":"):
            if s.startswith(".Lfunc_end"):
                cur = None
            continue
        mn = s.split()[0]
        if mn in ("s_and_saveexec_b64", "s_and_saveexec_b32"):
            mask_stack.append(block_in_loop)
        elif mn.startswith("s_or_b64") and "exec, exec" in s and mask_stack:
            mask_stack.pop()
        hw = hw_class(mn)
        if hw:
            if block_loop is None:
                cur.hw_outside[hw] += 1
            else:
                cur.hw_loops[block_loop][hw] += 1
        cat = category(mn)
        if cat is None and not _is_vector(mn):
            continue
        if block_loop is None:
            if cat:
                cur.outside[cat] += 1
        else:
            if cat:
                cur.loops[block_loop][cat] += 1
            if _is_vector(mn):
                cur.loop_vec[block_loop] += 1
                if any(mask_stack):
                    cur.loop_div[block_loop] += 1
    # registers and LDS from the code object metadata
    meta = re.search(r"\.amdgpu_metadata\n(---.*?\n\.\.\.)", text, re.S)
    if meta:
        doc = yaml.safe_load(meta.group(1))
        for k in doc.get("amdhsa.kernels", []):
            km = kernels.get(k.get(".name"))
            if km is not None:
                km.vgpr = int(k.get(".vgpr_count", 0))
                km.agpr = int(k.get(".agpr_count", 0))
                km.lds = int(k.get(".group_segment_fixed_size", 0))
    return {n: k for n, k in kernels.items() if n.startswith("_Z")}


def runtime_kernels(path: str | None = None) -> dict:
    """(family name, U) -> KernelMix for the measured families."""
    if path is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sa_runtime_gfx950.s")
    with open(path) as f:
        mixes = parse(f.read())
    out = {}
    pat = re.compile(r"rt_(matvec|stencil|reduce)ILi(\d+)E")
    for name, km in mixes.items():
        m = pat.search(name)
        if m:
            out[(m.group(1), int(m.group(2)))] = km
    return out
