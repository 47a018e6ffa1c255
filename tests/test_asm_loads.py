"""The BF16 layer-1 GEMM (k_l1rb) issues its weight-fragment loads as inline
assembly, each followed later by an explicit wait, so that its LDS pipeline's
fixed wait counts stay exact.  The compiler treats an inline load's
destination registers as written as soon as the instruction issues, so two
properties of the compiled device code have to hold, and are checked here on
the compiled assembly:

  (a) no instruction reads or overwrites a fragment load's destination
      registers before the MFMA that consumes it (a copy would read the
      registers early; a reuse would be overwritten by the load in flight);
  (b) on the straight-line path to that MFMA an s_waitcnt retires the load
      (vector-memory counter at most the number of vector-memory operations
      issued after it).

CPU only: it compiles nnp_mlp.hip for gfx950 to assembly (about 15 s)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

VM_OPS = ("global_load", "global_store", "global_atomic", "buffer_", "flat_", "scratch_")


def _regs(text):
    out = set()
    for m in re.finditer(r"v\[(\d+):(\d+)\]", text):
        out |= set(range(int(m.group(1)), int(m.group(2)) + 1))
    for m in re.finditer(r"(?<![\w\[])v(\d+)\b", text):
        out.add(int(m.group(1)))
    return out


def _instructions(lines):
    """(instruction, from inline asm) pairs, directives and labels left out"""
    inline = False
    for ln in lines:
        s = ln.strip()
        if s.startswith(";;#ASMSTART"):
            inline = True
        elif s.startswith(";;#ASMEND"):
            inline = False
        t = ln.split(";")[0].strip()
        if t and not t.startswith(".") and not t.endswith(":"):
            yield t, inline


@pytest.fixture(scope="module")
def l1rb_bodies(tmp_path_factory):
    from paper_2201_08110_amd import build as B
    try:
        cc = B.hipcc()
    except Exception:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("asm") / "mlp.s")
    r = subprocess.run([cc, *B.FLAGS, "--cuda-device-only", "-S",
                        os.path.join(B.CSRC, "nnp_mlp.hip"), "-o", out],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = open(out).read().split("\n")
    bodies = {}
    for i, ln in enumerate(lines):
        m = re.match(r"^(_ZN3nnp6k_l1rb\w+):", ln)
        if m:
            end = next(j for j in range(i + 1, len(lines)) if lines[j].startswith(".Lfunc_end"))
            bodies[m.group(1)] = lines[i:end]
    assert bodies, "no k_l1rb kernels in the assembly"
    return bodies


def inline_load_problems(body):
    """Violations of (a) and (b) in one kernel's assembly lines; also the
    number of inline fragment loads seen."""
    ins = list(_instructions(body))
    problems, n_loads = [], 0
    for i, (t, inline) in enumerate(ins):
        if not (inline and t.startswith("global_load_dwordx4 ")):
            continue
        dst = _regs(t.split(",")[0])
        n_loads += 1
        issued_after, retired = 0, False
        for u, _ in ins[i + 1:]:
            r = _regs(u)
            if u.startswith("s_waitcnt") and "vmcnt(" in u:
                n = int(re.search(r"vmcnt\((\d+)\)", u).group(1))
                retired = retired or n <= issued_after
            if u.startswith("v_mfma") and (r & dst):
                if not retired:
                    problems.append(f"MFMA reads {sorted(dst)} before a wait retires its load: {u}")
                break
            if r & dst:
                problems.append(f"{u!r} touches {sorted(dst)} while the load may be in flight")
                break
            if u.startswith(VM_OPS):
                issued_after += 1
        else:
            problems.append(f"load into {sorted(dst)} is never consumed")
    return problems, n_loads


def test_checker_on_hand_written_sequences():
    load = [";;#ASMSTART", "global_load_dwordx4 v[4:7], v[0:1], off", ";;#ASMEND"]
    mfma = "v_mfma_f32_16x16x32_bf16 a[0:3], v[4:7], v[8:11], a[0:3]"
    ok = load + ["global_load_dwordx4 v[12:15], v[2:3], off", "s_waitcnt vmcnt(1)", mfma]
    assert inline_load_problems(ok) == ([], 1)
    early = load + ["global_load_dwordx4 v[12:15], v[2:3], off", "s_waitcnt vmcnt(2)", mfma]
    assert "before a wait" in inline_load_problems(early)[0][0]
    copy = load + ["v_mov_b32_e32 v20, v5", "s_waitcnt vmcnt(0)", mfma]
    assert "touches" in inline_load_problems(copy)[0][0]
    reuse = load + ["v_add_u32_e32 v6, 4, v1", "s_waitcnt vmcnt(0)", mfma]
    assert "touches" in inline_load_problems(reuse)[0][0]
    unused = load + ["s_endpgm"]
    assert "never consumed" in inline_load_problems(unused)[0][0]


def test_inline_fragment_loads_are_consumed_after_a_wait(l1rb_bodies):
    for name, body in l1rb_bodies.items():
        problems, n_loads = inline_load_problems(body)
        assert not problems, f"{name}: {problems[:3]}"
        assert n_loads >= 8, f"{name}: expected the inline fragment loads, found {n_loads}"
