"""Shape checks on the gfx950 assembly of the kernels (CPU only: hipcc
cross-compiles).

Every persistent launch (the per-rig sweep and the pooled kernel) hands out
work by a claim loop: one counter atomic per wave, its old
value broadcast with readfirstlane, then a compare with the queue end that
the whole wave takes together.  That is correct only if the wave enters the
claim as a whole.  A form of the claim that lets a lane skip it on its own
(lanes other than lane 0 add nothing) was compiled into a second loop entry
between the atomic and the compare, which lanes 1..63 took after the body's
lane-0 epilogue split the wave: they then re-read a claim value of zero and
processed the first superpixel of the queue without end.  This test compiles
the kernels to assembly and checks that no branch from outside the claim
enters the span from the atomic to the compare.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1812_06856_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ATOMIC = re.compile(r"global_atomic_add v\d+, v\d+, v\d+, s\[\d+:\d+\] sc0")
LABEL = re.compile(r"^(\.LBB\w+):")


def _kernels(asm):
    """{symbol: [lines]} for every kernel of the slf namespace."""
    out, cur = {}, None
    for ln in asm.split("\n"):
        m = re.match(r"^(_ZN3slf\w+):", ln)
        if m:
            cur = m.group(1)
            out[cur] = []
        elif cur and ln.startswith(".Lfunc_end"):
            cur = None
        elif cur:
            out[cur].append(ln)
    return out


def claim_spans(lines):
    """(first, last) line index of each claim: the returning counter atomic
    up to the compare with the queue end."""
    spans = []
    for i, ln in enumerate(lines):
        if ATOMIC.search(ln):
            j = i
            while j < len(lines) and not re.match(r"\s+s_cmp_ge_i32", lines[j]):
                j += 1
            spans.append((i, j))
    return spans


def outside_entries(lines, span, slack=30):
    """Branches from outside the claim (allowing `slack` lines of set-up
    before the atomic) to labels inside it."""
    i, j = span
    bad = []
    for ln in lines[i:j]:
        m = LABEL.match(ln)
        if not m:
            continue
        lab = m.group(1)
        pat = re.compile(r"(?<![\w.])" + re.escape(lab) + r"(?!\w)")
        for t, other in enumerate(lines):
            if other.startswith(lab + ":") or i - slack <= t <= j:
                continue
            if pat.search(other):
                bad.append((lab, other.strip()))
    return bad


def test_outside_entry_detected():
    # A hand-made claim with a second entry (the broken shape) is flagged;
    # the clean shape is not.
    clean = """\ts_mov_b64 s[0:1], exec
\tglobal_atomic_add v2, v1, v2, s[4:5] sc0
.LBB1_9:
\ts_or_b64 exec, exec, s[2:3]
\tv_readfirstlane_b32 s0, v2
\ts_cmp_ge_i32 s0, s5
\ts_cbranch_scc1 .LBB1_20""".split("\n")
    # the execz branch into the span sits right before the atomic, inside the slack
    clean.insert(1, "\ts_cbranch_execz .LBB1_9")
    assert claim_spans(clean) and not outside_entries(clean, claim_spans(clean)[0])
    broken = clean[:3] + [".LBB1_13:"] + clean[3:] + ["\tv_mov_b32 v2, 0"] * 40 + ["\ts_branch .LBB1_13"]
    assert outside_entries(broken, claim_spans(broken)[0])


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not installed")
def test_claim_loops_entered_whole(tmp_path):
    out = tmp_path / "k.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-x", "hip",
           "--cuda-device-only", "-S", os.path.join(CSRC, "slf_kernels.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    kernels = _kernels(out.read_text())
    checked = 0
    for name, lines in kernels.items():
        # the templated kernels (their mangled names take template arguments: ...I)
        if not re.match(r"_ZN3slf(7k_sweep|6k_pool)I", name):
            continue
        spans = claim_spans(lines)
        assert spans, f"{name}: no claim found"
        for span in spans:
            assert not outside_entries(lines, span), f"{name}: claim entered from outside"
            checked += 1
    # three formats of the sweep, nine sweep and three refinement pool kernels
    assert checked == 15, checked
