"""Instruction schedule of the FP64 update kernel's main loop (CPU only).

The update kernel prefetches its MFMA fragments two k-steps ahead.  That
only pays if each fragment set waits for its own loads: a `s_waitcnt
vmcnt(0)` inside the loop means every trip waits for the whole prefetch queue
(the compiler produced exactly that when the reloads were conditional, and it
sank the reloads to their first use when they were not pinned).  The test
compiles the source for gfx950 to assembly and checks the loop of both
instantiations: MFMAs present, reloads present, no full-queue wait.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1203_1269_amd", "csrc", "chol.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _function_asm(asm: str, mangled_prefix: str) -> str:
    start = re.search(r"^" + re.escape(mangled_prefix) + r"[^:\n]*:", asm, re.M)
    assert start, mangled_prefix
    end = asm.find(".Lfunc_end", start.end())
    return asm[start.start():end]


def _main_loop(fn: str) -> str:
    """The last loop of the function: from the target of its back edge (the
    first branch after the loop header that jumps to a label at or before
    the header) to that branch."""
    headers = list(re.finditer(r"^(\.LBB[0-9_]+):[^\n]*Loop Header", fn, re.M))
    assert headers, "no loop found"
    h = headers[-1].start()
    labels = {m.group(1): m.start() for m in re.finditer(r"^(\.LBB[0-9_]+):", fn, re.M)}
    for br in re.finditer(r"s_c?branch\w* (\.LBB[0-9_]+)", fn[h:]):
        target = labels.get(br.group(1))
        if target is not None and target <= h:
            return fn[target:h + br.end()]
    raise AssertionError("no back branch")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc missing")
def test_update_loop_waits_only_for_its_own_fragments(tmp_path):
    out = tmp_path / "chol.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.dirname(SRC),
           "--cuda-device-only", "-S", SRC, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    asm = out.read_text()
    for tmpl in ("ILi2ELi2E", "ILi4ELi1E"):
        fn = _function_asm(asm, "_ZN3gpk12_GLOBAL__N_118syrk_update_kernel" + tmpl)
        loop = _main_loop(fn)
        assert loop.count("v_mfma_f64_16x16x4") >= 16, tmpl
        assert loop.count("global_load_dwordx2") >= 8, tmpl
        waits = [int(v) for v in re.findall(r"s_waitcnt vmcnt\((\d+)\)", loop)]
        assert waits, tmpl
        assert min(waits) > 0, f"{tmpl}: full-queue wait in the update loop: {waits}"
