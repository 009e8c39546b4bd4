"""Checks of the gfx950 code the kernels compile to (no GPU needed: hipcc cross-compiles).

* No kernel spills registers to scratch memory.
* The conv and lifting kernels reach HBM through global_* instructions only.  A flat_*
  access (what a generic pointer read from a descriptor in memory compiles to) also counts
  against the LDS wait counter, so every LDS wait in an MFMA loop would wait for the HBM
  loads in flight too.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2405_12631_amd import build as B

HIPCC = B.HIPCC
SOURCES = ["wv_conv.hip", "wv_conv_bf16.hip", "wv_lift_fused.hip", "wv_lift.hip", "wv_cdf.hip",
           "wv_stack_bf16.hip", "wv_lift_rows.hip", "wv_lstm_bf16.hip"]
FLAT_FREE = ("conv3x3", "lift_fused_k", "stack_bf16_k", "lift_rows_k", "lstm_bf16_k")


def _kernels(asm):
    """Kernel name -> (body text, ScratchSize) from a device assembly listing."""
    out = {}
    names = re.findall(r"^(_Z\S+):", asm, flags=re.M)
    for i, name in enumerate(names):
        start = asm.index(name + ":")
        end = asm.index(names[i + 1] + ":") if i + 1 < len(names) else len(asm)
        body = asm[start:end]
        m = re.search(r"; ScratchSize: (\d+)", body)
        out[name] = (body, int(m.group(1)) if m else 0)
    return out


@pytest.fixture(scope="module")
def listings():
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    tmp = tempfile.mkdtemp(prefix="wv_asm_")
    procs = []
    for src in SOURCES:
        out = os.path.join(tmp, src + ".s")
        cmd = [HIPCC, "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", out] + [
            f for f in B.HIP_FLAGS if f not in ("-fPIC",)]
        procs.append((src, out, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    res = {}
    for src, out, p in procs:
        log, _ = p.communicate()
        assert p.returncode == 0, f"{src}: {log[-2000:]}"
        with open(out) as f:
            res[src] = _kernels(f.read())
    shutil.rmtree(tmp, ignore_errors=True)
    return res


@pytest.mark.slow
def test_no_scratch_spills(listings):
    spills = [(src, k, sc) for src, ks in listings.items() for k, (_, sc) in ks.items() if sc > 0]
    assert not spills, spills


@pytest.mark.slow
def test_hot_kernels_use_global_memory_instructions(listings):
    seen, flat = 0, []
    for src, ks in listings.items():
        for k, (body, _) in ks.items():
            if any(t in k for t in FLAT_FREE):
                seen += 1
                if re.search(r"^\s*flat_(load|store|atomic)", body, flags=re.M):
                    flat.append(k)
    assert seen > 50, seen   # every conv instantiation and the lifting kernels were found
    assert not flat, flat
