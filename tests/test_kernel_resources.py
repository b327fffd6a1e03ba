"""Resource check of every stage, time-step and reduction kernel, from the
gfx950 assembly hipcc writes for the library's own sources (no GPU needed):
no kernel may use scratch memory (register spills, or an argument copy
moved to scratch by run-time indexing, which once made the batched
kernels 1.8x slower), and the LDS of a workgroup fits in the 160 KB of a
CU."""
import glob
import os
import re
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2004_08503_amd import build as hipbuild

CSRC = os.path.join(os.path.dirname(hipbuild.__file__), "csrc")
KEYS = ("private_segment_fixed_size", "group_segment_fixed_size", "vgpr_count")


def device_asm(src, out_dir):
    asm = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [hipbuild.HIPCC] + hipbuild.FLAGS + ["--cuda-device-only", "-S", src, "-o", asm]
    subprocess.run(cmd, check=True, capture_output=True)
    return asm


def parse(asm):
    """Kernel name -> metadata fields, from the code object's kernel list
    (one YAML item per kernel)."""
    text = open(asm).read()
    start = text.find("amdhsa.kernels:")
    out = {}
    for block in text[start:].split("\n  - ")[1:]:
        name = re.search(r"\.name:\s+(\S+)", block)
        if not name:
            continue
        d = {}
        for key in KEYS:
            m = re.search(r"\.%s:\s+(\d+)" % key, block)
            if m:
                d[key] = int(m.group(1))
        out[name.group(1)] = d
    return out


@pytest.fixture(scope="module")
def kernels():
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            asms = list(ex.map(lambda s: device_asm(s, tmp), srcs))
        meta = {}
        for a in asms:
            meta.update(parse(a))
    return meta


def test_every_kernel_fits_without_scratch(kernels):
    ours = {k: v for k, v in kernels.items() if k.startswith("_ZN3idp")}
    assert len(ours) > 100      # every equation, dimension and degree
    scratch = {k: v["private_segment_fixed_size"] for k, v in ours.items()
               if v.get("private_segment_fixed_size", 0) > 0}
    assert not scratch, scratch
    big = {k: v["group_segment_fixed_size"] for k, v in ours.items()
           if v.get("group_segment_fixed_size", 0) > 160 * 1024}
    assert not big, big
