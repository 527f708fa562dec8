"""The stage kernel's population loop is fully unrolled in every
instantiation: its accumulators are indexed by population, so a loop left
rolled keeps them in scratch memory and runs many times slower (the FP32
specular-x kernels did, under the compiler's default unroll size limit).
Compiles the device code to assembly with the library's own flags; CPU only."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1702_01690_amd import build as B


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_stage_kernels_fully_unrolled(tmp_path):
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-shared", "-Wall")]
    out = tmp_path / "stage.s"
    cmd = ["hipcc"] + flags + ["--offload-device-only", "-S", os.path.join(B.CSRC, "olb_kernels.hip"),
                               "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=900)
    lines = out.read_text().split("\n")
    starts = [i for i, l in enumerate(lines) if re.match(r"^_ZN4olbk12stage_kernelI\w+:", l)]
    # {FP64 BY 8, 16; FP32 BY 8, 12, 16} x walls x FN x specular x
    assert len(starts) == 40
    for i in starts:
        name = lines[i].split(":")[0]
        body = []
        for l in lines[i + 1:]:
            if l.startswith(".Lfunc_end"):
                break
            body.append(l.strip())
        barriers = sum(1 for l in body if l.startswith("s_barrier"))
        scratch = sum(1 for l in body if l.startswith("scratch_"))
        # one barrier before the force stencils and one per streamed population
        assert barriers == 25, (name, barriers)
        # at most a few spilled registers outside the loop, none at BY = 8 or 12
        assert scratch <= (0 if ("Li8E" in name or "Li12E" in name) else 8), (name, scratch)
