"""The per-phase kernels must not touch scratch memory: a kernel with scratch
pays for its set-up on every launch and reads its spilled values from memory.
hipcc reports each kernel's resource usage when cross-compiling for gfx950, so
this runs without a GPU."""
import os
import re
import subprocess

import pytest

from paper_1309_3848_amd import build as hipbuild

HOT = ["seeds_phase.hip", "seeds_kernels.hip", "seeds_quality.hip", "seeds_energy.hip"]


def _usage(src):
    cmd = [hipbuild.HIPCC, *[f for f in hipbuild.FLAGS if f not in ("-shared", "-fPIC")],
           "-I", hipbuild.INCLUDE, "-I", hipbuild.CSRC, "--cuda-device-only", "-c",
           os.path.join(hipbuild.CSRC, src), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert len(names) == len(scratch) and names
    return dict(zip(names, scratch))


@pytest.mark.parametrize("src", HOT)
def test_hot_kernels_use_no_scratch(src):
    usage = _usage(src)
    assert any(k in n for n in usage for k in ("k_phase", "k_init", "k_q_count", "k_energy"))
    assert {n: s for n, s in usage.items() if s} == {}
