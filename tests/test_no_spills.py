"""Every kernel compiles without scratch (spilled registers): spills are HBM
traffic on the hot path, and several kernels sit right at their register
budget.  Device code only, with the library's own flags."""
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2010_14333_amd import build

HIP_SOURCES = [s for s in build.SOURCES if s.endswith(".hip")]


def _resources(src):
    cmd = [build.HIPCC, *build.FLAGS, *build.EXTRA.get(src, []), "--cuda-device-only", "-c",
           os.path.join(build.SRC, src), "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(v) for v in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    assert names and len(names) == len(scratch), r.stderr[-2000:]
    return dict(zip(names, scratch))


@pytest.mark.skipif(not os.path.exists(build.HIPCC), reason="hipcc not found")
def test_no_kernel_spills():
    with ThreadPoolExecutor(len(HIP_SOURCES)) as ex:
        res = dict(zip(HIP_SOURCES, ex.map(_resources, HIP_SOURCES)))
    spilled = {(src, k): v for src, ks in res.items() for k, v in ks.items() if v}
    assert sum(len(ks) for ks in res.values()) >= 20
    assert not spilled, spilled
