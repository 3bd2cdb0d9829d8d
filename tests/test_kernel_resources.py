"""Every gfx950 kernel of the library keeps its values in registers: the
compiler's resource report shows no scratch (private stack) memory for any of
them.  A kernel that spills, or indexes a private array with a run-time index,
moves that data through memory on every access (the DIRK column kernel's stage
arrays once cost 560 bytes per lane and a third of the field solve).

Compiles each csrc/*.hip for the device only (no GPU needed)."""

import concurrent.futures
import os
import re
import shutil
import subprocess

import pytest

from paper_2410_18414_amd import build

HIPCC = build.HIPCC


def resource_report(src):
    cmd = [HIPCC] + build.FLAGS + ["--cuda-device-only", "-c", "-o", os.devnull, src,
                                   "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            kernels[name] = int(m.group(1))
    return kernels


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_no_kernel_uses_scratch():
    srcs = build.sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(srcs), 4)) as ex:
        reports = dict(zip(srcs, ex.map(resource_report, srcs)))
    assert sum(len(k) for k in reports.values()) > 20  # the report was parsed
    spills = {os.path.basename(s) + ":" + k: v for s, ks in reports.items() for k, v in ks.items() if v}
    assert not spills, spills
