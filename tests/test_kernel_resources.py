"""Every gfx950 kernel of the library keeps its values in registers: the
compiler's resource report shows no scratch (private stack) memory for any of
them.  A kernel that spills, or indexes a private array with a run-time index,
moves that data through memory on every access (the DIRK column kernel's stage
arrays once cost 560 bytes per lane and a third of the field solve).  And the
float32 fused pass of the default tile shape stays within 128 VGPRs: its LDS
admits four workgroups of four waves per CU, so four waves per SIMD, which a
larger register count would cut to three or two (measured 3-8% slower).

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
            kernels[name] = {}
            continue
        m = re.search(r"(ScratchSize \[bytes/lane\]|VGPRs): (\d+)", line)
        if m and name:
            kernels[name]["scratch" if m.group(1).startswith("Scratch") else "vgprs"] = int(m.group(2))
    return kernels


@pytest.fixture(scope="module")
def reports():
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    srcs = build.sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(srcs), 4)) as ex:
        return dict(zip((os.path.basename(s) for s in srcs), ex.map(resource_report, srcs)))


def test_no_kernel_uses_scratch(reports):
    assert sum(len(k) for k in reports.values()) > 20  # the report was parsed
    spills = {f + ":" + k: v["scratch"] for f, ks in reports.items() for k, v in ks.items() if v.get("scratch")}
    assert not spills, spills


def test_fused_pass_fits_four_waves_per_simd(reports):
    # k_tiled<float, 3 (cubic), 2 (fused), 16-cell tiles, slack 3>
    name = "_ZN3pic12_GLOBAL__N_17k_tiledIfLi3ELi2ELi16ELi3EEEvPKNS_8InstDescEiNS_8StepArgsE"
    assert name in reports["tiles.hip"]
    assert reports["tiles.hip"][name]["vgprs"] <= 128
