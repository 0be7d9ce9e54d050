"""Compiler resource checks of the hot kernels (CPU only: hipcc cross-compiles
for gfx950 here).  A register array that the compiler cannot keep in
registers is moved to per-lane scratch memory without any error, and the
pass then runs far slower; these tests fail instead."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_14211_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _resources(src, tmp_path):
    out = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                          "-I" + os.path.join(ROOT, "include"), "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops", "-Rpass-analysis=kernel-resource-usage", "-c",
                          os.path.join(CSRC, src), "-o", str(tmp_path / "k.o")],
                         capture_output=True, text=True, check=True).stderr
    res, name = {}, None
    for line in out.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            res[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^]]*\])?: (\d+)", line)
        if m and name:
            res[name][m.group(1).strip()] = int(m.group(2))
    return res


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
@pytest.mark.parametrize("src,kernels", [
    ("kernels.hip", ("fused_wave_kernel", "fused_pr_kernel")),
    ("spmm.hip", ("spmm_ppr_kernel", "spmm_packed_kernel")),
    ("many.hip", ("pr_many_kernel",)),
    ("stripe.hip", ("fused_stripe_kernel",)),
])
def test_hot_kernels_use_no_scratch(tmp_path, src, kernels):
    res = _resources(src, tmp_path)
    seen = 0
    for name, r in res.items():
        if any(k in name for k in kernels):
            seen += 1
            assert r.get("ScratchSize", 0) == 0, (name, r)
            assert r.get("LDS Size", 0) <= 160 * 1024, (name, r)
    assert seen >= len(kernels)
