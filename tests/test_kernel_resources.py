"""Register and scratch budget of the HIP kernels (gfx950, cross-compiled on
the host; no GPU needed).

The fused kernels' speed rests on two compile-time properties that no parity
test sees: no kernel keeps registers in scratch memory, and in FP32 a
workgroup of the R = 48 quarter (Q = 28) and one of the small-quarter launch
fit one compute unit together (the two launches of an apply run
concurrently; each workgroup puts two waves on every SIMD, and a SIMD lane
has 512 registers, VGPRs and AGPRs together).  A change that copies a larger
struct into a kernel's locals, or keeps more values live, breaks them
silently: a persistent form of the four-wave batch kernel spilled 34-38
registers at Q = 56 and ran the frequency 16 % slower, and forming the
float16 band fragments with a range multiply spilled 67 at Q = 40."""
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1704_05231_amd", "csrc")
FORMS = range(5)
# (source, form) pairs: the per-form objects and the form-independent ones
UNITS = ([("gabor_ws.hip", f) for f in FORMS] + [("gabor_fused.hip", f) for f in FORMS]
         + [(s, 0) for s in ("gabor_fp32.hip", "gabor_adjoint.hip", "gabor_iir.hip", "gabor_sdft.hip")])
REGS_PER_SIMD_LANE = 512
GRANULE = 8                     # register allocation granularity


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def _resources(unit, out_dir):
    """Per-kernel resource remarks of one source's device compile."""
    src, form = unit
    cmd = [_hipcc(), "-O3", "-std=c++17", "--offload-arch=gfx950", "--offload-device-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), f"-DGABOR_FORM={form}", "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", os.path.join(out_dir, f"{src}.{form}.o"),
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    res, cur = {}, None
    for ln in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", ln)
        if m:
            cur = m.group(1)
            res[cur] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|VGPRs Spill|SGPRs Spill|ScratchSize \[bytes/lane\]): (\d+)", ln)
        if m and cur:
            res[cur][m.group(1)] = int(m.group(2))
    return res


@pytest.fixture(scope="module")
def resources(tmp_path_factory):
    if _hipcc() is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("kernel_resources"))
    with ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 1)) as ex:
        found = list(ex.map(lambda u: _resources(u, out), UNITS))
    return dict(zip(UNITS, found))


def _kernel(res, pattern):
    hits = [k for k in res if re.search(pattern, k)]
    assert len(hits) == 1, (pattern, hits)
    return res[hits[0]]


def _regs(r):
    return -(-(r["VGPRs"] + r.get("AGPRs", 0)) // GRANULE) * GRANULE


def test_no_scratch(resources):
    for unit, res in resources.items():
        kernels = [k for k in res if "_ZN5gabor" in k and "k_" in k]
        assert kernels, (unit, sorted(res))
        for k in kernels:
            # (register spills into AGPRs or VGPR lanes need no scratch and are allowed)
            assert res[k].get("ScratchSize [bytes/lane]", 0) == 0, (unit, k, res[k])


def test_fp32_r48_and_small_launch_share_a_compute_unit(resources):
    res = resources[("gabor_ws.hip", 0)]
    big = _kernel(res, r"k_ws_tilesILi0ELi28EE")
    small = _kernel(res, r"k_ws_tiles_smallILi0EE")
    # two waves per SIMD from each workgroup
    assert 2 * _regs(big) + 2 * _regs(small) <= REGS_PER_SIMD_LANE, (big, small)
