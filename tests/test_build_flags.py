"""The library's compiler flags do what they claim (no GPU).

The device code must contain no packed-FP32 instructions.  The build passes
a target-feature switch for that; hipcc's host pass warns that it does not
know the feature, so this test checks on the device pass itself: a float2
kernel that hipcc -O3 turns into v_pk_* instructions without the switch
has none with the library's flags.  It also checks the built library's
sources compile to device assembly free of them.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2403_13287_amd import _build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void k(float2 *a, const float2 *b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float2 x = a[i];
    const float2 y = b[i];
    x.x = x.x * y.x + 1.0f;
    x.y = x.y * y.y + 1.0f;
    a[i] = x;
  }
}
"""
PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")

pytestmark = pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC),
                                reason="hipcc not available")


def _device_asm(src, flags, tmp_path, name):
    out = os.path.join(str(tmp_path), name + ".s")
    subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", src, "-o", out,
                    "-I", os.path.join(_build.ROOT, "include")], check=True,
                   stderr=subprocess.DEVNULL)
    return open(out).read()


def test_packed_fp32_switch_takes_effect_on_the_device_pass(tmp_path):
    src = os.path.join(str(tmp_path), "probe.hip")
    with open(src, "w") as f:
        f.write(PROBE)
    base = [f for f in _build.HIPCC_FLAGS if f not in ("-Xclang", "-target-feature",
                                                       "-packed-fp32-ops", "-fPIC")]
    without = _device_asm(src, base, tmp_path, "without")
    assert PACKED.search(without), "probe no longer produces packed FP32 code"
    with_flags = _device_asm(src, [f for f in _build.HIPCC_FLAGS if f != "-fPIC"], tmp_path, "with")
    assert not PACKED.search(with_flags)


@pytest.mark.parametrize("name", [os.path.basename(s) for s in _build.sources()])
def test_library_device_code_has_no_packed_fp32(name, tmp_path):
    src = os.path.join(_build.HERE, "csrc", name)
    flags = [f for f in _build.HIPCC_FLAGS if f != "-fPIC"]
    sched = _build.SCHEDULER.get(name)
    if sched:
        flags += ["-mllvm", f"-amdgpu-sched-strategy={sched}"]
    asm = _device_asm(src, flags, tmp_path, name)
    assert "v_fma_f64" in asm
    assert not PACKED.search(asm)
