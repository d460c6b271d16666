"""The device code is built without packed FP32 instructions.

hipcc's host pass warns that it does not know the `-packed-fp32-ops`
feature; the device pass honours it.  Shown on a probe kernel whose float2
arithmetic the compiler turns into packed instructions without the flag, and
checked on the library's own sources with the library's flags."""
import os
import shutil
import subprocess

import pytest

from paper_2109_08219_amd import build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
PACKED = ("v_pk_add_f32", "v_pk_mul_f32", "v_pk_fma_f32")

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(float2* a, const float2* b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) { float2 x = a[i], y = b[i]; x.x = x.x * y.x + 1.0f; x.y = x.y * y.y + 1.0f; a[i] = x; }
}
"""

pytestmark = pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")


def device_asm(src: str, flags: list, tmp_path) -> str:
    out = tmp_path / "out.s"
    subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(build.ROOT, "include"),
                    "-o", str(out), src], check=True, capture_output=True)
    return out.read_text()


def packed(asm: str) -> int:
    return sum(asm.count(p) for p in PACKED)


def test_flag_takes_effect_on_device_code(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    base = ["--offload-arch=gfx950", "-O3", "-std=c++17"]
    assert packed(device_asm(str(src), base, tmp_path)) > 0  # the probe does get packed code by default
    assert packed(device_asm(str(src), build.HIPCC_FLAGS, tmp_path)) == 0


@pytest.mark.parametrize("name", ["wide.hip", "codec_f32.hip"])
def test_library_sources_have_no_packed_fp32(name, tmp_path):
    asm = device_asm(os.path.join(build.CSRC, name), build.HIPCC_FLAGS, tmp_path)
    assert packed(asm) == 0
