"""The library's hipcc flags on a probe (CPU only, hipcc cross-compiles):
the device pass honours -packed-fp32-ops, so packed FP32 instructions
(v_pk_fma_f32 and kin), which hipcc -O3 otherwise forms from plain float2
code, are absent from the device code; hipcc's host pass warns that it does
not know the feature, which concerns the x86 target only."""
import os
import shutil
import subprocess

import pytest

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(float2* a, const float2* b, const float2* c) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  float2 x = a[i], y = b[i], z = c[i];
  x.x = x.x * y.x + z.x;
  x.y = x.y * y.y + z.y;
  a[i] = x;
}
"""


def _device_asm(tmp_path, flags):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    out = tmp_path / "probe.s"
    cmd = ["hipcc"] + flags + ["--cuda-device-only", "-S", str(src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=120)
    return out.read_text()


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_packed_fp32_is_off_in_device_code(tmp_path):
    from paper_2509_25347_amd import _lib
    lib_flags = [f for f in _lib.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    plain = [f for f in lib_flags
             if f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    # the probe contracts x*y+z into an FMA (the library itself uses explicit fma())
    with_flag = _device_asm(tmp_path, lib_flags + ["-ffp-contract=fast"])
    without = _device_asm(tmp_path, plain + ["-ffp-contract=fast"])
    packed = ("v_pk_fma_f32", "v_pk_mul_f32", "v_pk_add_f32")
    assert any(p in without for p in packed), "probe no longer forms packed FP32"
    assert not any(p in with_flag for p in packed)
    assert os.path.exists(tmp_path / "probe.s")
