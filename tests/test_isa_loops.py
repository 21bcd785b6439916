"""No barrier of a built kernel sits inside a lane-divergent loop.

A loop the compiler takes for lane-divergent runs while any lane of the
wave is left in it; with a barrier inside, part of a wave can meet the
block's barriers while another part is parked outside the loop.  The
persistent plan kernel once compiled that way (its claim and publish were
`threadIdx.x == 0` branches at the loop's head and latch) and its loop
never ended.  The checker (tests/isa_loops.py) is pinned first on two
minimal kernels of that shape, compiled here and never launched, then run
over every code object the build made.  CPU only: hipcc and the ROCm LLVM
tools, no device."""

import glob
import os
import subprocess

import pytest

from tests import isa_loops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

SHAPES = r"""
#include <hip/hip_runtime.h>
// claim and publish by the lane that has threadIdx.x == 0
__global__ void __launch_bounds__(256) lane0_loop(unsigned* ctr, const int* items, int n, float* out) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(ctr, 1u);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n) break;
    out[(size_t)it * 256 + threadIdx.x] += (float)items[it];
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(ctr + 1, 1u);
  }
}
// the same loop with wave-uniform branches only (wave 0 claims and publishes)
__global__ void __launch_bounds__(256) wave_loop(unsigned* ctr, const int* items, int n, float* out) {
  __shared__ int s_item;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (;;) {
    if (wave == 0)
      s_item = __builtin_amdgcn_readfirstlane((int)atomicAdd(ctr, (threadIdx.x & 63u) == 0u ? 1u : 0u));
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n) break;
    out[(size_t)it * 256 + threadIdx.x] += (float)items[it];
    __syncthreads();
    if (wave == 0) atomicAdd(ctr + 1, (threadIdx.x & 63u) == 0u ? 1u : 0u);
  }
}
"""


def _need_tools():
    if not os.path.exists(HIPCC) or not isa_loops.tools_present():
        pytest.skip("hipcc or the ROCm LLVM tools are missing")


def test_checker_flags_the_lane0_claim_loop(tmp_path):
    _need_tools()
    src = tmp_path / "shapes.hip"
    src.write_text(SHAPES)
    obj = tmp_path / "shapes.o"
    subprocess.run([HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                    "-Xclang", "-packed-fp32-ops", "-c", str(src), "-o", str(obj)],
                   check=True, capture_output=True)
    found = isa_loops.scan_object(str(obj), str(tmp_path))
    names = sorted(found)
    assert any("lane0_loop" in n for n in names), found
    assert not any("wave_loop" in n for n in names), found


def test_built_kernels_have_no_barrier_in_a_divergent_loop(tmp_path):
    _need_tools()
    objs = sorted(glob.glob(os.path.join(ROOT, "_build", "*.hip.o")))
    if not objs:
        pytest.skip("library not built")
    bad = {}
    for o in objs:
        for fn, msgs in isa_loops.scan_object(o, str(tmp_path)).items():
            bad[f"{os.path.basename(o)}:{fn}"] = msgs
    assert not bad, bad
