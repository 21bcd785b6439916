"""The ring tiles' prefetch of the next block is not waited for before the
spectrum's first barrier.

The register-ring tiles load block m+1 at the top of spectrum m and use it
only when the ring shifts at the end.  If the compiler places a wait for
those loads inside the FIR (it did while the prefetch was a conditional
load per word: the loop body was many basic blocks), every spectrum waits
out one HBM latency.  The check reads the largest loop of each kernel in
the built gfx950 code and lists the vector-memory waits between its first
global load and the first barrier after it.  It is pinned on two minimal
kernels compiled here and never launched: one uses its load before the
barrier (a wait must be found), one only after it (none).  CPU only."""

import os
import subprocess

import pytest

from tests import isa_loops

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

SHAPES = r"""
#include <hip/hip_runtime.h>
// the loaded value is used before the barrier
__global__ void __launch_bounds__(256) use_before(const float* x, float* out, int n) {
  __shared__ float s[256];
  float acc = 0.f;
  for (int m = 0; m < n; ++m) {
    const float v = x[(size_t)m * 256 + threadIdx.x];
    s[threadIdx.x] = v * 2.f;
    __syncthreads();
    acc += s[(threadIdx.x + 1) & 255];
    __syncthreads();
  }
  out[threadIdx.x] = acc;
}
// the loaded value (the next spectrum's) is used after the barriers
__global__ void __launch_bounds__(256) use_after(const float* x, float* out, int n) {
  __shared__ float s[256];
  float acc = 0.f, cur = x[threadIdx.x];
  for (int m = 0; m < n; ++m) {
    const float nxt = x[(size_t)(m + 1 < n ? m + 1 : m) * 256 + threadIdx.x];
    s[threadIdx.x] = cur * 2.f;
    __syncthreads();
    acc += s[(threadIdx.x + 1) & 255];
    __syncthreads();
    cur = nxt;
  }
  out[threadIdx.x] = acc;
}
"""

# the ring tiles: real-time fused kernel, in-place fused ring tile, ring
# F-engine (FP16 output, ping-pong buffers)
KERNELS = ["fx_fused_ring_pp_kernelILi4096ELi4ELi16ELi4E",
           "fx_fused_ring_kernelILi4096ELi4ELi16ELi4ELi0E",
           "chan_ring_kernelILi4096ELi4ELi16ELi4ELi1ELb1ELi0E"]


def _need_tools():
    if not os.path.exists(HIPCC) or not isa_loops.tools_present():
        pytest.skip("hipcc or the ROCm LLVM tools are missing")


def _waits(obj, tmp, name):
    fns = isa_loops.functions(isa_loops.disasm(obj, tmp))
    match = [f for f in fns if name in f]
    assert len(match) == 1, (name, match)
    return isa_loops.waits_before_first_barrier(isa_loops.main_loop(fns[match[0]]))


def test_checker_pins(tmp_path):
    _need_tools()
    src = tmp_path / "shapes.hip"
    src.write_text(SHAPES)
    obj = tmp_path / "shapes.o"
    subprocess.run([HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                    "-Xclang", "-packed-fp32-ops", "-c", str(src), "-o", str(obj)],
                   check=True, capture_output=True)
    assert _waits(str(obj), str(tmp_path), "use_before"), "a wait before the barrier was not found"
    assert _waits(str(obj), str(tmp_path), "use_after") == []


@pytest.mark.parametrize("name", KERNELS)
def test_ring_prefetch_not_waited_in_the_fir(tmp_path, name):
    _need_tools()
    obj = os.path.join(ROOT, "_build", "qc_fx.hip.o")
    if not os.path.exists(obj):
        pytest.skip("library not built")
    w = _waits(obj, str(tmp_path), name)
    assert w == [], w
