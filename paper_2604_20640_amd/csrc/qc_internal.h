// Host-side helpers of the C-ABI layer shared by its translation units:
// the thread-local error string behind qc_last_error() and the argument
// checks of the streaming entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qc.h"

namespace qc {

// Clears the calling thread's error string.
void api_clear_error();
// Records a formatted message as the calling thread's error; returns s.
qc_status api_fail(qc_status s, const char* fmt, ...);
// The checks qc_pfb_channelize and qc_xcorrelate apply to their int8 stream
// arguments (pfb parameters, sizes, strides, alignment, history aliasing).
qc_status api_check_stream_args(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                                const qc_pfb_params* p, const int8_t* hist, const int8_t* hist_out);
// The library's cached twiddle table exp(-2 pi i e / n), e = 0..n-1, on the
// current device (built once in float64 and rounded to float32).
qc_status api_twiddles(int n, float2** out);

}  // namespace qc
