/* Microbenchmarks of the chip's peaks (not part of the method): built into
 * their own library, libb3d_probe.so, which only the benchmark loads, so
 * that measured (not only published) VALU, HBM and LDS peaks can be stated
 * beside the kernels' rooflines.  Plain pointers and sizes; every call only
 * enqueues one kernel on `stream` (a hipStream_t, NULL = the default
 * stream) and returns 0, -1 for a bad argument (before any launch) or -3
 * when the launch fails.  The caller owns every buffer. */
#pragma once

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* blocks x 256 lanes each run iters x 128 FP32 FMAs in 8 independent
 * chains (2 flops each); out receives one float per lane (device
 * float[blocks * 256]).  1 <= blocks, iters <= 2^20.  Time it on `stream` to
 * measure the chip's FP32 vector FMA rate. */
int32_t b3d_probe_fma(float* out, int32_t blocks, int32_t iters, void* stream);

/* One pass of c = a + 1.5 b over n floats (n a positive multiple of 4;
 * device buffers, 16-byte aligned): 12 n bytes of HBM traffic when the
 * buffers exceed the caches. */
int32_t b3d_probe_hbm(const float* a, const float* b, float* c, int64_t n, void* stream);

/* blocks x 256 lanes each read iters x 32 16-byte LDS words
 * (conflict-free); out: device float[blocks * 256].  1 <= blocks, iters <=
 * 2^20.  Time it on `stream` to measure LDS read bandwidth. */
int32_t b3d_probe_lds(float* out, int32_t blocks, int32_t iters, void* stream);

#ifdef __cplusplus
}
#endif
