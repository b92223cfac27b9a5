// Measurement aids: ceilings of the two resources the detector and the
// pyramid spend most of their time on, measured on the device itself so
// that kernel figures are compared with what the chip delivers rather than
// with an estimate.
//
//  * VALU issue: every lane runs 8 independent float FMA chains (no chain
//    waits on its own previous result: 8 instructions apart), unrolled 16
//    times per loop trip, so the VALU instruction count per wave is
//    128 x iters plus a handful; launched with 8 waves per SIMD.
//  * LDS read bandwidth: every lane reads 16 bytes per ds_read_b128 from a
//    16 KB buffer at conflict-free addresses (consecutive lanes,
//    consecutive 16-byte words), folding them into two sums (two
//    three-input adds per read) so the reads cannot be dropped.
// Block 0's first lane records the shader clock and the constant-rate
// wall clock around its loop, which gives the clock frequency the device
// ran at.
#include "vsfe_internal.h"

namespace vsfe {

__global__ __launch_bounds__(256) void probe_valu_kernel(int iters, float a, float b, float *sink,
                                                         uint64_t *clocks) {
    uint64_t c0 = 0, w0 = 0;
    const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
    if (timer) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    float x0 = (float)threadIdx.x, x1 = x0 + 1.f, x2 = x0 + 2.f, x3 = x0 + 3.f;
    float x4 = x0 + 4.f, x5 = x0 + 5.f, x6 = x0 + 6.f, x7 = x0 + 7.f;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < 16; k++) {
            x0 = __builtin_fmaf(x0, a, b);
            x1 = __builtin_fmaf(x1, a, b);
            x2 = __builtin_fmaf(x2, a, b);
            x3 = __builtin_fmaf(x3, a, b);
            x4 = __builtin_fmaf(x4, a, b);
            x5 = __builtin_fmaf(x5, a, b);
            x6 = __builtin_fmaf(x6, a, b);
            x7 = __builtin_fmaf(x7, a, b);
        }
    }
    const float s = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
    if (s == 1234.5f) sink[blockIdx.x * 256 + threadIdx.x] = s;   // never true for a = 1, b = 0
    if (timer) {
        clocks[0] = clock64() - c0;
        clocks[1] = wall_clock64() - w0;
    }
}

__global__ __launch_bounds__(256) void probe_lds_kernel(int iters, uint32_t *sink, uint64_t *clocks) {
    __shared__ uint4 buf[1024];
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; k++) buf[tid + 256 * k] = make_uint4(tid, k, tid ^ k, 7u * tid);
    __syncthreads();
    uint64_t c0 = 0, w0 = 0;
    const bool timer = blockIdx.x == 0 && tid == 0;
    if (timer) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    // a wave's 16 reads of a trip cover the buffer once, lane l at byte
    // 16 l + 1024 k (immediate offsets from one base); the base flips
    // between lane pairs from trip to trip so the loads stay in the loop
    uint32_t acc0 = 0, acc1 = 0;
    const int lane = tid & 63;
    for (int i = 0; i < iters; i++) {
        const uint4 *p = buf + (lane ^ (i & 1));
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const uint4 v = p[64 * k];
            acc0 += v.x + v.y;
            acc1 += v.z + v.w;
        }
    }
    const uint4 acc = make_uint4(acc0, acc1, 0, 0);
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9E3779B9u) sink[blockIdx.x * 256 + tid] = acc.x;
    if (timer) {
        clocks[0] = clock64() - c0;
        clocks[1] = wall_clock64() - w0;
    }
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t vsfe_probe(int32_t kind, int32_t blocks, int32_t iters, void *sink, uint64_t *clocks,
                              void *stream) {
    if (kind != VSFE_PROBE_VALU && kind != VSFE_PROBE_LDS) return fail(VSFE_EINVAL, "unknown probe");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
        return fail(VSFE_EINVAL, "blocks and iters must be in 1..2^20");
    // bounded work: at most 2^26 block-trips (about 0.1 s of either probe)
    if ((int64_t)blocks * iters > ((int64_t)1 << 26))
        return fail(VSFE_EINVAL, "blocks x iters must be at most 2^26");
    if (!sink || !clocks) return fail(VSFE_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    if (kind == VSFE_PROBE_VALU)
        hipLaunchKernelGGL(probe_valu_kernel, dim3(blocks), dim3(256), 0, st, iters, 1.0f, 0.0f, (float *)sink,
                           clocks);
    else
        hipLaunchKernelGGL(probe_lds_kernel, dim3(blocks), dim3(256), 0, st, iters, (uint32_t *)sink, clocks);
    return check_launch("vsfe_probe");
}
