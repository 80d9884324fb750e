// Sustained int8 matrix-core rate of the device, for the roofline beside the
// published peak: every wave issues back-to-back v_mfma_i32_32x32x32_i8 on
// register operands into 16 independent accumulators, with no memory traffic
// in the loop.  Measurement infrastructure only (libmoco_probe.so, loaded by
// the benchmark); the search never calls it.
#include <hip/hip_runtime.h>

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kBlock = 256;
constexpr int kAcc = 16;

// VARY: every lane's operands are four different pairs of pseudo-random bytes
// (xorshift32), cycled so that consecutive MFMAs see different operands, as
// the correlation's digit planes do; otherwise the same two constant operands
// throughout.  The matrix core's power, and with it the clock it sustains,
// depends on how much its operand bits toggle.
__device__ inline unsigned xorshift32(unsigned x)
{
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

template <bool VARY>
__global__ __launch_bounds__(kBlock, 1) void k_mfma_i8_probe(int iters, int *__restrict__ out)
{
    v16i acc[kAcc];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] = v16i{0};
    v4i a[4], b[4];
    unsigned x = (blockIdx.x * kBlock + threadIdx.x) * 2654435761u + 0x9e3779b9u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (VARY) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                x = xorshift32(x);
                a[j][c] = (int)x;
                x = xorshift32(x);
                b[j][c] = (int)x;
            }
        } else {
            a[j] = v4i{(int)threadIdx.x, 0x01020304, 0x05060708, 0x090a0b0c};
            b[j] = v4i{(int)blockIdx.x, 0x0d0e0f10, 0x11121314, 0x15161718};
        }
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kAcc; ++k)
            acc[k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[k % 4], b[k / 4], acc[k], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int k = 0; k < kAcc; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[k][r];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

}  // namespace

extern "C" {

// Launch `blocks` blocks of four waves, each running `iters` iterations of 16
// MFMAs (32x32x32 int8, 65536 operations each), on `stream`; d_out holds
// blocks * 256 ints.  random_operands: pseudo-random operand bytes that change
// from one MFMA to the next (else constant operands).  Returns the launch status.
int probe_mfma_i8(int blocks, int iters, int random_operands, int *d_out, void *stream)
{
    if (blocks < 1 || iters < 1 || !d_out) return (int)hipErrorInvalidValue;
    if (random_operands)
        k_mfma_i8_probe<true><<<blocks, kBlock, 0, (hipStream_t)stream>>>(iters, d_out);
    else
        k_mfma_i8_probe<false><<<blocks, kBlock, 0, (hipStream_t)stream>>>(iters, d_out);
    return (int)hipGetLastError();
}

// Operations one launch performs.
double probe_mfma_i8_ops(int blocks, int iters)
{
    return (double)blocks * (kBlock / 64) * iters * kAcc * 32.0 * 32.0 * 32.0 * 2.0;
}

}  // extern "C"
