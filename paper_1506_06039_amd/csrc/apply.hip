// The corrected stack and its mean image (sec. 2: every frame moved by the
// translation found for it is the motion-corrected video; sec. 3: the mean of
// the corrected video, each frame black outside its overlap with the
// template).  HBM-bound: one read of every frame and one write of every
// corrected frame.
//
// k_apply: block (1024 pixel positions: 256 threads x four consecutive columns
// of one row, chunk of frames).  Frame k with shift (S,T) gives
// out[k][i][j] = a_k[i+S][j+T] inside the frame, else 0; the thread also sums
// its four pixels over the chunk's frames in frame order into FP64 partial
// sums [chunk][i][j].  k_apply_mean adds the chunks in order and divides by
// the frame count (for uint16 data every sum is an exact integer, so the mean
// is the correctly rounded quotient).
#include <hip/hip_runtime.h>

#include "moco_internal.h"

namespace moco {
namespace {

constexpr int kBlock = 256;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_apply(const T *__restrict__ frames,
                                                  const int32_t *__restrict__ shifts, int nframes,
                                                  int m, int n, int kchunk, T *__restrict__ out,
                                                  double *__restrict__ partial)
{
    const int nq = (n + 3) / 4;
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)m * nq) return;
    const int i = (int)(q / nq), j0 = 4 * (int)(q % nq);
    const int k0 = blockIdx.y * kchunk, k1 = min(nframes, k0 + kchunk);
    const size_t plane = (size_t)m * n;
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = k0; k < k1; ++k) {
        const long long r = (long long)i + shifts[2 * k];
        const long long c0 = (long long)j0 + shifts[2 * k + 1];
        const T *a = frames + (size_t)k * plane;
        const bool rin = r >= 0 && r < m;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const long long c = c0 + e;
            const T v = (rin && c >= 0 && c < n && j0 + e < n) ? a[(size_t)r * n + (size_t)c] : T(0);
            if (j0 + e < n) {
                if (out) out[(size_t)k * plane + (size_t)i * n + j0 + e] = v;
                sum[e] += (double)v;
            }
        }
    }
    if (partial) {
        double *p = partial + (size_t)blockIdx.y * plane + (size_t)i * n + j0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (j0 + e < n) p[e] = sum[e];
    }
}

// Bytes [b, b+16) of the 32 bytes lo:hi (b < 16), as two 64-bit halves.
__device__ __forceinline__ uint64_t funnel(uint64_t lo, uint64_t hi, int b)
{
    return b ? (lo >> (8 * b)) | (hi << (64 - 8 * b)) : lo;
}

// Same result as k_apply, 16 bytes per thread and frame (V = 16/sizeof(T)
// pixels of one row), for a frame plane and an output row length that are
// multiples of V and 16-byte aligned buffers.  A source span inside its row
// comes from two aligned 16-byte loads and a byte shift; spans that cross the
// frame's left or right edge, and the last V pixels of a frame, take the
// per-pixel path.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_apply_vec(const T *__restrict__ frames,
                                                      const int32_t *__restrict__ shifts,
                                                      int nframes, int m, int n, int kchunk,
                                                      T *__restrict__ out,
                                                      double *__restrict__ partial)
{
    constexpr int V = 16 / sizeof(T);
    const int nv = n / V;
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)m * nv) return;
    const int i = (int)(q / nv), j0 = V * (int)(q % nv);
    const int k0 = blockIdx.y * kchunk, k1 = min(nframes, k0 + kchunk);
    const size_t plane = (size_t)m * n;
    double sum[V];
#pragma unroll
    for (int e = 0; e < V; ++e) sum[e] = 0.0;
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
        const long long r = (long long)i + shifts[2 * k];
        const long long c0 = (long long)j0 + shifts[2 * k + 1];
        const T *a = frames + (size_t)k * plane;
        union {
            uint64_t u[2];
            T v[V];
        } x;
        // first source pixel, and the 16-byte aligned position at or before it
        const size_t e = (size_t)(r * n + c0), ea = e & ~(size_t)(V - 1);
        if (r < 0 || r >= m || c0 + V <= 0 || c0 >= n) {
            x.u[0] = x.u[1] = 0;
        } else if (c0 >= 0 && c0 + V <= n && (ea == e || ea + 2 * V <= plane)) {
            const uint4 w0 = *(const uint4 *)(a + ea);
            const uint4 w1 = (ea == e) ? uint4{0, 0, 0, 0} : *(const uint4 *)(a + ea + V);
            const uint64_t q0 = ((uint64_t)w0.y << 32) | w0.x, q1 = ((uint64_t)w0.w << 32) | w0.z;
            const uint64_t q2 = ((uint64_t)w1.y << 32) | w1.x, q3 = ((uint64_t)w1.w << 32) | w1.z;
            const int b = (int)(e - ea) * (int)sizeof(T);   // 0..15
            if (b < 8) {
                x.u[0] = funnel(q0, q1, b);
                x.u[1] = funnel(q1, q2, b);
            } else {
                x.u[0] = funnel(q1, q2, b - 8);
                x.u[1] = funnel(q2, q3, b - 8);
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const long long c = c0 + e;
                x.v[e] = (c >= 0 && c < n) ? a[(size_t)r * n + (size_t)c] : T(0);
            }
        }
        if (out) {
            uint4 st;
            st.x = (unsigned)x.u[0];
            st.y = (unsigned)(x.u[0] >> 32);
            st.z = (unsigned)x.u[1];
            st.w = (unsigned)(x.u[1] >> 32);
            *(uint4 *)(out + (size_t)k * plane + (size_t)i * n + j0) = st;
        }
#pragma unroll
        for (int e = 0; e < V; ++e) sum[e] += (double)x.v[e];
    }
    if (partial) {
        double *p = partial + (size_t)blockIdx.y * plane + (size_t)i * n + j0;
#pragma unroll
        for (int e = 0; e < V; ++e) p[e] = sum[e];
    }
}

__global__ __launch_bounds__(kBlock) void k_apply_mean(const double *__restrict__ partial,
                                                       int nchunks, size_t plane, double count,
                                                       double *__restrict__ mean)
{
    for (size_t p = (size_t)blockIdx.x * kBlock + threadIdx.x; p < plane;
         p += (size_t)gridDim.x * kBlock) {
        double s = 0.0;
        for (int c = 0; c < nchunks; ++c) s += partial[(size_t)c * plane + p];
        mean[p] = s / count;
    }
}

}  // namespace

int apply_chunk_frames(int T, int m, int n, size_t budget)
{
    // at most 32 chunks of at least 16 frames, and the partial sums within budget
    const size_t plane_bytes = (size_t)m * n * sizeof(double);
    int nchunks = (T + 15) / 16;
    if (nchunks > 32) nchunks = 32;
    if (nchunks < 1) nchunks = 1;
    while (nchunks > 1 && (size_t)nchunks * plane_bytes > budget) --nchunks;
    if ((size_t)nchunks * plane_bytes > budget) return 0;
    return (T + nchunks - 1) / nchunks;
}

hipError_t launch_apply(const void *frames, moco_dtype dt, const int32_t *shifts, int T, int m,
                        int n, int kchunk, void *out, double *partial, double *mean,
                        hipStream_t st)
{
    clear_stale_error();
    if (T == 0) return hipSuccess;
    const long long quads = (long long)m * ((n + 3) / 4);
    const int nchunks = (T + kchunk - 1) / kchunk;
    const long long bx = (quads + kBlock - 1) / kBlock;
    if (bx > INT32_MAX || nchunks > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)bx, nchunks);
    double *part = mean ? partial : nullptr;
    const size_t esz = dt == MOCO_U16 ? 2 : 4;
    const int V = (int)(16 / esz);
    const bool vec = n % V == 0 && ((uintptr_t)frames & 15) == 0 &&
                     (!out || ((uintptr_t)out & 15) == 0);
    if (vec) {
        const long long units = (long long)m * (n / V);
        const long long bv = (units + kBlock - 1) / kBlock;
        if (bv > INT32_MAX) return hipErrorInvalidValue;
        dim3 gv((unsigned)bv, nchunks);
        if (dt == MOCO_U16)
            k_apply_vec<uint16_t><<<gv, kBlock, 0, st>>>((const uint16_t *)frames, shifts, T, m, n,
                                                         kchunk, (uint16_t *)out, part);
        else
            k_apply_vec<float><<<gv, kBlock, 0, st>>>((const float *)frames, shifts, T, m, n,
                                                      kchunk, (float *)out, part);
    } else if (dt == MOCO_U16)
        k_apply<uint16_t><<<grid, kBlock, 0, st>>>((const uint16_t *)frames, shifts, T, m, n,
                                                   kchunk, (uint16_t *)out, part);
    else
        k_apply<float><<<grid, kBlock, 0, st>>>((const float *)frames, shifts, T, m, n, kchunk,
                                                (float *)out, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !mean) return e;
    const size_t plane = (size_t)m * n;
    size_t g = (plane + kBlock - 1) / kBlock;
    if (g > 65535) g = 65535;
    k_apply_mean<<<(unsigned)g, kBlock, 0, st>>>(partial, nchunks, plane, (double)T, mean);
    return hipGetLastError();
}

}  // namespace moco
