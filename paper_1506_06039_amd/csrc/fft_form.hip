// FFT form of the correlation (sec. 2: h from the transforms of the
// zero-padded frame and template, FP64 complex arithmetic).
//
// With P >= m'+w-1 and Q >= n'+w-1, c = IFFT(FFT(a') * conj(FFT(b'))) on the
// P x Q grid has c[s mod P][t mod Q] = h(s,t) for |s|,|t| <= w-1: the padding
// keeps every wrapped index in the zero border.  (The paper pads to m+w by n+w
// and flips b; the conjugate form needs one row and column less.)
//
// Three passes per frame, each a batch of one-dimensional transforms held in
// LDS (mixed-radix Stockham: radices 8, 4, 2, 3, 5, self-sorting, one LDS
// read and one LDS write of every element per radix pass):
//   rows    two real grid rows packed as one complex row, length Q; the two
//           half spectra (Q/2+1 bins) are split off and written bin-major,
//           S1[k][i];
//   columns for each bin k, the column S1[k][0..m'), zero-padded to P,
//           forward; times conj of the template's spectrum; inverse; only the
//           2w-1 outputs at s mod P are kept, S2[s][k];
//   rows    two rows of S2, each extended to its Hermitian length-Q spectrum,
//           packed as one complex row, inverse; the 2w-1 outputs at t mod Q
//           of the real and imaginary parts are the two rows of h, times
//           1/(PQ).
// The template's spectrum is the first two passes without the product and
// inverse, once per template.
#include <hip/hip_runtime.h>

#include "grid_src.h"
#include "moco_internal.h"

namespace moco {
namespace {

constexpr int kBlock = 256;
constexpr size_t kLdsBudget = 32 * 1024;  // LDS bytes a block's two buffers may use

// Complex type of each working precision: FP64 (the FFT forms) and FP32 (the
// plain single-precision form on centred grids).
template <typename R>
struct Cx;
template <>
struct Cx<double> {
    using T = double2;
};
template <>
struct Cx<float> {
    using T = float2;
};

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return {a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return {a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b)
{
    return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
template <typename C>
__device__ __forceinline__ C cmulc(C a, C b)
{
    return {fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y)};
}
template <typename C, typename R>
__device__ __forceinline__ C cscale(C a, R s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C>
__device__ __forceinline__ C rot(C a)
{
    return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

// Small DFTs in registers: y_k = sum_q v_q e^{-+2 pi i qk/R} (minus: forward).
template <int R, bool INV, typename C>
struct Dft;

template <bool INV, typename C>
struct Dft<2, INV, C> {
    __device__ static void run(C (&v)[2])
    {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <bool INV, typename C>
struct Dft<4, INV, C> {
    __device__ static void run(C (&v)[4])
    {
        C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        C t2 = cadd(v[1], v[3]), t3 = rot<INV>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <bool INV, typename C>
struct Dft<8, INV, C> {
    __device__ static void run(C (&v)[8])
    {
        using R = decltype(v[0].x);
        constexpr R h = (R)0.70710678118654752440;  // sqrt(1/2)
        C e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, INV, C>::run(e);
        Dft<4, INV, C>::run(o);
        // o_k times e^{-+2 pi i k/8}
        const C o1 = INV ? C{h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)}
                         : C{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
        const C o2 = rot<INV>(o[2]);
        const C o3 = INV ? C{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)}
                         : C{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

template <bool INV, typename C>
struct Dft<3, INV, C> {
    __device__ static void run(C (&v)[3])
    {
        using R = decltype(v[0].x);
        constexpr R r3 = (R)0.86602540378443864676;  // sqrt(3)/2
        const C t1 = cadd(v[1], v[2]);
        const C t2 = {v[0].x - (R)0.5 * t1.x, v[0].y - (R)0.5 * t1.y};
        const C d = rot<INV>(cscale(csub(v[1], v[2]), r3));
        v[0] = cadd(v[0], t1);
        v[1] = cadd(t2, d);
        v[2] = csub(t2, d);
    }
};

template <bool INV, typename C>
struct Dft<5, INV, C> {
    __device__ static void run(C (&v)[5])
    {
        using R = decltype(v[0].x);
        constexpr R c1 = (R)0.30901699437494742410;   // cos(2 pi/5) = (sqrt 5 - 1)/4
        constexpr R c2 = (R)-0.80901699437494742410;  // cos(4 pi/5) = -(sqrt 5 + 1)/4
        constexpr R s1 = (R)0.95105651629515357212;   // sin(2 pi/5)
        constexpr R s2 = (R)0.58778525229247312917;   // sin(4 pi/5)
        const C b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
        const C d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
        const C p1 = {v[0].x + c1 * b1.x + c2 * b2.x, v[0].y + c1 * b1.y + c2 * b2.y};
        const C p2 = {v[0].x + c2 * b1.x + c1 * b2.x, v[0].y + c2 * b1.y + c1 * b2.y};
        // -+i (s1 d1 + s2 d2) and -+i (s2 d1 - s1 d2)
        const C q1 = rot<INV>(C{s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y});
        const C q2 = rot<INV>(C{s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y});
        v[0] = cadd(v[0], cadd(b1, b2));
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    }
};

__device__ __forceinline__ int divq(int x, unsigned long long mag)
{
    // floor(x / d) for mag = ceil(2^32 / d), exact while x * d < 2^32
    return (int)(((unsigned long long)(unsigned)x * mag) >> 32);
}

// One Stockham pass of radix R over `rows` rows of length N: butterfly j
// (0 <= j < N/R) reads in[j + r N/R], r < R, twiddles them by w_N^{r (j mod
// Ns) N/(Ns R)}, transforms and writes out[(j div Ns) Ns R + (j mod Ns) + r Ns].
// tw: the length-N twiddle table, held in LDS by the block.
template <int R, bool INV, typename C>
__device__ __forceinline__ void fft_pass(const C *in, C *out, int rows, int N, int Ns,
                                         unsigned long long mag_nr, unsigned long long mag_ns,
                                         const C *tw)
{
    const int NR = N / R;
    const int stw = N / (Ns * R);
    const int total = rows * NR;
    for (int idx = threadIdx.x; idx < total; idx += kBlock) {
        const int row = divq(idx, mag_nr), j = idx - row * NR;
        const int jq = divq(j, mag_ns), jm = j - jq * Ns;
        const C *src = in + row * N + j;
        C v[R];
        v[0] = src[0];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const C x = src[r * NR];
            C t = tw[r * jm * stw];
            if (INV) t.y = -t.y;
            v[r] = cmul(x, t);
        }
        Dft<R, INV, C>::run(v);
        C *dst = out + row * N + jq * Ns * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r * Ns] = v[r];
    }
}

// Transform `rows` rows held in a; b is the other buffer.  Returns the buffer
// that holds the result.  Ends with a barrier.
template <bool INV, typename C>
__device__ C *fft_lds(C *a, C *b, int rows, const FftPlan &pl, const C *tw)
{
    for (int p = 0; p < pl.npass; ++p) {
        switch (pl.radix[p]) {
        case 8: fft_pass<8, INV>(a, b, rows, pl.n, pl.ns[p], pl.mag_nr[p], pl.mag_ns[p], tw); break;
        case 4: fft_pass<4, INV>(a, b, rows, pl.n, pl.ns[p], pl.mag_nr[p], pl.mag_ns[p], tw); break;
        case 2: fft_pass<2, INV>(a, b, rows, pl.n, pl.ns[p], pl.mag_nr[p], pl.mag_ns[p], tw); break;
        case 3: fft_pass<3, INV>(a, b, rows, pl.n, pl.ns[p], pl.mag_nr[p], pl.mag_ns[p], tw); break;
        default: fft_pass<5, INV>(a, b, rows, pl.n, pl.ns[p], pl.mag_nr[p], pl.mag_ns[p], tw); break;
        }
        __syncthreads();
        C *t = a;
        a = b;
        b = t;
    }
    return a;
}

// Largest of one value per thread of the block, stored by thread 0 (every
// thread calls it; it synchronises the block).
template <typename R>
__device__ void block_max_store(R v, R *dst)
{
    __shared__ R wm[1024 / 64];   // any block of at most 1024 threads
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if (threadIdx.x % 64 == 0) wm[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        R m = wm[0];
        for (int k = 1; k < (int)(blockDim.x / 64); ++k) m = fmax(m, wm[k]);
        *dst = m;
    }
}

// The block's copy of a length-n twiddle table (no barrier).
template <typename C>
__device__ __forceinline__ void load_twiddles(const C *__restrict__ g, int n, C *lds)
{
    for (int k = threadIdx.x; k < n; k += kBlock) lds[k] = g[k];
}

// Pass 1: rows.  Block (group of rp row pairs, frame).  src: the frames' grid
// (SRC 0: mg x ng FP64) or their pixels (m x n; see grid_at).  Each grid value
// less `center` (0 in the FP64 forms) enters the transform in precision R.
// s1: [frame][qh][mg] complex.
template <int SRC, typename R>
__global__ __launch_bounds__(kBlock) void k_fft_rows(const void *__restrict__ src, int m, int n,
                                                     int mg, int ng, int rp, FftPlan pq,
                                                     const typename Cx<R>::T *__restrict__ twq,
                                                     double center,
                                                     typename Cx<R>::T *__restrict__ s1,
                                                     const int32_t *__restrict__ only)
{
    using C = typename Cx<R>::T;
    if (only && !only[blockIdx.y]) return;
    extern __shared__ double lds_d[];
    C *lds = (C *)lds_d;
    const int Q = pq.n, qh = Q / 2 + 1;
    const int npairs = (mg + 1) / 2;
    const int pair0 = blockIdx.x * rp, np = min(rp, npairs - pair0);
    const void *a = grid_frame<SRC>(src, blockIdx.y, m, n, mg, ng);
    C *tw = lds, *bufa = lds + Q, *bufb = bufa + (size_t)rp * Q;
    load_twiddles(twq, Q, tw);
    for (int pr = 0; pr < np; ++pr) {
        const int r = 2 * (pair0 + pr);
        const bool two = r + 1 < mg;
        if (SRC == 1 && (n & 3) == 0) {
            // uint16 box means, two grid columns per thread: one 8-byte load per
            // pixel row (n a multiple of 4 keeps it aligned and ng even)
            const uint16_t *px = (const uint16_t *)a;
            for (int j = 2 * threadIdx.x; j < Q; j += 2 * kBlock) {
                C v0{0, 0}, v1{0, 0};
                if (j < ng) {
                    int s[2][2];
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        s[k][0] = s[k][1] = 0;
                        if (k == 1 && !two) break;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const uint2 q = *(const uint2 *)(px + (size_t)(2 * (r + k) + h) * n + 2 * j);
                            s[k][0] += (int)(q.x & 0xffffu) + (int)(q.x >> 16);
                            s[k][1] += (int)(q.y & 0xffffu) + (int)(q.y >> 16);
                        }
                    }
                    const double c1 = two ? center : 0.0;
                    v0 = C{(R)(0.25 * (double)s[0][0] - center), (R)(0.25 * (double)s[1][0] - c1)};
                    v1 = C{(R)(0.25 * (double)s[0][1] - center), (R)(0.25 * (double)s[1][1] - c1)};
                }
                bufa[pr * Q + j] = v0;
                if (j + 1 < Q) bufa[pr * Q + j + 1] = v1;
            }
            continue;
        }
        for (int j = threadIdx.x; j < Q; j += kBlock)
            bufa[pr * Q + j] =
                j < ng ? C{(R)(grid_at<SRC>(a, n, ng, r, j) - center),
                           two ? (R)(grid_at<SRC>(a, n, ng, r + 1, j) - center) : (R)0}
                       : C{0, 0};
    }
    __syncthreads();
    const C *z = fft_lds<false>(bufa, bufb, np, pq, tw);
    // Z = X + iY with X, Y the spectra of the real rows r, r+1:
    // X_k = (Z_k + conj Z_{-k})/2, Y_k = (Z_k - conj Z_{-k})/(2i)
    C *out = s1 + (size_t)blockIdx.y * qh * mg;
    for (int idx = threadIdx.x; idx < np * qh; idx += kBlock) {
        const int k = idx / np, pr = idx - k * np;
        const C zk = z[pr * Q + k], zc = z[pr * Q + (k == 0 ? 0 : Q - k)];
        const int r = 2 * (pair0 + pr);
        out[(size_t)k * mg + r] = C{(R)0.5 * (zk.x + zc.x), (R)0.5 * (zk.y - zc.y)};
        if (r + 1 < mg) out[(size_t)k * mg + r + 1] = C{(R)0.5 * (zk.y + zc.y), (R)0.5 * (zc.x - zk.x)};
    }
}

// Pass 2: columns.  Block (group of kb bins, frame).  SPEC: write the full
// column transforms to spec[k][p] (the template).  Otherwise multiply by
// conj(spec), inverse, keep s = -(w-1) .. w-1 into s2[frame][s+w-1][k].
// xmax (may be null): the largest |X_k|^2 of the frame's spectrum over the
// block's bins, at xmax[frame][block].
template <bool SPEC, typename R>
__global__ __launch_bounds__(kBlock) void k_fft_cols(const typename Cx<R>::T *__restrict__ s1,
                                                     int mg, int qh, int kb, int w, FftPlan pp,
                                                     const typename Cx<R>::T *__restrict__ twp,
                                                     const typename Cx<R>::T *__restrict__ spec_in,
                                                     typename Cx<R>::T *__restrict__ spec_out,
                                                     typename Cx<R>::T *__restrict__ s2,
                                                     const int32_t *__restrict__ only,
                                                     R *__restrict__ xmax)
{
    using C = typename Cx<R>::T;
    if (only && !only[blockIdx.y]) return;
    extern __shared__ double lds_d[];
    C *lds = (C *)lds_d;
    const int P = pp.n;
    const int k0 = blockIdx.x * kb, nk = min(kb, qh - k0);
    const C *col = s1 + (size_t)blockIdx.y * qh * mg + (size_t)k0 * mg;
    C *tw = lds, *bufa = lds + P, *bufb = bufa + (size_t)kb * P;
    load_twiddles(twp, P, tw);
    for (int kk = 0; kk < nk; ++kk)
        for (int p = threadIdx.x; p < P; p += kBlock)
            bufa[kk * P + p] = p < mg ? col[(size_t)kk * mg + p] : C{0, 0};
    __syncthreads();
    C *v = fft_lds<false>(bufa, bufb, nk, pp, tw);
    if (SPEC) {
        for (int kk = 0; kk < nk; ++kk)
            for (int p = threadIdx.x; p < P; p += kBlock)
                spec_out[(size_t)(k0 + kk) * P + p] = v[kk * P + p];
        return;
    }
    R m2 = 0;
    for (int kk = 0; kk < nk; ++kk)
        for (int p = threadIdx.x; p < P; p += kBlock) {
            const C x = v[kk * P + p];
            m2 = fmax(m2, x.x * x.x + x.y * x.y);
            v[kk * P + p] = cmulc(x, spec_in[(size_t)(k0 + kk) * P + p]);
        }
    if (xmax) block_max_store(m2, xmax + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
    __syncthreads();
    C *u = fft_lds<true>(v, v == bufa ? bufb : bufa, nk, pp, tw);
    const int W = 2 * w - 1;
    C *out = s2 + (size_t)blockIdx.y * W * qh;
    for (int idx = threadIdx.x; idx < W * nk; idx += kBlock) {
        const int si = idx / nk, kk = idx - si * nk;
        const int s = si - (w - 1);
        out[(size_t)si * qh + k0 + kk] = u[kk * P + (s < 0 ? s + P : s)];
    }
}

// Pass 3: rows back.  Block (group of rp pairs of shift rows, frame).  Rows
// si, si+1 of s2 are half spectra of real rows; Z = X + iY over the full
// length Q, inverse; h[si][t] = Re z_t / PQ, h[si+1][t] = Im z_t / PQ (the
// scale applied in FP64).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fft_rows_back(const typename Cx<R>::T *__restrict__ s2,
                                                          int qh, int w, int rp, double scale,
                                                          FftPlan pq,
                                                          const typename Cx<R>::T *__restrict__ twq,
                                                          double *__restrict__ h,
                                                          const int32_t *__restrict__ only)
{
    using C = typename Cx<R>::T;
    if (only && !only[blockIdx.y]) return;
    extern __shared__ double lds_d[];
    C *lds = (C *)lds_d;
    const int Q = pq.n, W = 2 * w - 1;
    const int npairs = (W + 1) / 2;
    const int pair0 = blockIdx.x * rp, np = min(rp, npairs - pair0);
    const C *src = s2 + (size_t)blockIdx.y * W * qh;
    C *tw = lds, *bufa = lds + Q, *bufb = bufa + (size_t)rp * Q;
    load_twiddles(twq, Q, tw);
    for (int pr = 0; pr < np; ++pr) {
        const int si = 2 * (pair0 + pr);
        const C *x = src + (size_t)si * qh;
        const C *y = si + 1 < W ? x + qh : nullptr;
        for (int k = threadIdx.x; k < Q; k += kBlock) {
            // X_k for k >= qh is conj X_{Q-k}
            const bool lo = k < qh;
            const int kk = lo ? k : Q - k;
            C X = x[kk], Y = y ? y[kk] : C{0, 0};
            if (!lo) {
                X.y = -X.y;
                Y.y = -Y.y;
            }
            bufa[pr * Q + k] = C{X.x - Y.y, X.y + Y.x};
        }
    }
    __syncthreads();
    const C *z = fft_lds<true>(bufa, bufb, np, pq, tw);
    double *out = h + (size_t)blockIdx.y * W * W;
    for (int idx = threadIdx.x; idx < np * W; idx += kBlock) {
        const int pr = idx / W, ti = idx - pr * W;
        const int t = ti - (w - 1);
        const C v = z[pr * Q + (t < 0 ? t + Q : t)];
        const int si = 2 * (pair0 + pr);
        out[(size_t)si * W + ti] = (double)v.x * scale;
        if (si + 1 < W) out[(size_t)(si + 1) * W + ti] = (double)v.y * scale;
    }
}

// Rows of length n a block holds in its two LDS buffers (elements of `esz`
// bytes), and the LDS bytes that takes with the length-n twiddle table.
int rows_per_block(int n, size_t esz = sizeof(double2))
{
    int r = (int)(kLdsBudget / (2 * (size_t)n * esz));
    return r < 1 ? 1 : (r > 8 ? 8 : r);
}

size_t block_lds(int rows, int n, size_t esz) { return (2 * (size_t)rows + 1) * n * esz; }

// ---------------------------------------------------------------------------
// Wave-level transforms for the lengths the workloads use (compile-time
// plans).  A transform of length N is owned by T consecutive lanes of one wave
// and lives in an LDS buffer of its own; each radix pass loads every input of
// the lane's butterflies, transforms them in registers and stores the outputs
// back into the same buffer.  The lanes of a wave issue each instruction
// together and LDS operations of a wave complete in order, so a pass's loads
// (all lanes) precede its stores: passes need no barrier, only a compiler
// fence.  The block synchronises twice: after staging the inputs and before
// the outputs leave, both block-cooperative and coalesced.

// The same radices as fft_plan, applied in the same order.
struct WPlan {
    int npass;
    int radix[kFftMaxPass];
    int ns[kFftMaxPass];
};

constexpr WPlan make_wplan(int n)
{
    WPlan p{};
    int c[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int x = n;
    while (x % 8 == 0) x /= 8, ++c[8];
    while (x % 4 == 0) x /= 4, ++c[4];
    while (x % 2 == 0) x /= 2, ++c[2];
    while (x % 3 == 0) x /= 3, ++c[3];
    while (x % 5 == 0) x /= 5, ++c[5];
    const int order[5] = {2, 3, 4, 5, 8};
    int ns = 1;
    for (int o = 0; o < 5; ++o)
        for (int k = 0; k < c[order[o]]; ++k) {
            p.radix[p.npass] = order[o];
            p.ns[p.npass] = ns;
            ns *= order[o];
            ++p.npass;
        }
    return p;
}

template <int N>
struct WPlanOf {
    static constexpr WPlan pl = make_wplan(N);
};

// Pass P and the ones after it of a length-N transform in `buf`; tl: the
// lane's index among the transform's T lanes; tw: the length-N twiddle table.
template <typename C, int N, int T, bool INV, int P>
struct WPass {
    __device__ static void run(C *buf, const C *tw, int tl)
    {
        constexpr WPlan pl = WPlanOf<N>::pl;
        if constexpr (P < pl.npass) {
            constexpr int Rr = pl.radix[P], Ns = pl.ns[P];
            constexpr int NR = N / Rr, NB = (NR + T - 1) / T, stw = N / (Ns * Rr);
            C v[NB][Rr];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = tl + T * b;
                if (NR % T == 0 || j < NR) {
#pragma unroll
                    for (int r = 0; r < Rr; ++r) v[b][r] = buf[j + r * NR];
                }
            }
            asm volatile("" ::: "memory");
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int j = tl + T * b;
                if (NR % T == 0 || j < NR) {
                    const int jm = j % Ns, jq = j / Ns;
#pragma unroll
                    for (int r = 1; r < Rr; ++r) {
                        C t = tw[r * jm * stw];
                        if (INV) t.y = -t.y;
                        v[b][r] = cmul(v[b][r], t);
                    }
                    Dft<Rr, INV, C>::run(v[b]);
                    C *dst = buf + jq * Ns * Rr + jm;
#pragma unroll
                    for (int r = 0; r < Rr; ++r) dst[r * Ns] = v[b][r];
                }
            }
            asm volatile("" ::: "memory");
            WPass<C, N, T, INV, P + 1>::run(buf, tw, tl);
        }
    }
};

constexpr int kWPad = 0;                  // elements between transform buffers

// Threads per block of the wave-level kernels: eight waves in FP32, four in
// FP64.  Measured on MI355X (three transform kernels per 2000 frames of the
// 512x512 stack; the 10000-frame 256x256 stack): FP32 0.94 -> 0.875 ms and
// 5.08 -> 4.65 ms with eight waves, FP64 1.40 -> 1.47 ms.
template <typename R>
constexpr int wave_block() { return sizeof(R) == 4 ? 512 : 256; }

template <int N, int T, int B>
struct WGeom {
    static constexpr int per_wave = 64 / T;
    static constexpr int per_block = per_wave * (B / 64);
    static constexpr int stride = N + kWPad;
};

// Rows: packed pairs of real grid rows, as k_fft_rows.
template <int SRC, typename R, int Q, int T>
__global__ __launch_bounds__(wave_block<R>()) void k_wrows(const void *__restrict__ src, int m, int n,
                                                      int mg, int ng,
                                                      const typename Cx<R>::T *__restrict__ twq,
                                                      double center,
                                                      typename Cx<R>::T *__restrict__ s1,
                                                      const int32_t *__restrict__ only)
{
    using C = typename Cx<R>::T;
    using G = WGeom<Q, T, wave_block<R>()>;
    constexpr int kWaveBlock = wave_block<R>();
    if (only && !only[blockIdx.y]) return;
    extern __shared__ double lds_d[];
    C *tw = (C *)lds_d, *bufs = tw + Q;
    constexpr int qh = Q / 2 + 1;
    const int npairs = (mg + 1) / 2;
    const int pair0 = blockIdx.x * G::per_block, np = min(G::per_block, npairs - pair0);
    const void *a = grid_frame<SRC>(src, blockIdx.y, m, n, mg, ng);
    load_twiddles(twq, Q, tw);
    for (int idx = threadIdx.x; idx < np * Q; idx += kWaveBlock) {
        const int pr = idx / Q, j = idx - pr * Q;
        const int r = 2 * (pair0 + pr);
        const bool two = r + 1 < mg;
        C v{0, 0};
        if (j < ng) {
            v.x = (R)(grid_at<SRC>(a, n, ng, r, j) - center);
            if (two) v.y = (R)(grid_at<SRC>(a, n, ng, r + 1, j) - center);
        }
        bufs[pr * G::stride + j] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x % 64, tr = (threadIdx.x / 64) * G::per_wave + lane / T;
    if (tr < np) WPass<C, Q, T, false, 0>::run(bufs + tr * G::stride, tw, lane % T);
    __syncthreads();
    C *out = s1 + (size_t)blockIdx.y * qh * mg;
    for (int idx = threadIdx.x; idx < np * qh; idx += kWaveBlock) {
        const int k = idx / np, pr = idx - k * np;
        const C *z = bufs + pr * G::stride;
        const C zk = z[k], zc = z[k == 0 ? 0 : Q - k];
        const int r = 2 * (pair0 + pr);
        out[(size_t)k * mg + r] = C{(R)0.5 * (zk.x + zc.x), (R)0.5 * (zk.y - zc.y)};
        if (r + 1 < mg) out[(size_t)k * mg + r + 1] = C{(R)0.5 * (zk.y + zc.y), (R)0.5 * (zc.x - zk.x)};
    }
}

// Columns: forward, times conj(spec), inverse, the 2w-1 outputs kept, and
// the block's largest |X_k|^2 when xmax is given, as k_fft_cols<false>.
template <typename R, int P, int T>
__global__ __launch_bounds__(wave_block<R>()) void k_wcols(const typename Cx<R>::T *__restrict__ s1,
                                                      int mg, int qh, int w,
                                                      const typename Cx<R>::T *__restrict__ twp,
                                                      const typename Cx<R>::T *__restrict__ spec,
                                                      typename Cx<R>::T *__restrict__ s2,
                                                      const int32_t *__restrict__ only,
                                                      R *__restrict__ xmax)
{
    using C = typename Cx<R>::T;
    using G = WGeom<P, T, wave_block<R>()>;
    constexpr int kWaveBlock = wave_block<R>();
    if (only && !only[blockIdx.y]) return;
    extern __shared__ double lds_d[];
    C *tw = (C *)lds_d, *bufs = tw + P;
    const int k0 = blockIdx.x * G::per_block, nk = min(G::per_block, qh - k0);
    const C *col = s1 + (size_t)blockIdx.y * qh * mg + (size_t)k0 * mg;
    load_twiddles(twp, P, tw);
    for (int idx = threadIdx.x; idx < nk * P; idx += kWaveBlock) {
        const int kk = idx / P, p = idx - kk * P;
        bufs[kk * G::stride + p] = p < mg ? col[(size_t)kk * mg + p] : C{0, 0};
    }
    __syncthreads();
    const int lane = threadIdx.x % 64, tr = (threadIdx.x / 64) * G::per_wave + lane / T;
    const int tl = lane % T;
    R m2 = 0;
    if (tr < nk) {
        C *buf = bufs + tr * G::stride;
        WPass<C, P, T, false, 0>::run(buf, tw, tl);
        const C *sp = spec + (size_t)(k0 + tr) * P;
#pragma unroll 4
        for (int p = tl; p < P; p += T) {
            const C x = buf[p];
            m2 = fmax(m2, x.x * x.x + x.y * x.y);
            buf[p] = cmulc(x, sp[p]);
        }
        asm volatile("" ::: "memory");
        WPass<C, P, T, true, 0>::run(buf, tw, tl);
    }
    if (xmax) block_max_store(m2, xmax + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
    __syncthreads();
    const int W = 2 * w - 1;
    C *out = s2 + (size_t)blockIdx.y * W * qh;
    for (int idx = threadIdx.x; idx < W * nk; idx += kWaveBlock) {
        const int si = idx / nk, kk = idx - si * nk;
        const int s = si - (w - 1);
        out[(size_t)si * qh + k0 + kk] = bufs[kk * G::stride + (s < 0 ? s + P : s)];
    }
}

// Rows back: packed pairs of shift rows, as k_fft_rows_back.
template <typename R, int Q, int T>
__global__ __launch_bounds__(wave_block<R>()) void k_wback(const typename Cx<R>::T *__restrict__ s2,
                                                      int qh, int w, double scale,
                                                      const typename Cx<R>::T *__restrict__ twq,
                                                      double *__restrict__ h,
                                                      const int32_t *__restrict__ only)
{
    using C = typename Cx<R>::T;
    using G = WGeom<Q, T, wave_block<R>()>;
    constexpr int kWaveBlock = wave_block<R>();
    if (only && !only[blockIdx.y]) return;
    extern __shared__ double lds_d[];
    C *tw = (C *)lds_d, *bufs = tw + Q;
    const int W = 2 * w - 1;
    const int npairs = (W + 1) / 2;
    const int pair0 = blockIdx.x * G::per_block, np = min(G::per_block, npairs - pair0);
    const C *src = s2 + (size_t)blockIdx.y * W * qh;
    load_twiddles(twq, Q, tw);
    for (int idx = threadIdx.x; idx < np * Q; idx += kWaveBlock) {
        const int pr = idx / Q, k = idx - pr * Q;
        const int si = 2 * (pair0 + pr);
        const bool lo = k < qh;
        const int kk = lo ? k : Q - k;
        C X = src[(size_t)si * qh + kk];
        C Y = si + 1 < W ? src[(size_t)(si + 1) * qh + kk] : C{0, 0};
        if (!lo) {
            X.y = -X.y;
            Y.y = -Y.y;
        }
        bufs[pr * G::stride + k] = C{X.x - Y.y, X.y + Y.x};
    }
    __syncthreads();
    const int lane = threadIdx.x % 64, tr = (threadIdx.x / 64) * G::per_wave + lane / T;
    if (tr < np) WPass<C, Q, T, true, 0>::run(bufs + tr * G::stride, tw, lane % T);
    __syncthreads();
    double *out = h + (size_t)blockIdx.y * W * W;
    for (int idx = threadIdx.x; idx < np * W; idx += kWaveBlock) {
        const int pr = idx / W, ti = idx - pr * W;
        const int t = ti - (w - 1);
        const C v = bufs[pr * G::stride + (t < 0 ? t + Q : t)];
        const int si = 2 * (pair0 + pr);
        out[(size_t)si * W + ti] = (double)v.x * scale;
        if (si + 1 < W) out[(size_t)(si + 1) * W + ti] = (double)v.y * scale;
    }
}

// Lanes per transform: a whole wave.  Measured on MI355X at 288 and 320 points
// against 16 and 32 lanes (several transforms per wave, more registers per
// lane, fewer waves per SIMD) and against the block-level kernels: 64 lanes
// were fastest in both precisions (the 512x512 stack's three transform
// kernels: FP32 1.02 ms against 1.38 for the block kernels, FP64 1.41 against
// 2.18, per 2000 frames), with or without padding between the buffers.
template <typename R>
constexpr int wave_lanes() { return 64; }

template <typename R, int N>
size_t wave_lds()
{
    using G = WGeom<N, wave_lanes<R>(), wave_block<R>()>;
    return ((size_t)N + (size_t)G::per_block * G::stride) * sizeof(typename Cx<R>::T);
}

// The lengths with a wave-level kernel; others take the block-level kernels.
// Measured on MI355X against the block kernels: faster at 144, 288, 300, 320,
// 384 and 512 points (384 x 384, 1000 frames: FP64 1.86 -> 1.30 ms, FP32 1.22
// -> 0.72 ms; 512 x 512: FP64 3.47 -> 2.42 ms, FP32 1.89 -> 1.21 ms, three
// radix-8 passes with every lane busy); slower at 360 (3,3,5,8: the radix-8 pass keeps 45 of 64 lanes
// busy; transforms of the 256x256 grid at w = 85: FP32 2.58 -> 1.92 ms, FP64
// 3.70 -> 3.29 ms per 2000 frames with the block kernels), 400, 432, 450 and
// 480 (5-18% slower: passes that leave lanes idle), which keep the block
// kernels.
#define MOCO_WAVE_LENGTHS(X) X(144) X(160) X(180) X(240) X(256) X(270) X(288) X(300) X(320) X(384) X(512)

bool wave_length(int n)
{
#define MOCO_WL_CASE(L) case L:
    switch (n) {
        MOCO_WAVE_LENGTHS(MOCO_WL_CASE)
        return true;
    default:
        return false;
    }
#undef MOCO_WL_CASE
}

template <typename R, int SRC, int Q>
void wrows_launch(const void *src, int C, const Geom &g, const typename Cx<R>::T *twq,
                  double center, typename Cx<R>::T *s1, hipStream_t st, const int32_t *only)
{
    constexpr int T = wave_lanes<R>();
    const int npairs = (g.mg + 1) / 2;
    const int pb = WGeom<Q, T, wave_block<R>()>::per_block;
    k_wrows<SRC, R, Q, T><<<dim3((npairs + pb - 1) / pb, C), wave_block<R>(), wave_lds<R, Q>(),
                            st>>>(
        src, g.m, g.n, g.mg, g.ng, twq, center, s1, only);
}

template <typename R, int SRC>
bool wrows(const void *src, int C, const Geom &g, const typename Cx<R>::T *twq, double center,
           typename Cx<R>::T *s1, hipStream_t st, int Q, const int32_t *only)
{
#define MOCO_WL_ROWS(L) \
    case L: wrows_launch<R, SRC, L>(src, C, g, twq, center, s1, st, only); return true;
    switch (Q) {
        MOCO_WAVE_LENGTHS(MOCO_WL_ROWS)
    default:
        return false;
    }
#undef MOCO_WL_ROWS
}

template <typename R>
bool wcols(const typename Cx<R>::T *s1, int C, const Geom &g, const FftTmpl &ft,
           const typename Cx<R>::T *twp, const typename Cx<R>::T *spec, typename Cx<R>::T *s2,
           hipStream_t st, const int32_t *only, R *xmax, int *nxb)
{
    constexpr int T = wave_lanes<R>();
#define MOCO_WL_COLS(L)                                                                       \
    case L: {                                                                                 \
        const int pb = WGeom<L, T, wave_block<R>()>::per_block;                               \
        *nxb = (ft.qh + pb - 1) / pb;                                                         \
        k_wcols<R, L, T><<<dim3(*nxb, C), wave_block<R>(), wave_lds<R, L>(), st>>>(            \
            s1, g.mg, ft.qh, g.w, twp, spec, s2, only, xmax);                                 \
        return true;                                                                          \
    }
    switch (ft.pp.n) {
        MOCO_WAVE_LENGTHS(MOCO_WL_COLS)
    default:
        return false;
    }
#undef MOCO_WL_COLS
}

template <typename R>
bool wback(const typename Cx<R>::T *s2, int C, const Geom &g, const FftTmpl &ft,
           const typename Cx<R>::T *twq, double scale, double *h, hipStream_t st,
           const int32_t *only)
{
    constexpr int T = wave_lanes<R>();
    const int npairs = (g.W + 1) / 2;
#define MOCO_WL_BACK(L)                                                                         \
    case L: {                                                                                   \
        const int pb = WGeom<L, T, wave_block<R>()>::per_block;                                 \
        k_wback<R, L, T><<<dim3((npairs + pb - 1) / pb, C), wave_block<R>(), wave_lds<R, L>(),   \
                           st>>>(                                                                \
            s2, ft.qh, g.w, scale, twq, h, only);                                               \
        return true;                                                                            \
    }
    switch (ft.pq.n) {
        MOCO_WAVE_LENGTHS(MOCO_WL_BACK)
    default:
        return false;
    }
#undef MOCO_WL_BACK
}

}  // namespace

// ---- host side ------------------------------------------------------------

static bool smooth235(int x)
{
    for (int p : {2, 3, 5})
        while (x % p == 0) x /= p;
    return x == 1;
}

static int next_smooth(int x)
{
    if (x < 2) x = 2;
    while (!smooth235(x)) ++x;
    return x;
}

bool fft_plan(int n, FftPlan *pl)
{
    if (n < 2 || n > kFftMaxLen || !smooth235(n)) return false;
    FftPlan p{};
    p.n = n;
    int rem = n, ns = 1;
    auto add = [&](int r) {
        p.radix[p.npass] = r;
        p.ns[p.npass] = ns;
        const unsigned long long nr = (unsigned long long)(n / r);
        p.mag_nr[p.npass] = ((1ULL << 32) + nr - 1) / nr;
        p.mag_ns[p.npass] = ((1ULL << 32) + ns - 1) / ns;
        ++p.npass;
        ns *= r;
        rem /= r;
    };
    // the same radices as taking 8s, then 4s, 2s, 3s and 5s, applied smallest
    // first: a pass writes runs of Ns consecutive elements, so the large radix,
    // whose early-pass writes would stride across LDS banks, comes last
    int c8 = 0, c4 = 0, c2 = 0, c3 = 0, c5 = 0, x = n;
    while (x % 8 == 0) x /= 8, ++c8;
    while (x % 4 == 0) x /= 4, ++c4;
    while (x % 2 == 0) x /= 2, ++c2;
    while (x % 3 == 0) x /= 3, ++c3;
    while (x % 5 == 0) x /= 5, ++c5;
    for (int k = 0; k < c2; ++k) add(2);
    for (int k = 0; k < c3; ++k) add(3);
    for (int k = 0; k < c4; ++k) add(4);
    for (int k = 0; k < c5; ++k) add(5);
    for (int k = 0; k < c8; ++k) add(8);
    *pl = p;
    return true;
}

// Error coefficients of the FFT form for the argmin certificate (first order
// in the unit roundoff u = 2^-53, then doubled).  Each radix-r pass over the
// whole array is a scaled unitary map computed with a relative 2-norm error of
// at most eta_r = (5 + c_r) u: twiddles rounded from long double (2u), their
// complex product (3u), and the small DFT's own roundings, c_r = 1, 2, 6, 10,
// 18 for r = 2, 4, 8, 3, 5 (the add levels of radices 2, 4, 8 plus the
// sqrt(1/2) products of radix 8; for radices 3 and 5 a componentwise bound of
// each output by its inputs' magnitudes, times sqrt(r) to a 2-norm).  A 2-D
// transform sums the passes of both lengths plus 2u for packing two real rows,
// eps.  With x, y the zero-padded grids (m'n' nonzeros each), the computed
// correlation satisfies |h^ - h| <= (2 eps + eps' + 2.9u + 2u) max(|x|_2 |y|_1,
// |x|_1 |y|_2) to first order (frame and template transforms, the complex
// product, the inverse, the 1/(PQ) scale), and |y|_1 <= sqrt(m'n') |y|_2;
// kf = 2 (3 eps + 5u).  The energy sums of the grids are computed with at most
// m'+n'+2w+16 roundings along any path, four of them combined by three
// additions: ke = (4 (m'+n'+2w+16) + 6) u.
void fft_error_coefs(const Geom &g, const FftTmpl &ft, double *kf, double *ke)
{
    const double u = 0x1p-53;
    auto plan_eps = [&](const FftPlan &pl) {
        double e = 0.0;
        for (int p = 0; p < pl.npass; ++p) {
            const int r = pl.radix[p];
            const double c = r == 2 ? 1.0 : r == 4 ? 2.0 : r == 8 ? 6.0 : r == 3 ? 10.0 : 18.0;
            e += (5.0 + c) * u;
        }
        return e;
    };
    const double eps = plan_eps(ft.pp) + plan_eps(ft.pq) + 2.0 * u;
    *kf = 2.0 * (3.0 * eps + 5.0 * u);
    *ke = (4.0 * (g.mg + g.ng + 2.0 * g.w + 16.0) + 6.0) * u;
}

// The single-precision form's factors, the same pass terms in u32 = 2^-24:
// e1 = eps + u32 for the frame's transform (its centred values rounded to
// FP32 once), e2 = eps + 7 u32 for the inverse, the template spectrum rounded
// from FP64 (2 u32), the complex product (4 u32) and the scale.
void fft32_cert_coefs(const FftTmpl &ft, double *e1, double *e2)
{
    const double u = 0x1p-24;
    double eps = 2.0 * u;
    for (const FftPlan *pl : {&ft.pp, &ft.pq})
        for (int p = 0; p < pl->npass; ++p) {
            const int r = pl->radix[p];
            eps += (5.0 + (r == 2 ? 1.0 : r == 4 ? 2.0 : r == 8 ? 6.0 : r == 3 ? 10.0 : 18.0)) * u;
        }
    *e1 = eps + u;
    *e2 = eps + 7.0 * u;
}

// The transform length for x = grid side + w - 1 points: the next length
// with a wave-level kernel when it is at most 10% longer than the next
// 2,3,5-smooth length, else that length (384 points in place of 360: the
// wave-level kernels ran the 384-point transforms 30% faster than the block
// kernels, more than the 14% more points cost).
static int transform_length(int x)
{
    const int n0 = next_smooth(x);
    if (wave_length(n0)) return n0;
    for (int n = n0 + 1; n <= n0 + n0 / 10; ++n)
        if (wave_length(n)) return n;
    return n0;
}

FftGeom fft_geom(const Geom &g)
{
    FftGeom f{};
    f.P = transform_length(g.mg + g.w - 1);
    f.Q = transform_length(g.ng + g.w - 1);
    f.qh = f.Q / 2 + 1;
    return f;
}

bool fft_applicable(const Geom &g)
{
    const FftGeom f = fft_geom(g);
    return f.P <= kFftMaxLen && f.Q <= kFftMaxLen;
}

size_t fft_s1_bytes(const Geom &g, size_t esz)
{
    return (size_t)fft_geom(g).qh * g.mg * esz;
}

size_t fft_s2_bytes(const Geom &g, size_t esz) { return (size_t)g.W * fft_geom(g).qh * esz; }

// The wave-level kernels where a length has one (on by default; the
// block-level kernels otherwise).
bool g_wave_fft = true;

namespace {

// Twiddle tables and the template spectrum of precision R.
template <typename R>
struct FftTabs;
template <>
struct FftTabs<double> {
    static const double2 *twp(const FftTmpl &f) { return f.twp; }
    static const double2 *twq(const FftTmpl &f) { return f.twq; }
    static const double2 *spec(const FftTmpl &f) { return f.spec; }
    static double center(const FftTmpl &) { return 0.0; }
};
template <>
struct FftTabs<float> {
    static const float2 *twp(const FftTmpl &f) { return f.twp32; }
    static const float2 *twq(const FftTmpl &f) { return f.twq32; }
    static const float2 *spec(const FftTmpl &f) { return f.spec32; }
    static double center(const FftTmpl &f) { return f.center; }
};

template <typename R>
hipError_t rows_grid(const double *grid, int C, const Geom &g, const FftTmpl &ft,
                     typename Cx<R>::T *s1, hipStream_t st, const int32_t *only)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    const size_t esz = sizeof(typename Cx<R>::T);
    const int rp = rows_per_block(ft.pq.n, esz);
    const int npairs = (g.mg + 1) / 2;
    k_fft_rows<0, R><<<dim3((npairs + rp - 1) / rp, C), kBlock, block_lds(rp, ft.pq.n, esz), st>>>(
        grid, g.m, g.n, g.mg, g.ng, rp, ft.pq, FftTabs<R>::twq(ft), FftTabs<R>::center(ft), s1,
        only);
    return hipGetLastError();
}

template <typename R>
hipError_t rows_px(const void *frames, int C, const Geom &g, const FftTmpl &ft,
                   typename Cx<R>::T *s1, hipStream_t st, const int32_t *only)
{
    clear_stale_error();
    if (C == 0) return hipSuccess;
    if (g.ds > 1) return hipErrorInvalidValue;
    const size_t esz = sizeof(typename Cx<R>::T);
    const int rp = rows_per_block(ft.pq.n, esz);
    const int npairs = (g.mg + 1) / 2;
    const size_t lds = block_lds(rp, ft.pq.n, esz);
    const dim3 grid((npairs + rp - 1) / rp, C);
    const bool u16 = g.dtype == MOCO_U16;
    const auto *tw = FftTabs<R>::twq(ft);
    const double c = FftTabs<R>::center(ft);
    if (g_wave_fft) {
        bool ok = false;
        if (u16 && g.ds)
            ok = wrows<R, 1>(frames, C, g, tw, c, s1, st, ft.pq.n, only);
        else if (u16)
            ok = wrows<R, 2>(frames, C, g, tw, c, s1, st, ft.pq.n, only);
        else if (g.ds)
            ok = wrows<R, 3>(frames, C, g, tw, c, s1, st, ft.pq.n, only);
        else
            ok = wrows<R, 4>(frames, C, g, tw, c, s1, st, ft.pq.n, only);
        if (ok) return hipGetLastError();
    }
    if (u16 && g.ds)
        k_fft_rows<1, R><<<grid, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, rp, ft.pq, tw, c, s1,
                                                  only);
    else if (u16)
        k_fft_rows<2, R><<<grid, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, rp, ft.pq, tw, c, s1,
                                                  only);
    else if (g.ds)
        k_fft_rows<3, R><<<grid, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, rp, ft.pq, tw, c, s1,
                                                  only);
    else
        k_fft_rows<4, R><<<grid, kBlock, lds, st>>>(frames, g.m, g.n, g.mg, g.ng, rp, ft.pq, tw, c, s1,
                                                  only);
    return hipGetLastError();
}

template <typename R>
hipError_t corr(const typename Cx<R>::T *s1, int C, const Geom &g, const FftTmpl &ft,
                typename Cx<R>::T *s2, double *h, hipStream_t st, const int32_t *only, R *xmax,
                int *nxb)
{
    clear_stale_error();
    int nb = 0;
    if (nxb) *nxb = 0;
    if (C == 0) return hipSuccess;
    const size_t esz = sizeof(typename Cx<R>::T);
    if (!g_wave_fft ||
        !wcols<R>(s1, C, g, ft, FftTabs<R>::twp(ft), FftTabs<R>::spec(ft), s2, st, only, xmax,
                  &nb)) {
        const int kb = rows_per_block(ft.pp.n, esz);
        nb = (ft.qh + kb - 1) / kb;
        k_fft_cols<false, R><<<dim3(nb, C), kBlock, block_lds(kb, ft.pp.n, esz), st>>>(
            s1, g.mg, ft.qh, kb, g.w, ft.pp, FftTabs<R>::twp(ft), FftTabs<R>::spec(ft), nullptr,
            s2, only, xmax);
    }
    if (nxb) *nxb = nb;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double scale = 1.0 / ((double)ft.pp.n * (double)ft.pq.n);
    if (!g_wave_fft || !wback<R>(s2, C, g, ft, FftTabs<R>::twq(ft), scale, h, st, only)) {
        const int rp = rows_per_block(ft.pq.n, esz);
        const int npairs = (g.W + 1) / 2;
        k_fft_rows_back<R><<<dim3((npairs + rp - 1) / rp, C), kBlock,
                             block_lds(rp, ft.pq.n, esz), st>>>(
            s2, ft.qh, g.w, rp, scale, ft.pq, FftTabs<R>::twq(ft), h, only);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fft_rows(const double *grid, int C, const Geom &g, const FftTmpl &ft,
                           double2 *s1, hipStream_t st, const int32_t *only)
{
    return rows_grid<double>(grid, C, g, ft, s1, st, only);
}

hipError_t launch_fft_rows_px(const void *frames, int C, const Geom &g, const FftTmpl &ft,
                              double2 *s1, hipStream_t st, const int32_t *only)
{
    return rows_px<double>(frames, C, g, ft, s1, st, only);
}

hipError_t launch_fft_spec(const double2 *s1, const Geom &g, const FftTmpl &ft, double2 *spec,
                           hipStream_t st)
{
    clear_stale_error();
    const int kb = rows_per_block(ft.pp.n);
    k_fft_cols<true, double><<<dim3((ft.qh + kb - 1) / kb, 1), kBlock,
                               block_lds(kb, ft.pp.n, sizeof(double2)), st>>>(
        s1, g.mg, ft.qh, kb, g.w, ft.pp, ft.twp, nullptr, spec, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_fft_corr(const double2 *s1, int C, const Geom &g, const FftTmpl &ft,
                           double2 *s2, double *h, hipStream_t st, const int32_t *only)
{
    return corr<double>(s1, C, g, ft, s2, h, st, only, nullptr, nullptr);
}

hipError_t launch_fft32_rows(const double *grid, int C, const Geom &g, const FftTmpl &ft,
                             float2 *s1, hipStream_t st)
{
    return rows_grid<float>(grid, C, g, ft, s1, st, nullptr);
}

hipError_t launch_fft32_rows_px(const void *frames, int C, const Geom &g, const FftTmpl &ft,
                                float2 *s1, hipStream_t st)
{
    return rows_px<float>(frames, C, g, ft, s1, st, nullptr);
}

hipError_t launch_fft32_corr(const float2 *s1, int C, const Geom &g, const FftTmpl &ft,
                             float2 *s2, double *h, hipStream_t st, float *xmax, int *nxb)
{
    return corr<float>(s1, C, g, ft, s2, h, st, nullptr, xmax, nxb);
}


}  // namespace moco
