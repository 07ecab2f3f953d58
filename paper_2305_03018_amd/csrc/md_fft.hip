// HIP kernels for exact grey-scale dilation / erosion on gfx950.
//
// The method (arXiv 2305.03018, Sec. 3): the one-hot "umbra" volumes of the
// image and of the structuring element (Step 1, Eqs. (7)-(8)) are convolved
// over the two image axes and the grey axis (Step 2) and each pixel's value
// is the top degree with a non-zero rounded coefficient (Step 3, Eq. (9)).
//
// How the volumes are handled here:
//   * Range (grey) axis.  The DFT of a one-hot column at grey value v is
//     exp(-2 pi i v m / nr); it is gathered from a table instead of being
//     transformed.  The convolved volume is real along this axis, so only
//     bins = nr/2 + 1 frequencies are kept (the rest are conjugates).
//   * Image axes.  Per (tile, bin) one workgroup builds the encoded tile in
//     LDS, runs an in-place radix-2^q FFT over rows and columns, multiplies by
//     the cached spectrum of the SE umbra, runs the inverse FFT and writes the
//     T x T valid outputs of the overlap-save tile (partitioned convolution,
//     the paper's Sec. 5 outlook) to the transform-domain buffer.
//   * Decode.  Per pixel, the inverse real DFT over the bins gives the
//     coefficients c_d; the output is the largest d with rint(c_d) != 0 and
//     the distance |c_d - rint(c_d)| is checked against the ambiguity band.
//   * Ambiguous tiles are recomputed exactly with FP64 transforms.
//   * Large tiles (FP32 256-1024, FP64 128-1024 points per side) run the
//     same steps through a per-block slab in global memory, a batch of lines
//     at a time in LDS.
//   * The classical max-plus window (direct path) is a separate kernel; a
//     measured cost model picks it or the transform path per job.
//
// LDS FFT layout: an N x N complex array with row pitch N + 1.  The forward
// transform is decimation-in-time with bit-reversed input (the encode writes
// bit-reversed positions) and natural-order output; the inverse is
// decimation-in-frequency with natural-order input and bit-reversed output,
// so no explicit permutation pass is needed.  Each pass fuses q <= 4
// radix-2 stages in registers; lanes of a wavefront walk the batch axis so
// both row and column passes touch consecutive LDS words.
#include "md_device.h"

#include <math.h>

#include <algorithm>
#include <type_traits>
#include <utility>

namespace md {
namespace {

// a * exp(-+2 pi i idx / kTwN), 0 <= idx < kTwN (both tables hold the full
// circle), with the twiddle held as hi + lo floats: the lo products are
// formed first so they are not lost against the hi products.
struct Tw32 {
    const TwF *__restrict__ p;
    __device__ __forceinline__ float2 mul(float2 a, int idx, bool inv) const {
        const TwF w = p[idx];
        const float hy = inv ? -w.hi.y : w.hi.y;
        const float ly = inv ? -w.lo.y : w.lo.y;
        const float sx = a.x * w.lo.x - a.y * ly;
        const float sy = a.x * ly + a.y * w.lo.x;
        float2 r;
        r.x = fmaf(a.x, w.hi.x, fmaf(-a.y, hy, sx));
        r.y = fmaf(a.x, hy, fmaf(a.y, w.hi.x, sy));
        return r;
    }
};

struct Tw64 {
    const double2 *__restrict__ p;
    __device__ __forceinline__ double2 mul(double2 a, int idx, bool inv) const {
        const double2 w = p[idx];
        const double wy = inv ? -w.y : w.y;
        double2 r;
        r.x = fma(a.x, w.x, -a.y * wy);
        r.y = fma(a.x, wy, a.y * w.x);
        return r;
    }
};

// x * w^(+-) where w = exp(-2 pi i idx / kTwN); when idx is a compile-time
// constant 0 or kTwN/4 (w = 1 or -i) no multiply is needed.
template <typename TW, typename C>
__device__ __forceinline__ C twmul(const TW &tw, C x, int idx, bool idx_known, bool inv) {
    if (idx_known && idx == 0) return x;
    if (idx_known && idx == kTwN / 4) {
        C r;
        if (inv) { r.x = -x.y; r.y = x.x; }   // * (+i)
        else { r.x = x.y; r.y = -x.x; }       // * (-i)
        return r;
    }
    return tw.mul(x, idx, inv);
}

template <typename R> struct TwSel;
template <> struct TwSel<float> { using T = Tw32; };
template <> struct TwSel<double> { using T = Tw64; };

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }
// Passes per 1-D transform of length 2^lg and the radix-2 stages fused into
// pass p (balanced, at most qm per pass: each pass is one LDS round trip;
// qm = 4 in FP32, 3 in FP64, whose 16-point registers would cost occupancy).
constexpr int npass(int lg, int qm) { return (lg + qm - 1) / qm; }
constexpr int passq(int lg, int qm, int p) { return lg / npass(lg, qm) + (p < lg % npass(lg, qm) ? 1 : 0); }
template <typename R> constexpr int max_q() { return sizeof(R) == 4 ? 4 : 3; }
constexpr int stages_before(int lg, int qm, int p) { return p == 0 ? 0 : stages_before(lg, qm, p - 1) + passq(lg, qm, p - 1); }

template <int LG>
__device__ __forceinline__ int brev(int i) { return (int)(__brev((unsigned)i) >> (32 - LG)); }

// q-bit reversal of a compile-time index
constexpr int brevc(int t, int q) { return q == 0 ? 0 : ((t & 1) << (q - 1)) | brevc(t >> 1, q - 1); }

// One fused decimation-in-time pass: radix-2 stages with half-sizes
// H0, 2 H0, ..., 2^(Q-1) H0 on each of LINES >= 64 lines of length N in an
// LDS array of row pitch N+1.  AXIS 0 transforms along rows (contiguous), AXIS 1
// along columns (then LINES == N).  Each thread combines RAD = 2^Q blocks of
// length H0 at offset o inside them: with the blocks in bit-reversed order,
// the q stages equal one twiddle per element, w_{RAD H0}^(o brev(t)), then a
// RAD-point DIT network whose twiddles w_{2h}^(t mod h) are compile-time
// constants (1 and -i cost no multiply).
template <typename R, int N, int Q, int H0, int AXIS, int BS, bool INV, int LINES = N>
__device__ __forceinline__ void pass_dit(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = LINES * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (LINES - 1);
        const int gi = __builtin_amdgcn_readfirstlane(u / LINES);   // LINES >= 64: uniform per wavefront
        const int o = gi % H0;
        const int base = (gi / H0) * (RAD * H0) + o;
        C *p = lds + line * LS + base * ES;
        C x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * H0 * ES];
        if constexpr (H0 > 1) {
            if (o != 0) {   // wave-uniform
#pragma unroll
                for (int t = 1; t < RAD; ++t) x[t] = tw.mul(x[t], o * brevc(t, Q) * (kTwN / (RAD * H0)), INV);
            }
        }
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = 1 << s;
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const C b = twmul(tw, x[t + hu], (t & (hu - 1)) * (kTwN / (2 * hu)), true, INV);
                const C a = x[t];
                x[t] = cadd(a, b);
                x[t + hu] = csub(a, b);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * H0 * ES] = x[t];
    }
}

// One fused decimation-in-frequency pass: half-sizes 2^(Q-1) HMIN, ..., HMIN;
// the transpose of pass_dit: the RAD-point DIF network with constant
// twiddles, then w_{RAD HMIN}^(o brev(t)) per element.
template <typename R, int N, int Q, int HMIN, int AXIS, int BS, bool INV, int LINES = N>
__device__ __forceinline__ void pass_dif(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = LINES * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (LINES - 1);
        const int gi = __builtin_amdgcn_readfirstlane(u / LINES);
        const int o = gi % HMIN;
        const int base = (gi / HMIN) * (RAD * HMIN) + o;
        C *p = lds + line * LS + base * ES;
        C x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * HMIN * ES];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = RAD >> (s + 1);
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const C a = x[t], b = x[t + hu];
                x[t] = cadd(a, b);
                x[t + hu] = twmul(tw, csub(a, b), (t & (hu - 1)) * (kTwN / (2 * hu)), true, INV);
            }
        }
        if constexpr (HMIN > 1) {
            if (o != 0) {   // wave-uniform
#pragma unroll
                for (int t = 1; t < RAD; ++t) x[t] = tw.mul(x[t], o * brevc(t, Q) * (kTwN / (RAD * HMIN)), INV);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * HMIN * ES] = x[t];
    }
}

// The same passes as radix-2 stages with their own twiddles
// w_{2h}^(o + (t mod h') H0): used when fewer than 64 lines share a pass, so
// the offset o varies inside a wavefront and every twiddle is a per-lane
// table read -- fewer of them are live at once than in the factored form.
template <typename R, int N, int Q, int H0, int AXIS, int BS, bool INV, int LINES>
__device__ __forceinline__ void pass_dit_staged(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = LINES * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (LINES - 1);
        const int gi = u / LINES;
        const int o = gi % H0;
        const int base = (gi / H0) * (RAD * H0) + o;
        C *p = lds + line * LS + base * ES;
        C x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * H0 * ES];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = 1 << s;
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const int j = o + (t & (hu - 1)) * H0;            // index inside the 2h block
                const C b = twmul(tw, x[t + hu], j * (kTwN / (2 * (H0 << s))), H0 == 1, INV);
                const C a = x[t];
                x[t] = cadd(a, b);
                x[t + hu] = csub(a, b);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * H0 * ES] = x[t];
    }
}

template <typename R, int N, int Q, int HMIN, int AXIS, int BS, bool INV, int LINES>
__device__ __forceinline__ void pass_dif_staged(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = LINES * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (LINES - 1);
        const int gi = u / LINES;
        const int o = gi % HMIN;
        const int base = (gi / HMIN) * (RAD * HMIN) + o;
        C *p = lds + line * LS + base * ES;
        C x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * HMIN * ES];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = RAD >> (s + 1);
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const int j = o + (t & (hu - 1)) * HMIN;
                const C a = x[t], b = x[t + hu];
                x[t] = cadd(a, b);
                x[t + hu] = twmul(tw, csub(a, b), j * (kTwN / (2 * hu * HMIN)), HMIN == 1, INV);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * HMIN * ES] = x[t];
    }
}

template <typename R, int N, int AXIS, int BS, bool INV, int LINES = N, int PASS = 0>
__device__ __forceinline__ void dit_axis(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    constexpr int lg = ilog2c(N);
    constexpr int qm = max_q<R>();
    if constexpr (PASS < npass(lg, qm)) {
        constexpr int Q = passq(lg, qm, PASS), H0 = 1 << stages_before(lg, qm, PASS);
        if constexpr (LINES >= 64) pass_dit<R, N, Q, H0, AXIS, BS, INV, LINES>(lds, tw);
        else pass_dit_staged<R, N, Q, H0, AXIS, BS, INV, LINES>(lds, tw);
        __syncthreads();
        dit_axis<R, N, AXIS, BS, INV, LINES, PASS + 1>(lds, tw);
    }
}

template <typename R, int N, int AXIS, int BS, bool INV, int LINES = N, int PASS = 0>
__device__ __forceinline__ void dif_axis(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    constexpr int lg = ilog2c(N);
    constexpr int qm = max_q<R>();
    if constexpr (PASS < npass(lg, qm)) {
        constexpr int Q = passq(lg, qm, PASS), HMIN = N >> (stages_before(lg, qm, PASS) + Q);
        if constexpr (LINES >= 64) pass_dif<R, N, Q, HMIN, AXIS, BS, INV, LINES>(lds, tw);
        else pass_dif_staged<R, N, Q, HMIN, AXIS, BS, INV, LINES>(lds, tw);
        __syncthreads();
        dif_axis<R, N, AXIS, BS, INV, LINES, PASS + 1>(lds, tw);
    }
}

// Runs use(q, load(q)) for q = threadIdx.x + e * BS < n, with the loads of
// CH consecutive iterations issued before any of them is used (a loop that
// loads and uses one element at a time waits a full memory latency per
// element).  `load` must accept any q < n.
template <int BS, int CH, typename LoadF, typename UseF>
__device__ __forceinline__ void batched(int n, LoadF load, UseF use) {
    for (int q0 = threadIdx.x; q0 < n; q0 += CH * BS) {
        decltype(load(0)) v[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = q0 + e * BS;
            v[e] = load(q < n ? q : q0);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = q0 + e * BS;
            if (q < n) use(q, v[e]);
        }
    }
}

// Order of the LDS walk in the encode and in the output of a tile.  Walking
// the LDS in order keeps a wavefront's LDS accesses on consecutive words
// and moves the bit reversal to the global side (scattered within one
// row); walking the image in order keeps the global accesses contiguous and
// puts the bit reversal on the LDS index, where lanes collide on banks.
//  * Encode: LDS order while a wavefront's 64 scattered pixel loads stay
//    within 512 bytes of the row (N <= 128); beyond that they touch up to
//    16 cache lines per load and the image order is faster.
//  * Output: LDS order in FP64 only.  FP64 elements span four banks, so the
//    conflicts cost more than the scatter; FP32 transforms are bound by
//    vector ALU issue, and the idle lanes and scattered stores of an
//    LDS-order output cost more than the conflicts they remove.
template <typename R, int N> constexpr bool kEncLdsOrder = N <= 128;
template <typename R> constexpr bool kOutLdsOrder = sizeof(R) == 8;

// Step 1 for `rows` x N input pixels starting at image pixel (gy0, gx0):
// out-of-image pixels are the zero polynomial, in-image grey values
// (complemented for erosion) become their range-DFT column enc_m[v].
// Calls put(l, c, value) for row l < rows and column c < N.  With XR the
// column c is the LDS column and holds image column gx0 + brev(c) (the
// forward transform wants bit-reversed input; reversing on the global side
// keeps a wavefront's LDS stores on consecutive words, where a bit-reversed
// LDS index puts 16 lanes on two banks); without XR, c is the image column.
// The pixel loads of CH elements go out together, then their table gathers;
// returns non-zero if an in-image value lies outside [0, L-1].
template <typename R, int N, int BS, int CH, bool XR, typename PutF>
__device__ __forceinline__ int encode_rows(int rows, const int32_t *__restrict__ img, int H, int W, int L, int op,
                                           int gy0, int gx0, const typename Cx<R>::T *__restrict__ enc_m, PutF put) {
    using C = typename Cx<R>::T;
    constexpr int LG = ilog2c(N);
    const int n = rows * N;
    const auto im = gld(img);
    int badv = 0;
    for (int q0 = threadIdx.x; q0 < n; q0 += CH * BS) {
        int val[CH];
        bool in[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = q0 + e * BS;
            const int gy = gy0 + (q >> LG), gx = gx0 + (XR ? brev<LG>(q & (N - 1)) : (q & (N - 1)));
            in[e] = q < n && (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
            val[e] = im[in[e] ? (size_t)gy * W + gx : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        C v[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            badv |= (int)(in[e] && (unsigned)val[e] >= (unsigned)L);
            int w = min(max(val[e], 0), L - 1);
            w = op ? L - 1 - w : w;
            v[e] = ldg(enc_m, in[e] ? w : 0);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = q0 + e * BS;
            if (q < n) put(q >> LG, q & (N - 1), in[e] ? v[e] : czero<C>());
        }
    }
    return badv;
}

// One (tile, bin) of Step 2.  The tile's outputs start at pixel (oy0, ox0);
// its N x N input window starts r pixels above/left of that (overlap-save):
// input index j holds f(o0 - r + j) and the SE umbra sits at [0, k) on both
// axes, so circular output index i >= k-1 is the linear result for pixel
// o0 + i - (k-1).  Out-of-image pixels are the zero polynomial (Sec. 3,
// Step 1).  Writes the T x T valid values (unscaled) to ydst, with `bump`
// added to their real parts (0 except under the perturbation test hook).
template <typename R, int N, int BS>
__device__ __forceinline__ void fft_tile_bin(typename Cx<R>::T *lds, const int32_t *__restrict__ img, int H,
                                             int W, int L, int op, int k, int oy0, int ox0,
                                             const typename Cx<R>::T *__restrict__ enc_m,
                                             const typename Cx<R>::T *__restrict__ spec_m,
                                             typename Cx<R>::T *__restrict__ ydst, int ybs,
                                             const typename TwSel<R>::T &tw, unsigned int *range_err, R bump) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, LG = ilog2c(N);
    constexpr int CH = N * N / BS < 16 ? N * N / BS : 16;
    const int r = (k - 1) >> 1, T = N - k + 1;
    const int iy0 = oy0 - r, ix0 = ox0 - r;
    const int bad = encode_rows<R, N, BS, CH, kEncLdsOrder<R, N>>(N, img, H, W, L, op, iy0, ix0, enc_m,
                                                                [&](int i, int c, C v) {
        lds[brev<LG>(i) * P + (kEncLdsOrder<R, N> ? c : brev<LG>(c))] = v;
    });
    if (bad && range_err) atomicOr(range_err, 1u);
    __syncthreads();
    dit_axis<R, N, 0, BS, false>(lds, tw);
    dit_axis<R, N, 1, BS, false>(lds, tw);
    // the spectrum is stored [kx][ky]: q walks ky fastest, down an LDS column
    batched<BS, CH>(
        N * N, [&](int q) { return ldg(spec_m, q); },
        [&](int q, C sv) {
            C *e = lds + (q & (N - 1)) * P + (q >> LG);
            *e = cmul(*e, sv);
        });
    __syncthreads();
    dif_axis<R, N, 1, BS, true>(lds, tw);
    dif_axis<R, N, 0, BS, true>(lds, tw);
    if constexpr (kOutLdsOrder<R>) {
        // LDS column b holds output column brev(b): walk the LDS rows in
        // order and scatter within the output row
        for (int q = threadIdx.x; q < T * N; q += BS) {
            const int i = (q >> LG) + (k - 1), b = q & (N - 1), j = brev<LG>(b);
            if (j >= k - 1) {
                C v = lds[brev<LG>(i) * P + b];
                v.x += bump;
                stg(ydst, ypix((size_t)(i - (k - 1)) * T + (j - (k - 1)), ybs), v);
            }
        }
    } else {
        for (int q = threadIdx.x; q < T * T; q += BS) {
            const int i = q / T + (k - 1), j = q % T + (k - 1);
            C v = lds[brev<LG>(i) * P + brev<LG>(j)];
            v.x += bump;
            stg(ydst, ypix(q, ybs), v);
        }
    }
    __syncthreads();
}

// Lines of length N held in LDS at a time by the large-tile transform
// (4096 points: in FP32 32 KiB, so up to four blocks fit a CU).
template <typename R, int N>
constexpr int big_lines() { return big_lines_of(N, sizeof(R) == 8); }

// One (tile, bin) of Step 2 for spatial lengths whose N x N array does not
// fit the LDS.  Same overlap-save geometry and bit-reversal bookkeeping as
// fft_tile_bin; the array lives in this block's scratch slab in global
// memory (mostly in L2 / Infinity Cache) and passes through the LDS in
// batches of LB lines:
//   1. encode LB image rows, forward DIT along x, write row i to slab row
//      brev(i) (the column transform then reads bit-reversed input);
//   2. LB slab columns: forward DIT along y, multiply by the SE spectrum,
//      inverse DIF along y (slab row r' then holds output row brev(r'));
//   3. LB slab rows: inverse DIF along x, write the valid outputs.
template <typename R, int N, int BS>
__device__ __forceinline__ void fft_big_tile_bin(typename Cx<R>::T *lds, typename Cx<R>::T *slab,
                                                 const int32_t *__restrict__ img, int H, int W, int L, int op,
                                                 int k, int oy0, int ox0, const typename Cx<R>::T *__restrict__ enc_m,
                                                 const typename Cx<R>::T *__restrict__ spec_m,
                                                 typename Cx<R>::T *__restrict__ ydst, int ybs,
                                                 const typename TwSel<R>::T &tw, unsigned int *range_err, R bump) {
    using C = typename Cx<R>::T;
    constexpr int LB = big_lines<R, N>();
    constexpr int P = N + 1, LG = ilog2c(N), LLB = ilog2c(LB);
    // 4 loads in flight per batch: more would cost the registers that let a
    // third block share the CU
    constexpr int CHM = sizeof(R) == 4 ? 4 : 16;
    constexpr int CH = LB * N / BS < CHM ? LB * N / BS : CHM;
    const int r = (k - 1) >> 1, T = N - k + 1;
    const int iy0 = oy0 - r, ix0 = ox0 - r;
    int bad = 0;
    // 1. rows
    for (int rb = 0; rb < N; rb += LB) {
        bad |= encode_rows<R, N, BS, CH, kEncLdsOrder<R, N>>(LB, img, H, W, L, op, iy0 + rb, ix0, enc_m, [&](int l, int c, C v) {
            lds[l * P + (kEncLdsOrder<R, N> ? c : brev<LG>(c))] = v;
        });
        __syncthreads();
        dit_axis<R, N, 0, BS, false, LB>(lds, tw);
        for (int q = threadIdx.x; q < LB * N; q += BS) {
            const int l = q >> LG, v = q & (N - 1);
            stg(slab, (size_t)brev<LG>(rb + l) * N + v, lds[l * P + v]);
        }
        __syncthreads();
    }
    if (bad && range_err) atomicOr(range_err, 1u);
    // 2. columns: multiply and back
    for (int cb = 0; cb < N; cb += LB) {
        batched<BS, CH>(
            LB * N, [&](int q) { return ldg(slab, (size_t)(q >> LLB) * N + cb + (q & (LB - 1))); },
            [&](int q, C v) { lds[(q & (LB - 1)) * P + (q >> LLB)] = v; });
        __syncthreads();
        dit_axis<R, N, 0, BS, false, LB>(lds, tw);
        // the spectrum is stored [kx][ky]: q walks ky fastest
        batched<BS, CH>(
            LB * N, [&](int q) { return ldg(spec_m, (size_t)(cb + (q >> LG)) * N + (q & (N - 1))); },
            [&](int q, C sv) {
                C *e = lds + (q >> LG) * P + (q & (N - 1));
                *e = cmul(*e, sv);
            });
        __syncthreads();
        dif_axis<R, N, 0, BS, true, LB>(lds, tw);
        for (int q = threadIdx.x; q < LB * N; q += BS) {
            const int rr = q >> LLB, l = q & (LB - 1);
            stg(slab, (size_t)rr * N + cb + l, lds[l * P + rr]);
        }
        __syncthreads();
    }
    // 3. rows back; slab row rb+l is output row y = brev(rb+l)
    for (int rb = 0; rb < N; rb += LB) {
        batched<BS, CH>(
            LB * N, [&](int q) { return ldg(slab, (size_t)(rb + (q >> LG)) * N + (q & (N - 1))); },
            [&](int q, C v) { lds[(q >> LG) * P + (q & (N - 1))] = v; });
        __syncthreads();
        dif_axis<R, N, 0, BS, true, LB>(lds, tw);
        if constexpr (kOutLdsOrder<R>) {
            for (int q = threadIdx.x; q < LB * N; q += BS) {
                const int l = q >> LG, b = q & (N - 1);
                const int y = brev<LG>(rb + l), x = brev<LG>(b);
                if (y >= k - 1 && x >= k - 1) {
                    C v = lds[l * P + b];
                    v.x += bump;
                    stg(ydst, ypix((size_t)(y - (k - 1)) * T + (x - (k - 1)), ybs), v);
                }
            }
        } else {
            for (int q = threadIdx.x; q < LB * T; q += BS) {
                const int l = q / T, xo = q - l * T;
                const int y = brev<LG>(rb + l);
                if (y >= k - 1) {
                    C v = lds[l * P + brev<LG>(xo + k - 1)];
                    v.x += bump;
                    stg(ydst, ypix((size_t)(y - (k - 1)) * T + xo, ybs), v);
                }
            }
        }
        __syncthreads();
    }
}


// Under the perturbation test hook (perturb non-null), bin 0 of a tile whose
// kPerturbFirst bit is set gets 0.4 nt^2 nr added to the real part of every
// output: after the decode's 1 / (nt^2 nr) scale every coefficient of its
// pixels moves by 0.4, so the band flags exactly those tiles.
template <typename R>
__device__ __forceinline__ R perturb_bump(const uint8_t *perturb, const JobDev &J, int tile, int m, uint8_t bit) {
    if (!perturb || m != 0 || !(perturb[J.flag0 + tile] & bit)) return R(0);
    return (R)(0.4 * (double)J.nt * J.nt * J.nr);
}

// Third word of a raw buffer resource on gfx9-class chips (32-bit data
// format, no swizzle).
constexpr int kBufWord3 = 0x00020000;

// 8- or 16-byte load through a buffer resource at voff + soff bytes (soff
// uniform across the wave)
template <typename C>
__device__ __forceinline__ C buf_load(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    if constexpr (sizeof(C) == 8)
        return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
    else
        return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

// 8- or 16-byte store through a buffer resource at voff + soff bytes; a
// store whose offset lies at or past the resource's size is dropped
template <typename C>
__device__ __forceinline__ void buf_store(C v, __amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    if constexpr (sizeof(C) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), rs,
                                              voff, soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), rs,
                                               voff, soff, 0);
}

// ---------------------------------------------------------------------------
// Spatial transform with register-resident lines (tiles of 16..128 points)
// ---------------------------------------------------------------------------
// One (tile, bin) work item per block of 4 N threads.  Every line of the
// N x N tile (a column, or a row) is held by the G = 4 lanes 16 apart in a
// wavefront, E = N / 4 points each: lane part g holds the points g + 4 e.  A
// line transform of length N = E G (Cooley-Tukey over n = g + G e,
// k = k1 + E k2) is
//   * an E-point DFT of each lane's points in registers,
//   * the turn w_N^(g k1) of its output k1 (a per-lane twiddle kept in
//     registers for the whole kernel),
//   * a 4-point DFT across the lanes of the line for every k1, as two
//     radix-2 stages whose operands are exchanged by the permlane swaps
//     (lanes 32 apart, then lanes 16 apart) with the turn -i between them.
// Lane g then holds the outputs k = k1 + E k2 for k1 in its chunk
// [g E/4, (g+1) E/4) and all four k2.  The inverse transform runs the same
// steps mirrored with conjugate twiddles and ends with the lane holding the
// points g + 4 e again.  The tile crosses the LDS twice:
//   1. columns: each lane encodes its points straight from the image (Step 1;
//      the lanes of a row of 16 walk 16 image columns), transforms along y and
//      stores its outputs;
//   2. rows: each lane loads its points of a row, transforms along x,
//      multiplies by the SE spectrum (stored transposed, [kx][ky], so that
//      lanes holding consecutive rows read consecutive words), transforms
//      back along x and stores them where it loaded them;
//   3. columns: each lane loads what it stored in 1, transforms back along
//      y and writes its valid outputs (rows and columns >= k - 1, the
//      overlap-save rule); waves whose 16 columns all lie left of the
//      overlap skip this phase.
// The LDS array has row pitch N + 1, so that the 16 lanes of a row of
// lanes touch 16 distinct bank pairs in both orientations.

// cos and sin of 2 pi j / n in double at compile time (Taylor series on an
// argument reduced to [0, pi / 2])
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double taylor_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int q = 1; q < 20; ++q) {
        t *= -x * x / ((2.0 * q - 1.0) * (2.0 * q));
        s += t;
    }
    return s;
}
constexpr double taylor_sin(double x) {
    double t = x, s = x;
    for (int q = 1; q < 20; ++q) {
        t *= -x * x / ((2.0 * q) * (2.0 * q + 1.0));
        s += t;
    }
    return s;
}
constexpr double cos2pi(int j, int n) {
    j = ((j % n) + n) % n;
    if (2 * j > n) j = n - j;                       // cos is even
    const double x = 2.0 * kPiD * j / n;            // [0, pi]
    return 2 * x > kPiD ? -taylor_cos(kPiD - x) : taylor_cos(x);
}
constexpr double sin2pi(int j, int n) {
    j = ((j % n) + n) % n;
    if (2 * j > n) return -sin2pi(n - j, n);        // sin is odd
    const double x = 2.0 * kPiD * j / n;            // [0, pi]
    return taylor_sin(2 * x > kPiD ? kPiD - x : x);
}

template <int V> using ic = std::integral_constant<int, V>;
template <typename F, int... I>
__device__ __forceinline__ void unroll_seq(F &&f, std::integer_sequence<int, I...>) {
    (f(ic<I>{}), ...);
}
// f(ic<0>), ..., f(ic<N-1>) with compile-time indices
template <int N, typename F>
__device__ __forceinline__ void unroll_c(F &&f) {
    unroll_seq(f, std::make_integer_sequence<int, N>{});
}

// x * exp(-+2 pi i J / NN) with a compile-time twiddle: free for multiples of
// a quarter turn, the eighth turns (+-1 +-i) c take a sum and a scaling, the
// others a full product.  In FP32 the constant is split into hi + lo floats
// (the lo products first), as the table twiddles are; SPLIT = false (the
// range-axis decodes, whose sums are short) rounds it to one float.
template <typename R, int J, int NN, bool INV, bool SPLIT = true, typename C>
__device__ __forceinline__ C twc(C x) {
    constexpr int j = ((J % NN) + NN) % NN;
    if constexpr (j == 0) return x;
    else if constexpr (4 * j == NN) {   // -i (forward), +i (inverse)
        C r;
        if (INV) { r.x = -x.y; r.y = x.x; } else { r.x = x.y; r.y = -x.x; }
        return r;
    } else if constexpr (2 * j == NN) {
        C r;
        r.x = -x.x;
        r.y = -x.y;
        return r;
    } else if constexpr (4 * j == 3 * NN) {
        C r;
        if (INV) { r.x = x.y; r.y = -x.x; } else { r.x = -x.y; r.y = x.x; }
        return r;
    } else {
        constexpr double wc = cos2pi(j, NN), ws0 = -sin2pi(j, NN);
        constexpr double ws = INV ? -ws0 : ws0;
        C r;
        if constexpr (8 * j == NN || 8 * j == 3 * NN || 8 * j == 5 * NN || 8 * j == 7 * NN) {
            // w = c (sx + i sy), sx, sy = +-1
            constexpr double c = wc < 0 ? -wc : wc;
            constexpr R sx = wc < 0 ? R(-1) : R(1), sy = ws < 0 ? R(-1) : R(1);
            const R t1 = sx * x.x - sy * x.y, t2 = sx * x.y + sy * x.x;
            if constexpr (sizeof(R) == 4 && SPLIT) {
                constexpr float ch = (float)c, cl = (float)(c - (double)ch);
                r.x = fmaf(t1, ch, t1 * cl);
                r.y = fmaf(t2, ch, t2 * cl);
            } else {
                r.x = t1 * (R)c;
                r.y = t2 * (R)c;
            }
        } else if constexpr (sizeof(R) == 4 && SPLIT) {
            constexpr float hx = (float)wc, hy = (float)ws;
            constexpr float lx = (float)(wc - (double)hx), ly = (float)(ws - (double)hy);
            const float sxx = fmaf(x.x, lx, -x.y * ly), syy = fmaf(x.x, ly, x.y * lx);
            r.x = fmaf(x.x, hx, fmaf(-x.y, hy, sxx));
            r.y = fmaf(x.x, hy, fmaf(x.y, hx, syy));
        } else {
            r.x = fma(x.x, (R)wc, -x.y * (R)ws);
            r.y = fma(x.x, (R)ws, x.y * (R)wc);
        }
        return r;
    }
}

// In-register DFT of E points, natural order in and out:
// y_s = sum_r v_r exp(-+2 pi i r s / E).  Radix-2 decimation in time after a
// bit reversal that full unrolling turns into register renaming.
// 4-point DFT in place, exp(-+2 pi i / 4) = -+i as operand swaps
template <bool INV, typename C>
__device__ __forceinline__ void dft4(C &a, C &b, C &c, C &d) {
    const C t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), u = csub(b, d);
    C t3;   // (b - d) * (-i) forward, * (+i) inverse
    if (INV) { t3.x = -u.y; t3.y = u.x; } else { t3.x = u.y; t3.y = -u.x; }
    a = cadd(t0, t2);
    c = csub(t0, t2);
    b = cadd(t1, t3);
    d = csub(t1, t3);
}

template <typename R, int E, bool INV, typename C>
__device__ __forceinline__ void reg_fft(C (&v)[E]) {
    if constexpr (E == 16) {
        // 16 = 4 x 4: n = r + 4 m, k = s + 4 t; four 4-point DFTs over m,
        // the turns w_16^(r s) (4 general, 4 eighth, 1 quarter: fewer than
        // the radix-2 split's 8 general and 6 eighth), four over r
        unroll_c<4>([&](auto rr) {
            constexpr int Rr = decltype(rr)::value;
            dft4<INV>(v[Rr], v[Rr + 4], v[Rr + 8], v[Rr + 12]);   // A[r][s] at v[r + 4 s]
            unroll_c<3>([&](auto ss) {
                constexpr int Ss = decltype(ss)::value + 1;
                v[Rr + 4 * Ss] = twc<R, Rr * Ss, 16, INV>(v[Rr + 4 * Ss]);
            });
        });
        C w[16];
        unroll_c<4>([&](auto ss) {
            constexpr int Ss = decltype(ss)::value;
            C a = v[4 * Ss], b = v[4 * Ss + 1], c = v[4 * Ss + 2], d = v[4 * Ss + 3];
            dft4<INV>(a, b, c, d);   // X[s + 4 t]
            w[Ss] = a;
            w[Ss + 4] = b;
            w[Ss + 8] = c;
            w[Ss + 12] = d;
        });
        unroll_c<16>([&](auto q) { v[decltype(q)::value] = w[decltype(q)::value]; });
        return;
    }
    constexpr int LE = ilog2c(E);
    unroll_c<E>([&](auto i) {
        constexpr int I = decltype(i)::value, J = brevc(I, LE);
        if constexpr (I < J) {
            const C t = v[I];
            v[I] = v[J];
            v[J] = t;
        }
    });
    unroll_c<LE>([&](auto st) {
        constexpr int H = 1 << decltype(st)::value;
        unroll_c<E / 2>([&](auto b) {
            constexpr int B = decltype(b)::value, T = B % H, I = (B / H) * 2 * H + T;
            const C y = twc<R, T, 2 * H, INV>(v[I + H]);
            const C x = v[I];
            v[I] = cadd(x, y);
            v[I + H] = csub(x, y);
        });
    });
}

// Per-lane twiddle w_N^(g k1) kept in registers: FP32 as split hi + lo
// floats, FP64 as one double pair.
template <typename R> struct LaneTw;
template <> struct LaneTw<float> {
    float hx, hy, lx, ly;
    __device__ __forceinline__ void load(const TwF *tw, int idx) {
        const TwF w = tw[idx];
        hx = w.hi.x; hy = w.hi.y; lx = w.lo.x; ly = w.lo.y;
    }
    template <bool INV>
    __device__ __forceinline__ float2 mul(float2 a) const {
        const float y_h = INV ? -hy : hy, y_l = INV ? -ly : ly;
        const float sx = fmaf(a.x, lx, -a.y * y_l), sy = fmaf(a.x, y_l, a.y * lx);
        float2 r;
        r.x = fmaf(a.x, hx, fmaf(-a.y, y_h, sx));
        r.y = fmaf(a.x, y_h, fmaf(a.y, hx, sy));
        return r;
    }
};
template <> struct LaneTw<double> {
    double x, y;
    __device__ __forceinline__ void load(const double2 *tw, int idx) {
        const double2 w = tw[idx];
        x = w.x; y = w.y;
    }
    template <bool INV>
    __device__ __forceinline__ double2 mul(double2 a) const {
        const double wy = INV ? -y : y;
        double2 r;
        r.x = fma(a.x, x, -a.y * wy);
        r.y = fma(a.x, wy, a.y * x);
        return r;
    }
};

// The lane twiddles w_N^(g k1), k1 < E, of a line transform: held in
// registers (RegTw), or read from a per-block LDS table of w_N^j, j < N
// (LdsTw: for the largest FP32 tile, whose registers are taken by its 32
// points per lane and the transform's constants).
template <typename R, int E> struct RegTw {
    LaneTw<R> w[E];
    template <typename TWT>
    __device__ __forceinline__ void init(const TWT *tw, int g, int stride) {
        unroll_c<E>([&](auto q) {
            constexpr int K1 = decltype(q)::value;
            w[K1].load(tw, (g * K1 * stride) & (kTwN - 1));
        });
    }
    template <bool INV, int K1, typename C>
    __device__ __forceinline__ C mul(ic<K1>, C x) const { return w[K1].template mul<INV>(x); }
};
template <typename R, int N> struct LdsTw {
    using TWT = typename std::conditional<sizeof(R) == 4, TwF, double2>::type;
    const __attribute__((address_space(3))) TWT *t;   // LDS, N entries
    int g;
    int z = 0;   // an opaque zero per transform (see fresh())
    // A new opaque zero added to the table index: the compiler can then
    // neither hoist the table reads out of the item loop nor share them
    // between the four transforms of an item, which would keep the whole
    // table live in the registers this form exists to save.
    __device__ __forceinline__ void fresh() {
        int q;
        asm volatile("v_mov_b32 %0, 0" : "=v"(q));
        z = q;
    }
    template <bool INV, int K1, typename C>
    __device__ __forceinline__ C mul(ic<K1>, C x) const {
        const int i = ((g * K1) & (N - 1)) + z;
        LaneTw<R> lw;
        if constexpr (sizeof(R) == 4) {
            typedef float f32x4 __attribute__((ext_vector_type(4)));
            const f32x4 w = ((const __attribute__((address_space(3))) f32x4 *)t)[i];
            lw.hx = w.x; lw.hy = w.y; lw.lx = w.z; lw.ly = w.w;
        } else {
            const f64x2 w = ((const __attribute__((address_space(3))) f64x2 *)t)[i];
            lw.x = w.x; lw.y = w.y;
        }
        return lw.template mul<INV>(x);
    }
};
template <typename T> __device__ __forceinline__ void tw_fresh(T &) {}
template <typename R, int N> __device__ __forceinline__ void tw_fresh(LdsTw<R, N> &t) { t.fresh(); }

// Exchange across lanes XOR apart (32 or 16) for a radix-2 stage: the lane
// with the lower partner bit ends with (its a, the partner's a), the other
// with (the partner's b, its b).
template <int XOR>
__device__ __forceinline__ void lane_swap32(uint32_t &a, uint32_t &b) {
    if constexpr (XOR == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}
template <int XOR>
__device__ __forceinline__ void lane_swap(float2 &a, float2 &b) {
    uint32_t ax = __float_as_uint(a.x), ay = __float_as_uint(a.y), bx = __float_as_uint(b.x), by = __float_as_uint(b.y);
    lane_swap32<XOR>(ax, bx);
    lane_swap32<XOR>(ay, by);
    a.x = __uint_as_float(ax); a.y = __uint_as_float(ay); b.x = __uint_as_float(bx); b.y = __uint_as_float(by);
}
template <int XOR>
__device__ __forceinline__ void lane_swap(double2 &a, double2 &b) {
    uint64_t A[2] = {(uint64_t)__double_as_longlong(a.x), (uint64_t)__double_as_longlong(a.y)};
    uint64_t B[2] = {(uint64_t)__double_as_longlong(b.x), (uint64_t)__double_as_longlong(b.y)};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        uint32_t alo = (uint32_t)A[q], ahi = (uint32_t)(A[q] >> 32), blo = (uint32_t)B[q], bhi = (uint32_t)(B[q] >> 32);
        lane_swap32<XOR>(alo, blo);
        lane_swap32<XOR>(ahi, bhi);
        A[q] = (uint64_t)ahi << 32 | alo;
        B[q] = (uint64_t)bhi << 32 | blo;
    }
    a.x = __longlong_as_double((long long)A[0]); a.y = __longlong_as_double((long long)A[1]);
    b.x = __longlong_as_double((long long)B[0]); b.y = __longlong_as_double((long long)B[1]);
}

// Line geometry of the register-resident transform: E points per lane, the
// frequency held in register s by lane part g after a forward transform.
template <int E>
__device__ __forceinline__ constexpr int line_freq_c(int s) {
    // s = j + (E/4) k2b + (E/2) k2a  ->  k = j + E (k2a + 2 k2b) (+ g E / 4)
    return (s % (E / 4)) + E * ((s / (E / 2)) + 2 * ((s / (E / 4)) % 2));
}

// Forward transform of one line held as v[e] = x[g + 4 e] (g: the lane's
// part, lanes 16 apart); afterwards v[s] = X[line_freq_c<E>(s) + g E / 4].
template <typename R, int E, typename C, typename TWS>
__device__ __forceinline__ void line_fwd(C (&v)[E], const TWS &ltw, bool g0) {
    reg_fft<R, E, false>(v);
    unroll_c<E - 1>([&](auto q) {
        constexpr int K1 = decltype(q)::value + 1;
        v[K1] = ltw.template mul<false>(ic<K1>{}, v[K1]);
    });
    // stage over lane-part bit 1 (lanes 32 apart)
    unroll_c<E / 2>([&](auto q) {
        constexpr int J = decltype(q)::value;
        lane_swap<32>(v[J], v[J + E / 2]);
        const C a = v[J], b = v[J + E / 2];
        v[J] = cadd(a, b);
        v[J + E / 2] = csub(a, b);
    });
    // stage over lane-part bit 0 (lanes 16 apart), with the turn -i of the
    // k2a = 1 values of the lane parts with bit 0 set: after the exchange the
    // second operand of every pair is such a part's value, so the turn is a
    // compile-time -i butterfly on the pairs of k2a = 1 in every lane
    unroll_c<E / 2>([&](auto q) {
        constexpr int Q = decltype(q)::value, J = Q % (E / 4) + (Q / (E / 4)) * (E / 2);
        lane_swap<16>(v[J], v[J + E / 4]);
        const C a = v[J];
        C b = v[J + E / 4];
        if constexpr (J >= E / 2) {   // k2a = 1: b * (-i)
            const R t = b.x;
            b.x = b.y;
            b.y = -t;
        }
        v[J] = cadd(a, b);
        v[J + E / 4] = csub(a, b);
    });
    (void)g0;
}

// Inverse (unnormalised) of line_fwd: takes v[s] = X[line_freq_c<E>(s) + g E / 4],
// leaves v[e] = N x[g + 4 e] with x the inverse DFT of X.
template <typename R, int E, typename C, typename TWS>
__device__ __forceinline__ void line_inv(C (&v)[E], const TWS &ltw, bool g0) {
    // mirror of the last stage of line_fwd: (p, q) -> (p + q, (p - q) * (+i)
    // for the pairs of k2a = 1), then the exchange
    unroll_c<E / 2>([&](auto q) {
        constexpr int Q = decltype(q)::value, J = Q % (E / 4) + (Q / (E / 4)) * (E / 2);
        const C a = v[J], b = v[J + E / 4];
        v[J] = cadd(a, b);
        C d = csub(a, b);
        if constexpr (J >= E / 2) {   // k2a = 1: d * (+i)
            const R t = d.x;
            d.x = -d.y;
            d.y = t;
        }
        v[J + E / 4] = d;
        lane_swap<16>(v[J], v[J + E / 4]);
    });
    (void)g0;
    unroll_c<E / 2>([&](auto q) {
        constexpr int J = decltype(q)::value;
        const C a = v[J], b = v[J + E / 2];
        v[J] = cadd(a, b);
        v[J + E / 2] = csub(a, b);
        lane_swap<32>(v[J], v[J + E / 2]);
    });
    unroll_c<E - 1>([&](auto q) {
        constexpr int K1 = decltype(q)::value + 1;
        v[K1] = ltw.template mul<true>(ic<K1>{}, v[K1]);
    });
    reg_fft<R, E, true>(v);
}

// Eight lanes per line (lanes 8 apart, E = N / 8 points each): the same
// Cooley-Tukey split with G = 8, its 8-point DFT across the lanes as three
// radix-2 stages over the lane-part bits (lanes 32, 16 and 8 apart).  With
// g = 4 g2 + 2 g1 + g0 and k2 = k2a + 2 k2b + 4 k2c,
//   w_8^(g k2) = (-1)^(g2 k2a) w_4^(g1 k2a) (-1)^(g1 k2b) w_8^(g0 (k2a + 2 k2b)) (-1)^(g0 k2c),
// so the turn before the second stage is -i (k2a = 1) and before the third
// w_8^(k2a + 2 k2b), each on the operand that the exchange brings from the
// part with that bit set, a compile-time turn per register.  Lane part g then
// holds k1 in [g E/8, (g+1) E/8) for every k2: register
// s = j + (E/8) k2c + (E/4) k2b + (E/2) k2a has k = j + g E/8 + E k2.
template <int E>
__device__ __forceinline__ constexpr int line_freq8_c(int s) {
    return (s % (E / 8)) + E * ((s / (E / 2)) + 2 * ((s / (E / 4)) % 2) + 4 * ((s / (E / 8)) % 2));
}

// Exchange across lanes 8 apart (the same semantics as lane_swap<32/16>),
// through a row rotation by 8 of the 16-lane DPP rows: each lane sends the
// value its partner keeps and takes the partner's.
__device__ __forceinline__ void lane_swap8_32(uint32_t &a, uint32_t &b, bool hi) {
    const uint32_t t = hi ? a : b;
    const uint32_t r = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0x128, 0xf, 0xf, false);   // row_ror:8
    a = hi ? r : a;
    b = hi ? b : r;
}
__device__ __forceinline__ void lane_swap8(float2 &a, float2 &b, bool hi) {
    uint32_t ax = __float_as_uint(a.x), ay = __float_as_uint(a.y), bx = __float_as_uint(b.x), by = __float_as_uint(b.y);
    lane_swap8_32(ax, bx, hi);
    lane_swap8_32(ay, by, hi);
    a.x = __uint_as_float(ax); a.y = __uint_as_float(ay); b.x = __uint_as_float(bx); b.y = __uint_as_float(by);
}

// Forward transform of one line held as v[e] = x[g + 8 e] (lane part g, lanes
// 8 apart; hi: bit 0 of g); afterwards v[s] = X[line_freq8_c<E>(s) + g E / 8].
template <typename R, int E, typename C, typename TWS>
__device__ __forceinline__ void line_fwd8(C (&v)[E], const TWS &ltw, bool hi) {
    reg_fft<R, E, false>(v);
    unroll_c<E - 1>([&](auto q) {
        constexpr int K1 = decltype(q)::value + 1;
        v[K1] = ltw.template mul<false>(ic<K1>{}, v[K1]);
    });
    // lane-part bit 2 (lanes 32 apart): k2a
    unroll_c<E / 2>([&](auto q) {
        constexpr int J = decltype(q)::value;
        lane_swap<32>(v[J], v[J + E / 2]);
        const C a = v[J], b = v[J + E / 2];
        v[J] = cadd(a, b);
        v[J + E / 2] = csub(a, b);
    });
    // bit 1 (lanes 16 apart): k2b, after the turn -i of k2a = 1
    unroll_c<E / 2>([&](auto q) {
        constexpr int Q = decltype(q)::value, J = Q % (E / 4) + (Q / (E / 4)) * (E / 2);
        lane_swap<16>(v[J], v[J + E / 4]);
        const C a = v[J];
        C b = v[J + E / 4];
        if constexpr (J >= E / 2) {
            const R t = b.x;
            b.x = b.y;
            b.y = -t;
        }
        v[J] = cadd(a, b);
        v[J + E / 4] = csub(a, b);
    });
    // bit 0 (lanes 8 apart): k2c, after the turn w_8^(k2a + 2 k2b)
    unroll_c<E / 2>([&](auto q) {
        constexpr int Q = decltype(q)::value, J = Q % (E / 8) + (Q / (E / 8)) * (E / 4);
        constexpr int TW = (J / (E / 2)) + 2 * ((J / (E / 4)) % 2);
        lane_swap8(v[J], v[J + E / 8], hi);
        const C a = v[J];
        const C b = twc<R, TW, 8, false>(v[J + E / 8]);
        v[J] = cadd(a, b);
        v[J + E / 8] = csub(a, b);
    });
}

// Inverse (unnormalised) of line_fwd8: takes v[s] = X[line_freq8_c<E>(s) + g E / 8],
// leaves v[e] = N x[g + 8 e].
template <typename R, int E, typename C, typename TWS>
__device__ __forceinline__ void line_inv8(C (&v)[E], const TWS &ltw, bool hi) {
    unroll_c<E / 2>([&](auto q) {
        constexpr int Q = decltype(q)::value, J = Q % (E / 8) + (Q / (E / 8)) * (E / 4);
        constexpr int TW = (J / (E / 2)) + 2 * ((J / (E / 4)) % 2);
        const C a = v[J], b = v[J + E / 8];
        v[J] = cadd(a, b);
        v[J + E / 8] = twc<R, TW, 8, true>(csub(a, b));
        lane_swap8(v[J], v[J + E / 8], hi);
    });
    unroll_c<E / 2>([&](auto q) {
        constexpr int Q = decltype(q)::value, J = Q % (E / 4) + (Q / (E / 4)) * (E / 2);
        const C a = v[J], b = v[J + E / 4];
        v[J] = cadd(a, b);
        C d = csub(a, b);
        if constexpr (J >= E / 2) {   // * (+i)
            const R t = d.x;
            d.x = -d.y;
            d.y = t;
        }
        v[J + E / 4] = d;
        lane_swap<16>(v[J], v[J + E / 4]);
    });
    unroll_c<E / 2>([&](auto q) {
        constexpr int J = decltype(q)::value;
        const C a = v[J], b = v[J + E / 2];
        v[J] = cadd(a, b);
        v[J + E / 2] = csub(a, b);
        lane_swap<32>(v[J], v[J + E / 2]);
    });
    unroll_c<E - 1>([&](auto q) {
        constexpr int K1 = decltype(q)::value + 1;
        v[K1] = ltw.template mul<true>(ic<K1>{}, v[K1]);
    });
    reg_fft<R, E, true>(v);
}

// XCD-aware walk of a persistent launch's items.  Workgroups are dealt to the
// eight XCDs in turn (workgroup b to XCD b mod 8), each XCD with its own L2.
// Striding the items by the grid would put consecutive items -- the tiles of
// one range bin, sharing its SE spectrum, and the bins of one tile, sharing
// its image rows -- on all eight XCDs at once, so every L2 would fetch the
// same data.  Instead each XCD walks its own contiguous eighth of the items
// (grid a multiple of 8; otherwise the plain stride).
struct XcdWalk {
    long long it, end, step;
    __device__ __forceinline__ XcdWalk(long long nitems) {
        const int grid = gridDim.x;
        if (grid % 8 == 0 && grid >= 8) {
            const int x = blockIdx.x & 7;
            const long long per = (nitems + 7) / 8;
            it = x * per + (blockIdx.x >> 3);
            end = min(nitems, (x + 1) * per);
            step = grid >> 3;
        } else {
            it = blockIdx.x;
            end = nitems;
            step = grid;
        }
    }
};

// Item order of k_fft_reg within a segment: groups of G tiles, all bins of a
// group before the next, bin-major inside it (the last group takes the
// remaining tiles).  With G a quarter of the walk's stride (the blocks of one
// XCD), a block's consecutive items are every fourth bin of one tile, which
// it keeps in its grey-value cache, and the XCD's blocks share G image
// windows and four bins' SE spectra at a time in their L2.  (G equal to the
// stride, every bin of a tile in one block, measured slower.)
__device__ __forceinline__ int tile_group_width(long long step) { return step >= 32 ? (int)(step / 4) : 8; }
__device__ __forceinline__ void tile_group_item(int local, int ntiles, int bins, int G, int &m, int &tl) {
    const int full = ntiles - ntiles % G;   // tiles in whole groups
    if (local < full * bins) {
        const int per = bins * G, grp = local / per, q = local - grp * per;
        m = q / G;
        tl = grp * G + (q - m * G);
    } else {
        const int rem = ntiles - full, q = local - full * bins;
        m = q / rem;
        tl = full + (q - m * rem);
    }
}

// waves per SIMD asked of k_fft_reg: the LDS allows four 64-point FP32 blocks
// (16 waves) per CU, and with the twiddle table in LDS they fit 128 VGPRs; the
// 128-point FP32 block of eight lanes per line is 16 waves, 4 per SIMD
// Number of SE cells y whose window pixel x - y lies in the image, for the
// pixel (gy, gx): the count of active cells (a, c) of the effective mask with
// a in [gy + r - H + 1, gy + r] and c in [gx + r - W + 1, gx + r], from the
// mask's prefix counts.  Every such pair adds 1 to exactly one coefficient of
// the pixel's product polynomial (Sec. 3.1), so the coefficients sum to it.
__device__ __forceinline__ int window_cells(const JobDev &J, int gy, int gx) {
    const int k = J.k, r = (k - 1) >> 1, kp = k + 1;
    const int a0 = max(0, gy + r - J.H + 1), a1 = min(k - 1, gy + r);
    const int c0 = max(0, gx + r - J.W + 1), c1 = min(k - 1, gx + r);
    if (a0 > a1 || c0 > c1) return 0;
    const auto P = gld(J.se_cnt);
    return P[(a1 + 1) * kp + c1 + 1] - P[a0 * kp + c1 + 1] - P[(a1 + 1) * kp + c0] + P[a0 * kp + c0];
}

// Bin 0 of every (tile, bin) item has a closed form.  At m = 0 the
// range-DFT column of every in-image grey value is 1 and that of every SE
// cell is 1 (Step 1), so the bin-0 product at a pixel is the count of SE
// cells whose window pixel lies in the image, window_cells, and the
// unscaled inverse 2-D transform holds nt^2 times it: an integer times a
// power of two, exact in either precision.  The transform kernels write
// that plane instead of transforming the item (the FP64 recompute of a
// flagged tile still transforms every bin).  L >= 2, so n_r >= 2 and every
// tile has a transformed bin whose encode checks the tile's values against
// [0, L-1].
template <typename R>
__device__ __forceinline__ typename Cx<R>::T dc_plane_value(const JobDev &J, int nt, int gy, int gx, R bump) {
    typename Cx<R>::T o;
    o.x = (R)((double)nt * nt) * (R)window_cells(J, gy, gx) + bump;
    o.y = R(0);
    return o;
}

template <typename R, int N, int G> constexpr int fft_reg_waves() {
    return sizeof(R) == 4 && (N == 64 || G == 8) ? 4 : 1;
}

// G lanes per line: 4 (lanes 16 apart), or 8 (lanes 8 apart, line_fwd8).
template <typename R, int N, int G = 4>
__global__ __launch_bounds__(G * N) __attribute__((amdgpu_waves_per_eu(fft_reg_waves<R, N, G>()))) void k_fft_reg(const JobDev *__restrict__ jobs, const Seg *__restrict__ segs,
                                                   int nseg, long long nitems, const TwF *__restrict__ tw32,
                                                   const double2 *__restrict__ tw64, StatsDev *st,
                                                   const uint8_t *__restrict__ perturb) {
    using C = typename Cx<R>::T;
    static_assert(G == 4 || G == 8, "four or eight lanes per line");
    // points per lane, lines per wave; LDS row pitch P (complex values): with
    // eight lanes per line a 16-lane group spans 8 lines and 2 lane parts, and
    // N + 4 puts both its row accesses (line P + g + 8 e) and its column
    // accesses ((2 g + f) P + line) in 32 distinct banks
    constexpr int E = N / G, P = G == 8 ? N + 4 : N + 1, LW = 64 / G;
    static_assert(E >= 4 && (E & (E - 1)) == 0 && (G == 4 || E >= 8), "E = N / G must be a power of two");
    using TWT = typename std::conditional<sizeof(R) == 4, TwF, double2>::type;
    constexpr bool TW_LDS = sizeof(R) == 4 && N >= 64;
    __shared__ C lds[N * P];
    __shared__ TWT tws[TW_LDS ? N : 1];
    // grey values of the block's current tile window, one byte each, for the
    // next items of the same tile (a lane reads back only what it wrote);
    // rows padded by a word so that a wave's four rows use distinct banks
    constexpr int VP = N + 4;
    __shared__ uint8_t vcache[N * VP];
    const int lane = threadIdx.x & 63, g = lane / LW;
    const bool g0 = (g & 1) != 0;
    const int line = (threadIdx.x >> 6) * LW + (lane & (LW - 1));   // column (phases 1, 3) or row (phase 2)
    const int lbase = (threadIdx.x >> 6) * LW;                       // first line of this wave
    // the frequency of register s after a forward line transform (plus g E / G)
    auto lfreq = [](auto q) constexpr {
        constexpr int Qv = decltype(q)::value;
        return G == 4 ? line_freq_c<E>(Qv) : line_freq8_c<E>(Qv);
    };
    const TWT *twg;
    if constexpr (sizeof(R) == 4) twg = tw32; else twg = tw64;
    // w_N^(g k1), k1 < E
    typename std::conditional<TW_LDS, LdsTw<R, N>, RegTw<R, E>>::type ltw;
    if constexpr (TW_LDS) {
        for (int j = threadIdx.x; j < N; j += G * N) tws[j] = twg[j * (kTwN / N)];
        ltw.t = (const __attribute__((address_space(3))) TWT *)tws;
        ltw.g = g;
        __syncthreads();
    } else {
        ltw.init(twg, g, kTwN / N);
    }
    // LDS row of register s in phases 1 and 3: the frequency it holds
    const int frow = g * (E / G);
    // byte offset of this lane's first spectrum value ([kx][ky], kx = frow + ...)
    const unsigned spec_voff = (unsigned)(frow * N + line) * sizeof(C);
    XcdWalk walk(nitems);
    const int tgw = tile_group_width(walk.step);
    long long cached = -1;    // (job, tile) whose grey values vcache holds
    unsigned inmask = 0;      // in-image bits of this lane's points, for that tile
    for (long long it = walk.it; it < walk.end; it += walk.step) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0);   // a segment holds fewer than 2^31 items
        // bin 0 of a tile is an item of its own, written in closed form:
        // the blocks walk the items in a fixed stride, so a cheap item only
        // lets its block finish early (bin 0 written with bin 1 made that
        // block the last one)
        int m, tl;
        tile_group_item(local, S.ntiles, J.bins, tgw, m, tl);
        const int tile = S.tile0 + tl;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const int k = J.k, r = (k - 1) >> 1, T = N - k + 1;
        const int iy0 = ty * J.T - r, ix0 = tx * J.T - r;
        if (m == 0) {
            // bin 0 in closed form (block-uniform; no LDS use, so the next
            // item needs no barrier after it); left to the decode for dc_dec
            // jobs
            C *yt = (C *)S.y + (size_t)tl * ytile_elems(J.bins, J.T, J.ybs) + ybin_offset(0, J.T, J.ybs);
            const R bump = perturb_bump<R>(perturb, J, tile, 0, kPerturbFirst);
            for (int q = threadIdx.x; q < (J.dc_dec ? 0 : T * T); q += G * N) {
                const int i = q / T, j = q - i * T;
                stg(yt, ypix(q, J.ybs), dc_plane_value<R>(J, N, ty * J.T + i, tx * J.T + j, bump));
            }
            continue;
        }
        // 1. columns: encode (Step 1) and forward transform along y.  The
        // range-DFT column of grey value w is read through a buffer resource
        // of the L table entries: an out-of-image pixel takes index L, past
        // the table, and reads the zero polynomial.
        C v[E];
        {
            const int W = J.W, H = J.H, L = J.L;
            const int gx = ix0 + line, y0 = iy0 + g;
            const bool colin = (unsigned)gx < (unsigned)W;
            const int32_t *col = J.img + ((ptrdiff_t)y0 * W + gx);   // pixel (y0, gx); read only in the image
            const __amdgpu_buffer_rsrc_t ers =
                __builtin_amdgcn_make_buffer_rsrc((void *)((const C *)J.enc + (size_t)m * L), (short)0,
                                                  (int)(L * sizeof(C)), kBufWord3);
            // erosion complements the values: w = (L - 1) - v = (v ^ -1) + L
            const unsigned wxor = J.op ? ~0u : 0u, wadd = J.op ? (unsigned)L : 0u;
            int val[E];
            bool in[E];
            const long long npx = (long long)H * W;
            const long long key = ((long long)S.job << 32) | (unsigned)(S.tile0 + tl);
            if (key == cached) {
                // the same tile as the block's previous item: its values
                // (checked against L when loaded) from the cache
                unroll_c<E>([&](auto q) {
                    constexpr int Q = decltype(q)::value;
                    in[Q] = (inmask >> Q) & 1u;
                    val[Q] = vcache[(g + G * Q) * VP + line];
                });
            } else if (npx < (1ll << 29) && W <= (1 << 22)) {
                // the image through a buffer resource: the pixel (y0 + G Q, gx)
                // at byte offset o0 + 4 G W Q, in 32-bit unsigned arithmetic.
                // An in-image pixel lies below 4 H W < 2^31; a row above the
                // image wraps to [2^31, 2^32), a row below stays under 2^32,
                // and a column outside the image starts at 2^31: all past the
                // resource, so their loads return 0 and the offset test marks
                // them out.
                const __amdgpu_buffer_rsrc_t irs =
                    __builtin_amdgcn_make_buffer_rsrc((void *)J.img, (short)0, (int)(npx * 4), kBufWord3);
                const unsigned o0 = colin ? ((unsigned)y0 * (unsigned)W + (unsigned)gx) * 4u : 0x80000000u;
                const unsigned step = 4u * G * (unsigned)W, lim = (unsigned)(npx * 4);
                unroll_c<E>([&](auto q) {
                    constexpr int Q = decltype(q)::value;
                    const unsigned o = o0 + (unsigned)Q * step;
                    in[Q] = o < lim;
                    val[Q] = __builtin_amdgcn_raw_buffer_load_b32(irs, o, 0, 0);
                });
            } else {
                unroll_c<E>([&](auto q) {
                    constexpr int Q = decltype(q)::value;
                    in[Q] = colin && (unsigned)(y0 + G * Q) < (unsigned)H;
                    val[Q] = in[Q] ? gld(col)[(ptrdiff_t)(G * Q) * W] : 0;
                });
            }
            unsigned top = 0;   // largest in-image value (as unsigned: negatives count as large)
            unroll_c<E>([&](auto q) {
                constexpr int Q = decltype(q)::value;
                top = max(top, (unsigned)val[Q]);
                const unsigned idx = in[Q] ? (((unsigned)val[Q] ^ wxor) + wadd) : (unsigned)L;
                v[Q] = buf_load<C>(ers, idx * (unsigned)sizeof(C), 0);
            });
            if (key != cached) {
                if (__any(top >= (unsigned)L) && lane == 0) atomicOr(&st->range_err, 1u);
                // values below L <= 256 fit a byte: keep them for this tile's
                // next items
                if (L <= 256) {
                    inmask = 0;
                    unroll_c<E>([&](auto q) {
                        constexpr int Q = decltype(q)::value;
                        vcache[(g + G * Q) * VP + line] = (uint8_t)val[Q];
                        inmask |= (unsigned)in[Q] << Q;
                    });
                    cached = key;
                } else {
                    cached = -1;
                }
            }
        }
        tw_fresh(ltw);
        if constexpr (G == 4) line_fwd<R, E>(v, ltw, g0); else line_fwd8<R, E>(v, ltw, g0);
        unroll_c<E>([&](auto q) {
            constexpr int Q = decltype(q)::value;
            lds[(frow + lfreq(ic<Q>{})) * P + line] = v[Q];
        });
        __syncthreads();
        // 2. rows: forward along x, times the SE spectrum, inverse along x
        unroll_c<E>([&](auto q) {
            constexpr int Q = decltype(q)::value;
            v[Q] = lds[line * P + g + G * Q];
        });
        tw_fresh(ltw);
        if constexpr (G == 4) line_fwd<R, E>(v, ltw, g0); else line_fwd8<R, E>(v, ltw, g0);
        {
            // spectrum values through a buffer resource: one offset register
            // per lane, the compile-time steps as uniform offsets; loads in
            // groups of up to 8 (register pressure)
            const __amdgpu_buffer_rsrc_t srs =
                __builtin_amdgcn_make_buffer_rsrc((void *)((const C *)J.se_spec + (size_t)m * N * N), (short)0,
                                                  (int)(N * N * sizeof(C)), kBufWord3);
            constexpr int SG = E < 8 ? E : 8;
            unroll_c<E / SG>([&](auto cg) {
                constexpr int Q0 = SG * decltype(cg)::value;
                C sv[SG];
                unroll_c<SG>([&](auto q) {
                    constexpr int Q = Q0 + decltype(q)::value;
                    sv[Q - Q0] = buf_load<C>(srs, spec_voff, (unsigned)(lfreq(ic<Q>{}) * N * sizeof(C)));
                });
                unroll_c<SG>([&](auto q) {
                    constexpr int Q = Q0 + decltype(q)::value;
                    v[Q] = cmul(v[Q], sv[Q - Q0]);
                });
            });
        }
        tw_fresh(ltw);
        if constexpr (G == 4) line_inv<R, E>(v, ltw, g0); else line_inv8<R, E>(v, ltw, g0);
        unroll_c<E>([&](auto q) {
            constexpr int Q = decltype(q)::value;
            lds[line * P + g + G * Q] = v[Q];
        });
        __syncthreads();
        // 3. columns: inverse along y and the valid outputs (rows and columns
        // >= k - 1); waves whose columns all lie left of them skip it
        if (lbase + LW - 1 >= k - 1) {
            unroll_c<E>([&](auto q) {
                constexpr int Q = decltype(q)::value;
                v[Q] = lds[(frow + lfreq(ic<Q>{})) * P + line];
            });
            tw_fresh(ltw);
            if constexpr (G == 4) line_inv<R, E>(v, ltw, g0); else line_inv8<R, E>(v, ltw, g0);
            const R bump = perturb_bump<R>(perturb, J, tile, m, kPerturbFirst);
            const int oc = line - (k - 1);
            if (oc >= 0) {
                // stores through a buffer resource over the tile's values; the
                // pixel index of row g + G Q is q0 + G T Q, negative for the
                // discarded rows, which then take an offset past the resource
                // and are dropped.  The [bins][T*T] layout is the blocked one
                // with 16-pixel blocks of pitch 16.  (Jobs on the short-length
                // decode in the bin-major layout, whose kept rows need no
                // per-row offset, measured slower.)
                const size_t te = ytile_elems(J.bins, J.T, J.ybs);
                const __amdgpu_buffer_rsrc_t ors = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)((C *)S.y + (size_t)tl * te), (short)0, (int)(te * sizeof(C)), kBufWord3);
                const int ybs = J.ybs ? J.ybs : 16;
                const int binoff = (int)ybin_offset(m, J.T, J.ybs);
                const int q0 = (g - (k - 1)) * T + oc;
                unroll_c<E>([&](auto q) {
                    constexpr int Q = decltype(q)::value;
                    const int qq = q0 + G * Q * T;
                    const unsigned e = (unsigned)(binoff + (qq >> 4) * ybs + (qq & 15));
                    C o = v[Q];
                    o.x += bump;
                    buf_store<C>(o, ors, qq >= 0 ? e * (unsigned)sizeof(C) : 0xfffffff0u, 0);
                });
            }
        }
        __syncthreads();
    }
}


// Step 3 on one coefficient c_d: the top degree with rint(c_d) != 0, and
// what the exactness checks need: the largest distance |c_d - rint(c_d)|, the
// sum of the rounded coefficients and whether any rounds below zero.
template <typename R>
struct PxDecode {
    int top = -1;
    R res = 0, sum = 0;
    bool neg = false;
    __device__ __forceinline__ void add(R c, int d) {
        const R rc = rint(c);
        res = fmax(res, fabs(c - rc));
        sum += rc;
        neg |= rc < R(0);
        if (rc != R(0)) top = max(top, d);
    }
};


// Whether a decoded pixel fails the exactness checks (band: the residual
// bound of the pass).
template <typename R>
__device__ __forceinline__ bool px_ambiguous(const PxDecode<R> &dd, float band, const JobDev &J, int gy, int gx) {
    return (float)dd.res >= band || dd.neg || (int)dd.sum != window_cells(J, gy, gx);
}

// Large tiles (FP32 256..1024 points per side, FP64 128..1024) in three
// grid-wide passes.  The N x N array of a (tile, bin) item does not fit the
// LDS, so each pass takes batches of LB = big_lines() lines of one item
// through the LDS, and the array lives in a per-item intermediate `mid` in
// global memory between passes.  A launch handles a chunk of `cn` items
// starting at `it0` (the chunk's intermediates are small enough to stay in
// the L2 and Infinity Cache between the passes):
//   PH 0: encode LB image rows in column order, forward DIF along x
//         (column c then holds kx = brev(c)), store row i at intermediate
//         row brev(i) (the columns then hold bit-reversed input for the DIT
//         along y);
//   PH 1: LB columns c: forward DIT along y, times the SE spectrum row
//         kx = brev(c) ([kx][ky]), inverse DIF along y (row r' then holds
//         output row brev(r')), stored back for the kept rows
//         brev(r') >= k - 1 only;
//   PH 2: LB kept output rows y = k - 1 + b LB + l (intermediate row
//         brev(y)): inverse DIT along x (bit-reversed kx in, x in column
//         order out) and the T x T valid outputs; the batches past the last
//         kept row return at once.
// Every LDS walk outside the butterflies is in column order: a bit-reversed
// LDS index would put the lanes of a wavefront on a few banks.  The items
// are bins 1 .. bins - 1; PH 2 writes bin 0's closed-form plane
// (dc_plane_value) with bin 1.
// Work units are (item, batch) pairs, walked per XCD (XcdWalk): item-major
// in PH 0 and 2, so that the blocks of one XCD share an item's image rows
// and intermediate lines in their L2; in PH 1 in pairs of batches, each
// pair over every item (see there).
template <typename R, int N, int PH>
__global__ __launch_bounds__(kBigThreads) void k_fft_big(const JobDev *__restrict__ jobs, const Seg *__restrict__ segs,
                                                         int nseg, long long it0, int cn, const TwF *__restrict__ tw32,
                                                         const double2 *__restrict__ tw64, void *mid, StatsDev *st,
                                                         const uint8_t *__restrict__ perturb) {
    using C = typename Cx<R>::T;
    constexpr int BS = kBigThreads, LB = big_lines<R, N>(), NB = N / LB;
    static_assert(NB % 2 == 0, "the column pass walks batches in pairs");
    constexpr int P = N + 1, LG = ilog2c(N), LLB = ilog2c(LB);
    constexpr int CHM = sizeof(R) == 4 ? 4 : 16;
    constexpr int CH = LB * N / BS < CHM ? LB * N / BS : CHM;
    __shared__ C lds[LB * P];
    typename TwSel<R>::T tw;
    if constexpr (sizeof(R) == 4) tw.p = tw32; else tw.p = tw64;
    // PH 0 and 2 deal the items to the XCDs in turn (item s to XCD s mod 8,
    // its NB batches consecutive there), so that items of unequal cost (PH 2
    // writes bin 0's plane with bin 1; edge tiles keep fewer rows) spread
    // over all of them.  PH 1 walks contiguous ranges of its batch-pair
    // order, which spans every item.
    const int grid = gridDim.x, xcd = blockIdx.x & 7;
    const bool deal = PH != 1 && grid % 8 == 0;
    XcdWalk walk((long long)cn * NB);
    if (deal) {
        walk.it = blockIdx.x >> 3;
        walk.end = (long long)((cn - xcd + 7) / 8) * NB;   // items xcd + 8 q
        walk.step = grid >> 3;
    }
    for (long long u = walk.it; u < walk.end; u += walk.step) {
        int i, b;
        if (deal) {
            const long long q = u / NB;
            i = xcd + 8 * (int)q;
            b = (int)(u - q * NB);
        } else if constexpr (PH == 1) {
            // pairs of column batches (at 512 points in FP32, whole 128-byte
            // lines of the intermediate rows), every item of the chunk per
            // pair: an XCD's blocks then share each pair's slice of the
            // spectra in their L2
            const long long pr = u / (2 * cn);
            const int rem = (int)(u - pr * 2 * cn);
            i = rem >> 1;
            b = (int)pr * 2 + (rem & 1);
        } else {
            i = (int)(u / NB);
            b = (int)(u - (long long)i * NB);
        }
        const long long it = it0 + i;
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0);   // a segment holds fewer than 2^31 items
        // the items are bins 1 .. bins - 1 of each tile (bin-major); bin 0,
        // in closed form, is written by PH 2 with bin 1
        const int mi = local / S.ntiles, tl = local - mi * S.ntiles, m = mi + 1;
        const int tile = S.tile0 + tl;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const int k = J.k, r = (k - 1) >> 1, T = N - k + 1;
        C *slab = (C *)mid + (size_t)i * N * N;
        if constexpr (PH == 0) {
            const int rb = b * LB;
            const C *enc_m = (const C *)J.enc + (size_t)m * J.L;
            const int bad = encode_rows<R, N, BS, CH, false>(
                LB, J.img, J.H, J.W, J.L, J.op, ty * J.T - r + rb, tx * J.T - r, enc_m,
                [&](int l, int c, C v) { lds[l * P + c] = v; });
            if (bad) atomicOr(&st->range_err, 1u);   // every transformed bin checks its rows
            __syncthreads();
            dif_axis<R, N, 0, BS, false, LB>(lds, tw);
            for (int q = threadIdx.x; q < LB * N; q += BS) {
                const int l = q >> LG, v = q & (N - 1);
                stg(slab, (size_t)brev<LG>(rb + l) * N + v, lds[l * P + v]);
            }
        } else if constexpr (PH == 1) {
            const int cb = b * LB;
            const C *spec_m = (const C *)J.se_spec + (size_t)m * N * N;
            batched<BS, CH>(
                LB * N, [&](int q) { return ldg(slab, (size_t)(q >> LLB) * N + cb + (q & (LB - 1))); },
                [&](int q, C v) { lds[(q & (LB - 1)) * P + (q >> LLB)] = v; });
            __syncthreads();
            dit_axis<R, N, 0, BS, false, LB>(lds, tw);
            // the spectrum is stored [kx][ky]: q walks ky fastest
            batched<BS, CH>(
                LB * N, [&](int q) { return ldg(spec_m, (size_t)brev<LG>(cb + (q >> LG)) * N + (q & (N - 1))); },
                [&](int q, C sv) {
                    C *e = lds + (q >> LG) * P + (q & (N - 1));
                    *e = cmul(*e, sv);
                });
            __syncthreads();
            dif_axis<R, N, 0, BS, true, LB>(lds, tw);
            for (int q = threadIdx.x; q < LB * N; q += BS) {
                const int rr = q >> LLB, l = q & (LB - 1);
                if (brev<LG>(rr) >= k - 1) stg(slab, (size_t)rr * N + cb + l, lds[l * P + rr]);
            }
        } else {
            // line l is output row y0 + l, intermediate row brev(y0 + l); the
            // lines of a last, partial batch past row N - 1 re-read row N - 1
            // and are not stored
            const int y0 = k - 1 + b * LB;
            if (y0 >= N) continue;   // block-uniform: the whole block skips the unit
            if (m == 1 && !J.dc_dec) {
                // the same rows of bin 0's plane (global stores only; for
                // dc_dec jobs the decode takes bin 0 in closed form)
                C *d0 = (C *)S.y + (size_t)tl * ytile_elems(J.bins, J.T, J.ybs) + ybin_offset(0, J.T, J.ybs);
                const R bump0 = perturb_bump<R>(perturb, J, tile, 0, kPerturbFirst);
                for (int q = threadIdx.x; q < LB * T; q += BS) {
                    const int l = q / T, xo = q - l * T, y = y0 + l;
                    if (y < N) {
                        const int yo = y - (k - 1);
                        stg(d0, ypix((size_t)yo * T + xo, J.ybs),
                            dc_plane_value<R>(J, N, ty * J.T + yo, tx * J.T + xo, bump0));
                    }
                }
            }
            C *ydst = (C *)S.y + (size_t)tl * ytile_elems(J.bins, J.T, J.ybs) + ybin_offset(m, J.T, J.ybs);
            const R bump = perturb_bump<R>(perturb, J, tile, m, kPerturbFirst);
            batched<BS, CH>(
                LB * N,
                [&](int q) {
                    const int y = min(y0 + (q >> LG), N - 1);
                    return ldg(slab, (size_t)brev<LG>(y) * N + (q & (N - 1)));
                },
                [&](int q, C v) { lds[(q >> LG) * P + (q & (N - 1))] = v; });
            __syncthreads();
            dit_axis<R, N, 0, BS, true, LB>(lds, tw);
            for (int q = threadIdx.x; q < LB * T; q += BS) {
                const int l = q / T, xo = q - l * T;
                if (y0 + l < N) {
                    C v = lds[l * P + xo + k - 1];
                    v.x += bump;
                    stg(ydst, ypix((size_t)(y0 + l - (k - 1)) * T + xo, J.ybs), v);
                }
            }
        }
        __syncthreads();
    }
}

// Inverse real DFT over the range axis for one pixel per lane, and Step 3:
// c_d = A_d - B_d and c_{nr-d} = A_d + B_d for d <= nr/2 (the coefficient
// vector is real), with A_d = sum_m w_m Re(X_m) cos(2 pi d m / nr) and
// B_d = sum_m w_m Im(X_m) sin(2 pi d m / nr); then the top degree with
// rint(c_d) != 0 and the largest distance |c_d - rint(c_d)| over all degrees.
//
// The [bin][degree] table is zero-padded (pitch `dp`, a multiple of 32, in
// both dimensions), so MB bins x DC degrees are accumulated per block with no
// branch: padded bins and degrees add zeros.  The twiddle index depends only
// on (bin, degree), so the table arrives through wave-uniform scalar loads.
// With bins <= MB and nr/2 < DC one pass covers the pixel and its bin values
// are loaded once.
template <typename R, int MB, int DC>
__device__ __forceinline__ void decode_px(const typename Cx<R>::T *X, size_t mstride, size_t p, bool valid,
                                          const typename Cx<R>::T *dec, int dp, int nr, int bins, R scale,
                                          PxDecode<R> &out) {
    using C = typename Cx<R>::T;
    const int dh = nr >> 1;
    out = PxDecode<R>();
    if (!__any(valid)) return;   // the whole wave lies outside the image
    for (int d0 = 0; d0 <= dh; d0 += DC) {
        R A[DC], B[DC];
#pragma unroll
        for (int dd = 0; dd < DC; ++dd) A[dd] = B[dd] = 0;
        for (int m0 = 0; m0 < bins; m0 += MB) {
            C x[MB];
#pragma unroll
            for (int mm = 0; mm < MB; ++mm) {
                x[mm] = czero<C>();
                if (valid && m0 + mm < bins) x[mm] = ldg(X, (size_t)(m0 + mm) * mstride + p);
            }
            const C *blk = dec + (size_t)m0 * dp + d0;
#pragma unroll
            for (int mm = 0; mm < MB; ++mm) {
#pragma unroll
                for (int dd = 0; dd < DC; ++dd) {
                    const C w = ldc(blk, (size_t)mm * dp + dd);
                    A[dd] = fma(x[mm].x, w.x, A[dd]);
                    B[dd] = fma(x[mm].y, w.y, B[dd]);
                }
            }
        }
#pragma unroll
        for (int dd = 0; dd < DC; ++dd) {
            const int d = d0 + dd;
            if (d <= dh) {
                out.add((A[dd] - B[dd]) * scale, d);
                if (d > 0 && 2 * d != nr) out.add((A[dd] + B[dd]) * scale, nr - d);
            }
        }
    }
}

// decode_px for at most MB bins and nr / 2 < MB degree pairs (one pass), with
// the pixel's bins already loaded (zero past the kept ones)
template <typename R, int MB>
__device__ __forceinline__ void decode_px_regs(const typename Cx<R>::T (&x)[MB], const typename Cx<R>::T *dec,
                                               int dp, int nr, R scale, PxDecode<R> &out) {
    using C = typename Cx<R>::T;
    const int dh = nr >> 1;
    out = PxDecode<R>();
    R A[MB], B[MB];
#pragma unroll
    for (int dd = 0; dd < MB; ++dd) A[dd] = B[dd] = 0;
#pragma unroll
    for (int mm = 0; mm < MB; ++mm) {
#pragma unroll
        for (int dd = 0; dd < MB; ++dd) {
            const C w = ldc(dec, (size_t)mm * dp + dd);
            A[dd] = fma(x[mm].x, w.x, A[dd]);
            B[dd] = fma(x[mm].y, w.y, B[dd]);
        }
    }
#pragma unroll
    for (int d = 0; d < MB; ++d) {
        if (d <= dh) {
            out.add((A[d] - B[d]) * scale, d);
            if (d > 0 && 2 * d != nr) out.add((A[d] + B[d]) * scale, nr - d);
        }
    }
}

// Decode variants by kept-bin count: one register pass for bins <= 4, <= 8,
// <= 12 and (FP32) <= 24; else blocks of 16 x 16 (FP32) or 8 x 8 (FP64).
enum : int { kDec8 = 0, kDec12 = 1, kDec24 = 2, kDecBlk = 3, kDec4 = 4 };

__host__ __device__ constexpr int decode_variant(int bins, int dbl) {
    return bins <= 4 ? kDec4 : bins <= 8 ? kDec8 : bins <= 12 ? kDec12 : (bins <= 24 && !dbl) ? kDec24 : kDecBlk;
}

template <typename R, int V>
__device__ __forceinline__ void decode_var(const typename Cx<R>::T *X, size_t mstride, size_t p, bool valid,
                                           const typename Cx<R>::T *dec, int dp, int nr, int bins, R scale,
                                           PxDecode<R> &out) {
    if constexpr (V == kDec4) decode_px<R, 4, 4>(X, mstride, p, valid, dec, dp, nr, bins, scale, out);
    else if constexpr (V == kDec8) decode_px<R, 8, 8>(X, mstride, p, valid, dec, dp, nr, bins, scale, out);
    else if constexpr (V == kDec12) decode_px<R, 12, 12>(X, mstride, p, valid, dec, dp, nr, bins, scale, out);
    else if constexpr (V == kDec24) decode_px<R, 24, 24>(X, mstride, p, valid, dec, dp, nr, bins, scale, out);
    else if constexpr (sizeof(R) == 4) decode_px<R, 16, 16>(X, mstride, p, valid, dec, dp, nr, bins, scale, out);
    else decode_px<R, 8, 8>(X, mstride, p, valid, dec, dp, nr, bins, scale, out);
}

// Sends a flagged tile to the next exact tier, once: FP32 jobs to the FP64
// recompute (fb_list), FP64 jobs to the exact window (win_list).
__device__ __forceinline__ void flag_tile(const JobDev &J, int job, int tile, unsigned int *tile_flags, int2 *fb_list,
                                          int2 *win_list, StatsDev *st) {
    const unsigned bit = J.fb_mode == kFbFFT64 ? kFlagFp64 : kFlagWindow;
    if (atomicOr(&tile_flags[J.flag0 + tile], bit) != 0u) return;
    if (bit == kFlagFp64) fb_list[atomicAdd(&st->fb_count, 1u)] = make_int2(job, tile);
    else win_list[atomicAdd(&st->win_count, 1u)] = make_int2(job, tile);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide max of a float (kDecThreads threads); result valid in thread 0.
__device__ __forceinline__ float block_max(float v, float *sh) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = sh[0];
#pragma unroll
    for (int q = 1; q < kDecThreads / 64; ++q) r = fmaxf(r, sh[q]);
    __syncthreads();
    return r;
}

template <typename R, int V>
__global__ __launch_bounds__(kDecThreads) void k_decode(const JobDev *__restrict__ jobs,
                                                        const Seg *__restrict__ segs, int nseg,
                                                        long long nitems, float band,
                                                        unsigned int *tile_flags, int2 *fb_list,
                                                        int2 *win_list, StatsDev *st,
                                                        const uint8_t *__restrict__ perturb) {
    using C = typename Cx<R>::T;
    __shared__ float s_red[kDecThreads / 64];
    float run_max = 0.f;          // largest residual this thread has seen (stats)
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0);
        const int tl = local / S.pblocks, pb = local - tl * S.pblocks;
        const int tile = S.tile0 + tl;
        const int T = J.T;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const size_t TT = (size_t)T * T;
        const C *X = (const C *)S.y + (size_t)tl * ytile_elems(J.bins, T, J.ybs);
        const size_t mstride = J.ybs ? 16 : TT;   // between bins of one pixel
        bool hit = false;
        if constexpr (V == kDec4 || V == kDec8) {
            // at most 4 or 8 bins: the bins of all kDecPixPerThread pixels
            // are loaded together (their loads in flight at once)
            constexpr int MB = V == kDec4 ? 4 : 8;
            C xs[kDecPixPerThread][MB];
            int gys[kDecPixPerThread], gxs[kDecPixPerThread];
            bool vals[kDecPixPerThread];
            unroll_c<kDecPixPerThread>([&](auto qq) {
                constexpr int Q = decltype(qq)::value;
                const int p = (pb * kDecPixPerThread + Q) * kDecThreads + threadIdx.x;
                const int ly = p / T, lx = p - ly * T;
                gys[Q] = ty * T + ly;
                gxs[Q] = tx * T + lx;
                vals[Q] = p < (int)TT && gys[Q] < J.H && gxs[Q] < J.W;
                const size_t b0 = ypix(vals[Q] ? p : 0, J.ybs);
                unroll_c<MB>([&](auto mq) {
                    constexpr int MM = decltype(mq)::value;
                    xs[Q][MM] = czero<C>();
                    if (vals[Q] && MM < J.bins) {
                        if (MM == 0 && J.dc_dec)   // bin 0 in closed form; the transforms left it unwritten
                            xs[Q][0] = dc_plane_value<R>(J, J.nt, gys[Q], gxs[Q],
                                                         perturb_bump<R>(perturb, J, tile, 0, kPerturbFirst));
                        else
                            xs[Q][MM] = ldg(X, (size_t)MM * mstride + b0);
                    }
                });
            });
            unroll_c<kDecPixPerThread>([&](auto qq) {
                constexpr int Q = decltype(qq)::value;
                PxDecode<R> dd;
                decode_px_regs<R, MB>(xs[Q], (const C *)J.dec, J.dec_pitch, J.nr, (R)J.scale, dd);
                if (vals[Q]) {
                    const int d = dd.top < 0 ? 0 : dd.top;
                    gst(J.out)[(size_t)gys[Q] * J.W + gxs[Q]] = J.op ? (J.L - 1 - d) : d;
                    run_max = fmaxf(run_max, (float)dd.res);
                    hit |= px_ambiguous(dd, band, J, gys[Q], gxs[Q]);
                }
            });
        } else {
        // kDecPixPerThread pixels per thread per item amortise the item setup
#pragma unroll 1
        for (int q = 0; q < kDecPixPerThread; ++q) {
            const int p = (pb * kDecPixPerThread + q) * kDecThreads + threadIdx.x;
            const int ly = p / T, lx = p - ly * T;
            const int gy = ty * T + ly, gx = tx * T + lx;
            const bool valid = p < (int)TT && gy < J.H && gx < J.W;
            PxDecode<R> dd;
            decode_var<R, V>(X, mstride, ypix(p, J.ybs), valid, (const C *)J.dec, J.dec_pitch, J.nr, J.bins,
                             (R)J.scale, dd);
            if (valid) {
                const int d = dd.top < 0 ? 0 : dd.top;
                gst(J.out)[(size_t)gy * J.W + gx] = J.op ? (J.L - 1 - d) : d;
                run_max = fmaxf(run_max, (float)dd.res);
                hit |= px_ambiguous(dd, band, J, gy, gx);
            }
        }
        }
        // a wave whose pixels fail a check flags the tile (rare); no barrier
        if (__any(hit) && (threadIdx.x & 63) == 0) flag_tile(J, S.job, tile, tile_flags, fb_list, win_list, st);
    }
    const float rm = block_max(run_max, s_red);
    if (threadIdx.x == 0 && rm > 0.f) atomicMax(&st->max_res_bits, __float_as_uint(rm));
}

// cos(2 pi q / 16) for q in [0, 8]
__host__ __device__ constexpr double cos16q(int q) {   // q in [0, 4]: 0 .. 90 degrees
    return q == 0 ? 1.0 : q == 1 ? 0.92387953251128675613 : q == 2 ? 0.70710678118654752440
         : q == 3 ? 0.38268343236508977173 : 0.0;
}
// (not recursive, so that every call inlines and folds to a constant)
__host__ __device__ constexpr double cos16(int q) { return q <= 4 ? cos16q(q) : -cos16q(8 - q); }
__host__ __device__ constexpr double sin16(int q) { return cos16(q <= 4 ? 4 - q : q - 4); }

// DFT of N <= 16 points held in registers, positive exponent,
// y_s = sum_r v_r exp(2 pi i r s / N), natural order in and out: radix-2
// decimation in time after a bit reversal that full unrolling turns into
// register renaming.
template <typename R, int N, typename C>
__device__ __forceinline__ void reg_dft(C (&v)[N]) {
    constexpr int LN = N == 2 ? 1 : N == 4 ? 2 : N == 8 ? 3 : 4;
    static_assert((1 << LN) == N, "N must be 2, 4, 8 or 16");
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int j = brevc(i, LN);
        if (i < j) {
            const C t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int h = 1; h < N; h *= 2) {
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += 2 * h) {
#pragma unroll
            for (int t = 0; t < h; ++t) {
                const int q = t * (8 / h);   // exp(2 pi i t / 2h) = exp(2 pi i q / 16)
                const C x0 = v[i0 + t], x1 = v[i0 + t + h];
                C y;
                if (q == 0) {
                    y = x1;
                } else if (q == 4) {
                    y.x = -x1.y;
                    y.y = x1.x;
                } else {
                    const R c = (R)cos16(q), s = (R)sin16(q);
                    y.x = c * x1.x - s * x1.y;
                    y.y = c * x1.y + s * x1.x;
                }
                v[i0 + t] = cadd(x0, y);
                v[i0 + t + h] = csub(x0, y);
            }
        }
    }
}

// cos(2 pi m / 24) and sin(2 pi m / 24) for any m >= 0
__host__ __device__ constexpr double cos24q(int m) {   // m in [0, 6]: 0 .. 90 degrees
    return m == 0 ? 1.0
         : m == 1 ? 0.96592582628906828675
         : m == 2 ? 0.86602540378443864676
         : m == 3 ? 0.70710678118654752440
         : m == 4 ? 0.5
         : m == 5 ? 0.25881904510252076235
                  : 0.0;
}
__host__ __device__ constexpr double cos24(int m) {   // not recursive: inlines to a constant
    return (m % 24) <= 6 ? cos24q(m % 24) : (m % 24) <= 12 ? -cos24q(12 - m % 24)
         : (m % 24) <= 18 ? -cos24q(m % 24 - 12) : cos24q(24 - m % 24);
}
__host__ __device__ constexpr double sin24(int m) { return cos24(m % 24 + 18); }

// DFT of 24 points in registers, positive exponent, natural order: for
// r = 3 r2 + r1 and s = s1 + 8 s2, three 8-point DFTs over r2, turns
// exp(2 pi i r1 s1 / 24), then eight 3-point DFTs over r1.
template <typename R, typename C>
__device__ __forceinline__ void reg_dft24(C (&v)[24]) {
    C a[3][8];
#pragma unroll
    for (int r1 = 0; r1 < 3; ++r1) {
#pragma unroll
        for (int r2 = 0; r2 < 8; ++r2) a[r1][r2] = v[3 * r2 + r1];
        reg_dft<R, 8>(a[r1]);
#pragma unroll
        for (int s1 = 1; s1 < 8; ++s1)
            if (r1 > 0) {
                const R c = (R)cos24(r1 * s1), sn = (R)sin24(r1 * s1);
                const C x = a[r1][s1];
                a[r1][s1].x = c * x.x - sn * x.y;
                a[r1][s1].y = c * x.y + sn * x.x;
            }
    }
    const R h = (R)0.86602540378443864676;   // sin(2 pi / 3)
#pragma unroll
    for (int s1 = 0; s1 < 8; ++s1) {
        const C a0 = a[0][s1], t = cadd(a[1][s1], a[2][s1]), u = csub(a[1][s1], a[2][s1]);
        C w;
        w.x = a0.x - (R)0.5 * t.x;
        w.y = a0.y - (R)0.5 * t.y;
        C iu;   // i sin(2 pi / 3) (a1 - a2)
        iu.x = -h * u.y;
        iu.y = h * u.x;
        v[s1] = cadd(a0, t);
        v[s1 + 8] = cadd(w, iu);
        v[s1 + 16] = csub(w, iu);
    }
}

// cos(2 pi m / 20) and sin(2 pi m / 20) for any m >= 0
__host__ __device__ constexpr double cos20q(int m) {   // m in [0, 5]: 0 .. 90 degrees
    return m == 0 ? 1.0
         : m == 1 ? 0.95105651629515357212
         : m == 2 ? 0.80901699437494742410
         : m == 3 ? 0.58778525229247312917
         : m == 4 ? 0.30901699437494742410
                  : 0.0;
}
__host__ __device__ constexpr double cos20(int m) {   // not recursive: inlines to a constant
    return (m % 20) <= 5 ? cos20q(m % 20) : (m % 20) <= 10 ? -cos20q(10 - m % 20)
         : (m % 20) <= 15 ? -cos20q(m % 20 - 10) : cos20q(20 - m % 20);
}
__host__ __device__ constexpr double sin20(int m) { return cos20(m % 20 + 15); }

// DFT of 20 points in registers, positive exponent, natural order: for
// r = 5 r2 + r1 and s = s1 + 4 s2, five 4-point DFTs over r2, turns
// exp(2 pi i r1 s1 / 20), then four 5-point DFTs over r1 (sums and
// differences of the conjugate pairs r1 = 1, 4 and 2, 3).
template <typename R, typename C>
__device__ __forceinline__ void reg_dft20(C (&v)[20]) {
    C a[5][4];
#pragma unroll
    for (int r1 = 0; r1 < 5; ++r1) {
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2) a[r1][r2] = v[5 * r2 + r1];
        reg_dft<R, 4>(a[r1]);
#pragma unroll
        for (int s1 = 1; s1 < 4; ++s1)
            if (r1 > 0) {
                const R c = (R)cos20(r1 * s1), sn = (R)sin20(r1 * s1);
                const C x = a[r1][s1];
                a[r1][s1].x = c * x.x - sn * x.y;
                a[r1][s1].y = c * x.y + sn * x.x;
            }
    }
    const R c1 = (R)cos20(4), c2 = (R)cos20(8), s1 = (R)sin20(4), s2 = (R)sin20(8);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const C a0 = a[0][q], t1 = cadd(a[1][q], a[4][q]), t2 = cadd(a[2][q], a[3][q]);
        const C d1 = csub(a[1][q], a[4][q]), d2 = csub(a[2][q], a[3][q]);
        C b1, b2, e1, e2;
        b1.x = a0.x + c1 * t1.x + c2 * t2.x;
        b1.y = a0.y + c1 * t1.y + c2 * t2.y;
        b2.x = a0.x + c2 * t1.x + c1 * t2.x;
        b2.y = a0.y + c2 * t1.y + c1 * t2.y;
        e1.x = s1 * d1.x + s2 * d2.x;   // e1 = s1 d1 + s2 d2, e2 = s2 d1 - s1 d2
        e1.y = s1 * d1.y + s2 * d2.y;
        e2.x = s2 * d1.x - s1 * d2.x;
        e2.y = s2 * d1.y - s1 * d2.y;
        v[q] = cadd(a0, cadd(t1, t2));
        v[q + 4].x = b1.x - e1.y;   // b1 + i e1
        v[q + 4].y = b1.y + e1.x;
        v[q + 16].x = b1.x + e1.y;   // b1 - i e1
        v[q + 16].y = b1.y - e1.x;
        v[q + 8].x = b2.x - e2.y;   // b2 + i e2
        v[q + 8].y = b2.y + e2.x;
        v[q + 12].x = b2.x + e2.y;   // b2 - i e2
        v[q + 12].y = b2.y - e2.x;
    }
}

// Range-axis FFT decode: Step 3 for a range length nr = 2M with M = 2^a
// (32 to 2048) or, in FP32, M = 3 2^a (48 to 768) or 5 2^a (40 to 320).
// A pixel's coefficient vector is the real inverse DFT of its Hermitian
// spectrum, of which the bins X_0 .. X_M are kept:
//   c_d = scale * sum_{m < nr} X_m w^(d m),  w = exp(2 pi i / nr),  X_{nr-m} = conj(X_m).
// Its even and odd samples are one complex inverse DFT of length M:
//   Z_k = (X_k + conj(X_{M-k})) + i w^k (X_k - conj(X_{M-k})),  k < M,
//   z_n = sum_{k<M} Z_k exp(2 pi i k n / M),  c_{2n} = scale Re z_n,  c_{2n+1} = scale Im z_n,
// about 2.5 nr log2(nr) flops per pixel where the dense decode takes
// nr (nr/2 + 1) products.  Thread (p, g), p < P, g < G = M / E, holds E
// points of pixel p (E = 16 for M = 2^a, 24 for M = 3 2^a, 20 for
// M = 5 2^a) through Stockham autosort passes: each pass of radix Q takes
// butterflies j, reads the points j + r M / Q (r < Q), turns them by
// exp(2 pi i r k / (S Q)) with k = j mod S (S: the length already
// transformed), takes a Q-point DFT in registers and leaves point s at
// (j - k) Q + k + s S.  A work item is the P = 256 E / M pixels of one tile
// whose transform-domain values are stored in blocks of 16 pixels with the
// bins contiguous (JobDev::ybs, the only layout these jobs use).
//   1. a radix-E pass straight from the bins: thread g loads X_k and X_{M-k}
//      for k = g + r G, packs Z_k and needs no turn (S = 1);
//   2. one or two more passes (M = 2^a: radix G up to 256, else radix 16
//      then M / 256; M = 3 2^a: radix min(G, 8), then G / 8; M = 5 2^a:
//      radix min(G, 4), then G / 4), through LDS rows of P points with one row of
//      padding after every E, so that the strided writes of the first pass
//      fall in distinct banks;
//   3. the last pass leaves each thread's points z_n in registers in
//      increasing n: it rounds them, keeps the index of its last non-zero
//      degree, and the threads of a pixel combine theirs by shuffles and one
//      LDS maximum per wave.
// Every job of one launch has the same range length, so the M twiddles are
// staged in LDS once per block.
template <typename R, int M>
__global__ __launch_bounds__(kDecThreads) void k_decode_fft(const JobDev *__restrict__ jobs,
                                                            const Seg *__restrict__ segs, int nseg,
                                                            long long nitems, float band,
                                                            unsigned int *tile_flags, int2 *fb_list,
                                                            int2 *win_list, StatsDev *st) {
    using C = typename Cx<R>::T;
    constexpr bool POW2 = (M & (M - 1)) == 0;
    constexpr int E = POW2 ? 16 : M % 3 == 0 ? 24 : 20, Q1 = E, G = M / E, P = kDecThreads / G;
    constexpr int Q2 = POW2 ? (M >= 256 ? 16 : G) : E == 24 ? (G < 8 ? G : 8) : (G < 4 ? G : 4), Q3 = M / (Q1 * Q2);
    constexpr int B2 = E / Q2, B3 = E / Q3, W = Q1 + 1;
    static_assert(G >= 2 && G * P == kDecThreads && (P & (P - 1)) == 0 && Q1 * Q2 * Q3 == M && E % Q2 == 0 &&
                      E % Q3 == 0 && (POW2 || sizeof(R) == 4),
                  "pass plan");
    __shared__ C zs[(M + M / Q1) * P];   // point n of pixel p at (n + n / E) P + p
    __shared__ C tws[M];                 // exp(2 pi i m / nr), m < M
    __shared__ C tw2[Q3 == 1 ? M : 1];   // exp(2 pi i m / M) for a last second pass
    __shared__ int s_top[P], s_sum[P];
    __shared__ float s_red[kDecThreads / 64];
    const int p = threadIdx.x & (P - 1), g = threadIdx.x / P;
    auto turn = [&](C x, int m) {   // x exp(2 pi i m / nr), m < nr
        C w = tws[m % M];
        if (m >= M) {
            w.x = -w.x;
            w.y = -w.y;
        }
        return cmul(x, w);
    };
    // LDS offset of row j + j / E, j = g + b G; for M = 2^a, G / 16 is whole
    // or zero, so b only adds a compile-time step
    auto row_base = [&](int b) {
        const int j = g + b * G;
        return POW2 ? (g + g / Q1) * P + p + b * (G + G / Q1) * P : (j + j / Q1) * P + p;
    };
    float run_max = 0.f;
    if (blockIdx.x < nitems) {
        const C *tw = (const C *)jobs[segs[find_seg(segs, nseg, blockIdx.x)].job].rtw;
        for (int m = threadIdx.x; m < M; m += kDecThreads) tws[m] = ldg(tw, m);
        if constexpr (Q3 == 1)
            for (int m = threadIdx.x; m < M; m += kDecThreads) {
                C w = ldg(tw, (2 * m) % M);
                if (2 * m >= M) {
                    w.x = -w.x;
                    w.y = -w.y;
                }
                tw2[m] = w;
            }
    }
    __syncthreads();
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0);
        const int tl = local / S.pblocks, pb = local - tl * S.pblocks;
        const int tile = S.tile0 + tl;
        const int T = J.T, TT = T * T;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const C *X = (const C *)S.y + (size_t)tl * ytile_elems(J.bins, T, J.ybs);
        const int p0 = pb * P;
        auto pixel_valid = [&](int pp) {
            const int q = p0 + pp, ly = q / T, lx = q - ly * T;
            return q < TT && ty * T + ly < J.H && tx * T + lx < J.W;
        };
        // 1. radix-E pass from the bins
        const bool pv = pixel_valid(p);
        C v[E];
        {
            // X_k and X_{M-k} (M - k = G - g + (E - 1 - r) G) through a buffer
            // resource over the item's 16-pixel blocks: one address register
            // per operand, the bin steps as uniform offsets.  A pixel outside
            // the image reads the bins of the item's first pixel (always
            // stored) and its results are dropped.
            C a[E], b[E];
            const int pl = pv ? p : 0;
            const int e0 = p0 & 15, blk = (e0 + pl) >> 4, pin = (p0 + pl) & 15;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(X + (size_t)(p0 >> 4) * J.ybs), (short)0,
                (int)((unsigned)((e0 + P + 15) >> 4) * J.ybs * sizeof(C)), kBufWord3);
            const unsigned va = (unsigned)(blk * J.ybs + pin + 16 * g) * sizeof(C);
            const unsigned vb = (unsigned)(blk * J.ybs + pin + 16 * (G - g)) * sizeof(C);
#pragma unroll
            for (int r = 0; r < E; ++r) {
                a[r] = buf_load<C>(rs, va, 16 * r * G * sizeof(C));
                b[r] = buf_load<C>(rs, vb, 16 * (E - 1 - r) * G * sizeof(C));
            }
#pragma unroll
            for (int r = 0; r < E; ++r) {
                // Z_k from (x, y) = (X_k, X_{M-k}): (x + conj y) + i w^k (x - conj y)
                const C x = a[r], y = b[r], w = tws[g + r * G];
                const R ox = x.x - y.x, oy = x.y + y.y;
                const R wx = w.x * ox - w.y * oy, wy = w.x * oy + w.y * ox;
                v[r].x = x.x + y.x - wy;
                v[r].y = x.y - y.y + wx;
            }
        }
        if constexpr (POW2) reg_dft<R, 16>(v);
        else if constexpr (E == 24) reg_dft24<R>(v);
        else reg_dft20<R>(v);
        const int base1 = W * g * P + p;   // rows E g + s
#pragma unroll
        for (int s = 0; s < E; ++s) zs[base1 + s * P] = v[s];
        if (threadIdx.x < P) {
            s_top[threadIdx.x] = -1;
            s_sum[threadIdx.x] = 0;
        }
        __syncthreads();
        // 2. the remaining passes (S = E, then E Q2)
        C u[B2][Q2];
#pragma unroll
        for (int b = 0; b < B2; ++b) {
            const int j = g + b * G, k = j % Q1, rb = row_base(b);   // rows j + r E Q3
#pragma unroll
            for (int r = 0; r < Q2; ++r) {
                const C x = zs[rb + r * Q3 * W * P];
                u[b][r] = r == 0 ? x : Q3 == 1 ? cmul(x, tw2[r * k]) : turn(x, r * k * (2 * M / (Q1 * Q2)));
            }
            reg_dft<R, Q2>(u[b]);
        }
        C w3[B3][Q3];
        if constexpr (Q3 > 1) {
            __syncthreads();   // every read of the first rows is done
#pragma unroll
            for (int b = 0; b < B2; ++b) {
                const int j = g + b * G, k = j % Q1, wb = ((j - k) / Q1 * Q2 * W + k) * P + p;
#pragma unroll
                for (int s = 0; s < Q2; ++s) zs[wb + s * W * P] = u[b][s];   // rows (j - k) Q2 + k + s E
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < B3; ++b) {
                const int j = g + b * G, rb = row_base(b);   // rows j + r E Q2
#pragma unroll
                for (int r = 0; r < Q3; ++r) {
                    const C x = zs[rb + r * Q2 * W * P];
                    w3[b][r] = r == 0 ? x : turn(x, 2 * r * j);   // exp(2 pi i r j / M)
                }
                reg_dft<R, Q3>(w3[b]);
            }
        }
        // 3. round every degree held in registers, in increasing degree
        // order (point n = g + b G + NS s), keeping the index of the last
        // non-zero one
        constexpr int NB = Q3 > 1 ? B3 : B2, NSP = Q3 > 1 ? Q3 : Q2, NS = Q3 > 1 ? Q1 * Q2 : Q1;
        // (with the exactness checks' inputs: residual, negative coefficients,
        // and the sum of the rounded coefficients)
        const R scale = (R)J.scale;
        int topi = -1;
        R res = 0, rsum = 0;
        bool neg = false;
#pragma unroll
        for (int s = 0; s < NSP; ++s)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const C z = Q3 > 1 ? w3[b][s] : u[b][s];
                const int i = 2 * (s * NB + b);
                const R cx = z.x * scale, cy = z.y * scale, rx = rint(cx), ry = rint(cy);
                res = fmax(res, fmax(fabs(cx - rx), fabs(cy - ry)));
                rsum += rx + ry;
                neg |= (rx < R(0)) | (ry < R(0));
                if (rx != R(0)) topi = i;
                if (ry != R(0)) topi = i + 1;
            }
        if (!pv) {
            topi = -1;
            res = 0;
            rsum = 0;
            neg = false;
        }
        int top = -1, isum = (int)rsum;
        if (topi >= 0) {
            const int q = topi >> 1, s = q / NB, b = q - s * NB;
            top = 2 * (g + b * G + NS * s) + (topi & 1);
        }
#pragma unroll
        for (int o = 32; o >= P; o >>= 1) {
            top = max(top, __shfl_xor(top, o, 64));
            isum += __shfl_xor(isum, o, 64);
        }
        if ((threadIdx.x & 63) < P) {
            if (top >= 0) atomicMax(&s_top[p], top);
            atomicAdd(&s_sum[p], isum);
        }
        run_max = fmaxf(run_max, (float)res);
        bool hit = (float)res >= band || neg;
        __syncthreads();
        if (threadIdx.x < P && pixel_valid(threadIdx.x)) {
            const int q = p0 + threadIdx.x, ly = q / T, lx = q - ly * T;
            const int gy = ty * T + ly, gx = tx * T + lx;
            const int d = s_top[threadIdx.x] < 0 ? 0 : s_top[threadIdx.x];
            gst(J.out)[(size_t)gy * J.W + gx] = J.op ? (J.L - 1 - d) : d;
            hit |= s_sum[threadIdx.x] != window_cells(J, gy, gx);
        }
        // a wave whose pixels fail a check flags the tile (rare)
        if (__any(hit) && (threadIdx.x & 63) == 0) flag_tile(J, S.job, tile, tile_flags, fb_list, win_list, st);
        __syncthreads();   // the rows and tops are rewritten by the next item
    }
    const float rm = block_max(run_max, s_red);
    if (threadIdx.x == 0 && rm > 0.f) atomicMax(&st->max_res_bits, __float_as_uint(rm));
}

// DFT with positive exponent of M = 2^a 3^b 5^c points in registers,
// natural order in and out: y_s = sum_r v_r exp(+2 pi i r s / M).  Mixed
// radix, decimation in time on the smallest factor, compile-time twiddles.
template <typename R, int M, typename C>
__device__ __forceinline__ void reg_idft(C (&v)[M]) {
    if constexpr (M == 2) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (M == 3) {
        const R h = (R)0.86602540378443864676;   // sin(2 pi / 3)
        const C a0 = v[0], t = cadd(v[1], v[2]), u = csub(v[1], v[2]);
        C w;
        w.x = a0.x - (R)0.5 * t.x;
        w.y = a0.y - (R)0.5 * t.y;
        v[0] = cadd(a0, t);
        v[1].x = w.x - h * u.y;   // w + i sin(2 pi / 3) (a1 - a2)
        v[1].y = w.y + h * u.x;
        v[2].x = w.x + h * u.y;
        v[2].y = w.y - h * u.x;
    } else if constexpr (M == 5) {
        const R c1 = (R)cos2pi(1, 5), c2 = (R)cos2pi(2, 5), s1 = (R)sin2pi(1, 5), s2 = (R)sin2pi(2, 5);
        const C a0 = v[0], t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        const C d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
        C b1, b2, e1, e2;
        b1.x = a0.x + c1 * t1.x + c2 * t2.x;
        b1.y = a0.y + c1 * t1.y + c2 * t2.y;
        b2.x = a0.x + c2 * t1.x + c1 * t2.x;
        b2.y = a0.y + c2 * t1.y + c1 * t2.y;
        e1.x = s1 * d1.x + s2 * d2.x;
        e1.y = s1 * d1.y + s2 * d2.y;
        e2.x = s2 * d1.x - s1 * d2.x;
        e2.y = s2 * d1.y - s1 * d2.y;
        v[0] = cadd(a0, cadd(t1, t2));
        v[1].x = b1.x - e1.y;   // b1 + i e1
        v[1].y = b1.y + e1.x;
        v[4].x = b1.x + e1.y;   // b1 - i e1
        v[4].y = b1.y - e1.x;
        v[2].x = b2.x - e2.y;   // b2 + i e2
        v[2].y = b2.y + e2.x;
        v[3].x = b2.x + e2.y;   // b2 - i e2
        v[3].y = b2.y - e2.x;
    } else {
        // outer factor: for M = 2^a 3^b 5^c with b + c > 0, 8 or 4 where they
        // divide M (fewer general turns than a radix-2 split: the turns by
        // multiples of M / 8 are eighth turns); powers of two split by 2
        constexpr bool POW2 = (M & (M - 1)) == 0;
        constexpr int P = !POW2 && M % 8 == 0 ? 8 : !POW2 && M % 4 == 0 ? 4 : M % 2 == 0 ? 2 : M % 3 == 0 ? 3 : 5,
                      Q = M / P;
        static_assert(P * Q == M && Q > 1, "M must factor into 2, 3 and 5");
        C a[P][Q];
        unroll_c<P>([&](auto r) {
            constexpr int RR = decltype(r)::value;
            unroll_c<Q>([&](auto j) {
                constexpr int JJ = decltype(j)::value;
                a[RR][JJ] = v[P * JJ + RR];
            });
            reg_idft<R, Q>(a[RR]);
            unroll_c<Q>([&](auto s) {
                constexpr int SS = decltype(s)::value;
                a[RR][SS] = twc<R, RR * SS, M, true, false>(a[RR][SS]);
            });
        });
        unroll_c<Q>([&](auto s) {
            constexpr int SS = decltype(s)::value;
            C b[P];
            unroll_c<P>([&](auto r) { b[decltype(r)::value] = a[decltype(r)::value][SS]; });
            reg_idft<R, P>(b);
            unroll_c<P>([&](auto t) { v[SS + Q * decltype(t)::value] = b[decltype(t)::value]; });
        });
    }
}

// Range-axis FFT decode for short range lengths nr = 2M, M from 4 to 45 in
// FP32 (to 24 in FP64) with no prime factor above 5, except 32: one pixel per
// thread, all of it in registers.
// The thread loads the pixel's bins X_0 .. X_M (16-pixel blocks, bins
// contiguous), packs
// Z_k = (X_k + conj X_{M-k}) + i w^k (X_k - conj X_{M-k}),
// w = exp(2 pi i / nr), takes the M-point inverse DFT z and reads
// c_{2n} = scale Re z_n, c_{2n+1} = scale Im z_n (the even and odd samples of
// the real inverse DFT of the Hermitian spectrum), then Step 3 and the
// exactness checks as the other decodes.  kDecSmallPix pixels of a tile per
// work item.
template <typename R, int M>
__global__ __launch_bounds__(kDecThreads) void k_decode_small(const JobDev *__restrict__ jobs,
                                                              const Seg *__restrict__ segs, int nseg,
                                                              long long nitems, float band,
                                                              unsigned int *tile_flags, int2 *fb_list,
                                                              int2 *win_list, StatsDev *st,
                                                              const uint8_t *__restrict__ perturb) {
    using C = typename Cx<R>::T;
    constexpr int PPT = kDecSmallPix / kDecThreads;   // pixels per thread per item
    __shared__ float s_red[kDecThreads / 64];
    float run_max = 0.f;
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0);
        const int tl = local / S.pblocks, pb = local - tl * S.pblocks;
        const int tile = S.tile0 + tl;
        const int T = J.T, TT = T * T;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const C *X = (const C *)S.y + (size_t)tl * ytile_elems(J.bins, T, J.ybs);
        const R scale = (R)J.scale;
        bool hit = false;
        // the bins of PF pixels are loaded together (their loads in flight at
        // once), as many as keep the loaded values within about 96 registers
        constexpr int PF = (M + 1) * (int)sizeof(C) / 4 * PPT <= 96 ? PPT : 1;
#pragma unroll 1
        for (int q0 = 0; q0 < PPT; q0 += PF) {
            int gy[PF], gx[PF], wc[PF];
            bool valid[PF];
            C x[PF][M + 1];
            unroll_c<PF>([&](auto qq) {
                constexpr int Q = decltype(qq)::value;
                const int p = (pb * PPT + q0 + Q) * kDecThreads + threadIdx.x;
                const int ly = p / T, lx = p - ly * T;
                gy[Q] = ty * T + ly;
                gx[Q] = tx * T + lx;
                valid[Q] = p < TT && gy[Q] < J.H && gx[Q] < J.W;
                const size_t b0 = ypix(valid[Q] ? p : 0, J.ybs);
                // bin 0 in closed form for dc_dec jobs (the transforms left
                // its plane unwritten); the count also serves the DC check
                wc[Q] = valid[Q] ? window_cells(J, gy[Q], gx[Q]) : 0;
                unroll_c<M + 1>([&](auto m) {
                    constexpr int MM = decltype(m)::value;
                    if (MM == 0 && J.dc_dec) {
                        x[Q][0].x = (R)((double)J.nt * J.nt) * (R)wc[Q] +
                                    perturb_bump<R>(perturb, J, tile, 0, kPerturbFirst);
                        x[Q][0].y = R(0);
                    } else {
                        x[Q][MM] = ldg(X, b0 + 16 * MM);
                    }
                });
            });
            unroll_c<PF>([&](auto qq) {
                constexpr int Q = decltype(qq)::value;
                C z[M];
                unroll_c<M>([&](auto kk) {
                    constexpr int K = decltype(kk)::value;
                    const C a = x[Q][K], b = x[Q][M - K];
                    C d;
                    d.x = a.x - b.x;
                    d.y = a.y + b.y;
                    const C t = twc<R, K, 2 * M, true, false>(d);   // w^k (x - conj y)
                    z[K].x = a.x + b.x - t.y;
                    z[K].y = a.y - b.y + t.x;
                });
                reg_idft<R, M>(z);
                PxDecode<R> dd;
                unroll_c<M>([&](auto n) {
                    constexpr int NN = decltype(n)::value;
                    dd.add(z[NN].x * scale, 2 * NN);
                    dd.add(z[NN].y * scale, 2 * NN + 1);
                });
                if (valid[Q]) {
                    const int d = dd.top < 0 ? 0 : dd.top;
                    gst(J.out)[(size_t)gy[Q] * J.W + gx[Q]] = J.op ? (J.L - 1 - d) : d;
                    run_max = fmaxf(run_max, (float)dd.res);
                    hit |= (float)dd.res >= band || dd.neg || (int)dd.sum != wc[Q];   // px_ambiguous
                }
            });
        }
        if (__any(hit) && (threadIdx.x & 63) == 0) flag_tile(J, S.job, tile, tile_flags, fb_list, win_list, st);
    }
    const float rm = block_max(run_max, s_red);
    if (threadIdx.x == 0 && rm > 0.f) atomicMax(&st->max_res_bits, __float_as_uint(rm));
}

// ---------------------------------------------------------------------------
// Measured comparison: batched 16-point DFTs on the vector ALU and on the
// matrix cores
// ---------------------------------------------------------------------------
// The question is whether the fixed-radix DFT stages of the spatial
// transform would run faster as dense products on the matrix cores than as
// butterflies.  Three kernels apply `reps` forward 16-point DFTs in a row to
// each of `lines` lines held in registers (one load and one store per line,
// so that the arithmetic dominates):
//   variant 0: the in-register radix-2 DFT of k_fft_reg (split hi + lo FP32
//              constants), one line per lane;
//   variant 1: FP32 products on v_mfma_f32_16x16x4_f32: a wavefront holds 64
//              lines as four 16 x 16 (point x line) blocks, lane (j, q) with
//              the points 4q + s (s < 4) of line j of each block; one DFT is
//              Z = F X with F the 16 x 16 DFT matrix, as 4 K-steps of the real
//              products Fr Xr - Fi Xi and Fi Xr + Fr Xi, and its output comes
//              back in the same layout (row 4q + r of D in lane group q);
//   variant 2: the same product on v_mfma_f32_16x16x32_bf16 with both
//              operands split into bf16 hi + lo and three products
//              (hi hi + hi lo + lo hi, FP32 accumulation): one K = 32 step per
//              real output ([Fr | -Fi] and [Fi | Fr] against [Xr; Xi]).
// The layouts are taken from the data placement of each kernel, so neither
// pays for moving data between lanes; inside k_fft_reg an MFMA stage would
// also need that movement.  Test and measurement hook only.
typedef float f32x4m __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8m __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_dft16_valu(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                     long long lines, int reps) {
    const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= lines) return;
    float2 v[16];
    unroll_c<16>([&](auto e) { v[decltype(e)::value] = ldg(in, (size_t)line * 16 + decltype(e)::value); });
    for (int r = 0; r < reps; ++r) reg_fft<float, 16, false>(v);
    unroll_c<16>([&](auto e) { stg(out, (size_t)line * 16 + decltype(e)::value, v[decltype(e)::value]); });
}

// DFT matrix entry exp(-2 pi i a b / 16)
__device__ __forceinline__ float dft16_re(int a, int b) { return (float)cospi(-2.0 * ((a * b) & 15) / 16.0); }
__device__ __forceinline__ float dft16_im(int a, int b) { return (float)sinpi(-2.0 * ((a * b) & 15) / 16.0); }

__global__ __launch_bounds__(256) void k_dft16_mfma32(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                       long long lines, int reps) {
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const long long w0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x - lane);   // first line of the wave
    if (w0 >= lines) return;
    // A operand of K-step s: lane (i = j, k = q) holds F[i][4k + s]
    float are[4], aim[4], anim[4];
    for (int s = 0; s < 4; ++s) {
        are[s] = dft16_re(j, 4 * q + s);
        aim[s] = dft16_im(j, 4 * q + s);
        anim[s] = -aim[s];
    }
    f32x4m xr[4], xi[4];   // block b: points 4q + s of line w0 + 16 b + j
    for (int b = 0; b < 4; ++b)
        for (int s = 0; s < 4; ++s) {
            const float2 x = ldg(in, (size_t)(w0 + 16 * b + j) * 16 + 4 * q + s);
            xr[b][s] = x.x;
            xi[b][s] = x.y;
        }
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            f32x4m dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                dr = __builtin_amdgcn_mfma_f32_16x16x4f32(are[s], xr[b][s], dr, 0, 0, 0);
                dr = __builtin_amdgcn_mfma_f32_16x16x4f32(anim[s], xi[b][s], dr, 0, 0, 0);
                di = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[s], xr[b][s], di, 0, 0, 0);
                di = __builtin_amdgcn_mfma_f32_16x16x4f32(are[s], xi[b][s], di, 0, 0, 0);
            }
            xr[b] = dr;   // row 4q + s of the output in lane group q
            xi[b] = di;
        }
    }
    for (int b = 0; b < 4; ++b)
        for (int s = 0; s < 4; ++s)
            stg(out, (size_t)(w0 + 16 * b + j) * 16 + 4 * q + s, make_float2(xr[b][s], xi[b][s]));
}

__device__ __forceinline__ void bf16_split(float x, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

__global__ __launch_bounds__(256) void k_dft16_mfma_bf16x3(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                            long long lines, int reps) {
    const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
    const long long w0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x - lane);
    if (w0 >= lines) return;
    // A operands: lane (i = j, k = q) holds K = 8q + t, t < 8: t < 4 the
    // coefficient of Re x[4q + t], t >= 4 that of Im x[4q + t - 4]
    bf16x8m arh, arl, aih, ail;   // rows of Re z: [Fr | -Fi]; of Im z: [Fi | Fr]
    for (int t = 0; t < 8; ++t) {
        const int e = 4 * q + (t & 3);
        const float fr = dft16_re(j, e), fi = dft16_im(j, e);
        __bf16 h, l;
        bf16_split(t < 4 ? fr : -fi, h, l);
        arh[t] = h;
        arl[t] = l;
        bf16_split(t < 4 ? fi : fr, h, l);
        aih[t] = h;
        ail[t] = l;
    }
    f32x4m xr[4], xi[4];
    for (int b = 0; b < 4; ++b)
        for (int s = 0; s < 4; ++s) {
            const float2 x = ldg(in, (size_t)(w0 + 16 * b + j) * 16 + 4 * q + s);
            xr[b][s] = x.x;
            xi[b][s] = x.y;
        }
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            bf16x8m bh, bl;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                __bf16 h, l;
                bf16_split(xr[b][s], h, l);
                bh[s] = h;
                bl[s] = l;
                bf16_split(xi[b][s], h, l);
                bh[s + 4] = h;
                bl[s + 4] = l;
            }
            f32x4m dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
            dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bh, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bl, dr, 0, 0, 0);
            dr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bh, dr, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, bh, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bl, di, 0, 0, 0);
            di = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bh, di, 0, 0, 0);
            xr[b] = dr;
            xi[b] = di;
        }
    }
    for (int b = 0; b < 4; ++b)
        for (int s = 0; s < 4; ++s)
            stg(out, (size_t)(w0 + 16 * b + j) * 16 + 4 * q + s, make_float2(xr[b][s], xi[b][s]));
}

// Exact recompute of the tiles listed by the decode: FP64 transforms on
// nt64-sized sub-tiles (LDS-resident up to 64, through this block's slab
// beyond), each decoded from this block's slot.  The decode applies the
// exactness checks with kExactBand; a tile that fails them here too goes on
// to the exact window (win_list).
template <int N>
__global__ __launch_bounds__(kDecThreads) void k_fallback(const JobDev *__restrict__ jobs,
                                                          const int2 *__restrict__ fb_list, StatsDev *st,
                                                          double2 *slots, size_t slot_elems,
                                                          const double2 *__restrict__ tw64, double2 *slabs,
                                                          unsigned int *tile_flags, int2 *win_list,
                                                          const uint8_t *__restrict__ perturb) {
    constexpr bool BIG = N > kMaxLdsN64;
    __shared__ double2 lds[BIG ? big_lines<double, N>() * (N + 1) : N * (N + 1)];
    Tw64 tw;
    tw.p = tw64;
    const unsigned cnt = __builtin_amdgcn_readfirstlane(*(volatile const unsigned *)&st->fb_count);
    double2 *slot = slots + (size_t)blockIdx.x * slot_elems;
    double2 *slab = BIG ? slabs + (size_t)blockIdx.x * N * N : nullptr;
    for (unsigned i = blockIdx.x; i < cnt; i += gridDim.x) {
        const int2 e = fb_list[i];
        const JobDev &J = jobs[e.x];
        if (J.fb_mode != kFbFFT64 || J.nt64 != N) continue;
        const int tile = e.y;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const int oy0 = ty * J.T, ox0 = tx * J.T;
        const int oh = min(J.T, J.H - oy0), ow = min(J.T, J.W - ox0);
        const int T64 = J.T64;
        const size_t TT = (size_t)T64 * T64;
        // the test hook's bump, in the units of this pass (nt64, not nt)
        const double bump = perturb && (perturb[J.flag0 + tile] & kPerturbFp64) ? 0.4 * N * N * J.nr : 0.0;
        bool hit = false;
        for (int sy = 0; sy < oh; sy += T64) {
            for (int sx = 0; sx < ow; sx += T64) {
                for (int m = 0; m < J.bins; ++m) {
                    if constexpr (BIG)
                        fft_big_tile_bin<double, N, kDecThreads>(lds, slab, J.img, J.H, J.W, J.L, J.op, J.k, oy0 + sy,
                                                                 ox0 + sx, J.enc64 + (size_t)m * J.L,
                                                                 J.se_spec64 + (size_t)m * N * N, slot + m * TT, 0,
                                                                 tw, nullptr, m == 0 ? bump : 0.0);
                    else
                        fft_tile_bin<double, N, kDecThreads>(lds, J.img, J.H, J.W, J.L, J.op, J.k, oy0 + sy, ox0 + sx,
                                                             J.enc64 + (size_t)m * J.L, J.se_spec64 + (size_t)m * N * N,
                                                             slot + m * TT, 0, tw, nullptr, m == 0 ? bump : 0.0);
                }
                const int sh = min(T64, oh - sy), sw = min(T64, ow - sx);
                for (int p0 = 0; p0 < (int)TT; p0 += kDecThreads) {
                    const int p = p0 + threadIdx.x;
                    const int ly = p / T64, lx = p - ly * T64;
                    const bool valid = p < (int)TT && ly < sh && lx < sw;
                    PxDecode<double> dd;
                    switch (decode_variant(J.bins, 1)) {
                        case kDec4:
                        case kDec8:
                            decode_var<double, kDec8>(slot, TT, p, valid, J.dec64, J.dec_pitch, J.nr, J.bins, J.scale64,
                                                      dd);
                            break;
                        case kDec12:
                            decode_var<double, kDec12>(slot, TT, p, valid, J.dec64, J.dec_pitch, J.nr, J.bins,
                                                       J.scale64, dd);
                            break;
                        default:
                            decode_var<double, kDecBlk>(slot, TT, p, valid, J.dec64, J.dec_pitch, J.nr, J.bins,
                                                        J.scale64, dd);
                    }
                    if (valid) {
                        const int gy = oy0 + sy + ly, gx = ox0 + sx + lx;
                        const int d = dd.top < 0 ? 0 : dd.top;
                        gst(J.out)[(size_t)gy * J.W + gx] = J.op ? (J.L - 1 - d) : d;
                        hit |= px_ambiguous(dd, kExactBand, J, gy, gx);
                    }
                }
                __syncthreads();   // the slot is rewritten by the next sub-tile
            }
        }
        if (__syncthreads_or(hit) && threadIdx.x == 0) {
            atomicOr(&tile_flags[J.flag0 + tile], kFlagWindow);
            win_list[atomicAdd(&st->win_count, 1u)] = e;
        }
    }
}

// The exact tier behind both transform passes: the classical window
// max { f(x-y) + b(y) } (Eq. (6new)) in int32 over every pixel of the tiles
// on win_list, for tiles whose FP64 coefficients still failed the checks.
// The effective SE comes in correlation order (sek, row i / column j holds
// the offset of cell (k-1-i, k-1-j), kNeg where masked), so the pixel (y, x)
// takes the image pixel (y + i - r, x + j - r); erosion complements the
// image values and the result (duality, Sec. 2.1).  A work item is one block
// of kDecThreads pixels of a listed tile.
__global__ __launch_bounds__(kDecThreads) void k_tile_window(const JobDev *__restrict__ jobs,
                                                             const int2 *__restrict__ win_list,
                                                             const StatsDev *__restrict__ st, int pblocks) {
    const unsigned cnt = __builtin_amdgcn_readfirstlane(*(volatile const unsigned *)&st->win_count);
    const long long items = (long long)cnt * pblocks;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const int2 e = win_list[it / pblocks];
        const JobDev &J = jobs[e.x];
        const int T = J.T, q = (int)(it % pblocks) * kDecThreads + threadIdx.x;
        const int ty = e.y / J.tiles_x, tx = e.y - ty * J.tiles_x;
        const int gy = ty * T + q / T, gx = tx * T + q % T;
        if (q >= T * T || gy >= J.H || gx >= J.W) continue;
        const int k = J.k, r = (k - 1) >> 1;
        const int i0 = max(0, r - gy), i1 = min(k, J.H - gy + r), j0 = max(0, r - gx), j1 = min(k, J.W - gx + r);
        const auto im = gld(J.img);
        int best = kNeg;
        for (int i = i0; i < i1; ++i) {
            const size_t row = (size_t)(gy + i - r) * J.W + (gx - r);
            const int32_t *srow = J.sek + (size_t)i * J.kpad;
            for (int j = j0; j < j1; ++j) {
                int v = min(max(im[row + j], 0), J.L - 1);
                v = J.op ? J.L - 1 - v : v;
                best = max(best, v + srow[j]);
            }
        }
        const int d = best < 0 ? 0 : best;
        gst(J.out)[(size_t)gy * J.W + gx] = J.op ? (J.L - 1 - d) : d;
    }
}

// ---------------------------------------------------------------------------
// tables (FP64 trigonometry; FP32 copies are rounded from it)
// ---------------------------------------------------------------------------
__global__ void k_twiddles(double2 *tw64, TwF *tw32) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kTwN) return;
    double s, c;
    sincospi(-2.0 * q / kTwN, &s, &c);
    tw64[q] = make_double2(c, s);
    TwF t;
    t.hi = make_float2((float)c, (float)s);
    t.lo = make_float2((float)(c - (double)t.hi.x), (float)(s - (double)t.hi.y));
    tw32[q] = t;
}

// enc[m][v] = exp(-2 pi i (v m mod nr) / nr): range-axis DFT of the one-hot
// column of grey value v (Eq. (7)).  dec[m][d] = w_m exp(+2 pi i (d m mod nr)
// / nr) for m, d < bins = nr/2+1 (w_m = 1 for m = 0 and m = nr/2, 2
// otherwise), zero-padded to dp x dp with dp = dec_pitch(nr): the inverse real
// DFT from the kept half of the bins (unscaled); degrees above nr/2 follow by
// symmetry in the decode.
__global__ void k_range_tables(int nr, int L, int bins, int dp, float2 *enc32, double2 *enc64, float2 *dec32,
                               double2 *dec64, float2 *rtw32, double2 *rtw64) {
    const long long ne = (long long)bins * L, nd = (long long)dp * dp, nw = nr / 2;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < ne + nd + nw;
         q += (long long)gridDim.x * blockDim.x) {
        double s, c;
        if (q >= ne + nd) {
            const long long m = q - ne - nd;
            sincospi(2.0 * (double)m / nr, &s, &c);
            rtw64[m] = make_double2(c, s);
            rtw32[m] = make_float2((float)c, (float)s);
        } else if (q < ne) {
            const long long m = q / L, v = q % L;
            const long long ph = (v * m) % nr;
            sincospi(-2.0 * (double)ph / nr, &s, &c);
            enc64[q] = make_double2(c, s);
            enc32[q] = make_float2((float)c, (float)s);
        } else {
            const long long e = q - ne;
            const long long m = e / dp, d = e % dp;
            double wc = 0, ws = 0;
            if (m < bins && d < bins) {
                const long long ph = (d * m) % nr;
                sincospi(2.0 * (double)ph / nr, &s, &c);
                const double wt = (m == 0 || 2 * m == nr) ? 1.0 : 2.0;
                wc = wt * c;
                ws = wt * s;
            }
            dec64[e] = make_double2(wc, ws);
            dec32[e] = make_float2((float)wc, (float)ws);
        }
    }
}

// Spectrum of the SE umbra (Eq. (8)) at spatial length nt, as a separable
// DFT in FP64: first along the SE columns for each of its k rows, then along
// the rows.  The umbra's value at cell (i, j), bin m, is
// exp(-2 pi i (b_ij m mod nr) / nr) on the mask and 0 off it.
__global__ void k_se_rows(const uint8_t *__restrict__ mask, const int32_t *__restrict__ off, int k, int nt,
                          int nr, const double2 *__restrict__ tw64, double2 *G) {
    const int m = blockIdx.x / k, i = blockIdx.x % k;
    const int step = kTwN / nt;
    for (int v = threadIdx.x; v < nt; v += blockDim.x) {
        double ax = 0, ay = 0;
        for (int j = 0; j < k; ++j) {
            if (!mask[i * k + j]) continue;
            const long long ph = ((long long)off[i * k + j] * m) % nr;
            double s, c;
            sincospi(-2.0 * (double)ph / nr, &s, &c);
            const double2 t = tw64[((v * j) % nt) * step];
            ax += c * t.x - s * t.y;
            ay += c * t.y + s * t.x;
        }
        G[((size_t)m * k + i) * nt + v] = make_double2(ax, ay);
    }
}

__global__ void k_se_cols(const double2 *__restrict__ G, int k, int nt, const double2 *__restrict__ tw64,
                          double2 *spec64, float2 *spec32) {
    const int m = blockIdx.x / nt, u = blockIdx.x % nt;
    const int step = kTwN / nt;
    for (int v = threadIdx.x; v < nt; v += blockDim.x) {
        double ax = 0, ay = 0;
        for (int i = 0; i < k; ++i) {
            const double2 g = G[((size_t)m * k + i) * nt + v];
            const double2 t = tw64[((u * i) % nt) * step];
            ax += g.x * t.x - g.y * t.y;
            ay += g.x * t.y + g.y * t.x;
        }
        const size_t o = ((size_t)m * nt + v) * nt + u;   // [m][kx][ky]
        if (spec64) spec64[o] = make_double2(ax, ay);
        if (spec32) spec32[o] = make_float2((float)ax, (float)ay);
    }
}

// Pseudo-random grey values in [0, L) from a 32-bit integer hash of the
// index (calibration images of the autotuner).
__global__ void k_fill_hash(int32_t *p, size_t n, int L, unsigned int seed) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        unsigned int h = (unsigned int)i * 0x9E3779B1u ^ seed;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        p[i] = (int32_t)(h % (unsigned int)L);
    }
}

// Elementwise steps of the compositions (grid-stride, one int32 per lane per
// step: these passes are bound by HBM and small next to the dilations).
__global__ void k_add_const(int32_t *out, const int32_t *in, int32_t c, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = in[i] + c;
}

__global__ void k_sub(int32_t *out, const int32_t *x, const int32_t *y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = x[i] - y[i];
}

__global__ void k_zero(uint32_t *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_or_flag(uint32_t *dst, const uint32_t *src) {
    if (threadIdx.x == 0) dst[0] |= src[0];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int fft_block_threads(int nt, int dbl) {
    if (nt > (dbl ? kMaxLdsN64 : kMaxLdsN32)) return nt <= kMaxN ? kBigThreads : 0;
    // k_fft_reg: four or eight lanes per line of the tile
    switch (nt) {
        case 16: case 32: case 64: case 128: return fft_reg_lanes(nt, dbl) * nt;
        default: return 0;
    }
}

size_t fft_lds_bytes(int nt, int dbl) {
    const size_t esz = dbl ? sizeof(double2) : sizeof(float2);
    if (nt > (dbl ? kMaxLdsN64 : kMaxLdsN32)) return (size_t)big_lines_of(nt, dbl) * (nt + 1) * esz;
    // k_fft_reg: the tile, the grey-value cache and (FP32 from 64 points) the
    // lane-twiddle table
    const size_t pitch = fft_reg_lanes(nt, dbl) == 8 ? nt + 4 : nt + 1;
    return (size_t)nt * pitch * esz + (size_t)nt * (nt + 4) + (!dbl && nt >= 64 ? (size_t)nt * sizeof(TwF) : 16);
}

hipError_t launch_add_const(int32_t *out, const int32_t *in, int32_t c, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    k_add_const<<<grid, 256, 0, s>>>(out, in, c, n);
    return hipGetLastError();
}

hipError_t launch_sub(int32_t *out, const int32_t *x, const int32_t *y, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 4096);
    k_sub<<<grid, 256, 0, s>>>(out, x, y, n);
    return hipGetLastError();
}

hipError_t launch_twiddles(double2 *tw64, TwF *tw32, hipStream_t s) {
    k_twiddles<<<(kTwN + 255) / 256, 256, 0, s>>>(tw64, tw32);
    return hipGetLastError();
}

hipError_t launch_range_tables(int nr, int L, float2 *enc32, double2 *enc64, float2 *dec32, double2 *dec64,
                               float2 *rtw32, double2 *rtw64, hipStream_t s) {
    const int bins = nr / 2 + 1, dp = dec_pitch(nr);
    const long long n = (long long)bins * L + (long long)dp * dp + nr / 2;
    const int grid = (int)std::min<long long>((n + 255) / 256, 4096);
    k_range_tables<<<grid, 256, 0, s>>>(nr, L, bins, dp, enc32, enc64, dec32, dec64, rtw32, rtw64);
    return hipGetLastError();
}

hipError_t launch_se_spectrum(const uint8_t *mask_d, const int32_t *off_d, int k, int nt, int nr,
                              const double2 *tw64, double2 *work, double2 *spec64, float2 *spec32,
                              hipStream_t s) {
    const int bins = nr / 2 + 1;
    const int threads = nt < 256 ? nt : 256;
    k_se_rows<<<bins * k, threads, 0, s>>>(mask_d, off_d, k, nt, nr, tw64, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_se_cols<<<bins * nt, threads, 0, s>>>(work, k, nt, tw64, spec64, spec32);
    return hipGetLastError();
}

hipError_t launch_fill_hash(int32_t *p, size_t n, int L, unsigned int seed, hipStream_t s) {
    const int grid = (int)std::min<size_t>((n + 255) / 256, 2048);
    k_fill_hash<<<grid, 256, 0, s>>>(p, n, L, seed);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 2048);
    k_zero<<<grid, 256, 0, s>>>((uint32_t *)p, n);
    return hipGetLastError();
}

hipError_t launch_or_flag(uint32_t *dst, const uint32_t *src, hipStream_t s) {
    k_or_flag<<<1, 64, 0, s>>>(dst, src);
    return hipGetLastError();
}

hipError_t launch_fft(int nt, int dbl, const JobDev *jobs, const Seg *segs, int nseg, long long nitems,
                      int grid, const TwF *tw32, const double2 *tw64, void *slabs, long long big_chunk,
                      StatsDev *st, const uint8_t *perturb, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
#define MD_FFT_CASE(R, N) \
    k_fft_reg<R, N, fft_reg_lanes(N, sizeof(R) == 8)><<<grid, fft_reg_lanes(N, sizeof(R) == 8) * N, 0, s>>>( \
        jobs, segs, nseg, nitems, tw32, tw64, st, perturb); break;
#define MD_FFT_BIG(R, N)                                                                                        \
    for (long long c0 = 0; c0 < nitems; c0 += big_chunk) {                                                      \
        const int cn = (int)std::min<long long>(big_chunk, nitems - c0);                                        \
        k_fft_big<R, N, 0><<<grid, kBigThreads, 0, s>>>(jobs, segs, nseg, c0, cn, tw32, tw64, slabs, st, perturb); \
        k_fft_big<R, N, 1><<<grid, kBigThreads, 0, s>>>(jobs, segs, nseg, c0, cn, tw32, tw64, slabs, st, perturb); \
        k_fft_big<R, N, 2><<<grid, kBigThreads, 0, s>>>(jobs, segs, nseg, c0, cn, tw32, tw64, slabs, st, perturb); \
        const hipError_t e_ = hipGetLastError();                                                                \
        if (e_ != hipSuccess) return e_;                                                                        \
    }                                                                                                           \
    break;
    if (!dbl) {
        switch (nt) {
            case 16: MD_FFT_CASE(float, 16)
            case 32: MD_FFT_CASE(float, 32)
            case 64: MD_FFT_CASE(float, 64)
            case 128: MD_FFT_CASE(float, 128)
            case 256: MD_FFT_BIG(float, 256)
            case 512: MD_FFT_BIG(float, 512)
            case 1024: MD_FFT_BIG(float, 1024)
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (nt) {
            case 16: MD_FFT_CASE(double, 16)
            case 32: MD_FFT_CASE(double, 32)
            case 64: MD_FFT_CASE(double, 64)
            case 128: MD_FFT_BIG(double, 128)
            case 256: MD_FFT_BIG(double, 256)
            case 512: MD_FFT_BIG(double, 512)
            case 1024: MD_FFT_BIG(double, 1024)
            default: return hipErrorInvalidValue;
        }
    }
#undef MD_FFT_CASE
#undef MD_FFT_BIG
    return hipGetLastError();
}

hipError_t launch_decode(int var, int dbl, const JobDev *jobs, const Seg *segs, int nseg, long long nitems,
                         int grid, float band, unsigned int *tile_flags, int2 *fb_list, int2 *win_list,
                         StatsDev *st, const uint8_t *perturb, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (var >= kDecFftVar) {
#define MD_DFFT(R, M) \
    k_decode_fft<R, M><<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems, band, tile_flags, fb_list, win_list, \
                                                     st); break
        const int dm = decode_fft_m(var);
        if (decode_small_m(dm, dbl)) {
#define MD_DSMALL(R, M) \
    k_decode_small<R, M><<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems, band, tile_flags, fb_list, win_list, \
                                                       st, perturb); break
            switch ((dbl ? 100000 : 0) + dm) {
                case 4: MD_DSMALL(float, 4);
                case 5: MD_DSMALL(float, 5);
                case 6: MD_DSMALL(float, 6);
                case 8: MD_DSMALL(float, 8);
                case 10: MD_DSMALL(float, 10);
                case 12: MD_DSMALL(float, 12);
                case 16: MD_DSMALL(float, 16);
                case 20: MD_DSMALL(float, 20);
                case 24: MD_DSMALL(float, 24);
                case 40: MD_DSMALL(float, 40);
                case 9: MD_DSMALL(float, 9);
                case 15: MD_DSMALL(float, 15);
                case 18: MD_DSMALL(float, 18);
                case 25: MD_DSMALL(float, 25);
                case 27: MD_DSMALL(float, 27);
                case 30: MD_DSMALL(float, 30);
                case 36: MD_DSMALL(float, 36);
                case 45: MD_DSMALL(float, 45);
                case 100004: MD_DSMALL(double, 4);
                case 100005: MD_DSMALL(double, 5);
                case 100006: MD_DSMALL(double, 6);
                case 100008: MD_DSMALL(double, 8);
                case 100010: MD_DSMALL(double, 10);
                case 100012: MD_DSMALL(double, 12);
                case 100016: MD_DSMALL(double, 16);
                case 100020: MD_DSMALL(double, 20);
                case 100024: MD_DSMALL(double, 24);
                case 100009: MD_DSMALL(double, 9);
                case 100015: MD_DSMALL(double, 15);
                case 100018: MD_DSMALL(double, 18);
                default: return hipErrorInvalidValue;
            }
#undef MD_DSMALL
            return hipGetLastError();
        }
        switch ((dbl ? 100000 : 0) + dm) {
            case 32: MD_DFFT(float, 32);
            case 64: MD_DFFT(float, 64);
            case 128: MD_DFFT(float, 128);
            case 256: MD_DFFT(float, 256);
            case 512: MD_DFFT(float, 512);
            case 1024: MD_DFFT(float, 1024);
            case 2048: MD_DFFT(float, 2048);
            case 48: MD_DFFT(float, 48);
            case 96: MD_DFFT(float, 96);
            case 192: MD_DFFT(float, 192);
            case 384: MD_DFFT(float, 384);
            case 768: MD_DFFT(float, 768);
            case 40: MD_DFFT(float, 40);
            case 80: MD_DFFT(float, 80);
            case 160: MD_DFFT(float, 160);
            case 320: MD_DFFT(float, 320);
            case 100032: MD_DFFT(double, 32);
            case 100064: MD_DFFT(double, 64);
            case 100128: MD_DFFT(double, 128);
            case 100256: MD_DFFT(double, 256);
            case 100512: MD_DFFT(double, 512);
            case 101024: MD_DFFT(double, 1024);
            case 102048: MD_DFFT(double, 2048);
            default: return hipErrorInvalidValue;
        }
#undef MD_DFFT
        return hipGetLastError();
    }
#define MD_DEC(R, V) \
    k_decode<R, V><<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems, band, tile_flags, fb_list, win_list, st, \
                                                perturb);                                                       \
    break
    if (!dbl) {
        switch (var) {
            case kDec4: MD_DEC(float, kDec4);
            case kDec8: MD_DEC(float, kDec8);
            case kDec12: MD_DEC(float, kDec12);
            case kDec24: MD_DEC(float, kDec24);
            default: MD_DEC(float, kDecBlk);
        }
    } else {
        switch (var) {
            case kDec4: MD_DEC(double, kDec4);
            case kDec8: MD_DEC(double, kDec8);
            case kDec12: MD_DEC(double, kDec12);
            default: MD_DEC(double, kDecBlk);
        }
    }
#undef MD_DEC
    return hipGetLastError();
}

int decode_group_variant(int bins, int dbl) { return decode_variant(bins, dbl); }

int dec_pitch(int nr) { return ((nr / 2 + 1) + 31) / 32 * 32; }

hipError_t launch_fallback(int nt64, const JobDev *jobs, const int2 *fb_list, StatsDev *st, double2 *slots,
                           size_t slot_elems, int grid, const double2 *tw64, double2 *slabs,
                           unsigned int *tile_flags, int2 *win_list, const uint8_t *perturb, hipStream_t s) {
#define MD_FB(N)                                                                                             \
    k_fallback<N><<<grid, kDecThreads, 0, s>>>(jobs, fb_list, st, slots, slot_elems, tw64, slabs, tile_flags, \
                                                win_list, perturb);                                          \
    break;
    switch (nt64) {
        case 16: MD_FB(16)
        case 32: MD_FB(32)
        case 64: MD_FB(64)
        case 128: MD_FB(128)
        case 256: MD_FB(256)
        case 512: MD_FB(512)
        case 1024: MD_FB(1024)
        default: return hipErrorInvalidValue;
    }
#undef MD_FB
    return hipGetLastError();
}

hipError_t launch_dft16(int variant, const float2 *in, float2 *out, long long lines, int reps, hipStream_t s) {
    if (lines <= 0) return hipSuccess;
    const int grid = (int)((lines + 255) / 256);
    switch (variant) {
        case 0: k_dft16_valu<<<grid, 256, 0, s>>>(in, out, lines, reps); break;
        case 1: k_dft16_mfma32<<<grid, 256, 0, s>>>(in, out, lines, reps); break;
        case 2: k_dft16_mfma_bf16x3<<<grid, 256, 0, s>>>(in, out, lines, reps); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tile_window(const JobDev *jobs, const int2 *win_list, const StatsDev *st, int pblocks, int grid,
                              hipStream_t s) {
    if (grid <= 0 || pblocks <= 0) return hipSuccess;
    k_tile_window<<<grid, kDecThreads, 0, s>>>(jobs, win_list, st, pblocks);
    return hipGetLastError();
}


}  // namespace md
