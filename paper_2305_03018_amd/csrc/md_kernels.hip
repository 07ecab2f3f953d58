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
//   * Ambiguous tiles are recomputed exactly: FP64 transforms, or the direct
//     max-plus window when the FP64 tile would be too small.
//
// LDS FFT layout: an N x N complex array with row pitch N + 1.  The forward
// transform is decimation-in-time with bit-reversed input (the encode writes
// bit-reversed positions) and natural-order output; the inverse is
// decimation-in-frequency with natural-order input and bit-reversed output,
// so no explicit permutation pass is needed.  Each pass fuses q <= 3
// radix-2 stages in registers; lanes of a wavefront walk the batch axis so
// both row and column passes touch consecutive LDS words.
#include "md_internal.h"

#include <math.h>

#include <algorithm>

namespace md {
namespace {

template <typename R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C>
__device__ __forceinline__ C czero() { C r; r.x = 0; r.y = 0; return r; }

// a * exp(-+2 pi i idx / kTwN) with the twiddle held as hi + lo floats: the lo
// products are formed first so they are not lost against the hi products.
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

template <typename R> struct TwSel;
template <> struct TwSel<float> { using T = Tw32; };
template <> struct TwSel<double> { using T = Tw64; };

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }
// Passes per 1-D transform of length 2^lg and the radix-2 stages fused into
// pass p (balanced, at most 3 per pass).
constexpr int npass(int lg) { return (lg + 2) / 3; }
constexpr int passq(int lg, int p) { return lg / npass(lg) + (p < lg % npass(lg) ? 1 : 0); }
constexpr int stages_before(int lg, int p) { return p == 0 ? 0 : stages_before(lg, p - 1) + passq(lg, p - 1); }

template <int LG>
__device__ __forceinline__ int brev(int i) { return (int)(__brev((unsigned)i) >> (32 - LG)); }

// One fused decimation-in-time pass: radix-2 stages with half-sizes
// H0, 2 H0, ..., 2^(Q-1) H0 on every line of the N x N LDS array.
// AXIS 0 transforms along rows (contiguous), AXIS 1 along columns.
template <typename R, int N, int Q, int H0, int AXIS, int BS, bool INV>
__device__ __forceinline__ void pass_dit(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = N * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (N - 1);
        int gi = u / N;
        if constexpr (N >= 64) gi = __builtin_amdgcn_readfirstlane(gi);   // uniform per wavefront
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
                const int idx = j * (kTwN / (2 * (H0 << s)));
                const C b = tw.mul(x[t + hu], idx, INV);
                const C a = x[t];
                x[t] = cadd(a, b);
                x[t + hu] = csub(a, b);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * H0 * ES] = x[t];
    }
}

// One fused decimation-in-frequency pass: half-sizes 2^(Q-1) HMIN, ..., HMIN.
template <typename R, int N, int Q, int HMIN, int AXIS, int BS, bool INV>
__device__ __forceinline__ void pass_dif(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = N * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (N - 1);
        int gi = u / N;
        if constexpr (N >= 64) gi = __builtin_amdgcn_readfirstlane(gi);
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
                const int idx = j * (kTwN / (2 * hu * HMIN));
                const C a = x[t], b = x[t + hu];
                x[t] = cadd(a, b);
                x[t + hu] = tw.mul(csub(a, b), idx, INV);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * HMIN * ES] = x[t];
    }
}

template <typename R, int N, int AXIS, int BS, bool INV, int PASS = 0>
__device__ __forceinline__ void dit_axis(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    constexpr int lg = ilog2c(N);
    if constexpr (PASS < npass(lg)) {
        pass_dit<R, N, passq(lg, PASS), (1 << stages_before(lg, PASS)), AXIS, BS, INV>(lds, tw);
        __syncthreads();
        dit_axis<R, N, AXIS, BS, INV, PASS + 1>(lds, tw);
    }
}

template <typename R, int N, int AXIS, int BS, bool INV, int PASS = 0>
__device__ __forceinline__ void dif_axis(typename Cx<R>::T *lds, const typename TwSel<R>::T &tw) {
    constexpr int lg = ilog2c(N);
    if constexpr (PASS < npass(lg)) {
        pass_dif<R, N, passq(lg, PASS), (N >> (stages_before(lg, PASS) + passq(lg, PASS))), AXIS, BS, INV>(lds, tw);
        __syncthreads();
        dif_axis<R, N, AXIS, BS, INV, PASS + 1>(lds, tw);
    }
}

// One (tile, bin) of Step 2.  The tile's outputs start at pixel (oy0, ox0);
// its N x N input window starts r pixels above/left of that (overlap-save):
// input index j holds f(o0 - r + j) and the SE umbra sits at [0, k) on both
// axes, so circular output index i >= k-1 is the linear result for pixel
// o0 + i - (k-1).  Out-of-image pixels are the zero polynomial (Sec. 3,
// Step 1).  Writes the T x T valid values (unscaled) to ydst.
template <typename R, int N, int BS>
__device__ __forceinline__ void fft_tile_bin(typename Cx<R>::T *lds, const int32_t *__restrict__ img, int H,
                                             int W, int L, int op, int k, int oy0, int ox0,
                                             const typename Cx<R>::T *__restrict__ enc_m,
                                             const typename Cx<R>::T *__restrict__ spec_m,
                                             typename Cx<R>::T *__restrict__ ydst,
                                             const typename TwSel<R>::T &tw, unsigned int *range_err) {
    using C = typename Cx<R>::T;
    constexpr int P = N + 1, LG = ilog2c(N);
    const int r = (k - 1) >> 1, T = N - k + 1;
    const int iy0 = oy0 - r, ix0 = ox0 - r;
    bool bad = false;
    for (int q = threadIdx.x; q < N * N; q += BS) {
        const int i = q >> LG, j = q & (N - 1);
        const int gy = iy0 + i, gx = ix0 + j;
        C v = czero<C>();
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            int val = img[(size_t)gy * W + gx];
            if ((unsigned)val >= (unsigned)L) {
                bad = true;
                val = val < 0 ? 0 : L - 1;
            }
            if (op) val = L - 1 - val;
            v = enc_m[val];
        }
        lds[brev<LG>(i) * P + brev<LG>(j)] = v;
    }
    if (bad && range_err) atomicOr(range_err, 1u);
    __syncthreads();
    dit_axis<R, N, 0, BS, false>(lds, tw);
    dit_axis<R, N, 1, BS, false>(lds, tw);
    for (int q = threadIdx.x; q < N * N; q += BS) {
        C *e = lds + (q >> LG) * P + (q & (N - 1));
        *e = cmul(*e, spec_m[q]);
    }
    __syncthreads();
    dif_axis<R, N, 1, BS, true>(lds, tw);
    dif_axis<R, N, 0, BS, true>(lds, tw);
    for (int q = threadIdx.x; q < T * T; q += BS) {
        const int i = q / T + (k - 1), j = q % T + (k - 1);
        ydst[q] = lds[brev<LG>(i) * P + brev<LG>(j)];
    }
    __syncthreads();
}

__device__ __forceinline__ int find_seg(const Seg *__restrict__ segs, int nseg, long long it) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].item0 <= it) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename R, int N, int BS>
__global__ __launch_bounds__(BS) void k_fft(const JobDev *__restrict__ jobs, const Seg *__restrict__ segs,
                                            int nseg, long long nitems, const TwF *__restrict__ tw32,
                                            const double2 *__restrict__ tw64, StatsDev *st) {
    using C = typename Cx<R>::T;
    __shared__ C lds[N * (N + 1)];
    typename TwSel<R>::T tw;
    if constexpr (sizeof(R) == 4) tw.p = tw32; else tw.p = tw64;
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const long long local = it - S.item0;
        const int m = (int)(local / S.ntiles), tl = (int)(local % S.ntiles);
        const int tile = S.tile0 + tl;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const size_t TT = (size_t)J.T * J.T;
        C *ydst = (C *)S.y + ((size_t)tl * J.bins + m) * TT;
        fft_tile_bin<R, N, BS>(lds, J.img, J.H, J.W, J.L, J.op, J.k, ty * J.T, tx * J.T,
                               (const C *)J.enc + (size_t)m * J.L, (const C *)J.se_spec + (size_t)m * N * N,
                               ydst, tw, m == 0 ? &st->range_err : nullptr);
    }
}

// Inverse real DFT over the range axis for one pixel per lane, and Step 3.
// Wave w of the block handles the degrees d = d0 + w + kDecTPP * j.  The
// twiddle index depends only on (w, j, m), so it is wave-uniform.
template <typename R, int DPT>
__device__ __forceinline__ void decode_px(const typename Cx<R>::T *__restrict__ X, size_t mstride, int p,
                                          bool valid, const typename Cx<R>::T *__restrict__ dec, int nr,
                                          int bins, R scale, int &top, R &res) {
    using C = typename Cx<R>::T;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    top = -1;
    res = 0;
    for (int d0 = 0; d0 < nr; d0 += kDecTPP * DPT) {
        R acc[DPT];
#pragma unroll
        for (int j = 0; j < DPT; ++j) acc[j] = 0;
        for (int m = 0; m < bins; ++m) {
            C x = czero<C>();
            if (valid) x = X[(size_t)m * mstride + p];
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                const int d = d0 + w + kDecTPP * j;
                if (d < nr) {
                    const C c = dec[(size_t)d * bins + m];
                    acc[j] = fma(x.x, c.x, fma(-x.y, c.y, acc[j]));
                }
            }
        }
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = d0 + w + kDecTPP * j;
            if (d < nr) {
                const R c = acc[j] * scale;
                const R rc = rint(c);
                res = fmax(res, fabs(c - rc));
                if (rc != R(0)) top = max(top, d);
            }
        }
    }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename R, int DPT>
__global__ __launch_bounds__(kDecThreads) void k_decode(const JobDev *__restrict__ jobs,
                                                        const Seg *__restrict__ segs, int nseg,
                                                        long long nitems, float band,
                                                        unsigned int *tile_flags, int2 *fb_list,
                                                        StatsDev *st) {
    using C = typename Cx<R>::T;
    __shared__ int s_top[kDecTPP][64];
    __shared__ float s_res[kDecTPP][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const long long local = it - S.item0;
        const int tl = (int)(local / S.pblocks), pb = (int)(local % S.pblocks);
        const int tile = S.tile0 + tl;
        const int T = J.T;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const int p = pb * 64 + lane;
        const int ly = p / T, lx = p - ly * T;
        const int gy = ty * T + ly, gx = tx * T + lx;
        const bool valid = p < T * T && gy < J.H && gx < J.W;
        const size_t TT = (size_t)T * T;
        const C *X = (const C *)S.y + (size_t)tl * J.bins * TT;
        int top;
        R res;
        decode_px<R, DPT>(X, TT, p, valid, (const C *)J.dec, J.nr, J.bins, (R)J.scale, top, res);
        s_top[w][lane] = top;
        s_res[w][lane] = (float)res;
        __syncthreads();
        if (w == 0) {
            float rr = (float)res;
#pragma unroll
            for (int v = 1; v < kDecTPP; ++v) {
                top = max(top, s_top[v][lane]);
                rr = fmaxf(rr, s_res[v][lane]);
            }
            if (valid) {
                const int d = top < 0 ? 0 : top;
                J.out[(size_t)gy * J.W + gx] = J.op ? (J.L - 1 - d) : d;
            }
            const float rm = wave_max(rr);
            if (lane == 0) {
                atomicMax(&st->max_res_bits, __float_as_uint(rm));
                if (rm >= band) {
                    if (J.fb_mode == kFbNone) {
                        atomicAdd(&st->pad, 1u);
                    } else if (atomicCAS(&tile_flags[J.flag0 + tile], 0u, 1u) == 0u) {
                        const unsigned idx = atomicAdd(&st->fb_count, 1u);
                        fb_list[idx] = make_int2(S.job, tile);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Direct max-plus window over one kDirBH x kDirBW block of outputs, clipped
// to [.., ye) x [.., xe).  The image block plus halo is staged in LDS as
// int32 with kNeg outside the image; the SE is held in correlation order
// (reflected for dilation) with kNeg on masked cells, so the inner loop is
// branch-free: acc = max(acc, in + b).  Erosion runs on the complement
// L-1-f with the unreflected SE and complements the result (Sec. 2.1).
__device__ __forceinline__ void direct_block(const JobDev &J, int by0, int bx0, int ye, int xe,
                                             int32_t *tile, unsigned int *range_err) {
    const int k = J.k, r = (k - 1) >> 1, kpad = J.kpad;
    const int TWD = kDirBW + kpad, TH = kDirBH + k - 1;
    const int H = J.H, W = J.W, L = J.L;
    bool bad = false;
    for (int q = threadIdx.x; q < TH * TWD; q += kDirThreads) {
        const int a = q / TWD, c = q - a * TWD;
        const int gy = by0 - r + a, gx = bx0 - r + c;
        int v = kNeg;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W && c < kDirBW + k - 1) {
            v = J.img[(size_t)gy * W + gx];
            if ((unsigned)v >= (unsigned)L) {
                bad = true;
                v = v < 0 ? 0 : L - 1;
            }
            if (J.op) v = L - 1 - v;
        }
        tile[q] = v;
    }
    if (bad && range_err) atomicOr(range_err, 1u);
    __syncthreads();
    const int ly = threadIdx.x / (kDirBW / kDirRX);
    const int lx0 = (threadIdx.x % (kDirBW / kDirRX)) * kDirRX;
    int acc[kDirRX];
#pragma unroll
    for (int t = 0; t < kDirRX; ++t) acc[t] = kNeg;
    for (int i = 0; i < k; ++i) {
        const int32_t *trow = tile + (ly + i) * TWD + lx0;
        const int32_t *brow = J.sek + (size_t)i * kpad;
        int in[2 * kDirRX];
#pragma unroll
        for (int t = 0; t < kDirRX; t += 4) {
            const int4 v = *(const int4 *)(trow + t);
            in[t] = v.x; in[t + 1] = v.y; in[t + 2] = v.z; in[t + 3] = v.w;
        }
        for (int jb = 0; jb < kpad; jb += kDirRX) {
#pragma unroll
            for (int t = 0; t < kDirRX; t += 4) {
                const int4 v = *(const int4 *)(trow + jb + kDirRX + t);
                in[kDirRX + t] = v.x; in[kDirRX + t + 1] = v.y; in[kDirRX + t + 2] = v.z; in[kDirRX + t + 3] = v.w;
            }
#pragma unroll
            for (int s = 0; s < kDirRX; ++s) {
                const int b = brow[jb + s];
#pragma unroll
                for (int t = 0; t < kDirRX; ++t) acc[t] = max(acc[t], in[t + s] + b);
            }
#pragma unroll
            for (int t = 0; t < kDirRX; ++t) in[t] = in[t + kDirRX];
        }
    }
    const int gy = by0 + ly;
    if (gy < ye) {
#pragma unroll
        for (int t = 0; t < kDirRX; ++t) {
            const int gx = bx0 + lx0 + t;
            if (gx < xe) {
                const int d = acc[t] < 0 ? 0 : acc[t];
                J.out[(size_t)gy * W + gx] = J.op ? (L - 1 - d) : d;
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kDirThreads) void k_direct(const JobDev *__restrict__ jobs,
                                                        const Seg *__restrict__ segs, int nseg,
                                                        long long nitems, StatsDev *st) {
    extern __shared__ int32_t dyn_lds[];
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const long long local = it - S.item0;
        const int byi = (int)(local / J.dir_bx), bxi = (int)(local % J.dir_bx);
        direct_block(J, byi * kDirBH, bxi * kDirBW, J.H, J.W, dyn_lds, &st->range_err);
    }
}

// Exact recompute of the tiles listed by the decode: FP64 transforms on
// nt64-sized sub-tiles, each decoded from this block's slot.
template <int N>
__global__ __launch_bounds__(256) void k_fallback(const JobDev *__restrict__ jobs,
                                                  const int2 *__restrict__ fb_list,
                                                  const StatsDev *__restrict__ st, double2 *slots,
                                                  size_t slot_elems, const double2 *__restrict__ tw64) {
    __shared__ double2 lds[N * (N + 1)];
    __shared__ int s_top[kDecTPP][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    Tw64 tw;
    tw.p = tw64;
    const unsigned cnt = __builtin_amdgcn_readfirstlane(*(volatile const unsigned *)&st->fb_count);
    double2 *slot = slots + (size_t)blockIdx.x * slot_elems;
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
        for (int sy = 0; sy < oh; sy += T64) {
            for (int sx = 0; sx < ow; sx += T64) {
                for (int m = 0; m < J.bins; ++m)
                    fft_tile_bin<double, N, 256>(lds, J.img, J.H, J.W, J.L, J.op, J.k, oy0 + sy, ox0 + sx,
                                                 J.enc64 + (size_t)m * J.L, J.se_spec64 + (size_t)m * N * N,
                                                 slot + m * TT, tw, nullptr);
                const int sh = min(T64, oh - sy), sw = min(T64, ow - sx);
                for (int p0 = 0; p0 < (int)TT; p0 += 64) {
                    const int p = p0 + lane;
                    const int ly = p / T64, lx = p - ly * T64;
                    const bool valid = p < (int)TT && ly < sh && lx < sw;
                    int top;
                    double res;
                    decode_px<double, 24>(slot, TT, p, valid, J.dec64, J.nr, J.bins, J.scale64, top, res);
                    s_top[w][lane] = top;
                    __syncthreads();
                    if (w == 0) {
#pragma unroll
                        for (int v = 1; v < kDecTPP; ++v) top = max(top, s_top[v][lane]);
                        if (valid) {
                            const int d = top < 0 ? 0 : top;
                            J.out[(size_t)(oy0 + sy + ly) * J.W + (ox0 + sx + lx)] = J.op ? (J.L - 1 - d) : d;
                        }
                    }
                    __syncthreads();
                }
            }
        }
    }
}

// Exact recompute by the direct window, for plans whose FP64 tiles would be
// too small to be worth transforming.
__global__ __launch_bounds__(kDirThreads) void k_fallback_direct(const JobDev *__restrict__ jobs,
                                                                 const int2 *__restrict__ fb_list,
                                                                 const StatsDev *__restrict__ st) {
    extern __shared__ int32_t dyn_lds[];
    const unsigned cnt = __builtin_amdgcn_readfirstlane(*(volatile const unsigned *)&st->fb_count);
    for (unsigned i = blockIdx.x; i < cnt; i += gridDim.x) {
        const int2 e = fb_list[i];
        const JobDev &J = jobs[e.x];
        if (J.fb_mode != kFbDirect) continue;
        const int tile = e.y;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const int oy0 = ty * J.T, ox0 = tx * J.T;
        const int ye = min(oy0 + J.T, J.H), xe = min(ox0 + J.T, J.W);
        for (int by0 = oy0; by0 < ye; by0 += kDirBH)
            for (int bx0 = ox0; bx0 < xe; bx0 += kDirBW) direct_block(J, by0, bx0, ye, xe, dyn_lds, nullptr);
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
    if (q < kTwN / 2) {
        TwF t;
        t.hi = make_float2((float)c, (float)s);
        t.lo = make_float2((float)(c - (double)t.hi.x), (float)(s - (double)t.hi.y));
        tw32[q] = t;
    }
}

// enc[m][v] = exp(-2 pi i (v m mod nr) / nr): range-axis DFT of the one-hot
// column of grey value v (Eq. (7)).  dec[d][m] = w_m exp(+2 pi i (d m mod nr)
// / nr), w_m = 1 for m = 0 and m = nr/2, 2 otherwise: the inverse real DFT
// from the kept half of the bins (unscaled).
__global__ void k_range_tables(int nr, int L, int bins, float2 *enc32, double2 *enc64, float2 *dec32,
                               double2 *dec64) {
    const long long ne = (long long)bins * L, nd = (long long)nr * bins;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < ne + nd;
         q += (long long)gridDim.x * blockDim.x) {
        double s, c;
        if (q < ne) {
            const long long m = q / L, v = q % L;
            const long long ph = (v * m) % nr;
            sincospi(-2.0 * (double)ph / nr, &s, &c);
            enc64[q] = make_double2(c, s);
            enc32[q] = make_float2((float)c, (float)s);
        } else {
            const long long e = q - ne;
            const long long d = e / bins, m = e % bins;
            const long long ph = (d * m) % nr;
            sincospi(2.0 * (double)ph / nr, &s, &c);
            const double wt = (m == 0 || 2 * m == nr) ? 1.0 : 2.0;
            dec64[e] = make_double2(wt * c, wt * s);
            dec32[e] = make_float2((float)(wt * c), (float)(wt * s));
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
        const size_t o = ((size_t)m * nt + u) * nt + v;
        if (spec64) spec64[o] = make_double2(ax, ay);
        if (spec32) spec32[o] = make_float2((float)ax, (float)ay);
    }
}

__global__ void k_zero(uint32_t *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int fft_block_threads(int nt, int dbl) {
    switch (nt) {
        case 16: return 64;
        case 32: return 128;
        case 64: return 256;
        case 128: return dbl ? 0 : 1024;
        default: return 0;
    }
}

hipError_t launch_twiddles(double2 *tw64, TwF *tw32, hipStream_t s) {
    k_twiddles<<<(kTwN + 255) / 256, 256, 0, s>>>(tw64, tw32);
    return hipGetLastError();
}

hipError_t launch_range_tables(int nr, int L, float2 *enc32, double2 *enc64, float2 *dec32, double2 *dec64,
                               hipStream_t s) {
    const int bins = nr / 2 + 1;
    const long long n = (long long)bins * L + (long long)nr * bins;
    const int grid = (int)std::min<long long>((n + 255) / 256, 4096);
    k_range_tables<<<grid, 256, 0, s>>>(nr, L, bins, enc32, enc64, dec32, dec64);
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

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 2048);
    k_zero<<<grid, 256, 0, s>>>((uint32_t *)p, n);
    return hipGetLastError();
}

hipError_t launch_fft(int nt, int dbl, const JobDev *jobs, const Seg *segs, int nseg, long long nitems,
                      int grid, const TwF *tw32, const double2 *tw64, StatsDev *st, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
#define MD_FFT_CASE(R, N, BS) \
    k_fft<R, N, BS><<<grid, BS, 0, s>>>(jobs, segs, nseg, nitems, tw32, tw64, st); break;
    if (!dbl) {
        switch (nt) {
            case 16: MD_FFT_CASE(float, 16, 64)
            case 32: MD_FFT_CASE(float, 32, 128)
            case 64: MD_FFT_CASE(float, 64, 256)
            case 128: MD_FFT_CASE(float, 128, 1024)
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (nt) {
            case 16: MD_FFT_CASE(double, 16, 64)
            case 32: MD_FFT_CASE(double, 32, 128)
            case 64: MD_FFT_CASE(double, 64, 256)
            default: return hipErrorInvalidValue;
        }
    }
#undef MD_FFT_CASE
    return hipGetLastError();
}

hipError_t launch_decode(int big, int dbl, const JobDev *jobs, const Seg *segs, int nseg, long long nitems,
                         int grid, float band, unsigned int *tile_flags, int2 *fb_list, StatsDev *st,
                         hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (!dbl) {
        if (big) k_decode<float, 24><<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems, band, tile_flags, fb_list, st);
        else k_decode<float, 8><<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems, band, tile_flags, fb_list, st);
    } else {
        if (big) k_decode<double, 24><<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems, band, tile_flags, fb_list, st);
        else k_decode<double, 8><<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems, band, tile_flags, fb_list, st);
    }
    return hipGetLastError();
}

size_t direct_lds_bytes(int k, int kpad) {
    return (size_t)(kDirBH + k - 1) * (kDirBW + kpad) * sizeof(int32_t);
}

hipError_t launch_direct(const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                         size_t lds_bytes, StatsDev *st, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    k_direct<<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
    return hipGetLastError();
}

hipError_t launch_fallback(int nt64, const JobDev *jobs, const int2 *fb_list, const StatsDev *st,
                           double2 *slots, size_t slot_elems, int grid, const double2 *tw64, hipStream_t s) {
    switch (nt64) {
        case 16: k_fallback<16><<<grid, 256, 0, s>>>(jobs, fb_list, st, slots, slot_elems, tw64); break;
        case 32: k_fallback<32><<<grid, 256, 0, s>>>(jobs, fb_list, st, slots, slot_elems, tw64); break;
        case 64: k_fallback<64><<<grid, 256, 0, s>>>(jobs, fb_list, st, slots, slot_elems, tw64); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fallback_direct(const JobDev *jobs, const int2 *fb_list, const StatsDev *st, int grid,
                                  size_t lds_bytes, hipStream_t s) {
    k_fallback_direct<<<grid, kDirThreads, lds_bytes, s>>>(jobs, fb_list, st);
    return hipGetLastError();
}

}  // namespace md
