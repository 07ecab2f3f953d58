// Exact transform path in a prime field for gfx950.
//
// The umbra convolution of Step 2 (Sec. 3) done with number-theoretic
// transforms instead of complex FFTs (the paper names them as the integer
// alternative): every coefficient of the product polynomial is a count of
// SE cells, at most |B| < p = 7 * 2^20 + 1, so the convolution computed
// modulo p is the exact integer result -- no rounding, no ambiguity band and
// no recompute.  Same structure as the FFT path:
//   * range axis: the transform of a one-hot column at grey value v is
//     w_n^(v m) (w_n a primitive n-th root of unity mod p, n | p - 1), read
//     from a table; all n bins are kept (no conjugate symmetry mod p);
//   * image axes: overlap-save tiles, one workgroup per (tile, bin):
//     bit-reversed encode into LDS, decimation-in-time over rows and columns,
//     product with the SE spectrum (scaled by nt^-2), decimation-in-frequency
//     back, T x T valid values written out;
//   * decode: per pixel c_d = n^-1 sum_m X_m w_n^(-d m), from the top degree
//     down in blocks, to the first non-zero count (Step 3, Eq. (9)).
// Every product has one operand that is fixed in advance (twiddles, SE
// spectrum, decode table), so it is done by Shoup's method with a stored
// companion floor(w 2^32 / p): one 32-bit high product and two 24-bit low
// products (p < 2^23 keeps every operand below 2^24).
#include "md_device.h"

#include <algorithm>

namespace md {
namespace {

constexpr uint32_t kP = kNttP;

// a * w mod p for a < 2^24, w < p, ws = floor(w 2^32 / p): the remainder
// a w - q p with q = floor(a ws / 2^32) lies in [0, 2p), so the low 32 bits
// of the two products give it exactly.
__device__ __forceinline__ uint32_t mulw_lazy(uint32_t a, uint32_t w, uint32_t ws) {
    const uint32_t q = __umulhi(a, ws);
    return __umul24(a, w) - __umul24(q, kP);
}
__device__ __forceinline__ uint32_t red1(uint32_t x) { return min(x, x - kP); }   // [0, 2p) -> [0, p)
__device__ __forceinline__ uint32_t mulw(uint32_t a, uint32_t w, uint32_t ws) { return red1(mulw_lazy(a, w, ws)); }
__device__ __forceinline__ uint32_t addm(uint32_t a, uint32_t b) { return red1(a + b); }
__device__ __forceinline__ uint32_t subm(uint32_t a, uint32_t b) { return red1(a + kP - b); }

// w_kNttTw^j and its Shoup companion, j < kNttTw
struct NTw {
    const uint32_t *__restrict__ w;
    const uint32_t *__restrict__ ws;
    template <bool INV>
    __device__ __forceinline__ uint32_t mul(uint32_t x, int idx) const {
        const int j = INV ? ((kNttTw - idx) & (kNttTw - 1)) : idx;
        return mulw(x, w[j], ws[j]);
    }
};

constexpr int nlog2(int n) { return n <= 1 ? 0 : 1 + nlog2(n >> 1); }
constexpr int nnpass(int lg) { return (lg + 3) / 4; }
constexpr int npassq(int lg, int p) { return lg / nnpass(lg) + (p < lg % nnpass(lg) ? 1 : 0); }
constexpr int nstages_before(int lg, int p) { return p == 0 ? 0 : nstages_before(lg, p - 1) + npassq(lg, p - 1); }

template <int LG>
__device__ __forceinline__ int nbrev(int i) { return (int)(__brev((unsigned)i) >> (32 - LG)); }

// One fused decimation-in-time pass (radix-2 stages with half-sizes H0 ...
// 2^(Q-1) H0) over LINES lines of length N in an LDS array of pitch N+1;
// AXIS 0 along rows, 1 along columns.  Twiddle of the butterfly at index j
// of a block of size 2h: w_2h^j = w_kNttTw^(j kNttTw / 2h).
template <int N, int Q, int H0, int AXIS, int BS, bool INV, int LINES>
__device__ __forceinline__ void npass_dit(uint32_t *lds, const NTw &tw) {
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = LINES * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (LINES - 1);
        int gi = u / LINES;
        if constexpr (LINES >= 64) gi = __builtin_amdgcn_readfirstlane(gi);
        const int o = gi % H0;
        const int base = (gi / H0) * (RAD * H0) + o;
        uint32_t *p = lds + line * LS + base * ES;
        uint32_t x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * H0 * ES];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = 1 << s;
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const int j = o + (t & (hu - 1)) * H0;
                const bool one = H0 == 1 && (t & (hu - 1)) == 0;   // w^0, known at compile time
                const uint32_t b = one ? x[t + hu] : tw.mul<INV>(x[t + hu], j * (kNttTw / (2 * (H0 << s))));
                const uint32_t a = x[t];
                x[t] = addm(a, b);
                x[t + hu] = subm(a, b);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * H0 * ES] = x[t];
    }
}

// One fused decimation-in-frequency pass: half-sizes 2^(Q-1) HMIN ... HMIN.
template <int N, int Q, int HMIN, int AXIS, int BS, bool INV, int LINES>
__device__ __forceinline__ void npass_dif(uint32_t *lds, const NTw &tw) {
    constexpr int P = N + 1, RAD = 1 << Q, UNITS = LINES * (N / RAD);
    constexpr int ES = AXIS == 0 ? 1 : P, LS = AXIS == 0 ? P : 1;
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int line = u & (LINES - 1);
        int gi = u / LINES;
        if constexpr (LINES >= 64) gi = __builtin_amdgcn_readfirstlane(gi);
        const int o = gi % HMIN;
        const int base = (gi / HMIN) * (RAD * HMIN) + o;
        uint32_t *p = lds + line * LS + base * ES;
        uint32_t x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * HMIN * ES];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = RAD >> (s + 1);
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const int j = o + (t & (hu - 1)) * HMIN;
                const bool one = HMIN == 1 && (t & (hu - 1)) == 0;
                const uint32_t a = x[t], b = x[t + hu];
                x[t] = addm(a, b);
                const uint32_t d = subm(a, b);
                x[t + hu] = one ? d : tw.mul<INV>(d, j * (kNttTw / (2 * hu * HMIN)));
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * HMIN * ES] = x[t];
    }
}

template <int N, int AXIS, int BS, bool INV, int PASS = 0>
__device__ __forceinline__ void ndit_axis(uint32_t *lds, const NTw &tw) {
    constexpr int lg = nlog2(N);
    if constexpr (PASS < nnpass(lg)) {
        npass_dit<N, npassq(lg, PASS), (1 << nstages_before(lg, PASS)), AXIS, BS, INV, N>(lds, tw);
        __syncthreads();
        ndit_axis<N, AXIS, BS, INV, PASS + 1>(lds, tw);
    }
}

template <int N, int AXIS, int BS, bool INV, int PASS = 0>
__device__ __forceinline__ void ndif_axis(uint32_t *lds, const NTw &tw) {
    constexpr int lg = nlog2(N);
    if constexpr (PASS < nnpass(lg)) {
        constexpr int Q = npassq(lg, PASS), HMIN = N >> (nstages_before(lg, PASS) + Q);
        npass_dif<N, Q, HMIN, AXIS, BS, INV, N>(lds, tw);
        __syncthreads();
        ndif_axis<N, AXIS, BS, INV, PASS + 1>(lds, tw);
    }
}

// One (tile, bin) of Step 2 modulo p.  Overlap-save geometry as on the FFT
// path: input index j holds f(o0 - r + j), the SE umbra sits at [0, k), and
// circular output index i >= k-1 is the linear result for pixel o0+i-(k-1).
// Loads of a thread's CH pixels (and then their table gathers) are issued
// together before any is used.  LDS column b holds image column brev(b), so
// a wavefront's LDS stores and loads stay on consecutive words; the bit
// reversal is paid on the global side, within one tile row.
template <int N, int BS>
__device__ __forceinline__ void ntt_tile_bin(uint32_t *lds, const int32_t *__restrict__ img, int H, int W, int L,
                                             int op, int k, int oy0, int ox0, const uint32_t *__restrict__ enc_m,
                                             const uint32_t *__restrict__ spec_m,
                                             const uint32_t *__restrict__ spec_s_m, uint32_t *__restrict__ ydst,
                                             const NTw &tw, unsigned int *range_err) {
    constexpr int P = N + 1, LG = nlog2(N), PER = N * N / BS, CH = PER < 16 ? PER : 16;
    static_assert(PER * BS == N * N, "block size must divide the tile");
    const int r = (k - 1) >> 1, T = N - k + 1;
    const int iy0 = oy0 - r, ix0 = ox0 - r;
    const auto im = gld(img);
    int badv = 0;
    for (int c0 = 0; c0 < PER; c0 += CH) {
        int val[CH];
        bool in[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            const int gy = iy0 + (q >> LG), gx = ix0 + nbrev<LG>(q & (N - 1));
            in[e] = (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
            val[e] = im[in[e] ? (size_t)gy * W + gx : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        uint32_t v[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            badv |= (int)(in[e] && (unsigned)val[e] >= (unsigned)L);
            int w = min(max(val[e], 0), L - 1);
            w = op ? L - 1 - w : w;
            v[e] = gld(enc_m)[in[e] ? w : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            lds[nbrev<LG>(q >> LG) * P + (q & (N - 1))] = in[e] ? v[e] : 0u;
        }
    }
    if (badv && range_err) atomicOr(range_err, 1u);
    __syncthreads();
    ndit_axis<N, 0, BS, false>(lds, tw);
    ndit_axis<N, 1, BS, false>(lds, tw);
    for (int c0 = 0; c0 < PER; c0 += CH) {
        uint32_t s[CH], ss[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            s[e] = gld(spec_m)[q];
            ss[e] = gld(spec_s_m)[q];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            uint32_t *x = lds + (q >> LG) * P + (q & (N - 1));
            *x = mulw(*x, s[e], ss[e]);
        }
    }
    __syncthreads();
    ndif_axis<N, 1, BS, true>(lds, tw);
    ndif_axis<N, 0, BS, true>(lds, tw);
    for (int q = threadIdx.x; q < T * N; q += BS) {
        const int i = (q >> LG) + (k - 1), b = q & (N - 1), j = nbrev<LG>(b);
        if (j >= k - 1) gst(ydst)[(size_t)(i - (k - 1)) * T + (j - (k - 1))] = lds[nbrev<LG>(i) * P + b];
    }
    __syncthreads();
}

template <int N, int BS>
__global__ __launch_bounds__(BS) void k_ntt(const JobDev *__restrict__ jobs, const Seg *__restrict__ segs, int nseg,
                                            long long nitems, const uint32_t *__restrict__ tw,
                                            const uint32_t *__restrict__ tws, StatsDev *st) {
    __shared__ uint32_t lds[N * (N + 1)];
    NTw t;
    t.w = tw;
    t.ws = tws;
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const long long local = it - S.item0;
        const int m = (int)(local / S.ntiles), tl = (int)(local % S.ntiles);
        const int tile = S.tile0 + tl;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const size_t TT = (size_t)J.T * J.T, NN = (size_t)N * N;
        uint32_t *ydst = (uint32_t *)S.y + ((size_t)tl * J.bins + m) * TT;
        ntt_tile_bin<N, BS>(lds, J.img, J.H, J.W, J.L, J.op, J.k, ty * J.T, tx * J.T,
                            (const uint32_t *)J.enc + (size_t)m * J.L, (const uint32_t *)J.se_spec + m * NN,
                            J.ntt_spec_s + m * NN, ydst, t, m == 0 ? &st->range_err : nullptr);
    }
}

// Step 3 modulo p: c_d = sum_m X_m dec[m][d] with dec[m][d] = n^-1 w_n^(-d m)
// (row pitch dp = n rounded up to kNdDC, rows padded to a multiple of kNdMC,
// zero beyond n in both), exact counts.  Degrees are taken in blocks
// of kNdDC from the block holding the largest possible degree (dtop = (L-1) +
// max offset) downwards, until every pixel of the wave has its top non-zero
// degree; bins in chunks of kNdMC (values loaded once per chunk), terms
// summed lazily in [0, 2p) and reduced every 128 bins.
constexpr int kNdDC = 8, kNdMC = 16;

__device__ __forceinline__ int ntt_top(const uint32_t *__restrict__ X, size_t mstride, int p, bool valid,
                                       const uint32_t *__restrict__ dec, const uint32_t *__restrict__ decs, int dp,
                                       int n, int dtop) {
    int top = -1;
    for (int d0 = (dtop / kNdDC) * kNdDC; d0 >= 0; d0 -= kNdDC) {
        if (!__any(valid && top < 0)) break;
        uint32_t acc[kNdDC], red[kNdDC];
#pragma unroll
        for (int dd = 0; dd < kNdDC; ++dd) acc[dd] = red[dd] = 0;
        for (int m0 = 0; m0 < n; m0 += kNdMC) {
            uint32_t x[kNdMC];
#pragma unroll
            for (int mm = 0; mm < kNdMC; ++mm) x[mm] = (valid && m0 + mm < n) ? gld(X)[(size_t)(m0 + mm) * mstride + p] : 0u;
            const auto cw = cst(dec + (size_t)m0 * dp + d0);
            const auto cs = cst(decs + (size_t)m0 * dp + d0);
#pragma unroll
            for (int mm = 0; mm < kNdMC; ++mm)   // rows past n are zero in the table (padded to kNdMC)
#pragma unroll
                for (int dd = 0; dd < kNdDC; ++dd) acc[dd] += mulw_lazy(x[mm], cw[mm * dp + dd], cs[mm * dp + dd]);
            if (((m0 + kNdMC) & 127) == 0) {   // at most 128 lazy terms (< 2^31) per partial sum
#pragma unroll
                for (int dd = 0; dd < kNdDC; ++dd) {
                    red[dd] = (uint32_t)(((uint64_t)red[dd] + acc[dd] % kP) % kP);
                    acc[dd] = 0;
                }
            }
        }
#pragma unroll
        for (int dd = kNdDC - 1; dd >= 0; --dd) {
            const uint32_t c = (uint32_t)(((uint64_t)red[dd] + acc[dd] % kP) % kP);
            if (top < 0 && c != 0) top = d0 + dd;
        }
    }
    return top;
}

__global__ __launch_bounds__(kDecThreads) void k_ntt_decode(const JobDev *__restrict__ jobs,
                                                            const Seg *__restrict__ segs, int nseg,
                                                            long long nitems) {
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0);
        const int tl = local / S.pblocks, pb = local - tl * S.pblocks;
        const int tile = S.tile0 + tl;
        const int T = J.T;
        const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
        const size_t TT = (size_t)T * T;
        const uint32_t *X = (const uint32_t *)S.y + (size_t)tl * J.bins * TT;
#pragma unroll 1
        for (int q = 0; q < kDecPixPerThread; ++q) {
            const int p = (pb * kDecPixPerThread + q) * kDecThreads + threadIdx.x;
            const int ly = p / T, lx = p - ly * T;
            const int gy = ty * T + ly, gx = tx * T + lx;
            const bool valid = p < (int)TT && gy < J.H && gx < J.W;
            const int top = ntt_top(X, TT, p, valid, (const uint32_t *)J.dec, J.ntt_dec_s, J.dec_pitch, J.nr,
                                    J.ntt_dtop);
            if (valid) {
                const int d = top < 0 ? 0 : top;
                gst(J.out)[(size_t)gy * J.W + gx] = J.op ? (J.L - 1 - d) : d;
            }
        }
    }
}

// SE spectrum modulo p at spatial length nt and range length n (Eq. (8) with
// the one-hot umbra of the SE): separable, first along the SE columns for
// each of its k rows, then along the rows; scaled by nt^-2 (the inverse
// spatial transform's factor) and stored with its Shoup companions.
__global__ void k_ntt_se_rows(const uint8_t *__restrict__ mask, const int32_t *__restrict__ off, int k, int nt,
                              int n, const uint32_t *__restrict__ rpow, const uint32_t *__restrict__ tw,
                              uint32_t *G) {
    const int m = blockIdx.x / k, i = blockIdx.x % k;
    const int step = kNttTw / nt;
    for (int v = threadIdx.x; v < nt; v += blockDim.x) {
        uint64_t acc = 0;
        for (int j = 0; j < k; ++j) {
            if (!mask[i * k + j]) continue;
            const uint64_t a = rpow[((long long)off[i * k + j] * m) % n];
            acc = (acc + a * tw[((v * j) % nt) * step]) % kP;
        }
        G[((size_t)m * k + i) * nt + v] = (uint32_t)acc;
    }
}

__global__ void k_ntt_se_cols(const uint32_t *__restrict__ G, int k, int nt, const uint32_t *__restrict__ tw,
                              uint32_t scale, uint32_t *spec, uint32_t *spec_s) {
    const int m = blockIdx.x / nt, u = blockIdx.x % nt;
    const int step = kNttTw / nt;
    for (int v = threadIdx.x; v < nt; v += blockDim.x) {
        uint64_t acc = 0;
        for (int i = 0; i < k; ++i)
            acc = (acc + (uint64_t)G[((size_t)m * k + i) * nt + v] * tw[((u * i) % nt) * step]) % kP;
        const uint32_t s = (uint32_t)(acc * scale % kP);
        const size_t o = ((size_t)m * nt + u) * nt + v;
        spec[o] = s;
        spec_s[o] = (uint32_t)(((uint64_t)s << 32) / kP);
    }
}

// ---- volumes: cubic tiles of N^3 points (Sec. 3 with N = 3 image axes: the
// umbra is 4-dimensional; the range axis is handled by the table as above,
// the three image axes by transforms of length N) ----
//
// LDS layout of one tile: point (z, y, x) at (z N + y)(N + 1) + x.  A pass
// along x takes lines (z, y) with stride N + 1 between lanes, along y and z
// it takes lines whose consecutive lanes differ in x: all three are free of
// bank conflicts.
template <int N>
struct Vol {
    static constexpr int P = N + 1;           // y pitch
    static constexpr int PZ = N * (N + 1);    // z pitch
    static constexpr int WORDS = N * PZ;
    __device__ static constexpr int at(int z, int y, int x) { return z * PZ + y * P + x; }
    // first element of line l (l < N^2) and element stride along AXIS 0 (x),
    // 1 (y), 2 (z)
    template <int AXIS>
    __device__ static int line(int l) {
        if (AXIS == 0) return l * P;                              // l = z N + y
        if (AXIS == 1) return (l / N) * PZ + (l & (N - 1));       // l = z N + x
        return (l / N) * P + (l & (N - 1));                       // l = y N + x
    }
    template <int AXIS>
    static constexpr int es() { return AXIS == 0 ? 1 : AXIS == 1 ? P : PZ; }
};

// One fused decimation-in-time pass (radix-2 stages with half-sizes H0 ...
// 2^(Q-1) H0) along AXIS over all N^2 lines of the tile.  The butterfly group
// index is the same for every lane of a wave (N^2 >= 64 lines), so twiddles
// are wave-uniform loads.
template <int N, int Q, int H0, int AXIS, int BS, bool INV>
__device__ __forceinline__ void vpass_dit(uint32_t *lds, const NTw &tw) {
    constexpr int RAD = 1 << Q, LINES = N * N, UNITS = LINES * (N / RAD), ES = Vol<N>::template es<AXIS>();
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int l = u & (LINES - 1);
        const int gi = __builtin_amdgcn_readfirstlane(u / LINES);
        const int o = gi % H0;
        const int base = (gi / H0) * (RAD * H0) + o;
        uint32_t *p = lds + Vol<N>::template line<AXIS>(l) + base * ES;
        uint32_t x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * H0 * ES];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = 1 << s;
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const int j = o + (t & (hu - 1)) * H0;
                const bool one = H0 == 1 && (t & (hu - 1)) == 0;
                const uint32_t b = one ? x[t + hu] : tw.mul<INV>(x[t + hu], j * (kNttTw / (2 * (H0 << s))));
                const uint32_t a = x[t];
                x[t] = addm(a, b);
                x[t + hu] = subm(a, b);
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * H0 * ES] = x[t];
    }
}

// One fused decimation-in-frequency pass: half-sizes 2^(Q-1) HMIN ... HMIN.
template <int N, int Q, int HMIN, int AXIS, int BS, bool INV>
__device__ __forceinline__ void vpass_dif(uint32_t *lds, const NTw &tw) {
    constexpr int RAD = 1 << Q, LINES = N * N, UNITS = LINES * (N / RAD), ES = Vol<N>::template es<AXIS>();
    for (int u = threadIdx.x; u < UNITS; u += BS) {
        const int l = u & (LINES - 1);
        const int gi = __builtin_amdgcn_readfirstlane(u / LINES);
        const int o = gi % HMIN;
        const int base = (gi / HMIN) * (RAD * HMIN) + o;
        uint32_t *p = lds + Vol<N>::template line<AXIS>(l) + base * ES;
        uint32_t x[RAD];
#pragma unroll
        for (int t = 0; t < RAD; ++t) x[t] = p[t * HMIN * ES];
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const int hu = RAD >> (s + 1);
#pragma unroll
            for (int t = 0; t < RAD; ++t) {
                if (t & hu) continue;
                const int j = o + (t & (hu - 1)) * HMIN;
                const bool one = HMIN == 1 && (t & (hu - 1)) == 0;
                const uint32_t a = x[t], b = x[t + hu];
                x[t] = addm(a, b);
                const uint32_t d = subm(a, b);
                x[t + hu] = one ? d : tw.mul<INV>(d, j * (kNttTw / (2 * hu * HMIN)));
            }
        }
#pragma unroll
        for (int t = 0; t < RAD; ++t) p[t * HMIN * ES] = x[t];
    }
}

template <int N, int AXIS, int BS, bool INV, int PASS = 0>
__device__ __forceinline__ void vdit_axis(uint32_t *lds, const NTw &tw) {
    constexpr int lg = nlog2(N);
    if constexpr (PASS < nnpass(lg)) {
        vpass_dit<N, npassq(lg, PASS), (1 << nstages_before(lg, PASS)), AXIS, BS, INV>(lds, tw);
        __syncthreads();
        vdit_axis<N, AXIS, BS, INV, PASS + 1>(lds, tw);
    }
}

template <int N, int AXIS, int BS, bool INV, int PASS = 0>
__device__ __forceinline__ void vdif_axis(uint32_t *lds, const NTw &tw) {
    constexpr int lg = nlog2(N);
    if constexpr (PASS < nnpass(lg)) {
        constexpr int Q = npassq(lg, PASS), HMIN = N >> (nstages_before(lg, PASS) + Q);
        vpass_dif<N, Q, HMIN, AXIS, BS, INV>(lds, tw);
        __syncthreads();
        vdif_axis<N, AXIS, BS, INV, PASS + 1>(lds, tw);
    }
}

// One (tile, bin) of Step 2 modulo p for a volume: input point (zz, yy, xx)
// holds f(o - r + (zz, yy, xx)) (minus-infinity = the zero column outside the
// volume), the SE umbra sits at [0, k)^3, and circular output index i >= k-1
// along each axis is the linear result for voxel o + i - (k-1).
template <int N, int BS>
__device__ __forceinline__ void ntt3_tile_bin(uint32_t *lds, const JobDev &J, int oz0, int oy0, int ox0,
                                              const uint32_t *__restrict__ enc_m,
                                              const uint32_t *__restrict__ spec_m,
                                              const uint32_t *__restrict__ spec_s_m, uint32_t *__restrict__ ydst,
                                              const NTw &tw, unsigned int *range_err) {
    constexpr int LG = nlog2(N), NN = N * N, PER = N * N * N / BS, CH = PER < 8 ? PER : 8;
    static_assert(PER * BS == N * N * N, "block size must divide the tile");
    const int k = J.k, r = (k - 1) >> 1, T = N - k + 1;
    const int iz0 = oz0 - r, iy0 = oy0 - r, ix0 = ox0 - r;
    const int D = J.D, H = J.H, W = J.W, L = J.L, op = J.op;
    const auto im = gld(J.img);
    int badv = 0;
    for (int c0 = 0; c0 < PER; c0 += CH) {
        int val[CH];
        bool in[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            const int gz = iz0 + q / NN, gy = iy0 + ((q >> LG) & (N - 1)), gx = ix0 + (q & (N - 1));
            in[e] = (unsigned)gz < (unsigned)D && (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
            val[e] = im[in[e] ? ((size_t)gz * H + gy) * W + gx : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        uint32_t v[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            badv |= (int)(in[e] && (unsigned)val[e] >= (unsigned)L);
            int w = min(max(val[e], 0), L - 1);
            w = op ? L - 1 - w : w;
            v[e] = gld(enc_m)[in[e] ? w : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            lds[Vol<N>::at(nbrev<LG>(q / NN), nbrev<LG>((q >> LG) & (N - 1)), nbrev<LG>(q & (N - 1)))] =
                in[e] ? v[e] : 0u;
        }
    }
    if (badv && range_err) atomicOr(range_err, 1u);
    __syncthreads();
    vdit_axis<N, 0, BS, false>(lds, tw);
    vdit_axis<N, 1, BS, false>(lds, tw);
    vdit_axis<N, 2, BS, false>(lds, tw);
    for (int c0 = 0; c0 < PER; c0 += CH) {
        uint32_t sv[CH], ss[CH];
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            sv[e] = gld(spec_m)[q];
            ss[e] = gld(spec_s_m)[q];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < CH; ++e) {
            const int q = (c0 + e) * BS + threadIdx.x;
            uint32_t *x = lds + Vol<N>::at(q / NN, (q >> LG) & (N - 1), q & (N - 1));
            *x = mulw(*x, sv[e], ss[e]);
        }
    }
    __syncthreads();
    vdif_axis<N, 2, BS, true>(lds, tw);
    vdif_axis<N, 1, BS, true>(lds, tw);
    vdif_axis<N, 0, BS, true>(lds, tw);
    const int TT = T * T;
    for (int q = threadIdx.x; q < TT * T; q += BS) {
        const int a = q / TT, rem = q - a * TT, b = rem / T, c = rem - b * T;
        gst(ydst)[q] = lds[Vol<N>::at(nbrev<LG>(a + k - 1), nbrev<LG>(b + k - 1), nbrev<LG>(c + k - 1))];
    }
    __syncthreads();
}

template <int N, int BS>
__global__ __launch_bounds__(BS) void k_ntt3(const JobDev *__restrict__ jobs, const Seg *__restrict__ segs, int nseg,
                                             long long nitems, const uint32_t *__restrict__ tw,
                                             const uint32_t *__restrict__ tws, StatsDev *st) {
    __shared__ uint32_t lds[Vol<N>::WORDS];
    NTw t;
    t.w = tw;
    t.ws = tws;
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const long long local = it - S.item0;
        const int m = (int)(local / S.ntiles), tl = (int)(local % S.ntiles);
        const int tile = S.tile0 + tl, txy = J.tiles_x * J.tiles_y;
        const int tz = tile / txy, rem = tile - tz * txy, ty = rem / J.tiles_x, tx = rem - ty * J.tiles_x;
        const size_t TTT = (size_t)J.T * J.T * J.T, NNN = (size_t)N * N * N;
        uint32_t *ydst = (uint32_t *)S.y + ((size_t)tl * J.bins + m) * TTT;
        ntt3_tile_bin<N, BS>(lds, J, tz * J.T, ty * J.T, tx * J.T, (const uint32_t *)J.enc + (size_t)m * J.L,
                             (const uint32_t *)J.se_spec + m * NNN, J.ntt_spec_s + m * NNN, ydst, t,
                             m == 0 ? &st->range_err : nullptr);
    }
}

// Step 3 modulo p for a volume tile: the T^3 voxels of each tile, decoded as
// on images.
__global__ __launch_bounds__(kDecThreads) void k_ntt3_decode(const JobDev *__restrict__ jobs,
                                                             const Seg *__restrict__ segs, int nseg,
                                                             long long nitems) {
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0);
        const int tl = local / S.pblocks, pb = local - tl * S.pblocks;
        const int tile = S.tile0 + tl, txy = J.tiles_x * J.tiles_y;
        const int tz = tile / txy, rem = tile - tz * txy, ty = rem / J.tiles_x, tx = rem - ty * J.tiles_x;
        const int T = J.T, TT = T * T;
        const size_t TTT = (size_t)TT * T;
        const uint32_t *X = (const uint32_t *)S.y + (size_t)tl * J.bins * TTT;
#pragma unroll 1
        for (int q = 0; q < kDecPixPerThread; ++q) {
            const int p = (pb * kDecPixPerThread + q) * kDecThreads + threadIdx.x;
            const int lz = p / TT, r2 = p - lz * TT, ly = r2 / T, lx = r2 - ly * T;
            const int gz = tz * T + lz, gy = ty * T + ly, gx = tx * T + lx;
            const bool valid = p < (int)TTT && gz < J.D && gy < J.H && gx < J.W;
            const int top = ntt_top(X, TTT, p, valid, (const uint32_t *)J.dec, J.ntt_dec_s, J.dec_pitch, J.nr,
                                    J.ntt_dtop);
            if (valid) {
                const int d = top < 0 ? 0 : top;
                gst(J.out)[((size_t)gz * J.H + gy) * J.W + gx] = J.op ? (J.L - 1 - d) : d;
            }
        }
    }
}

// Spectrum of a k x k x k SE umbra mod p, separable: along x for every SE row
// (a, i), then along y, then along z.
__global__ void k_ntt3_se_rows(const uint8_t *__restrict__ mask, const int32_t *__restrict__ off, int k, int nt,
                               int n, const uint32_t *__restrict__ rpow, const uint32_t *__restrict__ tw,
                               uint32_t *G) {
    const int kk = k * k, m = blockIdx.x / kk, row = blockIdx.x % kk;   // row = a k + i
    const int step = kNttTw / nt;
    for (int v = threadIdx.x; v < nt; v += blockDim.x) {
        uint64_t acc = 0;
        for (int j = 0; j < k; ++j) {
            const size_t c = (size_t)row * k + j;
            if (!mask[c]) continue;
            const uint64_t a = rpow[((long long)off[c] * m) % n];
            acc = (acc + a * tw[((v * j) % nt) * step]) % kP;
        }
        G[((size_t)m * kk + row) * nt + v] = (uint32_t)acc;
    }
}

// Y[o][u][e] = scale * sum_{i < len} X[o][i][e] w_nt^(u i), o < outer, u < nt,
// e < inner (one block per (o, u)); with `spec_s` set, also the Shoup
// companions of Y.
__global__ void k_ntt3_se_axis(const uint32_t *__restrict__ X, int len, int inner, int nt,
                               const uint32_t *__restrict__ tw, uint32_t scale, uint32_t *Y, uint32_t *Ys) {
    const int o = blockIdx.x / nt, u = blockIdx.x % nt;
    const int step = kNttTw / nt;
    for (int e = threadIdx.x; e < inner; e += blockDim.x) {
        uint64_t acc = 0;
        for (int i = 0; i < len; ++i)
            acc = (acc + (uint64_t)X[((size_t)o * len + i) * inner + e] * tw[((u * i) % nt) * step]) % kP;
        const uint32_t y = (uint32_t)(acc * scale % kP);
        const size_t dst = ((size_t)o * nt + u) * inner + e;
        Y[dst] = y;
        if (Ys) Ys[dst] = (uint32_t)(((uint64_t)y << 32) / kP);
    }
}

}  // namespace

int ntt3_block_threads(int nt) {
    switch (nt) {
        case 8: return 128;
        case 16: return 256;
        case 32: return 1024;
        default: return 0;
    }
}

hipError_t launch_ntt3(int nt, const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                       const uint32_t *tw, const uint32_t *tws, StatsDev *st, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (nt) {
        case 8: k_ntt3<8, 128><<<grid, 128, 0, s>>>(jobs, segs, nseg, nitems, tw, tws, st); break;
        case 16: k_ntt3<16, 256><<<grid, 256, 0, s>>>(jobs, segs, nseg, nitems, tw, tws, st); break;
        case 32: k_ntt3<32, 1024><<<grid, 1024, 0, s>>>(jobs, segs, nseg, nitems, tw, tws, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ntt3_decode(const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                              hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    k_ntt3_decode<<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems);
    return hipGetLastError();
}

hipError_t launch_ntt3_se_spectrum(const uint8_t *mask_d, const int32_t *off_d, int k, int nt, int n,
                                   const uint32_t *rpow, const uint32_t *tw, uint32_t scale, uint32_t *work,
                                   uint32_t *spec, uint32_t *spec_s, hipStream_t s) {
    const int threads = nt < 256 ? nt : 256;
    uint32_t *g1 = work;                                  // [n][k][k][nt]
    uint32_t *g2 = work + (size_t)n * k * k * nt;         // [n][k][nt][nt]
    k_ntt3_se_rows<<<n * k * k, threads, 0, s>>>(mask_d, off_d, k, nt, n, rpow, tw, g1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ntt3_se_axis<<<n * k * nt, threads, 0, s>>>(g1, k, nt, nt, tw, 1u, g2, nullptr);   // along y
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ntt3_se_axis<<<n * nt, 256, 0, s>>>(g2, k, nt * nt, nt, tw, scale, spec, spec_s);   // along z, scaled
    return hipGetLastError();
}

int ntt_block_threads(int nt) {
    switch (nt) {
        case 16: return 64;
        case 32: return 128;
        case 64: return 256;
        case 128: return 512;
        default: return 0;
    }
}

size_t ntt_lds_bytes(int nt) { return (size_t)nt * (nt + 1) * sizeof(uint32_t); }

hipError_t launch_ntt(int nt, const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                      const uint32_t *tw, const uint32_t *tws, StatsDev *st, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (nt) {
        case 16: k_ntt<16, 64><<<grid, 64, 0, s>>>(jobs, segs, nseg, nitems, tw, tws, st); break;
        case 32: k_ntt<32, 128><<<grid, 128, 0, s>>>(jobs, segs, nseg, nitems, tw, tws, st); break;
        case 64: k_ntt<64, 256><<<grid, 256, 0, s>>>(jobs, segs, nseg, nitems, tw, tws, st); break;
        case 128: k_ntt<128, 512><<<grid, 512, 0, s>>>(jobs, segs, nseg, nitems, tw, tws, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ntt_decode(const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                             hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    k_ntt_decode<<<grid, kDecThreads, 0, s>>>(jobs, segs, nseg, nitems);
    return hipGetLastError();
}

hipError_t launch_ntt_se_spectrum(const uint8_t *mask_d, const int32_t *off_d, int k, int nt, int n,
                                  const uint32_t *rpow, const uint32_t *tw, uint32_t scale, uint32_t *work,
                                  uint32_t *spec, uint32_t *spec_s, hipStream_t s) {
    const int threads = nt < 256 ? nt : 256;
    k_ntt_se_rows<<<n * k, threads, 0, s>>>(mask_d, off_d, k, nt, n, rpow, tw, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ntt_se_cols<<<n * nt, threads, 0, s>>>(work, k, nt, tw, scale, spec, spec_s);
    return hipGetLastError();
}

}  // namespace md
