// Direct max-plus window kernels for gfx950 (the classical form of the
// dilation, Eq. (6new); erosion by the complement duality of Sec. 2.1): the
// path a measured cost model picks over the transform path when the SE is
// small relative to the tonal range.
#include "md_device.h"

namespace md {
namespace {

// Direct max-plus window (the classical form of Eq. (6new)).  The image
// block plus halo is staged in LDS with "minus infinity" outside the image;
// the SE is held in correlation order (reflected for dilation) with minus
// infinity on masked cells, so the inner loop is branch-free:
// acc = max(acc, in + b).  Erosion runs on the complement L-1-f with the
// unreflected SE and complements the result (Sec. 2.1).
//
// Element formats:
//  * packed f16 (k_direct16<.., true>): two half-precision lanes per 32-bit
//    word holding vertically adjacent image rows, used when every reachable
//    sum is an integer of magnitude <= 2048 ((L-1) + max offset <= 2048),
//    which f16 holds exactly; minus infinity is the f16 infinity, so no sum
//    can wrap.  Two SE columns advance two outputs in three instructions:
//    two packed adds and one packed three-way maximum;
//  * packed int16 (k_direct16<.., false>): the same layout for values and
//    offsets <= 16383 with minus infinity = -16384, so sums stay within
//    [-32768, 16383]; one packed add and one packed max per SE column;
//  * plain int32 (k_direct32) for wider tonal ranges.
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
constexpr int kNeg16 = -16384;
constexpr unsigned kNegF16 = 0xFC00u;   // f16 minus infinity

template <bool F16> struct D16E {
    using V = s16x2;
    static constexpr unsigned kNegWord = ((unsigned)kNeg16 & 0xffffu) * 0x10001u;
};
template <> struct D16E<true> {
    using V = f16x2;
    static constexpr unsigned kNegWord = kNegF16 * 0x10001u;
};

// high 16 bits of lo-word, low 16 bits of hi-word: the packed pair of image
// rows (2p+1, 2p+2) from word rows p and p+1
__device__ __forceinline__ int straddle(int lo, int hi) {
    return (int)__builtin_amdgcn_alignbit((unsigned)hi, (unsigned)lo, 16u);
}

// Stages rows [by0 - rad, by0 - rad + TH) x columns [bx0 - rad,
// bx0 - rad + TC) of one H x W image (a volume slice) into LDS (columns up
// to `pitch`, minus infinity outside the image and past TC), complemented for
// erosion.  The 64 lanes of a wave cover
// consecutive columns (4 x 64 per row, pitch <= 256 + 4: words past 256 are
// never read), the waves take 4 consecutive rows each per pass.  The 16 loads
// of a pass are unconditional (pixel 0 stands in outside the image and the
// block) and issued together before any of them is used.  FMT 0: int32
// words; 1 (int16) and 2 (f16): LDS word (p, c) holds image rows 2p (low
// half) and 2p+1 (high half).  Returns non-zero if an in-image value lies
// outside [0, L-1].
template <int FMT, int RB = 4>
__device__ __forceinline__ int dir_stage(const JobDev &J, const int32_t *slice, int by0, int bx0, int rad, int TH,
                                         int TC, int pitch, int32_t *tile) {
    const int lane = threadIdx.x & 63;
    const auto img = gld(slice);
    const int H = J.H, W = J.W, L = J.L, op = J.op;
    constexpr bool PACK = FMT != 0;
    int badv = 0;
    for (int a0 = (threadIdx.x >> 6) * RB; a0 < TH; a0 += (kDirThreads / 64) * RB) {
        int raw[RB][4];
        bool in[RB][4];
#pragma unroll
        for (int h = 0; h < RB; ++h) {
            const int gy = by0 - rad + a0 + h;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = lane + 64 * u, gx = bx0 - rad + c;
                in[h][u] = a0 + h < TH && c < TC && (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
                raw[h][u] = img[in[h][u] ? (size_t)gy * W + gx : 0];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // grey value of staged pixel (h, u): clamped, complemented for
        // erosion; the caller's minus infinity outside the image
        auto value = [&](int h, int u) {
            int v = raw[h][u];
            badv |= (int)(in[h][u] && (unsigned)v >= (unsigned)L);
            v = min(max(v, 0), L - 1);
            return op ? L - 1 - v : v;
        };
        if constexpr (PACK) {
            // rows a, a+1 (a even) are the two halves of one LDS word: one
            // conversion of the pair and one 32-bit store.  TH is even, so
            // the pair is wholly inside the block or wholly outside.
            static_assert(RB % 2 == 0, "row pairs");
#pragma unroll
            for (int h = 0; h < RB; h += 2) {
                const int a = a0 + h;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = lane + 64 * u;
                    const int v0 = value(h, u), v1 = value(h + 1, u);
                    if (a < TH && c < pitch) {
                        unsigned w;
                        if constexpr (FMT == 2) {
                            // integers of magnitude <= 2048: exact under any rounding
                            const float f0 = in[h][u] ? (float)v0 : -__builtin_inff();
                            const float f1 = in[h + 1][u] ? (float)v1 : -__builtin_inff();
                            w = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(f0, f1));
                        } else {
                            const unsigned lo = (unsigned)(in[h][u] ? v0 : kNeg16) & 0xffffu;
                            const unsigned hi = (unsigned)(in[h + 1][u] ? v1 : kNeg16) & 0xffffu;
                            w = lo | hi << 16;
                        }
                        tile[(a >> 1) * pitch + c] = (int32_t)w;
                    }
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < RB; ++h) {
                const int a = a0 + h;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = lane + 64 * u;
                    const int v = value(h, u);
                    if (a < TH && c < pitch) tile[a * pitch + c] = in[h][u] ? v : kNeg;
                }
            }
        }
    }
    return badv;
}

// ---- 32-bit form: 128 x 16 outputs per 256-thread block, 8 consecutive
// outputs of one row per thread, SE rows one at a time over their active
// column span in 8-column steps ----

// 16 image words (this thread's 8 outputs plus the next 8 SE columns) and the
// 8 SE offsets of one 8-cell step
struct DirBuf {
    int4 w0, w1, w2, w3, b0, b1;
};

// SEL: the SE offsets are staged in LDS (else read with scalar loads from
// global memory, for SEs too large to share the LDS with the image block)
template <bool SEL>
__device__ __forceinline__ void dir_load(DirBuf &B, const int32_t *trow, const int32_t *brow, int jb) {
    B.w0 = *(const int4 *)(trow + jb);
    B.w1 = *(const int4 *)(trow + jb + 4);
    B.w2 = *(const int4 *)(trow + jb + 8);
    B.w3 = *(const int4 *)(trow + jb + 12);
    if constexpr (SEL) {
        B.b0 = *(const int4 *)(brow + jb);
        B.b1 = *(const int4 *)(brow + jb + 4);
    } else {
        const auto c = cst(brow + jb);
        B.b0 = make_int4(c[0], c[1], c[2], c[3]);
        B.b1 = make_int4(c[4], c[5], c[6], c[7]);
    }
}

__device__ __forceinline__ void dir_step(int (&acc)[kDirRX], const DirBuf &B) {
    const int in[2 * kDirRX] = {B.w0.x, B.w0.y, B.w0.z, B.w0.w, B.w1.x, B.w1.y, B.w1.z, B.w1.w,
                                B.w2.x, B.w2.y, B.w2.z, B.w2.w, B.w3.x, B.w3.y, B.w3.z, B.w3.w};
    const int b[kDirRX] = {B.b0.x, B.b0.y, B.b0.z, B.b0.w, B.b1.x, B.b1.y, B.b1.z, B.b1.w};
#pragma unroll
    for (int sj = 0; sj < kDirRX; ++sj)
#pragma unroll
        for (int t = 0; t < kDirRX; ++t) acc[t] = max(acc[t], in[t + sj] + b[sj]);
}

// One SE row over this thread's outputs: 8-cell steps from the row's first to
// its last active column, two register buffers in ping-pong (the next step's
// LDS words and offsets are in flight while the current step computes).  The
// prefetch may read up to 16 words past the active span, which the padding of
// the LDS block and of the SE arrays keeps in bounds (those values are never
// used).
template <bool SEL>
__device__ __forceinline__ void dir_row(int (&acc)[kDirRX], const int32_t *trow, const int32_t *brow, int jb0,
                                        int jhi) {
    DirBuf A, B;
    dir_load<SEL>(A, trow, brow, jb0);
    for (int jb = jb0;; jb += 2 * kDirRX) {
        dir_load<SEL>(B, trow, brow, jb + kDirRX);
        __builtin_amdgcn_sched_barrier(0);
        dir_step(acc, A);
        __builtin_amdgcn_sched_barrier(0);
        if (jb + kDirRX > jhi) break;
        dir_load<SEL>(A, trow, brow, jb + 2 * kDirRX);
        __builtin_amdgcn_sched_barrier(0);
        dir_step(acc, B);
        __builtin_amdgcn_sched_barrier(0);
        if (jb + 2 * kDirRX > jhi) break;
    }
}

// The 2-D window passes of one output slice z: for an image (nslab = 0) the
// job's own SE arrays over slice 0; for a volume, each active SE slab s over
// input slice z - dz_s (skipped when that slice lies outside the volume).
// Returns false when pass s has no input slice.
struct DirPass {
    const int32_t *slice, *sek, *sek16, *rows, *steps;
    int nsteps;
};

template <bool VOL>
__device__ __forceinline__ bool dir_pass(const JobDev &J, int z, int s, DirPass &p) {
    const size_t plane = (size_t)J.H * J.W;
    if (!VOL) {
        p.slice = J.img;
        p.sek = J.sek;
        p.sek16 = J.sek16;
        p.rows = J.sek_rows;
        p.steps = J.sek_steps;
        p.nsteps = J.dir_nsteps;
        return true;
    }
    const SlabDev &S = J.slabs[s];
    const int zi = z - S.dz;
    if ((unsigned)zi >= (unsigned)J.D) return false;
    p.slice = J.img + (size_t)zi * plane;
    p.sek = S.sek;
    p.sek16 = S.sek16;
    p.rows = S.sek_rows;
    p.steps = S.sek_steps;
    p.nsteps = S.dir_nsteps;
    return true;
}

// LDS of one 32-bit block: the image words (pitch kDirBW + kpad), each SE
// row's [first, last] active column, then (SEL) the SE offsets in correlation
// order (k rows of kpad words).  Output slice z of the job.
template <bool SEL, bool VOL>
__device__ __forceinline__ void direct32_block(const JobDev &J, int z, int by0, int bx0, int32_t *tile,
                                               unsigned int *range_err) {
    const int k = J.k, rad = (k - 1) >> 1, kpad = J.kpad;
    const int TWD = kDirBW + kpad;
    const int TH = kDirBH + k - 1;
    int32_t *rowL = tile + TH * TWD;
    int32_t *seL = rowL + ((2 * k + 3) & ~3);        // 16-byte aligned for the b128 reads
    const int trow0 = threadIdx.x / (kDirBW / kDirRX);
    const int lx0 = (threadIdx.x % (kDirBW / kDirRX)) * kDirRX;
    int acc[kDirRX];
#pragma unroll
    for (int t = 0; t < kDirRX; ++t) acc[t] = kNeg;
    const int npass = VOL ? J.nslab : 1;
    for (int s = 0; s < npass; ++s) {
        DirPass ps;
        if (!dir_pass<VOL>(J, z, s, ps)) continue;
        if (SEL)
            for (int q = threadIdx.x; q < k * kpad; q += kDirThreads) seL[q] = gld(ps.sek)[q];
        for (int q = threadIdx.x; q < 2 * k; q += kDirThreads) rowL[q] = gld(ps.rows)[q];
        const int bad = dir_stage<0>(J, ps.slice, by0, bx0, rad, TH, kDirBW + k - 1, TWD, tile);
        if (bad && range_err) atomicOr(range_err, 1u);
        __syncthreads();
        const int32_t *sebase = SEL ? seL : ps.sek;
        for (int i = 0; i < k; ++i) {
            const int jlo = rowL[2 * i], jhi = rowL[2 * i + 1];
            if (jlo > jhi) continue;
            dir_row<SEL>(acc, tile + (trow0 + i) * TWD + lx0, sebase + i * kpad, jlo & ~(kDirRX - 1), jhi);
        }
        __syncthreads();   // the LDS block is restaged by the next pass or item
    }
    const int gy = by0 + trow0, L = J.L, W = J.W;
    int32_t *out = J.out + (size_t)z * J.H * W;
    if (gy < J.H) {
#pragma unroll
        for (int t = 0; t < kDirRX; ++t) {
            const int gx = bx0 + lx0 + t;
            if (gx >= W) continue;
            const int d = acc[t] < 0 ? 0 : acc[t];
            gst(out)[(size_t)gy * W + gx] = J.op ? (L - 1 - d) : d;
        }
    }
}

template <bool SEL, bool VOL>
__global__ __launch_bounds__(kDirThreads) void k_direct32(const JobDev *__restrict__ jobs,
                                                          const Seg *__restrict__ segs, int nseg,
                                                          long long nitems, StatsDev *st) {
    extern __shared__ int32_t dyn_lds[];
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0), nb = J.dir_bx * J.dir_by;
        const int z = local / nb, rem = local - z * nb;
        const int byi = rem / J.dir_bx, bxi = rem - byi * J.dir_bx;
        direct32_block<SEL, VOL>(J, z, byi * kDirBH, bxi * kDirBW, dyn_lds, &st->range_err);
    }
}

// Packed direct window, register-blocked over output rows.  A block of
// 256 threads covers kD16BH x kDirBW outputs as 2 x 2 waves of 8 x 8 lanes;
// a lane owns 8 consecutive columns of kD16R packed output row pairs.  The
// loop runs over 8- (or 4-) column steps of the SE, and inside a step over
// SE row pairs (2s, 2s+1): output pair r reads LDS word row q+r+s (SE row 2s,
// whole words) and the straddle of word rows q+r+s, q+r+s+1 (SE row 2s+1),
// so the kD16R+1 word rows in registers slide down by one word row per SE row
// pair -- one new word row (16 words) is read from LDS per 2 x kD16R x 64
// packed add/max pairs.  The SE words (uniform across the wave) come through
// scalar loads.  Per column step, only the SE row pairs with an active cell
// in those columns are visited (sek_cols), so disk-shaped SEs skip their
// empty corners.
// R: packed output row pairs per lane (2 for images; 1 for volumes, whose
// window passes keep fewer registers live so that 4 blocks fit per CU); a
// block covers 32 R rows.
constexpr int kD16R = 2;
constexpr int kD16BH = 32 * kD16R;

// A column step covers NS SE columns starting at jb; the thread's LDS reads
// start O words earlier (O = 2 for a 2-column step at jb = 2 mod 4) so that
// every b128 read is 16-byte aligned, and take NW words: the 8 outputs plus
// NS - 1 columns, rounded up to whole b128 reads.
template <int NS, int O> struct D16 {
    static constexpr int NW = (O + NS + kDirRX - 1 + 3) & ~3;
};

template <int NW>
__device__ __forceinline__ void d16_load(int (&w)[NW], const int32_t *p) {
#pragma unroll
    for (int u = 0; u < NW / 4; ++u) {
        const int4 v = *(const int4 *)(p + 4 * u);
        w[4 * u] = v.x;
        w[4 * u + 1] = v.y;
        w[4 * u + 2] = v.z;
        w[4 * u + 3] = v.w;
    }
}

// acc = max(acc, in[t + sj] + b[sj]) over the NS SE columns of one SE row;
// all sums of a column before their maxima (a packed op that reads the result
// of the instruction right before it costs a wait state).  In f16 two
// columns share one three-way maximum.
template <int NS, bool F16>
__device__ __forceinline__ void d16_row(typename D16E<F16>::V (&acc)[kDirRX], const typename D16E<F16>::V *in,
                                        const typename D16E<F16>::V (&b)[NS]) {
    using V = typename D16E<F16>::V;
    if constexpr (F16) {
        static_assert(NS % 2 == 0, "f16 steps pair their SE columns");
#pragma unroll
        for (int sj = 0; sj < NS; sj += 2) {
            V s0[kDirRX], s1[kDirRX];
#pragma unroll
            for (int t = 0; t < kDirRX; ++t) s0[t] = in[t + sj] + b[sj];
#pragma unroll
            for (int t = 0; t < kDirRX; ++t) s1[t] = in[t + sj + 1] + b[sj + 1];
#pragma unroll
            for (int t = 0; t < kDirRX; ++t) {
                acc[t] = __builtin_elementwise_maximum(acc[t], __builtin_elementwise_maximum(s0[t], s1[t]));
                // the accumulator is opaque past this point, so the selector
                // cannot regroup maxima across column pairs or SE rows (which
                // turns one three-way maximum per two sums into three per four)
                asm("" : "+v"(acc[t]));
            }
        }
    } else {
#pragma unroll
        for (int sj = 0; sj < NS; ++sj) {
            V sum[kDirRX];
#pragma unroll
            for (int t = 0; t < kDirRX; ++t) sum[t] = in[t + sj] + b[sj];
#pragma unroll
            for (int t = 0; t < kDirRX; ++t) acc[t] = __builtin_elementwise_max(acc[t], sum[t]);
        }
    }
}

// NS SE offsets of one row at the step's first column (wave-uniform: scalar
// loads)
template <int NS>
__device__ __forceinline__ void d16_se(int (&b)[NS], const int32_t *p) {
    const auto c = cst(p);
#pragma unroll
    for (int sj = 0; sj < NS; ++sj) b[sj] = c[sj];
}

// One SE row pair (ODD) or the last, even SE row alone (!ODD) over the
// thread's kD16R output pairs, with the offsets be / bo of SE rows 2s and
// 2s+1 already in registers.  issue() runs after the first output pair: its
// arithmetic is the first use of the registers that the previous call's
// issue() filled, so their wait comes before the loads that issue() starts,
// and those loads stay in flight over the rest of the pair.
template <int R, int NS, int O, bool ODD, bool F16, typename F>
__device__ __forceinline__ void d16_pair(typename D16E<F16>::V (&acc)[R][kDirRX],
                                         const int (&win)[R + 1][D16<NS, O>::NW], const int (&be)[NS],
                                         const int (&bo)[NS], F &&issue) {
    using V = typename D16E<F16>::V;
    constexpr int NU = NS + kDirRX - 1;
    V b[NS];
#pragma unroll
    for (int sj = 0; sj < NS; ++sj) b[sj] = __builtin_bit_cast(V, be[sj]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r == (R > 1 ? 1 : 0)) {
            __builtin_amdgcn_sched_barrier(0);
            issue();
            __builtin_amdgcn_sched_barrier(0);
        }
        V in[NU];
#pragma unroll
        for (int t = 0; t < NU; ++t) in[t] = __builtin_bit_cast(V, win[r][O + t]);
        d16_row<NS, F16>(acc[r], in, b);
    }
    if constexpr (ODD) {
#pragma unroll
        for (int sj = 0; sj < NS; ++sj) b[sj] = __builtin_bit_cast(V, bo[sj]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            V in[NU];
#pragma unroll
            for (int t = 0; t < NU; ++t) in[t] = __builtin_bit_cast(V, straddle(win[r][O + t], win[r + 1][O + t]));
            d16_row<NS, F16>(acc[r], in, b);
        }
    }
}

// SE row pairs s0..s1 of one column step.  trow: LDS word row q of the
// thread at the step's first column minus O; se: SE row 0 at the step's
// first column.  Word row q+s+kD16R+1 and the offsets of SE rows 2s+2,
// 2s+3 are fetched while pair s computes, so the one wait per pair (LDS and
// scalar loads share a counter) comes after its arithmetic.  The fetches
// reach one word row past the staged block and SE row k at most, which the
// LDS allocation and the SE array's extra row cover.
template <int R, int NS, int O, bool F16>
__device__ __forceinline__ void d16_column(typename D16E<F16>::V (&acc)[R][kDirRX], const int32_t *trow, int P,
                                           const int32_t *se, int kpad, int k, int s0, int s1) {
    constexpr int NW = D16<NS, O>::NW;
    int win[R + 1][NW];
#pragma unroll
    for (int r = 0; r <= R; ++r) d16_load<NW>(win[r], trow + (s0 + r) * P);
    const int sfull = min(s1, (k - 3) >> 1);   // pairs with both rows inside the SE
    int be[NS], bo[NS];
    d16_se<NS>(be, se + 2 * s0 * kpad);
    d16_se<NS>(bo, se + (2 * s0 + 1) * kpad);
    int s = s0;
    // one pair: offsets in (ce, co), those of the next pair fetched into (ne, no)
    auto step = [&](const int (&ce)[NS], const int (&co)[NS], int (&ne)[NS], int (&no)[NS]) {
        int nxt[NW];
        d16_pair<R, NS, O, true, F16>(acc, win, ce, co, [&] {
            d16_load<NW>(nxt, trow + (s + R + 1) * P);
            d16_se<NS>(ne, se + (2 * s + 2) * kpad);
            d16_se<NS>(no, se + (2 * s + 3) * kpad);
        });
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int t = 0; t < NW; ++t) win[r][t] = win[r + 1][t];
#pragma unroll
        for (int t = 0; t < NW; ++t) win[R][t] = nxt[t];
        ++s;
    };
    // two pairs per trip, the offset registers alternating between them
    int be2[NS], bo2[NS];
    while (s < sfull) {
        step(be, bo, be2, bo2);
        step(be2, bo2, be, bo);
    }
    if (s == sfull) {
        step(be, bo, be2, bo2);
#pragma unroll
        for (int sj = 0; sj < NS; ++sj) {
            be[sj] = be2[sj];
            bo[sj] = bo2[sj];
        }
    }
    if (s <= s1) d16_pair<R, NS, O, false, F16>(acc, win, be, bo, [] {});   // s = (k-1)/2: SE row k-1 alone
}

// LDS words of one packed block: word rows of image rows 2p, 2p+1 (low,
// high half), one spare word row for the prefetch, pitch P = kDirBW + kpad + 4.
__host__ __device__ constexpr int d16_pitch(int kpad) { return kDirBW + kpad + 4; }
__host__ __device__ constexpr int d16_rows(int k, int R) { return (32 * R + k - 1) / 2 + 1; }

// Output slice z of the job (0 for an image).
template <bool VOL, bool F16>
__device__ __forceinline__ void direct16_block(const JobDev &J, int z, int by0, int bx0, int32_t *tile,
                                               unsigned int *range_err) {
    constexpr int R = VOL ? 1 : kD16R, BH = 32 * R;
    const int k = J.k, rad = (k - 1) >> 1, kpad = J.kpad;
    const int P = d16_pitch(kpad);
    const int TH = BH + k - 1;                     // image rows the block reads (even: k is odd)
    const int TC = kDirBW + k - 1;                 // image columns the block reads
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wx = wv & 1, wy = wv >> 1;
    const int cg = lane & 7, rg = lane >> 3;
    const int lx0 = wx * 64 + cg * kDirRX;         // first output column of the lane
    const int q = wy * 8 * R + rg * R;             // LDS word row = first output row / 2
    // a wave whose outputs all lie outside the image skips the window
    const bool live = bx0 + wx * 64 < J.W && by0 + wy * 16 * R < J.H;
    using V = typename D16E<F16>::V;
    V acc[R][kDirRX];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < kDirRX; ++t) acc[r][t] = __builtin_bit_cast(V, D16E<F16>::kNegWord);
    const int npass = VOL ? J.nslab : 1;
    for (int s = 0; s < npass; ++s) {
        DirPass ps;
        if (!dir_pass<VOL>(J, z, s, ps)) continue;
        // A volume restages while the accumulators are live: fewer loads in
        // flight, and the block origin is made opaque per pass so that the
        // staging addresses are recomputed rather than kept live across the
        // window.
        int oy = by0, ox = bx0;
        if (VOL) asm volatile("" : "+s"(oy), "+s"(ox));
        const int bad = dir_stage<F16 ? 2 : 1, VOL ? 2 : 4>(J, ps.slice, oy, ox, rad, TH, TC, P, tile);
        if (bad && range_err) atomicOr(range_err, 1u);
        __syncthreads();
        if (live) {
            // the SE's column steps: (first column, kind, first and last row
            // pair); kind 0: 8 columns, 1: 4 columns, 2: 2 columns, 3: 2
            // columns at a first column = 2 mod 4
            const auto steps = cst(ps.steps);
            const int32_t *base = tile + q * P + lx0;
            for (int i = 0; i < ps.nsteps; ++i) {
                const int jb = steps[4 * i], kind = steps[4 * i + 1], s0 = steps[4 * i + 2], s1 = steps[4 * i + 3];
                const int32_t *se = ps.sek16 + jb;
                switch (kind) {
                    case 0: d16_column<R, 8, 0, F16>(acc, base + jb, P, se, kpad, k, s0, s1); break;
                    case 1: d16_column<R, 4, 0, F16>(acc, base + jb, P, se, kpad, k, s0, s1); break;
                    case 2: d16_column<R, 2, 0, F16>(acc, base + jb, P, se, kpad, k, s0, s1); break;
                    default: d16_column<R, 2, 2, F16>(acc, base + jb - 2, P, se, kpad, k, s0, s1); break;
                }
            }
        }
        // every wave has finished reading the image block before it is
        // restaged or reused for the results
        __syncthreads();
    }
    // results (clamped at 0: a negative maximum is an empty window) go to LDS
    // as 16-bit values, one row of 8 per b128 write
    if (live) {
        uint16_t *ob = (uint16_t *)tile;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            V c[kDirRX];
#pragma unroll
            for (int t = 0; t < kDirRX; ++t) {
                if constexpr (F16) c[t] = __builtin_elementwise_maximum(acc[r][t], (V){0, 0});
                else c[t] = __builtin_elementwise_max(acc[r][t], (V){0, 0});
            }
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                int4 w;
                const unsigned sel = hh ? 0x07060302u : 0x05040100u;   // high or low halves of two words
                w.x = (int)__builtin_amdgcn_perm(__builtin_bit_cast(unsigned, c[1]), __builtin_bit_cast(unsigned, c[0]), sel);
                w.y = (int)__builtin_amdgcn_perm(__builtin_bit_cast(unsigned, c[3]), __builtin_bit_cast(unsigned, c[2]), sel);
                w.z = (int)__builtin_amdgcn_perm(__builtin_bit_cast(unsigned, c[5]), __builtin_bit_cast(unsigned, c[4]), sel);
                w.w = (int)__builtin_amdgcn_perm(__builtin_bit_cast(unsigned, c[7]), __builtin_bit_cast(unsigned, c[6]), sel);
                *(int4 *)(ob + (2 * (q + r) + hh) * kDirBW + lx0) = w;
            }
        }
    }
    __syncthreads();
    // rows of the block to global memory, 64 consecutive columns per wave store
    {
        const uint16_t *ob = (const uint16_t *)tile;
        const int L = J.L, W = J.W, op = J.op;
        int32_t *out = J.out + (size_t)z * J.H * W;
        const int cx = threadIdx.x & (kDirBW - 1), gx = bx0 + cx;
        if (gx < W) {
            for (int y = threadIdx.x / kDirBW; y < BH; y += kDirThreads / kDirBW) {
                const int gy = by0 + y;
                if (gy >= J.H) break;
                const uint16_t h = ob[y * kDirBW + cx];
                const int d = F16 ? (int)(float)__builtin_bit_cast(_Float16, h) : (int)h;
                gst(out)[(size_t)gy * W + gx] = op ? (L - 1 - d) : d;
            }
        }
    }
    __syncthreads();   // the LDS block is restaged by the next item
}

// The volume form asks for 4 waves per SIMD: its window loops fit, and the few
// values spilled to scratch are read and written outside them.
template <bool VOL, bool F16>
__global__ __launch_bounds__(kDirThreads) __attribute__((amdgpu_waves_per_eu(VOL ? 4 : 1))) void k_direct16(const JobDev *__restrict__ jobs,
                                                          const Seg *__restrict__ segs, int nseg,
                                                          long long nitems, StatsDev *st) {
    extern __shared__ int32_t dyn_lds[];
    for (long long it = blockIdx.x; it < nitems; it += gridDim.x) {
        const Seg S = segs[find_seg(segs, nseg, it)];
        const JobDev &J = jobs[S.job];
        const int local = (int)(it - S.item0), nb = J.dir_bx * J.dir_by;
        const int z = local / nb, rem = local - z * nb;
        const int byi = rem / J.dir_bx, bxi = rem - byi * J.dir_bx;
        direct16_block<VOL, F16>(J, z, byi * (VOL ? 32 : kD16BH), bxi * kDirBW, dyn_lds, &st->range_err);
    }
}

}  // namespace

int direct_block_rows(int pack, bool vol) { return pack ? (vol ? 32 : kD16BH) : kDirBH; }

size_t direct_lds_bytes(int k, int kpad, int pack, int sel, bool vol) {
    if (pack) return (size_t)d16_rows(k, vol ? 1 : kD16R) * d16_pitch(kpad) * sizeof(int32_t);
    const int rows = kDirBH + k - 1;
    return ((size_t)rows * (kDirBW + kpad) + (sel ? (size_t)k * kpad : 0) + (size_t)((2 * k + 3) & ~3) + 16) *
           sizeof(int32_t);
}

hipError_t launch_direct(int pack, int sel, const JobDev *jobs, const Seg *segs, int nseg, long long nitems,
                         int grid, size_t lds_bytes, StatsDev *st, hipStream_t s, bool vol) {
    if (nitems <= 0) return hipSuccess;
    if (vol) {
        if (pack == 2) k_direct16<true, true><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
        else if (pack) k_direct16<true, false><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
        else if (sel) k_direct32<true, true><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
        else k_direct32<false, true><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
    } else {
        if (pack == 2) k_direct16<false, true><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
        else if (pack) k_direct16<false, false><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
        else if (sel) k_direct32<true, false><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
        else k_direct32<false, false><<<grid, kDirThreads, lds_bytes, s>>>(jobs, segs, nseg, nitems, st);
    }
    return hipGetLastError();
}

}  // namespace md
