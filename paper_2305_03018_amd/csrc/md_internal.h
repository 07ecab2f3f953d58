// Internal declarations shared by the HIP kernels (md_fft.hip, md_direct.hip) and the
// host runtime (md_runtime.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace md {

// Length of the full-circle FP64 twiddle table; every spatial FFT length
// divides it (spatial lengths are powers of two up to kTwN).
constexpr int kTwN = 1024;

// Spatial FFT lengths: LDS-resident up to kMaxLdsN32 (FP32) / kMaxLdsN64
// (FP64) points per side, through a per-block global slab beyond, up to kMaxN.
constexpr int kMaxLdsN32 = 128;
constexpr int kMaxLdsN64 = 64;
constexpr int kMaxN = 1024;
constexpr int kBigThreads = 256;
constexpr int kMaxDirectK = 127;

// "Minus infinity" of the direct max-plus path: an out-of-image pixel or a
// masked-out SE cell.  Two of them still sum without overflow.
constexpr int32_t kNeg = -(1 << 29);

// Geometry of the direct max-plus kernel: each block produces a
// kDirBH x kDirBW output tile, each thread kDirRX consecutive outputs of a row.
constexpr int kDirRX = 8;
constexpr int kDirBW = 128;
constexpr int kDirBH = 16;
constexpr int kDirThreads = (kDirBW / kDirRX) * kDirBH;   // 256

// Decode kernel geometry: kDecThreads threads per block, each decoding
// kDecPixPerThread pixels of a work item.
constexpr int kDecThreads = 256;
constexpr int kDecPixPerThread = 4;

// FP32 twiddle stored as an unevaluated sum hi + lo of two floats, so that
// hi + lo carries about 48 significant bits of exp(-2 pi i j / kTwN).
struct TwF {
    float2 hi, lo;
};

// Exact transform path modulo the prime kNttP = 7 * 2^20 + 1 (primitive root
// kNttG): spatial lengths 16..kNttMaxN in LDS, range lengths n | kNttP - 1
// (2^a or 7 * 2^a) up to kNttMaxNr; the spatial twiddles are powers of a
// primitive kNttTw-th root of unity.
constexpr uint32_t kNttP = 7340033u;
constexpr uint32_t kNttG = 3u;
constexpr int kNttTw = 1024;
constexpr int kNttMaxN = 128;
constexpr int kNttMaxNr = 1024;

enum : int { kPathFFT = 1, kPathDirect = 2 };
enum : int { kPrecFP32 = 0, kPrecFP64 = 1, kPrecNTT = 2 };
enum : int { kFbNone = 0, kFbFFT64 = 1 };

// One SE slab of a volume job on the direct path: the 2-D window of SE slab
// a (correlation-order arrays as in JobDev) applied to input slice
// z - dz for output slice z, dz = a - r.
struct SlabDev {
    const int32_t *sek, *sek16, *sek_rows, *sek_steps;
    int dir_nsteps;
    int dz;
    int pad[2];
};

// One job as the kernels see it.  Complex arrays are float2 in the FP32 form
// and double2 in the FP64 form (the `dbl` flag of the job's plan).
struct JobDev {
    const int32_t *img;
    int32_t *out;
    int H, W, L, k, op;          // op 0 dilation, 1 erosion (complement + reflected SE)
    int path;                    // kPathFFT / kPathDirect
    // transform plan
    int nt, T, nr, bins, tiles_x, tiles_y;
    int dbl;                     // kPrecFP32 / kPrecFP64 / kPrecNTT (transform arithmetic)
    double scale;                // 1 / (nt^2 * nr)
    const void *se_spec;         // [bins][nt][nt] spectrum of the SE umbra
    const void *enc;             // [bins][L]  exp(-2 pi i (v m mod nr) / nr)
    const void *dec;             // [dp][dp] w_m exp(+2 pi i d m / nr) for m, d < bins, zero beyond
    int dec_pitch;               // dp: bins rounded up to a multiple of 32
    const void *rtw;             // [nr/2] exp(+2 pi i m / nr): twiddles of the range-axis FFT decode
    int ybs;                     // transform-domain layout of a tile: 0 = [bins][T*T]; else blocks of
                                 // 16 pixels, [ceil(T*T/16)][bins][16], and ybs = bins * 16
    long long flag0;             // first entry of this job in the tile-flag array
    int dc_dec;                  // 1: the decode computes bin 0 in closed form and the transforms
                                 // leave its plane unwritten (the register decodes: dense with
                                 // bins <= 8, and the short-length FFT decode)
    // exact recompute of ambiguous tiles
    int fb_mode;                 // kFbNone / kFbFFT64
    int nt64, T64;
    double scale64;
    const double2 *se_spec64;    // [bins][nt64][nt64]
    const double2 *enc64;        // [bins][L]
    const double2 *dec64;        // [dp][dp]
    // direct max-plus path
    const int32_t *sek;          // [k][kpad] offsets in correlation order, kNeg where masked
    const int32_t *sek16;        // same, as two equal 16-bit lanes per word: int16 (-16384 where
                                 // masked) or f16 (minus infinity where masked), per dir_pack
    const int32_t *sek_rows;     // [k][2] first and last active column of each row (first > last: none)
    const int32_t *sek_steps;    // packed form: [dir_nsteps][4] column steps (first column, kind, first
                                 // and last SE row pair (2s, 2s+1)); kind 0/1/2: 8/4/2 columns, 3: 2
                                 // columns starting at a column = 2 mod 4
    int dir_nsteps;
    int kpad;
    int dir_pack;                // element form of the window, direct_form()
    const int32_t *se_cnt;       // [k+1][k+1] prefix counts of the effective SE mask: cnt[i][j] = active
                                 // cells in rows < i, columns < j (transform jobs: the decode's count check)
    // exact transform path (dbl == kPrecNTT): se_spec / enc / dec hold uint32
    // residues mod kNttP, nr == bins == n, dec_pitch = n rounded up to 8
    const uint32_t *ntt_spec_s;  // Shoup companions of se_spec
    const uint32_t *ntt_dec_s;   // Shoup companions of dec
    int ntt_dtop;                // largest possible degree: (L-1) + max offset
    int dir_bx, dir_by;          // direct-path blocks per row / column
    // volumes (three image axes, z slowest): D slices of H x W; D = 1 and
    // nslab = 0 for images.  Direct path: the window runs once per active SE
    // slab (slabs[nslab]).  Transform path: cubic nt^3 tiles, tiles_z deep.
    int D, tiles_z;
    const SlabDev *slabs;
    int nslab;
};

// A contiguous run of work items of one job.  FFT segments cover
// ntiles * bins items (tile index fastest), decode segments ntiles * pblocks
// items, direct segments dir_bx * dir_by items.
struct Seg {
    long long item0;             // first global item index of the segment
    int job;
    int tile0, ntiles;           // tile range (FFT / decode)
    int pblocks;                 // decode: ceil(T*T / (kDecThreads * kDecPixPerThread))
    void *y;                     // transform-domain buffer [ntiles][bins][T*T]
};

// Transform-domain elements of one tile, and the position of (bin m, pixel q)
// in it, for either layout (JobDev::ybs).
__host__ __device__ inline size_t ytile_elems(int bins, int T, int ybs) {
    const size_t TT = (size_t)T * T;
    return ybs ? (TT + 15) / 16 * (size_t)ybs : (size_t)bins * TT;
}
__host__ __device__ inline size_t ybin_offset(int m, int T, int ybs) { return ybs ? (size_t)m * 16 : (size_t)m * T * T; }
__host__ __device__ inline size_t ypix(size_t q, int ybs) { return ybs ? (q >> 4) * (size_t)ybs + (q & 15) : q; }

struct StatsDev {
    unsigned int max_res_bits;   // float bits of the largest rounding residual
    unsigned int range_err;      // non-zero if an image value was outside [0, L-1]
    unsigned int fb_count;       // FP32 tiles appended to the FP64 recompute list
    unsigned int win_count;      // tiles appended to the exact window list (still ambiguous in FP64)
};

// Exactness checks of a decoded pixel (Step 3 on rounded coefficients).  A
// tile is sent on to the next exact tier when, for any of its in-image
// pixels and any degree d, |c_d - rint(c_d)| >= the band, or rint(c_d) < 0,
// or sum_d rint(c_d) differs from the number of SE cells whose window pixel
// lies in the image (the coefficients count those pairs).  The FP32 pass uses
// MD_OPT_BAND; the FP64 passes of the tiers behind it use kExactBand, the
// widest band within which rounding to the nearest integer is still sound
// for errors below 0.75.
constexpr float kExactBand = 0.25f;

// Tile flags (one word per transform tile of a batch): bit 0 set when the
// FP64 recompute took the tile, bit 1 when the exact window did.
enum : unsigned { kFlagFp64 = 1u, kFlagWindow = 2u };

// Test hook bits of the per-tile perturbation array: bit 0 perturbs the first
// transform pass of the tile, bit 1 the FP64 recompute.
enum : uint8_t { kPerturbFirst = 1, kPerturbFp64 = 2 };

// ---------------------------------------------------------------------------
// launchers (md_fft.hip, md_direct.hip); all enqueue on `s` and return the launch status
// ---------------------------------------------------------------------------
hipError_t launch_twiddles(double2 *tw64, TwF *tw32, hipStream_t s);
// rtw32 / rtw64: nr/2 entries exp(+2 pi i m / nr)
hipError_t launch_range_tables(int nr, int L, float2 *enc32, double2 *enc64, float2 *dec32,
                               double2 *dec64, float2 *rtw32, double2 *rtw64, hipStream_t s);
hipError_t launch_se_spectrum(const uint8_t *mask_d, const int32_t *off_d, int k, int nt, int nr,
                              const double2 *tw64, double2 *work, double2 *spec64, float2 *spec32,
                              hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// *dst |= *src (one word)
hipError_t launch_or_flag(uint32_t *dst, const uint32_t *src, hipStream_t s);
// out[i] = in[i] + c  /  out[i] = x[i] - y[i], i < n (int32; out may alias)
hipError_t launch_add_const(int32_t *out, const int32_t *in, int32_t c, size_t n, hipStream_t s);
hipError_t launch_sub(int32_t *out, const int32_t *x, const int32_t *y, size_t n, hipStream_t s);
hipError_t launch_fill_hash(int32_t *p, size_t n, int L, unsigned int seed, hipStream_t s);
// perturb: nullptr, or the test hook's per-tile bits (kPerturbFirst).
// Large tiles (big_tile()) run three passes per chunk of big_chunk items;
// `slabs` then holds big_chunk intermediates of nt x nt complex values and
// `grid` is the blocks of each pass.
hipError_t launch_fft(int nt, int dbl, const JobDev *jobs, const Seg *segs, int nseg, long long nitems,
                      int grid, const TwF *tw32, const double2 *tw64, void *slabs, long long big_chunk,
                      StatsDev *st, const uint8_t *perturb, hipStream_t s);
constexpr bool big_tile(int nt, int dbl) { return nt > (dbl ? kMaxLdsN64 : kMaxLdsN32); }
// Items per chunk of a large-tile launch: intermediates of about 256 MiB
// (the Infinity Cache), at least one item.
// lanes per tile line in k_fft_reg: eight for the 128-point FP32 tile (16
// waves per block, 4 per SIMD, where four lanes of 32 points would leave 2),
// four otherwise
constexpr int fft_reg_lanes(int nt, int dbl) { return !dbl && nt == 128 ? 8 : 4; }
// lines of one item that a large-tile pass takes through the LDS per block:
// 4096 points, 32 KiB (FP32) or 64 KiB (FP64); twice that in FP32 measured
// slower (fewer blocks per CU)
constexpr int big_lines_of(int nt, int dbl) { return (void)dbl, 4096 / nt; }
inline long long big_chunk_items(int nt, int dbl, long long nitems) {
    const long long per = (long long)nt * nt * (dbl ? 16 : 8);
    long long c = (256ll << 20) / per;
    if (c < 1) c = 1;
    return c < nitems ? c : nitems;
}
// decode kernel variant for a job's kept-bin count, and the zero-padded pitch
// (both dimensions) of the [bin][degree] decode table for a range length
int decode_group_variant(int bins, int dbl);
// Range-axis FFT decode: for nr = 2M with M = 2^a (nr 8..4096), M = 3 2^a
// (nr 12..1536) or M = 5 2^a (nr 10..640); lengths 3 2^a and 5 2^a from 96
// and 80 on are decoded so in FP32 only (the FP64 decode of those is dense).
// Short lengths (decode_small_m: M from 4 to 45 in FP32, to 24 in FP64, with
// no prime factor above 5, except 32) run k_decode_small, one pixel per
// thread in registers, with kDecSmallPix pixels of a tile per work item; the
// others run k_decode_fft, whose work item covers decode_fft_pixels(nr)
// pixels (256 E / M for E points per thread: 16, 24 or 20).  The decode
// variant of a range length is kDecFftVar + M.
constexpr int kDecFftVar = 16;
constexpr int kDecFftMinNr = 8, kDecFftMaxNr = 4096;
constexpr int kDecSmallPix = 512;
constexpr bool is_pow2c(int x) { return x > 0 && (x & (x - 1)) == 0; }
constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }
constexpr bool smooth235(int m) {
    if (m < 1) return false;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    while (m % 5 == 0) m /= 5;
    return m == 1;
}
constexpr bool decode_small_m(int m, int dbl) { return m >= 4 && m != 32 && m <= (dbl ? 24 : 45) && smooth235(m); }
constexpr bool decode_uses_fft(int nr, int dbl) {
    return (nr % 2 == 0 && decode_small_m(nr / 2, dbl)) ||
           (nr >= kDecFftMinNr && nr <= kDecFftMaxNr && is_pow2c(nr)) ||
           (dbl == 0 && nr >= 96 && nr <= 1536 && nr % 3 == 0 && is_pow2c(nr / 3)) ||
           (dbl == 0 && nr >= 80 && nr <= 640 && nr % 5 == 0 && is_pow2c(nr / 5));
}
constexpr int decode_fft_var(int nr) { return kDecFftVar + nr / 2; }
constexpr int decode_fft_m(int var) { return var - kDecFftVar; }
constexpr int decode_fft_pixels(int nr, int dbl) {
    return decode_small_m(nr / 2, dbl) ? kDecSmallPix : is_pow2c(nr) ? 8192 / nr : nr % 3 == 0 ? 12288 / nr : 10240 / nr;
}
int dec_pitch(int nr);
// Flagged tiles of FP32 jobs go to fb_list (the FP64 recompute), those of
// FP64 jobs to win_list (the exact window).
// perturb: as for launch_fft (the decodes that take bin 0 in closed form,
// JobDev::dc_dec, add its bump).
hipError_t launch_decode(int var, int dbl, const JobDev *jobs, const Seg *segs, int nseg,
                         long long nitems, int grid, float band, unsigned int *tile_flags,
                         int2 *fb_list, int2 *win_list, StatsDev *st, const uint8_t *perturb, hipStream_t s);
// vol: volume jobs (a window pass per active SE slab, JobDev::slabs);
// pack: direct_form()
hipError_t launch_direct(int pack, int sel, const JobDev *jobs, const Seg *segs, int nseg, long long nitems,
                         int grid, size_t lds_bytes, StatsDev *st, hipStream_t s, bool vol = false);
// FP64 recompute of the tiles on fb_list whose recompute length is nt64; a
// tile still ambiguous there is appended to win_list.
hipError_t launch_fallback(int nt64, const JobDev *jobs, const int2 *fb_list, StatsDev *st, double2 *slots,
                           size_t slot_elems, int grid, const double2 *tw64, double2 *slabs,
                           unsigned int *tile_flags, int2 *win_list, const uint8_t *perturb, hipStream_t s);
// Exact integer window (Eq. (6new)) over the tiles on win_list; each work
// item is one block of kDecThreads pixels of a tile, pblocks items per tile.
hipError_t launch_tile_window(const JobDev *jobs, const int2 *win_list, const StatsDev *st, int pblocks, int grid,
                              hipStream_t s);
// Measurement hook: `reps` forward 16-point DFTs of `lines` lines (a multiple
// of 64) of 16 complex FP32 values: variant 0 vector ALU, 1 FP32 matrix
// cores, 2 split-bf16 matrix cores.
hipError_t launch_dft16(int variant, const float2 *in, float2 *out, long long lines, int reps, hipStream_t s);
// vol: the volume form of the packed kernel (32-row blocks)
size_t direct_lds_bytes(int k, int kpad, int pack, int sel, bool vol = false);
// Element form of the direct window for the largest reachable sum
// top = (L-1) + max offset: 2 = packed f16 pairs (every sum an integer of
// magnitude <= 2048, exact in f16), 1 = packed int16 pairs (<= 16383),
// 0 = int32.  Both packed forms share block shape and LDS footprint.
constexpr int direct_form(long long top) { return top <= 2048 ? 2 : top <= 16383 ? 1 : 0; }
// exact transform path (md_ntt.hip)
int ntt_block_threads(int nt);
size_t ntt_lds_bytes(int nt);
hipError_t launch_ntt(int nt, const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                      const uint32_t *tw, const uint32_t *tws, StatsDev *st, hipStream_t s);
hipError_t launch_ntt_decode(const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                             hipStream_t s);
// volumes on the exact transform path (md_ntt.hip): cubic tiles of nt^3
// points, nt in {8, 16, 32}
int ntt3_block_threads(int nt);
hipError_t launch_ntt3(int nt, const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                       const uint32_t *tw, const uint32_t *tws, StatsDev *st, hipStream_t s);
hipError_t launch_ntt3_decode(const JobDev *jobs, const Seg *segs, int nseg, long long nitems, int grid,
                              hipStream_t s);
// spectrum of a k x k x k SE umbra mod p at spatial length nt and range
// length n, scaled by nt^-3: spec / spec_s [n][nt][nt][nt]; work holds
// n k^2 nt + n k nt^2 words
hipError_t launch_ntt3_se_spectrum(const uint8_t *mask_d, const int32_t *off_d, int k, int nt, int n,
                                   const uint32_t *rpow, const uint32_t *tw, uint32_t scale, uint32_t *work,
                                   uint32_t *spec, uint32_t *spec_s, hipStream_t s);
hipError_t launch_ntt_se_spectrum(const uint8_t *mask_d, const int32_t *off_d, int k, int nt, int n,
                                  const uint32_t *rpow, const uint32_t *tw, uint32_t scale, uint32_t *work,
                                  uint32_t *spec, uint32_t *spec_s, hipStream_t s);
constexpr size_t kLdsBytes = 160 * 1024;
int direct_block_rows(int pack, bool vol = false);
int fft_block_threads(int nt, int dbl);
size_t fft_lds_bytes(int nt, int dbl);

}  // namespace md
