/*
 * md.h -- exact grey-scale morphological dilation / erosion on AMD Instinct
 * MI355X (gfx950) through the max-plus -> polynomial homomorphism of
 * Sridhar, Shahin, Breuss, Reichenbach, "The Polynomial Connection between
 * Morphological Dilation and Discrete Convolution" (arXiv 2305.03018).
 *
 * Method (Sec. 3, Steps 1-3): each grey value v becomes the monomial t^v
 * (the one-hot "umbra" column of Eqs. (7)-(8)); image and structuring
 * element (SE) are multiplied as polynomials by a linear convolution over the
 * two image axes and the grey ("range") axis (Step 2, computed here with
 * FFTs); the dilated value of a pixel is the highest degree whose rounded
 * coefficient is non-zero (Step 3, Eq. (9)).  Theorem 1 (Sec. 2.2) makes the
 * result exact: it equals max { f(x-y) + b(y) : y in B, x-y in F }
 * (Sec. 2.1, Eq. (6new)), and 0 where that set is empty (Eq. (6)).
 * Erosion follows by the duality of Sec. 2.1.
 *
 * Conventions shared by every entry point
 *   - Images are row-major H x W int32 arrays in DEVICE memory (a HIP
 *     allocation on the current device); `out` has the same shape and must
 *     not overlap `img`.  The caller owns both.
 *   - The SE is given as two k x k row-major HOST arrays: `se_mask` (uint8,
 *     non-zero = the cell belongs to the SE domain B) and `se_offsets`
 *     (int32 additive offsets b(y) >= 0, ignored where the mask is 0).  k is
 *     odd, 1 <= k <= 1023 (the direct window path covers k <= 127, the FFT
 *     path every k), and the origin is the centre cell, so cell (i, j) is the offset
 *     y = (i - r, j - r), r = (k-1)/2.  A non-flat SE has offsets > 0, a flat
 *     one has all offsets 0 (Sec. 2.1).  The library copies what it needs;
 *     the host arrays may be freed when the call returns.
 *   - Image values must lie in [0, L-1], L >= 2 (the tonal range of
 *     Sec. 2.1, l = L-1).
 *   - Dilation:  out(x) = max { img(x-y) + b(y) : y in B, x-y in image },
 *                 0 where no cell qualifies (Eq. (6new), Eq. (6)).
 *     Erosion:   out(x) = min { img(x+y) - b(y) : y in B, x+y in image },
 *                 L-1 where no cell qualifies (Eq. (Erosion); the empty case
 *                 is not fixed by the paper and is chosen so that
 *                 erosion(f, b) = (L-1) - dilation((L-1) - f, reflected b)
 *                 holds everywhere, the complement duality of Sec. 2.1).
 *                 Erosion values can be negative, down to -max(b).
 *   - Results are exact integers for every precision setting.  The
 *     transform path checks every decoded pixel (Step 3 on rounded
 *     coefficients c_d): a tile fails if any in-image pixel has a degree d
 *     with |c_d - rint(c_d)| >= the band, or rint(c_d) < 0, or if the sum of
 *     its rounded coefficients differs from the number of SE cells whose
 *     window pixel lies in the image (the coefficients count exactly those
 *     pairs, Sec. 3.1).  A failing tile goes to the next exact tier: an FP32
 *     tile is recomputed with FP64 transforms (same checks, band 0.25); a
 *     tile that fails in FP64 (first pass or recompute) is recomputed by the
 *     integer window max of Eq. (6new).  FP32 is planned only where its
 *     worst-case rounding error, nt sqrt(|B|) 3 log2(nt^2 nr) (u + beta)
 *     with u = 2^-24, stays at most 0.25; other jobs take FP64.
 *   - Work is enqueued on the stream set by md_set_stream (default: the null
 *     stream).  With MD_OPT_SYNC = 1 (default) a call waits for its work and
 *     reports device-side errors and statistics; with 0 it returns after
 *     enqueueing (statistics then refer to the previous synchronised call).
 *   - Every function returns an md_status (0 = success).  No C++ exception
 *     crosses this interface.  On MD_ERR_ARG / MD_ERR_RANGE detected on the
 *     host nothing is enqueued and `out` is untouched.  An image value outside
 *     [0, L-1] is detected on the device: the call returns MD_ERR_RANGE (when
 *     synchronous) and the contents of `out` are unspecified.
 *   - The library is not thread-safe: serialise calls from several host
 *     threads.
 */
#ifndef MD_H_
#define MD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MD_OK = 0,
    MD_ERR_ARG = -1,          /* bad shape, pointer, k, L or option value        */
    MD_ERR_RANGE = -2,        /* image value outside [0, L-1] or negative offset */
    MD_ERR_NOMEM = -3,        /* device allocation failed                        */
    MD_ERR_DEVICE = -4,       /* a HIP runtime call failed                       */
    MD_ERR_UNSUPPORTED = -5   /* no plan covers this shape / forced setting      */
} md_status;

/* Option keys for md_set_option / md_get_option. */
typedef enum {
    MD_OPT_PRECISION = 0,  /* 0: FP32 transforms with split hi/lo twiddles and FP64
                              recompute of ambiguous tiles (default);
                              1: plain FP64 transforms everywhere;
                              2: exact number-theoretic transforms modulo the
                              prime 7340033 (no rounding, no recompute): tiles
                              of 16..128 points, range lengths 2^a or 7*2^a up
                              to 1024, so (L-1) + max offset < 1024           */
    MD_OPT_BAND = 1,       /* ambiguity band of the first transform pass: a tile
                              whose decoded coefficient c has |c - rint(c)| >=
                              band goes to the next exact tier (default 0.25; 0
                              sends every tile there: FP32 tiles to the FP64
                              recompute, FP64 tiles to the integer window)       */
    MD_OPT_PATH = 2,       /* 0: auto (cost model), 1: FFT convolution of umbras,
                              2: direct max-plus window (classical, Eq. (6new)) */
    MD_OPT_TILE = 3,       /* 0: auto, else the spatial FFT length per tile axis,
                              a power of two in [8, 1024] (images use 16 and
                              up, volumes 8, 16 or 32)                           */
    MD_OPT_NR = 4,         /* 0: auto, else the range-axis DFT length; must be at
                              least (L-1) + max offset + 1.  FP paths decode a
                              length 2^a from 8 to 4096, a length 2M with M in
                              [4, 24] (FP32: [4, 45]) having no prime factor
                              above 5, and in FP32 also 3 2^a up to 1536 and
                              5 2^a up to 640, by an FFT along the range axis,
                              any other by a dense DFT; auto weighs the
                              smallest length against the next such lengths
                              when the smallest has no FFT decode or passes
                              128                                               */
    MD_OPT_SYNC = 5,       /* 1 (default): wait for completion in every call    */
    MD_OPT_GRAPH = 6,      /* 1 (default): md_dilate_batch captures its launches
                              in a HIP graph per batch signature and replays it  */
    MD_OPT_WORKSPACE_MB = 7,/* cap on the transform-domain scratch per launch
                              group, MiB (default 8192)                           */
    MD_OPT_PROFILE = 8,    /* 1: bracket every kernel launch of a non-graph call
                              with HIP events and accumulate per-stage times
                              (read with md_profile_get); default 0              */
    MD_OPT_AUTOTUNE = 9,   /* 1 (default): the first auto-path call on a device
                              measures the kernels' rates and feeds them to the
                              cost model; 0 keeps the built-in estimates         */
    MD_OPT_STREAM_ROWS = 10,/* host-streamed calls: 0 (default) picks the band
                              height from MD_OPT_STREAM_MB, else the output
                              rows (volumes: slices) per band                    */
    MD_OPT_STREAM_MB = 11, /* device memory for the band buffers of the host-
                              streamed calls, MiB (default 2048)                 */
    MD_OPT_CACHE_MB = 12   /* bound on the device memory of the library's
                              caches (range tables, SE spectra, window tables),
                              MiB (default 16384): past it the least recently
                              used entries that no cached batch plan references
                              are freed; a single entry larger than the bound
                              is still kept while in use                        */
} md_option;

/* Dilation of one image (see the conventions above). */
int md_dilate(const int32_t *img, int H, int W, int L, const uint8_t *se_mask,
              const int32_t *se_offsets, int k, int32_t *out);

/* Erosion of one image (see the conventions above). */
int md_erode(const int32_t *img, int H, int W, int L, const uint8_t *se_mask,
             const int32_t *se_offsets, int k, int32_t *out);

/* Compositions of the exact dilation and erosion (the combinations named in
 * the paper's Sec. 5: opening, closing, Beucher gradient; and the top-hats).
 * With (+) dilation and (-) erosion by the SE b:
 *   MD_OPEN      (f (-) b) (+) b
 *   MD_CLOSE     (f (+) b) (-) b
 *   MD_GRADIENT  (f (+) b) - (f (-) b)
 *   MD_TOPHAT    f - open(f)
 *   MD_BLACKHAT  close(f) - f
 * An empty window takes the bottom (dilation) or top (erosion) of the range
 * its operand spans: [0, L-1] for the input (the 0 / L-1 rules of
 * md_dilate / md_erode), [-m, L-1] for an erosion result and [0, L-1+m] for a
 * dilation result, m = the largest offset of an active SE cell.  So the
 * opening of a pixel whose dilation window is empty is -m, the closing of a
 * pixel whose erosion window is empty is L-1+m; with these values opening is
 * anti-extensive and idempotent, closing extensive and idempotent, and the
 * two are dual under the complement with the reflected SE.
 * Arguments, layout and ownership as for md_dilate; the outputs are int32 in
 * [-m, L-1+m] (gradient and top-hats: differences of those).  Runs on the
 * library stream through two device intermediates of H x W int32 that the
 * library owns (kept for later calls, freed by md_release).  MD_ERR_ARG for
 * an unknown op; MD_ERR_RANGE if L + m exceeds 2^24.  Every path, precision
 * and option of md_dilate applies to each step. */
typedef enum {
    MD_DILATE = 0,
    MD_ERODE = 1,
    MD_OPEN = 2,
    MD_CLOSE = 3,
    MD_GRADIENT = 4,
    MD_TOPHAT = 5,
    MD_BLACKHAT = 6
} md_op;

int md_morph(int op, const int32_t *img, int H, int W, int L, const uint8_t *se_mask,
             const int32_t *se_offsets, int k, int32_t *out);

/* Images in HOST memory, possibly larger than the GPU's memory: the
 * partitioned convolution that the paper's conclusion proposes for very large
 * images (n_i >= 10^9).  The image is cut into bands of output rows; each
 * band is uploaded with r = (k-1)/2 halo rows on each side (fewer at the
 * image border), dilated or eroded on the device as an image of its own by
 * the same planner and kernels as md_dilate, and its interior rows are copied
 * back.  A window of an interior row never leaves its band, so the result is
 * exactly that of md_dilate / md_erode on the whole image.
 *   - `img` and `out` are H x W int32 row-major HOST arrays (H may exceed
 *     2^31; W >= 1; a band holds at most 2^31-1 pixels).  They must not
 *     overlap.  Pinned memory (hipHostMalloc) lets the copies run
 *     asynchronously; pageable memory works too.
 *   - SE arrays, L, k and every option as for md_dilate; MD_OPT_SYNC does not
 *     apply: the call returns when `out` is complete.
 *   - Device memory: two input and two output band buffers within
 *     MD_OPT_STREAM_MB (plus the transform workspace of one band), whatever
 *     the image size.  Uploads, compute and downloads of consecutive bands
 *     overlap on three HIP streams of default priority.
 *   - MD_ERR_RANGE if any pixel lies outside [0, L-1] (then `out` is
 *     unspecified); other errors as for md_dilate. */
int md_dilate_host(const int32_t *img, long long H, int W, int L, const uint8_t *se_mask,
                   const int32_t *se_offsets, int k, int32_t *out);
int md_erode_host(const int32_t *img, long long H, int W, int L, const uint8_t *se_mask,
                  const int32_t *se_offsets, int k, int32_t *out);

/* Volumes: dilation and erosion of a three-axis image.  Sec. 2.1 defines
 * both for N-dimensional images and Sec. 3 turns the N-dimensional dilation
 * into an (N+1)-dimensional umbra convolution, here a 4-dimensional one.
 *   - `vol` and `out` are D x H x W int32 DEVICE arrays, z slowest (voxel
 *     (z, y, x) at (z*H + y)*W + x), owned by the caller; they must not
 *     overlap.  Values in [0, L-1], 2 <= L <= 2^24.
 *   - The SE is two k x k x k HOST arrays, (a, i, j) row-major: `se_mask`
 *     (non-zero = in B) and `se_offsets` (b(y) >= 0 where the mask is set);
 *     k odd, 1 <= k <= 31, cell (a, i, j) is the offset
 *     y = (a-r, i-r, j-r), r = (k-1)/2.
 *   - Dilation: out(x) = max { vol(x-y) + b(y) : y in B, x-y in the volume },
 *     0 where no cell qualifies; erosion: min { vol(x+y) - b(y) }, L-1 where
 *     none does (the conventions of md_dilate / md_erode over three axes).
 *   - Paths (MD_OPT_PATH): the direct window, one 2-D window pass per active
 *     SE slab, accumulated in registers; or the transform path, which is
 *     exact: the 4-D umbra convolution by number-theoretic transforms modulo
 *     7*2^20+1 over cubic tiles of 8, 16 or 32 points per side (MD_OPT_TILE
 *     forces one) and a range length n >= L + max b of the form 2^a or 7*2^a,
 *     n <= 1024 (MD_OPT_NR forces one).  MD_OPT_PRECISION does not apply:
 *     volume transforms always run in the prime field.  Auto (0) picks by the
 *     cost model.  MD_ERR_UNSUPPORTED if the forced path has no plan.
 *   - Runs on the library stream after the work already on it (the call
 *     waits for that work before it rewrites its device tables); with
 *     MD_OPT_SYNC = 1 it waits for its own work and reports MD_ERR_RANGE for
 *     a voxel outside [0, L-1] that lies in some output's window (voxels in
 *     no window affect no output and may go unchecked).  Error behaviour
 *     otherwise as for md_dilate. */
int md_dilate3(const int32_t *vol, int D, int H, int W, int L, const uint8_t *se_mask,
               const int32_t *se_offsets, int k, int32_t *out);
int md_erode3(const int32_t *vol, int D, int H, int W, int L, const uint8_t *se_mask,
              const int32_t *se_offsets, int k, int32_t *out);

/* Compositions on volumes: md_morph's operations (MD_OPEN ... MD_BLACKHAT,
 * with the same empty-window values) over three axes, each step by
 * md_dilate3 / md_erode3.  Arguments, layout and errors as for md_dilate3;
 * two D x H x W int32 device intermediates are owned by the library (freed
 * by md_release). */
int md_morph3(int op, const int32_t *vol, int D, int H, int W, int L, const uint8_t *se_mask,
              const int32_t *se_offsets, int k, int32_t *out);

/* Volumes in HOST memory, streamed through the GPU in bands of output
 * slices with r = (k-1)/2 halo slices on each side, each band computed by
 * md_dilate3 / md_erode3 as a volume of its own (the partitioned convolution
 * of md_dilate_host along z).  `vol` / `out`: D x H x W int32 host arrays (D
 * may exceed 2^31 / (H W); a band holds at most 2^31-1 voxels).  Band height:
 * MD_OPT_STREAM_ROWS slices if set, else the most that four band buffers fit
 * into MD_OPT_STREAM_MB.  SE arrays, L, k, options and errors as for
 * md_dilate3; the call returns when `out` is complete. */
int md_dilate3_host(const int32_t *vol, long long D, int H, int W, int L, const uint8_t *se_mask,
                    const int32_t *se_offsets, int k, int32_t *out);
int md_erode3_host(const int32_t *vol, long long D, int H, int W, int L, const uint8_t *se_mask,
                   const int32_t *se_offsets, int k, int32_t *out);

/* One job of a batch.  Pointer and ownership rules as for md_dilate. */
typedef struct {
    const int32_t *img;          /* device, H x W                 */
    int H, W, L;
    const uint8_t *se_mask;      /* host, k x k                   */
    const int32_t *se_offsets;   /* host, k x k                   */
    int k;
    int32_t *out;                /* device, H x W                 */
    int op;                      /* 0 = dilation, 1 = erosion     */
} md_job;

/* Many images of uneven size, tonal range and SE in one go.  The planner
 * picks per job the transform lengths, tile shape and the FFT-versus-direct
 * path; the launches are stage-wise persistent kernels over device work
 * queues.  With MD_OPT_GRAPH = 1 they are captured once per batch signature
 * (shapes, L, k, SEs, op) into a HIP graph and replayed; image and output
 * pointers may change between calls with the same signature.  n >= 1.
 * `jobs` is a host array read during the call only. */
int md_dilate_batch(const md_job *jobs, int n);

/* Dilation for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, layout, result and host-side errors as md_dilate, computed by
 * the direct max-plus window of Eq. (6new) (the exact integer path md_dilate
 * takes for small SEs), with k <= 127 (MD_ERR_UNSUPPORTED beyond).
 *   - Allocates nothing: no hipMalloc, hipFree or allocating library call.
 *     Its device memory beyond `img` and `out` -- job and segment
 *     descriptors, the range-error word and the SE tables of the window --
 *     is a fixed 1 MiB array in the library's device code, which every GPU
 *     the library runs on holds until the process ends.  An SE whose tables
 *     would not fit it fails with MD_ERR_ARG (cannot happen for k <= 127).
 *   - Every call on a GPU shares that GPU's array and rewrites it, so calls
 *     that overlap on one GPU (several host threads, or streams without
 *     ordering between them) race; serialise them.
 *   - Runs on the stream of md_set_stream and always waits for its work
 *     (MD_OPT_SYNC does not apply): the SE tables are uploaded from host
 *     memory of the call.  Reports MD_ERR_RANGE for an image value outside
 *     [0, L-1].  Options, caches, plans and md_set_workspace do not apply;
 *     md_get_stats afterwards reports one direct-path job. */
int md_dilate_noalloc(const int32_t *img, int H, int W, int L, const uint8_t *se_mask,
                      const int32_t *se_offsets, int k, int32_t *out);

/* Caller-owned workspace for the transform path, for callers that own all
 * device scratch memory themselves.  `dev_ptr` is a DEVICE buffer of
 * `bytes` bytes, 256-byte aligned, that holds what a batch needs beyond its
 * inputs and outputs: the transform-domain buffer, the large-tile slabs, the
 * tile flags and tier lists, the FP64 recompute's slots and slabs.  It stays
 * the caller's: it must remain valid, and untouched by other work, while
 * calls may use it -- until md_set_workspace is called again or md_release.
 * Calls are ordered on the library stream, so successive calls share it.
 * (NULL, 0) returns to library-owned workspace (the default).  Setting it
 * waits for the device and drops cached batch plans.  A call whose plan needs
 * more than `bytes` fails with MD_ERR_ARG before enqueueing anything.
 * MD_ERR_ARG if only one of dev_ptr and bytes is 0 or the pointer is not
 * 256-byte aligned.  The library still owns its caches, plans and tables. */
int md_set_workspace(void *dev_ptr, size_t bytes);

/* Workspace bytes that md_dilate_batch(jobs, n) needs under the current
 * options (plans as that call would make them; the first auto-path call on a
 * device runs the autotuner first).  0 for a batch with no transform job, and
 * 0 on an invalid job (md_last_error then says why; it is empty otherwise).
 * A single image is the batch of one job (op 0 or 1). */
size_t md_workspace_size(const md_job *jobs, int n);

/* Device memory the library holds beyond the caller's buffers: *cache_bytes
 * for the cache of MD_OPT_CACHE_MB (range tables, SE spectra, window
 * tables), *plan_bytes for the workspace owned by its *plans cached batch
 * plans (each captured graph with its launch tables; at most 64, their
 * workspace also kept within MD_OPT_CACHE_MB by dropping the least recently
 * run ones).  Host pointers.  Excludes what the HIP runtime itself allocates
 * (graphs, kernel arguments). */
int md_memory_usage(size_t *cache_bytes, size_t *plan_bytes, int *plans);

/* The plan md_dilate_batch would make for one job under the current options
 * and cost model, computed on the host only: no device is touched and the
 * autotuner does not run (before the first auto-path call on a device the
 * cost model holds its built-in estimates).  batch = 0 plans the job as a
 * single-image call, 1 as one job of a larger batch (a lone job is priced as
 * if it filled the GPU's compute units).  Transform plans (path 1) use
 * overlap-save tiles of n_t points per side with T = n_t - k + 1 outputs,
 * tiles_x = ceil(W / T), tiles_y = ceil(H / T), and a range length
 * n_r >= (L-1) + max offset + 1 with `bins` kept range bins.  Errors as for
 * md_dilate_batch's host checks (MD_ERR_ARG, MD_ERR_RANGE,
 * MD_ERR_UNSUPPORTED).  `job` and `out` are host pointers; job->img and
 * job->out are only checked for being non-null and distinct. */
typedef struct {
    int path;            /* 1: transform (umbra convolution), 2: direct window       */
    int precision;       /* transform plans: 0 FP32 + exact tiers, 1 FP64, 2 mod p    */
    int n_t, T, n_r, bins, tiles_x, tiles_y;
    int decode_fft;      /* 1: the range-axis FFT decode, 0: the dense inverse DFT    */
    int n_t64;           /* FP32 plans: tile length of the FP64 recompute             */
    double fp32_bound;   /* transform plans: the FP32 worst-case error bound of n_t,
                            n_r and the SE (NaN for direct plans)                     */
    double cost_fft_ns;  /* cost model's estimates, INFINITY where no plan exists     */
    double cost_direct_ns;
} md_plan_info;

int md_plan(const md_job *job, int batch, md_plan_info *out);

/* Stream for subsequent calls (a hipStream_t, or NULL for the null stream). */
int md_set_stream(void *hip_stream);

int md_set_option(int key, double value);
double md_get_option(int key);  /* NaN for an unknown key */

/* Statistics of the last synchronised call. */
typedef struct {
    double max_residual;      /* max |c - rint(c)| over decoded coefficients (FFT path) */
    long long tiles;          /* FFT tiles processed                                     */
    long long fallback_tiles; /* FP32 tiles recomputed with FP64 transforms               */
    long long window_tiles;   /* tiles recomputed by the integer window (failed the
                                 checks in FP64)                                       */
    long long direct_jobs;    /* jobs that took the direct path                          */
    long long fft_jobs;       /* jobs that took the FFT path                             */
    int path, n_t, n_r;       /* plan of the last job: path 1 FFT / 2 direct, lengths    */
    int precision;            /* of the last job: 0 FP32 + fallback, 1 FP64, 2 exact
                                 mod p (a transform job planned FP64 because of the
                                 FP32 error bound reports 1)                          */
} md_stats;

int md_get_stats(md_stats *stats);

/* Text of the last error (never NULL; empty after success). */
const char *md_last_error(void);

/* Release every device buffer, cached plan, spectrum and graph. */
int md_release(void);

/* Per-stage launch timing collected while MD_OPT_PROFILE = 1 (HIP events on
 * the library's stream, synchronised calls only).  `alg_bytes` / `alg_ops`
 * are the algorithmic DRAM bytes and arithmetic operations the stage has to
 * perform for the work it was given (the figures a roofline is drawn with),
 * summed over its launches.  Stage names: transforms "fft32_nN",
 * "fft64_nN", "ntt_nN" (images) and "ntt3_nN" (volumes); decodes
 * "decode32", "decode64" (dense), "decode32_fft", "decode64_fft" (range-axis
 * FFT), "decode_ntt", "decode_ntt3"; exact recompute
 * "recompute64_nN"; direct window "direct16" (packed f16), "direct16i"
 * (packed int16), "direct32", and for volumes "direct3_16", "direct3_16i",
 * "direct3_32". */
typedef struct {
    char name[32];
    double ms;                /* summed event time                        */
    long long launches;
    double alg_bytes;
    double alg_ops;           /* flops (FFT/decode) or int ops (direct)   */
    double units;             /* work units the cost model prices the stage
                                 by: (tile, bin) items for the transforms,
                                 output pixels times SE cells stepped for
                                 the direct window, pixels times decode units
                                 for the decodes                          */
} md_stage_time;

/* Copies up to `max` stage records into `out` and the number available into
 * *n.  Host pointers. */
int md_profile_get(md_stage_time *out, int max, int *n);
int md_profile_reset(void);

/* Cost-model constants in use, in ns per work unit, into the host array
 * `dst` of capacity `n` (at least 24):
 *   [0] direct window, packed f16 form, per output pixel per SE cell
 *       stepped through, counted in 8-column-step equivalents (a narrower
 *       step's cells weighted by its higher issue cost per cell); the packed
 *       int16 form is priced at this times its issue-count ratio 580.5/461
 *   [1] the same, 32-bit form
 *   [2] direct window, per staged image word (block plus halo)
 *   [3] decode FP32, per pixel per (padded kept bins)^2
 *   [4] decode FP64, the same
 *   [5..11]  FFT stage per (tile, bin) item, FP32, lengths 16, 32, ..., 1024
 *   [12..18] the same, FP64
 *   [19..22] exact (mod p) transform stage per (tile, bin) item, lengths
 *            16, 32, 64, 128
 *   [23]     exact decode, per pixel per range bin (one block of degrees)
 * *measured = 1 if they come from the autotuner.  MD_ERR_ARG if n < 24. */
int md_cost_model(double *dst, int n, int *measured);

/* Test hook: per-bin transform-domain values of one tile just before the
 * inverse range transform, for measuring spectrum error against an FP64
 * reference.  Runs the FFT path of md_dilate (op 0) on `img` with the given
 * plan (n_t, n_r must be valid for k and L) and copies, for tile (ty, tx),
 * the values Y[m][p], m < n_r/2+1, p < T*T (T = n_t - k + 1, row-major over
 * the tile's T x T outputs starting at pixel (ty*T, tx*T)), scaled by
 * 1/n_t^2, into the HOST array `dst` as interleaved (re, im) doubles.
 * `dst` must hold 2*(n_r/2+1)*T*T doubles.  precision: 0 FP32, 1 FP64.
 * precision 2 (exact path, n_r a valid range length of that path): the n_r
 * bins Y[m][p] are residues mod 7340033 (already scaled by n_t^-2), copied
 * as (value, 0) pairs; `dst` must hold 2*n_r*T*T doubles. */
int md_debug_tile_values(const int32_t *img, int H, int W, int L, const uint8_t *se_mask,
                         const int32_t *se_offsets, int k, int n_t, int n_r, int precision,
                         int ty, int tx, double *dst);

/* Test hook for the exact tiers: from the next call on, perturb the listed
 * transform tiles.  A tile is named by its flat index over the call's
 * transform tiles: the tiles of its transform jobs in job order, each job's
 * tiles row-major (ty * tiles_x + tx).  bits[i]: 1 adds 0.4 to every decoded
 * coefficient of tile tiles[i] in the first transform pass, 2 does the same
 * in the FP64 recompute; so a tile with bit 1 fails the band and is
 * recomputed, and with bits 1|2 in FP32 (or 1 in FP64) reaches the integer
 * window.  The result must stay exact.  Calls run without a graph while the
 * list is set; indices beyond a call's tiles are ignored.  n = 0 clears the
 * list.  Host arrays, read during the call. */
int md_debug_perturb_tiles(const long long *tiles, const uint8_t *bits, int n);

/* Test hook: the per-tile tier flags of the last batch or single call
 * (bit 0: recomputed in FP64; bit 1: recomputed by the integer window), flat
 * tile order as for md_debug_perturb_tiles.  Copies min(cap, count) words to
 * the HOST array dst and the count into *n (0 when the last call had no
 * transform tile).  Waits for the library stream. */
int md_debug_tile_flags(uint32_t *dst, long long cap, long long *n);

/* Measurement hook for the choice between butterflies and matrix-core
 * products in the transform's fixed-radix stages: applies `reps` forward
 * 16-point DFTs, y_k = sum_n x_n exp(-2 pi i n k / 16), in a row to each of
 * `lines` lines of 16 complex FP32 values (interleaved re, im; DEVICE
 * arrays of 32 * lines floats, `in` and `out` may be equal), on the library
 * stream, waiting for completion.  variant 0: the vector-ALU radix-2 DFT the
 * spatial transform uses (split hi + lo FP32 constants); 1: FP32
 * matrix-core products (v_mfma_f32_16x16x4_f32, the DFT matrix rounded to
 * FP32); 2: split-bf16 matrix-core products (v_mfma_f32_16x16x32_bf16, both
 * operands as bf16 hi + lo, three products, FP32 accumulation).
 * MD_ERR_ARG unless lines is a positive multiple of 64, 1 <= reps <= 64 and
 * variant is 0, 1 or 2. */
int md_debug_dft16(int variant, const float *in, float *out, long long lines, int reps);

#ifdef __cplusplus
}
#endif

#endif /* MD_H_ */
