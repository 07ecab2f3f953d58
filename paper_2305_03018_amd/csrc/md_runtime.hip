// Host runtime behind the C ABI of include/md.h: argument checks, the
// planner / cost model, caches of twiddle tables, range tables and SE
// spectra, the stage-wise executor over device work queues, HIP-graph
// capture of whole batches, and statistics.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "md.h"
#include "md_internal.h"

namespace md {
namespace {

std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define MD_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? MD_ERR_NOMEM : MD_ERR_DEVICE,          \
                        "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define MD_TRY(expr)             \
    do {                         \
        int rc_ = (expr);        \
        if (rc_ != MD_OK) return rc_; \
    } while (0)

struct Options {
    int precision = 0;
    double band = 0.25;
    int path = 0;
    int tile = 0;
    int nr = 0;
    int sync = 1;
    int graph = 1;
    double ws_mb = 8192.0;
    int profile = 0;
    int autotune = 1;
    int stream_rows = 0;
    double stream_mb = 2048.0;
    double cache_mb = 16384.0;
    int dc_plane = 0;   // internal: every job's bin-0 plane is written (md_debug_tile_values reads it)
};

// Device buffer that only grows; freed when it is destroyed (a cache entry
// or executor going away releases its device memory).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    int ensure(size_t n) {
        if (n <= bytes) return MD_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (n == 0) return MD_OK;
        MD_HIP(hipMalloc(&p, n));
        bytes = n;
        return MD_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// Cached device objects: range tables, SE spectra (both transform
// families) and the direct window's SE tables.  They live in one cache keyed
// by their defining bytes and bounded in total size (MD_OPT_CACHE_MB):
// inserting past the bound evicts the least recently used objects that no
// cached executor references and that the current call has not touched.
struct CacheObj {
    virtual ~CacheObj() = default;
    virtual size_t bytes() const = 0;
};

struct RangeTables : CacheObj {
    DevBuf enc32, enc64, dec32, dec64, rtw32, rtw64;
    size_t bytes() const override {
        return enc32.bytes + enc64.bytes + dec32.bytes + dec64.bytes + rtw32.bytes + rtw64.bytes;
    }
};

struct SESpec : CacheObj {
    DevBuf s32, s64;
    size_t bytes() const override { return s32.bytes + s64.bytes; }
};

// Exact transform path: range-axis tables for (n, L) and an SE spectrum per
// (SE, nt, n), residues mod kNttP with Shoup companions.
struct NttRange : CacheObj {
    DevBuf enc, rpow, dec, dec_s;   // enc [n][L]; rpow [n] = w_n^e; dec [rows][dp] = n^-1 w_n^(-d m)
    int dp = 0;
    size_t bytes() const override { return enc.bytes + rpow.bytes + dec.bytes + dec_s.bytes; }
};

struct NttSpec : CacheObj {
    DevBuf spec, spec_s;            // [n][nt][nt]
    size_t bytes() const override { return spec.bytes + spec_s.bytes; }
};

// Per effective SE: the direct window's tables, and the 2-D prefix counts of
// its mask (cnt[i][j] = active cells in rows < i and columns < j, pitch
// k + 1) from which a decode derives how many window cells of a pixel lie in
// the image.
struct DirSE : CacheObj {
    DevBuf sek, sek16, sekh, rows, steps, cnt;
    int kpad = 0, nsteps = 0;
    size_t bytes() const override {
        return sek.bytes + sek16.bytes + sekh.bytes + rows.bytes + steps.bytes + cnt.bytes;
    }
};

struct CacheEntry {
    std::unique_ptr<CacheObj> obj;
    size_t bytes = 0;
    unsigned long long stamp = 0;   // call that last used it
    int refs = 0;                   // cached executors that hold its device pointers
};

// Per-job plan.
struct Plan {
    int path = kPathFFT;
    int dbl = 0;
    int nt = 0, T = 0, nr = 0, bins = 0, tiles_x = 0, tiles_y = 0;
    int fb_mode = kFbNone, nt64 = 0, T64 = 0;
    bool dec_fft = false;          // range-axis FFT decode (decode_uses_fft(nr, dbl))
    double cost_fft = 0, cost_dir = 0;
};

struct Group {
    int nt = 0, dbl = 0, big = 0;   // big: decode variant (decode groups), blocks per CU (direct groups)
    int pack = 0, sel = 0;        // direct groups: element form, SE staged in LDS
    size_t lds = 0;               // dynamic LDS per block (direct groups)
    void *slabs = nullptr;        // large-tile FFT groups: big_chunk x nt x nt complex intermediates
    long long big_chunk = 0;      // large-tile FFT groups: items per chunk of three passes
    std::vector<Seg> segs;
    long long nitems = 0;
    Seg *segs_d = nullptr;
    int grid = 0;
    // algorithmic DRAM bytes / operations of the whole launch, and the work
    // units the cost model prices it by; transform and decode groups also
    // count the in-image pixels they produce and (transforms) the complex
    // transform-domain values they write
    double alg_bytes = 0, alg_ops = 0, units = 0, pixels = 0, vol_elems = 0;
};

struct Wave {
    std::vector<Group> fft;
    std::vector<Group> dec;
};

struct Exec {
    std::vector<JobDev> jobs_h;
    std::vector<Plan> plans;
    std::vector<CacheEntry *> pins;   // cache entries whose device pointers jobs_h holds
    JobDev *jobs_d = nullptr;
    JobDev *jobs_pin = nullptr;
    hipEvent_t copy_done = nullptr;
    bool copy_pending = false;
    // direct-window launches, one per (element form, SE in LDS, blocks per CU
    // allowed by the LDS footprint, capped at 4)
    std::vector<Group> direct;
    std::vector<Wave> waves;
    DevBuf segbuf;
    // workspace: the transform-domain buffer, the large-tile groups' slabs,
    // the tile flags, the FP64-recompute and window lists, the recompute's
    // slots and slabs; carved from the caller's buffer (md_set_workspace) or
    // from ws_own
    DevBuf ws_own;
    size_t ws_need = 0;
    void *ybuf = nullptr;
    unsigned int *flags = nullptr;
    int2 *list = nullptr, *wlist = nullptr;
    double2 *slots = nullptr, *fb_slabs = nullptr;
    long long nflags = 0;
    // exact recompute, one launch per FP64 length: the per-block slot of the
    // largest job of that length and the launch's block count
    struct FbClass {
        int nt64 = 0;
        size_t slot_elems = 0;
        int grid = 0;
    };
    std::vector<FbClass> fb_classes;
    // exact window tier: pixel blocks per listed tile and the launch's blocks
    int win_pblocks = 0, win_grid = 0;
    long long fft_tiles = 0;
    int n_direct = 0, n_fft = 0;
    unsigned long long stamp = 0;   // call that last ran it
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t graph_stream = nullptr;
    ~Exec() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (copy_done) (void)hipEventDestroy(copy_done);
        if (jobs_pin) (void)hipHostFree(jobs_pin);
        if (jobs_d) (void)hipFree(jobs_d);
        segbuf.release();
        ws_own.release();
        for (CacheEntry *e : pins) --e->refs;
    }
};

// Cost model (nanoseconds of whole-GPU time).  The constants are replaced by
// measured rates when the autotuner has run on this device.
// values reported by md_cost_model and persisted in the tune file
constexpr int kCostValues = 24;

struct CostModel {
    // per (tile, bin) item, index log2(nt): FP32 / FP64
    // index 0 FP32, 1 FP64, 2 exact (mod p; lengths up to kNttMaxN)
    double fft_item[3][11] = {{0, 0, 0, 0, 2.0, 8.0, 30.0, 130.0, 700.0, 3200.0, 14000.0},
                              {0, 0, 0, 0, 5.0, 20.0, 75.0, 900.0, 3800.0, 16000.0, 70000.0},
                              {0, 0, 0, 0, 3.0, 12.0, 45.0, 200.0, 0, 0, 0}};
    // FP: per pixel * (padded bins)^2; exact: per pixel * n (one degree block)
    double dec_unit[3] = {1.5e-3, 3.0e-3, 5.0e-2};
    // direct window: per output pixel * SE cells stepped through (16-bit
    // packed / 32-bit form), and per staged image word
    double dir_cell[2] = {2.5e-5, 5.0e-5};
    double dir_stage = 2.0e-3;
    double launch = 3000.0;                  // fixed cost per job class
};

struct Ctx {
    bool inited = false;
    int device = -1;
    int cu = 256;
    hipStream_t stream = nullptr;
    Options opt;
    double2 *tw64 = nullptr;
    TwF *tw32 = nullptr;
    StatsDev *st_d = nullptr;
    StatsDev *st_h = nullptr;
    md_stats last{};
    CostModel cost;
    // cached device objects (see CacheObj), their total size, the number of
    // the current call (an object it has touched is never evicted during it)
    // and, while an executor is built, where the entries it uses are pinned
    std::unordered_map<std::string, CacheEntry> cache;
    size_t cache_bytes = 0;
    unsigned long long call_id = 0;
    std::vector<CacheEntry *> *pin_sink = nullptr;
    // caller-owned workspace (md_set_workspace); null: each executor owns its own
    void *ws_ptr = nullptr;
    size_t ws_bytes = 0;
    // perturbation test hook: (flat transform tile index, kPerturb* bits), and
    // the per-tile byte array a call built from it
    std::vector<std::pair<long long, uint8_t>> perturb;
    DevBuf perturb_d;
    uint32_t *ntw = nullptr, *ntws = nullptr;   // w_kNttTw^j and Shoup companions
    std::unordered_map<std::string, std::unique_ptr<Exec>> execs;
    // repeat-call fast path: the previous batch call's job array, the bytes
    // of its SE arrays, the options it ran with and its executor
    std::vector<md_job> last_jobs;
    std::string last_se;
    Options last_opt;
    Exec *last_exec = nullptr;
    DevBuf se_work, se_in;
    DevBuf morph_a, morph_b;      // intermediates of md_morph
    DevBuf vjob, vseg, vslabs, vy;  // volume path: job, segments, slab table, transform buffer
    std::string vtab;               // host image of what vjob / vseg / vslabs hold
    // side stream of a batch: the direct-window launches run on it beside the
    // transform path's launches (fork / join events on the library stream)
    hipStream_t s_side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // host-streamed images: upload / download streams, two band buffers per
    // direction, their events, and an accumulated range-error flag
    hipStream_t s_up = nullptr, s_down = nullptr;
    hipEvent_t ev_up[2] = {nullptr, nullptr}, ev_comp[2] = {nullptr, nullptr}, ev_down[2] = {nullptr, nullptr};
    DevBuf hs_in[2], hs_out[2], hs_flag;
    // profiling
    struct Pending {
        std::string name;
        hipEvent_t a, b;
        double bytes, ops, units;
    };
    struct Total {
        double ms = 0;
        long long launches = 0;
        double bytes = 0, ops = 0, units = 0;
    };
    std::vector<Pending> pending;
    std::map<std::string, Total> prof;
    std::vector<hipEvent_t> evpool;
    bool tuned = false, tuning = false, cost_measured = false;
};

// The context lives until the process ends and is never destroyed: its
// destructor would free device memory and graphs after the HIP runtime has
// been torn down at exit.  md_release frees everything explicitly.
Ctx &g = *new Ctx;

// arithmetic mod kNttP on the host (table generation)
uint32_t pmul(uint64_t a, uint64_t b) { return (uint32_t)(a * b % kNttP); }
uint32_t ppow(uint64_t a, uint64_t e) {
    uint64_t r = 1;
    a %= kNttP;
    while (e) {
        if (e & 1) r = r * a % kNttP;
        a = a * a % kNttP;
        e >>= 1;
    }
    return (uint32_t)r;
}
uint32_t pinv(uint32_t a) { return ppow(a, kNttP - 2); }
uint32_t shoup(uint32_t w) { return (uint32_t)(((uint64_t)w << 32) / kNttP); }

// Smallest range length n >= nmin that divides kNttP - 1 = 7 * 2^20 (a power
// of two or 7 times one), 0 if it would exceed kNttMaxNr.
int ntt_length(long long nmin) {
    int best = 0;
    for (int a = 0; a <= 20; ++a)
        for (int c : {1, 7}) {
            const long long n = (long long)c << a;
            if (n >= nmin && n <= kNttMaxNr && (best == 0 || n < best)) best = (int)n;
        }
    return best;
}

int ilog2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

int init() {
    int dev = 0;
    MD_HIP(hipGetDevice(&dev));
    if (g.inited && g.device == dev) return MD_OK;
    if (g.inited && g.device != dev)
        return fail(MD_ERR_UNSUPPORTED, "the library was initialised on device %d, now %d is current; call md_release first",
                    g.device, dev);
    hipDeviceProp_t prop;
    MD_HIP(hipGetDeviceProperties(&prop, dev));
    g.cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    MD_HIP(hipMalloc(&g.tw64, sizeof(double2) * kTwN));
    MD_HIP(hipMalloc(&g.tw32, sizeof(TwF) * kTwN));
    MD_HIP(hipMalloc(&g.st_d, sizeof(StatsDev)));
    MD_HIP(hipHostMalloc((void **)&g.st_h, sizeof(StatsDev), 0));
    MD_HIP(launch_twiddles(g.tw64, g.tw32, nullptr));
    {
        // spatial twiddles of the exact path: powers of a primitive
        // kNttTw-th root of unity mod kNttP
        std::vector<uint32_t> w(kNttTw), ws(kNttTw);
        const uint32_t root = ppow(kNttG, (kNttP - 1) / kNttTw);
        uint32_t x = 1;
        for (int j = 0; j < kNttTw; ++j) {
            w[j] = x;
            ws[j] = shoup(x);
            x = pmul(x, root);
        }
        MD_HIP(hipMalloc(&g.ntw, sizeof(uint32_t) * kNttTw));
        MD_HIP(hipMalloc(&g.ntws, sizeof(uint32_t) * kNttTw));
        MD_HIP(hipMemcpy(g.ntw, w.data(), sizeof(uint32_t) * kNttTw, hipMemcpyHostToDevice));
        MD_HIP(hipMemcpy(g.ntws, ws.data(), sizeof(uint32_t) * kNttTw, hipMemcpyHostToDevice));
    }
    MD_HIP(launch_zero(g.st_d, sizeof(StatsDev), nullptr));
    MD_HIP(hipStreamCreateWithFlags(&g.s_side, hipStreamNonBlocking));
    MD_HIP(hipEventCreateWithFlags(&g.ev_fork, hipEventDisableTiming));
    MD_HIP(hipEventCreateWithFlags(&g.ev_join, hipEventDisableTiming));
    MD_HIP(hipDeviceSynchronize());
    g.device = dev;
    g.inited = true;
    // registered after the HIP runtime is up, so it runs before the runtime's
    // own exit handlers: graphs and buffers are released while HIP still works
    static bool exit_hook = false;
    if (!exit_hook) {
        exit_hook = true;
        atexit([] { md_release(); });
    }
    return MD_OK;
}

// ---------------------------------------------------------------------------
// caches
// ---------------------------------------------------------------------------
// Key of a cached object: a tag for its kind, then its defining values.
template <class... A> std::string cache_key(char tag, const A &...vals) {
    std::string k(1, tag);
    (k.append((const char *)&vals, sizeof vals), ...);
    return k;
}

void cache_pin(CacheEntry &e) {
    e.stamp = g.call_id;
    if (g.pin_sink) {
        ++e.refs;
        g.pin_sink->push_back(&e);
    }
}

// The cached object under `key`, marked as used by the current call and
// pinned to the executor being built; nullptr if absent.
template <class T> T *cache_get(const std::string &key) {
    auto it = g.cache.find(key);
    if (it == g.cache.end()) return nullptr;
    cache_pin(it->second);
    return static_cast<T *>(it->second.obj.get());
}

// Makes room for `need` more bytes under MD_OPT_CACHE_MB: evicts, least
// recently used first, objects that no cached executor pins and the current
// call has not touched; if that is not enough, drops the cached executors
// (they are rebuilt on their next call) and evicts again.  An object larger
// than the bound still goes in.
int cache_reserve(size_t need) {
    const double cap = g.opt.cache_mb * 1024.0 * 1024.0;
    if ((double)(g.cache_bytes + need) <= cap) return MD_OK;
    MD_HIP(hipDeviceSynchronize());   // evicted objects may still be read by enqueued work
    for (int pass = 0; pass < 2 && (double)(g.cache_bytes + need) > cap; ++pass) {
        if (pass == 1) g.execs.clear(), g.last_exec = nullptr;
        std::vector<std::pair<unsigned long long, std::string>> cand;
        for (auto &kv : g.cache)
            if (kv.second.refs == 0 && kv.second.stamp != g.call_id) cand.push_back({kv.second.stamp, kv.first});
        std::sort(cand.begin(), cand.end());
        for (auto &c : cand) {
            if ((double)(g.cache_bytes + need) <= cap) break;
            auto it = g.cache.find(c.second);
            g.cache_bytes -= it->second.bytes;
            g.cache.erase(it);
        }
    }
    return MD_OK;
}

// Stores a newly built object and pins it as cache_get does.
template <class T> T *cache_put(const std::string &key, std::unique_ptr<T> obj) {
    T *p = obj.get();
    CacheEntry &e = g.cache[key];
    e.obj = std::move(obj);
    e.bytes = p->bytes();
    g.cache_bytes += e.bytes;
    cache_pin(e);
    return p;
}

// Brings an entry's recorded size up to date after buffers were added to it.
void cache_resize(const std::string &key) {
    auto it = g.cache.find(key);
    if (it == g.cache.end()) return;
    g.cache_bytes -= it->second.bytes;
    it->second.bytes = it->second.obj->bytes();
    g.cache_bytes += it->second.bytes;
}

int get_range(int nr, int L, RangeTables **out) {
    const std::string key = cache_key('R', nr, L);
    if ((*out = cache_get<RangeTables>(key))) return MD_OK;
    auto rt = std::make_unique<RangeTables>();
    const size_t bins = nr / 2 + 1;
    const size_t ne = bins * (size_t)L, nd = (size_t)dec_pitch(nr) * dec_pitch(nr);
    MD_TRY(cache_reserve((ne + nd + bins) * (sizeof(float2) + sizeof(double2))));
    MD_TRY(rt->enc32.ensure(ne * sizeof(float2)));
    MD_TRY(rt->enc64.ensure(ne * sizeof(double2)));
    MD_TRY(rt->dec32.ensure(nd * sizeof(float2)));
    MD_TRY(rt->dec64.ensure(nd * sizeof(double2)));
    MD_TRY(rt->rtw32.ensure(bins * sizeof(float2)));
    MD_TRY(rt->rtw64.ensure(bins * sizeof(double2)));
    MD_HIP(launch_range_tables(nr, L, (float2 *)rt->enc32.p, (double2 *)rt->enc64.p, (float2 *)rt->dec32.p,
                               (double2 *)rt->dec64.p, (float2 *)rt->rtw32.p, (double2 *)rt->rtw64.p, g.stream));
    *out = cache_put(key, std::move(rt));
    return MD_OK;
}

// Effective SE as the transform path uses it: the SE itself for dilation,
// its reflection for erosion (duality, Sec. 2.1).
struct SEData {
    int k = 0;
    std::vector<uint8_t> mask;
    std::vector<int32_t> off;   // zero where masked out
    int maxoff = 0;
    int ncells = 0;
    std::string key;
    double dir_cells[2] = {0, 0};   // cells the direct window steps through per output pixel (packed, 32-bit)
};

// Column steps of the packed direct window for one SE, in its correlation
// order (row i, column j <-> SE cell (k-1-i, k-1-j)).  Each 2-column group g
// (columns 2g, 2g+1) has the range of SE row pairs (2s, 2s+1) with an active
// cell there.  A step of 8, 4 or 2 columns runs over the union of its groups'
// ranges (8- and 4-column steps start at a multiple of 4); the steps are
// chosen by dynamic programming over the groups to minimise the issue cost of
// the window, kDirPairCost per row pair and step width (instructions of one
// pair in the f16 kernel's unrolled loops), so neighbouring groups with nearly
// equal ranges share a wider step even where that covers a few masked cells.
// Each step is {first column, kind, first pair, last pair}, kind 0/1/2 =
// 8/4/2 columns, 3 = 2 columns at 2 mod 4.  The int16 form (one max per SE
// column rather than half a three-way max) issues 580.5 / 311.5 / 177.5 and
// takes the same steps.
constexpr double kDirPairCost[3] = {461.0, 250.0, 146.0};   // 8, 4, 2 columns
constexpr double kDirPairCostI16 = 580.5;                    // 8 columns, int16 form

// row pairs a step over pairs s0..s1 runs (the last, even SE row of an odd k
// alone counts as one)
int dir_pairs(int k, int s0, int s1) {
    const int last = (k - 1) / 2, sfull = (k - 3) / 2;
    return std::max(0, std::min(s1, sfull) - s0 + 1) + (s1 == last && 2 * last + 1 == k ? 1 : 0);
}

std::vector<int32_t> dir_steps(const SEData &se) {
    const int k = se.k, kpad = (k + kDirRX - 1) / kDirRX * kDirRX, ng = kpad / 2;
    std::vector<int> lo(ng, k), hi(ng, -1);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            if (se.mask[(size_t)(k - 1 - i) * k + (k - 1 - j)]) {
                lo[j / 2] = std::min(lo[j / 2], i / 2);
                hi[j / 2] = std::max(hi[j / 2], i / 2);
            }
    // best[g]: least cost covering groups [0, g); from[g]: the step that ends
    // there (width in groups, 0 = an empty group skipped)
    std::vector<double> best(ng + 1, INFINITY);
    std::vector<int> from(ng + 1, -1);
    best[0] = 0;
    for (int g = 0; g < ng; ++g) {
        if (!(best[g] < INFINITY)) continue;
        if (lo[g] > hi[g] && best[g] < best[g + 1]) {
            best[g + 1] = best[g];
            from[g + 1] = 0;
        }
        for (int w : {1, 2, 4}) {   // groups per step: 2, 4, 8 columns
            if (g + w > ng || (w > 1 && (2 * g) % 4 != 0)) continue;
            int s0 = k, s1 = -1;
            for (int q = g; q < g + w; ++q) {
                s0 = std::min(s0, lo[q]);
                s1 = std::max(s1, hi[q]);
            }
            if (s0 > s1) continue;
            const double c = best[g] + kDirPairCost[w == 4 ? 0 : w == 2 ? 1 : 2] * dir_pairs(k, s0, s1);
            if (c < best[g + w]) {
                best[g + w] = c;
                from[g + w] = w;
            }
        }
    }
    std::vector<int32_t> st;
    for (int g = ng; g > 0;) {
        const int w = from[g];
        if (w <= 0) {
            --g;
            continue;
        }
        const int g0 = g - w;
        int s0 = k, s1 = -1;
        for (int q = g0; q < g; ++q) {
            s0 = std::min(s0, lo[q]);
            s1 = std::max(s1, hi[q]);
        }
        const int c = 2 * g0, kind = w == 4 ? 0 : w == 2 ? 1 : (c % 4 == 2 ? 3 : 2);
        st.insert(st.begin(), {c, kind, s0, s1});
        g = g0;
    }
    return st;
}

// Work of the direct window per output pixel.  Packed form: in 8-column-step
// equivalents -- each step's row pairs weighted by their issue cost relative
// to an 8-column pair of 16 cells -- so that one calibrated per-cell cost
// prices every step width.  32-bit form: each row's active span from its
// first column rounded down to 8, in 8-column steps.
void dir_work(SEData &se) {
    const int k = se.k;
    const std::vector<int32_t> st = dir_steps(se);
    double e16 = 0;
    for (size_t i = 0; i < st.size(); i += 4) {
        const int kind = st[i + 1];
        const double w = kDirPairCost[kind == 0 ? 0 : kind == 1 ? 1 : 2] / kDirPairCost[0];
        e16 += 16.0 * w * dir_pairs(k, st[i + 2], st[i + 3]);
    }
    std::vector<int> lo(k, k), hi(k, -1);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            if (se.mask[(size_t)(k - 1 - i) * k + (k - 1 - j)]) {
                lo[i] = std::min(lo[i], j);
                hi[i] = std::max(hi[i], j);
            }
    double e32 = 0;
    for (int i = 0; i < k; ++i) {
        if (lo[i] > hi[i]) continue;
        const int jb = lo[i] & ~(kDirRX - 1);
        e32 += (double)kDirRX * ((hi[i] - jb) / kDirRX + 1);
    }
    se.dir_cells[0] = e16;
    se.dir_cells[1] = e32;
}

// Image words the direct window stages per output pixel (block plus halo).
double dir_staged(int k, int pack) {
    const int bh = direct_block_rows(pack), kpad = (k + kDirRX - 1) / kDirRX * kDirRX;
    return (double)(bh + k - 1) * (kDirBW + kpad) / ((double)bh * kDirBW);
}

// The per-unit costs are measured with the GPU full, several blocks sharing
// each CU.  A job that runs alone (`lone`) and has fewer blocks than CUs
// leaves CUs idle: it is priced as one block per CU (a block alone on a CU
// runs about as many times faster as the blocks it would otherwise share the
// CU with, so one round of resident blocks would overprice it).
// Per-cell cost of a direct_form(): the packed f16 form is the calibrated
// one; the int16 form issues one max per SE column where f16 issues half a
// three-way max, kDirPairCostI16 / kDirPairCost more per 8-column pair.
double dir_cell_cost(int form) {
    return form == 2 ? g.cost.dir_cell[0] : form == 1 ? g.cost.dir_cell[0] * (kDirPairCostI16 / kDirPairCost[0])
                                                      : g.cost.dir_cell[1];
}

// The per-cell cost is calibrated with 4 packed blocks per CU.  An SE whose
// LDS footprint leaves fewer blocks per CU has fewer waves to hide latency
// with: measured on 2048^2 images, k = 95 (2 blocks per CU) runs 3% and
// k = 127 (1 block per CU) 10% above the calibrated figure.
double dir_occupancy(int k, int form) {
    if (!form) return 1.0;
    const int kpad = (k + kDirRX - 1) / kDirRX * kDirRX;
    const size_t per_cu = kLdsBytes / direct_lds_bytes(k, kpad, form, 0);
    return per_cu >= 3 ? 1.0 : per_cu == 2 ? 1.03 : 1.10;
}

double dir_block_cost(int k, const SEData &se, int form) {
    return dir_staged(k, form) * g.cost.dir_stage +
           se.dir_cells[form ? 0 : 1] * dir_cell_cost(form) * dir_occupancy(k, form);
}

double dir_cost(const md_job &j, const SEData &se, int pack, bool lone = false) {
    double px = (double)j.H * j.W;
    if (lone) px = std::max(px, (double)g.cu * direct_block_rows(pack) * kDirBW);
    return px * dir_block_cost(j.k, se, pack);
}

// Kept bins rounded up as the decode variant for that count accumulates them.
double dec_padded_bins(int bins, int dbl);

// Transform-domain layout of a plan's tiles (JobDev::ybs): blocks of 16
// pixels with their bins contiguous for the range-axis FFT decode, which
// reads all bins of a few pixels; bin-major otherwise.
int plan_ybs(const Plan &p) { return p.dec_fft ? p.bins * 16 : 0; }

// Decode work per pixel in the dense decode's units (padded bins squared).
// The range-axis FFT decode is priced at kDecFftRatio[precision] of those
// units per nr log2 nr (time per nr log2 nr over the dense decode's time per
// unit at nr - 1, on 2048^2 images: FP32 1.37 at nr = 128, 1.08 at 256,
// 0.73 at 512, 0.85 at 1024; FP64 0.88, 0.55, 0.49, 0.46).  The FP32
// lengths 3 2^a take 1.4 times that (1.19 at 192, 1.14 at 384, 1.0 at 768),
// the lengths 5 2^a 1.3 times (1.38 at 160, 1.05 at 320, 0.78 at 640).
constexpr double kDecFftRatio[2] = {0.8, 0.5};
double dec_units(int nr, int dbl) {
    if (decode_uses_fft(nr, dbl))
        return kDecFftRatio[dbl ? 1 : 0] * (is_pow2c(nr) ? 1.0 : nr % 3 == 0 ? 1.4 : 1.3) * nr *
               std::log2((double)nr);
    const double pb = dec_padded_bins(nr / 2 + 1, dbl);
    return pb * pb;
}

double dec_padded_bins(int bins, int dbl) {
    switch (decode_group_variant(bins, dbl)) {
        case 4: return 4;
        case 0: return 8;
        case 1: return 12;
        case 2: return 24;
        default: {
            const int b = dbl ? 8 : 16;
            return (double)((bins + b - 1) / b * b);
        }
    }
}

void make_se(const uint8_t *mask, const int32_t *off, int k, int op, SEData &se) {
    se.k = k;
    se.mask.assign((size_t)k * k, 0);
    se.off.assign((size_t)k * k, 0);
    se.maxoff = 0;
    se.ncells = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            const int si = op ? (k - 1 - i) : i, sj = op ? (k - 1 - j) : j;
            const size_t src = (size_t)si * k + sj, dst = (size_t)i * k + j;
            if (mask[src]) {
                se.mask[dst] = 1;
                se.off[dst] = off[src];
                se.maxoff = std::max(se.maxoff, (int)off[src]);
                ++se.ncells;
            }
        }
    se.key.assign((const char *)&k, sizeof k);
    se.key.append((const char *)se.mask.data(), se.mask.size());
    se.key.append((const char *)se.off.data(), se.off.size() * sizeof(int32_t));
    dir_work(se);
}

int get_spectrum(const SEData &se, int nt, int nr, bool need32, bool need64, SESpec **out) {
    std::string key = "S" + se.key;
    key.append((const char *)&nt, sizeof nt);
    key.append((const char *)&nr, sizeof nr);
    SESpec *sp = cache_get<SESpec>(key);
    if (sp && (!need32 || sp->s32.p) && (!need64 || sp->s64.p)) {
        *out = sp;
        return MD_OK;
    }
    const int k = se.k, bins = nr / 2 + 1;
    const size_t nspec = (size_t)bins * nt * nt;
    const bool add32 = need32 && !(sp && sp->s32.p), add64 = need64 && !(sp && sp->s64.p);
    MD_TRY(cache_reserve(nspec * ((add32 ? sizeof(float2) : 0) + (add64 ? sizeof(double2) : 0))));
    if (!sp) sp = cache_put(key, std::make_unique<SESpec>());
    if (add32) MD_TRY(sp->s32.ensure(nspec * sizeof(float2)));
    if (add64) MD_TRY(sp->s64.ensure(nspec * sizeof(double2)));
    cache_resize(key);
    MD_TRY(g.se_work.ensure((size_t)bins * k * nt * sizeof(double2)));
    const size_t kk = (size_t)k * k;
    MD_TRY(g.se_in.ensure(kk * (sizeof(int32_t) + 1) + 64));
    MD_HIP(hipStreamSynchronize(g.stream));   // se_in may still be read by an earlier build
    int32_t *off_d = (int32_t *)g.se_in.p;
    uint8_t *mask_d = (uint8_t *)((char *)g.se_in.p + kk * sizeof(int32_t));
    MD_HIP(hipMemcpy(off_d, se.off.data(), kk * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(mask_d, se.mask.data(), kk, hipMemcpyHostToDevice));
    MD_HIP(launch_se_spectrum(mask_d, off_d, k, nt, nr, g.tw64, (double2 *)g.se_work.p,
                              sp->s64.p ? (double2 *)sp->s64.p : nullptr, sp->s32.p ? (float2 *)sp->s32.p : nullptr,
                              g.stream));
    MD_HIP(hipStreamSynchronize(g.stream));
    *out = sp;
    return MD_OK;
}

// Range-axis tables of the exact path for range length n and L grey values:
// enc[m][v] = w_n^(v m), rpow[e] = w_n^e, dec[m][d] = n^-1 w_n^(-d m) with
// pitch dp = n rounded up to 8 and rows padded to a multiple of 16 (zeros).
int get_nrange(int n, int L, NttRange **out) {
    const std::string key = cache_key('N', n, L);
    if ((*out = cache_get<NttRange>(key))) return MD_OK;
    auto rt = std::make_unique<NttRange>();
    const uint32_t wn = ppow(kNttG, (kNttP - 1) / n), ninv = pinv((uint32_t)n);
    std::vector<uint32_t> pw(n);
    uint32_t x = 1;
    for (int e = 0; e < n; ++e) {
        pw[e] = x;
        x = pmul(x, wn);
    }
    std::vector<uint32_t> enc((size_t)n * L);
    for (int m = 0; m < n; ++m)
        for (int v = 0; v < L; ++v) enc[(size_t)m * L + v] = pw[(size_t)((long long)v * m % n)];
    rt->dp = (n + 7) / 8 * 8;
    const int rows = (n + 15) / 16 * 16;
    std::vector<uint32_t> dec((size_t)rows * rt->dp, 0), decs((size_t)rows * rt->dp, 0);
    for (int m = 0; m < n; ++m)
        for (int d = 0; d < n; ++d) {
            const uint32_t w = pmul(ninv, pw[(size_t)((n - (long long)d * m % n) % n)]);
            dec[(size_t)m * rt->dp + d] = w;
            decs[(size_t)m * rt->dp + d] = shoup(w);
        }
    MD_TRY(cache_reserve((enc.size() + pw.size() + dec.size() + decs.size()) * 4));
    MD_TRY(rt->enc.ensure(enc.size() * 4));
    MD_TRY(rt->rpow.ensure(pw.size() * 4));
    MD_TRY(rt->dec.ensure(dec.size() * 4));
    MD_TRY(rt->dec_s.ensure(decs.size() * 4));
    MD_HIP(hipMemcpy(rt->enc.p, enc.data(), enc.size() * 4, hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(rt->rpow.p, pw.data(), pw.size() * 4, hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(rt->dec.p, dec.data(), dec.size() * 4, hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(rt->dec_s.p, decs.data(), decs.size() * 4, hipMemcpyHostToDevice));
    *out = cache_put(key, std::move(rt));
    return MD_OK;
}

// SE spectrum of the exact path at spatial length nt and range length n,
// scaled by nt^-2.
int get_nspectrum(const SEData &se, int nt, int n, const NttRange *rt, NttSpec **out) {
    std::string key = "P" + se.key;
    key.append((const char *)&nt, sizeof nt);
    key.append((const char *)&n, sizeof n);
    if ((*out = cache_get<NttSpec>(key))) return MD_OK;
    auto sp = std::make_unique<NttSpec>();
    const int k = se.k;
    const size_t nspec = (size_t)n * nt * nt;
    MD_TRY(cache_reserve(nspec * 8));
    MD_TRY(sp->spec.ensure(nspec * 4));
    MD_TRY(sp->spec_s.ensure(nspec * 4));
    MD_TRY(g.se_work.ensure((size_t)n * k * nt * 4));
    const size_t kk = (size_t)k * k;
    MD_TRY(g.se_in.ensure(kk * (sizeof(int32_t) + 1) + 64));
    MD_HIP(hipStreamSynchronize(g.stream));   // se_in may still be read by an earlier build
    int32_t *off_d = (int32_t *)g.se_in.p;
    uint8_t *mask_d = (uint8_t *)((char *)g.se_in.p + kk * sizeof(int32_t));
    MD_HIP(hipMemcpy(off_d, se.off.data(), kk * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(mask_d, se.mask.data(), kk, hipMemcpyHostToDevice));
    const uint32_t scale = pinv(pmul((uint32_t)nt, (uint32_t)nt));
    MD_HIP(launch_ntt_se_spectrum(mask_d, off_d, k, nt, n, (const uint32_t *)rt->rpow.p, g.ntw, scale,
                                  (uint32_t *)g.se_work.p, (uint32_t *)sp->spec.p, (uint32_t *)sp->spec_s.p,
                                  g.stream));
    MD_HIP(hipStreamSynchronize(g.stream));
    *out = cache_put(key, std::move(sp));
    return MD_OK;
}

// IEEE half-precision bits of an integer 0 <= v <= 2048 (exact: at most 11
// significant bits).
uint32_t f16_bits(int v) {
    if (v <= 0) return 0;
    int e = 0;
    while ((v >> (e + 1)) != 0) ++e;                       // 2^e <= v < 2^(e+1)
    const uint32_t frac = e <= 10 ? ((uint32_t)v << (10 - e)) & 0x3ffu : ((uint32_t)v >> (e - 10)) & 0x3ffu;
    return (uint32_t)(e + 15) << 10 | frac;
}

// Host images of the direct window's SE tables: correlation-order offsets
// (the effective SE reflected) as int32 and as packed 16-bit pairs (int16
// and f16), each row's span of active cells, the column steps of the packed
// form, and the 2-D prefix counts of the mask.
struct DirTables {
    int kpad = 0;
    std::vector<int32_t> h, h16, hh, rows, steps, cnt;
};

void dir_tables(const SEData &se, DirTables &t) {
    const int k = se.k;
    t.kpad = (k + kDirRX - 1) / kDirRX * kDirRX;
    // 16 words of padding after the last row: the direct kernel prefetches
    // past the end of a row's active span; the packed form also reads one
    // whole row past the SE (SE row k, all minus infinity) ahead of use
    t.h.assign((size_t)k * t.kpad + 16, kNeg);
    const uint32_t neg16 = 0xC000C000u;   // -16384 in both lanes
    const uint32_t negh = 0xFC00FC00u;    // f16 minus infinity in both lanes
    t.h16.assign((size_t)(k + 1) * t.kpad + 16, (int32_t)neg16);
    t.hh.assign(t.h16.size(), (int32_t)negh);
    t.rows.assign((size_t)2 * k, 0);
    for (int i = 0; i < k; ++i) {
        int lo = k, hi = -1;
        for (int j = 0; j < k; ++j) {
            const size_t src = (size_t)(k - 1 - i) * k + (k - 1 - j);
            if (!se.mask[src]) continue;
            const int32_t b = se.off[src];
            t.h[(size_t)i * t.kpad + j] = b;
            t.h16[(size_t)i * t.kpad + j] = (int32_t)(((uint32_t)b & 0xffffu) * 0x10001u);
            // offsets above 2048 never reach the f16 form (direct_form)
            if (b <= 2048) t.hh[(size_t)i * t.kpad + j] = (int32_t)(f16_bits(b) * 0x10001u);
            lo = std::min(lo, j);
            hi = std::max(hi, j);
        }
        t.rows[2 * i] = lo;
        t.rows[2 * i + 1] = hi;
    }
    t.steps = dir_steps(se);
    // prefix counts of the mask
    t.cnt.assign((size_t)(k + 1) * (k + 1), 0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j)
            t.cnt[(size_t)(i + 1) * (k + 1) + j + 1] = t.cnt[(size_t)i * (k + 1) + j + 1] +
                                                       t.cnt[(size_t)(i + 1) * (k + 1) + j] -
                                                       t.cnt[(size_t)i * (k + 1) + j] +
                                                       (se.mask[(size_t)i * k + j] ? 1 : 0);
}

// The direct window's SE tables on the device (cached per effective SE).
int get_dirse(const SEData &se, DirSE **out) {
    const std::string key = "D" + se.key;
    if ((*out = cache_get<DirSE>(key))) return MD_OK;
    auto d = std::make_unique<DirSE>();
    DirTables t;
    dir_tables(se, t);
    d->kpad = t.kpad;
    d->nsteps = (int)t.steps.size() / 4;
    MD_TRY(cache_reserve((t.h.size() + t.h16.size() + t.hh.size() + t.rows.size() + t.steps.size() + t.cnt.size()) * 4));
    MD_TRY(d->sek.ensure(t.h.size() * sizeof(int32_t)));
    MD_TRY(d->sek16.ensure(t.h16.size() * sizeof(int32_t)));
    MD_TRY(d->sekh.ensure(t.hh.size() * sizeof(int32_t)));
    MD_TRY(d->rows.ensure(t.rows.size() * sizeof(int32_t)));
    MD_TRY(d->steps.ensure(std::max<size_t>(1, t.steps.size()) * sizeof(int32_t)));
    if (!t.steps.empty())
        MD_HIP(hipMemcpy(d->steps.p, t.steps.data(), t.steps.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(d->sek.p, t.h.data(), t.h.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(d->sek16.p, t.h16.data(), t.h16.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(d->sekh.p, t.hh.data(), t.hh.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(d->rows.p, t.rows.data(), t.rows.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_TRY(d->cnt.ensure(t.cnt.size() * sizeof(int32_t)));
    MD_HIP(hipMemcpy(d->cnt.p, t.cnt.data(), t.cnt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    *out = cache_put(key, std::move(d));
    return MD_OK;
}

// ---------------------------------------------------------------------------
// planner
// ---------------------------------------------------------------------------
int check_job(const md_job &j) {
    if (!j.img || !j.out) return fail(MD_ERR_ARG, "null image or output pointer");
    if ((const void *)j.img == (const void *)j.out) return fail(MD_ERR_ARG, "output must not alias the input");
    if (!j.se_mask || !j.se_offsets) return fail(MD_ERR_ARG, "null SE array");
    if (j.H < 1 || j.W < 1) return fail(MD_ERR_ARG, "image shape %dx%d", j.H, j.W);
    if ((long long)j.H * j.W > 0x7fffffffLL) return fail(MD_ERR_ARG, "image has more than 2^31-1 pixels");
    if (j.L < 2 || j.L > (1 << 24)) return fail(MD_ERR_ARG, "L=%d outside [2, 2^24]", j.L);
    if (j.k < 1 || j.k > kMaxN - 1 || (j.k % 2) == 0) return fail(MD_ERR_ARG, "k=%d must be odd in [1,%d]", j.k, kMaxN - 1);
    if (j.op != 0 && j.op != 1) return fail(MD_ERR_ARG, "op=%d must be 0 (dilation) or 1 (erosion)", j.op);
    for (int q = 0; q < j.k * j.k; ++q)
        if (j.se_mask[q] && (j.se_offsets[q] < 0 || j.se_offsets[q] > (1 << 24)))
            return fail(MD_ERR_RANGE, "SE offset %d at cell %d outside [0, 2^24]", j.se_offsets[q], q);
    return MD_OK;
}

// Floor of a lone transform launch: one item per CU for the LDS-resident
// kernels (bound by the ALU and the LDS, so an item alone on a CU runs
// correspondingly faster).  A large-tile item spreads over its nt^2 / 4096
// line batches in each of its three passes, so items enough for four blocks
// per CU fill the GPU.
double lone_items(int nt, int dbl) {
    if (dbl != kPrecNTT && big_tile(nt, dbl)) return std::max(1.0, 4.0 * g.cu * 4096.0 / ((double)nt * nt));
    return g.cu;
}

double fft_cost(const md_job &j, int nt, int nr, int dbl, bool lone = false) {
    const int T = nt - j.k + 1;
    if (T < 1) return INFINITY;
    const long long tiles = (long long)((j.H + T - 1) / T) * ((j.W + T - 1) / T);
    if (dbl == kPrecNTT) {
        if (nt > kNttMaxN) return INFINITY;
        const double item = g.cost.fft_item[2][ilog2i(nt)];
        if (item <= 0) return INFINITY;
        double items = (double)tiles * nr;
        if (lone) items = std::max(items, lone_items(nt, dbl));
        return items * item + (double)tiles * T * T * nr * g.cost.dec_unit[2];
    }
    const int bins = nr / 2 + 1;
    const double item = g.cost.fft_item[dbl][ilog2i(nt)];
    if (item <= 0) return INFINITY;
    // bin 0 is written in closed form (its plane is priced with the decode)
    double items = (double)tiles * (bins - 1);
    if (lone) items = std::max(items, lone_items(nt, dbl));
    return items * item + (double)tiles * T * T * dec_units(nr, dbl) * g.cost.dec_unit[dbl];
}

// Worst-case rounding error of a decoded coefficient from the FP32 pass of
// one tile: |a|_2 |b|_2 3 log2(nt^2 nr) (u + beta) with u = 2^-24, the tile
// umbra's 2-norm |a|_2 <= nt (one unit entry per pixel at each bin), the SE
// umbra's |b|_2 = sqrt(|B|) (one per SE cell), the spatial stages' twiddle
// error beta ~ 0 (split hi/lo twiddles) and the range stages' beta ~ u
// (single-float twiddles in the decode), so the range stages count twice.
// The band check is sound while the true error stays below 0.75 (a larger
// one can round to a wrong integer unflagged); FP32 plans are kept where
// this bound is at most kFp32BoundMax.
double fp32_error_bound(int nt, int nr, long long ncells) {
    return nt * std::sqrt((double)ncells) * 3.0 * (std::log2((double)nt * nt) + 2.0 * std::log2((double)nr)) *
           std::ldexp(1.0, -24);
}
constexpr double kFp32BoundMax = 0.25;

int plan_job(const md_job &j, const SEData &se, Plan &p, bool lone) {
    const long long nr_min = (long long)(j.L - 1) + se.maxoff + 1;
    int nr = (int)std::min<long long>(nr_min, 1 << 30);
    if (g.opt.nr > 0) {
        if (g.opt.nr < nr_min)
            return fail(MD_ERR_ARG, "forced range length %d < (L-1)+max offset+1 = %lld", g.opt.nr, nr_min);
        nr = g.opt.nr;
    }
    int dbl = g.opt.precision;   // kPrecFP32 / kPrecFP64 / kPrecNTT
    bool ntt_ok = true;
    if (dbl == kPrecNTT) {
        // a range length that divides p - 1 (forced lengths must, too)
        if (g.opt.nr > 0) {
            if (ntt_length(nr) != nr)
                return fail(MD_ERR_ARG, "range length %d of the exact path must be 2^a or 7*2^a, <= %d", nr, kNttMaxNr);
        } else {
            nr = ntt_length(nr_min);
        }
        ntt_ok = nr > 0;
    }
    p = Plan();
    const int form = direct_form((long long)(j.L - 1) + se.maxoff);
    const bool dir_ok = j.k <= kMaxDirectK;
    p.cost_dir = dir_ok ? dir_cost(j, se, form, lone) : INFINITY;
    const bool fft_ok = nr_min <= 4096 && se.ncells > 0 && ntt_ok;
    // transform plan: best spatial length and, on the FP paths, range length
    // by the cost model: the smallest range length, or the next lengths with
    // a range-axis FFT decode (2^a, 3 2^a, 5 2^a, and the shortest length with
    // any FFT decode), at the price of more kept bins.  Past 128 they are offered always: on 2048^2 images the power of
    // two wins from about 150 on (FP32 12.9 against 6.5 ms at 230, FP64 42.1
    // against 17.6 ms).  Up to 128 they are offered only when the smallest
    // length has no FFT decode (dense decode, 4 nr bins flops a pixel,
    // against the short decode's one read of the bins): from one FFT-decoded
    // length to a longer one the extra bins cost more than the decode saves.
    // FP32 candidates whose error bound exceeds kFp32BoundMax are skipped; if
    // none is left the job runs in FP64.
    double best = INFINITY;
    int best_nt = 0, best_nr = nr;
    auto search = [&](int prec) {
        int nrs[5] = {nr, 0, 0, 0, 0};
        if (prec != kPrecNTT && g.opt.nr <= 0 && (nr > 128 || !decode_uses_fft(nr, prec))) {
            int nr2 = 1;
            while (nr2 < nr) nr2 <<= 1;
            if (nr2 != nr && decode_uses_fft(nr2, prec)) nrs[1] = nr2;
            int nr3 = 6;
            while (nr3 < nr) nr3 <<= 1;
            if (nr3 != nr && nr3 < nr2 && decode_uses_fft(nr3, prec)) nrs[2] = nr3;
            int nr5 = 10;
            while (nr5 < nr) nr5 <<= 1;
            if (nr5 != nr && nr5 < nr2 && nr5 < nr3 && decode_uses_fft(nr5, prec)) nrs[3] = nr5;
            // and the shortest length above nr with any FFT decode (the short
            // decode's lengths 2M, M with no prime factor above 5)
            for (int n = nr + 1; n < 2 * nr && n <= 4096; ++n)
                if (decode_uses_fft(n, prec)) {
                    if (n != nrs[1] && n != nrs[2] && n != nrs[3]) nrs[4] = n;
                    break;
                }
        }
        best = INFINITY;
        best_nt = 0;
        best_nr = nr;
        for (int c = 0; c < 5; ++c)
            for (int nt = 16; fft_ok && nrs[c] > 0 && nt <= kMaxN; nt *= 2) {
                if (g.opt.tile > 0 && nt != g.opt.tile) continue;
                if (prec == kPrecFP32 && fp32_error_bound(nt, nrs[c], se.ncells) > kFp32BoundMax) continue;
                const double cst = fft_cost(j, nt, nrs[c], prec, lone);
                if (cst < best) {
                    best = cst;
                    best_nt = nt;
                    best_nr = nrs[c];
                }
            }
    };
    search(dbl);
    if (dbl == kPrecFP32 && fft_ok && !best_nt) {
        dbl = kPrecFP64;
        search(dbl);
    }
    p.dbl = dbl;
    p.nr = best_nr;
    p.bins = dbl == kPrecNTT ? p.nr : p.nr / 2 + 1;
    p.dec_fft = dbl != kPrecNTT && decode_uses_fft(p.nr, dbl);
    p.cost_fft = best;
    if (g.opt.path == kPathFFT) {
        if (!fft_ok)
            return fail(MD_ERR_UNSUPPORTED, "FFT path needs 1 <= SE cells and (L-1)+max offset+1 <= %d",
                        dbl == kPrecNTT ? kNttMaxNr : 4096);
        if (!best_nt) return fail(MD_ERR_UNSUPPORTED, "no FFT tile length fits k=%d (tile %d)", j.k, g.opt.tile);
        p.path = kPathFFT;
    } else if (g.opt.path == kPathDirect) {
        if (!dir_ok) return fail(MD_ERR_UNSUPPORTED, "the direct window supports k <= %d (k=%d)", kMaxDirectK, j.k);
        p.path = kPathDirect;
    } else {
        if (!best_nt && !dir_ok) return fail(MD_ERR_UNSUPPORTED, "no path covers k=%d with an empty SE", j.k);
        p.path = (best_nt && best < p.cost_dir) ? kPathFFT : kPathDirect;
    }
    if (p.path == kPathDirect) return MD_OK;
    p.nt = best_nt;
    p.T = best_nt - j.k + 1;
    p.tiles_x = (j.W + p.T - 1) / p.T;
    p.tiles_y = (j.H + p.T - 1) / p.T;
    if (dbl == kPrecFP32) {
        // exact recompute of ambiguous tiles in FP64: the smallest length
        // whose tile covers the FP32 tile, else the largest
        p.fb_mode = kFbFFT64;
        p.nt64 = kMaxN;
        for (int nt64 = 16; nt64 <= kMaxN; nt64 *= 2)
            if (nt64 - j.k + 1 >= p.T) {
                p.nt64 = nt64;
                break;
            }
        p.T64 = p.nt64 - j.k + 1;
    }
    return MD_OK;
}

// ---------------------------------------------------------------------------
// executor
// ---------------------------------------------------------------------------
// bytes of one transform-domain value
size_t elem_bytes(int dbl) {
    return dbl == kPrecNTT ? sizeof(uint32_t) : dbl == kPrecFP64 ? sizeof(double2) : sizeof(float2);
}

int occupancy_grid(long long nitems, size_t lds, int threads) {
    int per_cu = 2048 / threads;
    if (lds > 0) per_cu = std::min<int>(per_cu, (int)((160 * 1024) / lds));
    per_cu = std::max(per_cu, 1);
    const long long cap = (long long)g.cu * per_cu;
    return (int)std::max<long long>(1, std::min(nitems, cap));
}

Group *find_group(std::vector<Group> &v, int nt, int dbl, int big) {
    for (auto &gr : v)
        if (gr.nt == nt && gr.dbl == dbl && gr.big == big) return &gr;
    v.push_back(Group());
    v.back().nt = nt;
    v.back().dbl = dbl;
    v.back().big = big;
    return &v.back();
}

std::string signature(const md_job *jobs, int n, const std::vector<SEData> &ses) {
    std::string s;
    const Options &o = g.opt;
    s.append((const char *)&o.precision, sizeof o.precision);
    s.append((const char *)&o.band, sizeof o.band);
    s.append((const char *)&o.path, sizeof o.path);
    s.append((const char *)&o.tile, sizeof o.tile);
    s.append((const char *)&o.nr, sizeof o.nr);
    s.append((const char *)&o.ws_mb, sizeof o.ws_mb);
    for (int i = 0; i < n; ++i) {
        const int hdr[5] = {jobs[i].H, jobs[i].W, jobs[i].L, jobs[i].k, jobs[i].op};
        s.append((const char *)hdr, sizeof hdr);
        s.append(ses[i].key);
    }
    return s;
}

// Builds a batch's executor: plans, device job and segment tables, launch
// groups and the workspace layout.  With layout_only it stops once the
// workspace size (ex.ws_need) is known, touching no device memory.
int build_exec(const md_job *jobs, int n, const std::vector<SEData> &ses, Exec &ex, bool layout_only = false) {
    struct PinScope {   // cache entries used from here on are pinned to ex
        explicit PinScope(std::vector<CacheEntry *> *p) { g.pin_sink = p; }
        ~PinScope() { g.pin_sink = nullptr; }
    } pin_scope(layout_only ? nullptr : &ex.pins);
    ex.jobs_h.resize(n);
    ex.plans.resize(n);
    std::vector<size_t> dir_lds(n, 0);
    std::vector<int> dir_sel(n, 0);
    long long flag_total = 0;
    int win_tmax = 0;
    const size_t cap_bytes = (size_t)std::max(1.0, g.opt.ws_mb) * 1024 * 1024;
    // per-job plans and device descriptors
    for (int i = 0; i < n; ++i) {
        const md_job &j = jobs[i];
        Plan &p = ex.plans[i];
        MD_TRY(plan_job(j, ses[i], p, n == 1));
        JobDev &d = ex.jobs_h[i];
        memset(&d, 0, sizeof d);
        d.D = 1;
        d.img = j.img;
        d.out = j.out;
        d.H = j.H;
        d.W = j.W;
        d.L = j.L;
        d.k = j.k;
        d.op = j.op;
        d.path = p.path;
        d.kpad = (j.k + kDirRX - 1) / kDirRX * kDirRX;
        DirSE *ds = nullptr;
        // window tables: the direct path, and the exact window tier behind
        // the FP transform passes
        if (!layout_only && (p.path == kPathDirect || p.dbl != kPrecNTT)) {
            MD_TRY(get_dirse(ses[i], &ds));
            d.sek = (const int32_t *)ds->sek.p;
            d.se_cnt = (const int32_t *)ds->cnt.p;
        }
        if (p.path == kPathDirect) {
            d.dir_pack = direct_form((long long)(j.L - 1) + ses[i].maxoff);
            if (ds) {
                d.sek16 = (const int32_t *)(d.dir_pack == 2 ? ds->sekh.p : ds->sek16.p);
                d.sek_rows = (const int32_t *)ds->rows.p;
                d.sek_steps = (const int32_t *)ds->steps.p;
                d.dir_nsteps = ds->nsteps;
            }
            d.dir_bx = (j.W + kDirBW - 1) / kDirBW;
            d.dir_by = (j.H + direct_block_rows(d.dir_pack) - 1) / direct_block_rows(d.dir_pack);
            // the packed form reads the SE through scalar loads; the 32-bit form
            // stages it in LDS when it fits
            const int sel = !d.dir_pack && direct_lds_bytes(j.k, d.kpad, 0, 1) <= kLdsBytes ? 1 : 0;
            dir_sel[i] = sel;
            dir_lds[i] = direct_lds_bytes(j.k, d.kpad, d.dir_pack, sel);
            if (dir_lds[i] > kLdsBytes) return fail(MD_ERR_UNSUPPORTED, "direct window for k=%d exceeds the LDS", j.k);
            ++ex.n_direct;
            continue;
        }
        ++ex.n_fft;
        d.nt = p.nt;
        d.T = p.T;
        d.nr = p.nr;
        d.bins = p.bins;
        d.tiles_x = p.tiles_x;
        d.tiles_y = p.tiles_y;
        d.dbl = p.dbl;
        if (p.dbl == kPrecNTT) {
            if (!layout_only) {
                NttRange *nrt = nullptr;
                MD_TRY(get_nrange(p.nr, j.L, &nrt));
                NttSpec *nsp = nullptr;
                MD_TRY(get_nspectrum(ses[i], p.nt, p.nr, nrt, &nsp));
                d.se_spec = nsp->spec.p;
                d.ntt_spec_s = (const uint32_t *)nsp->spec_s.p;
                d.enc = nrt->enc.p;
                d.dec = nrt->dec.p;
                d.ntt_dec_s = (const uint32_t *)nrt->dec_s.p;
                d.dec_pitch = nrt->dp;
            }
            d.ntt_dtop = (j.L - 1) + ses[i].maxoff;
            d.fb_mode = kFbNone;
            ex.fft_tiles += (long long)p.tiles_x * p.tiles_y;
            continue;
        }
        RangeTables *rt = nullptr;
        if (!layout_only) {
            MD_TRY(get_range(p.nr, j.L, &rt));
            SESpec *sp = nullptr;
            MD_TRY(get_spectrum(ses[i], p.nt, p.nr, !p.dbl, p.dbl != 0, &sp));
            d.se_spec = p.dbl ? sp->s64.p : sp->s32.p;
            d.enc = p.dbl ? rt->enc64.p : rt->enc32.p;
            d.dec = p.dbl ? rt->dec64.p : rt->dec32.p;
            d.rtw = p.dbl ? rt->rtw64.p : rt->rtw32.p;
        }
        d.scale = 1.0 / ((double)p.nt * p.nt * p.nr);
        d.dec_pitch = dec_pitch(p.nr);
        d.ybs = plan_ybs(p);
        // the register decodes (the dense ones of at most 8 bins and the
        // short-length FFT ones) take bin 0 in closed form: its plane need
        // not be written or read
        d.dc_dec = ((!p.dec_fft && p.bins <= 8) || (p.dec_fft && decode_small_m(p.nr / 2, p.dbl))) &&
                   !g.opt.dc_plane;
        d.flag0 = flag_total;
        flag_total += (long long)p.tiles_x * p.tiles_y;
        ex.fft_tiles += (long long)p.tiles_x * p.tiles_y;
        win_tmax = std::max(win_tmax, p.T);
        d.fb_mode = p.fb_mode;
        if (p.fb_mode == kFbFFT64) {
            if (!layout_only) {
                SESpec *sp64 = nullptr;
                MD_TRY(get_spectrum(ses[i], p.nt64, p.nr, false, true, &sp64));
                d.se_spec64 = (const double2 *)sp64->s64.p;
                d.enc64 = (const double2 *)rt->enc64.p;
                d.dec64 = (const double2 *)rt->dec64.p;
            }
            d.nt64 = p.nt64;
            d.T64 = p.T64;
            d.scale64 = 1.0 / ((double)p.nt64 * p.nt64 * p.nr);
            auto fc = std::find_if(ex.fb_classes.begin(), ex.fb_classes.end(),
                                   [&](const Exec::FbClass &c) { return c.nt64 == p.nt64; });
            if (fc == ex.fb_classes.end()) {
                ex.fb_classes.emplace_back();
                fc = ex.fb_classes.end() - 1;
                fc->nt64 = p.nt64;
            }
            fc->slot_elems = std::max(fc->slot_elems, (size_t)p.bins * p.T64 * p.T64);
        }
    }
    // direct groups: one segment per direct job, in decreasing cost per
    // block, so that the persistent blocks end on the cheapest items
    std::vector<int> dir_order;
    for (int i = 0; i < n; ++i)
        if (ex.plans[i].path == kPathDirect) dir_order.push_back(i);
    auto block_cost = [&](int i) { return dir_block_cost(jobs[i].k, ses[i], ex.jobs_h[i].dir_pack); };
    std::stable_sort(dir_order.begin(), dir_order.end(), [&](int a, int b) { return block_cost(a) > block_cost(b); });
    for (int i : dir_order) {
        const int pack = ex.jobs_h[i].dir_pack, sel = dir_sel[i];
        // blocks per CU the job's LDS footprint allows; footprints that allow 4
        // or more share one launch at 4 (16 waves per CU keep the VALU busy),
        // so the batch drains through one tail instead of one per class
        const int per_cu = std::max(1, std::min(4, (int)(kLdsBytes / dir_lds[i])));
        Group *grp = nullptr;
        for (auto &gq : ex.direct)
            if (gq.pack == pack && gq.sel == sel && gq.big == per_cu) grp = &gq;
        if (!grp) {
            ex.direct.push_back(Group());
            grp = &ex.direct.back();
            grp->pack = pack;
            grp->sel = sel;
            grp->big = per_cu;
        }
        Group &gr = *grp;
        gr.lds = std::max(gr.lds, dir_lds[i]);
        Seg s{};
        s.item0 = gr.nitems;
        s.job = i;
        gr.segs.push_back(s);
        gr.nitems += (long long)ex.jobs_h[i].dir_bx * ex.jobs_h[i].dir_by;
        const double px = (double)jobs[i].H * jobs[i].W;
        gr.alg_bytes += px * 8.0;
        gr.alg_ops += px * ses[i].ncells * 2.0;
        gr.units += px * ses[i].dir_cells[gr.pack ? 0 : 1];
    }

    // FFT jobs: split tile ranges into waves bounded by the workspace cap
    std::vector<std::vector<std::pair<int, std::pair<int, int>>>> wave_chunks(1);   // (job, (tile0, ntiles))
    std::vector<size_t> wave_bytes(1, 0);
    for (int i = 0; i < n; ++i) {
        const Plan &p = ex.plans[i];
        if (p.path != kPathFFT) continue;
        const size_t per_tile = ytile_elems(p.bins, p.T, plan_ybs(p)) * elem_bytes(p.dbl);
        const int ntiles = p.tiles_x * p.tiles_y;
        int t = 0;
        while (t < ntiles) {
            size_t room = cap_bytes > wave_bytes.back() ? cap_bytes - wave_bytes.back() : 0;
            int fit = (int)std::min<size_t>((size_t)(ntiles - t), room / per_tile);
            if (fit == 0) {
                if (wave_bytes.back() == 0) fit = 1;   // a single tile larger than the cap
                else {
                    wave_chunks.emplace_back();
                    wave_bytes.push_back(0);
                    continue;
                }
            }
            wave_chunks.back().push_back({i, {t, fit}});
            wave_bytes.back() += per_tile * fit;
            t += fit;
        }
    }
    size_t ymax = 0;
    for (size_t w = 0; w < wave_chunks.size(); ++w) ymax = std::max(ymax, wave_bytes[w]);
    for (size_t w = 0; w < wave_chunks.size(); ++w) {
        if (wave_chunks[w].empty()) continue;
        Wave wv;
        size_t off = 0;
        for (auto &ch : wave_chunks[w]) {
            const int i = ch.first, tile0 = ch.second.first, nt_ = ch.second.second;
            const Plan &p = ex.plans[i];
            const size_t per_tile = ytile_elems(p.bins, p.T, plan_ybs(p)) * elem_bytes(p.dbl);
            Seg s{};
            s.job = i;
            s.tile0 = tile0;
            s.ntiles = nt_;
            const int dpix = p.dec_fft ? decode_fft_pixels(p.nr, p.dbl) : kDecThreads * kDecPixPerThread;
            s.pblocks = (p.T * p.T + dpix - 1) / dpix;
            s.y = (void *)(uintptr_t)off;   // an offset into the transform-domain buffer until it is placed
            off += per_tile * nt_;
            const bool ntt = p.dbl == kPrecNTT;
            const double esz = (double)elem_bytes(p.dbl), N2 = (double)p.nt * p.nt, TT = (double)p.T * p.T;
            const double items = (double)nt_ * p.bins;
            // items the transform kernels transform: bin 0 of the floating-
            // point paths is written in closed form instead
            const double fitems = ntt ? items : (double)nt_ * (p.bins - 1);
            // planes stored in the transform-domain buffer: every bin, but
            // bin 0 where the decode takes it in closed form (JobDev::dc_dec)
            const double planes = ex.jobs_h[i].dc_dec ? (double)nt_ * (p.bins - 1) : items;
            // pixels of these tiles that lie inside the image
            double inside = 0;
            for (int t = tile0; t < tile0 + nt_; ++t) {
                const int ty = t / p.tiles_x, tx = t % p.tiles_x;
                inside += (double)std::min(p.T, jobs[i].H - ty * p.T) * std::min(p.T, jobs[i].W - tx * p.T);
            }
            Group *gf = find_group(wv.fft, p.nt, p.dbl, 0);
            s.item0 = gf->nitems;
            gf->segs.push_back(s);
            // the large-tile kernel has no bin-0 items (it writes bin 0 with
            // bin 1); the LDS-resident one keeps them as cheap items
            gf->nitems += (long long)nt_ * (!ntt && big_tile(p.nt, p.dbl) ? p.bins - 1 : p.bins);
            // HBM bytes the transform must move: the valid outputs of every
            // item out, and in the int32 tile once and the SE spectrum of
            // each transformed bin once (each then serves its other items
            // from L2/MALL)
            gf->alg_bytes += planes * TT * esz + (fitems > 0 ? (double)nt_ * N2 * 4.0 : 0.0) +
                             (fitems / nt_) * N2 * esz;
            // FP: flops of the forward and inverse 2-D FFTs and the product;
            // exact: modular products (one per butterfly and per point)
            gf->alg_ops += ntt ? items * (N2 * log2(N2) + N2) : fitems * (2.0 * 5.0 * N2 * log2(N2) + 6.0 * N2);
            gf->units += fitems;
            gf->pixels += inside;
            gf->vol_elems += items * TT;
            const int dvar = ntt ? 0 : p.dec_fft ? decode_fft_var(p.nr) : decode_group_variant(p.bins, p.dbl);
            Group *gd = find_group(wv.dec, 0, p.dbl, dvar);
            s.item0 = gd->nitems;
            gd->segs.push_back(s);
            gd->nitems += (long long)nt_ * s.pblocks;
            gd->alg_bytes += inside * ((ex.jobs_h[i].dc_dec ? p.bins - 1 : p.bins) * esz + 4.0);
            gd->pixels += inside;
            if (ntt) {
                // one block of 8 degrees per pixel, over all n bins
                gd->alg_ops += inside * p.nr * 8.0;
                gd->units += (double)nt_ * TT * p.nr;
            } else if (p.dec_fft) {
                // packing (10 flops per point of the half-length transform)
                // and a complex inverse FFT of length nr/2
                const double h = p.nr / 2.0;
                gd->alg_ops += inside * (5.0 * h * std::log2(h) + 10.0 * h);
                gd->units += (double)nt_ * TT * dec_units(p.nr, p.dbl);
            } else {
                gd->alg_ops += inside * p.nr * p.bins * 4.0;
                gd->units += (double)nt_ * TT * dec_units(p.nr, p.dbl);
            }
        }
        ex.waves.push_back(std::move(wv));
    }
    // segment tables (device copies below) and launch grids
    size_t nseg_total = 0;
    for (auto &gr : ex.direct) nseg_total += gr.segs.size();
    for (auto &wv : ex.waves) {
        for (auto &gr : wv.fft) nseg_total += gr.segs.size();
        for (auto &gr : wv.dec) nseg_total += gr.segs.size();
    }
    for (auto &gr : ex.direct) gr.grid = occupancy_grid(gr.nitems, gr.lds, kDirThreads);
    std::vector<std::pair<Group *, size_t>> slab_groups;   // large-tile groups and their slab bytes
    for (auto &wv : ex.waves) {
        for (auto &gr : wv.fft) {
            if (gr.dbl == kPrecNTT) {
                gr.grid = occupancy_grid(gr.nitems, ntt_lds_bytes(gr.nt), ntt_block_threads(gr.nt));
                continue;
            }
            if (big_tile(gr.nt, gr.dbl)) {
                // three passes per chunk of items, each over (item, line batch)
                // units, through the chunk's intermediates
                gr.big_chunk = big_chunk_items(gr.nt, gr.dbl, gr.nitems);
                const long long units = gr.big_chunk * (gr.nt / big_lines_of(gr.nt, gr.dbl));
                gr.grid = occupancy_grid(units, fft_lds_bytes(gr.nt, gr.dbl), fft_block_threads(gr.nt, gr.dbl));
                slab_groups.push_back({&gr, (size_t)gr.big_chunk * gr.nt * gr.nt *
                                                (gr.dbl ? sizeof(double2) : sizeof(float2))});
            } else {
                gr.grid = occupancy_grid(gr.nitems, fft_lds_bytes(gr.nt, gr.dbl), fft_block_threads(gr.nt, gr.dbl));
            }
        }
        for (auto &gr : wv.dec) {
            // the range-axis FFT decode holds 256 E complex values (E = 16, 24
            // or 20 points per thread), one row of padding per E rows, and its
            // M twiddles in LDS (2 M when the second pass is the last); the
            // short-length form keeps everything in registers
            const size_t elem = gr.dbl == kPrecFP64 ? sizeof(double2) : sizeof(float2);
            const size_t dm = gr.big >= kDecFftVar ? (size_t)decode_fft_m(gr.big) : 0;
            const bool p2 = (dm & (dm - 1)) == 0, m3 = dm % 3 == 0;
            const size_t pts = p2 ? 4352 : m3 ? 6400 : 5376;
            const bool last2 = p2 ? dm <= 256 : m3 ? dm <= 192 : dm <= 80;
            const size_t lds = dm && !decode_small_m((int)dm, gr.dbl) ? (pts + (last2 ? 2 * dm : dm)) * elem : 0;
            gr.grid = occupancy_grid(gr.nitems, lds, kDecThreads);
        }
    }
    // recompute tiers
    ex.nflags = flag_total;
    size_t slot_bytes = 0, fb_slab_bytes = 0;
    if (!ex.fb_classes.empty()) {
        // recompute blocks per length: two per CU (the kernel's LDS holds two),
        // bounded so that that launch's slots and slabs stay under ~2 GiB.  Each
        // length sizes its own grid, so a long tile's large slots do not starve
        // the launches of shorter ones; the buffers fit the largest launch.
        for (auto &c : ex.fb_classes) {
            const double slab = c.nt64 > kMaxLdsN64 ? (double)c.nt64 * c.nt64 * sizeof(double2) : 0.0;
            const double per_block = (double)c.slot_elems * sizeof(double2) + slab;
            const int cap = (int)std::max(1.0, std::min(2.0 * g.cu, (double)(2ll << 30) / per_block));
            c.grid = (int)std::max<long long>(1, std::min<long long>(flag_total, cap));
            slot_bytes = std::max(slot_bytes, (size_t)c.grid * c.slot_elems * sizeof(double2));
            if (slab > 0) fb_slab_bytes = std::max(fb_slab_bytes, (size_t)c.grid * c.nt64 * c.nt64 * sizeof(double2));
        }
    }
    if (flag_total > 0) {
        ex.win_pblocks = (win_tmax * win_tmax + kDecThreads - 1) / kDecThreads;
        ex.win_grid = (int)std::max<long long>(1, std::min<long long>(flag_total * ex.win_pblocks, 8LL * g.cu));
    }
    // workspace layout, 256-byte aligned regions
    size_t ws = 0;
    auto region = [&](size_t bytes) {
        const size_t at = ws;
        ws += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t o_y = region(ymax);
    std::vector<size_t> o_slab;
    for (auto &sg : slab_groups) o_slab.push_back(region(sg.second));
    const size_t o_flags = region((size_t)flag_total * sizeof(unsigned int));
    const size_t o_list = region((size_t)flag_total * sizeof(int2));
    const size_t o_wlist = region((size_t)flag_total * sizeof(int2));
    const size_t o_slots = region(slot_bytes);
    const size_t o_fbslab = region(fb_slab_bytes);
    ex.ws_need = ws;
    if (layout_only) return MD_OK;
    char *base = nullptr;
    if (g.ws_ptr) {
        if (ws > g.ws_bytes)
            return fail(MD_ERR_ARG, "the workspace holds %zu bytes, this batch needs %zu (md_workspace_size)", g.ws_bytes,
                        ws);
        base = (char *)g.ws_ptr;
    } else {
        MD_TRY(ex.ws_own.ensure(ws));
        base = (char *)ex.ws_own.p;
    }
    ex.ybuf = base + o_y;
    for (size_t q = 0; q < slab_groups.size(); ++q) slab_groups[q].first->slabs = base + o_slab[q];
    ex.flags = (unsigned int *)(base + o_flags);
    ex.list = (int2 *)(base + o_list);
    ex.wlist = (int2 *)(base + o_wlist);
    ex.slots = (double2 *)(base + o_slots);
    ex.fb_slabs = (double2 *)(base + o_fbslab);
    // segment tables on the device, transform-domain offsets made pointers
    MD_TRY(ex.segbuf.ensure(std::max<size_t>(1, nseg_total) * sizeof(Seg)));
    std::vector<Seg> all;
    all.reserve(nseg_total);
    auto place = [&](Group &gr) {
        for (auto &sg : gr.segs)
            if (sg.y || ex.plans[sg.job].path == kPathFFT) sg.y = (char *)ex.ybuf + (uintptr_t)sg.y;
        gr.segs_d = (Seg *)ex.segbuf.p + all.size();
        all.insert(all.end(), gr.segs.begin(), gr.segs.end());
    };
    for (auto &gr : ex.direct) place(gr);
    for (auto &wv : ex.waves) {
        for (auto &gr : wv.fft) place(gr);
        for (auto &gr : wv.dec) place(gr);
    }
    if (!all.empty()) MD_HIP(hipMemcpy(ex.segbuf.p, all.data(), all.size() * sizeof(Seg), hipMemcpyHostToDevice));
    // job table
    MD_HIP(hipMalloc(&ex.jobs_d, sizeof(JobDev) * n));
    MD_HIP(hipHostMalloc((void **)&ex.jobs_pin, sizeof(JobDev) * n, 0));
    MD_HIP(hipEventCreateWithFlags(&ex.copy_done, hipEventDisableTiming));
    memcpy(ex.jobs_pin, ex.jobs_h.data(), sizeof(JobDev) * n);
    MD_HIP(hipMemcpy(ex.jobs_d, ex.jobs_pin, sizeof(JobDev) * n, hipMemcpyHostToDevice));
    return MD_OK;
}

hipEvent_t ev_get() {
    if (!g.evpool.empty()) {
        hipEvent_t e = g.evpool.back();
        g.evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Event pair around one launch when profiling (never inside a capture).
struct ProfScope {
    bool on;
    hipStream_t s;
    hipEvent_t a = nullptr;
    std::string name;
    double bytes, ops, units;
    ProfScope(bool on_, hipStream_t s_, std::string n, double b, double o, double u)
        : on(on_), s(s_), name(std::move(n)), bytes(b), ops(o), units(u) {
        if (on && (a = ev_get())) (void)hipEventRecord(a, s);
    }
    void done() {
        if (!on || !a) return;
        hipEvent_t b = ev_get();
        if (!b) return;
        (void)hipEventRecord(b, s);
        g.pending.push_back({name, a, b, bytes, ops, units});
        a = nullptr;
    }
};

void resolve_profile() {
    for (auto &p : g.pending) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &t = g.prof[p.name];
            t.ms += ms;
            t.launches += 1;
            t.bytes += p.bytes;
            t.ops += p.ops;
            t.units += p.units;
        }
        g.evpool.push_back(p.a);
        g.evpool.push_back(p.b);
    }
    g.pending.clear();
}

// Stream-ordered launches of one batch.  perturb: the test hook's per-tile
// bits (never set while capturing).
int enqueue(Exec &ex, hipStream_t s, bool skip_decode = false, bool capturing = false,
            const uint8_t *perturb = nullptr) {
    const bool prof = g.opt.profile && !capturing;
    MD_HIP(launch_zero(g.st_d, sizeof(StatsDev), s));
    if (ex.nflags > 0) MD_HIP(launch_zero(ex.flags, ex.nflags * sizeof(unsigned int), s));
    // With both paths in the batch, the direct-window launches go to a side
    // stream, so the transform path's launches take the CUs that the direct
    // grid's last blocks leave idle; the library stream joins the side stream
    // before the recompute.  Profiled calls keep one stream, so that each
    // stage's event time is its own.
    bool any_direct = false, any_fft = false;
    for (auto &gr : ex.direct) any_direct |= gr.nitems > 0;
    for (auto &wv : ex.waves)
        for (auto &gr : wv.fft) any_fft |= gr.nitems > 0;
    const bool fork = any_direct && any_fft && !skip_decode && !prof;
    hipStream_t sd = s;
    // joins the side stream back into the library stream exactly once, also
    // on an early error return (a capture with an unjoined stream is invalid)
    struct Join {
        bool pending = false;
        hipStream_t side = nullptr, main = nullptr;
        hipError_t run() {
            if (!pending) return hipSuccess;
            pending = false;
            hipError_t e = hipEventRecord(g.ev_join, side);
            if (e == hipSuccess) e = hipStreamWaitEvent(main, g.ev_join, 0);
            return e;
        }
        ~Join() { (void)run(); }
    } join;
    if (fork) {
        MD_HIP(hipEventRecord(g.ev_fork, s));
        MD_HIP(hipStreamWaitEvent(g.s_side, g.ev_fork, 0));
        sd = g.s_side;
        join.pending = true;
        join.side = sd;
        join.main = s;
    }
    for (auto &gr : ex.direct) {
        if (gr.nitems <= 0) continue;
        ProfScope ps(prof, sd, gr.pack == 2 ? "direct16" : gr.pack ? "direct16i" : "direct32", gr.alg_bytes,
                     gr.alg_ops, gr.units);
        MD_HIP(launch_direct(gr.pack, gr.sel, ex.jobs_d, gr.segs_d, (int)gr.segs.size(), gr.nitems, gr.grid, gr.lds,
                             g.st_d, sd));
        ps.done();
    }
    const float band = (float)g.opt.band;
    for (auto &wv : ex.waves) {
        for (auto &gr : wv.fft) {
            if (gr.dbl == kPrecNTT) {
                ProfScope ps(prof, s, "ntt_n" + std::to_string(gr.nt), gr.alg_bytes, gr.alg_ops, gr.units);
                MD_HIP(launch_ntt(gr.nt, ex.jobs_d, gr.segs_d, (int)gr.segs.size(), gr.nitems, gr.grid, g.ntw, g.ntws,
                                  g.st_d, s));
                ps.done();
                continue;
            }
            ProfScope ps(prof, s, std::string(gr.dbl ? "fft64_n" : "fft32_n") + std::to_string(gr.nt), gr.alg_bytes,
                         gr.alg_ops, gr.units);
            MD_HIP(launch_fft(gr.nt, gr.dbl, ex.jobs_d, gr.segs_d, (int)gr.segs.size(), gr.nitems, gr.grid, g.tw32,
                              g.tw64, gr.slabs, gr.big_chunk, g.st_d, perturb, s));
            ps.done();
        }
        if (skip_decode) continue;
        for (auto &gr : wv.dec) {
            if (gr.dbl == kPrecNTT) {
                ProfScope ps(prof, s, "decode_ntt", gr.alg_bytes, gr.alg_ops, gr.units);
                MD_HIP(launch_ntt_decode(ex.jobs_d, gr.segs_d, (int)gr.segs.size(), gr.nitems, gr.grid, s));
                ps.done();
                continue;
            }
            const bool dfft = gr.big >= kDecFftVar;   // the range-axis FFT decode
            ProfScope ps(prof, s, gr.dbl ? (dfft ? "decode64_fft" : "decode64") : (dfft ? "decode32_fft" : "decode32"),
                         gr.alg_bytes, gr.alg_ops, gr.units);
            MD_HIP(launch_decode(gr.big, gr.dbl, ex.jobs_d, gr.segs_d, (int)gr.segs.size(), gr.nitems, gr.grid,
                                 band, ex.flags, ex.list, ex.wlist, g.st_d, perturb, s));
            ps.done();
        }
    }
    MD_HIP(join.run());
    if (skip_decode) return MD_OK;
    for (const auto &c : ex.fb_classes) {
        ProfScope ps(prof, s, "recompute64_n" + std::to_string(c.nt64), 0, 0, 0);
        MD_HIP(launch_fallback(c.nt64, ex.jobs_d, ex.list, g.st_d, ex.slots, c.slot_elems, c.grid, g.tw64,
                               ex.fb_slabs, ex.flags, ex.wlist, perturb, s));
        ps.done();
    }
    if (ex.win_grid > 0) {
        ProfScope ps(prof, s, "window_exact", 0, 0, 0);
        MD_HIP(launch_tile_window(ex.jobs_d, ex.wlist, g.st_d, ex.win_pblocks, ex.win_grid, s));
        ps.done();
    }
    return MD_OK;
}

int collect_stats(Exec &ex, int *range_err) {
    MD_HIP(hipStreamSynchronize(g.stream));
    resolve_profile();
    MD_HIP(hipMemcpy(g.st_h, g.st_d, sizeof(StatsDev), hipMemcpyDeviceToHost));
    md_stats &st = g.last;
    float res;
    memcpy(&res, &g.st_h->max_res_bits, sizeof res);
    st.max_residual = res;
    st.tiles = ex.fft_tiles;
    st.fallback_tiles = g.st_h->fb_count;
    st.window_tiles = g.st_h->win_count;
    st.direct_jobs = ex.n_direct;
    st.fft_jobs = ex.n_fft;
    const Plan &p = ex.plans.back();
    st.path = p.path;
    st.n_t = p.nt;
    st.n_r = p.path == kPathFFT ? p.nr : 0;
    st.precision = p.path == kPathFFT ? p.dbl : g.opt.precision;
    *range_err = g.st_h->range_err != 0;
    return MD_OK;
}

int run(const md_job *jobs, int n, bool use_graph);

// Autotuner: time each kernel family on calibration images on this device
// and replace the cost model's built-in estimates with the measured rates.
int autotune_body() {
    // calibration images: 1024^2 for the LDS-resident lengths, 2048^2 for 256
    // (FP32) / 128-256 (FP64), 4096^2 for 512 and 1024 and for the direct
    // window (enough (tile, bin) items or blocks to load the whole GPU); grey
    // values in [0, 16)
    const int HS = 4096;
    DevBuf img, out;
    MD_TRY(img.ensure((size_t)HS * HS * 4));
    MD_TRY(out.ensure((size_t)HS * HS * 4));
    MD_HIP(launch_fill_hash((int32_t *)img.p, (size_t)HS * HS, 16, 12345u, g.stream));
    g.opt.sync = 1;
    g.opt.graph = 0;
    g.opt.profile = 1;
    g.opt.nr = 0;
    g.opt.band = 0.25;
    // runs one job 3 times after a warm-up; *ms = mean time of `stage` per
    // run, *per_unit = the same per work unit
    auto measure = [&](int k, int L, int side, int path, int prec, int tile, const std::string &stage, double *ms,
                       double *per_unit, SEData *se_out) -> int {
        std::vector<uint8_t> mask((size_t)k * k, 1);
        std::vector<int32_t> off((size_t)k * k);
        for (size_t q = 0; q < off.size(); ++q) off[q] = (int32_t)(q % 4);
        if (se_out) make_se(mask.data(), off.data(), k, 0, *se_out);
        md_job j{(const int32_t *)img.p, side, side, L, mask.data(), off.data(), k, (int32_t *)out.p, 0};
        g.opt.path = path;
        g.opt.precision = prec;
        g.opt.tile = tile;
        MD_TRY(run(&j, 1, false));
        g.prof.clear();
        for (int r = 0; r < 3; ++r) MD_TRY(run(&j, 1, false));
        auto it = g.prof.find(stage);
        if (it == g.prof.end() || it->second.units <= 0) return fail(MD_ERR_DEVICE, "calibration: no %s stage", stage.c_str());
        if (ms) *ms = it->second.ms / 3.0;
        if (per_unit) *per_unit = it->second.ms * 1e6 / it->second.units;
        return MD_OK;
    };
    // direct window: staging and per-cell costs from a small and a large SE
    // (16-bit packed form), then the 32-bit per-cell cost (L = 32768), on the
    // 4096^2 image: 2048 blocks, so the GPU is as full as in a large batch
    // (a smaller image leaves CUs idle and inflates the per-pixel costs)
    {
        const int side = HS;
        const double px = (double)side * side;
        SEData s3, s41, s15;
        double t3 = 0, t41 = 0, t15 = 0;
        MD_TRY(measure(3, 16, side, kPathDirect, 0, 0, "direct16", &t3, nullptr, &s3));
        MD_TRY(measure(41, 16, side, kPathDirect, 0, 0, "direct16", &t41, nullptr, &s41));
        MD_TRY(measure(15, 32768, side, kPathDirect, 0, 0, "direct32", &t15, nullptr, &s15));
        const double a1 = dir_staged(3, 1), b1 = s3.dir_cells[0], y1 = t3 * 1e6 / px;
        const double a2 = dir_staged(41, 1), b2 = s41.dir_cells[0], y2 = t41 * 1e6 / px;
        double cc = (y2 - y1 * a2 / a1) / (b2 - b1 * a2 / a1);
        double cs = (y1 - b1 * cc) / a1;
        if (!(cc > 0) || !(cs > 0)) {   // degenerate fit: all of it per cell
            cs = 0;
            cc = y2 / b2;
        }
        g.cost.dir_cell[0] = cc;
        g.cost.dir_stage = cs;
        const double y3 = t15 * 1e6 / px - dir_staged(15, 0) * cs;
        g.cost.dir_cell[1] = y3 > 0 ? y3 / s15.dir_cells[1] : 2 * cc;
    }
    // FFT lengths: SE side nt/8*2+1 up to 33 (the item cost does not depend
    // on it; the spectrum build does), on images that give every resident
    // block many items (2048^2: at 128 points tens per CU; on 1024^2
    // the last round's tail inflated the 128-point cost against the 64-point
    // one by some 5%, which sent jobs to the slower 64-point plans)
    auto side_for = [](int nt, int prec) { return (void)prec, nt >= 512 ? 4096 : 2048; };
    for (int prec = 0; prec < 2; ++prec) {
        const std::string pre = prec ? "fft64_n" : "fft32_n";
        for (int nt = 16; nt <= kMaxN; nt *= 2) {
            MD_TRY(measure(std::min(nt / 8 * 2 + 1, 33), 16, side_for(nt, prec), kPathFFT, prec, nt,
                           pre + std::to_string(nt), nullptr, &g.cost.fft_item[prec][ilog2i(nt)], nullptr));
            if (nt == 64) {   // the dense decode, at the smallest range length (19)
                g.opt.nr = 19;
                const int rc = measure(17, 16, 1024, kPathFFT, prec, nt, prec ? "decode64" : "decode32", nullptr,
                                       &g.cost.dec_unit[prec], nullptr);
                g.opt.nr = 0;
                MD_TRY(rc);
            }
        }
    }
    // exact path: lengths 16..128 and its decode
    for (int nt = 16; nt <= kNttMaxN; nt *= 2) {
        MD_TRY(measure(std::min(nt / 8 * 2 + 1, 33), 16, 1024, kPathFFT, kPrecNTT, nt, "ntt_n" + std::to_string(nt),
                       nullptr, &g.cost.fft_item[2][ilog2i(nt)], nullptr));
        if (nt == 64)
            MD_TRY(measure(17, 16, 1024, kPathFFT, kPrecNTT, nt, "decode_ntt", nullptr, &g.cost.dec_unit[2], nullptr));
    }
    return MD_OK;
}

// Persisted cost model: MD_TUNE_FILE names a text file of "key value" lines,
// valid for the device whose name and compute-unit count it records.  A file
// that lacks any key (one written for other kernel forms) is ignored and the
// model is measured again.
std::string device_key() {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g.device) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
}

bool load_tune_file() {
    const char *path = getenv("MD_TUNE_FILE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char key[128], dev[256] = {0};
    double v;
    CostModel c = g.cost;
    int got = 0;
    bool dev_ok = false;
    if (fscanf(f, "device %255s", dev) == 1 && device_key() == dev) dev_ok = true;
    while (dev_ok && fscanf(f, "%127s %lf", key, &v) == 2) {
        const std::string k(key);
        if (k == "direct_f16_cell") c.dir_cell[0] = v, ++got;
        else if (k == "direct32_cell") c.dir_cell[1] = v, ++got;
        else if (k == "direct_stage") c.dir_stage = v, ++got;
        else if (k == "decode32") c.dec_unit[0] = v, ++got;
        else if (k == "decode64") c.dec_unit[1] = v, ++got;
        else if (k == "decode_ntt") c.dec_unit[2] = v, ++got;
        else if (k.rfind("ntt_n", 0) == 0) c.fft_item[2][ilog2i(atoi(k.c_str() + 5))] = v, ++got;
        else if (k.rfind("fft32_n", 0) == 0) c.fft_item[0][ilog2i(atoi(k.c_str() + 7))] = v, ++got;
        else if (k.rfind("fft64_n", 0) == 0) c.fft_item[1][ilog2i(atoi(k.c_str() + 7))] = v, ++got;
    }
    fclose(f);
    if (!dev_ok || got < kCostValues) return false;
    g.cost = c;
    return true;
}

void save_tune_file() {
    const char *path = getenv("MD_TUNE_FILE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "device %s\n", device_key().c_str());
    fprintf(f, "direct_f16_cell %.9g\ndirect32_cell %.9g\ndirect_stage %.9g\ndecode32 %.9g\ndecode64 %.9g\n",
            g.cost.dir_cell[0], g.cost.dir_cell[1], g.cost.dir_stage, g.cost.dec_unit[0], g.cost.dec_unit[1]);
    for (int nt = 16; nt <= kMaxN; nt *= 2) fprintf(f, "fft32_n%d %.9g\n", nt, g.cost.fft_item[0][ilog2i(nt)]);
    for (int nt = 16; nt <= kMaxN; nt *= 2) fprintf(f, "fft64_n%d %.9g\n", nt, g.cost.fft_item[1][ilog2i(nt)]);
    for (int nt = 16; nt <= kNttMaxN; nt *= 2) fprintf(f, "ntt_n%d %.9g\n", nt, g.cost.fft_item[2][ilog2i(nt)]);
    fprintf(f, "decode_ntt %.9g\n", g.cost.dec_unit[2]);
    fclose(f);
}

int autotune() {
    if (g.tuned || g.tuning) return MD_OK;
    if (load_tune_file()) {
        g.tuned = true;
        g.cost_measured = true;
        return MD_OK;
    }
    g.tuning = true;
    const Options saved = g.opt;
    const auto saved_prof = g.prof;
    const md_stats saved_stats = g.last;
    const int rc = autotune_body();
    g.opt = saved;
    g.prof = saved_prof;
    g.last = saved_stats;
    g.execs.clear(), g.last_exec = nullptr;
    g.tuning = false;
    g.tuned = rc == MD_OK;
    g.cost_measured = rc == MD_OK;
    if (rc == MD_OK) save_tune_file();
    return rc;
}

// Bytes of a batch's SE arrays as the caller passed them (masks, then
// offsets, job by job): the repeat-call fast path compares them with the
// previous call's.
std::string se_bytes(const md_job *jobs, int n) {
    size_t total = 0;
    for (int i = 0; i < n; ++i) total += (size_t)jobs[i].k * jobs[i].k * (1 + sizeof(int32_t));
    std::string b;
    b.reserve(total);
    for (int i = 0; i < n; ++i) {
        const size_t kk = (size_t)jobs[i].k * jobs[i].k;
        b.append((const char *)jobs[i].se_mask, kk);
        b.append((const char *)jobs[i].se_offsets, kk * sizeof(int32_t));
    }
    return b;
}

bool same_options(const Options &a, const Options &b) {
    return a.precision == b.precision && a.band == b.band && a.path == b.path && a.tile == b.tile && a.nr == b.nr &&
           a.ws_mb == b.ws_mb;
}

bool same_se_bytes(const md_job *jobs, int n, const std::string &prev) {
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const size_t kk = (size_t)jobs[i].k * jobs[i].k;
        if (off + kk * (1 + sizeof(int32_t)) > prev.size()) return false;
        if (memcmp(prev.data() + off, jobs[i].se_mask, kk) != 0) return false;
        off += kk;
        if (memcmp(prev.data() + off, jobs[i].se_offsets, kk * sizeof(int32_t)) != 0) return false;
        off += kk * sizeof(int32_t);
    }
    return off == prev.size();
}

// Room for a new cached executor whose own workspace takes `adding` bytes:
// the cached executors are kept to at most kMaxExecs, and their workspace
// together with the new one's within MD_OPT_CACHE_MB, by dropping the least
// recently run ones (they are rebuilt on their next call).
constexpr size_t kMaxExecs = 64;
int trim_execs(size_t adding) {
    const double cap = g.opt.cache_mb * 1024.0 * 1024.0;
    auto total = [&] {
        size_t t = adding;
        for (auto &kv : g.execs) t += kv.second->ws_own.bytes;
        return t;
    };
    if (g.execs.size() < kMaxExecs && (double)total() <= cap) return MD_OK;
    MD_HIP(hipDeviceSynchronize());   // their graphs and buffers may still be in use
    while (!g.execs.empty() && (g.execs.size() >= kMaxExecs || (double)total() > cap)) {
        auto lru = g.execs.begin();
        for (auto it = g.execs.begin(); it != g.execs.end(); ++it)
            if (it->second->stamp < lru->second->stamp) lru = it;
        if (lru->second.get() == g.last_exec) g.last_exec = nullptr;
        g.execs.erase(lru);
    }
    return MD_OK;
}

int run(const md_job *jobs, int n, bool use_graph) {
    MD_TRY(init());
    ++g.call_id;
    if (g.opt.path == 0 && g.opt.autotune && !g.tuned && !g.tuning) MD_TRY(autotune());
    if (n < 1 || !jobs) return fail(MD_ERR_ARG, "empty batch");
    // A call identical to the previous one (job array, SE contents, options)
    // runs its executor again without re-validating, re-planning or hashing
    // the batch signature; everything was checked when that executor was
    // built and the inputs have not changed since.
    Exec *ex = nullptr;
    if (g.last_exec && (int)g.last_jobs.size() == n && same_options(g.opt, g.last_opt) &&
        memcmp(g.last_jobs.data(), jobs, sizeof(md_job) * n) == 0 && same_se_bytes(jobs, n, g.last_se))
        ex = g.last_exec;
    const bool repeat = ex != nullptr;
    std::vector<SEData> ses;
    if (!ex) {
        ses.resize(n);
        for (int i = 0; i < n; ++i) {
            MD_TRY(check_job(jobs[i]));
            make_se(jobs[i].se_mask, jobs[i].se_offsets, jobs[i].k, jobs[i].op, ses[i]);
        }
    }
    const std::string sig = ex ? std::string() : signature(jobs, n, ses);
    auto it = ex ? g.execs.end() : g.execs.find(sig);
    if (ex) {
    } else if (it == g.execs.end()) {
        auto e = std::make_unique<Exec>();
        const int rc = build_exec(jobs, n, ses, *e);
        if (rc != MD_OK) return rc;
        ex = e.get();
        MD_TRY(trim_execs(e->ws_own.bytes));
        g.execs[sig] = std::move(e);
    } else {
        ex = it->second.get();
    }
    ex->stamp = g.call_id;
    if (!repeat) {
        g.last_jobs.assign(jobs, jobs + n);
        g.last_se = se_bytes(jobs, n);
        g.last_opt = g.opt;
        g.last_exec = ex;
    }
    // refresh image / output pointers in the device job table if they moved
    bool changed = false;
    for (int i = 0; i < n; ++i) {
        if (ex->jobs_h[i].img != jobs[i].img || ex->jobs_h[i].out != jobs[i].out) {
            ex->jobs_h[i].img = jobs[i].img;
            ex->jobs_h[i].out = jobs[i].out;
            changed = true;
        }
    }
    if (changed) {
        if (ex->copy_pending) MD_HIP(hipEventSynchronize(ex->copy_done));
        memcpy(ex->jobs_pin, ex->jobs_h.data(), sizeof(JobDev) * n);
        MD_HIP(hipMemcpyAsync(ex->jobs_d, ex->jobs_pin, sizeof(JobDev) * n, hipMemcpyHostToDevice, g.stream));
        MD_HIP(hipEventRecord(ex->copy_done, g.stream));
        ex->copy_pending = true;
    }
    // the perturbation test hook: a per-tile byte array for this call, no graph
    const uint8_t *perturb = nullptr;
    if (!g.perturb.empty() && ex->nflags > 0) {
        std::vector<uint8_t> bits((size_t)ex->nflags, 0);
        for (auto &pt : g.perturb)
            if (pt.first >= 0 && pt.first < ex->nflags) bits[(size_t)pt.first] |= pt.second;
        MD_HIP(hipStreamSynchronize(g.stream));
        MD_TRY(g.perturb_d.ensure(bits.size()));
        MD_HIP(hipMemcpy(g.perturb_d.p, bits.data(), bits.size(), hipMemcpyHostToDevice));
        perturb = (const uint8_t *)g.perturb_d.p;
    }
    const bool graph = use_graph && g.opt.graph && g.stream != nullptr && !perturb;
    if (graph) {
        if (!ex->gexec || ex->graph_stream != g.stream) {
            if (ex->gexec) (void)hipGraphExecDestroy(ex->gexec);
            if (ex->graph) (void)hipGraphDestroy(ex->graph);
            ex->gexec = nullptr;
            ex->graph = nullptr;
            MD_HIP(hipStreamBeginCapture(g.stream, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue(*ex, g.stream, false, true);
            hipGraph_t gr = nullptr;
            const hipError_t ee = hipStreamEndCapture(g.stream, &gr);
            if (rc != MD_OK) {
                if (gr) (void)hipGraphDestroy(gr);
                return rc;
            }
            MD_HIP(ee);
            ex->graph = gr;
            MD_HIP(hipGraphInstantiate(&ex->gexec, gr, nullptr, nullptr, 0));
            ex->graph_stream = g.stream;
        }
        MD_HIP(hipGraphLaunch(ex->gexec, g.stream));
    } else {
        MD_TRY(enqueue(*ex, g.stream, false, false, perturb));
    }
    if (g.opt.sync) {
        int range_err = 0;
        MD_TRY(collect_stats(*ex, &range_err));
        if (range_err) return fail(MD_ERR_RANGE, "an image value lies outside [0, L-1]");
    }
    g_err.clear();
    return MD_OK;
}

// ---------------------------------------------------------------------------
// allocation-free dilation (md_dilate_noalloc)
// ---------------------------------------------------------------------------
// Device memory of md_dilate_noalloc: the job and segment descriptors, the
// statistics word and the SE tables of the direct window live in this array.
// Each device holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
constexpr size_t kNoAllocBytes = 1u << 20;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
void *noalloc_base[kNoAllocDevices] = {};

// This device's address of `scratch`, looked up once per device.
int noalloc_scratch(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kNoAllocDevices)
        return fail(MD_ERR_UNSUPPORTED, "md_dilate_noalloc supports devices 0..%d, not %d", kNoAllocDevices - 1, dev);
    if (!noalloc_base[dev]) {
        void *p = nullptr;
        MD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MD_ERR_DEVICE, "hipGetSymbolAddress returned a null address for the scratch array");
        noalloc_base[dev] = p;
    }
    *out = (unsigned char *)noalloc_base[dev];
    return MD_OK;
}

// Dilation by the direct max-plus window (Eq. (6new)) with every device
// buffer beyond the image and output taken from `scratch`: no allocation,
// no cache, no plan kept.  Synchronous: the tables are uploaded from host
// memory that lives on this call's stack, so it waits for its work.
int noalloc_dilate(const int32_t *img, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k,
                   int32_t *out) {
    const md_job j{img, H, W, L, mask, off, k, out, 0};
    MD_TRY(check_job(j));
    if (k > kMaxDirectK)
        return fail(MD_ERR_UNSUPPORTED, "md_dilate_noalloc runs the direct window, k <= %d (k=%d)", kMaxDirectK, k);
    SEData se;
    make_se(mask, off, k, 0, se);
    DirTables t;
    dir_tables(se, t);
    const int pack = direct_form((long long)(L - 1) + se.maxoff);
    const int sel = !pack && direct_lds_bytes(k, t.kpad, 0, 1) <= kLdsBytes ? 1 : 0;
    const size_t lds = direct_lds_bytes(k, t.kpad, pack, sel);
    if (lds > kLdsBytes) return fail(MD_ERR_UNSUPPORTED, "direct window for k=%d exceeds the LDS", k);
    const std::vector<int32_t> &packed = pack == 2 ? t.hh : t.h16;
    // scratch layout, 256-byte aligned regions
    size_t at = 0;
    auto region = [&](size_t bytes) {
        const size_t o = at;
        at += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_job = region(sizeof(JobDev)), o_seg = region(sizeof(Seg)), o_st = region(sizeof(StatsDev));
    const size_t o_sek = region(t.h.size() * 4), o_pk = region(packed.size() * 4), o_rows = region(t.rows.size() * 4);
    const size_t o_steps = region(std::max<size_t>(1, t.steps.size()) * 4);
    if (at > kNoAllocBytes)
        return fail(MD_ERR_ARG, "md_dilate_noalloc needs %zu bytes of scratch for k=%d, the maximum is %zu", at, k,
                    kNoAllocBytes);
    int dev = 0;
    MD_HIP(hipGetDevice(&dev));
    unsigned char *base = nullptr;
    MD_TRY(noalloc_scratch(dev, &base));
    int cu = 0;
    MD_HIP(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
    JobDev d;
    memset(&d, 0, sizeof d);
    d.img = img;
    d.out = out;
    d.H = H;
    d.W = W;
    d.L = L;
    d.k = k;
    d.op = 0;
    d.path = kPathDirect;
    d.D = 1;
    d.kpad = t.kpad;
    d.dir_pack = pack;
    d.sek = (const int32_t *)(base + o_sek);
    d.sek16 = (const int32_t *)(base + o_pk);
    d.sek_rows = (const int32_t *)(base + o_rows);
    d.sek_steps = (const int32_t *)(base + o_steps);
    d.dir_nsteps = (int)t.steps.size() / 4;
    d.dir_bx = (W + kDirBW - 1) / kDirBW;
    d.dir_by = (H + direct_block_rows(pack) - 1) / direct_block_rows(pack);
    Seg sg;
    memset(&sg, 0, sizeof sg);
    sg.job = 0;
    const long long nitems = (long long)d.dir_bx * d.dir_by;
    const int per_cu = std::max(1, std::min(2048 / kDirThreads, (int)(kLdsBytes / lds)));
    const int grid = (int)std::max<long long>(1, std::min<long long>(nitems, (long long)std::max(cu, 1) * per_cu));
    const hipStream_t s = g.stream;
    StatsDev *st = (StatsDev *)(base + o_st);
    MD_HIP(hipMemcpyAsync(base + o_job, &d, sizeof d, hipMemcpyHostToDevice, s));
    MD_HIP(hipMemcpyAsync(base + o_seg, &sg, sizeof sg, hipMemcpyHostToDevice, s));
    MD_HIP(hipMemcpyAsync(base + o_sek, t.h.data(), t.h.size() * 4, hipMemcpyHostToDevice, s));
    MD_HIP(hipMemcpyAsync(base + o_pk, packed.data(), packed.size() * 4, hipMemcpyHostToDevice, s));
    MD_HIP(hipMemcpyAsync(base + o_rows, t.rows.data(), t.rows.size() * 4, hipMemcpyHostToDevice, s));
    if (!t.steps.empty())
        MD_HIP(hipMemcpyAsync(base + o_steps, t.steps.data(), t.steps.size() * 4, hipMemcpyHostToDevice, s));
    // the range-error word starts at zero on every call (a fill kernel, not a
    // memset node)
    MD_HIP(launch_zero(st, sizeof(StatsDev), s));
    MD_HIP(launch_direct(pack, sel, (const JobDev *)(base + o_job), (const Seg *)(base + o_seg), 1, nitems, grid, lds,
                         st, s));
    StatsDev sh;
    MD_HIP(hipMemcpyAsync(&sh, st, sizeof sh, hipMemcpyDeviceToHost, s));
    MD_HIP(hipStreamSynchronize(s));
    md_stats &ls = g.last;
    ls = md_stats{};
    ls.direct_jobs = 1;
    ls.path = kPathDirect;
    ls.precision = g.opt.precision;
    if (sh.range_err) return fail(MD_ERR_RANGE, "image value outside [0, L-1] (L=%d)", L);
    return MD_OK;
}

// One dilation (op 0) or erosion (op 1) of an image whose values lie in
// [0, L-1], through the same planner and kernels as md_dilate.
int single(int op, const int32_t *img, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k,
           int32_t *out) {
    md_job j{img, H, W, L, mask, off, k, out, op};
    return run(&j, 1, false);
}

// Compositions of n-element images (or volumes): apply(o, src, Lr, dst)
// enqueues the dilation (o = 0) or erosion (o = 1) of src, values in
// [0, Lr-1], into dst.  m is the largest offset of an active SE cell.
//   opening: the erosion lies in [-m, L-1]; shifted by m it is an image of
//     range L+m, whose dilation (0 on an empty window) shifted back gives -m
//     there;
//   closing: the dilation lies in [0, L-1+m], an image of range L+m, whose
//     erosion gives L-1+m on an empty window.
template <typename A>
int compose(int op, const int32_t *img, size_t n, int L, int m, int32_t *out, A &&apply) {
    MD_TRY(g.morph_a.ensure(n * sizeof(int32_t)));
    MD_TRY(g.morph_b.ensure(n * sizeof(int32_t)));
    int32_t *a = (int32_t *)g.morph_a.p, *b = (int32_t *)g.morph_b.p;
    auto opening_into = [&](int32_t *tmp, int32_t *dst) -> int {
        MD_TRY(apply(1, img, L, tmp));
        if (m) MD_HIP(launch_add_const(tmp, tmp, m, n, g.stream));
        MD_TRY(apply(0, tmp, L + m, dst));
        if (m) MD_HIP(launch_add_const(dst, dst, -m, n, g.stream));
        return MD_OK;
    };
    auto closing_into = [&](int32_t *tmp, int32_t *dst) -> int {
        MD_TRY(apply(0, img, L, tmp));
        return apply(1, tmp, L + m, dst);
    };
    switch (op) {
        case MD_OPEN: MD_TRY(opening_into(a, out)); break;
        case MD_CLOSE: MD_TRY(closing_into(a, out)); break;
        case MD_GRADIENT:
            MD_TRY(apply(0, img, L, a));
            MD_TRY(apply(1, img, L, b));
            MD_HIP(launch_sub(out, a, b, n, g.stream));
            break;
        case MD_TOPHAT:
            MD_TRY(opening_into(a, b));
            MD_HIP(launch_sub(out, img, b, n, g.stream));
            break;
        default:   // MD_BLACKHAT
            MD_TRY(closing_into(a, b));
            MD_HIP(launch_sub(out, b, img, n, g.stream));
            break;
    }
    if (g.opt.sync) MD_HIP(hipStreamSynchronize(g.stream));
    return MD_OK;
}

int max_active_offset(const uint8_t *mask, const int32_t *off, size_t cells) {
    int m = 0;
    for (size_t q = 0; q < cells; ++q)
        if (mask[q]) m = std::max(m, (int)off[q]);
    return m;
}

int morph(int op, const int32_t *img, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k,
          int32_t *out) {
    if (op == MD_DILATE || op == MD_ERODE) return single(op, img, H, W, L, mask, off, k, out);
    if (op < MD_OPEN || op > MD_BLACKHAT) return fail(MD_ERR_ARG, "unknown morphological operation %d", op);
    md_job j{img, H, W, L, mask, off, k, out, 0};
    MD_TRY(check_job(j));
    MD_TRY(init());
    const int m = max_active_offset(mask, off, (size_t)k * k);
    if ((long long)L + m > (1 << 24)) return fail(MD_ERR_RANGE, "L + max offset = %lld exceeds 2^24", (long long)L + m);
    return compose(op, img, (size_t)H * W, L, m, out, [&](int o, const int32_t *src, int Lr, int32_t *dst) {
        return single(o, src, H, W, Lr, mask, off, k, dst);
    });
}

int vol_run(int op, const int32_t *vol, int D, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k,
            int32_t *out);

int morph3(int op, const int32_t *vol, int D, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k,
           int32_t *out) {
    if (op == MD_DILATE || op == MD_ERODE) return vol_run(op, vol, D, H, W, L, mask, off, k, out);
    if (op < MD_OPEN || op > MD_BLACKHAT) return fail(MD_ERR_ARG, "unknown morphological operation %d", op);
    if (!vol || !out || (const void *)vol == (const void *)out) return fail(MD_ERR_ARG, "null or aliased volume");
    if (!mask || !off) return fail(MD_ERR_ARG, "null SE array");
    if (D < 1 || H < 1 || W < 1 || (long long)D * H * W > 0x7fffffffLL)
        return fail(MD_ERR_ARG, "volume shape %dx%dx%d", D, H, W);
    if (k < 1 || k > 31 || (k % 2) == 0) return fail(MD_ERR_ARG, "k=%d must be odd in [1,31]", k);
    MD_TRY(init());
    const int m = max_active_offset(mask, off, (size_t)k * k * k);
    if ((long long)L + m > (1 << 24)) return fail(MD_ERR_RANGE, "L + max offset = %lld exceeds 2^24", (long long)L + m);
    return compose(op, vol, (size_t)D * H * W, L, m, out, [&](int o, const int32_t *src, int Lr, int32_t *dst) {
        return vol_run(o, src, D, H, W, Lr, mask, off, k, dst);
    });
}

// ---------------------------------------------------------------------------
// host-streamed images (partitioned convolution over bands of rows)
// ---------------------------------------------------------------------------
constexpr int kVolMaxK = 31;   // volume SE side

// Bands of H "rows" of `W` words each (image rows, or volume slices of
// H x W voxels), r = (k-1)/2 halo rows on each side; `compute(din, rows,
// dout)` enqueues one band's dilation / erosion on the library stream.
template <typename F>
int stream_bands(const int32_t *img, long long H, size_t W, int k, int32_t *out, F &&compute);

int stream_run(int op, const int32_t *img, long long H, int W, int L, const uint8_t *mask, const int32_t *off, int k,
               int32_t *out) {
    MD_TRY(init());
    if (!img || !out) return fail(MD_ERR_ARG, "null image or output pointer");
    if (!mask || !off) return fail(MD_ERR_ARG, "null SE array");
    if (H < 1 || W < 1) return fail(MD_ERR_ARG, "image shape %lldx%d", H, W);
    if (k < 1 || k > kMaxN - 1 || (k % 2) == 0) return fail(MD_ERR_ARG, "k=%d must be odd in [1,%d]", k, kMaxN - 1);
    return stream_bands(img, H, (size_t)W, k, out, [&](const int32_t *din, long long rows, int32_t *dout) {
        return single(op, din, (int)rows, W, L, mask, off, k, dout);
    });
}

// The same over bands of volume slices.
int stream_run3(int op, const int32_t *vol, long long D, int H, int W, int L, const uint8_t *mask, const int32_t *off,
                int k, int32_t *out) {
    MD_TRY(init());
    if (!vol || !out) return fail(MD_ERR_ARG, "null volume or output pointer");
    if (!mask || !off) return fail(MD_ERR_ARG, "null SE array");
    if (D < 1 || H < 1 || W < 1) return fail(MD_ERR_ARG, "volume shape %lldx%dx%d", D, H, W);
    if (k < 1 || k > kVolMaxK || (k % 2) == 0) return fail(MD_ERR_ARG, "k=%d must be odd in [1,%d]", k, kVolMaxK);
    return stream_bands(vol, D, (size_t)H * W, k, out, [&](const int32_t *din, long long slices, int32_t *dout) {
        return vol_run(op, din, (int)slices, H, W, L, mask, off, k, dout);
    });
}

template <typename F>
int stream_bands(const int32_t *img, long long H, size_t W, int k, int32_t *out, F &&compute) {
    const size_t bytes_all = (size_t)H * W * sizeof(int32_t);
    if ((const char *)img < (const char *)out + bytes_all && (const char *)out < (const char *)img + bytes_all)
        return fail(MD_ERR_ARG, "output must not overlap the input");
    const int r = (k - 1) / 2;
    // output rows per band: forced, or the most that four buffers of
    // (rows + 2r) x W words fit into the budget; a band image stays below 2^31
    // pixels
    long long R = g.opt.stream_rows;
    if (R <= 0) {
        const double budget = g.opt.stream_mb * 1024.0 * 1024.0;
        R = (long long)(budget / (4.0 * sizeof(int32_t) * W)) - 2 * r;
    }
    R = std::min<long long>(R, (long long)(0x7fffffffLL / W) - 2 * r);
    if (R < 1)
        return fail(MD_ERR_ARG, "a band of %zu words per row with %d halo rows does not fit (MD_OPT_STREAM_MB)", W, 2 * r);
    R = std::min<long long>(R, H);
    const long long nb = (H + R - 1) / R;
    const size_t band_bytes = (size_t)(std::min<long long>(H, R + 2 * r)) * W * sizeof(int32_t);
    if (!g.s_up) {
        MD_HIP(hipStreamCreateWithFlags(&g.s_up, hipStreamNonBlocking));
        MD_HIP(hipStreamCreateWithFlags(&g.s_down, hipStreamNonBlocking));
        for (int i = 0; i < 2; ++i) {
            MD_HIP(hipEventCreateWithFlags(&g.ev_up[i], hipEventDisableTiming));
            MD_HIP(hipEventCreateWithFlags(&g.ev_comp[i], hipEventDisableTiming));
            MD_HIP(hipEventCreateWithFlags(&g.ev_down[i], hipEventDisableTiming));
        }
    }
    // calibration (first auto-path call) before any band is in flight
    if (g.opt.path == 0 && g.opt.autotune && !g.tuned && !g.tuning) MD_TRY(autotune());
    MD_HIP(hipStreamSynchronize(g.stream));   // the band buffers may still be in use
    for (int i = 0; i < 2; ++i) {
        MD_TRY(g.hs_in[i].ensure(band_bytes));
        MD_TRY(g.hs_out[i].ensure(band_bytes));
    }
    MD_TRY(g.hs_flag.ensure(sizeof(uint32_t)));
    MD_HIP(launch_zero(g.hs_flag.p, sizeof(uint32_t), g.stream));
    // bands run with MD_OPT_SYNC = 0 so that their work overlaps; every call
    // below is stream-ordered on the library stream
    const Options saved = g.opt;
    g.opt.sync = 0;
    auto band = [&](long long b, long long &y0, long long &y1, long long &a0, long long &a1) {
        y0 = b * R;
        y1 = std::min(H, y0 + R);
        a0 = std::max(0LL, y0 - r);
        a1 = std::min(H, y1 + r);
    };
    auto download = [&](long long b) -> int {
        long long y0, y1, a0, a1;
        band(b, y0, y1, a0, a1);
        const int i = (int)(b & 1);
        MD_HIP(hipStreamWaitEvent(g.s_down, g.ev_comp[i], 0));
        MD_HIP(hipMemcpyAsync(out + (size_t)y0 * W, (const int32_t *)g.hs_out[i].p + (size_t)(y0 - a0) * W,
                              (size_t)(y1 - y0) * W * sizeof(int32_t), hipMemcpyDeviceToHost, g.s_down));
        MD_HIP(hipEventRecord(g.ev_down[i], g.s_down));
        return MD_OK;
    };
    int rc = MD_OK;
    for (long long b = 0; b < nb && rc == MD_OK; ++b) {
        long long y0, y1, a0, a1;
        band(b, y0, y1, a0, a1);
        const int i = (int)(b & 1);
        int32_t *din = (int32_t *)g.hs_in[i].p, *dout = (int32_t *)g.hs_out[i].p;
        // buffer i was last read by the compute of band b-2 and written back by
        // its download
        if (b >= 2) {
            if (hipStreamWaitEvent(g.s_up, g.ev_comp[i], 0) != hipSuccess ||
                hipStreamWaitEvent(g.stream, g.ev_down[i], 0) != hipSuccess) {
                rc = fail(MD_ERR_DEVICE, "stream wait failed");
                break;
            }
        }
        if (hipMemcpyAsync(din, img + (size_t)a0 * W, (size_t)(a1 - a0) * W * sizeof(int32_t), hipMemcpyHostToDevice,
                           g.s_up) != hipSuccess ||
            hipEventRecord(g.ev_up[i], g.s_up) != hipSuccess || hipStreamWaitEvent(g.stream, g.ev_up[i], 0) != hipSuccess) {
            rc = fail(MD_ERR_DEVICE, "band upload failed");
            break;
        }
        rc = compute(din, a1 - a0, dout);
        if (rc != MD_OK) break;
        if (launch_or_flag((uint32_t *)g.hs_flag.p, &g.st_d->range_err, g.stream) != hipSuccess ||
            hipEventRecord(g.ev_comp[i], g.stream) != hipSuccess) {
            rc = fail(MD_ERR_DEVICE, "band completion record failed");
            break;
        }
        // the previous band goes back while this one computes
        if (b >= 1) rc = download(b - 1);
    }
    if (rc == MD_OK) rc = download(nb - 1);
    const std::string err = g_err;
    // drain everything before returning (also after an error: no copy may
    // still target the caller's arrays)
    const hipError_t e1 = hipStreamSynchronize(g.s_up), e2 = hipStreamSynchronize(g.stream),
                     e3 = hipStreamSynchronize(g.s_down);
    g.opt = saved;
    if (rc != MD_OK) {
        g_err = err;
        return rc;
    }
    MD_HIP(e1);
    MD_HIP(e2);
    MD_HIP(e3);
    uint32_t flag = 0;
    MD_HIP(hipMemcpy(&flag, g.hs_flag.p, sizeof flag, hipMemcpyDeviceToHost));
    if (flag) return fail(MD_ERR_RANGE, "an image value lies outside [0, L-1]");
    g_err.clear();
    return MD_OK;
}

// ---------------------------------------------------------------------------
// volumes (three image axes, Sec. 2.1 / Sec. 3 with N = 3)
// ---------------------------------------------------------------------------
// Effective volume SE: the SE for dilation, its reflection through the
// centre for erosion (duality, Sec. 2.1); k^3 cells, (a, i, j) row-major.
struct VolSE {
    int k = 0;
    std::vector<uint8_t> mask;
    std::vector<int32_t> off;
    int maxoff = 0;
    long long ncells = 0;
    std::string key;
};

void make_vol_se(const uint8_t *mask, const int32_t *off, int k, int op, VolSE &se) {
    const size_t n = (size_t)k * k * k;
    se.k = k;
    se.mask.assign(n, 0);
    se.off.assign(n, 0);
    se.maxoff = 0;
    se.ncells = 0;
    for (size_t c = 0; c < n; ++c) {
        const size_t src = op ? n - 1 - c : c;   // reflection through the centre
        if (!mask[src]) continue;
        se.mask[c] = 1;
        se.off[c] = off[src];
        se.maxoff = std::max(se.maxoff, (int)off[src]);
        ++se.ncells;
    }
    se.key = "vol";
    se.key.append((const char *)&k, sizeof k);
    se.key.append((const char *)se.mask.data(), n);
    se.key.append((const char *)se.off.data(), n * sizeof(int32_t));
}

// One slab of the effective SE as a 2-D SE (already in effective form).
void vol_slab(const VolSE &se, int a, SEData &sd) {
    const size_t kk = (size_t)se.k * se.k;
    make_se(se.mask.data() + a * kk, se.off.data() + a * kk, se.k, 0, sd);
}

// Exact-path SE spectrum of a volume SE at cubic length nt and range length n,
// scaled by nt^-3, cached with the image spectra.
int get_vspectrum(const VolSE &se, int nt, int n, const NttRange *rt, NttSpec **out) {
    std::string key = "Q" + se.key;
    key.append((const char *)&nt, sizeof nt);
    key.append((const char *)&n, sizeof n);
    if ((*out = cache_get<NttSpec>(key))) return MD_OK;
    auto sp = std::make_unique<NttSpec>();
    const int k = se.k;
    const size_t nspec = (size_t)n * nt * nt * nt, kkk = (size_t)k * k * k;
    MD_TRY(cache_reserve(nspec * 8));
    MD_TRY(sp->spec.ensure(nspec * 4));
    MD_TRY(sp->spec_s.ensure(nspec * 4));
    MD_TRY(g.se_work.ensure(((size_t)n * k * k * nt + (size_t)n * k * nt * nt) * 4));
    MD_TRY(g.se_in.ensure(kkk * (sizeof(int32_t) + 1) + 64));
    MD_HIP(hipStreamSynchronize(g.stream));   // se_in may still be read by an earlier build
    int32_t *off_d = (int32_t *)g.se_in.p;
    uint8_t *mask_d = (uint8_t *)((char *)g.se_in.p + kkk * sizeof(int32_t));
    MD_HIP(hipMemcpy(off_d, se.off.data(), kkk * sizeof(int32_t), hipMemcpyHostToDevice));
    MD_HIP(hipMemcpy(mask_d, se.mask.data(), kkk, hipMemcpyHostToDevice));
    const uint32_t scale = pinv(pmul(pmul((uint32_t)nt, (uint32_t)nt), (uint32_t)nt));
    MD_HIP(launch_ntt3_se_spectrum(mask_d, off_d, k, nt, n, (const uint32_t *)rt->rpow.p, g.ntw, scale,
                                   (uint32_t *)g.se_work.p, (uint32_t *)sp->spec.p, (uint32_t *)sp->spec_s.p,
                                   g.stream));
    MD_HIP(hipStreamSynchronize(g.stream));
    *out = cache_put(key, std::move(sp));
    return MD_OK;
}

// Modular products of one cubic (tile, bin) item: one per butterfly of the
// forward and inverse transforms along the three axes and one per point.
double ntt3_item_products(int nt) {
    const double n3 = (double)nt * nt * nt;
    return n3 * std::log2(n3) + n3;
}

// Cost of one cubic item, scaled from the measured image item at length 16
// by the modular products (both are LDS-resident transforms of the same
// passes).
double ntt3_item_cost(int nt) {
    const double per = g.cost.fft_item[2][4] / (256.0 * 8.0 + 256.0);
    return per * ntt3_item_products(nt);
}

struct VolPlan {
    int path = kPathDirect;
    int pack = 1, sel = 0;
    size_t lds = 0;
    int nt = 0, T = 0, n = 0, tiles_x = 0, tiles_y = 0, tiles_z = 0;
    double cost_dir = INFINITY, cost_ntt = INFINITY;
    std::vector<SEData> slabs;   // active slabs (direct)
    std::vector<int> slab_a;
};

int vol_plan(int D, int H, int W, int L, const VolSE &se, VolPlan &p) {
    const int k = se.k, r = (k - 1) / 2;
    const double vox = (double)D * H * W;
    // direct window: one pass per active slab
    p.pack = direct_form((long long)(L - 1) + se.maxoff);
    double cells = 0;
    for (int a = 0; a < k; ++a) {
        bool any = false;
        for (size_t c = (size_t)a * k * k; c < (size_t)(a + 1) * k * k; ++c) any |= se.mask[c] != 0;
        if (!any) continue;
        p.slabs.emplace_back();
        vol_slab(se, a, p.slabs.back());
        p.slab_a.push_back(a);
        cells += p.slabs.back().dir_cells[p.pack ? 0 : 1];
    }
    const int kpad = (k + kDirRX - 1) / kDirRX * kDirRX;
    p.sel = !p.pack && direct_lds_bytes(k, kpad, 0, 1, true) <= kLdsBytes ? 1 : 0;
    p.lds = direct_lds_bytes(k, kpad, p.pack, p.sel, true);
    const int bh = direct_block_rows(p.pack, true);
    const double staged = (double)(bh + k - 1) * (kDirBW + kpad) / ((double)bh * kDirBW);
    p.cost_dir = vox * ((double)p.slabs.size() * staged * g.cost.dir_stage + cells * dir_cell_cost(p.pack));
    // exact transform: range length n >= L + max offset, cubic tiles 8 / 16 / 32
    long long nmin = (long long)(L - 1) + se.maxoff + 1;
    int n = ntt_length(nmin);
    if (g.opt.nr > 0) {
        if (g.opt.nr < nmin) return fail(MD_ERR_ARG, "forced range length %d < (L-1)+max offset+1 = %lld", g.opt.nr, nmin);
        if (ntt_length(g.opt.nr) != g.opt.nr)
            return fail(MD_ERR_ARG, "range length %d is not 2^a or 7*2^a up to %d", g.opt.nr, kNttMaxNr);
        n = g.opt.nr;
    }
    if (n > 0 && n <= kNttMaxNr) {
        for (int nt = 8; nt <= 32; nt *= 2) {
            if (g.opt.tile > 0 && g.opt.tile != nt) continue;
            const int T = nt - k + 1;
            if (T < 1) continue;
            const double tiles = (double)((D + T - 1) / T) * ((H + T - 1) / T) * ((W + T - 1) / T);
            const double c = tiles * n * ntt3_item_cost(nt) + tiles * T * T * T * n * g.cost.dec_unit[2];
            if (c < p.cost_ntt) {
                p.cost_ntt = c;
                p.nt = nt;
                p.T = T;
                p.n = n;
            }
        }
    }
    const bool ntt_ok = p.nt > 0;
    switch (g.opt.path) {
        case kPathFFT:
            if (!ntt_ok)
                return fail(MD_ERR_UNSUPPORTED,
                            g.opt.tile > 0 ? "no volume transform plan with tile %d for k=%d, L+max offset=%lld"
                                           : "no volume transform plan (tile %d) for k=%d, L+max offset=%lld",
                            g.opt.tile, k, nmin);
            p.path = kPathFFT;
            break;
        case kPathDirect: p.path = kPathDirect; break;
        default: p.path = ntt_ok && p.cost_ntt < p.cost_dir ? kPathFFT : kPathDirect; break;
    }
    if (p.path == kPathFFT) {
        p.tiles_z = (D + p.T - 1) / p.T;
        p.tiles_y = (H + p.T - 1) / p.T;
        p.tiles_x = (W + p.T - 1) / p.T;
    } else if (p.lds > kLdsBytes) {
        return fail(MD_ERR_UNSUPPORTED, "direct window for k=%d exceeds the LDS", k);
    }
    (void)r;
    return MD_OK;
}

int vol_run(int op, const int32_t *vol, int D, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k,
            int32_t *out) {
    MD_TRY(init());
    ++g.call_id;
    if (!vol || !out) return fail(MD_ERR_ARG, "null volume or output pointer");
    if ((const void *)vol == (const void *)out) return fail(MD_ERR_ARG, "output must not alias the input");
    if (!mask || !off) return fail(MD_ERR_ARG, "null SE array");
    if (D < 1 || H < 1 || W < 1) return fail(MD_ERR_ARG, "volume shape %dx%dx%d", D, H, W);
    if ((long long)D * H * W > 0x7fffffffLL) return fail(MD_ERR_ARG, "volume has more than 2^31-1 voxels");
    if (L < 2 || L > (1 << 24)) return fail(MD_ERR_ARG, "L=%d outside [2, 2^24]", L);
    if (k < 1 || k > kVolMaxK || (k % 2) == 0) return fail(MD_ERR_ARG, "k=%d must be odd in [1,%d]", k, kVolMaxK);
    for (int q = 0; q < k * k * k; ++q)
        if (mask[q] && (off[q] < 0 || off[q] > (1 << 24)))
            return fail(MD_ERR_RANGE, "SE offset %d at cell %d outside [0, 2^24]", off[q], q);
    VolSE se;
    make_vol_se(mask, off, k, op, se);
    VolPlan p;
    MD_TRY(vol_plan(D, H, W, L, se, p));
    const bool prof = g.opt.profile != 0;
    const double vox = (double)D * H * W;
    JobDev d;
    memset(&d, 0, sizeof d);
    d.img = vol;
    d.out = out;
    d.D = D;
    d.H = H;
    d.W = W;
    d.L = L;
    d.k = k;
    d.op = op;
    d.path = p.path;
    // device tables: job, segments, slabs; uploaded only when they differ
    // from what the buffers hold (a rewrite first waits for earlier work on
    // the stream, which may still read them)
    long long tiles = 0;
    std::vector<SlabDev> sl;
    std::vector<Seg> segs;
    long long dir_items = 0, chunk = 0;
    size_t TTT = 0, per_tile = 0;
    int pblocks = 0;
    if (p.path == kPathDirect) {
        sl.resize(p.slabs.size());
        for (size_t i = 0; i < p.slabs.size(); ++i) {
            DirSE *ds = nullptr;
            MD_TRY(get_dirse(p.slabs[i], &ds));
            SlabDev &e = sl[i];
            memset(&e, 0, sizeof e);
            e.sek = (const int32_t *)ds->sek.p;
            e.sek16 = (const int32_t *)(p.pack == 2 ? ds->sekh.p : ds->sek16.p);
            e.sek_rows = (const int32_t *)ds->rows.p;
            e.sek_steps = (const int32_t *)ds->steps.p;
            e.dir_nsteps = ds->nsteps;
            e.dz = p.slab_a[i] - (k - 1) / 2;
        }
        d.kpad = (k + kDirRX - 1) / kDirRX * kDirRX;
        if (g.vslabs.bytes < std::max<size_t>(1, sl.size()) * sizeof(SlabDev)) {
            MD_HIP(hipStreamSynchronize(g.stream));   // the table may still be in use
            MD_TRY(g.vslabs.ensure(std::max<size_t>(1, sl.size()) * sizeof(SlabDev)));
        }
        d.slabs = (const SlabDev *)g.vslabs.p;
        d.nslab = (int)sl.size();
        d.dir_pack = p.pack;
        d.dir_bx = (W + kDirBW - 1) / kDirBW;
        d.dir_by = (H + direct_block_rows(p.pack, true) - 1) / direct_block_rows(p.pack, true);
        segs.push_back(Seg{});
        dir_items = (long long)D * d.dir_by * d.dir_bx;
    } else {
        NttRange *nrt = nullptr;
        MD_TRY(get_nrange(p.n, L, &nrt));
        NttSpec *nsp = nullptr;
        MD_TRY(get_vspectrum(se, p.nt, p.n, nrt, &nsp));
        d.nt = p.nt;
        d.T = p.T;
        d.nr = p.n;
        d.bins = p.n;
        d.tiles_x = p.tiles_x;
        d.tiles_y = p.tiles_y;
        d.tiles_z = p.tiles_z;
        d.dbl = kPrecNTT;
        d.se_spec = nsp->spec.p;
        d.ntt_spec_s = (const uint32_t *)nsp->spec_s.p;
        d.enc = nrt->enc.p;
        d.dec = nrt->dec.p;
        d.ntt_dec_s = (const uint32_t *)nrt->dec_s.p;
        d.dec_pitch = nrt->dp;
        d.ntt_dtop = (L - 1) + se.maxoff;
        tiles = (long long)p.tiles_x * p.tiles_y * p.tiles_z;
        TTT = (size_t)p.T * p.T * p.T;
        per_tile = (size_t)p.n * TTT * sizeof(uint32_t);
        const size_t cap = (size_t)(g.opt.ws_mb * 1024.0 * 1024.0);
        chunk = std::max<long long>(1, std::min<long long>(tiles, (long long)(cap / per_tile)));
        pblocks = (int)((TTT + kDecThreads * kDecPixPerThread - 1) / (kDecThreads * kDecPixPerThread));
        for (long long t0 = 0; t0 < tiles; t0 += chunk) {
            Seg sg{};
            sg.tile0 = (int)t0;
            sg.ntiles = (int)std::min(chunk, tiles - t0);
            sg.pblocks = pblocks;
            segs.push_back(sg);
        }
        if (g.vy.bytes < (size_t)chunk * per_tile) {
            MD_HIP(hipStreamSynchronize(g.stream));   // the buffer may still be in use
            MD_TRY(g.vy.ensure((size_t)chunk * per_tile));
        }
        for (auto &sg : segs) sg.y = g.vy.p;
    }
    std::string tab((const char *)&d, sizeof d);
    tab.append((const char *)segs.data(), segs.size() * sizeof(Seg));
    tab.append((const char *)sl.data(), sl.size() * sizeof(SlabDev));
    if (tab != g.vtab || g.vjob.bytes < sizeof(JobDev) || g.vseg.bytes < segs.size() * sizeof(Seg)) {
        MD_HIP(hipStreamSynchronize(g.stream));
        MD_TRY(g.vjob.ensure(sizeof(JobDev)));
        MD_TRY(g.vseg.ensure(segs.size() * sizeof(Seg)));
        MD_HIP(hipMemcpy(g.vjob.p, &d, sizeof(JobDev), hipMemcpyHostToDevice));
        MD_HIP(hipMemcpy(g.vseg.p, segs.data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice));
        if (!sl.empty()) MD_HIP(hipMemcpy(g.vslabs.p, sl.data(), sl.size() * sizeof(SlabDev), hipMemcpyHostToDevice));
        g.vtab = tab;
    }
    MD_HIP(launch_zero(g.st_d, sizeof(StatsDev), g.stream));
    if (p.path == kPathDirect) {
        double units = 0;
        for (auto &sd : p.slabs) units += sd.dir_cells[p.pack ? 0 : 1];
        ProfScope ps(prof, g.stream, p.pack == 2 ? "direct3_16" : p.pack ? "direct3_16i" : "direct3_32", vox * 8.0, vox * se.ncells * 2.0,
                     vox * units);
        MD_HIP(launch_direct(p.pack, p.sel, (const JobDev *)g.vjob.p, (const Seg *)g.vseg.p, 1, dir_items,
                             occupancy_grid(dir_items, p.lds, kDirThreads), p.lds, g.st_d, g.stream, true));
        ps.done();
    } else {
        const int threads = ntt3_block_threads(p.nt);
        const size_t lds = (size_t)p.nt * p.nt * (p.nt + 1) * sizeof(uint32_t);
        for (size_t c = 0; c < segs.size(); ++c) {
            const Seg *sd = (const Seg *)g.vseg.p + c;
            const long long nt_ = segs[c].ntiles, items = nt_ * p.n;
            const double n3 = (double)p.nt * p.nt * p.nt;
            {
                ProfScope ps(prof, g.stream, "ntt3_n" + std::to_string(p.nt),
                             (double)items * TTT * 4.0 + (double)nt_ * n3 * 4.0,
                             (double)items * ntt3_item_products(p.nt), (double)items);
                MD_HIP(launch_ntt3(p.nt, (const JobDev *)g.vjob.p, sd, 1, items, occupancy_grid(items, lds, threads),
                                   g.ntw, g.ntws, g.st_d, g.stream));
                ps.done();
            }
            {
                const double v = (double)nt_ * TTT;
                const long long ditems = nt_ * pblocks;
                ProfScope ps(prof, g.stream, "decode_ntt3", v * p.n * 4.0 + v * 4.0, v * 8.0 * p.n, v * p.n);
                MD_HIP(launch_ntt3_decode((const JobDev *)g.vjob.p, sd, 1, ditems,
                                          occupancy_grid(ditems, 0, kDecThreads), g.stream));
                ps.done();
            }
        }
    }
    if (g.opt.sync) {
        MD_HIP(hipStreamSynchronize(g.stream));
        resolve_profile();
        MD_HIP(hipMemcpy(g.st_h, g.st_d, sizeof(StatsDev), hipMemcpyDeviceToHost));
        md_stats &st = g.last;
        memset(&st, 0, sizeof st);
        st.tiles = tiles;
        st.direct_jobs = p.path == kPathDirect;
        st.fft_jobs = p.path == kPathFFT;
        st.path = p.path;
        st.n_t = p.path == kPathFFT ? p.nt : 0;
        st.n_r = p.path == kPathFFT ? p.n : 0;
        st.precision = p.path == kPathFFT ? kPrecNTT : g.opt.precision;
        if (g.st_h->range_err) return fail(MD_ERR_RANGE, "a volume value lies outside [0, L-1]");
    }
    g_err.clear();
    return MD_OK;
}

}  // namespace
}  // namespace md

using namespace md;

extern "C" {

int md_dilate(const int32_t *img, int H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets, int k,
              int32_t *out) {
    md_job j{img, H, W, L, se_mask, se_offsets, k, out, 0};
    return run(&j, 1, false);
}

int md_dilate_noalloc(const int32_t *img, int H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets,
                      int k, int32_t *out) {
    g_err.clear();
    return noalloc_dilate(img, H, W, L, se_mask, se_offsets, k, out);
}

int md_erode(const int32_t *img, int H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets, int k,
             int32_t *out) {
    md_job j{img, H, W, L, se_mask, se_offsets, k, out, 1};
    return run(&j, 1, false);
}

int md_dilate_batch(const md_job *jobs, int n) { return run(jobs, n, true); }

int md_dilate_host(const int32_t *img, long long H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets,
                   int k, int32_t *out) {
    return stream_run(0, img, H, W, L, se_mask, se_offsets, k, out);
}

int md_erode_host(const int32_t *img, long long H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets,
                  int k, int32_t *out) {
    return stream_run(1, img, H, W, L, se_mask, se_offsets, k, out);
}

int md_morph3(int op, const int32_t *vol, int D, int H, int W, int L, const uint8_t *se_mask,
              const int32_t *se_offsets, int k, int32_t *out) {
    return morph3(op, vol, D, H, W, L, se_mask, se_offsets, k, out);
}

int md_dilate3_host(const int32_t *vol, long long D, int H, int W, int L, const uint8_t *se_mask,
                    const int32_t *se_offsets, int k, int32_t *out) {
    return stream_run3(0, vol, D, H, W, L, se_mask, se_offsets, k, out);
}

int md_erode3_host(const int32_t *vol, long long D, int H, int W, int L, const uint8_t *se_mask,
                   const int32_t *se_offsets, int k, int32_t *out) {
    return stream_run3(1, vol, D, H, W, L, se_mask, se_offsets, k, out);
}

int md_dilate3(const int32_t *vol, int D, int H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets,
               int k, int32_t *out) {
    return vol_run(0, vol, D, H, W, L, se_mask, se_offsets, k, out);
}

int md_erode3(const int32_t *vol, int D, int H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets,
              int k, int32_t *out) {
    return vol_run(1, vol, D, H, W, L, se_mask, se_offsets, k, out);
}

int md_morph(int op, const int32_t *img, int H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets,
             int k, int32_t *out) {
    return morph(op, img, H, W, L, se_mask, se_offsets, k, out);
}

int md_set_workspace(void *dev_ptr, size_t bytes) {
    if ((dev_ptr == nullptr) != (bytes == 0)) return fail(MD_ERR_ARG, "workspace pointer and size must both be set or both be 0");
    if (dev_ptr && ((uintptr_t)dev_ptr & 255u)) return fail(MD_ERR_ARG, "workspace must be 256-byte aligned");
    if (g.inited) {
        // executors hold pointers into the previous workspace, and their
        // graphs may still run on it
        MD_HIP(hipDeviceSynchronize());
        g.execs.clear(), g.last_exec = nullptr;
    }
    g.ws_ptr = dev_ptr;
    g.ws_bytes = bytes;
    g_err.clear();
    return MD_OK;
}

size_t md_workspace_size(const md_job *jobs, int n) {
    g_err.clear();
    if (n < 1 || !jobs) return fail(MD_ERR_ARG, "empty batch"), 0;
    if (init() != MD_OK) return 0;
    ++g.call_id;
    if (g.opt.path == 0 && g.opt.autotune && !g.tuned && !g.tuning && autotune() != MD_OK) return 0;
    std::vector<SEData> ses(n);
    for (int i = 0; i < n; ++i) {
        if (check_job(jobs[i]) != MD_OK) return 0;
        make_se(jobs[i].se_mask, jobs[i].se_offsets, jobs[i].k, jobs[i].op, ses[i]);
    }
    Exec ex;
    if (build_exec(jobs, n, ses, ex, true) != MD_OK) return 0;
    return ex.ws_need;
}

int md_memory_usage(size_t *cache_bytes, size_t *plan_bytes, int *plans) {
    if (!cache_bytes || !plan_bytes || !plans) return fail(MD_ERR_ARG, "null pointer");
    *cache_bytes = g.cache_bytes;
    size_t t = 0;
    for (auto &kv : g.execs) t += kv.second->ws_own.bytes;
    *plan_bytes = t;
    *plans = (int)g.execs.size();
    return MD_OK;
}

int md_plan(const md_job *job, int batch, md_plan_info *out) {
    if (!job || !out) return fail(MD_ERR_ARG, "null pointer");
    MD_TRY(check_job(*job));
    SEData se;
    make_se(job->se_mask, job->se_offsets, job->k, job->op, se);
    Plan p;
    MD_TRY(plan_job(*job, se, p, batch == 0));
    memset(out, 0, sizeof *out);
    out->path = p.path;
    out->precision = p.dbl;
    out->cost_fft_ns = p.cost_fft;
    out->cost_direct_ns = p.cost_dir;
    out->fp32_bound = NAN;
    if (p.path == kPathFFT) {
        out->n_t = p.nt;
        out->T = p.T;
        out->n_r = p.nr;
        out->bins = p.bins;
        out->tiles_x = p.tiles_x;
        out->tiles_y = p.tiles_y;
        out->decode_fft = p.dec_fft ? 1 : 0;
        out->n_t64 = p.nt64;
        out->fp32_bound = fp32_error_bound(p.nt, p.nr, se.ncells);
    }
    g_err.clear();
    return MD_OK;
}

int md_debug_dft16(int variant, const float *in, float *out, long long lines, int reps) {
    g_err.clear();
    if (variant < 0 || variant > 2) return fail(MD_ERR_ARG, "variant %d must be 0, 1 or 2", variant);
    if (lines <= 0 || lines % 64 != 0) return fail(MD_ERR_ARG, "lines=%lld must be a positive multiple of 64", lines);
    if (reps < 1 || reps > 64) return fail(MD_ERR_ARG, "reps=%d outside [1, 64]", reps);
    if (!in || !out) return fail(MD_ERR_ARG, "null pointer");
    MD_TRY(init());
    MD_HIP(launch_dft16(variant, (const float2 *)in, (float2 *)out, lines, reps, g.stream));
    MD_HIP(hipStreamSynchronize(g.stream));
    return MD_OK;
}

int md_debug_perturb_tiles(const long long *tiles, const uint8_t *bits, int n) {
    if (n < 0 || (n > 0 && (!tiles || !bits))) return fail(MD_ERR_ARG, "null tile list");
    g.perturb.clear();
    for (int i = 0; i < n; ++i) {
        if (tiles[i] < 0) return fail(MD_ERR_ARG, "negative tile index");
        g.perturb.push_back({tiles[i], bits[i]});
    }
    g_err.clear();
    return MD_OK;
}

int md_debug_tile_flags(uint32_t *dst, long long cap, long long *n) {
    if (!n || (cap > 0 && !dst)) return fail(MD_ERR_ARG, "null pointer");
    *n = 0;
    if (!g.inited || !g.last_exec) return MD_OK;
    Exec &ex = *g.last_exec;
    *n = ex.nflags;
    const long long c = std::min(cap, ex.nflags);
    if (c > 0) {
        MD_HIP(hipStreamSynchronize(g.stream));
        MD_HIP(hipMemcpy(dst, ex.flags, (size_t)c * sizeof(uint32_t), hipMemcpyDeviceToHost));
    }
    g_err.clear();
    return MD_OK;
}

int md_set_stream(void *hip_stream) {
    g.stream = (hipStream_t)hip_stream;
    return MD_OK;
}

int md_set_option(int key, double v) {
    Options &o = g.opt;
    switch (key) {
        case MD_OPT_PRECISION:
            if (v != 0 && v != 1 && v != 2) return fail(MD_ERR_ARG, "precision must be 0, 1 or 2");
            o.precision = (int)v;
            break;
        case MD_OPT_BAND:
            if (!(v >= 0 && v <= 0.5)) return fail(MD_ERR_ARG, "band must lie in [0, 0.5]");
            o.band = v;
            break;
        case MD_OPT_PATH:
            if (v != 0 && v != 1 && v != 2) return fail(MD_ERR_ARG, "path must be 0, 1 or 2");
            o.path = (int)v;
            break;
        case MD_OPT_TILE:
            if (v != 0 && !(v >= 8 && v <= kMaxN && v == floor(v) && ((int)v & ((int)v - 1)) == 0))
                return fail(MD_ERR_ARG, "tile must be 0 or a power of two in [8, %d]", kMaxN);
            o.tile = (int)v;
            break;
        case MD_OPT_NR:
            if (v < 0 || v > 4096 || v != floor(v)) return fail(MD_ERR_ARG, "range length must be an integer in [0, 4096]");
            o.nr = (int)v;
            break;
        case MD_OPT_SYNC: o.sync = v != 0; break;
        case MD_OPT_GRAPH: o.graph = v != 0; break;
        case MD_OPT_WORKSPACE_MB:
            if (!(v >= 1)) return fail(MD_ERR_ARG, "workspace cap must be >= 1 MiB");
            o.ws_mb = v;
            break;
        case MD_OPT_PROFILE: o.profile = v != 0; break;
        case MD_OPT_AUTOTUNE: o.autotune = v != 0; break;
        case MD_OPT_STREAM_ROWS:
            if (!(v >= 0 && v <= 0x7fffffff) || v != floor(v)) return fail(MD_ERR_ARG, "band rows must be an integer >= 0");
            o.stream_rows = (int)v;
            break;
        case MD_OPT_STREAM_MB:
            if (!(v >= 1)) return fail(MD_ERR_ARG, "band buffer budget must be >= 1 MiB");
            o.stream_mb = v;
            break;
        case MD_OPT_CACHE_MB:
            if (!(v >= 1)) return fail(MD_ERR_ARG, "cache bound must be >= 1 MiB");
            o.cache_mb = v;
            break;
        default: return fail(MD_ERR_ARG, "unknown option %d", key);
    }
    g_err.clear();
    return MD_OK;
}

double md_get_option(int key) {
    const Options &o = g.opt;
    switch (key) {
        case MD_OPT_PRECISION: return o.precision;
        case MD_OPT_BAND: return o.band;
        case MD_OPT_PATH: return o.path;
        case MD_OPT_TILE: return o.tile;
        case MD_OPT_NR: return o.nr;
        case MD_OPT_SYNC: return o.sync;
        case MD_OPT_GRAPH: return o.graph;
        case MD_OPT_WORKSPACE_MB: return o.ws_mb;
        case MD_OPT_PROFILE: return o.profile;
        case MD_OPT_AUTOTUNE: return o.autotune;
        case MD_OPT_STREAM_ROWS: return o.stream_rows;
        case MD_OPT_STREAM_MB: return o.stream_mb;
        case MD_OPT_CACHE_MB: return o.cache_mb;
        default: return NAN;
    }
}

int md_get_stats(md_stats *s) {
    if (!s) return fail(MD_ERR_ARG, "null stats pointer");
    *s = g.last;
    return MD_OK;
}

const char *md_last_error(void) { return g_err.c_str(); }

int md_profile_get(md_stage_time *out, int max, int *n) {
    if (!n || (max > 0 && !out)) return fail(MD_ERR_ARG, "null pointer");
    if (g.inited && !g.pending.empty()) {
        MD_HIP(hipStreamSynchronize(g.stream));
        resolve_profile();
    }
    int q = 0;
    for (auto &kv : g.prof) {
        if (q < max) {
            md_stage_time &t = out[q];
            memset(&t, 0, sizeof t);
            snprintf(t.name, sizeof t.name, "%s", kv.first.c_str());
            t.ms = kv.second.ms;
            t.launches = kv.second.launches;
            t.alg_bytes = kv.second.bytes;
            t.alg_ops = kv.second.ops;
            t.units = kv.second.units;
        }
        ++q;
    }
    *n = q;
    return MD_OK;
}

int md_profile_reset(void) {
    if (g.inited && !g.pending.empty()) {
        MD_HIP(hipStreamSynchronize(g.stream));
        resolve_profile();
    }
    g.prof.clear();
    return MD_OK;
}

int md_cost_model(double *dst, int n, int *measured) {
    if (!dst || !measured) return fail(MD_ERR_ARG, "null pointer");
    if (n < kCostValues) return fail(MD_ERR_ARG, "cost model needs %d values (n=%d)", kCostValues, n);
    dst[0] = g.cost.dir_cell[0];
    dst[1] = g.cost.dir_cell[1];
    dst[2] = g.cost.dir_stage;
    dst[3] = g.cost.dec_unit[0];
    dst[4] = g.cost.dec_unit[1];
    for (int q = 0; q < 7; ++q) dst[5 + q] = g.cost.fft_item[0][4 + q];
    for (int q = 0; q < 7; ++q) dst[12 + q] = g.cost.fft_item[1][4 + q];
    for (int q = 0; q < 4; ++q) dst[19 + q] = g.cost.fft_item[2][4 + q];
    dst[23] = g.cost.dec_unit[2];
    *measured = g.cost_measured ? 1 : 0;
    return MD_OK;
}

int md_release(void) {
    if (!g.inited) return MD_OK;
    (void)hipDeviceSynchronize();
    g.execs.clear(), g.last_exec = nullptr;
    g.cache.clear();
    g.cache_bytes = 0;
    g.se_work.release();
    g.se_in.release();
    g.morph_a.release();
    g.morph_b.release();
    g.vjob.release();
    g.vseg.release();
    g.vslabs.release();
    g.vy.release();
    g.vtab.clear();
    for (int i = 0; i < 2; ++i) {
        g.hs_in[i].release();
        g.hs_out[i].release();
        for (hipEvent_t *e : {&g.ev_up[i], &g.ev_comp[i], &g.ev_down[i]})
            if (*e) (void)hipEventDestroy(*e), *e = nullptr;
    }
    g.hs_flag.release();
    if (g.ev_fork) (void)hipEventDestroy(g.ev_fork);
    if (g.ev_join) (void)hipEventDestroy(g.ev_join);
    if (g.s_side) (void)hipStreamDestroy(g.s_side);
    g.ev_fork = g.ev_join = nullptr;
    g.s_side = nullptr;
    if (g.s_up) (void)hipStreamDestroy(g.s_up);
    if (g.s_down) (void)hipStreamDestroy(g.s_down);
    g.s_up = g.s_down = nullptr;
    if (g.tw64) (void)hipFree(g.tw64);
    if (g.tw32) (void)hipFree(g.tw32);
    if (g.ntw) (void)hipFree(g.ntw);
    if (g.ntws) (void)hipFree(g.ntws);
    g.ntw = g.ntws = nullptr;
    if (g.st_d) (void)hipFree(g.st_d);
    if (g.st_h) (void)hipHostFree(g.st_h);
    g.tw64 = nullptr;
    g.tw32 = nullptr;
    g.st_d = nullptr;
    g.st_h = nullptr;
    g.inited = false;
    g.device = -1;
    return MD_OK;
}

int md_debug_tile_values(const int32_t *img, int H, int W, int L, const uint8_t *se_mask, const int32_t *se_offsets,
                         int k, int n_t, int n_r, int precision, int ty, int tx, double *dst) {
    MD_TRY(init());
    ++g.call_id;
    if (!dst) return fail(MD_ERR_ARG, "null destination");
    const Options saved = g.opt;
    g.opt.path = kPathFFT;
    g.opt.tile = n_t;
    g.opt.nr = n_r;
    g.opt.precision = precision;
    g.opt.ws_mb = 1e9;
    g.opt.dc_plane = 1;   // the read-back includes bin 0
    md_job j{img, H, W, L, se_mask, se_offsets, k, nullptr, 0};
    int32_t dummy_out_marker = 0;
    (void)dummy_out_marker;
    std::vector<SEData> ses(1);
    int rc = MD_OK;
    Exec ex;
    do {
        if (!img || !se_mask || !se_offsets) { rc = fail(MD_ERR_ARG, "null pointer"); break; }
        j.out = (int32_t *)(uintptr_t)1;   // never written: decode is skipped
        rc = check_job(j);
        if (rc != MD_OK) break;
        make_se(se_mask, se_offsets, k, 0, ses[0]);
        rc = build_exec(&j, 1, ses, ex);
        if (rc != MD_OK) break;
        const Plan &p = ex.plans[0];
        if (ty < 0 || ty >= p.tiles_y || tx < 0 || tx >= p.tiles_x) { rc = fail(MD_ERR_ARG, "tile index out of range"); break; }
        rc = enqueue(ex, g.stream, true);
        if (rc != MD_OK) break;
        if (hipStreamSynchronize(g.stream) != hipSuccess) { rc = fail(MD_ERR_DEVICE, "synchronise failed"); break; }
        const int tile = ty * p.tiles_x + tx;
        const Seg &s = ex.waves[0].fft[0].segs[0];
        const size_t TT = (size_t)p.T * p.T, n = (size_t)p.bins * TT;
        const int ybs = plan_ybs(p);
        const size_t nt_elems = ytile_elems(p.bins, p.T, ybs);
        const double sc = 1.0 / ((double)p.nt * p.nt);
        const size_t esz = elem_bytes(p.dbl);
        std::vector<char> hb(nt_elems * esz), h(n * esz);
        const char *src = (const char *)s.y + (size_t)(tile - s.tile0) * nt_elems * esz;
        if (hipMemcpy(hb.data(), src, nt_elems * esz, hipMemcpyDeviceToHost) != hipSuccess) { rc = fail(MD_ERR_DEVICE, "copy failed"); break; }
        for (int m = 0; m < p.bins; ++m)   // bin-major, whatever the device layout
            for (size_t q = 0; q < TT; ++q)
                memcpy(h.data() + ((size_t)m * TT + q) * esz, hb.data() + (ybin_offset(m, p.T, ybs) + ypix(q, ybs)) * esz,
                       esz);
        for (size_t q = 0; q < n; ++q) {
            if (p.dbl == kPrecNTT) {   // residues mod p, already scaled by n_t^-2
                dst[2 * q] = ((const uint32_t *)h.data())[q];
                dst[2 * q + 1] = 0;
            } else if (p.dbl) {
                const double2 v = ((const double2 *)h.data())[q];
                dst[2 * q] = v.x * sc;
                dst[2 * q + 1] = v.y * sc;
            } else {
                const float2 v = ((const float2 *)h.data())[q];
                dst[2 * q] = v.x * sc;
                dst[2 * q + 1] = v.y * sc;
            }
        }
    } while (0);
    g.opt = saved;
    if (rc == MD_OK) g_err.clear();
    return rc;
}

}  // extern "C"
