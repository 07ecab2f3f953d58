/*
 * Driver for a sanitizer build of the CPU oracle (test infrastructure):
 * compiled together with oracle/oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py.  It calls
 * every exported oracle function on exactly sized heap buffers over
 * degenerate and ragged shapes (1 x 1 images, SEs larger than the image,
 * empty masks, single-cell masks far from the origin) and checks a few
 * identities that need no second implementation:
 *   - a 1 x 1 SE with offset c shifts every pixel by c (dilation) or -c
 *     (erosion);
 *   - the exact coefficients of a pixel sum to the number of SE cells whose
 *     window pixel lies in the image, and their top degree is the dilation;
 *   - the sampled forms agree with the whole-image forms.
 * Exit status 0 when all checks pass; the sanitizers abort on any error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_dilate(const int32_t *f, int H, int W, const uint8_t *mask, const int32_t *off, int k, int32_t *out);
void oracle_erode(const int32_t *f, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k, int32_t *out);
void oracle_at(const int32_t *f, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k, int op, int n,
               const int32_t *ys, const int32_t *xs, int32_t *out);
void oracle_counts_at(const int32_t *f, int H, int W, const uint8_t *mask, const int32_t *off, int k, int n,
                      const int32_t *ys, const int32_t *xs, int nd, int32_t *out, int64_t *overflow);
void oracle_dilate3_e(const int32_t *f, int D, int H, int W, const uint8_t *mask, const int32_t *off, int k,
                      int32_t empty, int32_t *out);
void oracle_erode3_e(const int32_t *f, int D, int H, int W, const uint8_t *mask, const int32_t *off, int k,
                     int32_t empty, int32_t *out);
void oracle_at3(const int32_t *f, int D, int H, int W, int L, const uint8_t *mask, const int32_t *off, int k, int op,
                int n, const int32_t *zs, const int32_t *ys, const int32_t *xs, int32_t *out);

static unsigned long long rng_state = 88172645463325252ull;
static unsigned rnd(unsigned n) {   /* xorshift64, uniform enough for test inputs */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (unsigned)(rng_state % n);
}

static int failures = 0;
#define CHECK(c, ...)                        \
    do {                                     \
        if (!(c)) {                          \
            fprintf(stderr, __VA_ARGS__);    \
            fputc('\n', stderr);             \
            ++failures;                      \
        }                                    \
    } while (0)

static void image_case(int H, int W, int L, int k, int pmask, int maxoff) {
    const size_t n = (size_t)H * W, kk = (size_t)k * k;
    int32_t *f = malloc(n * sizeof *f), *dil = malloc(n * sizeof *dil), *ero = malloc(n * sizeof *ero);
    uint8_t *mask = malloc(kk);
    int32_t *off = malloc(kk * sizeof *off);
    for (size_t i = 0; i < n; ++i) f[i] = (int32_t)rnd((unsigned)L);
    int top = 0;
    for (size_t c = 0; c < kk; ++c) {
        mask[c] = rnd(100) < (unsigned)pmask;
        off[c] = mask[c] ? (int32_t)rnd((unsigned)maxoff + 1) : 0;
        if (mask[c] && off[c] > top) top = off[c];
    }
    oracle_dilate(f, H, W, mask, off, k, dil);
    oracle_erode(f, H, W, L, mask, off, k, ero);
    const int m = 2 * (int)n < 64 ? 2 * (int)n : 64;
    int32_t *ys = malloc((size_t)m * sizeof *ys), *xs = malloc((size_t)m * sizeof *xs);
    int32_t *got = malloc((size_t)m * sizeof *got);
    for (int i = 0; i < m; ++i) {
        ys[i] = (int32_t)rnd((unsigned)H);
        xs[i] = (int32_t)rnd((unsigned)W);
    }
    oracle_at(f, H, W, L, mask, off, k, 0, m, ys, xs, got);
    for (int i = 0; i < m; ++i) CHECK(got[i] == dil[(size_t)ys[i] * W + xs[i]], "at/dilate differ");
    oracle_at(f, H, W, L, mask, off, k, 1, m, ys, xs, got);
    for (int i = 0; i < m; ++i) CHECK(got[i] == ero[(size_t)ys[i] * W + xs[i]], "at/erode differ");
    const int nd = L + top;
    int32_t *cnt = malloc((size_t)m * nd * sizeof *cnt);
    int64_t ovf = -1;
    oracle_counts_at(f, H, W, mask, off, k, m, ys, xs, nd, cnt, &ovf);
    CHECK(ovf == 0, "counts overflow %lld", (long long)ovf);
    const int r = (k - 1) / 2;
    for (int i = 0; i < m; ++i) {
        int cells = 0;
        for (int a = 0; a < k; ++a)
            for (int c = 0; c < k; ++c) {
                const int y = ys[i] - (a - r), x = xs[i] - (c - r);
                if (mask[a * k + c] && y >= 0 && y < H && x >= 0 && x < W) ++cells;
            }
        int sum = 0, hi = -1;
        for (int d = 0; d < nd; ++d) {
            sum += cnt[(size_t)i * nd + d];
            if (cnt[(size_t)i * nd + d]) hi = d;
        }
        CHECK(sum == cells, "counts sum %d, window cells %d", sum, cells);
        CHECK((hi < 0 ? 0 : hi) == dil[(size_t)ys[i] * W + xs[i]], "top degree %d vs dilation", hi);
    }
    free(f), free(dil), free(ero), free(mask), free(off), free(ys), free(xs), free(got), free(cnt);
}

static void shift_case(int H, int W, int L, int c) {
    const size_t n = (size_t)H * W;
    int32_t *f = malloc(n * sizeof *f), *o = malloc(n * sizeof *o);
    uint8_t mask = 1;
    int32_t off = c;
    for (size_t i = 0; i < n; ++i) f[i] = (int32_t)rnd((unsigned)L);
    oracle_dilate(f, H, W, &mask, &off, 1, o);
    for (size_t i = 0; i < n; ++i) CHECK(o[i] == f[i] + c, "1x1 dilation shift");
    oracle_erode(f, H, W, L, &mask, &off, 1, o);
    for (size_t i = 0; i < n; ++i) CHECK(o[i] == f[i] - c, "1x1 erosion shift");
    free(f), free(o);
}

static void volume_case(int D, int H, int W, int L, int k) {
    const size_t n = (size_t)D * H * W, kkk = (size_t)k * k * k;
    int32_t *f = malloc(n * sizeof *f), *dil = malloc(n * sizeof *dil), *ero = malloc(n * sizeof *ero);
    uint8_t *mask = malloc(kkk);
    int32_t *off = malloc(kkk * sizeof *off);
    for (size_t i = 0; i < n; ++i) f[i] = (int32_t)rnd((unsigned)L);
    for (size_t c = 0; c < kkk; ++c) {
        mask[c] = rnd(100) < 60;
        off[c] = mask[c] ? (int32_t)rnd(4) : 0;
    }
    oracle_dilate3_e(f, D, H, W, mask, off, k, 0, dil);
    oracle_erode3_e(f, D, H, W, mask, off, k, L - 1, ero);
    const int m = 32;
    int32_t zs[32], ys[32], xs[32], got[32];
    for (int i = 0; i < m; ++i) {
        zs[i] = (int32_t)rnd((unsigned)D);
        ys[i] = (int32_t)rnd((unsigned)H);
        xs[i] = (int32_t)rnd((unsigned)W);
    }
    oracle_at3(f, D, H, W, L, mask, off, k, 0, m, zs, ys, xs, got);
    for (int i = 0; i < m; ++i) CHECK(got[i] == dil[((size_t)zs[i] * H + ys[i]) * W + xs[i]], "at3/dilate3 differ");
    oracle_at3(f, D, H, W, L, mask, off, k, 1, m, zs, ys, xs, got);
    for (int i = 0; i < m; ++i) CHECK(got[i] == ero[((size_t)zs[i] * H + ys[i]) * W + xs[i]], "at3/erode3 differ");
    free(f), free(dil), free(ero), free(mask), free(off);
}

int main(void) {
    static const int shapes[][2] = {{1, 1}, {1, 37}, {41, 1}, {2, 2}, {7, 5}, {33, 60}, {64, 64}};
    static const int ks[] = {1, 3, 5, 9, 41};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        for (size_t q = 0; q < sizeof ks / sizeof ks[0]; ++q)
            for (int pm = 0; pm <= 100; pm += 50) image_case(shapes[s][0], shapes[s][1], 16, ks[q], pm, 5);
    image_case(40, 50, 256, 17, 70, 255);
    image_case(3, 70, 2, 63, 3, 0);
    shift_case(9, 13, 16, 0);
    shift_case(9, 13, 16, 7);
    volume_case(1, 1, 1, 8, 3);
    volume_case(5, 9, 7, 16, 5);
    volume_case(12, 6, 20, 4, 7);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitize driver: OK\n");
    return 0;
}
