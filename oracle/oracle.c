/*
 * CPU oracle for exact grey-scale dilation / erosion.  TEST INFRASTRUCTURE
 * ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg may
 * call it; the product library never does, and the two share no code.
 *
 * Everything here is the plain definition, written as nested loops:
 *
 *   dilation   (f (+) b)(x) = max { f(x-y) + b(y) : y in B, x-y in F }   Sec. 2.1, Eq. (6new)
 *              and 0 when that set is empty                             Eq. (6), Eq. (9)
 *   erosion    (f (-) b)(x) = min { f(x+y) - b(y) : y in B, x+y in F }   Sec. 2.1, Eq. (Erosion)
 *              and L-1 when that set is empty (the paper leaves this case
 *              open; L-1 is the complement-duality image of the 0 rule)
 *   compositions (Sec. 5 names them; assembled in the Python layer from the
 *              two definitions above with explicit empty-window values)
 *   counts     c_x(d) = #{ y in B : x-y in F, f(x-y) + b(y) = d }
 *              = the integer coefficients of the polynomial that the
 *              umbra convolution yields at pixel x (Sec. 3.1, Eq. (Obs7)
 *              with the one-hot umbras of Eqs. (7)-(8): every admissible
 *              pair (x-y, y) contributes the monomial t^(f(x-y)+b(y))).
 *
 * Conventions: images are row-major H x W int32; the SE is a k x k array,
 * k odd, origin at the centre cell (r, r) with r = (k-1)/2, so cell (i, j)
 * is the offset y = (i - r, j - r); mask[i*k+j] != 0 marks y in B and
 * off[i*k+j] is b(y).  Rows of the output are independent and are split
 * across OpenMP threads.
 */
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

int oracle_num_threads(void) { return omp_get_max_threads(); }

void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* One output pixel of the dilation; returns 1 and the max in *v if the window
   is non-empty, 0 otherwise. */
static int dil_px(const int32_t *f, int H, int W, const uint8_t *mask,
                  const int32_t *off, int k, int x0, int x1, int64_t *v)
{
    const int r = (k - 1) / 2;
    int any = 0;
    int64_t best = 0;
    for (int i = 0; i < k; ++i) {
        const int s0 = x0 - (i - r);          /* row of x - y */
        if (s0 < 0 || s0 >= H) continue;
        for (int j = 0; j < k; ++j) {
            if (!mask[i * k + j]) continue;
            const int s1 = x1 - (j - r);      /* column of x - y */
            if (s1 < 0 || s1 >= W) continue;
            const int64_t val = (int64_t)f[(size_t)s0 * W + s1] + off[i * k + j];
            if (!any || val > best) { best = val; any = 1; }
        }
    }
    *v = best;
    return any;
}

static int ero_px(const int32_t *f, int H, int W, const uint8_t *mask,
                  const int32_t *off, int k, int x0, int x1, int64_t *v)
{
    const int r = (k - 1) / 2;
    int any = 0;
    int64_t best = 0;
    for (int i = 0; i < k; ++i) {
        const int s0 = x0 + (i - r);          /* row of x + y */
        if (s0 < 0 || s0 >= H) continue;
        for (int j = 0; j < k; ++j) {
            if (!mask[i * k + j]) continue;
            const int s1 = x1 + (j - r);
            if (s1 < 0 || s1 >= W) continue;
            const int64_t val = (int64_t)f[(size_t)s0 * W + s1] - off[i * k + j];
            if (!any || val < best) { best = val; any = 1; }
        }
    }
    *v = best;
    return any;
}

/* Dilation / erosion of an image with any int32 values (an intermediate of a
   composition may be negative or exceed L-1), `empty` where the window is
   empty. */
void oracle_dilate_e(const int32_t *f, int H, int W, const uint8_t *mask,
                     const int32_t *off, int k, int32_t empty, int32_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int x0 = 0; x0 < H; ++x0)
        for (int x1 = 0; x1 < W; ++x1) {
            int64_t v;
            out[(size_t)x0 * W + x1] = dil_px(f, H, W, mask, off, k, x0, x1, &v) ? (int32_t)v : empty;
        }
}

void oracle_erode_e(const int32_t *f, int H, int W, const uint8_t *mask,
                    const int32_t *off, int k, int32_t empty, int32_t *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int x0 = 0; x0 < H; ++x0)
        for (int x1 = 0; x1 < W; ++x1) {
            int64_t v;
            out[(size_t)x0 * W + x1] = ero_px(f, H, W, mask, off, k, x0, x1, &v) ? (int32_t)v : empty;
        }
}

void oracle_dilate(const int32_t *f, int H, int W, const uint8_t *mask,
                   const int32_t *off, int k, int32_t *out)
{
    oracle_dilate_e(f, H, W, mask, off, k, 0, out);
}

void oracle_erode(const int32_t *f, int H, int W, int L, const uint8_t *mask,
                  const int32_t *off, int k, int32_t *out)
{
    oracle_erode_e(f, H, W, mask, off, k, L - 1, out);
}

/* Dilation (op 0) or erosion (op 1) at n listed pixels (ys[i], xs[i]). */
void oracle_at(const int32_t *f, int H, int W, int L, const uint8_t *mask,
               const int32_t *off, int k, int op, int n, const int32_t *ys,
               const int32_t *xs, int32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        int64_t v;
        if (op == 0)
            out[i] = dil_px(f, H, W, mask, off, k, ys[i], xs[i], &v) ? (int32_t)v : 0;
        else
            out[i] = ero_px(f, H, W, mask, off, k, ys[i], xs[i], &v) ? (int32_t)v : L - 1;
    }
}

/* Exact polynomial coefficients c_x(d), d in [0, nd), at n listed pixels;
   out is n x nd.  Pairs whose degree falls outside [0, nd) are counted in
   *overflow so a caller can tell that nd was too small. */
void oracle_counts_at(const int32_t *f, int H, int W, const uint8_t *mask,
                      const int32_t *off, int k, int n, const int32_t *ys,
                      const int32_t *xs, int nd, int32_t *out, int64_t *overflow)
{
    const int r = (k - 1) / 2;
    int64_t ovf = 0;
#pragma omp parallel for schedule(static) reduction(+ : ovf)
    for (int p = 0; p < n; ++p) {
        int32_t *c = out + (size_t)p * nd;
        for (int d = 0; d < nd; ++d) c[d] = 0;
        for (int i = 0; i < k; ++i) {
            const int s0 = ys[p] - (i - r);
            if (s0 < 0 || s0 >= H) continue;
            for (int j = 0; j < k; ++j) {
                if (!mask[i * k + j]) continue;
                const int s1 = xs[p] - (j - r);
                if (s1 < 0 || s1 >= W) continue;
                const int64_t d = (int64_t)f[(size_t)s0 * W + s1] + off[i * k + j];
                if (d >= 0 && d < nd) c[d] += 1; else ovf += 1;
            }
        }
    }
    *overflow = ovf;
}

/* ---- volumes (N = 3; Sec. 2.1 states the definitions for N-dimensional
   images) --------------------------------------------------------------
   Volumes are D x H x W int32, z slowest; the SE is a k x k x k array (k
   odd, origin at the centre cell (r, r, r)), cell (a, i, j) is the offset
   y = (a - r, i - r, j - r), mask[(a*k + i)*k + j] != 0 marks y in B and
   off[...] is b(y).  Dilation / erosion as above, with x - y (x + y) taken
   over all three axes. */
static int vol_px(const int32_t *f, int D, int H, int W, const uint8_t *mask,
                  const int32_t *off, int k, int sgn, int z, int y, int x, int64_t *v)
{
    const int r = (k - 1) / 2;
    int any = 0;
    int64_t best = 0;
    for (int a = 0; a < k; ++a) {
        const int s0 = z - sgn * (a - r);
        if (s0 < 0 || s0 >= D) continue;
        for (int i = 0; i < k; ++i) {
            const int s1 = y - sgn * (i - r);
            if (s1 < 0 || s1 >= H) continue;
            for (int j = 0; j < k; ++j) {
                const size_t c = ((size_t)a * k + i) * k + j;
                if (!mask[c]) continue;
                const int s2 = x - sgn * (j - r);
                if (s2 < 0 || s2 >= W) continue;
                const int64_t fv = f[((size_t)s0 * H + s1) * W + s2];
                /* dilation (sgn = +1): f(x-y) + b(y), largest;
                   erosion (sgn = -1): f(x+y) - b(y), smallest */
                const int64_t val = sgn > 0 ? fv + off[c] : fv - off[c];
                if (!any || (sgn > 0 ? val > best : val < best)) { best = val; any = 1; }
            }
        }
    }
    *v = best;
    return any;
}

void oracle_dilate3_e(const int32_t *f, int D, int H, int W, const uint8_t *mask,
                      const int32_t *off, int k, int32_t empty, int32_t *out)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t v;
                out[((size_t)z * H + y) * W + x] =
                    vol_px(f, D, H, W, mask, off, k, 1, z, y, x, &v) ? (int32_t)v : empty;
            }
}

void oracle_erode3_e(const int32_t *f, int D, int H, int W, const uint8_t *mask,
                     const int32_t *off, int k, int32_t empty, int32_t *out)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t v;
                out[((size_t)z * H + y) * W + x] =
                    vol_px(f, D, H, W, mask, off, k, -1, z, y, x, &v) ? (int32_t)v : empty;
            }
}

/* Dilation (op 0, 0 if empty) or erosion (op 1, L-1 if empty) at n listed
   voxels (zs[i], ys[i], xs[i]). */
void oracle_at3(const int32_t *f, int D, int H, int W, int L, const uint8_t *mask,
                const int32_t *off, int k, int op, int n, const int32_t *zs,
                const int32_t *ys, const int32_t *xs, int32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        int64_t v;
        const int any = vol_px(f, D, H, W, mask, off, k, op == 0 ? 1 : -1, zs[i], ys[i], xs[i], &v);
        out[i] = any ? (int32_t)v : (op == 0 ? 0 : L - 1);
    }
}
