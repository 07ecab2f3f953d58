"""CPU oracle for exact grey-scale dilation / erosion.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import this package; the product library
(``paper_2305_03018_amd``) never does, and the two share no code.

Two layers, both plain and slow on purpose:

* ``oracle.c`` (loaded here through ctypes): the definitions of dilation
  (Sec. 2.1, Eq. (6new) with the empty-window rule of Eq. (6)), erosion
  (Eq. (Erosion)) and of the exact integer polynomial coefficients that the
  umbra convolution produces at each pixel (Sec. 3.1, Eq. (Obs7)).
* Python/numpy below: the paper's own objects, used to pin the C layer on
  small inputs -- the degree function and its one-hot inverse (Sec. 2.2,
  Eqs. (Degree) and (InvDelta)), polynomial products summed per pixel
  (Theorem 1), the umbras of Step 1 (Eqs. (7)-(8)), the full-mode umbra
  convolution of Step 2 done with numpy's FFT as the paper does (Sec. 4.1),
  and the top-degree read-out of Step 3 (Eq. (9)).

Readings of points the paper leaves open (listed with the design notes):
odd k with the SE origin at the centre cell; an empty erosion window gives
L-1; out-of-domain pixels and SE cells are the zero polynomial.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "oracle.c")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc + OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-std=c11", "-Wall", _SRC_PATH, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_dilate.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _u8p, _i32p, ctypes.c_int, _i32p]
        lib.oracle_erode.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u8p, _i32p,
                                     ctypes.c_int, _i32p]
        lib.oracle_at.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u8p, _i32p,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i32p]
        lib.oracle_counts_at.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _u8p, _i32p, ctypes.c_int,
                                         ctypes.c_int, _i32p, _i32p, ctypes.c_int, _i32p, _i64p]
        lib.oracle_dilate_e.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _u8p, _i32p, ctypes.c_int,
                                        ctypes.c_int32, _i32p]
        lib.oracle_erode_e.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, _u8p, _i32p, ctypes.c_int,
                                       ctypes.c_int32, _i32p]
        lib.oracle_dilate3_e.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u8p, _i32p,
                                         ctypes.c_int, ctypes.c_int32, _i32p]
        lib.oracle_erode3_e.argtypes = lib.oracle_dilate3_e.argtypes
        lib.oracle_at3.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _u8p, _i32p,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i32p, _i32p]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _prep(img, mask, off):
    img = np.ascontiguousarray(img, dtype=np.int32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int32)
    if img.ndim != 2 or mask.ndim != 2 or mask.shape != off.shape or mask.shape[0] != mask.shape[1]:
        raise ValueError("img must be 2-D and mask/off k x k")
    if mask.shape[0] % 2 != 1:
        raise ValueError("SE side must be odd")
    return img, mask, off


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


# ----------------------------------------------------------------------------
# definitions (C layer)
# ----------------------------------------------------------------------------
def dilate(img, mask, off) -> np.ndarray:
    """Eq. (6new) / (6): max of f(x-y)+b(y) over the window, 0 if empty."""
    img, mask, off = _prep(img, mask, off)
    out = np.empty_like(img)
    _load().oracle_dilate(_p(img, _i32p), img.shape[0], img.shape[1], _p(mask, _u8p),
                          _p(off, _i32p), mask.shape[0], _p(out, _i32p))
    return out


def erode(img, mask, off, L: int) -> np.ndarray:
    """Eq. (Erosion): min of f(x+y)-b(y) over the window, L-1 if empty."""
    img, mask, off = _prep(img, mask, off)
    out = np.empty_like(img)
    _load().oracle_erode(_p(img, _i32p), img.shape[0], img.shape[1], int(L), _p(mask, _u8p),
                         _p(off, _i32p), mask.shape[0], _p(out, _i32p))
    return out


def at(img, mask, off, L: int, op: int, ys, xs) -> np.ndarray:
    """Dilation (op 0) or erosion (op 1) at the listed pixels only."""
    img, mask, off = _prep(img, mask, off)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    out = np.empty(ys.shape[0], np.int32)
    _load().oracle_at(_p(img, _i32p), img.shape[0], img.shape[1], int(L), _p(mask, _u8p),
                      _p(off, _i32p), mask.shape[0], int(op), ys.shape[0], _p(ys, _i32p),
                      _p(xs, _i32p), _p(out, _i32p))
    return out


def counts_at(img, mask, off, ys, xs, nd: int) -> np.ndarray:
    """Exact coefficients c_x(d), d < nd, of the per-pixel polynomial that the
    umbra convolution gives (Sec. 3.1, Eq. (Obs7)); shape (n, nd)."""
    img, mask, off = _prep(img, mask, off)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    out = np.empty((ys.shape[0], nd), np.int32)
    ovf = np.zeros(1, np.int64)
    _load().oracle_counts_at(_p(img, _i32p), img.shape[0], img.shape[1], _p(mask, _u8p),
                             _p(off, _i32p), mask.shape[0], ys.shape[0], _p(ys, _i32p),
                             _p(xs, _i32p), int(nd), _p(out, _i32p), _p(ovf, _i64p))
    if ovf[0]:
        raise ValueError(f"{int(ovf[0])} degrees fall outside [0, {nd})")
    return out


def counts(img, mask, off, nd: int) -> np.ndarray:
    """counts_at over every pixel; shape (H, W, nd)."""
    H, W = np.asarray(img).shape
    ys, xs = np.divmod(np.arange(H * W, dtype=np.int64), W)
    return counts_at(img, mask, off, ys, xs, nd).reshape(H, W, nd)


# ----------------------------------------------------------------------------
# compositions (Sec. 5: opening, closing, Beucher gradient "combined" from the
# exact dilation and erosion)
# ----------------------------------------------------------------------------
def dilate_e(img, mask, off, empty: int) -> np.ndarray:
    """Dilation of any int32 image, `empty` where the window is empty."""
    img, mask, off = _prep(img, mask, off)
    out = np.empty_like(img)
    _load().oracle_dilate_e(_p(img, _i32p), img.shape[0], img.shape[1], _p(mask, _u8p), _p(off, _i32p),
                            mask.shape[0], int(empty), _p(out, _i32p))
    return out


def erode_e(img, mask, off, empty: int) -> np.ndarray:
    """Erosion of any int32 image, `empty` where the window is empty."""
    img, mask, off = _prep(img, mask, off)
    out = np.empty_like(img)
    _load().oracle_erode_e(_p(img, _i32p), img.shape[0], img.shape[1], _p(mask, _u8p), _p(off, _i32p),
                           mask.shape[0], int(empty), _p(out, _i32p))
    return out


def max_offset(mask, off) -> int:
    """Largest offset over the active SE cells (0 for an empty SE)."""
    m = np.asarray(mask) != 0
    return int(np.asarray(off)[m].max()) if m.any() else 0


# An empty window takes the bottom (dilation) or the top (erosion) of the range
# its operand can span: [0, L-1] for an input image (the 0 / L-1 rules),
# [-m, L-1] for an erosion result and [0, L-1+m] for a dilation result, with
# m the largest SE offset.
def opening(img, mask, off, L: int) -> np.ndarray:
    """(f erosion b) dilation b."""
    m = max_offset(mask, off)
    return dilate_e(erode_e(img, mask, off, L - 1), mask, off, -m)


def closing(img, mask, off, L: int) -> np.ndarray:
    """(f dilation b) erosion b."""
    m = max_offset(mask, off)
    return erode_e(dilate_e(img, mask, off, 0), mask, off, L - 1 + m)


def gradient(img, mask, off, L: int) -> np.ndarray:
    """Beucher gradient: dilation minus erosion."""
    return dilate(img, mask, off) - erode(img, mask, off, L)


def tophat(img, mask, off, L: int) -> np.ndarray:
    """White top-hat: f minus its opening."""
    return np.asarray(img, np.int32) - opening(img, mask, off, L)


def blackhat(img, mask, off, L: int) -> np.ndarray:
    """Black top-hat: the closing minus f."""
    return closing(img, mask, off, L) - np.asarray(img, np.int32)


MORPH = {0: lambda f, m, o, L: dilate(f, m, o), 1: erode, 2: opening, 3: closing, 4: gradient, 5: tophat,
         6: blackhat}


def morph(op: int, img, mask, off, L: int) -> np.ndarray:
    """Operation `op`: 0 dilation, 1 erosion, 2 opening, 3 closing, 4 Beucher
    gradient, 5 white top-hat, 6 black top-hat."""
    return MORPH[op](img, mask, off, L)


# ----------------------------------------------------------------------------
# volumes (N = 3: the definitions of Sec. 2.1 for three image axes)
# ----------------------------------------------------------------------------
def _prep3(vol, mask, off):
    vol = np.ascontiguousarray(vol, dtype=np.int32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int32)
    if vol.ndim != 3 or mask.ndim != 3 or mask.shape != off.shape or len(set(mask.shape)) != 1:
        raise ValueError("vol must be 3-D and mask/off k x k x k")
    if mask.shape[0] % 2 != 1:
        raise ValueError("SE side must be odd")
    return vol, mask, off


def dilate3_e(vol, mask, off, empty: int = 0) -> np.ndarray:
    """Eq. (6new) over three axes: max of f(x-y)+b(y), `empty` (Eq. (6): 0)
    where the window is empty."""
    vol, mask, off = _prep3(vol, mask, off)
    out = np.empty_like(vol)
    _load().oracle_dilate3_e(_p(vol, _i32p), *vol.shape, _p(mask, _u8p), _p(off, _i32p), mask.shape[0],
                             int(empty), _p(out, _i32p))
    return out


def erode3_e(vol, mask, off, empty: int) -> np.ndarray:
    """Eq. (Erosion) over three axes: min of f(x+y)-b(y), `empty` where the
    window is empty."""
    vol, mask, off = _prep3(vol, mask, off)
    out = np.empty_like(vol)
    _load().oracle_erode3_e(_p(vol, _i32p), *vol.shape, _p(mask, _u8p), _p(off, _i32p), mask.shape[0],
                            int(empty), _p(out, _i32p))
    return out


def dilate3(vol, mask, off) -> np.ndarray:
    return dilate3_e(vol, mask, off, 0)


def erode3(vol, mask, off, L: int) -> np.ndarray:
    return erode3_e(vol, mask, off, L - 1)


def at3(vol, mask, off, L: int, op: int, zs, ys, xs) -> np.ndarray:
    """Volume dilation (op 0) or erosion (op 1) at the listed voxels only."""
    vol, mask, off = _prep3(vol, mask, off)
    zs, ys, xs = (np.ascontiguousarray(a, dtype=np.int32) for a in (zs, ys, xs))
    out = np.empty(zs.shape[0], np.int32)
    _load().oracle_at3(_p(vol, _i32p), *vol.shape, int(L), _p(mask, _u8p), _p(off, _i32p), mask.shape[0],
                       int(op), zs.shape[0], _p(zs, _i32p), _p(ys, _i32p), _p(xs, _i32p), _p(out, _i32p))
    return out


def opening3(vol, mask, off, L: int) -> np.ndarray:
    """Volume opening: the erosion lies in [-m, L-1], so an empty dilation
    window gives -m (as for images)."""
    m = max_offset(mask, off)
    return dilate3_e(erode3_e(vol, mask, off, L - 1), mask, off, -m)


def closing3(vol, mask, off, L: int) -> np.ndarray:
    m = max_offset(mask, off)
    return erode3_e(dilate3_e(vol, mask, off, 0), mask, off, L - 1 + m)


MORPH3 = {0: lambda f, m, o, L: dilate3(f, m, o), 1: erode3, 2: opening3, 3: closing3,
          4: lambda f, m, o, L: dilate3(f, m, o) - erode3(f, m, o, L),
          5: lambda f, m, o, L: np.asarray(f, np.int32) - opening3(f, m, o, L),
          6: lambda f, m, o, L: closing3(f, m, o, L) - np.asarray(f, np.int32)}


def morph3(op: int, vol, mask, off, L: int) -> np.ndarray:
    """Volume operation `op`, numbered as for morph."""
    return MORPH3[op](vol, mask, off, L)


def run_job(job) -> np.ndarray:
    """Oracle result for a ``synthetic.Job``."""
    if job.op == 0:
        return dilate(job.img, job.mask, job.off)
    return erode(job.img, job.mask, job.off, job.L)


# ----------------------------------------------------------------------------
# the paper's objects (Python; small inputs only)
# ----------------------------------------------------------------------------
NEG_INF = float("-inf")


def delta(p: list[int]) -> float:
    """Degree function, Eq. (Degree): highest power with a non-zero
    coefficient, -inf for the zero polynomial."""
    for d in range(len(p) - 1, -1, -1):
        if p[d] != 0:
            return d
    return NEG_INF


def delta_inv(a) -> list[int]:
    """One-hot inverse, Eq. (InvDelta): -inf -> 0, 0 -> 1, a -> x^a."""
    if a == NEG_INF:
        return []
    return [0] * int(a) + [1]


def poly_add(p: list[int], q: list[int]) -> list[int]:
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]


def poly_mul(p: list[int], q: list[int]) -> list[int]:
    """Product of polynomials = full-mode convolution of coefficient lists
    (Sec. 3.1, Eq. (Obs1)), written as the double loop."""
    if not p or not q:
        return []
    out = [0] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def maxplus_by_polynomials(a_list, b_list) -> float:
    """Right-hand side of Theorem 1: delta(sum_i p_{a_i} * p_{b_i})."""
    acc: list[int] = []
    for a, b in zip(a_list, b_list):
        acc = poly_add(acc, poly_mul(delta_inv(a), delta_inv(b)))
    return delta(acc)


def poly_dilate(img, mask, off) -> np.ndarray:
    """Dilation by Theorem 1 applied pixel by pixel: out-of-domain image
    pixels and masked-out SE cells are -inf (Sec. 2.2), every pixel's value
    is the degree of sum_y delta'(f(x-y)) * delta'(b(y)); a zero polynomial
    (empty window) maps to 0 as in Eq. (6)."""
    img = np.asarray(img)
    H, W = img.shape
    k = mask.shape[0]
    r = (k - 1) // 2
    out = np.zeros((H, W), np.int32)
    for x0 in range(H):
        for x1 in range(W):
            a_list, b_list = [], []
            for i in range(k):
                for j in range(k):
                    s0, s1 = x0 - (i - r), x1 - (j - r)
                    a = int(img[s0, s1]) if (0 <= s0 < H and 0 <= s1 < W) else NEG_INF
                    b = int(off[i, j]) if mask[i, j] else NEG_INF
                    a_list.append(a)
                    b_list.append(b)
            d = maxplus_by_polynomials(a_list, b_list)
            out[x0, x1] = 0 if d == NEG_INF else int(d)
    return out


def umbra(values: np.ndarray, valid: np.ndarray, lR: int) -> np.ndarray:
    """Eqs. (7)/(8): one-hot along a new last ('range') axis of length lR+1;
    positions outside the domain get the all-zero vector."""
    values = np.asarray(values)
    u = np.zeros(values.shape + (lR + 1,), np.float64)
    idx = np.nonzero(valid)
    u[idx + (values[idx].astype(np.int64),)] = 1.0
    return u


def method_umbra_conv(img, mask, off) -> tuple[np.ndarray, int]:
    """Steps 1-2 in fp64 as the paper computes them: build the umbras with
    lR = max f + max b (Step 1), then the full-mode convolution on the two
    domain axes and the range axis by numpy's fftn/ifftn (Step 2).  Returns
    the real convolution volume restricted to x in F (shape (H, W, lR+1))
    and lR."""
    img = np.asarray(img, np.int64)
    mask = np.asarray(mask).astype(bool)
    off = np.asarray(off, np.int64)
    H, W = img.shape
    k = mask.shape[0]
    r = (k - 1) // 2
    lR = int(img.max()) + int(off[mask].max() if mask.any() else 0)
    fU = umbra(img, np.ones_like(mask, shape=img.shape), lR)
    bU = umbra(off, mask, lR)
    full = (H + k - 1, W + k - 1, 2 * lR + 1)
    ax = (0, 1, 2)
    conv = np.fft.ifftn(np.fft.fftn(fU, full, axes=ax) * np.fft.fftn(bU, full, axes=ax), axes=ax).real
    # SE index i is the offset y = i - r, so the full-mode output index a is
    # x + r for the pixel x.
    return conv[r:r + H, r:r + W, :lR + 1], lR


def method_dilate(img, mask, off) -> np.ndarray:
    """Steps 1-3: umbra convolution, then Eq. (9): the highest y whose
    (rounded) coefficient is >= 1, or 0 where no coefficient is."""
    conv, lR = method_umbra_conv(img, mask, off)
    c = np.rint(conv)
    hit = c >= 1
    top = (lR - np.argmax(hit[..., ::-1], axis=-1)).astype(np.int32)
    return np.where(hit.any(axis=-1), top, 0).astype(np.int32)


def poly_dilate_nd(img, mask, off) -> np.ndarray:
    """poly_dilate for any number of image axes N (the SE has the same N
    axes, each of odd length, origin at the centre): Theorem 1 applied voxel
    by voxel.  Tiny inputs only."""
    img = np.asarray(img)
    mask = np.asarray(mask)
    r = np.array([(s - 1) // 2 for s in mask.shape])
    out = np.zeros(img.shape, np.int32)
    cells = list(np.ndindex(*mask.shape))
    for x in np.ndindex(*img.shape):
        a_list, b_list = [], []
        for c in cells:
            s = tuple(np.array(x) - (np.array(c) - r))
            inside = all(0 <= s[d] < img.shape[d] for d in range(img.ndim))
            a_list.append(int(img[s]) if inside else NEG_INF)
            b_list.append(int(off[c]) if mask[c] else NEG_INF)
        d = maxplus_by_polynomials(a_list, b_list)
        out[x] = 0 if d == NEG_INF else int(d)
    return out


def method_umbra_conv_nd(img, mask, off) -> tuple[np.ndarray, int]:
    """Steps 1-2 for N image axes (Sec. 3: an N-dimensional image gives an
    (N+1)-dimensional umbra): one-hot umbras with lR = max f + max b, full-mode
    convolution over the N domain axes and the range axis by numpy's fftn in
    fp64.  Returns the convolution restricted to x in F and lR."""
    img = np.asarray(img, np.int64)
    mask = np.asarray(mask).astype(bool)
    off = np.asarray(off, np.int64)
    n = img.ndim
    r = [(s - 1) // 2 for s in mask.shape]
    lR = int(img.max()) + int(off[mask].max() if mask.any() else 0)
    fU = umbra(img, np.ones(img.shape, bool), lR)
    bU = umbra(off, mask, lR)
    full = tuple(img.shape[d] + mask.shape[d] - 1 for d in range(n)) + (2 * lR + 1,)
    ax = tuple(range(n + 1))
    conv = np.fft.ifftn(np.fft.fftn(fU, full, axes=ax) * np.fft.fftn(bU, full, axes=ax), axes=ax).real
    # the full-mode output index along a domain axis is x + r for the voxel x
    sl = tuple(slice(r[d], r[d] + img.shape[d]) for d in range(n)) + (slice(0, lR + 1),)
    return conv[sl], lR


def method_dilate_nd(img, mask, off) -> np.ndarray:
    """Steps 1-3 for N image axes: the umbra convolution, then Eq. (9) -- the
    highest degree whose rounded coefficient is >= 1, 0 where none is."""
    conv, lR = method_umbra_conv_nd(img, mask, off)
    hit = np.rint(conv) >= 1
    top = (lR - np.argmax(hit[..., ::-1], axis=-1)).astype(np.int32)
    return np.where(hit.any(axis=-1), top, 0).astype(np.int32)


def range_spectrum_ref(counts_px: np.ndarray, nr: int) -> np.ndarray:
    """Forward DFT along the range axis of exact coefficient vectors:
    Y_m = sum_d c(d) exp(-2 pi i d m / nr) for m in [0, nr//2].  This is the
    per-bin value a transform-domain implementation holds for a pixel just
    before its inverse range transform; used to report spectrum error."""
    c = np.asarray(counts_px, np.float64)
    nd = c.shape[-1]
    if nd > nr:
        raise ValueError("nr shorter than the coefficient vector")
    m = np.arange(nr // 2 + 1)
    d = np.arange(nd)
    ph = np.exp(-2j * np.pi * np.outer(d, m) / nr)
    return c @ ph
