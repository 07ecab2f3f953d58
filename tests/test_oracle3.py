"""Pins for the volume (three image axes) oracle, no GPU.

The definitions of Sec. 2.1 hold for N-dimensional images, and Sec. 3 turns
an N-dimensional dilation into an (N+1)-dimensional umbra convolution.  Each
check ties ``oracle.dilate3`` / ``oracle.erode3`` to something other than
itself: scipy's N-dimensional grey-scale morphology, Theorem 1 applied voxel
by voxel, the umbra convolution of Steps 1-3 computed in four dimensions with
numpy's FFT, the 2-D oracle (itself pinned to the paper's worked examples) on
volumes and SEs that have one slice, and the algebra of dilation / erosion.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from paper_2305_03018_amd import synthetic


def reflect3(a):
    return np.ascontiguousarray(a[::-1, ::-1, ::-1])


def test_vs_scipy_nd_grey_morphology():
    rng = np.random.default_rng(31)
    for _ in range(12):
        D, H, W = (int(v) for v in rng.integers(3, 14, 3))
        k = int(rng.integers(0, 3)) * 2 + 1
        L = 32
        job = synthetic.random_vol_job(rng, D, H, W, L, k, p=0.6, max_off=9)
        job.mask[k // 2, k // 2, k // 2] = 1     # scipy needs a non-empty window everywhere
        fp = job.mask.astype(bool)
        g = ndi.grey_dilation(job.vol.astype(np.float64), footprint=fp,
                              structure=job.off.astype(np.float64), mode="constant", cval=-1e9)
        assert np.array_equal(oracle.dilate3(job.vol, job.mask, job.off), g.astype(np.int32))
        e = ndi.grey_erosion(job.vol.astype(np.float64), footprint=fp,
                             structure=job.off.astype(np.float64), mode="constant", cval=1e9)
        assert np.array_equal(oracle.erode3(job.vol, job.mask, job.off, L), e.astype(np.int32))


def test_flat_cube_is_moving_max():
    rng = np.random.default_rng(32)
    vol = rng.integers(0, 256, (9, 13, 17)).astype(np.int32)
    for k in (1, 3, 5):
        mask = synthetic.cube_mask3(k)
        off = np.zeros((k, k, k), np.int32)
        assert np.array_equal(oracle.dilate3(vol, mask, off),
                              ndi.maximum_filter(vol, size=k, mode="constant", cval=-1))
        assert np.array_equal(oracle.erode3(vol, mask, off, 256),
                              ndi.minimum_filter(vol, size=k, mode="constant", cval=1 << 20))


def test_theorem1_voxel_by_voxel_tiny():
    rng = np.random.default_rng(33)
    for _ in range(4):
        job = synthetic.random_vol_job(rng, 3, 4, 5, 8, 3, p=0.5, max_off=3)
        assert np.array_equal(oracle.dilate3(job.vol, job.mask, job.off),
                              oracle.poly_dilate_nd(job.vol, job.mask, job.off))


def test_four_dimensional_umbra_convolution():
    """Steps 1-3 with N = 3: one-hot umbras of the volume and the SE, their
    full 4-D convolution by FFT, and the top degree (Eq. (9))."""
    rng = np.random.default_rng(34)
    for _ in range(6):
        D, H, W = (int(v) for v in rng.integers(3, 9, 3))
        k = int(rng.integers(0, 3)) * 2 + 1
        job = synthetic.random_vol_job(rng, D, H, W, 16, k, p=0.6, max_off=5)
        if not job.mask.any():
            continue
        assert np.array_equal(oracle.dilate3(job.vol, job.mask, job.off),
                              oracle.method_dilate_nd(job.vol, job.mask, job.off))


def test_nd_method_agrees_with_2d_method():
    """The N-D form of Steps 1-3 reduces to the 2-D one."""
    rng = np.random.default_rng(35)
    job = synthetic.random_job(rng, 11, 9, 16, 5, p=0.6, max_off=4)
    assert np.array_equal(oracle.method_dilate_nd(job.img, job.mask, job.off),
                          oracle.method_dilate(job.img, job.mask, job.off))


def test_one_slice_reduces_to_2d():
    """A volume of one slice with any SE, and any volume with an SE that lives
    in its centre slab, act slice by slice as the 2-D dilation with that slab."""
    rng = np.random.default_rng(36)
    k = 5
    for op in (0, 1):
        job = synthetic.random_vol_job(rng, 6, 12, 10, 32, k, p=0.6, max_off=6)
        slab = job.mask[k // 2].copy(), job.off[k // 2].copy()
        m3 = np.zeros_like(job.mask)
        m3[k // 2] = slab[0]
        o3 = np.zeros_like(job.off)
        o3[k // 2] = slab[1]
        if op == 0:
            got = oracle.dilate3(job.vol, m3, o3)
            want = np.stack([oracle.dilate(s, *slab) for s in job.vol])
            one = oracle.dilate3(job.vol[:1], job.mask, job.off)
            want1 = oracle.dilate(job.vol[0], *slab)
        else:
            got = oracle.erode3(job.vol, m3, o3, 32)
            want = np.stack([oracle.erode(s, *slab, 32) for s in job.vol])
            one = oracle.erode3(job.vol[:1], job.mask, job.off, 32)
            want1 = oracle.erode(job.vol[0], *slab, 32)
        assert np.array_equal(got, want)
        assert np.array_equal(one[0], want1)


def test_slab_decomposition():
    """max over SE slabs of 2-D dilations of shifted slices (a volume SE is
    the union of its slabs): voxel (z, y, x) takes slab a from slice z-(a-r)."""
    rng = np.random.default_rng(37)
    k, D = 3, 5
    job = synthetic.random_vol_job(rng, D, 8, 9, 16, k, p=0.7, max_off=4)
    r = k // 2
    want = np.full(job.vol.shape, -(1 << 20), np.int64)
    for a in range(k):
        if not job.mask[a].any():
            continue
        for z in range(D):
            s = z - (a - r)
            if 0 <= s < D:
                d2 = oracle.dilate_e(job.vol[s], job.mask[a], job.off[a], -(1 << 20))
                want[z] = np.maximum(want[z], d2)
    want = np.where(want < 0, 0, want)
    assert np.array_equal(oracle.dilate3(job.vol, job.mask, job.off), want)


def test_duality_and_empty_windows():
    rng = np.random.default_rng(38)
    L = 24
    job = synthetic.random_vol_job(rng, 7, 6, 8, L, 5, p=0.5, max_off=7)
    # erosion(f, b) = (L-1) - dilation((L-1) - f, reflected b)
    e = oracle.erode3(job.vol, job.mask, job.off, L)
    d = oracle.dilate3(L - 1 - job.vol, reflect3(job.mask), reflect3(job.off))
    assert np.array_equal(e, L - 1 - d)
    # an SE cell far outside a 2 x 2 x 2 volume: every window is empty
    k = 7
    mask = np.zeros((k, k, k), np.uint8)
    mask[0, 0, 0] = 1
    off = np.zeros((k, k, k), np.int32)
    off[0, 0, 0] = 5
    vol = rng.integers(0, L, (2, 2, 2)).astype(np.int32)
    assert np.array_equal(oracle.dilate3(vol, mask, off), np.zeros_like(vol))
    assert np.array_equal(oracle.erode3(vol, mask, off, L), np.full_like(vol, L - 1))
    # an empty SE
    assert np.array_equal(oracle.dilate3(vol, np.zeros_like(mask), off), np.zeros_like(vol))


def test_at3_matches_full():
    rng = np.random.default_rng(39)
    job = synthetic.random_vol_job(rng, 6, 7, 9, 16, 3, p=0.7, max_off=3)
    full_d = oracle.dilate3(job.vol, job.mask, job.off)
    full_e = oracle.erode3(job.vol, job.mask, job.off, 16)
    zs, ys, xs = (rng.integers(0, n, 40) for n in job.vol.shape)
    assert np.array_equal(oracle.at3(job.vol, job.mask, job.off, 16, 0, zs, ys, xs), full_d[zs, ys, xs])
    assert np.array_equal(oracle.at3(job.vol, job.mask, job.off, 16, 1, zs, ys, xs), full_e[zs, ys, xs])


def test_volume_recipes():
    v = synthetic.blurred_volume(0, shape=(8, 16, 16), L=16, k=5, max_off=3)
    assert v.vol.shape == (8, 16, 16) and v.vol.min() >= 0 and v.vol.max() <= 15
    assert v.mask.shape == (5, 5, 5) and v.mask[2, 2, 2] == 1 and v.mask[0, 0, 0] == 0
    assert (v.off[v.mask == 0] == 0).all() and v.off.max() <= 3
    b = synthetic.ball_mask3(7)
    assert b.sum() == sum(1 for a in range(7) for i in range(7) for j in range(7)
                          if (a - 3) ** 2 + (i - 3) ** 2 + (j - 3) ** 2 <= 9)


def test_volume_compositions_reduce_to_2d():
    """On a one-slice volume with an SE in its centre slab, every volume
    composition equals the (pinned) image composition of the slice."""
    rng = np.random.default_rng(40)
    k, L = 5, 16
    job = synthetic.random_vol_job(rng, 1, 23, 19, L, k, p=0.6, max_off=4)
    slab_m, slab_o = job.mask[k // 2].copy(), job.off[k // 2].copy()
    m3 = np.zeros_like(job.mask)
    m3[k // 2] = slab_m
    o3 = np.zeros_like(job.off)
    o3[k // 2] = slab_o
    for op in range(7):
        assert np.array_equal(oracle.morph3(op, job.vol, m3, o3, L)[0], oracle.morph(op, job.vol[0], slab_m, slab_o, L)), op


def test_volume_compositions_algebra():
    rng = np.random.default_rng(41)
    L = 16
    for p in (0.5, 1.0):
        job = synthetic.random_vol_job(rng, 7, 9, 10, L, 3, p=p, max_off=3)
        f, mk, of = job.vol, job.mask, job.off
        o = oracle.opening3(f, mk, of, L)
        c = oracle.closing3(f, mk, of, L)
        assert (o <= f).all() and (c >= f).all()
        m = oracle.max_offset(mk, of)
        # idempotence: the second pass runs on the first result's range
        assert np.array_equal(oracle.dilate3_e(oracle.erode3_e(o, mk, of, L - 1), mk, of, -m), o)
        assert np.array_equal(oracle.erode3_e(oracle.dilate3_e(c, mk, of, -m), mk, of, L - 1 + m), c)
        # complement duality with the reflected SE
        cd = oracle.closing3(L - 1 - f, reflect3(mk), reflect3(of), L)
        assert np.array_equal(o, L - 1 - cd)


def test_volume_flat_opening_vs_scipy_interior():
    rng = np.random.default_rng(42)
    vol = rng.integers(0, 32, (12, 14, 15)).astype(np.int32)
    k = 3
    mask = synthetic.cube_mask3(k)
    off = np.zeros((k, k, k), np.int32)
    r = 2 * (k // 2)    # two SE radii: untouched by the border in both steps
    inner = (slice(r, -r),) * 3
    assert np.array_equal(oracle.opening3(vol, mask, off, 32)[inner], ndi.grey_opening(vol, size=k)[inner])
    assert np.array_equal(oracle.closing3(vol, mask, off, 32)[inner], ndi.grey_closing(vol, size=k)[inner])
