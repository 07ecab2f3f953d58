"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Dilation and erosion results are integers, so every comparison is bit-exact
(numpy array_equal), for every path (FFT of umbras / direct window), every
precision (FP64, FP32 + exact recompute) and every tile length.
"""
import numpy as np
import pytest

import oracle
import paper_2305_03018_amd as md
from paper_2305_03018_amd import synthetic

pytestmark = pytest.mark.gpu

FFT64 = dict(precision=1, path=1)
FFT32 = dict(precision=0, path=1)
DIRECT = dict(path=2)
NTT = dict(precision=2, path=1)
MODES = {"fft64": FFT64, "fft32": FFT32, "direct": DIRECT, "ntt": NTT}


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    md.load()
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)


def run_job(job, dev, **opts):
    import torch

    img = torch.from_numpy(job.img).to(dev)
    with md.options(**opts):
        f = md.dilate if job.op == 0 else md.erode
        out = f(img, job.mask, job.off, job.L)
        st = md.get_stats()
    return out.cpu().numpy(), st


def assert_parity(job, dev, want=None, **opts):
    if want is None:
        want = oracle.run_job(job)
    _say(f"  case {job.name} op={job.op} opts={opts}")
    got, st = run_job(job, dev, **opts)
    bad = got != want
    assert not bad.any(), (f"{job.name} op={job.op} {opts}: {int(bad.sum())} of {bad.size} pixels differ; "
                           f"first at {np.argwhere(bad)[0].tolist()} got {got[bad][0]} want {want[bad][0]}")
    return st


def embed_1d(values, origin):
    n = len(values)
    r = max(origin, n - 1 - origin)
    k = 2 * r + 1
    mask = np.zeros((k, k), np.uint8)
    off = np.zeros((k, k), np.int32)
    for idx, v in enumerate(values):
        if v is not None:
            mask[r, idx - origin + r] = 1
            off[r, idx - origin + r] = v
    return mask, off


# ----------------------------------------------------------------------------
# the paper's worked example (Sec. 2.1, Example 2; Sec. 3, Example 5)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["fft64", "fft32", "direct", "ntt"])
@pytest.mark.parametrize("tile", [0, 16, 64])
def test_paper_example2(dev, mode, tile):
    mask, off = embed_1d([1, 2, None, 0], 1)
    job = synthetic.Job(np.array([[3, 0, 7, 6, 2, 7]], np.int32), 8, mask, off, 0, "example2")
    got, _ = run_job(job, dev, tile=tile, **MODES[mode])
    assert got[0].tolist() == [5, 8, 9, 8, 8, 9]
    job.op = 1
    got, _ = run_job(job, dev, tile=tile, **MODES[mode])
    assert got[0].tolist() == [1, -2, -1, 4, 0, 1]


# ----------------------------------------------------------------------------
# seeded random cases spanning several tiles and ragged tails
# ----------------------------------------------------------------------------
RANDOM_CASES = [
    # H, W, L, k, p, max_off, op
    (150, 203, 16, 7, 0.7, 3, 0),
    (150, 203, 16, 7, 0.7, 3, 1),
    (97, 131, 2, 3, 1.0, 0, 0),
    (61, 300, 64, 15, 0.5, 16, 0),
    (61, 300, 64, 15, 0.5, 16, 1),
    (257, 129, 8, 1, 1.0, 5, 0),
    (33, 33, 32, 31, 0.4, 8, 1),
    (200, 45, 256, 11, 0.6, 40, 0),
]


@pytest.mark.parametrize("case", RANDOM_CASES, ids=lambda c: "x".join(map(str, c)))
def test_random_parity(dev, case):
    H, W, L, k, p, max_off, op = case
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    job = synthetic.random_job(rng, H, W, L, k, p=p, max_off=max_off, op=op)
    want = oracle.run_job(job)
    for name, opts in MODES.items():
        tiles = [0] if name == "direct" else [t for t in (16, 32, 64, 128) if t >= k and not (t == 128 and name == "fft64")]
        for t in tiles:
            assert_parity(job, dev, want=want, tile=t, **opts)


def test_forced_nr_lengths(dev):
    rng = np.random.default_rng(21)
    job = synthetic.random_job(rng, 120, 90, 16, 9, p=0.6, max_off=6)
    want = oracle.run_job(job)
    nr_min = 15 + int(job.off.max()) + 1
    for nr in (nr_min, nr_min + 1, 32, 77):
        for opts in (FFT32, FFT64):
            assert_parity(job, dev, want=want, nr=nr, **opts)
    with pytest.raises(md.MDError):
        run_job(job, dev, nr=nr_min - 1, **FFT32)


# ----------------------------------------------------------------------------
# exact recompute of ambiguous tiles
# ----------------------------------------------------------------------------
def test_forced_recompute_all_and_none(dev):
    job = synthetic.blurred_512(0)
    want = oracle.run_job(job)
    st = assert_parity(job, dev, want=want, band=0.0, **FFT32)
    assert st["fallback_tiles"] == st["tiles"] > 0
    st = assert_parity(job, dev, want=want, band=0.5, **FFT32)
    assert st["fallback_tiles"] == 0


def test_recompute_large_se_fp64_large_tile(dev):
    rng = np.random.default_rng(22)
    job = synthetic.random_job(rng, 140, 170, 8, 61, p=0.5, max_off=2)
    want = oracle.run_job(job)
    st = assert_parity(job, dev, want=want, band=0.0, **FFT32)
    assert st["fallback_tiles"] == st["tiles"] > 0


# ----------------------------------------------------------------------------
# edge cases
# ----------------------------------------------------------------------------
def test_edge_shapes_and_masks(dev):
    rng = np.random.default_rng(23)
    cases = []
    for H, W in ((1, 1), (1, 37), (41, 1), (2, 2)):
        cases.append(synthetic.random_job(rng, H, W, 16, 5, p=0.8, max_off=3))
    j = synthetic.random_job(rng, 40, 50, 16, 7, p=0.5, max_off=3)
    j.mask[:] = 0
    j.off[:] = 0
    j.name = "empty_mask"
    cases.append(j)
    j = synthetic.random_job(rng, 3, 70, 16, 9, p=0.5, max_off=3)
    j.mask[4, 4] = 0
    j.mask[:, :] = 0
    j.mask[0, 0] = 1      # only y = (-4, -4): every window of a 3-row image is empty
    j.off[:] = 0
    j.name = "all_windows_empty"
    cases.append(j)
    j = synthetic.random_job(rng, 64, 64, 16, 1, p=1.0, max_off=0)
    j.name = "identity_1x1"
    cases.append(j)
    for job in cases:
        for op in (0, 1):
            job.op = op
            want = oracle.run_job(job)
            for name, opts in MODES.items():
                if name != "direct" and not job.mask.any():
                    continue   # the FFT path needs at least one SE cell
                assert_parity(job, dev, want=want, **opts)
            assert_parity(job, dev, want=want)


def test_largest_se_and_widest_range(dev):
    rng = np.random.default_rng(24)
    job = synthetic.random_job(rng, 300, 280, 4, 127, p=0.3, max_off=1)
    want = oracle.run_job(job)
    assert_parity(job, dev, want=want, **DIRECT)
    assert_parity(job, dev, want=want, **FFT32)          # 128-point tiles, 2 outputs per side
    job = synthetic.random_job(rng, 70, 90, 4000, 3, p=1.0, max_off=90)   # nr up to 4090
    want = oracle.run_job(job)
    assert_parity(job, dev, want=want, **FFT32)
    assert_parity(job, dev, want=want, **FFT64)
    assert_parity(job, dev, want=want)


def test_direct_32bit_form(dev):
    """Tonal ranges where (L-1) + max offset exceeds 16383 take the int32 form
    of the direct window (SE staged in LDS up to the LDS size, else read
    through scalar loads); the transform path does not cover them."""
    rng = np.random.default_rng(27)
    cases = [(77, 190, 20000, 7, 0.7, 100, 0), (77, 190, 20000, 7, 0.7, 100, 1),
             (130, 260, 1 << 20, 41, 0.5, 1000, 0), (40, 300, 30000, 127, 0.2, 5, 1),
             (1, 129, 17000, 3, 1.0, 0, 0)]
    for H, W, L, k, p, max_off, op in cases:
        job = synthetic.random_job(rng, H, W, L, k, p=p, max_off=max_off, op=op)
        want = oracle.run_job(job)
        assert_parity(job, dev, want=want, **DIRECT)
        assert_parity(job, dev, want=want)


def _with_top(job, max_off):
    """Sets the first active SE cell's offset to max_off, so that the largest
    reachable sum is exactly (L-1) + max_off."""
    i, j = np.argwhere(job.mask)[0]
    job.off[i, j] = max_off
    return job


def _direct_stage(job, dev):
    md.profile_reset()
    with md.options(profile=1, graph=0):
        run_job(job, dev, **DIRECT)
    return [s for s in md.profile_get() if s.startswith("direct")]


def test_direct_packed_forms(dev):
    """The packed direct window computes in f16 while every reachable sum
    (L-1) + max offset is at most 2048 (integers that f16 holds exactly), in
    int16 up to 16383, and in int32 beyond.  Cases at and just past each
    boundary, with masked cells, erosion and empty windows, match the oracle
    exactly and run the form their range selects."""
    rng = np.random.default_rng(31)
    cases = [
        # H, W, L, k, p, max_off, op, stage
        (70, 150, 2049, 3, 1.0, 0, 0, "direct16"),       # top 2048: f16, sums reach it
        (70, 150, 2049, 5, 0.6, 0, 1, "direct16"),
        (90, 140, 2000, 7, 0.7, 47, 0, "direct16"),      # top 2046
        (90, 140, 2000, 9, 0.7, 49, 1, "direct16"),      # top 2048
        (90, 140, 2000, 7, 0.7, 50, 0, "direct16i"),     # top 2049: int16
        (90, 140, 2000, 41, 0.3, 50, 1, "direct16i"),
        (65, 257, 16000, 15, 0.5, 384, 0, "direct16i"),  # top 16383
        (65, 257, 16000, 15, 0.5, 384, 1, "direct16i"),
        (65, 257, 16000, 15, 0.5, 385, 0, "direct32"),   # top 16384: int32
    ]
    for H, W, L, k, p, max_off, op, stage in cases:
        job = _with_top(synthetic.random_job(rng, H, W, L, k, p=p, max_off=max_off, op=op), max_off)
        want = oracle.run_job(job)
        assert_parity(job, dev, want=want, **DIRECT)
        assert _direct_stage(job, dev) == [stage], (job.name, stage)
    # one SE cell far from the origin: windows near the borders are empty
    # (dilation 0, erosion L-1)
    for L, max_off, stage in ((2049, 0, "direct16"), (3000, 77, "direct16i")):
        for op in (0, 1):
            img = rng.integers(0, L, (50, 300)).astype(np.int32)
            mask = np.zeros((41, 41), np.uint8)
            off = np.zeros((41, 41), np.int32)
            mask[0, 40] = 1
            off[0, 40] = max_off
            job = synthetic.Job(img, L, mask, off, op, f"corner41_L{L}")
            assert_parity(job, dev, **DIRECT)
            assert _direct_stage(job, dev) == [stage]


def test_range_fft_decode(dev):
    """Power-of-two range lengths from 8 to 4096, the short lengths 2M (M
    from 4 to 24 in FP64 and to 45 in FP32 with no prime factor above 5), and
    in FP32 the lengths 3 2^a up to 1536 and 5 2^a up to 640, decode by a
    range-axis FFT (even and odd
    coefficients from one complex inverse transform of half length) instead
    of the dense inverse DFT.  Forced lengths in both
    precisions, erosion, several tiles with ragged edges, and the exact
    recompute of every tile (band 0), all bit-exact."""
    rng = np.random.default_rng(41)
    cases = [
        # H, W, L, k, p, max_off, op, nr
        # short lengths: one pixel per thread in registers
        (61, 77, 6, 5, 0.8, 2, 0, 8),
        (90, 45, 8, 13, 0.6, 2, 1, 10),
        (33, 140, 9, 7, 0.7, 3, 0, 12),
        (100, 99, 12, 3, 1.0, 4, 1, 16),
        (71, 129, 16, 21, 0.5, 4, 0, 20),
        (130, 64, 18, 9, 0.6, 5, 1, 24),
        (57, 88, 25, 11, 0.7, 7, 0, 32),
        (120, 111, 32, 31, 0.6, 8, 1, 40),
        (66, 95, 40, 15, 0.6, 8, 0, 48),
        # short lengths with factors 3 and 5 beyond one (M = 9 .. 45)
        (77, 91, 12, 9, 0.7, 5, 1, 18),
        (95, 60, 20, 7, 0.6, 8, 0, 30),
        (64, 130, 28, 11, 0.8, 7, 1, 36),
        (101, 83, 40, 5, 0.7, 9, 0, 50),
        (58, 147, 44, 13, 0.6, 9, 1, 54),
        (120, 75, 48, 9, 0.7, 11, 0, 60),
        (93, 118, 60, 17, 0.6, 10, 1, 72),
        (81, 139, 70, 7, 0.8, 18, 0, 90),
        (133, 171, 48, 9, 0.7, 12, 1, 64),
        (150, 203, 100, 7, 0.7, 27, 0, 128),
        (97, 181, 200, 9, 0.6, 50, 1, 256),
        (130, 140, 256, 15, 0.5, 255, 0, 512),
        (70, 260, 900, 5, 0.8, 100, 1, 1024),
        (40, 90, 1800, 3, 1.0, 200, 0, 2048),
        (60, 70, 4000, 3, 1.0, 90, 0, 4096),
        # 3 2^a lengths (the FP32 FFT decode; FP64 decodes them, and the 5 2^a
        # lengths below, densely)
        (141, 99, 70, 11, 0.6, 20, 0, 96),
        (120, 170, 150, 9, 0.6, 40, 0, 192),
        (100, 150, 300, 11, 0.7, 80, 1, 384),
        (64, 200, 600, 5, 0.9, 160, 0, 768),
        (50, 80, 1200, 3, 1.0, 300, 1, 1536),
        # 5 2^a lengths (FP32 FFT decode)
        (157, 203, 64, 21, 0.6, 16, 0, 80),
        (88, 131, 50, 41, 0.8, 12, 1, 80),
        (110, 160, 120, 7, 0.6, 35, 1, 160),
        (90, 140, 250, 9, 0.7, 60, 0, 320),
        (60, 150, 500, 5, 0.9, 130, 1, 640),
    ]
    for H, W, L, k, p, max_off, op, nr in cases:
        job = _with_top(synthetic.random_job(rng, H, W, L, k, p=p, max_off=max_off, op=op), max_off)
        want = oracle.run_job(job)
        for opts in (FFT32, FFT64):
            st = assert_parity(job, dev, want=want, nr=nr, **opts)
            assert st["n_r"] == nr and st["max_residual"] < 0.25, st
        assert_parity(job, dev, want=want, nr=nr, band=0.0, **FFT32)


def test_planner_picks_fft_decode(dev):
    """An 8-bit range (n_r >= 287), and one of 230, on the transform path:
    the planner prices the smallest range length with the dense decode
    against the next power of two with the FFT decode; either way the result
    is exact."""
    rng = np.random.default_rng(43)
    img = rng.integers(0, 256, (300, 280)).astype(np.int32)
    mask = synthetic.disk_mask(31)
    off = (rng.integers(0, 32, (31, 31)) * mask).astype(np.int32)
    for op in (0, 1):
        job = synthetic.Job(img, 256, mask, off, op, "octave_like_300x280_L256_disk31")
        want = oracle.run_job(job)
        for opts in (FFT32, FFT64):
            st = assert_parity(job, dev, want=want, **opts)
            assert st["n_r"] in (int((mask * off).max()) + 256, 320, 384, 512), st
    # a range length between 128 and 256: the smallest length or 256
    img = rng.integers(0, 115, (260, 230)).astype(np.int32)
    off = (rng.integers(0, 116, (31, 31)) * mask).astype(np.int32)
    off[15, 15] = 115
    job = synthetic.Job(img, 115, mask, off, 0, "mid_range_260x230_L115_disk31")
    want = oracle.run_job(job)
    for opts in (FFT32, FFT64):
        st = assert_parity(job, dev, want=want, **opts)
        assert st["n_r"] in (230, 256), st


def test_large_se_fft_only(dev):
    """SEs beyond the direct window's limit (k > 127) go through the FFT path
    with spatial tiles larger than the LDS (256 to 1024 points per side)."""
    rng = np.random.default_rng(25)
    job = synthetic.random_job(rng, 520, 610, 8, 151, p=0.5, max_off=2)
    want = oracle.run_job(job)
    for t in (256, 512, 1024):
        assert_parity(job, dev, want=want, tile=t, **FFT32)
    for t in (256, 512):
        assert_parity(job, dev, want=want, tile=t, **FFT64)
    st = assert_parity(job, dev, want=want)              # auto: must take the FFT path
    assert st["fft_jobs"] == 1 and st["n_t"] >= 256
    job.op = 1
    want = oracle.run_job(job)
    assert_parity(job, dev, want=want, tile=256, **FFT32)
    with pytest.raises(md.MDError) as ei:
        run_job(job, dev, **DIRECT)
    assert ei.value.code == -5


def test_large_tiles_mid_se_and_recompute(dev):
    """Large tiles for moderate SEs, in both precisions, and the FP64
    recompute on large tiles (every tile forced through it)."""
    rng = np.random.default_rng(26)
    job = synthetic.random_job(rng, 700, 333, 16, 41, p=0.6, max_off=4)
    want = oracle.run_job(job)
    assert_parity(job, dev, want=want, tile=256, **FFT32)
    assert_parity(job, dev, want=want, tile=128, **FFT64)
    assert_parity(job, dev, want=want, tile=256, **FFT64)
    st = assert_parity(job, dev, want=want, tile=256, band=0.0, **FFT32)
    assert st["fallback_tiles"] == st["tiles"] > 0
    st = assert_parity(job, dev, want=want, tile=128, band=0.0, **FFT32)
    assert st["fallback_tiles"] == st["tiles"] > 0


def test_errors(dev):
    import torch

    job = synthetic.small_uniform(0)
    img = torch.from_numpy(job.img).to(dev)
    bad = img.clone()
    bad[3, 5] = 16
    # the range check on every transform form: LDS-resident tiles and the
    # large-tile passes (whose bin-0 items are written in closed form)
    for opts in (FFT32, FFT64, DIRECT, dict(FFT32, tile=256), dict(FFT64, tile=128), dict(FFT64, tile=256)):
        with md.options(**opts), pytest.raises(md.MDError) as ei:
            md.dilate(bad, job.mask, job.off, 16)
        assert ei.value.code == -2, opts
    neg = job.off.copy()
    neg[0, 0] = -1
    with pytest.raises(md.MDError) as ei:
        md.dilate(img, job.mask, neg, 16)
    assert ei.value.code == -2
    with pytest.raises(md.MDError) as ei:
        md.dilate(img, np.ones((4, 4)), np.zeros((4, 4)), 16)
    assert ei.value.code == -1
    with pytest.raises(md.MDError) as ei:
        md.dilate(img, job.mask, job.off, 1)
    assert ei.value.code == -1
    out = torch.full_like(img, 123)
    with pytest.raises(md.MDError):
        md.dilate(img, np.ones((4, 4)), np.zeros((4, 4)), 16, out=out)
    assert (out == 123).all()
    # the library still works after errors
    assert_parity(job, dev)


def test_wide_rows_and_value_cache_bounds(dev):
    """Image rows wider than 2^22 pixels take the transform's plain image
    loads instead of the 32-bit buffer offsets; grey ranges up to 256 keep a
    tile's values in the per-block byte cache, wider ones reload them; a value
    past the range (256 with L = 256, which the byte cache would wrap to 0)
    is still reported."""
    import torch

    rng = np.random.default_rng(47)
    wide = synthetic.random_job(rng, 3, (1 << 22) + 37, 16, 5, p=0.7, max_off=3)
    want = oracle.run_job(wide)
    for opts in (FFT32, FFT64):
        _say(f"  wide rows {opts}")
        assert_parity(wide, dev, want=want, **opts)
    for L in (256, 257):
        job = synthetic.random_job(rng, 150, 170, L, 9, p=0.6, max_off=6, op=L % 2)
        assert_parity(job, dev, tile=32, **FFT32)
    job = synthetic.random_job(rng, 100, 120, 256, 7, p=0.6, max_off=5)
    bad = torch.from_numpy(job.img).to(dev)
    bad[57, 33] = 256
    for opts in (FFT32, FFT64):
        with md.options(**opts), pytest.raises(md.MDError) as ei:
            md.dilate(bad, job.mask, job.off, 256)
        assert ei.value.code == -2


# ----------------------------------------------------------------------------
# transform-domain values against the FP64 reference
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("nr", [24, 128])
def test_spectrum_error_report(dev, nr):
    """Transform-domain values of one tile against the DFT of the oracle's
    exact coefficients; at a power-of-two range length the tile is stored in
    blocks of 16 pixels (the FFT decode's layout) and read back bin-major."""
    import torch

    job = synthetic.blurred_512(0)
    img = torch.from_numpy(job.img).to(dev)
    for nt in (64, 128):   # four and (FP32) eight lanes per tile line
        T = nt - job.k + 1
        for ty, tx in ((2, 3), (0, 0)):   # an inner tile and a corner tile (partial windows)
            ys, xs = np.divmod(np.arange(T * T), T)
            counts = oracle.counts_at(job.img, job.mask, job.off, ty * T + ys, tx * T + xs, nr)
            ref = oracle.range_spectrum_ref(counts, nr).T           # (bins, T*T)
            for prec, tol in ((0, 2e-5), (1, 1e-12)):
                got = md.debug_tile_values(img, job.mask, job.off, job.L, nt, nr, prec, ty, tx)
                rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                mx = np.abs(got - ref).max()
                _say(f"  nt={nt} tile=({ty},{tx}) precision={prec}: relative L2 {rel:.3e}, max abs {mx:.3e}")
                assert rel < tol
                # bin 0 is the sum of the pixel's exact coefficients (the DFT at
                # m = 0), written in closed form: equal in every precision
                assert np.array_equal(got[0].real, counts.sum(axis=1).astype(np.float64))
                assert not got[0].imag.any()


def test_tile_values_dense_decode_plan(dev):
    """A plan whose decode takes bin 0 in closed form (n_r = 5, 3 bins): the
    read-back still holds bin 0's plane, the exact coefficient sums, and the
    other bins within the spectrum tolerance."""
    import torch

    rng = np.random.default_rng(41)
    job = synthetic.random_job(rng, 160, 150, 4, 9, p=0.6, max_off=1)
    img = torch.from_numpy(job.img).to(dev)
    nt, nr = 64, 5
    T = nt - job.k + 1
    for ty, tx in ((0, 0), (1, 2)):
        ys, xs = np.divmod(np.arange(T * T), T)
        counts = oracle.counts_at(job.img, job.mask, job.off, ty * T + ys, tx * T + xs, nr)
        ref = oracle.range_spectrum_ref(counts, nr).T
        for prec, tol in ((0, 2e-5), (1, 1e-12)):
            got = md.debug_tile_values(img, job.mask, job.off, job.L, nt, nr, prec, ty, tx)
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < tol
            assert np.array_equal(got[0].real, counts.sum(axis=1).astype(np.float64))
    want = oracle.run_job(job)
    for opts in (FFT32, FFT64):
        for t in (64, 256):
            st = assert_parity(job, dev, want=want, tile=t, nr=nr, **opts)
            assert st["n_r"] == nr, st


def test_ntt_exact_counts(dev):
    """The exact path's transform-domain values of one tile, inverted over
    the range axis on the host with Python integers, are the exact polynomial
    coefficients c_x(d) of every degree (not only the top one)."""
    import torch

    p, g = 7340033, 3
    job = synthetic.blurred_512(0)
    img = torch.from_numpy(job.img).to(dev)
    nt, n = 64, 28                      # (L-1) + max offset + 1 = 23 <= 28 = 7 * 4
    T = nt - job.k + 1
    for ty, tx in ((0, 0), (2, 3), (7, 9)):
        y = md.debug_tile_values(img, job.mask, job.off, job.L, nt, n, 2, ty, tx).real.astype(np.int64)
        assert y.shape == (n, T * T) and y.min() >= 0 and y.max() < p
        w = pow(g, (p - 1) // n, p)
        ninv = pow(n, p - 2, p)
        ys, xs = np.divmod(np.arange(T * T), T)
        want = oracle.counts_at(job.img, job.mask, job.off, ty * T + ys, tx * T + xs, n)
        yl = [[int(v) for v in row] for row in y]
        for q in range(0, T * T, 7):
            for d in range(n):
                c = sum(yl[m][q] * pow(w, (n - d * m % n) % n, p) for m in range(n)) % p * ninv % p
                assert c == want[q, d], (ty, tx, q, d, c, want[q, d])


def test_repeatable(dev):
    job = synthetic.blurred_512(0)
    a, sa = run_job(job, dev, **FFT32)
    b, sb = run_job(job, dev, **FFT32)
    assert np.array_equal(a, b) and sa["max_residual"] == sb["max_residual"]


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["fft64", "fft32", "direct"])
def test_small_uniform_64(dev, mode):
    job = synthetic.small_uniform(0)
    assert_parity(job, dev, **MODES[mode])


@pytest.mark.parametrize("op", [0, 1])
def test_blurred_512(dev, op):
    job = synthetic.blurred_512(0, op=op)
    want = oracle.run_job(job)
    for name, opts in MODES.items():
        assert_parity(job, dev, want=want, **opts)
    for tile in (32, 64, 128):
        assert_parity(job, dev, want=want, tile=tile, **FFT32)
    st = assert_parity(job, dev, want=want)   # auto plan
    assert st["window_tiles"] == 0


@pytest.mark.parametrize("flat", [True, False])
def test_large_random_mask_2048(dev, flat):
    job = synthetic.large_random_mask(0, flat=flat)
    want = oracle.run_job(job)
    st = assert_parity(job, dev, want=want, **FFT32)
    _say(f"  stats {st}")
    assert st["max_residual"] < 0.25
    assert_parity(job, dev, want=want, **DIRECT)
    if flat:
        assert_parity(job, dev, want=want, **FFT64)


@pytest.mark.parametrize("op", [0, 1])
def test_octave_noise_4096(dev, op):
    """The 4096^2 8-bit workload at full size, every pixel: FP32 + exact
    recompute, plain FP64, the direct window and the auto plan, for dilation
    and erosion."""
    job = synthetic.octave_noise_4096(0)
    job.op = op
    want = oracle.run_job(job)
    st = assert_parity(job, dev, want=want, **FFT32)
    _say(f"  stats {st}")
    assert st["max_residual"] < 0.25 and st["window_tiles"] == 0
    st = assert_parity(job, dev, want=want, **FFT64)
    _say(f"  stats {st}")
    assert st["max_residual"] < 1e-6 and st["window_tiles"] == 0
    assert_parity(job, dev, want=want, **DIRECT)
    assert_parity(job, dev, want=want)


_BATCH_WANT = {}


def _batch_want(jobs):
    """Oracle results of the 256-job batch, computed once per module."""
    if "uneven" not in _BATCH_WANT:
        _BATCH_WANT["uneven"] = [oracle.run_job(j) for j in jobs]
    return _BATCH_WANT["uneven"]


def _batch_parity(jobs, outs):
    for job, out, want in zip(jobs, outs, _batch_want(jobs)):
        got = out.cpu().numpy()
        assert np.array_equal(got, want), f"{job.name}: {int((got != want).sum())} pixels differ"


@pytest.mark.parametrize("mode", ["auto", "fft32", "fft64", "ntt"])
def test_uneven_batch_256(dev, mode):
    """All 256 jobs of the uneven batch, every pixel, in each mode."""
    import torch

    jobs = synthetic.uneven_batch(0, 256)
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    opts = {"auto": {}, "fft32": FFT32, "fft64": FFT64, "ntt": NTT}[mode]
    _say(f"  batch of {len(jobs)} mode={mode}")
    with md.options(**opts):
        outs = md.dilate_batch([(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)])
        st = md.get_stats()
        _say(f"  stats {st}")
        _batch_parity(jobs, outs)
        assert st["window_tiles"] == 0
        # replay with new output buffers (same signature -> graph replay)
        outs2 = [torch.full_like(o, -7) for o in outs]
        md.dilate_batch([(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)], outs=outs2)
        for a, b in zip(outs, outs2):
            assert torch.equal(a, b)


@pytest.mark.parametrize("mode", ["auto", "fft32", "direct"])
def test_many_tiny_jobs(dev, mode):
    """1500 jobs of 1x1 to 40x40 pixels in one batch call: segment tables
    and their binary search over many short segments, a graph with many
    segments, k from 1 to 9, L from 2 to 300, both operations, masks that
    can be empty; every job exact."""
    import torch

    rng = np.random.default_rng(77)
    jobs = []
    for i in range(1500):
        H, W = (int(v) for v in rng.integers(1, 41, 2))
        L = int(rng.choice([2, 5, 16, 64, 300]))
        k = int(rng.integers(0, 5)) * 2 + 1
        jobs.append(synthetic.random_job(rng, H, W, L, k, p=float(rng.choice([0.0, 0.4, 1.0])),
                                         max_off=int(rng.integers(0, 8)), op=i % 2))
    if mode == "fft32":   # the transform path needs at least one SE cell
        jobs = [j for j in jobs if j.mask.any()]
    opts = {"auto": {}, "fft32": FFT32, "direct": DIRECT}[mode]
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    _say(f"  {len(jobs)} tiny jobs mode={mode}")
    with md.options(**opts):
        outs = md.dilate_batch([(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)])
    for q, (j, o) in enumerate(zip(jobs, outs)):
        got, want = o.cpu().numpy(), oracle.run_job(j)
        assert np.array_equal(got, want), f"{mode} job {q} ({j.name}, op {j.op}): {int((got != want).sum())} differ"
