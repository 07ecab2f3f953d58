"""CPU tests of the host-side planner (md_plan): no GPU involved.

They check the rules every plan must satisfy whatever the cost model picks:
the overlap-save tiling covers the image, the range length holds every
reachable degree, FP32 is planned only under the worst-case error bound of
the exact tiers, the exact path's range lengths divide p - 1, and the
planner's errors."""
import math

import numpy as np
import pytest

import paper_2305_03018_amd as md
from paper_2305_03018_amd import synthetic

U32 = 2.0 ** -24


def _se(rng, k, p, max_off):
    mask = synthetic.bernoulli_mask(rng, k, p, centre=True)
    off = (rng.integers(0, max_off + 1, (k, k)) * mask).astype(np.int32)
    return mask, off


def _bound(nt, nr, cells):
    # nt sqrt(|B|) 3 log2(nt^2 nr) (u + beta): the range stages count twice
    return nt * math.sqrt(cells) * 3.0 * (math.log2(nt * nt) + 2.0 * math.log2(nr)) * U32


def test_overlap_save_tiles_cover_the_image():
    rng = np.random.default_rng(1)
    for _ in range(60):
        k = int(rng.integers(0, 40)) * 2 + 1
        H, W = (int(v) for v in rng.integers(1, 3000, 2))
        L = int(rng.choice([2, 8, 16, 64, 256]))
        mask, off = _se(rng, k, 0.6, L // 4)
        for tile in (t for t in (16, 32, 64, 128, 256, 512, 1024) if t >= k):
            with md.options(path=1, tile=tile, precision=int(rng.integers(0, 2))):
                p = md.plan((H, W), mask, off, L, batch=True)
            assert p["path"] == 1 and p["n_t"] == tile
            T = tile - k + 1
            assert p["T"] == T
            assert p["tiles_x"] == -(-W // T) and p["tiles_y"] == -(-H // T)
            assert (p["tiles_x"] - 1) * T < W <= p["tiles_x"] * T
            assert (p["tiles_y"] - 1) * T < H <= p["tiles_y"] * T


def test_range_length_holds_every_degree():
    rng = np.random.default_rng(2)
    for _ in range(80):
        k = int(rng.integers(0, 8)) * 2 + 1
        L = int(rng.integers(2, 600))
        mask, off = _se(rng, k, 0.7, int(rng.integers(0, 300)))
        top = (L - 1) + int(off[mask != 0].max())
        for prec in (0, 1):
            with md.options(path=1, precision=prec):
                p = md.plan((300, 200), mask, off, L, op=int(rng.integers(0, 2)))
            assert p["n_r"] >= top + 1
            assert p["bins"] == p["n_r"] // 2 + 1
            n = p["n_r"]
            pow2 = lambda x: x > 0 and x & (x - 1) == 0
            assert p["decode_fft"] == (1 if _fft_decodable(n, p["precision"]) else 0), p


def _smooth(m):
    for f in (2, 3, 5):
        while m % f == 0:
            m //= f
    return m == 1


def _fft_decodable(n, prec):
    """Range lengths with a range-axis FFT decode: 2^a (8..4096); 3 2^a and
    5 2^a up to 1536 and 640 in FP32; and the short decode's 2M with M from 4
    to 45 (FP32) or 24 (FP64), no prime factor above 5, M != 32."""
    pow2 = lambda x: x > 0 and x & (x - 1) == 0
    small = n % 2 == 0 and 4 <= n // 2 <= (24 if prec else 45) and n // 2 != 32 and _smooth(n // 2)
    return small or (8 <= n <= 4096 and pow2(n)) or (prec == 0 and (
        (n % 3 == 0 and 96 <= n <= 1536 and pow2(n // 3)) or (n % 5 == 0 and 80 <= n <= 640 and pow2(n // 5))))


def test_fp32_only_under_the_error_bound():
    """A transform job asked for FP32 is planned FP32 only where the bound
    is at most 0.25; otherwise FP64, at the same forced tile."""
    rng = np.random.default_rng(3)
    seen = set()
    for k, p_mask, tile in ((151, 0.5, 1024), (151, 0.5, 512), (255, 0.9, 512), (255, 0.9, 1024), (41, 1.0, 256),
                            (127, 0.3, 128), (401, 0.5, 1024), (15, 1.0, 64)):
        mask, off = _se(rng, k, p_mask, 2)
        cells = int(mask.sum())
        with md.options(path=1, tile=tile, precision=0):
            p = md.plan((900, 1000), mask, off, 8)
        want = _bound(tile, p["n_r"], cells)
        assert p["fp32_bound"] == pytest.approx(want, rel=1e-12)
        assert p["precision"] == (0 if want <= 0.25 else 1), (k, tile, want, p)
        seen.add(p["precision"])
    assert seen == {0, 1}
    # auto tiles: whatever is picked in FP32 is under the bound
    for _ in range(40):
        k = int(rng.integers(0, 200)) * 2 + 1
        mask, off = _se(rng, k, float(rng.uniform(0.2, 1.0)), int(rng.integers(0, 16)))
        with md.options(path=1, precision=0):
            p = md.plan((2000, 2000), mask, off, int(rng.choice([4, 16, 64])), batch=True)
        if p["precision"] == 0:
            assert p["fp32_bound"] <= 0.25
            assert p["n_t64"] >= p["T"] + k - 1 or p["n_t64"] == 1024


def test_fp32_recompute_tile_covers_the_fp32_tile():
    rng = np.random.default_rng(4)
    for k in (3, 15, 31, 61):
        mask, off = _se(rng, k, 0.8, 3)
        for tile in (t for t in (64, 128, 256) if t > k):
            with md.options(path=1, tile=tile, precision=0):
                p = md.plan((700, 800), mask, off, 16)
            if p["precision"] != 0:
                continue
            nt64 = p["n_t64"]
            assert nt64 & (nt64 - 1) == 0 and nt64 - k + 1 >= p["T"]
            assert nt64 // 2 - k + 1 < p["T"] or nt64 == 16


def test_exact_path_range_lengths():
    rng = np.random.default_rng(5)
    for _ in range(40):
        k = int(rng.integers(0, 10)) * 2 + 1
        L = int(rng.integers(2, 700))
        mask, off = _se(rng, k, 0.6, int(rng.integers(0, 300)))
        top = (L - 1) + int(off[mask != 0].max())
        with md.options(path=1, precision=2):
            if top + 1 > 1024:
                with pytest.raises(md.MDError) as ei:
                    md.plan((200, 200), mask, off, L)
                assert ei.value.code == -5
                continue
            p = md.plan((200, 200), mask, off, L)
        n = p["n_r"]
        cands = [c << a for a in range(11) for c in (1, 7) if (c << a) >= top + 1 and (c << a) <= 1024]
        assert n == min(cands) and p["bins"] == n and p["n_t"] <= 128


def test_paths_and_errors():
    rng = np.random.default_rng(6)
    mask, off = _se(rng, 151, 0.5, 2)
    p = md.plan((600, 600), mask, off, 8)
    assert p["path"] == 1                                   # only the transform covers k > 127
    with md.options(path=2), pytest.raises(md.MDError) as ei:
        md.plan((600, 600), mask, off, 8)
    assert ei.value.code == -5
    empty = np.zeros((9, 9), np.uint8)
    assert md.plan((50, 50), empty, np.zeros((9, 9), np.int32), 16)["path"] == 2
    with md.options(path=1), pytest.raises(md.MDError) as ei:
        md.plan((50, 50), empty, np.zeros((9, 9), np.int32), 16)
    assert ei.value.code == -5
    m5, o5 = _se(rng, 5, 1.0, 3)
    bad = o5.copy()
    bad[2, 2] = -1
    with pytest.raises(md.MDError) as ei:
        md.plan((40, 40), m5, bad, 16)
    assert ei.value.code == -2
    with pytest.raises(md.MDError) as ei:
        md.plan((40, 40), np.ones((4, 4), np.uint8), np.zeros((4, 4), np.int32), 16)
    assert ei.value.code == -1
    with md.options(path=1, nr=10), pytest.raises(md.MDError) as ei:
        md.plan((40, 40), m5, o5, 16)                      # (L-1) + 3 + 1 = 19 > 10
    assert ei.value.code == -1
    with md.options(path=1, nr=19):
        assert md.plan((40, 40), m5, o5, 16)["n_r"] == 19


def test_range_length_candidates():
    """FP paths: the range length is the smallest one, (L-1) + max offset + 1,
    or above it the next 2^a, 3 2^a or 5 2^a, or the shortest length, that
    has a range-axis FFT decode; up to 128 a smallest length that has an FFT
    decode is kept."""
    rng = np.random.default_rng(8)
    for _ in range(120):
        k = int(rng.integers(0, 8)) * 2 + 1
        L = int(rng.choice([int(rng.integers(2, 140)), int(rng.integers(2, 1000))]))
        mask, off = _se(rng, k, 0.7, int(rng.integers(0, max(1, L // 4))))
        nr_min = (L - 1) + int(off[mask != 0].max()) + 1
        for prec in (0, 1):
            with md.options(path=1, precision=prec):
                p = md.plan((400, 300), mask, off, L)
            n = p["n_r"]
            if n == nr_min:
                continue
            prec_p = p["precision"]
            assert p["decode_fft"] == 1 and _fft_decodable(n, prec_p), (nr_min, p)
            nxt = [min(c << a for a in range(13) if (c << a) >= nr_min) for c in (1, 3, 5)]
            first = next(m for m in range(nr_min + 1, 2 * nr_min) if _fft_decodable(m, prec_p))
            assert n in nxt or n == first, (nr_min, n)
            if nr_min <= 128:
                with md.options(path=1, precision=p["precision"], nr=nr_min):
                    assert md.plan((400, 300), mask, off, L)["decode_fft"] == 0, (nr_min, n)
