"""GPU: the exact tiers behind the transform passes, through the C ABI.

A decoded tile that fails the exactness checks (residual band, a negative
rounded coefficient, or a rounded-coefficient sum different from the number
of in-image window cells) goes on: FP32 tiles to the FP64 recompute, tiles
that fail in FP64 to the integer window.  The perturbation hook pushes chosen
tiles over the band; the per-tile flags then show exactly which tiles each
tier took, and every output pixel must still equal the oracle's.

Also here: the caller-owned workspace (md_set_workspace /
md_workspace_size) and the bounded device caches.
"""
import numpy as np
import pytest

import oracle
import paper_2305_03018_amd as md
from paper_2305_03018_amd import synthetic

pytestmark = pytest.mark.gpu

FFT64 = dict(precision=1, path=1)
FFT32 = dict(precision=0, path=1)


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    md.load()
    yield torch.device("cuda:0")
    md.debug_perturb_tiles([], [])


def _say(msg):
    print(msg, flush=True)


def _run_batch(jobs, dev, **opts):
    import torch

    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    with md.options(**opts):
        outs = md.dilate_batch([(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)])
        st = md.get_stats()
    return [o.cpu().numpy() for o in outs], st


def _expect_exact(jobs, outs, wants):
    for j, got, want in zip(jobs, outs, wants):
        bad = got != want
        assert not bad.any(), f"{j.name} op={j.op}: {int(bad.sum())} pixels differ"


def _tiles_of(job, nt):
    T = nt - job.k + 1
    H, W = job.img.shape
    return ((H + T - 1) // T) * ((W + T - 1) // T)


def _perturbed(jobs, dev, tiles, bits, **opts):
    md.debug_perturb_tiles(tiles, bits)
    try:
        outs, st = _run_batch(jobs, dev, **opts)
        flags = md.debug_tile_flags()
    finally:
        md.debug_perturb_tiles([], [])
    return outs, st, flags


@pytest.mark.parametrize("nr", [0, 256])
def test_selective_fp64_recompute(dev, nr):
    """FP32: tiles perturbed in the first pass (bit 1) are recomputed in FP64
    and nothing else; a tile perturbed in the FP64 recompute too (bits 1|2)
    reaches the integer window.  Dense decode (nr auto, 23) and the range-axis
    FFT decode (nr 256)."""
    jobs = [synthetic.blurred_512(0, op=0), synthetic.blurred_512(0, op=1)]
    wants = [oracle.run_job(j) for j in jobs]
    n0 = _tiles_of(jobs[0], 64)
    first = [3, 17, 60, n0 + 5, n0 + 44]
    both = [40, n0 + 100]
    tiles = first + both
    bits = [1] * len(first) + [3] * len(both)
    _say(f"  FP32 nr={nr}: {2 * n0} tiles, perturbed {tiles}")
    outs, st, flags = _perturbed(jobs, dev, tiles, bits, tile=64, nr=nr, **FFT32)
    _expect_exact(jobs, outs, wants)
    assert flags.shape == (2 * n0,)
    want_flags = np.zeros(2 * n0, np.uint32)
    want_flags[first] = 1
    want_flags[both] = 3
    assert np.array_equal(flags, want_flags), (np.nonzero(flags)[0], flags[np.nonzero(flags)[0]])
    assert st["fallback_tiles"] == len(tiles) and st["window_tiles"] == len(both), st


@pytest.mark.parametrize("nr", [0, 128])
def test_fp64_flagged_tiles_take_the_window(dev, nr):
    """Plain FP64: a flagged tile goes straight to the integer window."""
    job = synthetic.blurred_512(0, op=0)
    want = oracle.run_job(job)
    tiles = [0, 9, 77, _tiles_of(job, 64) - 1]
    outs, st, flags = _perturbed([job], dev, tiles, [1] * len(tiles), tile=64, nr=nr, **FFT64)
    _expect_exact([job], outs, [want])
    want_flags = np.zeros(_tiles_of(job, 64), np.uint32)
    want_flags[tiles] = 2
    assert np.array_equal(flags, want_flags)
    assert st["fallback_tiles"] == 0 and st["window_tiles"] == len(tiles), st


def test_band_zero_sends_every_tile_on(dev):
    """Band 0: every FP32 tile goes to the FP64 recompute (whose own band stays
    0.25, so none goes further); every FP64 tile goes to the window."""
    rng = np.random.default_rng(5)
    jobs = [synthetic.random_job(rng, 150, 203, 16, 7, p=0.7, max_off=3, op=0),
            synthetic.random_job(rng, 97, 260, 64, 15, p=0.5, max_off=16, op=1)]
    wants = [oracle.run_job(j) for j in jobs]
    outs, st = _run_batch(jobs, dev, band=0.0, **FFT32)
    _expect_exact(jobs, outs, wants)
    assert st["fallback_tiles"] == st["tiles"] > 0 and st["window_tiles"] == 0, st
    assert (md.debug_tile_flags() == 1).all()
    outs, st = _run_batch(jobs, dev, band=0.0, **FFT64)
    _expect_exact(jobs, outs, wants)
    assert st["window_tiles"] == st["tiles"] > 0 and st["fallback_tiles"] == 0, st
    assert (md.debug_tile_flags() == 2).all()


def test_default_band_flags_nothing(dev):
    """At the default band no tile of these workloads fails a check."""
    rng = np.random.default_rng(6)
    jobs = [synthetic.blurred_512(0), synthetic.random_job(rng, 300, 280, 256, 31, p=0.6, max_off=31)]
    wants = [oracle.run_job(j) for j in jobs]
    for opts in (FFT32, FFT64):
        outs, st = _run_batch(jobs, dev, **opts)
        _expect_exact(jobs, outs, wants)
        assert st["fallback_tiles"] == 0 and st["window_tiles"] == 0, st
        assert not md.debug_tile_flags().any()


def test_perturbed_large_tiles_and_every_decode(dev):
    """The hook on the large-tile kernels (FP32 256-point tiles, FP64
    recompute through its slab) and on each decode variant: kept bins <= 8,
    <= 12, <= 24, blocks, and the range-axis FFT decode at 3 2^a and 5 2^a."""
    rng = np.random.default_rng(7)
    cases = [  # H, W, L, k, max_off, tile, nr
        (300, 330, 8, 41, 2, 256, 0),
        (180, 170, 8, 9, 3, 64, 0),       # bins 6
        (180, 170, 16, 9, 4, 64, 0),      # bins 11
        (180, 170, 32, 9, 8, 64, 0),      # bins 20
        (180, 170, 64, 9, 16, 64, 0),     # bins 40
        (150, 160, 100, 7, 40, 64, 192),
        (150, 160, 100, 7, 40, 64, 160),
        # dense register decodes (n_r without an FFT decode, at most 8 bins),
        # which take bin 0 in closed form and so add the bump themselves
        (200, 190, 4, 9, 1, 64, 5),       # bins 3
        (300, 330, 4, 41, 1, 256, 5),     # bins 3, large tiles
        (200, 190, 8, 9, 4, 64, 15),      # bins 8
    ]
    for H, W, L, k, max_off, tile, nr in cases:
        job = synthetic.random_job(rng, H, W, L, k, p=0.6, max_off=max_off, op=int(rng.integers(0, 2)))
        want = oracle.run_job(job)
        n = _tiles_of(job, tile)
        tiles = sorted({0, n // 2, n - 1})
        for opts, bits, want_bit in ((FFT32, 1, 1), (FFT32, 3, 3), (FFT64, 1, 2)):
            _say(f"  {job.name} tile={tile} nr={nr} {opts} bits={bits}")
            outs, st, flags = _perturbed([job], dev, tiles, [bits] * len(tiles), tile=tile, nr=nr, **opts)
            _expect_exact([job], outs, [want])
            want_flags = np.zeros(n, np.uint32)
            want_flags[tiles] = want_bit
            assert np.array_equal(flags, want_flags), (job.name, opts, bits)


def test_fp32_error_bound_moves_jobs_to_fp64(dev):
    """A forced FP32 plan whose worst-case error bound exceeds 0.25 (here
    1024-point tiles for a 151 x 151 SE) runs in FP64 and stays exact."""
    rng = np.random.default_rng(25)
    job = synthetic.random_job(rng, 520, 610, 8, 151, p=0.5, max_off=2)
    want = oracle.run_job(job)
    outs, st = _run_batch([job], dev, tile=1024, **FFT32)
    _expect_exact([job], outs, [want])
    assert st["precision"] == 1 and st["n_t"] == 1024, st
    outs, st = _run_batch([job], dev, tile=256, **FFT32)
    _expect_exact([job], outs, [want])
    assert st["precision"] == 0, st


def test_caller_workspace(dev):
    """md_set_workspace: a batch runs bit-exact inside a caller buffer of
    md_workspace_size bytes; one byte less fails with MD_ERR_ARG before
    anything runs; NULL returns to library-owned workspace."""
    import torch

    rng = np.random.default_rng(8)
    jobs = [synthetic.random_job(rng, 200, 230, 16, 11, p=0.6, max_off=4, op=q % 2) for q in range(3)]
    jobs.append(synthetic.random_job(rng, 260, 250, 8, 61, p=0.5, max_off=2))
    wants = [oracle.run_job(j) for j in jobs]
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    spec = [(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)]
    try:
        for opts in (FFT32, FFT64, dict(FFT32, tile=256)):
            with md.options(**opts):
                need = md.workspace_size(spec)
                _say(f"  workspace {opts}: {need} bytes")
                assert need > 0
                ws = torch.empty(need, dtype=torch.uint8, device=dev)
                md.set_workspace(ws)
                outs = md.dilate_batch(spec)
                _expect_exact(jobs, [o.cpu().numpy() for o in outs], wants)
                outs2 = [torch.full_like(o, -3) for o in outs]
                md.dilate_batch(spec, outs=outs2)    # graph replay inside the workspace
                for a, b in zip(outs, outs2):
                    assert torch.equal(a, b)
                small = torch.empty(need - 256, dtype=torch.uint8, device=dev)
                md.set_workspace(small)
                marker = [torch.full_like(o, 123) for o in outs]
                with pytest.raises(md.MDError) as ei:
                    md.dilate_batch(spec, outs=marker)
                assert ei.value.code == -1
                assert all(bool((m == 123).all()) for m in marker)
                md.set_workspace(None)
        direct_only = [spec[0]]
        with md.options(path=2):
            assert md.workspace_size(direct_only) == 0
    finally:
        md.set_workspace(None)
    outs = md.dilate_batch(spec)
    _expect_exact(jobs, [o.cpu().numpy() for o in outs], wants)


def test_cache_bound_keeps_memory_flat(dev):
    """Batches with fresh SEs under a small bound (MD_OPT_CACHE_MB = 64): the
    library's cache stays within it, the cached plans are dropped least
    recently run first, device memory stays flat, and results stay exact.
    With graphs on, what the HIP runtime keeps per instantiated graph is
    reported as well."""
    import torch

    rng = np.random.default_rng(9)
    cap = 64 << 20
    drift = {}
    for graph in (0, 1):
        free = []
        with md.options(cache_mb=64, graph=graph, **FFT32):
            for it in range(24):
                jobs = [synthetic.random_job(rng, 160, 170, 64, 15, p=0.6, max_off=16) for _ in range(4)]
                outs, st = _run_batch(jobs, dev)
                if it % 6 == 0:
                    _expect_exact(jobs, outs, [oracle.run_job(j) for j in jobs])
                use = md.memory_usage()
                assert use["cache_bytes"] <= cap, use
                assert use["plans"] <= 2, use
                torch.cuda.synchronize()
                free.append(torch.cuda.mem_get_info(dev)[0])
        drift[graph] = (free[5] - min(free[6:])) / (1 << 20)
        _say(f"  graph={graph}: free MiB {[f // (1 << 20) for f in free]}, usage {md.memory_usage()}")
    _say(f"  drift after warm-up, MiB: {drift}")
    # without the bound each batch would keep about 70 MiB more (1.2 GiB over
    # the last 17 batches)
    assert drift[0] < 256, drift
