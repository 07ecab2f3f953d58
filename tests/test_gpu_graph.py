"""Graph replay of md_dilate_batch: one batch signature captured once and
replayed several times, with eager torch work and synchronisations between
the replays and new image contents and output buffers each time; every
replay is checked against the oracle.  Covers the direct window, the FP32
transform path, the exact recompute (band 0 sends every tile through it, so
the device-built recompute list and its counters are reset and rebuilt
inside the graph at every replay), the exact mod-p path and the range-axis
FFT decode in both precisions."""
import numpy as np
import pytest

import oracle
import paper_2305_03018_amd as md
from paper_2305_03018_amd import synthetic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    md.load()
    return torch.device("cuda:0")


def batch_jobs(rng):
    shapes = [(130, 170, 16, 7), (64, 300, 32, 15), (257, 129, 8, 3), (90, 90, 64, 21), (200, 150, 16, 31),
              (33, 47, 16, 5)]
    return [synthetic.random_job(rng, H, W, L, k, p=0.7, max_off=L // 4, op=i % 2)
            for i, (H, W, L, k) in enumerate(shapes)]


def fft_decode_jobs(rng, nr):
    """Jobs for a forced range length nr (512, or the FP32 lengths 320 and
    384): the range-axis FFT decode and its pixel-block layout of the
    transform-domain tiles."""
    L2, off2 = (256, 255) if nr >= 512 else (200, 100)
    return [synthetic.random_job(rng, 150, 170, 100, 7, p=0.7, max_off=27, op=0),
            synthetic.random_job(rng, 90, 260, L2, 15, p=0.5, max_off=off2, op=1)]


@pytest.mark.parametrize("mode", ["auto", "fft32", "recompute_all", "ntt", "direct", "fft_decode32",
                                  "fft_decode64", "fft_decode32_n320", "fft_decode32_n384"])
def test_graph_replays(dev, mode):
    import torch

    opts = {"auto": {}, "fft32": dict(precision=0, path=1), "recompute_all": dict(precision=0, path=1, band=0.0),
            "ntt": dict(precision=2, path=1), "direct": dict(path=2),
            "fft_decode32": dict(precision=0, path=1, nr=512), "fft_decode64": dict(precision=1, path=1, nr=512),
            "fft_decode32_n320": dict(precision=0, path=1, nr=320),
            "fft_decode32_n384": dict(precision=0, path=1, nr=384)}[mode]
    rng = np.random.default_rng(71)
    jobs = fft_decode_jobs(rng, opts["nr"]) if mode.startswith("fft_decode") else batch_jobs(rng)
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    side = torch.randn(512, 512, device=dev)
    stream = torch.cuda.Stream()   # graphs are captured on a non-default stream only
    with torch.cuda.stream(stream), md.options(graph=1, sync=1, **opts):
        for rep in range(5):
            # new contents, same shapes / L / SEs: the same signature, so the
            # captured graph is replayed
            for j, im in zip(jobs, imgs):
                j.img = rng.integers(0, j.L, j.img.shape).astype(np.int32)
                im.copy_(torch.from_numpy(j.img))
            outs = [torch.full_like(im, -9) for im in imgs]
            print(f"  {mode} replay {rep}", flush=True)
            md.dilate_batch([(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)], outs=outs)
            st = md.get_stats()
            if mode == "recompute_all":
                assert st["fallback_tiles"] == st["tiles"] > 0
            # eager work on the same device between replays
            side = (side @ side.T).tanh()
            torch.cuda.synchronize()
            for q, (j, o) in enumerate(zip(jobs, outs)):
                want = oracle.run_job(j)
                got = o.cpu().numpy()
                assert np.array_equal(got, want), f"{mode} replay {rep} job {q} ({j.name}): {int((got != want).sum())} differ"


def test_repeat_calls_see_in_place_changes(dev):
    """The library reuses the previous call's executor only when the job
    array, the SE bytes and the planning options are all unchanged: an SE
    array edited in place, an offset changed under a masked cell, new image
    contents and a changed precision must each give the new exact result."""
    import torch

    rng = np.random.default_rng(72)
    jobs = batch_jobs(rng)
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    batch = md.Batch([(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)])

    def check(tag):
        outs = batch.run()
        torch.cuda.synchronize()
        for q, (j, o) in enumerate(zip(jobs, outs)):
            want = oracle.run_job(j)
            got = o.cpu().numpy()
            assert np.array_equal(got, want), f"{tag}: job {q} ({j.name}) {int((got != want).sum())} differ"

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        check("first call")
        check("identical repeat")
        # the Batch holds the same numpy arrays the jobs hold: edit in place
        j = jobs[1]
        j.off[j.mask != 0] = (j.off[j.mask != 0] + 1) % (j.L // 4 + 1)
        check("offsets edited in place")
        j = jobs[3]
        cells = np.argwhere(j.mask == 0)
        if len(cells):
            j.off[tuple(cells[0])] = 7          # under a masked cell: no effect on the result
            check("offset under a masked cell")
        j = jobs[0]
        j.mask[:] = 0
        j.mask[j.k // 2, 0] = 1
        j.off[:] = 0
        check("mask edited in place")
        for j, im in zip(jobs, imgs):
            j.img = rng.integers(0, j.L, j.img.shape).astype(np.int32)
            im.copy_(torch.from_numpy(j.img))
        check("new image contents")
        with md.options(precision=1):
            check("precision changed")
        check("precision restored")
