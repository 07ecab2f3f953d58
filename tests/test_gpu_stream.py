"""GPU parity of the host-streamed entry points (md_dilate_host /
md_erode_host): images in host memory, cut into bands of output rows with
their halo, each band computed on the device.  Bit-exact against the oracle
on the whole image, on every path, for band heights from 1 row to the whole
image, pageable and pinned host memory, and the range check."""
import numpy as np
import pytest

import oracle
import paper_2305_03018_amd as md
from paper_2305_03018_amd import synthetic

pytestmark = pytest.mark.gpu

MODES = {"auto": {}, "direct": dict(path=2), "fft32": dict(precision=0, path=1),
         "fft64": dict(precision=1, path=1), "ntt": dict(precision=2, path=1)}


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    md.load()
    return torch.device("cuda:0")


def want_of(job, op):
    return oracle.dilate(job.img, job.mask, job.off) if op == 0 else oracle.erode(job.img, job.mask, job.off, job.L)


def check(job, rows, modes=MODES, ops=(0, 1), pinned=False):
    import torch

    img = job.img
    if pinned:
        t = torch.empty(img.shape, dtype=torch.int32, pin_memory=True)
        t.copy_(torch.from_numpy(img))
        img = t
    for op in ops:
        want = want_of(job, op)
        for name, opts in modes.items():
            if name in ("fft32", "fft64", "ntt") and not job.mask.any():
                continue
            print(f"  case {job.name} rows={rows} op={op} {name} pinned={pinned}", flush=True)
            out = torch.empty(img.shape, dtype=torch.int32, pin_memory=True) if pinned else None
            with md.options(stream_rows=rows, **opts):
                fn = md.dilate_host if op == 0 else md.erode_host
                got = fn(img, job.mask, job.off, job.L, out=out)
            got = got.numpy() if isinstance(got, torch.Tensor) else got
            bad = got != want
            assert not bad.any(), (f"{job.name} rows={rows} op={op} {name}: {int(bad.sum())} differ; first at "
                                   f"{np.argwhere(bad)[0].tolist()} got {got[bad][0]} want {want[bad][0]}")


@pytest.mark.parametrize("case", [(613, 517, 16, 7, 0.7, 3, 50), (300, 200, 64, 15, 0.6, 16, 37),
                                  (257, 130, 8, 31, 0.3, 2, 64), (90, 1000, 32, 1, 1.0, 5, 7)],
                         ids=lambda c: "x".join(map(str, c)))
def test_bands(dev, case):
    H, W, L, k, p, max_off, rows = case
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    check(synthetic.random_job(rng, H, W, L, k, p=p, max_off=max_off), rows)


def test_band_heights(dev):
    rng = np.random.default_rng(61)
    job = synthetic.random_job(rng, 41, 150, 16, 5, p=0.7, max_off=3)
    for rows in (1, 2, 3, 40, 41, 1000, 0):
        check(job, rows, modes={"auto": {}, "fft32": dict(precision=0, path=1)}, ops=(0,))


def test_pinned_host_memory(dev):
    rng = np.random.default_rng(62)
    check(synthetic.random_job(rng, 500, 333, 32, 9, p=0.6, max_off=8), 60, pinned=True)


def test_budget_sets_band_height(dev):
    """MD_OPT_STREAM_MB alone (band height 0 = auto) on a 4096 x 3000 image:
    an 8 MiB budget gives bands of about 170 rows; sampled pixels against the
    oracle."""
    rng = np.random.default_rng(63)
    job = synthetic.random_job(rng, 4096, 3000, 64, 11, p=0.6, max_off=16)
    ys, xs = rng.integers(0, 4096, 6000), rng.integers(0, 3000, 6000)
    ys[:4] = [0, 4095, 170, 171]
    for op in (0, 1):
        want = oracle.at(job.img, job.mask, job.off, job.L, op, ys, xs)
        with md.options(stream_rows=0, stream_mb=8):
            got = (md.dilate_host if op == 0 else md.erode_host)(job.img, job.mask, job.off, job.L)
        assert np.array_equal(got[ys, xs], want)


def test_range_error_and_arguments(dev):
    rng = np.random.default_rng(64)
    job = synthetic.random_job(rng, 200, 100, 16, 3, p=1.0, max_off=2)
    bad = job.img.copy()
    bad[150, 40] = 16
    with md.options(stream_rows=30), pytest.raises(md.MDError) as e:
        md.dilate_host(bad, job.mask, job.off, job.L)
    assert e.value.code == -2
    # a band that cannot fit the budget
    with md.options(stream_rows=0, stream_mb=1), pytest.raises(md.MDError):
        md.dilate_host(np.zeros((4, 200000), np.int32), job.mask, job.off, 16)
    # the library still works after the errors
    with md.options(stream_rows=30):
        got = md.dilate_host(job.img, job.mask, job.off, job.L)
    assert np.array_equal(got, oracle.dilate(job.img, job.mask, job.off))


@pytest.mark.parametrize("case", [(23, 40, 50, 16, 5, 0.7, 3, 4), (17, 33, 70, 8, 7, 0.5, 2, 1), (9, 20, 30, 32, 3, 1.0, 8, 2)],
                         ids=lambda c: "x".join(map(str, c)))
def test_volume_bands(dev, case):
    """md_dilate3_host / md_erode3_host: bands of slices with their halo,
    on the direct window and on the exact transform path."""
    D, H, W, L, k, p, max_off, slices = case
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    job = synthetic.random_vol_job(rng, D, H, W, L, k, p=p, max_off=max_off)
    for op in (0, 1):
        want = oracle.dilate3(job.vol, job.mask, job.off) if op == 0 else oracle.erode3(job.vol, job.mask, job.off, L)
        for name, opts in {"auto": {}, "direct": dict(path=2), "ntt16": dict(path=1, tile=16)}.items():
            print(f"  case {case} op={op} {name}", flush=True)
            with md.options(stream_rows=slices, **opts):
                got = (md.dilate3_host if op == 0 else md.erode3_host)(job.vol, job.mask, job.off, L)
            bad = got != want
            assert not bad.any(), f"{case} op={op} {name}: {int(bad.sum())} differ"


def test_volume_bands_range_error(dev):
    rng = np.random.default_rng(65)
    job = synthetic.random_vol_job(rng, 12, 10, 12, 16, 3, p=1.0, max_off=2)
    bad = job.vol.copy()
    bad[9, 5, 5] = 99
    with md.options(stream_rows=2), pytest.raises(md.MDError) as e:
        md.dilate3_host(bad, job.mask, job.off, job.L)
    assert e.value.code == -2
