"""GPU parity of the volume entry points (md_dilate3 / md_erode3) against
the volume oracle, bit-exact, on the direct window (packed 16-bit and 32-bit
forms) and on the exact transform path at every cubic tile length, with
ragged volumes that span several blocks / tiles, the degenerate cases, the
range check, and sampled voxels of a full-size volume."""
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


def modes_for(k):
    m = {"auto": {}, "direct": dict(path=2)}
    for nt in (8, 16, 32):
        if nt - k + 1 >= 1:
            m[f"ntt{nt}"] = dict(path=1, tile=nt)
    return m


def want_of(job, op):
    if op == 0:
        return oracle.dilate3(job.vol, job.mask, job.off)
    return oracle.erode3(job.vol, job.mask, job.off, job.L)


def check(job, dev, modes=None, ops=(0, 1)):
    import torch

    vol = torch.from_numpy(job.vol).to(dev)
    for op in ops:
        want = want_of(job, op)
        for name, opts in (modes or modes_for(job.k)).items():
            print(f"  case {job.name} op={op} {name}", flush=True)
            with md.options(**opts):
                fn = md.dilate3 if op == 0 else md.erode3
                got = fn(vol, job.mask, job.off, job.L).cpu().numpy()
                st = md.get_stats()
            bad = got != want
            assert not bad.any(), (f"{job.name} op={op} {name}: {int(bad.sum())} of {bad.size} differ; first at "
                                   f"{np.argwhere(bad)[0].tolist()} got {got[bad][0]} want {want[bad][0]}")
            if name.startswith("ntt"):
                assert st["path"] == 1 and st["n_t"] == int(name[3:]) and st["precision"] == 2
            if name == "direct":
                assert st["path"] == 2


CASES = [
    # D, H, W, L, k, p, max_off
    (9, 70, 150, 16, 3, 0.7, 3),
    (13, 29, 41, 32, 5, 0.6, 8),
    (30, 17, 23, 8, 7, 0.5, 2),
    (6, 66, 131, 64, 9, 0.4, 16),
    (5, 12, 34, 4, 15, 0.3, 1),
    (3, 40, 40, 16, 31, 0.05, 4),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_random_volumes(dev, case):
    D, H, W, L, k, p, max_off = case
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    check(synthetic.random_vol_job(rng, D, H, W, L, k, p=p, max_off=max_off), dev)


def test_ball_se_blurred_volume(dev):
    check(synthetic.blurred_volume(3, shape=(21, 37, 45), L=16, k=7, max_off=3), dev)


def test_wide_range_uses_32bit_window(dev):
    """L + max offset beyond the packed 16-bit range: the 32-bit direct form;
    the transform path has no range length for it."""
    rng = np.random.default_rng(51)
    job = synthetic.random_vol_job(rng, 7, 20, 140, 40000, 5, p=0.6, max_off=3000)
    check(job, dev, modes={"auto": {}, "direct": dict(path=2)})
    with md.options(path=1), pytest.raises(md.MDError):
        md.dilate3(__import__("torch").from_numpy(job.vol).to(dev), job.mask, job.off, job.L)


def test_packed_forms(dev):
    """The packed window's f16 form up to a reachable sum of 2048 and its
    int16 form just past it, on volumes (one window pass per SE slab)."""
    rng = np.random.default_rng(53)
    for D, H, W, L, k, p, max_off in ((7, 20, 70, 2049, 3, 0.7, 0), (6, 25, 90, 1900, 5, 0.6, 148),
                                      (7, 20, 70, 2000, 5, 0.6, 49), (5, 30, 75, 2000, 7, 0.4, 60)):
        job = synthetic.random_vol_job(rng, D, H, W, L, k, p=p, max_off=max_off)
        a, i, j = np.argwhere(job.mask)[0]
        job.off[a, i, j] = max_off
        check(job, dev, modes={"auto": {}, "direct": dict(path=2)})


def test_degenerate_volumes(dev):
    rng = np.random.default_rng(52)
    # one slice, one voxel, k = 1
    check(synthetic.random_vol_job(rng, 1, 33, 70, 16, 5, p=0.7, max_off=3), dev)
    check(synthetic.random_vol_job(rng, 1, 1, 1, 16, 3, p=1.0, max_off=3), dev)
    check(synthetic.random_vol_job(rng, 4, 9, 11, 16, 1, p=1.0, max_off=5), dev)
    # empty SE: every window is empty
    j = synthetic.random_vol_job(rng, 5, 9, 10, 16, 5, p=0.5, max_off=3)
    j.mask[:] = 0
    j.off[:] = 0
    j.name = "empty_se"
    check(j, dev)
    # only a far corner cell: most windows are empty, and for D = 2 the
    # corner slab never meets an input slice for half of the outputs
    j = synthetic.random_vol_job(rng, 2, 6, 7, 16, 7, p=0.0, max_off=3)
    j.mask[0, 0, 0] = 1
    j.off[0, 0, 0] = 2
    j.name = "corner_only"
    check(j, dev)


def test_range_error(dev):
    import torch

    rng = np.random.default_rng(53)
    job = synthetic.random_vol_job(rng, 6, 20, 30, 16, 3, p=1.0, max_off=2)
    bad = job.vol.copy()
    bad[3, 10, 15] = 16
    for opts in (dict(path=2), dict(path=1, tile=16)):
        with md.options(**opts), pytest.raises(md.MDError) as e:
            md.dilate3(torch.from_numpy(bad).to(dev), job.mask, job.off, job.L)
        assert e.value.code == -2


def test_argument_errors(dev):
    import torch

    vol = torch.zeros((4, 5, 6), dtype=torch.int32, device=dev)
    m = np.ones((3, 3, 3), np.uint8)
    o = np.zeros((3, 3, 3), np.int32)
    with pytest.raises(md.MDError):
        md.dilate3(vol, np.ones((33, 33, 33), np.uint8), np.zeros((33, 33, 33), np.int32), 16)   # k > 31
    with pytest.raises(md.MDError):
        md.dilate3(vol, m, o, 1)                                                              # L < 2
    with pytest.raises(md.MDError):
        md.dilate3(vol, m, np.full((3, 3, 3), -1, np.int32), 16)                              # negative offset
    with md.options(path=1, tile=8), pytest.raises(md.MDError):
        md.dilate3(vol, np.ones((9, 9, 9), np.uint8), np.zeros((9, 9, 9), np.int32), 16)      # no 8-point plan


def test_full_size_sampled(dev):
    """The benchmark volume (128 x 256 x 256, L = 16, 7 x 7 x 7 ball) on each
    path: sampled voxels against the oracle, computed one by one."""
    import torch

    job = synthetic.blurred_volume(0)
    vol = torch.from_numpy(job.vol).to(dev)
    rng = np.random.default_rng(54)
    n = 4000
    zs, ys, xs = (rng.integers(0, s, n) for s in job.vol.shape)
    # borders and corners too
    zs[:8] = [0, 0, 127, 127, 0, 127, 64, 64]
    ys[:8] = [0, 255, 0, 255, 128, 128, 0, 255]
    xs[:8] = [0, 255, 255, 0, 0, 255, 255, 0]
    for op in (0, 1):
        want = oracle.at3(job.vol, job.mask, job.off, job.L, op, zs, ys, xs)
        for name, opts in {"auto": {}, "direct": dict(path=2), "ntt16": dict(path=1, tile=16),
                           "ntt32": dict(path=1, tile=32)}.items():
            print(f"  full-size op={op} {name}", flush=True)
            with md.options(**opts):
                fn = md.dilate3 if op == 0 else md.erode3
                got = fn(vol, job.mask, job.off, job.L)[zs, ys, xs].cpu().numpy()
            assert np.array_equal(got, want), f"op={op} {name}: {int((got != want).sum())} samples differ"


@pytest.mark.parametrize("case", [(11, 37, 45, 16, 5, 0.6, 3), (6, 20, 130, 8, 7, 1.0, 2)],
                         ids=lambda c: "x".join(map(str, c)))
def test_volume_compositions(dev, case):
    """md_morph3 (opening, closing, Beucher gradient, top-hats on volumes)
    against the oracle's volume compositions on both volume paths."""
    import torch

    D, H, W, L, k, p, max_off = case
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    job = synthetic.random_vol_job(rng, D, H, W, L, k, p=p, max_off=max_off)
    vol = torch.from_numpy(job.vol).to(dev)
    for op in range(2, 7):
        want = oracle.morph3(op, job.vol, job.mask, job.off, L)
        for name, opts in {"direct": dict(path=2), "ntt16": dict(path=1, tile=16)}.items():
            print(f"  case {case} op={op} {name}", flush=True)
            with md.options(**opts):
                got = md.morph3(op, vol, job.mask, job.off, L).cpu().numpy()
            bad = got != want
            assert not bad.any(), f"{case} op={op} {name}: {int(bad.sum())} differ"
