"""GPU parity of the compositions (opening, closing, Beucher gradient,
top-hats; md_morph) against the oracle's compositions, bit-exact, on every
path and precision of the underlying dilation and erosion."""
import numpy as np
import pytest

import oracle
import paper_2305_03018_amd as md
from paper_2305_03018_amd import synthetic

pytestmark = pytest.mark.gpu

MODES = {"auto": {}, "fft64": dict(precision=1, path=1), "fft32": dict(precision=0, path=1),
         "direct": dict(path=2)}
OPS = {md.OPEN: "open", md.CLOSE: "close", md.GRADIENT: "gradient", md.TOPHAT: "tophat",
       md.BLACKHAT: "blackhat"}


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    md.load()
    return torch.device("cuda:0")


def check(job, dev, ops=OPS, modes=MODES):
    import torch

    img = torch.from_numpy(job.img).to(dev)
    for op, name in ops.items():
        want = oracle.morph(op, job.img, job.mask, job.off, job.L)
        for mname, opts in modes.items():
            if mname != "direct" and mname != "auto" and not job.mask.any():
                continue   # the FFT path needs at least one SE cell
            print(f"  case {job.name} {name} {mname}", flush=True)
            with md.options(**opts):
                got = md.morph(op, img, job.mask, job.off, job.L).cpu().numpy()
            bad = got != want
            assert not bad.any(), (f"{job.name} {name} {mname}: {int(bad.sum())} of {bad.size} differ; first at "
                                   f"{np.argwhere(bad)[0].tolist()} got {got[bad][0]} want {want[bad][0]}")


@pytest.mark.parametrize("case", [(150, 203, 16, 7, 0.7, 3), (61, 300, 64, 15, 0.5, 16), (97, 131, 2, 3, 1.0, 0),
                                  (33, 33, 32, 31, 0.4, 8), (200, 45, 256, 11, 0.6, 40)],
                         ids=lambda c: "x".join(map(str, c)))
def test_random_compositions(dev, case):
    H, W, L, k, p, max_off = case
    rng = np.random.default_rng(abs(hash(case)) % (2 ** 32))
    check(synthetic.random_job(rng, H, W, L, k, p=p, max_off=max_off), dev)


def test_composition_edges(dev):
    rng = np.random.default_rng(41)
    j = synthetic.random_job(rng, 40, 50, 16, 7, p=0.5, max_off=3)
    j.mask[:] = 0
    j.off[:] = 0
    j.name = "empty_mask"
    check(j, dev)
    j = synthetic.random_job(rng, 3, 70, 16, 9, p=0.5, max_off=3)
    j.mask[:, :] = 0
    j.mask[0, 0] = 1
    j.off[:] = 0
    j.off[0, 0] = 3
    j.name = "all_windows_empty"
    check(j, dev)
    j = synthetic.random_job(rng, 1, 1, 16, 5, p=0.8, max_off=3)
    j.name = "one_pixel"
    check(j, dev)
    j = synthetic.random_job(rng, 64, 64, 16, 1, p=1.0, max_off=4)
    j.name = "one_cell"
    check(j, dev)


def test_composition_large_se_and_range(dev):
    rng = np.random.default_rng(42)
    j = synthetic.random_job(rng, 300, 280, 4, 127, p=0.3, max_off=1)
    check(j, dev, ops={md.OPEN: "open", md.CLOSE: "close"}, modes={"direct": dict(path=2), "auto": {}})
    j = synthetic.random_job(rng, 90, 100, 20000, 5, p=0.8, max_off=300)   # 32-bit direct form
    check(j, dev, modes={"auto": {}})


def test_composition_blurred_512(dev):
    job = synthetic.blurred_512(0, 0)
    check(job, dev, modes={"auto": {}, "fft32": dict(precision=0, path=1)})


def test_composition_errors(dev):
    import torch

    img = torch.zeros((8, 8), dtype=torch.int32, device=dev)
    mask = np.ones((3, 3), np.uint8)
    off = np.zeros((3, 3), np.int32)
    with pytest.raises(md.MDError) as e:
        md.morph(7, img, mask, off, 16)
    assert e.value.code == -1
    big = np.full((3, 3), (1 << 23) + 1, np.int32)
    with pytest.raises(md.MDError) as e:
        md.morph(md.OPEN, img, mask, big, 1 << 23)
    assert e.value.code == -2
