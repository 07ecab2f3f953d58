"""GPU: the paper's exactness experiment (Sec. 4.3, Fig. ErrorGraph), seeded.

The paper draws, with numpy's randint over [0, 255] (8-bit), 100 random
pairs of a 99 x 99 image and a full square non-flat SE for each SE side
3, 5, ..., 17, and 100 pairs of an image and a 5 x 5 SE for each image side
100, 200, ..., 600, and reports a mean absolute error of 0 against the
classical dilation.  Here each group of 100 pairs is one batch call, run
through the FP32 transform path with its exact tiers, plain FP64 and the
auto plan; every pixel of every image must equal the oracle's, so the mean
absolute error is 0 as in the paper.

With SE offsets up to 255 the range length is at least 511, so the FP32 plan
decodes with the range-axis FFT at 512 (or 640) points.
"""
import numpy as np
import pytest

import oracle
import paper_2305_03018_amd as md
from paper_2305_03018_amd import synthetic

pytestmark = pytest.mark.gpu

MODES = {"fft32": dict(precision=0, path=1), "fft64": dict(precision=1, path=1), "auto": {}}
PAIRS = 100


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    md.load()
    return torch.device("cuda:0")


def _group(dev, jobs, label):
    import torch

    wants = [oracle.run_job(j) for j in jobs]
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    spec = [(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)]
    for mode, opts in MODES.items():
        with md.options(**opts):
            outs = md.dilate_batch(spec)
            st = md.get_stats()
        err = 0.0
        for j, o, w in zip(jobs, outs, wants):
            err += float(np.abs(o.cpu().numpy().astype(np.int64) - w).mean())
        print(f"  {label} {mode}: mean abs error {err / len(jobs):.3g}, stats {st}", flush=True)
        assert err == 0.0, f"{label} {mode}: mean absolute error {err / len(jobs)}"


@pytest.mark.parametrize("k", [3, 5, 7, 9, 11, 13, 15, 17])
def test_se_size_sweep_99x99(dev, k):
    rng = np.random.default_rng(1000 + k)
    _group(dev, [synthetic.exactness_pair(rng, 99, k) for _ in range(PAIRS)], f"99x99 k={k}")


@pytest.mark.parametrize("side", [100, 200, 300, 400, 500, 600])
def test_image_size_sweep_5x5(dev, side):
    rng = np.random.default_rng(2000 + side)
    _group(dev, [synthetic.exactness_pair(rng, side, 5) for _ in range(PAIRS)], f"{side}x{side} k=5")
