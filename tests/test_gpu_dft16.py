"""GPU: the measurement hook behind the choice of butterflies over
matrix-core products for the transform's radix stages (md_debug_dft16).

Each variant's batched 16-point DFTs against numpy's FP64 FFT of the same
lines: the vector-ALU and FP32 matrix-core forms to FP32 rounding, the
split-bf16 form to its own (about 2^-16 relative) precision; and four DFTs in
a row against the identity F^4 = 256 I.  Argument errors through the C ABI.
"""
import numpy as np
import pytest

import paper_2305_03018_amd as md

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    md.load()
    return torch.device("cuda:0")


def _lines(rng, n):
    return (rng.uniform(-1, 1, (n, 16)) + 1j * rng.uniform(-1, 1, (n, 16))).astype(np.complex64)


@pytest.mark.parametrize("variant,tol", [(0, 3e-7), (1, 3e-7), (2, 6e-5)])
def test_dft16_variants(dev, variant, tol):
    import torch

    rng = np.random.default_rng(5 + variant)
    x = _lines(rng, 64 * 37)
    want = np.fft.fft(x.astype(np.complex128), axis=1)
    got = md.debug_dft16(variant, torch.from_numpy(x).to(dev), reps=1).cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"  variant {variant}: max error / max |y| = {err:.3g}", flush=True)
    assert err < tol
    # F^4 = 16^2 I
    got4 = md.debug_dft16(variant, torch.from_numpy(x).to(dev), reps=4).cpu().numpy()
    err4 = np.abs(got4 - 256.0 * x).max() / (256.0 * np.abs(x).max())
    assert err4 < 4 * tol


def test_dft16_arguments(dev):
    import torch

    x = torch.zeros((64, 16), dtype=torch.complex64, device=dev)
    lib = md.load()
    assert lib.md_debug_dft16(3, x.data_ptr(), x.data_ptr(), 64, 1) == -1
    assert lib.md_debug_dft16(0, x.data_ptr(), x.data_ptr(), 32, 1) == -1
    assert lib.md_debug_dft16(0, x.data_ptr(), x.data_ptr(), 64, 0) == -1
    assert lib.md_debug_dft16(0, None, x.data_ptr(), 64, 1) == -1
