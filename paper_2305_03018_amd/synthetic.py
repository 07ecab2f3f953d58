"""Seeded synthetic workloads for exact grey-scale dilation / erosion.

This module only draws inputs: images, structuring-element (SE) masks and
SE offsets.  It holds none of the morphology or transform arithmetic, so the
HIP path, the CPU oracle, the tests and the benchmark can all share it.

Value domains follow the paper's model (Section 2.1): an image takes values
in {0, ..., L-1}; a non-flat SE is a mask (the domain B) plus non-negative
additive offsets.  SE arrays are k x k with odd k and the origin at the
centre cell; offsets are drawn for every cell and zeroed where the mask is 0.

The paper's own workloads draw image and SE values i.i.d. uniform with
numpy's ``randint`` (Section 4.1 and the exactness experiment of
Section 4.3).  The five named workloads below add structure (smoothed
noise, disk masks, salt-and-pepper) and a batch of uneven jobs; every
recipe is seeded and deterministic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    """One dilation (op=0) or erosion (op=1) request."""

    img: np.ndarray          # (H, W) int32, values in [0, L-1]
    L: int                   # number of grey levels
    mask: np.ndarray         # (k, k) uint8, 1 = cell in the SE domain B
    off: np.ndarray          # (k, k) int32 >= 0, zero where mask == 0
    op: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def k(self) -> int:
        return int(self.mask.shape[0])


# ----------------------------------------------------------------------------
# masks
# ----------------------------------------------------------------------------
def disk_mask(k: int) -> np.ndarray:
    """Cells (i, j) with (i-r)^2 + (j-r)^2 <= r^2, r = (k-1)/2."""
    r = (k - 1) // 2
    i, j = np.mgrid[0:k, 0:k]
    return (((i - r) ** 2 + (j - r) ** 2) <= r * r).astype(np.uint8)


def square_mask(k: int) -> np.ndarray:
    return np.ones((k, k), np.uint8)


def bernoulli_mask(rng: np.random.Generator, k: int, p: float, centre: bool) -> np.ndarray:
    m = (rng.random((k, k)) < p).astype(np.uint8)
    if centre:
        m[k // 2, k // 2] = 1
    return m


def _offsets(rng: np.random.Generator, k: int, hi_inclusive: int, mask: np.ndarray) -> np.ndarray:
    off = rng.integers(0, hi_inclusive + 1, (k, k)).astype(np.int32)
    off[mask == 0] = 0
    return off


def _normalise_to_levels(g: np.ndarray, L: int) -> np.ndarray:
    lo, hi = float(g.min()), float(g.max())
    scale = (L - 1) / (hi - lo) if hi > lo else 0.0
    return np.rint((g - lo) * scale).astype(np.int32)


# ----------------------------------------------------------------------------
# the five named workloads
# ----------------------------------------------------------------------------
def small_uniform(seed: int = 0) -> Job:
    """64x64, L=16 i.i.d. uniform; 7x7 full-square SE, offsets in [0,3]."""
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 16, (64, 64)).astype(np.int32)
    mask = square_mask(7)
    off = _offsets(rng, 7, 3, mask)
    return Job(img, 16, mask, off, 0, "small_uniform_64x64_L16_k7")


def blurred_512(seed: int = 0, op: int = 0) -> Job:
    """512x512, L=16: Gaussian-blurred (sigma 4) uniform noise quantised to
    [0,15]; 15x15 disk SE, offsets in [0,7]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    u = rng.random((512, 512))
    g = gaussian_filter(u, 4.0, mode="reflect", truncate=4.0)
    img = _normalise_to_levels(g, 16)
    mask = disk_mask(15)
    off = _offsets(rng, 15, 7, mask)
    return Job(img, 16, mask, off, op, "blurred_512x512_L16_disk15")


def large_random_mask(seed: int = 0, flat: bool = True) -> Job:
    """2048x2048, L=32 i.i.d. uniform; 63x63 Bernoulli(0.5) mask with the
    centre set; offsets 0 (flat) or uniform in [0,15]."""
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 32, (2048, 2048)).astype(np.int32)
    mask = bernoulli_mask(rng, 63, 0.5, centre=True)
    if flat:
        off = np.zeros((63, 63), np.int32)
    else:
        off = _offsets(rng, 63, 15, mask)
    return Job(img, 32, mask, off, 0,
               "random_2048x2048_L32_bern63_" + ("flat" if flat else "nonflat"))


def large_disk_2048(seed: int = 13) -> Job:
    """2048x2048, L=4 i.i.d. uniform; 127x127 disk SE with offsets uniform in
    [0, 1]: a large SE over few grey levels, where the transform's work per
    pixel (independent of the SE's cells) is below the window's."""
    rng = np.random.default_rng(seed)
    side, L, k = 2048, 4, 127
    img = rng.integers(0, L, (side, side)).astype(np.int32)
    mask = disk_mask(k)
    off = (rng.integers(0, 2, (k, k)) * mask).astype(np.int32)
    return Job(img, L, mask, off, 0, f"uniform_{side}x{side}_L{L}_disk{k}")


def uneven_batch(seed: int = 0, n: int = 256) -> list[Job]:
    """n images with sides uniform in [128,1024] (non-square), L drawn from
    {8,16,32,64}, uniform values; odd SE side in [3,41], disk / square /
    Bernoulli(0.6) mask (centre not forced), offsets uniform in [0, L/4]."""
    jobs = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(n)):
        rng = np.random.default_rng(child)
        H, W = (int(v) for v in rng.integers(128, 1025, 2))
        L = int(rng.choice([8, 16, 32, 64]))
        img = rng.integers(0, L, (H, W)).astype(np.int32)
        k = int(rng.integers(1, 21)) * 2 + 1
        shape = int(rng.integers(0, 3))
        if shape == 0:
            mask, sname = disk_mask(k), "disk"
        elif shape == 1:
            mask, sname = square_mask(k), "square"
        else:
            mask, sname = bernoulli_mask(rng, k, 0.6, centre=False), "bern"
        off = _offsets(rng, k, L // 4, mask)
        jobs.append(Job(img, L, mask, off, 0, f"batch{i}_{H}x{W}_L{L}_{sname}{k}"))
    return jobs


def octave_noise_4096(seed: int = 0, side: int = 4096) -> Job:
    """side x side 8-bit image: three octaves of smoothed Gaussian noise
    (sigma 16/2^o, weight 2^-o, each normalised to unit std), min-max
    quantised to [0,255], then 5% salt-and-pepper; 31x31 disk SE, offsets in
    [0,31]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    acc = np.zeros((side, side), np.float64)
    for o in range(3):
        n = gaussian_filter(rng.standard_normal((side, side)), 16.0 / 2 ** o, mode="wrap")
        n /= n.std()
        acc += n * 2.0 ** (-o)
    img = _normalise_to_levels(acc, 256)
    npx = side * side
    sel = rng.choice(npx, size=npx // 20, replace=False)
    flat = img.reshape(-1)
    half = len(sel) // 2
    flat[sel[:half]] = 255
    flat[sel[half:]] = 0
    mask = disk_mask(31)
    off = _offsets(rng, 31, 31, mask)
    return Job(img, 256, mask, off, 0, f"octaves_{side}x{side}_L256_disk31")


def exactness_pair(rng: np.random.Generator, side: int, k: int, L: int = 256) -> Job:
    """The exactness protocol of Section 4.3: random image and random full
    square non-flat SE, both drawn uniformly from [0, L-1]."""
    img = rng.integers(0, L, (side, side)).astype(np.int32)
    mask = square_mask(k)
    off = rng.integers(0, L, (k, k)).astype(np.int32)
    return Job(img, L, mask, off, 0, f"exact_{side}_k{k}")


def random_job(rng: np.random.Generator, H: int, W: int, L: int, k: int,
               p: float = 0.7, max_off: int | None = None, op: int = 0) -> Job:
    """Generic random case for parity tests: Bernoulli(p) mask (centre not
    forced), offsets uniform in [0, max_off]."""
    if max_off is None:
        max_off = max(1, L // 4)
    img = rng.integers(0, L, (H, W)).astype(np.int32)
    mask = bernoulli_mask(rng, k, p, centre=False)
    off = _offsets(rng, k, max_off, mask)
    return Job(img, L, mask, off, op, f"rand_{H}x{W}_L{L}_k{k}")


# ----------------------------------------------------------------------------
# volumes (three image axes; SE arrays k x k x k, origin at the centre cell)
# ----------------------------------------------------------------------------
@dataclass
class VolJob:
    """One volume dilation (op=0) or erosion (op=1) request."""

    vol: np.ndarray          # (D, H, W) int32, values in [0, L-1]
    L: int
    mask: np.ndarray         # (k, k, k) uint8
    off: np.ndarray          # (k, k, k) int32 >= 0, zero where mask == 0
    op: int = 0
    name: str = ""

    @property
    def k(self) -> int:
        return int(self.mask.shape[0])


def ball_mask3(k: int) -> np.ndarray:
    """Cells (a, i, j) within distance r = (k-1)/2 of the centre."""
    r = (k - 1) // 2
    a, i, j = np.mgrid[0:k, 0:k, 0:k]
    return (((a - r) ** 2 + (i - r) ** 2 + (j - r) ** 2) <= r * r).astype(np.uint8)


def cube_mask3(k: int) -> np.ndarray:
    return np.ones((k, k, k), np.uint8)


def bernoulli_mask3(rng: np.random.Generator, k: int, p: float, centre: bool) -> np.ndarray:
    m = (rng.random((k, k, k)) < p).astype(np.uint8)
    if centre:
        m[k // 2, k // 2, k // 2] = 1
    return m


def _offsets3(rng: np.random.Generator, k: int, hi_inclusive: int, mask: np.ndarray) -> np.ndarray:
    off = rng.integers(0, hi_inclusive + 1, (k, k, k)).astype(np.int32)
    off[mask == 0] = 0
    return off


def random_vol_job(rng: np.random.Generator, D: int, H: int, W: int, L: int, k: int,
                   p: float = 0.7, max_off: int | None = None, op: int = 0) -> VolJob:
    """Generic random volume case for parity tests: i.i.d. uniform voxels,
    Bernoulli(p) mask (centre not forced), offsets uniform in [0, max_off]."""
    if max_off is None:
        max_off = max(1, L // 4)
    vol = rng.integers(0, L, (D, H, W)).astype(np.int32)
    mask = bernoulli_mask3(rng, k, p, centre=False)
    off = _offsets3(rng, k, max_off, mask)
    return VolJob(vol, L, mask, off, op, f"vol_{D}x{H}x{W}_L{L}_k{k}")


def blurred_volume(seed: int = 0, shape=(128, 256, 256), L: int = 16, k: int = 7,
                   max_off: int = 3, op: int = 0) -> VolJob:
    """A D x H x W volume with L grey levels: Gaussian-blurred (sigma 2)
    uniform noise, min-max quantised; k x k x k ball SE with offsets uniform
    in [0, max_off].  The volume counterpart of blurred_512."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    g = gaussian_filter(rng.random(shape), 2.0, mode="reflect", truncate=3.0)
    vol = _normalise_to_levels(g, L)
    mask = ball_mask3(k)
    off = _offsets3(rng, k, max_off, mask)
    D, H, W = shape
    return VolJob(vol, L, mask, off, op, f"blurred_vol_{D}x{H}x{W}_L{L}_ball{k}")


WORKLOADS = {
    "small_uniform": small_uniform,
    "blurred_512": blurred_512,
    "large_random_mask": large_random_mask,
    "uneven_batch": uneven_batch,
    "octave_noise_4096": octave_noise_4096,
}
