"""Throughput benchmark: exact dilated Mpixels/s on one MI355X.

Workload (default): the uneven batch -- 256 seeded synthetic images with
sides uniform in [128, 1024], L in {8, 16, 32, 64}, odd SE sides 3..41 with
disk / square / Bernoulli(0.6) masks and offsets in [0, L/4] -- run as one
md_dilate_batch call per step.  Inputs are resident in HBM before timing
starts.

Headline (`value`): every job through the transform path (the paper's
Steps 1-3: one-hot umbra encode, FFT convolution, top-degree decode) with
FP32 transforms and split twiddles, the exact tiers behind them (FP64
recompute of tiles that fail the decode's checks, then the integer window),
HIP-graph replay.  Beside it in the same line: the plain FP64 transform path
on the same batch and the ratio; the autotuned batch (which picks the
classical window for every job of this batch) as a named extra; the exact
mod-p path, the window forced, the recompute of every tile; a 2048^2 image
with 4 grey levels and a 127 x 127 disk, where the transform path beats the
window; the volume path; and a 16384^2 image streamed from host memory
(PCIe included; a context figure).  Every output of the headline and of
the FP64 leg is compared with the CPU oracle, all pixels of all 256 jobs;
the oracle's run over the batch is the CPU baseline.  A profiled pass (HIP
events on the library stream around every launch) gives the dominant
kernel's average launch duration for the roofline figure.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_TFLOPS = 157.3
FP64_VECTOR_TFLOPS = 78.6
CUS, CLOCK_GHZ, LANES_PER_CU = 256, 2.4, 64
FP32_NONPACKED_TFLOPS = CUS * LANES_PER_CU * 2 * CLOCK_GHZ / 1000.0   # one FMA per lane per clock
INT32_ALU_TOPS = CUS * LANES_PER_CU * CLOCK_GHZ / 1000.0   # one 32-bit integer op per lane per clock
INT16X2_ALU_TOPS = 2 * INT32_ALU_TOPS                       # packed 16-bit: two ops per lane per clock
# packed f16 window: two packed adds and one packed three-way max take two SE
# cells of two pixels (8 add/max ops) in three issue slots
F16X2_ADDMAX_TOPS = INT32_ALU_TOPS * 8.0 / 3.0


# the forced-path comparison legs on the batch
LEG_OPTS = {"fft64": dict(precision=1, path=1), "fft32": dict(precision=0, path=1),
            "ntt": dict(precision=2, path=1), "direct": dict(precision=0, path=2),
            # band 0: every tile of the FP32 path is recomputed exactly in FP64
            "fft32_recompute_all": dict(precision=0, path=1, band=0.0)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload(name):
    from paper_2305_03018_amd import synthetic

    if name == "uneven_batch":
        return synthetic.uneven_batch(0, 256)
    if name == "blurred_512":
        return [synthetic.blurred_512(0, 0), synthetic.blurred_512(0, 1)]
    if name == "large_random_mask":
        return [synthetic.large_random_mask(0, True), synthetic.large_random_mask(0, False)]
    if name == "octave_noise_4096":
        return [synthetic.octave_noise_4096(0)]
    if name == "large_disk_2048":
        return [synthetic.large_disk_2048()]
    if name == "small_uniform":
        return [synthetic.small_uniform(0)]
    raise SystemExit(f"unknown workload {name}")


def timed_steps(md, torch, stream, args_list, outs, steps, warmup, host=None, **opts):
    """warmup + timed steps of one md_dilate_batch call each (the batch
    marshalled once, as a serving loop would); returns ms/step.  With `host`
    a dict, host["ms"] gets the mean host time of one call."""
    batch = md.Batch(args_list, outs)
    with md.options(sync=0, **opts):
        for _ in range(warmup):
            batch.run()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        h = 0.0
        for _ in range(steps):
            c0 = time.perf_counter()
            batch.run()
            h += time.perf_counter() - c0
        t1.record(stream)
        torch.cuda.synchronize()
    if host is not None:
        host["ms"] = h * 1e3 / steps
    return t0.elapsed_time(t1) / steps


def stage_dtype(stage):
    """Arithmetic type a profiled stage computes in."""
    if stage in ("direct16", "direct3_16"):
        return "f16"          # integers of magnitude <= 2048, exact in f16
    if stage in ("direct16i", "direct3_16i"):
        return "i16"
    if stage.startswith("direct"):
        return "i32"
    if stage.startswith(("ntt", "decode_ntt")):
        return "u32"          # residues mod 7 * 2^20 + 1
    if stage.startswith(("fft64", "decode64", "recompute64")):
        return "f64"
    return "f32"


def kernel_of(stage):
    """HIP kernel that a profiled stage launches."""
    if stage in ("direct16", "direct16i"):
        return f"k_direct16<false, {'true' if stage == 'direct16' else 'false'}>"
    if stage == "direct32":
        return "k_direct32<sel, false>"
    if stage in ("direct3_16", "direct3_16i"):
        return f"k_direct16<true, {'true' if stage == 'direct3_16' else 'false'}>"
    if stage == "direct3_32":
        return "k_direct32<sel, true>"
    if stage == "decode_ntt3":
        return "k_ntt3_decode"
    if stage.startswith("ntt3"):
        return f"k_ntt3<{stage.split('_n')[1]}>"
    if stage.startswith("fft"):
        prec, n = ("float" if stage.startswith("fft32") else "double"), int(stage.split("_n")[1])
        big = n > (128 if prec == "float" else 64)
        lanes = 8 if (prec == "float" and n == 128) else 4   # lanes per tile line
        return f"k_fft_big<{prec}, {n}>" if big else f"k_fft_reg<{prec}, {n}, {lanes}>"
    if stage == "decode_ntt":
        return "k_ntt_decode"
    if stage.startswith("ntt"):
        return f"k_ntt<{stage.split('_n')[1]}>"
    if stage in ("decode32_fft", "decode64_fft"):
        return f"k_decode_fft<{'float' if stage == 'decode32_fft' else 'double'}>"
    if stage.startswith("decode"):
        return f"k_decode<{'float' if stage == 'decode32' else 'double'}>"
    if stage.startswith("recompute64"):
        return f"k_fallback<{stage.split('_n')[1]}>"
    return stage


def measured_traffic(kernel, workload, with_alg=False):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record (FETCH_SIZE and WRITE_SIZE, scaled by the copy-probe factors), or
    None when there is no record or the kernel source changed since it was
    taken.  With `with_alg`, (bytes, algorithmic bytes of the profiled
    launch or None): the autotuner's tile mix, and so the bytes per launch,
    follow each box's calibration, so the ratio is what carries over."""
    import hashlib

    inst = kernel.replace("<", "_").replace(">", "").replace(", ", "_")
    path = os.path.join(ROOT, "profiles", f"{inst}_{workload}_traffic.txt")
    if not os.path.exists(path):
        path = os.path.join(ROOT, "profiles", f"{kernel.split('<')[0]}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return (None, None) if with_alg else None
    rec = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            key, val = line.split(None, 1)
            rec[key] = val
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return (None, None) if with_alg else None
    b = 1024.0 * (float(rec["fetch_kib"]) * float(rec["fetch_scale"]) +
                  float(rec["write_kib"]) * float(rec["write_scale"]))
    if with_alg:
        return b, (float(rec["alg_bytes"]) if "alg_bytes" in rec else None)
    return b


def roofline_for(stage, prof, workload, launch_ms=None):
    """Roofline figures of one profiled stage; `launch_ms` (if given) replaces
    the profiled calls' mean launch time."""
    rec = prof[stage]
    per_launch_ms = rec["ms"] / rec["launches"] if launch_ms is None else launch_ms
    ops = rec["alg_ops"] / rec["launches"]
    achieved = ops / (per_launch_ms * 1e-3) / 1e12
    kernel = kernel_of(stage)
    traffic, traffic_alg = measured_traffic(kernel, workload, with_alg=True)
    base = {"achieved": achieved, "traffic": traffic, "kernel": kernel,
            "stage": stage, "avg_launch_ms": per_launch_ms,
            "alg_bytes_per_launch": rec["alg_bytes"] / rec["launches"]}
    if traffic is not None and traffic_alg:
        # the profiled launch's algorithmic bytes and the counted/algorithmic
        # ratio (the tile mix of this run may differ)
        base["traffic_alg_bytes"] = traffic_alg
        base["traffic_ratio"] = traffic / traffic_alg
    if stage.startswith("direct"):
        peak = (F16X2_ADDMAX_TOPS if stage in ("direct16", "direct3_16") else
                INT16X2_ALU_TOPS if stage in ("direct16i", "direct3_16i") else INT32_ALU_TOPS)
        return {"bound": "alu", "peak": peak, "unit": "TOP/s", "frac": achieved / peak, **base}
    if stage.startswith(("ntt", "decode_ntt")):
        # modular products (Shoup): one 32-bit high multiply (4 issue slots at
        # quarter rate), two 24-bit multiplies, a subtract and a two-op
        # reduction on the int32 ALU -- 9 slots each
        peak = INT32_ALU_TOPS / 9.0
        return {"bound": "alu", "peak": peak, "unit": "T modmul/s", "frac": achieved / peak, **base}
    fp64 = stage.startswith(("fft64", "decode64", "recompute64"))
    if fp64:
        return {"bound": "alu", "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_TFLOPS, **base}
    # FP32: the kernels are built without packed FP32 instructions, so the
    # vector ALU's FMA rate is 256 CUs x 64 lanes x 2 flops x 2.4 GHz; the
    # published 157.3 counts packed FP32
    out = {"bound": "alu", "peak": FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved / FP32_NONPACKED_TFLOPS, "peak_published_fp32": FP32_VECTOR_TFLOPS,
           "frac_published_fp32": achieved / FP32_VECTOR_TFLOPS, **base}
    if stage.startswith("fft32"):
        # the transform-domain volume a two-pass (unfused) design would move:
        # nt^2 complex FP32 values per (tile, bin) item, V = (nt/T)^2 bins per
        # output pixel; the fused kernel keeps it in LDS
        n = int(stage.split("_n")[1])
        vol = rec["units"] / rec["launches"] * n * n * 8.0
        gbs = vol / (per_launch_ms * 1e-3) / 1e9
        out["volume_view"] = {"bytes_per_launch": vol, "achieved_GBs": gbs, "peak_GBs": HBM_PEAK_GBS,
                              "frac": gbs / HBM_PEAK_GBS}
    return out


def volume_leg(md, torch, dev, stream, steps):
    """The volume path on a 128 x 256 x 256 blurred volume (L = 16, 7 x 7 x 7
    ball SE, offsets in [0, 3]): auto, direct window and exact transform, each
    timed over `steps` calls with per-stage figures from a profiled pass and
    sampled voxels checked against the oracle."""
    import oracle
    from paper_2305_03018_amd import synthetic

    job = synthetic.blurred_volume(0)
    vol = torch.from_numpy(job.vol).to(dev)
    out = torch.empty_like(vol)
    nvox = int(job.vol.size)
    rng = np.random.default_rng(9)
    zs, ys, xs = (rng.integers(0, n, 2048) for n in job.vol.shape)
    want = oracle.at3(job.vol, job.mask, job.off, job.L, 0, zs, ys, xs)
    res = {"workload": job.name, "voxels": nvox}
    for name, opts in (("auto", {}), ("direct", dict(path=2)), ("ntt", dict(path=1))):
        with md.options(sync=0, **opts):
            md.dilate3(vol, job.mask, job.off, job.L, out=out)
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(steps):
                md.dilate3(vol, job.mask, job.off, job.L, out=out)
            t1.record(stream)
            torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        md.profile_reset()
        with md.options(profile=1, sync=1, **opts):
            for _ in range(2):
                md.dilate3(vol, job.mask, job.off, job.L, out=out)
            st = md.get_stats()
        sp = md.profile_get()
        md.profile_reset()
        got = out[zs, ys, xs].cpu().numpy()
        if not np.array_equal(got, want):
            raise SystemExit(f"bench: volume parity failure ({name})")
        res[name] = {"ms": ms, "mvoxels_s": nvox / (ms * 1e-3) / 1e6, "path": "direct" if st["path"] == 2 else "ntt",
                     "n_t": st["n_t"], "n_r": st["n_r"],
                     "stages": {k: {q: v for q, v in roofline_for(k, sp, "volume").items() if not q.startswith("traffic")}
                                for k in sp if sp[k]["alg_ops"] > 0}}
        log(f"bench: volume {name} {ms:.3f} ms ({res[name]['mvoxels_s']:.0f} Mvoxel/s)")
    return res


def host_stream_leg(md, torch, dev, steps):
    """A 16384 x 16384 image (1 GiB, L = 16 uniform, 15 x 15 disk SE with
    offsets in [0, 7]) in pinned host memory, streamed through the GPU in
    bands within a 256 MiB band budget (md_dilate_host): wall time per call
    including the PCIe transfers, against the same dilation with the image
    already resident in HBM; sampled pixels checked against the oracle."""
    import oracle
    from paper_2305_03018_amd import synthetic

    side = 16384
    rng = np.random.default_rng(11)
    host = torch.empty((side, side), dtype=torch.int32, pin_memory=True)
    host.copy_(torch.from_numpy(rng.integers(0, 16, (side, side), dtype=np.int32)))
    out = torch.empty_like(host, pin_memory=True)
    mask = synthetic.disk_mask(15)
    off = rng.integers(0, 8, (15, 15)).astype(np.int32) * mask
    res = {"workload": f"uniform_{side}x{side}_L16_disk15", "pixels": side * side, "band_budget_mb": 256}
    with md.options(stream_rows=0, stream_mb=256):
        md.dilate_host(host, mask, off, 16, out=out)
        t0 = time.perf_counter()
        for _ in range(steps):
            md.dilate_host(host, mask, off, 16, out=out)
        dt = (time.perf_counter() - t0) / steps
    ys, xs = rng.integers(0, side, 2048), rng.integers(0, side, 2048)
    want = oracle.at(host.numpy(), mask, off, 16, 0, ys, xs)
    if not np.array_equal(out.numpy()[ys, xs], want):
        raise SystemExit("bench: host-streamed parity failure")
    res["ms"] = dt * 1e3
    res["mpx_s_pcie_inclusive"] = side * side / dt / 1e6
    res["pcie_gb_s"] = 2 * side * side * 4 / dt / 1e9
    dimg = host.to(dev)
    dout = torch.empty_like(dimg)
    md.dilate(dimg, mask, off, 16, out=dout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        md.dilate(dimg, mask, off, 16, out=dout)
    torch.cuda.synchronize()
    dt2 = (time.perf_counter() - t0) / steps
    res["resident_ms"] = dt2 * 1e3
    res["resident_mpx_s"] = side * side / dt2 / 1e6
    log(f"bench: host-streamed {res['ms']:.1f} ms ({res['mpx_s_pcie_inclusive']:.0f} Mpx/s incl. PCIe), "
        f"resident {res['resident_ms']:.1f} ms")
    del host, out, dimg, dout
    return res


def large_se_leg(md, torch, dev, stream, steps):
    """The transform path's niche: a 2048 x 2048 image with L = 4 grey levels
    (uniform) and a 127 x 127 disk SE (offsets in [0, 1]), where the
    transform's work per pixel, independent of the SE's 12 649 cells, is below
    the window's.  Auto, the direct window and the FP32 transform path, each
    over `steps` calls; sampled pixels checked against the oracle."""
    import oracle
    from paper_2305_03018_amd import synthetic

    job = synthetic.large_disk_2048()
    img_np, mask, off, L, k, side = job.img, job.mask, job.off, job.L, job.k, job.img.shape[0]
    rng = np.random.default_rng(14)
    img = torch.from_numpy(img_np).to(dev)
    out = torch.empty_like(img)
    ys, xs = rng.integers(0, side, 1024), rng.integers(0, side, 1024)
    want = oracle.at(img_np, mask, off, L, 0, ys, xs)
    res = {"workload": f"uniform_{side}x{side}_L{L}_disk{k}"}
    for name, opts in (("auto", {}), ("direct", dict(path=2)), ("fft32", dict(precision=0, path=1))):
        batch = md.Batch([(img, mask, off, L, 0)], [out])
        with md.options(**opts):
            batch.run()
            st = md.get_stats()
            with md.options(sync=0):
                t0 = torch.cuda.Event(enable_timing=True)
                t1 = torch.cuda.Event(enable_timing=True)
                t0.record(stream)
                for _ in range(steps):
                    batch.run()
                t1.record(stream)
                torch.cuda.synchronize()
        if not np.array_equal(out.cpu().numpy()[ys, xs], want):
            raise SystemExit(f"bench: large-SE parity failure ({name})")
        ms = t0.elapsed_time(t1) / steps
        res[name] = {"ms": ms, "mpx_s": side * side / (ms * 1e-3) / 1e6,
                     "path": "direct" if st["path"] == 2 else "fft", "n_t": st["n_t"], "n_r": st["n_r"]}
        log(f"bench: large SE {name} {ms:.3f} ms ({res[name]['path']})")
    return res


def paper_shapes_leg(md, torch, dev, stream, steps):
    """The paper's own workload shapes (Sec. 4.1: i.i.d. uniform image and SE
    values over the tonal range, square SEs; Sec. 4.2: 5 x 5 SE, 2- to 5-bit
    images of side FFT size - 4), run through the auto path: a cold call
    (plan, SE tables), then `steps` timed calls, with sampled pixels checked
    against the oracle.  Odd SE sides stand in for the paper's even ones (the
    SE origin is its centre cell)."""
    import oracle
    from paper_2305_03018_amd import synthetic

    rng = np.random.default_rng(17)
    cases = ([("se_size", 512, bits, k) for bits in (4, 8) for k in (33, 65, 129, 255)] +
             [("image_size", n, 4, (n // 10) | 1) for n in (512, 1024, 2048, 4096)] +
             [("image_size", n, 8, (n // 10) | 1) for n in (512, 1024, 2048)] +
             [("fpga", n - 4, 5, 5) for n in (128, 512, 1024)])
    res = []
    for exp, side, bits, k in cases:
        L = 1 << bits
        img_np = rng.integers(0, L, (side, side)).astype(np.int32)
        mask = synthetic.square_mask(k)
        off = rng.integers(0, L, (k, k)).astype(np.int32)
        img = torch.from_numpy(img_np).to(dev)
        out = torch.empty_like(img)
        batch = md.Batch([(img, mask, off, L, 0)], [out])
        c0 = time.perf_counter()
        batch.run()
        cold = (time.perf_counter() - c0) * 1e3
        st = md.get_stats()
        with md.options(sync=0):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(steps):
                batch.run()
            t1.record(stream)
            torch.cuda.synchronize()
        ys, xs = rng.integers(0, side, 256), rng.integers(0, side, 256)
        if not np.array_equal(out.cpu().numpy()[ys, xs], oracle.at(img_np, mask, off, L, 0, ys, xs)):
            raise SystemExit(f"bench: paper-shape parity failure ({exp} {side} {bits}-bit k={k})")
        ms = t0.elapsed_time(t1) / steps
        res.append({"experiment": exp, "side": side, "bits": bits, "k": k, "ms": ms, "cold_ms": cold,
                    "mpx_s": side * side / (ms * 1e-3) / 1e6, "path": "direct" if st["path"] == 2 else "fft",
                    "n_t": st["n_t"], "n_r": st["n_r"]})
        log(f"bench: paper shape {exp} {side}^2 {bits}-bit k={k}: {ms:.3f} ms ({res[-1]['path']})")
        del batch, img, out
    return res


def spectrum_error(md, torch, dev):
    """Transform-domain values of one tile of the 512 x 512 blurred image
    (15 x 15 disk, n_t = 128, n_r = 24) just before the inverse range
    transform, FP32 and FP64, against the DFT of the exact per-pixel
    coefficient vectors from the oracle."""
    import oracle
    from paper_2305_03018_amd import synthetic

    job = synthetic.blurred_512(0)
    img = torch.from_numpy(job.img).to(dev)
    nt, nr, ty, tx = 128, 24, 1, 2
    T = nt - job.k + 1
    ys, xs = np.divmod(np.arange(T * T), T)
    counts = oracle.counts_at(job.img, job.mask, job.off, ty * T + ys, tx * T + xs, nr)
    ref = oracle.range_spectrum_ref(counts, nr).T
    out = {"config": f"{job.name}, tile ({ty},{tx}) of {T}x{T}, n_t={nt}, n_r={nr}"}
    for prec, name in ((0, "fp32"), (1, "fp64")):
        got = md.debug_tile_values(img, job.mask, job.off, job.L, nt, nr, prec, ty, tx)
        out[f"{name}_rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out[f"{name}_max_abs"] = float(np.abs(got - ref).max())
    return out


def dft16_leg(md, torch, dev, stream, lines=1 << 20, reps=32, runs=5):
    """Batched 16-point DFTs (md_debug_dft16), `reps` in a row per line, by
    the vector-ALU butterflies of the spatial transform, FP32 matrix-core
    products and split-bf16 matrix-core products: mean event time per call
    and the rate in 16-point DFTs per second and in algorithmic flops
    (5 N log2 N = 320 per DFT)."""
    rng = np.random.default_rng(23)
    x = torch.from_numpy((rng.uniform(-1, 1, (lines, 16)) + 1j * rng.uniform(-1, 1, (lines, 16)))
                         .astype(np.complex64)).to(dev)
    out = torch.empty_like(x)
    res = {"lines": lines, "reps": reps}
    for v, name in ((0, "valu_butterflies"), (1, "mfma_fp32"), (2, "mfma_bf16x3")):
        md.debug_dft16(v, x, reps=reps, out=out)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(runs):
            md.debug_dft16(v, x, reps=reps, out=out)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / runs
        dfts = lines * reps
        res[name] = {"ms": ms, "gdft_s": dfts / (ms * 1e-3) / 1e9, "tflops_alg": dfts * 320.0 / (ms * 1e-3) / 1e12}
        log(f"bench: dft16 {name} {ms:.3f} ms ({res[name]['tflops_alg']:.1f} TFLOP/s algorithmic)")
    return res


def stream_probe(torch, dev, gib=4, runs=10):
    """Device-memory rate of torch's own streaming kernels: a copy (read
    and write) and a full-tensor sum (read), timed with HIP events."""
    n = gib << 28
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    res = {}
    for name, f, nbytes in (("copy", lambda: y.copy_(x), 2 * 4 * n), ("sum", lambda: x.sum(), 4 * n)):
        f()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(runs):
            f()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / runs
        res[name] = {"ms": ms, "bytes": nbytes, "TB_s": nbytes / (ms * 1e-3) / 1e12}
        log(f"bench: stream probe {name} {gib} GiB: {ms:.3f} ms, {res[name]['TB_s']:.2f} TB/s")
    del x, y
    return res


def cpu_baseline(jobs, budget_s):
    import oracle

    t0 = time.perf_counter()
    px = 0
    n = 0
    for job in jobs:
        oracle.run_job(job)
        px += job.img.size
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": px / dt / 1e6, "unit": "Mpixels/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {n} of {len(jobs)} jobs ({px} px), {dt:.1f} s, direct max over the SE (C, OpenMP)"}


def parity_full(jobs, outs, wants, what):
    """Every pixel of every job against the oracle."""
    for q, (j, o, w) in enumerate(zip(jobs, outs, wants)):
        got = o.cpu().numpy()
        if not np.array_equal(got, w):
            raise SystemExit(f"bench: parity failure ({what}) on job {q} ({j.name}): "
                             f"{int((got != w).sum())} pixels differ")


def leg_stats(md, batch, **opts):
    """One synchronised call of a forced leg and its statistics."""
    with md.options(sync=1, **opts):
        batch.run()
        return md.get_stats()


def profiled(md, batch, calls, **opts):
    """Per-stage event times of `calls` synchronised calls without a graph."""
    md.profile_reset()
    with md.options(profile=1, graph=0, sync=1, **opts):
        for _ in range(calls):
            batch.run()
    sp = md.profile_get()
    md.profile_reset()
    return sp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uneven_batch")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="also run the paper's own timing shapes through the auto path (context only)")
    ap.add_argument("--leg", choices=sorted(LEG_OPTS),
                    help="run only this forced path on the batch (warm-up, --steps timed steps, one profiled "
                         "step) and print its own JSON line; for hardware-counter runs of its kernels")
    ap.add_argument("--dft16", action="store_true",
                    help="only the batched 16-point DFT comparison (vector ALU against matrix cores), one JSON line")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only time torch's own streaming kernels (a 4 GiB device copy and a full-tensor sum) "
                         "with HIP events: the rate this GPU reaches for plain streaming access, one JSON line")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain device copy of 256 MiB (a known-size reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path shards by tiles/images "
              "across GPUs but this build measures a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2305_03018_amd as md

    dev = torch.device("cuda:0")
    if args.stream_probe:
        print(json.dumps({"stream_probe": stream_probe(torch, dev)}), flush=True)
        return
    if args.copy_probe:
        src = torch.arange(64 << 20, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy probe {src.numel() * 4} bytes read, {dst.numel() * 4} bytes written")
        del src, dst
    if args.dft16:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            print(json.dumps({"dft16": dft16_leg(md, torch, dev, stream)}), flush=True)
        md.release()
        return
    jobs = build_workload(args.workload)
    total_px = sum(j.img.size for j in jobs)
    log(f"bench: workload {args.workload}: {len(jobs)} jobs, {total_px / 1e6:.2f} Mpx")
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    outs = [torch.empty_like(t) for t in imgs]
    arglist = [(im, j.mask, j.off, j.L, j.op) for im, j in zip(imgs, jobs)]
    stream = torch.cuda.Stream()
    if args.leg:
        opts = LEG_OPTS[args.leg]
        with torch.cuda.stream(stream):
            # one auto-path call first: it calibrates the cost model (or loads
            # the tune file), so the forced path plans as in the full run
            with md.options(precision=0, path=0):
                md.dilate_batch(arglist, outs=outs)
            m = timed_steps(md, torch, stream, arglist, outs, args.steps, args.warmup, **opts)
            sp = profiled(md, md.Batch(arglist, outs), 1, **opts)
        print(json.dumps({"leg": args.leg, "workload": args.workload, "ms_per_step": m,
                          "stages": {st: roofline_for(st, sp, args.workload) for st in sp if sp[st]["alg_ops"] > 0}}),
              flush=True)
        md.release()
        return
    import oracle

    # the oracle over the whole batch: parity reference for every leg, and
    # the CPU baseline (its wall time on all host threads)
    log("bench: oracle over the batch")
    t0 = time.perf_counter()
    wants = [oracle.run_job(j) for j in jobs]
    cpu_s = time.perf_counter() - t0
    head = LEG_OPTS["fft32"]
    res = {}
    with torch.cuda.stream(stream):
        # calibration first (one small auto-path call), then the headline
        # leg's first call builds its plans, SE spectra and graph
        with md.options(sync=1, precision=0, path=0):
            md.dilate_batch(arglist[:1], outs=outs[:1])
        with md.options(sync=1, **head):
            t0 = time.perf_counter()
            md.dilate_batch(arglist, outs=outs)
            res["cold_ms"] = (time.perf_counter() - t0) * 1e3
        log(f"bench: cold call of the FP32 transform leg {res['cold_ms']:.1f} ms")
        batch = md.Batch(arglist, outs)
        # headline: FP32 transforms + exact tiers, graph replay
        host = {}
        ms = timed_steps(md, torch, stream, arglist, outs, args.steps, args.warmup, host=host, **head)
        stats = leg_stats(md, batch, **head)
        parity_full(jobs, outs, wants, "fp32 transform leg")
        log(f"bench: FP32 transform leg {ms:.3f} ms/step, host {host['ms']:.3f} ms per call, stats {stats}")
        # the plain FP64 transform path on the same batch
        ms64 = timed_steps(md, torch, stream, arglist, outs, max(3, args.steps // 2), 1, **LEG_OPTS["fft64"])
        stats64 = leg_stats(md, batch, **LEG_OPTS["fft64"])
        parity_full(jobs, outs, wants, "fp64 transform leg")
        log(f"bench: FP64 transform leg {ms64:.3f} ms/step, stats {stats64}")
        # per-stage event times of the headline leg (the roofline's launch
        # durations) and of the FP64 leg
        prof = profiled(md, batch, max(2, args.steps // 4), **head)
        prof64 = profiled(md, batch, 2, **LEG_OPTS["fft64"])
        log(f"bench: profile {json.dumps(prof)}")
        cmp = {}
        if not args.no_compare:
            for name, opts in (("autotuned", dict(precision=0, path=0)), ("direct", LEG_OPTS["direct"]),
                               ("ntt", LEG_OPTS["ntt"]), ("fft32_recompute_all", LEG_OPTS["fft32_recompute_all"])):
                m = timed_steps(md, torch, stream, arglist, outs, max(3, args.steps // 4), 1, **opts)
                st = leg_stats(md, batch, **opts)
                parity_full(jobs, outs, wants, name)
                sp = profiled(md, batch, 2, **opts)
                cmp[name] = {"ms_per_step": m, "mpx_s": total_px / (m * 1e-3) / 1e6,
                             "stats": {k: st[k] for k in ("fft_jobs", "direct_jobs", "tiles", "fallback_tiles",
                                                          "window_tiles", "max_residual")},
                             "stages": {q: {k: v for k, v in roofline_for(q, sp, args.workload).items()
                                            if not k.startswith("traffic")} for q in sp if sp[q]["alg_ops"] > 0}}
                if name == "fft32_recompute_all":
                    rec = {q: v for q, v in sp.items() if q.startswith("recompute")}
                    ms_rec = sum(v["ms"] for v in rec.values()) / 2
                    cmp[name]["recompute"] = {"tiles": st["fallback_tiles"], "ms_per_step": ms_rec,
                                              "us_per_tile": ms_rec * 1e3 / max(1, st["fallback_tiles"])}
                log(f"bench: {name} {m:.3f} ms/step")
            cmp["volume"] = volume_leg(md, torch, dev, stream, max(3, args.steps // 4))
            cmp["large_se"] = large_se_leg(md, torch, dev, stream, 3)
            cmp["host_stream"] = host_stream_leg(md, torch, dev, 3)
            cmp["dft16"] = dft16_leg(md, torch, dev, stream)
            if args.paper_shapes:
                cmp["paper_shapes"] = paper_shapes_leg(md, torch, dev, stream, 3)
        spec_err = spectrum_error(md, torch, dev)
    fft_stages = [k for k in prof if k.startswith("fft32")]
    dominant = max(fft_stages or list(prof), key=lambda k: prof[k]["ms"])
    roof = roofline_for(dominant, prof, args.workload)
    roof["share_of_step"] = prof[dominant]["ms"] / sum(v["ms"] for v in prof.values())
    value = total_px / (ms * 1e-3) / 1e6
    line = {
        "metric": "exact dilated Mpixels/s, batched FP32+fallback vs FP64 FFT path, 1 MI355X",
        "value": value,
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "jobs": len(jobs), "pixels": total_px,
                   "path": "transform (umbra FFT convolution) for every job",
                   "precision": "fp32 split twiddles; exact tiers: fp64 recompute, then integer window",
                   "launch": "hipGraph replay of stage-wise persistent kernels"},
        "fp64_fft": {"ms_per_step": ms64, "mpx_s": total_px / (ms64 * 1e-3) / 1e6,
                     "stages": {k: {q: v for q, v in roofline_for(k, prof64, args.workload).items() if not q.startswith("traffic")}
                                for k in prof64 if prof64[k]["alg_ops"] > 0}},
        "speedup_vs_fp64_fft": ms64 / ms,
        "roofline": roof,
        "stats": {"max_residual": stats["max_residual"], "tiles": stats["tiles"],
                  "fallback_tiles": stats["fallback_tiles"], "window_tiles": stats["window_tiles"],
                  "fallback_fraction": stats["fallback_tiles"] / max(1, stats["tiles"]),
                  "fft_jobs": stats["fft_jobs"], "direct_jobs": stats["direct_jobs"],
                  "fp64_max_residual": stats64["max_residual"], "spectrum_error": spec_err,
                  "parity": "all pixels of all jobs equal the oracle (fp32 and fp64 legs"
                            + (", and every compare leg)" if cmp else ")")},
        "stage_ms_per_step": {k: v["ms"] / max(2, args.steps // 4) for k, v in prof.items()},
        "cold_ms": res["cold_ms"],
        "host_ms_per_call": host["ms"],
        "compare": cmp,
        "cost_model": md.cost_model(),
    }
    if "autotuned" in cmp:
        line["autotuned_mpx_s"] = cmp["autotuned"]["mpx_s"]
    if not args.no_cpu:
        threads = oracle.num_threads()
        line["cpu_baseline"] = {"value": total_px / cpu_s / 1e6, "unit": "Mpixels/s", "cores": threads,
                                "kind": "oracle",
                                "sample": f"all {len(jobs)} jobs ({total_px} px), {cpu_s:.1f} s: the direct max "
                                          f"over the SE (C, OpenMP, {threads} threads)"}
        oracle.set_threads(1)
        line["cpu_1core"] = cpu_baseline(jobs, 4.0)
        oracle.set_threads(threads)
    print(json.dumps(line), flush=True)
    md.release()


if __name__ == "__main__":
    main()
