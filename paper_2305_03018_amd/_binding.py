"""ctypes binding of libmd.so (include/md.h).  Argument marshalling only."""
from __future__ import annotations

import contextlib
import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libmd.so")
_HEADER = os.path.join(os.path.dirname(_PKG), "include", "md.h")
_lib = None

(OPT_PRECISION, OPT_BAND, OPT_PATH, OPT_TILE, OPT_NR, OPT_SYNC, OPT_GRAPH, OPT_WORKSPACE_MB,
 OPT_PROFILE, OPT_AUTOTUNE, OPT_STREAM_ROWS, OPT_STREAM_MB, OPT_CACHE_MB) = range(13)
_OPT_NAMES = {"precision": OPT_PRECISION, "band": OPT_BAND, "path": OPT_PATH, "tile": OPT_TILE,
              "nr": OPT_NR, "sync": OPT_SYNC, "graph": OPT_GRAPH, "workspace_mb": OPT_WORKSPACE_MB,
              "profile": OPT_PROFILE, "autotune": OPT_AUTOTUNE, "stream_rows": OPT_STREAM_ROWS,
              "stream_mb": OPT_STREAM_MB, "cache_mb": OPT_CACHE_MB}
_STATUS = {0: "MD_OK", -1: "MD_ERR_ARG", -2: "MD_ERR_RANGE", -3: "MD_ERR_NOMEM",
           -4: "MD_ERR_DEVICE", -5: "MD_ERR_UNSUPPORTED"}


class MDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _Job(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("H", ctypes.c_int), ("W", ctypes.c_int), ("L", ctypes.c_int),
                ("se_mask", ctypes.c_void_p), ("se_offsets", ctypes.c_void_p), ("k", ctypes.c_int),
                ("out", ctypes.c_void_p), ("op", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("max_residual", ctypes.c_double), ("tiles", ctypes.c_longlong),
                ("fallback_tiles", ctypes.c_longlong), ("window_tiles", ctypes.c_longlong),
                ("direct_jobs", ctypes.c_longlong), ("fft_jobs", ctypes.c_longlong),
                ("path", ctypes.c_int), ("n_t", ctypes.c_int), ("n_r", ctypes.c_int),
                ("precision", ctypes.c_int)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("precision", ctypes.c_int), ("n_t", ctypes.c_int), ("T", ctypes.c_int),
                ("n_r", ctypes.c_int), ("bins", ctypes.c_int), ("tiles_x", ctypes.c_int), ("tiles_y", ctypes.c_int),
                ("decode_fft", ctypes.c_int), ("n_t64", ctypes.c_int), ("fp32_bound", ctypes.c_double),
                ("cost_fft_ns", ctypes.c_double), ("cost_direct_ns", ctypes.c_double)]


class _StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("ms", ctypes.c_double), ("launches", ctypes.c_longlong),
                ("alg_bytes", ctypes.c_double), ("alg_ops", ctypes.c_double), ("units", ctypes.c_double)]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libmd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise MDError(-4, f"{_LIB_PATH} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i, u8 = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p
    for name in ("md_dilate", "md_erode", "md_dilate_noalloc"):
        f = getattr(lib, name)
        f.argtypes = [vp, i, i, i, u8, vp, i, vp]
        f.restype = i
    for name in ("md_dilate_host", "md_erode_host"):
        f = getattr(lib, name)
        f.argtypes = [vp, ctypes.c_longlong, i, i, u8, vp, i, vp]
        f.restype = i
    for name in ("md_dilate3_host", "md_erode3_host"):
        f = getattr(lib, name)
        f.argtypes = [vp, ctypes.c_longlong, i, i, i, u8, vp, i, vp]
        f.restype = i
    for name in ("md_dilate3", "md_erode3"):
        f = getattr(lib, name)
        f.argtypes = [vp, i, i, i, i, u8, vp, i, vp]
        f.restype = i
    lib.md_dilate_batch.argtypes = [ctypes.POINTER(_Job), i]
    lib.md_dilate_batch.restype = i
    lib.md_set_stream.argtypes = [vp]
    lib.md_set_stream.restype = i
    lib.md_set_option.argtypes = [i, ctypes.c_double]
    lib.md_set_option.restype = i
    lib.md_get_option.argtypes = [i]
    lib.md_get_option.restype = ctypes.c_double
    lib.md_get_stats.argtypes = [ctypes.POINTER(_Stats)]
    lib.md_get_stats.restype = i
    lib.md_last_error.argtypes = []
    lib.md_last_error.restype = ctypes.c_char_p
    lib.md_release.argtypes = []
    lib.md_release.restype = i
    lib.md_debug_tile_values.argtypes = [vp, i, i, i, u8, vp, i, i, i, i, i, i, vp]
    lib.md_debug_tile_values.restype = i
    lib.md_profile_get.argtypes = [ctypes.POINTER(_StageTime), i, ctypes.POINTER(ctypes.c_int)]
    lib.md_profile_get.restype = i
    lib.md_profile_reset.argtypes = []
    lib.md_profile_reset.restype = i
    lib.md_morph.argtypes = [i, vp, i, i, i, u8, vp, i, vp]
    lib.md_morph.restype = i
    lib.md_morph3.argtypes = [i, vp, i, i, i, i, u8, vp, i, vp]
    lib.md_morph3.restype = i
    lib.md_cost_model.argtypes = [ctypes.POINTER(ctypes.c_double), i, ctypes.POINTER(ctypes.c_int)]
    lib.md_cost_model.restype = i
    lib.md_memory_usage.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_int)]
    lib.md_memory_usage.restype = i
    lib.md_plan.argtypes = [ctypes.POINTER(_Job), i, ctypes.POINTER(_PlanInfo)]
    lib.md_plan.restype = i
    lib.md_set_workspace.argtypes = [vp, ctypes.c_size_t]
    lib.md_set_workspace.restype = i
    lib.md_workspace_size.argtypes = [ctypes.POINTER(_Job), i]
    lib.md_workspace_size.restype = ctypes.c_size_t
    lib.md_debug_perturb_tiles.argtypes = [ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_uint8), i]
    lib.md_debug_perturb_tiles.restype = i
    lib.md_debug_tile_flags.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.c_longlong,
                                        ctypes.POINTER(ctypes.c_longlong)]
    lib.md_debug_tile_flags.restype = i
    lib.md_debug_dft16.argtypes = [i, vp, vp, ctypes.c_longlong, i]
    lib.md_debug_dft16.restype = i
    _lib = lib
    return lib


def header_symbols() -> list[str]:
    """Function names declared in include/md.h."""
    text = open(_HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(md_\w+)\s*\(", text, re.M)))


def exported_symbols() -> dict[str, bool]:
    lib = load()
    out = {}
    for name in header_symbols():
        try:
            getattr(lib, name)
            out[name] = True
        except AttributeError:
            out[name] = False
    return out


def _check(rc: int):
    if rc != 0:
        raise MDError(rc, load().md_last_error().decode())


def _se_arrays(mask, off):
    mask = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
    off = np.ascontiguousarray(np.asarray(off), dtype=np.int32)
    if mask.ndim != 2 or mask.shape != off.shape or mask.shape[0] != mask.shape[1]:
        raise ValueError("mask and offsets must be k x k arrays of the same shape")
    return mask, off


def _device_image(img):
    import torch

    if not isinstance(img, torch.Tensor) or not img.is_cuda:
        raise TypeError("image must be a torch tensor on a HIP device")
    if img.dtype != torch.int32 or img.dim() != 2:
        raise TypeError("image must be a 2-D torch.int32 tensor")
    return img.contiguous()


def _bind_stream(dev):
    import torch

    load().md_set_stream(ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))


def _run_single(fname, img, mask, off, L, out):
    import torch

    lib = load()
    img = _device_image(img)
    mask, off = _se_arrays(mask, off)
    if out is None:
        out = torch.empty_like(img)
    elif out.shape != img.shape or out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor shaped like the image")
    with torch.cuda.device(img.device):
        _bind_stream(img.device)
        rc = getattr(lib, fname)(img.data_ptr(), img.shape[0], img.shape[1], int(L),
                                 mask.ctypes.data, off.ctypes.data, mask.shape[0], out.data_ptr())
    _check(rc)
    return out


def dilate(img, mask, off, L: int, out=None):
    """Exact dilation: max over the SE of img(x-y) + b(y), 0 on empty windows."""
    return _run_single("md_dilate", img, mask, off, L, out)


def dilate_noalloc(img, mask, off, L: int, out=None):
    """md_dilate_noalloc: the same dilation through the direct window with no
    device allocation in the library (k <= 127)."""
    return _run_single("md_dilate_noalloc", img, mask, off, L, out)


def erode(img, mask, off, L: int, out=None):
    """Exact erosion: min over the SE of img(x+y) - b(y), L-1 on empty windows."""
    return _run_single("md_erode", img, mask, off, L, out)


def _run_host(fname, img, mask, off, L, out):
    """img / out: C-contiguous int32 numpy arrays or CPU torch tensors (pinned
    or not) of shape (H, W)."""
    import torch

    lib = load()

    def ptr_of(a, what):
        if isinstance(a, torch.Tensor):
            if a.is_cuda or a.dtype != torch.int32 or a.dim() != 2 or not a.is_contiguous():
                raise TypeError(f"{what} must be a contiguous 2-D int32 host tensor")
            return a.data_ptr(), tuple(a.shape)
        if not isinstance(a, np.ndarray) or a.dtype != np.int32 or a.ndim != 2 or not a.flags.c_contiguous:
            raise TypeError(f"{what} must be a C-contiguous 2-D int32 numpy array")
        return a.ctypes.data, a.shape

    ip, shape = ptr_of(img, "image")
    if out is None:
        out = np.empty(shape, np.int32)
    op_, oshape = ptr_of(out, "out")
    if oshape != shape:
        raise ValueError("out must have the image's shape")
    mask, off = _se_arrays(mask, off)
    rc = getattr(lib, fname)(ip, shape[0], shape[1], int(L), mask.ctypes.data, off.ctypes.data, mask.shape[0], op_)
    _check(rc)
    return out


def dilate_host(img, mask, off, L: int, out=None):
    """Exact dilation of an image in host memory, streamed through the GPU in
    bands of rows (md_dilate_host)."""
    return _run_host("md_dilate_host", img, mask, off, L, out)


def erode_host(img, mask, off, L: int, out=None):
    """Exact erosion of an image in host memory (md_erode_host)."""
    return _run_host("md_erode_host", img, mask, off, L, out)


def _run_volume_host(fname, vol, mask, off, L, out):
    """vol / out: C-contiguous int32 numpy arrays or CPU torch tensors of
    shape (D, H, W)."""
    import torch

    lib = load()

    def ptr_of(a, what):
        if isinstance(a, torch.Tensor):
            if a.is_cuda or a.dtype != torch.int32 or a.dim() != 3 or not a.is_contiguous():
                raise TypeError(f"{what} must be a contiguous 3-D int32 host tensor")
            return a.data_ptr(), tuple(a.shape)
        if not isinstance(a, np.ndarray) or a.dtype != np.int32 or a.ndim != 3 or not a.flags.c_contiguous:
            raise TypeError(f"{what} must be a C-contiguous 3-D int32 numpy array")
        return a.ctypes.data, a.shape

    vp_, shape = ptr_of(vol, "volume")
    if out is None:
        out = np.empty(shape, np.int32)
    op_, oshape = ptr_of(out, "out")
    if oshape != shape:
        raise ValueError("out must have the volume's shape")
    mask = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
    off = np.ascontiguousarray(np.asarray(off), dtype=np.int32)
    if mask.ndim != 3 or mask.shape != off.shape or len(set(mask.shape)) != 1:
        raise ValueError("mask and offsets must be k x k x k arrays of the same shape")
    rc = getattr(lib, fname)(vp_, shape[0], shape[1], shape[2], int(L), mask.ctypes.data, off.ctypes.data,
                             mask.shape[0], op_)
    _check(rc)
    return out


def dilate3_host(vol, mask, off, L: int, out=None):
    """Exact volume dilation of a volume in host memory, streamed through the
    GPU in bands of slices (md_dilate3_host)."""
    return _run_volume_host("md_dilate3_host", vol, mask, off, L, out)


def erode3_host(vol, mask, off, L: int, out=None):
    """Exact volume erosion from host memory (md_erode3_host)."""
    return _run_volume_host("md_erode3_host", vol, mask, off, L, out)


def _run_volume(fname, vol, mask, off, L, out):
    import torch

    lib = load()
    if not isinstance(vol, torch.Tensor) or not vol.is_cuda:
        raise TypeError("volume must be a torch tensor on a HIP device")
    if vol.dtype != torch.int32 or vol.dim() != 3:
        raise TypeError("volume must be a 3-D torch.int32 tensor")
    vol = vol.contiguous()
    mask = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
    off = np.ascontiguousarray(np.asarray(off), dtype=np.int32)
    if mask.ndim != 3 or mask.shape != off.shape or len(set(mask.shape)) != 1:
        raise ValueError("mask and offsets must be k x k x k arrays of the same shape")
    if out is None:
        out = torch.empty_like(vol)
    elif out.shape != vol.shape or out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor shaped like the volume")
    with torch.cuda.device(vol.device):
        _bind_stream(vol.device)
        rc = getattr(lib, fname)(vol.data_ptr(), vol.shape[0], vol.shape[1], vol.shape[2], int(L),
                                 mask.ctypes.data, off.ctypes.data, mask.shape[0], out.data_ptr())
    _check(rc)
    return out


def morph3(op: int, vol, mask, off, L: int, out=None):
    """md_morph3: a volume composition (op as for morph: 0 dilation ... 6
    black top-hat) over three axes."""
    import torch

    lib = load()
    if not isinstance(vol, torch.Tensor) or not vol.is_cuda or vol.dtype != torch.int32 or vol.dim() != 3:
        raise TypeError("volume must be a 3-D torch.int32 tensor on a HIP device")
    vol = vol.contiguous()
    mask = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
    off = np.ascontiguousarray(np.asarray(off), dtype=np.int32)
    if mask.ndim != 3 or mask.shape != off.shape or len(set(mask.shape)) != 1:
        raise ValueError("mask and offsets must be k x k x k arrays of the same shape")
    if out is None:
        out = torch.empty_like(vol)
    with torch.cuda.device(vol.device):
        _bind_stream(vol.device)
        rc = lib.md_morph3(int(op), vol.data_ptr(), vol.shape[0], vol.shape[1], vol.shape[2], int(L),
                           mask.ctypes.data, off.ctypes.data, mask.shape[0], out.data_ptr())
    _check(rc)
    return out


def dilate3(vol, mask, off, L: int, out=None):
    """Exact volume dilation (md_dilate3): max over the k x k x k SE of
    vol(x-y) + b(y), 0 on empty windows."""
    return _run_volume("md_dilate3", vol, mask, off, L, out)


def erode3(vol, mask, off, L: int, out=None):
    """Exact volume erosion (md_erode3): min over the SE of vol(x+y) - b(y),
    L-1 on empty windows."""
    return _run_volume("md_erode3", vol, mask, off, L, out)


# md_op codes of include/md.h
DILATE, ERODE, OPEN, CLOSE, GRADIENT, TOPHAT, BLACKHAT = range(7)


def morph(op: int, img, mask, off, L: int, out=None):
    """Dilation, erosion or one of their compositions (md_morph): op 0
    dilation, 1 erosion, 2 opening, 3 closing, 4 Beucher gradient, 5 white
    top-hat, 6 black top-hat."""
    import torch

    lib = load()
    img = _device_image(img)
    mask, off = _se_arrays(mask, off)
    if out is None:
        out = torch.empty_like(img)
    elif out.shape != img.shape or out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor shaped like the image")
    with torch.cuda.device(img.device):
        _bind_stream(img.device)
        rc = lib.md_morph(int(op), img.data_ptr(), img.shape[0], img.shape[1], int(L), mask.ctypes.data,
                          off.ctypes.data, mask.shape[0], out.data_ptr())
    _check(rc)
    return out


def opening(img, mask, off, L: int, out=None):
    """(img erosion b) dilation b; -m where the dilation window is empty."""
    return morph(OPEN, img, mask, off, L, out)


def closing(img, mask, off, L: int, out=None):
    """(img dilation b) erosion b; L-1+m where the erosion window is empty."""
    return morph(CLOSE, img, mask, off, L, out)


def gradient(img, mask, off, L: int, out=None):
    """Beucher gradient: dilation minus erosion."""
    return morph(GRADIENT, img, mask, off, L, out)


def tophat(img, mask, off, L: int, out=None):
    """White top-hat: img minus its opening."""
    return morph(TOPHAT, img, mask, off, L, out)


def blackhat(img, mask, off, L: int, out=None):
    """Black top-hat: the closing minus img."""
    return morph(BLACKHAT, img, mask, off, L, out)


class Batch:
    """A batch for md_dilate_batch, marshalled once: jobs is a sequence of
    (img, mask, off, L, op) with op 0 = dilation, 1 = erosion and images
    int32 device tensors; outs (optional) the output tensors.  run() makes
    the call and returns the outputs; a loop that runs the same jobs on the
    same buffers pays the marshalling once.  The object keeps the tensors and
    SE arrays alive; SE arrays changed in place are seen by the library (it
    compares their contents with the previous call's)."""

    def __init__(self, jobs, outs=None):
        import torch

        self.lib = load()
        self.n = len(jobs)
        self.arr = (_Job * self.n)()
        self.keep = []
        self.outs = []
        self.dev = None
        for q, (img, mask, off, L, op) in enumerate(jobs):
            img = _device_image(img)
            self.dev = img.device if self.dev is None else self.dev
            mask, off = _se_arrays(mask, off)
            out = torch.empty_like(img) if outs is None else outs[q]
            self.keep.append((img, mask, off))
            self.outs.append(out)
            self.arr[q] = _Job(img.data_ptr(), img.shape[0], img.shape[1], int(L), mask.ctypes.data,
                               off.ctypes.data, mask.shape[0], out.data_ptr(), int(op))

    def run(self):
        import torch

        with torch.cuda.device(self.dev):
            _bind_stream(self.dev)
            rc = self.lib.md_dilate_batch(self.arr, self.n)
        _check(rc)
        return self.outs


def set_workspace(buf=None):
    """md_set_workspace: a caller-owned device buffer (a torch tensor on the
    device, 256-byte aligned; the library carves its transform workspace from
    it) or None for library-owned workspace.  Keep the tensor alive while it
    is set."""
    if buf is None:
        _check(load().md_set_workspace(None, 0))
    else:
        _check(load().md_set_workspace(ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))


def workspace_size(jobs) -> int:
    """md_workspace_size for jobs given as for dilate_batch (outputs are not
    needed: a placeholder pointer is passed)."""
    lib = load()
    n = len(jobs)
    arr = (_Job * n)()
    keep = []
    for q, (img, mask, off, L, op) in enumerate(jobs):
        img = _device_image(img)
        mask, off = _se_arrays(mask, off)
        keep.append((img, mask, off))
        arr[q] = _Job(img.data_ptr(), img.shape[0], img.shape[1], int(L), mask.ctypes.data, off.ctypes.data,
                      mask.shape[0], img.data_ptr() + 4, int(op))
    size = lib.md_workspace_size(arr, n)
    err = lib.md_last_error().decode()
    if err:
        raise MDError(-1, err)
    return int(size)


def memory_usage() -> dict:
    """md_memory_usage: bytes of the library's cache and of its cached batch
    plans' workspace, and the number of cached plans."""
    c, p, n = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_int(0)
    _check(load().md_memory_usage(ctypes.byref(c), ctypes.byref(p), ctypes.byref(n)))
    return {"cache_bytes": c.value, "plan_bytes": p.value, "plans": n.value}


def plan(shape, mask, off, L: int, op: int = 0, batch: bool = False) -> dict:
    """md_plan: the host-side plan of one job of the given (H, W) shape (no
    device involved; placeholder image pointers are passed)."""
    mask, off = _se_arrays(mask, off)
    H, W = shape
    job = _Job(16, int(H), int(W), int(L), mask.ctypes.data, off.ctypes.data, mask.shape[0], 32, int(op))
    info = _PlanInfo()
    _check(load().md_plan(ctypes.byref(job), 1 if batch else 0, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in _PlanInfo._fields_}


def debug_perturb_tiles(tiles, bits):
    """md_debug_perturb_tiles: flat transform-tile indices and their bits (1:
    first pass, 2: FP64 recompute); empty lists clear the hook."""
    t = np.ascontiguousarray(np.asarray(tiles, dtype=np.int64))
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
    if t.shape != b.shape or t.ndim != 1:
        raise ValueError("tiles and bits must be 1-D of the same length")
    _check(load().md_debug_perturb_tiles(t.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                         b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), t.shape[0]))


def debug_dft16(variant: int, x, reps: int = 1, out=None):
    """md_debug_dft16 on a complex64 HIP tensor x of shape (lines, 16):
    `reps` forward 16-point DFTs per line by the vector ALU (0), FP32
    matrix cores (1) or split-bf16 matrix cores (2)."""
    import torch

    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.complex64 or x.dim() != 2 \
            or x.shape[1] != 16:
        raise TypeError("x must be a complex64 HIP tensor of shape (lines, 16)")
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    with torch.cuda.device(x.device):
        _bind_stream(x.device)
        _check(load().md_debug_dft16(int(variant), x.data_ptr(), out.data_ptr(), x.shape[0], int(reps)))
    return out


def debug_tile_flags() -> np.ndarray:
    """md_debug_tile_flags: per-tile tier bits of the last call (1: FP64
    recompute, 2: integer window), flat tile order."""
    lib = load()
    n = ctypes.c_longlong(0)
    _check(lib.md_debug_tile_flags(None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), np.uint32)
    _check(lib.md_debug_tile_flags(out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), n.value, ctypes.byref(n)))
    return out[:n.value]


def dilate_batch(jobs, outs=None):
    """jobs: sequence of (img, mask, off, L, op) with op 0 = dilation, 1 =
    erosion; images are int32 device tensors.  Returns the output tensors."""
    return Batch(jobs, outs).run()


def set_option(key, value: float):
    key = _OPT_NAMES.get(key, key)
    _check(load().md_set_option(int(key), float(value)))


def get_option(key) -> float:
    key = _OPT_NAMES.get(key, key)
    return float(load().md_get_option(int(key)))


@contextlib.contextmanager
def options(**kw):
    """Temporarily set options by name, e.g. options(precision=1, path=1)."""
    saved = {k: get_option(k) for k in kw}
    try:
        for k, v in kw.items():
            set_option(k, v)
        yield
    finally:
        for k, v in saved.items():
            set_option(k, v)


def get_stats() -> dict:
    st = _Stats()
    _check(load().md_get_stats(ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in _Stats._fields_}


def release():
    _check(load().md_release())


def profile_reset():
    _check(load().md_profile_reset())


def profile_get() -> dict:
    """Per-stage totals collected while the 'profile' option is 1:
    {name: {ms, launches, alg_bytes, alg_ops}}."""
    lib = load()
    n = ctypes.c_int(0)
    _check(lib.md_profile_get(None, 0, ctypes.byref(n)))
    arr = (_StageTime * max(1, n.value))()
    _check(lib.md_profile_get(arr, n.value, ctypes.byref(n)))
    return {arr[q].name.decode(): {"ms": arr[q].ms, "launches": arr[q].launches,
                                   "alg_bytes": arr[q].alg_bytes, "alg_ops": arr[q].alg_ops,
                                   "units": arr[q].units}
            for q in range(n.value)}


def cost_model() -> dict:
    """Cost-model constants in use (ns per work unit) and whether the
    autotuner measured them."""
    n = 24
    v = (ctypes.c_double * n)()
    measured = ctypes.c_int(0)
    _check(load().md_cost_model(v, n, ctypes.byref(measured)))
    lens = [16 << q for q in range(7)]
    return {"direct16_per_px_cell": v[0], "direct32_per_px_cell": v[1], "direct_per_staged_word": v[2],
            "decode32_per_px_bins2": v[3], "decode64_per_px_bins2": v[4],
            "fft32_item": {n: v[5 + q] for q, n in enumerate(lens)},
            "fft64_item": {n: v[12 + q] for q, n in enumerate(lens)},
            "ntt_item": {n: v[19 + q] for q, n in enumerate(lens[:4])}, "decode_ntt_per_px_bin": v[23],
            "measured": bool(measured.value)}


def debug_tile_values(img, mask, off, L: int, n_t: int, n_r: int, precision: int, ty: int, tx: int):
    """Per-bin values of one tile before the inverse range transform
    (see md_debug_tile_values); returns complex128 (n_r//2+1, T*T)."""
    import torch

    lib = load()
    img = _device_image(img)
    mask, off = _se_arrays(mask, off)
    k = mask.shape[0]
    T = n_t - k + 1
    bins = n_r if int(precision) == 2 else n_r // 2 + 1
    dst = np.zeros(2 * bins * T * T, np.float64)
    with torch.cuda.device(img.device):
        _bind_stream(img.device)
        rc = lib.md_debug_tile_values(img.data_ptr(), img.shape[0], img.shape[1], int(L), mask.ctypes.data,
                                      off.ctypes.data, k, int(n_t), int(n_r), int(precision), int(ty), int(tx),
                                      dst.ctypes.data)
    _check(rc)
    return (dst[0::2] + 1j * dst[1::2]).reshape(bins, T * T)
