"""Python binding of the C ABI in include/phgrms.h (argument marshalling only).

Every step of the method runs in the HIP library; PyTorch supplies device
memory and streams.  If the library has not been built, every call raises
PhgrmsError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libphgrms.so")

STATUS = {
    0: "PHGRMS_OK", -1: "PHGRMS_EINVAL", -2: "PHGRMS_ENOSPC", -3: "PHGRMS_EDEVICE",
    -4: "PHGRMS_EUNSUPPORTED", -5: "PHGRMS_EBUSY", -6: "PHGRMS_ENOTFOUND",
    -7: "PHGRMS_EAGAIN",
}
BETA_MAX = 4
K_MAX = 1024
COUNT_SLOTS = 512   # PHGRMS_COUNT_SLOTS: int64 count slots per pass
STOP_ON_CYCLE = 1   # PHGRMS_STOP_ON_CYCLE: flag of phgrms_denoise_ex


class PhgrmsError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), message))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("k", ctypes.c_int32)]


class Item(ctypes.Structure):
    _fields_ = [("in_off", ctypes.c_uint64), ("out_off", ctypes.c_uint64), ("p", Params)]


_lib = None
_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load (once) and declare the C ABI.  Raises if the library is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise PhgrmsError(-3, "HIP library %s is not built; run "
                              "`python -m paper_1306_5390_amd.build`" % path)
        lib = ctypes.CDLL(path)
        vp, sz, i32, i64p, i32p = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int32))
        lib.phgrms_status_str.argtypes = [ctypes.c_int]
        lib.phgrms_status_str.restype = ctypes.c_char_p
        lib.phgrms_last_error.argtypes = []
        lib.phgrms_last_error.restype = ctypes.c_char_p
        lib.phgrms_version.argtypes = []
        lib.phgrms_version.restype = ctypes.c_int
        lib.phgrms_workspace_bytes.argtypes = [Params]
        lib.phgrms_workspace_bytes.restype = sz
        for name in ("phgrms_denoise", "phgrms_denoise_plain"):
            f = getattr(lib, name)
            f.argtypes = [vp, vp, Params, vp, sz, i64p, i32p, vp]
            f.restype = ctypes.c_int
        lib.phgrms_denoise_async.argtypes = [vp, vp, Params, vp, sz, vp, vp, vp]
        lib.phgrms_denoise_ex.restype = ctypes.c_int
        lib.phgrms_denoise_ex.argtypes = [vp, vp, Params, i32, vp, sz, vp, vp, vp]
        lib.phgrms_denoise_async.restype = ctypes.c_int
        lib.phgrms_cardinality.argtypes = [vp, i32, i32, i32, i32, vp, vp]
        lib.phgrms_cardinality.restype = ctypes.c_int
        lib.phgrms_run_passes.argtypes = [vp, vp, Params, i32, i32, vp, vp, vp]
        lib.phgrms_run_passes.restype = ctypes.c_int
        lib.phgrms_change_map_bytes.argtypes = [Params]
        lib.phgrms_change_map_bytes.restype = sz
        lib.phgrms_shape_tracks_changes.argtypes = [i32]
        lib.phgrms_shape_tracks_changes.restype = ctypes.c_int
        lib.phgrms_shape_skips_unchanged.argtypes = [i32]
        lib.phgrms_shape_skips_unchanged.restype = ctypes.c_int
        lib.phgrms_cardinality_scatter.argtypes = [vp, i32, i32, i32, i32, vp, vp]
        lib.phgrms_cardinality_scatter.restype = ctypes.c_int
        lib.phgrms_salt_pepper.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_uint32, vp]
        lib.phgrms_salt_pepper.restype = ctypes.c_int
        lib.phgrms_sq_diff_sum.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
        lib.phgrms_sq_diff_sum.restype = ctypes.c_int
        lib.phgrms_selftest.argtypes = [vp, vp]
        lib.phgrms_selftest.restype = ctypes.c_int
        lib.phgrms_num_shapes.argtypes = []
        lib.phgrms_num_shapes.restype = ctypes.c_int
        lib.phgrms_shape_info.argtypes = [i32, i32p, i32p, i32p]
        lib.phgrms_shape_info.restype = ctypes.c_int
        lib.phgrms_set_tuning.argtypes = [i32, i32]
        lib.phgrms_set_tuning.restype = ctypes.c_int
        lib.phgrms_get_tuning.argtypes = [i32]
        lib.phgrms_get_tuning.restype = ctypes.c_int
        lib.phgrms_batch_plan.argtypes = [ctypes.c_void_p, i32, ctypes.c_char_p,
                                          ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_size_t)]
        lib.phgrms_batch_plan.restype = ctypes.c_int
        lib.phgrms_batch_run.argtypes = [vp, vp, sz, vp, sz, vp, sz, vp, vp, vp]
        lib.phgrms_batch_run.restype = ctypes.c_int
        lib.phgrms_batch_launches.argtypes = [vp]
        lib.phgrms_batch_launches.restype = ctypes.c_int
        lib.phgrms_plan_destroy.argtypes = [vp]
        lib.phgrms_plan_destroy.restype = None
        lib.phgrms_server_create.argtypes = [vp, vp, sz, ctypes.POINTER(ctypes.c_void_p)]
        lib.phgrms_server_create.restype = ctypes.c_int
        lib.phgrms_server_submit.argtypes = [vp, vp, Params, ctypes.POINTER(ctypes.c_uint64)]
        lib.phgrms_server_submit_host.restype = ctypes.c_int
        lib.phgrms_server_submit_host.argtypes = [vp, vp, vp, Params,
                                                  ctypes.POINTER(ctypes.c_uint64)]
        lib.phgrms_server_submit.restype = ctypes.c_int
        lib.phgrms_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p),
                                           i32p, i64p, ctypes.POINTER(ctypes.c_double)]
        lib.phgrms_server_poll.restype = ctypes.c_int
        lib.phgrms_server_next_done.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32]
        lib.phgrms_server_next_done.restype = ctypes.c_int
        lib.phgrms_server_release.argtypes = [vp, ctypes.c_uint64]
        lib.phgrms_server_release.restype = ctypes.c_int
        lib.phgrms_server_get_stats.argtypes = [vp, vp]
        lib.phgrms_server_get_stats.restype = ctypes.c_int
        lib.phgrms_server_destroy.argtypes = [vp]
        lib.phgrms_server_destroy.restype = None
        lib.phgrms_autotune_workspace_bytes.argtypes = [Params]
        lib.phgrms_autotune_workspace_bytes.restype = sz
        lib.phgrms_autotune.argtypes = [Params, vp, vp, sz, i32, i32p,
                                        ctypes.POINTER(ctypes.c_float), ctypes.c_char_p, vp]
        lib.phgrms_load_tuning.argtypes = [ctypes.c_char_p]
        lib.phgrms_load_tuning.restype = ctypes.c_int
        lib.phgrms_save_tuning.argtypes = [ctypes.c_char_p]
        lib.phgrms_save_tuning.restype = ctypes.c_int
        lib.phgrms_autotune.restype = ctypes.c_int
        lib.phgrms_set_tuning_class.argtypes = [i32, i32, i32]
        lib.phgrms_set_batch_tuning_class.argtypes = [i32, i32, i32]
        lib.phgrms_set_batch_tuning_class.restype = ctypes.c_int
        lib.phgrms_get_batch_tuning_class.argtypes = [i32, i32]
        lib.phgrms_get_batch_tuning_class.restype = ctypes.c_int
        lib.phgrms_set_tuning_class.restype = ctypes.c_int
        lib.phgrms_get_tuning_class.argtypes = [i32, i32]
        lib.phgrms_get_tuning_class.restype = ctypes.c_int
        lib.phgrms_set_grid_mode.argtypes = [i32]
        lib.phgrms_set_grid_mode.restype = ctypes.c_int
        lib.phgrms_get_grid_mode.argtypes = []
        lib.phgrms_get_grid_mode.restype = ctypes.c_int
        lib.phgrms_calib_copy.argtypes = [vp, vp, sz, vp]
        lib.phgrms_calib_copy.restype = ctypes.c_int
        lib.phgrms_calib_valu.argtypes = [vp, i32, i32, i32, ctypes.POINTER(ctypes.c_uint64), vp]
        lib.phgrms_calib_valu.restype = ctypes.c_int
        _lib = lib
        return lib


def check(rc: int) -> None:
    if rc != 0:
        lib = load_library()
        raise PhgrmsError(rc, lib.phgrms_last_error().decode(errors="replace"))


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_image(img: torch.Tensor) -> None:
    if not isinstance(img, torch.Tensor):
        raise TypeError("image must be a torch.Tensor")
    if img.device.type != "cuda":
        raise PhgrmsError(-1, "image must be a device (cuda) tensor")
    if img.dtype != torch.uint8 or img.dim() != 2:
        raise PhgrmsError(-1, "image must be a 2-D uint8 tensor")
    if not img.is_contiguous():
        raise PhgrmsError(-1, "image must be contiguous (row pitch == cols)")


def version() -> int:
    return int(load_library().phgrms_version())


def workspace_bytes(rows: int, cols: int, alpha: int, beta: int, k: int) -> int:
    return int(load_library().phgrms_workspace_bytes(Params(rows, cols, alpha, beta, k)))


def _prepare(img, alpha, beta, k, out, workspace):
    _check_image(img)
    lib = load_library()
    rows, cols = img.shape
    p = Params(rows, cols, alpha, beta, k)
    nbytes = lib.phgrms_workspace_bytes(p)
    if nbytes == 0:
        # invalid parameters: let the library produce the message
        rc = lib.phgrms_denoise(None, None, p, None, 0, None, None, None)
        check(rc)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=img.device)
    if out is None:
        out = torch.empty_like(img)
    else:
        _check_image(out)
        if out.shape != img.shape:
            raise PhgrmsError(-1, "out has a different shape")
    return lib, p, out, workspace


def denoise(img: torch.Tensor, alpha: int, beta: int, k: int, out=None, workspace=None,
            stream=None, plain: bool = False, stop_on_cycle: bool = False):
    """Run the pass loop on a device image.

    Returns (out, iterations, changed) where changed[t] is the number of
    pixels pass t changed.  `plain=True` runs one launch per pass with a
    host read-back after each (the paper's host loop).  `stop_on_cycle=True`
    (opt-in) also stops after the first pass whose image equals the image
    two passes before it."""
    if stop_on_cycle:
        if plain:
            raise PhgrmsError(-1, "stop_on_cycle has no plain path")
        s = torch.cuda.current_stream(img.device) if stream is None else stream
        out, ch, it = denoise_async(img, alpha, beta, k, out=out, workspace=workspace,
                                    stream=s, stop_on_cycle=True)
        s.synchronize()
        n = int(it.item())
        return out, n, [int(x) for x in ch[:n].cpu().tolist()]
    lib, p, out, workspace = _prepare(img, alpha, beta, k, out, workspace)
    changed = (ctypes.c_int64 * max(k, 1))()
    it = ctypes.c_int32(0)
    fn = lib.phgrms_denoise_plain if plain else lib.phgrms_denoise
    with torch.cuda.device(img.device):
        rc = fn(img.data_ptr(), out.data_ptr(), p, workspace.data_ptr(),
                workspace.numel(), changed, ctypes.byref(it), _stream_handle(stream))
    check(rc)
    n = it.value
    return out, n, [int(changed[i]) for i in range(n)]


def denoise_async(img: torch.Tensor, alpha: int, beta: int, k: int, out=None,
                  workspace=None, changed=None, iterations=None, stream=None,
                  stop_on_cycle: bool = False):
    """Enqueue the pass loop; nothing synchronises.  Returns (out, changed,
    iterations) as device tensors (int64[k], int32[1]).  `stop_on_cycle`
    as in denoise()."""
    lib, p, out, workspace = _prepare(img, alpha, beta, k, out, workspace)
    if changed is None:
        changed = torch.empty(max(k, 1), dtype=torch.int64, device=img.device)
    if iterations is None:
        iterations = torch.empty(1, dtype=torch.int32, device=img.device)
    with torch.cuda.device(img.device):
        if stop_on_cycle:
            rc = lib.phgrms_denoise_ex(img.data_ptr(), out.data_ptr(), p, STOP_ON_CYCLE,
                                       workspace.data_ptr(), workspace.numel(),
                                       changed.data_ptr(), iterations.data_ptr(),
                                       _stream_handle(stream))
        else:
            rc = lib.phgrms_denoise_async(img.data_ptr(), out.data_ptr(), p,
                                          workspace.data_ptr(), workspace.numel(),
                                          changed.data_ptr(), iterations.data_ptr(),
                                          _stream_handle(stream))
    check(rc)
    return out, changed, iterations


def cardinality(img: torch.Tensor, alpha: int, beta: int, stream=None) -> torch.Tensor:
    """Algorithm 1's cardinality matrix, as a device int32 tensor."""
    _check_image(img)
    lib = load_library()
    rows, cols = img.shape
    card = torch.empty((rows, cols), dtype=torch.int16, device=img.device)
    with torch.cuda.device(img.device):
        rc = lib.phgrms_cardinality(img.data_ptr(), rows, cols, alpha, beta,
                                    card.data_ptr(), _stream_handle(stream))
    check(rc)
    return card.to(torch.int32) & 0xFFFF


def cardinality_scatter(img: torch.Tensor, alpha: int, beta: int, stream=None) -> torch.Tensor:
    """Algorithm 1 in the printed scatter form with atomic increments
    (int32 tensor, same values as cardinality())."""
    _check_image(img)
    rows, cols = img.shape
    card = torch.empty((rows, cols), dtype=torch.int32, device=img.device)
    with torch.cuda.device(img.device):
        check(load_library().phgrms_cardinality_scatter(img.data_ptr(), rows, cols, alpha, beta,
                                                        card.data_ptr(), _stream_handle(stream)))
    return card


def count_slots(npasses: int, device) -> torch.Tensor:
    """Zeroed count slots for run_passes (npasses x COUNT_SLOTS int64)."""
    return torch.zeros(npasses * COUNT_SLOTS, dtype=torch.int64, device=device)


def pass_counts(slots: torch.Tensor) -> list:
    """Per-pass changed counts from run_passes' count slots."""
    v = slots.view(-1, COUNT_SLOTS)[:, ::16]
    return [int(x) for x in v.sum(dim=1).cpu().tolist()]


def change_maps(rows: int, cols: int, device) -> torch.Tensor:
    """Device buffer for run_passes' change maps of a rows x cols image.
    Uninitialised: a sequence's first launch reads no map, and every launch
    writes its whole map before the next one reads it (nothing is enqueued
    here, so the buffer needs no ordering against other streams)."""
    n = load_library().phgrms_change_map_bytes(Params(rows, cols, 0, 1, 0))
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def run_passes(src: torch.Tensor, dst: torch.Tensor, alpha: int, beta: int, npasses: int,
               shape: int, slots: torch.Tensor, stream=None, pass_index: int = 0,
               maps: torch.Tensor = None) -> None:
    """One pass-kernel launch (npasses passes) from src to dst; `slots`
    (see count_slots / pass_counts, zeroed by the caller) accumulates the
    changed counts.  With `maps` (see change_maps; change-tracking shapes
    only, see shape_tracks_changes),
    launch `pass_index` of a sequence over one image copies through the rows
    the previous launch's change map shows cannot change."""
    _check_image(src)
    _check_image(dst)
    if slots.numel() < npasses * COUNT_SLOTS or slots.dtype != torch.int64:
        raise PhgrmsError(-1, "slots must hold npasses * COUNT_SLOTS int64 values")
    lib = load_library()
    rows, cols = src.shape
    p = Params(rows, cols, alpha, beta, npasses)
    if maps is not None and (maps.dtype != torch.uint8 or not maps.is_cuda or
                             maps.numel() < lib.phgrms_change_map_bytes(p)):
        raise PhgrmsError(-1, "maps must be a device uint8 tensor of change_maps' size")
    with torch.cuda.device(src.device):
        rc = lib.phgrms_run_passes(src.data_ptr(), dst.data_ptr(), p, shape, pass_index,
                                   slots.data_ptr(), None if maps is None else maps.data_ptr(),
                                   _stream_handle(stream))
    check(rc)


def salt_pepper(img: torch.Tensor, seed: int, t_pepper: int, t_salt: int,
                out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Salt-and-pepper noise on a device image (see phgrms_salt_pepper;
    synth.noise_thresholds gives the thresholds of a density).  Enqueued on
    `stream`, no synchronisation."""
    _check_image(img)
    if out is None:
        out = torch.empty_like(img)
    else:
        _check_image(out)
        if out.shape != img.shape:
            raise PhgrmsError(-1, "output shape differs")
    with torch.cuda.device(img.device):
        check(load_library().phgrms_salt_pepper(
            img.data_ptr(), out.data_ptr(), img.numel(), ctypes.c_uint64(seed),
            ctypes.c_uint32(t_pepper), ctypes.c_uint32(t_salt), _stream_handle(stream)))
    return out


def sq_diff_sum(a: torch.Tensor, b: torch.Tensor, stream=None) -> torch.Tensor:
    """Device int64 scalar: sum of squared differences of two equal-shape
    device uint8 images (enqueued, not synchronised)."""
    _check_image(a)
    _check_image(b)
    if a.shape != b.shape:
        raise PhgrmsError(-1, "shapes differ")
    res = torch.empty(1, dtype=torch.int64, device=a.device)
    with torch.cuda.device(a.device):
        check(load_library().phgrms_sq_diff_sum(a.data_ptr(), b.data_ptr(), a.numel(),
                                                res.data_ptr(), _stream_handle(stream)))
    return res


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    """Peak signal-to-noise ratio in dB, 10 log10(255^2 n / SSD), of two
    device images (the restoration measure of the paper's Table 2);
    infinite for equal images.  Synchronises."""
    ssd = int(sq_diff_sum(a, b).item())
    if ssd == 0:
        return float("inf")
    return 10.0 * math.log10(255.0 ** 2 * a.numel() / ssd)


def selftest(device="cuda:0") -> tuple:
    """(wrong quotients, wrong square roots) of the kernels' integer routines
    over their whole input domains (see phgrms_selftest)."""
    out = torch.zeros(2, dtype=torch.int64, device=device)
    with torch.cuda.device(out.device):
        check(load_library().phgrms_selftest(out.data_ptr(), _stream_handle(None)))
    v = out.cpu().tolist()
    return int(v[0]), int(v[1])


def calib_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """Stream copy of src's bytes into dst (see phgrms_calib_copy); enqueued
    on the stream, not synchronised."""
    if src.device != dst.device or not src.is_contiguous() or not dst.is_contiguous():
        raise PhgrmsError(-1, "contiguous tensors on one device expected")
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise PhgrmsError(-1, "destination smaller than source")
    with torch.cuda.device(src.device):
        check(load_library().phgrms_calib_copy(src.data_ptr(), dst.data_ptr(), n,
                                               _stream_handle(stream)))


def calib_valu(out: torch.Tensor, blocks: int, trips: int, kind: int, stream=None) -> int:
    """Integer VALU issue loop (see phgrms_calib_valu) writing blocks * 256
    words of `out` (int32 or uint32 storage); returns the VALU instructions
    each wave issues.  Enqueued on the stream, not synchronised."""
    if out.element_size() != 4 or out.numel() < blocks * 256 or not out.is_contiguous():
        raise PhgrmsError(-1, "out must hold blocks * 256 contiguous 32-bit words")
    per_wave = ctypes.c_uint64(0)
    with torch.cuda.device(out.device):
        check(load_library().phgrms_calib_valu(out.data_ptr(), blocks, trips, kind,
                                               ctypes.byref(per_wave), _stream_handle(stream)))
    return int(per_wave.value)


def shape_tracks_changes(shape: int) -> bool:
    """Whether kernel shape `shape` keeps change maps (see run_passes)."""
    rc = load_library().phgrms_shape_tracks_changes(shape)
    check(rc if rc < 0 else 0)
    return rc == 1


def shape_skips_unchanged(shape: int) -> bool:
    """Whether kernel shape `shape` leaves tiles and rows that cannot change
    untouched from the third pass on (see run_passes)."""
    rc = load_library().phgrms_shape_skips_unchanged(shape)
    check(rc if rc < 0 else 0)
    return rc == 1


def autotune_native(img: torch.Tensor, alpha: int, beta: int, k: int, reps: int = 3,
                    stream=None, cache_path=None):
    """The library's own autotuner (phgrms_autotune): times the pass loop on
    `img` with every compiled shape, one run at a time, and uses the fastest
    for beta and the image's size class (also written into the tuning cache
    `cache_path` if given).  Returns (best shape, microseconds per run for
    each shape)."""
    _check_image(img)
    lib = load_library()
    rows, cols = img.shape
    p = Params(rows, cols, alpha, beta, k)
    nbytes = lib.phgrms_autotune_workspace_bytes(p)
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=img.device)
    best = ctypes.c_int32(-1)
    us = (ctypes.c_float * lib.phgrms_num_shapes())()
    with torch.cuda.device(img.device):
        s = torch.cuda.current_stream(img.device) if stream is None else stream
        s.wait_stream(torch.cuda.current_stream(img.device))
        check(lib.phgrms_autotune(p, img.data_ptr(), ws.data_ptr(), ws.numel(), reps,
                                  ctypes.byref(best), us,
                                  None if cache_path is None else os.fsencode(cache_path),
                                  _stream_handle(s)))
    return best.value, [float(x) for x in us]


def load_tuning(path) -> None:
    """Apply a tuning cache file to the library's shape tables
    (phgrms_load_tuning)."""
    check(load_library().phgrms_load_tuning(os.fsencode(path)))


def save_tuning(path) -> None:
    """Write the library's shape tables as a tuning cache (phgrms_save_tuning)."""
    check(load_library().phgrms_save_tuning(os.fsencode(path)))


def shapes():
    """Compiled kernel shapes: list of (passes_per_launch, rows_per_wave, waves)."""
    lib = load_library()
    out = []
    for s in range(lib.phgrms_num_shapes()):
        t, r, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib.phgrms_shape_info(s, ctypes.byref(t), ctypes.byref(r), ctypes.byref(w)))
        out.append((t.value, r.value, w.value))
    return out


def set_tuning(beta: int, shape: int) -> None:
    check(load_library().phgrms_set_tuning(beta, shape))


def set_grid_mode(mode: int) -> None:
    """0: one workgroup per tile; 1: persistent workgroups."""
    check(load_library().phgrms_set_grid_mode(mode))


def get_grid_mode() -> int:
    return int(load_library().phgrms_get_grid_mode())


SIZE_CLASS_LIMITS = (1 << 20, 1 << 24)   # pixels: class 0 below, class 1 below, class 2


def size_class(npx: int) -> int:
    return 0 if npx < SIZE_CLASS_LIMITS[0] else (1 if npx < SIZE_CLASS_LIMITS[1] else 2)


def set_tuning_class(beta: int, cls: int, shape: int) -> None:
    check(load_library().phgrms_set_tuning_class(beta, cls, shape))


def set_batch_tuning_class(beta: int, cls: int, shape: int) -> None:
    """Shape of the batch path's launches for beta and size class (-1: every
    class); applies to Batch objects made afterwards."""
    check(load_library().phgrms_set_batch_tuning_class(beta, cls, shape))


def get_batch_tuning_class(beta: int, cls: int) -> int:
    rc = load_library().phgrms_get_batch_tuning_class(beta, cls)
    if rc < 0:
        check(rc)
    return rc


def get_tuning_class(beta: int, cls: int) -> int:
    rc = load_library().phgrms_get_tuning_class(beta, cls)
    if rc < 0:
        check(rc)
    return rc


def get_tuning(beta: int) -> int:
    rc = load_library().phgrms_get_tuning(beta)
    if rc < 0:
        check(rc)
    return rc


class Batch:
    """Many images, each with its own (rows, cols, alpha, beta, k), run as one
    multi-image launch sequence (phgrms_batch_*).

    `specs` is a list of (rows, cols, alpha, beta, k).  Inputs and outputs
    live in two device arenas at 256-byte aligned offsets (or at the offsets
    given).  run() enqueues the batch on a stream; the first run with a set
    of pointers captures a HIP graph that later runs replay.  `tune_cache`:
    a tuning cache file whose batch shapes this plan uses (else the
    process's current ones)."""

    def __init__(self, specs, device="cuda:0", in_offsets=None, out_offsets=None,
                 tune_cache=None):
        lib = load_library()
        self.lib = lib
        self.device = torch.device(device)
        n = len(specs)
        if n < 1:
            raise PhgrmsError(-1, "empty batch")
        items = (Item * n)()
        off = 0
        self.in_offsets, self.out_offsets = [], []
        for i, (r, c, a, b, k) in enumerate(specs):
            io = off if in_offsets is None else int(in_offsets[i])
            oo = off if out_offsets is None else int(out_offsets[i])
            items[i] = Item(io, oo, Params(r, c, a, b, k))
            self.in_offsets.append(io)
            self.out_offsets.append(oo)
            off += (r * c + 255) // 256 * 256
        self.specs = [tuple(s) for s in specs]
        self.arena_bytes = max(off, 1)
        plan = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        check(lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), n,
                                    None if tune_cache is None else os.fsencode(tune_cache),
                                    ctypes.byref(plan), ctypes.byref(ws)))
        self.plan = plan
        self.ws_bytes = ws.value
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.k_offsets = []
        acc = 0
        for s in self.specs:
            self.k_offsets.append(acc)
            acc += s[4]
        self.changed = torch.zeros(max(acc, 1), dtype=torch.int64, device=self.device)
        self.iterations = torch.zeros(n, dtype=torch.int32, device=self.device)

    def launches(self) -> int:
        return int(self.lib.phgrms_batch_launches(self.plan))

    def new_arena(self) -> torch.Tensor:
        return torch.zeros(self.arena_bytes, dtype=torch.uint8, device=self.device)

    def view(self, arena: torch.Tensor, i: int, out: bool = False) -> torch.Tensor:
        r, c = self.specs[i][0], self.specs[i][1]
        o = (self.out_offsets if out else self.in_offsets)[i]
        return arena[o:o + r * c].view(r, c)

    def run(self, in_arena: torch.Tensor, out_arena: torch.Tensor, stream=None) -> None:
        with torch.cuda.device(self.device):
            check(self.lib.phgrms_batch_run(
                self.plan, in_arena.data_ptr(), in_arena.numel(), out_arena.data_ptr(),
                out_arena.numel(), self.workspace.data_ptr(), self.ws_bytes,
                self.changed.data_ptr(), self.iterations.data_ptr(), _stream_handle(stream)))

    def results(self):
        """[(iterations, changed list)] per image (synchronises)."""
        its = self.iterations.cpu().tolist()
        ch = self.changed.cpu().tolist()
        out = []
        for i, s in enumerate(self.specs):
            o = self.k_offsets[i]
            out.append((its[i], ch[o:o + its[i]]))
        return out

    def close(self):
        if getattr(self, "plan", None):
            self.lib.phgrms_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerCfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("passes_per_step", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("cap_bytes", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("active", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64)]


class Server:
    """Continuous-batching request server (phgrms_server_*) on a device
    arena allocated here with PyTorch.  submit() returns a request id;
    poll() returns None until the request is done, then (out, iterations,
    changed, latency_s) with `out` a view into the arena that stays valid
    until release()."""

    def __init__(self, arena_bytes: int, device="cuda:0", max_active: int = 256,
                 passes_per_step: int = 0, max_queue: int = 65536, cap_bytes: int = 0):
        lib = load_library()
        self.lib = lib
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        cfg = ServerCfg(self.device.index or 0, max_active, passes_per_step, max_queue,
                        int(cap_bytes))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            torch.cuda.synchronize()
            check(lib.phgrms_server_create(ctypes.byref(cfg), self.arena.data_ptr(),
                                           self.arena.numel(), ctypes.byref(h)))
        self.handle = h
        self._inputs = {}
        self._host_out = {}
        self._shapes = {}

    def submit(self, img: torch.Tensor, alpha: int, beta: int, k: int) -> int:
        _check_image(img)
        rows, cols = img.shape
        rid = ctypes.c_uint64()
        check(self.lib.phgrms_server_submit(self.handle, img.data_ptr(),
                                            Params(rows, cols, alpha, beta, k), ctypes.byref(rid)))
        self._inputs[rid.value] = img
        self._shapes[rid.value] = (rows, cols, k)
        return rid.value

    def submit_host(self, img: torch.Tensor, out: torch.Tensor, alpha: int, beta: int,
                    k: int) -> int:
        """Submit an image in host memory; the result is copied to `out`
        (host, same shape) when the request finishes (the end-to-end form:
        both PCIe copies are part of the request).  Page-locked tensors
        (pin_memory) keep the copies asynchronous.  poll() then returns
        `out` as the image."""
        for t in (img, out):
            if not isinstance(t, torch.Tensor) or t.device.type != "cpu":
                raise PhgrmsError(-1, "host request buffers must be CPU tensors")
            if t.dtype != torch.uint8 or t.dim() != 2 or not t.is_contiguous():
                raise PhgrmsError(-1, "host request buffers must be contiguous 2-D uint8")
        if out.shape != img.shape:
            raise PhgrmsError(-1, "out has a different shape")
        rows, cols = img.shape
        rid = ctypes.c_uint64()
        check(self.lib.phgrms_server_submit_host(self.handle, img.data_ptr(), out.data_ptr(),
                                                 Params(rows, cols, alpha, beta, k),
                                                 ctypes.byref(rid)))
        self._inputs[rid.value] = (img, out)
        self._host_out[rid.value] = out
        self._shapes[rid.value] = (rows, cols, k)
        return rid.value

    def poll(self, rid: int):
        rows, cols, k = self._shapes[rid]
        out = ctypes.c_void_p()
        it = ctypes.c_int32()
        ch = (ctypes.c_int64 * max(k, 1))()
        lat = ctypes.c_double()
        rc = self.lib.phgrms_server_poll(self.handle, rid, ctypes.byref(out), ctypes.byref(it),
                                         ch, ctypes.byref(lat))
        if rc == -7:
            return None
        check(rc)
        self._inputs.pop(rid, None)
        host = self._host_out.pop(rid, None)
        if host is not None:
            view = host
        else:
            off = (out.value or self.arena.data_ptr()) - self.arena.data_ptr()
            view = self.arena[off:off + rows * cols].view(rows, cols)
        n = it.value
        return view, n, [int(ch[i]) for i in range(n)], lat.value

    def next_done(self, max_ids: int = 4096) -> list:
        """Ids completed since the last call, in completion order."""
        buf = (ctypes.c_uint64 * max_ids)()
        n = self.lib.phgrms_server_next_done(self.handle, buf, max_ids)
        if n < 0:
            check(n)
        return [int(buf[i]) for i in range(n)]

    def release(self, rid: int) -> None:
        check(self.lib.phgrms_server_release(self.handle, rid))
        self._shapes.pop(rid, None)
        self._host_out.pop(rid, None)
        self._inputs.pop(rid, None)

    def stats(self) -> dict:
        st = ServerStats()
        check(self.lib.phgrms_server_get_stats(self.handle, ctypes.byref(st)))
        return {f[0]: int(getattr(st, f[0])) for f in ServerStats._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.lib.phgrms_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
