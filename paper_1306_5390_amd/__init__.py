"""MI355X (gfx950) implementation of the P-HGRMS pass loop.

The compute path is the HIP library libphgrms.so (C ABI in include/phgrms.h);
this package holds that library's sources (csrc/), its build step (build.py),
the Python binding (_api.py), and the seeded input generator (synth.py).

The binding is loaded lazily so that `paper_1306_5390_amd.synth` can be used
without PyTorch or a built library.
"""
_API_NAMES = {
    "PhgrmsError", "Params", "denoise", "denoise_async", "cardinality",
    "workspace_bytes", "shapes", "set_tuning", "get_tuning", "load_library",
    "version", "check", "run_passes", "change_maps", "shape_tracks_changes", "shape_skips_unchanged", "salt_pepper", "sq_diff_sum", "psnr", "cardinality_scatter", "count_slots", "pass_counts",
    "COUNT_SLOTS", "set_grid_mode", "get_grid_mode", "Batch", "Item", "Server", "ServerCfg", "selftest", "set_tuning_class",
    "get_tuning_class", "size_class", "LIB_PATH", "BETA_MAX", "K_MAX", "autotune_native",
    "STOP_ON_CYCLE", "set_batch_tuning_class", "get_batch_tuning_class", "load_tuning",
    "save_tuning", "calib_copy", "calib_valu",
}


def __getattr__(name):
    if name in _API_NAMES:
        from . import _api
        return getattr(_api, name)
    raise AttributeError(name)
