"""CPU tests of the C ABI: the library loads, exports every function the
header declares, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phgrms.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(phgrms_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1306_5390_amd import _api
    if not os.path.exists(_api.LIB_PATH):
        from paper_1306_5390_amd import build
        build.build()
    return _api.load_library()


def test_header_declares_the_path():
    names = declared_functions()
    for must in ["phgrms_denoise", "phgrms_denoise_async", "phgrms_denoise_plain",
                 "phgrms_cardinality", "phgrms_workspace_bytes", "phgrms_last_error",
                 "phgrms_status_str"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    assert lib.phgrms_status_str(0) == b"PHGRMS_OK"
    assert lib.phgrms_status_str(-1) == b"PHGRMS_EINVAL"
    assert lib.phgrms_status_str(-4) == b"PHGRMS_EUNSUPPORTED"


def test_workspace_bytes(lib):
    from paper_1306_5390_amd._api import Params
    n = lib.phgrms_workspace_bytes(Params(100, 37, 20, 1, 10))
    assert n >= 100 * 37 + 8 * 10
    assert lib.phgrms_workspace_bytes(Params(100, 37, 300, 1, 10)) == 0
    assert lib.phgrms_workspace_bytes(Params(-1, 37, 20, 1, 10)) == 0
    assert lib.phgrms_workspace_bytes(Params(10, 37, 20, 0, 10)) == 0
    assert lib.phgrms_workspace_bytes(Params(10, 37, 20, 1, 1025)) == 0


def test_invalid_arguments_rejected_before_any_launch(lib):
    from paper_1306_5390_amd._api import Params
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        (Params(10, 10, -1, 1, 3), -1),      # alpha < 0
        (Params(10, 10, 256, 1, 3), -1),     # alpha > 255
        (Params(10, 10, 20, 0, 3), -1),      # beta < 1
        (Params(10, 10, 20, 5, 3), -4),      # beta above the built maximum
        (Params(10, 10, 20, 1, -1), -1),     # k < 0
        (Params(10, 10, 20, 1, 2000), -1),   # k too large
        (Params(-3, 10, 20, 1, 3), -1),      # negative size
        (Params(70000, 70000, 20, 1, 3), -1),  # more than 2^31 pixels
    ]
    for p, code in cases:
        rc = lib.phgrms_denoise(fake, fake, p, fake, 1 << 30, None, None, None)
        assert rc == code, (p.rows, p.cols, p.alpha, p.beta, p.k, rc)
        assert lib.phgrms_last_error() != b""
    p = Params(10, 10, 20, 1, 3)
    # workspace too small
    assert lib.phgrms_denoise(fake, ctypes.c_void_p(0x100000), p, ctypes.c_void_p(0x200000),
                              16, None, None, None) == -2
    # overlapping but not identical input/output
    assert lib.phgrms_denoise(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1005), p,
                              ctypes.c_void_p(0x200000), 1 << 20, None, None, None) == -1
    # workspace overlapping an image
    assert lib.phgrms_denoise(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), p,
                              ctypes.c_void_p(0x1010), 1 << 20, None, None, None) == -1
    # null image pointers
    assert lib.phgrms_denoise(None, None, p, fake, 1 << 20, None, None, None) == -1
    assert lib.phgrms_cardinality(None, 4, 4, 20, 1, None, None) == -1
    assert lib.phgrms_cardinality(fake, 4, 4, 20, 9, fake, None) == -4
    assert lib.phgrms_cardinality_scatter(None, 4, 4, 20, 1, None, None) == -1
    assert lib.phgrms_cardinality_scatter(fake, 4, 4, 20, 9, fake, None) == -4
    assert lib.phgrms_cardinality_scatter(fake, 4, 4, 300, 1, fake, None) == -1
    assert lib.phgrms_cardinality_scatter(fake, -4, 4, 20, 1, fake, None) == -1


def test_denoise_ex_validation(lib):
    from paper_1306_5390_amd._api import Params, STOP_ON_CYCLE
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    p = Params(10, 10, 20, 1, 3)
    assert STOP_ON_CYCLE == 1
    # unknown flag bits
    for flags in (2, 4, -1, 1 << 30):
        assert lib.phgrms_denoise_ex(fake, fake, p, flags, fake, 1 << 30, None, None,
                                     None) == -1, flags
        assert lib.phgrms_last_error() != b""
    # invalid parameters, a short workspace and overlaps as for phgrms_denoise
    assert lib.phgrms_denoise_ex(fake, fake, Params(10, 10, 256, 1, 3), 1, fake, 1 << 30,
                                 None, None, None) == -1
    assert lib.phgrms_denoise_ex(fake, fake, Params(10, 10, 20, 5, 3), 1, fake, 1 << 30,
                                 None, None, None) == -4
    assert lib.phgrms_denoise_ex(fake, ctypes.c_void_p(0x100000), p, 1,
                                 ctypes.c_void_p(0x200000), 16, None, None, None) == -2
    assert lib.phgrms_denoise_ex(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1005), p, 1,
                                 ctypes.c_void_p(0x200000), 1 << 20, None, None, None) == -1
    assert lib.phgrms_denoise_ex(None, None, p, 1, fake, 1 << 20, None, None, None) == -1


def test_autotune_validation(lib):
    from paper_1306_5390_amd._api import Params
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    best = ctypes.c_int32()
    p = Params(64, 64, 20, 1, 4)
    need = lib.phgrms_autotune_workspace_bytes(p)
    assert need >= 64 * 64 + lib.phgrms_workspace_bytes(p)
    assert lib.phgrms_autotune_workspace_bytes(Params(64, 64, 300, 1, 4)) == 0
    big = ctypes.c_void_p(0x10000000)
    # nothing to time, bad reps, null pointers, short or overlapping workspace
    assert lib.phgrms_autotune(Params(0, 64, 20, 1, 4), fake, big, need, 2, ctypes.byref(best), None, None, None) == -1
    assert lib.phgrms_autotune(Params(64, 64, 20, 1, 0), fake, big, need, 2, ctypes.byref(best), None, None, None) == -1
    assert lib.phgrms_autotune(p, fake, big, need, 0, ctypes.byref(best), None, None, None) == -1
    assert lib.phgrms_autotune(p, None, big, need, 2, ctypes.byref(best), None, None, None) == -1
    assert lib.phgrms_autotune(p, fake, big, need, 2, None, None, None, None) == -1
    assert lib.phgrms_autotune(p, fake, big, need - 1, 2, ctypes.byref(best), None, None, None) == -2
    assert lib.phgrms_autotune(p, ctypes.c_void_p(0x10000010), big, need, 2, ctypes.byref(best),
                               None, None, None) == -1
    assert lib.phgrms_autotune(Params(64, 64, 20, 7, 4), fake, big, need, 2, ctypes.byref(best),
                               None, None, None) == -4


def test_change_maps_and_run_passes_validation(lib):
    from paper_1306_5390_amd._api import Params
    # two maps of one byte per (row, 256-column tile column), padded to 256
    # bytes, then the tile lists: 3 x 16 counts of 16 words, and per tile of
    # at least 16 rows a mark and an entry in each of 3 x 16 list shards
    def expect(rows, cols):
        tx = (cols + 255) // 256
        cap = (rows + 15) // 16 * tx
        return (2 * rows * tx + 255) // 256 * 256 + 4 * (3 * 16 * 16 + cap * (1 + 3 * 16))
    assert lib.phgrms_change_map_bytes(Params(100, 300, 20, 1, 1)) == expect(100, 300) == 6328
    assert lib.phgrms_change_map_bytes(Params(7, 256, 20, 2, 1)) == expect(7, 256)
    assert lib.phgrms_change_map_bytes(Params(7, 257, 20, 2, 1)) == expect(7, 257)
    assert lib.phgrms_change_map_bytes(Params(8192, 8192, 20, 2, 1)) == expect(8192, 8192)
    assert lib.phgrms_change_map_bytes(Params(7, 257, 300, 2, 1)) == 0
    shapes = [(i, lib.phgrms_num_shapes()) for i in range(lib.phgrms_num_shapes())]
    T = []
    for i, _ in shapes:
        t, r, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert lib.phgrms_shape_info(i, ctypes.byref(t), ctypes.byref(r), ctypes.byref(w)) == 0
        T.append(t.value)
    tracked = [i for i in range(len(T)) if lib.phgrms_shape_tracks_changes(i) == 1]
    assert tracked and all(T[i] == 1 for i in tracked)
    assert lib.phgrms_shape_tracks_changes(len(T)) == -1
    one = tracked[0]
    untracked_one = next(i for i, t in enumerate(T) if t == 1 and i not in tracked)
    multi = next(i for i, t in enumerate(T) if t > 1)
    src, dst, cnt = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    maps = ctypes.c_void_p(0x400000)
    p1 = Params(64, 64, 20, 1, 1)
    # maps need a change-tracking shape and k == 1
    assert lib.phgrms_run_passes(src, dst, p1, multi, 0, cnt, maps, None) == -1
    assert lib.phgrms_run_passes(src, dst, p1, untracked_one, 0, cnt, maps, None) == -1
    assert lib.phgrms_run_passes(src, dst, Params(64, 64, 20, 1, 2), multi, 0, cnt, maps,
                                 None) == -1
    # negative pass index
    assert lib.phgrms_run_passes(src, dst, p1, one, -1, cnt, maps, None) == -1
    # maps overlapping an image
    assert lib.phgrms_run_passes(src, dst, p1, one, 1, cnt, ctypes.c_void_p(0x100010),
                                 None) == -1
    # k above the shape's passes per launch, bad shape
    assert lib.phgrms_run_passes(src, dst, Params(64, 64, 20, 1, 2), one, 0, cnt, None,
                                 None) == -1
    assert lib.phgrms_run_passes(src, dst, p1, 99, 0, cnt, None, None) == -1


def test_quality_calls_validate_before_launch(lib):
    fake = ctypes.c_void_p(0x1000)
    assert lib.phgrms_salt_pepper(fake, fake, -1, 0, 0, 0, None) == -1
    assert lib.phgrms_salt_pepper(fake, fake, 10, 0, 5, 4, None) == -1      # t_pepper > t_salt
    assert lib.phgrms_salt_pepper(None, None, 10, 0, 0, 1, None) == -1
    assert lib.phgrms_salt_pepper(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1004), 10, 0, 0, 1,
                                  None) == -1                               # partial overlap
    assert lib.phgrms_salt_pepper(None, None, 0, 0, 0, 0, None) == 0        # nothing to do
    assert lib.phgrms_sq_diff_sum(fake, fake, -1, fake, None) == -1
    assert lib.phgrms_sq_diff_sum(fake, fake, 10, None, None) == -1
    assert lib.phgrms_sq_diff_sum(None, fake, 10, fake, None) == -1


def test_noise_thresholds():
    from paper_1306_5390_amd import synth
    assert synth.noise_thresholds(0.0) == (0, 0)
    assert synth.noise_thresholds(1.0) == ((2 ** 32 - 1) // 2, 2 ** 32 - 1)
    tp, ts = synth.noise_thresholds(0.2)
    assert ts == round(0.2 * 2 ** 32) and tp == ts // 2
    with pytest.raises(ValueError):
        synth.noise_thresholds(1.5)


def test_tuning_calls(lib):
    n = lib.phgrms_num_shapes()
    assert n >= 1
    t, r, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    for s in range(n):
        assert lib.phgrms_shape_info(s, ctypes.byref(t), ctypes.byref(r), ctypes.byref(w)) == 0
        assert t.value >= 1 and r.value >= 1 and w.value >= 1
    assert lib.phgrms_shape_info(n, None, None, None) == -1
    old = lib.phgrms_get_tuning(2)
    assert lib.phgrms_set_tuning(2, n - 1) == 0
    assert lib.phgrms_get_tuning(2) == n - 1
    assert lib.phgrms_set_tuning(2, old) == 0
    assert lib.phgrms_set_tuning(0, 0) == -1
    assert lib.phgrms_set_tuning(2, n) == -1
    # the batch path's own table
    old = [lib.phgrms_get_batch_tuning_class(1, c) for c in range(3)]
    assert all(0 <= x < n for x in old)
    assert lib.phgrms_set_batch_tuning_class(1, -1, 0) == 0
    assert [lib.phgrms_get_batch_tuning_class(1, c) for c in range(3)] == [0, 0, 0]
    assert lib.phgrms_set_batch_tuning_class(1, 1, n - 1) == 0
    assert lib.phgrms_get_batch_tuning_class(1, 1) == n - 1
    for c, x in enumerate(old):
        assert lib.phgrms_set_batch_tuning_class(1, c, x) == 0
    assert lib.phgrms_set_batch_tuning_class(1, 3, 0) == -1
    assert lib.phgrms_set_batch_tuning_class(1, 0, n) == -1
    assert lib.phgrms_get_batch_tuning_class(0, 0) == -1
    assert lib.phgrms_get_batch_tuning_class(1, 3) == -1


def test_batch_plan_validation(lib):
    from paper_1306_5390_amd._api import Item, Params
    plan = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    items = (Item * 3)(Item(0, 0, Params(10, 10, 20, 1, 3)), Item(256, 256, Params(5, 7, 0, 2, 1)),
                       Item(512, 512, Params(0, 0, 20, 1, 0)))
    assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 3, None, ctypes.byref(plan),
                                 ctypes.byref(ws)) == 0
    assert ws.value > 0 and plan.value
    assert lib.phgrms_batch_launches(plan) >= 3
    fake_in, fake_out = 0x10000000, 0x20000000
    wsp = 0x40000000
    # arenas too small
    assert lib.phgrms_batch_run(plan, fake_in, 100, fake_out, 1 << 20, wsp, ws.value,
                                None, None, None) == -1
    # workspace too small
    assert lib.phgrms_batch_run(plan, fake_in, 1 << 20, fake_out, 1 << 20, wsp, 16,
                                None, None, None) == -2
    # output overlapping another item's input (same arena, shifted offsets)
    lib.phgrms_plan_destroy(plan)
    items = (Item * 2)(Item(0, 50, Params(10, 10, 20, 1, 3)), Item(100, 150, Params(10, 10, 20, 1, 3)))
    assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 2, None, ctypes.byref(plan),
                                 ctypes.byref(ws)) == 0
    assert lib.phgrms_batch_run(plan, fake_in, 1 << 20, fake_in, 1 << 20, wsp, ws.value,
                                None, None, None) == -1
    # overlapping outputs
    lib.phgrms_plan_destroy(plan)
    items = (Item * 2)(Item(0, 0, Params(10, 10, 20, 1, 3)), Item(100, 50, Params(10, 10, 20, 1, 3)))
    assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 2, None, ctypes.byref(plan),
                                 ctypes.byref(ws)) == 0
    assert lib.phgrms_batch_run(plan, fake_in, 1 << 20, fake_out, 1 << 20, wsp, ws.value,
                                None, None, None) == -1
    lib.phgrms_plan_destroy(plan)
    # invalid item parameters
    items = (Item * 2)(Item(0, 0, Params(10, 10, 20, 1, 3)), Item(0, 0, Params(10, 10, 300, 1, 3)))
    assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 2, None, ctypes.byref(plan),
                                 ctypes.byref(ws)) == -1
    items = (Item * 1)(Item(0, 0, Params(10, 10, 20, 7, 3)))
    assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 1, None, ctypes.byref(plan),
                                 ctypes.byref(ws)) == -4
    assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 0, None, ctypes.byref(plan),
                                 ctypes.byref(ws)) == -1
    lib.phgrms_plan_destroy(None)


def test_server_config_validation(lib):
    from paper_1306_5390_amd._api import ServerCfg
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x10000000)
    for cfg in [ServerCfg(0, 0, 0, 16, 0), ServerCfg(0, 8, -2, 16, 0), ServerCfg(0, 8, 0, 0, 0)]:
        assert lib.phgrms_server_create(ctypes.byref(cfg), fake, 1 << 30, ctypes.byref(h)) == -1
    assert lib.phgrms_server_create(ctypes.byref(ServerCfg(0, 8, 0, 16, 0)), None, 1 << 30,
                                    ctypes.byref(h)) == -1
    # an arena too small for the descriptor slots
    assert lib.phgrms_server_create(ctypes.byref(ServerCfg(0, 8, 0, 16, 0)), fake, 1 << 16,
                                    ctypes.byref(h)) == -2
    lib.phgrms_server_destroy(None)
    assert lib.phgrms_server_poll(None, 1, None, None, None, None) == -1
    from paper_1306_5390_amd._api import Params
    rid = ctypes.c_uint64()
    assert lib.phgrms_server_submit_host(None, fake, ctypes.c_void_p(0x20000000),
                                         Params(8, 8, 20, 1, 2), ctypes.byref(rid)) == -1
    assert lib.phgrms_server_submit_host(None, None, None, Params(8, 8, 20, 1, 2),
                                         ctypes.byref(rid)) == -1


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it exits with a
    message, before touching a GPU."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_tuning_cache_load(lib, tmp_path):
    """The tuning cache applies the per-class choices and the batch path's
    table; entries that are not betas (notes) are skipped."""
    import json
    from paper_1306_5390_amd import _api, autotune
    saved = {b: ([_api.get_tuning_class(b, c) for c in range(3)],
                 [_api.get_batch_tuning_class(b, c) for c in range(3)]) for b in (1, 2)}
    try:
        p = tmp_path / "tuning.json"
        p.write_text(json.dumps({
            "choice": {"1": {"0": {"shape": 2}, "1": {"shape": 9}}, "2": {"2": {"shape": 4}}},
            "batch_choice": {"1": {"shape": 5}, "2": {"shape": 0}, "note": "not a beta"}}))
        assert autotune.load(str(p))
        assert _api.get_tuning_class(1, 0) == 2 and _api.get_tuning_class(1, 1) == 9
        assert _api.get_tuning_class(2, 2) == 4
        assert [_api.get_batch_tuning_class(1, c) for c in range(3)] == [5, 5, 5]
        assert [_api.get_batch_tuning_class(2, c) for c in range(3)] == [0, 0, 0]
        assert not autotune.load(str(tmp_path / "missing.json"))
    finally:
        for b, (fused, batch) in saved.items():
            for c in range(3):
                _api.set_tuning_class(b, c, fused[c])
                _api.set_batch_tuning_class(b, c, batch[c])


# ---- tuning cache through the C ABI -----------------------------------------

def _tables(lib):
    fused = {(b, c): lib.phgrms_get_tuning_class(b, c) for b in (1, 2, 3, 4) for c in (0, 1, 2)}
    batch = {(b, c): lib.phgrms_get_batch_tuning_class(b, c) for b in (1, 2, 3, 4)
             for c in (0, 1, 2)}
    return fused, batch


def _restore(lib, saved):
    fused, batch = saved
    for (b, c), s in fused.items():
        assert lib.phgrms_set_tuning_class(b, c, s) == 0
    for (b, c), s in batch.items():
        assert lib.phgrms_set_batch_tuning_class(b, c, s) == 0


def test_tuning_cache_round_trip(lib, tmp_path):
    import json
    saved = _tables(lib)
    try:
        path = str(tmp_path / "tune.json").encode()
        assert lib.phgrms_set_tuning_class(2, 1, 5) == 0
        assert lib.phgrms_set_batch_tuning_class(1, 2, 6) == 0
        assert lib.phgrms_save_tuning(path) == 0
        data = json.load(open(path))
        assert data["format"] == "phgrms-tuning-1"
        assert len(data["shapes"]) == lib.phgrms_num_shapes()
        assert data["choice"]["2"]["1"]["shape"] == 5
        assert data["batch_choice"]["1"]["classes"]["2"] == 6
        # other values, then the file brings the saved ones back
        assert lib.phgrms_set_tuning_class(2, 1, 0) == 0
        assert lib.phgrms_set_batch_tuning_class(1, 2, 0) == 0
        assert lib.phgrms_load_tuning(path) == 0
        assert lib.phgrms_get_tuning_class(2, 1) == 5
        assert lib.phgrms_get_batch_tuning_class(1, 2) == 6
        assert _tables(lib) == _tables(lib)
    finally:
        _restore(lib, saved)


def test_tuning_cache_committed_file(lib):
    """The committed cache (written by the Python autotuner, with its rates
    and notes) reads through the C reader into exactly its choices."""
    import json
    from paper_1306_5390_amd import autotune
    saved = _tables(lib)
    try:
        data = json.load(open(autotune.DEFAULT_CACHE))
        assert lib.phgrms_load_tuning(autotune.DEFAULT_CACHE.encode()) == 0
        for beta, per in data["choice"].items():
            for cls, c in per.items():
                assert lib.phgrms_get_tuning_class(int(beta), int(cls)) == c["shape"]
        for beta, c in data.get("batch_choice", {}).items():
            if beta.isdigit():
                want = c.get("classes", {}) or {str(k): c["shape"] for k in range(3)}
                for cls, s in want.items():
                    assert lib.phgrms_get_batch_tuning_class(int(beta), int(cls)) == s
    finally:
        _restore(lib, saved)


def test_tuning_cache_errors_change_nothing(lib, tmp_path):
    import json
    saved = _tables(lib)
    try:
        missing = str(tmp_path / "none.json").encode()
        assert lib.phgrms_load_tuning(missing) == -6
        n = lib.phgrms_num_shapes()
        bad = {
            "syntax": '{"choice": {"1": {"0": {"shape": 3}}',
            "not_object": "[1, 2]",
            "shape_range": json.dumps({"choice": {"1": {"0": {"shape": n}}}}),
            "shape_fraction": json.dumps({"choice": {"1": {"0": {"shape": 1.5}}}}),
            "beta_range": json.dumps({"choice": {"9": {"0": {"shape": 1}}}}),
            "class_range": json.dumps({"choice": {"1": {"3": {"shape": 1}}}}),
            "batch_shape": json.dumps({"batch_choice": {"2": {"shape": -1}}}),
            "other_shapes": json.dumps({"shapes": [[9, 9, 9]], "choice": {}}),
        }
        for name, text in bad.items():
            p = tmp_path / (name + ".json")
            p.write_text(text)
            # a partly valid file changes nothing either
            before = _tables(lib)
            assert lib.phgrms_load_tuning(str(p).encode()) == -1, name
            assert _tables(lib) == before, name
            assert lib.phgrms_last_error()
            # and is never overwritten
            assert lib.phgrms_save_tuning(str(p).encode()) == -1, name
            assert p.read_text() == text
        assert lib.phgrms_load_tuning(None) == -1
    finally:
        _restore(lib, saved)


def test_tuning_cache_rewrite_keeps_other_keys(lib, tmp_path):
    import json
    saved = _tables(lib)
    try:
        p = tmp_path / "rich.json"
        p.write_text(json.dumps({
            "device": "x", "note": "kept é\\n",
            "choice": {"1": {"2": {"shape": 4, "rates": [1.5, 2.0]}}},
            "batch_choice": {"note": "also kept", "2": {"shape": 5, "rates": [3]}}}))
        assert lib.phgrms_load_tuning(str(p).encode()) == 0
        assert lib.phgrms_get_tuning_class(1, 2) == 4
        assert all(lib.phgrms_get_batch_tuning_class(2, c) == 5 for c in range(3))
        assert lib.phgrms_set_tuning_class(1, 2, 7) == 0
        assert lib.phgrms_save_tuning(str(p).encode()) == 0
        d = json.loads(p.read_text())
        assert d["device"] == "x" and d["note"] == "kept é\\n"
        assert d["choice"]["1"]["2"] == {"shape": 7, "rates": [1.5, 2.0]}
        assert d["batch_choice"]["note"] == "also kept"
        assert d["batch_choice"]["2"]["rates"] == [3]
        assert d["batch_choice"]["2"]["classes"] == {"0": 5, "1": 5, "2": 5}
        assert "shape" not in d["batch_choice"]["2"]
    finally:
        _restore(lib, saved)


def test_batch_plan_takes_the_cache_shapes(lib, tmp_path):
    """A plan made with a cache path uses that cache's batch shapes (here 4
    passes per launch: 2 launches for k = 8) without changing the process's
    table (1 pass per launch: 8 launches)."""
    import json
    from paper_1306_5390_amd._api import Item, Params
    saved = _tables(lib)
    try:
        T = [ctypes.c_int32() for _ in range(3)]
        four = next(s for s in range(lib.phgrms_num_shapes())
                    if lib.phgrms_shape_info(s, ctypes.byref(T[0]), ctypes.byref(T[1]),
                                             ctypes.byref(T[2])) == 0 and T[0].value == 4)
        assert lib.phgrms_set_batch_tuning_class(1, -1, 3) == 0
        p = tmp_path / "batch.json"
        p.write_text(json.dumps({"batch_choice": {"1": {"shape": four}}}))
        items = (Item * 1)(Item(0, 0, Params(300, 300, 20, 1, 8)))
        plan, ws = ctypes.c_void_p(), ctypes.c_size_t()
        assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 1, None,
                                     ctypes.byref(plan), ctypes.byref(ws)) == 0
        plain_launches = lib.phgrms_batch_launches(plan)
        lib.phgrms_plan_destroy(plan)
        assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 1, str(p).encode(),
                                     ctypes.byref(plan), ctypes.byref(ws)) == 0
        cached_launches = lib.phgrms_batch_launches(plan)
        lib.phgrms_plan_destroy(plan)
        assert cached_launches == plain_launches - 6
        assert lib.phgrms_get_batch_tuning_class(1, 0) == 3
        assert lib.phgrms_batch_plan(ctypes.cast(items, ctypes.c_void_p), 1,
                                     str(tmp_path / "missing.json").encode(),
                                     ctypes.byref(plan), ctypes.byref(ws)) == -6
    finally:
        _restore(lib, saved)


def test_calibration_arguments_rejected_before_any_launch(lib):
    """The roofline calibration entry points validate on the host: no GPU
    call happens for any of these (the pointers are never dereferenced)."""
    vp = ctypes.c_void_p
    a, b = vp(0x100000), vp(0x200000)
    assert lib.phgrms_calib_copy(a, b, 0, None) == 0                    # nothing to do
    assert lib.phgrms_calib_copy(None, b, 64, None) == -1               # null source
    assert lib.phgrms_calib_copy(a, None, 64, None) == -1               # null destination
    assert lib.phgrms_calib_copy(a, b, 40, None) == -1                  # size not a multiple of 16
    assert lib.phgrms_calib_copy(vp(0x100008), b, 64, None) == -1       # misaligned source
    assert lib.phgrms_calib_copy(a, vp(0x100010), 64, None) == -1       # overlapping regions
    assert lib.phgrms_calib_copy(vp(0x100010), a, 64, None) == -1
    per_wave = ctypes.c_uint64(123)
    assert lib.phgrms_calib_valu(None, 1, 1, 0, ctypes.byref(per_wave), None) == -1
    for blocks, trips, kind in [(0, 1, 0), (1 << 21, 1, 0), (1, 0, 0), (1, 1 << 25, 0),
                                (1, 1, 9), (1, 1, -1)]:
        assert lib.phgrms_calib_valu(a, blocks, trips, kind, ctypes.byref(per_wave), None) == -1
        assert lib.phgrms_last_error() != b""
    assert per_wave.value == 123                                        # untouched on error
