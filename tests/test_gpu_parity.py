"""GPU parity: the HIP path against the CPU oracle, bit for bit (image,
iteration count and per-pass changed counts), through the C ABI.

Cases span several 256-column tiles with ragged tails, every compiled kernel
shape (1, 2 and 4 passes per launch), every beta the kernels are built for,
alpha at the band edges (0, 1, 255), byte-misaligned and in-place buffers,
and the degenerate images (empty, one row, one column, smaller than a window).
"""
import numpy as np
import pytest
import torch

import oracle
import pins
import golden_io
from paper_1306_5390_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def phg():
    import paper_1306_5390_amd as m
    m.load_library()
    return m


def say(*a):
    print(*a, flush=True)


def _num_shapes():
    try:
        from paper_1306_5390_amd import _api
        return int(_api.load_library().phgrms_num_shapes())
    except Exception:
        return 7


NUM_SHAPES = _num_shapes()
MODES = ["plain"] + list(range(NUM_SHAPES))


def run_gpu(img: np.ndarray, alpha, beta, k, mode):
    m = phg()
    t = torch.from_numpy(np.ascontiguousarray(img)).to(DEV)
    if mode == "plain":
        out, it, ch = m.denoise(t, alpha, beta, k, plain=True)
    else:
        old = m.get_tuning(beta)
        m.set_tuning(beta, mode)
        try:
            out, it, ch = m.denoise(t, alpha, beta, k)
        finally:
            m.set_tuning(beta, old)
    return out.cpu().numpy(), it, ch


def assert_same(img, alpha, beta, k, mode, tag=""):
    say("case", tag, img.shape, "alpha", alpha, "beta", beta, "k", k, "mode", mode)
    ref, rit, rch = oracle.denoise(img, alpha, beta, k)
    got, it, ch = run_gpu(img, alpha, beta, k, mode)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError("%s: %d pixels differ, first %s (gpu %d, oracle %d)" % (
            tag, len(bad), bad[0].tolist(), got[tuple(bad[0])], ref[tuple(bad[0])]))
    assert it == rit, (tag, it, rit)
    assert ch == rch, (tag, ch, rch)


@pytest.mark.parametrize("mode", MODES)
def test_goldens(mode):
    for path in golden_io.golden_files():
        g = golden_io.load(path)
        got, it, ch = run_gpu(g["input"], g["alpha"], g["beta"], g["k"], mode)
        assert np.array_equal(got, g["output"]), (g["name"], mode)
        assert it == g["iterations"] and ch == g["changed"], (g["name"], mode, it, ch)


@pytest.mark.parametrize("beta", [1, 2, 3, 4])
@pytest.mark.parametrize("mode", MODES)
def test_random_tiles(beta, mode):
    rng = np.random.Generator(np.random.PCG64(100 + beta))
    for (h, w) in [(70, 600), (37, 257), (131, 130)]:
        for alpha in (1, 20, 40):
            img = pins.boundary_image(rng, h, w, alpha)
            assert_same(img, alpha, beta, 5, mode, "boundary")
    img = synth.noisy_image(90, 520, 0.3, 21 + beta)
    for alpha in (10, 20):
        assert_same(img, alpha, beta, 9, mode, "synth")


@pytest.mark.parametrize("mode", MODES)
def test_alpha_extremes(mode):
    rng = np.random.Generator(np.random.PCG64(7))
    img = rng.integers(0, 256, size=(45, 300)).astype(np.uint8)
    for beta in (1, 2):
        assert_same(img, 0, beta, 3, mode, "alpha0")
        assert_same(img, 255, beta, 3, mode, "alpha255")
        assert_same(img, 1, beta, 4, mode, "alpha1")


@pytest.mark.parametrize("mode", MODES)
def test_degenerate_shapes(mode):
    rng = np.random.Generator(np.random.PCG64(8))
    for (h, w) in [(0, 0), (0, 5), (5, 0), (1, 1), (1, 700), (700, 1), (2, 2), (3, 300),
                   (300, 3), (4, 4), (5, 5), (6, 259)]:
        img = pins.boundary_image(rng, h, w, 20) if h * w else np.zeros((h, w), np.uint8)
        assert_same(img, 20, 1, 4, mode, "degenerate")
        assert_same(img, 20, 2, 4, mode, "degenerate")


@pytest.mark.parametrize("mode", MODES)
def test_k_values(mode):
    img = synth.noisy_image(60, 290, 0.25, 31)
    for k in (0, 1, 2, 3, 4, 5, 7, 8, 9):
        assert_same(img, 20, 1, k, mode, "k")
    # period-2 oscillation: iterations == k
    g = golden_io.load(golden_io.GOLDEN_DIR + "/p_period2_k5.txt")
    for k in (1, 16, 33, 1024):
        assert_same(g["input"], 20, 1, k, mode, "oscillation")


@pytest.mark.parametrize("cols", [299, 300])
def test_unaligned_and_in_place(cols):
    """Byte offsets 0-4 of input and output: 300 columns with offsets 0 and 4
    take the aligned dword path, everything else the re-aligning path."""
    m = phg()
    saved = {b: m.get_tuning(b) for b in (1, 2)}
    img = synth.noisy_image(53, cols, 0.3, 41)
    ref, rit, rch = oracle.denoise(img, 20, 1, 6)
    n = img.size
    try:
        for off_in in range(5):
            for off_out in range(5):
                say("offsets", off_in, off_out, "cols", cols)
                big_in = torch.zeros(n + 64, dtype=torch.uint8, device=DEV)
                big_out = torch.zeros(n + 64, dtype=torch.uint8, device=DEV)
                tin = big_in[off_in:off_in + n].view(53, cols)
                tin.copy_(torch.from_numpy(img).to(DEV))
                tout = big_out[off_out:off_out + n].view(53, cols)
                for mode in ["plain"] + list(range(NUM_SHAPES)):
                    if mode == "plain":
                        out, it, ch = m.denoise(tin, 20, 1, 6, out=tout, plain=True)
                    else:
                        m.set_tuning(1, mode)
                        out, it, ch = m.denoise(tin, 20, 1, 6, out=tout)
                    assert np.array_equal(out.cpu().numpy(), ref), (off_in, off_out, mode)
                    assert (it, ch) == (rit, rch)
                    # bytes around the output are untouched
                    assert int(big_out[:off_out].sum()) == 0
                    assert int(big_out[off_out + n:].sum()) == 0
        # in place, both parities of the launch count
        for k in (5, 6):
            ref, rit, rch = oracle.denoise(img, 20, 2, k)
            for mode in ["plain"] + list(range(NUM_SHAPES)):
                t = torch.from_numpy(img).to(DEV)
                if mode == "plain":
                    out, it, ch = m.denoise(t, 20, 2, k, out=t, plain=True)
                else:
                    m.set_tuning(2, mode)
                    out, it, ch = m.denoise(t, 20, 2, k, out=t)
                assert out.data_ptr() == t.data_ptr()
                assert np.array_equal(t.cpu().numpy(), ref), (k, mode)
                assert (it, ch) == (rit, rch)
    finally:
        for b, v in saved.items():
            m.set_tuning(b, v)


def test_async_results_on_device():
    m = phg()
    img = synth.noisy_image(100, 333, 0.2, 51)
    ref, rit, rch = oracle.denoise(img, 20, 1, 7)
    t = torch.from_numpy(img).to(DEV)
    out, d_changed, d_it = m.denoise_async(t, 20, 1, 7)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert int(d_it.item()) == rit
    assert d_changed.cpu().tolist()[:rit] == rch
    assert all(v == 0 for v in d_changed.cpu().tolist()[rit:])


@pytest.mark.parametrize("beta", [1, 2, 3, 4])
def test_cardinality_matches_algorithm1(beta):
    m = phg()
    rng = np.random.Generator(np.random.PCG64(60 + beta))
    for (h, w, alpha) in [(33, 301, 20), (7, 9, 0), (64, 64, 255), (1, 50, 10)]:
        img = pins.boundary_image(rng, h, w, max(alpha, 1))
        ref = oracle.cardinality(img, alpha, beta, scatter=True).astype(np.int64)
        got = m.cardinality(torch.from_numpy(img).to(DEV), alpha, beta).cpu().numpy()
        assert np.array_equal(got, ref), (h, w, alpha, beta)


def test_single_481x321_config():
    spec = synth.single_481x321()
    img = spec.image()
    for mode in MODES:
        assert_same(img, spec.alpha, spec.beta, spec.k, mode, "481x321")


def test_integer_routines_exhaustive():
    """The fast floor(S/F) and floor(sqrt(q)) of the candidate evaluation are
    exact over their whole domains."""
    m = phg()
    assert m.selftest(DEV) == (0, 0)


def streak_image(rng, h, w, beta, n_streaks=12):
    """Smooth background (level 100, small texture) with dotted streaks of
    level ~200, dots every `beta` pixels along a row or a column.  A streak's
    end dot has a single in-band dot in its window and is replaced; the next
    dot becomes an end: each streak erodes one dot per pass from both ends,
    so changes move across tile boundaries pass after pass."""
    img = np.clip(100 + rng.normal(0, 2, size=(h, w)), 0, 255).round().astype(np.uint8)
    for _ in range(n_streaks):
        if rng.random() < 0.5:
            r = int(rng.integers(beta, h - beta))
            c0 = int(rng.integers(beta, w // 2))
            c1 = int(rng.integers(min(c0 + 10 * beta, w - beta - 1), w - beta))
            img[r, c0:c1:beta] = 200 + rng.integers(-3, 4, size=len(range(c0, c1, beta)))
        else:
            c = int(rng.integers(beta, w - beta))
            r0 = int(rng.integers(beta, h // 2))
            r1 = int(rng.integers(min(r0 + 10 * beta, h - beta - 1), h - beta))
            img[r0:r1:beta, c] = 200 + rng.integers(-3, 4, size=len(range(r0, r1, beta)))
    return img


@pytest.mark.parametrize("beta", [1, 2, 3, 4])
@pytest.mark.parametrize("mode", MODES)
def test_eroding_streaks_across_tiles(beta, mode):
    # few changes per pass, moving across tile rows and tile columns: rows
    # whose neighbourhood did not change are copied through untested, and a
    # missed dependency would show here
    rng = np.random.Generator(np.random.PCG64(500 + beta))
    for (h, w) in [(100, 600), (70, 520)]:
        img = streak_image(rng, h, w, beta)
        assert_same(img, 20, beta, 48, mode, "streaks")


@pytest.mark.parametrize("beta", [1, 2])
def test_skipping_shapes_ignore_stale_buffers(beta):
    """The skipping shapes leave unchanged tiles and rows untouched from the
    third pass on, so the first two passes must write both ping-pong buffers
    whole: an output and a workspace that hold another image's run, or
    random bytes, give the oracle's results (k = 1..4 and 33, both launch
    parities, in place too)."""
    m = phg()
    skips = [s for s in range(NUM_SHAPES) if m.shape_skips_unchanged(s)]
    assert skips
    rng = np.random.Generator(np.random.PCG64(650 + beta))
    img = streak_image(rng, 150, 900, beta, n_streaks=20)
    other = torch.from_numpy(synth.noisy_image(150, 900, 0.4, 77)).to(DEV)
    t = torch.from_numpy(img).to(DEV)
    saved = m.get_tuning(beta)
    try:
        for s in skips:
            m.set_tuning(beta, s)
            for k in (1, 2, 3, 4, 33):
                ref, rit, rch = oracle.denoise(img, 20, beta, k)
                ws = torch.empty(m.workspace_bytes(150, 900, 20, beta, k), dtype=torch.uint8,
                                 device=DEV)
                out = torch.empty_like(t)
                for stale in ("other", "random"):
                    say("skip shape", s, "beta", beta, "k", k, stale)
                    if stale == "other":
                        m.denoise(other, 20, beta, k, out=out, workspace=ws)
                    else:
                        ws.random_(0, 256)
                        out.random_(0, 256)
                    got, it, ch = m.denoise(t, 20, beta, k, out=out, workspace=ws)
                    assert np.array_equal(got.cpu().numpy(), ref), (s, k, stale)
                    assert (it, ch) == (rit, rch), (s, k, stale)
                # in place, over a workspace holding another run
                m.denoise(other, 20, beta, k, out=torch.empty_like(t), workspace=ws)
                tt = t.clone()
                got, it, ch = m.denoise(tt, 20, beta, k, out=tt, workspace=ws)
                assert np.array_equal(tt.cpu().numpy(), ref), (s, k, "in place")
                assert (it, ch) == (rit, rch)
    finally:
        m.set_tuning(beta, saved)


@pytest.mark.parametrize("beta", [1, 2, 3])
def test_run_passes_with_change_maps(beta):
    # a run_passes sequence with change maps equals the oracle pass by pass
    m = phg()
    shapes = m.shapes()
    rng = np.random.Generator(np.random.PCG64(600 + beta))
    img = streak_image(rng, 90, 700, beta)
    ref = img
    for si, (T, R, W) in enumerate(shapes):
        if not m.shape_tracks_changes(si):
            continue
        say("run_passes maps shape", si, "beta", beta)
        cur = torch.from_numpy(img).to(DEV)
        bufs = (torch.empty_like(cur), torch.empty_like(cur))
        maps = m.change_maps(*img.shape, DEV)
        ref = img
        for t in range(20):
            slots = m.count_slots(1, DEV)
            dst = bufs[t % 2]
            m.run_passes(cur, dst, 20, beta, 1, si, slots, pass_index=t, maps=maps)
            ref, rch = oracle.one_pass(ref, 20, beta)
            assert m.pass_counts(slots)[0] == rch, (si, t)
            assert np.array_equal(dst.cpu().numpy(), ref), (si, t)
            cur = dst


@pytest.mark.parametrize("beta", [1, 2, 3, 4])
def test_cardinality_scatter_form(beta):
    # the printed scatter form (atomic increments) equals the gather form
    # on the GPU and the oracle's scatter form
    m = phg()
    rng = np.random.Generator(np.random.PCG64(700 + beta))
    for (h, w) in [(1, 1), (5, 700), (37, 257), (70, 600), (131, 130)]:
        for alpha in (0, 1, 20, 255):
            img = pins.boundary_image(rng, h, w, max(alpha, 1)) if h * w > 1 else \
                rng.integers(0, 256, size=(h, w)).astype(np.uint8)
            say("scatter card", (h, w), alpha, beta)
            t = torch.from_numpy(img).to(DEV)
            sc = m.cardinality_scatter(t, alpha, beta).cpu().numpy()
            ga = m.cardinality(t, alpha, beta).cpu().numpy()
            ref = oracle.cardinality(img, alpha, beta, scatter=True).astype(np.int32)
            assert np.array_equal(sc, ref), ((h, w), alpha, beta)
            assert np.array_equal(ga, ref), ((h, w), alpha, beta)


def test_native_autotune_picks_a_shape_and_keeps_results():
    """phgrms_autotune times every shape on one image, uses the fastest for
    the image's size class, and the pass loop's results stay the oracle's."""
    m = phg()
    img = synth.noisy_image(300, 520, 0.3, 51)
    t = torch.from_numpy(img).to(DEV)
    cls = m.size_class(img.size)
    saved = m.get_tuning_class(2, cls)
    try:
        best, us = m.autotune_native(t, 20, 2, 6, reps=2)
        say("autotune", best, ["%.1f" % x for x in us])
        assert 0 <= best < NUM_SHAPES and len(us) == NUM_SHAPES
        assert all(x > 0 for x in us) and us[best] == min(us)
        assert m.get_tuning_class(2, cls) == best
        ref, rit, rch = oracle.denoise(img, 20, 2, 6)
        out, it, ch = m.denoise(t, 20, 2, 6)
        assert np.array_equal(out.cpu().numpy(), ref) and (it, ch) == (rit, rch)
    finally:
        m.set_tuning_class(2, cls, saved)
