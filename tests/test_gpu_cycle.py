"""GPU parity of the opt-in period-2 stop (phgrms_denoise_ex with
PHGRMS_STOP_ON_CYCLE) against the oracle's stop rule, bit for bit: image,
iteration count and per-pass changed counts.

Cases: the worked period-2 example (stops after pass 2 with the input
restored), tilted-plane images with salt and pepper that end in a cycle, a
fixed point or the k cap, inputs spanning several 256-column tiles with
ragged tails, byte-misaligned and in-place buffers (both launch parities),
the 481 x 321 workload, and every compiled kernel shape chosen as the tuned
shape (shapes with several passes per launch fall back to a one-pass shape).
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


SHAPES = list(range(_num_shapes()))


def run_cycle(img, alpha, beta, k, shape, out=None, tin=None):
    m = phg()
    old = m.get_tuning(beta)
    m.set_tuning(beta, shape)
    try:
        t = tin if tin is not None else torch.from_numpy(np.ascontiguousarray(img)).to(DEV)
        res, it, ch = m.denoise(t, alpha, beta, k, out=out, stop_on_cycle=True)
    finally:
        m.set_tuning(beta, old)
    return res, it, ch


def assert_cycle_same(img, alpha, beta, k, shape, tag=""):
    say("case", tag, img.shape, "alpha", alpha, "beta", beta, "k", k, "shape", shape)
    ref, rit, rch = oracle.denoise_cycle(img, alpha, beta, k)
    got, it, ch = run_cycle(img, alpha, beta, k, shape)
    got = got.cpu().numpy()
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        raise AssertionError("%s: %d pixels differ, first %s (gpu %d, oracle %d)" % (
            tag, len(bad), bad[0].tolist(), got[tuple(bad[0])], ref[tuple(bad[0])]))
    assert it == rit, (tag, it, rit)
    assert ch == rch, (tag, ch, rch)
    return rit, rch


@pytest.mark.parametrize("shape", SHAPES)
def test_cycle_worked_example_and_goldens(shape):
    g = golden_io.load(golden_io.GOLDEN_DIR + "/p_period2_k5.txt")
    for k in (1, 2, 5, 1024):
        rit, rch = assert_cycle_same(g["input"], 20, 1, k, shape, "period2")
        assert rit == min(k, 2)
    for path in golden_io.golden_files():
        g = golden_io.load(path)
        assert_cycle_same(g["input"], g["alpha"], g["beta"], g["k"], shape, g["name"])


@pytest.mark.parametrize("beta", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", SHAPES)
def test_cycle_random_tiles(beta, shape):
    rng = np.random.Generator(np.random.PCG64(300 + beta))
    kinds = set()
    for (h, w) in [(70, 600), (37, 257), (131, 130), (9, 11)]:
        for alpha in (10, 20):
            img = pins.noisy_ramp(rng, h, w, 0.2)
            for k in (3, 40):
                rit, rch = assert_cycle_same(img, alpha, beta, k, shape, "ramp")
                kinds.add("zero" if rch and rch[-1] == 0 else ("cap" if rit == k else "cycle"))
    img = synth.noisy_image(90, 520, 0.3, 21 + beta)
    assert_cycle_same(img, 20, beta, 30, shape, "synth")
    if beta <= 2:
        assert "cycle" in kinds, kinds


@pytest.mark.parametrize("cols", [299, 300])
def test_cycle_unaligned_and_in_place(cols):
    m = phg()
    rng = np.random.Generator(np.random.PCG64(77))
    img = pins.noisy_ramp(rng, 53, cols, 0.2)
    for alpha in (10, 20):
        ref, rit, rch = oracle.denoise_cycle(img, alpha, 1, 40)
        say("unaligned", cols, "alpha", alpha, "oracle iterations", rit)
        n = img.size
        for off_in in range(5):
            for off_out in range(5):
                big_in = torch.zeros(n + 64, dtype=torch.uint8, device=DEV)
                big_out = torch.zeros(n + 64, dtype=torch.uint8, device=DEV)
                tin = big_in[off_in:off_in + n].view(53, cols)
                tin.copy_(torch.from_numpy(img).to(DEV))
                tout = big_out[off_out:off_out + n].view(53, cols)
                for shape in (3, 7, 9):
                    out, it, ch = run_cycle(img, alpha, 1, 40, shape, out=tout, tin=tin)
                    assert np.array_equal(out.cpu().numpy(), ref), (off_in, off_out, shape)
                    assert (it, ch) == (rit, rch)
                    assert int(big_out[:off_out].sum()) == 0
                    assert int(big_out[off_out + n:].sum()) == 0
    # in place: the stop after an odd and after an even number of passes,
    # and k of both parities (which buffer launch 0 writes)
    g = golden_io.load(golden_io.GOLDEN_DIR + "/p_period2_k5.txt")
    cases = [(img, 10, k) for k in (39, 40)] + [(g["input"], 20, k) for k in (1, 5, 6)]
    for (im, alpha, k) in cases:
        ref, rit, rch = oracle.denoise_cycle(im, alpha, 1, k)
        for shape in SHAPES:
            t = torch.from_numpy(np.ascontiguousarray(im)).to(DEV)
            out, it, ch = run_cycle(im, alpha, 1, k, shape, out=t, tin=t)
            assert out.data_ptr() == t.data_ptr()
            assert np.array_equal(t.cpu().numpy(), ref), (k, shape)
            assert (it, ch) == (rit, rch)


def test_cycle_481x321_workload():
    spec = synth.single_481x321()
    img = spec.image()
    ref, rit, rch = oracle.denoise_cycle(img, spec.alpha, spec.beta, spec.k)
    _, pit, _ = oracle.denoise(img, spec.alpha, spec.beta, spec.k)
    say("481x321: cycle stop after", rit, "of", pit, "passes")
    assert rit < pit
    for shape in SHAPES:
        assert_cycle_same(img, spec.alpha, spec.beta, spec.k, shape, "481x321")


def test_cycle_off_is_the_plain_rule():
    """Without the flag the same entry point keeps the paper's stop rule."""
    m = phg()
    spec = synth.single_481x321()
    img = spec.image()
    ref, rit, rch = oracle.denoise(img, spec.alpha, spec.beta, spec.k)
    t = torch.from_numpy(img).to(DEV)
    out, ch, it = m.denoise_async(t, spec.alpha, spec.beta, spec.k, stop_on_cycle=False)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert int(it.item()) == rit
    assert ch[:rit].cpu().tolist() == rch


def test_cycle_full_size_sweep_image():
    """The 2048^2 benchmark image (30 % noise) with the tuning cache the
    benchmark applies: beta = 2 runs stop on a period-2 cycle well before
    k = 32; the image, the count and every per-pass count equal the
    oracle's (computed here, a few seconds on one core)."""
    from paper_1306_5390_amd import autotune
    m = phg()
    saved = {b: [m.get_tuning_class(b, c) for c in range(3)] for b in (1, 2)}
    try:
        autotune.load()
        spec = synth.sweep_2048()[0]
        img = spec.image()
        t = torch.from_numpy(img).to(DEV)
        for alpha in (20,):
            ref, rit, rch = oracle.denoise_cycle(img, alpha, 2, 32)
            say("2048^2 beta 2 alpha", alpha, "oracle stops after", rit)
            assert rit < 32
            out, it, ch = m.denoise(t, alpha, 2, 32, stop_on_cycle=True)
            assert np.array_equal(out.cpu().numpy(), ref)
            assert (it, ch) == (rit, rch)
    finally:
        for b, v in saved.items():
            for c, s in enumerate(v):
                m.set_tuning_class(b, c, s)


def test_denoise_ex_without_flags_is_denoise_async():
    """phgrms_denoise_ex with flags = 0 keeps the paper's stop rule and the
    tuned shape: the same image, count and per-pass counts as the oracle."""
    import ctypes
    from paper_1306_5390_amd import _api
    m = phg()
    lib = m.load_library()
    spec = synth.single_481x321()
    img = spec.image()
    ref, rit, rch = oracle.denoise(img, spec.alpha, spec.beta, spec.k)
    t = torch.from_numpy(img).to(DEV)
    out = torch.empty_like(t)
    p = _api.Params(img.shape[0], img.shape[1], spec.alpha, spec.beta, spec.k)
    ws = torch.empty(lib.phgrms_workspace_bytes(p), dtype=torch.uint8, device=DEV)
    ch = torch.zeros(spec.k, dtype=torch.int64, device=DEV)
    it = torch.zeros(1, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    rc = lib.phgrms_denoise_ex(t.data_ptr(), out.data_ptr(), p, 0, ws.data_ptr(), ws.numel(),
                               ch.data_ptr(), it.data_ptr(), None)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert int(it.item()) == rit and ch[:rit].cpu().tolist() == rch
