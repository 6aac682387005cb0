"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (the autotuner cache applied): the output image's SHA-256,
the iteration count and every per-pass changed count equal the oracle's,
stored by tests/golden/make_expected.py (which calls only the oracle).
The 8192^2 and 16384^2 images are also run with other kernel shapes (one
pass per launch dense, four per launch, change tracking, tile skipping) and
the plain path; the 16384^2 image is further checked at sampled pixels, each
computed by the oracle on its crop of radius k*beta, and against the
border-frame invariant."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
import golden_io
from paper_1306_5390_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def phg():
    import paper_1306_5390_amd as m
    from paper_1306_5390_amd import autotune
    m.load_library()
    autotune.load()
    return m


def expected(name):
    path = os.path.join(golden_io.GOLDEN_DIR, "expected_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("no stored oracle results for %s" % name)
    with open(path) as f:
        return json.load(f)["results"]


def sha(t: torch.Tensor) -> str:
    return hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest()


def check_one(m, spec, exp, img=None, plain=False):
    img = spec.image() if img is None else img
    assert hashlib.sha256(img.tobytes()).hexdigest() == exp["input_sha256"], "generator drift"
    out, it, ch = m.denoise(torch.from_numpy(img).to(DEV), spec.alpha, spec.beta, spec.k,
                            plain=plain)
    assert sha(out) == exp["output_sha256"], (spec, plain)
    assert it == exp["iterations"] and ch == exp["changed"], (spec, it, exp["iterations"])


def test_single_481x321():
    m = phg()
    (exp,) = expected("single481")
    check_one(m, synth.single_481x321(), exp)


def test_sweep2048():
    m = phg()
    exps = expected("sweep2048")
    specs = synth.sweep_2048()
    img = specs[0].image()
    for spec, exp in zip(specs, exps):
        print("sweep", spec.alpha, spec.beta, flush=True)
        check_one(m, spec, exp, img=img)
    check_one(m, specs[0], exps[0], img=img, plain=True)


def other_shapes(m):
    """Dense one pass per launch, four passes per launch, change tracking
    and the skipping shapes."""
    out = [3, 6]
    for s in range(len(m.shapes())):
        if m.shape_tracks_changes(s):
            out.append(s)
    return out


def test_large8192():
    m = phg()
    (exp,) = expected("large8192")
    spec = synth.large_single(8192)
    print("generating 8192^2", flush=True)
    img = spec.image()
    check_one(m, spec, exp, img=img)
    saved = m.get_tuning_class(2, 2)
    try:
        for s in other_shapes(m):
            print("8192^2 shape", s, flush=True)
            m.set_tuning_class(2, 2, s)
            check_one(m, spec, exp, img=img)
    finally:
        m.set_tuning_class(2, 2, saved)
    print("8192^2 plain", flush=True)
    check_one(m, spec, exp, img=img, plain=True)


def test_batch512():
    m = phg()
    exps = expected("batch512")
    specs_full = synth.batch_512(n=512, seed=5)
    print("generating 512 images", flush=True)
    imgs = synth.generate_many(specs_full, workers=min(16, os.cpu_count() or 1))
    specs = [(s.rows, s.cols, s.alpha, s.beta, s.k) for s in specs_full]
    b = m.Batch(specs, device=DEV)
    ain = b.new_arena()
    for i, img in enumerate(imgs):
        b.view(ain, i).copy_(torch.from_numpy(img).to(DEV))
    aout = b.new_arena()
    for rep in range(2):
        print("batch run", rep, flush=True)
        b.run(ain, aout)
        torch.cuda.synchronize()
        res = b.results()
        for i, exp in enumerate(exps):
            assert sha(b.view(aout, i, out=True)) == exp["output_sha256"], (rep, i)
            assert res[i] == (exp["iterations"], exp["changed"]), (rep, i)
    b.close()


def test_large16384():
    """Output SHA-256, iterations and every per-pass count against the
    oracle's stored results, in the benchmark's configuration and with the
    dense one-pass and skipping shapes; then sampled pixels against the
    oracle on crops, and invariants."""
    m = phg()
    (exp,) = expected("large16384")
    spec = synth.large_single(16384)
    print("generating 16384^2", flush=True)
    img = spec.image()
    check_one(m, spec, exp, img=img)
    saved = m.get_tuning_class(2, 2)
    try:
        for s in [3] + [s for s in range(len(m.shapes())) if m.shape_skips_unchanged(s)]:
            print("16384^2 shape", s, flush=True)
            m.set_tuning_class(2, 2, s)
            check_one(m, spec, exp, img=img)
    finally:
        m.set_tuning_class(2, 2, saved)
    out, it, ch = m.denoise(torch.from_numpy(img).to(DEV), spec.alpha, spec.beta, spec.k)
    got = out.cpu().numpy()
    b = spec.beta
    # border frame unchanged
    assert np.array_equal(got[:b], img[:b]) and np.array_equal(got[-b:], img[-b:])
    assert np.array_equal(got[:, :b], img[:, :b]) and np.array_equal(got[:, -b:], img[:, -b:])
    # changed counts are consistent with the run: nothing changes after a zero
    assert len(ch) == it and all(c >= 0 for c in ch)
    rng = np.random.Generator(np.random.PCG64(16384))
    pts = [(int(rng.integers(0, 16384)), int(rng.integers(0, 16384))) for _ in range(40)]
    pts += [(0, 0), (16383, 16383), (b, b), (16383 - b, 8000), (255, 256), (256, 255)]
    for (r, c) in pts:
        assert got[r, c] == oracle.denoise_window(img, spec.alpha, b, spec.k, r, c), (r, c)
    # pixels where the first pass changed something, sampled
    d1, it1, ch1 = m.denoise(torch.from_numpy(img).to(DEV), spec.alpha, b, 1)
    moved = np.argwhere(d1.cpu().numpy() != img)
    assert len(moved) == ch1[0] == ch[0]
    for (r, c) in moved[rng.integers(0, len(moved), size=20)]:
        assert got[r, c] == oracle.denoise_window(img, spec.alpha, b, spec.k, int(r), int(c))
