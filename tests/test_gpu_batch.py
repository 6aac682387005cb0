"""GPU parity of the batch path (phgrms_batch_*): every image of a mixed
batch equals the oracle's result for that image alone (image, iterations,
per-pass changed counts), on the first run and on the graph replays."""
import numpy as np
import pytest
import torch

import oracle
import pins
from paper_1306_5390_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def phg():
    import paper_1306_5390_amd as m
    m.load_library()
    return m


def make_batch(seed, n, max_side, kmax, betas=(1, 2, 3, 4)):
    rng = np.random.Generator(np.random.PCG64(seed))
    specs, imgs = [], []
    for i in range(n):
        r = int(rng.integers(0, max_side + 1)) if i % 7 == 3 else int(rng.integers(5, max_side + 1))
        c = int(rng.integers(1, max_side + 1))
        alpha = int(rng.choice([0, 1, 10, 20, 40, 255])) if i % 5 == 0 else int(rng.integers(10, 41))
        beta = int(rng.choice(betas))
        k = int(rng.integers(0, kmax + 1))
        if i % 3 == 0:
            img = synth.noisy_image(r, c, float(rng.uniform(0.05, 0.6)), seed * 1000 + i)
        else:
            img = pins.boundary_image(rng, r, c, max(alpha, 1)) if r * c else np.zeros((r, c), np.uint8)
        specs.append((r, c, alpha, beta, k))
        imgs.append(img)
    return specs, imgs


def check_batch(m, specs, imgs, in_place=False, runs=3):
    b = m.Batch(specs, device=DEV)
    ain = b.new_arena()
    for i, img in enumerate(imgs):
        if img.size:
            b.view(ain, i).copy_(torch.from_numpy(img).to(DEV))
    refs = [oracle.denoise(img, s[2], s[3], s[4]) for img, s in zip(imgs, specs)]
    for rep in range(runs):
        print("run", rep, "images", len(specs), flush=True)
        if in_place:
            arena = ain.clone()
            b.run(arena, arena)
            aout = arena
        else:
            aout = b.new_arena()
            b.run(ain, aout)
        torch.cuda.synchronize()
        res = b.results()
        for i, (ref, rit, rch) in enumerate(refs):
            got = b.view(aout, i, out=True).cpu().numpy()
            assert np.array_equal(got, ref), (rep, i, specs[i])
            assert res[i] == (rit, rch), (rep, i, specs[i], res[i], (rit, rch))
    b.close()


def test_mixed_batch():
    m = phg()
    specs, imgs = make_batch(1, 40, 300, 9)
    check_batch(m, specs, imgs)


def test_mixed_batch_in_place():
    m = phg()
    specs, imgs = make_batch(2, 24, 200, 7)
    check_batch(m, specs, imgs, in_place=True)


@pytest.mark.parametrize("shape", [0, 3, 5, 6, 7, 10, 11, 12])
def test_batch_shapes(shape):
    m = phg()
    saved = {b: [m.get_batch_tuning_class(b, c) for c in range(3)] for b in (1, 2)}
    try:
        for b in (1, 2):
            m.set_batch_tuning_class(b, -1, shape)
        specs, imgs = make_batch(10 + shape, 16, 280, 9, betas=(1, 2))
        check_batch(m, specs, imgs, runs=2)
    finally:
        for b, v in saved.items():
            for c, sh in enumerate(v):
                m.set_batch_tuning_class(b, c, sh)


@pytest.mark.parametrize("shape", [11, 12])
def test_batch_skipping_shapes_longer_runs(shape):
    # the skipping shapes' tile lists over many images: k up to 20 (many
    # listed launches), in place and not, graph replays
    m = phg()
    saved = {b: [m.get_batch_tuning_class(b, c) for c in range(3)] for b in (1, 2)}
    try:
        for b in (1, 2):
            m.set_batch_tuning_class(b, -1, shape)
        specs, imgs = make_batch(40 + shape, 20, 330, 20, betas=(1, 2))
        check_batch(m, specs, imgs, runs=2)
        check_batch(m, specs, imgs, in_place=True, runs=2)
    finally:
        for b, v in saved.items():
            for c, sh in enumerate(v):
                m.set_batch_tuning_class(b, c, sh)


def test_batch_equals_single_image_path_at_scale():
    """A batch of the workload's kind (sides log-uniform, mixed density, alpha,
    beta, k = 32) against the single-image path, which the oracle checks
    elsewhere, plus sampled pixels against the oracle directly."""
    m = phg()
    specs_full = synth.batch_512(n=24, seed=5)
    specs = [(s.rows, s.cols, s.alpha, s.beta, s.k) for s in specs_full]
    imgs = [s.image() for s in specs_full]
    b = m.Batch(specs, device=DEV)
    ain = b.new_arena()
    for i, img in enumerate(imgs):
        b.view(ain, i).copy_(torch.from_numpy(img).to(DEV))
    aout = b.new_arena()
    b.run(ain, aout)
    torch.cuda.synchronize()
    res = b.results()
    rng = np.random.Generator(np.random.PCG64(99))
    for i, (img, s) in enumerate(zip(imgs, specs)):
        out, it, ch = m.denoise(torch.from_numpy(img).to(DEV), s[2], s[3], s[4])
        got = b.view(aout, i, out=True)
        assert torch.equal(got, out), (i, s)
        assert res[i] == (it, ch), (i, s)
        if i < 6:
            g = got.cpu().numpy()
            for _ in range(4):
                r = int(rng.integers(0, s[0]))
                c = int(rng.integers(0, s[1]))
                assert g[r, c] == oracle.denoise_window(img, s[2], s[3], s[4], r, c), (i, r, c)
    b.close()
