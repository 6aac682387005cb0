"""GPU parity of the experiments' noise and quality measure (Section 3):
salt-and-pepper noise bit for bit against the oracle (whose generator is
pinned to the generator's published outputs), and the exact sum of squared
differences behind PSNR."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1306_5390_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def phg():
    import paper_1306_5390_amd as m
    m.load_library()
    return m


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (37, 53), (321, 481), (1024, 1031)])
@pytest.mark.parametrize("density", [0.0, 0.05, 0.2, 0.6, 1.0])
def test_salt_pepper_matches_oracle(shape, density):
    m = phg()
    rng = np.random.Generator(np.random.PCG64(hash((shape, density)) & 0xFFFF))
    img = rng.integers(0, 256, size=shape).astype(np.uint8)
    tp, ts = synth.noise_thresholds(density)
    for seed in (0, 12345, (1 << 63) + 5):
        print("noise", shape, density, seed, flush=True)
        want = oracle.salt_pepper(img, seed, tp, ts)
        got = m.salt_pepper(torch.from_numpy(img).to(DEV), seed, tp, ts).cpu().numpy()
        assert np.array_equal(got, want), (shape, density, seed)


def test_salt_pepper_in_place_and_large():
    m = phg()
    img = synth.clean_image(2048, 2048, 2)
    tp, ts = synth.noise_thresholds(0.3)
    want = oracle.salt_pepper(img, 77, tp, ts)
    t = torch.from_numpy(img).to(DEV)
    m.salt_pepper(t, 77, tp, ts, out=t)          # in place
    assert np.array_equal(t.cpu().numpy(), want)


def test_sq_diff_sum_and_psnr():
    m = phg()
    rng = np.random.Generator(np.random.PCG64(3))
    for shape in [(1, 1), (5, 3), (333, 517), (2048, 2048)]:
        a = rng.integers(0, 256, size=shape).astype(np.uint8)
        b = rng.integers(0, 256, size=shape).astype(np.uint8)
        da, db = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
        ssd = int(m.sq_diff_sum(da, db).item())
        assert ssd == oracle.sq_diff_sum(a, b)
        assert m.psnr(da, db) == pytest.approx(10 * math.log10(255.0 ** 2 * a.size / ssd))
        assert m.psnr(da, da) == float("inf")
