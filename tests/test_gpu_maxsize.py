"""GPU runs at the largest image the interface accepts (rows * cols just
under 2^31 pixels), where the kernels' 32-bit pixel offsets come closest to
their limit.  The oracle cannot run at this size, so the inputs are built
so that the exact result follows from the method's definition (Section 2):

* a constant field with isolated salt pixels far apart: each salt pixel has
  every other window pixel outside its band, so it is replaced by the root
  mean square of equal values, i.e. the field's value; no other pixel has
  fewer than 3 window pixels in its band.  One changing pass, then one
  with no change: 2 iterations, changed = [number of salt pixels, 0].
  The same construction at a small size is pinned to the oracle first.
* one-row and one-column images of about 2^31 random bytes: every pixel
  lies on the border frame, which is never replaced, so the output equals
  the input.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1306_5390_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SIDE = 46340                 # 46340^2 = 2,147,395,600 < 2^31
BG, SALT, STEP, OFF = 100, 255, 1000, 500


def phg():
    import paper_1306_5390_amd as m
    from paper_1306_5390_amd import autotune
    m.load_library()
    autotune.load()
    return m


def salted(side):
    img = np.full((side, side), BG, dtype=np.uint8)
    img[OFF::STEP, OFF::STEP] = SALT
    return img


@pytest.mark.parametrize("beta", [1, 2])
def test_salt_field_construction_matches_oracle(beta):
    img = salted(1700)
    out, it, ch = oracle.denoise(img, 20, beta, 3)
    n_salt = int((img == SALT).sum())
    assert n_salt == 4
    assert it == 2 and list(ch[:it]) == [n_salt, 0]
    assert (out == BG).all()


@pytest.mark.parametrize("beta", [1, 2])
def test_largest_square_image(beta):
    m = phg()
    print("max-size square", SIDE, "beta", beta, flush=True)
    img = torch.from_numpy(salted(SIDE)).to(DEV)
    n_salt = int((img == SALT).sum().item())
    assert n_salt == ((SIDE - OFF + STEP - 1) // STEP) ** 2
    out, it, ch = m.denoise(img, 20, beta, 3)
    assert it == 2 and ch == [n_salt, 0], (it, ch)
    assert int((out != BG).sum().item()) == 0
    del out
    # the opt-in period-2 stop: the zero-change pass still ends the run
    out, it, ch = m.denoise(img, 20, beta, 3, stop_on_cycle=True)
    assert it == 2 and ch == [n_salt, 0], (it, ch)
    assert int((out != BG).sum().item()) == 0
    del img, out
    torch.cuda.empty_cache()


def equal_in_chunks(a, b, chunk=1 << 26):
    a, b = a.reshape(-1), b.reshape(-1)
    return all(torch.equal(a[i:i + chunk], b[i:i + chunk]) for i in range(0, a.numel(), chunk))


@pytest.mark.parametrize("shape", [(1, (1 << 31) - 1), (1, (1 << 31) - 8), ((1 << 31) - 1, 1)])
def test_largest_one_row_and_one_column_images(shape):
    # (the rounding up of a side near 2^31 to whole tiles once overflowed:
    # every pixel came out 0)
    m = phg()
    print("max-size line", shape, flush=True)
    g = torch.Generator(device=DEV).manual_seed(7)
    img = torch.randint(0, 256, shape, dtype=torch.uint8, device=DEV, generator=g)
    out, it, ch = m.denoise(img, 20, 1, 2)
    assert it == 1 and ch == [0], (it, ch)
    assert equal_in_chunks(out, img)
    del img, out
    torch.cuda.empty_cache()


def test_batch_with_a_largest_image():
    # the batch path's tile tables, tile lists and grids at a near-2^31-pixel
    # image, next to small images checked against the oracle
    m = phg()
    big = (1, (1 << 31) - 1)
    small = [synth.noisy_image(300, 400, 0.3, 12), salted(1700)[1400:1700, 1400:1700].copy()]
    specs = [(big[0], big[1], 20, 1, 3)] + [(s.shape[0], s.shape[1], 20, b, 3)
                                            for s, b in zip(small, (1, 2))]
    print("batch with", big, flush=True)
    b = m.Batch(specs, device=DEV)
    ain = b.new_arena()
    g = torch.Generator(device=DEV).manual_seed(11)
    big_in = b.view(ain, 0)
    big_in.copy_(torch.randint(0, 256, big, dtype=torch.uint8, device=DEV, generator=g))
    for i, s in enumerate(small):
        b.view(ain, i + 1).copy_(torch.from_numpy(s).to(DEV))
    aout = b.new_arena()
    b.run(ain, aout)
    torch.cuda.synchronize()
    res = b.results()
    assert res[0] == (1, [0]), res[0]
    assert equal_in_chunks(b.view(aout, 0, out=True), big_in)
    for i, s in enumerate(small):
        ref, rit, rch = oracle.denoise(s, 20, specs[i + 1][3], 3)
        assert np.array_equal(b.view(aout, i + 1, out=True).cpu().numpy(), ref), i
        assert res[i + 1] == (rit, list(rch[:rit])), (i, res[i + 1])
    b.close()
    del ain, aout
    torch.cuda.empty_cache()


def test_server_with_a_largest_image():
    # a served request of 46340^2 pixels beside a small one
    import time
    m = phg()
    srv = m.Server(6 << 30, device=DEV, max_active=4)
    big = torch.from_numpy(salted(SIDE)).to(DEV)
    n_salt = int((big == SALT).sum().item())
    small = synth.noisy_image(200, 300, 0.3, 13)
    print("serving", SIDE, flush=True)
    ids = [srv.submit(big, 20, 1, 3), srv.submit(torch.from_numpy(small).to(DEV), 20, 2, 3)]
    done, t0 = {}, time.time()
    while len(done) < 2:
        for rid in ids:
            if rid not in done:
                r = srv.poll(rid)
                if r is not None:
                    done[rid] = r
        assert time.time() - t0 < 120, "server did not finish: %s" % srv.stats()
        time.sleep(0.001)
    view, it, ch, _ = done[ids[0]]
    assert (it, ch) == (2, [n_salt, 0])
    assert int((view != BG).sum().item()) == 0
    ref, rit, rch = oracle.denoise(small, 20, 2, 3)
    view, it, ch, _ = done[ids[1]]
    assert np.array_equal(view.cpu().numpy(), ref) and (it, ch) == (rit, rch)
    for rid in ids:
        srv.release(rid)
    srv.close()
    del big
    torch.cuda.empty_cache()


def expected_line_card(v, alpha):
    """Gather cardinality (beta = 1) of a line image given as a flat int32
    tensor: the pixel itself (for alpha >= 1) and each in-image neighbour
    along the line within the strict band."""
    x = v[1:-1]
    c = (alpha > 0) * torch.ones_like(x)
    for y in (v[:-2], v[2:]):
        c += ((y - x).abs() < alpha).int()
    return c


@pytest.mark.parametrize("shape", [(1, (1 << 31) - 1), ((1 << 31) - 1, 1)])
def test_cardinality_at_the_largest_sizes(shape):
    m = phg()
    print("max-size cardinality", shape, flush=True)
    g = torch.Generator(device=DEV).manual_seed(9)
    img = torch.randint(0, 256, shape, dtype=torch.uint8, device=DEV, generator=g)
    card = m.cardinality(img, 20, 1)
    torch.cuda.synchronize()
    flat, cf = img.reshape(-1), card.reshape(-1)
    n, chunk = flat.numel(), 1 << 26
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        lo, hi = max(a - 1, 0), min(b + 1, n)
        v = flat[lo:hi].int()
        # pad the line's two ends with values outside every band
        v = torch.cat([torch.full((1,), -1000, dtype=torch.int32, device=DEV) if a == 0 else v[:0],
                       v,
                       torch.full((1,), -1000, dtype=torch.int32, device=DEV) if b == n else v[:0]])
        want = expected_line_card(v, 20)
        assert torch.equal(cf[a:b].int(), want), (shape, a)
    if shape[0] == 1:
        sc = m.cardinality_scatter(img, 20, 1)
        torch.cuda.synchronize()
        sf = sc.reshape(-1)
        for a in range(0, n, chunk):
            assert torch.equal(sf[a:a + chunk], cf[a:a + chunk].int()), a
        del sc, sf
    del img, card, flat, cf
    torch.cuda.empty_cache()
