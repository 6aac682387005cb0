"""Pins of the CPU oracle against facts the paper and mathematics fix.

Each check takes an `oracle.Oracle` instance so the same checks can be run on
deliberately broken builds of the oracle (test_oracle_mutants.py) and must
fail there.  None of these checks re-types the oracle's own steps:

* hand-derived golden examples (tests/golden/, Section 2 rules worked by hand);
* alpha = 0: the band is empty, so the method reduces to the interior floor
  root-mean-square box filter, computed here with scipy's 2-D convolution and
  math.isqrt;
* Algorithm 1's scatter count equals a gather count, because the band
  relation |I_p - I_q| < alpha is symmetric; the gather count is re-derived
  here with shifted numpy views;
* the gate-free closed form of Algorithm 2: for an interior pixel the window
  holds all N positions, so flag = N - K with K = #{q : -alpha < I_q - I_p <=
  alpha}; flag > N - 3 iff K <= 2, and K <= 2 implies C <= 2, so a pass
  replaces exactly the interior pixels with K <= 2; a border pixel sees at
  most N - (2*beta + 1) <= N - 3 window positions inside the image and is
  never replaced;
* invariants: output range, border frame unchanged, the 8 symmetries of the
  square commute with the method, a pass is a function of the image alone
  (resume), constant images and k = 0 are identities, a replaced value lies
  between the smallest and largest outside value.
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

import golden_io  # noqa: E402


# ---------------------------------------------------------------------------
# independent formulations used as references
# ---------------------------------------------------------------------------

def isqrt_array(q: np.ndarray) -> np.ndarray:
    return np.array([math.isqrt(int(v)) for v in q.ravel()],
                    dtype=np.int64).reshape(q.shape)


def gather_cardinality(img: np.ndarray, alpha: int, beta: int) -> np.ndarray:
    """C(p) = #{q in window(p), q in image : |I_q - I_p| < alpha}."""
    a = img.astype(np.int64)
    h, w = a.shape
    pad = np.full((h + 2 * beta, w + 2 * beta), -10_000, dtype=np.int64)
    pad[beta:beta + h, beta:beta + w] = a
    card = np.zeros((h, w), dtype=np.int64)
    for dr in range(-beta, beta + 1):
        for dc in range(-beta, beta + 1):
            y = pad[beta + dr:beta + dr + h, beta + dc:beta + dc + w]
            card += (np.abs(y - a) < alpha) & (y >= 0)
    return card


def closed_form_pass(img: np.ndarray, alpha: int, beta: int):
    """One pass by the gate-free rule: (image, changed)."""
    h, w = img.shape
    out = img.copy()
    n = (2 * beta + 1) ** 2
    if h < 2 * beta + 1 or w < 2 * beta + 1:
        return out, 0
    a = img.astype(np.int64)
    x = a[beta:h - beta, beta:w - beta]
    kin = np.zeros_like(x)
    s = np.zeros_like(x)
    for dr in range(-beta, beta + 1):
        for dc in range(-beta, beta + 1):
            y = a[beta + dr:h - beta + dr, beta + dc:w - beta + dc]
            d = y - x
            inside = (d > -alpha) & (d <= alpha)
            kin += inside
            s += np.where(inside, 0, y * y)
    f = n - kin
    rep = kin <= 2
    val = x.copy()
    if rep.any():
        val[rep] = isqrt_array(s[rep] // f[rep])
    out[beta:h - beta, beta:w - beta] = val.astype(np.uint8)
    return out, int((out != img).sum())


def closed_form_denoise(img: np.ndarray, alpha: int, beta: int, k: int):
    cur = img.copy()
    changed = []
    for _ in range(k):
        cur, ch = closed_form_pass(cur, alpha, beta)
        changed.append(ch)
        if ch == 0:
            break
    return cur, len(changed), changed


def boundary_image(rng: np.random.Generator, h: int, w: int, alpha: int) -> np.ndarray:
    """Values clustered at alpha-band boundaries around a few centres, plus
    salt and pepper: the inputs on which band-edge mistakes show."""
    centres = rng.integers(0, 256, size=3)
    offs = np.array([0, alpha - 1, alpha, alpha + 1, -(alpha - 1), -alpha,
                     -(alpha + 1)])
    vals = (centres[rng.integers(0, 3, size=(h, w))]
            + offs[rng.integers(0, len(offs), size=(h, w))])
    vals = np.clip(vals, 0, 255)
    noise = rng.random((h, w))
    vals[noise < 0.15] = 0
    vals[(noise >= 0.15) & (noise < 0.3)] = 255
    return vals.astype(np.uint8)


D4 = [
    (lambda a: a, lambda a: a),
    (lambda a: np.rot90(a, 1), lambda a: np.rot90(a, -1)),
    (lambda a: np.rot90(a, 2), lambda a: np.rot90(a, -2)),
    (lambda a: np.rot90(a, 3), lambda a: np.rot90(a, -3)),
    (lambda a: a[::-1, :], lambda a: a[::-1, :]),
    (lambda a: a[:, ::-1], lambda a: a[:, ::-1]),
    (lambda a: a.T, lambda a: a.T),
    (lambda a: np.rot90(a, 1).T, lambda a: np.rot90(a.T, -1)),
]


# ---------------------------------------------------------------------------
# the checks
# ---------------------------------------------------------------------------

def check_golden(o, path: str):
    g = golden_io.load(path)
    out, it, ch = o.denoise(g["input"], g["alpha"], g["beta"], g["k"])
    assert np.array_equal(out, g["output"]), (g["name"], out)
    assert it == g["iterations"], (g["name"], it)
    assert ch == g["changed"], (g["name"], ch)


def check_goldens(o):
    for p in golden_io.golden_files():
        check_golden(o, p)


def check_isqrt(o):
    for q in list(range(0, 65026)) + [2**20 + 7, 2**31 - 1, 2**32 - 1]:
        assert o.isqrt(q) == math.isqrt(q), q


def check_alpha0_box(o, seed=11):
    from scipy.signal import convolve2d
    rng = np.random.Generator(np.random.PCG64(seed))
    for (h, w, beta) in [(7, 13, 1), (12, 9, 2), (5, 5, 2), (16, 23, 3), (9, 31, 1)]:
        img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
        out, ch = o.one_pass(img, 0, beta)
        n = (2 * beta + 1) ** 2
        sq = img.astype(np.int64) ** 2
        box = convolve2d(sq, np.ones((2 * beta + 1, 2 * beta + 1), np.int64),
                         mode="valid")
        ref = img.copy()
        if box.size:
            ref[beta:h - beta, beta:w - beta] = isqrt_array(box // n).astype(np.uint8)
        assert np.array_equal(out, ref), (h, w, beta)
        assert ch == int((ref != img).sum())


def check_scatter_gather(o, seed=12):
    rng = np.random.Generator(np.random.PCG64(seed))
    for (h, w, alpha, beta) in [(9, 14, 20, 1), (17, 11, 10, 2), (6, 6, 0, 1),
                                (20, 25, 40, 3), (1, 30, 20, 1), (3, 2, 255, 2)]:
        img = boundary_image(rng, h, w, max(alpha, 1))
        cs = o.cardinality(img, alpha, beta, scatter=True)
        cg = o.cardinality(img, alpha, beta, scatter=False)
        ref = gather_cardinality(img, alpha, beta)
        assert np.array_equal(cs.astype(np.int64), ref), (h, w, alpha, beta)
        assert np.array_equal(cg.astype(np.int64), ref), (h, w, alpha, beta)


def check_closed_form_random(o, seed=13, count=60):
    rng = np.random.Generator(np.random.PCG64(seed))
    for i in range(count):
        beta = 1 + (i % 3)
        alpha = int(rng.choice([1, 2, 10, 20, 40, 128, 255]))
        h = int(rng.integers(1, 24))
        w = int(rng.integers(1, 24))
        img = boundary_image(rng, h, w, alpha)
        k = int(rng.integers(1, 6))
        ref, rit, rch = closed_form_denoise(img, alpha, beta, k)
        out, it, ch = o.denoise(img, alpha, beta, k)
        assert np.array_equal(out, ref), (h, w, alpha, beta, k)
        assert (it, ch) == (rit, rch), (h, w, alpha, beta, k)


def check_exhaustive_3x3(o):
    """Every 3x3 image over a 3-symbol band-edge alphabet: one interior pixel."""
    import itertools
    alpha = 20
    for alphabet in ([100, 120, 80], [100, 121, 81], [0, 20, 255]):
        for vals in itertools.product(range(3), repeat=9):
            img = np.array([alphabet[v] for v in vals], dtype=np.uint8).reshape(3, 3)
            out, ch = o.one_pass(img, alpha, 1)
            ref, rch = closed_form_pass(img, alpha, 1)
            if not np.array_equal(out, ref) or ch != rch:
                raise AssertionError(("3x3", img.tolist(), out.tolist(), ref.tolist()))


def check_invariants(o, seed=14):
    rng = np.random.Generator(np.random.PCG64(seed))
    for i in range(12):
        beta = 1 + (i % 2)
        alpha = int(rng.choice([5, 20, 40]))
        h = int(rng.integers(5, 20))
        w = int(rng.integers(5, 20))
        img = boundary_image(rng, h, w, alpha)
        k = 6
        out, it, ch = o.denoise(img, alpha, beta, k)
        # range and border frame
        assert out.dtype == np.uint8
        fr = np.ones_like(img, dtype=bool)
        fr[beta:h - beta, beta:w - beta] = False
        assert np.array_equal(out[fr], img[fr])
        # symmetries of the square
        for fwd, inv in D4:
            o2, it2, ch2 = o.denoise(np.ascontiguousarray(fwd(img)), alpha, beta, k)
            assert np.array_equal(inv(o2), out), ("D4", i)
            assert (it2, ch2) == (it, ch)
        # resume: the pass loop is a function of the current image only
        if it >= 3 and all(c > 0 for c in ch[:2]):
            mid, it_a, ch_a = o.denoise(img, alpha, beta, 2)
            fin, it_b, ch_b = o.denoise(mid, alpha, beta, k - 2)
            assert np.array_equal(fin, out)
            assert it_a + it_b == it and ch_a + ch_b == ch
        # k = 0 is the identity
        z, itz, chz = o.denoise(img, alpha, beta, 0)
        assert np.array_equal(z, img) and itz == 0 and chz == []
        # a replaced value lies within the outside values of its window
        p1, _ = o.one_pass(img, alpha, beta)
        a = img.astype(np.int64)
        for (r, c) in zip(*np.nonzero(p1 != img)):
            win = a[r - beta:r + beta + 1, c - beta:c + beta + 1].ravel()
            d = win - a[r, c]
            outside = win[~((d > -alpha) & (d <= alpha))]
            assert outside.min() <= p1[r, c] <= outside.max()
    # constant images and windows larger than the image
    for v in (0, 17, 255):
        img = np.full((9, 11), v, np.uint8)
        out, it, ch = o.denoise(img, 20, 2, 5)
        assert np.array_equal(out, img) and it == 1 and ch == [0]
    img = rng.integers(0, 256, size=(4, 40)).astype(np.uint8)
    out, it, ch = o.denoise(img, 20, 2, 5)
    assert np.array_equal(out, img) and it == 1 and ch == [0]
    # empty image
    e = np.zeros((0, 7), np.uint8)
    out, it, ch = o.denoise(e, 20, 1, 3)
    assert out.shape == (0, 7) and it == 1 and ch == [0]


def check_window_crop(o, seed=15):
    """The crop evaluation used for sampled parity equals the full run."""
    rng = np.random.Generator(np.random.PCG64(seed))
    img = boundary_image(rng, 40, 37, 20)
    for (alpha, beta, k) in [(20, 1, 4), (10, 2, 3)]:
        full, _, _ = o.denoise(img, alpha, beta, k)
        for _ in range(12):
            r = int(rng.integers(0, 40))
            c = int(rng.integers(0, 37))
            assert o.denoise_window(img, alpha, beta, k, r, c) == full[r, c]


# ---- the experiments' noise and quality measure (Section 3) ----------------

def check_splitmix64(o):
    """The oracle's generator reproduces the generator's published outputs."""
    import json
    with open(os.path.join(HERE, "golden", "splitmix64_reference.json")) as f:
        ref = json.load(f)
    assert o.splitmix64(1234567, 5) == ref["seed_1234567_first5"]
    xs = np.array(o.splitmix64(987654321, 100000), dtype=np.uint64)
    buckets = (xs >> np.uint64(32)).astype(np.float64) * 5.0 / 2.0 ** 32
    counts = np.bincount(buckets.astype(np.int64), minlength=5)
    assert counts.tolist() == ref["seed_987654321_first100000_bucket_counts_of_5"]


def check_salt_pepper(o, seed=16):
    """Noise: each pixel follows the threshold rule on its own generator
    output (checked against the pinned generator), zero thresholds are the
    identity, and densities come out within binomial bounds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    img = rng.integers(1, 255, size=(37, 53)).astype(np.uint8)   # no 0/255 inputs
    n = img.size
    tp, ts = 1 << 29, 3 << 29                 # 1/8 pepper, 1/4 salt
    out = o.salt_pepper(img, 99, tp, ts)
    u = np.array(o.splitmix64(99, n), dtype=np.uint64) >> np.uint64(32)
    u = u.reshape(img.shape)
    assert np.array_equal(out[u < tp], np.zeros(int((u < tp).sum()), np.uint8))
    sel = (u >= tp) & (u < ts)
    assert np.array_equal(out[sel], np.full(int(sel.sum()), 255, np.uint8))
    keep = u >= ts
    assert np.array_equal(out[keep], img[keep])
    assert np.array_equal(o.salt_pepper(img, 5, 0, 0), img)
    # densities on a large image (binomial, 6 sigma)
    big = np.full((1000, 1000), 128, np.uint8)
    rho = 0.2
    t_s = int(round(rho * 2 ** 32))
    t_p = t_s // 2
    nb = o.salt_pepper(big, 2024, t_p, t_s)
    for frac, p in (((nb == 0).mean(), rho / 2), ((nb == 255).mean(), rho / 2)):
        sd = (p * (1 - p) / big.size) ** 0.5
        assert abs(frac - p) < 6 * sd, (frac, p)


def check_sq_diff_sum(o, seed=17):
    """The sum of squared differences equals numpy's."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for shape in [(1, 1), (3, 7), (64, 257), (300, 301)]:
        a = rng.integers(0, 256, size=shape).astype(np.uint8)
        b = rng.integers(0, 256, size=shape).astype(np.uint8)
        want = int(((a.astype(np.int64) - b.astype(np.int64)) ** 2).sum())
        assert o.sq_diff_sum(a, b) == want
        assert o.sq_diff_sum(a, a) == 0


def noisy_ramp(rng: np.random.Generator, h: int, w: int, density: float = 0.2) -> np.ndarray:
    """A tilted plane with +-15 texture and salt and pepper at `density`:
    small inputs on which the pass loop often ends in a period-2 cycle."""
    yy, xx = np.mgrid[0:h, 0:w]
    base = (int(rng.integers(40, 200)) + int(rng.integers(-4, 5)) * yy
            + int(rng.integers(-4, 5)) * xx + rng.integers(-15, 16, (h, w)))
    img = np.clip(base, 0, 255).astype(np.uint8)
    u = rng.random((h, w))
    img[u < density / 2] = 0
    img[(u >= density / 2) & (u < density)] = 255
    return img


def check_cycle_stop(o, seed=18):
    """The opt-in period-2 stop against its definition: with I_0 the input
    and I_t the closed-form pass applied t times, the run ends after pass
    t* = the first t >= 1 with I_t == I_{t-1} (nothing changed) or, for
    t >= 2, I_t == I_{t-2}; at most k passes.  Every pass up to t* is an
    ordinary pass, so the image and counts are those of t* plain passes, and
    once I_t* == I_{t*-2} every later plain pass alternates between
    I_{t*-1} and I_t*."""
    # worked example: the centre goes 117 -> 120 -> 117, so pass 2 restores
    # the input and the run stops there
    g = golden_io.load(os.path.join(golden_io.GOLDEN_DIR, "p_period2_k5.txt"))
    out, it, ch = o.denoise_cycle(g["input"], g["alpha"], g["beta"], g["k"])
    assert it == 2 and ch == [1, 1], (it, ch)
    assert np.array_equal(out, g["input"])
    out, it, ch = o.denoise_cycle(g["input"], g["alpha"], g["beta"], 1)
    assert it == 1 and ch == [1] and out[2, 2] == 120, (it, ch)
    rng = np.random.default_rng(seed)
    kinds = set()
    for case in range(36):
        h, w = int(rng.integers(5, 25)), int(rng.integers(5, 31))
        alpha, beta = [(20, 1), (10, 1), (20, 2)][case % 3]
        img = noisy_ramp(rng, h, w)
        k = [0, 1, 2, 3, 40][case % 5]
        seq, changed = [img], []
        t_star = 0
        for t in range(1, k + 1):
            nxt, c = closed_form_pass(seq[-1], alpha, beta)
            seq.append(nxt)
            changed.append(c)
            t_star = t
            if c == 0 or (t >= 2 and np.array_equal(nxt, seq[t - 2])):
                break
        out, it, ch = o.denoise_cycle(img, alpha, beta, k)
        assert it == t_star and ch == changed, (case, it, t_star, ch, changed)
        assert np.array_equal(out, seq[t_star]), case
        if t_star >= 2 and changed[-1] != 0 and np.array_equal(seq[t_star], seq[t_star - 2]):
            kinds.add("cycle")
            for extra in (1, 2, 3):
                later, _, _ = closed_form_denoise(img, alpha, beta, t_star + extra)
                assert np.array_equal(later, seq[t_star - (extra % 2)]), (case, extra)
        elif t_star > 0 and changed[-1] == 0:
            kinds.add("fixed point")
        elif t_star == k:
            kinds.add("k cap")
    assert kinds == {"cycle", "fixed point", "k cap"}, kinds


ALL_CHECKS = [check_goldens, check_isqrt, check_alpha0_box, check_scatter_gather,
              check_closed_form_random, check_exhaustive_3x3, check_invariants,
              check_window_crop, check_splitmix64, check_salt_pepper, check_sq_diff_sum,
              check_cycle_stop]


def run_all(o):
    for chk in ALL_CHECKS:
        chk(o)


if __name__ == "__main__":
    # Used by the mutation test: run every pin against the library given on
    # the command line; exit status 0 iff all pins hold.
    sys.path.insert(0, os.path.dirname(HERE))
    import oracle as _oracle
    run_all(_oracle.Oracle(sys.argv[1]))
