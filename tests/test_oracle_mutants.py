"""The pins pin: each plausible mistake, planted in a temporary copy of the
oracle source and built on the CPU, must make at least one pin fail.

Each mutant is a small textual change of oracle/phgrms_oracle.c; all keep
memory accesses in bounds.  The pins run in a child process.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

MUTANTS = {
    # Algorithm 2 band read symmetrically (|d| >= alpha outside)
    "band2_symmetric": ("return !(y > x - alpha && y <= x + alpha);",
                        "return !(y > x - alpha && y < x + alpha);"),
    # Algorithm 2 band with the sign of the asymmetry flipped
    "band2_flipped": ("return !(y > x - alpha && y <= x + alpha);",
                      "return !(y >= x - alpha && y < x + alpha);"),
    # Algorithm 1 band not strict
    "band1_closed": ("return y > x - alpha && y < x + alpha;",
                     "return y >= x - alpha && y <= x + alpha;"),
    # the window size counting only positions inside the image
    "pixcount_in_image": (
        "const int64_t window_size = side * side;",
        "const int64_t window_size = ((r + beta < im->rows ? r + beta : im->rows - 1) -"
        " (r - beta > 0 ? r - beta : 0) + 1) * ((c + beta < im->cols ? c + beta : im->cols - 1) -"
        " (c - beta > 0 ? c - beta : 0) + 1) + 0 * side;"),
    # window of Algorithm 2 one column short (a dropped term)
    "window_short": ("for (int ox = -beta; ox <= beta; ox++)", "for (int ox = -beta; ox < beta; ox++)"),
    # window of Algorithm 1 one row short
    "card_window_short": ("for (int di = -beta; di <= beta; di++)",
                          "for (int di = -beta; di < beta; di++)"),
    # gate threshold
    "gate_lt2": ("if (card > 2) return x;", "if (card >= 2) return x;"),
    # replacement threshold
    "flag_ge": ("if (o.count <= window_size - 3) return x;", "if (o.count < window_size - 3) return x;"),
    # rounded instead of floored mean
    "mean_rounded": ("(uint32_t)(o.sq_sum / (uint64_t)o.count)",
                     "(uint32_t)((o.sq_sum + (uint64_t)o.count / 2) / (uint64_t)o.count)"),
    # mean of values instead of squares
    "sum_not_squared": ("o.sq_sum += (uint64_t)y * (uint64_t)y;", "o.sq_sum += (uint64_t)y * 255u;"),
    # integer square root off by one
    "isqrt_strict": ("(uint64_t)(n + 1) * (uint64_t)(n + 1) <= (uint64_t)q",
                     "(uint64_t)(n + 1) * (uint64_t)(n + 1) < (uint64_t)q"),
    # in-place (Gauss-Seidel) update instead of the temporary image
    "in_place": ("out[r * cols + c] = noise_rule(&before, r, c, alpha, beta, card[r * cols + c]);",
                 "{ const image_view now = {out, rows, cols};\n"
                 "        out[r * cols + c] = noise_rule(&now, r, c, alpha, beta, card[r * cols + c]); }"),
    # no early stop
    "no_stop": ("if (moved == 0) break; /* R12 */", "(void)0;"),
    # cardinality counted twice at the centre
    "card_double_count": ("card[(r + di) * im->cols + (c + dj)] += 1;",
                          "card[r * im->cols + c] += 2;"),
    # generator: a wrong shift in the output function
    "splitmix_shift": ("z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;",
                       "z = (z ^ (z >> 28)) * 0x94d049bb133111ebull;"),
    # generator: output taken before the state advances (index off by one)
    "splitmix_pre_step": ("    state += 0x9e3779b97f4a7c15ull;\n    uint64_t z = state;",
                          "    uint64_t z = state;\n    state += 0x9e3779b97f4a7c15ull;"),
    # noise: salt and pepper swapped
    "noise_swapped": ("    if (u < t_pepper)\n      v = 0;\n    else if (u < t_salt)\n      v = 255;",
                      "    if (u < t_pepper)\n      v = 255;\n    else if (u < t_salt)\n      v = 0;"),
    # noise: the low half of the output instead of the top 32 bits
    "noise_low_bits": ("const uint32_t u = (uint32_t)(r >> 32);", "const uint32_t u = (uint32_t)r;"),
    # quality sum: absolute instead of squared differences
    "ssd_abs": ("    s += d * d;", "    s += d < 0 ? -d : d;"),
    # period-2 stop: the first possible cycle (after pass 2) missed
    "cycle_from_3": ("if (t >= 2) same_as_older", "if (t >= 3) same_as_older"),
    # period-2 stop: compared with the previous image (never fires on a cycle)
    "cycle_vs_previous": ("memcmp(nxt, older, (size_t)n) == 0", "memcmp(nxt, cur, (size_t)n) == 0"),
    # period-2 stop: returns the other image of the cycle
    "cycle_returns_older": ("if (ch == 0 || same_as_older) break;",
                            "if (same_as_older) memcpy(cur, older, (size_t)n);\n"
                            "    if (ch == 0 || same_as_older) break;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    with open(oracle.SOURCE) as f:
        src = f.read()
    assert src.count(old) == 1, "mutation anchor not found once: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    oracle.compile_oracle(str(mut), lib)
    r = subprocess.run([sys.executable, os.path.join(HERE, "pins.py"), lib],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "mutant %s passed every pin" % name
    assert "AssertionError" in r.stderr, r.stderr[-2000:]


def test_unmutated_passes(tmp_path):
    lib = str(tmp_path / "libplain.so")
    oracle.compile_oracle(oracle.SOURCE, lib)
    r = subprocess.run([sys.executable, os.path.join(HERE, "pins.py"), lib],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
