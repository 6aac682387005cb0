"""Write the oracle's results for the full-size workloads to
tests/golden/expected_*.json (SHA-256 of the output image, iteration count,
per-pass changed counts).  Calls only the oracle and the seeded input
generator; run from the repository root:

    python tests/golden/make_expected.py [NAME ...] [--out-dir DIR]

NAME is one of single481, sweep2048, large8192, large16384, batch512,
serve8, serve256 (default: all of them).

Each image is computed by one single-threaded oracle call; independent
images run in parallel processes.
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1306_5390_amd import synth  # noqa: E402


def _one(args):
    spec = synth.ImageSpec(*args)
    img = spec.image()
    t0 = time.time()
    out, it, ch = oracle.denoise(img, spec.alpha, spec.beta, spec.k)
    return {"rows": spec.rows, "cols": spec.cols, "density": spec.density,
            "alpha": spec.alpha, "beta": spec.beta, "k": spec.k, "seed": spec.seed,
            "input_sha256": hashlib.sha256(img.tobytes()).hexdigest(),
            "output_sha256": hashlib.sha256(out.tobytes()).hexdigest(),
            "iterations": it, "changed": ch, "oracle_seconds": round(time.time() - t0, 2)}


def serve8_indices(pool):
    """Eight requests of the serving pool at full size: the largest image,
    the largest with the other beta, and six more at evenly spaced ranks of
    the pool sorted by area (largest first)."""
    order = sorted(range(len(pool)), key=lambda i: (-pool[i].rows * pool[i].cols, i))
    first = order[0]
    other = next(i for i in order if pool[i].beta != pool[first].beta)
    pick = [first, other]
    for rank in (32, 64, 96, 128, 176, 240):
        i = order[rank]
        if i not in pick:
            pick.append(i)
    return pick


def workload(name):
    if name == "single481":
        return [synth.single_481x321()]
    if name == "sweep2048":
        return synth.sweep_2048()
    if name == "large8192":
        return [synth.large_single(8192)]
    if name == "large16384":
        return [synth.large_single(16384)]
    if name == "serve8":
        pool = synth.serve_pool(n=256, seed=6)
        return [pool[i] for i in serve8_indices(pool)]
    if name == "serve256":
        # every image of the serving pool with its own alpha, beta and k
        return synth.serve_pool(n=256, seed=6)
    if name == "batch512":
        return synth.batch_512(n=512, seed=5)
    raise ValueError(name)


def main(names, out_dir=HERE):
    oracle.build(force=False)
    for name in names:
        specs = workload(name)
        t0 = time.time()
        args = [(s.rows, s.cols, s.density, s.alpha, s.beta, s.k, s.seed) for s in specs]
        with mp.get_context("fork").Pool(min(len(args), os.cpu_count() or 1)) as pool:
            # largest first, so the slow ones start early
            order = sorted(range(len(args)), key=lambda i: -args[i][0] * args[i][1])
            res = pool.map(_one, [args[i] for i in order], chunksize=1)
            pool.close()
            pool.join()
        out = [None] * len(args)
        for i, r in zip(order, res):
            out[i] = r
        path = os.path.join(out_dir, "expected_%s.json" % name)
        with open(path, "w") as f:
            json.dump({"workload": name, "generator": "paper_1306_5390_amd.synth",
                       "results": out}, f, indent=0)
        print(name, len(out), "images", round(time.time() - t0, 1), "s ->", path, flush=True)


if __name__ == "__main__":
    argv = sys.argv[1:]
    out_dir = HERE
    if "--out-dir" in argv:
        i = argv.index("--out-dir")
        out_dir = argv[i + 1]
        del argv[i:i + 2]
    main(argv or ["single481", "sweep2048", "large8192", "large16384", "batch512", "serve8",
                  "serve256"],
         out_dir)
