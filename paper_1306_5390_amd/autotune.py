"""Autotuner: pick, per beta and image size class, the compiled kernel shape
(passes per launch, rows per wave, waves per workgroup) that runs the pass
loop fastest on this GPU, and keep the choice in a JSON cache.

    python -m paper_1306_5390_amd.autotune [--out tuning.json] [--betas 1,2]
    python -m paper_1306_5390_amd.autotune --batch-only [--out tuning.json]

For each (beta, size class) it times the pass loop with k = 16 and every
shape, three independent runs at a time on three streams, exactly as
phgrms_denoise_async launches them (replayed as a graph), on a seeded noisy
image of a representative size, and keeps the shape with the most
pixel-passes per second.  With --batch-only it tunes the batch path's own
table instead (see tune_batch) and adds it to the cache.  Results never
depend on the shape; only speed does.
"""
from __future__ import annotations

import argparse
import json
import os

import torch

from . import _api
from . import synth

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
# representative square side per size class (pixels: <2^20, <2^24, >=2^24)
CLASS_SIDES = {0: 768, 1: 2048, 2: 8192}


def _time_shape(img, alpha, beta, shape, T, stream, passes=16, reps=3, concurrent=3):
    """Pixel-passes per second of `concurrent` independent runs of the pass
    loop (k = `passes`) on `img`, each on its own stream, with kernel shape
    `shape` forced for the image's beta and size class: the launch sequence
    phgrms_denoise_async enqueues (change maps and tile lists for the
    shapes that keep them, dense first launches), captured as one graph and
    replayed.  Concurrent runs measure throughput as the benchmark, batches
    and servers use the GPU, not the latency of a lone run.  (T is the
    shape's passes per launch; the loop takes it from the shape itself.)"""
    dev = img.device
    rows, cols = img.shape
    cls = _api.size_class(rows * cols)
    saved = _api.get_tuning_class(beta, cls)
    _api.set_tuning_class(beta, cls, shape)
    try:
        side = [torch.cuda.Stream(device=dev) for _ in range(concurrent)]
        work = []
        for _ in range(concurrent):
            work.append((torch.empty_like(img),
                         torch.empty(_api.workspace_bytes(rows, cols, alpha, beta, passes),
                                     dtype=torch.uint8, device=dev),
                         torch.zeros(max(passes, 1), dtype=torch.int64, device=dev),
                         torch.zeros(1, dtype=torch.int32, device=dev)))
        stream.wait_stream(torch.cuda.current_stream(dev))

        def step():
            for st in side:
                st.wait_stream(stream)
            for st, (out, ws, ch, it) in zip(side, work):
                _api.denoise_async(img, alpha, beta, passes, out=out, workspace=ws, changed=ch,
                                   iterations=it, stream=st)
            for st in side:
                stream.wait_stream(st)

        with torch.cuda.stream(stream):
            step()
        torch.cuda.synchronize()
        iters = int(work[0][3].item())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            g.replay()
            e0.record(stream)
            for _ in range(reps):
                g.replay()
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        return img.numel() * iters * concurrent / (ms * 1e-3)
    finally:
        _api.set_tuning_class(beta, cls, saved)


def autotune(betas=(1, 2), classes=(0, 1, 2), density=0.3, alpha=20, device="cuda:0",
             out_path=DEFAULT_CACHE, apply=True, log=print):
    dev = torch.device(device)
    shapes = _api.shapes()
    stream = torch.cuda.Stream(device=dev)
    result = {"device": torch.cuda.get_device_name(dev), "shapes": shapes, "choice": {}}
    for cls in classes:
        side = CLASS_SIDES[cls]
        img = torch.from_numpy(synth.noisy_image(side, side, density, 900 + cls)).to(dev)
        for beta in betas:
            rates = []
            for si, (T, R, W) in enumerate(shapes):
                r = _time_shape(img, alpha, beta, si, T, stream)
                rates.append(r)
                if log:
                    log("beta %d class %d shape %d %s: %.3f Tpx*pass/s" % (beta, cls, si, (T, R, W), r / 1e12))
            best = max(range(len(shapes)), key=lambda i: rates[i])
            result["choice"].setdefault(str(beta), {})[str(cls)] = {
                "shape": best, "rate_px_pass_s": rates[best],
                "rates": [round(x / 1e9, 2) for x in rates],
                "tuner": "autotune.py: three concurrent pass loops (k = 16) as "
                         "phgrms_denoise_async launches them, seeded image of the "
                         "class's side, %d%% noise" % round(100 * density)}
            if apply:
                _api.set_tuning_class(beta, cls, best)
    if out_path:
        # the classes and betas tuned here over the cache's other entries
        data = {}
        if os.path.exists(out_path):
            with open(out_path) as f:
                data = json.load(f)
        data["device"] = result["device"]
        data["shapes"] = [list(s) for s in shapes]
        for beta, per in result["choice"].items():
            data.setdefault("choice", {}).setdefault(beta, {}).update(per)
        with open(out_path, "w") as f:
            json.dump(data, f, indent=1)
    return result


def tune_batch(betas=(1, 2), n=512, seed=7, device="cuda:0", reps=3, apply=True, log=print):
    """The batch path's own shape per beta (the same for every size class):
    time phgrms_batch_run on `n` images drawn like the 512-image mixed
    workload (sides log-uniform in [128, 4096], density U[5%,60%], alpha
    U{10..40}, beta U{1,2}, k = 32) with every compiled shape for one beta
    while the other betas keep their current shape, one beta after the
    other, and keep the fastest (the change-tracking shapes keep change maps
    per image, the skipping shapes also one set of tile lists per launch).
    Returns {beta: {"shape", "rates"}}."""
    import time
    dev = torch.device(device)
    full = synth.batch_512(n=n, seed=seed)
    imgs = synth.generate_many(full, workers=min(16, os.cpu_count() or 1))
    specs = [(s.rows, s.cols, s.alpha, s.beta, s.k) for s in full]
    nshapes = len(_api.shapes())
    stream = torch.cuda.Stream(device=dev)

    def rate():
        b = _api.Batch(specs, device=dev)
        ain, aout = b.new_arena(), b.new_arena()
        for i, img in enumerate(imgs):
            b.view(ain, i).copy_(torch.from_numpy(img).to(dev))
        stream.wait_stream(torch.cuda.current_stream(dev))
        b.run(ain, aout, stream=stream)     # uploads and captures
        torch.cuda.synchronize()
        px_iters = sum(sp[0] * sp[1] * r[0] for sp, r in zip(specs, b.results()))
        t0 = time.perf_counter()
        for _ in range(reps):
            b.run(ain, aout, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        b.close()
        return px_iters / dt

    out = {}
    for beta in betas:
        saved = [_api.get_batch_tuning_class(beta, c) for c in range(3)]
        rates = []
        for si in range(nshapes):
            _api.set_batch_tuning_class(beta, -1, si)
            rates.append(rate())
            if log:
                log("batch beta %d shape %d: %.0f Mpx*iter/s" % (beta, si, rates[-1] / 1e6))
        best = max(range(nshapes), key=lambda i: rates[i])
        out[str(beta)] = {"shape": best, "rates": [round(x / 1e6, 1) for x in rates]}
        if apply:
            _api.set_batch_tuning_class(beta, -1, best)
        else:
            for c, sh in enumerate(saved):
                _api.set_batch_tuning_class(beta, c, sh)
    return out


def load(path=DEFAULT_CACHE) -> bool:
    """Apply a tuning cache (the library's own reader, phgrms_load_tuning);
    False if there is none."""
    if not os.path.exists(path):
        return False
    _api.load_tuning(path)
    return True


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--betas", default="1,2")
    ap.add_argument("--classes", default="0,1,2")
    ap.add_argument("--batch-only", action="store_true",
                    help="tune only the batch path's shapes and add them to the cache")
    ap.add_argument("--batch-images", type=int, default=512)
    a = ap.parse_args()
    betas = [int(x) for x in a.betas.split(",")]
    if a.batch_only:
        data = {}
        if os.path.exists(a.out):
            with open(a.out) as f:
                data = json.load(f)
        load(a.out)
        data["batch_choice"] = tune_batch(betas=betas, n=a.batch_images)
        with open(a.out, "w") as f:
            json.dump(data, f, indent=1)
    else:
        autotune(betas=betas, classes=[int(x) for x in a.classes.split(",")], out_path=a.out)
