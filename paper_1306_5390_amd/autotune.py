"""Autotuner: pick, per beta and image size class, the compiled kernel shape
(passes per launch, rows per wave, waves per workgroup) that runs the pass
loop fastest on this GPU, and keep the choice in a JSON cache.

    python -m paper_1306_5390_amd.autotune [--out tuning.json] [--betas 1,2]

For each (beta, size class) it times the first 16 passes of the pass loop
with every shape, three independent runs at a time on three streams,
launched as the pass loop launches them (replayed as a graph), on a seeded
noisy image of a representative size, and keeps the shape with the most
pixel-passes per second.  Results never depend on the
shape; only speed does.
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
    """Pixel-passes per second of `concurrent` independent runs of `passes`
    passes from `img`, each on its own stream and launched as the pass loop
    launches them (T passes per launch; change maps for a change-tracking
    shape), captured as one graph and replayed.  Concurrent runs measure
    throughput as the benchmark, batches and servers use the GPU, not the
    latency of a lone run."""
    dev = img.device
    track = _api.shape_tracks_changes(shape)
    side = [torch.cuda.Stream(device=dev) for _ in range(concurrent)]
    work = []
    for _ in range(concurrent):
        work.append(((torch.empty_like(img), torch.empty_like(img)), _api.count_slots(T, dev),
                     _api.change_maps(img.shape[0], img.shape[1], dev) if track else None))

    def sequence(st, bufs, slots, maps):
        src, n, p = img, 0, 0
        while p < passes:
            m = min(T, passes - p)
            _api.run_passes(src, bufs[n % 2], alpha, beta, m, shape, slots, stream=st,
                            pass_index=n, maps=maps)
            src, n, p = bufs[n % 2], n + 1, p + m

    # the count slots were zeroed on the current stream
    stream.wait_stream(torch.cuda.current_stream(dev))

    def step():
        for st in side:
            st.wait_stream(stream)
        for st, (bufs, slots, maps) in zip(side, work):
            sequence(st, bufs, slots, maps)
        for st in side:
            stream.wait_stream(st)

    with torch.cuda.stream(stream):
        step()
    torch.cuda.synchronize()
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
    return img.numel() * passes * concurrent / (ms * 1e-3)


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
                "rates": [round(x / 1e9, 2) for x in rates]}
            if apply:
                _api.set_tuning_class(beta, cls, best)
    if out_path:
        with open(out_path, "w") as f:
            json.dump(result, f, indent=1)
    return result


def load(path=DEFAULT_CACHE) -> bool:
    """Apply a tuning cache; False if there is none."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        data = json.load(f)
    n = _api.load_library().phgrms_num_shapes()
    for beta, per in data.get("choice", {}).items():
        for cls, c in per.items():
            if 0 <= int(c["shape"]) < n:
                _api.set_tuning_class(int(beta), int(cls), int(c["shape"]))
    return True


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--betas", default="1,2")
    ap.add_argument("--classes", default="0,1,2")
    a = ap.parse_args()
    autotune(betas=[int(x) for x in a.betas.split(",")],
             classes=[int(x) for x in a.classes.split(",")], out_path=a.out)
