"""The asynchronous entry points captured into a HIP graph (through torch's
CUDAGraph) and replayed several times, with other work and
synchronisations between the replays: every replay's image, per-pass
counts and iteration count equal the oracle's.  The pass loop clears its
count slots and tile lists with kernels (no memset nodes), so a replay
starts from the same state as the first run."""
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


@pytest.mark.parametrize("shape", [3, 6, 7, 12])
@pytest.mark.parametrize("stop_on_cycle", [False, True])
def test_graph_replays_equal_the_oracle(shape, stop_on_cycle):
    # (with the period-2 stop a shape of several passes per launch falls
    # back to the one-pass dense shape)
    m = phg()
    rows, cols, alpha, beta, k = 600, 900, 20, 2, 12
    img_np = synth.noisy_image(rows, cols, 0.3, 21)
    if stop_on_cycle:
        ref, rit, rch = oracle.denoise_cycle(img_np, alpha, beta, k)
    else:
        ref, rit, rch = oracle.denoise(img_np, alpha, beta, k)
    cls = m.size_class(rows * cols)
    saved = m.get_tuning_class(beta, cls)
    m.set_tuning_class(beta, cls, shape)
    try:
        img = torch.from_numpy(img_np).to(DEV)
        out = torch.empty_like(img)
        ws = torch.empty(m.workspace_bytes(rows, cols, alpha, beta, k), dtype=torch.uint8,
                         device=DEV)
        ch = torch.zeros(k, dtype=torch.int64, device=DEV)
        it = torch.zeros(1, dtype=torch.int32, device=DEV)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            m.denoise_async(img, alpha, beta, k, out=out, workspace=ws, changed=ch,
                            iterations=it, stream=s, stop_on_cycle=stop_on_cycle)
        other = torch.from_numpy(synth.noisy_image(200, 300, 0.4, 22)).to(DEV)
        for rep in range(4):
            print("shape", shape, "cycle", stop_on_cycle, "replay", rep, flush=True)
            out.fill_(0xAB)
            ch.fill_(-1)
            it.fill_(-1)
            ws.fill_(0x5A)          # stale workspace: the replay must not depend on it
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            n = int(it.item())
            assert n == rit, (rep, n, rit)
            assert ch.cpu().tolist()[:n] == list(rch[:n]), rep
            assert np.array_equal(out.cpu().numpy(), ref), rep
            # other work between replays, on the default stream
            m.denoise(other, 30, 1, 5)
            torch.cuda.synchronize()
    finally:
        m.set_tuning_class(beta, cls, saved)
