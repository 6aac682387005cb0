"""Benchmark of the P-HGRMS pass loop on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload (`large8192`): one 8192x8192 seeded synthetic image at 50%
salt-and-pepper density, alpha 20, beta 2, k = 32 (iterate until a pass
changes nothing, cap 32).  One step = one denoise of the image with the
tuned kernel shape, input resident in device memory, results (image,
iteration count, changed counts) left in device memory, replayed as a HIP
graph.  Throughput is Mpixel*iter/s: rows*cols*iterations per second.

Other workloads: `large16384` (16384^2, same parameters), `sweep2048`
(2048^2 at 30%, alpha in {10, 20, 40} x beta in {1, 2}, six runs per step
on three streams), `single481` (481x321, 10%, alpha 20, beta 1, k 10).

The JSON line also carries:
  roofline      the pass kernel as the step launches it (its average launch
                duration from HIP events on its stream) against HBM: 2 B per
                pixel and pass (read I, write I') over 8 TB/s -- for a shape
                that skips unchanged tiles this is a dense-equivalent rate;
                traffic: measured HBM bytes per launch (rocprof counters)
  roofline_dense  the same for the dense one-pass kernel (every pixel of
                every pass tested, every byte moved)
  kernels       the whole pass loop with each kernel shape: one launch per
                pass with a host read-back per pass (the plain path), one
                pass per launch dense, 2 and 4 passes per launch (temporal
                blocking), change tracking, tile skipping
  sync_call     one synchronous denoise call of the first run (results and
                counts copied to the host), median wall time
  ceilings      the two ceilings measured on this GPU with the library's
                calibration kernels: stream-copy bandwidth and the VALU issue
                rate; each roofline also gives its fraction of the measured
                copy, and the dense kernel its VALU issue fraction
  cpu_baseline  the CPU oracle (single-threaded C, pinned to one core) on a
                bounded sample of the same workload
  batch         the 512-image mixed batch against per-image launches
  serve         the continuous-batching server under Poisson arrivals, at
                saturation, and against plain per-image calls
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpixel·iter/s & % HBM roofline, batched vs per-image launch; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_1306_5390_amd", "csrc", "pass_kernel.hpp")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large8192",
                    choices=["large8192", "large16384", "sweep2048", "single481"])
    ap.add_argument("--graph", type=int, default=1, help="replay each step as a HIP graph")
    ap.add_argument("--streams", type=int, default=3,
                    help="streams the step's independent denoise runs are spread over "
                         "(round-robin; 1: one after another)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernels", type=int, default=1,
                    help="time the pass loop with each kernel shape (0: skip)")
    ap.add_argument("--kernel-reps", type=int, default=5)
    ap.add_argument("--ceilings", type=int, default=1,
                    help="measure stream-copy bandwidth and VALU issue rate (0: skip)")
    ap.add_argument("--ceilings-only", action="store_true",
                    help="print only the measured ceilings, the VALU rates at 1-16 waves "
                         "per SIMD, and exit")
    ap.add_argument("--cycle", type=int, default=1,
                    help="also time each run with the opt-in period-2 stop (not the headline)")
    ap.add_argument("--quality", type=int, default=1,
                    help="noise / denoise / PSNR section on 481x321 images (0: skip)")
    ap.add_argument("--batch", type=int, default=512,
                    help="images in the batched-vs-per-image section (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="seconds of Poisson arrivals per rate in the serving section (0: skip)")
    ap.add_argument("--serve-rates", default="200,500,1000,2000,5000")
    ap.add_argument("--serve-passes", type=int, default=4,
                    help="server passes per step: 4 (default), 2, 1, 0 tuned shape, -1 adaptive")
    ap.add_argument("--serve-e2e-rates", default="200,2000",
                    help="rates of the end-to-end serving rows (host buffers, PCIe included)")
    ap.add_argument("--serve-cap-gb", type=float, default=200.0,
                    help="admission cap of the server (GB)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a plain 64 MiB device copy (scales rocprof byte counters)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="no GPU work: summarise rocprofv3 --pmc runs of this benchmark "
                         "(directories of FETCH_SIZE, WRITE_SIZE [, SQ counters]) into "
                         "profiles/pass_kernel_<workload>_traffic.json and print a table")
    return ap.parse_args()


def kernel_source_hash() -> str:
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload, shape, avg_launch_s):
    """HBM bytes per pass-kernel launch of `shape` from rocprof FETCH_SIZE /
    WRITE_SIZE runs of this workload (profiles/), each scaled by the same
    counter on a 64 MiB copy; (None, reason) when there are none or they
    predate the current kernel source."""
    path = os.path.join(ROOT, "profiles", "pass_kernel_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None, {"stale": True, "measured_for": t.get("kernel_source_sha256")}
    row = t.get("shapes", {}).get(str(shape))
    if row is None:
        return None, None
    b = row["bytes_per_launch"]
    return round(b / avg_launch_s / 1e9, 1), {
        "bytes_per_launch": b, "algorithmic_bytes_per_launch": row["algorithmic_bytes_per_launch"],
        "ratio_to_algorithmic": round(b / row["algorithmic_bytes_per_launch"], 4),
        "fetch_scale": t["fetch_scale"], "write_scale": t["write_scale"], "unit": "GB/s"}


def _dispatches(csv_dir):
    """{dispatch id: (kernel name, {counter: value})} of a rocprofv3 --pmc
    output directory (csv)."""
    import csv
    import glob
    out = {}
    for path in glob.glob(os.path.join(csv_dir, "*counter_collection.csv")):
        with open(path) as f:
            for r in csv.DictReader(f):
                d = out.setdefault(int(r["Dispatch_Id"]), (r["Kernel_Name"], {}))
                d[1][r["Counter_Name"]] = d[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def _pass_signature(name):
    """(beta, T, rows, waves, TRACK) of a pass_kernel name, else None."""
    import re
    m = re.search(r"pass_kernel<(\d+), (\d+), (\d+), (\d+), (\d+), (false|true)>", name)
    if not m or "multi_pass" in name:
        return None
    return tuple(int(m.group(i)) for i in range(1, 6))


def _runs(disp):
    """Pass loops of the benchmark in dispatch order: each begins with the
    loop's clearing kernel (zero2_u64_kernel) and ends with finish_kernel;
    the plain path (zero_u64_kernel) is left out."""
    runs, cur = [], None
    for i in sorted(disp):
        name = disp[i][0]
        if "zero2_u64_kernel" in name:
            cur = []
        elif "finish_kernel" in name and cur is not None:
            runs.append(cur)
            cur = None
        elif cur is not None and _pass_signature(name) is not None:
            cur.append(i)
    return runs


def summarize_counters(workload, dirs, out_path=None):
    """HBM bytes per pass-kernel launch of every shape the benchmark's
    kernel section ran (FETCH_SIZE and WRITE_SIZE runs, each scaled by the
    same counter on the 64 MiB calibration copies), and, with a third
    directory, SQ counters per launch; written to
    profiles/pass_kernel_<workload>_traffic.json."""
    import paper_1306_5390_amd as phg
    spec = workload_specs(workload)[0]
    shapes = phg.shapes()
    sig_of = {}
    # the first two launches of a change-tracking loop run the dense
    # one-pass kernel of shape 3, (1, 8, 4); a skipping shape's loop then
    # runs its list-building kernel (TRACK 2) and its listed one (TRACK 3)
    T3, R3, W3 = shapes[3]
    dense0 = (spec.beta, T3, R3, W3, 0)
    for s, (T, R, W) in enumerate(shapes):
        tr = 2 if phg.shape_skips_unchanged(s) else 1 if phg.shape_tracks_changes(s) else 0
        sig = {(spec.beta, T, R, W, tr)} if tr < 2 else {(spec.beta, 1, R, W, t) for t in (2, 3)}
        if tr > 0:
            sig.add(dense0)
        sig_of[frozenset(sig)] = s
    res = {}
    counters = []
    for d in dirs:
        disp = _dispatches(d)
        copies = [disp[i][1] for i in sorted(disp) if "copyBuffer" in disp[i][0]][-3:]
        counters.append((disp, copies))
    (fd, fcopies), (wd, wcopies) = counters[0], counters[1]
    fetch_scale = 65536.0 / (sum(c["FETCH_SIZE"] for c in fcopies) / len(fcopies))
    write_scale = 65536.0 / (sum(c["WRITE_SIZE"] for c in wcopies) / len(wcopies))
    for disp, key, scale in ((fd, "FETCH_SIZE", fetch_scale), (wd, "WRITE_SIZE", write_scale)):
        for run in _runs(disp):
            sig = frozenset(_pass_signature(disp[i][0]) for i in run)
            s = sig_of.get(sig)
            if s is None:
                continue
            r = res.setdefault(str(s), {"runs": 0, "launches": len(run), "FETCH_SIZE": [],
                                        "WRITE_SIZE": []})
            r[key].append([disp[i][1][key] * 1024.0 * scale for i in run])
    sq = {}
    if len(dirs) > 2:
        sd = counters[2][0]
        for run in _runs(sd):
            sig = frozenset(_pass_signature(sd[i][0]) for i in run)
            s = sig_of.get(sig)
            if s is None or str(s) in sq:
                continue
            names = sorted(sd[run[0]][1])
            sq[str(s)] = {n: [round(sd[i][1][n], 3) for i in run] for n in names}
    out_shapes = {}
    T_of = {str(s): shapes[s][0] for s in range(len(shapes))}
    for s, r in res.items():
        per_launch_f = [sum(x) / len(x) for x in zip(*r["FETCH_SIZE"])]
        per_launch_w = [sum(x) / len(x) for x in zip(*r["WRITE_SIZE"])]
        per_launch = [a + b for a, b in zip(per_launch_f, per_launch_w)]
        row = {"bytes_per_launch": sum(per_launch) / len(per_launch),
               "algorithmic_bytes_per_launch": 2.0 * spec.rows * spec.cols * T_of[s],
               "bytes_per_launch_in_order": [round(x) for x in per_launch],
               "launches": len(per_launch)}
        if s in sq:
            row["sq_per_launch_in_order"] = sq[s]
        out_shapes[s] = row
    data = {"workload": workload, "kernel_source_sha256": kernel_source_hash(),
            "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
            "copy64MiB_fetch_kib": [c["FETCH_SIZE"] for c in fcopies],
            "copy64MiB_write_kib": [c["WRITE_SIZE"] for c in wcopies],
            "shapes": out_shapes}
    path = out_path or os.path.join(ROOT, "profiles", "pass_kernel_%s_traffic.json" % workload)
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print("| shape | kind | launches | HBM bytes per launch | algorithmic | ratio |")
    print("|---|---|---|---|---|---|")
    for s, row in sorted(out_shapes.items(), key=lambda kv: int(kv[0])):
        print("| %s | %s | %d | %.0f | %.0f | %.4f |" % (
            s, shape_name(phg, int(s))["kind"], row["launches"], row["bytes_per_launch"],
            row["algorithmic_bytes_per_launch"],
            row["bytes_per_launch"] / row["algorithmic_bytes_per_launch"]))
    print("fetch scale %.4f, write scale %.4f -> %s" % (fetch_scale, write_scale, path))


def host_cpu():
    """Logical CPUs of the host and its CPU model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def _oracle_on_core(args):
    """Child process: pin to one CPU, run the oracle on the band, return its
    seconds and iteration count."""
    cpu, band, alpha, beta, k = args
    os.sched_setaffinity(0, {cpu})
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    _, it, _ = oracle.denoise(band, alpha, beta, k)
    return time.perf_counter() - t0, it


def cpu_baseline(specs, images, band_rows=1024, band_cols=2048):
    """The oracle, single-threaded and pinned to one core (in a child
    process), on the first band_rows x band_cols of each image with every
    (alpha, beta) of the workload and its full k: about 10-30 s of CPU work."""
    import multiprocessing as mp
    cpus = sorted(os.sched_getaffinity(0))
    cpu = cpus[0]
    px_iters, dt = 0, 0.0
    with mp.get_context("spawn").Pool(1) as pool:
        for spec, img in zip(specs, images):
            band = img[: min(band_rows, img.shape[0]), : min(band_cols, img.shape[1])].copy()
            sec, it = pool.apply(_oracle_on_core, ((cpu, band, spec.alpha, spec.beta, spec.k),))
            px_iters += band.size * it
            dt += sec
        pool.close()
        pool.join()
    nproc, model = host_cpu()
    rows = min(band_rows, specs[0].rows)
    cols = min(band_cols, specs[0].cols)
    return {"value": round(px_iters / dt / 1e6, 2), "unit": "Mpixel·iter/s", "cores": 1,
            "kind": "oracle",
            "sample": "first %dx%d band of each image of the workload, every (alpha, beta), "
                      "full k; %.1f s on one pinned core" % (rows, cols, dt),
            "pinned_cpu": cpu, "nproc": nproc, "cpu_model": model}


def shape_name(phg, s):
    T, R, W = phg.shapes()[s]
    kind = ("skipping" if phg.shape_skips_unchanged(s) else
            "tracked" if phg.shape_tracks_changes(s) else "dense")
    return {"shape": s, "passes_per_launch": T, "rows_per_wave": R, "waves": W, "kind": kind}


def time_denoise(phg, spec, d_in, dev, shape, reps):
    """The whole pass loop with kernel shape `shape` (forced for the image's
    beta and size class), as phgrms_denoise_async enqueues it, captured as a
    graph and replayed `reps` times between two events on its stream.
    Returns (ms per run, iterations, launches, output)."""
    import torch
    cls = phg.size_class(spec.rows * spec.cols)
    saved = phg.get_tuning_class(spec.beta, cls)
    phg.set_tuning_class(spec.beta, cls, shape)
    try:
        ws = torch.empty(phg.workspace_bytes(spec.rows, spec.cols, spec.alpha, spec.beta, spec.k),
                         dtype=torch.uint8, device=dev)
        out = torch.empty_like(d_in)
        ch = torch.zeros(max(spec.k, 1), dtype=torch.int64, device=dev)
        it = torch.zeros(1, dtype=torch.int32, device=dev)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            phg.denoise_async(d_in, spec.alpha, spec.beta, spec.k, out=out, workspace=ws,
                              changed=ch, iterations=it, stream=s)
        torch.cuda.synchronize()
        iters = int(it.item())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            phg.denoise_async(d_in, spec.alpha, spec.beta, spec.k, out=out, workspace=ws,
                              changed=ch, iterations=it, stream=s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s):
            g.replay()
            e0.record(s)
            for _ in range(reps):
                g.replay()
            e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        T = phg.shapes()[shape][0]
        launches = (spec.k + T - 1) // T
        assert int(it.item()) == iters
        return ms, iters, launches, out
    finally:
        phg.set_tuning_class(spec.beta, cls, saved)


def time_sync_call(phg, spec, d_in, reps=5, warmup=2):
    """One synchronous phgrms_denoise call (the whole loop, then the changed
    counts and the iteration count copied to the host), wall clock around
    the call, median of `reps` after `warmup` calls."""
    import torch
    ws = torch.empty(phg.workspace_bytes(spec.rows, spec.cols, spec.alpha, spec.beta, spec.k),
                     dtype=torch.uint8, device=d_in.device)
    out = torch.empty_like(d_in)
    ts, iters = [], 0
    for r in range(warmup + reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, iters, _ = phg.denoise(d_in, spec.alpha, spec.beta, spec.k, out=out, workspace=ws)
        if r >= warmup:
            ts.append(time.perf_counter() - t0)
    ts.sort()
    ms = ts[len(ts) // 2] * 1e3
    return {"ms_median": round(ms, 4), "iterations": iters, "reps": reps,
            "Mpx_iter_s": round(spec.rows * spec.cols * iters / (ms * 1e-3) / 1e6, 1)}, out


def time_plain(phg, spec, d_in, reps=3):
    """phgrms_denoise_plain (one launch per pass, a host read-back of the
    changed count after each), wall clock, median of `reps`."""
    import torch
    ws = torch.empty(phg.workspace_bytes(spec.rows, spec.cols, spec.alpha, spec.beta, spec.k),
                     dtype=torch.uint8, device=d_in.device)
    out = torch.empty_like(d_in)
    ts, iters = [], 0
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, iters, _ = phg.denoise(d_in, spec.alpha, spec.beta, spec.k, out=out, workspace=ws,
                                  plain=True)
        if r:
            ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2] * 1e3, iters, out


def measured_valu(workload, shape):
    """Mean VALU wave-instructions per pass-kernel launch of `shape` from the
    rocprof SQ_INSTS_VALU run of this workload (profiles/), or None when
    there is none or it predates the current kernel source."""
    path = os.path.join(ROOT, "profiles", "pass_kernel_%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    v = t.get("shapes", {}).get(str(shape), {}).get("sq_per_launch_in_order", {}).get("SQ_INSTS_VALU")
    return sum(v) / len(v) if v else None


VALU_KINDS = ("v_add_u32", "v_lerp_u8", "v_xor_b32", "v_bitop3_b32", "v_add3_u32",
              "v_alignbyte_b32", "v_pk_add_u16", "v_dot4_u32_u8", "band_test_mix")


def ceilings_section(phg, dev, copy_bytes=1 << 30, reps=10, waves_per_simd=(8,)):
    """The two ceilings measured on this GPU with the library's calibration
    kernels (HIP events on their stream): stream-copy bandwidth (2 B moved
    per byte copied) and the VALU issue rate of each integer instruction
    the pass kernels issue most, against the specification's figures."""
    import torch
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count
    st = torch.cuda.Stream()
    src = torch.full((copy_bytes,), 7, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()

    def timed(fn):
        ts = []
        for i in range(3 + reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn()
            e1.record(st)
            e1.synchronize()
            if i >= 3:
                ts.append(e0.elapsed_time(e1) * 1e-3)
        ts.sort()
        return ts[len(ts) // 2], ts[0]

    with torch.cuda.stream(st):
        med, best = timed(lambda: phg.calib_copy(src, dst, stream=st))
    torch.cuda.synchronize()
    assert torch.equal(dst[:: 1 << 20], src[:: 1 << 20])
    copy = {"bytes_copied": copy_bytes, "GB_s_median": round(2 * copy_bytes / med / 1e9, 1),
            "GB_s_best": round(2 * copy_bytes / best / 1e9, 1), "spec_GB_s": HBM_PEAK_GBS,
            "frac_of_spec": round(2 * copy_bytes / med / 1e9 / HBM_PEAK_GBS, 4)}
    del src, dst
    # one workgroup of 4 waves per CU puts one wave on each SIMD
    out = torch.empty(cus * max(waves_per_simd) * 256, dtype=torch.int32, device=dev)
    spec_rate = cus * 4 * 2.4e9 / 4       # wave64 VALU: 4 cycles per SIMD at 2.4 GHz
    valu = {"waves_per_simd": 8, "spec_wave_instr_per_s": spec_rate}
    by_occupancy = {}
    for wps in waves_per_simd:
        blocks = cus * wps
        for kind, name in enumerate(VALU_KINDS):
            trips = 1024
            with torch.cuda.stream(st):
                per_wave = phg.calib_valu(out, blocks, trips, kind, stream=st)
                med, best = timed(lambda: phg.calib_valu(out, blocks, trips, kind, stream=st))
            rate = blocks * 4 * per_wave / med
            by_occupancy.setdefault(str(wps), {})[name] = round(rate / 1e9, 1)
            if wps == 8:
                valu[name] = {"instr_per_wave": per_wave, "wave_instr_per_s": round(rate, -6),
                              "T_lane_ops_per_s": round(rate * 64 / 1e12, 2),
                              "frac_of_spec": round(rate / spec_rate, 4)}
    if len(waves_per_simd) > 1:
        valu["G_wave_instr_per_s_by_waves_per_simd"] = by_occupancy
    torch.cuda.synchronize()
    return {"copy": copy, "valu": valu, "cus": cus}


def roofline_of(spec, ms, launches, T, traffic=None, traffic_detail=None, kernel="pass_kernel",
                dense_equivalent=False):
    """HBM roofline of one pass-kernel launch: 2 B per pixel and pass."""
    avg_s = ms * 1e-3 / launches
    alg_bytes = 2.0 * spec.rows * spec.cols * T
    achieved = alg_bytes / avg_s / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
         "kernel": kernel, "avg_launch_us": round(avg_s * 1e6, 2),
         "algorithmic_bytes_per_launch": int(alg_bytes),
         "launches": launches, "dense_equivalent": dense_equivalent}
    if traffic_detail is not None:
        r["traffic_detail"] = traffic_detail
    return r


def kernels_section(phg, spec, d_in, dev, reps, workload, ref_out):
    """The whole pass loop on the workload's first run with each kernel
    shape kind, and the plain path; every output must equal `ref_out`."""
    import torch
    pick = {}
    for s in range(len(phg.shapes())):
        T, R, W = phg.shapes()[s]
        n = shape_name(phg, s)
        key = None
        if n["kind"] == "dense" and (R, W) == (8, 4) and T == 1:
            key = "dense_T1"
        elif n["kind"] == "dense" and (R, W) == (16, 4) and T in (2, 4):
            key = "dense_T%d" % T
        elif n["kind"] == "tracked" and (R, W) == (8, 4):
            key = "tracked"
        elif n["kind"] == "skipping":
            key = "skipping_%dw" % W
        if key and key not in pick:
            pick[key] = s
    rows = {}
    for key, s in pick.items():
        ms, iters, launches, out = time_denoise(phg, spec, d_in, dev, s, reps)
        assert torch.equal(out, ref_out), "shape %d differs from the headline output" % s
        T = phg.shapes()[s][0]
        traffic, detail = measured_traffic(workload, s, ms * 1e-3 / launches)
        rows[key] = {**shape_name(phg, s), "ms_per_run": round(ms, 4), "iterations": iters,
                     "Mpx_iter_s": round(spec.rows * spec.cols * iters / (ms * 1e-3) / 1e6, 1),
                     "hbm_frac_dense_equivalent": round(
                         2.0 * spec.rows * spec.cols * iters / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "avg_launch_us": round(ms * 1e3 / launches, 2), "launches": launches,
                     "traffic": traffic}
        if detail:
            rows[key]["traffic_detail"] = detail
    ms, iters, out = time_plain(phg, spec, d_in)
    assert torch.equal(out, ref_out), "plain path differs from the headline output"
    rows["plain"] = {"kind": "one launch per pass, host read-back of each pass's count",
                     "ms_per_run": round(ms, 4), "iterations": iters,
                     "Mpx_iter_s": round(spec.rows * spec.cols * iters / (ms * 1e-3) / 1e6, 1),
                     "hbm_frac_dense_equivalent": round(
                         2.0 * spec.rows * spec.cols * iters / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return rows, pick


def _drain(srv, n_expect, t_limit, on_done):
    done = 0
    t0 = time.perf_counter()
    while done < n_expect:
        for rid in srv.next_done():
            on_done(rid)
            done += 1
        if time.perf_counter() - t0 > t_limit:
            raise RuntimeError("server did not finish: %s" % srv.stats())


def serve_section(seconds, rates, dev, e2e_rates=(), passes=4, cap_gb=200.0):
    """Continuous-batching server under Poisson arrivals.  Request i denoises
    pool image i mod 256 (device resident; sides log-uniform in [256, 8192],
    density U[5%,50%], alpha 20, beta U{1,2}, k = 16).  Latency is submit to
    completion on the device, measured by the server.  Each rate runs for
    `seconds` of arrivals.  The saturation row keeps 64 requests queued for
    `seconds` (served capacity); the plain row denoises the 256 pool images
    one after another with phgrms_denoise_plain (one launch per pass, a host
    read-back per pass).  The end-to-end rows (`e2e_rates`) submit the same
    pool from page-locked host memory: the server copies each image in and
    its result out over PCIe, inside the request's latency."""
    import numpy as np
    import torch
    import paper_1306_5390_amd as phg
    from paper_1306_5390_amd import synth

    pool = synth.serve_pool(n=256, seed=6)
    imgs = synth.generate_many(pool, workers=min(16, os.cpu_count() or 1))
    d_pool = [torch.from_numpy(im).to(dev) for im in imgs]
    del imgs
    free, _total = torch.cuda.mem_get_info()
    cap = int(cap_gb * 1e9)
    # the cap plus the server's descriptor slots, within the free memory
    arena = int(min(cap + (1 << 30), free - (8 << 30)))
    srv = phg.Server(arena, device=dev, max_active=1024, passes_per_step=passes,
                     cap_bytes=min(cap, arena - (1 << 30)))
    # warm-up: every pool image once
    for i, spec in enumerate(pool):
        srv.submit(d_pool[i], spec.alpha, spec.beta, spec.k)
    _drain(srv, len(pool), 120, srv.release)

    def run_rate(lam, seed, host=None):
        arrivals = synth.poisson_arrivals(lam, max(1, int(lam * seconds)), seed=seed)
        lat, px_iters, n, submitted, done, moved = [], 0, len(arrivals), 0, 0, 0
        t_start = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t_start
            while submitted < n and arrivals[submitted] <= now:
                j = submitted % len(pool)
                spec = pool[j]
                if host is None:
                    srv.submit(d_pool[j], spec.alpha, spec.beta, spec.k)
                else:
                    srv.submit_host(host[0][j], host[1][j], spec.alpha, spec.beta, spec.k)
                    moved += 2 * host[0][j].numel()
                submitted += 1
            for rid in srv.next_done():
                r = srv.poll(rid)
                lat.append(r[3])
                px_iters += r[0].numel() * r[1]
                srv.release(rid)
                done += 1
            if now > seconds * 20 + 60:
                raise RuntimeError("serving at %g req/s did not drain: %s" % (lam, srv.stats()))
        wall = time.perf_counter() - t_start
        lat_ms = np.array(lat) * 1e3
        row = {"rate_req_s": lam, "requests": n, "wall_s": round(wall, 3),
               "achieved_req_s": round(n / wall, 1),
               "Mpx_iter_s": round(px_iters / wall / 1e6, 1),
               "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
               "p99_ms": round(float(np.percentile(lat_ms, 99)), 3)}
        if host is not None:
            row["pcie_GB_s"] = round(moved / wall / 1e9, 2)
        return row

    results = [run_rate(lam, 60 + li) for li, lam in enumerate(rates)]

    # saturation: 64 requests always waiting
    lat, px_iters, submitted, done = [], 0, 0, 0
    depth = 64
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < seconds:
        while submitted - done < depth:
            j = submitted % len(pool)
            srv.submit(d_pool[j], pool[j].alpha, pool[j].beta, pool[j].k)
            submitted += 1
        for rid in srv.next_done():
            r = srv.poll(rid)
            lat.append(r[3])
            px_iters += r[0].numel() * r[1]
            srv.release(rid)
            done += 1
    wall = time.perf_counter() - t_start
    served_rate = px_iters / wall
    lat_ms = np.array(lat) * 1e3
    saturated = {"queue_depth": depth, "requests_completed": done, "wall_s": round(wall, 3),
                 "req_s": round(done / wall, 1), "Mpx_iter_s": round(served_rate / 1e6, 1),
                 "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                 "p99_ms": round(float(np.percentile(lat_ms, 99)), 3)}

    def on_tail(rid):
        srv.release(rid)
    _drain(srv, submitted - done, 120, on_tail)

    # plain per-image calls on the same 256 images
    ws = torch.empty(max(phg.workspace_bytes(s.rows, s.cols, s.alpha, s.beta, s.k) for s in pool),
                     dtype=torch.uint8, device=dev)
    outs = torch.empty(max(s.rows * s.cols for s in pool), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    px_plain = 0
    for j, s in enumerate(pool):
        o = outs[: s.rows * s.cols].view(s.rows, s.cols)
        _, it, _ = phg.denoise(d_pool[j], s.alpha, s.beta, s.k, out=o, workspace=ws, plain=True)
        px_plain += s.rows * s.cols * it
    torch.cuda.synchronize()
    plain_rate = px_plain / (time.perf_counter() - t0)
    del ws, outs

    e2e = []
    if e2e_rates:
        # the same pool in page-locked host memory, one host output per image
        h_pool = [t.cpu().pin_memory() for t in d_pool]
        h_out = [torch.empty_like(t).pin_memory() for t in h_pool]
        e2e = [run_rate(lam, 80 + li, host=(h_pool, h_out)) for li, lam in enumerate(e2e_rates)]
        del h_pool, h_out
    st = srv.stats()
    srv.close()
    return {"pool_images": len(pool), "arena_bytes": arena, "cap_bytes": min(cap, arena - (1 << 30)),
            "passes_per_step": passes, "seconds_per_rate": seconds, "rates": results,
            "saturated": saturated,
            "plain_per_image_Mpx_iter_s": round(plain_rate / 1e6, 1),
            "served_vs_plain": round(served_rate / plain_rate, 2),
            "end_to_end_host": e2e, "steps": st["steps"]}


def batch_section(n, steps, dev):
    """Batched path vs per-image launches on the 512-image mixed workload:
    sides log-uniform in [128, 4096], density U[5%,60%], alpha U{10..40},
    beta U{1,2}, k = 32."""
    import torch
    import paper_1306_5390_amd as phg
    from paper_1306_5390_amd import synth

    specs_full = synth.batch_512(n=n, seed=5)
    imgs = synth.generate_many(specs_full, workers=min(16, os.cpu_count() or 1))
    specs = [(s.rows, s.cols, s.alpha, s.beta, s.k) for s in specs_full]
    b = phg.Batch(specs, device=dev)
    ain = b.new_arena()
    for i, img in enumerate(imgs):
        b.view(ain, i).copy_(torch.from_numpy(img).to(dev))
    del imgs
    aout = b.new_arena()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())   # the arena copies above
    b.run(ain, aout, stream=stream)          # uploads descriptors, captures the graph
    torch.cuda.synchronize()
    res = b.results()
    px_iters = sum(s[0] * s[1] * r[0] for s, r in zip(specs, res))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        b.run(ain, aout, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    dt_batch = e0.elapsed_time(e1) * 1e-3 / steps
    # pixel-passes a launch sequence visits (every launch of an image up to
    # k, converged or not) against the passes that ran
    px_passes_planned = sum(s[0] * s[1] * s[4] for s in specs)
    # per-image comparators on the same images and outputs
    ws = torch.empty(max(phg.workspace_bytes(s[0], s[1], s[2], s[3], s[4]) for s in specs),
                     dtype=torch.uint8, device=dev)
    views_in = [b.view(ain, i) for i in range(n)]
    views_out = [b.view(aout, i, out=True) for i in range(n)]
    mism = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i, s in enumerate(specs):
            _, it, _ = phg.denoise(views_in[i], s[2], s[3], s[4], out=views_out[i], workspace=ws,
                                   stream=stream, plain=True)
            mism += it != res[i][0]
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i, s in enumerate(specs):
            phg.denoise_async(views_in[i], s[2], s[3], s[4], out=views_out[i], workspace=ws,
                              stream=stream)
    torch.cuda.synchronize()
    dt_fused = time.perf_counter() - t0
    hbm = 2.0 * px_iters / dt_batch / 1e9
    out = {
        "images": n, "total_pixels": int(sum(s[0] * s[1] for s in specs)),
        "launches_per_run": b.launches(),
        "batched_Mpx_iter_s": round(px_iters / dt_batch / 1e6, 1),
        "batched_ms": round(dt_batch * 1e3, 3),
        "per_image_plain_Mpx_iter_s": round(px_iters / dt_plain / 1e6, 1),
        "per_image_plain_ms": round(dt_plain * 1e3, 3),
        "per_image_fused_Mpx_iter_s": round(px_iters / dt_fused / 1e6, 1),
        "per_image_fused_ms": round(dt_fused * 1e3, 3),
        "speedup_vs_plain": round(dt_plain / dt_batch, 2),
        "speedup_vs_fused_per_image": round(dt_fused / dt_batch, 2),
        "iteration_mismatches": int(mism),
        "passes_run_of_planned": round(px_iters / px_passes_planned, 4),
        "roofline": {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(hbm / HBM_PEAK_GBS, 4),
                     "kernel": "multi_pass_kernel (whole batch run, events)",
                     "note": "2 B per pixel and pass that ran, over the run's duration"},
        "batch_shapes": {str(bb): [phg.get_batch_tuning_class(bb, c) for c in range(3)]
                         for bb in (1, 2)},
    }
    b.close()
    return out


def quality_section(dev, images=5, densities=(0.05, 0.10, 0.15, 0.20), alpha=20, beta=1, k=10):
    """The shape of the paper's Tables 1-2 (Section 3) on synthetic clean
    images of the segmentation benchmark's 481x321 frame: salt-and-pepper
    noise at 5-20 % (counter-based generator, on the GPU), the pass loop,
    PSNR against the clean image before and after, and the time of one
    denoise call (events, inputs resident).  The paper's images and its
    alpha, beta are not available; these stand in for them."""
    import torch
    import paper_1306_5390_amd as phg
    from paper_1306_5390_amd import synth
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    clean = [torch.from_numpy(synth.clean_image(321, 481, 100 + i)).to(dev) for i in range(images)]
    ws = torch.empty(phg.workspace_bytes(321, 481, alpha, beta, k), dtype=torch.uint8, device=dev)
    rows = []
    for rho in densities:
        tp, ts = synth.noise_thresholds(rho)
        ps_noisy, ps_out, ms, its, ps_cyc, its_cyc = [], [], [], [], [], []
        for i, c in enumerate(clean):
            noisy = phg.salt_pepper(c, 1000 + i, tp, ts, stream=stream)
            out = torch.empty_like(c)
            ch = torch.zeros(k, dtype=torch.int64, device=dev)
            it = torch.zeros(1, dtype=torch.int32, device=dev)
            stream.wait_stream(torch.cuda.current_stream())   # the buffers zeroed above
            for rep in range(4):             # warm, then three timed calls
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                with torch.cuda.stream(stream):
                    e0.record(stream)
                    phg.denoise_async(noisy, alpha, beta, k, out=out, workspace=ws,
                                      changed=ch, iterations=it, stream=stream)
                    e1.record(stream)
                torch.cuda.synchronize()
                if rep:
                    ms.append(e0.elapsed_time(e1))
            ps_noisy.append(phg.psnr(c, noisy))
            ps_out.append(phg.psnr(c, out))
            its.append(int(it.item()))
            # the same call with the opt-in period-2 stop
            with torch.cuda.stream(stream):
                phg.denoise_async(noisy, alpha, beta, k, out=out, workspace=ws, changed=ch,
                                  iterations=it, stream=stream, stop_on_cycle=True)
            torch.cuda.synchronize()
            ps_cyc.append(phg.psnr(c, out))
            its_cyc.append(int(it.item()))
        rows.append({"density": rho, "psnr_noisy_db": round(sum(ps_noisy) / images, 2),
                     "psnr_denoised_db": round(sum(ps_out) / images, 2),
                     "psnr_denoised_per_image": [round(x, 2) for x in ps_out],
                     "denoise_ms": round(sum(ms) / len(ms), 4), "iterations": its,
                     "stop_on_cycle": {"iterations": its_cyc,
                                       "psnr_denoised_db": round(sum(ps_cyc) / images, 2)}})
    return {"images": images, "shape": [321, 481], "alpha": alpha, "beta": beta, "k": k,
            "rows": rows}


def cycle_section(runs, stream):
    """The opt-in period-2 stop on the workload's own runs: per run, one
    denoise call under the paper's stop rule and one with stop_on_cycle
    (events on the call's stream, inputs resident, warm call first), with
    the passes each ran.  Not part of the headline, which keeps the
    paper's rule."""
    import torch
    import paper_1306_5390_amd as phg
    rows = []
    for (s, d_in, out, ws, ch, it) in runs:
        res = {}
        for mode, flag in (("paper_rule", False), ("stop_on_cycle", True)):
            ms = []
            for rep in range(4):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                with torch.cuda.stream(stream):
                    e0.record(stream)
                    phg.denoise_async(d_in, s.alpha, s.beta, s.k, out=out, workspace=ws,
                                      changed=ch, iterations=it, stream=stream,
                                      stop_on_cycle=flag)
                    e1.record(stream)
                torch.cuda.synchronize()
                if rep:
                    ms.append(e0.elapsed_time(e1))
            res[mode] = {"iterations": int(it.item()), "ms": round(sum(ms) / len(ms), 4)}
        rows.append({"alpha": s.alpha, "beta": s.beta, "k": s.k, **res})
    return rows


def workload_specs(name):
    from paper_1306_5390_amd import synth
    if name == "sweep2048":
        return synth.sweep_2048()
    if name == "single481":
        return [synth.single_481x321()]
    if name == "large8192":
        return [synth.large_single(8192)]
    if name == "large16384":
        return [synth.large_single(16384)]
    raise ValueError(name)


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(args.workload, args.summarize_counters)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this implementation has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1306_5390_amd as phg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    phg.load_library()
    if args.ceilings_only:
        print(json.dumps({"ceilings": ceilings_section(phg, dev, waves_per_simd=(1, 2, 4, 8, 16))}),
              flush=True)
        return
    from paper_1306_5390_amd import autotune
    tuned = autotune.load()          # the committed autotuner cache, if any
    specs = workload_specs(args.workload)
    print("workload %s: generating %d run(s)" % (args.workload, len(specs)), file=sys.stderr,
          flush=True)
    # one image per distinct seed/size (the sweep shares one image)
    cache = {}
    images = []
    for s in specs:
        key = (s.rows, s.cols, s.density, s.seed)
        if key not in cache:
            cache[key] = s.image()
        images.append(cache[key])
    d_imgs = {key: torch.from_numpy(img).to(dev) for key, img in cache.items()}
    runs = []
    for s in specs:
        key = (s.rows, s.cols, s.density, s.seed)
        d_in = d_imgs[key]
        ws = torch.empty(phg.workspace_bytes(s.rows, s.cols, s.alpha, s.beta, s.k),
                         dtype=torch.uint8, device=dev)
        out = torch.empty_like(d_in)
        ch = torch.zeros(max(s.k, 1), dtype=torch.int64, device=dev)
        it = torch.zeros(1, dtype=torch.int32, device=dev)
        runs.append((s, d_in, out, ws, ch, it))

    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())   # the buffers zeroed above
    # Several runs (the 2048^2 sweep): three at a time fill the GPU.
    nstreams = max(1, min(args.streams, len(runs)))
    side = [torch.cuda.Stream() for _ in range(nstreams)] if nstreams > 1 else None

    def step():
        # each run is the single-image path; with several streams run i goes
        # to stream i mod n, the streams forked from and joined to `stream`
        if side is None:
            for (s, d_in, out, ws, ch, it) in runs:
                phg.denoise_async(d_in, s.alpha, s.beta, s.k, out=out, workspace=ws,
                                  changed=ch, iterations=it, stream=stream)
            return
        for st in side:
            st.wait_stream(stream)
        for i, (s, d_in, out, ws, ch, it) in enumerate(runs):
            phg.denoise_async(d_in, s.alpha, s.beta, s.k, out=out, workspace=ws,
                              changed=ch, iterations=it, stream=side[i % nstreams])
        for st in side:
            stream.wait_stream(st)

    with torch.cuda.stream(stream):
        step()
    torch.cuda.synchronize()
    iters = [int(r[5].item()) for r in runs]
    px_iters = sum(r[0].rows * r[0].cols * i for r, i in zip(runs, iters))

    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            step()
        torch.cuda.synchronize()

    def replay():
        if graph is not None:
            graph.replay()
        else:
            with torch.cuda.stream(stream):
                step()

    for _ in range(args.warmup):
        replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = px_iters * args.steps / dt / 1e6
    # the graph replays must give the eager results
    iters2 = [int(r[5].item()) for r in runs]
    assert iters2 == iters, (iters, iters2)
    print("headline: %.1f Mpixel*iter/s, %.4f ms per step" % (value, ms_per_step),
          file=sys.stderr, flush=True)

    # ---- the dominant kernel and the kernel shapes ----------------------------
    # The first run's pass loop with each kernel shape (events on the stream
    # its kernels run on); the tuned shape's row is the headline step's own
    # launch sequence when the workload is one run.
    s0, d0, out0 = runs[0][0], runs[0][1], runs[0][2]
    tuned_shape = phg.get_tuning_class(s0.beta, phg.size_class(s0.rows * s0.cols))
    kernels, picked = None, {}
    ms_t, it_t, L_t, o_t = time_denoise(phg, s0, d0, dev, tuned_shape, args.kernel_reps)
    assert torch.equal(o_t, out0)
    T_t = phg.shapes()[tuned_shape][0]
    traffic, detail = measured_traffic(args.workload, tuned_shape, ms_t * 1e-3 / L_t)
    nm = shape_name(phg, tuned_shape)
    roofline = roofline_of(s0, ms_t, L_t, T_t, traffic, detail,
                           kernel="pass_kernel<beta=%d, T=%d, rows=%d, waves=%d, %s>" % (
                               s0.beta, T_t, nm["rows_per_wave"], nm["waves"], nm["kind"]),
                           dense_equivalent=nm["kind"] != "dense")
    if nm["kind"] != "dense":
        roofline["launch_kernels"] = (
            "launches 0-1: the dense one-pass kernel (1, 8, 4); then the shape's own"
            + (" (launch 2 builds the tile lists, later launches run the listed tiles)"
               if nm["kind"] == "skipping" else ""))
    roofline["run"] = {"alpha": s0.alpha, "beta": s0.beta, "k": s0.k, "iterations": it_t,
                       "ms_per_run": round(ms_t, 4)}
    # one synchronous call with its results read back to the host (hipEvents
    # are not needed: the call returns after its stream is synchronised)
    sync_call, o_s = time_sync_call(phg, s0, d0, reps=5 if s0.rows * s0.cols >= 1 << 24 else 10)
    assert torch.equal(o_s, out0)
    roofline_dense = None
    if args.kernels:
        kernels, picked = kernels_section(phg, s0, d0, dev, args.kernel_reps, args.workload, out0)
        if "dense_T1" in kernels:
            kd = kernels["dense_T1"]
            td, dd = measured_traffic(args.workload, picked["dense_T1"],
                                      kd["ms_per_run"] * 1e-3 / kd["launches"])
            roofline_dense = roofline_of(s0, kd["ms_per_run"], kd["launches"], 1, td, dd,
                                         kernel="pass_kernel<beta=%d, T=1, rows=8, waves=4, dense>"
                                         % s0.beta)
    print("kernels done", file=sys.stderr, flush=True)

    ceilings = None
    if args.ceilings:
        ceilings = ceilings_section(phg, dev)
        cgb = ceilings["copy"]["GB_s_median"]
        roofline["frac_of_measured_copy"] = round(roofline["achieved"] / cgb, 4)
        if roofline_dense is not None:
            roofline_dense["frac_of_measured_copy"] = round(roofline_dense["achieved"] / cgb, 4)
            vi = measured_valu(args.workload, picked["dense_T1"])
            if vi is not None:
                rate = vi / (roofline_dense["avg_launch_us"] * 1e-6)
                roofline_dense["valu"] = {
                    "wave_instr_per_launch": round(vi), "wave_instr_per_s": round(rate, -6),
                    "frac_of_measured_issue": round(rate / ceilings["valu"]["v_add_u32"]["wave_instr_per_s"], 4),
                    "frac_of_band_test_mix": round(rate / ceilings["valu"]["band_test_mix"]["wave_instr_per_s"], 4),
                    "frac_of_spec_issue": round(rate / ceilings["valu"]["spec_wave_instr_per_s"], 4)}
        print("ceilings done", file=sys.stderr, flush=True)

    batch = None
    if args.batch > 0:
        batch = batch_section(args.batch, args.batch_steps, dev)
        print("batch done", file=sys.stderr, flush=True)

    serve = None
    if args.serve_seconds > 0:
        serve = serve_section(args.serve_seconds,
                              [float(x) for x in args.serve_rates.split(",") if x], dev,
                              [float(x) for x in args.serve_e2e_rates.split(",") if x],
                              args.serve_passes, args.serve_cap_gb)
        print("serve done", file=sys.stderr, flush=True)

    cycle = None
    if args.cycle:
        cycle = cycle_section(runs, stream)

    quality = None
    if args.quality:
        quality = quality_section(dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(specs, images)
        print("cpu baseline done", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel·iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded piecewise-constant + gradient + texture, salt-and-pepper)",
        "config": {"workload": args.workload, "rows": s0.rows, "cols": s0.cols,
                   "density": s0.density,
                   "params": [[s.alpha, s.beta, s.k] for s in specs],
                   "iterations": iters, "graph": bool(args.graph),
                   "streams": nstreams, "tuning_cache": bool(tuned),
                   "shapes": {str(b): shape_name(phg, phg.get_tuning_class(
                       b, phg.size_class(s0.rows * s0.cols))) for b in (1, 2)}},
        "roofline": roofline, "roofline_dense": roofline_dense, "kernels": kernels,
        "cpu_baseline": cpu, "batch": batch, "serve": serve, "quality": quality,
        "cycle_stop": cycle, "ceilings": ceilings, "sync_call": sync_call,
    }
    print(json.dumps(line), flush=True)
    if args.copy_calibration:
        a = torch.ones(64 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
