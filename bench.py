"""Throughput of the fused FIR -> IIR-SOS chain on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the mid-size chain): 8 channels x 5,760,000 samples (120 s at
48 kHz), fp32, per-channel seeded 1/f noise plus a 20 Hz-20 kHz log sweep;
chain = 1023-tap Hamming band-pass FIR | 8th-order Chebyshev-I low-pass
(4 sections) | 2 peaking EQs, i.e. one FIR plus a 6-section cascade.

A step is one full tfx_chain call on the resident input: the device table
build (tfx_chain_prepare) followed by the fused filter kernel
(tfx_chain_run).  W untimed steps, then K timed steps between two device
synchronisations.  HIP events recorded on the launch stream around every
tfx_chain_run give the dominant kernel's average duration for the roofline
(algorithmic bytes = 8 B per channel-sample: read x once, write y once).

The CPU baseline runs the FP64 oracle (test infrastructure, plain C with one
OpenMP thread per channel) on the same input and reports its throughput and
the GPU result's error against it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also time a plain device copy of the same size (bandwidth reference)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); "
              "the channels of a multi-GPU job would shard with no communication." % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_08624_amd import lib, workloads
    from paper_2504_08624_amd.functional import _stages

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print("bench: generating chain_mid inputs (8 x 5,760,000)", file=sys.stderr, flush=True)
    w = workloads.chain_mid()
    C, N = w.x.shape
    x = torch.from_numpy(w.x).to(dev)
    y = torch.empty_like(x)
    kept, desc = _stages(w.stages, dev)
    arr = lib.stage_array(desc)
    nst = len(desc)
    L = lib.load()
    nb = lib.size_out()
    lib.call("tfx_chain_workspace_size", C, N, arr, nst, 0, nb)
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream

    def prepare():
        lib.check(L.tfx_chain_prepare(C, N, arr, nst, 0, ws.data_ptr(), ws.numel(), sp), "tfx_chain_prepare")

    def run():
        lib.check(L.tfx_chain_run(x.data_ptr(), y.data_ptr(), C, N, N, N, arr, nst, 0, None,
                                  ws.data_ptr(), ws.numel(), sp), "tfx_chain_run")

    print("bench: warmup %d" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        prepare()
        run()
    torch.cuda.synchronize()

    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        prepare()
        ev[i][0].record(stream)
        run()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    print("bench: timed %d steps in %.3f s" % (K, wall), file=sys.stderr, flush=True)

    samples = C * N
    ms_step = wall / K * 1e3
    value = samples / (wall / K) / 1e6
    alg_bytes = 8.0 * samples
    kern_s = float(kern_ms.mean()) / 1e3
    achieved = alg_bytes / kern_s / 1e9

    copy = None
    if args.copy_probe:
        z = torch.empty_like(x)
        for _ in range(3):
            z.copy_(x)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(10):
            z.copy_(x)
        b.record(stream)
        torch.cuda.synchronize()
        cs = a.elapsed_time(b) / 10 / 1e3
        copy = {"bytes": 2 * 4 * samples, "us": cs * 1e6, "GB/s": 2 * 4 * samples / cs / 1e9}
        del z

    out = y.cpu().numpy()

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.build()
        threads = min(C, len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "1024")))
        print("bench: oracle on the full input (%d threads)" % threads, file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        ref = O.chain(w.x, w.stages)
        c1 = time.perf_counter()
        cpu = {"value": samples / (c1 - c0) / 1e6, "unit": "Msamples/s", "cores": threads,
               "kind": "oracle",
               "sample": "the full chain_mid input (8 x 5,760,000, all stages), FP64, %.1f s" % (c1 - c0)}
        num = np.linalg.norm(out.astype(np.float64) - ref, axis=1)
        den = np.linalg.norm(ref, axis=1)
        err = float((num / den).max())

    rec = {
        "metric": "Msamples/s (ch x samples) fwd, % HBM roofline, at stated error",
        "value": round(value, 3),
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "chain_mid: 8 ch x 5,760,000 samples @48 kHz, 1/f noise + log sweep; "
                               "FIR 1023-tap band-pass | Chebyshev-I 8th order (4 SOS) | 2 peaking EQ",
                   "channels": C, "samples": N, "fir_taps": int(w.stages[0][1].size),
                   "sections": int(sum(s[1].shape[0] for s in w.stages if s[0] == "sos")),
                   "fir_algo": "fft" if 48 < w.stages[0][1].size <= 1025 else "direct", "step": "tfx_chain_prepare + tfx_chain_run"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "chain_kernel<FIR_FFT, true>", "kernel_us": round(kern_s * 1e6, 2),
                     "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": err,
        "tolerance": 1e-4,
    }
    if copy is not None:
        rec["copy_probe"] = copy
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
