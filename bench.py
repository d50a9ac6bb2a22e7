#!/usr/bin/env python3
"""Benchmark of the qudit state-vector hot path on one MI355X.

One step = |0...0> init, the depth-10 qutrit ansatz on n = 16 qudits
(3^16 = 43,046,721 complex64 amplitudes: per layer R_x, R_y, R_z on level
pairs (0,1), (1,2) of every qudit, clock Z^a, CSUM ring; 1280 gates), the full
probability vector and <Z_0>.  Inputs and outputs stay resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--cpu-seconds S]

Prints one JSON line.  value = amplitude updates per second
= (gates of the circuit as written) * 3^16 / step time.  The roofline entry
covers the dominant kernel (the fused LDS stage), timed with HIP events
recorded around each of its launches on the launch stream during the timed
steps; its algorithmic traffic is one read and one write of the state per
launch.  cpu_baseline times the FP64 oracle on a bounded sample of the same
workload on one host core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_d3_n16_traffic.json")


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the ragged-batch measurement")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="run only the counter workload: two plain copies of the state size, then one step")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs of --pmc-workload (FETCH_SIZE, WRITE_SIZE) into "
                         "profiles/stage_d3_n16_traffic.json")
    return ap.parse_args()


def _source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_stage.hip", "qf_internal.h", "qf_common.h"):
        with open(os.path.join(ROOT, "paper_2409_17716_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic():
    """HBM bytes per stage launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE
    (scaled by a plain copy of known size), if taken on the current kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != _source_hash():
        return None
    return t.get("bytes_per_launch")


def write_traffic(fetch_dir: str, write_dir: str) -> None:
    """Per-launch HBM bytes of the stage kernel from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the plain
    copy of the state size that --pmc-workload runs first."""
    import collections
    import csv
    import glob
    import re

    N = 3 ** 16

    def per_kernel(d, counter):
        out = collections.defaultdict(list)
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                if r["Counter_Name"] == counter:
                    out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return out

    f = per_kernel(fetch_dir, "FETCH_SIZE")
    w = per_kernel(write_dir, "WRITE_SIZE")
    copyk = next(k for k in f if "copyBuffer" in k or "copy" in k.lower())
    stagek = next(k for k in f if "k_stage" in k)
    copy_kib = N * 8 / 1024
    cal_f = copy_kib / (sum(f[copyk]) / 2)
    cal_w = copy_kib / (sum(w[copyk]) / 2)
    sf = sum(f[stagek]) / len(f[stagek])
    sw = sum(w[stagek]) / len(w[stagek])
    bpl = (sf * cal_f + sw * cal_w) * 1024
    m = re.search(r"k_stage\w*(<[^>]*>)?", stagek)
    rec = {"kernel": m.group(0) if m else stagek, "launches": len(f[stagek]),
           "workload": "qutrit ansatz D=3 n=16 complex64, default plan",
           "source_hash": _source_hash(), "fetch_kib_per_launch": sf, "write_kib_per_launch": sw,
           "copy_calibration": {"bytes": N * 8, "fetch_scale": cal_f, "write_scale": cal_w},
           "bytes_per_launch": round(bpl), "algorithmic_bytes_per_launch": 2 * N * 8,
           "ratio": bpl / (2 * N * 8),
           "commands": ["timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch "
                        "-o run -- python3 bench.py --pmc-workload",
                        "timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write "
                        "-o run -- python3 bench.py --pmc-workload",
                        "python3 bench.py --write-traffic gpurun_out/pmc_fetch gpurun_out/pmc_write"]}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def batched_measurement(steps: int) -> dict:
    """Ragged batch of 1024 circuits (768 qutrit, n ~ U{6..10}; 256 ququart,
    n ~ U{5..8}; depth-6 ansatz, own angles): init + forward + <sum Z_i> + adjoint
    gradient of every circuit, as one HIP graph replay per step, against the same
    circuits looped one at a time through the per-circuit path."""
    import numpy as np
    import torch

    import qf_inputs as qi
    from paper_2409_17716_amd.batched import PlainLoop, RaggedBatch
    circ = qi.config4()
    rb = RaggedBatch(circ)
    rb.capture()
    for _ in range(2):
        rb.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rb.replay()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / steps
    pl = PlainLoop(circ)
    pl.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.step()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    gb = rb.gradients()
    rel = max(float(np.abs(gb[i] - pl.grads[i]).max() / max(1e-12, np.abs(pl.grads[i]).max()))
              for i in range(len(circ)))
    return {"workload": "1024 circuits: 768 qutrit (n ~ U{6..10}) + 256 ququart (n ~ U{5..8}), depth-6 ansatz, "
                        "complex64; forward + Re<sum Z_i> + adjoint gradient per circuit",
            "circuits": len(circ), "amplitudes": int(sum(c.dim ** c.n for c in circ)), "groups": len(rb.groups),
            "batched_ms_per_step": round(tb * 1e3, 3), "batched_circuits_per_s": len(circ) / tb,
            "plain_ms_per_step": round(tp * 1e3, 2), "plain_circuits_per_s": len(circ) / tp,
            "speedup": tp / tb, "max_rel_grad_diff_vs_plain": rel}


def cpu_baseline(c, seconds: float) -> dict:
    """The FP64 oracle, as it stands, on the first gates of the same workload."""
    from threadpoolctl import threadpool_limits

    from oracle import sim
    D, n = c.dim, c.n
    N = D ** n
    psi = sim.basis_state(D, n)
    done = 0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for op in c.ops:
            psi = sim.apply_op(psi, D, n, op, c.theta)
            done += 1
            if time.perf_counter() - t0 >= seconds:
                break
        el = time.perf_counter() - t0
    kinds = sorted({op[0] for op in c.ops[:done]})
    return {"value": done * N / el, "unit": "amp-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {len(c.ops)} gates ({', '.join(kinds)}) of the same circuit on the full "
                      f"3^16 state in complex128, {el:.1f} s on one host core"}


def main() -> int:
    a = _args()
    if a.write_traffic:
        write_traffic(*a.write_traffic)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU; --gpus above 1 is not supported", file=sys.stderr)
        return 2
    import torch

    import paper_2409_17716_amd as qf
    import qf_inputs as qi

    torch.cuda.set_device(0)
    c = qi.config2()
    D, n = c.dim, c.n
    N = D ** n
    plan = qf.plan_for(c, "c64")
    psi = qf.new_state(n, D, "c64")
    probs = torch.empty(N, dtype=torch.float32, device="cuda")
    z0 = torch.empty(2, dtype=torch.float64, device="cuda")
    terms = qi.z0_terms()

    def step():
        qf.qf_state_init(psi, n, D, None)
        plan.forward(psi, c.theta)
        qf.qf_probs(psi, n, D, out=probs)
        qf.qf_expect(psi, n, D, terms, out=z0)

    if a.pmc_workload:
        src = torch.zeros(N, dtype=torch.complex64, device="cuda")
        for _ in range(2):
            psi.copy_(src)
        torch.cuda.synchronize()
        step()
        torch.cuda.synchronize()
        return 0

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.read_profile()
    plan.set_profiling(False)
    ms = (t1 - t0) / a.steps * 1e3
    value = len(c.ops) * N / (ms * 1e-3)

    launches, total_ms, nbytes = prof["stage"]
    avg_ms = total_ms / launches
    per_launch = nbytes / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    traffic = _traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_stage_rounds<float, 3, 2>", "launches_per_step": launches // a.steps,
                "avg_launch_us": round(avg_ms * 1e3, 2), "bytes_per_launch": per_launch}
    ev = z0.cpu().numpy()
    out = {
        "metric": "amplitude-updates/s (%HBM peak); batched fwd+adjoint circuits/s vs plain",
        "value": value,
        "unit": "amp-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "qutrit HEA, D=3, n=16 (3^16 amplitudes, complex64), depth 10, batch 1: "
                               "init + 1280 gates + full probabilities + <Z_0>",
                   "dim": D, "n": n, "layers": 10, "gates": len(c.ops), "amplitudes": N, "batch": 1,
                   "forward_passes": plan.num_stages},
        "roofline": roofline,
        "z0": [float(ev[0]), float(ev[1])],
    }
    if not a.no_batched:
        out["batched"] = batched_measurement(max(1, a.steps // 2))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, a.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
