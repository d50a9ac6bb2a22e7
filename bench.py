#!/usr/bin/env python3
"""Benchmark of the qudit state-vector hot path on one MI355X.

One step = |0...0> init, the depth-10 qutrit ansatz on n = 16 qudits
(3^16 = 43,046,721 complex64 amplitudes: per layer R_x, R_y, R_z on level
pairs (0,1), (1,2) of every qudit, clock Z^a, CSUM ring; 1280 gates), the full
probability vector and <Z_0>.  Inputs and outputs stay resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-batched] [--no-legs] [--no-cpu-baseline]
    python bench.py --profile-workload {stage,axis,fused,adjoint,batched}   (for rocprofv3)

Prints one JSON line.  value = amplitude updates per second
= (gates of the circuit as written) * 3^16 / step time.  The roofline entry
covers the dominant kernel (the fused LDS stage), timed with HIP events
recorded around each of its launches on the launch stream during the timed
steps; its algorithmic traffic is one read and one write of the state per
launch.  cpu_baseline times the FP64 oracle on a bounded sample of the same
workload (the circuit's mix of rotations, clock gates and CSUM) on one host
core and on several at once.  Extra records: one D x D gate on every qudit of
the same register through the single-qudit sweep kernels (each launch's HBM
fraction), the ragged 1024-circuit batch (graph replay vs the plain
per-circuit loop) and two gradient legs (D=5 n=10 forward + adjoint; D=10 n=8
forward + checkpointed adjoint).
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the ragged-batch measurement")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="run only the counter workload: two plain copies of the state size, then one step")
    ap.add_argument("--profile-workload", choices=["stage", "axis", "fused", "adjoint", "batched", "next"],
                    help="run only a short workload for rocprofv3 (kernel traces and counters), printing its "
                         "own HIP-event timings: stage = --pmc-workload; axis = one random unitary on each of "
                         "the 16 qudits of the 3^16 state; fused = dense blocks K = 100 (real, D=10 n=8) and "
                         "K = 49 (complex, D=7 n=9); adjoint = the D=5 n=10 forward + adjoint gradient; "
                         "batched = one graph replay of the 1024-circuit batch; next = the controlled-rotation, "
                         "slab, SWAP, MCX, shots and mixed-register kernels")
    ap.add_argument("--no-legs", action="store_true", help="skip the D=5 n=10 and D=10 n=8 gradient legs")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the controlled-rotation, slab, SWAP, MCX, shots and mixed-register record")
    ap.add_argument("--write-traffic", nargs="+", metavar="DIR",
                    help="turn rocprofv3 --pmc runs of --profile-workload stage (FETCH_SIZE, WRITE_SIZE, and "
                         "optionally the read- and write-request counters) into profiles/stage_d3_n16_traffic.json")
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


def _counter_rows(d, counters):
    """{kernel name: {counter: [value per dispatch]}} from a rocprofv3 --pmc run."""
    import collections
    import csv
    import glob
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] in counters:
                out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def write_traffic(fetch_dir: str, write_dir: str, rdreq_dir: str | None = None, wrreq_dir: str | None = None) -> None:
    """Per-launch HBM bytes of the stage kernel from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the two
    plain copies of the state size that --pmc-workload runs first.  With the
    request counters (TCC_EA0_RDREQ / _32B, TCC_BUBBLE, TCC_EA0_RDREQ_DRAM;
    TCC_EA0_WRREQ / _64B / _DRAM) the same bytes are also counted from raw
    requests, 128 B per read request (what the copy of known size shows on
    gfx950) and 64 / 32 B per write request."""
    import re

    N = 3 ** 16
    state = N * 8
    f = _counter_rows(fetch_dir, ("FETCH_SIZE",))
    w = _counter_rows(write_dir, ("WRITE_SIZE",))
    copyk = next(k for k in f if "copyBuffer" in k)
    stagek = next(k for k in f if "k_stage" in k)
    # the calibration copies are the two dispatches of the state size (the plan's matrix upload is another copy)
    cf = sorted(f[copyk]["FETCH_SIZE"])[-2:]
    cw = sorted(w[copyk]["WRITE_SIZE"])[-2:]
    cal_f = (state / 1024) / (sum(cf) / 2)
    cal_w = (state / 1024) / (sum(cw) / 2)
    sf = sum(f[stagek]["FETCH_SIZE"]) / len(f[stagek]["FETCH_SIZE"])
    sw = sum(w[stagek]["WRITE_SIZE"]) / len(w[stagek]["WRITE_SIZE"])
    bpl = (sf * cal_f + sw * cal_w) * 1024
    m = re.search(r"k_stage\w*(<[^>]*>)?", stagek)
    rec = {"kernel": m.group(0) if m else stagek, "launches": len(f[stagek]["FETCH_SIZE"]),
           "workload": "qutrit ansatz D=3 n=16 complex64, default plan",
           "source_hash": _source_hash(), "fetch_kib_per_launch": sf, "write_kib_per_launch": sw,
           "copy_calibration": {"bytes": state, "fetch_scale": cal_f, "write_scale": cal_w},
           "bytes_per_launch": round(bpl), "algorithmic_bytes_per_launch": 2 * state,
           "ratio": bpl / (2 * state),
           "commands": ["timeout -s KILL 150 rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof/stage_fetch "
                        "-o run -- python3 bench.py --profile-workload stage",
                        "timeout -s KILL 150 rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof/stage_write "
                        "-o run -- python3 bench.py --profile-workload stage"]}
    if rdreq_dir and wrreq_dir:
        rd = _counter_rows(rdreq_dir, ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_BUBBLE_sum",
                                       "TCC_EA0_RDREQ_DRAM_sum"))
        wr = _counter_rows(wrreq_dir, ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_WRREQ_DRAM_sum"))
        ck = next(k for k in rd if "copyBuffer" in k)
        sk = next(k for k in rd if "k_stage" in k)

        def avg(rows, c):
            return sum(rows[c]) / len(rows[c])
        copy_rd = sorted(rd[ck]["TCC_EA0_RDREQ_sum"])[-1]
        read_bytes_per_req = state / copy_rd
        rq = avg(rd[sk], "TCC_EA0_RDREQ_sum")
        wq = avg(wr[sk], "TCC_EA0_WRREQ_sum")
        wq64 = avg(wr[sk], "TCC_EA0_WRREQ_64B_sum")
        rbytes = rq * read_bytes_per_req
        wbytes = wq64 * 64 + (wq - wq64) * 32
        rec["request_cross_check"] = {
            "copy_read_requests": copy_rd, "bytes_per_read_request": read_bytes_per_req,
            "read_requests_per_launch": rq, "read_requests_32B": avg(rd[sk], "TCC_EA0_RDREQ_32B_sum"),
            "read_requests_bubble": avg(rd[sk], "TCC_BUBBLE_sum"),
            "read_requests_to_dram": avg(rd[sk], "TCC_EA0_RDREQ_DRAM_sum"),
            "write_requests_per_launch": wq, "write_requests_64B": wq64,
            "write_requests_to_dram": avg(wr[sk], "TCC_EA0_WRREQ_DRAM_sum"),
            "bytes_per_launch": round(rbytes + wbytes), "ratio": (rbytes + wbytes) / (2 * state),
            "commands": ["timeout -s KILL 150 rocprofv3 --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_BUBBLE_sum "
                         "TCC_EA0_RDREQ_DRAM_sum --output-format csv -d gpurun_out/prof/stage_rdreq -o run -- "
                         "python3 bench.py --profile-workload stage",
                         "timeout -s KILL 150 rocprofv3 --pmc TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum "
                         "TCC_EA0_WRREQ_DRAM_sum --output-format csv -d gpurun_out/prof/stage_wrreq -o run -- "
                         "python3 bench.py --profile-workload stage"]}
    rec["commands"].append("python3 bench.py --write-traffic gpurun_out/prof/stage_fetch gpurun_out/prof/stage_write"
                           + (" gpurun_out/prof/stage_rdreq gpurun_out/prof/stage_wrreq" if rdreq_dir else ""))
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def batched_measurement(steps: int) -> dict:
    """Ragged batch of 1024 circuits (768 qutrit, n ~ U{6..10}; 256 ququart,
    n ~ U{5..8}; depth-6 ansatz, own angles): init + forward + <sum Z_i> + adjoint
    gradient of every circuit, as one HIP graph replay per step.  Two set-ups:
    default schedules on one stream, and the autotuned schedules (forward +
    adjoint timed in the device-parameter mode at each group's batch) with one
    stream per group; both against the same circuits looped one at a time
    through the per-circuit path."""
    import numpy as np
    import torch

    import qf_inputs as qi
    from paper_2409_17716_amd.batched import PlainLoop, RaggedBatch
    circ = qi.config4()

    def run(**kw):
        t0 = time.perf_counter()
        rb = RaggedBatch(circ, **kw)
        setup = time.perf_counter() - t0
        rb.capture()
        for _ in range(2):
            rb.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rb.replay()
        torch.cuda.synchronize()
        return rb, (time.perf_counter() - t0) / steps, setup

    rb0, t_default, _ = run(tune=False, streams=0)
    g_default = rb0.gradients()
    del rb0
    torch.cuda.empty_cache()
    rb, tb, setup = run(tune=True, streams=4)
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
    rel0 = max(float(np.abs(g_default[i] - pl.grads[i]).max() / max(1e-12, np.abs(pl.grads[i]).max()))
               for i in range(len(circ)))
    return {"workload": "1024 circuits: 768 qutrit (n ~ U{6..10}) + 256 ququart (n ~ U{5..8}), depth-6 ansatz, "
                        "complex64; forward + Re<sum Z_i> + adjoint gradient per circuit",
            "circuits": len(circ), "amplitudes": int(sum(c.dim ** c.n for c in circ)), "groups": len(rb.groups),
            "batched_ms_per_step": round(tb * 1e3, 3), "batched_circuits_per_s": len(circ) / tb,
            "batched_setup": "autotuned schedules, groups on 4 streams (longest processing time first)",
            "tune_and_build_s": round(setup, 2), "stream_bytes": [int(b) for b in rb.chain_bytes],
            "default_single_stream_ms_per_step": round(t_default * 1e3, 3),
            "plain_ms_per_step": round(tp * 1e3, 2), "plain_circuits_per_s": len(circ) / tp,
            "speedup": tp / tb, "max_rel_grad_diff_vs_plain": rel, "default_max_rel_grad_diff_vs_plain": rel0,
            "schedules": rb.schedules()}


def _median_launch_ms(fn, reps: int = 5, per: int = 3) -> float:
    """Milliseconds per launch of fn(): the median over reps trials, each timing
    per back-to-back launches with HIP events on the current stream (a stray
    stall of the host or the GPU affects one trial)."""
    return sorted(_event_time(fn, per) for _ in range(reps))[reps // 2]


def sweep_measurement(psi, n: int, D: int) -> dict:
    """One Haar-random D x D gate on every qudit of the bench register through
    qf_apply_1q (the single-qudit sweep kernels), each qudit's launch time the
    median of 5 trials of 3 back-to-back launches (HIP events) after a warm-up;
    algorithmic traffic 2 N b per launch (one read and one write of the state)."""
    import numpy as np

    import paper_2409_17716_amd as qf
    import qf_inputs as qi
    N = D ** n
    nbytes = 2 * N * psi.element_size()
    rng = np.random.default_rng(11)
    per = []
    for q in range(n):
        U = qi.random_unitary(D, rng)
        qf.qf_apply_1q(psi, n, D, q, U)
        ms = _median_launch_ms(lambda: qf.qf_apply_1q(psi, n, D, q, U))
        per.append(nbytes / (ms * 1e-3) / 1e9)
    fr = [g / HBM_PEAK_GBS for g in per]
    return {"kernel": "k_axis_wide / k_axis_narrow (qf_apply_1q)", "bytes_per_launch": nbytes,
            "per_qudit_GBps": [round(g, 1) for g in per], "frac_mean": round(sum(fr) / len(fr), 4),
            "frac_min": round(min(fr), 4), "frac_max": round(max(fr), 4), "peak": HBM_PEAK_GBS, "unit": "GB/s"}


def next_rows_measurement() -> dict:
    """The kernels of the controlled rotation, the slab rotation, SWAP, MCX and
    shots on the 3^16 complex64 register, and one-qudit sweeps plus a plan on a
    mixed register of dims [2, 3, 4, 5] x 4 (120^4 = 207.4M amplitudes), each
    timed with HIP events (warm-up, then the median of 5 trials of 3 launches) against its algorithmic
    bytes: the amplitudes the operation must read and write (a gate reads and
    writes only the amplitudes it changes; shots read the state and write the
    histogram).  Where the changed amplitudes are spread over every 128-byte
    line of a region (a stride-1 target or control), line_bytes counts those
    lines, the least traffic such an access pattern can cause."""
    import numpy as np
    import torch

    import paper_2409_17716_amd as qf
    import qf_inputs as qi
    D, n = 3, 16
    N, b = D ** n, 8
    psi = qf.new_state(n, D, "c64")
    qf.qf_state_init(psi, n, D, None)
    for q in range(n):
        qf.qf_apply_1q(psi, n, D, q, qi.random_unitary(D, q))
    rec = {"register": "3^16 complex64 (344.4 MB)"}

    def measure(name, fn, nbytes, line_bytes=None, reps=5):
        fn()
        ms = _median_launch_ms(fn, reps)
        gbps = nbytes / (ms * 1e-3) / 1e9
        rec[name] = {"us": round(ms * 1e3, 2), "algorithmic_bytes": int(nbytes), "GBps": round(gbps, 1),
                     "frac": round(gbps / HBM_PEAK_GBS, 4)}
        if line_bytes is not None:
            rec[name]["line_bytes"] = int(line_bytes)
            rec[name]["line_frac"] = round(line_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    moved = 2 * b * N  # read and write of every amplitude
    # controlled rotation: fibres at control levels 1..D-1, x/y types touch 2 of D levels, z type j + 1
    measure("crx_c0_t15", lambda: qf.qf_apply_crot(psi, n, D, "crx", 0, 15, 0, 1, 0.3), moved * (D - 1) / D * 2 / D,
            moved * (D - 1) / D)
    measure("cry_c15_t0", lambda: qf.qf_apply_crot(psi, n, D, "cry", 15, 0, 1, 2, 0.3), moved * (D - 1) / D * 2 / D,
            moved * 2 / D)
    measure("crz_c4_t9", lambda: qf.qf_apply_crot(psi, n, D, "crz", 4, 9, 1, 0, 0.3), moved * (D - 1) / D * 2 / D)
    measure("slab_rx_q0", lambda: qf.qf_apply_rot(psi, n, D, "rx", 0, 0, 2, 0.3), moved * 2 / D)
    measure("slab_ry_q15", lambda: qf.qf_apply_rot(psi, n, D, "ry", 15, 0, 1, 0.3), moved * 2 / D, moved)
    measure("swap_0_15", lambda: qf.qf_apply_swap(psi, n, D, 0, 15), moved * (D - 1) / D, moved)
    measure("swap_7_8", lambda: qf.qf_apply_swap(psi, n, D, 7, 8), moved * (D - 1) / D)
    # x_15 += x_0 x_1 mod 3 moves the fibres whose two control digits are both non-zero
    measure("mcx_c01_t15", lambda: qf.qf_apply_mcx(psi, n, D, [0, 1], 15), moved * ((D - 1) / D) ** 2)
    pf = torch.empty(N, dtype=torch.float32, device="cuda")
    pm = torch.empty(9, dtype=torch.float32, device="cuda")
    measure("probs_full", lambda: qf.qf_probs(psi, n, D, out=pf), N * b + 4 * N)
    measure("probs_marginal_q0q15", lambda: qf.qf_probs(psi, n, D, qudits=[0, 15], out=pm), N * b)
    zb = torch.empty(2, dtype=torch.float64, device="cuda")
    measure("expect_z0", lambda: qf.qf_expect(psi, n, D, qi.z0_terms(), out=zb), N * b)
    measure("expect_sum_z", lambda: qf.qf_expect(psi, n, D, qi.zsum_terms(n), out=zb), N * b)
    p27 = torch.empty(27, dtype=torch.float32, device="cuda")
    measure("probs_marginal_q3q7q11", lambda: qf.qf_probs(psi, n, D, qudits=[3, 7, 11], out=p27), N * b)
    shots = 1 << 20
    u = torch.from_numpy(qi.uniforms(shots, 1)).cuda()
    measure("shots_full_2^20", lambda: qf.qf_sample(psi, n, D, shots, u), N * b + 8 * N)
    measure("shots_marginal_q0q15_2^20", lambda: qf.qf_sample(psi, n, D, shots, u, qudits=[0, 15]), N * b + 8 * 9)
    del psi, u
    torch.cuda.empty_cache()
    dims = [2, 3, 4, 5] * 4
    nm = len(dims)
    Nm = int(np.prod(dims))
    x = qf.new_state(nm, dims, "c64")
    qf.qf_state_init(x, nm, dims, None)
    fr = []
    for q in range(nm):
        U = qi.random_unitary(dims[q], q)
        qf.qf_apply_1q(x, nm, dims, q, U)
        ms = _median_launch_ms(lambda: qf.qf_apply_1q(x, nm, dims, q, U))
        fr.append(2 * b * Nm / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    c = qi.mixed_hea(dims, 1, 5)
    p = qf.plan_for(c, "c64")
    qf.qf_state_init(x, nm, dims, None)
    p.forward(x, c.theta)
    ms = _event_time(lambda: p.forward(x, c.theta), 2)
    rec["mixed"] = {"dims": "[2,3,4,5] x 4", "amplitudes": Nm, "sweep_frac_per_qudit": [round(f, 4) for f in fr],
                    "sweep_frac_mean": round(float(np.mean(fr)), 4), "sweep_frac_min": round(float(min(fr)), 4),
                    "plan": f"mixed ansatz, 1 layer ({len(c.ops)} gates), per-qudit runs", "plan_ms": round(ms, 3),
                    "plan_steps": p.num_stages, "plan_amp_updates_per_s": len(c.ops) * Nm / (ms * 1e-3)}
    del x
    torch.cuda.empty_cache()
    return rec


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(c, n_rot: int, n_clock: int, n_csum: int):
    """Gates of the circuit in the proportion it holds them (rotations, clock
    gates, CSUM), taken in circuit order."""
    want = {"rot": n_rot, "clock": n_clock, "csum": n_csum}
    out = []
    for op in c.ops:
        k = "rot" if op[0] in ("rx", "ry", "rz") else op[0]
        if want.get(k, 0) > 0:
            out.append(op)
            want[k] -= 1
    return out


def _oracle_run(mix):
    """One host process: the FP64 oracle applying the sample to the full state."""
    from threadpoolctl import threadpool_limits

    import qf_inputs as qi
    from oracle import sim
    c = qi.config2()
    ops = _oracle_sample(c, *mix)
    psi = sim.basis_state(c.dim, c.n)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for op in ops:
            psi = sim.apply_op(psi, c.dim, c.n, op, c.theta)
        return len(ops), time.perf_counter() - t0


def cpu_baseline(c) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    6 rotations, 1 clock gate and 1 CSUM (the circuit's 6 : 1 : 1 mix) on the
    full 3^16 state, first on one host core, then as independent copies on
    several cores at once (aggregate rate; copies limited by free memory, the
    oracle's digit maps take about 12 GB each)."""
    import concurrent.futures as cf

    import psutil
    N = c.dim ** c.n
    mix = (6, 1, 1)
    ngates, el = _oracle_run(mix)
    single = ngates * N / el
    ncpu = os.cpu_count() or 1
    try:
        ncpu = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    par = max(1, min(ncpu, 16, int(psutil.virtual_memory().available // (12 << 30))))
    agg = None
    if par > 1:
        with cf.ProcessPoolExecutor(max_workers=par) as ex:
            t0 = time.perf_counter()
            res = list(ex.map(_oracle_run, [mix] * par))
            wall = time.perf_counter() - t0
        agg = sum(r[0] for r in res) * N / wall
    return {"value": agg if agg else single, "unit": "amp-updates/s", "cores": par, "kind": "oracle",
            "single_core": single, "nproc": ncpu, "cpu_model": _cpu_model(),
            "sample": f"{ngates} gates in the circuit's mix (6 rotations, 1 clock, 1 CSUM) on the full 3^16 "
                      f"state in complex128: {el:.1f} s on one core; value = {par} independent copies on "
                      f"{par} cores at once (aggregate)"}


def _event_time(fn, reps: int) -> float:
    """Mean milliseconds of fn() over reps, with HIP events on the current stream."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def gradient_legs() -> dict:
    """D=5 n=10 (960 angles) forward + adjoint gradient, and D=10 n=8 (864
    angles) forward + adjoint with a checkpoint every 4 layers, default plans,
    complex64, host-returned gradients (the adjoint call synchronises)."""
    import torch

    import paper_2409_17716_amd as qf
    import qf_inputs as qi
    out = {}
    for name, c, kw in (("d5_n10_fwd_grad", qi.config3(), {}),
                        ("d10_n8_fwd_ckpt_grad", qi.config5(), {"ckpt_every": 320})):
        p = qf.plan_for(c, "c64", **kw)
        psi = qf.new_state(c.n, c.dim, "c64")
        lam = qf.new_state(c.n, c.dim, "c64")
        terms = qi.zsum_terms(c.n)

        def fwd():
            qf.qf_state_init(psi, c.n, c.dim, None)
            p.forward(psi, c.theta)

        def step():
            fwd()
            p.adjoint_grad(psi, lam, c.theta, terms)
        step()
        torch.cuda.synchronize()
        reps = 5 if c.dim == 5 else 2
        t_fwd = _event_time(fwd, reps)
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / reps * 1e3
        out[name] = {"amplitudes": c.dim ** c.n, "gates": len(c.ops), "params": c.nparams,
                     "forward_passes": p.num_stages, "adjoint_passes": p.num_adjoint_stages,
                     "forward_ms": round(t_fwd, 3), "forward_plus_gradient_ms": round(t_step, 3),
                     "forward_amp_updates_per_s": len(c.ops) * c.dim ** c.n / (t_fwd * 1e-3)}
        del p, psi, lam
        torch.cuda.empty_cache()
    return out


def profile_workload(kind: str) -> int:
    """Short workloads for rocprofv3; each prints its own HIP-event timings."""
    import numpy as np
    import torch

    import paper_2409_17716_amd as qf
    import qf_inputs as qi
    torch.cuda.set_device(0)
    rec = {"workload": kind}
    if kind == "axis":
        D, n = 3, 16
        N = D ** n
        psi = qf.new_state(n, D, "c64")
        src = torch.zeros(N, dtype=torch.complex64, device="cuda")
        for _ in range(2):
            psi.copy_(src)  # calibration copies of the state size for the traffic counters
        qf.qf_state_init(psi, n, D, None)
        rng = np.random.default_rng(7)
        per = []
        for q in range(n):
            U = qi.random_unitary(D, rng)
            qf.qf_apply_1q(psi, n, D, q, U)  # warm-up
            ms = _event_time(lambda: qf.qf_apply_1q(psi, n, D, q, U), 3)
            per.append({"qudit": q, "stride": D ** (n - 1 - q), "us": round(ms * 1e3, 2),
                        "GBps": round(2 * N * 8 / (ms * 1e-3) / 1e9, 1)})
        rec["per_axis"] = per
    elif kind == "fused":
        for D, n, k, real in ((10, 8, 2, True), (7, 9, 2, False)):
            K = D ** k
            psi = qf.new_state(n, D, "c64")
            qf.qf_state_init(psi, n, D, None)
            rng = np.random.default_rng(K)
            if real:
                q, _ = np.linalg.qr(rng.standard_normal((K, K)))
                B = q.astype(np.complex128)
            else:
                B = qi.random_unitary(K, rng)
            positions = list(range(0, n - k + 1, 2))
            # the block as a custom gate of a one-gate plan: the plan knows from
            # the host matrix whether it is real (and then skips the imaginary
            # products), which qf_apply_fused, given a device matrix, does not
            plans = {q0: qf.Plan(D, n, [("u", q0, k, B)], 0, "c64") for q0 in positions}
            no_angles = np.zeros(0)
            for q0 in positions:
                plans[q0].forward(psi, no_angles)
            ms = {q0: _event_time(lambda: plans[q0].forward(psi, no_angles), 3) for q0 in positions}
            N = D ** n
            flops = (4 if real else 8) * K * N
            rec[f"K{K}_{'real' if real else 'complex'}"] = {
                "D": D, "n": n, "flops_per_launch": flops,
                "per_position": {str(q0): {"us": round(v * 1e3, 1), "TFLOPs": round(flops / (v * 1e-3) / 1e12, 2)}
                                 for q0, v in ms.items()}}
            del psi
            torch.cuda.empty_cache()
    elif kind == "adjoint":
        c = qi.config3()
        terms = qi.zsum_terms(c.n)
        p = qf.plan_for(c, "c64")
        psi = qf.new_state(c.n, c.dim, "c64")
        lam = qf.new_state(c.n, c.dim, "c64")
        for i in range(3):
            if i == 2:
                p.set_profiling(True)
            qf.qf_state_init(psi, c.n, c.dim, None)
            p.forward(psi, c.theta)
            p.adjoint_grad(psi, lam, c.theta, terms)
        prof = p.read_profile()
        rec["families"] = {k: {"launches": v[0], "ms": round(v[1], 3),
                               "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1)} for k, v in prof.items()}
    elif kind == "next":
        rec.update(next_rows_measurement())
    elif kind == "batched":
        from paper_2409_17716_amd.batched import RaggedBatch
        rb = RaggedBatch(qi.config4(), tune=True)
        rb.capture()
        rb.replay()
        torch.cuda.synchronize()
        rec["replay_ms"] = round(_event_time(rb.replay, 3), 3)
    torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)
    return 0


def main() -> int:
    a = _args()
    if a.write_traffic:
        if len(a.write_traffic) not in (2, 4):
            print("bench.py: --write-traffic takes FETCH_DIR WRITE_DIR [RDREQ_DIR WRREQ_DIR]", file=sys.stderr)
            return 2
        write_traffic(*a.write_traffic)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU; --gpus above 1 is not supported", file=sys.stderr)
        return 2
    if a.profile_workload and a.profile_workload != "stage":
        return profile_workload(a.profile_workload)
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

    if a.pmc_workload or a.profile_workload == "stage":
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
                "kernel": "k_stage_rounds_w8<float, 3, 2>", "launches_per_step": launches // a.steps,
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "qutrit HEA, D=3, n=16 (3^16 amplitudes, complex64), depth 10, batch 1: "
                               "init + 1280 gates + full probabilities + <Z_0>",
                   "dim": D, "n": n, "layers": 10, "gates": len(c.ops), "amplitudes": N, "batch": 1,
                   "forward_passes": plan.num_stages,
                   "state": "complex64 (FP32 arithmetic, FP64 reductions)"},
        "roofline": roofline,
        "z0": [float(ev[0]), float(ev[1])],
        "sweeps": sweep_measurement(psi, n, D),
    }
    if not a.no_batched:
        out["batched"] = batched_measurement(max(1, a.steps // 2))
    if not a.no_legs:
        out["legs"] = gradient_legs()
    if not a.no_next:
        out["next_rows"] = next_rows_measurement()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
