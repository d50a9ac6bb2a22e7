#!/usr/bin/env python3
"""Writes the full-size expected values the GPU tests compare against.

Calls only the FP64 oracle (``oracle/``) on the seeded workload descriptions of
``qf_inputs``; nothing here touches the HIP library.

    python tests/golden/make_fullsize_goldens.py [--workers 8] [--only config3|config2]

* ``config3_d5_n10_full.json`` - D=5, n=10, depth 8 (1120 gates, 960 angles):
  the loss Re<sum_i Z_i>, all 960 oracle-adjoint gradients and the FP64 central
  finite differences (h = 1e-6) of the 16 parameters the workload names.
* ``config2_d3_n16_full.json`` - D=3, n=16, depth 10 (1280 gates): <Z_0> and
  the marginal distribution of every single qudit.

The finite differences run as separate processes (two forwards each); one
oracle forward of config 3 takes about six minutes on one core, one of
config 2 about forty.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

H_FD = 1e-6


def _one_thread():
    from threadpoolctl import threadpool_limits
    return threadpool_limits(1)


def _loss_at(args):
    """Oracle loss of config 3 with parameter i moved by delta."""
    i, delta = args
    import numpy as np

    import qf_inputs as qi
    from oracle import grad
    c = qi.config3()
    th = np.array(c.theta, dtype=np.float64)
    th[i] += delta
    with _one_thread():
        return i, delta, grad.loss(c, qi.zsum_terms(c.n), th)


def _adjoint_c3():
    import numpy as np

    import qf_inputs as qi
    from oracle import grad, measure, sim
    c = qi.config3()
    terms = qi.zsum_terms(c.n)
    with _one_thread():
        psi = sim.run(c)
        loss = float(measure.expect_diag(psi, c.dim, c.n, terms).real)
        g = grad.adjoint(c, terms, psi_final=psi)
    return loss, np.asarray(g).tolist()


def _config2():
    import qf_inputs as qi
    from oracle import measure, sim
    c = qi.config2()
    with _one_thread():
        psi = sim.run(c)
        z0 = measure.expect_diag(psi, c.dim, c.n, qi.z0_terms())
        marg = [measure.marginal(psi, c.dim, c.n, [q]).tolist() for q in range(c.n)]
        zsum = measure.expect_diag(psi, c.dim, c.n, qi.zsum_terms(c.n))
    return {"z0": [z0.real, z0.imag], "zsum": [zsum.real, zsum.imag], "marginals": marg}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--only", choices=["config3", "config2"], default=None)
    a = ap.parse_args()
    import numpy as np

    import qf_inputs as qi
    t0 = time.time()
    jobs = {}
    with ProcessPoolExecutor(max_workers=a.workers) as ex:
        if a.only in (None, "config2"):
            jobs["c2"] = ex.submit(_config2)
        if a.only in (None, "config3"):
            c = qi.config3()
            idx = [int(i) for i in qi.config3_fd_params(c, 16)]
            jobs["adj"] = ex.submit(_adjoint_c3)
            jobs["fd"] = [ex.submit(_loss_at, (i, s * H_FD)) for i in idx for s in (1.0, -1.0)]
        if "fd" in jobs:
            vals = {}
            for f in jobs["fd"]:
                i, d, L = f.result()
                vals[(i, d > 0)] = L
                print(f"[golden] config3 loss(theta{'+' if d > 0 else '-'}h e_{i}) = {L!r} "
                      f"({time.time() - t0:.0f} s)", flush=True)
            fd = [(vals[(i, True)] - vals[(i, False)]) / (2 * H_FD) for i in idx]
            loss, g = jobs["adj"].result()
            rec = {
                "_source": "written by tests/golden/make_fullsize_goldens.py from the FP64 oracle only",
                "workload": "D=5, n=10, depth-8 ansatz (R_x, R_y, R_z on the 4 adjacent level pairs of every "
                            "qudit, CSUM ring, CZ(i, i+2)), seed 2, from |0...0>",
                "gates": len(c.ops), "nparams": c.nparams,
                "loss": loss,
                "grad_adjoint": g,
                "fd_h": H_FD, "fd_params": idx, "grad_fd": fd,
            }
            with open(os.path.join(HERE, "config3_d5_n10_full.json"), "w") as fh:
                json.dump(rec, fh, indent=0)
            print(f"[golden] config3 done: loss {loss!r}, max|adj - fd| on the 16 = "
                  f"{np.abs(np.array(g)[idx] - np.array(fd)).max():.3e} ({time.time() - t0:.0f} s)", flush=True)
        if "c2" in jobs:
            r = jobs["c2"].result()
            c2 = qi.config2()
            rec = {"_source": "written by tests/golden/make_fullsize_goldens.py from the FP64 oracle only",
                   "workload": "D=3, n=16, depth-10 ansatz (R_x, R_y, R_z on level pairs (0,1), (1,2), clock Z^a, "
                               "CSUM ring), seed 1, from |0...0>",
                   "gates": len(c2.ops), **r}
            with open(os.path.join(HERE, "config2_d3_n16_full.json"), "w") as fh:
                json.dump(rec, fh, indent=0)
            print(f"[golden] config2 done: z0 = {r['z0']} ({time.time() - t0:.0f} s)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
