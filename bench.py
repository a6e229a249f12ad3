"""Throughput of the multicomponent TSLB step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload jet128] [--storage fp32]

One step = the boundary-layer fill plus the fused pull-stream-collide step over
the whole lattice (every row of the hot path).  The state is resident in HBM
before the timed region.  Prints one JSON line with GLUPS (n_x n_y n_z n_steps
/ (1e9 T)), the roofline of the dominant kernel (the fused step: algorithmic
bytes = the state read once and written once, 88 B/node in binary32 and 48 B/node
with 16-bit moments) measured with HIP events on the library's stream, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
BYTES_PER_NODE = {"fp32": 88, "fp16": 48, "bf16": 48}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="jet128", choices=["jet128", "jet512", "droplet32"])
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-oracle sample budget (0 = skip)")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the copy-kernel ceiling probe (0 = skip)")
    ap.add_argument("--kernel", default="fused", choices=["fused", "gather"])
    return ap.parse_args()


def workload_state(name):
    from paper_2403_15773_amd import inputs
    w = inputs.WORKLOADS[name]
    p = w["params"]
    if w["init"] == "droplet":
        st = inputs.droplet(p["nx"], 8.0, p["width"], noise_amp=1e-3, seed=1)
    else:
        st = inputs.quiescent(p["nx"], p["ny"], p["nz"])
    return p, st


def describe(name, p):
    if name.startswith("jet"):
        d, u = p["inlet_d"], p["inlet_u"]
        return {"workload": "round jet %dx%dx%d, D=%g, U=%g, Re=%g, We=%g, inlet noise %g, outflow at z max, "
                            "free-slip lateral walls" % (p["nx"], p["ny"], p["nz"], d, u, round(u * d / p["nu"]),
                                                         round(u * u * d / p["sigma"]), p["inlet_noise"]),
                "nodes": p["nx"] * p["ny"] * p["nz"]}
    return {"workload": "periodic droplet %d^3, R=8, W=3, nu=%g, sigma=%g" % (p["nx"], p["nu"], p["sigma"]),
            "nodes": p["nx"] * p["ny"] * p["nz"]}


def cpu_baseline(name, p, st, budget_s):
    """The FP64 oracle as it stands, on this host's cores, for a bounded number of
    steps of the same workload; rate in GLUPS."""
    if budget_s <= 0:
        return None
    import numpy as np

    from oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    o = Oracle(p["nx"], p["ny"], p["nz"], nu=p["nu"], sigma=p["sigma"], width=p["width"], eps=1e-4, bc=p["bc"],
               inlet_u=p.get("inlet_u", 0.0), inlet_d=p.get("inlet_d", 0.0), inlet_noise=p.get("inlet_noise", 0.0),
               seed=p.get("seed", 0))
    o.set_physical(**{k: np.asarray(v, np.float64) for k, v in st.items()})
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    n = max(1, min(1000, int(budget_s / max(t1 - t0, 1e-6)) - 1))
    o.step(n)
    t2 = time.perf_counter()
    steps = n + 1
    nodes = p["nx"] * p["ny"] * p["nz"]
    o.close()
    return {"value": nodes * steps / (t2 - t0) / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d steps of the full %dx%dx%d workload (FP64 populations, OpenMP), %.1f s"
                      % (steps, p["nx"], p["ny"], p["nz"], t2 - t0)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_2403_15773_amd.tslb import Simulation
    import numpy as np

    p, st = workload_state(a.workload)
    nodes = p["nx"] * p["ny"] * p["nz"]
    from paper_2403_15773_amd.tslb import copy_bandwidth
    copy = None
    if a.copy_mib > 0:
        gbps, cms = copy_bandwidth(a.copy_mib << 20, iters=20)
        copy = {"gbps": gbps, "ms": cms, "bytes_moved": 2 * (a.copy_mib << 20)}
        print("bench: copy-kernel ceiling %.0f GB/s (%d MiB read + written, %.3f ms)" % (gbps, 2 * a.copy_mib, cms),
              file=sys.stderr, flush=True)
    sim = Simulation(**p, eps=1e-4, storage=a.storage, device=0)
    sim.set_kernel(a.kernel)
    sim.set_state(rho_dev=np.asarray(st["rho"] - 1.0, np.float32), u=np.asarray(st["u"], np.float32),
                  P=np.asarray(st["P"], np.float32), phi=np.asarray(st["phi"], np.float32))
    print("bench: %s %s, warmup %d" % (a.workload, a.storage, a.warmup), file=sys.stderr, flush=True)
    sim.step(a.warmup)
    sim.sync()
    sim.set_timing(True)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(a.steps)
    sim.sync()
    t1 = time.perf_counter()
    kernel_ms = sim.last_step_kernel_ms()
    diag = sim.diagnostics()
    sim.close()
    T = t1 - t0
    glups = nodes * a.steps / T / 1e9
    bpn = BYTES_PER_NODE[a.storage]
    achieved = bpn * nodes / (kernel_ms * 1e-3) / 1e9 if kernel_ms > 0 else None
    print("bench: %.3f s for %d steps, kernel %.4f ms/launch, finite=%s" % (T, a.steps, kernel_ms, diag["finite"]),
          file=sys.stderr, flush=True)
    rec = {
        "metric": "GLUPS (lattice-node updates per second / 1e9) and fraction of the HBM roofline",
        "value": glups,
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": T / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.storage == "fp32" else "f32 (%s-stored moments)" % a.storage,
        "data": "synthetic",
        "config": describe(a.workload, p) | {"storage": a.storage, "finite": diag["finite"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
                     "kernel": "%s step" % a.kernel, "bytes_per_node": bpn, "kernel_ms": kernel_ms,
                     "copy_ceiling": copy["gbps"] if copy else None,
                     "frac_of_copy_ceiling": achieved / copy["gbps"] if (copy and achieved) else None},
        "cpu_baseline": cpu_baseline(a.workload, p, st, a.cpu_seconds),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
