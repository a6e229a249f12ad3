"""Throughput of the multicomponent TSLB step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload jet512] [--storage fp32]
                    [--variants fp16,bf16,fp16q] [--secondary jet128] [--serve 256] [--cpu-seconds 15]

One step = the fused pull-stream-collide step over the whole lattice, which also
writes the boundary layers of the state it produces (every row of the hot path).
The state is resident in HBM before the timed region.  Prints one JSON line:
  value / roofline  GLUPS (n_x n_y n_z n_steps / (1e9 T)) of the main run (by
                    default the 512 x 512 x 2048 jet, the largest workload on one
                    GPU) and the roofline of its dominant kernel (the fused step;
                    algorithmic bytes = the state read once and written once:
                    88 B/node in binary32, 48 B/node with 16-bit moments), the
                    kernel time measured with HIP events on the library's stream
                    around every launch of the timed region;
  storage_variants  the same workload with FP16/BF16-stored moments;
  secondary         the 128 x 128 x 512 jet in binary32;
  serving           the seeded request stream run by continuous batching
                    (p50/p99 latency, aggregate GLUPS);
  cpu_baseline      the FP64 CPU oracle timed on a bounded sample of the workload
                    (of the 128 x 128 x 512 jet when the workload's FP64
                    populations do not fit in host memory: 292 GB for the
                    512 x 512 x 2048 jet).
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
BYTES_PER_NODE = {"fp32": 88, "fp16": 48, "bf16": 48, "fp16q": 64}
BYTES_PER_NODE_1C = {"fp32": 80, "fp16": 40, "bf16": 40, "fp16q": 56}  # one component: no phase plane
# HBM traffic of the fused step from rocprofv3 counters, valid while the kernel
# sources hash to the value recorded next to the figures
TRAFFIC_FILES = {"jet128": os.path.join(ROOT, "profiles", "fused_step_jet128_traffic.txt"),
                 "tgv256": os.path.join(ROOT, "profiles", "fused_step_tgv256_1c_traffic.txt"),
                 "jet512": os.path.join(ROOT, "profiles", "fused_step_jet512_traffic.txt")}
KERNEL_SOURCES = ["paper_2403_15773_amd/csrc/tslb_step_fused.hip", "paper_2403_15773_amd/csrc/tslb_device.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="jet512",
                    choices=["jet128", "jet512", "jet400", "droplet32", "tgv256", "jet128vd"])
    ap.add_argument("--paper-domain", type=int, default=1,
                    help="also time the paper's 400x400x800 jet domain, for context beside its GLUPS (0 = skip)")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16", "fp16q"])
    ap.add_argument("--variants", default="fp16,bf16,fp16q", help="other storage types timed on the same workload")
    ap.add_argument("--secondary", default="jet128", help="another workload timed in binary32 ('' = skip)")
    ap.add_argument("--serve", type=int, default=256, help="requests in the serving stream (0 = skip)")
    ap.add_argument("--single", type=int, default=1, help="also time the one-component Taylor-Green vortex (0 = skip)")
    ap.add_argument("--vd", type=int, default=1, help="also time the variable-density 128x128x512 jet (0 = skip)")
    ap.add_argument("--busy", type=int, default=1,
                    help="also time the workload from a smooth state with no quiescent node (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-oracle sample budget (0 = skip)")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the copy-kernel ceiling probe (0 = skip)")
    ap.add_argument("--kernel", default="fused", choices=["fused", "gather"])
    ap.add_argument("--repeats", type=int, default=4,
                    help="further timed runs of the headline's steps after its timed region (median of all reported)")
    ap.add_argument("--probe", type=int, default=1, help="time the projection on ALU and matrix cores (0 = skip)")
    return ap.parse_args()


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def workload_state(name):
    """(parameters, physical initial fields or None for a quiescent start)."""
    from paper_2403_15773_amd import inputs
    w = inputs.WORKLOADS[name]
    p = w["params"]
    if w["init"] == "droplet":
        return p, inputs.droplet(p["nx"], 8.0, p["width"], noise_amp=1e-3, seed=1)
    if w["init"] == "taylor_green":
        return p, inputs.taylor_green(p["nx"])
    return p, None


def describe(name, p):
    if name.startswith("tgv"):
        return {"workload": "Taylor-Green vortex %d^3, one component, U0=0.05, Re=1600, periodic" % p["nx"],
                "nodes": p["nx"] * p["ny"] * p["nz"]}
    if name == "jet128vd":
        return {"workload": "round jet %dx%dx%d, D=%g, U=%g, jet/ambient density %g/%g, nu %g, We=%g, variable-density "
                            "step" % (p["nx"], p["ny"], p["nz"], p["inlet_d"], p["inlet_u"], p["density_a"],
                                      p["density_b"], p["nu_a"], round(p["inlet_u"] ** 2 * p["inlet_d"] / p["sigma"])),
                "nodes": p["nx"] * p["ny"] * p["nz"]}
    if name.startswith("jet"):
        d, u = p["inlet_d"], p["inlet_u"]
        return {"workload": "round jet %dx%dx%d, D=%g, U=%g, Re=%g, We=%g, inlet noise %g, outflow at z max, "
                            "free-slip lateral walls" % (p["nx"], p["ny"], p["nz"], d, u, round(u * d / p["nu"]),
                                                         round(u * u * d / p["sigma"]), p["inlet_noise"]),
                "nodes": p["nx"] * p["ny"] * p["nz"]}
    return {"workload": "periodic droplet %d^3, R=8, W=3, nu=%g, sigma=%g" % (p["nx"], p["nu"], p["sigma"]),
            "nodes": p["nx"] * p["ny"] * p["nz"]}


def sources_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, storage):
    """HBM bytes per fused-step launch from the committed counter summary, or
    None when it covers another workload or the kernel changed since."""
    path = TRAFFIC_FILES.get(workload)
    if storage != "fp32" or path is None or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != sources_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_lattice(name, storage, steps, warmup, kernel="fused", smooth=False, repeats=0):
    """Time `steps` steps of workload `name`; returns the measurements.  smooth:
    start from inputs.smooth_state (no quiescent node) instead of the workload's
    own initial state.  repeats: after the timed region, time that many more
    batches of `steps` steps of the same lattice (continuing its run), each by
    the wall clock around it, for the spread of whole timed runs."""
    import numpy as np

    from paper_2403_15773_amd import inputs
    from paper_2403_15773_amd.tslb import Simulation
    p, st = workload_state(name)
    if smooth:
        s = inputs.smooth_state(p["nx"], p["ny"], p["nz"])
        st = {"rho_dev": s["rho_dev"], "u": s["u"], "P": s["P"], "phi": s["phi"]}
    nodes = p["nx"] * p["ny"] * p["nz"]
    sim = Simulation(**p, eps=1e-4, storage=storage, u_scale=0.05, device=0)
    sim.set_kernel(kernel)
    if st is None:
        sim.set_state_rest(step=0)  # quiescent: rho = 1, u = 0, P = 0, phi = 0
    elif smooth:
        sim.set_state(rho_dev=st["rho_dev"], u=st["u"], P=st["P"],
                      phi=None if p.get("components", 2) == 1 else st["phi"])
        st = s = None  # the host copy is no longer needed
    else:
        one = p.get("components", 2) == 1
        sim.set_state(rho_dev=np.asarray(st["rho"] - 1.0, np.float32), u=np.asarray(st["u"], np.float32),
                      P=np.asarray(st["P"], np.float32), phi=None if one else np.asarray(st["phi"], np.float32))
    log("%s %s%s, warmup %d" % (name, storage, " (smooth state)" if smooth else "", warmup))
    sim.step(warmup)
    sim.sync()
    sim.set_timing(True)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    t1 = time.perf_counter()
    kernel_ms = sim.last_step_kernel_ms()
    times = sim.step_kernel_times()
    rep = []
    if repeats > 0:
        sim.set_timing(False)
        for _ in range(repeats):
            sim.sync()
            r0 = time.perf_counter()
            sim.step(steps)
            sim.sync()
            rep.append(nodes * steps / (time.perf_counter() - r0) / 1e9)
    diag = sim.diagnostics()
    sim.close()
    T = t1 - t0
    bpn = (BYTES_PER_NODE_1C if p.get("components", 2) == 1 else BYTES_PER_NODE)[storage]
    achieved = bpn * nodes / (kernel_ms * 1e-3) / 1e9 if kernel_ms > 0 else None
    log("%s %s: %.3f s for %d steps, kernel %.4f ms/launch, finite=%s" % (name, storage, T, steps, kernel_ms,
                                                                          diag["finite"]))
    spread = {"median": float(np.median(times)), "min": float(times.min()), "max": float(times.max()),
              "launches": int(times.size)} if times.size else None
    return {"p": p, "st": st, "nodes": nodes, "T": T, "glups": nodes * steps / T / 1e9, "kernel_ms": kernel_ms,
            "kernel_ms_spread": spread, "achieved": achieved, "bpn": bpn, "finite": diag["finite"], "repeats": rep}


def serving(n_requests):
    """The seeded request stream (Poisson arrivals at 20/s, boxes 32..128,
    droplet/jet, Re 500..5000, We 10..2000, 500..5000 steps) through the
    serving group."""
    from paper_2403_15773_amd import serve
    from paper_2403_15773_amd.tslb import Group, device_memory
    reqs = serve.make_requests(n_requests, rate=20.0, master_seed=5)
    free, total = device_memory(0)
    budget = max(0, free - total // 16)  # admission by free HBM, less a reserve of 1/16 of the device
    log("serving %d requests, budget %.1f GB of free HBM" % (n_requests, budget / 1e9))
    t0 = time.perf_counter()
    with Group(hbm_budget_bytes=budget, max_domains=64) as g:
        backend = serve.GpuBackend(g)
        recs = serve.serve(reqs, backend, budget, max_domains=64)
        busy = backend.busy_seconds()
    s = serve.summarise(recs, busy_s=busy)
    log("serving: p50 %.2f s, p99 %.2f s, %.2f GLUPS aggregate (offered %.2f), device busy %.1f %%, %d unstable, "
        "%.1f s wall" % (s["p50_latency_s"], s["p99_latency_s"], s["aggregate_glups"], s["offered_glups"],
                         100 * s["device_busy_frac"], s["unstable"], time.perf_counter() - t0))
    s["budget_bytes"] = budget
    s["stream"] = ("%d requests, Poisson arrivals 20/s (master seed 5), cubic L in {32,48,64,96,128}, droplet/jet "
                   "50/50, Re log-U[500,5000], We log-U[10,2000], steps U{500..5000}, FP32, admitted by free HBM "
                   "(hipMemGetInfo at the start, less 1/16 of the device), 64 domain slots" % n_requests)
    return s


# Workloads whose FP64 population oracle does not fit in host memory take the
# oracle's rate on a smaller lattice of the same set-up (the rate is per node).
CPU_SAMPLE_WORKLOAD = {"jet512": "jet128"}


def cpu_baseline(name, p, st, budget_s):
    """The FP64 oracle as it stands, on this host's cores, for a bounded number of
    steps of the same workload (or of CPU_SAMPLE_WORKLOAD's stand-in); rate in GLUPS."""
    if budget_s <= 0:
        return None
    import numpy as np

    quoted = CPU_SAMPLE_WORKLOAD.get(name)
    if quoted is not None:
        p, st = workload_state(quoted)

    from oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    o = Oracle(p["nx"], p["ny"], p["nz"], nu=p["nu"], sigma=p["sigma"], width=p["width"], eps=1e-4, bc=p["bc"],
               inlet_u=p.get("inlet_u", 0.0), inlet_d=p.get("inlet_d", 0.0), inlet_noise=p.get("inlet_noise", 0.0),
               seed=p.get("seed", 0), rho_a=p.get("density_a"), rho_b=p.get("density_b"), nu_a=p.get("nu_a"),
               nu_b=p.get("nu_b"))
    if st is None:
        from paper_2403_15773_amd import inputs
        st = inputs.quiescent(p["nx"], p["ny"], p["nz"])
    o.set_physical(**{k: np.asarray(v, np.float64) for k, v in st.items()})
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    n = max(1, min(1000, int(budget_s / max(t1 - t0, 1e-6)) - 1))
    o.step(n)
    t2 = time.perf_counter()
    steps = n + 1
    nodes = p["nx"] * p["ny"] * p["nz"]
    # the same oracle on one core, continuing from the state reached (OpenMP is its only parallelism)
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(1)
    try:
        t3 = time.perf_counter()
        o.step(1)
        t4 = time.perf_counter()
        n1 = max(0, min(100, int(budget_s / 3 / max(t4 - t3, 1e-6)) - 1))
        o.step(n1)
        t5 = time.perf_counter()
    finally:
        gomp.omp_set_num_threads(threads)
    o.close()
    one = {"value": nodes * (n1 + 1) / (t5 - t3) / 1e9, "unit": "GLUPS", "cores": 1,
           "sample": "%d step%s of the same workload on one thread, %.1f s" % (n1 + 1, "" if n1 == 0 else "s", t5 - t3)}
    what = ("%d steps of the full %dx%dx%d workload (FP64 populations, OpenMP), %.1f s"
            % (steps, p["nx"], p["ny"], p["nz"], t2 - t0))
    if quoted is not None:
        what = ("quoted from the %dx%dx%d jet of the same set-up (the %s lattice's FP64 populations do not fit in "
                "host memory): %s" % (p["nx"], p["ny"], p["nz"], name, what))
    return {"value": nodes * steps / (t2 - t0) / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": what, "single_core": one}


def projection_probe(nodes, reps):
    """The moment-to-population projection timed on the vector ALU (the step's
    tensor product) and as FP32 matrix-core tiles, on the same seeded inputs."""
    import numpy as np

    from paper_2403_15773_amd.tslb import PROJECTION_MFMA, PROJECTION_VALU
    from paper_2403_15773_amd.tslb import projection_probe as probe
    coef = np.random.default_rng(3).uniform(-0.05, 0.05, (16, nodes)).astype(np.float32)
    flops = 2.0 * 27 * 16 * nodes * reps  # the map as a dense 27 x 16 product
    res = {"nodes": nodes, "reps": reps, "flop_per_projection": 2 * 27 * 16}
    for name, kind in (("valu", PROJECTION_VALU), ("mfma_fp32", PROJECTION_MFMA)):
        ms, _ = probe(kind, coef, reps, iters=10, want_out=False)
        res[name] = {"ms": ms, "tflops_equivalent": flops / (ms * 1e-3) / 1e12}
    res["mfma_over_valu_time"] = res["mfma_fp32"]["ms"] / res["valu"]["ms"]
    log("projection probe: valu %.4f ms, mfma fp32 %.4f ms (%.2fx the time)" % (
        res["valu"]["ms"], res["mfma_fp32"]["ms"], res["mfma_over_valu_time"]))
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: the TSLB step here runs on one GPU (multi-GPU sharding is a design only); --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_2403_15773_amd.tslb import copy_bandwidth

    copy = None
    if a.copy_mib > 0:
        gbps, cms = copy_bandwidth(a.copy_mib << 20, iters=20)
        copy = {"gbps": gbps, "ms": cms, "bytes_moved": 2 * (a.copy_mib << 20)}
        log("copy-kernel ceiling %.0f GB/s (%d MiB read + written, %.3f ms)" % (gbps, 2 * a.copy_mib, cms))
    m = run_lattice(a.workload, a.storage, a.steps, a.warmup, a.kernel, repeats=a.repeats)
    p, nodes, achieved = m["p"], m["nodes"], m["achieved"]
    traffic = measured_traffic(a.workload, a.storage) if a.kernel == "fused" else None
    variants = {}
    for v in [s for s in a.variants.split(",") if s and s != a.storage]:
        r = run_lattice(a.workload, v, a.steps, a.warmup, a.kernel)
        variants[v] = {"value": r["glups"], "unit": "GLUPS", "kernel_ms": r["kernel_ms"],
                       "roofline_frac": r["achieved"] / HBM_PEAK_GBS if r["achieved"] else None,
                       "bytes_per_node": r["bpn"], "speedup_vs_%s" % a.storage: r["glups"] / m["glups"],
                       "finite": r["finite"]}
    secondary = None
    if a.secondary and a.secondary != a.workload:
        r = run_lattice(a.secondary, "fp32", a.steps, a.warmup, a.kernel)
        t2 = measured_traffic(a.secondary, "fp32") if a.kernel == "fused" else None
        secondary = describe(a.secondary, r["p"]) | {
            "storage": "fp32", "value": r["glups"], "unit": "GLUPS", "ms_per_step": r["T"] / a.steps * 1e3,
            "kernel_ms": r["kernel_ms"], "kernel_ms_spread": r["kernel_ms_spread"], "bytes_per_node": r["bpn"],
            "roofline_frac": r["achieved"] / HBM_PEAK_GBS if r["achieved"] else None,
            "traffic": t2, "traffic_vs_algorithmic": t2 / (r["bpn"] * r["nodes"]) if t2 else None,
            "finite": r["finite"]}
    single = None
    if a.single and a.workload != "tgv256":
        r = run_lattice("tgv256", "fp32", a.steps, a.warmup, a.kernel)
        t1 = measured_traffic("tgv256", "fp32") if a.kernel == "fused" else None
        single = {"workload": describe("tgv256", r["p"])["workload"], "nodes": r["nodes"], "value": r["glups"],
                  "traffic": t1, "traffic_vs_algorithmic": t1 / (r["bpn"] * r["nodes"]) if t1 else None,
                  "unit": "GLUPS", "kernel_ms": r["kernel_ms"], "bytes_per_node": r["bpn"],
                  "roofline_frac": r["achieved"] / HBM_PEAK_GBS if r["achieved"] else None,
                  "frac_of_copy_ceiling": r["achieved"] / copy["gbps"] if (copy and r["achieved"]) else None,
                  "finite": r["finite"]}
    paper = None
    if a.paper_domain and a.workload != "jet400":
        r = run_lattice("jet400", "fp32", a.steps, a.warmup, a.kernel)
        paper = describe("jet400", r["p"]) | {
            "value": r["glups"], "unit": "GLUPS", "kernel_ms": r["kernel_ms"], "bytes_per_node": r["bpn"],
            "roofline_frac": r["achieved"] / HBM_PEAK_GBS if r["achieved"] else None, "finite": r["finite"],
            "paper_glups_other_hardware": {"RTX 3090": 1.5, "A100": 2.0},
            "note": "the paper's own jet domain (128 million nodes) and its quoted GLUPS on other hardware and "
                    "code: context, not a baseline of this metric"}
    vd = None
    if a.vd and a.workload != "jet128vd":
        r = run_lattice("jet128vd", "fp32", a.steps, a.warmup, a.kernel)
        vd = describe("jet128vd", r["p"]) | {
            "value": r["glups"], "unit": "GLUPS", "kernel_ms": r["kernel_ms"], "bytes_per_node": r["bpn"],
            "roofline_frac": r["achieved"] / HBM_PEAK_GBS if r["achieved"] else None, "finite": r["finite"]}
    busy = None
    if a.busy:
        r = run_lattice(a.workload, a.storage, a.steps, a.warmup, a.kernel, smooth=True)
        busy = {"value": r["nodes"] / (r["kernel_ms"] * 1e-3) / 1e9, "unit": "GLUPS (kernel time)",
                "kernel_ms": r["kernel_ms"], "kernel_ms_spread": r["kernel_ms_spread"],
                "roofline_frac": r["achieved"] / HBM_PEAK_GBS if r["achieved"] else None,
                "time_vs_config_start": r["kernel_ms"] / m["kernel_ms"], "finite": r["finite"],
                "note": "the same lattice and step from a smooth state with no quiescent node (phi in [0.1, 0.9], "
                        "|u| <= 0.02 on every node); the headline starts as its configuration does, from rest, "
                        "and the step's time depends on the data it moves"}
    rec = {
        "metric": "GLUPS (lattice-node updates per second / 1e9) and fraction of the HBM roofline",
        "value": m["glups"],
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": m["T"] / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.storage == "fp32" else "f32 (%s-stored moments)" % a.storage,
        "data": "synthetic",
        "config": describe(a.workload, p) | {"storage": a.storage, "finite": m["finite"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, copy-kernel scaled)",
                     "traffic_vs_algorithmic": traffic / (m["bpn"] * nodes) if traffic else None,
                     "kernel": "%s step" % a.kernel, "bytes_per_node": m["bpn"], "kernel_ms": m["kernel_ms"],
                     "kernel_ms_spread": m["kernel_ms_spread"],
                     "copy_ceiling": copy["gbps"] if copy else None,
                     "frac_of_copy_ceiling": achieved / copy["gbps"] if (copy and achieved) else None},
        "repeat_runs": ({"glups": [m["glups"]] + m["repeats"],
                         "median_glups": float(statistics.median([m["glups"]] + m["repeats"])),
                         "note": "the timed region (value) and %d further runs of the same number of steps on the same "
                                 "lattice right after it, each by the wall clock around it" % len(m["repeats"])}
                        if m["repeats"] else None),
        "busy_state": busy,
        "storage_variants": variants,
        "secondary": secondary,
        "single_component": single,
        "variable_density": vd,
        "paper_domain": paper,
        "projection_probe": projection_probe(1 << 22, 64) if a.probe else None,
        "serving": serving(a.serve) if a.serve > 0 else None,
        "cpu_baseline": cpu_baseline(a.workload, p, m["st"], a.cpu_seconds),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
