"""Time-averaged statistics of a round jet (Results, self-similarity of the jets).

Runs a jet from rest, accumulates on the device the time averages of phi, u and
u_z^2 every `every` steps from step `avg_from` on, and fits:
* U/U_c(z) and 1/phi_c(z) = (z - z0)/(B D) over a window beyond the potential
  core (the paper finds slopes 1/B near 1/6.5 per diameter);
* the Gaussian exponents K of the mean axial-velocity and phase profiles at a
  distance from the nozzle (the paper shows K = 75 for the velocity at 12 D and
  K = 80 for the phase field at We = 2000).

Prints one JSON line; with --out also writes the centreline arrays and the
mid-plane (y = ny/2) slices of the averages to an .npz file.

    python -m paper_2403_15773_amd.jetstats --nx 200 --ny 200 --nz 400 --d 20 \\
        --re 5000 --we 2000 --steps 60000 --avg-from 20000 --every 10
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import analysis, inputs


def log(msg):
    print("[jetstats] " + msg, file=sys.stderr, flush=True)


def run(nx, ny, nz, d, u, re, we, steps, avg_from, every, seed=2, chunk=2000, z_window=None, z_profile=12.0,
        storage="fp32"):
    from .tslb import Simulation
    p = inputs.jet_params(nx, ny, nz, d=d, u=u, re=re, we=we, seed=seed)
    res = {"config": {"nx": nx, "ny": ny, "nz": nz, "D": d, "U": u, "Re": re, "We": we, "steps": steps,
                      "avg_from": avg_from, "every": every, "storage": storage}}
    with Simulation(**p, eps=1e-4, storage=storage, u_scale=u) as s:
        s.set_state_raw(np.zeros(s.state_bytes, np.uint8), step=0)  # rest: rho = 1, u = 0, P = 0, phi = 0
        t_plain = t_stats = 0.0
        n_plain = n_stats = 0
        done = 0
        while done < steps:
            if done == avg_from:
                s.stats_start(every)
            n = min(chunk, steps - done, avg_from - done if done < avg_from else steps)
            s.sync()
            t0 = time.perf_counter()
            s.step(n)
            s.sync()
            dt = time.perf_counter() - t0
            if done >= avg_from:
                t_stats, n_stats = t_stats + dt, n_stats + n
            else:
                t_plain, n_plain = t_plain + dt, n_plain + n
            done += n
            diag = s.diagnostics()
            log("step %d of %d (%.3f ms/step) finite=%s" % (done, steps, 1e3 * dt / n, diag["finite"]))
            if not diag["finite"]:
                res["finite"] = False
                return res, None
        st = s.stats()
    res["finite"] = True
    res["samples"] = st["samples"]
    res["ms_per_step"] = 1e3 * t_plain / n_plain if n_plain else None
    res["ms_per_step_with_stats"] = 1e3 * t_stats / n_stats if n_stats else None
    res["glups"] = nx * ny * nz / (t_plain / n_plain) / 1e9 if n_plain else None

    mphi, uz = st["mean_phi"], st["mean_u"][2]
    phic, uc = analysis.centreline(mphi), analysis.centreline(uz)
    # beyond the potential core (about 6-7 D at high We) and clear of the last
    # 8 D, where the outflow layer bends the mean flow of a 20 D box
    zw = z_window or (int(8 * d), int(nz - 8 * d))
    if zw[1] - zw[0] < 2:  # a short box: the middle of it
        zw = (int(0.45 * nz), int(0.75 * nz))
    B_u, z0_u = analysis.decay_constant(uc, u, d, zw)
    B_phi, z0_phi = analysis.decay_constant(phic, 1.0, d, zw)
    zp = min(int(round(z_profile * d)), nz - 1 - int(d))  # stay a diameter clear of the outflow
    res.update({"z_window_D": [zw[0] / d, zw[1] / d], "B_u": B_u, "z0_u_D": z0_u, "B_phi": B_phi,
                "z0_phi_D": z0_phi, "z_profile_D": zp / d,
                "K_u": analysis.gaussian_exponent(uz[zp], zp, z0_u * d),
                "K_phi": analysis.gaussian_exponent(mphi[zp], zp, z0_phi * d),
                "half_width_u_D": analysis.half_width(uz[zp]) / d})
    arrays = {"phi_c": phic, "u_c": uc, "mean_phi_xz": mphi[:, ny // 2, :], "mean_uz_xz": uz[:, ny // 2, :],
              "rms_uz_xz": st["rms_uz"][:, ny // 2, :], "mean_uz_zp": uz[zp], "mean_phi_zp": mphi[zp]}
    return res, arrays


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--nx", type=int, default=200)
    ap.add_argument("--ny", type=int, default=200)
    ap.add_argument("--nz", type=int, default=400)
    ap.add_argument("--d", type=float, default=20.0)
    ap.add_argument("--u", type=float, default=0.05)
    ap.add_argument("--re", type=float, default=5000.0)
    ap.add_argument("--we", type=float, default=2000.0)
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--avg-from", type=int, default=20000)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--chunk", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--storage", default="fp32")
    ap.add_argument("--z-profile", type=float, default=12.0, help="distance of the radial profiles, in D")
    ap.add_argument("--z-window", type=float, nargs=2, default=None, help="fit window of the decay laws, in D")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if not 0 <= a.avg_from < a.steps:
        ap.error("need 0 <= avg-from < steps")
    res, arrays = run(a.nx, a.ny, a.nz, a.d, a.u, a.re, a.we, a.steps, a.avg_from, a.every, seed=a.seed,
                      chunk=a.chunk, z_window=None if a.z_window is None else (int(a.z_window[0] * a.d), int(a.z_window[1] * a.d)),
                      z_profile=a.z_profile, storage=a.storage)
    if a.out and arrays is not None:
        np.savez_compressed(a.out, **arrays)
    print(json.dumps(res), flush=True)
    return 0 if res["finite"] else 1


if __name__ == "__main__":
    sys.exit(main())
