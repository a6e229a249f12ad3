"""On-device time averages (tslb_stats_*) against time averages of the FP64
oracle's fields over the same steps, and their bookkeeping."""
import numpy as np
import pytest

from paper_2403_15773_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 1e-4
TOL = 1e-5


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def test_jet_time_averages_match_oracle():
    """24 x 24 x 40 mini-jet from step 5: sampling every 4 steps over steps 41..200
    (40 samples); mean phi and mean u per field within 1e-5 of the oracle's
    relative to the field's largest value, rms u_z within 1e-5 of U."""
    from oracle import Oracle
    from paper_2403_15773_amd.tslb import Simulation
    from test_gpu_parity import _f32, _oracle_inputs
    _say("stats mini-jet 24x24x40 fp32, every 4 steps over 41..200")
    p = inputs.jet_params(24, 24, 40, d=8.0, u=0.05, re=400.0, we=40.0, seed=9)
    st = _f32(inputs.quiescent(24, 24, 40))
    every, first, last = 4, 40, 200
    with Simulation(**p, eps=EPS) as s:
        s.set_state(**st, step=5)
        s.step(first - 5)
        s.stats_start(every)
        s.step(last - first)
        g = s.stats()
    o = Oracle(p["nx"], p["ny"], p["nz"], nu=p["nu"], sigma=p["sigma"], width=p["width"], eps=EPS, bc=p["bc"],
               inlet_u=p["inlet_u"], inlet_d=p["inlet_d"], inlet_noise=p["inlet_noise"], seed=p["seed"])
    o.set_physical(**_oracle_inputs(st), step=5)
    o.step(first - 5)
    acc = {"phi": 0.0, "u": 0.0, "uz2": 0.0}
    n = 0
    for _ in range(last - first):
        o.step(1)
        if o.step_count % every == 0:
            r = o.physical()
            acc["phi"] = acc["phi"] + r["phi"]
            acc["u"] = acc["u"] + r["u"]
            acc["uz2"] = acc["uz2"] + r["u"][2] ** 2
            n += 1
    o.close()
    assert g["samples"] == n == 40
    mphi, mu = acc["phi"] / n, acc["u"] / n
    rms = np.sqrt(np.maximum(acc["uz2"] / n - mu[2] ** 2, 0.0))
    errs = {"phi": np.abs(g["mean_phi"] - mphi).max() / np.abs(mphi).max()}
    for a in range(3):
        errs["u" + "xyz"[a]] = np.abs(g["mean_u"][a] - mu[a]).max() / np.abs(mu[a]).max()
    errs["rms_uz/U"] = np.abs(g["rms_uz"] - rms).max() / p["inlet_u"]
    _say("stats vs oracle: " + " ".join("%s=%.2e" % kv for kv in errs.items()) +
         " (max rms u_z %.3e)" % rms.max())
    assert rms.max() > 1e-4  # the window holds a developing jet, not a steady state
    assert max(errs.values()) <= TOL


def test_stats_bookkeeping():
    """No samples before start or at steps off the period; a restart clears the
    sums; stop freezes them; a steady field averages to itself with zero rms."""
    from paper_2403_15773_amd.tslb import Simulation, TslbError
    _say("stats bookkeeping 16^3 periodic uniform flow")
    st = inputs.quiescent(16, 16, 16)
    st["u"][0] = 0.02
    st["rho_dev"] = np.zeros((16, 16, 16), np.float32)
    del st["rho"]
    with Simulation(nx=16, ny=16, nz=16, nu=0.05, sigma=0.01, width=3.0, eps=EPS) as s:
        s.set_state(**{k: np.asarray(v, np.float32) for k, v in st.items()}, step=0)
        assert s.stats_samples() == 0
        with pytest.raises(TslbError):
            s.stats()
        s.stats_start(3)
        s.step(2)
        assert s.stats_samples() == 0
        with pytest.raises(TslbError):
            s.stats()
        s.step(7)  # steps 3, 6, 9
        assert s.stats()["samples"] == s.stats_samples() == 3
        s.stats_start(1)
        s.step(2)
        g = s.stats()
        assert g["samples"] == 2
        assert np.allclose(g["mean_u"][0], 0.02, rtol=1e-6, atol=0) and np.abs(g["mean_u"][1:]).max() < 1e-7
        assert g["rms_uz"].max() < 1e-6
        s.stats_stop()
        s.step(3)
        assert s.stats_samples() == 2
        with pytest.raises(TslbError):
            s.stats_start(0)


def test_single_component_time_averages_match_oracle():
    """One component (no phase plane): the 24 x 24 x 40 single-phase jet, sampling every
    5 steps over steps 21..120; mean u and rms u_z against the sigma = 0 oracle's fields,
    mean phi identically zero."""
    from oracle import Oracle
    from paper_2403_15773_amd.tslb import Simulation
    from test_gpu_parity import _f32, _oracle_inputs
    _say("stats single component mini-jet 24x24x40")
    p = inputs.jet_params(24, 24, 40, d=8.0, u=0.05, re=400.0, we=40.0, seed=9)
    st = _f32(inputs.quiescent(24, 24, 40))
    every, first, last = 5, 20, 120
    with Simulation(**p, components=1) as s:
        s.set_state(rho_dev=st["rho_dev"], u=st["u"], P=st["P"], phi=None, step=0)
        s.step(first)
        s.stats_start(every)
        s.step(last - first)
        g = s.stats()
    o = Oracle(p["nx"], p["ny"], p["nz"], nu=p["nu"], sigma=0.0, width=p["width"], eps=EPS, bc=p["bc"],
               inlet_u=p["inlet_u"], inlet_d=p["inlet_d"], inlet_noise=p["inlet_noise"], seed=p["seed"])
    o.set_physical(**_oracle_inputs(st), step=0)
    o.step(first)
    su, suz2, n = 0.0, 0.0, 0
    for _ in range(last - first):
        o.step(1)
        if o.step_count % every == 0:
            r = o.physical()
            su = su + r["u"]
            suz2 = suz2 + r["u"][2] ** 2
            n += 1
    o.close()
    assert g["samples"] == n == 20
    mu = su / n
    rms = np.sqrt(np.maximum(suz2 / n - mu[2] ** 2, 0.0))
    errs = {"u" + "xyz"[a]: np.abs(g["mean_u"][a] - mu[a]).max() / np.abs(mu[a]).max() for a in range(3)}
    errs["rms_uz/U"] = np.abs(g["rms_uz"] - rms).max() / p["inlet_u"]
    _say("single-component stats vs oracle: " + " ".join("%s=%.2e" % kv for kv in errs.items()))
    assert not g["mean_phi"].any()
    assert max(errs.values()) <= TOL
