"""GPU checks of the serving group (continuous batching through the C-ABI).

The step of one lattice reads and writes only that lattice, so a request run
inside a mixed group must give bitwise the state it gets when run alone with
tslb_step; admission by HBM budget must defer and later accept; a member is
locked while the group owns it."""
import numpy as np
import pytest

from paper_2403_15773_amd import serve

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def _mix_requests():
    """8 requests covering both set-ups and every box side, short runs."""
    spec = [(32, "droplet", 800.0, 50.0, 37), (48, "jet", 2000.0, 300.0, 52), (64, "droplet", 1500.0, 20.0, 45),
            (96, "jet", 600.0, 1000.0, 30), (128, "droplet", 3000.0, 100.0, 24), (32, "jet", 500.0, 10.0, 61),
            (48, "droplet", 4000.0, 2000.0, 40), (128, "jet", 1000.0, 150.0, 28)]
    return [serve.Request(i, 0.0, L, s, re, we, n, 1000 + i) for i, (L, s, re, we, n) in enumerate(spec)]


def _alone(req):
    from paper_2403_15773_amd.tslb import Simulation
    p, f = serve.request_setup(req)
    with Simulation(**p) as s:
        s.set_state(**f)
        s.step(req.steps)
        return s.get_state_raw(), s.step_index


def test_group_results_equal_alone_runs_bitwise():
    from paper_2403_15773_amd.tslb import Group, Simulation
    reqs = _mix_requests()
    _say("group mix of %d requests (sides %s)" % (len(reqs), sorted({r.L for r in reqs})))
    alone = {r.id: _alone(r) for r in reqs}
    got = {}
    with Group(hbm_budget_bytes=8 << 30, max_domains=8) as g:
        sims = {}
        waves = [reqs[:3], reqs[3:6], reqs[6:]]
        polls = 0
        while waves or g.status()["members"]:
            if waves and polls % 9 == 0:  # requests join while others run
                for r in waves.pop(0):
                    p, f = serve.request_setup(r)
                    s = Simulation(**p)
                    s.set_state(**f)
                    assert g.admit(s, r.steps)
                    sims[s.h.value] = (r, s)
            for s in g.poll():
                r, _ = sims[s.h.value]
                got[r.id] = (s.get_state_raw(), s.step_index)
                s.close()
            polls += 1
            assert polls < 10000
    assert sorted(got) == sorted(alone)
    for r in reqs:
        assert got[r.id][1] == alone[r.id][1] == r.steps
        assert np.array_equal(got[r.id][0], alone[r.id][0]), "request %d (%s L=%d) differs" % (r.id, r.setup, r.L)


def test_group_budget_defers_then_admits():
    from paper_2403_15773_amd.tslb import Group, Simulation
    _say("group HBM budget deferral")
    a = serve.Request(0, 0.0, 32, "droplet", 1000.0, 100.0, 10, 1)
    b = serve.Request(1, 0.0, 32, "jet", 1000.0, 100.0, 5, 2)
    pa, fa = serve.request_setup(a)
    pb, fb = serve.request_setup(b)
    sa, sb = Simulation(**pa), Simulation(**pb)
    sa.set_state(**fa)
    sb.set_state(**fb)
    from paper_2403_15773_amd.tslb import required_bytes
    assert required_bytes(sa.params) == required_bytes(sb.params) == 2 * sa.state_bytes  # both state buffers
    need = sa.device_bytes  # the state buffers and the diagnostics partials: what the lattice holds
    assert need == sb.device_bytes and 2 * sa.state_bytes < need < 2 * sa.state_bytes + (1 << 20)
    with Group(hbm_budget_bytes=need + need // 2, max_domains=4) as g:
        assert g.admit(sa, a.steps)
        assert not g.admit(sb, b.steps)  # over budget: defer
        assert g.status()["bytes_in_use"] == need
        done = []
        while not done:
            done = g.poll()
        assert done[0] is sa and sa.step_index == 10
        assert g.admit(sb, b.steps)
        done = []
        while not done:
            done = g.poll()
        assert done[0] is sb and sb.step_index == 5
        assert g.status()["members"] == 0 and g.status()["bytes_in_use"] == 0
    sa.close()
    sb.close()


def test_group_charge_matches_the_device_memory_a_member_holds():
    """Admission charges what a lattice holds between calls: its state buffers
    and diagnostics partials.  The staging and geometry planes of set-state and
    readout are released before those calls return."""
    from paper_2403_15773_amd.tslb import Group, Simulation, device_memory
    _say("group charge vs device memory held")
    r = serve.Request(0, 0.0, 128, "droplet", 1000.0, 100.0, 3, 5)
    p, f = serve.request_setup(r)
    with Simulation(**p) as w:  # code objects and runtime pools loaded before the measurement
        w.set_state(**f)
        w.moments()
    free0, _ = device_memory(0)
    s = Simulation(**p)
    s.set_state(**f)
    s.moments()
    free1, _ = device_memory(0)
    held = free0 - free1
    charge = s.device_bytes
    assert charge > 2 * s.state_bytes
    # allocation granularity and the stream's own runtime memory: within 16 MiB
    assert abs(held - charge) <= 16 << 20, (held, charge)
    with Group(hbm_budget_bytes=charge, max_domains=2) as g:
        assert g.admit(s, r.steps)
        assert g.status()["bytes_in_use"] == charge
        while not g.poll():
            pass
    s.close()


def test_group_member_is_locked_and_zero_steps_retire():
    from paper_2403_15773_amd.tslb import E_STATE, Group, Simulation, TslbError
    _say("group member lock, zero-step admission")
    r = serve.Request(0, 0.0, 32, "droplet", 1000.0, 100.0, 3, 5)
    p, f = serve.request_setup(r)
    s = Simulation(**p)
    s.set_state(**f)
    raw0 = s.get_state_raw()
    with Group(hbm_budget_bytes=1 << 30, max_domains=2) as g:
        assert g.admit(s, 0)
        with pytest.raises(TslbError) as e:
            s.step(1)
        assert e.value.code == E_STATE
        done = []
        for _ in range(100):
            done = g.poll()
            if done:
                break
        assert done == [s] and s.step_index == 0
        assert np.array_equal(s.get_state_raw(), raw0)
        assert g.admit(s, 3)
        with pytest.raises(TslbError):
            g.admit(s, 1)  # already a member
        assert g.poll() == []  # launches step 1 of 3
    # destroying the group frees its members at the step they reached
    assert s.step_index == 1
    s.step(1)
    assert s.step_index == 2
    s.close()


def test_small_serving_stream_completes():
    from paper_2403_15773_amd.tslb import Group
    reqs = serve.make_requests(12, rate=200.0, master_seed=9, sizes=(32, 48), re=(200.0, 600.0), steps=(50, 150))
    _say("serving stream of %d requests" % len(reqs))
    with Group(hbm_budget_bytes=256 << 20, max_domains=6) as g:
        recs = serve.serve(reqs, serve.GpuBackend(g), 256 << 20, max_domains=6)
    s = serve.summarise(recs)
    _say("p50 %.3f s p99 %.3f s aggregate %.2f GLUPS unstable %d" % (
        s["p50_latency_s"], s["p99_latency_s"], s["aggregate_glups"], s["unstable"]))
    assert s["unstable"] == 0 and s["requests"] == 12
    for rec in recs:
        assert rec.extra["step"] == rec.req.steps
        assert rec.req.arrival <= rec.admitted <= rec.done


def test_group_mixes_one_and_two_component_lattices_bitwise():
    """A group holding one- and two-component lattices of several storage types
    launches one kernel per class; every member still ends bitwise equal to its
    run alone."""
    from paper_2403_15773_amd.tslb import Group, Simulation
    _say("group mix of one- and two-component lattices")
    reqs = _mix_requests()[:7]
    cases = [(reqs[0], 1, "fp32"), (reqs[1], 2, "fp32"), (reqs[2], 1, "fp16q"), (reqs[3], 2, "fp16"),
             (reqs[4], 2, "bf16"), (reqs[5], 2, "fp16q"), (reqs[6], 1, "bf16")]

    def make(r, comps, storage):
        p, f = serve.request_setup(r)
        s = Simulation(**p, components=comps, storage=storage)
        s.set_state(**f) if comps == 2 else s.set_state(f["rho_dev"], f["u"], f["P"])
        return s

    alone = []
    for r, comps, storage in cases:
        with make(r, comps, storage) as s:
            s.step(r.steps)
            alone.append(s.get_state_raw())
    sims = [make(r, comps, storage) for r, comps, storage in cases]
    with Group(hbm_budget_bytes=8 << 30, max_domains=8) as g:
        for s, (r, _, _) in zip(sims, cases):
            assert g.admit(s, r.steps)
        left, polls = len(sims), 0
        while left:
            left -= len(g.poll())
            polls += 1
            assert polls < 10000
    for s, a, (r, comps, storage) in zip(sims, alone, cases):
        assert np.array_equal(s.get_state_raw(), a), "L=%d %d component(s) %s differs" % (r.L, comps, storage)
        s.close()


def test_group_of_walled_boxes_is_bitwise_equal_to_alone_runs():
    """Lattices whose faces take different rules (closed no-slip box, channel,
    outflow lid, a jet) in one multi-lattice launch: each member reads its own
    rule table, so each ends bitwise equal to its run alone."""
    from paper_2403_15773_amd import inputs
    from paper_2403_15773_amd.tslb import Group, Simulation
    _say("group of walled boxes")
    nx, ny, nz = 36, 20, 24
    node = np.arange(nx * ny * nz, dtype=np.uint64)
    x, y, z = inputs.grid_coords(nx, ny, nz)
    st = inputs.quiescent(nx, ny, nz)
    st["phi"] = 0.5 * (1 - np.tanh(2 * (np.sqrt((x - 17.2) ** 2 + (y - 9.6) ** 2 + (z - 11.3) ** 2) - 5.5) / 3.0))
    st["u"] = 0.01 * np.stack([inputs.noise(7, 0, 0, node, a).reshape(nz, ny, nx) for a in range(3)])
    fields = dict(rho_dev=np.zeros((nz, ny, nx), np.float32), u=st["u"].astype(np.float32),
                  P=np.zeros((6, nz, ny, nx), np.float32), phi=st["phi"].astype(np.float32))
    cases = [((4, 4, 4, 4, 4, 4), 40), ((1, 1, 4, 4, 0, 0), 33), ((4, 1, 1, 4, 4, 3), 27)]

    def make(bc):
        s = Simulation(nx=nx, ny=ny, nz=nz, nu=0.03, sigma=0.01, width=3.0, bc=bc, eps=1e-4)
        s.set_state(**fields)
        return s

    jet_p = inputs.jet_params(24, 24, 40, d=8.0, u=0.05, re=400.0, we=40.0, seed=9)

    def make_jet():
        s = Simulation(**jet_p, eps=1e-4)
        q = inputs.quiescent(24, 24, 40)
        s.set_state(rho_dev=np.zeros((40, 24, 24), np.float32), u=q["u"].astype(np.float32),
                    P=q["P"].astype(np.float32), phi=q["phi"].astype(np.float32))
        return s

    alone = []
    for bc, n in cases:
        with make(bc) as s:
            s.step(n)
            alone.append(s.get_state_raw())
    with make_jet() as s:
        s.step(31)
        alone.append(s.get_state_raw())
    sims = [make(bc) for bc, _ in cases] + [make_jet()]
    steps = [n for _, n in cases] + [31]
    with Group(hbm_budget_bytes=1 << 30, max_domains=8) as g:
        for s, n in zip(sims, steps):
            assert g.admit(s, n)
        left, polls = len(sims), 0
        while left:
            left -= len(g.poll())
            polls += 1
            assert polls < 10000
    for s, a, n in zip(sims, alone, steps):
        assert s.step_index == n
        assert np.array_equal(s.get_state_raw(), a), "bc %s differs" % (s.params.bc[:],)
        s.close()
