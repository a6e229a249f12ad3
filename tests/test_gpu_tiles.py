"""The fused step's two tile heights (32 x 16 and 32 x 20 destination columns
per workgroup): the library's choice per lattice, and the result bitwise the
same at either height, alone and in a serving group, on lattices whose tiles
are partial in y."""
import numpy as np
import pytest

from paper_2403_15773_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def _run(p, st, steps, rows, chunk=0):
    from paper_2403_15773_amd.tslb import Simulation
    with Simulation(**p, eps=1e-4) as s:
        s.set_kernel("fused", chunk)
        s.set_tile(rows)
        assert s.tile_rows == rows
        s.set_state(rho_dev=np.asarray(st["rho"] - 1.0, np.float32), u=np.asarray(st["u"], np.float32),
                    P=np.asarray(st["P"], np.float32), phi=np.asarray(st["phi"], np.float32))
        s.step(steps)
        return s.get_state_raw(), s.diagnostics()


@pytest.mark.parametrize("case", ["droplet", "jet"])
def test_result_is_bitwise_the_same_at_16_and_20_rows(case):
    if case == "droplet":
        st = inputs.droplet(40, 9.0, seed=3)
        p = dict(nx=40, ny=40, nz=40, nu=0.02, sigma=0.01, width=3.0)
    else:  # inlet, outflow and free-slip walls; 44 rows: partial tiles at both heights
        p = inputs.jet_params(48, 44, 60, d=10.0, u=0.05, re=500.0, we=50.0, seed=7)
        st = inputs.quiescent(48, 44, 60)
    _say("%s: 16 against 20 rows, 60 steps" % case)
    a, da = _run(p, st, 60, 16)
    b, db = _run(p, st, 60, 20)
    c, _ = _run(p, st, 60, 20, chunk=7)  # and a short chunk on the 20-row tiles
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert da["finite"] and da["mass"] == db["mass"] and da["phase"] == db["phase"]


def test_library_choice_of_tile_height():
    """The cost model takes 20 rows where it gives every compute unit less time
    (the 512 x 512 x 2048 jet) and 16 where 20-row tiles fill the device worse
    (the 128 x 128 x 512 jet); one component and variable density take 16, and
    20 rows are refused for them."""
    from paper_2403_15773_amd.tslb import Simulation, TslbError
    big = inputs.WORKLOADS["jet512"]["params"]
    with Simulation(**big, eps=1e-4) as s:
        assert s.tile_rows == 20
    with Simulation(**inputs.WORKLOADS["jet128"]["params"], eps=1e-4) as s:
        assert s.tile_rows == 16
        s.set_tile(20)
        assert s.tile_rows == 20
        s.set_tile(0)
        assert s.tile_rows == 16
    with Simulation(**inputs.WORKLOADS["tgv256"]["params"], eps=1e-4) as s:
        assert s.tile_rows == 16
        with pytest.raises(TslbError):
            s.set_tile(20)
    with Simulation(nx=32, ny=32, nz=32, nu=0.1, sigma=0.01, width=3.0, eps=1e-4,
                    density_a=2.0, density_b=1.0, nu_a=0.05, nu_b=0.05) as s:
        assert s.tile_rows == 16
        with pytest.raises(TslbError):
            s.set_tile(20)


def test_twenty_row_member_in_a_group_is_bitwise_alone():
    from paper_2403_15773_amd.tslb import Group, Simulation
    _say("20-row and 16-row members in one serving group")
    st = inputs.droplet(36, 8.0, seed=4)
    f32 = {"rho_dev": np.asarray(st["rho"] - 1.0, np.float32), "u": np.asarray(st["u"], np.float32),
           "P": np.asarray(st["P"], np.float32), "phi": np.asarray(st["phi"], np.float32)}
    p = dict(nx=36, ny=36, nz=36, nu=0.03, sigma=0.01, width=3.0, eps=1e-4)
    alone = []
    for rows, n in ((20, 13), (16, 9)):
        with Simulation(**p) as s:
            s.set_tile(rows)
            s.set_state(**f32)
            s.step(n)
            alone.append(s.get_state_raw())
    sims = []
    for rows in (20, 16):
        s = Simulation(**p)
        s.set_tile(rows)
        s.set_state(**f32)
        sims.append(s)
    with Group(hbm_budget_bytes=1 << 30, max_domains=4) as grp:
        for s, n in zip(sims, (13, 9)):
            assert grp.admit(s, n)
        left = 2
        while left:
            left -= len(grp.poll())
    for s, a in zip(sims, alone):
        assert np.array_equal(s.get_state_raw(), a)
        s.close()
