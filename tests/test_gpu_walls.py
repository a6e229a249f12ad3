"""The walled-step flows that pin the oracle (tests/test_oracle_walls.py), run
on the HIP path: the no-slip and free-slip channel shear modes (against the
oracle node by node after 200 steps, 1e-5 relative L-infinity of the velocity
and of the shear stress, and their decay rate against the closed form over 650
steps) and the uniform stream through inlet, outflow and free-slip faces."""
import numpy as np
import pytest

from paper_2403_15773_amd import inputs

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0
EPS = 1e-4
P_INDEX = {(0, 1): 3, (0, 2): 4, (1, 2): 5}


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def _mode_state(n, wall_axis, comp, rule, omega):
    dims = [4, 4, 4]
    dims[wall_axis] = n
    nx, ny, nz = dims
    st = inputs.quiescent(nx, ny, nz)
    s = inputs.grid_coords(nx, ny, nz)[wall_axis]
    if rule == 4:
        H, s0, mode, dmode = n - 1, 0.0, np.sin, np.cos
    else:
        H, s0, mode, dmode = n - 2, 0.5, np.cos, lambda v: -np.sin(v)
    k, A = np.pi / H, 1e-3
    st["u"][comp] = A * mode(k * (s - s0))
    st["P"][P_INDEX[tuple(sorted((wall_axis, comp)))]] = -(CS2 / omega) * A * k * dmode(k * (s - s0))
    bc = [0] * 6
    bc[2 * wall_axis] = bc[2 * wall_axis + 1] = rule
    return (nx, ny, nz), tuple(bc), st, k, mode(k * (np.arange(n) - s0))


@pytest.mark.parametrize("rule,n,wall_axis,comp", [(4, 65, 1, 0), (4, 65, 2, 1), (1, 129, 0, 2)])
def test_channel_shear_mode_against_oracle_and_closed_form(rule, n, wall_axis, comp):
    from oracle import Oracle
    from paper_2403_15773_amd.tslb import Simulation
    nu = 0.05
    omega = 1.0 / (3 * nu + 0.5)
    (nx, ny, nz), bc, st, k, basis = _mode_state(n, wall_axis, comp, rule, omega)
    _say("channel shear mode rule %d, %dx%dx%d" % (rule, nx, ny, nz))
    f32 = {"rho_dev": np.zeros((nz, ny, nx), np.float32), "u": st["u"].astype(np.float32),
           "P": st["P"].astype(np.float32), "phi": st["phi"].astype(np.float32)}
    sim = Simulation(nx=nx, ny=ny, nz=nz, nu=nu, sigma=0.0, eps=EPS, bc=bc)
    o = Oracle(nx, ny, nz, nu=nu, sigma=0.0, eps=EPS, bc=bc)
    sim.set_state(**f32)
    o.set_physical(rho=np.ones((nz, ny, nx)), u=f32["u"].astype(np.float64), P=f32["P"].astype(np.float64),
                   phi=f32["phi"].astype(np.float64))
    mean_axes = tuple(a for a in range(3) if a != 2 - wall_axis)
    sim.step(200)
    o.step(200)
    g = sim.physical()
    r = o.physical()
    o.close()
    ts, amps = [], []
    for _ in range(10):
        sim.step(50)
        u = sim.physical()["u"][comp].astype(np.float64).mean(axis=mean_axes)
        ts.append(sim.step_index)
        amps.append((u * basis).sum() / (basis ** 2).sum())
    sim.close()
    # the velocity against its own scale; the shear stress (nu k u, about 1 % of u here, below the
    # rounding of the populations that carry u) against the velocity scale; rho - 1 (rounding level
    # in this incompressible mode) by an absolute bound
    su = np.abs(r["u"][comp]).max()
    sP = P_INDEX[tuple(sorted((wall_axis, comp)))]
    for name, a, b, scale in [("u", g["u"][comp], r["u"][comp], su), ("P", g["P"][sP], r["P"][sP], su)]:
        err = np.abs(np.asarray(a, np.float64) - b).max() / scale
        _say("  %s: %.2e (scale %.2e, own max %.2e)" % (name, err, scale, np.abs(b).max()))
        assert err <= 1e-5, name
    assert np.abs(g["rho_dev"].astype(np.float64) - (r["rho"] - 1.0)).max() <= 1e-9
    rate = -np.polyfit(ts, np.log(amps), 1)[0]
    ratio = rate / (k ** 2 * CS2 * (1 / omega - 0.5))
    if rule == 4:
        assert ratio == pytest.approx(1.0, abs=5e-3)
    else:
        assert ratio == pytest.approx(1.0, abs=2e-2)


def test_uniform_stream_stays_uniform():
    from paper_2403_15773_amd.tslb import Simulation
    _say("uniform stream through inlet/outflow/free-slip")
    nx, ny, nz, U = 40, 36, 50, 0.05
    sim = Simulation(nx=nx, ny=ny, nz=nz, nu=0.02, sigma=1e-3, width=3.0, eps=EPS, bc=(1, 1, 1, 1, 2, 3),
                     inlet_u=U, inlet_d=1e6, inlet_noise=0.0, seed=1)
    st = inputs.quiescent(nx, ny, nz, phi=1.0)
    u = st["u"].astype(np.float32)
    u[2] = U
    sim.set_state(rho_dev=np.zeros((nz, ny, nx), np.float32), u=u, P=st["P"].astype(np.float32),
                  phi=st["phi"].astype(np.float32))
    sim.step(60)
    g = sim.physical()
    sim.close()
    # steady to binary32 rounding (an ulp of U is 3.7e-9)
    assert np.abs(g["rho_dev"]).max() <= 1e-7
    assert np.abs(g["u"][2] - np.float32(U)).max() <= 2e-6 * U
    assert np.abs(g["u"][:2]).max() <= 1e-7
    assert np.abs(g["P"]).max() <= 1e-7
    assert np.abs(g["phi"] - 1.0).max() == 0.0  # the phase streams in exact integers
