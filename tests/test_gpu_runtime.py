"""GPU checks of the runtime around the step: a caller-owned device buffer
(hipMalloc, or a torch allocation) and a caller's stream give results bitwise
equal to the library's own; every node of the state a step produces is written (the buffer
is poisoned first); the rest state; per-launch timing; the mass-drift bound."""
import numpy as np
import pytest

from paper_2403_15773_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 1e-4


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def _droplet(nx, ny, nz, seed=3):
    """A ragged droplet with velocity noise: (params, float32 fields)."""
    x, y, z = inputs.grid_coords(nx, ny, nz)
    st = inputs.quiescent(nx, ny, nz)
    r = np.sqrt((x - 0.45 * nx) ** 2 + (y - 0.55 * ny) ** 2 + (z - 0.5 * nz) ** 2)
    st["phi"] = 0.5 * (1 - np.tanh(2 * (r - 6.0) / 3.0))
    node = np.arange(nx * ny * nz, dtype=np.uint64)
    st["u"] = 0.01 * np.stack([inputs.noise(seed, 0, 0, node, a).reshape(nz, ny, nx) for a in range(3)])
    p = dict(nx=nx, ny=ny, nz=nz, nu=0.03, sigma=0.02, width=3.0, bc=(0,) * 6, eps=EPS)
    f = {"rho_dev": np.zeros((nz, ny, nx), np.float32), "u": st["u"].astype(np.float32),
         "P": st["P"].astype(np.float32), "phi": st["phi"].astype(np.float32)}
    return p, f


def _jet(nx=40, ny=36, nz=50):
    return inputs.jet_params(nx, ny, nz, d=10.0, u=0.05, re=1000.0, we=50.0, seed=7) | {"eps": EPS}


@pytest.mark.parametrize("case", ["droplet", "jet"])
def test_caller_buffer_every_node_written(case):
    """The state lives in a caller's device allocation; the buffer a step writes
    is filled with NaN words (0xFF bytes; the phase plane then holds -1
    fixed-point units, and 0x7F7F7F7F in the jet case, far outside the clamp
    range) before the step.  The step must overwrite every node, boundary layers
    included: the device words equal those of a run on library-owned memory,
    bit for bit."""
    from hip_runtime import DeviceBuffer
    from paper_2403_15773_amd.tslb import Simulation, required_bytes, make_params
    _say("caller-owned buffer, poisoned output, %s" % case)
    if case == "droplet":
        p, f = _droplet(40, 36, 44)
        steps = 3
    else:
        p, f = _jet(), None
        steps = 5
    with Simulation(**p) as own:
        if f is None:
            own.set_state_rest()
        else:
            own.set_state(**f)
        own.step(steps - 1)
        start = own.get_state_raw()
        own.step(1)
        want = own.get_state_raw()
    # N is a multiple of 64 here, so the planes have no padding words (the
    # comparison below covers every word of the buffer)
    assert (p["nx"] * p["ny"] * p["nz"]) % 64 == 0
    need = required_bytes(make_params(**p))
    with DeviceBuffer(need) as buf:
        sim = Simulation(**p, device_buffer=buf.ptr, device_buffer_bytes=need)
        sb = sim.state_bytes
        assert 2 * sb == need
        sim.set_state_raw(start, step=steps - 1)  # into the first half (the current buffer)
        assert np.array_equal(buf.download(sb), start)
        buf.fill(0xFF if case == "droplet" else 0x7F, nbytes=sb, offset=sb)
        sim.step(1)
        sim.sync()
        got = buf.download(sb, offset=sb)  # the device words directly: no boundary refill on the way
        sim.close()
    assert np.array_equal(got, want)


def test_caller_stream_matches_own_stream():
    from hip_runtime import Stream
    from paper_2403_15773_amd.tslb import Simulation
    _say("caller stream vs own stream")
    p, f = _droplet(33, 31, 29, seed=5)
    with Simulation(**p) as own:
        own.set_state(**f)
        own.step(7)
        want = own.get_state_raw()
    with Stream() as stream:
        with Simulation(**p, stream=stream.handle) as sim:
            sim.set_state(**f)
            sim.step(7)
            stream.synchronize()
            got = sim.get_state_raw()
    assert np.array_equal(got, want)


_TORCH_CHILD = r"""
import sys, numpy as np
import torch                      # torch's bundled ROCm runtime starts first in this process
assert torch.cuda.is_available()
sys.path.insert(0, sys.argv[1])
from paper_2403_15773_amd import inputs
from paper_2403_15773_amd.tslb import Simulation, make_params, required_bytes
p = inputs.jet_params(40, 36, 50, d=10.0, u=0.05, re=1000.0, we=50.0, seed=7) | {"eps": 1e-4}
with Simulation(**p) as own:
    own.set_state_rest()
    own.step(6)
    want = own.get_state_raw()
need = required_bytes(make_params(**p))
buf = torch.empty(need, dtype=torch.uint8, device="cuda")
torch.cuda.synchronize()
with Simulation(**p, device_buffer=buf.data_ptr(), device_buffer_bytes=need) as sim:
    sim.set_state_rest()
    sim.step(6)
    got = sim.get_state_raw()
    sim.sync()
    dev = buf[need // 2:].cpu().numpy() if sim.step_index % 2 else buf[:need // 2].cpu().numpy()
assert np.array_equal(got, want), "torch-buffer run differs"
assert np.array_equal(dev, want), "device words differ"
print("torch buffer OK", need)
"""


def test_torch_allocation_as_the_state_buffer():
    """A torch tensor's device memory as device_buffer, in a child process where
    torch's runtime starts before the library's: bitwise the library-owned run,
    and the current state read back through torch equals it too."""
    import os
    import subprocess
    import sys
    _say("torch allocation as device_buffer (child process)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _TORCH_CHILD, root], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "torch buffer OK" in r.stdout


@pytest.mark.parametrize("storage", ["fp32", "fp16q"])
def test_rest_state_is_the_all_zero_state(storage):
    from paper_2403_15773_amd.tslb import Simulation
    _say("rest state, %s" % storage)
    p = _jet(32, 28, 40)
    with Simulation(**p, storage=storage) as a, Simulation(**p, storage=storage) as b:
        a.set_state_rest(step=4)
        b.set_state_raw(np.zeros(b.state_bytes, np.uint8), step=4)
        assert a.step_index == 4
        d, e = a.diagnostics(), b.diagnostics()  # boundary layers filled first: the inlet disc brings phase
        assert d["mass"] == 32 * 28 * 40 and d["finite"] and d["phase"] == e["phase"] > 0
        a.step(12)
        b.step(12)
        assert np.array_equal(a.get_state_raw(), b.get_state_raw())


def test_per_launch_kernel_times():
    from paper_2403_15773_amd.tslb import Simulation
    _say("per-launch kernel times")
    with Simulation(**_jet()) as s:
        s.set_state_rest()
        s.set_timing(True)
        s.step(6)
        t = s.step_kernel_times()
        assert t.shape == (6,) and np.all(t > 0)
        assert np.isclose(t.mean(), s.last_step_kernel_ms(), rtol=1e-5)
        s.set_timing(False)
        s.step(2)
        assert s.step_kernel_times().shape == (0,)


def test_mass_drift_bound():
    """Closed box: the mass stays within a tight bound.  A box with an outflow
    face and a denser interior loses mass through that face (the rule imposes
    rho = 1 there): the bound trips at the first check past it."""
    from paper_2403_15773_amd.tslb import E_UNSTABLE, Simulation, TslbError
    _say("mass-drift bound")
    p, f = _droplet(24, 24, 24)
    with Simulation(**p, check_interval=5, max_mass_drift=1e-6) as s:
        s.set_state(**f)
        s.step(40)
        assert s.step_index == 40
    n = 20
    q = dict(nx=n, ny=n, nz=n, nu=0.05, sigma=0.0, width=3.0, eps=EPS, bc=(1, 1, 1, 1, 4, 3))
    st = inputs.quiescent(n, n, n)
    fields = {"rho_dev": np.full((n, n, n), 0.01, np.float32), "u": st["u"].astype(np.float32),
              "P": st["P"].astype(np.float32), "phi": st["phi"].astype(np.float32)}
    with Simulation(**q, check_interval=4) as free:  # no bound: runs
        free.set_state(**fields)
        m0 = free.diagnostics()["mass"]
        free.step(40)
        drift = abs(free.diagnostics()["mass"] - m0) / m0
    assert drift > 1e-4
    with Simulation(**q, check_interval=4, max_mass_drift=1e-4) as s:
        s.set_state(**fields)
        with pytest.raises(TslbError) as ei:
            s.step(40)
        assert ei.value.code == E_UNSTABLE and "mass drifted" in str(ei.value)
        assert s.step_index % 4 == 0 and 0 < s.step_index <= 40
