"""Reduced-precision storage (moments stored as FP16 or BF16 scaled deviations
rho'/U^2, u/U, Q/U^2 with U = 0.05; arithmetic and the phase field unchanged).

Bars:
* Laplace's law (static droplet, R = 6, 8, 10, 3000 steps): the pressure jump
  with 16-bit storage within 2 % of the binary32 one, and binary32 within 5 %
  of 2 sigma / R (the physics pin of the whole GPU path);
* the 1e-3 per-field target against the FP64 oracle on the 32^3 droplet is NOT
  met by all-16-bit storage (measured worst field: FP16 1.3e-2, BF16 1.1e-1,
  both in the stress P); the test bounds the measured error so that a
  regression shows, and the target is kept as an expected failure;
* FP16Q (rho' and ubar binary32, the stress binary16) meets the 1e-3 target;
* conservation: the phase sum stays exact (fixed point), the mass drifts by the
  storage rounding only.
"""
import numpy as np
import pytest

from paper_2403_15773_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 1e-4
CS2 = 1.0 / 3.0
# measured worst per-field relative L-inf error after 200 steps of the 32^3
# droplet (FP16 1.27e-2, BF16 1.11e-1), with head room for regressions only
BOUND = {"fp16": 2.5e-2, "bf16": 2.0e-1}
# the 2000-step jets against binary32: relative L2 of u_z and phi, and the relative change of the
# penetration length and of the axis-mean u_z (the chaotic divergence included)
# (measured at We 10/100/2000: L2 of u_z and phi up to 2.3e-3 and 1.2e-2 for FP16, 3.2e-5 and 2.0e-4 for
# FP16Q, 0.28 and 0.44 for BF16; penetration and axis-mean u_z unchanged with FP16 and FP16Q, 4-11 % lower
# with BF16)
L2_BOUND = {"fp16": 0.05, "fp16q": 1e-3, "bf16": 0.8}
INTEGRAL_BOUND = {"fp16": 0.02, "fp16q": 0.01, "bf16": 0.2}


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def _droplet_errors(storage):
    from test_gpu_parity import _f32, field_errors, run_both
    p = inputs.droplet_params(32)
    g, r = run_both(p, inputs.droplet(32, 8.0, 3.0, noise_amp=1e-3, seed=1), 200, storage=storage)
    e = {k: v[0] for k, v in field_errors(g, r).items()}
    _say("droplet32 %s vs oracle: " % storage + " ".join("%s=%.1e" % kv for kv in e.items()))
    return e


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_reduced_storage_error_is_bounded(storage):
    e = _droplet_errors(storage)
    assert max(e.values()) <= BOUND[storage]
    assert e["rho-1"] <= BOUND[storage] / 10 and e["phi"] <= BOUND[storage] / 10


@pytest.mark.xfail(strict=True, reason="16-bit moment storage misses the 1e-3 per-field target (FP16 1.3e-2 in P)")
def test_fp16_meets_1e3_target():
    assert max(_droplet_errors("fp16").values()) <= 1e-3


def test_fp16_stress_storage_meets_1e3_target():
    """rho' and ubar in binary32, the stress in binary16 (32 B per node and
    buffer): every field within 1e-3 of the oracle after 200 steps."""
    e = _droplet_errors("fp16q")
    assert max(e.values()) <= 1e-3


def _laplace_dp(radius, storage, steps=3000):
    from paper_2403_15773_amd.tslb import Simulation
    from test_gpu_parity import _f32
    n, W, sigma = 32, 3.0, 0.01
    st = _f32(inputs.droplet(n, radius, W, noise_amp=0.0, rho_inside=2 * sigma / (radius * CS2)))
    with Simulation(nx=n, ny=n, nz=n, nu=0.1, sigma=sigma, width=W, eps=EPS, storage=storage) as s:
        s.set_state(**st)
        s.step(steps)
        rho = 1.0 + s.moments()[0].astype(np.float64)
        d = s.diagnostics()
    x, y, z = inputs.grid_coords(n, n, n)
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2)
    dp = CS2 * (rho[r <= radius - W].mean() - rho[r >= radius + W + 2].mean())
    return dp * radius / (2 * sigma), d


@pytest.mark.parametrize("radius", [6.0, 8.0, 10.0])
def test_laplace_law_binary32_and_16_bit(radius):
    ref, d32 = _laplace_dp(radius, "fp32")
    _say("Laplace R=%g fp32: dp R/(2 sigma) = %.4f" % (radius, ref))
    assert ref == pytest.approx(1.0, abs=0.05)
    for storage in ("fp16", "bf16", "fp16q"):
        v, d = _laplace_dp(radius, storage)
        _say("Laplace R=%g %s: %.4f (%.2e vs fp32)" % (radius, storage, v, v / ref - 1))
        assert v == pytest.approx(ref, rel=0.02)
        assert d["finite"]
        # the phase field is stored in fixed point whatever the moment storage
        assert d["phase"] == d32["phase"]


def _jet_fields(p, storage, steps):
    from paper_2403_15773_amd.tslb import Simulation
    with Simulation(**p, eps=EPS, storage=storage, u_scale=0.05) as s:
        s.set_state_raw(np.zeros(s.state_bytes, np.uint8), step=0)  # quiescent: the all-zero raw state
        s.step(steps)
        g = s.physical()
        d = s.diagnostics()
    return g, d


def _jet_integrals(g, d_nozzle):
    """(penetration: the furthest z whose axis-averaged phi exceeds 1/2, in nozzle
    diameters; axis-mean u_z over the column of the four central nodes)."""
    nz, ny, nx = g["phi"].shape
    cy, cx = (ny - 1) // 2, (nx - 1) // 2
    phi_axis = g["phi"][:, cy:cy + 2, cx:cx + 2].astype(np.float64).mean(axis=(1, 2))
    uz_axis = g["u"][2][:, cy:cy + 2, cx:cx + 2].astype(np.float64).mean(axis=(1, 2))
    inside = np.nonzero(phi_axis > 0.5)[0]
    return (inside.max() + 1 if inside.size else 0) / d_nozzle, uz_axis.mean()


def _l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300))


# the 128 x 128 x 512 jet (We = 100) after 200 steps from rest, worst field against binary32 (the
# flow is still laminar: the difference is the storage rounding, not chaos).  FP16Q: the 1e-3 target
# (measured 9.3e-4); FP16 measured 1.4e-2, BF16 1.1e-1
SHORT_BOUND = {"fp16q": 1e-3, "fp16": 2.5e-2, "bf16": 2.0e-1}


@pytest.mark.parametrize("storage", ["fp16q", "fp16", "bf16"])
def test_jet_16_bit_storage_before_divergence(storage):
    """The 128 x 128 x 512 jet (We = 100) after 200 steps from rest, before the
    instability amplifies rounding differences: per-field relative L-infinity
    error against binary32 within the storage's bound (FP16Q: the 1e-3 target)."""
    from test_gpu_parity import field_errors
    p = inputs.jet_params(128, 128, 512, d=20.0, u=0.05, re=5000.0, we=100.0, seed=2)
    _say("jet 128x128x512 We=100, 200 steps: binary32 vs %s" % storage)
    g32, _ = _jet_fields(p, "fp32", 200)
    ref = {k: v.astype(np.float64) for k, v in g32.items() if k != "rho_dev"}
    ref["rho"] = 1.0 + g32["rho_dev"].astype(np.float64)
    g, d = _jet_fields(p, storage, 200)
    e = {k: v[0] for k, v in field_errors(g, ref).items()}
    _say("  %s: worst %.2e (%s)" % (storage, max(e.values()), " ".join("%s=%.1e" % kv for kv in e.items())))
    assert d["finite"] and max(e.values()) <= SHORT_BOUND[storage]


@pytest.mark.parametrize("we", [10.0, 100.0, 2000.0])
def test_jet_16_bit_storage_against_binary32(we):
    """The 128 x 128 x 512 jet geometry (D = 20, Re = 5000) at We = 10, 100, 2000, 2000 steps from
    rest: each 16-bit storage against binary32.  The jet is unstable at Re = 5000, so rounding
    differences grow along the run and the per-field error includes that divergence: the bounds
    keep the measured values (FP16 up to 0.18, FP16Q smaller, BF16 decorrelated at ~2) from
    regressing, and mass and phase must drift only by the storage rounding."""
    from test_gpu_parity import field_errors
    p = inputs.jet_params(128, 128, 512, d=20.0, u=0.05, re=5000.0, we=we, seed=2)
    _say("jet 128x128x512 We=%g: binary32, 2000 steps" % we)
    g32, d32 = _jet_fields(p, "fp32", 2000)
    ref = {k: v.astype(np.float64) for k, v in g32.items() if k != "rho_dev"}
    ref["rho"] = 1.0 + g32["rho_dev"].astype(np.float64)
    assert d32["finite"] and g32["u"][2].max() > 0.04
    pen32, uz32 = _jet_integrals(g32, 20.0)
    bounds = {"fp16": 0.5, "fp16q": 0.5, "bf16": 5.0}
    for storage in ("fp16", "fp16q", "bf16"):
        g, d = _jet_fields(p, storage, 2000)
        e = {k: v[0] for k, v in field_errors(g, ref).items()}
        dm = abs(d["mass"] - d32["mass"]) / d32["mass"]
        dp = abs(d["phase"] - d32["phase"]) / d32["phase"]
        pen, uz = _jet_integrals(g, 20.0)
        l2u, l2phi = _l2(g["u"][2], ref["u"][2]), _l2(g["phi"], ref["phi"])
        _say("We=%g %s vs binary32: worst %.2e (%s) mass %.1e phase %.1e; L2 u_z %.2e phi %.2e; "
             "penetration %.2f D (binary32 %.2f D), axis u_z %.4f (binary32 %.4f)" % (
                 we, storage, max(e.values()), max(e, key=e.get), dm, dp, l2u, l2phi, pen, pen32, uz, uz32))
        assert d["finite"]
        assert max(e.values()) <= bounds[storage]
        assert dm <= 1e-4 and dp <= 1e-3
        # L2 and integral quantities of the chaotic jet
        assert l2u <= L2_BOUND[storage] and l2phi <= L2_BOUND[storage]
        assert abs(pen - pen32) <= INTEGRAL_BOUND[storage] * pen32
        assert abs(uz - uz32) <= INTEGRAL_BOUND[storage] * abs(uz32)


def _bf16_rne_bits(x):
    """binary32 -> bfloat16 bits by round to nearest, ties to even, on the upper
    16 bits of the binary32 word (finite inputs)."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)


def test_bf16_store_rounds_to_nearest_even():
    """The BF16 store (the hardware conversion of gfx950) against the definition
    of round to nearest even: exact ties with even and odd kept bits, one unit
    on either side of a tie, exact values and random words, both signs, from
    1e-30 to 1e3.  rho' is stored scaled by 1/U^2, so U = 1 stores it as given
    in plane 0 of the raw state."""
    from paper_2403_15773_amd.tslb import Simulation
    n = 16
    rng = np.random.default_rng(11)
    N = n * n * n
    hi = rng.integers(0, 1 << 16, N, dtype=np.uint64)
    expo = rng.integers(27, 137, N, dtype=np.uint64)  # about 1e-30 .. 1e3
    lows = np.array([0x8000, 0x7FFF, 0x8001, 0x0000, 0xFFFF], np.uint64)
    low = np.where(np.arange(N) % 6 < 5, lows[np.arange(N) % 6 % 5],
                   rng.integers(0, 1 << 16, N, dtype=np.uint64)).astype(np.uint64)
    sign = ((np.arange(N) // 6) % 2).astype(np.uint64)
    words = (sign << 31) | (expo << 23) | ((hi & 0x7F) << 16) | low
    rho = words.astype(np.uint32).view(np.float32).reshape(n, n, n).copy()
    assert np.all(np.isfinite(rho)) and np.all(np.abs(rho) < 1e4)
    zero3 = np.zeros((3, n, n, n), np.float32)
    zero6 = np.zeros((6, n, n, n), np.float32)
    _say("bf16 store: %d words, %d exact ties" % (N, int(np.sum((low == 0x8000)))))
    with Simulation(nx=n, ny=n, nz=n, nu=0.05, components=1, storage="bf16", u_scale=1.0) as s:
        s.set_state(rho_dev=rho, u=zero3, P=zero6)
        raw = s.get_state_raw().view(np.uint16)
    got = raw[:N]
    want = _bf16_rne_bits(rho.reshape(-1))
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "first mismatches: " + ", ".join(
        "%08x -> %04x (want %04x)" % (int(words[i]), int(got[i]), int(want[i])) for i in bad[:5])
