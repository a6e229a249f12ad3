"""The projection probe: both evaluations of the moment-to-population map (the
vector-ALU tensor product the step uses, and FP32 matrix-core tiles) against the
map written out on the host from its definition."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


def _projection_matrix():
    """A[m, k]: tau at velocity m = 9 (cz+1) + (cx+1) + 3 (cy+1) per unit coefficient k of
    tau(c) = K1.c + K2_aa h(c_a) + K2_ab c_a c_b + K3_aab h(c_a) c_b + K3_xyz cx cy cz."""
    h = lambda c: c * c - 1.0 / 3.0  # noqa: E731
    A = np.zeros((27, 16))
    for cz in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cx in (-1, 0, 1):
                m = 9 * (cz + 1) + (cx + 1) + 3 * (cy + 1)
                A[m] = [cx, cy, cz, h(cx), h(cy), h(cz), cx * cy, cx * cz, cy * cz,
                        h(cx) * cy, h(cx) * cz, h(cy) * cx, h(cy) * cz, h(cz) * cx, h(cz) * cy, cx * cy * cz]
    return A


@pytest.mark.parametrize("kind", [0, 1])
def test_projection_probe_matches_the_map(kind):
    from paper_2403_15773_amd.tslb import projection_probe
    nodes, reps, step = 64 * 70, 4, 1.0e-3  # 70 waves: a partial last block of 256 threads
    rng = np.random.default_rng(11)
    coef = rng.uniform(-0.05, 0.05, (16, nodes)).astype(np.float32)
    _say("projection probe kind %d, %d nodes, %d reps" % (kind, nodes, reps))
    ms, out = projection_probe(kind, coef, reps, iters=2)
    A = _projection_matrix()
    expect = reps * (A @ coef.astype(np.float64)) + step * reps * (reps - 1) / 2 * A.sum(axis=1)[:, None]
    err = np.abs(out - expect).max() / np.abs(expect).max()
    _say("kind %d: relative error %.2e, %.4f ms" % (kind, err, ms))
    assert err < 1e-5
