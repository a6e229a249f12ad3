"""Second, independent FP64 route: the thread-safe step itself, in numpy.

TEST INFRASTRUCTURE ONLY.  Where ``tslb_oracle.c`` keeps 27 + 7 populations in
two arrays and pushes them, this route keeps only the moments (rho, j, Pi, phi)
and, each step, rebuilds every post-collision population at the neighbour
x - c_i and sums it into x (Methodology, Eqs. 6 and 8 and the thread-safe
sketch).  The collision is written in its closed scalar form (the Hermite
contractions of Eqs. 16 and 19 worked out by hand for c_s^2 = 1/3) rather than
with tensor loops, so the two routes share neither storage, streaming nor the
way the collision is written.  Periodic boxes only.

Fields are numpy arrays of shape (nz, ny, nx); vectors (3, ...), symmetric
tensors (6, ...) in the order xx, yy, zz, xy, xz, yz.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0


def _velocities():
    c = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)])
    s = (c * c).sum(1)
    w = np.choose(s, [8 / 27, 2 / 27, 1 / 54, 1 / 216])
    return c, w


C27, W27 = _velocities()
C7 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
W7 = np.array([0.25] + [0.125] * 6)
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def _shift(a, c):
    """value at x of a(x + c) (periodic)."""
    return np.roll(a, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2))


def _pull(a, c):
    """value at x of a(x - c) (periodic)."""
    return np.roll(a, shift=(c[2], c[1], c[0]), axis=(0, 1, 2))


def geometry(phi, sigma, eps=1e-12):
    """G = 3 sum w c phi(x+c), n = G/(|G|+eps), kappa = 3 sum w c.n(x+c), F = -sigma kappa G."""
    G = np.zeros((3,) + phi.shape)
    for c, w in zip(C27, W27):
        if not c.any():
            continue
        ps = _shift(phi, c)
        for a in range(3):
            if c[a]:
                G[a] += 3.0 * w * c[a] * ps
    mag = np.sqrt((G * G).sum(0))
    n = G / (mag + eps)
    kappa = np.zeros_like(phi)
    for c, w in zip(C27, W27):
        if not c.any():
            continue
        kappa += 3.0 * w * sum(c[a] * _shift(n[a], c) for a in range(3) if c[a])
    F = -sigma * kappa * G
    return G, n, kappa, F


def post_collision(rho, u, P, F, omega, c, w):
    """f_i^post at every node for one velocity c (closed form, c_s^2 = 1/3)."""
    cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
    cF = c[0] * F[0] + c[1] * F[1] + c[2] * F[2]
    uu = (u * u).sum(0)
    uF = (u * F).sum(0)
    cPc = sum((1 if a == b else 2) * c[a] * c[b] * P[s] for s, (a, b) in enumerate(PAIRS))
    trP = P[0] + P[1] + P[2]
    Pu = [P[0] * u[0] + P[3] * u[1] + P[4] * u[2],
          P[3] * u[0] + P[1] * u[1] + P[5] * u[2],
          P[4] * u[0] + P[5] * u[1] + P[2] * u[2]]
    cPu = c[0] * Pu[0] + c[1] * Pu[1] + c[2] * Pu[2]
    eq = rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu + 4.5 * cu * (cu * cu - uu))
    neq = 4.5 * cPc - 1.5 * trP + 13.5 * cu * cPc - 4.5 * cu * trP - 9.0 * cPu
    force = 1.5 * cF + 4.5 * cu * cF - 1.5 * uF
    return w * (eq + (1.0 - omega) * neq + force)


def from_physical(rho, u, P, phi, sigma, eps=1e-12):
    """Moments (rho, j, Pi, phi) of the initial state (same convention as the C oracle)."""
    _, _, _, F = geometry(phi, sigma, eps)
    j = rho * u - 0.5 * F
    Pi = np.empty_like(P)
    for s, (a, b) in enumerate(PAIRS):
        Pi[s] = P[s] + (rho * CS2 if a == b else 0.0) + rho * u[a] * u[b] - 0.5 * (u[a] * F[b] + F[a] * u[b])
    return {"rho": rho.copy(), "j": j, "Pi": Pi, "phi": phi.copy()}


def to_physical(m, sigma, eps=1e-12):
    rho, j, Pi, phi = m["rho"], m["j"], m["Pi"], m["phi"]
    _, _, _, F = geometry(phi, sigma, eps)
    u = (j + 0.5 * F) / rho
    P = np.empty_like(Pi)
    for s, (a, b) in enumerate(PAIRS):
        P[s] = Pi[s] - (rho * CS2 if a == b else 0.0) - rho * u[a] * u[b] + 0.5 * (u[a] * F[b] + F[a] * u[b])
    return {"rho": rho, "u": u, "P": P, "phi": phi}


def step(m, nu, sigma, width=3.0, gamma=0.0, eps=1e-12):
    """One thread-safe step: read moments at x - c_i, rebuild f_i^post there, sum at x."""
    omega = 1.0 / (3.0 * nu + 0.5)
    gamma = gamma if gamma > 0 else 2.0 / width
    phys = to_physical(m, sigma, eps)
    rho, u, P, phi = phys["rho"], phys["u"], phys["P"], phys["phi"]
    _, n, _, F = geometry(phi, sigma, eps)
    new_rho = np.zeros_like(rho)
    new_j = np.zeros_like(m["j"])
    new_Pi = np.zeros_like(m["Pi"])
    for c, w in zip(C27, W27):
        f = _pull(post_collision(rho, u, P, F, omega, c, w), c)
        new_rho += f
        for a in range(3):
            if c[a]:
                new_j[a] += c[a] * f
        for s, (a, b) in enumerate(PAIRS):
            if c[a] * c[b]:
                new_Pi[s] += c[a] * c[b] * f
    new_phi = np.zeros_like(phi)
    for c, w in zip(C7, W7):
        cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
        cn = c[0] * n[0] + c[1] * n[1] + c[2] * n[2]
        g = w * phi * (1.0 + 4.0 * cu) + w * gamma * phi * (1.0 - phi) * cn
        new_phi += _pull(g, c)
    return {"rho": new_rho, "j": new_j, "Pi": new_Pi, "phi": new_phi}


def run(state, nu, sigma, steps, width=3.0, gamma=0.0, eps=1e-12):
    """Physical state after ``steps`` thread-safe steps (periodic box)."""
    m = from_physical(state["rho"], state["u"], state["P"], state["phi"], sigma, eps)
    for _ in range(steps):
        m = step(m, nu, sigma, width, gamma, eps)
    return to_physical(m, sigma, eps)
