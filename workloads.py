"""Seeded synthetic workloads shared by the tests, the smoke check and the
benchmark.

This module holds no arithmetic of the simulation method: it only names the
workload shapes (code distance, rounds, noise parameters, trajectory counts)
of the paper's experiment (Sec. III.B: d=5, five noisy rounds, 10^4
trajectories per (p, c) point) and of the benchmark configurations, and draws
seeded random inputs (per-site over-rotation angles, random states and
matrices) with numpy.  The per-trajectory random draws of the method itself
(noise locations, measurement outcomes) are made inside the simulators from a
counter-based generator and are not produced here.
"""
import numpy as np

CR = "cr"              # cross-resonance gate set (Sec. III.A)
TEXTBOOK = "textbook"  # H / CNOT / CZ circuits (Fig. 1 of the paper)

# Named workloads.  theta = over-rotation angle range in radians; the exponent
# of the over-rotation exp(-i eps A) is eps = theta / 2 (theta = 2 c sqrt(p)).
CONFIGS = {
    # d=3, 10 qubits, textbook circuit, exp(-i 0.02 X) after each H.
    "d3_textbook_c128": dict(d=3, gateset=TEXTBOOK, rounds=3, p=1e-3, eps=0.02,
                             theta=None, zeta=0.0, n_traj=1000, seed=0, dtype="c128"),
    # d=5, 26 qubits, cross-resonance circuit, theta ~ U[0, 0.05) per gate site,
    # ZZ crosstalk zeta = 0.01 on nearest-neighbour data pairs.
    "d5_cr_c128": dict(d=5, gateset=CR, rounds=5, p=1e-3, eps=None,
                       theta=(0.0, 0.05), zeta=0.01, n_traj=100, seed=1, dtype="c128"),
    # precision comparison: fixed theta for every site.
    "d5_cr_theta0.01": dict(d=5, gateset=CR, rounds=5, p=1e-3, eps=0.005, theta=None,
                            zeta=0.01, n_traj=20, seed=1, dtype="c64"),
    "d5_cr_theta0.03": dict(d=5, gateset=CR, rounds=5, p=1e-3, eps=0.015, theta=None,
                            zeta=0.01, n_traj=20, seed=1, dtype="c64"),
    "d5_cr_theta0.05": dict(d=5, gateset=CR, rounds=5, p=1e-3, eps=0.025, theta=None,
                            zeta=0.01, n_traj=20, seed=1, dtype="c64"),
}


def eps_sites(n_sites, theta, seed):
    """Per-gate-site over-rotation exponents eps = theta/2 with theta drawn
    once per site and job, uniform on [theta[0], theta[1])."""
    rng = np.random.default_rng([0x5EED, int(seed)])
    return rng.uniform(theta[0], theta[1], size=n_sites) / 2.0


def batch_params(n_traj, n_sites, seed, rounds=(1, 9), p=(5e-4, 5e-3), theta=(0.0, 0.05)):
    """Per-trajectory parameters of a batched small-distance launch: rounds
    uniform on {rounds[0]..rounds[1]}, p uniform on [p0, p1), and per-site
    exponents eps = theta/2 with theta uniform on [theta0, theta1)."""
    rng = np.random.default_rng([0xBA7C, int(seed)])
    r = rng.integers(rounds[0], rounds[1] + 1, size=n_traj).astype(np.int32)
    pp = rng.uniform(p[0], p[1], size=n_traj)
    eps = rng.uniform(theta[0], theta[1], size=(n_traj, n_sites)) / 2.0
    return r, pp, eps


def random_state(n, seed, dtype=np.complex128):
    """Normalised random state of n qubits (Gaussian amplitudes)."""
    rng = np.random.default_rng([0x57A7E, int(n), int(seed)])
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    v /= np.linalg.norm(v)
    return v.astype(dtype)


def random_matrix(k, seed, unitary=True):
    """Random 2^k x 2^k complex matrix (Haar-like unitary via QR if asked)."""
    rng = np.random.default_rng([0x3A7, int(k), int(seed)])
    a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
    if not unitary:
        return a
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def serving_stream(window_s, seed=2, rate=200.0, companion=False, n_sites=None):
    """Poisson job stream of the serving workload: arrivals at `rate` jobs/s
    over `window_s` seconds; distance 3/4/5 with probabilities 0.6/0.3/0.1,
    rounds uniform on 1..10, trajectories log-uniform on [10, 10^4], p uniform
    on [5e-4, 5e-3), per-site theta uniform on [0, 0.05) (eps = theta/2),
    complex64 or complex128 with probability 1/2 each.

    companion=True scales the offered load down to fit one GPU: d=4 jobs get a
    tenth of the trajectories and d=5 jobs one trajectory.  `n_sites(d)` gives
    the gate-site count per round.  Returns a list of (arrival_s, job dict)."""
    rng = np.random.default_rng([0x5E4E, int(seed), int(companion)])
    t, out, tag = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= window_s:
            break
        d = int(rng.choice([3, 4, 5], p=[0.6, 0.3, 0.1]))
        rounds = int(rng.integers(1, 11))
        n_traj = int(round(np.exp(rng.uniform(np.log(10.0), np.log(1e4)))))
        if companion:
            n_traj = 1 if d == 5 else (max(1, n_traj // 10) if d == 4 else n_traj)
        p = float(rng.uniform(5e-4, 5e-3))
        eps = rng.uniform(0.0, 0.05, size=n_sites(d)) / 2.0
        dtype = "c64" if rng.random() < 0.5 else "c128"
        out.append((t, dict(tag=tag, d=d, gateset="cr", rounds=rounds, n_traj=n_traj,
                            seed=int(rng.integers(0, 2 ** 62)), p=p, eps_site=eps, zeta=0.0,
                            dtype=dtype, traj0=0)))
        tag += 1
    return out
