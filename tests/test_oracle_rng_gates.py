"""Pins of the oracle's random-number generator and gate arithmetic."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import statevec as sv

# Known-answer vectors of Philox4x32-10 published with the Random123 library
# (Salmon, Moraes, Dror, Shaw, SC'11): (counter, key) -> output.
PHILOX_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX_KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(int(v) for v in oracle.philox4x32_10(ctr, key)) == want


def test_uniform_layout_of_counter_and_key():
    # u(seed, t, k) uses counter (k_lo, k_hi, t_lo, t_hi), key (s_lo, s_hi)
    seed, t, k = 0x0123456789ABCDEF, 0x1122334455667788, 0x99AABBCCDDEEFF00
    w = oracle.philox4x32_10(
        (k & 0xFFFFFFFF, k >> 32, t & 0xFFFFFFFF, t >> 32), (seed & 0xFFFFFFFF, seed >> 32))
    bits = ((int(w[1]) << 32) | int(w[0])) >> 11
    assert oracle.uniform(seed, t, k) == bits * 2.0 ** -53


def test_uniform_statistics():
    u = np.array([oracle.uniform(3, t, k) for t in range(20) for k in range(1000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = np.sum((hist - u.size / 20) ** 2 / (u.size / 20))
    assert chi2 < 45.3  # 19 dof, p = 1e-3


def _rot(P, beta):
    return np.cos(beta) * np.eye(P.shape[0]) - 1j * np.sin(beta) * P


def test_gate_set_identities():
    """Gate-set equations of Sec. III.A: exp(-i beta P) = cos b I - i sin b P
    (checked against scipy's matrix exponential), Rx(pi/2)^2 = -iX,
    Rzx(pi/2)^4 = -I, all unitary."""
    X, Z = sv.pauli("X"), sv.pauli("Z")
    ZX = np.kron(X, Z)  # matrix with bit0 = first qubit (Z), bit1 = second (X)
    for P in (X, Z, ZX):
        for beta in (np.pi / 4, np.pi / 4 + 0.013, -0.2):
            R = _rot(P, beta)
            assert np.allclose(R, scipy.linalg.expm(-1j * beta * P), atol=1e-15)
            assert np.allclose(R @ R.conj().T, np.eye(P.shape[0]), atol=1e-15)
    Rx = _rot(X, np.pi / 4)
    assert np.allclose(Rx @ Rx, -1j * X, atol=1e-15)
    Rzx = _rot(ZX, np.pi / 4)
    assert np.allclose(np.linalg.matrix_power(Rzx, 4), -np.eye(4), atol=1e-15)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_statevec_gate_vs_kronecker(n):
    rng = np.random.default_rng(n)
    for qs in ([0], [n - 1], [1, 0], [0, n - 1], [n - 1, 1], [2, 0, 1]):
        k = len(qs)
        m = rng.normal(size=(2 ** k, 2 ** k)) + 1j * rng.normal(size=(2 ** k, 2 ** k))
        s = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
        ref = sv.kron_gate(n, qs, m) @ s
        assert np.allclose(sv.apply_gate(s, qs, m), ref, atol=1e-12)
        if k <= 2:
            assert np.allclose(oracle.apply_gate_cpp(s, qs, m), ref, atol=1e-12)


def test_kronecker_brute_force_matches_textbook_kron():
    # kron_gate on qubits (0, 1) of 2 qubits with bit j = qubits[j] is the
    # matrix itself; on (1, 0) it is the swapped-basis matrix.
    rng = np.random.default_rng(1)
    A = rng.normal(size=(2, 2)) + 0j
    B = rng.normal(size=(2, 2)) + 0j
    # bit0 = qubit 0 -> np.kron(B, A) acts with A on bit 0 (little-endian)
    assert np.allclose(sv.kron_gate(2, [0], A), np.kron(np.eye(2), A))
    assert np.allclose(sv.kron_gate(2, [1], B), np.kron(B, np.eye(2)))
    assert np.allclose(sv.kron_gate(2, [0, 1], np.kron(B, A)), np.kron(B, A))


def test_measure_reset_definition():
    rng = np.random.default_rng(2)
    s = rng.normal(size=16) + 1j * rng.normal(size=16)
    s /= np.linalg.norm(s)
    S1 = np.sum(np.abs(s[8:]) ** 2)
    m, p1, out = sv.measure_reset(s, 3, u=0.0)
    assert m == 1 and np.isclose(p1, S1)
    assert np.allclose(out[:8], s[8:] / np.sqrt(S1)) and np.all(out[8:] == 0)
    m, p1, out = sv.measure_reset(s, 3, u=0.999999)
    assert m == 0 and np.allclose(out[:8], s[:8] / np.sqrt(1 - S1))
    assert np.isclose(np.linalg.norm(out), 1.0, atol=1e-14)
