"""Plain numpy definitions of the state-vector primitives (test infrastructure).

Conventions: an n-qubit state is a complex128 vector of length 2^n; qubit q is
bit q of the basis index (little-endian).  A k-qubit matrix acts on the local
index whose bit j is qubit ``qubits[j]``.

* :func:`apply_gate` -- the definition psi'[.., i, ..] = sum_j M[i, j] psi[.., j, ..]
  written as a tensor contraction.
* :func:`kron_gate` -- the full 2^n x 2^n matrix built from Kronecker products
  and a basis permutation (brute force for n <= 8, used to pin the above).
* :func:`measure_reset` -- Z measurement of one qubit with outcome decided by a
  supplied uniform, renormalisation by the kept half's own norm and reset of
  the measured qubit to |0> (the reused-ancilla step of Sec. II.B).
"""
import numpy as np

TAU = 1e-10


def apply_gate(state, qubits, m):
    """Apply a dense 2^k x 2^k matrix to the listed qubits (tensor contraction)."""
    state = np.asarray(state, dtype=np.complex128)
    n = int(np.log2(state.size))
    k = len(qubits)
    m = np.asarray(m, dtype=np.complex128).reshape([2] * (2 * k))
    # numpy axis a of the (2,)*n tensor is qubit n-1-a.
    psi = state.reshape([2] * n)
    axes = [n - 1 - q for q in qubits]
    # matrix row/col index bits: bit j = qubits[j] -> reshaped axis (k-1-j)
    m_axes_in = [2 * k - 1 - j for j in range(k)]
    out = np.tensordot(m, psi, axes=(m_axes_in, axes))
    # out axes: matrix output axes (bit k-1 .. bit 0) then remaining psi axes
    rest = [a for a in range(n) if a not in axes]
    order = [None] * n
    for j in range(k):
        order[axes[j]] = k - 1 - j
    for i, a in enumerate(rest):
        order[a] = k + i
    return np.transpose(out, order).reshape(-1).copy()


def apply_diag(state, qubits, phases):
    """Multiply each amplitude by phases[local index of the listed qubits]."""
    state = np.asarray(state, dtype=np.complex128)
    idx = np.arange(state.size, dtype=np.int64)
    loc = np.zeros(state.size, dtype=np.int64)
    for j, q in enumerate(qubits):
        loc |= ((idx >> q) & 1) << j
    return state * np.asarray(phases, dtype=np.complex128)[loc]


def kron_gate(n, qubits, m):
    """Full 2^n x 2^n matrix of a k-qubit gate, by brute force over basis states."""
    m = np.asarray(m, dtype=np.complex128)
    k = len(qubits)
    N = 1 << n
    full = np.zeros((N, N), dtype=np.complex128)
    for col in range(N):
        jloc = 0
        for j, q in enumerate(qubits):
            jloc |= ((col >> q) & 1) << j
        base = col
        for q in qubits:
            base &= ~(1 << q)
        for iloc in range(1 << k):
            row = base
            for j, q in enumerate(qubits):
                if (iloc >> j) & 1:
                    row |= 1 << q
            full[row, col] += m[iloc, jloc]
    return full


def pauli(P):
    """2x2 Pauli matrix for 'I', 'X', 'Y', 'Z' (Y = [[0,-i],[i,0]])."""
    return {
        "I": np.eye(2, dtype=np.complex128),
        "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
        "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
        "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
    }[P]


def half_norms(state, q):
    """(S0, S1): squared norms of the halves with bit q equal to 0 and 1."""
    idx = np.arange(state.size, dtype=np.int64)
    w = np.abs(state) ** 2
    one = ((idx >> q) & 1).astype(bool)
    return float(np.sum(w[~one])), float(np.sum(w[one]))


def measure_reset(state, q, u=None, forced=None, tau=TAU):
    """Measure qubit q in Z, keep the outcome's half renormalised, reset q to 0.

    Outcome m = [u < p1] with p1 = S1 / (S0 + S1) clamped to 0 below tau and
    to 1 above 1 - tau; or m = forced.  Returns (m, p1, new_state)."""
    S0, S1 = half_norms(state, q)
    p1 = S1 / (S0 + S1)
    if p1 < tau:
        p1 = 0.0
    elif p1 > 1.0 - tau:
        p1 = 1.0
    m = int(forced) if forced is not None else int(u < p1)
    Sm = S1 if m else S0
    idx = np.arange(state.size, dtype=np.int64)
    lo = idx[((idx >> q) & 1) == 0]
    out = np.zeros_like(state)
    out[lo] = state[lo | (m << q)] / np.sqrt(Sm)
    return m, p1, out
