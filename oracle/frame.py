"""Pauli-frame sampler for Pauli-only runs (test infrastructure).

With no coherent error (eps = zeta = 0) every gate of both syndrome circuits is
Clifford and every noise location is a stochastic Pauli channel, so the
circuit can be sampled efficiently (the Gottesman-Knill special case the paper
contrasts with its full simulation, Introduction).  A frame of X/Z bits per
qubit and per shot is pushed through the circuit; a Z measurement flips
relative to the noiseless reference exactly when the frame has an X component
on the measured qubit.

The reference run of a noiseless circuit on logical |0> gives deterministic
syndromes r0 (raw ancilla bits) and deterministic Z-stabilizer and logical-Z
parities of the final data bits, so the sampler returns flips of those
quantities.  It is independent of the state-vector oracle except for the code
layout.

Frame update rules (E -> U E U^dag, signs dropped):
  * exp(-i pi/4 P) for a Pauli string P: E -> E P if E anticommutes with P;
  * H: swap x and z; CNOT(c -> t): x_t ^= x_c, z_c ^= z_t;
    CZ(a, b): z_a ^= x_b, z_b ^= x_a.
"""
import numpy as np

from . import layout as _layout

_PAULI_XZ = {1: (1, 0), 2: (1, 1), 3: (0, 1)}  # X, Y, Z -> (x, z)


class FrameSampler:
    def __init__(self, d, gateset, shots, rng, idle=False):
        self.d = d
        self.idle = idle
        self.gateset = gateset
        self.stabs = _layout(d)
        self.nq = d * d + 1
        self.anc = d * d
        self.shots = shots
        self.rng = rng
        self.x = np.zeros((shots, self.nq), dtype=np.uint8)
        self.z = np.zeros((shots, self.nq), dtype=np.uint8)

    # --- Clifford gates -------------------------------------------------
    def rot_pauli(self, xs, zs):
        """exp(-i pi/4 P), P given by per-qubit (x, z) lists of (qubit, bit)."""
        # symplectic product <E, P> = sum_q x_E z_P + z_E x_P (mod 2)
        anti = np.zeros(self.shots, dtype=np.uint8)
        for q, (px, pz) in zip(xs, zs):
            if pz:
                anti ^= self.x[:, q]
            if px:
                anti ^= self.z[:, q]
        for q, (px, pz) in zip(xs, zs):
            if px:
                self.x[:, q] ^= anti
            if pz:
                self.z[:, q] ^= anti

    def rx(self, q):
        self.rot_pauli([q], [(1, 0)])

    def rz(self, q):
        self.rot_pauli([q], [(0, 1)])

    def rzx(self, qc, qt):
        self.rot_pauli([qc, qt], [(0, 1), (1, 0)])

    def h(self, q):
        self.x[:, q], self.z[:, q] = self.z[:, q].copy(), self.x[:, q].copy()

    def cnot(self, c, t):
        self.x[:, t] ^= self.x[:, c]
        self.z[:, c] ^= self.z[:, t]

    def cz(self, a, b):
        self.z[:, a] ^= self.x[:, b]
        self.z[:, b] ^= self.x[:, a]

    # --- noise ------------------------------------------------------------
    def noise1(self, q, p):
        u = self.rng.random(self.shots)
        j = np.where(u < p, 1 + np.minimum((u / (p / 3.0)).astype(np.int64), 2), 0)
        for P, (px, pz) in _PAULI_XZ.items():
            hit = (j == P).astype(np.uint8)
            if px:
                self.x[:, q] ^= hit
            if pz:
                self.z[:, q] ^= hit

    def noise2(self, q1, q2, p):
        u = self.rng.random(self.shots)
        j = np.where(u < p, 1 + np.minimum((u / (p / 15.0)).astype(np.int64), 14), 0)
        for qq, Pj in ((q1, j >> 2), (q2, j & 3)):
            for P, (px, pz) in _PAULI_XZ.items():
                hit = ((Pj == P) & (j > 0)).astype(np.uint8)
                if px:
                    self.x[:, qq] ^= hit
                if pz:
                    self.z[:, qq] ^= hit

    # --- circuit ------------------------------------------------------------
    def waiting(self, slots, busy, p):
        """Idle noise of one step: N1 on the check's data qubits other than
        `busy` (a label, or 0), in slot order."""
        if self.idle:
            for q in slots:
                if q and q != busy:
                    self.noise1(q - 1, p)

    def stabilizer(self, typ, slots, p):
        a = self.anc
        if self.gateset == 0:
            if typ == "X":
                self.rx(a)          # Rx^dag: same Clifford frame action as Rx
                self.noise1(a, p)
                self.waiting(slots, 0, p)
                for q in slots:
                    if q:
                        self.rzx(a, q - 1)
                        self.noise2(a, q - 1, p)
                    else:
                        self.noise1(a, p)
                    self.waiting(slots, q, p)
                self.rx(a)
                self.noise1(a, p)
                for q in slots:
                    if q:
                        self.rx(q - 1)
                        self.noise1(q - 1, p)
            else:
                for q in slots:
                    if q:
                        self.rzx(q - 1, a)
                        self.noise2(q - 1, a, p)
                    else:
                        self.noise1(a, p)
                    self.waiting(slots, q, p)
                for q in slots:
                    if q:
                        self.rz(q - 1)
                        self.noise1(q - 1, p)
                if self.idle:
                    self.noise1(a, p)
        else:
            self.h(a)
            self.noise1(a, p)
            self.waiting(slots, 0, p)
            for q in slots:
                if q:
                    if typ == "X":
                        self.cnot(a, q - 1)
                    else:
                        self.cz(a, q - 1)
                    self.noise2(a, q - 1, p)
                    self.waiting(slots, q, p)
            self.h(a)
            self.noise1(a, p)
            self.waiting(slots, 0, p)
        flip = self.x[:, a].copy()
        self.x[:, a] = 0
        self.z[:, a] = 0
        return flip

    def run(self, rounds, p, basis="Z"):
        """Returns (record flips [shots, rounds, n_stab], final data flips
        [shots, d*d]); basis "X": the data are measured in the X basis, which
        flips where the frame has a Z component."""
        ns = len(self.stabs)
        rec = np.zeros((self.shots, rounds, ns), dtype=np.uint8)
        for r in range(rounds):
            for i, (typ, slots) in enumerate(self.stabs):
                rec[:, r, i] = self.stabilizer(typ, slots, p)
        frame_bits = self.x if basis == "Z" else self.z
        final = frame_bits[:, : self.d * self.d].copy()
        return rec, final


def sample(d, gateset, rounds, p, shots, seed=0, basis="Z", idle=False):
    """Record flips and final-bit flips relative to the noiseless reference;
    idle: one-qubit noise on the waiting qubits of every step."""
    fs = FrameSampler(d, gateset, shots, np.random.default_rng(seed), idle)
    return fs.run(rounds, p, basis)
