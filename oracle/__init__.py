"""CPU oracle for the rotated-surface-code trajectory simulator (arXiv:2204.11404).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only callers.  It shares no code with the GPU path and
imports nothing from it.

Parts:
  * ``liboracle.so`` (built from ``qec_oracle.cpp``): complex128 gate-by-gate
    simulation of one trajectory on d^2 data qubits plus one reused ancilla, in
    the order of Sec. II (code, CNOT order, delayed measurement) and Sec. III
    (gate set, noise, protocol) of the paper.
  * :mod:`oracle.statevec`: plain numpy definitions of a k-qubit gate, a
    diagonal, and the ancilla measurement with reset, plus Kronecker-product
    brute force for n <= 8.
  * :mod:`oracle.frame`: Pauli-frame sampler for Pauli-only (Clifford) runs.
  * :mod:`oracle.decoder`: detection events and a minimum-weight matching
    decoder for the logical Z readout.
"""
import contextlib
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

GATESET_CR = 0
GATESET_TEXTBOOK = 1


class _Job(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int),
        ("gateset", ctypes.c_int),
        ("rounds", ctypes.c_int),
        ("twirl", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("p", ctypes.c_double),
        ("zeta", ctypes.c_double),
        ("eps_site", ctypes.POINTER(ctypes.c_double)),
        ("eps", ctypes.c_double),
        ("xbasis", ctypes.c_int),
        ("virtual_z", ctypes.c_int),
        ("idle", ctypes.c_int),
        ("zzp", ctypes.c_int),
        ("max_blocks", ctypes.c_int),
    ]


_lib = None


def lib():
    """Load liboracle.so (built by oracle/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH}; run oracle/build.py")
        _lib = _load(LIB_PATH)
    return _lib


@contextlib.contextmanager
def library_override(path):
    """Route this module's calls to another build of qec_oracle.cpp for the
    duration of the block (the pins' own check that a mistake planted in an
    edited copy of the oracle is caught); the usual library is back after."""
    global _lib
    saved = lib()
    _lib = _load(path)
    try:
        yield _lib
    finally:
        _lib = saved


def _load(path):
    """Open a build of qec_oracle.cpp and declare its entry points."""
    L = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_philox4x32_10.restype = None
    L.orc_uniform.argtypes = [ctypes.c_ulonglong] * 3
    L.orc_uniform.restype = ctypes.c_double
    ip = ctypes.POINTER(ctypes.c_int)
    L.orc_layout.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int]
    L.orc_layout.restype = ctypes.c_int
    L.orc_template_counts.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, ip]
    L.orc_template_counts.restype = ctypes.c_int
    u8p = ctypes.POINTER(ctypes.c_uint8)
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_run_trajectory.argtypes = [ctypes.POINTER(_Job), ctypes.c_ulonglong, u8p, u8p, dp, dp]
    L.orc_run_trajectory.restype = ctypes.c_int
    L.orc_logical_state.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
    L.orc_logical_state.restype = ctypes.c_int
    L.orc_apply_gate.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, dp]
    L.orc_apply_gate.restype = ctypes.c_int
    L.orc_time_blocks.argtypes = [ctypes.POINTER(_Job), ctypes.c_ulonglong, ctypes.c_int, ip]
    L.orc_time_blocks.restype = ctypes.c_double
    L.orc_time_block_range.argtypes = [ctypes.POINTER(_Job), ctypes.c_ulonglong, ctypes.c_int,
                                       ctypes.c_int, ip]
    L.orc_time_block_range.restype = ctypes.c_double
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = None
    return L


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11): 4 counter words, 2 key words."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def uniform(seed, t, k):
    """The uniform draw number k of trajectory t under `seed`."""
    return lib().orc_uniform(int(seed), int(t), int(k))


def layout(d):
    """Stabilizers of the distance-d rotated surface code in measurement order.

    Returns a list of (type, slots) with type 'X' or 'Z' and slots the four
    CNOT partners in circuit order (data labels 1..d^2, 0 = wait)."""
    types = np.zeros(64, dtype=np.int32)
    slots = np.zeros(256, dtype=np.int32)
    n = lib().orc_layout(d, _ptr(types, ctypes.c_int), _ptr(slots, ctypes.c_int), 64)
    if n < 0:
        raise ValueError(f"bad distance {d}")
    return [("X" if types[i] == 0 else "Z", tuple(int(v) for v in slots[4 * i:4 * i + 4])) for i in range(n)]


def template_counts(d, gateset):
    """(stabilizers, gate sites, random draws) per round."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    if lib().orc_template_counts(d, gateset, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) != 0:
        raise ValueError("bad arguments")
    return a.value, b.value, c.value


def run_trajectory(d, gateset, rounds, seed, t, p, zeta=0.0, eps=0.0, eps_site=None,
                   want_state=False, twirl=False, xbasis=False, virtual_z=False, idle=False,
                   zz_plaquette=False, max_blocks=0):
    """One Monte Carlo trajectory.

    twirl: Pauli-twirled over-rotations; xbasis: X-basis memory (logical |+>,
    final X measurement of the data qubits); virtual_z: the Rz restores of the
    cross-resonance Z checks without over-rotation; idle: one-qubit noise on
    the waiting qubits of the circuit at every step; zz_plaquette: the
    crosstalk exp(-i zeta Z_anc Z_q) between the ancilla and every data qubit
    of the running check after each step; max_blocks > 0: stop after that
    many noisy circuits (records and p1 beyond them stay 0, no final
    measurement, `state` is the register at that point).  Returns
    dict(records=uint8[rounds, n_stab], final_bits=uint8[d*d],
    p1=float64[rounds, n_stab], state=complex128[2^(d*d)] or None) where
    `state` is the data register just before the final measurement."""
    n_stab, n_sites, _ = template_counts(d, gateset)
    job = _Job()
    job.d, job.gateset, job.rounds = d, gateset, rounds
    job.seed, job.p, job.zeta, job.eps = int(seed), float(p), float(zeta), float(eps)
    job.twirl = 1 if twirl else 0
    job.xbasis = 1 if xbasis else 0
    job.virtual_z = 1 if virtual_z else 0
    job.idle = 1 if idle else 0
    job.zzp = 1 if zz_plaquette else 0
    job.max_blocks = int(max_blocks)
    keep = None
    if eps_site is not None:
        keep = np.ascontiguousarray(eps_site, dtype=np.float64)
        if keep.shape != (n_sites,):
            raise ValueError(f"eps_site must have {n_sites} entries")
        job.eps_site = _ptr(keep, ctypes.c_double)
    rec = np.zeros((max(rounds, 1), n_stab), dtype=np.uint8)
    fb = np.zeros(d * d, dtype=np.uint8)
    p1 = np.zeros((max(rounds, 1), n_stab), dtype=np.float64)
    st = np.zeros(2 << (d * d), dtype=np.float64) if want_state else None
    rc = lib().orc_run_trajectory(
        ctypes.byref(job), int(t), _ptr(rec, ctypes.c_uint8), _ptr(fb, ctypes.c_uint8),
        _ptr(p1, ctypes.c_double), _ptr(st, ctypes.c_double) if st is not None else None)
    if rc != 0:
        raise RuntimeError("oracle trajectory failed")
    del keep
    return dict(records=rec[:rounds], final_bits=fb, p1=p1[:rounds],
                state=st.view(np.complex128) if st is not None else None)


def logical_zero(d, gateset=GATESET_CR):
    """Logical |0> of the data register after the noise-free projection."""
    out = np.zeros(2 << (d * d), dtype=np.float64)
    if lib().orc_logical_state(d, gateset, 0, _ptr(out, ctypes.c_double)) != 0:
        raise RuntimeError("projection failed")
    return out.view(np.complex128)


def logical_plus(d, gateset=GATESET_CR):
    """Logical |+> of the data register: |+...+> after the noise-free
    projection onto the trivial syndromes."""
    out = np.zeros(2 << (d * d), dtype=np.float64)
    if lib().orc_logical_state(d, gateset, 1, _ptr(out, ctypes.c_double)) != 0:
        raise RuntimeError("projection failed")
    return out.view(np.complex128)


def apply_gate_cpp(state, qubits, m):
    """The C++ oracle's own 1- or 2-qubit gate loop (used to pin it)."""
    s = np.ascontiguousarray(state, dtype=np.complex128).copy()
    n = int(np.log2(s.size))
    q = np.asarray(qubits, dtype=np.int32)
    mm = np.ascontiguousarray(m, dtype=np.complex128)
    rc = lib().orc_apply_gate(_ptr(s.view(np.float64), ctypes.c_double), n, len(q),
                              _ptr(q, ctypes.c_int), _ptr(mm.view(np.float64), ctypes.c_double))
    if rc != 0:
        raise ValueError("bad gate")
    return s


def set_threads(n):
    """OpenMP threads of the oracle's amplitude loops from now on."""
    lib().orc_set_threads(int(n))


def time_blocks(d, gateset, seed, t, p, n_blocks, zeta=0.0, eps=0.0, eps_site=None, first=0):
    """Wall time (s) of n_blocks noisy circuits of the round template from
    circuit `first` on, and the OpenMP thread count used."""
    job = _Job()
    job.d, job.gateset, job.rounds = d, gateset, 1
    job.seed, job.p, job.zeta, job.eps = int(seed), float(p), float(zeta), float(eps)
    keep = None
    if eps_site is not None:
        keep = np.ascontiguousarray(eps_site, dtype=np.float64)
        job.eps_site = _ptr(keep, ctypes.c_double)
    th = ctypes.c_int()
    sec = lib().orc_time_block_range(ctypes.byref(job), int(t), int(first), int(n_blocks),
                                     ctypes.byref(th))
    del keep
    if sec < 0:
        raise ValueError("bad arguments")
    return sec, th.value
