"""GPU parity of the register ops behind the C ABI against the numpy oracle.

Each case runs the HIP kernel through libqecsv on a seeded random state and
compares element by element with oracle.statevec (the plain definition),
which is itself pinned to Kronecker brute force in the CPU tests.
Tolerances: complex128 1e-12 absolute (unit-norm states, O(n) rounding steps);
complex64 2e-6 (float32 rounding of O(1)-magnitude sums of up to 32 terms
on normalised states, whose amplitudes are <= 1).
"""
import numpy as np
import pytest

import paper_2204_11404_amd as qs
import workloads
from oracle import statevec as sv

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-6}


def _state(n, dtype, seed):
    psi = workloads.random_state(n, seed)
    s = qs.State(n, dtype)
    s.set(psi)
    # the reference starts from the same rounded values
    return s, s.get().astype(np.complex128)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [5, 11, 18])
def test_apply_gate_every_position(dtype, n):
    for k in (1, 2):
        for trial, q0 in enumerate(range(n)):
            qubits = [q0] if k == 1 else [q0, (q0 + 1 + trial % (n - 1)) % n]
            if k == 2 and qubits[0] == qubits[1]:
                continue
            print(f"case gate k={k} n={n} {dtype} qubits={qubits}", flush=True)
            s, ref = _state(n, dtype, 100 * k + q0)
            m = workloads.random_matrix(k, 7 * q0 + k)
            s.apply_gate(qubits, m)
            got = s.get()
            want = sv.apply_gate(ref, qubits, m)
            assert np.max(np.abs(got - want)) < TOL[dtype]
            s.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_gate_low_pairs(dtype):
    """Two-qubit gates on low qubits: every ordered pair below 4, on registers
    of 8, 9 (one block of the lane kernels) and 12 qubits; (0, 1) and (1, 0)
    exchange the quadruple between lanes (complex128: one amplitude per lane,
    DPP quads; complex64: two per lane, DPP lane pairs)."""
    for n in (8, 9, 12):
        for q0 in range(4):
            for q1 in range(4):
                if q0 == q1:
                    continue
                print(f"case gate low pair n={n} {dtype} qubits={[q0, q1]}", flush=True)
                s, ref = _state(n, dtype, 300 + 10 * q0 + q1)
                m = workloads.random_matrix(2, 400 + 10 * q0 + q1)
                s.apply_gate([q0, q1], m)
                assert np.max(np.abs(s.get() - sv.apply_gate(ref, [q0, q1], m))) < TOL[dtype]
                s.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_apply_diag(dtype, k):
    n = 14
    rng = np.random.default_rng(k)
    qubits = list(rng.choice(n, size=k, replace=False))
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, size=1 << k))
    print(f"case diag k={k} {dtype} qubits={qubits}", flush=True)
    s, ref = _state(n, dtype, 40 + k)
    s.apply_diag(qubits, ph)
    assert np.max(np.abs(s.get() - sv.apply_diag(ref, qubits, ph))) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_apply_fused(dtype, k):
    n = 16
    rng = np.random.default_rng(10 + k)
    for rep in range(3):
        qubits = [int(x) for x in rng.choice(n, size=k, replace=False)]
        print(f"case fused k={k} {dtype} qubits={qubits}", flush=True)
        s, ref = _state(n, dtype, 60 + 3 * k + rep)
        m = workloads.random_matrix(k, 90 + k + rep)
        s.apply_fused(qubits, m)
        assert np.max(np.abs(s.get() - sv.apply_gate(ref, qubits, m))) < TOL[dtype] * (1 << k)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k,n,qubits", [
    (5, 9, [4, 0, 8, 2, 6]),          # one 16-group MFMA tile
    (4, 8, [7, 1, 0, 5]),
    (5, 8, [0, 1, 2, 3, 4]),          # fewer than 16 groups: scalar kernel
    (5, 22, [0, 1, 2, 3, 4]),         # contiguous low block, many tiles per wave
    (5, 22, [21, 17, 20, 18, 19]),    # high block, unsorted
    (4, 22, [3, 12, 0, 21]),
    # targets = the k lowest bits in any order: contiguous groups staged
    # through LDS
    (5, 9, [2, 4, 0, 3, 1]),          # exactly one tile
    (5, 16, [3, 0, 4, 1, 2]),
    (4, 12, [2, 0, 3, 1]),
    (4, 20, [0, 1, 2, 3]),
])
def test_apply_fused_tiles(dtype, k, n, qubits):
    """The matrix-core path (k = 4, 5 with at least 16 groups) at the tile
    edge, with low, high and scattered target qubits, and the scalar kernel
    below one tile; three calls in a row reuse the matrix slots."""
    print(f"case fused tiles k={k} n={n} {dtype} qubits={qubits}", flush=True)
    s, ref = _state(n, dtype, 500 + n + k)
    want = ref
    for rep in range(3):
        m = workloads.random_matrix(k, 700 + 10 * n + rep)
        s.apply_fused(qubits, m)
        want = sv.apply_gate(want, qubits, m)
    assert np.max(np.abs(s.get() - want)) < 3 * TOL[dtype] * (1 << k)
    s.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_fused_many_calls(dtype):
    """More calls than matrix slots without a synchronisation in between:
    each call's matrix must be the one its kernel reads."""
    n, k = 12, 5
    print(f"case fused ring {dtype}", flush=True)
    s, ref = _state(n, dtype, 77)
    want = ref
    rng = np.random.default_rng(5)
    for rep in range(20):
        qubits = [int(x) for x in rng.choice(n, size=k, replace=False)]
        m = workloads.random_matrix(k, 1000 + rep)
        s.apply_fused(qubits, m)
        m[:] = 0.0       # the caller may reuse its buffer once the call returns
        want = sv.apply_gate(want, qubits, workloads.random_matrix(k, 1000 + rep))
    assert np.max(np.abs(s.get() - want)) < 20 * TOL[dtype] * (1 << k)
    s.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_measure_reset(dtype):
    n = 16
    for anc in (0, 7, n - 1):
        for u in (0.0, 0.3, 0.999):
            print(f"case measure anc={anc} u={u} {dtype}", flush=True)
            s, ref = _state(n, dtype, anc + 1)
            m, p1 = s.measure_reset(anc, u)
            mo, p1o, out = sv.measure_reset(ref, anc, u=u)
            assert m == mo
            assert abs(p1 - p1o) < 1e-12
            assert np.max(np.abs(s.get() - out)) < TOL[dtype] * 4


def test_measure_reset_forced_and_enumeric():
    n = 10
    s = qs.State(n, "c128")
    s.set_basis(0b1000000000)  # qubit 9 in |1>
    with pytest.raises(qs.SvError) as e:
        s.measure_reset_forced(9, 0)
    assert e.value.status == qs.SV_ENUMERIC
    p1 = s.measure_reset_forced(9, 1)
    assert p1 == 1.0
    got = s.get()
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = 1.0
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_load_logical0(dtype, d):
    from test_oracle_circuit import closed_form_logical_zero
    print(f"case logical0 d={d} {dtype}", flush=True)
    s = qs.State(d * d + 1, dtype)
    s.load_logical0(d)
    got = s.get()
    want = np.zeros(2 << (d * d), dtype=np.complex128)
    want[: 1 << (d * d)] = closed_form_logical_zero(d)
    assert np.max(np.abs(got - want)) < TOL[dtype]


def test_wrap_torch_tensor_and_stream():
    import torch
    n = 12
    t = torch.zeros(2 << n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    s = qs.State(n, "c128", stream=stream, tensor=t)
    s.set_basis(5)
    s.synchronize()
    host = t.cpu().numpy().view(np.complex128)
    assert host[5] == 1.0 and np.count_nonzero(host) == 1
    s.free()
    assert t.abs().sum().item() == 1.0  # memory still owned by torch


def test_invalid_arguments_rejected_before_launch():
    s = qs.State(6, "c128")
    for bad in ([6], [-1]):
        with pytest.raises(qs.SvError) as e:
            s.apply_gate(bad, np.eye(2))
        assert e.value.status == qs.SV_EINVAL
    with pytest.raises(qs.SvError):
        s.apply_gate([1, 1], np.eye(4))
    with pytest.raises(qs.SvError):
        s.apply_fused([0, 1, 2, 3, 4, 5], np.eye(64))
    with pytest.raises(qs.SvError):
        s.load_logical0(3)  # 6 qubits < 9
    assert np.array_equal(s.get(), np.eye(1, 64, 0, dtype=np.complex128)[0])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_copy_state(dtype):
    n = 15
    a, ref = _state(n, dtype, 77)
    b = qs.State(n, dtype)
    b.copy_from(a)
    assert np.array_equal(b.get(), a.get())
    with pytest.raises(qs.SvError):
        b.copy_from(qs.State(n - 1, dtype))
