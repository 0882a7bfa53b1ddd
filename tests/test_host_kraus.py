"""Host-side checks of the trajectory engine's formulation (no GPU).

The engine folds each stabilizer circuit, with its sampled Paulis and
over-rotations, into the operator K_m = <m|_anc U |0>_anc on the block's data
qubits, in the monomial form K_m = B P_F diag(D_m) B returned by the
library's host builder (sv_block_kraus).  Applying these operators with numpy
must reproduce the oracle's gate-by-gate trajectory (records, p1, and the data
register before the final measurement), which pins the template, the noise
enumeration and the Kraus builder before any kernel runs.
"""
import numpy as np
import pytest

import oracle
import paper_2204_11404_amd as qs
from oracle import statevec as sv
from test_oracle_circuit import closed_form_logical_zero

CR, TB = "cr", "textbook"
GS = {CR: oracle.GATESET_CR, TB: oracle.GATESET_TEXTBOOK}


def _kraus_dense(k):
    w = len(k["qubits"])
    n = 1 << w
    PF = np.zeros((n, n))
    for x in range(n):
        PF[x ^ k["F"], x] = 1.0
    Wh = np.array([[(-1) ** bin(a & b).count("1") for b in range(n)] for a in range(n)], dtype=float)
    out = []
    for m in (0, 1):
        K = PF @ np.diag(k["D"][m])
        if k["type"] == "X":
            K = Wh @ K @ Wh
        out.append(K)
    return out


def _zz_phase(d, zeta):
    n = d * d
    idx = np.arange(1 << n)
    s = np.zeros(1 << n)
    for row in range(d):
        for col in range(d):
            b = d * row + col
            for c in ([b + 1] if col + 1 < d else []) + ([b + d] if row + 1 < d else []):
                s += np.where(((idx >> b) & 1) == ((idx >> c) & 1), 1.0, -1.0)
    return np.exp(-1j * zeta * s)


def emulate(d, gateset, R, seed, t, p, eps=0.0, eps_site=None, zeta=0.0):
    ns = d * d - 1
    psi = closed_form_logical_zero(d)
    zz = _zz_phase(d, zeta)
    rec = np.zeros((R, ns), dtype=np.uint8)
    p1s = np.zeros((R, ns))
    for r in range(R):
        for s in range(ns):
            k = qs.block_kraus(d, gateset, s, r, seed, t, p, eps, eps_site)
            K = _kraus_dense(k)
            outs = [sv.apply_gate(psi, k["qubits"], K[m]) for m in (0, 1)]
            S = [float(np.vdot(o, o).real) for o in outs]
            p1 = S[1] / (S[0] + S[1])
            p1 = 0.0 if p1 < 1e-10 else (1.0 if p1 > 1 - 1e-10 else p1)
            m = int(k["u"] < p1)
            psi = zz * outs[m] / np.sqrt(S[m])
            rec[r, s], p1s[r, s] = m, p1
    return rec, p1s, psi


@pytest.mark.parametrize("gateset,d,p,eps,zeta", [
    (CR, 2, 0.05, 0.03, 0.04),
    (CR, 3, 0.02, 0.02, 0.01),
    (TB, 3, 0.02, 0.02, 0.0),
    (TB, 2, 0.1, 0.05, 0.05),
])
def test_engine_formulation_matches_oracle(gateset, d, p, eps, zeta):
    R = 3
    for t in range(6):
        rec, p1, psi = emulate(d, gateset, R, 23, t, p, eps=eps, zeta=zeta)
        o = oracle.run_trajectory(d, GS[gateset], R, seed=23, t=t, p=p, eps=eps, zeta=zeta,
                                  want_state=True)
        assert np.array_equal(rec, o["records"])
        assert np.allclose(p1, o["p1"], atol=1e-12)
        assert np.allclose(psi, o["state"], atol=1e-12)


def test_engine_formulation_per_site_angles():
    d, R = 3, 2
    n_sites = oracle.template_counts(d, oracle.GATESET_CR)[1]
    es = np.random.default_rng(5).uniform(0, 0.05, n_sites) / 2
    for t in range(4):
        rec, p1, psi = emulate(d, CR, R, 3, t, 0.01, eps_site=es, zeta=0.01)
        o = oracle.run_trajectory(d, oracle.GATESET_CR, R, seed=3, t=t, p=0.01, eps_site=es,
                                  zeta=0.01, want_state=True)
        assert np.array_equal(rec, o["records"])
        assert np.allclose(psi, o["state"], atol=1e-12)


@pytest.mark.parametrize("d", [2, 3, 4, 5])
@pytest.mark.parametrize("gateset", [CR, TB])
def test_template_counts_agree_with_oracle(d, gateset):
    assert qs.template_info(d, gateset) == oracle.template_counts(d, GS[gateset])


def test_block_qubits_follow_table1_slot_order():
    lay = oracle.layout(5)
    for s, (typ, slots) in enumerate(lay):
        k = qs.block_kraus(5, CR, s, 0, 0, 0, 0.0)
        assert k["type"] == typ
        assert k["qubits"] == [q - 1 for q in slots if q]


def test_draw_stream_matches_oracle():
    for (s, t, k) in [(0, 0, 0), (1, 2, 3), (2 ** 40 + 7, 2 ** 33 + 5, 2 ** 35 + 11)]:
        assert qs.uniform(s, t, k) == oracle.uniform(s, t, k)


def test_library_exports_every_declared_symbol():
    import ctypes
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "qecsv.h")).read()
    declared = set(re.findall(r"^\s*(?:sv_status|const char\*|int|double)\s+(sv_\w+)\(", hdr, re.M))
    assert declared == set(qs.exported_symbols())
    L = ctypes.CDLL(qs.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


def test_argument_errors_are_reported_on_host():
    with pytest.raises(qs.SvError) as e:
        qs.template_info(7, CR)
    assert e.value.status == qs.SV_EINVAL
    with pytest.raises(qs.SvError):
        qs.block_kraus(3, CR, 99, 0, 0, 0, 0.0)
    with pytest.raises(qs.SvError) as e:
        qs.run_rounds(3, CR, 0, 1, 0, 0.0)
    assert e.value.status == qs.SV_EINVAL
    with pytest.raises(qs.SvError):
        qs.run_rounds(3, CR, 1, 1, 0, 1.5)


@pytest.mark.parametrize("gateset", [CR, TB])
@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_pass_layouts_are_consistent(d, gateset):
    """Every register-pass layout of every chain length partitions its tile
    between lanes and register slots consistently (host-side builder)."""
    for zchain in (1, 2, 3, 4, 5, 6):
        n_x = sum(1 for t, _ in oracle.layout(d) if t == "X")
        n_z = (d * d - 1) - n_x
        # one pass per X check and per chain, plus the first and the last
        assert qs.check_pass_layouts(d, gateset, zchain) == n_x + -(-n_z // zchain) + 2
        assert qs.check_pass_layouts(d, gateset, zchain, 0) == n_x + -(-n_z // zchain) + 2
    with pytest.raises(qs.SvError):
        qs.check_pass_layouts(d, gateset, 7)


def _pair_fits(qubit_sets):
    """A pass with a pair needs the qubits of the X members of both its units
    and the three lowest bits in one tile of 2^12 amplitudes."""
    u = set(range(3))
    for q in qubit_sets:
        u |= q
    return len(u) <= 12


@pytest.mark.parametrize("gateset", [CR, TB])
@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_x_pair_layouts(d, gateset):
    """With pairs of consecutive X checks (xpair = 1) every pass layout still
    checks out.  Below 12 qubits no pairs form.  At d = 4 and 5 the X checks
    of a round take the fewest units whose passes fit one tile (brute force
    over the cuts of Table I's X order into singles and pairs, with the
    neighbouring Z chain and logical |0> around the run)."""
    xs = [frozenset(q - 1 for q in s if q) for t, s in oracle.layout(d) if t == "X"]
    n_x, n_z = len(xs), (d * d - 1) - len(xs)

    def cuts(i):
        if i == n_x:
            yield []
            return
        for l in (1, 2):
            if i + l <= n_x:
                for rest in cuts(i + l):
                    yield [xs[i:i + l]] + rest

    best = n_x
    if d * d >= 12:
        for c in cuts(0):
            ok = all(_pair_fits(a + b) for a, b in zip(c, c[1:]) if len(a) == 2 or len(b) == 2)
            ok = ok and all(_pair_fits(u) for u in (c[0], c[-1]))  # from |0>, into the Z chain
            if ok:
                best = min(best, len(c))
    assert best < n_x or d < 4
    for zchain in (1, 2, 3, 4, 5, 6):
        assert qs.check_pass_layouts(d, gateset, zchain, 1) == best + -(-n_z // zchain) + 2
    with pytest.raises(qs.SvError):
        qs.check_pass_layouts(d, gateset, 4, 2)


@pytest.mark.parametrize("gateset", [CR, TB])
@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_spec_layouts(d, gateset):
    """Speculative passes (no data ZZ layer): consecutive X checks two by two
    where the pair's tile (both members' qubits and the three lowest bits)
    fits 2^12 amplitudes, then the Z chains; every layout checks out
    (host-side builder).  Below 12 qubits, and at d = 4 with chains of five or
    six (a chain no four tile bits avoid, summed amplitude by amplitude), the
    plain passes run (0 units)."""
    xs = [frozenset(q - 1 for q in s if q) for t, s in oracle.layout(d) if t == "X"]
    n_x, n_z = len(xs), (d * d - 1) - len(xs)
    units_x, i = 0, 0
    while i < n_x:
        i += 2 if i + 1 < n_x and _pair_fits([xs[i] | xs[i + 1]]) else 1
        units_x += 1
    for zchain in (1, 2, 3, 4, 5, 6):
        plain = d * d < 12 or (d == 4 and zchain >= 5)
        want = 0 if plain else units_x + -(-n_z // zchain)
        assert qs.check_spec_layouts(d, gateset, zchain) == want
    if d >= 4:
        assert units_x == (n_x + 1) // 2  # every pair fits at d = 4, 5
    with pytest.raises(qs.SvError):
        qs.check_spec_layouts(d, gateset, 7)
