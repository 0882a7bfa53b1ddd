"""Pins of the oracle's code layout against what the paper prints (Sec. II.A,
Table I) and against the algebra of stabilizer codes."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_d5.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            idx, xs, zs = line.split()
            rows.append((int(idx), [int(v) for v in xs.split(",")], [int(v) for v in zs.split(",")]))
    return rows


def test_table1_verbatim_and_in_order():
    st = oracle.layout(5)
    xs = [s for t, s in st if t == "X"]
    zs = [s for t, s in st if t == "Z"]
    rows = _read_table1()
    assert len(xs) == len(zs) == len(rows) == 12
    # the round measures every X stabilizer, then every Z stabilizer
    assert [t for t, _ in st] == ["X"] * 12 + ["Z"] * 12
    for (idx, xsup, zsup), xsl, zsl in zip(rows, xs, zs):
        assert sorted(q for q in xsl if q) == sorted(xsup), idx
        assert sorted(q for q in zsl if q) == sorted(zsup), idx


def test_cnot_order_examples():
    st = oracle.layout(5)
    with open(os.path.join(GOLDEN, "cnot_order_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            typ, sup, order = line.split()
            sup = sorted(int(v) for v in sup.split(","))
            want = tuple(0 if v == "W" else int(v) for v in order.split(","))
            got = [s for t, s in st if t == typ and sorted(q for q in s if q) == sup]
            assert got == [want]


@pytest.mark.parametrize("d,nx,nz", [(2, 2, 1), (3, 4, 4), (4, 8, 7), (5, 12, 12)])
def test_counts(d, nx, nz):
    st = oracle.layout(d)
    assert sum(t == "X" for t, _ in st) == nx
    assert sum(t == "Z" for t, _ in st) == nz
    assert len(st) == d * d - 1
    # every data qubit is covered, weights are 2 or 4
    for _, s in st:
        assert sum(1 for q in s if q) in (2, 4)


def _supports(d):
    return [(t, {q for q in s if q}) for t, s in oracle.layout(d)]


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_stabilizers_commute(d):
    sup = _supports(d)
    for ta, a in sup:
        for tb, b in sup:
            if ta != tb:
                assert len(a & b) % 2 == 0


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_logical_operators(d):
    """Z_L on the top row and X_L on the left column commute with every
    stabilizer and anticommute with each other; they are independent of the
    stabilizers (rank check over GF(2))."""
    sup = _supports(d)
    zl = set(range(1, d + 1))
    xl = {d * r + 1 for r in range(d)}
    for t, s in sup:
        if t == "X":
            assert len(s & zl) % 2 == 0
        else:
            assert len(s & xl) % 2 == 0
    assert len(zl & xl) % 2 == 1

    def rank(rows):
        m = np.array(rows, dtype=np.uint8) % 2
        r = 0
        for c in range(m.shape[1]):
            piv = [i for i in range(r, m.shape[0]) if m[i, c]]
            if not piv:
                continue
            m[[r, piv[0]]] = m[[piv[0], r]]
            for i in range(m.shape[0]):
                if i != r and m[i, c]:
                    m[i] ^= m[r]
            r += 1
        return r

    vec = lambda s: [1 if q in s else 0 for q in range(1, d * d + 1)]
    zrows = [vec(s) for t, s in sup if t == "Z"]
    assert rank(zrows + [vec(zl)]) == rank(zrows) + 1


def test_paper_logical_z_is_not_a_logical_operator():
    """The printed Z_L = Z1 Z7 Z13 Z19 Z25 (Sec. III.B) anticommutes with X
    stabilizers of Table I; the top-row operator is used instead."""
    diag = {1, 7, 13, 19, 25}
    bad = [s for t, s in _supports(5) if t == "X" and len(s & diag) % 2]
    assert len(bad) == 8


@pytest.mark.parametrize("d,gateset,sites,draws", [
    (5, oracle.GATESET_CR, 184, 224),     # 12 X (8 w4, 4 w2), 12 Z (8 w4, 4 w2)
    (3, oracle.GATESET_CR, 56, 72),
    (3, oracle.GATESET_TEXTBOOK, 16, 48),
])
def test_template_counts_closed_form(d, gateset, sites, draws):
    # CR: X-check 2 + 2w sites, 1+4+1+w+1 draws; Z-check 2w sites, 4+w+1 draws.
    # textbook: 2 sites, 1+w+1+1 draws per check.
    ns, s, k = oracle.template_counts(d, gateset)
    assert (ns, s, k) == (d * d - 1, sites, draws)
