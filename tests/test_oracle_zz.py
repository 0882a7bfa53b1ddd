"""Pins of the oracle's data ZZ crosstalk layer exp(-i zeta sum_E Z_i Z_j),
E = the horizontal and vertical nearest-neighbour data pairs of the d x d grid
of Table I (Sec. II.A), applied once per stabilizer circuit just before its
ancilla measurement.  The paper names ZZ crosstalk as the next coherent error
source (Introduction, Conclusion) without simulating it, so its placement is a
reading; what the reading fixes is pinned here by closed forms derived by hand
from Table I's geometry, not by re-running the layer's own loop.

Derivation used by the p1 pins.  Noise off (p = 0, eps = 0): every circuit is
an exact projective measurement of its stabilizer.  Logical |0> (psi0) is a
+1 eigenstate of every check, so the first X check is deterministic and
leaves psi0 unchanged; its ZZ layer U = exp(-i zeta A) then acts.  The second
check S (an X check) sees <U^dag S U> = <psi0| exp(2 i zeta A_S) |psi0>, where
A_S is the sum of the ZZ terms with exactly one end in supp(S) (the others
commute with S).  Expanding prod_k (c + i s P_k), c = cos 2 zeta,
s = sin 2 zeta, a product of terms has expectation 1 on psi0 when it commutes
with every X check and 0 otherwise.  The outcome -1 has probability
(1 - <U^dag S U>) / 2.
"""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import oracle

CR, TB = oracle.GATESET_CR, oracle.GATESET_TEXTBOOK
ZETAS = [0.03, 0.07]


def _flip_probability(d, zeta):
    """P(second X check reads -1) after the first check's ZZ layer.

    d = 3: the checks are X1X2, then S = X2X3X5X6.  Terms with one end in
    {2,3,5,6}: Z1Z2, Z4Z5 (horizontal), Z5Z8, Z6Z9 (vertical).  Z1Z2 and Z4Z5
    anticommute only with S; Z5Z8 and Z6Z9 also with X8X9.  Commuting products:
    {}, {Z1Z2 Z4Z5}, {Z5Z8 Z6Z9}, all four ->
    <.> = c^4 - 2 c^2 s^2 + s^4 = cos^2(4 zeta), P = sin^2(4 zeta) / 2.

    d = 5: the checks are X1X2, then S = X3X4.  Terms: Z2Z3, Z4Z5 (horizontal),
    Z3Z8, Z4Z9 (vertical).  Z2Z3 also anticommutes with X1X2; Z4Z5 only with
    S; Z3Z8 and Z4Z9 also with X8X9X13X14.  Commuting products: {}, {Z3Z8 Z4Z9}
    -> <.> = c^4 - c^2 s^2 = cos^2(2 zeta) cos(4 zeta),
    P = (1 - cos^2(2 zeta) cos(4 zeta)) / 2.
    """
    if d == 3:
        return np.sin(4 * zeta) ** 2 / 2
    if d == 5:
        return (1 - np.cos(2 * zeta) ** 2 * np.cos(4 * zeta)) / 2
    raise ValueError(d)


def _raw_p1(gateset, w, p_minus):
    """Probability of raw ancilla bit 1: the cross-resonance circuit flips the
    ancilla for eigenvalue +1 of a weight-2 check (trivial bit (w/2) mod 2),
    the textbook circuit reads 1 for eigenvalue -1."""
    trivial = (w // 2) % 2 if gateset == CR else 0
    return 1.0 - p_minus if trivial else p_minus


def _check_second_x(run, d, gateset, zeta):
    r = run(d, gateset, 1, seed=1, t=0, p=0.0, zeta=zeta, max_blocks=2)
    lay = oracle.layout(d)
    assert lay[1][0] == "X"
    w = sum(1 for q in lay[1][1] if q)
    return abs(r["p1"][0, 1] - _raw_p1(gateset, w, _flip_probability(d, zeta))) < 1e-13


def _check_d2_phase(run, gateset, zeta):
    """d = 2, one round: X1X2, X3X4, Z1Z2Z3Z4, edges (1,2), (3,4), (1,3),
    (2,4).  psi0 = (|0000> + |1100> + |0011> + |1111>)/2 in label order
    (register indices 0, 3, 12, 15).  U multiplies indices 0 and 15 by
    exp(-4 i zeta) (all four pairs aligned) and 3, 12 by 1 (two aligned, two
    anti-aligned).  X1X2 is trivial; measuring X3X4 on U psi0 reads -1 with
    probability sin^2(2 zeta); either projection is, up to a factor,
    |0> + e|3> + e|12> + |15> with e = +1 (outcome +1) or -1 (outcome -1); two
    more layers (X3X4's and the trivial Z check's) make the final ratio
    amp(0) / amp(3) = e exp(-8 i zeta).  The sign of the exponent pins the sign
    of zeta, which no probability of this real circuit can see."""
    r = run(2, gateset, 1, seed=3, t=0, p=0.0, zeta=zeta, want_state=True)
    st = r["state"]
    trivial = 1 if gateset == CR else 0
    e = 1.0 if int(r["records"][0, 1]) == trivial else -1.0
    ok = abs(r["p1"][0, 1] - _raw_p1(gateset, 2, np.sin(2 * zeta) ** 2)) < 1e-13
    ok &= np.allclose(np.abs(st[[0, 3, 12, 15]]), 0.5, atol=1e-12)
    ok &= abs(st[0] / st[3] - e * np.exp(-8j * zeta)) < 1e-12
    ok &= abs(st[15] - st[0]) < 1e-12 and abs(st[12] - st[3]) < 1e-12
    return bool(ok)


@pytest.mark.parametrize("zeta", ZETAS)
@pytest.mark.parametrize("gateset", [TB, CR])
def test_second_x_check_flip_closed_form_d3(gateset, zeta):
    assert _check_second_x(oracle.run_trajectory, 3, gateset, zeta)


@pytest.mark.parametrize("gateset,zeta", [(TB, 0.07), (CR, 0.03)])
def test_second_x_check_flip_closed_form_d5(gateset, zeta):
    # 26 qubits: one noise-free preparation and two circuits per case
    assert _check_second_x(oracle.run_trajectory, 5, gateset, zeta)


@pytest.mark.parametrize("zeta", ZETAS)
@pytest.mark.parametrize("gateset", [TB, CR])
def test_d2_round_phase_closed_form(gateset, zeta):
    assert _check_d2_phase(oracle.run_trajectory, gateset, zeta)


# Each planted mistake is a textual edit of the oracle's ZZ layer; the edited
# copy is compiled and loaded on the CPU, and at least one pin must reject it.
_SRC = os.path.join(os.path.dirname(oracle.__file__), "qec_oracle.cpp")
_MUTANTS = {
    "no_vertical_edges": ("if (row + 1 < d) edges.push_back({b, b + d});", ""),
    "no_horizontal_edges": ("if (col + 1 < d) edges.push_back({b, b + 1});", ""),
    "zeta_sign_flipped": ("cplx(0.0, -zeta * (double)sum)", "cplx(0.0, zeta * (double)sum)"),
    "extra_diagonal_edge": (
        "if (row + 1 < d) edges.push_back({b, b + d});",
        "if (row + 1 < d) edges.push_back({b, b + d});\n"
        "      if (row + 1 < d && col + 1 < d) edges.push_back({b, b + d + 1});"),
}


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_pins_reject_planted_zz_mistakes(name, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    old, new = _MUTANTS[name]
    src = open(_SRC).read()
    assert src.count(old) == 1, "the ZZ layer's source changed; update the planted mistake"
    mutated = tmp_path / "mutant.cpp"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-fcx-limited-range", "-fopenmp",
                    "-fPIC", "-shared", str(mutated), "-o", str(so)], check=True)
    with oracle.library_override(str(so)):
        caught = []
        for zeta in ZETAS:
            for gs in (TB, CR):
                caught.append(not _check_second_x(oracle.run_trajectory, 3, gs, zeta))
                caught.append(not _check_d2_phase(oracle.run_trajectory, gs, zeta))
    assert any(caught), f"no pin catches the planted mistake {name}"
    # the unmodified library is back
    assert _check_second_x(oracle.run_trajectory, 3, TB, ZETAS[0])
    assert re.search(r"liboracle\.so$", oracle.lib()._name)
