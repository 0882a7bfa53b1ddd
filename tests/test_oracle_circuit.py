"""Pins of the oracle's trajectories against facts fixed by the paper and by
the mathematics of stabilizer measurement (Sec. II-III of arXiv:2204.11404)."""
import numpy as np
import pytest

import oracle
from oracle import frame
from oracle import statevec as sv

CR, TB = oracle.GATESET_CR, oracle.GATESET_TEXTBOOK


def trivial_bits(d, gateset):
    """Raw ancilla bit of a +1 eigenvalue: w/2 mod 2 for the cross-resonance
    circuit (product of w rotations by pi/4 about Z_q X_a), 0 for textbook."""
    return np.array([(sum(1 for q in s if q) // 2) % 2 if gateset == CR else 0
                     for _, s in oracle.layout(d)], dtype=np.uint8)


def closed_form_logical_zero(d):
    """2^(-n_X/2) on every data basis state in the GF(2) span of the X
    stabilizer supports (the orbit of |0...0> under the X stabilizer group)."""
    gens = []
    for t, s in oracle.layout(d):
        if t == "X":
            v = 0
            for q in s:
                if q:
                    v |= 1 << (q - 1)
            gens.append(v)
    span = {0}
    for g in gens:
        span |= {x ^ g for x in span}
    psi = np.zeros(1 << (d * d), dtype=np.complex128)
    psi[list(span)] = 2.0 ** (-len(gens) / 2)
    assert len(span) == 2 ** len(gens)
    return psi


@pytest.mark.parametrize("gateset", [CR, TB])
@pytest.mark.parametrize("d", [2, 3, 4])
def test_logical_zero_closed_form(d, gateset):
    # Sec. III.B: |0...0> projected by noise-free syndrome measurements with
    # trivial outcomes; phase fixed so <0...0|psi> > 0.
    assert np.allclose(oracle.logical_zero(d, gateset), closed_form_logical_zero(d), atol=1e-12)


@pytest.mark.parametrize("gateset", [CR, TB])
@pytest.mark.parametrize("d", [2, 3, 4])
def test_noiseless_rounds_are_trivial_and_leave_code_state(d, gateset):
    r = oracle.run_trajectory(d, gateset, 3, seed=5, t=1, p=0.0, want_state=True)
    assert np.array_equal(r["records"], np.tile(trivial_bits(d, gateset), (3, 1)))
    assert set(np.unique(r["p1"])) <= {0.0, 1.0}
    lz = closed_form_logical_zero(d)
    # invariant up to a global phase
    assert abs(abs(np.vdot(lz, r["state"])) - 1.0) < 1e-12
    # final Z measurement gives a codeword of the X orbit: Z stabilizers and
    # the top-row logical Z have even parity
    fb = r["final_bits"]
    for t, s in oracle.layout(d):
        if t == "Z":
            assert sum(int(fb[q - 1]) for q in s if q) % 2 == 0
    assert sum(int(fb[q]) for q in range(d)) % 2 == 0


def test_textbook_first_block_over_rotation():
    """Textbook circuit with exp(-i eps X) after each H and no other noise: the
    first check (X1X2 on logical 0) reads 1 with probability sin^2(eps)
    (the over-rotation relation of Sec. III.A with theta = 2 eps)."""
    eps = 0.02
    r = oracle.run_trajectory(3, TB, 1, seed=0, t=0, p=0.0, eps=eps)
    assert abs(r["p1"][0, 0] - np.sin(eps) ** 2) < 1e-14
    assert abs(np.sin(eps) ** 2 - 3.9995e-4) < 1e-8


def _cr_sites(d):
    """Kind of each gate site of the cross-resonance round template."""
    kinds = []
    for t, s in oracle.layout(d):
        w = sum(1 for q in s if q)
        if t == "X":
            kinds += ["anc"] + ["cr"] * w + ["anc"] + ["restore"] * w
        else:
            kinds += ["cr"] * w + ["restore"] * w
    return kinds


@pytest.mark.parametrize("d", [2, 3, 4])
def test_cr_first_block_over_rotation_on_cr_gates(d):
    """Over-rotation eps only on the two CR gates of X1X2: the ancilla turns by
    2(pi/4 + eps) instead of pi/2, so the check misses its trivial bit with
    probability sin^2(2 eps)."""
    eps = 0.013
    kinds = _cr_sites(d)
    es = np.array([eps if k == "cr" else 0.0 for k in kinds])
    r = oracle.run_trajectory(d, CR, 1, seed=0, t=0, p=0.0, eps_site=es)
    # raw trivial bit of a weight-2 check is 1
    assert abs((1.0 - r["p1"][0, 0]) - np.sin(2 * eps) ** 2) < 1e-13


@pytest.mark.parametrize("gateset", [CR, TB])
def test_norm_preserved(gateset):
    r = oracle.run_trajectory(3, gateset, 4, seed=9, t=3, p=0.02, eps=0.03, zeta=0.02,
                              want_state=True)
    assert abs(np.linalg.norm(r["state"]) - 1.0) < 1e-12


def test_zz_only_never_fires_z_checks_or_flips_logical_z():
    """ZZ crosstalk is diagonal: it commutes with Z checks and Z_L, so with no
    other noise Z records stay trivial and the top-row parity stays even."""
    d = 3
    tb = trivial_bits(d, CR)
    isz = np.array([t == "Z" for t, _ in oracle.layout(d)])
    fired_x = 0
    for t in range(40):
        r = oracle.run_trajectory(d, CR, 3, seed=4, t=t, p=0.0, zeta=0.15)
        assert np.array_equal(r["records"][:, isz], np.tile(tb[isz], (3, 1)))
        assert sum(int(r["final_bits"][q]) for q in range(d)) % 2 == 0
        fired_x += int(np.any(r["records"][:, ~isz] != tb[~isz]))
    assert fired_x > 0  # but X checks do see it


def _detectors(flips):
    prev = np.concatenate([np.zeros_like(flips[:, :1]), flips[:, :-1]], axis=1)
    return (flips ^ prev).reshape(flips.shape[0], -1)


@pytest.mark.parametrize("gateset,d,p", [(CR, 3, 0.01), (TB, 3, 0.01), (CR, 2, 0.03)])
def test_pauli_only_matches_frame_sampler(gateset, d, p):
    """Pauli-only noise makes the circuit Clifford; detector and logical-Z flip
    rates of the oracle agree with the Pauli-frame sampler."""
    R, N = 3, 2500
    tb = trivial_bits(d, gateset)
    recs, zl = [], []
    for t in range(N):
        r = oracle.run_trajectory(d, gateset, R, seed=11, t=t, p=p)
        recs.append(r["records"] ^ tb)
        zl.append(sum(int(r["final_bits"][q]) for q in range(d)) % 2)
    recs = np.array(recs)
    frec, ffin = frame.sample(d, gateset, R, p, 200000, seed=2)
    a = _detectors(recs).mean(0)
    b = _detectors(frec).mean(0)
    sig = np.sqrt(np.maximum(b * (1 - b), 1.0 / N) / N)
    z = (a - b) / sig
    assert np.max(np.abs(z)) < 4.0
    assert np.sum(z ** 2) < len(z) + 4.0 * np.sqrt(2 * len(z)) + 10
    zl_f = np.bitwise_xor.reduce(ffin[:, :d], axis=1).mean()
    zl_o = np.mean(zl)
    assert abs(zl_o - zl_f) < 4.0 * np.sqrt(max(zl_f * (1 - zl_f), 1.0 / N) / N)


def test_final_measurement_is_born_sampling():
    """The sequential MSB-first Z measurement of the data register samples the
    Born distribution: for noiseless d=2 the four X-orbit codewords appear
    uniformly and nothing else appears."""
    d = 2
    lz = closed_form_logical_zero(d)
    allowed = set(np.nonzero(np.abs(lz) > 0)[0].tolist())
    counts = {}
    N = 2000
    for t in range(N):
        fb = oracle.run_trajectory(d, CR, 1, seed=21, t=t, p=0.0)["final_bits"]
        x = sum(int(b) << q for q, b in enumerate(fb))
        counts[x] = counts.get(x, 0) + 1
    assert set(counts) == allowed
    exp = N / len(allowed)
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 16.3  # 3 dof, p = 1e-3


# ---- dense brute force of a whole d=2 trajectory with the same draws ------

def _dense_trajectory(d, gateset, rounds, seed, t, p, eps, zeta, twirl=False, idle=False, zzp=False):
    nd = d * d
    n = nd + 1
    anc = nd
    X, Y, Z = sv.pauli("X"), sv.pauli("Y"), sv.pauli("Z")
    P = [sv.pauli("I"), X, Y, Z]
    H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)

    def rot(M, beta):
        return np.cos(beta) * np.eye(M.shape[0]) - 1j * np.sin(beta) * M

    def g(qs, m):
        return sv.kron_gate(n, qs, m)

    psi = np.kron(np.array([1, 0]), closed_form_logical_zero(d)).astype(np.complex128)
    k = 0
    rec = np.zeros((rounds, nd - 1), dtype=np.uint8)

    def draw():
        nonlocal k
        u = oracle.uniform(seed, t, k)
        k += 1
        return u

    def n1(q):
        nonlocal psi
        u = draw()
        for j in (1, 2, 3):
            if u < j * p / 3.0:
                psi = g([q], P[j]) @ psi
                return

    def n2(q1, q2):
        nonlocal psi
        u = draw()
        for j in range(1, 16):
            if u < j * p / 15.0:
                psi = g([q1, q2], np.kron(P[j & 3], P[j >> 2])) @ psi
                return

    def site(qs, M, sign, base):
        """Gate site: exp(-i sign (base + eps) M), or in the twirled model the
        base rotation and then, on one draw u < sin^2 eps, the Pauli M."""
        nonlocal psi
        if not twirl:
            psi = g(qs, rot(M, sign * (base + eps))) @ psi
            return
        psi = g(qs, rot(M, sign * base)) @ psi
        if draw() < np.sin(eps) ** 2:
            psi = g(qs, M) @ psi

    def wait(slots, busy):
        """End of a step: idle noise (N1 on the check's other data qubits, slot
        order), then the ancilla-plaquette crosstalk exp(-i zeta Z_anc Z_q) on
        each of the check's data qubits."""
        nonlocal psi
        if idle and busy is not None:
            for q in slots:
                if q and q != busy:
                    n1(q - 1)
        if zzp:
            for q in slots:
                if q:
                    psi = g([anc, q - 1], np.diag(np.exp(-1j * zeta * np.array([1, -1, -1, 1])))) @ psi

    # ZX with bit0 = control (Z), bit1 = target (X): kron(X, Z)
    ZX = np.kron(X, Z)
    edges = []
    for row in range(d):
        for col in range(d):
            b = d * row + col
            if col + 1 < d:
                edges.append((b, b + 1))
            if row + 1 < d:
                edges.append((b, b + d))
    idx = np.arange(1 << n)
    zzsum = np.zeros(1 << n)
    for a, b in edges:
        zzsum += np.where(((idx >> a) & 1) == ((idx >> b) & 1), 1.0, -1.0)
    zzphase = np.exp(-1j * zeta * zzsum)
    q4 = np.pi / 4
    for r in range(rounds):
        for i, (typ, slots) in enumerate(oracle.layout(d)):
            if gateset == CR:
                if typ == "X":
                    site([anc], X, -1, q4); n1(anc); wait(slots, 0)
                    for q in slots:
                        if q:
                            site([anc, q - 1], ZX, 1, q4); n2(anc, q - 1)
                        else:
                            n1(anc)
                        wait(slots, q)
                    site([anc], X, 1, q4); n1(anc)
                    for q in slots:
                        if q:
                            site([q - 1], X, 1, q4); n1(q - 1)
                    wait(slots, None)  # no waiting qubit in the last step
                else:
                    for q in slots:
                        if q:
                            site([q - 1, anc], ZX, 1, q4); n2(q - 1, anc)
                        else:
                            n1(anc)
                        wait(slots, q)
                    for q in slots:
                        if q:
                            site([q - 1], Z, 1, q4); n1(q - 1)
                    if idle:
                        n1(anc)
                    wait(slots, None)
            else:
                psi = g([anc], H) @ psi; site([anc], X, 1, 0.0); n1(anc); wait(slots, 0)
                for q in slots:
                    if q:
                        if typ == "X":
                            m = np.zeros((4, 4)); m[0, 0] = m[2, 2] = m[3, 1] = m[1, 3] = 1
                        else:
                            m = np.diag([1, 1, 1, -1]).astype(float)
                        psi = g([anc, q - 1], m) @ psi; n2(anc, q - 1); wait(slots, q)
                psi = g([anc], H) @ psi; site([anc], X, 1, 0.0); n1(anc); wait(slots, 0)
            psi = zzphase * psi
            m, _, psi = sv.measure_reset(psi, anc, u=draw())
            rec[r, i] = m
    state = psi[: 1 << nd].copy()
    fb = np.zeros(nd, dtype=np.uint8)
    for q in range(nd, 0, -1):
        S0, S1 = sv.half_norms(psi, q - 1)
        p1 = S1 / (S0 + S1)
        p1 = 0.0 if p1 < 1e-10 else (1.0 if p1 > 1 - 1e-10 else p1)
        b = int(draw() < p1)
        keep = ((idx >> (q - 1)) & 1) == b
        psi = np.where(keep, psi, 0) / np.sqrt(S1 if b else S0)
        fb[q - 1] = b
    return rec, fb, state


@pytest.mark.parametrize("gateset", [CR, TB])
def test_dense_brute_force_d2_trajectories(gateset):
    d, R = 2, 3
    for t, (p, eps, zeta) in enumerate([(0.05, 0.0, 0.0), (0.08, 0.04, 0.0), (0.1, 0.03, 0.05),
                                        (0.2, 0.1, 0.1)]):
        rec, fb, st = _dense_trajectory(d, gateset, R, 17, t, p, eps, zeta)
        o = oracle.run_trajectory(d, gateset, R, seed=17, t=t, p=p, eps=eps, zeta=zeta,
                                  want_state=True)
        assert np.array_equal(o["records"], rec)
        assert np.array_equal(o["final_bits"], fb)
        assert np.allclose(o["state"], st, atol=1e-12)


@pytest.mark.parametrize("gateset", [CR, TB])
def test_dense_brute_force_d2_twirled_trajectories(gateset):
    """Pauli-twirled over-rotations (one draw after each rotation; its
    generator with probability sin^2 eps) against the dense brute force."""
    d, R = 2, 3
    hits = 0
    for t, (p, eps, zeta) in enumerate([(0.05, 0.3, 0.0), (0.1, 0.25, 0.05), (0.0, 0.4, 0.02)]):
        rec, fb, st = _dense_trajectory(d, gateset, R, 23, t, p, eps, zeta, twirl=True)
        o = oracle.run_trajectory(d, gateset, R, seed=23, t=t, p=p, eps=eps, zeta=zeta,
                                  want_state=True, twirl=True)
        assert np.array_equal(o["records"], rec)
        assert np.array_equal(o["final_bits"], fb)
        assert np.allclose(o["state"], st, atol=1e-12)
        hits += int(np.any(rec != trivial_bits(d, gateset)))
    assert hits > 0


def test_twirled_textbook_first_check_flips_with_sin2_eps():
    """Twirled textbook circuit, no other noise: the X after the last H of the
    first check flips its outcome with probability sin^2 eps, the same as the
    coherent error (whose p1 is sin^2 eps exactly)."""
    eps, n = 0.2, 4000
    flips = sum(int(oracle.run_trajectory(2, TB, 1, seed=3, t=t, p=0.0, eps=eps,
                                          twirl=True)["records"][0, 0]) for t in range(n))
    q = np.sin(eps) ** 2
    assert abs(flips / n - q) < 4 * np.sqrt(q * (1 - q) / n)


# ---- X-basis memory ---------------------------------------------------------

def closed_form_logical_plus(d):
    """Uniform superposition over the data strings with even parity on every
    Z check: |+...+> projected onto the trivial Z syndromes."""
    n = d * d
    zs = [[q - 1 for q in s if q] for t, s in oracle.layout(d) if t == "Z"]
    idx = np.arange(1 << n)
    ok = np.ones(1 << n, dtype=bool)
    for sup in zs:
        par = np.zeros(1 << n, dtype=np.int64)
        for q in sup:
            par ^= (idx >> q) & 1
        ok &= par == 0
    v = ok.astype(np.complex128)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("gateset", [CR, TB])
@pytest.mark.parametrize("d", [2, 3])
def test_logical_plus_closed_form(d, gateset):
    ref = closed_form_logical_plus(d)
    assert int(np.count_nonzero(ref)) == 1 << (d * d - (d * d - 1) // 2)
    assert np.allclose(oracle.logical_plus(d, gateset), ref, atol=1e-12)


@pytest.mark.parametrize("gateset", [CR, TB])
def test_noiseless_x_memory_is_trivial(gateset):
    """Logical |+>: every X check reads its trivial bit from round 1, every
    Z check stays constant after round 1, and the final X outcomes have even
    parity on every X check and on X_L (the first column)."""
    d, R = 3, 3
    for t in range(4):
        o = oracle.run_trajectory(d, gateset, R, seed=2, t=t, p=0.0, xbasis=True)
        r0 = trivial_bits(d, gateset)
        layout = oracle.layout(d)
        xi = [i for i, (typ, _) in enumerate(layout) if typ == "X"]
        zi = [i for i, (typ, _) in enumerate(layout) if typ == "Z"]
        assert np.array_equal(o["records"][:, xi], np.broadcast_to(r0[xi], (R, len(xi))))
        assert np.array_equal(o["records"][1:, zi], np.broadcast_to(o["records"][0, zi], (R - 1, len(zi))))
        fb = o["final_bits"]
        for i in xi:
            assert sum(int(fb[q - 1]) for q in layout[i][1] if q) % 2 == 0
        assert sum(int(fb[d * r]) for r in range(d)) % 2 == 0


@pytest.mark.parametrize("gateset", [CR, TB])
def test_x_memory_pauli_only_matches_frame_sampler(gateset):
    """X-basis memory with Pauli-only noise: X-check detector rates and the X_L
    flip rate (final X outcomes on the first column) agree with the
    Pauli-frame sampler read out in the X basis."""
    d, R, N, p = 3, 3, 2500, 0.01
    layout = oracle.layout(d)
    xi = [i for i, (typ, _) in enumerate(layout) if typ == "X"]
    tb = trivial_bits(d, gateset)
    recs, xl = [], []
    for t in range(N):
        r = oracle.run_trajectory(d, gateset, R, seed=13, t=t, p=p, xbasis=True)
        recs.append((r["records"] ^ tb)[:, xi])
        xl.append(sum(int(r["final_bits"][d * k]) for k in range(d)) % 2)
    recs = np.array(recs)
    frec, ffin = frame.sample(d, gateset, R, p, 200000, seed=3, basis="X")
    a = _detectors(recs).mean(0)
    b = _detectors(frec[:, :, xi]).mean(0)
    sig = np.sqrt(np.maximum(b * (1 - b), 1.0 / N) / N)
    assert np.max(np.abs((a - b) / sig)) < 4.0
    xl_f = np.bitwise_xor.reduce(ffin[:, 0:d * d:d], axis=1).mean()
    assert abs(np.mean(xl) - xl_f) < 4.0 * np.sqrt(max(xl_f * (1 - xl_f), 1.0 / N) / N)


def test_virtual_z_restores_carry_no_over_rotation():
    """virtual_z: over-rotation placed only on the Rz restores of the Z checks
    changes nothing -- p1, records and register equal the eps = 0 run."""
    d = 3
    kinds = []
    for t, s in oracle.layout(d):
        w = sum(1 for q in s if q)
        kinds += (["anc"] + ["cr"] * w + ["anc"] + ["restore"] * w) if t == "X" else (["cr"] * w + ["rz"] * w)
    es = np.array([0.07 if k == "rz" else 0.0 for k in kinds])
    a = oracle.run_trajectory(d, CR, 2, seed=4, t=0, p=0.0, eps_site=es, virtual_z=True, want_state=True)
    b = oracle.run_trajectory(d, CR, 2, seed=4, t=0, p=0.0, want_state=True)
    c = oracle.run_trajectory(d, CR, 2, seed=4, t=0, p=0.0, eps_site=es, want_state=True)
    assert np.array_equal(a["p1"], b["p1"]) and np.allclose(a["state"], b["state"], atol=1e-14)
    assert np.max(np.abs(c["p1"] - b["p1"])) > 1e-6   # without the flag they do act


# ---- idle noise on the waiting qubits of each step --------------------------

@pytest.mark.parametrize("gateset", [CR, TB])
def test_dense_brute_force_d2_idle_trajectories(gateset):
    """Idle noise (N1 on the check's data qubits that a step leaves alone, and
    on the ancilla during the Z check's restores) against the dense brute force
    with the same draws, also with twirled over-rotations."""
    d, R = 2, 2
    for t, (p, eps, zeta, tw) in enumerate([(0.1, 0.0, 0.0, False), (0.15, 0.05, 0.03, False),
                                            (0.12, 0.2, 0.02, True)]):
        rec, fb, st = _dense_trajectory(d, gateset, R, 29, t, p, eps, zeta, twirl=tw, idle=True)
        o = oracle.run_trajectory(d, gateset, R, seed=29, t=t, p=p, eps=eps, zeta=zeta,
                                  want_state=True, twirl=tw, idle=True)
        assert np.array_equal(o["records"], rec)
        assert np.array_equal(o["final_bits"], fb)
        assert np.allclose(o["state"], st, atol=1e-12)


@pytest.mark.parametrize("gateset", [CR, TB])
def test_idle_noise_first_check_flip_probability(gateset):
    """First check of round 1 (X1X2, slots 2, 1, wait, wait) on logical |0>,
    Pauli noise only.  Propagating the measured Z of the ancilla back through
    the circuit gives the operator each location must anticommute with to flip
    the outcome: a one-qubit location flips with probability 2p/3, a two-qubit
    one with 8p/15.  Cross-resonance circuit: four one-qubit and two two-qubit
    flipping locations, plus three idle ones (data 1 and 2 waiting during
    Rx^dag, data 1 waiting during the first cross-resonance gate).  Textbook:
    two and two, plus three idle ones (data 1 and 2 after the first H, data 1
    during the first CNOT).  P(flip) = (1 - prod(1 - 2 q)) / 2."""
    p, n = 0.03, 20000
    r0 = trivial_bits(2, gateset)[0]
    k1 = 4 if gateset == CR else 2
    for idle, extra in ((False, 0), (True, 3)):
        flips = sum(int(oracle.run_trajectory(2, gateset, 1, seed=31, t=t, p=p, idle=idle)["records"][0, 0]) ^ int(r0)
                    for t in range(n))
        q = 0.5 * (1.0 - (1 - 4 * p / 3) ** (k1 + extra) * (1 - 16 * p / 15) ** 2)
        assert abs(flips / n - q) < 4 * np.sqrt(q * (1 - q) / n), (idle, flips / n, q)


@pytest.mark.parametrize("gateset", [CR, TB])
def test_idle_noise_pauli_only_matches_frame_sampler(gateset):
    """Idle noise in a Pauli-only d=3 run: detector and logical-Z flip rates
    agree with the Pauli-frame sampler run with the same step schedule."""
    d, R, N, p = 3, 2, 2500, 0.008
    tb = trivial_bits(d, gateset)
    recs, zl = [], []
    for t in range(N):
        r = oracle.run_trajectory(d, gateset, R, seed=37, t=t, p=p, idle=True)
        recs.append(r["records"] ^ tb)
        zl.append(sum(int(r["final_bits"][q]) for q in range(d)) % 2)
    recs = np.array(recs)
    frec, ffin = frame.sample(d, gateset, R, p, 200000, seed=5, idle=True)
    a = _detectors(recs).mean(0)
    b = _detectors(frec).mean(0)
    sig = np.sqrt(np.maximum(b * (1 - b), 1.0 / N) / N)
    assert np.max(np.abs((a - b) / sig)) < 4.0
    zl_f = np.bitwise_xor.reduce(ffin[:, :d], axis=1).mean()
    assert abs(np.mean(zl) - zl_f) < 4.0 * np.sqrt(max(zl_f * (1 - zl_f), 1.0 / N) / N)
    # idle noise raises the detector rates over the run without it
    f0, _ = frame.sample(d, gateset, R, p, 200000, seed=5)
    assert _detectors(frec).mean() > 1.2 * _detectors(f0).mean()



# ---- ancilla-plaquette ZZ crosstalk after every step ------------------------

@pytest.mark.parametrize("gateset", [CR, TB])
def test_dense_brute_force_d2_zz_plaquette_trajectories(gateset):
    """Per-step crosstalk exp(-i zeta Z_anc Z_q) on the running check's data
    qubits (with the once-per-circuit data ZZ layer), also with idle noise and
    twirled over-rotations, against the dense brute force with the same draws."""
    d, R = 2, 2
    for t, (p, eps, zeta, tw, idle) in enumerate([(0.0, 0.0, 0.15, False, False),
                                                  (0.08, 0.05, 0.1, False, False),
                                                  (0.1, 0.2, 0.07, True, True)]):
        rec, fb, st = _dense_trajectory(d, gateset, R, 43, t, p, eps, zeta, twirl=tw, idle=idle, zzp=True)
        o = oracle.run_trajectory(d, gateset, R, seed=43, t=t, p=p, eps=eps, zeta=zeta, want_state=True,
                                  twirl=tw, idle=idle, zz_plaquette=True)
        assert np.array_equal(o["records"], rec)
        assert np.array_equal(o["final_bits"], fb)
        assert np.allclose(o["state"], st, atol=1e-12)


def test_zz_plaquette_acts_on_the_first_check():
    """The crosstalk alone changes the first X check's outcome probability
    (the data ZZ layer does not: it commutes with that measurement); zeta = 0
    leaves every trajectory unchanged."""
    d = 3
    a = oracle.run_trajectory(d, CR, 1, seed=5, t=0, p=0.0, zeta=0.2, zz_plaquette=True)
    b = oracle.run_trajectory(d, CR, 1, seed=5, t=0, p=0.0, zeta=0.2)
    assert abs(a["p1"][0, 0] - b["p1"][0, 0]) > 1e-4
    c = oracle.run_trajectory(d, CR, 2, seed=5, t=1, p=0.02, eps=0.03, zeta=0.0, zz_plaquette=True,
                              want_state=True)
    e = oracle.run_trajectory(d, CR, 2, seed=5, t=1, p=0.02, eps=0.03, zeta=0.0, want_state=True)
    assert np.array_equal(c["records"], e["records"]) and np.allclose(c["state"], e["state"], atol=1e-14)
