"""The library's native decoder (sv_decode_z: exact minimum-weight matching
by dynamic programming over event subsets) against the oracle's networkx
matching on the same detection events.  Matching weights must agree for
every trajectory; failure flags wherever the minimum is unique in its logical
parity (where corrections of both parities reach the minimum, both decoders
are correct and may differ)."""
import numpy as np
import pytest

import oracle
from oracle import decoder, frame
import paper_2204_11404_amd as qs


def _r0(d, gateset):
    return np.array([(sum(1 for q in s if q) // 2) % 2 if gateset == 0 else 0
                     for _, s in oracle.layout(d)], dtype=np.uint8)


@pytest.mark.parametrize("d,p,shots", [(3, 2e-2, 400), (5, 6e-3, 300)])
@pytest.mark.parametrize("gateset", [0, 1])
def test_matches_oracle_decoder(d, p, shots, gateset):
    R = 4
    flips, fin = frame.sample(d, gateset, R, p, shots, seed=11 + d)
    rec = flips ^ _r0(d, gateset)
    out = qs.decode_z(d, "cr" if gateset == 0 else "textbook", rec, fin)
    assert out["overflow"] == 0
    dec = decoder.ZDecoder(d, R, gateset)
    n_amb = 0
    for i in range(shots):
        det = dec.detectors(rec[i], fin[i])
        par, w = dec.matching(det)
        assert out["weight"][i] == w, f"trajectory {i}"
        if out["ambiguous"][i]:
            n_amb += 1
            continue
        assert out["failed"][i] == dec.logical_raw(fin[i]) ^ par, f"trajectory {i}"
    # unit weights leave many ties (e.g. the two boundary qubits of a corner
    # check, one on Z_L and one not); enough trajectories stay unique
    assert shots - n_amb >= shots // 2


@pytest.mark.parametrize("gateset", [0, 1])
def test_x_basis_matches_oracle_decoder(gateset):
    d, R, p, shots = 3, 4, 2e-2, 400
    flips, fin = frame.sample(d, gateset, R, p, shots, seed=21, basis="X")
    rec = flips ^ _r0(d, gateset)
    out = qs.decode_x(d, "cr" if gateset == 0 else "textbook", rec, fin)
    dec = decoder.MemoryDecoder(d, R, gateset, basis="X")
    n_amb = 0
    for i in range(shots):
        par, w = dec.matching(dec.detectors(rec[i], fin[i]))
        assert out["weight"][i] == w, f"trajectory {i}"
        if out["ambiguous"][i]:
            n_amb += 1
            continue
        assert out["failed"][i] == dec.logical_raw(fin[i]) ^ par, f"trajectory {i}"
    assert shots - n_amb >= shots // 2


def test_no_events_reads_the_raw_logical():
    d, R = 3, 2
    rec = np.broadcast_to(_r0(d, 0), (2, R, d * d - 1)).copy()
    fin = np.zeros((2, d * d), dtype=np.uint8)
    fin[1, [0, 3, 6]] = 1          # X_L on the first column: every Z check even, Z_L odd
    out = qs.decode_z(d, "cr", rec, fin)
    assert list(out["weight"]) == [0, 0]
    assert list(out["failed"]) == [0, 1]


def test_too_many_events_are_flagged():
    d, R = 5, 5
    rng = np.random.default_rng(3)
    rec = rng.integers(0, 2, size=(3, R, d * d - 1), dtype=np.uint8)
    fin = rng.integers(0, 2, size=(3, d * d), dtype=np.uint8)
    out = qs.decode_z(d, "cr", rec, fin)
    assert out["overflow"] >= 1
    assert all(f == 2 for f in out["failed"][out["weight"] < 0])


def test_rejects_bad_shapes():
    with pytest.raises(ValueError):
        qs.decode_z(3, "cr", np.zeros((2, 2, 7), np.uint8), np.zeros((2, 9), np.uint8))


def test_power_law_fit_recovers_exact_points():
    from paper_2204_11404_amd.sweep import fit_power_law
    A, xi = 6.5e5, 2.92
    pts = [{"p": p, "p_L": A * p ** xi, "trajectories": 10 ** 6,
            "failures": int(A * p ** xi * 10 ** 6)} for p in (1e-3, 2e-3, 3e-3)]
    f = fit_power_law(pts)
    assert abs(f["xi"] - xi) < 1e-9 and abs(f["A"] / A - 1) < 1e-9
    assert fit_power_law(pts[:1]) is None


@pytest.mark.gpu
def test_decodes_engine_trajectories_like_the_oracle():
    """Records of the GPU engine with coherent over-rotation (c = 1): the
    native decoder agrees with the oracle's matching."""
    d, R, p = 3, 4, 8e-3
    g = qs.run_rounds(d, "cr", R, 300, 5, p, eps=np.sqrt(p), zeta=0.01)
    out = qs.decode_z(d, "cr", g["records"], g["final_bits"])
    dec = decoder.ZDecoder(d, R, 0)
    for i in range(300):
        par, w = dec.matching(dec.detectors(g["records"][i], g["final_bits"][i]))
        assert out["weight"][i] == w
        if not out["ambiguous"][i]:
            assert out["failed"][i] == dec.logical_raw(g["final_bits"][i]) ^ par


@pytest.mark.gpu
def test_sweep_point_runs():
    from paper_2204_11404_amd.sweep import run_point
    q = run_point(3, 5e-3, 0.5, 400, rounds=3, chunk=150)
    assert q["trajectories"] == 400 and q["undecoded"] == 0
    assert 0.0 <= q["p_L"] < 0.2


def test_effective_model_fit_recovers_alpha():
    from paper_2204_11404_amd.sweep import fit_effective_model
    A, xi, alpha = 2e5, 3.0, 0.8
    pts = []
    for c in (0.0, 0.5, 1.0):
        for p in (1.5e-3, 3e-3):
            pl = A * ((1 + alpha * c * c) * p) ** xi
            pts.append({"p": p, "c": c, "p_L": pl, "trajectories": 10 ** 6, "failures": int(pl * 1e6)})
    f = fit_effective_model(pts, A, xi)
    assert abs(f["B"][0.0][0] - 1.0) < 1e-9
    assert abs(f["alpha"] - alpha) < 1e-9
