"""Pins of the decoder used for logical error rates (Sec. III.B procedure)."""
import numpy as np
import pytest

import oracle
from oracle import decoder, frame


def _r0(d):
    return np.array([(sum(1 for q in s if q) // 2) % 2 for _, s in oracle.layout(d)], dtype=np.uint8)


@pytest.mark.parametrize("d", [3, 5])
def test_no_events_no_failure(d):
    dec = decoder.ZDecoder(d, 3, oracle.GATESET_CR)
    rec = np.tile(_r0(d), (3, 1))
    assert dec.failed(rec, np.zeros(d * d, dtype=np.uint8)) == 0


@pytest.mark.parametrize("d", [3, 5])
def test_every_single_final_flip_is_corrected(d):
    """A single X error before the final measurement flips one data bit; the
    matching must undo it whether or not the bit is on the logical support."""
    dec = decoder.ZDecoder(d, 2, oracle.GATESET_CR)
    rec = np.tile(_r0(d), (2, 1))
    for q in range(d * d):
        fb = np.zeros(d * d, dtype=np.uint8)
        fb[q] = 1
        assert dec.failed(rec, fb) == 0, q


def test_single_measurement_error_is_corrected():
    d = 5
    dec = decoder.ZDecoder(d, 4, oracle.GATESET_CR)
    zidx = [i for i, (t, _) in enumerate(oracle.layout(d)) if t == "Z"]
    for k in zidx:
        for r in range(4):
            rec = np.tile(_r0(d), (4, 1))
            rec[r, k] ^= 1
            assert dec.failed(rec, np.zeros(d * d, dtype=np.uint8)) == 0


def test_logical_operator_is_detected_as_failure():
    d = 3
    dec = decoder.ZDecoder(d, 1, oracle.GATESET_CR)
    rec = np.tile(_r0(d), (1, 1))
    fb = np.zeros(d * d, dtype=np.uint8)
    fb[[0, 3, 6]] = 1  # X on the left column: a logical X flips Z_L, no detection event
    assert dec.failed(rec, fb) == 1


def test_distance_helps_below_threshold():
    """Frame-sampled Pauli-only runs: the decoded rate is below the raw
    logical flip rate, and d=5 beats d=3 at p = 1e-3 (same rounds)."""
    rates = {}
    for d in (3, 5):
        rec, fin = frame.sample(d, 0, 3, 1e-3, 30000, seed=4)
        dec = decoder.ZDecoder(d, 3, 0)
        fails = sum(dec.failed(rec[i] ^ _r0(d), fin[i]) for i in range(rec.shape[0]))
        raw = np.mean(np.bitwise_xor.reduce(fin[:, :d], axis=1))
        rates[d] = fails / rec.shape[0]
        assert rates[d] < raw / 5
    assert rates[5] < rates[3]


@pytest.mark.parametrize("gateset", [oracle.GATESET_CR, oracle.GATESET_TEXTBOOK])
def test_error_between_two_checks_of_a_round_is_one_fault(gateset):
    """Checks of a round are measured one after another: an X error on a data
    qubit shared by Z checks a (measured first) and b, striking between their
    measurements of round 0, shows in b from round 0 and in a from round 1 --
    one fault, matched at weight 1 and corrected."""
    d, R = 3, 3
    dec = decoder.ZDecoder(d, R, gateset)
    owners = {}
    for k, sup in enumerate(dec.zsup):
        for q in sup:
            owners.setdefault(q, []).append(k)
    for q, ks in owners.items():
        if len(ks) != 2:
            continue
        a, b = ks
        rec = np.zeros((R, d * d - 1), dtype=np.uint8)
        rec[:, dec.zidx] = dec.r0
        rec[0:, dec.zidx[b]] ^= 1
        rec[1:, dec.zidx[a]] ^= 1
        fin = np.zeros(d * d, dtype=np.uint8)
        fin[q - 1] = 1
        det = dec.detectors(rec, fin)
        assert sorted(zip(*np.nonzero(det))) == sorted([(b, 0), (a, 1)])
        assert dec.matching(det)[1] == 1
        assert dec.failed(rec, fin) == 0
