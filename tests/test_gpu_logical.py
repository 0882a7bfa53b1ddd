"""Logical error probabilities from GPU trajectories agree with independent
oracle and frame-sampler estimates within 3 sigma (binomial)."""
import numpy as np
import pytest

import oracle
import paper_2204_11404_amd as qs
from oracle import decoder, frame

pytestmark = pytest.mark.gpu


def _sigma(p, n):
    return np.sqrt(max(p * (1 - p), 1.0 / n) / n)


def test_logical_rate_gpu_vs_oracle_independent_seeds():
    d, R, p, eps = 3, 3, 0.01, 0.02
    ng, no = 20000, 1500
    rg = np.full(ng, R, dtype=np.int32)
    g = qs.run_batch(d, "cr", rg, np.full(ng, p), seed=101, eps=eps, dtype="c128")
    pl_g, _ = decoder.logical_error_rate(d, 0, g["records"], g["final_bits"])
    recs, fins = [], []
    for t in range(no):
        o = oracle.run_trajectory(d, 0, R, 202, t, p, eps=eps)
        recs.append(o["records"])
        fins.append(o["final_bits"])
    pl_o, _ = decoder.logical_error_rate(d, 0, np.array(recs), np.array(fins))
    assert abs(pl_g - pl_o) < 3 * np.hypot(_sigma(pl_g, ng), _sigma(pl_o, no))


def test_logical_rate_pauli_only_vs_frame_sampler():
    d, R, p = 3, 3, 0.01
    ng = 20000
    g = qs.run_batch(d, "cr", np.full(ng, R, dtype=np.int32), np.full(ng, p), seed=7, dtype="c64")
    pl_g, _ = decoder.logical_error_rate(d, 0, g["records"], g["final_bits"])
    rec, fin = frame.sample(d, 0, R, p, 40000, seed=9)
    r0 = np.array([(sum(1 for q in s if q) // 2) % 2 for _, s in oracle.layout(d)], dtype=np.uint8)
    pl_f, _ = decoder.logical_error_rate(d, 0, rec ^ r0, fin)
    assert abs(pl_g - pl_f) < 3 * np.hypot(_sigma(pl_g, ng), _sigma(pl_f, 40000))
