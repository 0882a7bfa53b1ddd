"""Write the d=5 oracle fixtures used by the full-size GPU parity tests.

Calls only the CPU oracle (oracle/).  Workload: the 26-qubit cross-resonance
circuit with p = 1e-3, per-site over-rotation theta ~ U[0, 0.05) (eps =
theta/2, drawn by workloads.eps_sites with the job seed) and ZZ crosstalk
zeta = 0.01; seed 1, trajectories 0 and 1, two rounds.  Stored: records,
p1 trace, final bits, and the data register before the final measurement at
4096 sampled indices (plus its norm).

Usage: python tests/golden/make_d5_golden.py   (about 3 minutes on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

D, ROUNDS, SEED, P, ZETA = 5, 2, 1, 1e-3, 0.01
TRAJ = (0, 1)
OUT = os.path.join(HERE, "d5_cr_oracle.npz")


def main():
    n_sites = oracle.template_counts(D, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), SEED)
    rng = np.random.default_rng(12345)
    idx = np.unique(rng.integers(0, 1 << (D * D), size=4096))
    out = dict(eps=eps, idx=idx, traj=np.array(TRAJ), rounds=ROUNDS, seed=SEED, p=P, zeta=ZETA)
    for t in TRAJ:
        r = oracle.run_trajectory(D, oracle.GATESET_CR, ROUNDS, SEED, t, P, zeta=ZETA, eps_site=eps,
                                  want_state=True)
        out[f"records_{t}"] = r["records"]
        out[f"p1_{t}"] = r["p1"]
        out[f"final_bits_{t}"] = r["final_bits"]
        out[f"amps_{t}"] = r["state"][idx]
        out[f"norm_{t}"] = np.linalg.norm(r["state"])
        # the largest amplitudes, where relative errors are easiest to see
        top = np.argsort(-np.abs(r["state"]))[:256]
        out[f"top_idx_{t}"] = top
        out[f"top_amps_{t}"] = r["state"][top]
        print("trajectory", t, "records", r["records"].tolist(), flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
