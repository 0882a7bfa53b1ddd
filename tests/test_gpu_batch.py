"""GPU parity of the batched small-distance launch (sv_run_batch) against the
CPU oracle, trajectory by trajectory: each trajectory has its own round count,
depolarizing probability and per-site over-rotation angles (the batched
workload's shape: rounds uniform in 1..9, p and theta drawn per trajectory).
Records and final bits must agree bit for bit."""
import numpy as np
import pytest

import oracle
import paper_2204_11404_amd as qs
import workloads

pytestmark = pytest.mark.gpu

GS = {"cr": oracle.GATESET_CR, "textbook": oracle.GATESET_TEXTBOOK}


def _check(d, gateset, dtype, n_traj, seed, p_range, zeta=0.0, traj0=0):
    n_stab, n_sites, _ = qs.template_info(d, gateset)
    R, p, eps = workloads.batch_params(n_traj, n_sites, seed, p=p_range)
    print(f"case batch d={d} {gateset} {dtype} n={n_traj} p={p_range} zeta={zeta}", flush=True)
    g = qs.run_batch(d, gateset, R, p, seed, eps_site=eps, zeta=zeta, dtype=dtype, traj0=traj0,
                     max_rounds=9)
    for i in range(n_traj):
        o = oracle.run_trajectory(d, GS[gateset], int(R[i]), seed, traj0 + i, p[i], zeta=zeta,
                                  eps_site=eps[i])
        assert np.array_equal(g["records"][i, :R[i]], o["records"]), f"trajectory {i}"
        assert not g["records"][i, R[i]:].any()
        assert np.array_equal(g["final_bits"][i], o["final_bits"]), f"trajectory {i}"
    return g


# waves per trajectory of the LDS-resident kernel (1: eight amplitudes per
# lane, one check qubit on a lane bit; 2 and 4: four and two amplitudes per
# lane, two and three check qubits on lane bits); the default picks by size
SPLITS = ["1", "2", "4"]


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("gateset", ["cr", "textbook"])
def test_batch_d3_parity(gateset, dtype, split, monkeypatch):
    monkeypatch.setenv("QECSV_BATCH_SPLIT", split)
    print(f"waves per trajectory {split}", flush=True)
    _check(3, gateset, dtype, 400, seed=31, p_range=(5e-3, 5e-2), zeta=0.01)


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("gateset", ["cr", "textbook"])
def test_batch_d2_parity(gateset, split, monkeypatch):
    monkeypatch.setenv("QECSV_BATCH_SPLIT", split)
    print(f"waves per trajectory {split}", flush=True)
    _check(2, gateset, "c128", 200, seed=5, p_range=(1e-2, 1e-1), zeta=0.02)


def test_batch_matches_run_rounds():
    d, n = 3, 64
    n_stab, n_sites, _ = qs.template_info(d, "cr")
    eps = workloads.eps_sites(n_sites, (0, 0.05), 4)
    R = np.full(n, 4, dtype=np.int32)
    p = np.full(n, 0.01)
    a = qs.run_batch(d, "cr", R, p, 4, eps_site=np.tile(eps, (n, 1)), traj0=100, dtype="c128")
    b = qs.run_rounds(d, "cr", 4, n, 4, 0.01, eps_site=eps, traj0=100)
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["final_bits"], b["final_bits"])


def test_batch_workload_shape_small_p():
    """The batched benchmark's parameters (p in [5e-4, 5e-3), theta in [0, 0.05),
    complex64) on a sample of trajectories."""
    _check(3, "cr", "c64", 300, seed=2, p_range=(5e-4, 5e-3))


def test_batch_rejects_bad_arguments():
    with pytest.raises(qs.SvError):
        qs.run_batch(3, "cr", [0], [0.01], 0)            # rounds < 1
    with pytest.raises(qs.SvError):
        qs.run_batch(3, "cr", [2], [1.5], 0)             # p > 1
    with pytest.raises(qs.SvError):
        qs.run_batch(3, "cr", [5], [0.01], 0, max_rounds=4)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("gateset", ["cr", "textbook"])
def test_batch_d4_parity(gateset, dtype):
    """d=4 (16 data qubits, 2^16 amplitudes per trajectory, streamed from HBM
    by one workgroup per trajectory), several tiles per pass."""
    _check(4, gateset, dtype, 24 if dtype == "c128" else 12, seed=17, p_range=(5e-3, 3e-2),
           zeta=0.01)


def test_batch_d4_chain_of_two(monkeypatch):
    """Lockstep d=4 batches with Z chains of at most two checks per pass."""
    monkeypatch.setenv("QECSV_ZCHAIN", "2")
    _check(4, "cr", "c128", 8, seed=19, p_range=(1e-2, 4e-2), zeta=0.01)


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("gateset,d,dtype", [("textbook", 3, "c128"), ("cr", 3, "c64"), ("cr", 2, "c128")])
def test_batch_common_angles_parity(gateset, d, dtype, split, monkeypatch):
    """One over-rotation angle for every site and trajectory: the angle table
    and noise-free Kraus pairs are computed once for the launch (and copied
    per trajectory); per-trajectory rounds and p still vary."""
    monkeypatch.setenv("QECSV_BATCH_SPLIT", split)
    n = 300
    rng = np.random.default_rng(44)
    R = rng.integers(1, 6, n).astype(np.int32)
    p = rng.uniform(5e-3, 4e-2, n)
    eps, zeta, seed = 0.03, 0.01, 44
    print(f"case batch common angles d={d} {gateset} {dtype} waves per trajectory {split}", flush=True)
    g = qs.run_batch(d, gateset, R, p, seed, eps=eps, zeta=zeta, dtype=dtype, max_rounds=5)
    for i in range(n):
        o = oracle.run_trajectory(d, GS[gateset], int(R[i]), seed, i, p[i], eps=eps, zeta=zeta)
        assert np.array_equal(g["records"][i, :R[i]], o["records"]), f"trajectory {i}"
        assert np.array_equal(g["final_bits"][i], o["final_bits"]), f"trajectory {i}"
