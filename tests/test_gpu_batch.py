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


# -------------------------------------------------- the batched launch's real shape
# 16 384 d=3 trajectories: far more than the persistent grid holds at once
# (at most CUs * 32 waves), so every workgroup runs several trajectories one
# after another and reuses its LDS slot, angle tables and cached noise-free
# Kraus pairs.  The oracle runs a spread sample (every 16th trajectory and the
# last 64) once per parameter set; every launch variant is compared with it.
N_REAL = 16384
_ORACLE_CACHE = {}


def _real_shape_sample(n):
    return np.unique(np.concatenate([np.arange(0, n, 16), np.arange(n - 64, n)]))


def _oracle_sample(d, gateset, n, seed, p_range):
    key = (d, gateset, n, seed, p_range)
    if key not in _ORACLE_CACHE:
        n_sites = qs.template_info(d, gateset)[1]
        R, p, eps = workloads.batch_params(n, n_sites, seed, p=p_range)
        idx = _real_shape_sample(n) if d == 3 else np.unique(np.concatenate(
            [np.arange(0, n, n // 48), np.arange(n - 16, n)]))
        print(f"oracle sample d={d} {gateset} n={n}: {idx.size} trajectories", flush=True)
        out = {}
        for i in idx:
            o = oracle.run_trajectory(d, GS[gateset], int(R[i]), seed, int(i), p[i], eps_site=eps[i])
            out[int(i)] = (o["records"], o["final_bits"])
        _ORACLE_CACHE[key] = (R, p, eps, out)
    return _ORACLE_CACHE[key]


def _grid_bound(d, dtype, nw):
    """Most workgroups the persistent launch can have: CUs x the tuned waves
    per CU / waves per trajectory."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    per_cu = max(1, qs.tuning_get(d, dtype)["batch_waves_per_cu"] // nw)
    return cus * per_cu


def _check_sample(d, gateset, dtype, n, seed, p_range):
    R, p, eps, ref = _oracle_sample(d, gateset, n, seed, p_range)
    g = qs.run_batch(d, gateset, R, p, seed, eps_site=eps, dtype=dtype, max_rounds=9)
    for i, (rec, fb) in ref.items():
        assert np.array_equal(g["records"][i, :R[i]], rec), f"trajectory {i}"
        assert not g["records"][i, R[i]:].any(), f"trajectory {i}"
        assert np.array_equal(g["final_bits"][i], fb), f"trajectory {i}"
    return g


@pytest.mark.parametrize("waves_per_cu", [None, "1"])
@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batch_d3_persistent_real_shape(dtype, split, waves_per_cu, monkeypatch):
    """The batched workload's shape (rounds 1..9, p in [5e-4, 5e-3), theta in
    [0, 0.05) per site and trajectory) at 16 384 trajectories per launch, with
    the tuned occupancy and with one resident workgroup per CU (each then runs
    at least 64 trajectories)."""
    monkeypatch.setenv("QECSV_BATCH_SPLIT", split)
    if waves_per_cu:
        monkeypatch.setenv("QECSV_BATCH_WAVES_PER_CU", waves_per_cu)
    print(f"case batch real shape d=3 {dtype} split={split} waves_per_cu={waves_per_cu}", flush=True)
    assert N_REAL > 2 * _grid_bound(3, dtype, int(split))
    _check_sample(3, "cr", dtype, N_REAL, seed=61, p_range=(5e-4, 5e-3))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_d4_lockstep_groups(dtype, monkeypatch):
    """d=4 registers run in lockstep groups of QECSV_LOCKSTEP_MIB; 2 MiB holds
    two complex128 or four complex64 registers, so 24 trajectories take 12 or
    6 consecutive groups (slots, tables and decisions reused from group to
    group)."""
    monkeypatch.setenv("QECSV_LOCKSTEP_MIB", "2")
    per_reg = (2 << 16) * (8 if dtype == "c128" else 4)
    assert 24 // ((2 << 20) // per_reg) >= 3
    print(f"case batch d=4 lockstep groups {dtype}", flush=True)
    _check(4, "cr", dtype, 24, seed=63, p_range=(5e-3, 3e-2), zeta=0.01)


def test_batch_d4_real_shape_sample():
    """4096 d=4 complex64 trajectories in one launch with the tuned lockstep
    groups, a spread sample of 64 (including the last 16) against the
    oracle."""
    print("case batch real shape d=4 c64 n=4096", flush=True)
    _check_sample(4, "cr", "c64", 4096, seed=65, p_range=(5e-4, 5e-3))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_d4_x_pairs(dtype, monkeypatch):
    """Lockstep d=4 passes with pairs of X checks (QECSV_XPAIR=1), over
    several lockstep groups."""
    monkeypatch.setenv("QECSV_XPAIR", "1")
    monkeypatch.setenv("QECSV_LOCKSTEP_MIB", "2")
    print(f"case batch d=4 x pairs {dtype}", flush=True)
    _check(4, "cr", dtype, 12, seed=67, p_range=(5e-3, 3e-2), zeta=0.01)


# ------------------------------------------- speculative lockstep passes
# Without the data ZZ layer (zeta = 0) the lockstep passes are speculative
# (a pair of X checks or a chain of Z checks summed and applied in one pass
# with predicted outcomes, redone per slot when a prediction fails); with
# QECSV_SPEC=1 also at zeta = 0.01 and high noise, where predictions fail
# often.  Several lockstep groups (each slot then holds two registers).
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_d4_speculative_groups(dtype, monkeypatch):
    monkeypatch.delenv("QECSV_SPEC", raising=False)
    monkeypatch.setenv("QECSV_LOCKSTEP_MIB", "2")
    print(f"case batch d=4 speculative groups {dtype}", flush=True)
    _check(4, "cr", dtype, 16, seed=81, p_range=(5e-4, 2e-2))


@pytest.mark.parametrize("gateset", ["cr", "textbook"])
def test_batch_d4_speculative_forced(gateset, monkeypatch):
    monkeypatch.setenv("QECSV_SPEC", "1")
    print(f"case batch d=4 speculative forced {gateset}", flush=True)
    _check(4, gateset, "c128", 12, seed=83, p_range=(1e-2, 5e-2), zeta=0.01)


def test_batch_d4_speculative_matches_plain(monkeypatch):
    """The same launch with speculation on and off: identical records and
    final bits."""
    n_sites = qs.template_info(4, "cr")[1]
    R, p, eps = workloads.batch_params(64, n_sites, 85, p=(5e-4, 5e-3))
    out = []
    for spec in ("1", "0"):
        monkeypatch.setenv("QECSV_SPEC", spec)
        out.append(qs.run_batch(4, "cr", R, p, 85, eps_site=eps, dtype="c64", max_rounds=9))
    assert np.array_equal(out[0]["records"], out[1]["records"])
    assert np.array_equal(out[0]["final_bits"], out[1]["final_bits"])
    assert out[0]["passes_per_round"] < out[1]["passes_per_round"] and out[1]["redo_passes"] == 0
