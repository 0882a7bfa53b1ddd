"""GPU parity of sv_run_rounds (the trajectory engine) against the CPU oracle.

Same seeded draws on both sides (Philox4x32-10 keyed by the seed, counter =
(draw index, trajectory)): syndrome records and final data bits must agree
bit for bit; p1 and the data register before the final measurement to 1e-10
in complex128.  In complex64 (amplitudes in float32, probabilities and
renormalisation in float64) the register must agree to 1e-5 and records bit
for bit for these seeds.
"""
import os

import numpy as np
import pytest

import oracle
import paper_2204_11404_amd as qs
import workloads

pytestmark = pytest.mark.gpu

GS = {"cr": oracle.GATESET_CR, "textbook": oracle.GATESET_TEXTBOOK}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d5_cr_oracle.npz")


def _compare(d, gateset, R, n_traj, seed, p, eps=0.0, eps_site=None, zeta=0.0, dtype="c128",
             traj0=0, atol=1e-10, twirl=False, xbasis=False, virtual_z=False, idle=False, zzp=False):
    print(f"case rounds d={d} {gateset} R={R} n={n_traj} p={p} eps={eps} zeta={zeta} {dtype}"
          f" twirl={twirl} xbasis={xbasis} vz={virtual_z} idle={idle} zzp={zzp}", flush=True)
    g = qs.run_rounds(d, gateset, R, n_traj, seed, p, eps=eps, eps_site=eps_site, zeta=zeta,
                      dtype=dtype, traj0=traj0, want_p1=True, want_states=True, twirl=twirl,
                      xbasis=xbasis, virtual_z=virtual_z, idle_noise=idle, zz_plaquette=zzp)
    for i in range(n_traj):
        o = oracle.run_trajectory(d, GS[gateset], R, seed, traj0 + i, p, eps=eps, eps_site=eps_site,
                                  zeta=zeta, want_state=True, twirl=twirl, xbasis=xbasis,
                                  virtual_z=virtual_z, idle=idle, zz_plaquette=zzp)
        assert np.array_equal(g["records"][i], o["records"]), f"trajectory {i}"
        assert np.array_equal(g["final_bits"][i], o["final_bits"]), f"trajectory {i}"
        assert np.max(np.abs(g["p1"][i] - o["p1"])) < atol
        assert np.max(np.abs(g["states"][i] - o["state"])) < atol
    return g


@pytest.mark.parametrize("gateset", ["cr", "textbook"])
@pytest.mark.parametrize("d", [2, 3])
def test_small_distance_parity(gateset, d):
    _compare(d, gateset, 3, 40, seed=7, p=0.02, eps=0.03, zeta=0.02)


def test_d3_textbook_workload_parity():
    c = workloads.CONFIGS["d3_textbook_c128"]
    _compare(3, "textbook", c["rounds"], 200, c["seed"], c["p"], eps=c["eps"])


def test_d4_parity_spans_several_tiles():
    # 16 data qubits: 2^16 amplitudes = 16 tiles of 2^12
    n_sites = oracle.template_counts(4, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 3)
    _compare(4, "cr", 2, 4, seed=3, p=0.01, eps_site=eps, zeta=0.01)


def test_noiseless_records_are_trivial():
    g = qs.run_rounds(3, "cr", 4, 8, 0, 0.0)
    r0 = np.array([(sum(1 for q in s if q) // 2) % 2 for _, s in oracle.layout(3)], dtype=np.uint8)
    assert np.array_equal(g["records"], np.broadcast_to(r0, g["records"].shape))


@pytest.mark.parametrize("d", [3, 4])
def test_complex64_parity(d):
    n_sites = oracle.template_counts(d, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 11)
    _compare(d, "cr", 2, 6 if d == 4 else 30, seed=11, p=0.01, eps_site=eps, zeta=0.01,
             dtype="c64", atol=1e-5)


def test_deterministic_and_resumable():
    kw = dict(d=4, gateset="cr", rounds=2, seed=5, p=0.02, eps=0.02, zeta=0.01, want_p1=True)
    a = qs.run_rounds(n_traj=4, traj0=0, **kw)
    b = qs.run_rounds(n_traj=4, traj0=0, **kw)
    c = qs.run_rounds(n_traj=2, traj0=2, **kw)
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["p1"], b["p1"])  # bitwise: fixed reduction order
    assert np.array_equal(a["final_bits"], b["final_bits"])
    assert np.array_equal(a["records"][2:], c["records"])
    assert np.array_equal(a["final_bits"][2:], c["final_bits"])


def test_d5_full_size_against_stored_oracle():
    """26-qubit cross-resonance workload (p=1e-3, theta ~ U[0,0.05) per site,
    zeta=0.01) with the launch parameters in effect (one tile per pass
    workgroup unless tuned): records, p1, final bits and 4096 sampled
    amplitudes against the oracle's stored run.  The benchmark's tuned
    configuration and the whole register are compared with the live oracle in
    test_gpu_d5_live.py."""
    z = np.load(GOLDEN)
    traj = [int(t) for t in z["traj"]]
    R, seed = int(z["rounds"]), int(z["seed"])
    print(f"case d5 golden traj={traj} R={R}", flush=True)
    g = qs.run_rounds(5, "cr", R, len(traj), seed, float(z["p"]), eps_site=z["eps"],
                      zeta=float(z["zeta"]), traj0=traj[0], want_p1=True, want_states=True)
    for i, t in enumerate(traj):
        assert np.array_equal(g["records"][i], z[f"records_{t}"])
        assert np.array_equal(g["final_bits"][i], z[f"final_bits_{t}"])
        assert np.max(np.abs(g["p1"][i] - z[f"p1_{t}"])) < 1e-10
        st = g["states"][i]
        assert np.max(np.abs(st[z["idx"]] - z[f"amps_{t}"])) < 1e-10
        assert np.max(np.abs(st[z[f"top_idx_{t}"]] - z[f"top_amps_{t}"])) < 1e-10
        assert abs(np.linalg.norm(st) - 1.0) < 1e-10


def test_d5_bench_config_properties():
    """The full d=5, 5-round benchmark workload for two trajectories: the
    register stays normalised, runs are bit-reproducible, and since draws are
    enumerated round by round, the first two rounds equal the oracle's stored
    two-round run of the same job."""
    c = workloads.CONFIGS["d5_cr_c128"]
    n_sites = qs.template_info(5, "cr")[1]
    eps = workloads.eps_sites(n_sites, c["theta"], c["seed"])
    kw = dict(d=5, gateset="cr", rounds=c["rounds"], n_traj=2, seed=c["seed"], p=c["p"],
              eps_site=eps, zeta=c["zeta"])
    a = qs.run_rounds(want_states=True, want_p1=True, **kw)
    b = qs.run_rounds(want_p1=True, **kw)
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["p1"], b["p1"])
    for st in a["states"]:
        assert abs(np.linalg.norm(st) - 1.0) < 1e-10
    z = np.load(GOLDEN)
    assert np.array_equal(z["eps"], eps) and int(z["seed"]) == c["seed"]
    for t in (0, 1):
        assert np.array_equal(a["records"][t, :2], z[f"records_{t}"])
        assert np.max(np.abs(a["p1"][t, :2] - z[f"p1_{t}"])) < 1e-10


@pytest.mark.parametrize("chain", [1, 2, 3, 5, 6])
@pytest.mark.parametrize("d", [3, 4])
def test_z_chain_lengths_parity(monkeypatch, d, chain):
    """Passes that apply and decide chains of 1..3, 5 and 6 Z checks
    (QECSV_ZCHAIN; d=4 has seven: chains (5, 2) and (6, 1), the six-chain
    summed amplitude by amplitude as no four tile bits avoid its qubits)
    give the oracle's records, p1 and register, with enough noise that most
    Z checks carry an X-type Pauli (a non-trivial Pauli-X frame)."""
    monkeypatch.setenv("QECSV_ZCHAIN", str(chain))
    n_sites = oracle.template_counts(d, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 21)
    _compare(d, "cr", 2, 3 if d == 4 else 12, seed=21, p=0.04, eps_site=eps, zeta=0.015)


def test_high_noise_frames_d4():
    """p = 0.08: nearly every Z check moves amplitudes (XOR permutations kept
    as a frame); the register handed back and the final bits are in the
    logical frame."""
    _compare(4, "textbook", 2, 3, seed=33, p=0.08, eps=0.02, zeta=0.01)


@pytest.mark.parametrize("d,dtype", [(3, "c128"), (4, "c64"), (5, "c128")])
def test_graph_replay_matches_stream_launches(monkeypatch, d, dtype):
    """SV_RUN_GRAPH (one trajectory's launch sequence captured once, replayed
    per trajectory with a device-side trajectory counter) gives the records,
    p1 and final bits of the stream launches, for every replay; an eager run
    sits between two graph runs.  Graph runs use the plain passes, as do the
    stream launches here (no speculative units)."""
    monkeypatch.setenv("QECSV_SPEC", "0")
    n_sites = oracle.template_counts(d, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 8)
    n = {3: 24, 4: 6, 5: 2}[d]
    kw = dict(d=d, gateset="cr", rounds=2, n_traj=n, seed=8, p=0.01 if d < 5 else 2e-3,
              eps_site=eps, zeta=0.01, dtype=dtype, traj0=3, want_p1=True)
    g1 = qs.run_rounds(graph=True, **kw)
    e = qs.run_rounds(**kw)
    g2 = qs.run_rounds(graph=True, **kw)
    for g in (g1, g2):
        assert np.array_equal(g["records"], e["records"])
        assert np.array_equal(g["final_bits"], e["final_bits"])
        assert np.array_equal(g["p1"], e["p1"])


def test_graph_rejects_final_states():
    with pytest.raises(qs.SvError):
        qs.run_rounds(3, "cr", 1, 1, 0, 0.01, graph=True, want_states=True)


@pytest.mark.parametrize("gateset", ["cr", "textbook"])
@pytest.mark.parametrize("d", [3, 4])
def test_twirled_over_rotation_parity(gateset, d):
    """SV_RUN_TWIRL: every rotation by its base angle plus its generator with
    probability sin^2 eps (one extra draw per rotation)."""
    n_sites = oracle.template_counts(d, GS[gateset])[1]
    eps = workloads.eps_sites(n_sites, (0.1, 0.5), 5)
    _compare(d, gateset, 2, 3 if d == 4 else 12, seed=41, p=0.01, eps_site=eps, zeta=0.01, twirl=True)


@pytest.mark.parametrize("gateset,d,dtype", [("cr", 3, "c128"), ("textbook", 3, "c128"),
                                             ("cr", 4, "c128"), ("cr", 3, "c64")])
def test_x_basis_memory_parity(gateset, d, dtype):
    """SV_RUN_XBASIS: logical |+> written by the first pass, the data measured
    in the X basis after a Walsh-Hadamard transform of the register."""
    n_sites = oracle.template_counts(d, GS[gateset])[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 12)
    _compare(d, gateset, 2, 3 if d == 4 else 12, seed=12, p=0.02, eps_site=eps, zeta=0.01,
             dtype=dtype, atol=1e-10 if dtype == "c128" else 1e-5, xbasis=True)


def test_x_basis_noiseless_reads_trivial_logical():
    g = qs.run_rounds(3, "cr", 3, 8, 0, 0.0, xbasis=True)
    d = 3
    xl = np.bitwise_xor.reduce(g["final_bits"][:, 0:d * d:d], axis=1)
    assert not xl.any()
    assert not qs.decode_x(d, "cr", g["records"], g["final_bits"])["failed"].any()


def test_x_basis_twirled_parity():
    n_sites = oracle.template_counts(3, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.1, 0.4), 13)
    _compare(3, "cr", 2, 10, seed=13, p=0.01, eps_site=eps, twirl=True, xbasis=True)


@pytest.mark.parametrize("twirl", [False, True])
def test_virtual_z_parity(twirl):
    """SV_RUN_VIRTUAL_Z: exact Rz restores after the Z checks."""
    n_sites = oracle.template_counts(3, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.05, 0.3), 14)
    _compare(3, "cr", 2, 10, seed=14, p=0.01, eps_site=eps, zeta=0.01, twirl=twirl, virtual_z=True)


@pytest.mark.parametrize("gateset,d,dtype,twirl,xbasis", [
    ("cr", 3, "c128", False, False), ("textbook", 3, "c128", False, False),
    ("cr", 4, "c128", True, False), ("cr", 3, "c64", False, False), ("cr", 3, "c128", False, True)])
def test_idle_noise_parity(gateset, d, dtype, twirl, xbasis):
    """SV_RUN_IDLE_NOISE: one-qubit noise on the waiting qubits of every step
    (the largest block template: d=4 weight-4 X checks with twirled rotations,
    36 ops).  High p so that idle locations fire in most blocks."""
    n_sites = oracle.template_counts(d, GS[gateset])[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.3 if twirl else 0.05), 15)
    _compare(d, gateset, 2, 3 if d == 4 else 10, seed=15, p=0.03, eps_site=eps, zeta=0.01,
             dtype=dtype, atol=1e-10 if dtype == "c128" else 1e-5, twirl=twirl, xbasis=xbasis,
             idle=True)


def test_idle_noise_d5_noiseless_is_trivial():
    """d=5 (26 qubits) with SV_RUN_IDLE_NOISE and p = 0: every record is its
    trivial bit and the final bits satisfy every Z check and Z_L."""
    d = 5
    g = qs.run_rounds(d, "cr", 2, 1, 3, 0.0, eps=0.0, zeta=0.0, dtype="c64", idle_noise=True)
    tb = np.array([(sum(1 for q in s if q) // 2) % 2 for _, s in oracle.layout(d)], dtype=np.uint8)
    assert np.array_equal(g["records"][0], np.broadcast_to(tb, (2, len(tb))))
    fb = g["final_bits"][0]
    for typ, s in oracle.layout(d):
        if typ == "Z":
            assert sum(int(fb[q - 1]) for q in s if q) % 2 == 0
    assert sum(int(fb[q]) for q in range(d)) % 2 == 0


def test_grid_stride_passes_match(monkeypatch):
    """Register passes with fewer workgroups than tiles (each takes tiles
    grid-stride and sums its tiles before the fixed-order reduction) give the
    same records and final bits, and p1 up to the rounding of the different
    summation order."""
    n_sites = oracle.template_counts(5, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 1)
    kw = dict(d=5, gateset="cr", rounds=1, n_traj=1, seed=3, p=5e-3, eps_site=eps, zeta=0.01,
              dtype="c64", want_p1=True)
    monkeypatch.setenv("QECSV_PASS_WGS_PER_CU", "0")
    a = qs.run_rounds(**kw)
    monkeypatch.setenv("QECSV_PASS_WGS_PER_CU", "1")
    b = qs.run_rounds(**kw)
    assert np.array_equal(a["records"], b["records"])
    assert np.max(np.abs(a["p1"] - b["p1"])) < 1e-12
    assert np.array_equal(a["final_bits"], b["final_bits"])



@pytest.mark.parametrize("gateset,d,dtype,twirl,idle,xbasis", [
    ("cr", 3, "c128", False, False, False), ("textbook", 3, "c128", False, False, False),
    ("cr", 4, "c128", False, True, False), ("cr", 3, "c64", True, False, False),
    ("cr", 3, "c128", False, False, True),
    # d = 4: whole waves of lanes, so the dense products run on the matrix
    # cores (FP64 and FP32 operand layouts)
    ("cr", 4, "c64", False, False, False), ("textbook", 4, "c128", False, False, False),
    ("cr", 4, "c128", True, False, True)])
def test_zz_plaquette_parity(gateset, d, dtype, twirl, idle, xbasis):
    """SV_RUN_ZZ_PLAQUETTE: the ancilla-plaquette crosstalk after every step
    makes the X checks' Kraus pairs dense (k_prepare_dense, dense pass
    kernels); records, p1 and register against the oracle."""
    n_sites = oracle.template_counts(d, GS[gateset])[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.3 if twirl else 0.05), 17)
    _compare(d, gateset, 2, 3 if d == 4 else 8, seed=17, p=0.02, eps_site=eps, zeta=0.08,
             dtype=dtype, atol=1e-10 if dtype == "c128" else 1e-5, twirl=twirl, idle=idle,
             xbasis=xbasis, zzp=True)


def test_zz_plaquette_graph_and_d5():
    """The crosstalk runs under graph replay (same records as the stream) and
    at d=5 (26 qubits)."""
    kw = dict(d=3, gateset="cr", rounds=2, n_traj=6, seed=18, p=0.01, eps=0.02, zeta=0.05,
              dtype="c128", want_p1=True, zz_plaquette=True)
    a = qs.run_rounds(**kw)
    b = qs.run_rounds(graph=True, **kw)
    assert np.array_equal(a["records"], b["records"]) and np.array_equal(a["p1"], b["p1"])
    g = qs.run_rounds(5, "cr", 1, 1, 18, 1e-3, eps=0.01, zeta=0.01, dtype="c64", zz_plaquette=True)
    assert g["records"].shape == (1, 1, 24)


# ---------------------------------------------------- pairs of X checks
# With QECSV_XPAIR=1 a pass sums two consecutive X checks (the second for
# each outcome of the first, after the first's Kraus operator and ZZ layer)
# wherever both units' qubits fit one tile; d=4 then runs 7 passes a round
# (pairs (X0,X1), (X2,X3), (X6,X7)), d=5 12.  Enough noise that frames of the
# pair members and Pauli-X frames occur.
@pytest.mark.parametrize("chain", [1, 2, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_x_pairs_parity_d4(monkeypatch, dtype, chain):
    monkeypatch.setenv("QECSV_SPEC", "0")
    monkeypatch.setenv("QECSV_XPAIR", "1")
    monkeypatch.setenv("QECSV_ZCHAIN", str(chain))
    n_sites = oracle.template_counts(4, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 71)
    g = _compare(4, "cr", 3, 4, seed=71, p=0.03, eps_site=eps, zeta=0.02, dtype=dtype,
                 atol=1e-10 if dtype == "c128" else 1e-5)
    assert g["passes_per_round"] == qs.check_pass_layouts(4, "cr", chain, 1) - 2
    assert g["passes_per_round"] < qs.check_pass_layouts(4, "cr", chain, 0) - 2


@pytest.mark.parametrize("flags", ["textbook", "xbasis", "idle", "twirl", "virtual_z"])
def test_x_pairs_parity_d4_flags(monkeypatch, flags):
    """Pairs under the textbook gate set and the physical-schedule flags (the
    X basis starts from logical |+> in the pass that sums the first pair)."""
    monkeypatch.setenv("QECSV_SPEC", "0")
    monkeypatch.setenv("QECSV_XPAIR", "1")
    gs = "textbook" if flags == "textbook" else "cr"
    _compare(4, gs, 2, 3, seed=73, p=0.02, eps=0.03, zeta=0.01, xbasis=flags == "xbasis",
             idle=flags == "idle", twirl=flags == "twirl", virtual_z=flags == "virtual_z")


def test_x_pairs_graph_replay(monkeypatch):
    monkeypatch.setenv("QECSV_SPEC", "0")
    monkeypatch.setenv("QECSV_XPAIR", "1")
    kw = dict(d=4, gateset="cr", rounds=2, n_traj=3, seed=77, p=0.02, eps=0.02, zeta=0.01, want_p1=True)
    a = qs.run_rounds(**kw)
    b = qs.run_rounds(graph=True, **kw)
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["final_bits"], b["final_bits"])
    assert np.max(np.abs(a["p1"] - b["p1"])) < 1e-12
