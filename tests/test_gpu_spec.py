"""Speculative units of sv_run_rounds (registers of 2^12 amplitudes and more).

Each unit (two consecutive X checks, a single X check, or a chain of Z checks)
is summed and applied in one pass with predicted outcomes: the trivial outcome
in the first round, the same check's outcome one round earlier after that.
The decision confirms the members in order and has the pass run again from
the untouched input when a drawn outcome differs (Sec. III.B's sequential
measure-and-reset, one check at a time, is what is computed).  Parity with
the oracle as for the plain passes: records and final bits bit for bit, p1 and
the register to 1e-10 (complex128) or 1e-5 (complex64).  Noise levels from
the benchmark's to p = 0.05 make the predictions fail often, so every redo
path runs; the number of redos is checked against a model of the decision
rule computed from the records.
"""
import numpy as np
import pytest

import oracle
import paper_2204_11404_amd as qs
import workloads

pytestmark = pytest.mark.gpu

GS = {"cr": oracle.GATESET_CR, "textbook": oracle.GATESET_TEXTBOOK}


def _units(d, zchain):
    """Speculative units of a round, every pair of consecutive X checks
    formed (kind, first, len)."""
    lay = oracle.layout(d)
    nx = sum(1 for t, _ in lay if t == "X")
    u = [("XP", i, 2) for i in range(0, nx - 1, 2)]
    if nx % 2:
        u.append(("X", nx - 1, 1))
    i = nx
    while i < len(lay):
        ln = min(zchain, len(lay) - i)
        u.append(("Z", i, ln))
        i += ln
    return u


def _expected_redos(d, gateset, records, zchain):
    """Redos the decision rule calls for: a pair whose first member's
    prediction fails runs again, and once more if the second member's fails
    too; a pair whose first member holds but whose second fails, a single X
    check or a Z chain with any failed prediction, once."""
    lay = oracle.layout(d)
    w = np.array([sum(1 for q in s if q) for _, s in lay])
    triv = ((w // 2) % 2).astype(np.uint8) if gateset == "cr" else np.zeros(len(lay), np.uint8)
    units = _units(d, zchain)
    n = 0
    for rec in records:  # [rounds][n_stab]
        for r in range(rec.shape[0]):
            pred = triv if r == 0 else rec[r - 1]
            for kind, f, ln in units:
                miss = [int(rec[r, f + l] != pred[f + l]) for l in range(ln)]
                if kind == "XP":
                    n += (1 + miss[1]) if miss[0] else miss[1]
                else:
                    n += int(any(miss))
    return n, len(units)


def _run(monkeypatch, d, gateset, R, n_traj, seed, p, zchain=4, dtype="c128", atol=None, **kw):
    monkeypatch.setenv("QECSV_SPEC", "1")
    monkeypatch.setenv("QECSV_ZCHAIN", str(zchain))
    print(f"case spec d={d} {gateset} R={R} n={n_traj} seed={seed} p={p} chain={zchain} {dtype} {kw}",
          flush=True)
    g = qs.run_rounds(d, gateset, R, n_traj, seed, p, dtype=dtype, want_p1=True, want_states=True, **kw)
    okw = {k: v for k, v in kw.items() if k in ("eps", "eps_site", "zeta", "twirl", "xbasis", "virtual_z")}
    if "idle_noise" in kw:
        okw["idle"] = kw["idle_noise"]
    atol = atol or (1e-10 if dtype == "c128" else 1e-5)
    for i in range(n_traj):
        o = oracle.run_trajectory(d, GS[gateset], R, seed, i, p, want_state=True, **okw)
        assert np.array_equal(g["records"][i], o["records"]), f"trajectory {i}"
        assert np.array_equal(g["final_bits"][i], o["final_bits"]), f"trajectory {i}"
        assert np.max(np.abs(g["p1"][i] - o["p1"])) < atol
        assert np.max(np.abs(g["states"][i].astype(np.complex128) - o["state"])) < atol
    n_redo, n_units = _expected_redos(d, gateset, g["records"], zchain)
    print(f"  redos {g['redo_passes']} (model {n_redo}), units per round {g['passes_per_round']}", flush=True)
    assert g["passes_per_round"] == n_units
    assert g["redo_passes"] == n_redo
    return g


@pytest.mark.parametrize("zchain", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_spec_parity_d4(monkeypatch, dtype, zchain):
    n_sites = oracle.template_counts(4, oracle.GATESET_CR)[1]
    eps = workloads.eps_sites(n_sites, (0.0, 0.05), 41)
    g = _run(monkeypatch, 4, "cr", 3, 4, 41, 0.03, zchain=zchain, dtype=dtype, eps_site=eps, zeta=0.02)
    assert g["redo_passes"] > 0


@pytest.mark.parametrize("p", [0.0, 1e-3, 0.05])
def test_spec_noise_levels_d4(monkeypatch, p):
    """p = 0: after the first round every prediction holds (no redo); p =
    0.05: predictions fail often, with Pauli-X frames."""
    g = _run(monkeypatch, 4, "textbook", 4, 3, 43, p, eps=0.02 if p else 0.0, zeta=0.01 if p else 0.0)
    if p == 0.0:
        n_first, _ = _expected_redos(4, "textbook", g["records"][:, :1], 4)
        assert g["redo_passes"] == n_first


@pytest.mark.parametrize("flags", ["xbasis", "idle", "twirl", "virtual_z"])
def test_spec_flags_d4(monkeypatch, flags):
    _run(monkeypatch, 4, "cr", 3, 3, 47, 0.02, eps=0.03, zeta=0.01, xbasis=flags == "xbasis",
         idle_noise=flags == "idle", twirl=flags == "twirl", virtual_z=flags == "virtual_z")


def test_spec_matches_plain_passes(monkeypatch):
    """The same trajectories with speculation off: identical records and
    final bits; p1 and the register agree to rounding."""
    n_sites = oracle.template_counts(4, oracle.GATESET_CR)[1]
    kw = dict(d=4, gateset="cr", rounds=3, n_traj=6, seed=49, p=0.02,
              eps_site=workloads.eps_sites(n_sites, (0.0, 0.05), 49), zeta=0.01, want_p1=True,
              want_states=True)
    monkeypatch.setenv("QECSV_SPEC", "1")
    a = qs.run_rounds(**kw)
    monkeypatch.setenv("QECSV_SPEC", "0")
    b = qs.run_rounds(**kw)
    assert a["passes_per_round"] < b["passes_per_round"] and b["redo_passes"] == 0
    assert np.array_equal(a["records"], b["records"])
    assert np.array_equal(a["final_bits"], b["final_bits"])
    assert np.max(np.abs(a["p1"] - b["p1"])) < 1e-12
    assert np.max(np.abs(a["states"] - b["states"])) < 1e-12


def test_spec_grid_and_traversal_variants(monkeypatch):
    """Pass grids of one tile per workgroup and of 1 workgroup per CU (tiles
    taken grid-stride), with and without alternating traversal: the same
    records and final bits; p1 to rounding."""
    kw = dict(d=4, gateset="cr", rounds=2, n_traj=3, seed=51, p=0.03, eps=0.02, zeta=0.01,
              want_p1=True)
    monkeypatch.setenv("QECSV_SPEC", "1")
    out = []
    for wgs, snake in (("0", "1"), ("1", "0"), ("16", "1")):
        monkeypatch.setenv("QECSV_PASS_WGS_PER_CU", wgs)
        monkeypatch.setenv("QECSV_SNAKE", snake)
        out.append(qs.run_rounds(**kw))
    for g in out[1:]:
        assert np.array_equal(g["records"], out[0]["records"])
        assert np.array_equal(g["final_bits"], out[0]["final_bits"])
        assert np.max(np.abs(g["p1"] - out[0]["p1"])) < 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_spec_graph_replay(monkeypatch, dtype):
    """A trajectory's speculative launch sequence captured once and replayed
    per trajectory (its redos are launched every time, run when needed): the
    stream launches' records, p1 and final bits for every replay, with an
    eager run between two graph runs."""
    monkeypatch.setenv("QECSV_SPEC", "1")
    kw = dict(d=4, gateset="cr", rounds=3, n_traj=5, seed=55, p=0.02, eps=0.02, zeta=0.0, dtype=dtype,
              traj0=2, want_p1=True)
    g1 = qs.run_rounds(graph=True, **kw)
    e = qs.run_rounds(**kw)
    g2 = qs.run_rounds(graph=True, **kw)
    assert e["redo_passes"] > 0 and g1["redo_passes"] == e["redo_passes"]
    for g in (g1, g2):
        assert g["passes_per_round"] == e["passes_per_round"]
        assert np.array_equal(g["records"], e["records"])
        assert np.array_equal(g["final_bits"], e["final_bits"])
        assert np.array_equal(g["p1"], e["p1"])


def test_spec_runs_without_the_zz_layer(monkeypatch):
    """Unless QECSV_SPEC says otherwise, the speculative units run exactly
    when the data ZZ layer is off (zeta = 0), where outcomes repeat from round
    to round; with it the plain passes run."""
    monkeypatch.delenv("QECSV_SPEC", raising=False)
    monkeypatch.setenv("QECSV_ZCHAIN", "4")
    kw = dict(d=4, gateset="cr", rounds=2, n_traj=2, seed=53, p=1e-3, eps=0.02)
    a = qs.run_rounds(zeta=0.0, **kw)
    b = qs.run_rounds(zeta=0.01, **kw)
    assert a["passes_per_round"] == len(_units(4, 4))
    assert b["passes_per_round"] > a["passes_per_round"] and b["redo_passes"] == 0
