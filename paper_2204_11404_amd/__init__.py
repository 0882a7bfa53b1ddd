"""Python binding of libqecsv (include/qecsv.h): argument marshalling only.

Every step of the simulation runs in the HIP kernels of the shared library;
this module converts numpy / torch arguments to the C ABI and back.  It never
falls back to a CPU path: if the library is missing, every call raises.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqecsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_ENUMERIC, SV_EBUSY = 0, -1, -2, -3, -4, -5
SV_C64, SV_C128 = 0, 1
SV_GATESET_CR, SV_GATESET_TEXTBOOK = 0, 1
TAU = 1e-10

_DTYPES = {"c64": SV_C64, "c128": SV_C128, SV_C64: SV_C64, SV_C128: SV_C128}
_NP = {SV_C64: np.complex64, SV_C128: np.complex128}
_GATESETS = {"cr": SV_GATESET_CR, "textbook": SV_GATESET_TEXTBOOK,
             SV_GATESET_CR: SV_GATESET_CR, SV_GATESET_TEXTBOOK: SV_GATESET_TEXTBOOK}


class SvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qecsv error {status}: {msg}")
        self.status = status


class Job(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int), ("gateset", ctypes.c_int), ("rounds", ctypes.c_int),
        ("dtype", ctypes.c_int), ("n_traj", ctypes.c_int), ("flags", ctypes.c_int),
        ("traj0", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("p", ctypes.c_double),
        ("eps", ctypes.c_double), ("eps_site", ctypes.POINTER(ctypes.c_double)),
        ("zeta", ctypes.c_double), ("hip_stream", ctypes.c_void_p),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("records", ctypes.POINTER(ctypes.c_uint8)), ("final_bits", ctypes.POINTER(ctypes.c_uint8)),
        ("p1_trace", ctypes.POINTER(ctypes.c_double)), ("final_states", ctypes.c_void_p),
        ("gpu_ms", ctypes.c_double), ("pass_ms", ctypes.c_double),
        ("passes_per_round", ctypes.c_int), ("redo_passes", ctypes.c_int),
    ]


class BatchJob(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int), ("gateset", ctypes.c_int), ("dtype", ctypes.c_int),
        ("n_traj", ctypes.c_int), ("max_rounds", ctypes.c_int), ("flags", ctypes.c_int),
        ("traj0", ctypes.c_uint64), ("seed", ctypes.c_uint64),
        ("rounds", ctypes.POINTER(ctypes.c_int)), ("p", ctypes.POINTER(ctypes.c_double)),
        ("eps_site", ctypes.POINTER(ctypes.c_double)), ("eps", ctypes.c_double),
        ("zeta", ctypes.c_double), ("hip_stream", ctypes.c_void_p),
    ]


class BatchResult(ctypes.Structure):
    _fields_ = [
        ("records", ctypes.POINTER(ctypes.c_uint8)), ("final_bits", ctypes.POINTER(ctypes.c_uint8)),
        ("gpu_ms", ctypes.c_double), ("passes_per_round", ctypes.c_int), ("redo_passes", ctypes.c_int),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("zchain", ctypes.c_int), ("snake", ctypes.c_int),
                ("batch_waves_per_cu", ctypes.c_int), ("lockstep_mib", ctypes.c_int),
                ("pass_wgs_per_cu", ctypes.c_int), ("xpair", ctypes.c_int)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("big_streams", ctypes.c_int),
                ("max_batch_traj", ctypes.c_int), ("flags", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("job", Job), ("records", ctypes.POINTER(ctypes.c_uint8)),
                ("final_bits", ctypes.POINTER(ctypes.c_uint8)), ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("pad", ctypes.c_int),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("hbm_in_use", ctypes.c_size_t), ("hbm_high_water", ctypes.c_size_t),
                ("pending", ctypes.c_int), ("running", ctypes.c_int), ("completed", ctypes.c_int),
                ("launches", ctypes.c_int)]


# name -> (restype, argtypes)
_SIGS = {
    "sv_last_error": (ctypes.c_char_p, []),
    "sv_version": (ctypes.c_int, []),
    "sv_alloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sv_wrap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                               ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sv_free": (ctypes.c_int, [ctypes.c_void_p]),
    "sv_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sv_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sv_set_basis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "sv_copy_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sv_load_logical0": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sv_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "sv_apply_gate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double)]),
    "sv_apply_diag": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double)]),
    "sv_apply_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_double)]),
    "sv_measure_reset_ancilla": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    "sv_measure_reset_ancilla_forced": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                       ctypes.POINTER(ctypes.c_double)]),
    "sv_check_pass_layouts": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int)]),
    "sv_check_spec_layouts": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int)]),
    "sv_template_info": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "sv_run_rounds": (ctypes.c_int, [ctypes.POINTER(Job), ctypes.POINTER(Result)]),
    "sv_run_rounds_async": (ctypes.c_int, [ctypes.POINTER(Job), ctypes.POINTER(Result), ctypes.c_void_p]),
    "sv_run_batch": (ctypes.c_int, [ctypes.POINTER(BatchJob), ctypes.POINTER(BatchResult)]),
    "sv_run_batch_noalloc": (ctypes.c_int, [ctypes.POINTER(BatchJob), ctypes.POINTER(BatchResult)]),
    "sv_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "sv_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request)]),
    "sv_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Completion), ctypes.c_int]),
    "sv_server_wait_idle": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "sv_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "sv_server_clock": (ctypes.c_double, [ctypes.c_void_p]),
    "sv_server_destroy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sv_decode_z": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "sv_decode_x": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "sv_tuning_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "sv_tuning_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "sv_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_double)]),
    "sv_tuning_save": (ctypes.c_int, [ctypes.c_char_p]),
    "sv_tuning_load": (ctypes.c_int, [ctypes.c_char_p]),
    "sv_uniform": (ctypes.c_double, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]),
    "sv_block_kraus": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]),
}

_lib = None


def lib():
    """Load libqecsv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP extension missing: {LIB_PATH} (run __graft_entry__.build())")
        # torch ships its own HIP runtime under the same soname as the system
        # one; load it first so the library binds to the runtime that owns
        # torch's device memory and streams (one runtime per process).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status):
    if status != SV_OK:
        raise SvError(status, lib().sv_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def template_info(d, gateset):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().sv_template_info(d, _GATESETS[gateset], ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def check_pass_layouts(d, gateset, zchain=4, xpair=0):
    """sv_check_pass_layouts: host-side consistency of the register-pass
    layouts; returns the pass count of one round sequence."""
    n = ctypes.c_int()
    _check(lib().sv_check_pass_layouts(d, _GATESETS[gateset], int(zchain), int(xpair), ctypes.byref(n)))
    return n.value


def check_spec_layouts(d, gateset, zchain=4):
    """sv_check_spec_layouts: host-side consistency of the speculative
    passes' layouts; returns the units per round (0: the plain passes run)."""
    n = ctypes.c_int()
    _check(lib().sv_check_spec_layouts(d, _GATESETS[gateset], int(zchain), ctypes.byref(n)))
    return n.value


def uniform(seed, t, k):
    return lib().sv_uniform(int(seed), int(t), int(k))


def block_kraus(d, gateset, stab, rnd, seed, t, p, eps=0.0, eps_site=None):
    """sv_block_kraus: returns dict(D=complex[2, 2^w], F, u, type ('X'/'Z'), qubits)."""
    D = np.zeros(64, dtype=np.float64)
    F, u, typ, w = ctypes.c_uint32(), ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
    q = np.zeros(4, dtype=np.int32)
    es = None
    if eps_site is not None:
        es = np.ascontiguousarray(eps_site, dtype=np.float64)
    _check(lib().sv_block_kraus(d, _GATESETS[gateset], stab, rnd, int(seed), int(t), float(p),
                                float(eps), _dptr(es) if es is not None else None, _dptr(D),
                                ctypes.byref(F), ctypes.byref(u), ctypes.byref(typ), ctypes.byref(w),
                                _iptr(q)))
    n = 1 << w.value
    Dc = D.view(np.complex128).reshape(2, 16)[:, :n].copy()
    return dict(D=Dc, F=F.value, u=u.value, type="X" if typ.value == 0 else "Z",
                qubits=[int(x) for x in q[: w.value]])


class State:
    """A register on the GPU (sv_alloc / sv_wrap)."""

    def __init__(self, n_qubits, dtype="c128", stream=None, tensor=None):
        self.n = n_qubits
        self.dtype = _DTYPES[dtype]
        self._tensor = tensor
        h = ctypes.c_void_p()
        if tensor is None:
            _check(lib().sv_alloc(n_qubits, self.dtype, _stream_ptr(stream), ctypes.byref(h)))
        else:
            nbytes = tensor.numel() * tensor.element_size()
            _check(lib().sv_wrap(ctypes.c_void_p(tensor.data_ptr()), nbytes, n_qubits, self.dtype,
                                 _stream_ptr(stream), ctypes.byref(h)))
        self.h = h

    @property
    def nbytes(self):
        return (16 if self.dtype == SV_C128 else 8) << self.n

    def free(self):
        if self.h:
            _check(lib().sv_free(self.h))
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set(self, host):
        a = np.ascontiguousarray(host, dtype=_NP[self.dtype])
        _check(lib().sv_set_state(self.h, a.ctypes.data, a.nbytes))

    def get(self):
        a = np.empty(1 << self.n, dtype=_NP[self.dtype])
        _check(lib().sv_get_state(self.h, a.ctypes.data, a.nbytes))
        return a

    def copy_from(self, other):
        _check(lib().sv_copy_state(self.h, other.h))

    def set_basis(self, index):
        _check(lib().sv_set_basis(self.h, int(index)))

    def load_logical0(self, d):
        _check(lib().sv_load_logical0(self.h, d))

    def synchronize(self):
        _check(lib().sv_synchronize(self.h))

    def _mat(self, qubits, m):
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        mm = np.ascontiguousarray(m, dtype=np.complex128).view(np.float64)
        return q, mm

    def apply_gate(self, qubits, m):
        q, mm = self._mat(qubits, m)
        _check(lib().sv_apply_gate(self.h, len(q), _iptr(q), _dptr(mm)))

    def apply_diag(self, qubits, phases):
        q, mm = self._mat(qubits, phases)
        _check(lib().sv_apply_diag(self.h, len(q), _iptr(q), _dptr(mm)))

    def apply_fused(self, qubits, m):
        q, mm = self._mat(qubits, m)
        _check(lib().sv_apply_fused(self.h, len(q), _iptr(q), _dptr(mm)))

    def measure_reset(self, anc, u):
        m, p1 = ctypes.c_int(), ctypes.c_double()
        _check(lib().sv_measure_reset_ancilla(self.h, anc, float(u), ctypes.byref(m), ctypes.byref(p1)))
        return m.value, p1.value

    def measure_reset_forced(self, anc, outcome):
        p1 = ctypes.c_double()
        _check(lib().sv_measure_reset_ancilla_forced(self.h, anc, int(outcome), ctypes.byref(p1)))
        return p1.value


SV_RUN_GRAPH = 1
SV_RUN_TWIRL = 2
SV_RUN_XBASIS = 4
SV_RUN_VIRTUAL_Z = 8
SV_RUN_IDLE_NOISE = 16
SV_RUN_ZZ_PLAQUETTE = 32


def _rounds_job(d, gateset, rounds, n_traj, seed, p, eps, eps_site, zeta, dtype, traj0, stream, graph,
                twirl, xbasis, virtual_z, idle_noise, zz_plaquette):
    n_stab, n_sites, _ = template_info(d, gateset)
    job = Job()
    job.d, job.gateset, job.rounds = d, _GATESETS[gateset], rounds
    job.dtype, job.n_traj = _DTYPES[dtype], n_traj
    job.flags = ((SV_RUN_GRAPH if graph else 0) | (SV_RUN_TWIRL if twirl else 0)
                 | (SV_RUN_XBASIS if xbasis else 0) | (SV_RUN_VIRTUAL_Z if virtual_z else 0)
                 | (SV_RUN_IDLE_NOISE if idle_noise else 0)
                 | (SV_RUN_ZZ_PLAQUETTE if zz_plaquette else 0))
    job.traj0, job.seed, job.p, job.eps, job.zeta = int(traj0), int(seed), float(p), float(eps), float(zeta)
    job.hip_stream = _stream_ptr(stream)
    keep = None
    if eps_site is not None:
        keep = np.ascontiguousarray(eps_site, dtype=np.float64)
        if keep.shape != (n_sites,):
            raise ValueError(f"eps_site must have {n_sites} entries")
        job.eps_site = _dptr(keep)
    return job, keep, n_stab


def run_rounds(d, gateset, rounds, n_traj, seed, p, eps=0.0, eps_site=None, zeta=0.0,
               dtype="c128", traj0=0, want_p1=False, want_states=False, stream=None, graph=False,
               twirl=False, xbasis=False, virtual_z=False, idle_noise=False, zz_plaquette=False):
    """sv_run_rounds: returns dict(records[n_traj, rounds, n_stab], final_bits[n_traj, d*d],
    p1 or None, states or None, gpu_ms, pass_ms, passes_per_round).  Flags:
    graph (HIP graph replay), twirl (Pauli-twirled over-rotations), xbasis
    (X-basis memory), virtual_z (exact Rz restores), idle_noise (one-qubit
    noise on the waiting qubits of every step), zz_plaquette (crosstalk
    exp(-i zeta Z_anc Z_q) with the check's data qubits after every step)."""
    job, keep, n_stab = _rounds_job(d, gateset, rounds, n_traj, seed, p, eps, eps_site, zeta, dtype, traj0,
                                    stream, graph, twirl, xbasis, virtual_z, idle_noise, zz_plaquette)
    rec = np.zeros((n_traj, rounds, n_stab), dtype=np.uint8)
    fb = np.zeros((n_traj, d * d), dtype=np.uint8)
    p1 = np.zeros((n_traj, rounds, n_stab), dtype=np.float64) if want_p1 else None
    states = np.zeros((n_traj, 1 << (d * d)), dtype=_NP[job.dtype]) if want_states else None
    res = Result()
    res.records = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    res.final_bits = fb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    if p1 is not None:
        res.p1_trace = _dptr(p1)
    if states is not None:
        res.final_states = states.ctypes.data
    _check(lib().sv_run_rounds(ctypes.byref(job), ctypes.byref(res)))
    del keep
    return dict(records=rec, final_bits=fb, p1=p1, states=states, gpu_ms=res.gpu_ms, pass_ms=res.pass_ms,
                passes_per_round=res.passes_per_round, redo_passes=res.redo_passes)


class AsyncRun:
    """An sv_run_rounds_async call in flight: its pinned host outputs and the
    event recorded after their copies.  wait() returns the run_rounds dict."""

    def __init__(self, event, out, res, n_passes):
        self.event, self._out, self._res, self._n_passes = event, out, res, n_passes

    def done(self):
        return self.event.query()

    def wait(self):
        self.event.synchronize()
        o = self._out
        return dict(records=o["records"].numpy(), final_bits=o["final_bits"].numpy(),
                    p1=o["p1"].numpy() if o["p1"] is not None else None, states=None,
                    gpu_ms=None, pass_ms=None, passes_per_round=self._n_passes)


def run_rounds_async(d, gateset, rounds, n_traj, seed, p, stream, eps=0.0, eps_site=None, zeta=0.0,
                     dtype="c128", traj0=0, want_p1=False, twirl=False, xbasis=False, virtual_z=False,
                     idle_noise=False, zz_plaquette=False):
    """sv_run_rounds_async on `stream` (a torch.cuda.Stream): the outputs go
    to pinned host tensors; returns an AsyncRun at once."""
    import torch
    job, keep, n_stab = _rounds_job(d, gateset, rounds, n_traj, seed, p, eps, eps_site, zeta, dtype, traj0,
                                    stream, False, twirl, xbasis, virtual_z, idle_noise, zz_plaquette)
    out = dict(records=torch.zeros((n_traj, rounds, n_stab), dtype=torch.uint8, pin_memory=True),
               final_bits=torch.zeros((n_traj, d * d), dtype=torch.uint8, pin_memory=True),
               p1=torch.zeros((n_traj, rounds, n_stab), dtype=torch.float64, pin_memory=True)
               if want_p1 else None)
    res = Result()
    res.records = ctypes.cast(out["records"].data_ptr(), ctypes.POINTER(ctypes.c_uint8))
    res.final_bits = ctypes.cast(out["final_bits"].data_ptr(), ctypes.POINTER(ctypes.c_uint8))
    if out["p1"] is not None:
        res.p1_trace = ctypes.cast(out["p1"].data_ptr(), ctypes.POINTER(ctypes.c_double))
    # torch creates the HIP event when it is first recorded; the library then
    # records it again after the run's work
    event = torch.cuda.Event()
    event.record(stream)
    _check(lib().sv_run_rounds_async(ctypes.byref(job), ctypes.byref(res), ctypes.c_void_p(event.cuda_event)))
    del keep
    return AsyncRun(event, out, res, res.passes_per_round)


def run_batch(d, gateset, rounds, p, seed, eps=0.0, eps_site=None, zeta=0.0, dtype="c64", traj0=0,
              max_rounds=None, stream=None, no_alloc=False):
    """sv_run_batch (no_alloc: sv_run_batch_noalloc, d <= 3): rounds and p
    are per-trajectory arrays; eps_site is None or [n_traj, n_sites].  Returns
    dict(records[n_traj, max_rounds, n_stab], final_bits[n_traj, d*d], gpu_ms)."""
    rounds = np.ascontiguousarray(rounds, dtype=np.int32)
    p = np.ascontiguousarray(p, dtype=np.float64)
    n_traj = int(rounds.size)
    if p.shape != (n_traj,):
        raise ValueError("p must have one entry per trajectory")
    n_stab, n_sites, _ = template_info(d, gateset)
    mr = int(max_rounds if max_rounds is not None else (rounds.max() if n_traj else 1))
    job = BatchJob()
    job.d, job.gateset, job.dtype = d, _GATESETS[gateset], _DTYPES[dtype]
    job.n_traj, job.max_rounds, job.flags = n_traj, mr, 0
    job.traj0, job.seed = int(traj0), int(seed)
    job.rounds = rounds.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    job.p = _dptr(p)
    keep = None
    if eps_site is not None:
        keep = np.ascontiguousarray(eps_site, dtype=np.float64)
        if keep.shape != (n_traj, n_sites):
            raise ValueError(f"eps_site must be [{n_traj}, {n_sites}]")
        job.eps_site = _dptr(keep)
    job.eps, job.zeta = float(eps), float(zeta)
    job.hip_stream = _stream_ptr(stream)
    rec = np.zeros((n_traj, mr, n_stab), dtype=np.uint8)
    fb = np.zeros((n_traj, d * d), dtype=np.uint8)
    res = BatchResult()
    res.records = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    res.final_bits = fb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    entry = lib().sv_run_batch_noalloc if no_alloc else lib().sv_run_batch
    _check(entry(ctypes.byref(job), ctypes.byref(res)))
    del keep
    return dict(records=rec, final_bits=fb, gpu_ms=res.gpu_ms, passes_per_round=res.passes_per_round,
                redo_passes=res.redo_passes)


class Server:
    """sv_server: continuous batching with HBM-budget admission.  Output
    buffers of each job are kept here until its completion is polled."""

    def __init__(self, hbm_budget, big_streams=2, max_batch_traj=65536):
        cfg = ServerConfig(int(hbm_budget), int(big_streams), int(max_batch_traj), 0)
        h = ctypes.c_void_p()
        _check(lib().sv_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self._jobs = {}

    def submit(self, tag, d, gateset, rounds, n_traj, seed, p, eps=0.0, eps_site=None, zeta=0.0,
               dtype="c128", traj0=0):
        n_stab, n_sites, _ = template_info(d, gateset)
        req = Request()
        j = req.job
        j.d, j.gateset, j.rounds, j.dtype = d, _GATESETS[gateset], rounds, _DTYPES[dtype]
        j.n_traj, j.flags, j.traj0, j.seed = n_traj, 0, int(traj0), int(seed)
        j.p, j.eps, j.zeta = float(p), float(eps), float(zeta)
        keep = None
        if eps_site is not None:
            keep = np.ascontiguousarray(eps_site, dtype=np.float64)
            if keep.shape != (n_sites,):
                raise ValueError(f"eps_site must have {n_sites} entries")
            j.eps_site = _dptr(keep)
        rec = np.zeros((n_traj, rounds, n_stab), dtype=np.uint8)
        fb = np.zeros((n_traj, d * d), dtype=np.uint8)
        req.records = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        req.final_bits = fb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        req.tag = int(tag)
        self._jobs[int(tag)] = (rec, fb)
        try:
            _check(lib().sv_server_submit(self.h, ctypes.byref(req)))
        except SvError:
            del self._jobs[int(tag)]
            raise
        del keep

    def poll(self, max_n=1024):
        buf = (Completion * max_n)()
        k = lib().sv_server_poll(self.h, buf, max_n)
        out = []
        for c in buf[:k]:
            rec, fb = self._jobs.pop(int(c.tag))
            out.append(dict(tag=int(c.tag), status=int(c.status), t_submit=c.t_submit,
                            t_admit=c.t_admit, t_done=c.t_done, records=rec, final_bits=fb))
        return out

    def wait_idle(self, timeout_s=600.0):
        _check(lib().sv_server_wait_idle(self.h, float(timeout_s)))

    def stats(self):
        st = ServerStats()
        _check(lib().sv_server_stats_get(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def clock(self):
        return lib().sv_server_clock(self.h)

    def close(self, cancel=False):
        if self.h:
            _check(lib().sv_server_destroy(self.h, 1 if cancel else 0))
            self.h = None

    def __del__(self):
        try:
            self.close(cancel=True)
        except Exception:
            pass


def _tuning_dict(t):
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


def tuning_get(d, dtype):
    """sv_tuning_get: effective launch parameters for (d, dtype)."""
    t = Tuning()
    _check(lib().sv_tuning_get(d, _DTYPES[dtype], ctypes.byref(t)))
    return _tuning_dict(t)


def tuning_set(d, dtype, **kw):
    """sv_tuning_set: replace fields of the current parameters for (d, dtype)."""
    cur = tuning_get(d, dtype)
    cur.update(kw)
    t = Tuning(**cur)
    _check(lib().sv_tuning_set(d, _DTYPES[dtype], ctypes.byref(t)))


def autotune(d, dtype, gateset="cr"):
    """sv_autotune: time candidate launch parameters and keep the fastest;
    returns (parameters, device ms of the winning trial)."""
    t, ms = Tuning(), ctypes.c_double()
    _check(lib().sv_autotune(d, _DTYPES[dtype], _GATESETS[gateset], ctypes.byref(t), ctypes.byref(ms)))
    return _tuning_dict(t), ms.value


def tuning_save(path):
    _check(lib().sv_tuning_save(os.fsencode(path)))


def tuning_load(path):
    _check(lib().sv_tuning_load(os.fsencode(path)))


def decode_x(d, gateset, records, final_bits):
    """sv_decode_x: the X-basis memory's records and final X outcomes."""
    return decode_z(d, gateset, records, final_bits, basis="X")


def decode_z(d, gateset, records, final_bits, basis="Z"):
    """sv_decode_z (basis "X": sv_decode_x): records [n_traj, rounds, d*d-1]
    raw bits, final_bits [n_traj, d*d].  Returns dict(failed, ambiguous,
    weight) arrays; failed is 2 for trajectories with too many detection
    events (then `overflow` > 0)."""
    rec = np.ascontiguousarray(records, dtype=np.uint8)
    fb = np.ascontiguousarray(final_bits, dtype=np.uint8)
    n_traj, rounds, n_stab = rec.shape
    if n_stab != d * d - 1 or fb.shape != (n_traj, d * d):
        raise ValueError("records / final_bits shape does not match d")
    failed = np.zeros(n_traj, dtype=np.uint8)
    amb = np.zeros(n_traj, dtype=np.uint8)
    w = np.zeros(n_traj, dtype=np.int32)
    fn = lib().sv_decode_z if basis == "Z" else lib().sv_decode_x
    st = fn(d, _GATESETS[gateset], rounds, n_traj, rec.ctypes.data, fb.ctypes.data,
            failed.ctypes.data, amb.ctypes.data, w.ctypes.data)
    if st not in (SV_OK, SV_ENUMERIC):
        _check(st)
    return dict(failed=failed, ambiguous=amb, weight=w, overflow=int(np.sum(failed == 2)))
