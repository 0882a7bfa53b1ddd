/* qecsv: state-vector Monte Carlo trajectories of rotated-surface-code syndrome
 * extraction on an AMD Instinct MI355X (gfx950).
 *
 * The method is that of Katsuda, Mitarai and Fujii, "Simulation and
 * performance analysis of quantum error correction with a rotated surface code
 * under a realistic noise model" (arXiv:2204.11404):
 *   - Sec. II.A, Table I: the d x d rotated surface code, its d^2-1
 *     stabilizers and the CNOT order inside each plaquette, with "wait" slots on
 *     the boundary;
 *   - Sec. II.B: the stabilizer circuits are delayed so that one runs at a
 *     time, and a single ancilla is measured, reset and reused, so that d=5
 *     needs 26 simulated qubits instead of 49;
 *   - Sec. III.A: the cross-resonance gate set, depolarizing noise after every
 *     gate and on waiting qubits, coherent over-rotation exp(-i eps A) of every
 *     rotation gate (theta = 2 eps = 2 c sqrt(p));
 *   - Sec. III.B: logical |0> prepared by noise-free syndrome measurements with
 *     trivial outcomes, noisy rounds, a final Z measurement of the data.
 * ZZ crosstalk, named by the paper as a further coherent source (Introduction,
 * Conclusion), is supported as exp(-i zeta Z_i Z_j) on nearest-neighbour data
 * pairs once per stabilizer circuit.
 *
 * Conventions used throughout:
 *   - qubit q is bit q of the amplitude index (little-endian); data qubit label
 *     i (1-based, Table I) is qubit i-1; in a full register of d^2+1 qubits the
 *     ancilla is qubit d^2;
 *   - amplitudes are interleaved (re, im): SV_C128 = two doubles (16 B),
 *     SV_C64 = two floats (8 B);
 *   - matrices are passed from the host as row-major interleaved complex128;
 *     for a k-qubit matrix, bit j of the row/column index is qubits[j].
 *
 * Errors: every call returns an sv_status; arguments are checked on the host
 * before anything is launched and nothing is written on error.  HIP errors map
 * to SV_EDEVICE.  sv_last_error() returns a thread-local message describing the
 * last failure on the calling thread.  No call throws across this boundary.
 *
 * Streams: every sv_state is bound to one HIP stream (may be NULL = the legacy
 * default stream); the ops are enqueued on it and are asynchronous unless
 * noted.  One sv_state must not be used from two threads at once.
 */
#ifndef QECSV_H
#define QECSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SV_OK = 0,
  SV_EINVAL = -1,   /* bad argument (range, duplicate qubit, size) */
  SV_ENOMEM = -2,   /* device allocation failed or budget exceeded */
  SV_EDEVICE = -3,  /* a HIP call failed */
  SV_ENUMERIC = -4, /* a forced outcome has probability below the clamp */
  SV_EBUSY = -5     /* resource in use */
} sv_status;

typedef enum { SV_C64 = 0, SV_C128 = 1 } sv_dtype;

typedef enum {
  SV_GATESET_CR = 0,       /* Sec. III.A cross-resonance circuit */
  SV_GATESET_TEXTBOOK = 1  /* H / CNOT / CZ circuit of Fig. 1 */
} sv_gateset;

/* Probabilities below this are clamped to 0 (above 1 - SV_TAU to 1) before an
 * outcome is decided. */
#define SV_TAU 1e-10

/* sv_job.flags for sv_run_rounds */
#define SV_RUN_GRAPH 1 /* capture one trajectory's launch sequence (draws,
                          passes, decisions, final measurement, record copy)
                          in a HIP graph once and replay it per trajectory;
                          results are identical to the stream launches */
#define SV_RUN_XBASIS 4 /* X-basis memory: logical |+> instead of |0> (the
                           2^(n - n_z) strings with even parity on every Z
                           check, equal amplitudes), and the data qubits
                           measured in the X basis at the end (final_bits =
                           X outcomes, 1 for eigenvalue -1); final_states is
                           the register before that measurement */
#define SV_RUN_VIRTUAL_Z 8 /* the Rz(pi/2) restores after cross-resonance Z
                              checks are virtual Z gates without
                              over-rotation (their sites keep their place in
                              eps_site but are not used) */
#define SV_RUN_TWIRL 2 /* Pauli-twirled over-rotations: every rotation turns by
                          its base angle only, and one draw right after it
                          applies its generator (Rx: X, Rz: Z, Rzx: Z x X, the
                          textbook exp(-i eps X): X) with probability sin^2 of
                          the site's exponent -- the Pauli channel with the
                          same error probability as the coherent error
                          (Sec. III.A); the draw enumeration gains one draw per
                          rotation, placed before that gate's noise draw */
#define SV_RUN_IDLE_NOISE 16 /* one-qubit depolarizing noise on the waiting
                                qubits of every step (Sec. III.A: the channel
                                acts on every qubit of the measurement circuit
                                at each step).  Steps: cross-resonance X check
                                Rx^dag | each slot | Rx with the restores; Z
                                check each slot | the restores; textbook H |
                                each data qubit | H.  After a step, one N1 draw
                                per data qubit of the check that the step does
                                not touch (slot order), and one on the ancilla
                                after the Z check's restores */
#define SV_RUN_ZZ_PLAQUETTE 32 /* crosstalk between the ancilla and the running
                                  check's data qubits: after every step (as
                                  for SV_RUN_IDLE_NOISE, after its noise),
                                  exp(-i zeta Z_anc Z_q) for each data qubit
                                  q of the check, in addition to the
                                  once-per-circuit data ZZ layer; X checks
                                  then get dense Kraus pairs (no effect when
                                  zeta = 0) */

typedef struct sv_state_s* sv_state;

/* Thread-local description of the last error on this thread ("" if none). */
const char* sv_last_error(void);

/* Library ABI version (major * 100 + minor). */
int sv_version(void);

/* ------------------------------------------------------------------ memory */

/* Allocate a register of n_qubits (1..34) in dtype on the current HIP device,
 * bound to hip_stream (a hipStream_t, may be NULL).  The library owns the
 * memory; sv_free releases it.  The register starts in |0...0>. */
sv_status sv_alloc(int n_qubits, sv_dtype dtype, void* hip_stream, sv_state* out);

/* Wrap caller-owned device memory (e.g. a torch tensor) of at least
 * 2^n_qubits amplitudes as a register.  The library never frees dev_ptr.
 * dev_ptr must be 16-byte aligned. */
sv_status sv_wrap(void* dev_ptr, size_t bytes, int n_qubits, sv_dtype dtype,
                  void* hip_stream, sv_state* out);

/* Release the handle (and the memory if sv_alloc made it).  Waits for the
 * stream.  NULL is accepted. */
sv_status sv_free(sv_state s);

/* Copy 2^n amplitudes from / to host memory (bytes must equal the register
 * size).  Synchronous. */
sv_status sv_set_state(sv_state s, const void* host, size_t bytes);
sv_status sv_get_state(sv_state s, void* host, size_t bytes);

/* Copy the amplitudes of src into dst (same n_qubits and dtype) with a
 * streaming device kernel on dst's stream (waits for src's stream first if it
 * differs).  Asynchronous on dst's stream. */
sv_status sv_copy_state(sv_state dst, sv_state src);

/* |index>. */
sv_status sv_set_basis(sv_state s, uint64_t index);

/* Logical |0> of the distance-d code on data qubits 0..d^2-1 (Sec. III.B):
 * amplitude 2^(-n_X/2) on every basis state of the orbit of |0...0> under the
 * X-stabilizer group, zero elsewhere (ancilla and higher qubits 0).  This is
 * the state the noise-free projection with trivial outcomes produces, with
 * its global phase fixed real and positive.  Needs n_qubits >= d^2. */
sv_status sv_load_logical0(sv_state s, int d);

/* Wait for the register's stream. */
sv_status sv_synchronize(sv_state s);

/* --------------------------------------------------------------------- ops */

/* Dense k-qubit gate, k in {1, 2}: m is 2^k x 2^k row-major interleaved
 * complex128 (host pointer, copied before return); distinct qubits < n. */
sv_status sv_apply_gate(sv_state s, int k, const int* qubits, const double* m);

/* Diagonal on k <= 5 qubits: amplitude *= phases[local index] (2^k
 * interleaved complex128, host pointer). */
sv_status sv_apply_diag(sv_state s, int k, const int* qubits, const double* phases);

/* Dense fused k-qubit matrix, 1 <= k <= 5 (up to 32 x 32 complex) applied to
 * all 2^(n-k) vectors (the gate action of Sec. II.B written as one matrix);
 * same layout as sv_apply_gate.  Used for runs of gates multiplied on the host
 * into one matrix.  k = 4, 5 run on the matrix cores when n - k >= 4.  m is a
 * host pointer, copied before return (the caller may reuse it at once); the
 * call is stream-ordered and returns without waiting for the kernel, except
 * when eight earlier calls on this state are still in flight.  Errors:
 * SV_EINVAL (qubits, k, NULL m), SV_ENOMEM (the 128 KiB of matrix slots, on
 * the first call), SV_EDEVICE (launch or copy failure). */
sv_status sv_apply_fused(sv_state s, int k, const int* qubits, const double* m);

/* ------------------------------------------------------------- measurement */

/* Measure qubit anc in Z and reset it (Sec. II.B): S0, S1 = squared norms of
 * the halves with anc = 0 / 1 (FP64), p1 = S1/(S0+S1) clamped by SV_TAU,
 * outcome = [u < p1]; the kept half is scaled by 1/sqrt(S_outcome) and moved
 * to anc = 0, the other half is zeroed.  Synchronous: waits for the stream.
 * outcome and p1 may be NULL. */
sv_status sv_measure_reset_ancilla(sv_state s, int anc, double u, int* outcome, double* p1);

/* Same with the outcome given; returns SV_ENUMERIC (state unchanged) if the
 * outcome's probability is below SV_TAU. */
sv_status sv_measure_reset_ancilla_forced(sv_state s, int anc, int outcome, double* p1);

/* ------------------------------------------------------------- whole runs */

/* One round of the template: number of stabilizers (d^2-1), gate sites (each
 * rotation gate instance, the unit of the per-site over-rotation) and random
 * draws (noise locations plus one per measurement). */
sv_status sv_template_info(int d, int gateset, int* n_stab, int* n_sites, int* n_draws_per_round);

/* Host-side self-check of the register-pass layouts that sv_run_rounds would
 * use for (d, gateset) with Z chains of at most zchain checks and, when xpair
 * is 1, pairs of consecutive X checks (sv_tuning.xpair): every tile layout
 * partitions its bits between lanes and register slots, the regrouping
 * layouts cover the same tile, and each unit's qubits sit where its mode needs
 * them; for d <= 3 also the layouts of sv_run_batch's LDS-resident kernel for
 * one, two and four waves per trajectory.  No device work.  *n_passes
 * (optional) receives the pass count of one round sequence; SV_EINVAL names
 * the first failing pass or block. */
sv_status sv_check_pass_layouts(int d, int gateset, int zchain, int xpair, int* n_passes);

/* Host-side self-check of the speculative passes sv_run_rounds and
 * sv_run_batch use for (d, gateset) with Z chains of at most zchain checks
 * when the data ZZ layer is off: for each unit (a pair of consecutive X
 * checks, a single X check or a Z chain) its pass fits a tile; a pair's tile
 * holds both members' qubits, the second member's layout covers the same
 * tile bits with that member's qubits on its register slots, and a pair
 * stored from that layout keeps the three lowest bits on its first lanes.  No
 * device work.  *n_units receives the units per round, or 0 when the plain
 * passes run instead (fewer than 12 qubits, or a chain that would have to be
 * summed amplitude by amplitude); SV_EINVAL names the first failing unit. */
sv_status sv_check_spec_layouts(int d, int gateset, int zchain, int* n_units);

typedef struct sv_job {
  int d;               /* code distance, 2..5 */
  int gateset;         /* sv_gateset */
  int rounds;          /* noisy rounds, >= 1 */
  int dtype;           /* sv_dtype of the state */
  int n_traj;          /* trajectories */
  int flags;           /* SV_RUN_GRAPH | SV_RUN_TWIRL | SV_RUN_XBASIS |
                          SV_RUN_VIRTUAL_Z | SV_RUN_IDLE_NOISE |
                          SV_RUN_ZZ_PLAQUETTE
                          (sv_run_rounds only; with
                          SV_RUN_GRAPH final_states must be NULL) */
  uint64_t traj0;      /* first trajectory index (draw stream id) */
  uint64_t seed;       /* Philox key */
  double p;            /* depolarizing probability, [0, 1] */
  double eps;          /* over-rotation exponent for every site (if eps_site NULL) */
  const double* eps_site; /* host array of n_sites exponents, or NULL */
  double zeta;         /* ZZ crosstalk strength */
  void* hip_stream;    /* stream to run on (NULL = default) */
} sv_job;

typedef struct sv_result {
  uint8_t* records;     /* host [n_traj][rounds][d^2-1] raw ancilla bits (required) */
  uint8_t* final_bits;  /* host [n_traj][d^2], index q-1 for data qubit q (required) */
  double* p1_trace;     /* host [n_traj][rounds][d^2-1] clamped p1, or NULL */
  void* final_states;   /* host [n_traj][2^(d^2)] amplitudes of dtype before the
                           final measurement, or NULL */
  double gpu_ms;        /* out: device time of the whole run (hipEvents) */
  double pass_ms;       /* out: mean device time per register pass of the last
                           trajectory (one pass applies an X check, a pair of
                           them or a chain of Z checks; with speculative
                           units, their prediction passes) */
  int passes_per_round; /* out: register passes per round (speculative units:
                           prediction passes per round) */
  int redo_passes;      /* out: speculative units' redo passes that ran, over
                           the whole run (0 without speculative units and for
                           sv_run_rounds_async, which does not wait for it) */
} sv_result;

/* Run job->n_traj trajectories (indices traj0 ..): logical |0>, `rounds`
 * noisy rounds of the d^2-1 stabilizer circuits in Table I order (all X
 * checks, then all Z checks), each followed by an ancilla measurement and
 * reset, then a Z measurement of every data qubit from label d^2 down to 1.
 * Draw k of trajectory t is uniform(seed, t, k) from Philox4x32-10; the draws
 * are enumerated in circuit order: per round, per stabilizer, one per noise
 * location and then one for the measurement; after the last round one per
 * final data measurement.  Synchronous.  Records are the raw ancilla bits.
 * With zeta = 0 and d >= 4 (outcomes then mostly repeat from round to round)
 * the register passes are speculative: a pair of X checks or a chain of Z
 * checks is summed and applied in one pass with predicted outcomes (the
 * trivial ones in the first round, the previous round's after that) and the
 * pass runs again when a drawn outcome differs; records, p1 and states are
 * those of the plain passes.  The environment variable QECSV_SPEC = 0 / 1
 * turns this off / on whatever zeta is (not with the dense crosstalk, which
 * always uses the plain passes). */
sv_status sv_run_rounds(const sv_job* job, sv_result* res);

/* The same run enqueued without waiting, so that jobs on several streams
 * overlap on the device (the paper's workload is many independent
 * trajectories, Sec. III.B).  Every kernel and copy goes to job->hip_stream;
 * done_event (a hipEvent_t the caller created) is recorded on that stream
 * after records, final_bits and p1_trace (if given) have been copied into
 * res's host buffers, and the call returns without waiting for the device.
 * The caller keeps those buffers valid and unread until done_event has
 * completed; with pinned host buffers (hipHostMalloc) the copies run
 * asynchronously, with pageable ones the runtime may wait for them.  job and
 * eps_site are copied before return.  Results are those of sv_run_rounds.
 * Not available: SV_RUN_GRAPH and final_states (SV_EINVAL).  res->gpu_ms and
 * res->pass_ms are set to -1 (time with events on the stream);
 * res->passes_per_round is set.  Errors are reported before anything is
 * enqueued, except HIP failures during enqueueing (SV_EDEVICE; work already
 * enqueued then still runs and done_event is not recorded). */
sv_status sv_run_rounds_async(const sv_job* job, sv_result* res, void* done_event);

/* Decoding of the Z-basis memory experiment (Sec. III.B; host only).
 * Detection events: Z-check syndromes (raw record XOR its trivial bit, which
 * is (w/2) mod 2 for a weight-w check of the cross-resonance circuit and 0
 * for the textbook circuit) compared between consecutive rounds, plus a last
 * layer recomputed from the final data bits.  They are paired by an exact
 * minimum-weight perfect matching on the unit-weight space-time graph with one
 * boundary node (dynamic programming over subsets, at most 22 events per
 * trajectory).  records: host [n_traj][rounds][d^2-1] raw bits as written by
 * sv_run_rounds; final_bits: host [n_traj][d^2].  Outputs (host, n_traj
 * entries): failed = 1 if the corrected Z_L = Z_1...Z_d reads -1, else 0 (2
 * if the trajectory has too many events); ambiguous (optional) = 1 if
 * minimum-weight corrections of both logical parities exist; weight
 * (optional) = the matching's total weight (-1 if undecoded).  SV_ENUMERIC if
 * any trajectory has more than 22 events (the others are still decoded). */
sv_status sv_decode_z(int d, int gateset, int rounds, int n_traj, const uint8_t* records,
                      const uint8_t* final_bits, uint8_t* failed, uint8_t* ambiguous, int* weight);
/* The same for the X-basis memory (SV_RUN_XBASIS): X-check events, final_bits
 * are X outcomes, failed = 1 if the corrected X_L (X on the first column,
 * labels 1, d+1, ..., (d-1)d+1) reads -1. */
sv_status sv_decode_x(int d, int gateset, int rounds, int n_traj, const uint8_t* records,
                      const uint8_t* final_bits, uint8_t* failed, uint8_t* ambiguous, int* weight);

/* Launch parameters of the trajectory engine for (d, dtype) on the current
 * device.  They change speed only: results agree up to the order of
 * floating-point sums.  The environment variables QECSV_ZCHAIN, QECSV_SNAKE,
 * QECSV_BATCH_WAVES_PER_CU, QECSV_LOCKSTEP_MIB, QECSV_PASS_WGS_PER_CU and
 * QECSV_XPAIR override them. */
typedef struct sv_tuning {
  int zchain;             /* longest chain of Z checks applied per register pass, 1..6 */
  int snake;              /* 1: consecutive passes walk the tiles in opposite orders */
  int batch_waves_per_cu; /* sv_run_batch, d <= 3: resident waves per compute unit, 1..32 */
  int lockstep_mib;       /* sv_run_batch, d = 4: MiB of registers run in lockstep */
  int pass_wgs_per_cu;    /* sv_run_rounds: workgroups per compute unit of a register
                             pass, each taking tiles grid-stride; 0 = one tile
                             per workgroup (0..64) */
  int xpair;              /* 1: d >= 4 register passes may sum two consecutive X
                             checks at once (the second for each outcome of the
                             first) and apply both in the next pass, wherever
                             both units' qubits fit one tile of 2^12
                             amplitudes; 0: one X check per pass */
} sv_tuning;

/* Effective parameters (set, tuned or built-in, then the environment). */
sv_status sv_tuning_get(int d, int dtype, sv_tuning* out);
/* Replace the parameters for (d, dtype) on the current device; SV_EINVAL if
 * a field is out of range. */
sv_status sv_tuning_set(int d, int dtype, const sv_tuning* in);
/* Time candidate parameters on synthetic work of this shape (tens of ms of
 * device time) and keep the fastest for (d, dtype) on the current device:
 * d = 5, sv_run_rounds (one trajectory, one round): xpair x zchain x snake x
 *   pass_wgs_per_cu;
 * d = 4, sv_run_batch (4096 trajectories, 3 rounds): xpair x zchain x
 *   lockstep_mib;
 * d <= 3, sv_run_batch (16384 trajectories, 3 rounds): batch_waves_per_cu.
 * Writes the winner to *best and its device time to *best_ms (either may be
 * NULL).  Synchronous, on the default stream; call it before serving, not
 * while other threads run jobs of the same shape. */
sv_status sv_autotune(int d, int dtype, int gateset, sv_tuning* best, double* best_ms);
/* Write / read the parameters of the current device's architecture as text
 * lines "arch d dtype zchain snake batch_waves_per_cu lockstep_mib
 * pass_wgs_per_cu xpair"; load (lines without the last field: xpair 0)
 * keeps only lines for this architecture.  SV_EINVAL on I/O or parse errors. */
sv_status sv_tuning_save(const char* path);
sv_status sv_tuning_load(const char* path);

/* Batched small-distance trajectories: one persistent launch runs n_traj
 * trajectories, each with its own round count, depolarizing probability and
 * per-site over-rotation exponents.  Trajectory i uses draw stream traj0 + i
 * and is the same trajectory sv_run_rounds computes for those parameters
 * (same draw enumeration, same records and final bits).  d = 2 or 3 keep the
 * whole data register in LDS (one persistent launch, a workgroup of one or
 * two waves per trajectory: two when the launch has at most two trajectories
 * per SIMD; the environment variable QECSV_BATCH_SPLIT = 1, 2 or 4 forces the
 * count); d = 4 keeps the registers in HBM and runs the trajectories in
 * lockstep through the register passes, the trajectory being a grid
 * dimension; with zeta = 0 those passes are speculative as in sv_run_rounds
 * (each slot then holds two registers; QECSV_SPEC = 0 / 1 forces the mode).
 * Synchronous. */
typedef struct sv_batch_job {
  int d;                    /* 2..4 */
  int gateset;              /* sv_gateset */
  int dtype;                /* sv_dtype */
  int n_traj;
  int max_rounds;           /* >= every rounds[i] */
  int flags;                /* reserved, must be 0 */
  uint64_t traj0;
  uint64_t seed;
  const int* rounds;        /* host [n_traj], each in 1..max_rounds */
  const double* p;          /* host [n_traj], each in [0, 1] */
  const double* eps_site;   /* host [n_traj][n_sites] exponents, or NULL */
  double eps;               /* every site of every trajectory if eps_site is NULL */
  double zeta;
  void* hip_stream;
} sv_batch_job;

typedef struct sv_batch_result {
  uint8_t* records;     /* host [n_traj][max_rounds][d^2-1]; rows past rounds[i] are 0 */
  uint8_t* final_bits;  /* host [n_traj][d^2] */
  double gpu_ms;        /* out: device time of the launch (hipEvents) */
  int passes_per_round; /* out: d = 4: register passes per round (speculative
                           units: prediction passes); 0 for d <= 3 */
  int redo_passes;      /* out: speculative redos that ran (one per trajectory
                           and unit); 0 without speculative units */
} sv_batch_result;

sv_status sv_run_batch(const sv_batch_job* job, sv_batch_result* res);

/* sv_run_batch for d <= 3 without any device allocation, for callers that
 * cannot allocate (tight serving loops, harnesses that forbid hipMalloc): the
 * same job, kernels and results, with every device buffer of the launch
 * (staged parameters, per-trajectory tables, records, final bits) carved
 * from a static 64 MiB array that each GPU the library runs on holds until
 * the process ends.  Its address is taken once per device on the first call
 * there.  Calls on one device are serialised by a lock and each call clears
 * what must start at zero; a call leaves its data in the array.  Errors:
 * SV_EINVAL as sv_run_batch, and for d = 4; SV_ENOMEM if the job's buffers
 * exceed the 64 MiB (about 100 000 d=3 trajectories with per-site angles, 9
 * rounds), checked before anything is enqueued.  Synchronous. */
sv_status sv_run_batch_noalloc(const sv_batch_job* job, sv_batch_result* res);

/* ---------------------------------------------------------------- serving */

/* A server runs submitted jobs (each an sv_job: distance, rounds, dtype, noise
 * parameters, trajectory range) with continuous batching: jobs are admitted
 * in arrival order while the device bytes they hold fit in hbm_budget;
 * admitted jobs with d <= 4 join a lane per (d, gate set, dtype, zeta) whose
 * worker merges the waiting trajectories of any number of jobs into one
 * persistent batched launch (a job arriving during a launch joins the next);
 * d = 5 jobs run on one of big_streams workers with their own HIP streams, so
 * their passes overlap on the device.  A job's records and final bits are the
 * same as those of sv_run_rounds for the same job.  All calls are thread-safe.
 */
typedef struct sv_server_s* sv_server;

typedef struct sv_server_config {
  size_t hbm_budget;   /* device bytes admitted jobs may hold at once (> 0) */
  int big_streams;     /* d = 5 jobs running at once, 1..16 */
  int max_batch_traj;  /* trajectories per merged launch, >= 1 */
  int flags;           /* reserved, must be 0 */
} sv_server_config;

typedef struct sv_request {
  sv_job job;          /* hip_stream ignored; eps_site copied at submission */
  uint8_t* records;    /* host [n_traj][rounds][d^2-1], caller-owned until completion */
  uint8_t* final_bits; /* host [n_traj][d^2] */
  uint64_t tag;        /* returned with the completion */
} sv_request;

typedef struct sv_completion {
  uint64_t tag;
  int status;          /* sv_status of the job (SV_EBUSY: cancelled) */
  int pad;
  double t_submit;     /* server clock, seconds */
  double t_admit;
  double t_done;
} sv_completion;

typedef struct sv_server_stats {
  size_t hbm_in_use;      /* bytes held by admitted, unfinished jobs */
  size_t hbm_high_water;  /* maximum of hbm_in_use so far (<= hbm_budget) */
  int pending;            /* submitted, not admitted */
  int running;            /* launches in flight */
  int completed;
  int launches;           /* batched launches plus d = 5 jobs run */
} sv_server_stats;

sv_status sv_server_create(const sv_server_config* cfg, sv_server* out);

/* Enqueue a job; returns at once.  SV_ENOMEM if the job alone exceeds the
 * budget, SV_EINVAL for bad arguments (nothing is queued). */
sv_status sv_server_submit(sv_server s, const sv_request* req);

/* Move up to max completions (oldest first) into out; returns how many. */
int sv_server_poll(sv_server s, sv_completion* out, int max);

/* Wait until every submitted job has completed, or SV_EBUSY after timeout_s. */
sv_status sv_server_wait_idle(sv_server s, double timeout_s);

sv_status sv_server_stats_get(sv_server s, sv_server_stats* out);

/* Seconds since the server was created (the clock of the completions). */
double sv_server_clock(sv_server s);

/* Finish and free the server.  cancel = 0 waits for every job; cancel = 1
 * completes queued jobs with SV_EBUSY and stops admitted ones at their next
 * trajectory or launch. */
sv_status sv_server_destroy(sv_server s, int cancel);

/* Philox4x32-10 uniform used by the device code, evaluated on the host (for
 * tests of the draw stream). */
double sv_uniform(uint64_t seed, uint64_t t, uint64_t k);

/* Host-side evaluation (no GPU) of the operator the trajectory engine applies
 * for stabilizer `stab` (0-based, Table I order) in round `round` of
 * trajectory t.  With the ancilla starting in |0>, the circuit's unitary U and
 * the outcome m, K_m = <m|_anc U |0>_anc acts on the block's w data qubits;
 * for this noise model it is monomial in the block basis B (Hadamard on the
 * data qubits for X checks, identity for Z checks):
 *   K_m = B . P_F . diag(D_m) . B,   P_F |x> = |x XOR F>.
 * Outputs: D = [2][2^w] interleaved complex128 (host buffer of 64 doubles,
 * entries beyond 2^w are 0; for X checks the two unnormalised Walsh-Hadamard
 * factors 2^-w are folded in), *F, *u (the measurement draw), *type (0 = X,
 * 1 = Z), *w, qubits[0..w-1] (data qubit indices in CNOT-slot order).
 * Returns SV_EINVAL if the circuit is not monomial in that basis. */
sv_status sv_block_kraus(int d, int gateset, int stab, int round, uint64_t seed, uint64_t t,
                         double p, double eps, const double* eps_site, double* D, uint32_t* F,
                         double* u, int* type, int* w, int* qubits);

#ifdef __cplusplus
}
#endif

#endif /* QECSV_H */
