// CPU oracle for rotated-surface-code syndrome extraction by full state-vector
// Monte Carlo trajectories (Katsuda, Mitarai, Fujii, arXiv:2204.11404).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark use it.  It shares no code, header, table or constant
// generator with the GPU path.
//
// What it computes, in the paper's own order and in complex128:
//   * the d x d rotated surface code and its stabilizer list (Sec. II.A,
//     Table I) with the CNOT order inside each plaquette and the boundary
//     "wait" slots (Sec. II.A);
//   * one stabilizer circuit at a time on the register of d^2 data qubits plus
//     ONE reused ancilla, which is measured and reset after each circuit
//     (Sec. II.B, the delayed-measurement construction that takes d=5 from 49
//     to 26 simulated qubits);
//   * the cross-resonance gate set {Rx(pi/2), Rx^dag(pi/2), Rzx(pi/2),
//     Rz(pi/2)} and its three rewrites of the textbook circuit (Sec. III.A,
//     gate-set equations), or the textbook H/CNOT/CZ circuit;
//   * the noise model: one-qubit depolarizing noise after every gate and on
//     waiting qubits, two-qubit depolarizing noise after every two-qubit gate
//     (Sec. III.A, channel equations), and coherent over-rotation of every
//     rotation gate by exp(-i eps A) (Sec. III.A, over-rotation channel);
//     stochastic channels are unravelled by sampling one Pauli per location;
//   * the protocol of Sec. III.B: data qubits start in |0>, are projected onto
//     the code space by noise-free syndrome measurements with trivial outcome,
//     then several noisy rounds run, then every data qubit is measured in Z.
//   * ZZ crosstalk exp(-i zeta Z_i Z_j) on nearest-neighbour data pairs, the
//     coherent source the paper names as a straightforward extension
//     (Introduction; Conclusion).
//
// Every gate is applied separately as a plain loop over amplitude pairs or
// quadruples; no gates are fused.  Reductions use fixed chunks so results do
// not depend on the number of OpenMP threads.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11), key = seed, counter = (draw index,
// trajectory index).  One uniform per draw.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTau = 1e-10;  // clamp for deterministic outcomes

// ---------------------------------------------------------------- Philox --
// Philox4x32 round function and Weyl key schedule as defined by Salmon et al.
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                   uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    const uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Uniform in [0, 1) on the 2^-53 grid from the first two output words of the
// Philox block addressed by (draw index k, trajectory t) under key = seed.
double uniform01(uint64_t seed, uint64_t t, uint64_t k) {
  const uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), (uint32_t)t,
                           (uint32_t)(t >> 32)};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  philox4x32_10(ctr, key, w);
  const uint64_t bits = (((uint64_t)w[1] << 32) | w[0]) >> 11;
  return (double)bits * 0x1p-53;
}

// ---------------------------------------------------------------- layout --
// A stabilizer: type (0 = X, 1 = Z) and four CNOT slots in the order of
// Sec. II.A (X: clockwise from bottom-right, Z: clockwise from top-right);
// slot value = data-qubit label 1..d^2, or 0 for "wait".
struct Stab {
  int type;
  int slot[4];
  int r, c;
};

// Plaquette (r, c) has corners TL=(r,c), TR=(r,c+1), BL=(r+1,c), BR=(r+1,c+1)
// on the d x d grid of data qubits labelled d*row + col + 1 (Table I).  X-type
// where r+c is odd.  Bulk plaquettes are all kept; weight-2 X plaquettes sit on
// the top and bottom edges, weight-2 Z plaquettes on the left and right edges.
// X plaquettes are listed by (row, column), Z plaquettes by column and then by
// descending row: this is the order of Table I.
std::vector<Stab> build_layout(int d) {
  auto label = [d](int row, int col) {
    return (row >= 0 && row < d && col >= 0 && col < d) ? d * row + col + 1 : 0;
  };
  std::vector<Stab> xs, zs;
  for (int r = -1; r <= d - 1; ++r) {
    for (int c = -1; c <= d - 1; ++c) {
      const int tl = label(r, c), tr = label(r, c + 1);
      const int bl = label(r + 1, c), br = label(r + 1, c + 1);
      const bool is_x = ((r + c) & 1) != 0;
      const int weight = (tl != 0) + (tr != 0) + (bl != 0) + (br != 0);
      const bool bulk = r >= 0 && r <= d - 2 && c >= 0 && c <= d - 2;
      bool keep = bulk;
      if (!bulk && weight == 2) {
        if (is_x && (r == -1 || r == d - 1) && c >= 0 && c <= d - 2) keep = true;
        if (!is_x && (c == -1 || c == d - 1) && r >= 0 && r <= d - 2) keep = true;
      }
      if (!keep) continue;
      Stab s;
      s.r = r;
      s.c = c;
      if (is_x) {
        s.type = 0;
        s.slot[0] = br; s.slot[1] = bl; s.slot[2] = tl; s.slot[3] = tr;
        xs.push_back(s);
      } else {
        s.type = 1;
        s.slot[0] = tr; s.slot[1] = br; s.slot[2] = bl; s.slot[3] = tl;
        zs.push_back(s);
      }
    }
  }
  std::stable_sort(xs.begin(), xs.end(), [](const Stab& a, const Stab& b) {
    return a.r != b.r ? a.r < b.r : a.c < b.c;
  });
  std::stable_sort(zs.begin(), zs.end(), [](const Stab& a, const Stab& b) {
    return a.c != b.c ? a.c < b.c : a.r > b.r;
  });
  std::vector<Stab> all = xs;
  all.insert(all.end(), zs.begin(), zs.end());
  return all;
}

// ----------------------------------------------------------- state vector --
struct State {
  int n = 0;
  std::vector<cplx> a;
  explicit State(int nq) : n(nq), a((size_t)1 << nq, cplx(0.0, 0.0)) {
    a[0] = 1.0;
  }
  int64_t size() const { return (int64_t)a.size(); }
};

// 2x2 matrix m (row-major) on qubit q: amplitude pairs differing in bit q.
void apply_1q(State& s, int q, const cplx m[4]) {
  const int64_t N = s.size();
  const int64_t bit = (int64_t)1 << q;
  cplx* a = s.a.data();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    if (i & bit) continue;
    const cplx a0 = a[i], a1 = a[i | bit];
    a[i] = m[0] * a0 + m[1] * a1;
    a[i | bit] = m[2] * a0 + m[3] * a1;
  }
}

// 4x4 matrix m (row-major) on qubits (q0, q1); local index = b(q0) + 2*b(q1).
void apply_2q(State& s, int q0, int q1, const cplx m[16]) {
  const int64_t N = s.size();
  const int64_t b0 = (int64_t)1 << q0, b1 = (int64_t)1 << q1;
  cplx* a = s.a.data();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    if ((i & b0) || (i & b1)) continue;
    const int64_t idx[4] = {i, i | b0, i | b1, i | b0 | b1};
    cplx v[4];
    for (int r = 0; r < 4; ++r) v[r] = a[idx[r]];
    for (int r = 0; r < 4; ++r) {
      cplx acc = 0.0;
      for (int c = 0; c < 4; ++c) acc += m[4 * r + c] * v[c];
      a[idx[r]] = acc;
    }
  }
}

// Pauli matrices, index 0..3 = I, X, Y, Z.  Y = [[0,-i],[i,0]].
void pauli_matrix(int P, cplx m[4]) {
  const cplx I(0.0, 1.0);
  switch (P) {
    case 0: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = 1; break;
    case 1: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; break;
    case 2: m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; break;
    default: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; break;
  }
}

// exp(-i beta P) = cos(beta) I - i sin(beta) P on one qubit.
void rot1(State& s, int q, int P, double beta) {
  cplx p[4], m[4];
  pauli_matrix(P, p);
  const cplx I(0.0, 1.0);
  const double cb = std::cos(beta), sb = std::sin(beta);
  for (int e = 0; e < 4; ++e) m[e] = (e == 0 || e == 3 ? cb : 0.0) - I * sb * p[e];
  apply_1q(s, q, m);
}

// exp(-i beta Z_qc X_qt): Z on the first qubit, X on the second.
void rot_zx(State& s, int qc, int qt, double beta) {
  // local index li = b(qc) + 2*b(qt); (Z (x) X)|bc,bt> = (-1)^bc |bc, 1-bt>.
  cplx zx[16] = {};
  for (int bc = 0; bc < 2; ++bc)
    for (int bt = 0; bt < 2; ++bt)
      zx[4 * (bc + 2 * (1 - bt)) + (bc + 2 * bt)] = (bc ? -1.0 : 1.0);
  const cplx I(0.0, 1.0);
  const double cb = std::cos(beta), sb = std::sin(beta);
  cplx m[16];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      m[4 * r + c] = (r == c ? cb : 0.0) - I * sb * zx[4 * r + c];
  apply_2q(s, qc, qt, m);
}

void hadamard(State& s, int q) {
  const double h = 1.0 / std::sqrt(2.0);
  const cplx m[4] = {h, h, h, -h};
  apply_1q(s, q, m);
}

void cnot(State& s, int qc, int qt) {
  cplx m[16] = {};
  // li = b(qc) + 2 b(qt); flips target when control is 1.
  m[4 * 0 + 0] = 1; m[4 * 2 + 2] = 1; m[4 * 3 + 1] = 1; m[4 * 1 + 3] = 1;
  apply_2q(s, qc, qt, m);
}

void cz(State& s, int q0, int q1) {
  cplx m[16] = {};
  m[0] = 1; m[5] = 1; m[10] = 1; m[15] = -1;
  apply_2q(s, q0, q1, m);
}

void apply_pauli(State& s, int q, int P) {
  if (P == 0) return;
  cplx m[4];
  pauli_matrix(P, m);
  apply_1q(s, q, m);
}

// Fixed-chunk sums of |a|^2 split by bit q (chunk = 2^14 amplitudes).
void half_norms(const State& s, int q, double* S0, double* S1) {
  const int64_t N = s.size();
  const int64_t chunk = std::min<int64_t>(N, (int64_t)1 << 14);
  const int64_t nchunks = N / chunk;
  std::vector<double> c0(nchunks, 0.0), c1(nchunks, 0.0);
  const int64_t bit = (int64_t)1 << q;
  const cplx* a = s.a.data();
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; ++c) {
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = c * chunk; i < (c + 1) * chunk; ++i) {
      const double w = std::norm(a[i]);
      if (i & bit) s1 += w; else s0 += w;
    }
    c0[c] = s0;
    c1[c] = s1;
  }
  double s0 = 0.0, s1 = 0.0;
  for (int64_t c = 0; c < nchunks; ++c) { s0 += c0[c]; s1 += c1[c]; }
  *S0 = s0;
  *S1 = s1;
}

// Keep the half with bit q == m, scaled by 1/sqrt(S_m); if `reset`, move it to
// bit q == 0 (ancilla reset); the other half becomes zero.
void project(State& s, int q, int m, double Sm, bool reset) {
  const int64_t N = s.size();
  const int64_t bit = (int64_t)1 << q;
  const double scale = 1.0 / std::sqrt(Sm);
  cplx* a = s.a.data();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    if (i & bit) continue;
    const cplx keep = (m ? a[i | bit] : a[i]) * scale;
    if (reset || m == 0) {
      a[i] = keep;
      a[i | bit] = 0.0;
    } else {
      a[i] = 0.0;
      a[i | bit] = keep;
    }
  }
}

// exp(-i zeta sum_{(i,j) in E} Z_i Z_j) over horizontal and vertical
// nearest-neighbour pairs of data qubits on the d x d grid.
void zz_layer(State& s, int d, double zeta) {
  std::vector<std::pair<int, int>> edges;
  for (int row = 0; row < d; ++row)
    for (int col = 0; col < d; ++col) {
      const int b = d * row + col;  // bit = label - 1
      if (col + 1 < d) edges.push_back({b, b + 1});
      if (row + 1 < d) edges.push_back({b, b + d});
    }
  const int64_t N = s.size();
  cplx* a = s.a.data();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    int sum = 0;
    for (const auto& e : edges) {
      const int zi = (i >> e.first) & 1, zj = (i >> e.second) & 1;
      sum += (zi == zj) ? 1 : -1;
    }
    a[i] *= std::exp(cplx(0.0, -zeta * (double)sum));
  }
}

// ------------------------------------------------------------- the circuit --
struct Job {
  int d;
  int gateset;  // 0 = cross-resonance gate set, 1 = textbook H/CNOT/CZ
  int rounds;
  uint64_t seed;
  double p;
  double zeta;
  const double* eps_site;  // per gate site (length = sites per round) or null
  double eps;              // used for every site when eps_site is null
  int twirl;               // 1: Pauli-twirled over-rotations (see site_rot1)
  int xbasis;              // 1: X-basis memory (logical |+>, final X measurement)
  int virtual_z;           // 1: Rz restores are exact (virtual Z, Fig. 4)
  int idle;                // 1: one-qubit noise on the circuit's waiting qubits at each step
  int zzp;                 // 1: exp(-i zeta Z_anc Z_q) on the check's data qubits after each step
  int max_blocks;          // > 0: stop after this many noisy circuits (no final measurement)
};

struct Ctx {
  const Job* job;
  uint64_t t;
  uint64_t k;  // next draw index
  bool noisy;
  int site;    // site index within the round template
};

double next_eps(Ctx& cx) {
  const int s = cx.site++;
  if (!cx.noisy) return 0.0;
  return cx.job->eps_site ? cx.job->eps_site[s] : cx.job->eps;
}

// Rotation exp(-i sign (base + eps) P) of the next gate site.  Twirled model
// (Sec. III.A: the coherent error exp(-i eps P) next to its Pauli channel):
// the rotation by sign*base only, then one draw u and the Pauli P when
// u < sin^2 eps.  Outside the noisy part (state preparation) nothing is drawn.
void site_rot1(State& s, Ctx& cx, int q, int P, double sign, double base) {
  const double e = next_eps(cx);
  if (!cx.job->twirl || !cx.noisy) {
    if (base != 0.0 || e != 0.0) rot1(s, q, P, sign * (base + e));
    return;
  }
  if (base != 0.0) rot1(s, q, P, sign * base);
  const double u = uniform01(cx.job->seed, cx.t, cx.k++);
  const double sn = std::sin(e);
  if (u < sn * sn) apply_pauli(s, q, P);
}

// exp(-i (base + eps) Z_qc X_qt); twirled: Z on qc and X on qt with
// probability sin^2 eps after the base rotation.
void site_rzx(State& s, Ctx& cx, int qc, int qt, double base) {
  const double e = next_eps(cx);
  if (!cx.job->twirl || !cx.noisy) {
    rot_zx(s, qc, qt, base + e);
    return;
  }
  rot_zx(s, qc, qt, base);
  const double u = uniform01(cx.job->seed, cx.t, cx.k++);
  const double sn = std::sin(e);
  if (u < sn * sn) {
    apply_pauli(s, qc, 3);
    apply_pauli(s, qt, 1);
  }
}

// One-qubit depolarizing channel (Sec. III.A): with probability p/3 each, X, Y
// or Z.  One uniform u per location; Pauli j for the first j with u < j*p/3.
void noise1(State& s, Ctx& cx, int q) {
  if (!cx.noisy) return;
  const double u = uniform01(cx.job->seed, cx.t, cx.k++);
  const double p = cx.job->p;
  for (int j = 1; j <= 3; ++j) {
    if (u < (double)j * p / 3.0) {
      apply_pauli(s, q, j);
      return;
    }
  }
}

// Two-qubit depolarizing channel: each of the 15 non-identity products A(x)B
// with probability p/15.  Pair index j = 4*a + b, A = P[a] on q1, B = P[b] on q2.
void noise2(State& s, Ctx& cx, int q1, int q2) {
  if (!cx.noisy) return;
  const double u = uniform01(cx.job->seed, cx.t, cx.k++);
  const double p = cx.job->p;
  for (int j = 1; j <= 15; ++j) {
    if (u < (double)j * p / 15.0) {
      apply_pauli(s, q1, j >> 2);
      apply_pauli(s, q2, j & 3);
      return;
    }
  }
}

// Idle noise of one step (Sec. III.A: the one-qubit channel acts on every
// qubit of the measurement circuit at each step, waiting qubits included):
// N1 on each data qubit of the check, in slot order, except `busy` (the label
// of the data qubit the step's gate acts on, or 0).  Only with job.idle.
void idle_data(State& s, Ctx& cx, const Stab& st, int busy) {
  if (!cx.job->idle) return;
  for (int j = 0; j < 4; ++j) {
    const int q = st.slot[j];
    if (q && q != busy) noise1(s, cx, q - 1);
  }
}

// Crosstalk between the ancilla and the plaquette's data qubits (only with
// job.zzp): exp(-i zeta Z_anc Z_q) for every data qubit q of the running
// check, after each step of its circuit (after the step's noise).  Diagonal:
// phase exp(-i zeta) where the two bits agree, exp(+i zeta) where they differ.
void zz_plaquette(State& s, const Ctx& cx, const Stab& st, int anc) {
  if (!cx.job->zzp || !cx.noisy || cx.job->zeta == 0.0) return;
  const cplx same = std::exp(cplx(0.0, -cx.job->zeta)), diff = std::exp(cplx(0.0, cx.job->zeta));
  for (int j = 0; j < 4; ++j) {
    const int q = st.slot[j] - 1;
    if (q < 0) continue;
    cplx* a = s.a.data();
    const int64_t N = s.size();
    for (int64_t i = 0; i < N; ++i) a[i] *= (((i >> anc) ^ (i >> q)) & 1) ? diff : same;
  }
}

// Gates and noise of one stabilizer circuit on ancilla `anc`.  With job.idle
// the circuit runs in steps (cross-resonance X check: Rx^dag | one per slot |
// Rx with the restores; Z check: one per slot | the restores; textbook: H |
// one per data qubit | H) and after each step the check's data qubits that
// the step leaves alone get N1, and in the Z check's restore step the ancilla.
// With job.zzp the ancilla-plaquette crosstalk follows every step.
void run_stabilizer_gates(State& s, Ctx& cx, const Stab& st, int anc) {
  const double q4 = kPi / 4.0;
  const int gateset = cx.job->gateset;
  if (gateset == 0) {
    if (st.type == 0) {
      // Rx^dag(pi/2) on the ancilla: rotation about -X.
      site_rot1(s, cx, anc, 1, -1.0, q4);
      noise1(s, cx, anc);
      idle_data(s, cx, st, 0);
      zz_plaquette(s, cx, st, anc);
      for (int j = 0; j < 4; ++j) {
        const int q = st.slot[j];
        if (q) {
          site_rzx(s, cx, anc, q - 1, q4);
          noise2(s, cx, anc, q - 1);
        } else {
          noise1(s, cx, anc);
        }
        idle_data(s, cx, st, q);
        zz_plaquette(s, cx, st, anc);
      }
      site_rot1(s, cx, anc, 1, 1.0, q4);
      noise1(s, cx, anc);
      for (int j = 0; j < 4; ++j) {
        const int q = st.slot[j];
        if (!q) continue;
        site_rot1(s, cx, q - 1, 1, 1.0, q4);
        noise1(s, cx, q - 1);
      }
      zz_plaquette(s, cx, st, anc);
    } else {
      for (int j = 0; j < 4; ++j) {
        const int q = st.slot[j];
        if (q) {
          site_rzx(s, cx, q - 1, anc, q4);
          noise2(s, cx, q - 1, anc);
        } else {
          noise1(s, cx, anc);
        }
        idle_data(s, cx, st, q);
        zz_plaquette(s, cx, st, anc);
      }
      for (int j = 0; j < 4; ++j) {
        const int q = st.slot[j];
        if (!q) continue;
        if (cx.job->virtual_z) {  // a frame change: no over-rotation, no draw
          next_eps(cx);
          rot1(s, q - 1, 3, q4);
        } else {
          site_rot1(s, cx, q - 1, 3, 1.0, q4);
        }
        noise1(s, cx, q - 1);
      }
      if (cx.job->idle) noise1(s, cx, anc);  // the ancilla waits during the restores
      zz_plaquette(s, cx, st, anc);
    }
  } else {
    // Textbook circuit: H, entangling gates, H on the ancilla; each H is
    // followed by the coherent error exp(-i eps X) on the ancilla.
    hadamard(s, anc);
    site_rot1(s, cx, anc, 1, 1.0, 0.0);
    noise1(s, cx, anc);
    idle_data(s, cx, st, 0);
    zz_plaquette(s, cx, st, anc);
    for (int j = 0; j < 4; ++j) {
      const int q = st.slot[j];
      if (!q) continue;
      if (st.type == 0) cnot(s, anc, q - 1); else cz(s, anc, q - 1);
      noise2(s, cx, anc, q - 1);
      idle_data(s, cx, st, q);
      zz_plaquette(s, cx, st, anc);
    }
    hadamard(s, anc);
    site_rot1(s, cx, anc, 1, 1.0, 0.0);
    noise1(s, cx, anc);
    idle_data(s, cx, st, 0);
    zz_plaquette(s, cx, st, anc);
  }
}

int weight(const Stab& st) {
  return (st.slot[0] != 0) + (st.slot[1] != 0) + (st.slot[2] != 0) + (st.slot[3] != 0);
}

// Raw ancilla bit that signals stabilizer eigenvalue +1: always 0 for the
// textbook circuit; for the cross-resonance circuit the product of w rotations
// by pi/4 flips the ancilla on eigenvalue +1 exactly when w/2 is odd.
int trivial_bit(int gateset, const Stab& st) {
  return gateset == 0 ? (weight(st) / 2) % 2 : 0;
}

void apply_measure_clamp(double* p1) {
  if (*p1 < kTau) *p1 = 0.0;
  else if (*p1 > 1.0 - kTau) *p1 = 1.0;
}

// Logical |0>: |0...0> projected by noise-free syndrome circuits with the
// trivial outcome forced (Sec. III.B).  The global phase is fixed so that the
// amplitude of |0...0> is real and positive.  Returns 0 or -1 if a forced
// outcome has probability below the clamp.
// Logical |0> (|+> for the X-basis memory): from |0...0> (|+...+>), run every
// stabilizer circuit noise-free with its outcome forced to the trivial bit;
// the global phase makes the amplitude of |0...0> real and positive.
int prepare_logical_zero(State& s, const Job& job, const std::vector<Stab>& stabs) {
  const int d = job.d, anc = d * d;
  if (job.xbasis)
    for (int q = 0; q < d * d; ++q) hadamard(s, q);
  Ctx cx{&job, 0, 0, false, 0};
  for (const Stab& st : stabs) {
    run_stabilizer_gates(s, cx, st, anc);
    double S0, S1;
    half_norms(s, anc, &S0, &S1);
    const int m = trivial_bit(job.gateset, st);
    const double Sm = m ? S1 : S0;
    if (Sm / (S0 + S1) < kTau) return -1;
    project(s, anc, m, Sm, true);
  }
  const cplx a0 = s.a[0];
  if (std::abs(a0) == 0.0) return -1;
  const cplx ph = std::conj(a0) / std::abs(a0);
  for (auto& v : s.a) v *= ph;
  return 0;
}

struct Output {
  uint8_t* records;     // [rounds][n_stab]
  uint8_t* final_bits;  // [d*d], index q-1 for data qubit q
  double* p1_trace;     // [rounds][n_stab] or null
  double* final_state;  // interleaved complex, 2^(d*d) entries, or null
};

int run_trajectory(const Job& job, uint64_t t, const Output& out) {
  const int d = job.d, nd = d * d, anc = nd;
  const std::vector<Stab> stabs = build_layout(d);
  const int ns = (int)stabs.size();
  State s(nd + 1);
  if (prepare_logical_zero(s, job, stabs) != 0) return -1;

  Ctx cx{&job, t, 0, true, 0};
  int done = 0;  // noisy circuits run so far
  bool stopped = false;
  for (int r = 0; r < job.rounds && !stopped; ++r) {
    cx.site = 0;
    for (int i = 0; i < ns; ++i) {
      if (job.max_blocks > 0 && done == job.max_blocks) {
        stopped = true;
        break;
      }
      ++done;
      const Stab& st = stabs[i];
      run_stabilizer_gates(s, cx, st, anc);
      if (job.zeta != 0.0) zz_layer(s, d, job.zeta);
      double S0, S1;
      half_norms(s, anc, &S0, &S1);
      double p1 = S1 / (S0 + S1);
      apply_measure_clamp(&p1);
      const double u = uniform01(job.seed, t, cx.k++);
      const int m = (u < p1) ? 1 : 0;
      project(s, anc, m, m ? S1 : S0, true);
      out.records[r * ns + i] = (uint8_t)m;
      if (out.p1_trace) out.p1_trace[r * ns + i] = p1;
    }
  }
  if (out.final_state) {
    for (int64_t x = 0; x < ((int64_t)1 << nd); ++x) {
      out.final_state[2 * x] = s.a[x].real();
      out.final_state[2 * x + 1] = s.a[x].imag();
    }
  }
  if (job.max_blocks > 0 && done == job.max_blocks) return 0;  // a partial trajectory
  // Final Z (X-basis memory: X) measurement of every data qubit, highest label
  // first; an X measurement is a Z measurement after a Hadamard.
  if (job.xbasis)
    for (int q = 0; q < nd; ++q) hadamard(s, q);
  for (int q = nd; q >= 1; --q) {
    double S0, S1;
    half_norms(s, q - 1, &S0, &S1);
    double p1 = S1 / (S0 + S1);
    apply_measure_clamp(&p1);
    const double u = uniform01(job.seed, t, cx.k++);
    const int b = (u < p1) ? 1 : 0;
    project(s, q - 1, b, b ? S1 : S0, false);
    out.final_bits[q - 1] = (uint8_t)b;
  }
  return 0;
}

// Gate sites (rotation gates carrying over-rotation) and random draws of one
// stabilizer circuit with the default noise options.
void block_counts(int gateset, const Stab& st, int* sites, int* draws) {
  const int w = weight(st);
  if (gateset == 0) {
    if (st.type == 0) { *sites = 2 + 2 * w; *draws = 1 + 4 + 1 + w + 1; }
    else { *sites = 2 * w; *draws = 4 + w + 1; }
  } else {
    *sites = 2;
    *draws = 1 + w + 1 + 1;
  }
}

// Number of gate sites and of random draws in one round.
void template_counts(int d, int gateset, int* n_stab, int* n_sites, int* n_draws) {
  const std::vector<Stab> stabs = build_layout(d);
  int sites = 0, draws = 0;
  for (const Stab& st : stabs) {
    int a, b;
    block_counts(gateset, st, &a, &b);
    sites += a;
    draws += b;
  }
  *n_stab = (int)stabs.size();
  *n_sites = sites;
  *n_draws = draws;
}

}  // namespace

// ------------------------------------------------------------- C interface --
extern "C" {

typedef struct {
  int d;
  int gateset;
  int rounds;
  int twirl;  // 1: Pauli-twirled over-rotations
  unsigned long long seed;
  double p;
  double zeta;
  const double* eps_site;
  double eps;
  int xbasis;     // 1: X-basis memory
  int virtual_z;  // 1: Rz restores exact
  int idle;       // 1: idle noise on the waiting qubits of every step
  int zzp;        // 1: ancilla-plaquette ZZ crosstalk after every step
  int max_blocks; // > 0: only the first max_blocks noisy circuits (then no final measurement)
} orc_job;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox4x32_10(ctr, key, out);
}

double orc_uniform(unsigned long long seed, unsigned long long t, unsigned long long k) {
  return uniform01(seed, t, k);
}

// Writes type[i] (0 = X, 1 = Z) and slots[4*i + j]; returns the count.
int orc_layout(int d, int* type, int* slots, int max_n) {
  if (d < 2 || d > 7) return -1;
  const std::vector<Stab> st = build_layout(d);
  if ((int)st.size() > max_n) return -1;
  for (size_t i = 0; i < st.size(); ++i) {
    type[i] = st[i].type;
    for (int j = 0; j < 4; ++j) slots[4 * i + j] = st[i].slot[j];
  }
  return (int)st.size();
}

int orc_template_counts(int d, int gateset, int* n_stab, int* n_sites, int* n_draws) {
  if (d < 2 || d > 7 || gateset < 0 || gateset > 1) return -1;
  template_counts(d, gateset, n_stab, n_sites, n_draws);
  return 0;
}

int orc_run_trajectory(const orc_job* j, unsigned long long t, uint8_t* records,
                       uint8_t* final_bits, double* p1_trace, double* final_state) {
  if (!j || j->d < 2 || j->d > 5 || j->rounds < 0) return -1;
  Job job{j->d,     j->gateset, j->rounds, j->seed,   j->p,         j->zeta,
          j->eps_site, j->eps,   j->twirl,  j->xbasis, j->virtual_z, j->idle, j->zzp,
          j->max_blocks};
  Output out{records, final_bits, p1_trace, final_state};
  return run_trajectory(job, t, out);
}

// Logical |0> (xbasis = 1: logical |+>) on the data register (ancilla 0),
// 2^(d*d) interleaved complex.
int orc_logical_state(int d, int gateset, int xbasis, double* out) {
  if (d < 2 || d > 5) return -1;
  Job job{d, gateset, 0, 0, 0.0, 0.0, nullptr, 0.0, 0, xbasis, 0, 0, 0, 0};
  const std::vector<Stab> stabs = build_layout(d);
  State s(d * d + 1);
  if (prepare_logical_zero(s, job, stabs) != 0) return -1;
  for (int64_t x = 0; x < ((int64_t)1 << (d * d)); ++x) {
    out[2 * x] = s.a[x].real();
    out[2 * x + 1] = s.a[x].imag();
  }
  return 0;
}

// Apply a dense k-qubit gate (k = 1 or 2) to an n-qubit state in place:
// m is 2^k x 2^k row-major interleaved complex, local index bit j = qubits[j].
int orc_apply_gate(double* state, int n, int k, const int* qubits, const double* m) {
  if (n < 1 || n > 28 || k < 1 || k > 2) return -1;
  State s(n);
  for (int64_t x = 0; x < s.size(); ++x) s.a[x] = cplx(state[2 * x], state[2 * x + 1]);
  cplx mm[16];
  for (int e = 0; e < (1 << (2 * k)); ++e) mm[e] = cplx(m[2 * e], m[2 * e + 1]);
  if (k == 1) apply_1q(s, qubits[0], mm);
  else apply_2q(s, qubits[0], qubits[1], mm);
  for (int64_t x = 0; x < s.size(); ++x) {
    state[2 * x] = s.a[x].real();
    state[2 * x + 1] = s.a[x].imag();
  }
  return 0;
}

// Benchmark sample: run n_blocks noisy stabilizer circuits of the round
// template starting at circuit `first` (gates, noise, ZZ layer, measurement
// and reset; default noise options) from |0...0> and return the wall time in
// seconds; *threads receives the OpenMP thread count.  The cost of a circuit
// does not depend on the state, so this times the same work as the
// corresponding part of a trajectory.
double orc_time_block_range(const orc_job* j, unsigned long long t, int first, int n_blocks,
                            int* threads) {
  if (!j || j->d < 2 || j->d > 5 || n_blocks < 1 || first < 0) return -1.0;
  if (j->twirl || j->idle || j->zzp) return -1.0;
  Job job{j->d,     j->gateset, 1,         j->seed,   j->p,         j->zeta,
          j->eps_site, j->eps,     0,        j->xbasis, j->virtual_z, 0,       0, 0};
  const int d = job.d, anc = d * d;
  const std::vector<Stab> stabs = build_layout(d);
  const int ns = (int)stabs.size();
  State s(d * d + 1);
  Ctx cx{&job, t, 0, true, 0};
  // sites and draws of the circuits before `first` (within its round)
  for (int i = 0; i < first % ns; ++i) {
    int a, b;
    block_counts(job.gateset, stabs[i], &a, &b);
    cx.site += a;
    cx.k += (uint64_t)b;
  }
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = first; i < first + n_blocks; ++i) {
    const Stab& st = stabs[i % ns];
    if (i % ns == 0) cx.site = 0;
    run_stabilizer_gates(s, cx, st, anc);
    if (job.zeta != 0.0) zz_layer(s, d, job.zeta);
    double S0, S1;
    half_norms(s, anc, &S0, &S1);
    double p1 = S1 / (S0 + S1);
    apply_measure_clamp(&p1);
    const double u = uniform01(job.seed, t, cx.k++);
    const int m = (u < p1) ? 1 : 0;
    project(s, anc, m, m ? S1 : S0, true);
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (threads) {
#ifdef _OPENMP
    *threads = omp_get_max_threads();
#else
    *threads = 1;
#endif
  }
  return std::chrono::duration<double>(t1 - t0).count();
}

double orc_time_blocks(const orc_job* j, unsigned long long t, int n_blocks, int* threads) {
  return orc_time_block_range(j, t, 0, n_blocks, threads);
}

// OpenMP threads of the amplitude loops from now on (n >= 1).
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
