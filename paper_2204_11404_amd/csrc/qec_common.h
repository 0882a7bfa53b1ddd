// Host/device definitions shared by the qecsv runtime and its HIP kernels:
// the counter-based generator, the encoded stabilizer-circuit template, and
// the per-block Kraus builder used by the trajectory engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#define QEC_HD __host__ __device__ __forceinline__

namespace qec {

// ------------------------------------------------------------------ Philox --
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 32x32->64 multiplies
// per round with constants M0, M1, key bumped by the Weyl constants W0, W1.
struct U4 {
  uint32_t x, y, z, w;
};

QEC_HD U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = (uint64_t)0xD2511F53u * c.x;
    const uint64_t b = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(b >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)b;
    n.z = (uint32_t)(a >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)a;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Draw k of trajectory t: counter (k, t), key = seed, 53 random bits from the
// first two output words, scaled to [0, 1).
QEC_HD double uniform(uint64_t seed, uint64_t t, uint64_t k) {
  U4 c{(uint32_t)k, (uint32_t)(k >> 32), (uint32_t)t, (uint32_t)(t >> 32)};
  const U4 o = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t bits = ((((uint64_t)o.y) << 32) | o.x) >> 11;
  return (double)bits * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------- complex helpers --
struct cd {
  double re, im;
};
QEC_HD cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
QEC_HD cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
QEC_HD cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }
QEC_HD cd cexpi(double th) { return {cos(th), sin(th)}; }  // e^{i th}

// ---------------------------------------------------- circuit template --
// One stabilizer circuit is a list of ops on the ancilla and the block's data
// qubits (local index j = position among the block's data qubits in CNOT
// slot order).  Rotation ops carry a gate site (index into the per-round
// over-rotation table) and an angle base (pi/4 for the cross-resonance gate
// set, 0 for the textbook over-rotation gate).  Noise ops carry a local draw
// index.
enum OpKind : uint8_t {
  OP_ROT_ANC = 1,   // exp(-i beta sgn P) on the ancilla, P = axis
  OP_ROT_DATA = 2,  // exp(-i beta P) on data j
  OP_CR_AD = 3,     // exp(-i beta Z_anc X_j)
  OP_CR_DA = 4,     // exp(-i beta Z_j X_anc)
  OP_H_ANC = 5,     // Hadamard on the ancilla
  OP_CNOT_AD = 6,   // CNOT control ancilla, target data j
  OP_CZ_AD = 7,     // CZ ancilla, data j
  OP_N1_ANC = 8,    // one-qubit depolarizing location on the ancilla
  OP_N1_DATA = 9,   // ... on data j
  OP_N2_AD = 10,    // two-qubit location, first qubit ancilla, second data j
  OP_N2_DA = 11,    // two-qubit location, first qubit data j, second ancilla
  OP_ZZ_AD = 12,    // exp(-i beta Z_anc Z_j): ancilla-plaquette crosstalk (beta from its site)
};

struct TOp {
  uint8_t kind;
  uint8_t j;        // local data index
  uint8_t axis;     // 1 = X, 2 = Y, 3 = Z
  int8_t sgn;       // +1 / -1 generator sign
  uint8_t quarter;  // 1: angle base pi/4; 0: base 0
  uint8_t exact;    // 1: no over-rotation at this site (virtual Z)
  int16_t site;     // gate site within the round, -1 if none
  int16_t draw;     // local draw index, -1 if none
  int16_t pad2;
};

constexpr int kMaxOps = 64;       // cross-resonance X check with idle noise and per-step ZZ: 60
constexpr int kMaxOpsBatch = 24;  // templates of the batched paths (no idle noise): 20

struct TBlock {
  int type;          // 0 = X check (data in the X basis), 1 = Z check
  int w;             // data qubits (2 or 4)
  int qubit[4];      // data qubit (bit index) per local index
  int n_ops;
  int n_draws;       // noise draws + 1 measurement draw
  int dense;         // 1: not monomial in the block basis (dense Kraus pair, BlockDense)
  int draw_off;      // first draw of this block within the round
  int site_off;      // first site of this block within the round
  uint64_t n2mask;   // bit k set if noise draw k is a two-qubit location
  TOp ops[kMaxOps];
};

// Per (trajectory, block instance) result of the Kraus builder.  With B the
// block basis (Hadamard on the block's data for X checks, identity for Z
// checks), the post-measurement operator of outcome m on the data register is
// K_m = B Pi_F diag(D_m) B, a monomial matrix: the kernels apply it as
// WHT -> diag -> WHT -> sign pattern (X checks) or diag -> XOR permutation (Z
// checks).  D holds D_m with 2^-w folded in for X checks; W holds the weights
// |D_m|^2 (again with 2^-w for X checks) that give S_m from the transformed
// amplitudes.
struct BlockRT {
  double D[2][16][2];
  double W[2][16];
  double u;       // measurement draw
  uint32_t F;     // XOR pattern (local data bits)
  uint32_t pad;
};

// Dense Kraus pair of a block that is not monomial in its basis:
// K[m][i][x] = <anc m, data i| U |anc 0, data x>, data labels in the
// computational basis of the block's qubits (bit l = block qubit l).
struct BlockDense {
  double K[2][16][16][2];
};

// Thresholds of the depolarizing channels: Pauli j is chosen for the first
// j with u < j p / 3 (one-qubit, j = 1..3 -> X, Y, Z) or u < j p / 15
// (two-qubit, j = 1..15 -> P[j >> 2] (x) P[j & 3] on (first, second)).
QEC_HD int pick_pauli1(double u, double p) {
  for (int j = 1; j <= 3; ++j)
    if (u < (double)j * p / 3.0) return j;
  return 0;
}
QEC_HD int pick_pauli2(double u, double p) {
  for (int j = 1; j <= 15; ++j)
    if (u < (double)j * p / 15.0) return j;
  return 0;
}

// Pauli P (1 X, 2 Y, 3 Z) on the ancilla 2-vector.
QEC_HD void anc_pauli(int P, cd& v0, cd& v1) {
  if (P == 1) {
    cd t = v0; v0 = v1; v1 = t;
  } else if (P == 2) {  // Y = [[0,-i],[i,0]]
    cd t = v0;
    v0 = {v1.im, -v1.re};   // -i * v1
    v1 = {-t.im, t.re};     //  i * v0
  } else if (P == 3) {
    v1 = {-v1.re, -v1.im};
  }
}

// Pauli P on data bit j of the block-basis label `cur`: returns the phase
// and flips cur if needed.  In the X basis X is diagonal (eigenvalue +-1),
// Z flips |+> <-> |->, Y|+> = -i|->, Y|-> = i|+>.  In the Z basis Z is
// diagonal, X flips, Y|0> = i|1>, Y|1> = -i|0>.
QEC_HD cd data_pauli(int P, bool xbasis, int j, uint32_t& cur) {
  const int bit = (cur >> j) & 1;
  const double e = bit ? -1.0 : 1.0;
  cd ph{1.0, 0.0};
  if (P == 0) return ph;
  const int diag_axis = xbasis ? 1 : 3;
  if (P == diag_axis) return {e, 0.0};
  if (P == 2) {
    // X basis: bit 0 -> -i, bit 1 -> +i;  Z basis: bit 0 -> +i, bit 1 -> -i
    const double s = xbasis ? -e : e;
    ph = {0.0, s};
  }
  cur ^= (1u << j);
  return ph;
}

// exp(-i theta P) on the ancilla 2-vector given c = cos(theta), s = sin(theta).
QEC_HD void anc_rot_cs(int axis, double c, double s, cd& v0, cd& v1) {
  if (axis == 1) {  // [[c, -is], [-is, c]]
    cd a{c * v0.re + s * v1.im, c * v0.im - s * v1.re};
    cd b{c * v1.re + s * v0.im, c * v1.im - s * v0.re};
    v0 = a; v1 = b;
  } else if (axis == 2) {  // [[c, -s], [s, c]]
    cd a{c * v0.re - s * v1.re, c * v0.im - s * v1.im};
    cd b{s * v0.re + c * v1.re, s * v0.im + c * v1.im};
    v0 = a; v1 = b;
  } else {  // diag(e^{-i th}, e^{i th})
    v0 = cmul(v0, cd{c, -s});
    v1 = cmul(v1, cd{c, s});
  }
}

// Angle of a rotation op: pi/4 (cross-resonance gate set) or 0 (textbook
// over-rotation gate) plus the over-rotation exponent of its site.  A
// rotation op that carries a draw belongs to the Pauli-twirled model (its
// over-rotation is replaced by the generator applied with probability
// sin^2 eps, Sec. III.A): it rotates by the base angle only.
QEC_HD double op_angle(const TOp& op, const double* eps_site) {
  return (op.quarter ? 0.78539816339744830962 : 0.0) +
         (op.site >= 0 && op.draw < 0 && !op.exact ? eps_site[op.site] : 0.0);
}

QEC_HD bool is_rotation(uint8_t kind) {
  return kind == OP_ROT_ANC || kind == OP_ROT_DATA || kind == OP_CR_AD || kind == OP_CR_DA;
}

// Accessor evaluating cos/sin of each op's angle on the fly.
struct CsFromEps {
  const double* eps;
  QEC_HD cd operator()(const TOp& op) const {
    const double beta = op_angle(op, eps);
    return {cos(beta), sin(beta)};
  }
};

// Accessor reading a per-site (cos, sin) table.
struct CsFromTable {
  const double* cs;  // [site][2]
  QEC_HD cd operator()(const TOp& op) const { return {cs[2 * op.site], cs[2 * op.site + 1]}; }
};

// Runs the ops of a block (type xb: X check; n_ops ops) on the ancilla
// 2-vector for the block-basis input label x (ancilla starting in |0>).  The
// op source `src` gives op i (src.op(i)), the Pauli code drawn for it
// (src.code(i): 0 = none; for two-qubit locations the pair index 1..15) and,
// for a rotation, (cos beta, sin beta) of its angle beta = base + eps of its
// site (src.angle(i, op)); rotations by +-beta only flip the sine.  Returns
// the ancilla amplitudes (v0, v1) = (D_0(x), D_1(x)) before normalisation
// and the output label in *cur; false if an op is not monomial in the block
// basis.
template <class SRC>
QEC_HD bool track_ops(bool xb, int n_ops, const SRC& src, int x, cd& v0, cd& v1, uint32_t* cur_out) {
  v0 = {1.0, 0.0};
  v1 = {0.0, 0.0};
  uint32_t cur = (uint32_t)x;
  for (int i = 0; i < n_ops; ++i) {
    const TOp op = src.op(i);
    const int code = src.code(i);
    switch (op.kind) {
      case OP_ROT_ANC: {
        const cd c = src.angle(i, op);
        anc_rot_cs(op.axis, c.re, c.im * (double)op.sgn, v0, v1);
        if (code) anc_pauli(op.axis, v0, v1);  // twirled: the generator
        break;
      }
      case OP_ROT_DATA: {
        if ((xb && op.axis != 1) || (!xb && op.axis != 3)) return false;
        const double e = ((cur >> op.j) & 1) ? -1.0 : 1.0;
        const cd c = src.angle(i, op);
        const cd ph{c.re, -c.im * e * (double)op.sgn};  // exp(-i beta e sgn)
        v0 = cmul(v0, ph);
        v1 = cmul(v1, ph);
        if (code) {
          const cd g = data_pauli(op.axis, xb, op.j, cur);
          v0 = cmul(v0, g);
          v1 = cmul(v1, g);
        }
        break;
      }
      case OP_CR_AD: {
        if (!xb) return false;
        const double e = ((cur >> op.j) & 1) ? -1.0 : 1.0;
        const cd c = src.angle(i, op);
        v0 = cmul(v0, cd{c.re, -c.im * e});
        v1 = cmul(v1, cd{c.re, c.im * e});
        if (code) {  // Z on the ancilla, X on data j
          anc_pauli(3, v0, v1);
          const cd g = data_pauli(1, xb, op.j, cur);
          v0 = cmul(v0, g);
          v1 = cmul(v1, g);
        }
        break;
      }
      case OP_CR_DA: {
        if (xb) return false;
        const double e = ((cur >> op.j) & 1) ? -1.0 : 1.0;
        const cd c = src.angle(i, op);
        anc_rot_cs(1, c.re, c.im * e, v0, v1);
        if (code) {  // Z on data j, X on the ancilla
          const cd g = data_pauli(3, xb, op.j, cur);
          v0 = cmul(v0, g);
          v1 = cmul(v1, g);
          anc_pauli(1, v0, v1);
        }
        break;
      }
      case OP_H_ANC: {
        const double h = 0.70710678118654752440;
        cd a{(v0.re + v1.re) * h, (v0.im + v1.im) * h};
        cd c{(v0.re - v1.re) * h, (v0.im - v1.im) * h};
        v0 = a; v1 = c;
        break;
      }
      case OP_CNOT_AD: {
        if (!xb) return false;
        if ((cur >> op.j) & 1) v1 = {-v1.re, -v1.im};
        break;
      }
      case OP_CZ_AD: {
        if (xb) return false;
        if ((cur >> op.j) & 1) v1 = {-v1.re, -v1.im};
        break;
      }
      case OP_N1_ANC:
        anc_pauli(code, v0, v1);
        break;
      case OP_N1_DATA: {
        const cd ph = data_pauli(code, xb, op.j, cur);
        v0 = cmul(v0, ph);
        v1 = cmul(v1, ph);
        break;
      }
      case OP_N2_AD: {
        const int pj = code;
        anc_pauli(pj >> 2, v0, v1);
        const cd ph = data_pauli(pj & 3, xb, op.j, cur);
        v0 = cmul(v0, ph);
        v1 = cmul(v1, ph);
        break;
      }
      case OP_N2_DA: {
        const int pj = code;
        const cd ph = data_pauli(pj >> 2, xb, op.j, cur);
        v0 = cmul(v0, ph);
        v1 = cmul(v1, ph);
        anc_pauli(pj & 3, v0, v1);
        break;
      }
      case OP_ZZ_AD: {  // diagonal only in the computational basis of the data
        if (xb) return false;
        const double e = ((cur >> op.j) & 1) ? -1.0 : 1.0;
        const cd c = src.angle(i, op);
        v0 = cmul(v0, cd{c.re, -c.im * e});
        v1 = cmul(v1, cd{c.re, c.im * e});
        break;
      }
      default:
        return false;
    }
  }
  *cur_out = cur;
  return true;
}

// Op source of track_ops over an op array, a Pauli-code array and an angle
// accessor `cs(op)`.
template <class CS>
struct OpList {
  const TOp* ops;
  const uint8_t* pauli;
  CS cs;
  QEC_HD TOp op(int i) const { return ops[i]; }
  QEC_HD int code(int i) const { return pauli[i]; }
  QEC_HD cd angle(int, const TOp& o) const { return cs(o); }
};

// track_ops over the op list of block b with Pauli codes pauli[i].
template <class CS>
QEC_HD bool track_column(const TBlock& b, CS cs, const uint8_t* pauli, int x, cd& v0, cd& v1,
                         uint32_t* cur_out) {
  return track_ops(b.type == 0, b.n_ops, OpList<CS>{b.ops, pauli, cs}, x, v0, v1, cur_out);
}

// Builds BlockRT for one block instance from the Pauli codes of its noise
// locations.  Returns false if an op is not monomial in the block basis.
QEC_HD bool build_block(const TBlock& b, const double* eps_site, const uint8_t* pauli,
                        BlockRT& out) {
  const bool xb = (b.type == 0);
  const int n = 1 << b.w;
  const double norm = xb ? 1.0 / (double)n : 1.0;
  uint32_t F = 0;
  for (int x = 0; x < n; ++x) {
    cd v0, v1;
    uint32_t cur = 0;
    if (!track_column(b, CsFromEps{eps_site}, pauli, x, v0, v1, &cur)) return false;
    F = cur ^ (uint32_t)x;
    out.D[0][x][0] = v0.re * norm;
    out.D[0][x][1] = v0.im * norm;
    out.D[1][x][0] = v1.re * norm;
    out.D[1][x][1] = v1.im * norm;
    out.W[0][x] = (v0.re * v0.re + v0.im * v0.im) * norm;
    out.W[1][x] = (v1.re * v1.re + v1.im * v1.im) * norm;
  }
  for (int x = n; x < 16; ++x) {
    out.D[0][x][0] = out.D[0][x][1] = out.D[1][x][0] = out.D[1][x][1] = 0.0;
    out.W[0][x] = out.W[1][x] = 0.0;
  }
  out.F = F;
  return true;
}

// ---- dense Kraus pairs (blocks that are not monomial in their basis) ------
// The circuit's ops on the 32-amplitude register of the ancilla (bit 4) and
// the block's data qubits (bits 0..3, bit l = block qubit l), computational
// basis.
QEC_HD void dn_gate1(cd* psi, uint32_t mask, cd m00, cd m01, cd m10, cd m11) {
  for (uint32_t i = 0; i < 32; ++i) {
    if (i & mask) continue;
    const cd a = psi[i], b = psi[i | mask];
    psi[i] = cd{m00.re * a.re - m00.im * a.im + m01.re * b.re - m01.im * b.im,
                m00.re * a.im + m00.im * a.re + m01.re * b.im + m01.im * b.re};
    psi[i | mask] = cd{m10.re * a.re - m10.im * a.im + m11.re * b.re - m11.im * b.im,
                       m10.re * a.im + m10.im * a.re + m11.re * b.im + m11.im * b.re};
  }
}

// exp(-i theta P) (P = 1 X, 2 Y, 3 Z) with c = cos theta, s = sin theta.
QEC_HD void dn_rot(cd* psi, uint32_t mask, int axis, double c, double s) {
  if (axis == 1) dn_gate1(psi, mask, {c, 0}, {0, -s}, {0, -s}, {c, 0});
  else if (axis == 2) dn_gate1(psi, mask, {c, 0}, {-s, 0}, {s, 0}, {c, 0});
  else dn_gate1(psi, mask, {c, -s}, {0, 0}, {0, 0}, {c, s});
}

// Pauli P (1 X, 2 Y = [[0,-i],[i,0]], 3 Z).
QEC_HD void dn_pauli(cd* psi, uint32_t mask, int P) {
  if (P == 1) dn_gate1(psi, mask, {0, 0}, {1, 0}, {1, 0}, {0, 0});
  else if (P == 2) dn_gate1(psi, mask, {0, 0}, {0, -1}, {0, 1}, {0, 0});
  else if (P == 3) dn_gate1(psi, mask, {1, 0}, {0, 0}, {0, 0}, {-1, 0});
}

// exp(-i theta Z_c X_t): on qubit t, [[c, -i z s], [-i z s, c]] with z = +-1
// the eigenvalue of Z_c.
QEC_HD void dn_zx(cd* psi, uint32_t cmask, uint32_t tmask, double c, double s) {
  for (uint32_t i = 0; i < 32; ++i) {
    if (i & tmask) continue;
    const double z = (i & cmask) ? -1.0 : 1.0;
    const cd a = psi[i], b = psi[i | tmask];
    // c a - i z s b,  -i z s a + c b
    psi[i] = cd{c * a.re + z * s * b.im, c * a.im - z * s * b.re};
    psi[i | tmask] = cd{z * s * a.im + c * b.re, -z * s * a.re + c * b.im};
  }
}

// Column x of the dense Kraus pair: runs the block's ops on |anc 0, data x>
// and returns the final 32 amplitudes (ancilla bit 4).  Returns false for an
// op kind it does not know.
template <typename CS>
QEC_HD bool dense_column(const TBlock& b, CS cs, const uint8_t* pauli, int x, cd* psi) {
  for (int i = 0; i < 32; ++i) psi[i] = {0.0, 0.0};
  psi[x] = {1.0, 0.0};
  const uint32_t A = 16u;
  for (int i = 0; i < b.n_ops; ++i) {
    const TOp& op = b.ops[i];
    const uint32_t Q = 1u << op.j;
    switch (op.kind) {
      case OP_ROT_ANC: {
        const cd c = cs(op);
        dn_rot(psi, A, op.axis, c.re, c.im * (double)op.sgn);
        if (pauli[i]) dn_pauli(psi, A, op.axis);
        break;
      }
      case OP_ROT_DATA: {
        const cd c = cs(op);
        dn_rot(psi, Q, op.axis, c.re, c.im * (double)op.sgn);
        if (pauli[i]) dn_pauli(psi, Q, op.axis);
        break;
      }
      case OP_CR_AD: {
        const cd c = cs(op);
        dn_zx(psi, A, Q, c.re, c.im);
        if (pauli[i]) { dn_pauli(psi, A, 3); dn_pauli(psi, Q, 1); }
        break;
      }
      case OP_CR_DA: {
        const cd c = cs(op);
        dn_zx(psi, Q, A, c.re, c.im);
        if (pauli[i]) { dn_pauli(psi, Q, 3); dn_pauli(psi, A, 1); }
        break;
      }
      case OP_H_ANC: {
        const double h = 0.70710678118654752440;
        dn_gate1(psi, A, {h, 0}, {h, 0}, {h, 0}, {-h, 0});
        break;
      }
      case OP_CNOT_AD:
        for (uint32_t k = 0; k < 32; ++k)
          if ((k & A) && !(k & Q)) { const cd t = psi[k]; psi[k] = psi[k | Q]; psi[k | Q] = t; }
        break;
      case OP_CZ_AD:
        for (uint32_t k = 0; k < 32; ++k)
          if ((k & A) && (k & Q)) psi[k] = {-psi[k].re, -psi[k].im};
        break;
      case OP_N1_ANC:
        dn_pauli(psi, A, pauli[i]);
        break;
      case OP_N1_DATA:
        dn_pauli(psi, Q, pauli[i]);
        break;
      case OP_N2_AD:
        dn_pauli(psi, A, pauli[i] >> 2);
        dn_pauli(psi, Q, pauli[i] & 3);
        break;
      case OP_N2_DA:
        dn_pauli(psi, Q, pauli[i] >> 2);
        dn_pauli(psi, A, pauli[i] & 3);
        break;
      case OP_ZZ_AD: {
        const cd c = cs(op);
        for (uint32_t k = 0; k < 32; ++k) {
          const double z = (((k >> 4) ^ (k >> op.j)) & 1) ? -1.0 : 1.0;  // Z_anc Z_j eigenvalue
          psi[k] = cmul(psi[k], cd{c.re, -c.im * z});
        }
        break;
      }
      default:
        return false;
    }
  }
  return true;
}

// Draws of one block instance: Pauli choices per op (for a twirled rotation:
// 1 if its generator is applied, u < twirl_thr[site] = sin^2 eps),
// measurement uniform.
QEC_HD void draw_block(const TBlock& b, uint64_t seed, uint64_t t, uint64_t k0, double p,
                       uint8_t* pauli, double* u_meas, const double* twirl_thr = nullptr) {
  for (int i = 0; i < b.n_ops; ++i) {
    const TOp& op = b.ops[i];
    pauli[i] = 0;
    if (op.draw < 0) continue;
    const double u = uniform(seed, t, k0 + (uint64_t)op.draw);
    if (is_rotation(op.kind))
      pauli[i] = (uint8_t)(twirl_thr && u < twirl_thr[op.site] ? 1 : 0);
    else if (op.kind == OP_N1_ANC || op.kind == OP_N1_DATA)
      pauli[i] = (uint8_t)pick_pauli1(u, p);
    else
      pauli[i] = (uint8_t)pick_pauli2(u, p);
  }
  *u_meas = uniform(seed, t, k0 + (uint64_t)(b.n_draws - 1));
}

// Longest chain of Z checks one register pass applies or sums, and the sums
// of a full chain (every outcome prefix: 2^(L+1) - 2).
constexpr int kChainMax = 6;
constexpr int kChainAcc = (2 << kChainMax) - 2;

struct JobConst {
  int d;
  int n;               // data qubits
  int n_x;             // X stabilizers (rank of the X-support span)
  int n_edges;         // ZZ pairs
  uint32_t hmask, vmask;
  double amp0;         // 2^(-n_x/2)
  uint32_t span_vec[16];   // echelon basis of the X supports
  uint32_t span_piv[16];   // pivot bit of each basis vector
  double zz[2 * 64];       // exp(-i zeta (|E| - 2k)), k = 0..|E|
  int use_zz;
  int init_plus;           // 1: the first pass writes logical |+> (X-basis memory)
  // L consecutive ZZ layers: exp(-i zeta (L |E| - 2K)), K = 0..L|E|, L = 1..kChainMax
  double zzl[kChainMax][2 * (kChainMax * 40 + 1)];
  int n_zc;                // Z checks
  uint32_t zc_mask[16];    // data bits of each Z check
};

// Outcome of one pass unit (a single check, or a chain of Z checks: bit i of
// m is the outcome of chain member i), the norm^2 of the kept branch, and the
// register's Pauli-X frame before the unit is applied (see UnitPass).
struct Decision {
  double Sm;
  int m;
  uint32_t phi;
};

// ------------------------------------------------------------ pass units --
// The trajectory engine runs one HBM pass per "unit": a single X check, or a
// chain of up to kChainMax (six) consecutive Z checks.  Z checks are monomial in the
// computational basis (diag(D_m), then an XOR permutation by F), so a chain is
// pointwise on the amplitude index: its S_m for every prefix of outcomes
// (a binary tree of 2^(L+1) - 2 sums) comes out of one read of the register,
// and the next pass applies the whole decided chain.  The XOR permutations are
// never carried out in memory: the register is kept in a Pauli-X frame phi,
// physical index p holding logical amplitude p ^ phi.  A Z check then rewrites
// every amplitude in place and updates phi; an X check commutes with the frame
// up to the global sign (-1)^{popcount(phi_b & F)} (phi_b: phi on the check's
// qubits); S_m of an X check does not depend on phi; the final measurement
// reads logical bit q as physical bit q ^ phi_q.
// Two consecutive X checks can also form one unit (U_XP, a pair): the pass
// that sums the pair evaluates the first member's S_m and, for each outcome m
// of the first member, the second member's sums after the first member's
// Kraus operator for m and its ZZ layer (six sums laid out as a chain of two:
// index 2 + m0 + 2 m1 for the second member); the next pass applies both.
// A pair's members may have weight 2 or 4: a weight-2 member is handled as a
// 16-element group over four register slots (its two qubits and two others)
// with its tables repeated over the other two bits and divided by 4.
// Speculative units (the single-register trajectory, Sec. III.B): a unit
// whose outcomes are predicted (the same check's outcome one round earlier,
// the trivial outcome in the first round) is summed and applied in the same
// pass, which writes the other of two register buffers.  An X check or pair
// is summed along the predicted outcomes (its first member's S_0, S_1, then
// the second member's after the first member's predicted Kraus operator and
// ZZ layer: index 2 l + m for member l); a Z chain is summed over every
// outcome string as a B unit is, after a U_SC "unit" that only applies the
// pending renormalisation.  The decision confirms the members in order; at
// the first member whose drawn outcome differs from the one applied it fixes
// that outcome and has the pass run again from the untouched input (a redo).
// Applied outcomes are never wrong in the register the next unit reads.
enum : int { U_NONE = 0, U_X = 1, U_Z = 2, U_INIT = 3, U_XP = 4, U_SC = 5 };

// Control record of one speculative unit instance: m, the outcome bits the
// last pass applied (bit l: member l); the members below `known` are decided;
// run = 1 while a redo is due.  The prediction pass writes it, the decision
// updates it, a redo reads it.
struct SpecCtl {
  int m;
  int known;
  int run;
  int pad;
};
// Sums a pass leaves for the decision of a unit of len members: every outcome
// prefix (2^(len+1) - 2: an X check 2, a pair or a chain of two 6), or for a
// chain of three or more only its last level (2^len; the prefixes are its
// marginals, each member's outcome weights adding up to one).
__host__ __device__ constexpr int unit_sums(int len) { return len >= 3 ? (1 << len) : (2 << len) - 2; }

// Layout and unit description of one pass: apply unit A (decided), accumulate
// the sums of unit B.  Tiles of 2^tb amplitudes; a thread owns 16 amplitudes
// (register slot j) at a time.  Phase 1 (apply A) uses layout 1, whose slot
// bits are A's qubits for an X check, or for a Z chain bits outside A's qubits
// where possible (then the chain's factor is the same for the thread's 16
// amplitudes: amode = 1).  Phase 2 (sums of B) either stays in layout 1
// (bmode 1: an X check B whose qubits are the slot bits, or a Z chain B whose
// qubits avoid the slot bits, summed once per thread), regroups the tile
// through LDS into layout 2 (bmode 2: slot bits = B's qubits for an X check,
// bits outside B's qubits for a Z chain), or evaluates a Z chain amplitude by
// amplitude in layout 1 (bmode 0, when no 4 tile bits avoid B's qubits).
struct UnitPass {
  int tb, n_outer;
  int akind, la, wa;       // A: U_INIT / U_X / U_Z / U_XP, members, X weight (first member)
  int bkind, lb, wb;       // B: U_NONE / U_X / U_Z / U_XP
  int amode, bmode;
  uint32_t outer_bit[32];
  // LDS slots (tid_l, j_l, b_tid_l, b_j_l) are already swizzled: the slot of
  // a thread's value is the XOR of its thread-index bits' and its slot's entries
  uint32_t tid_g[8], tid_l[8];     // layout 1: global bit / LDS slot of each thread-index bit
  uint32_t j_g[16], j_l[16];       // layout 1: global bits / LDS slot of register slot j
  uint32_t b_tid_g[8], b_tid_l[8];  // layout 2
  uint32_t b_j_l[16];
  uint32_t b_j_g[16];               // layout 2: global bits of slot j (host checks)
  // X pairs: layout of the second member's register slots, [0] for an A
  // pair (the tile goes layout 1 -> p[0] -> layout 1), [1] for a B pair
  // (layout 2 holds B's first member, p[1] its second)
  uint32_t p_tid_g[2][8], p_tid_l[2][8], p_j_g[2][16], p_j_l[2][16];
  // amix = 1: X check A on bit 0 or 1 keeps its qubits below bit 4 on the
  // lanes (so lanes still run over the lowest bits) and the others in the low
  // amix_r register slots; its local index is the XOR of a_tx[i] over the
  // thread's index bits i and a_jx[j] of register slot j; amix_lanes: the
  // lane bits (0..3) that carry qubits of A
  int amix, amix_r, amix_lanes, pad_amix;
  int adense, bdense;  // the X check A / B has a dense Kraus pair (BlockDense)
  // an X pair A with no B: the tile is stored from layout p[0] (its lanes
  // keep the three lowest bits: runs of at least 8 amplitudes), not
  // regrouped back to layout 1 first
  int pstore, pad_pstore;
  uint32_t a_tx[8], a_jx[16];
  uint32_t aq[kChainMax][4];     // global bit of local bit l of A's member i
  uint32_t bq[kChainMax][4];
  int aw[kChainMax], bw[kChainMax];
  uint32_t a_j_loc[kChainMax][16];  // member-i local index carried by slot j's bits (layout 1)
  uint32_t b_j_loc[kChainMax][16];
};

}  // namespace qec
