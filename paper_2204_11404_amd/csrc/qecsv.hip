// qecsv host runtime and C ABI (see include/qecsv.h).
//
// Host side of the trajectory engine: the code layout of Sec. II.A (Table I
// order, CNOT slot order, boundary waits), the encoded stabilizer-circuit
// template of Sec. III.A (cross-resonance or textbook gate set, noise
// locations, over-rotation sites), the units and tile descriptors of the
// register passes, the launch sequence of one trajectory (Sec. III.B), the
// batched and served runs, the launch-parameter table and the decoder.  All
// simulation arithmetic runs in the kernels of kernels.hip and
// kernels_batch.hip.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "qecsv.h"
#include "qec_common.h"
#include "kernels.hip"
#include "kernels_ops.hip"
#include "kernels_batch.hip"

using namespace qec;

namespace {

thread_local std::string g_err;

sv_status fail(sv_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(SV_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define SV_OK_OR_RETURN(expr)                \
  do {                                       \
    const sv_status s_ = (expr);             \
    if (s_ != SV_OK) return s_;              \
  } while (0)

// Device buffers for one call, allocated and released in stream order from
// the device's default pool (no device-wide synchronisation, memory is reused
// across calls).
void keep_pool_memory(int dev) {
  static std::once_flag once[64];
  if (dev < 0 || dev >= 64) return;
  std::call_once(once[dev], [dev] {
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
      uint64_t keep = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
  });
}

struct DevBufs {
  hipStream_t s;
  std::vector<void*> ptrs;
  explicit DevBufs(hipStream_t stream) : s(stream) {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) keep_pool_memory(dev);
  }
  ~DevBufs() {
    for (void* p : ptrs) (void)hipFreeAsync(p, s);
  }
  template <typename P>
  hipError_t alloc(P** out, size_t bytes) {
    void* p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes ? bytes : 16, s);
    if (e == hipSuccess) {
      ptrs.push_back(p);
      *out = reinterpret_cast<P*>(p);
    }
    return e;
  }
};

// --------------------------------------------------------------- layout --
struct Stab {
  int type;     // 0 X, 1 Z
  int slot[4];  // data labels 1..d^2 in CNOT order, 0 = wait
};

// Rotated surface code of distance d.  Faces sit between data rows r, r+1
// and columns c, c+1 for r, c in -1..d-1; a face is X-type when r + c is odd.
// Interior faces have four data qubits; the weight-2 faces kept on the border
// are X-type on the top/bottom edges and Z-type on the left/right edges.  X
// faces are measured in row-major order, Z faces column by column from the
// bottom row up (Table I).  CNOT slots: X faces bottom-right, bottom-left,
// top-left, top-right; Z faces top-right, bottom-right, bottom-left,
// top-left (Sec. II.A).
std::vector<Stab> code_layout(int d) {
  auto q = [d](int row, int col) -> int {
    if (row < 0 || col < 0 || row >= d || col >= d) return 0;
    return row * d + col + 1;
  };
  std::vector<Stab> out;
  // X faces, row-major
  for (int r = -1; r < d; ++r)
    for (int c = -1; c < d; ++c) {
      if (((r + c) & 1) == 0) continue;
      const bool interior = r >= 0 && c >= 0 && r < d - 1 && c < d - 1;
      const bool edge = (r == -1 || r == d - 1) && c >= 0 && c < d - 1;
      if (!interior && !edge) continue;
      out.push_back({0, {q(r + 1, c + 1), q(r + 1, c), q(r, c), q(r, c + 1)}});
    }
  // Z faces, by column, bottom row first
  for (int c = -1; c < d; ++c)
    for (int r = d - 1; r >= -1; --r) {
      if ((r + c) & 1) continue;
      const bool interior = r >= 0 && c >= 0 && r < d - 1 && c < d - 1;
      const bool edge = (c == -1 || c == d - 1) && r >= 0 && r < d - 1;
      if (!interior && !edge) continue;
      out.push_back({1, {q(r, c + 1), q(r + 1, c + 1), q(r + 1, c), q(r, c)}});
    }
  return out;
}

// ------------------------------------------------------------- template --
struct Template {
  std::vector<TBlock> blocks;
  int n_sites = 0;   // gate sites of the round (the per-site over-rotation table)
  int n_draws = 0;
  int zz_site = -1;  // >= 0: angle-table entry n_sites holds the per-step crosstalk zeta
  bool any_dense = false;
};

struct OpSink {
  TBlock& b;
  int site_base;
  bool twirl;  // rotations draw their twirled over-rotation
  bool vz;     // Rz restores are virtual: exact, no draw
  int sites = 0;
  int draws = 0;
  // The largest block (cross-resonance X check of weight 4 with idle noise,
  // twirled rotations and per-step crosstalk) needs 60 ops and 36 noise draws:
  // within kMaxOps and the 64-bit n2mask for every template the builder makes.
  TOp& next() {
    if (b.n_ops >= kMaxOps || draws >= 63) {
      std::fprintf(stderr, "qecsv: block template exceeds kMaxOps\n");
      std::abort();
    }
    return b.ops[b.n_ops++];
  }
  void gate(uint8_t kind, int j, int axis, int sgn, int quarter) {
    TOp& o = next();
    o = TOp{};
    o.kind = kind; o.j = (uint8_t)j; o.axis = (uint8_t)axis; o.sgn = (int8_t)sgn;
    o.quarter = (uint8_t)quarter;
    o.site = (int16_t)(site_base + sites++);
    o.exact = (uint8_t)(vz && kind == OP_ROT_DATA && axis == 3);
    o.draw = (twirl && !o.exact) ? (int16_t)draws++ : (int16_t)-1;
  }
  void plain(uint8_t kind, int j) {
    TOp& o = next();
    o = TOp{};
    o.kind = kind; o.j = (uint8_t)j; o.site = -1; o.draw = -1;
  }
  // exp(-i zeta Z_anc Z_j); its angle is the angle-table entry zz_site
  void zz(int j, int zz_site) {
    TOp& o = next();
    o = TOp{};
    o.kind = OP_ZZ_AD; o.j = (uint8_t)j; o.site = (int16_t)zz_site; o.draw = -1;
  }
  void noise(uint8_t kind, int j) {
    TOp& o = next();
    o = TOp{};
    o.kind = kind; o.j = (uint8_t)j; o.site = -1;
    if (kind == OP_N2_AD || kind == OP_N2_DA) b.n2mask |= 1ull << draws;
    o.draw = (int16_t)draws++;
  }
};

// twirl: Pauli-twirled over-rotations -- each rotation by its base angle,
// then one draw deciding whether its generator is applied (probability
// sin^2 eps of its site), drawn right after the rotation.
// vz: the Rz restores of the cross-resonance Z checks are virtual Z gates
// (frame changes, Fig. 4): no over-rotation; their sites stay in the table.
// idle: the one-qubit channel also acts on the waiting qubits of each step
// (Sec. III.A): after a step, N1 on every data qubit of the check that the
// step leaves alone, in slot order; the ancilla waits during the Z check's
// restores.
// zzp: after each step (after its noise), the crosstalk exp(-i zeta Z_anc Z_q)
// between the ancilla and every data qubit of the check; its angle sits in
// the angle table after the n_sites gate sites.  X checks then stop being
// monomial in their Hadamard basis and get dense Kraus pairs.
Template build_template(int d, int gateset, bool twirl = false, bool vz = false, bool idle = false,
                        bool zzp = false) {
  Template T;
  if (zzp)  // the crosstalk entry follows every gate site
    T.zz_site = build_template(d, gateset, twirl, vz, idle, false).n_sites;
  for (const Stab& st : code_layout(d)) {
    TBlock b{};
    b.type = st.type;
    b.w = 0;
    int local[4];
    for (int s = 0; s < 4; ++s) {
      local[s] = -1;
      if (st.slot[s]) {
        local[s] = b.w;
        b.qubit[b.w++] = st.slot[s] - 1;
      }
    }
    b.draw_off = T.n_draws;
    b.site_off = T.n_sites;
    OpSink o{b, T.n_sites, twirl, vz};
    auto waiting = [&](int busy_slot) {  // end of a step: idle data qubits, crosstalk
      if (idle && busy_slot != -2)
        for (int s = 0; s < 4; ++s)
          if (local[s] >= 0 && s != busy_slot) o.noise(OP_N1_DATA, local[s]);
      if (zzp)
        for (int l = 0; l < b.w; ++l) o.zz(l, T.zz_site);
    };
    if (gateset == SV_GATESET_CR) {
      if (st.type == 0) {
        o.gate(OP_ROT_ANC, 0, 1, -1, 1);  // Rx^dag(pi/2)
        o.noise(OP_N1_ANC, 0);
        waiting(-1);
        for (int s = 0; s < 4; ++s) {
          if (local[s] >= 0) {
            o.gate(OP_CR_AD, local[s], 0, 1, 1);
            o.noise(OP_N2_AD, local[s]);
          } else {
            o.noise(OP_N1_ANC, 0);  // wait
          }
          waiting(s);
        }
        o.gate(OP_ROT_ANC, 0, 1, 1, 1);  // Rx(pi/2)
        o.noise(OP_N1_ANC, 0);
        for (int l = 0; l < b.w; ++l) {
          o.gate(OP_ROT_DATA, l, 1, 1, 1);  // restoring Rx(pi/2) on data
          o.noise(OP_N1_DATA, l);
        }
        waiting(-2);  // nobody waits in this step
      } else {
        for (int s = 0; s < 4; ++s) {
          if (local[s] >= 0) {
            o.gate(OP_CR_DA, local[s], 0, 1, 1);
            o.noise(OP_N2_DA, local[s]);
          } else {
            o.noise(OP_N1_ANC, 0);
          }
          waiting(s);
        }
        for (int l = 0; l < b.w; ++l) {
          o.gate(OP_ROT_DATA, l, 3, 1, 1);  // restoring Rz(pi/2) on data
          o.noise(OP_N1_DATA, l);
        }
        if (idle) o.noise(OP_N1_ANC, 0);  // the ancilla waits during the restores
        waiting(-2);
      }
    } else {
      o.plain(OP_H_ANC, 0);
      o.gate(OP_ROT_ANC, 0, 1, 1, 0);  // coherent error exp(-i eps X) after H
      o.noise(OP_N1_ANC, 0);
      waiting(-1);
      for (int s = 0; s < 4; ++s) {
        if (local[s] < 0) continue;
        o.plain(st.type == 0 ? OP_CNOT_AD : OP_CZ_AD, local[s]);
        o.noise(OP_N2_AD, local[s]);
        waiting(s);
      }
      o.plain(OP_H_ANC, 0);
      o.gate(OP_ROT_ANC, 0, 1, 1, 0);
      o.noise(OP_N1_ANC, 0);
      waiting(-1);
    }
    b.n_draws = o.draws + 1;  // + measurement
    T.n_sites += o.sites;
    T.n_draws += b.n_draws;
    // not monomial in the block basis (an X check with crosstalk): dense Kraus pair
    {
      const std::vector<double> zero(T.zz_site + 2 + T.n_sites, 0.0);
      const uint8_t none[kMaxOps] = {};
      cd v0, v1;
      uint32_t cur = 0;
      b.dense = track_column(b, CsFromEps{zero.data()}, none, 0, v0, v1, &cur) ? 0 : 1;
      T.any_dense = T.any_dense || b.dense;
    }
    T.blocks.push_back(b);
  }
  return T;
}

// ------------------------------------------------------- job constants --
JobConst make_job_const(int d, double zeta, bool init_plus = false) {
  JobConst jc{};
  jc.d = d;
  jc.n = d * d;
  jc.init_plus = init_plus ? 1 : 0;
  for (const Stab& st : code_layout(d)) {
    if (st.type != 1) continue;
    uint32_t m = 0;
    for (int q : st.slot)
      if (q) m |= 1u << (q - 1);
    jc.zc_mask[jc.n_zc++] = m;
  }
  // reduced echelon basis of the X-stabilizer supports over GF(2)
  std::vector<uint32_t> basis;
  for (const Stab& st : code_layout(d)) {
    if (st.type != 0) continue;
    uint32_t v = 0;
    for (int s = 0; s < 4; ++s)
      if (st.slot[s]) v |= 1u << (st.slot[s] - 1);
    for (uint32_t bv : basis) {
      const uint32_t piv = 1u << (31 - __builtin_clz(bv));
      if (v & piv) v ^= bv;
    }
    if (!v) continue;
    const uint32_t piv = 1u << (31 - __builtin_clz(v));
    for (uint32_t& bv : basis)
      if (bv & piv) bv ^= v;
    basis.push_back(v);
  }
  jc.n_x = (int)basis.size();
  for (int i = 0; i < jc.n_x; ++i) {
    jc.span_vec[i] = basis[i];
    jc.span_piv[i] = 1u << (31 - __builtin_clz(basis[i]));
  }
  // logical |0>: 2^n_x strings of the X-stabilizer orbit of 0; logical |+>:
  // the 2^(n - n_z) strings with even parity on every Z check
  jc.amp0 = init_plus ? std::pow(2.0, -0.5 * (d * d - jc.n_zc)) : std::pow(2.0, -0.5 * jc.n_x);
  uint32_t hm = 0, vm = 0;
  int ne = 0;
  for (int i = 0; i < d * d; ++i) {
    if (i % d != d - 1) { hm |= 1u << i; ++ne; }
    if (i + d < d * d) { vm |= 1u << i; ++ne; }
  }
  jc.hmask = hm;
  jc.vmask = vm;
  jc.n_edges = ne;
  for (int k = 0; k <= ne; ++k) {
    const double th = -zeta * (double)(ne - 2 * k);
    jc.zz[2 * k] = std::cos(th);
    jc.zz[2 * k + 1] = std::sin(th);
  }
  jc.use_zz = zeta != 0.0;
  for (int L = 1; L <= kChainMax; ++L)
    for (int k = 0; k <= L * ne; ++k) {
      const double th = -zeta * (double)(L * ne - 2 * k);
      jc.zzl[L - 1][2 * k] = std::cos(th);
      jc.zzl[L - 1][2 * k + 1] = std::sin(th);
    }
  return jc;
}

// ------------------------------------------------------------ pass units --
struct Unit {
  int kind;   // U_X or U_Z
  int first;  // template index of the first member
  int len;    // members (1 for an X check)
};

// ---------------------------------------------------------------- tuning --
// Launch parameters per (device, d, dtype): built-in defaults, replaced by
// values set with sv_tuning_set or found by sv_autotune, in turn overridden by
// the QECSV_* environment variables.  None of them changes what is computed
// beyond the order of floating-point sums.
struct TuneKey {
  int dev, d, dtype;
  bool operator<(const TuneKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (d != o.d) return d < o.d;
    return dtype < o.dtype;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, sv_tuning> g_tune;

sv_tuning default_tuning() {
  sv_tuning t{};
  t.zchain = 4;  // chains of five or six: the autotuner's choice
  t.snake = 1;
  t.batch_waves_per_cu = 8;
  t.lockstep_mib = 4096;
  t.pass_wgs_per_cu = 0;
  t.xpair = 0;
  return t;
}

int current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  return dev;
}

sv_status check_tuning(const sv_tuning& t) {
  if (t.zchain < 1 || t.zchain > kChainMax) return fail(SV_EINVAL, "zchain %d out of 1..%d", t.zchain, kChainMax);
  if (t.snake != 0 && t.snake != 1) return fail(SV_EINVAL, "snake must be 0 or 1");
  if (t.batch_waves_per_cu < 1 || t.batch_waves_per_cu > 32)
    return fail(SV_EINVAL, "batch_waves_per_cu %d out of 1..32", t.batch_waves_per_cu);
  if (t.lockstep_mib < 1 || t.lockstep_mib > (1 << 20)) return fail(SV_EINVAL, "lockstep_mib out of range");
  if (t.pass_wgs_per_cu < 0 || t.pass_wgs_per_cu > 64) return fail(SV_EINVAL, "pass_wgs_per_cu out of 0..64");
  if (t.xpair != 0 && t.xpair != 1) return fail(SV_EINVAL, "xpair must be 0 or 1");
  return SV_OK;
}

int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

sv_tuning tuning_for(int d, int dtype) {
  sv_tuning t = default_tuning();
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(TuneKey{current_device(), d, dtype});
    if (it != g_tune.end()) t = it->second;
  }
  if (const char* e = std::getenv("QECSV_ZCHAIN")) t.zchain = std::max(1, std::min(kChainMax, std::atoi(e)));
  if (const char* e = std::getenv("QECSV_SNAKE")) t.snake = std::atoi(e) != 0;
  if (const char* e = std::getenv("QECSV_BATCH_WAVES_PER_CU")) t.batch_waves_per_cu = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("QECSV_LOCKSTEP_MIB")) t.lockstep_mib = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("QECSV_PASS_WGS_PER_CU"))
    t.pass_wgs_per_cu = std::max(0, std::min(64, std::atoi(e)));
  if (const char* e = std::getenv("QECSV_XPAIR")) t.xpair = std::atoi(e) != 0;
  return t;
}

// Units of one round: every X check alone, runs of consecutive Z checks cut
// into chains of at most max_chain members.
std::vector<Unit> make_units(const Template& tp, int max_chain) {
  std::vector<Unit> u;
  for (int s = 0; s < (int)tp.blocks.size(); ++s) {
    if (tp.blocks[s].type == 0)
      u.push_back({U_X, s, 1});
    else if (!u.empty() && u.back().kind == U_Z && u.back().len < max_chain &&
             u.back().first + u.back().len == s)
      u.back().len++;
    else
      u.push_back({U_Z, s, 1});
  }
  return u;
}

// Pass descriptor: apply unit A (nullptr: write logical |0>), sum unit B
// (nullptr: none).  Slot bits of a layout: an X check's qubits (then further
// bits as needed), or four bits outside the qubits of the chain(s) to be
// evaluated per thread, taken from bit tb - 4 upwards so that the
// thread-index bits are the lowest tile bits (coalesced runs).  The tile
// holds both layouts' slot bits and then the lowest remaining bits.
UnitPass make_unit_pass(int n, int tb_max, const Template& tp, const Unit* A, const Unit* B,
                        bool* fits = nullptr) {
  UnitPass pd{};
  const int tb = std::min(tb_max, n);
  pd.tb = tb;
  pd.akind = A ? A->kind : U_INIT;
  pd.la = A ? A->len : 0;
  pd.bkind = B ? B->kind : U_NONE;
  pd.lb = B ? B->len : 0;
  const bool apair = A && A->kind == U_XP, bpair = B && B->kind == U_XP;
  const bool pairpass = apair || bpair;
  pd.wa = (A && (A->kind == U_X || apair)) ? tp.blocks[A->first].w : 0;
  pd.wb = (B && (B->kind == U_X || bpair)) ? tp.blocks[B->first].w : 0;
  auto members = [&](const Unit* U, uint32_t (*q)[4], int* w) {
    if (!U) return;
    for (int i = 0; i < U->len; ++i) {
      const TBlock& b = tp.blocks[U->first + i];
      w[i] = b.w;
      for (int l = 0; l < b.w; ++l) q[i][l] = 1u << b.qubit[l];
    }
  };
  members(A, pd.aq, pd.aw);
  members(B, pd.bq, pd.bw);
  auto xqubits = [&](const Unit* U, int i = 0) {  // qubits of X member i
    std::vector<int> qs;
    const TBlock& b = tp.blocks[U->first + i];
    for (int l = 0; l < b.w; ++l) qs.push_back(b.qubit[l]);
    return qs;
  };
  auto umask = [&](const Unit* U) {  // union of a unit's qubits
    uint32_t m = 0;
    if (U)
      for (int i = 0; i < U->len; ++i)
        for (int l = 0; l < tp.blocks[U->first + i].w; ++l) m |= 1u << tp.blocks[U->first + i].qubit[l];
    return m;
  };
  const uint32_t UA = (A && A->kind == U_Z) ? umask(A) : 0u;
  const uint32_t UB = (B && B->kind == U_Z) ? umask(B) : 0u;
  // `fixed` first, then bits outside `avoid` until 4 bits: upward from just
  // above the thread-index bits, then downward below them, so that the lowest
  // bits stay with the lanes (contiguous runs per load) as long as possible;
  // false if there are not enough such bits
  auto slots = [&](std::vector<int> fixed, uint32_t avoid, std::vector<int>& out) {
    out = fixed;
    uint32_t used = avoid;
    for (int q : fixed) used |= 1u << q;
    for (int k = 0; k < n && (int)out.size() < 4; ++k) {
      const int bit = k < n - (tb - 4) ? tb - 4 + k : n - 1 - k;
      if (!((used >> bit) & 1)) { out.push_back(bit); used |= 1u << bit; }
    }
    return (int)out.size() == 4;
  };
  auto disjoint = [](const std::vector<int>& qs, uint32_t m) {
    for (int q : qs) if ((m >> q) & 1) return false;
    return true;
  };
  auto jmask_of = [](const std::vector<int>& J) {
    uint32_t m = 0;
    for (int q : J) m |= 1u << q;
    return m;
  };
  // passes with an X pair: the qubits of every X member of A and B, where the
  // fillers of the layouts' slots are taken first (from bit 4 upward, then
  // below bit 4 unless avoided) so that the tile stays small and keeps the
  // lowest bits for the lanes; then as `slots`
  uint32_t UX = 0;
  if (pairpass) {
    for (const Unit* U : {A, B})
      if (U && (U->kind == U_X || U->kind == U_XP))
        for (int i = 0; i < U->len; ++i)
          for (int q : xqubits(U, i)) UX |= 1u << q;
  }
  auto pslots = [&](std::vector<int> fixed, uint32_t avoid, uint32_t low_ok, std::vector<int>& out) {
    out = fixed;
    uint32_t used = avoid;
    for (int q : fixed) used |= 1u << q;
    for (int pass = 0; pass < 2; ++pass)
      for (int bit = 0; bit < n && (int)out.size() < 4; ++bit) {
        const bool low = bit < 4;
        if (pass == 0 ? low : !(low && ((low_ok >> bit) & 1))) continue;
        if (((UX >> bit) & 1) && !((used >> bit) & 1)) {
          out.push_back(bit);
          used |= 1u << bit;
        }
      }
    for (int k = 0; k < n && (int)out.size() < 4; ++k) {
      const int bit = k < n - (tb - 4) ? tb - 4 + k : n - 1 - k;
      if (!((used >> bit) & 1)) { out.push_back(bit); used |= 1u << bit; }
    }
    return (int)out.size() == 4;
  };
  std::vector<int> J1, J2, Jp[2];
  bool have2 = false;
  pd.amode = 0;
  pd.bmode = 0;
  const bool ax = A && (A->kind == U_X || apair), az = A && A->kind == U_Z;
  const bool bx = B && (B->kind == U_X || bpair), bz = B && B->kind == U_Z;
  // an X check's qubits serve as layout-1 slot bits only if that keeps the
  // four lowest bits for the thread index (runs of >= 256 bytes)
  const bool bx_high = bx && disjoint(xqubits(B), 0xFu);
  pd.amix = 0;
  pd.adense = ax && tp.blocks[A->first].dense;
  pd.bdense = bx && tp.blocks[B->first].dense;
  std::vector<int> a_high;  // amix: A's qubits held in register slots
  if (ax && pairpass) {
    uint32_t am = 0;
    for (int q : xqubits(A)) am |= 1u << q;
    if ((am & 0x3u) && tb >= 8) {
      for (int q : xqubits(A))
        if (q >= 4) a_high.push_back(q);
      if (pslots(a_high, UB | 0xFu, 0u, J1) || pslots(a_high, 0xFu, 0u, J1)) pd.amix = 1;
    }
    if (!pd.amix && !pslots(xqubits(A), UB, 0u, J1)) pslots(xqubits(A), 0u, 0u, J1);
  } else if (ax) {
    uint32_t am = 0;
    for (int q : xqubits(A)) am |= 1u << q;
    if ((am & 0x3u) && tb >= 8 && !pd.adense) {
      for (int q : xqubits(A))
        if (q >= 4) a_high.push_back(q);
      if (slots(a_high, UB | 0xFu, J1) || slots(a_high, 0xFu, J1)) pd.amix = 1;
    }
    if (!pd.amix && !slots(xqubits(A), UB, J1)) slots(xqubits(A), 0u, J1);
  } else if (az && bpair) {
    if (!pslots({}, UA, 0u, J1)) slots({}, 0u, J1);
    pd.amode = (jmask_of(J1) & UA) == 0;
  } else if (az) {
    if (bx_high && disjoint(xqubits(B), UA) && slots(xqubits(B), UA, J1)) {
      pd.amode = 1;
    } else if (slots({}, UA | UB, J1) || slots({}, UA, J1)) {
      pd.amode = 1;
    } else {
      slots({}, 0u, J1);
    }
  } else if (bpair) {  // logical |0>, then the sums of a pair
    pslots({}, 0u, 0u, J1);
  } else {  // logical |0>
    if (bx_high) slots(xqubits(B), 0u, J1);
    else if (!(bz && slots({}, UB, J1))) slots({}, 0u, J1);
  }
  auto jmask = [](const std::vector<int>& J) {
    uint32_t m = 0;
    for (int q : J) m |= 1u << q;
    return m;
  };
  // slots of the regrouping layout 2: `fixed` first, then layout 1's slot
  // bits, then the lowest bits, outside `avoid`.  Layout 2's slot bits join
  // the tile and take the place of low bits among layout 1's thread bits, so
  // reusing layout 1's bits, else low ones, keeps layout 1's lanes on the
  // lowest bits (long contiguous runs per load and store)
  auto slots2 = [&](std::vector<int> fixed, uint32_t avoid, std::vector<int>& out) {
    out = fixed;
    uint32_t used = avoid;
    for (int q : fixed) used |= 1u << q;
    for (int q : J1)
      if ((int)out.size() < 4 && !((used >> q) & 1)) { out.push_back(q); used |= 1u << q; }
    for (int bit = 0; bit < n && (int)out.size() < 4; ++bit)
      if (!((used >> bit) & 1)) { out.push_back(bit); used |= 1u << bit; }
    return (int)out.size() == 4;
  };
  if (pairpass) {
    // second members: their qubits on the register slots (fillers anywhere)
    if (apair) pslots(xqubits(A, 1), 0u, 0xFu, Jp[0]);
    if (bpair) pslots(xqubits(B, 1), 0u, 0xFu, Jp[1]);
  }
  if (bx && pairpass) {
    pslots(xqubits(B), 0u, 0xFu, J2);
    have2 = true;
    pd.bmode = 2;
  } else if (bz && pairpass) {
    if ((jmask(J1) & UB) == 0) {
      pd.bmode = 1;
    } else if (pslots({}, UB, 0xFu, J2)) {
      have2 = true;
      pd.bmode = 2;
    } else {
      pd.bmode = 0;
    }
  } else if (bx) {
    const std::vector<int> bq = xqubits(B);
    bool in_regs = !ax && J1.size() >= bq.size();
    for (size_t l = 0; l < bq.size() && in_regs; ++l) in_regs = J1[l] == bq[l];
    if (in_regs) {
      pd.bmode = 1;
    } else {
      slots2(bq, 0u, J2);
      have2 = true;
      pd.bmode = 2;
    }
  } else if (bz) {
    if ((jmask(J1) & UB) == 0) {
      pd.bmode = 1;
    } else if (slots2({}, UB, J2)) {
      have2 = true;
      pd.bmode = 2;
    } else {
      pd.bmode = 0;
    }
  }
  // tile: slot bits of both layouts, then the lowest remaining bits
  std::vector<bool> in_t(n, false);
  int cnt = 0;
  for (int x : J1) if (!in_t[x]) { in_t[x] = true; ++cnt; }
  if (have2)
    for (int x : J2) if (!in_t[x]) { in_t[x] = true; ++cnt; }
  for (const std::vector<int>& J : Jp)
    for (int x : J) if (!in_t[x]) { in_t[x] = true; ++cnt; }
  const bool over = cnt > tb;  // the slots alone exceed the tile
  for (int bit = 0; bit < n && cnt < tb; ++bit)
    if (!in_t[bit]) { in_t[bit] = true; ++cnt; }
  {
    // a pass fits when its slots leave room for the lowest three bits
    // (lanes over runs of at least 8 amplitudes); one that does not is
    // returned with tb = -1 (never launched)
    bool ok = !over;
    if (pairpass)
      for (int bit = 0; bit < std::min(3, n) && ok; ++bit) ok = in_t[bit];
    if (fits) *fits = ok;
    if (!ok) {
      pd.tb = -1;
      return pd;
    }
  }
  std::vector<int> rank(n, -1);
  int r = 0;
  pd.n_outer = 0;
  for (int bit = 0; bit < n; ++bit) {
    if (in_t[bit]) rank[bit] = r++;
    else pd.outer_bit[pd.n_outer++] = 1u << bit;
  }
  auto fill = [&](const std::vector<int>& J, uint32_t* tid_g, uint32_t* tid_l, uint32_t* j_g,
                  uint32_t* j_l) {
    std::vector<int> rest;
    for (int bit = 0; bit < n; ++bit)
      if (in_t[bit] && std::find(J.begin(), J.end(), bit) == J.end()) rest.push_back(bit);
    for (int i = 0; i < tb - 4; ++i) {
      tid_g[i] = 1u << rest[i];
      tid_l[i] = 1u << rank[rest[i]];
    }
    for (int j = 0; j < 16; ++j) {
      uint32_t g = 0, l = 0;
      for (int b = 0; b < 4; ++b)
        if ((j >> b) & 1) { g |= 1u << J[b]; l |= 1u << rank[J[b]]; }
      if (j_g) j_g[j] = g;
      j_l[j] = l;
    }
  };
  fill(J1, pd.tid_g, pd.tid_l, pd.j_g, pd.j_l);
  if (pd.amix) {
    // local index of A: bit l for A's qubit l, from lanes or register slots
    const std::vector<int> aq = xqubits(A);
    pd.amix_r = (int)a_high.size();
    pd.amix_lanes = 0;
    for (int i = 0; i < tb - 4; ++i) {
      pd.a_tx[i] = 0;
      for (size_t l = 0; l < aq.size(); ++l)
        if (pd.tid_g[i] == (1u << aq[l])) pd.a_tx[i] = 1u << l;
      if (pd.a_tx[i]) pd.amix_lanes |= 1 << i;
    }
    for (int j = 0; j < 16; ++j) {
      pd.a_jx[j] = 0;
      for (size_t l = 0; l < aq.size(); ++l)
        if (pd.j_g[j] & (1u << aq[l])) pd.a_jx[j] |= 1u << l;
    }
  }
  for (int k = 0; k < 2; ++k)
    if (!Jp[k].empty()) fill(Jp[k], pd.p_tid_g[k], pd.p_tid_l[k], pd.p_j_g[k], pd.p_j_l[k]);
  pd.pstore = apair && !B && tb - 4 >= 3 && pd.p_tid_g[0][0] == 1u && pd.p_tid_g[0][1] == 2u &&
              pd.p_tid_g[0][2] == 4u;
  if (have2) fill(J2, pd.b_tid_g, pd.b_tid_l, pd.b_j_g, pd.b_j_l);
  if (have2 || pairpass) {
    // LDS swizzle for the regrouping: slot = l ^ f(l), where f folds each tile
    // bit i >= 4 onto one of the four lowest bits (mask M[i]).  A wave's 64
    // lanes then spread over the 16-byte bank groups when their lane bits map
    // to four independent low bits, in both layouts; search the foldings for
    // one that does that (the first candidate is the plain fold i -> i mod 4).
    const int nl = std::min(6, tb - 4);
    auto rank_ok = [&](const uint32_t* tl, const uint32_t* M) {
      uint32_t basis[4] = {0, 0, 0, 0};
      int r = 0;
      for (int k = 0; k < nl; ++k) {
        const int b = __builtin_ctz(tl[k]);
        uint32_t v = b < 4 ? 1u << b : M[b];
        for (int q = 0; q < r; ++q) v = std::min(v, v ^ basis[q]);
        if (v) basis[r++] = v;
      }
      return r >= std::min(4, nl);
    };
    uint32_t M[32] = {};
    uint32_t best[32] = {};
    bool found = false;
    for (uint32_t code = 0; code < (1u << (2 * 8)) && !found; ++code) {
      // M[i] = one low bit for i = 4..11; code 0 is the plain fold
      for (int i = 4; i < 12; ++i) M[i] = 1u << (((i & 3) + ((code >> (2 * (i - 4))) & 3)) & 3);
      if (rank_ok(pd.tid_l, M) && (!have2 || rank_ok(pd.b_tid_l, M)) && (Jp[0].empty() || rank_ok(pd.p_tid_l[0], M)) &&
          (Jp[1].empty() || rank_ok(pd.p_tid_l[1], M))) {
        found = true;
        std::copy(M, M + 32, best);
      }
    }
    if (!found)
      for (int i = 4; i < 12; ++i) best[i] = 1u << (i & 3);
    auto swz = [&](uint32_t l) {
      uint32_t f = 0;
      for (int i = 4; i < 12; ++i)
        if ((l >> i) & 1) f ^= best[i];
      return l ^ f;
    };
    for (int i = 0; i < tb - 4; ++i) {
      pd.tid_l[i] = swz(pd.tid_l[i]);
      pd.b_tid_l[i] = swz(pd.b_tid_l[i]);
      for (int k = 0; k < 2; ++k) pd.p_tid_l[k][i] = swz(pd.p_tid_l[k][i]);
    }
    for (int j = 0; j < 16; ++j) {
      pd.j_l[j] = swz(pd.j_l[j]);
      pd.b_j_l[j] = swz(pd.b_j_l[j]);
      for (int k = 0; k < 2; ++k) pd.p_j_l[k][j] = swz(pd.p_j_l[k][j]);
    }
  }
  auto loc = [](uint32_t g, const uint32_t* q, int w) {
    uint32_t x = 0;
    for (int l = 0; l < w; ++l)
      if (g & q[l]) x |= 1u << l;
    return x;
  };
  for (int i = 0; i < pd.la; ++i)
    for (int j = 0; j < 16; ++j) pd.a_j_loc[i][j] = loc(pd.j_g[j], pd.aq[i], pd.aw[i]);
  for (int i = 0; i < pd.lb; ++i)
    for (int j = 0; j < 16; ++j) pd.b_j_loc[i][j] = loc(pd.j_g[j], pd.bq[i], pd.bw[i]);
  return pd;
}


// H on every one of the n register qubits, in groups of up to five, scaled
// by 2^(-n/2) in the last group.
template <typename T>
void launch_wht_all(hipStream_t s, T* st, int n) {
  for (int q0 = 0; q0 < n; q0 += 5) {
    const int K = std::min(5, n - q0);
    const double scale = (q0 + K == n) ? std::pow(2.0, -0.5 * n) : 1.0;
    const uint64_t groups = 1ull << (n - K);
    const dim3 grid((unsigned)((groups + 255) / 256)), block(256);
    const int q[5] = {q0, q0 + 1, q0 + 2, q0 + 3, q0 + 4};
#define QEC_WHT(KK)                                                                              \
  if (K == KK) hipLaunchKernelGGL((k_wht_group<T, KK>), grid, block, 0, s, st, groups, q[0], q[1], \
                                  q[2], q[3], q[4], scale);
    QEC_WHT(1) QEC_WHT(2) QEC_WHT(3) QEC_WHT(4) QEC_WHT(5)
#undef QEC_WHT
  }
}

// One pass kernel launch; the instantiation with the dense Kraus code exists
// only for unit pairs with an X check, the one summing a Z chain amplitude by
// amplitude (bmode 0) only for a Z chain B.
template <typename T, int AK, int AP, int BK, int BP>
void launch_pass(bool dense, bool bm0, dim3 g, dim3 b, hipStream_t s, T* st, const UnitPass* pd,
                 const JobConst* jc, const BlockRT* rta, const BlockRT* rtb, const Decision* da, Decision* db,
                 double* part, int rev, SlotStrides ss, const BlockDense* dna, const BlockDense* dnb) {
#define QEC_K(DNV, BMV)                                                                                  \
  hipLaunchKernelGGL((k_upass<T, AK, AP, BK, BP, DNV, BMV, 0>), g, b, 0, s, st, pd, jc, rta, rtb, da, db, part, \
                     rev, ss, dna, dnb, SpecArgs{})
  if constexpr (BK == U_Z) {
    if (bm0) {
      if constexpr (AK == U_X) {
        if (dense) {
          QEC_K(true, true);
          return;
        }
      }
      QEC_K(false, true);
      return;
    }
  }
  if constexpr ((AK == U_X || BK == U_X) && AK != U_XP && BK != U_XP) {  // pairs are never dense
    if (dense) {
      QEC_K(true, false);
      return;
    }
  }
  QEC_K(false, false);
#undef QEC_K
}

// Launches the pass kernel instantiated for the descriptor's unit kinds.
template <typename T>
sv_status launch_upass(const UnitPass& h, dim3 g, dim3 b, hipStream_t s, T* st, const UnitPass* pd,
                       const JobConst* jc, const BlockRT* rta, const BlockRT* rtb,
                       const Decision* da, Decision* db, double* part, int rev,
                       SlotStrides ss = SlotStrides{0, 0, 0}, const BlockDense* dna = nullptr,
                       const BlockDense* dnb = nullptr) {
#define QEC_UP(AK, AP, BK, BP)                                                                      \
  if (h.akind == AK && ap == AP && h.bkind == BK && bp == BP) {                                     \
    launch_pass<T, AK, AP, BK, BP>(h.adense || h.bdense, h.bkind == U_Z && h.bmode == 0, g, b, s, st, pd, jc, \
                                   rta, rtb, da, db, part, \
                                   rev, ss, dna, dnb);                                              \
    return SV_OK;                                                                                   \
  }
#define QEC_UP_B(AK, AP) \
  QEC_UP(AK, AP, U_X, 2) QEC_UP(AK, AP, U_X, 4) QEC_UP(AK, AP, U_Z, 1) QEC_UP(AK, AP, U_Z, 2) \
  QEC_UP(AK, AP, U_Z, 3) QEC_UP(AK, AP, U_Z, 4) QEC_UP(AK, AP, U_Z, 5) QEC_UP(AK, AP, U_Z, 6)
  if ((h.adense && !dna) || (h.bdense && !dnb)) return fail(SV_EINVAL, "dense unit without its Kraus table");
  if (h.tb <= 0) return fail(SV_EINVAL, "pass layout does not fit a tile");
  const int ap = h.akind == U_X ? h.wa : (h.akind == U_Z ? h.la : 0);
  const int bp = h.bkind == U_X ? h.wb : (h.bkind == U_Z ? h.lb : 0);
  QEC_UP_B(U_INIT, 0)
  QEC_UP_B(U_X, 2) QEC_UP_B(U_X, 4) QEC_UP(U_X, 2, U_NONE, 0) QEC_UP(U_X, 4, U_NONE, 0)
  QEC_UP_B(U_Z, 1) QEC_UP_B(U_Z, 2) QEC_UP_B(U_Z, 3) QEC_UP_B(U_Z, 4) QEC_UP_B(U_Z, 5) QEC_UP_B(U_Z, 6)
  QEC_UP(U_Z, 1, U_NONE, 0) QEC_UP(U_Z, 2, U_NONE, 0) QEC_UP(U_Z, 3, U_NONE, 0) QEC_UP(U_Z, 4, U_NONE, 0)
  QEC_UP(U_Z, 5, U_NONE, 0) QEC_UP(U_Z, 6, U_NONE, 0)
  // X pairs (weights handled at run time)
  QEC_UP(U_INIT, 0, U_XP, 0) QEC_UP(U_X, 2, U_XP, 0) QEC_UP(U_X, 4, U_XP, 0)
  QEC_UP(U_Z, 1, U_XP, 0) QEC_UP(U_Z, 2, U_XP, 0) QEC_UP(U_Z, 3, U_XP, 0) QEC_UP(U_Z, 4, U_XP, 0)
  QEC_UP(U_Z, 5, U_XP, 0) QEC_UP(U_Z, 6, U_XP, 0)
  QEC_UP_B(U_XP, 0) QEC_UP(U_XP, 0, U_XP, 0) QEC_UP(U_XP, 0, U_NONE, 0)
  QEC_UP(U_INIT, 0, U_NONE, 0)  // logical |0> alone (speculative runs)
#undef QEC_UP_B
#undef QEC_UP
  return fail(SV_EINVAL, "no pass kernel for units (%d,%d)->(%d,%d)", h.akind, h.wa, h.bkind, h.wb);
}

// A speculative unit's prediction pass (redo = false) or redo: reads st,
// writes sa.out; the unit is A (an X check or pair, B none) or B (a Z chain,
// A the pending renormalisation).
template <typename T>
sv_status launch_spass(const UnitPass& h, bool redo, dim3 g, dim3 b, hipStream_t s, T* st, const UnitPass* pd,
                       const JobConst* jc, const BlockRT* rta, const BlockRT* rtb, const Decision* da,
                       Decision* db, double* part, int rev, SpecArgs sa, SlotStrides ss) {
#define QEC_SP(AK, AP, BK, BP)                                                                              \
  if (h.akind == AK && ap == AP && h.bkind == BK && bp == BP) {                                             \
    if (redo)                                                                                               \
      hipLaunchKernelGGL((k_uredo<T, AK, AP, BK, BP>), g, b, 0, s, st, pd, jc, rta, rtb, da, db, part, rev, \
                         ss, nullptr, nullptr, sa);                                                         \
    else                                                                                                    \
      hipLaunchKernelGGL((k_upass<T, AK, AP, BK, BP, false, false, 1>), g, b, 0, s, st, pd, jc, rta, rtb,   \
                         da, db, part, rev, ss, nullptr, nullptr, sa);                                      \
    return SV_OK;                                                                                           \
  }
  if (h.tb <= 0) return fail(SV_EINVAL, "pass layout does not fit a tile");
  if (h.adense || h.bdense || (h.bkind == U_Z && h.bmode == 0))
    return fail(SV_EINVAL, "no speculative pass for this unit");
  const int ap = h.akind == U_X ? h.wa : 0;
  const int bp = h.bkind == U_Z ? h.lb : 0;
  QEC_SP(U_X, 2, U_NONE, 0) QEC_SP(U_X, 4, U_NONE, 0) QEC_SP(U_XP, 0, U_NONE, 0)
  QEC_SP(U_SC, 0, U_Z, 1) QEC_SP(U_SC, 0, U_Z, 2) QEC_SP(U_SC, 0, U_Z, 3) QEC_SP(U_SC, 0, U_Z, 4)
  QEC_SP(U_SC, 0, U_Z, 5) QEC_SP(U_SC, 0, U_Z, 6)
#undef QEC_SP
  return fail(SV_EINVAL, "no speculative pass for units (%d,%d)->(%d,%d)", h.akind, h.wa, h.bkind, h.lb);
}


// Units of one round with X pairs (pairs on): each run of consecutive X
// checks is cut into single checks and pairs of consecutive checks, the
// fewest units whose passes fit a tile (a pass with a pair needs the qubits
// of every X member of both its units, and the lowest three bits, in one tile
// of 2^12 amplitudes), counting the passes from the unit before the run and
// into the unit after it (around the round, and from logical |0>).  Dense
// checks stay single; below 12 qubits no pairs.
std::vector<Unit> make_units_paired(const Template& tp, int max_chain, int n, int xpair) {
  const std::vector<Unit> base = make_units(tp, max_chain);
  if (!xpair || n < kTileMax) return base;
  const int nb = (int)base.size();
  auto fit = [&](const Unit* a, const Unit* b) {
    if (!((a && a->kind == U_XP) || (b && b->kind == U_XP))) return true;
    bool ok = false;
    (void)make_unit_pass(n, kTileMax, tp, a, b, &ok);
    return ok;
  };
  std::vector<Unit> out;
  for (int i = 0; i < nb;) {
    if (base[i].kind != U_X) {
      out.push_back(base[i++]);
      continue;
    }
    int j = i;
    while (j < nb && base[j].kind == U_X) ++j;  // X run [i, j)
    const Unit* L = &base[(i + nb - 1) % nb];
    const Unit* R = &base[j % nb];
    const int len = j - i;
    auto unit_at = [&](int p, int l) {
      return l == 2 ? Unit{U_XP, base[i + p].first, 2} : base[i + p];
    };
    // best[p][k]: fewest units for checks p.. given the previous unit (k = 0:
    // L, 1: single p - 1, 2: pair p - 2, p - 1); choice[p][k]: its first unit's length
    const int INF = 1 << 20;
    std::vector<std::array<int, 3>> best(len + 1), choice(len + 1);
    for (int p = len; p >= 0; --p)
      for (int k = 0; k < 3; ++k) {
        best[p][k] = INF;
        choice[p][k] = 0;
        if ((k == 0) != (p == 0) || p < k) continue;
        Unit prev_u{};
        const Unit* prev = L;
        if (k > 0) {
          prev_u = unit_at(p - k, k);
          prev = &prev_u;
        }
        if (p == len) {
          if (fit(prev, R)) best[p][k] = 0;
          continue;
        }
        for (int l = 1; l <= 2; ++l) {
          if (p + l > len) continue;
          if (l == 2 && (tp.blocks[base[i + p].first].dense || tp.blocks[base[i + p + 1].first].dense)) continue;
          const Unit u = unit_at(p, l);
          if (!fit(prev, &u)) continue;
          if (i == 0 && p == 0 && !fit(nullptr, &u)) continue;
          const int c = best[p + l][l];
          if (c < INF && 1 + c < best[p][k]) {
            best[p][k] = 1 + c;
            choice[p][k] = l;
          }
        }
      }
    if (best[0][0] >= INF) {  // keep the run's single checks
      for (int p = i; p < j; ++p) out.push_back(base[p]);
    } else {
      for (int p = 0, k = 0; p < len;) {
        const int l = choice[p][k];
        out.push_back(unit_at(p, l));
        p += l;
        k = l;
      }
    }
    i = j;
  }
  // every pass of the sequence must fit (also around the round)
  const int nu = (int)out.size();
  bool ok = fit(nullptr, &out[0]) && fit(&out[nu - 1], nullptr);
  for (int u = 0; u < nu && ok; ++u) ok = fit(&out[u], &out[(u + 1) % nu]);
  return ok ? out : base;
}

// Passes of a round sequence: [0] writes logical |0> and sums unit 0;
// [1 + u] applies unit u and sums unit u + 1 (unit 0 of the next round after
// the last); [nu + 1] applies the last unit and sums nothing.
std::vector<UnitPass> make_unit_passes(int n, int tb, const Template& tp,
                                       const std::vector<Unit>& units) {
  const int nu = (int)units.size();
  std::vector<UnitPass> pds(nu + 2);
  pds[0] = make_unit_pass(n, tb, tp, nullptr, &units[0]);
  for (int u = 0; u < nu; ++u) pds[1 + u] = make_unit_pass(n, tb, tp, &units[u], &units[(u + 1) % nu]);
  pds[nu + 1] = make_unit_pass(n, tb, tp, &units[nu - 1], nullptr);
  return pds;
}

// Units of one round for speculative passes: consecutive X checks two by two
// where the pair's pass fits a tile (else alone), Z checks in chains of at
// most max_chain members.  Passes: [0] writes logical |0>; [1 + u] is unit u's
// pass (an X unit as A, a Z chain as B after the pending renormalisation).
std::vector<Unit> make_spec_units(const Template& tp, int max_chain, int n) {
  const std::vector<Unit> base = make_units(tp, max_chain);
  std::vector<Unit> out;
  for (size_t i = 0; i < base.size();) {
    if (base[i].kind == U_X && i + 1 < base.size() && base[i + 1].kind == U_X) {
      const Unit pr{U_XP, base[i].first, 2};
      bool ok = false;
      (void)make_unit_pass(n, kTileMax, tp, &pr, nullptr, &ok);
      if (ok) {
        out.push_back(pr);
        i += 2;
        continue;
      }
    }
    out.push_back(base[i++]);
  }
  return out;
}
std::vector<UnitPass> make_spec_passes(int n, int tb, const Template& tp, const std::vector<Unit>& units) {
  std::vector<UnitPass> pds(units.size() + 1);
  pds[0] = make_unit_pass(n, tb, tp, nullptr, nullptr);
  const Unit sc{U_SC, 0, 0};
  for (size_t u = 0; u < units.size(); ++u)
    pds[1 + u] = units[u].kind == U_Z ? make_unit_pass(n, tb, tp, &sc, &units[u])
                                      : make_unit_pass(n, tb, tp, &units[u], nullptr);
  return pds;
}

}  // namespace

namespace {

// Host-side inputs of one run's set-up copies.  An asynchronous run keeps
// them alive until its stream has passed the copies (a host function on the
// stream deletes them), so they may come from pageable memory.
struct RunStage {
  std::vector<TBlock> blocks;
  std::vector<UnitPass> pds;
  JobConst jc;
  std::vector<double> eps, thr;
  std::vector<UnitPass> spds;   // speculative passes
  std::vector<uint8_t> pred0;   // first-round predictions
};

// Every block of the template builds a monomial Kraus pair with no Pauli
// drawn (Paulis keep that form), i.e. the device-side check of the prepare
// kernels cannot fire; used where the run cannot wait to read that check.
bool template_is_monomial(const Template& tp, const std::vector<double>& eps) {
  const uint8_t none[kMaxOps] = {};
  for (const TBlock& b : tp.blocks) {
    if (b.dense) continue;
    BlockRT rt;
    if (!build_block(b, eps.data(), none, rt)) return false;
  }
  return true;
}

int env_int(const char* name, int dflt);

// done == nullptr: synchronous.  Otherwise every step is enqueued on the
// job's stream, `done` is recorded after the results' copies to the host and
// the call returns without waiting (no graph replay, no final states).
// Speculative units (stream launches, asynchronous runs and graph replay of
// a register of at least 2^12 amplitudes whose blocks are all monomial): each
// unit is summed and applied in one pass with predicted outcomes, then
// confirmed or redone (see k_sdecide); two register buffers.  They pay when
// outcomes repeat from round to round, i.e. without the data ZZ layer: at
// d = 5, p = 1e-3 a round takes 2.1 ms instead of 2.9 (complex128); with
// zeta = 0.01 the layer turns 15 % of the X checks' outcomes from one round to
// the next and the redos make them slower (3.1 against 3.0 ms).  So they run
// when zeta = 0; QECSV_SPEC = 0 / 1 turns them off / on whatever zeta is.
template <typename T>
sv_status run_rounds_t(const sv_job* job, sv_result* res, const Template& tp,
                       const std::atomic<int>* cancel = nullptr, hipEvent_t done = nullptr) {
  const bool async = done != nullptr;
  const int d = job->d, n = d * d, ns = (int)tp.blocks.size(), R = job->rounds;
  const int tb = std::min(kTileMax, n);
  const int per_traj = R * ns;  // block instances (records) per trajectory
  const sv_tuning tune = tuning_for(d, job->dtype);
  const std::vector<Unit> units = make_units_paired(tp, tune.zchain, n, tune.xpair);
  const int nu = (int)units.size();
  const int per_units = R * nu;  // passes per trajectory after the first
  const int spec_env = env_int("QECSV_SPEC", -1);
  bool spec = (spec_env < 0 ? job->zeta == 0.0 : spec_env != 0) && n >= kTileMax && !tp.any_dense;
  std::vector<Unit> sunits;
  std::vector<UnitPass> spds;
  if (spec) {
    sunits = make_spec_units(tp, tune.zchain, n);
    spds = make_spec_passes(n, tb, tp, sunits);
    // a chain that has to be summed amplitude by amplitude keeps the plain passes
    for (const UnitPass& h : spds)
      if (h.tb <= 0 || (h.bkind == U_Z && h.bmode == 0)) spec = false;
  }
  if (!spec) sunits.clear();
  const int nus = (int)sunits.size();
  const int per_units_s = R * nus;
  // decision record of the register the final measurement reads
  const int fin = spec ? per_units_s : per_units;
  hipStream_t s = (hipStream_t)job->hip_stream;
  DevBufs M(s);
  T* st = nullptr;
  double* partials = nullptr;
  TBlock* dblocks = nullptr;
  UnitPass* dpass = nullptr;
  JobConst* djc = nullptr;
  double* deps = nullptr;
  Decision* ddec = nullptr;
  uint8_t* drec = nullptr;
  uint8_t* dbits = nullptr;
  double* dp1 = nullptr;
  double* dsums = nullptr;
  int* derr = nullptr;
  BlockRT* drt = nullptr;
  const uint64_t na = 1ull << n;
  const int cb = std::min(12, n);
  const size_t n_tiles = (size_t)1 << (n - tb);
  // trajectories per prepare chunk: keep the block tables under 64 MiB
  const size_t rt_per_traj = sizeof(BlockRT) * (size_t)per_traj;
  const size_t dn_per_traj = tp.any_dense ? sizeof(BlockDense) * (size_t)per_traj : 0;
  const int chunk = (int)std::max<size_t>(
      1, std::min<size_t>((size_t)job->n_traj, ((size_t)64 << 20) / (rt_per_traj + dn_per_traj)));
  const int n_angles = std::max(1, tp.zz_site >= 0 ? tp.zz_site + 1 : tp.n_sites);
  const size_t nrec = (size_t)job->n_traj * per_traj;
  HIP_OK(M.alloc(&st, sizeof(T) * 2 * na));
  HIP_OK(M.alloc(&partials, sizeof(double) * kChainAcc * n_tiles));
  double* dacc = nullptr;
  unsigned* dticket = nullptr;
  HIP_OK(M.alloc(&dacc, sizeof(double) * kChainAcc));
  HIP_OK(M.alloc(&dticket, sizeof(unsigned)));
  HIP_OK(hipMemsetAsync(dticket, 0, sizeof(unsigned), s));
  HIP_OK(M.alloc(&dblocks, sizeof(TBlock) * ns));
  HIP_OK(M.alloc(&dpass, sizeof(UnitPass) * (nu + 2)));
  HIP_OK(M.alloc(&djc, sizeof(JobConst)));
  HIP_OK(M.alloc(&deps, sizeof(double) * n_angles));
  const int n_dec = std::max(per_units, per_units_s) + 1;
  HIP_OK(M.alloc(&ddec, sizeof(Decision) * n_dec));
  HIP_OK(M.alloc(&drec, nrec));
  HIP_OK(M.alloc(&dbits, (size_t)job->n_traj * n));
  if (res->p1_trace) HIP_OK(M.alloc(&dp1, sizeof(double) * nrec));
  HIP_OK(M.alloc(&dsums, sizeof(double) << (n - cb)));
  HIP_OK(M.alloc(&derr, sizeof(int)));
  HIP_OK(M.alloc(&drt, rt_per_traj * chunk));
  BlockDense* ddn = nullptr;  // dense Kraus pairs (blocks with crosstalk inside)
  if (tp.any_dense) HIP_OK(M.alloc(&ddn, dn_per_traj * chunk));

  const std::vector<UnitPass> pds = make_unit_passes(n, tb, tp, units);
  const bool xbasis = (job->flags & SV_RUN_XBASIS) != 0;
  // speculative runs: the second register, pass descriptors, control records,
  // first-round predictions (the trivial outcome of every check), redo count
  T* st2 = nullptr;
  UnitPass* dspass = nullptr;
  SpecCtl* dctl = nullptr;
  uint8_t* dpred0 = nullptr;
  int* dredos = nullptr;
  std::vector<uint8_t> pred0;
  if (spec) {
    for (const TBlock& b : tp.blocks)
      pred0.push_back(job->gateset == SV_GATESET_CR ? (uint8_t)((b.w / 2) % 2) : (uint8_t)0);
    HIP_OK(M.alloc(&st2, sizeof(T) * 2 * na));
    HIP_OK(M.alloc(&dspass, sizeof(UnitPass) * spds.size()));
    HIP_OK(M.alloc(&dctl, sizeof(SpecCtl) * per_units_s));
    HIP_OK(M.alloc(&dpred0, pred0.size()));
    HIP_OK(M.alloc(&dredos, sizeof(int)));
    HIP_OK(hipMemsetAsync(dredos, 0, sizeof(int), s));
  }
  std::vector<double> eps(n_angles, job->eps);
  if (job->eps_site)
    for (int i = 0; i < tp.n_sites; ++i) eps[i] = job->eps_site[i];
  if (tp.zz_site >= 0) eps[tp.zz_site] = job->zeta;  // the per-step crosstalk angle
  if (async && !template_is_monomial(tp, eps))
    return fail(SV_EINVAL, "circuit template is not monomial in its block basis");
  // Pauli-twirled over-rotations: per-site probability sin^2 eps, computed
  // here so that every implementation compares its draws with the same value
  std::vector<double> thr;
  double* dthr = nullptr;
  if (job->flags & SV_RUN_TWIRL) {
    thr.resize(eps.size());
    for (size_t i = 0; i < eps.size(); ++i) {
      const double sn = std::sin(eps[i]);
      thr[i] = sn * sn;
    }
    HIP_OK(M.alloc(&dthr, sizeof(double) * thr.size()));
  }
  {
    // set-up copies from a staging block that a host function on the stream
    // deletes once the stream has passed them (the call may return first)
    RunStage* stage = new RunStage{tp.blocks, pds, make_job_const(d, job->zeta, xbasis), eps, thr, spds, pred0};
    const hipError_t e = [&]() -> hipError_t {
      hipError_t r;
      if ((r = hipMemcpyAsync(dblocks, stage->blocks.data(), sizeof(TBlock) * ns, hipMemcpyHostToDevice, s)))
        return r;
      if ((r = hipMemcpyAsync(dpass, stage->pds.data(), sizeof(UnitPass) * (nu + 2), hipMemcpyHostToDevice,
                              s)))
        return r;
      if ((r = hipMemcpyAsync(djc, &stage->jc, sizeof(JobConst), hipMemcpyHostToDevice, s))) return r;
      if ((r = hipMemcpyAsync(deps, stage->eps.data(), sizeof(double) * stage->eps.size(),
                              hipMemcpyHostToDevice, s)))
        return r;
      if (dthr && (r = hipMemcpyAsync(dthr, stage->thr.data(), sizeof(double) * stage->thr.size(),
                                      hipMemcpyHostToDevice, s)))
        return r;
      if (spec && (r = hipMemcpyAsync(dspass, stage->spds.data(), sizeof(UnitPass) * stage->spds.size(),
                                      hipMemcpyHostToDevice, s)))
        return r;
      if (spec && (r = hipMemcpyAsync(dpred0, stage->pred0.data(), stage->pred0.size(), hipMemcpyHostToDevice, s)))
        return r;
      return hipLaunchHostFunc(s, [](void* q) { delete static_cast<RunStage*>(q); }, stage);
    }();
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      delete stage;
      return fail(SV_EDEVICE, "set-up copies: %s", hipGetErrorString(e));
    }
  }
  HIP_OK(hipMemsetAsync(derr, 0, sizeof(int), s));
  HIP_OK(hipMemsetAsync(ddec, 0, sizeof(Decision) * n_dec, s));
  if (spec) {  // the register logical |0> is written in: norm 1, frame 0
    static const Decision d0{1.0, 0, 0u};
    HIP_OK(hipMemcpyAsync(ddec, &d0, sizeof d0, hipMemcpyHostToDevice, s));
  }

  // whole-run events plus one pair around every pass of the last trajectory
  struct Events {
    std::vector<hipEvent_t> ev;
    ~Events() {
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
  } E;
  E.ev.resize(async ? 0 : 2 + 2 * std::max(per_units, per_units_s), nullptr);
  for (auto& e : E.ev) HIP_OK(hipEventCreate(&e));
  hipEvent_t ev0 = async ? nullptr : E.ev[0], ev1 = async ? nullptr : E.ev[1];
  hipEvent_t* evs = async ? nullptr : E.ev.data() + 2;
  if (!async) HIP_OK(hipEventRecord(ev0, s));

  // alternate the tile traversal between consecutive passes: a pass starts on
  // the lines its predecessor wrote last
  const int snake = tune.snake;
  const size_t pass_wgs = tune.pass_wgs_per_cu == 0
                              ? n_tiles
                              : std::min<size_t>(n_tiles, (size_t)device_cu_count() * tune.pass_wgs_per_cu);
  const dim3 grid((unsigned)pass_wgs), block((unsigned)std::max(64, 1 << (tb - 4)));
  const SlotStrides ss0{0, 0, 0};
  const int draws_round = tp.n_draws;
  const int last_t = job->n_traj - 1;
  // block instance of the first member of unit instance ui
  auto inst = [&](int ui) { return (ui / nu) * ns + units[ui % nu].first; };
  // passes and decisions of one trajectory whose block tables are at rt
  auto traj_passes = [&](hipStream_t q, const BlockRT* rt, const BlockDense* dn, uint8_t* rec, double* p1,
                         bool timed) -> sv_status {
    auto dense = [&](int ui) { return dn ? dn + inst(ui) : (const BlockDense*)nullptr; };
    auto decide = [&](int ui) {
      const int bi = inst(ui);
      const int lb = units[ui % nu].len;
      // one partial per pass workgroup
      hipLaunchKernelGGL(k_udecide, dim3(unit_sums(lb)), dim3(256), 0, q, partials, (int)grid.x, lb,
                         rt + bi, &ddec[ui], rec + bi, p1 ? p1 + bi : nullptr, ss0, (size_t)0, dacc,
                         dticket, 1);
    };
    SV_OK_OR_RETURN(launch_upass<T>(pds[0], grid, block, q, st, &dpass[0], djc, nullptr, rt + inst(0),
                                    nullptr, &ddec[0], partials, 0, ss0, nullptr, dense(0)));
    decide(0);
    for (int ui = 0; ui < per_units; ++ui) {
      const int u = ui % nu;
      const bool last = (ui == per_units - 1);
      const int pidx = last ? nu + 1 : 1 + u;
      if (timed) HIP_OK(hipEventRecord(evs[2 * ui], q));
      SV_OK_OR_RETURN(launch_upass<T>(pds[pidx], grid, block, q, st, &dpass[pidx], djc, rt + inst(ui),
                                      last ? nullptr : rt + inst(ui + 1), &ddec[ui], &ddec[ui + 1],
                                      partials, snake ? ((ui + 1) & 1) : 0, ss0, dense(ui),
                                      last ? nullptr : dense(ui + 1)));
      if (timed) HIP_OK(hipEventRecord(evs[2 * ui + 1], q));
      if (!last) decide(ui + 1);
    }
    HIP_OK(hipGetLastError());
    return SV_OK;
  };
  // speculative passes of one trajectory: logical |0> into st, then per unit
  // instance its prediction pass (st <-> st2 alternate), the decision and the
  // redos it may need (an X pair two, with a decision between them; a single
  // check or a chain one).  Returns the register that holds the result.
  auto traj_spec = [&](hipStream_t q, const BlockRT* rt, uint8_t* rec, double* p1, bool timed,
                       T** out) -> sv_status {
    T* cur = st;
    T* oth = st2;
    SV_OK_OR_RETURN(launch_upass<T>(spds[0], grid, block, q, cur, &dspass[0], djc, nullptr, nullptr, nullptr,
                                    &ddec[0], partials, 0, ss0));
    for (int ui = 0; ui < per_units_s; ++ui) {
      const int u = ui % nus, r = ui / nus;
      const Unit& U = sunits[u];
      const bool zb = U.kind == U_Z;
      const size_t bi = (size_t)r * ns + U.first;
      const uint8_t* pred = r == 0 ? dpred0 + U.first : rec + bi - ns;
      const SpecArgs sa{oth, &dctl[ui], pred, dredos, 0, 0};
      const BlockRT* rta = zb ? nullptr : rt + bi;
      const BlockRT* rtb = zb ? rt + bi : nullptr;
      const int rev = snake ? (ui & 1) : 0;
      auto pass = [&](bool redo) {
        return launch_spass<T>(spds[1 + u], redo, grid, block, q, cur, &dspass[1 + u], djc, rta, rtb, &ddec[ui],
                               &ddec[ui + 1], partials, rev, sa, ss0);
      };
      auto decide = [&]() {
        hipLaunchKernelGGL(k_sdecide, dim3(zb ? unit_sums(U.len) : 2 * U.len), dim3(256), 0, q, partials,
                           (int)grid.x, U.len, zb ? 1 : 0, rt + bi, &ddec[ui], &ddec[ui + 1], rec + bi,
                           p1 ? p1 + bi : nullptr, &dctl[ui], dacc, dticket, ss0, (size_t)0, (size_t)0, 1);
      };
      if (timed) HIP_OK(hipEventRecord(evs[2 * ui], q));
      SV_OK_OR_RETURN(pass(false));
      if (timed) HIP_OK(hipEventRecord(evs[2 * ui + 1], q));
      decide();
      const int redos = (!zb && U.len == 2) ? 2 : 1;
      for (int k = 0; k < redos; ++k) {
        SV_OK_OR_RETURN(pass(true));
        if (k + 1 < redos) decide();
      }
      std::swap(cur, oth);
    }
    HIP_OK(hipGetLastError());
    *out = cur;
    return SV_OK;
  };
  // final Z measurement of the data register buf (draw stream t, or *tptr);
  // in the X basis a Walsh-Hadamard transform of the whole register first,
  // which removes the Pauli-X frame from the outcome probabilities (the
  // outcome probabilities are ratios: a pending renormalisation is harmless)
  auto traj_final = [&](hipStream_t q, T* buf, uint8_t* bits, uint64_t t, const uint64_t* tptr) {
    if (xbasis) launch_wht_all<T>(q, buf, n);
    hipLaunchKernelGGL(k_final_sums<T>, dim3(1u << (n - cb)), dim3(256), 0, q, buf, cb, dsums,
                       (size_t)0);
    hipLaunchKernelGGL(k_final_measure<T>, dim3(1), dim3(1024), 0, q, buf, n, cb, dsums, job->seed, t,
                       (uint64_t)R * (uint64_t)draws_round, bits, (size_t)0, (const uint64_t*)nullptr,
                       tptr, (const int*)nullptr, (uint64_t)0,
                       xbasis ? (const Decision*)nullptr : (const Decision*)&ddec[fin],
                       (size_t)0);
  };
  double pass_ms_graph = -1.0;
  std::vector<uint32_t> phi_host(res->final_states ? job->n_traj : 0);
  if (job->flags & SV_RUN_GRAPH) {
    // one trajectory's sequence, staged through fixed buffers and a device
    // trajectory counter, captured once and replayed n_traj times
    BlockRT* rt_s = nullptr;
    BlockDense* dn_s = nullptr;
    uint8_t *rec_s = nullptr, *bits_s = nullptr;
    double* p1_s = nullptr;
    uint64_t* dcur = nullptr;  // [0] trajectory counter, [1] its draw stream
    HIP_OK(M.alloc(&rt_s, rt_per_traj));
    if (tp.any_dense) HIP_OK(M.alloc(&dn_s, dn_per_traj));
    HIP_OK(M.alloc(&rec_s, (size_t)per_traj));
    HIP_OK(M.alloc(&bits_s, (size_t)n));
    if (dp1) HIP_OK(M.alloc(&p1_s, sizeof(double) * per_traj));
    HIP_OK(M.alloc(&dcur, 2 * sizeof(uint64_t)));
    const uint64_t cur0[2] = {0, job->traj0};
    HIP_OK(hipMemcpyAsync(dcur, cur0, sizeof cur0, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    struct GraphRes {
      hipStream_t q = nullptr;
      hipGraph_t g = nullptr;
      hipGraphExec_t x = nullptr;
      hipEvent_t a = nullptr, b = nullptr;
      ~GraphRes() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (q) (void)hipStreamDestroy(q);
      }
    } G;
    HIP_OK(hipStreamCreateWithFlags(&G.q, hipStreamNonBlocking));
    HIP_OK(hipEventCreate(&G.a));
    HIP_OK(hipEventCreate(&G.b));
    HIP_OK(hipStreamBeginCapture(G.q, hipStreamCaptureModeThreadLocal));
    sv_status cst = SV_OK;
    {
      hipLaunchKernelGGL(k_prepare, dim3((unsigned)((per_traj + 127) / 128)), dim3(128), 0, G.q,
                         dblocks, ns, R, draws_round, job->seed, job->traj0, 1, job->p, deps, rt_s,
                         derr, (const uint64_t*)(dcur + 1), (const double*)dthr);
      if (dn_s)
        hipLaunchKernelGGL(k_prepare_dense, dim3((unsigned)((per_traj * 16 + 127) / 128)), dim3(128), 0, G.q,
                           dblocks, ns, R, draws_round, job->seed, job->traj0, 1, job->p, deps, dn_s, derr,
                           (const uint64_t*)(dcur + 1), (const double*)dthr);
      T* fbuf = st;
      cst = spec ? traj_spec(G.q, rt_s, rec_s, p1_s, false, &fbuf) : traj_passes(G.q, rt_s, dn_s, rec_s, p1_s, false);
      if (cst == SV_OK) {
        traj_final(G.q, fbuf, bits_s, 0, dcur + 1);
        hipLaunchKernelGGL(k_commit, dim3(1), dim3(256), 0, G.q, rec_s, p1_s, bits_s, drec, dp1, dbits,
                           per_traj, n, dcur, dcur + 1, job->traj0);
      }
    }
    const hipError_t ce = hipStreamEndCapture(G.q, &G.g);
    if (cst != SV_OK) return cst;
    HIP_OK(ce);
    HIP_OK(hipGraphInstantiate(&G.x, G.g, nullptr, nullptr, 0));
    HIP_OK(hipEventRecord(ev0, G.q));
    for (int t = 0; t < job->n_traj; ++t) {
      if (cancel && cancel->load(std::memory_order_relaxed)) {
        (void)hipStreamSynchronize(G.q);
        return fail(SV_EBUSY, "cancelled");
      }
      if (t == last_t) HIP_OK(hipEventRecord(G.a, G.q));
      HIP_OK(hipGraphLaunch(G.x, G.q));
      if (t == last_t) HIP_OK(hipEventRecord(G.b, G.q));
    }
    HIP_OK(hipEventRecord(ev1, G.q));
    HIP_OK(hipStreamSynchronize(G.q));
    float tm = 0.f;
    HIP_OK(hipEventElapsedTime(&tm, G.a, G.b));
    pass_ms_graph = tm / ((spec ? per_units_s : per_units) + 1);
  } else {
    for (int c0 = 0; c0 < job->n_traj; c0 += chunk) {
      const int cn = std::min(chunk, job->n_traj - c0);
      const int64_t nthreads = (int64_t)cn * per_traj;
      hipLaunchKernelGGL(k_prepare, dim3((unsigned)((nthreads + 127) / 128)), dim3(128), 0, s, dblocks,
                         ns, R, draws_round, job->seed, job->traj0 + (uint64_t)c0, cn, job->p, deps,
                         drt, derr, (const uint64_t*)nullptr, (const double*)dthr);
      if (ddn)
        hipLaunchKernelGGL(k_prepare_dense, dim3((unsigned)((nthreads * 16 + 127) / 128)), dim3(128), 0, s,
                           dblocks, ns, R, draws_round, job->seed, job->traj0 + (uint64_t)c0, cn, job->p, deps,
                           ddn, derr, (const uint64_t*)nullptr, (const double*)dthr);
      HIP_OK(hipGetLastError());
      for (int ti = 0; ti < cn; ++ti) {
        if (cancel && cancel->load(std::memory_order_relaxed)) {
          (void)hipStreamSynchronize(s);
          return fail(SV_EBUSY, "cancelled");
        }
        const int tg = c0 + ti;
        T* buf = st;
        if (spec) {
          SV_OK_OR_RETURN(traj_spec(s, drt + (size_t)ti * per_traj, drec + (size_t)tg * per_traj,
                                    dp1 ? dp1 + (size_t)tg * per_traj : nullptr, tg == last_t && !async, &buf));
        } else {
          SV_OK_OR_RETURN(traj_passes(s, drt + (size_t)ti * per_traj, ddn ? ddn + (size_t)ti * per_traj : nullptr,
                                      drec + (size_t)tg * per_traj,
                                      dp1 ? dp1 + (size_t)tg * per_traj : nullptr, tg == last_t && !async));
        }
        if (res->final_states) {
          // a speculative run leaves the last unit's renormalisation pending
          if (spec)
            hipLaunchKernelGGL(k_renorm<T>, dim3((unsigned)std::min<uint64_t>(na / 256, 65536)), dim3(256), 0, s,
                               buf, na, (const Decision*)&ddec[fin]);
          HIP_OK(hipMemcpyAsync((char*)res->final_states + (size_t)tg * sizeof(T) * 2 * na, buf,
                                sizeof(T) * 2 * na, hipMemcpyDeviceToHost, s));
          Decision fd{};
          HIP_OK(hipMemcpyAsync(&fd, &ddec[fin], sizeof fd, hipMemcpyDeviceToHost, s));
          HIP_OK(hipStreamSynchronize(s));
          phi_host[tg] = fd.phi;
        }
        traj_final(s, buf, dbits + (size_t)tg * n, job->traj0 + (uint64_t)tg, nullptr);
        HIP_OK(hipGetLastError());
      }
    }
    if (async) {
      HIP_OK(hipMemcpyAsync(res->records, drec, nrec, hipMemcpyDeviceToHost, s));
      HIP_OK(hipMemcpyAsync(res->final_bits, dbits, (size_t)job->n_traj * n, hipMemcpyDeviceToHost, s));
      if (res->p1_trace)
        HIP_OK(hipMemcpyAsync(res->p1_trace, dp1, sizeof(double) * nrec, hipMemcpyDeviceToHost, s));
      HIP_OK(hipEventRecord(done, s));
      // the device buffers are released in stream order when M goes out of
      // scope
      res->gpu_ms = -1.0;
      res->pass_ms = -1.0;
      res->passes_per_round = spec ? nus : nu;
      res->redo_passes = 0;  // not waited for
      return SV_OK;
    }
    HIP_OK(hipEventRecord(ev1, s));
  }
  int herr = 0;
  HIP_OK(hipMemcpyAsync(&herr, derr, sizeof herr, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (herr) return fail(SV_EINVAL, "circuit template is not monomial in its block basis");
  HIP_OK(hipMemcpyAsync(res->records, drec, nrec, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(res->final_bits, dbits, (size_t)job->n_traj * n, hipMemcpyDeviceToHost, s));
  if (res->p1_trace)
    HIP_OK(hipMemcpyAsync(res->p1_trace, dp1, sizeof(double) * nrec, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  // registers handed back in the logical frame: amplitude x sits at x ^ phi
  if (res->final_states)
    for (int t = 0; t < job->n_traj; ++t) {
      const uint32_t phi = phi_host[t];
      if (!phi) continue;
      C2<T>* a = reinterpret_cast<C2<T>*>((char*)res->final_states + (size_t)t * sizeof(T) * 2 * na);
      for (uint64_t x = 0; x < na; ++x) {
        const uint64_t y = x ^ phi;
        if (x < y) std::swap(a[x], a[y]);
      }
    }
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, ev0, ev1));
  double pass_sum = 0.0;
  const int timed_units = spec ? per_units_s : per_units;
  if (pass_ms_graph < 0.0) {
    for (int ui = 0; ui < timed_units; ++ui) {
      float pm = 0.f;
      HIP_OK(hipEventElapsedTime(&pm, evs[2 * ui], evs[2 * ui + 1]));
      pass_sum += pm;
    }
  }
  res->gpu_ms = ms;
  // replayed graphs: the last trajectory's device time per pass (an upper
  // bound that includes its decisions, draws and final measurement)
  res->pass_ms = pass_ms_graph >= 0.0 ? pass_ms_graph : pass_sum / timed_units;
  res->passes_per_round = spec ? nus : nu;
  res->redo_passes = 0;
  if (spec) {  // on the job's stream (a plain copy would wait for every stream of the device)
    HIP_OK(hipMemcpyAsync(&res->redo_passes, dredos, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  return SV_OK;
}

// Lane / register maps of the small-register batch kernel for each block
// template: a lane's 8 registers span three of a weight-4 check's qubits (its
// fourth is lane bit 0), or a weight-2 check's two qubits and the lowest other
// bit; the remaining bits index lanes, lowest first.
// Register layout of every block template for a trajectory run by nw waves:
// 2^rb amplitudes per thread (rb = 3, 2, 1 for nw = 1, 2, 4).  The check's
// first qubits go to register bits (at most rb, and at most 2 for a weight-2
// check when rb >= 2), its other qubits to the lowest thread-index bits (lane
// bits: their Walsh-Hadamard stages are lane exchanges); the remaining
// register bits fill the free register slots, then the higher thread bits.
std::vector<SmallDesc> make_small_descs(int n, const Template& tp, int nw) {
  const int rb = nw == 1 ? 3 : nw == 2 ? 2 : 1;
  std::vector<SmallDesc> out(tp.blocks.size());
  for (size_t i = 0; i < tp.blocks.size(); ++i) {
    const TBlock& b = tp.blocks[i];
    SmallDesc sd{};
    std::vector<int> rest;
    for (int bit = 0; bit < n; ++bit) {
      bool in = false;
      for (int l = 0; l < b.w; ++l) in = in || (b.qubit[l] == bit);
      if (!in) rest.push_back(bit);
    }
    const int xreg = std::min(rb, b.w == 4 ? 4 : 2);
    std::vector<int> regs, lanes;
    for (int l = 0; l < xreg; ++l) regs.push_back(b.qubit[l]);
    for (int l = xreg; l < b.w; ++l) lanes.push_back(b.qubit[l]);
    size_t r = 0;
    while ((int)regs.size() < rb) regs.push_back(rest[r++]);
    for (; r < rest.size(); ++r) lanes.push_back(rest[r]);
    sd.xreg = xreg;
    sd.xlanes = b.w - xreg;
    sd.xmask = (1u << xreg) - 1u;
    for (int j = 0; j < (1 << rb); ++j) {
      uint32_t g = 0;
      for (int k = 0; k < rb; ++k)
        if ((j >> k) & 1) g |= 1u << regs[k];
      sd.j_off[j] = g;
    }
    sd.n_lane_bits = n - rb;
    for (int k = 0; k < n - rb; ++k) sd.lane_bit[k] = 1u << lanes[k];
    for (int l = 0; l < b.w; ++l) sd.q_bit[l] = 1u << b.qubit[l];
    out[i] = sd;
  }
  return out;
}

int env_int(const char* name, int dflt) {
  if (const char* e = std::getenv(name)) return std::atoi(e);
  return dflt;
}

// Inputs of one batched launch; every array has one entry per trajectory
// (eps: eps_stride doubles per trajectory, stride 0 = shared by all).
struct BatchInputs {
  int d, gateset, n_traj, max_rounds;
  double zeta;
  const uint64_t* seed;
  const uint64_t* stream;
  const int* rounds;
  const double* p;
  const double* eps;
  int eps_stride;
  uint8_t* records;     // host [n_traj][max_rounds][n_stab]
  uint8_t* final_bits;  // host [n_traj][d^2]
  hipStream_t hs;
  double gpu_ms;
  int passes_per_round = 0;  // out: register passes per round (lockstep launches)
  int redo_passes = 0;       // out: speculative redos that ran, one per slot and unit
};

template <typename T>
sv_status run_batch_lockstep(BatchInputs& in, const Template& tp);

// Device buffers of one call carved from a fixed region (the no-allocation
// entry point's scratch array): 256-byte aligned, never freed.
struct Arena {
  char* base;
  size_t cap, used;
  bool overflow;
  template <typename P>
  hipError_t alloc(P** out, size_t bytes) {
    const size_t off = (used + 255) & ~(size_t)255;
    if (off + bytes > cap) {
      overflow = true;
      return hipErrorOutOfMemory;
    }
    *out = reinterpret_cast<P*>(base + off);
    used = off + bytes;
    return hipSuccess;
  }
};

// The batched kernels draw a block with one lane per draw (16 lanes) and keep
// kMaxOpsBatch Pauli choices per lane.
bool batch_template_fits(const Template& tp) {
  for (const TBlock& b : tp.blocks)
    if (b.n_draws > 16 || b.n_ops > kMaxOpsBatch) return false;
  return true;
}

// d <= 3: the register fits in LDS (k_batch_small).
bool batch_is_small(const Template& tp, int d) {
  return d * d <= kSmallBits && (int)tp.blocks.size() <= kSmallStab && tp.n_sites <= kSmallSites &&
         tp.n_draws <= kSmallDraws;
}

// The LDS-resident launch with its device buffers from M (DevBufs or Arena);
// ev_a / ev_b bracket the kernel.  Every buffer is taken before anything is
// enqueued, so a failed allocation leaves nothing in flight.
template <typename T, typename Alloc>
sv_status run_batch_small(BatchInputs& in, const Template& tp, Alloc& M, hipEvent_t ev_a, hipEvent_t ev_b);

template <typename T>
sv_status run_batch_core(BatchInputs& in, const Template& tp) {
  const int d = in.d, n = d * d;
  if (!batch_template_fits(tp)) return fail(SV_EINVAL, "block template too large for the batched path");
  if (!batch_is_small(tp, d)) {
    if (n > 16) return fail(SV_EINVAL, "d=%d batch path not available", d);
    return run_batch_lockstep<T>(in, tp);
  }
  DevBufs M(in.hs);
  struct Ev {
    hipEvent_t a = nullptr, b = nullptr;
    ~Ev() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  HIP_OK(hipEventCreate(&ev.a));
  HIP_OK(hipEventCreate(&ev.b));
  return run_batch_small<T>(in, tp, M, ev.a, ev.b);
}

template <typename T, typename Alloc>
sv_status run_batch_small(BatchInputs& in, const Template& tp, Alloc& M, hipEvent_t ev_a, hipEvent_t ev_b) {
  const int d = in.d, n = d * d, ns = (int)tp.blocks.size();
  const int nt = in.n_traj;
  hipStream_t s = in.hs;
  TBlock* dblocks = nullptr;
  SmallDesc* dsd = nullptr;
  JobConst* djc = nullptr;
  int *dorder = nullptr, *drounds = nullptr, *derr = nullptr;
  double *dp = nullptr, *deps = nullptr;
  uint64_t *dseed = nullptr, *dstream = nullptr;
  uint8_t *drec = nullptr, *dbits = nullptr;
  const size_t nrec = (size_t)nt * in.max_rounds * ns;
  const size_t neps = in.eps_stride ? (size_t)nt * in.eps_stride : (size_t)std::max(1, tp.n_sites);
  HIP_OK(M.alloc(&dblocks, sizeof(TBlock) * ns));
  HIP_OK(M.alloc(&dsd, sizeof(SmallDesc) * ns));
  HIP_OK(M.alloc(&djc, sizeof(JobConst)));
  HIP_OK(M.alloc(&dorder, sizeof(int) * nt));
  HIP_OK(M.alloc(&drounds, sizeof(int) * nt));
  HIP_OK(M.alloc(&derr, sizeof(int)));
  HIP_OK(M.alloc(&dp, sizeof(double) * nt));
  HIP_OK(M.alloc(&dseed, sizeof(uint64_t) * nt));
  HIP_OK(M.alloc(&dstream, sizeof(uint64_t) * nt));
  HIP_OK(M.alloc(&deps, sizeof(double) * neps));
  HIP_OK(M.alloc(&drec, nrec));
  HIP_OK(M.alloc(&dbits, (size_t)nt * n));
  TOp* dsites = nullptr;
  HIP_OK(M.alloc(&dsites, sizeof(TOp) * std::max(1, tp.n_sites)));
  SmallShared<T>* dshared = nullptr;
  if (in.eps_stride == 0) HIP_OK(M.alloc(&dshared, sizeof(SmallShared<T>)));
  uint32_t* dinit = nullptr;
  HIP_OK(M.alloc(&dinit, sizeof(uint32_t) * 16));
  uint8_t* dkind = nullptr;
  HIP_OK(M.alloc(&dkind, (size_t)std::max(1, tp.n_draws)));
  // longest trajectories first, so the static assignment balances
  std::vector<int> order(nt);
  for (int i = 0; i < nt; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return in.rounds[a] > in.rounds[b]; });
  // waves per trajectory: a launch of at most two trajectories per SIMD
  // splits each one over 2 waves (more waves hide the latency of the
  // per-circuit chain: 1000 d=3 trajectories 0.090 -> 0.085 ms; 4 waves take
  // 0.138 ms, the per-circuit reduction and decision then dominate);
  // QECSV_BATCH_SPLIT forces 1, 2 or 4
  const int simds = 4 * device_cu_count();
  int nw = nt <= 2 * simds ? 2 : 1;
  const int forced = env_int("QECSV_BATCH_SPLIT", 0);
  if (forced == 1 || forced == 2 || forced == 4) nw = forced;
  const std::vector<SmallDesc> sd = make_small_descs(n, tp, nw);
  const JobConst jc = make_job_const(d, in.zeta);
  // the op of every gate site (index = site)
  std::vector<TOp> sites(std::max(1, tp.n_sites));
  for (const TBlock& b : tp.blocks)
    for (int i = 0; i < b.n_ops; ++i)
      if (b.ops[i].site >= 0) sites[b.ops[i].site] = b.ops[i];
  HIP_OK(hipMemcpyAsync(dsites, sites.data(), sizeof(TOp) * sites.size(), hipMemcpyHostToDevice, s));
  // angles common to every trajectory: the angle table and noise-free Kraus
  // pairs once, here
  if (in.eps_stride == 0) {
    SmallShared<T> sh{};
    for (int k = 0; k < tp.n_sites; ++k) {
      const double beta = op_angle(sites[k], in.eps);
      sh.cs[2 * k] = std::cos(beta);
      sh.cs[2 * k + 1] = std::sin(beta);
    }
    const uint8_t none[kMaxOpsBatch] = {};
    for (int b = 0; b < ns; ++b)
      for (int x = 0; x < (1 << tp.blocks[b].w); ++x) {
        cd v0, v1;
        uint32_t cur = 0;
        if (!track_column(tp.blocks[b], CsFromTable{sh.cs}, none, x, v0, v1, &cur))
          return fail(SV_EINVAL, "circuit template is not monomial in its block basis");
        const double norm = tp.blocks[b].type == 0 ? 1.0 / (double)(1 << tp.blocks[b].w) : 1.0;
        sh.Dc[b][0][x] = C2<T>{(T)(v0.re * norm), (T)(v0.im * norm)};
        sh.Dc[b][1][x] = C2<T>{(T)(v1.re * norm), (T)(v1.im * norm)};
        sh.Wc[b][0][x] = (v0.re * v0.re + v0.im * v0.im) * norm;
        sh.Wc[b][1][x] = (v1.re * v1.re + v1.im * v1.im) * norm;
      }
    HIP_OK(hipMemcpyAsync(dshared, &sh, sizeof sh, hipMemcpyHostToDevice, s));
  }
  // logical |0> of the register: bit x set on the X-stabilizer orbit of 0
  std::vector<uint32_t> init_mask(16, 0u);
  for (uint32_t x = 0; x < (1u << n); ++x) {
    uint32_t r = x;
    for (int i = 0; i < jc.n_x; ++i)
      if (r & jc.span_piv[i]) r ^= jc.span_vec[i];
    if (r == 0) init_mask[x >> 5] |= 1u << (x & 31);
  }
  HIP_OK(hipMemcpyAsync(dinit, init_mask.data(), sizeof(uint32_t) * init_mask.size(), hipMemcpyHostToDevice, s));
  // kind of every draw of a round: 0 one-qubit location, 1 two-qubit
  // location, 2 measurement
  std::vector<uint8_t> kind(std::max(1, tp.n_draws), 2);
  for (const TBlock& b : tp.blocks)
    for (int k = 0; k + 1 < b.n_draws; ++k) kind[b.draw_off + k] = (uint8_t)((b.n2mask >> k) & 1);
  HIP_OK(hipMemcpyAsync(dkind, kind.data(), kind.size(), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dblocks, tp.blocks.data(), sizeof(TBlock) * ns, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dsd, sd.data(), sizeof(SmallDesc) * ns, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(djc, &jc, sizeof jc, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dorder, order.data(), sizeof(int) * nt, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(drounds, in.rounds, sizeof(int) * nt, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dp, in.p, sizeof(double) * nt, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dseed, in.seed, sizeof(uint64_t) * nt, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dstream, in.stream, sizeof(uint64_t) * nt, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(deps, in.eps, sizeof(double) * neps, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemsetAsync(drec, 0, nrec, s));
  HIP_OK(hipMemsetAsync(derr, 0, sizeof(int), s));
  {
    // a persistent launch: no more workgroups than stay resident at once
    // (the tuned waves per CU, nw waves per workgroup)
    auto launch = [&](auto kernel, int nwv) -> hipError_t {
      int per_cu = std::max(1, tuning_for(in.d, sizeof(T) == 8 ? SV_C128 : SV_C64).batch_waves_per_cu / nwv);
      int resident = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kernel, 64 * nwv, 0) == hipSuccess &&
          resident > 0)
        per_cu = std::min(per_cu, resident);
      const int max_wg = device_cu_count() * per_cu;
      const int grid = std::max(1, std::min(nt, max_wg));  // one trajectory per workgroup at a time
      hipError_t e = hipEventRecord(ev_a, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(64 * nwv), 0, s, dblocks, dsd, ns, n, tp.n_draws, djc,
                         dseed, dstream, dorder, nt, drounds, dp, deps, in.eps_stride, drec,
                         in.max_rounds, dbits, derr, (const TOp*)dsites, tp.n_sites,
                         (const SmallShared<T>*)dshared, (const uint32_t*)dinit, (const uint8_t*)dkind);
      return hipGetLastError();
    };
    if (nw == 4) HIP_OK(launch(k_batch_small<T, 4>, 4));
    else if (nw == 2) HIP_OK(launch(k_batch_small<T, 2>, 2));
    else HIP_OK(launch(k_batch_small<T, 1>, 1));
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(ev_b, s));
  int herr = 0;
  HIP_OK(hipMemcpyAsync(&herr, derr, sizeof herr, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(in.records, drec, nrec, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(in.final_bits, dbits, (size_t)nt * n, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (herr) return fail(SV_EINVAL, "circuit template is not monomial in its block basis");
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, ev_a, ev_b));
  in.gpu_ms = ms;
  return SV_OK;
}

// Batched trajectories too large for LDS, run in lockstep: every launch of
// the register pass covers (tile, trajectory) pairs, so thousands of
// 2^16-amplitude registers fill the GPU like one 2^25-amplitude register does.  Slots are the
// trajectories sorted by round count (longest first), so the trajectories still
// running in round r are always the first A(r) slots.
template <typename T>
sv_status run_batch_lockstep(BatchInputs& in, const Template& tp) {
  const int d = in.d, n = d * d, ns = (int)tp.blocks.size(), nt = in.n_traj;
  const int tb = std::min(kTileMax, n);
  const size_t n_tiles = (size_t)1 << (n - tb);
  const int cb = std::min(12, n);
  const size_t reg = (size_t)2 << n;  // T elements per register
  const size_t per_reg_bytes = reg * sizeof(T);
  const sv_tuning tune = tuning_for(d, sizeof(T) == 8 ? SV_C128 : SV_C64);
  const size_t cap = (size_t)tune.lockstep_mib << 20;
  const int per_traj = in.max_rounds * ns;
  const std::vector<Unit> units = make_units_paired(tp, tune.zchain, n, tune.xpair);
  const int nu = (int)units.size();
  // speculative units (as for one register: on when zeta = 0 unless
  // QECSV_SPEC says otherwise); each slot then holds two registers
  const int spec_env = env_int("QECSV_SPEC", -1);
  bool spec = (spec_env < 0 ? in.zeta == 0.0 : spec_env != 0) && !tp.any_dense;
  std::vector<Unit> sunits;
  std::vector<UnitPass> spds;
  if (spec) {
    sunits = make_spec_units(tp, tune.zchain, n);
    spds = make_spec_passes(n, tb, tp, sunits);
    for (const UnitPass& h : spds)
      if (h.tb <= 0 || (h.bkind == U_Z && h.bmode == 0)) spec = false;
  }
  const int nus = spec ? (int)sunits.size() : 0;
  const int G = (int)std::max<size_t>(1, std::min<size_t>((size_t)nt, cap / (per_reg_bytes * (spec ? 2 : 1))));
  const size_t dec_stride = (size_t)in.max_rounds * (spec ? nus : nu) + 1;
  const size_t ctl_stride = (size_t)in.max_rounds * nus;
  const int n_sites = std::max(1, tp.n_sites);
  hipStream_t s = in.hs;
  DevBufs M(s);
  TBlock* dblocks = nullptr;
  UnitPass* dpass = nullptr;
  JobConst* djc = nullptr;
  T* st = nullptr;
  double* partials = nullptr;
  Decision* ddec = nullptr;
  BlockRT *rtA = nullptr, *rtB = nullptr;
  uint64_t *dseed = nullptr, *dstream = nullptr;
  double *dp = nullptr, *deps = nullptr, *dsums = nullptr;
  int *drounds = nullptr, *derr = nullptr;
  uint8_t *drec = nullptr, *dbits = nullptr;
  HIP_OK(M.alloc(&dblocks, sizeof(TBlock) * ns));
  HIP_OK(M.alloc(&dpass, sizeof(UnitPass) * (nu + 2)));
  HIP_OK(M.alloc(&djc, sizeof(JobConst)));
  HIP_OK(M.alloc(&st, per_reg_bytes * G));
  HIP_OK(M.alloc(&partials, sizeof(double) * kChainAcc * n_tiles * G));
  double* dacc = nullptr;
  unsigned* dticket = nullptr;
  HIP_OK(M.alloc(&dacc, sizeof(double) * kChainAcc * G));
  HIP_OK(M.alloc(&dticket, sizeof(unsigned) * G));
  HIP_OK(hipMemsetAsync(dticket, 0, sizeof(unsigned) * G, s));
  HIP_OK(M.alloc(&ddec, sizeof(Decision) * dec_stride * G));
  HIP_OK(M.alloc(&rtA, sizeof(BlockRT) * (size_t)ns * G));
  HIP_OK(M.alloc(&rtB, sizeof(BlockRT) * (size_t)ns * G));
  HIP_OK(M.alloc(&dseed, sizeof(uint64_t) * G));
  HIP_OK(M.alloc(&dstream, sizeof(uint64_t) * G));
  HIP_OK(M.alloc(&dp, sizeof(double) * G));
  HIP_OK(M.alloc(&deps, sizeof(double) * (size_t)n_sites * G));
  double* dcs = nullptr;
  HIP_OK(M.alloc(&dcs, sizeof(double) * 2 * (size_t)n_sites * G));
  HIP_OK(M.alloc(&dsums, (sizeof(double) << (n - cb)) * G));
  HIP_OK(M.alloc(&drounds, sizeof(int) * G));
  HIP_OK(M.alloc(&derr, sizeof(int)));
  HIP_OK(M.alloc(&drec, (size_t)per_traj * G));
  HIP_OK(M.alloc(&dbits, (size_t)n * G));
  T* st2 = nullptr;
  UnitPass* dspass = nullptr;
  SpecCtl* dctl = nullptr;
  uint8_t* dpred0 = nullptr;
  int* dredos = nullptr;
  std::vector<uint8_t> pred0;
  if (spec) {
    for (const TBlock& b : tp.blocks)
      pred0.push_back(in.gateset == SV_GATESET_CR ? (uint8_t)((b.w / 2) % 2) : (uint8_t)0);
    HIP_OK(M.alloc(&st2, per_reg_bytes * G));
    HIP_OK(M.alloc(&dspass, sizeof(UnitPass) * spds.size()));
    HIP_OK(M.alloc(&dctl, sizeof(SpecCtl) * ctl_stride * G));
    HIP_OK(M.alloc(&dpred0, pred0.size()));
    HIP_OK(M.alloc(&dredos, sizeof(int)));
    HIP_OK(hipMemcpyAsync(dspass, spds.data(), sizeof(UnitPass) * spds.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(dpred0, pred0.data(), pred0.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemsetAsync(dredos, 0, sizeof(int), s));
  }

  const std::vector<UnitPass> pds = make_unit_passes(n, tb, tp, units);
  const JobConst jc = make_job_const(d, in.zeta);
  HIP_OK(hipMemcpyAsync(dblocks, tp.blocks.data(), sizeof(TBlock) * ns, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dpass, pds.data(), sizeof(UnitPass) * (nu + 2), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(djc, &jc, sizeof jc, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemsetAsync(derr, 0, sizeof(int), s));

  std::vector<int> order(nt);
  for (int i = 0; i < nt; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return in.rounds[a] > in.rounds[b]; });
  // a: start, b: end; fork/join: the next round's Kraus pairs are built on a
  // second stream while the current round's passes run
  struct Ev {
    hipEvent_t a = nullptr, b = nullptr, fork = nullptr, join = nullptr;
    hipStream_t s2 = nullptr;
    ~Ev() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      if (fork) (void)hipEventDestroy(fork);
      if (join) (void)hipEventDestroy(join);
      if (s2) (void)hipStreamDestroy(s2);
    }
  } ev;
  HIP_OK(hipEventCreate(&ev.a));
  HIP_OK(hipEventCreate(&ev.b));
  HIP_OK(hipEventCreateWithFlags(&ev.fork, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&ev.join, hipEventDisableTiming));
  HIP_OK(hipStreamCreateWithFlags(&ev.s2, hipStreamNonBlocking));
  const dim3 block((unsigned)std::max(64, 1 << (tb - 4)));
  const SlotStrides ss{reg, (size_t)ns, dec_stride};
  // pass workgroups per slot, each taking tiles grid-stride: four tiles each
  // for passes that sum a Z chain or write logical |0> (their tables - up to
  // four chain members' weights, a phase table per layer count - are loaded
  // once for four tiles: d=4 Z-chain passes 216-253 -> 201-202 ns per slot),
  // one tile each for the X-check passes (183 ns per slot; 199 with four)
  auto gx_of = [&](const UnitPass& p) {
    const bool heavy = p.bkind == U_Z || p.akind == U_INIT;
    return (unsigned)std::max<size_t>(1, heavy ? n_tiles / 4 : n_tiles);
  };
  std::vector<uint64_t> hseed(G), hstream(G);
  std::vector<double> hp(G), heps((size_t)n_sites * G);
  std::vector<int> hrounds(G);
  std::vector<uint8_t> hrec((size_t)per_traj * G), hbits((size_t)n * G);
  std::memset(in.records, 0, (size_t)nt * per_traj);
  int pass_no = 0;
  HIP_OK(hipEventRecord(ev.a, s));
  for (int g0 = 0; g0 < nt; g0 += G) {
    const int gn = std::min(G, nt - g0);
    for (int i = 0; i < gn; ++i) {
      const int t = order[g0 + i];
      hseed[i] = in.seed[t];
      hstream[i] = in.stream[t];
      hp[i] = in.p[t];
      hrounds[i] = in.rounds[t];
      for (int k = 0; k < tp.n_sites; ++k)
        heps[(size_t)i * n_sites + k] = in.eps[(size_t)t * in.eps_stride + k];
    }
    HIP_OK(hipMemcpyAsync(dseed, hseed.data(), sizeof(uint64_t) * gn, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(dstream, hstream.data(), sizeof(uint64_t) * gn, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(dp, hp.data(), sizeof(double) * gn, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(deps, heps.data(), sizeof(double) * n_sites * gn, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(drounds, hrounds.data(), sizeof(int) * gn, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemsetAsync(drec, 0, (size_t)per_traj * gn, s));
    auto active = [&](int r) {  // slots with more than r rounds (a prefix)
      int a = 0;
      while (a < gn && hrounds[a] > r) ++a;
      return a;
    };
    {
      const int64_t nth = (int64_t)gn * ns * kMaxOps;
      hipLaunchKernelGGL(k_site_cs, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, s, dblocks, ns,
                         deps, n_sites, n_sites, gn, dcs);
    }
    auto prepare = [&](hipStream_t q, int r, BlockRT* out, int slots) {
      const int64_t nth = (int64_t)slots * ns * 16;
      hipLaunchKernelGGL(k_prepare_round, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, q, dblocks,
                         ns, r, tp.n_draws, dseed, dstream, dp, dcs, n_sites, slots, out, derr);
    };
    // outcomes of unit u of round r (tables of that round at rt) from the
    // partials of a pass of gx workgroups per slot
    auto decide = [&](int slots, const BlockRT* rt, int r, int u, unsigned gx) {
      const int bi = r * ns + units[u].first;
      const int lb = units[u].len;
      hipLaunchKernelGGL(k_udecide, dim3(slots), dim3(64), 0, s, partials, (int)gx, lb,
                         rt + units[u].first, ddec + (size_t)r * nu + u, drec + bi, (double*)nullptr,
                         ss, (size_t)per_traj, dacc, dticket, 0);
    };
    prepare(s, 0, rtA, gn);
    const int R0 = hrounds[0];
    // final Z measurement of the slots [from, from + cnt) on register buffer
    // buf, their frames in the decision records at dfin
    auto measure = [&](const T* buf, int from, int cnt, const Decision* dfin) {
      hipLaunchKernelGGL(k_final_sums<T>, dim3(1u << (n - cb), cnt), dim3(256), 0, s, buf + (size_t)from * reg, cb,
                         dsums, reg);
      hipLaunchKernelGGL(k_final_measure<T>, dim3(cnt), dim3(1024), 0, s, buf + (size_t)from * reg, n, cb, dsums,
                         (uint64_t)0, (uint64_t)0, (uint64_t)0, dbits + (size_t)from * n, reg, dseed + from,
                         dstream + from, drounds + from, (uint64_t)tp.n_draws, dfin, dec_stride);
    };
    if (spec) {
      // speculative units: logical |0> into st, then per unit of every round
      // its prediction pass over the active slots (st <-> st2 for all of
      // them), the decision and the redos (see run_rounds_t)
      T* cur = st;
      T* oth = st2;
      hipLaunchKernelGGL(k_dec_init, dim3((unsigned)((gn + 255) / 256)), dim3(256), 0, s, ddec, gn, dec_stride);
      SV_OK_OR_RETURN(launch_upass<T>(spds[0], dim3(gx_of(spds[0]), gn), block, s, cur, &dspass[0], djc, nullptr,
                                      nullptr, nullptr, ddec, partials, 0, ss));
      int ui = 0;
      for (int r = 0; r < R0; ++r) {
        const int Ar = active(r), An = active(r + 1);
        BlockRT* rt_cur = (r & 1) ? rtB : rtA;
        BlockRT* rt_nxt = (r & 1) ? rtA : rtB;
        if (An > 0) {
          HIP_OK(hipEventRecord(ev.fork, s));
          HIP_OK(hipStreamWaitEvent(ev.s2, ev.fork, 0));
          prepare(ev.s2, r + 1, rt_nxt, An);
          HIP_OK(hipEventRecord(ev.join, ev.s2));
        }
        for (int u = 0; u < nus; ++u, ++ui) {
          const Unit& U = sunits[u];
          const bool zb = U.kind == U_Z;
          const UnitPass& h = spds[1 + u];
          const unsigned gx = gx_of(h);
          const int bi = r * ns + U.first;
          const SpecArgs sa{oth, dctl + ui, r == 0 ? dpred0 + U.first : drec + bi - ns, dredos, ctl_stride,
                            r == 0 ? (size_t)0 : (size_t)per_traj};
          const BlockRT* rtu = rt_cur + U.first;
          const int rev = (++pass_no) & 1;
          // redo grid: a quarter of the pass's workgroups per slot.  Nearly
          // every redo launch has some slot to redo among thousands, and a
          // full-width grid mostly dispatches workgroups that return at once
          // (d=4, 4096 trajectories: 38.7 ms per launch; 39.0 full width,
          // 40.7 with two and 44.9 with one workgroup per slot)
          const unsigned gr = std::max(1u, gx / 4);
          auto pass = [&](bool redo) {
            return launch_spass<T>(h, redo, dim3(redo ? gr : gx, Ar), block, s, cur, &dspass[1 + u], djc,
                                   zb ? nullptr : rtu, zb ? rtu : nullptr, ddec + ui, ddec + ui + 1, partials, rev,
                                   sa, ss);
          };
          auto sdecide = [&](unsigned parts) {
            hipLaunchKernelGGL(k_sdecide, dim3(Ar), dim3(64), 0, s, partials, (int)parts, U.len, zb ? 1 : 0, rtu,
                               ddec + ui, ddec + ui + 1, drec + bi, (double*)nullptr, dctl + ui, dacc, dticket, ss,
                               (size_t)per_traj, ctl_stride, 0);
          };
          SV_OK_OR_RETURN(pass(false));
          sdecide(gx);
          const int redos = (!zb && U.len == 2) ? 2 : 1;
          for (int k = 0; k < redos; ++k) {
            SV_OK_OR_RETURN(pass(true));
            if (k + 1 < redos) sdecide(gr);
          }
          std::swap(cur, oth);
        }
        if (An > 0) HIP_OK(hipStreamWaitEvent(s, ev.join, 0));
        if (Ar > An) measure(cur, An, Ar - An, ddec + (size_t)An * dec_stride + ui);
        HIP_OK(hipGetLastError());
      }
    } else {
    SV_OK_OR_RETURN(launch_upass<T>(pds[0], dim3(gx_of(pds[0]), gn), block, s, st, &dpass[0], djc,
                                    nullptr, rtA + units[0].first, nullptr, ddec, partials, 0, ss));
    decide(gn, rtA, 0, 0, gx_of(pds[0]));
    for (int r = 0; r < R0; ++r) {
      const int Ar = active(r), An = active(r + 1);
      BlockRT* rt_cur = (r & 1) ? rtB : rtA;
      BlockRT* rt_nxt = (r & 1) ? rtA : rtB;
      if (An > 0) {
        // rt_nxt was last read by the previous round's passes, enqueued above
        HIP_OK(hipEventRecord(ev.fork, s));
        HIP_OK(hipStreamWaitEvent(ev.s2, ev.fork, 0));
        prepare(ev.s2, r + 1, rt_nxt, An);
        HIP_OK(hipEventRecord(ev.join, ev.s2));
      }
      for (int u = 0; u < nu; ++u) {
        const int ui = r * nu + u;
        // the round's last pass sums the next round's first unit
        if (u == nu - 1 && An > 0) HIP_OK(hipStreamWaitEvent(s, ev.join, 0));
        const int rev = (++pass_no) & 1;
        const BlockRT* rta = rt_cur + units[u].first;
        if (u < nu - 1) {
          SV_OK_OR_RETURN(launch_upass<T>(pds[1 + u], dim3(gx_of(pds[1 + u]), Ar), block, s, st,
                                          &dpass[1 + u], djc, rta, rt_cur + units[u + 1].first,
                                          ddec + ui, ddec + ui + 1, partials, rev, ss));
          decide(Ar, rt_cur, r, u + 1, gx_of(pds[1 + u]));
          continue;
        }
        if (An > 0) {
          SV_OK_OR_RETURN(launch_upass<T>(pds[1 + u], dim3(gx_of(pds[1 + u]), An), block, s, st,
                                          &dpass[1 + u], djc, rta, rt_nxt + units[0].first,
                                          ddec + ui, ddec + ui + 1, partials, rev, ss));
          decide(An, rt_nxt, r + 1, 0, gx_of(pds[1 + u]));
        }
        if (Ar > An) {  // trajectories ending with this round
          const int cnt = Ar - An;
          Decision* dfin = ddec + (size_t)An * dec_stride + ui + 1;
          SV_OK_OR_RETURN(launch_upass<T>(pds[nu + 1], dim3(gx_of(pds[nu + 1]), cnt), block, s,
                                          st + (size_t)An * reg, &dpass[nu + 1], djc,
                                          rta + (size_t)An * ns, nullptr,
                                          ddec + (size_t)An * dec_stride + ui, dfin, partials, rev, ss));
          measure(st, An, cnt, dfin);
        }
      }
      HIP_OK(hipGetLastError());
    }
    }
    HIP_OK(hipMemcpyAsync(hrec.data(), drec, (size_t)per_traj * gn, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hbits.data(), dbits, (size_t)n * gn, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < gn; ++i) {
      const int t = order[g0 + i];
      std::memcpy(in.records + (size_t)t * per_traj, hrec.data() + (size_t)i * per_traj,
                  (size_t)hrounds[i] * ns);
      std::memcpy(in.final_bits + (size_t)t * n, hbits.data() + (size_t)i * n, n);
    }
  }
  HIP_OK(hipEventRecord(ev.b, s));
  int herr = 0;
  HIP_OK(hipMemcpyAsync(&herr, derr, sizeof herr, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (herr) return fail(SV_EINVAL, "circuit template is not monomial in its block basis");
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, ev.a, ev.b));
  in.gpu_ms = ms;
  in.passes_per_round = spec ? nus : nu;
  in.redo_passes = 0;
  if (spec) {
    HIP_OK(hipMemcpyAsync(&in.redo_passes, dredos, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  return SV_OK;
}

// Device bytes one batched launch of n_traj trajectories holds (admission).
size_t batch_footprint(int d, int dtype, int n_traj, int max_rounds, int n_sites) {
  const int n = d * d;
  const size_t elem = dtype == SV_C128 ? 16 : 8;
  size_t b = (size_t)n_traj * ((size_t)max_rounds * (n + 1) + n + 40 + 8 * (size_t)n_sites);
  if (n > kSmallBits) {
    // lockstep: G registers with their partial sums and decisions
    const size_t reg = elem << n;
    const size_t cap = (size_t)tuning_for(d, dtype).lockstep_mib << 20;
    const size_t G = std::max<size_t>(1, std::min<size_t>((size_t)n_traj, cap / reg));
    // speculative units hold two registers per slot in groups half as large
    const size_t G2 = std::max<size_t>(1, std::min<size_t>((size_t)n_traj, cap / (2 * reg)));
    const size_t n_tiles = (size_t)1 << (n - std::min(kTileMax, n));
    b += std::max(G, 2 * G2) * reg +
         G * (sizeof(double) * kChainAcc * n_tiles + sizeof(Decision) * (size_t)max_rounds * n);
  }
  return b + (1 << 20);
}

}  // namespace

// ==================================================================== ABI ==
struct sv_state_s {
  void* ptr = nullptr;
  size_t bytes = 0;
  int n = 0;
  sv_dtype dt = SV_C128;
  hipStream_t stream = nullptr;
  bool owned = false;
  double2* partials = nullptr;
  MeasOut* mo = nullptr;
  // Matrix uploads of sv_apply_fused: a ring of pinned host slots and device
  // slots; a slot is reused once the event recorded after its kernel fired.
  double* mat_host = nullptr;
  double* mat_dev = nullptr;
  hipEvent_t mat_ev[8] = {};
  bool mat_used[8] = {};
  int mat_next = 0;
};

static constexpr int kMeasGrid = 1024;
static constexpr int kMatSlots = 8;
static constexpr size_t kMatDoubles = 2 * 32 * 32;

extern "C" {

const char* sv_last_error(void) { return g_err.c_str(); }

int sv_version(void) { return 100; }

static size_t elem_size(sv_dtype dt) { return dt == SV_C128 ? 16 : 8; }

static sv_status make_state(void* ptr, size_t bytes, int n, sv_dtype dt, void* stream, bool owned,
                            sv_state* out) {
  sv_state s = new (std::nothrow) sv_state_s;
  if (!s) return fail(SV_ENOMEM, "host allocation failed");
  s->ptr = ptr;
  s->bytes = bytes;
  s->n = n;
  s->dt = dt;
  s->stream = (hipStream_t)stream;
  s->owned = owned;
  void* scratch = nullptr;
  const size_t sb = sizeof(double2) * kMeasGrid + 256 + sizeof(MeasOut);
  if (hipMalloc(&scratch, sb) != hipSuccess) {
    delete s;
    return fail(SV_ENOMEM, "scratch allocation failed");
  }
  s->partials = (double2*)scratch;
  s->mo = (MeasOut*)((char*)scratch + sizeof(double2) * kMeasGrid + 256);
  *out = s;
  return SV_OK;
}

sv_status sv_alloc(int n_qubits, sv_dtype dtype, void* hip_stream, sv_state* out) {
  if (!out) return fail(SV_EINVAL, "out is NULL");
  if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d out of 1..34", n_qubits);
  if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  const size_t bytes = elem_size(dtype) << n_qubits;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(SV_ENOMEM, "hipMalloc(%zu) failed", bytes);
  sv_status st = make_state(p, bytes, n_qubits, dtype, hip_stream, true, out);
  if (st != SV_OK) {
    (void)hipFree(p);
    return st;
  }
  return sv_set_basis(*out, 0);
}

sv_status sv_wrap(void* dev_ptr, size_t bytes, int n_qubits, sv_dtype dtype, void* hip_stream,
                  sv_state* out) {
  if (!out || !dev_ptr) return fail(SV_EINVAL, "NULL pointer");
  if (n_qubits < 1 || n_qubits > 34) return fail(SV_EINVAL, "n_qubits %d out of 1..34", n_qubits);
  if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  if (((uintptr_t)dev_ptr) % 16) return fail(SV_EINVAL, "dev_ptr not 16-byte aligned");
  const size_t need = elem_size(dtype) << n_qubits;
  if (bytes < need) return fail(SV_EINVAL, "buffer of %zu bytes < %zu needed", bytes, need);
  return make_state(dev_ptr, need, n_qubits, dtype, hip_stream, false, out);
}

sv_status sv_free(sv_state s) {
  if (!s) return SV_OK;
  (void)hipStreamSynchronize(s->stream);
  if (s->owned) (void)hipFree(s->ptr);
  (void)hipFree(s->partials);
  if (s->mat_dev) {
    for (int i = 0; i < kMatSlots; ++i) (void)hipEventDestroy(s->mat_ev[i]);
    (void)hipHostFree(s->mat_host);
    (void)hipFree(s->mat_dev);
  }
  delete s;
  return SV_OK;
}

sv_status sv_synchronize(sv_state s) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  HIP_OK(hipStreamSynchronize(s->stream));
  return SV_OK;
}

sv_status sv_set_state(sv_state s, const void* host, size_t bytes) {
  if (!s || !host) return fail(SV_EINVAL, "NULL pointer");
  if (bytes != s->bytes) return fail(SV_EINVAL, "expected %zu bytes, got %zu", s->bytes, bytes);
  HIP_OK(hipStreamSynchronize(s->stream));
  HIP_OK(hipMemcpy(s->ptr, host, bytes, hipMemcpyHostToDevice));
  return SV_OK;
}

sv_status sv_get_state(sv_state s, void* host, size_t bytes) {
  if (!s || !host) return fail(SV_EINVAL, "NULL pointer");
  if (bytes != s->bytes) return fail(SV_EINVAL, "expected %zu bytes, got %zu", s->bytes, bytes);
  HIP_OK(hipStreamSynchronize(s->stream));
  HIP_OK(hipMemcpy(host, s->ptr, bytes, hipMemcpyDeviceToHost));
  return SV_OK;
}

static unsigned grid_for(uint64_t n, unsigned block) {
  return (unsigned)((n + block - 1) / block);
}

sv_status sv_copy_state(sv_state dst, sv_state src) {
  if (!dst || !src) return fail(SV_EINVAL, "NULL state");
  if (dst->n != src->n || dst->dt != src->dt) return fail(SV_EINVAL, "registers differ in size or dtype");
  if (dst->ptr == src->ptr) return SV_OK;
  // order the copy after both registers' pending work, on dst's stream
  if (src->stream != dst->stream) HIP_OK(hipStreamSynchronize(src->stream));
  const uint64_t n16 = dst->bytes / 16;
  const unsigned grid = (unsigned)std::min<uint64_t>((n16 + 4 * 256 - 1) / (4 * 256), 1u << 20);
  hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, dst->stream, (double2*)dst->ptr,
                     (const double2*)src->ptr, n16);
  HIP_OK(hipGetLastError());
  return SV_OK;
}

sv_status sv_set_basis(sv_state s, uint64_t index) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  const uint64_t na = 1ull << s->n;
  if (index >= na) return fail(SV_EINVAL, "basis index out of range");
  if (s->dt == SV_C128)
    hipLaunchKernelGGL(k_fill_basis<double>, dim3(grid_for(na, 256)), dim3(256), 0, s->stream,
                       (double*)s->ptr, na, index);
  else
    hipLaunchKernelGGL(k_fill_basis<float>, dim3(grid_for(na, 256)), dim3(256), 0, s->stream,
                       (float*)s->ptr, na, index);
  HIP_OK(hipGetLastError());
  return SV_OK;
}

sv_status sv_load_logical0(sv_state s, int d) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (s->n < d * d) return fail(SV_EINVAL, "register of %d qubits < d^2 = %d", s->n, d * d);
  JobConst jc = make_job_const(d, 0.0);
  JobConst* djc = nullptr;
  HIP_OK(hipMalloc(&djc, sizeof(JobConst)));
  hipError_t e = hipMemcpyAsync(djc, &jc, sizeof jc, hipMemcpyHostToDevice, s->stream);
  const uint64_t na = 1ull << s->n;
  if (e == hipSuccess) {
    if (s->dt == SV_C128)
      hipLaunchKernelGGL(k_logical0<double>, dim3(grid_for(na, 256)), dim3(256), 0, s->stream,
                         (double*)s->ptr, na, djc);
    else
      hipLaunchKernelGGL(k_logical0<float>, dim3(grid_for(na, 256)), dim3(256), 0, s->stream,
                         (float*)s->ptr, na, djc);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(djc);
  if (e != hipSuccess) return fail(SV_EDEVICE, "logical0: %s", hipGetErrorString(e));
  return SV_OK;
}

static sv_status check_qubits(const sv_state s, int k, const int* qubits, int kmax) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  if (!qubits) return fail(SV_EINVAL, "NULL qubits");
  if (k < 1 || k > kmax) return fail(SV_EINVAL, "k=%d out of 1..%d", k, kmax);
  if (k > s->n) return fail(SV_EINVAL, "k=%d > n=%d", k, s->n);
  for (int i = 0; i < k; ++i) {
    if (qubits[i] < 0 || qubits[i] >= s->n) return fail(SV_EINVAL, "qubit %d out of range", qubits[i]);
    for (int j = 0; j < i; ++j)
      if (qubits[i] == qubits[j]) return fail(SV_EINVAL, "duplicate qubit %d", qubits[i]);
  }
  return SV_OK;
}

sv_status sv_apply_gate(sv_state s, int k, const int* qubits, const double* m) {
  sv_status st = check_qubits(s, k, qubits, 2);
  if (st != SV_OK) return st;
  if (!m) return fail(SV_EINVAL, "NULL matrix");
  const uint64_t na = 1ull << s->n;
  if (k == 1) {
    Mat2 M;
    std::memcpy(M.m, m, sizeof M.m);
    const uint64_t np = na >> 1;
    if (s->dt == SV_C128)
      hipLaunchKernelGGL(k_gate1<double>, dim3(grid_for(np, 256)), dim3(256), 0, s->stream,
                         (double*)s->ptr, np, qubits[0], M);
    else
      hipLaunchKernelGGL(k_gate1<float>, dim3(grid_for(np, 256)), dim3(256), 0, s->stream,
                         (float*)s->ptr, np, qubits[0], M);
  } else if (qubits[0] + qubits[1] == 1 && s->n >= 9) {
    // qubits 0 and 1: one amplitude per thread, quadruples exchanged within
    // DPP quads (whole 256-thread blocks)
    Mat4 M;
    std::memcpy(M.m, m, sizeof M.m);
    const dim3 g((unsigned)(na / 256)), b(256);
    const int swap = qubits[0] == 1;
    if (s->dt == SV_C128)
      hipLaunchKernelGGL(k_gate2_quad<double>, g, b, 0, s->stream, (double*)s->ptr, swap, M);
    else  // two amplitudes per thread: half the threads
      hipLaunchKernelGGL(k_gate2_pair_f32, dim3((unsigned)(na / 512)), b, 0, s->stream, (float*)s->ptr,
                         swap, M);
  } else {
    Mat4 M;
    std::memcpy(M.m, m, sizeof M.m);
    const uint64_t nq = na >> 2;
    if (s->dt == SV_C128)
      hipLaunchKernelGGL(k_gate2<double>, dim3(grid_for(nq, 256)), dim3(256), 0, s->stream,
                         (double*)s->ptr, nq, qubits[0], qubits[1], M);
    else
      hipLaunchKernelGGL(k_gate2<float>, dim3(grid_for(nq, 256)), dim3(256), 0, s->stream,
                         (float*)s->ptr, nq, qubits[0], qubits[1], M);
  }
  HIP_OK(hipGetLastError());
  return SV_OK;
}

sv_status sv_apply_diag(sv_state s, int k, const int* qubits, const double* phases) {
  sv_status st = check_qubits(s, k, qubits, 5);
  if (st != SV_OK) return st;
  if (!phases) return fail(SV_EINVAL, "NULL phases");
  Diag32 D{};
  std::memcpy(D.ph, phases, sizeof(double) * 2 * (1 << k));
  int q[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < k; ++i) q[i] = qubits[i];
  const uint64_t na = 1ull << s->n;
  if (s->dt == SV_C128)
    hipLaunchKernelGGL(k_diag<double>, dim3(grid_for(na, 256)), dim3(256), 0, s->stream,
                       (double*)s->ptr, na, k, q[0], q[1], q[2], q[3], q[4], D);
  else
    hipLaunchKernelGGL(k_diag<float>, dim3(grid_for(na, 256)), dim3(256), 0, s->stream,
                       (float*)s->ptr, na, k, q[0], q[1], q[2], q[3], q[4], D);
  HIP_OK(hipGetLastError());
  return SV_OK;
}

}  // extern "C"

// Whether the MFMA fused kernel prefetches the next tile (more loads in
// flight per wave, more registers).  Measured on the 26-qubit register: it
// pays only for complex64 with k = 5 (254 -> 245 us); for complex128, k = 5 it
// costs a wave per SIMD of occupancy (441 -> 457 us).
template <typename T, int K> struct FusedPF {
  static constexpr bool value = sizeof(T) == 4 && K == 5;
};

// Persistent grid for the MFMA fused kernels: every resident workgroup, at
// most one wave per 16-group tile.
template <typename T, int K, bool LOW>
static unsigned fused_mfma_grid(uint64_t n_tiles) {
  static const int per_cu = [] {
    int b = 0;
    hipError_t e;
    if constexpr (LOW)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_fused_mfma_low<T, K>, 256, 0);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_fused_mfma<T, K, FusedPF<T, K>::value>, 256, 0);
    if (e != hipSuccess || b < 1) b = 1;
    return b;
  }();
  const uint64_t want = (n_tiles + 3) / 4, cap = (uint64_t)device_cu_count() * per_cu;
  return (unsigned)std::min(want, cap);
}

extern "C" {

static sv_status fused_slots(sv_state s) {
  if (s->mat_dev) return SV_OK;
  const size_t bytes = sizeof(double) * kMatDoubles * kMatSlots;
  if (hipHostMalloc((void**)&s->mat_host, bytes, hipHostMallocDefault) != hipSuccess) {
    s->mat_host = nullptr;
    return fail(SV_ENOMEM, "pinned matrix slots (%zu bytes) failed", bytes);
  }
  if (hipMalloc((void**)&s->mat_dev, bytes) != hipSuccess) {
    (void)hipHostFree(s->mat_host);
    s->mat_host = nullptr;
    s->mat_dev = nullptr;
    return fail(SV_ENOMEM, "device matrix slots (%zu bytes) failed", bytes);
  }
  for (int i = 0; i < kMatSlots; ++i) {
    if (hipEventCreateWithFlags(&s->mat_ev[i], hipEventDisableTiming) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(s->mat_ev[j]);
      (void)hipHostFree(s->mat_host);
      (void)hipFree(s->mat_dev);
      s->mat_host = nullptr;
      s->mat_dev = nullptr;
      return fail(SV_EDEVICE, "event creation failed");
    }
    s->mat_used[i] = false;
  }
  return SV_OK;
}

sv_status sv_apply_fused(sv_state s, int k, const int* qubits, const double* m) {
  sv_status st = check_qubits(s, k, qubits, 5);
  if (st != SV_OK) return st;
  if (!m) return fail(SV_EINVAL, "NULL matrix");
  st = fused_slots(s);
  if (st != SV_OK) return st;
  const size_t nd = 2u << (2 * k), mb = sizeof(double) * nd;
  const int slot = s->mat_next;
  // the slot's previous copy and kernel must be done before it is rewritten
  if (s->mat_used[slot]) HIP_OK(hipEventSynchronize(s->mat_ev[slot]));
  double* hm = s->mat_host + kMatDoubles * slot;
  double* dm = s->mat_dev + kMatDoubles * slot;
  std::memcpy(hm, m, mb);
  HIP_OK(hipMemcpyAsync(dm, hm, mb, hipMemcpyHostToDevice, s->stream));
  int q[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < k; ++i) q[i] = qubits[i];
  const uint64_t ng = 1ull << (s->n - k);
  // 16x16 MFMA tiles need 16 rows (k >= 4) and 16 groups per tile
  const bool mfma = k >= 4 && s->n - k >= 4;
  // complex64, targets = the k lowest bits: contiguous groups, staged through
  // LDS (26 qubits, k = 5: 298 -> 222 us; complex128 gains nothing there,
  // 436 -> 472 us, and keeps the direct kernel)
  bool low = mfma && s->dt == SV_C64;
  for (int i = 0; i < k; ++i) low = low && q[i] < k;
  const dim3 g(grid_for(ng, 256)), b(256);
#define QEC_FUSED(K)                                                                             \
  case K:                                                                                       \
    if (s->dt == SV_C128)                                                                       \
      hipLaunchKernelGGL((k_fused<double, K>), g, b, 0, s->stream, (double*)s->ptr, ng, dm, q[0], \
                         q[1], q[2], q[3], q[4]);                                               \
    else                                                                                        \
      hipLaunchKernelGGL((k_fused<float, K>), g, b, 0, s->stream, (float*)s->ptr, ng, dm, q[0],   \
                         q[1], q[2], q[3], q[4]);                                               \
    break;
#define QEC_FUSED_MFMA(K)                                                                        \
  case K:                                                                                       \
    if (low)                                                                                    \
      hipLaunchKernelGGL((k_fused_mfma_low<float, K>), dim3(fused_mfma_grid<float, K, true>(ng / 16)), \
                         b, 0, s->stream, (float*)s->ptr, ng / 16, dm, q[0], q[1], q[2], q[3], q[4]); \
    else if (s->dt == SV_C128)                                                                  \
      hipLaunchKernelGGL((k_fused_mfma<double, K, FusedPF<double, K>::value>),                  \
                         dim3(fused_mfma_grid<double, K, false>(ng / 16)), b, 0, s->stream,       \
                         (double*)s->ptr, ng / 16, dm, q[0], q[1], q[2], q[3], q[4]);            \
    else                                                                                        \
      hipLaunchKernelGGL((k_fused_mfma<float, K, FusedPF<float, K>::value>),                    \
                         dim3(fused_mfma_grid<float, K, false>(ng / 16)), b, 0, s->stream,        \
                         (float*)s->ptr, ng / 16, dm, q[0], q[1], q[2], q[3], q[4]);             \
    break;
  if (mfma) {
    switch (k) { QEC_FUSED_MFMA(4) QEC_FUSED_MFMA(5) }
  } else {
    switch (k) { QEC_FUSED(1) QEC_FUSED(2) QEC_FUSED(3) QEC_FUSED(4) QEC_FUSED(5) }
  }
#undef QEC_FUSED
#undef QEC_FUSED_MFMA
  hipError_t e = hipGetLastError();
  // the copy is queued whatever the launch did: the slot stays busy until
  // the stream has passed this point
  s->mat_next = (slot + 1) % kMatSlots;
  const hipError_t er = hipEventRecord(s->mat_ev[slot], s->stream);
  if (er == hipSuccess) {
    s->mat_used[slot] = true;
  } else {
    s->mat_used[slot] = false;
    (void)hipStreamSynchronize(s->stream);
  }
  if (e == hipSuccess) e = er;
  if (e != hipSuccess) return fail(SV_EDEVICE, "apply_fused: %s", hipGetErrorString(e));
  return SV_OK;
}

static sv_status measure_common(sv_state s, int anc, double u, int forced, int* outcome, double* p1) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  if (anc < 0 || anc >= s->n) return fail(SV_EINVAL, "qubit %d out of range", anc);
  const uint64_t na = 1ull << s->n;
  const unsigned grid = (unsigned)std::min<uint64_t>(kMeasGrid, std::max<uint64_t>(1, na / 1024));
  if (s->dt == SV_C128)
    hipLaunchKernelGGL(k_measure_sums<double>, dim3(grid), dim3(256), 0, s->stream,
                       (const double*)s->ptr, na, anc, s->partials);
  else
    hipLaunchKernelGGL(k_measure_sums<float>, dim3(grid), dim3(256), 0, s->stream,
                       (const float*)s->ptr, na, anc, s->partials);
  hipLaunchKernelGGL(k_measure_decide, dim3(1), dim3(256), 0, s->stream, s->partials, (int)grid, u,
                     forced, s->mo);
  HIP_OK(hipGetLastError());
  if (forced >= 0) {
    MeasOut mo;
    HIP_OK(hipMemcpyAsync(&mo, s->mo, sizeof mo, hipMemcpyDeviceToHost, s->stream));
    HIP_OK(hipStreamSynchronize(s->stream));
    const double pf = (forced ? mo.S1 : mo.S0) / (mo.S0 + mo.S1);
    if (!(pf >= SV_TAU))
      return fail(SV_ENUMERIC, "forced outcome %d has probability %.3e < %.1e", forced, pf, SV_TAU);
  }
  const uint64_t np = na >> 1;
  if (s->dt == SV_C128)
    hipLaunchKernelGGL(k_project<double>, dim3(grid_for(np, 256)), dim3(256), 0, s->stream,
                       (double*)s->ptr, np, anc, s->mo);
  else
    hipLaunchKernelGGL(k_project<float>, dim3(grid_for(np, 256)), dim3(256), 0, s->stream,
                       (float*)s->ptr, np, anc, s->mo);
  HIP_OK(hipGetLastError());
  MeasOut mo;
  HIP_OK(hipMemcpyAsync(&mo, s->mo, sizeof mo, hipMemcpyDeviceToHost, s->stream));
  HIP_OK(hipStreamSynchronize(s->stream));
  if (outcome) *outcome = mo.m;
  if (p1) *p1 = mo.p1;
  return SV_OK;
}

sv_status sv_measure_reset_ancilla(sv_state s, int anc, double u, int* outcome, double* p1) {
  if (!(u >= 0.0 && u < 1.0)) return fail(SV_EINVAL, "u must be in [0, 1)");
  return measure_common(s, anc, u, -1, outcome, p1);
}

sv_status sv_measure_reset_ancilla_forced(sv_state s, int anc, int outcome, double* p1) {
  if (outcome != 0 && outcome != 1) return fail(SV_EINVAL, "outcome must be 0 or 1");
  return measure_common(s, anc, 0.0, outcome, nullptr, p1);
}

sv_status sv_template_info(int d, int gateset, int* n_stab, int* n_sites, int* n_draws_per_round) {
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (gateset != SV_GATESET_CR && gateset != SV_GATESET_TEXTBOOK) return fail(SV_EINVAL, "bad gateset");
  const Template T = build_template(d, gateset);
  if (n_stab) *n_stab = (int)T.blocks.size();
  if (n_sites) *n_sites = T.n_sites;
  if (n_draws_per_round) *n_draws_per_round = T.n_draws;
  return SV_OK;
}

sv_status sv_check_spec_layouts(int d, int gateset, int zchain, int* n_units) {
  if (!n_units) return fail(SV_EINVAL, "NULL n_units");
  *n_units = 0;
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (gateset != SV_GATESET_CR && gateset != SV_GATESET_TEXTBOOK) return fail(SV_EINVAL, "bad gateset");
  if (zchain < 1 || zchain > kChainMax) return fail(SV_EINVAL, "zchain %d out of 1..%d", zchain, kChainMax);
  const Template tp = build_template(d, gateset);
  const int n = d * d;
  if (n < kTileMax) return SV_OK;  // the plain passes
  const int tb = std::min(kTileMax, n);
  const std::vector<Unit> units = make_spec_units(tp, zchain, n);
  const std::vector<UnitPass> pds = make_spec_passes(n, tb, tp, units);
  for (const UnitPass& h : pds)
    if (h.tb <= 0 || (h.bkind == U_Z && h.bmode == 0)) return SV_OK;  // the plain passes
  auto bits_of = [](const uint32_t* m, int k) {
    uint32_t r = 0;
    for (int i = 0; i < k; ++i) r |= m[i];
    return r;
  };
  for (size_t u = 0; u < units.size(); ++u) {
    const UnitPass& h = pds[1 + u];
    if (units[u].kind != U_XP) continue;
    const uint32_t tile = bits_of(h.tid_g, h.tb - 4) | bits_of(h.j_g, 16);
    const uint32_t tile_p = bits_of(h.p_tid_g[0], h.tb - 4) | bits_of(h.p_j_g[0], 16);
    uint32_t q0 = 0, q1 = 0;
    for (int l = 0; l < h.aw[0]; ++l) q0 |= h.aq[0][l];
    for (int l = 0; l < h.aw[1]; ++l) q1 |= h.aq[1][l];
    if (__builtin_popcount(tile) != h.tb || tile_p != tile || (q0 & ~tile) || (q1 & ~tile))
      return fail(SV_EINVAL, "speculative unit %zu: the pair's tile does not hold both members", u);
    if ((q1 & ~bits_of(h.p_j_g[0], 16)) != 0)
      return fail(SV_EINVAL, "speculative unit %zu: second member not on its layout's register slots", u);
    if (h.pstore && (h.p_tid_g[0][0] != 1u || h.p_tid_g[0][1] != 2u || h.p_tid_g[0][2] != 4u))
      return fail(SV_EINVAL, "speculative unit %zu: stored from a layout without the lowest bits on its lanes", u);
  }
  *n_units = (int)units.size();
  return SV_OK;
}

sv_status sv_check_pass_layouts(int d, int gateset, int zchain, int xpair, int* n_passes) {
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (gateset != SV_GATESET_CR && gateset != SV_GATESET_TEXTBOOK) return fail(SV_EINVAL, "bad gateset");
  if (zchain < 1 || zchain > kChainMax) return fail(SV_EINVAL, "zchain %d out of 1..%d", zchain, kChainMax);
  if (xpair != 0 && xpair != 1) return fail(SV_EINVAL, "xpair must be 0 or 1");
  const Template tp = build_template(d, gateset);
  const int n = d * d;
  const std::vector<Unit> units = make_units_paired(tp, zchain, n, xpair);
  const std::vector<UnitPass> pds = make_unit_passes(n, kTileMax, tp, units);
  const uint32_t all = (uint32_t)((1ull << n) - 1);
  auto bits_of = [](const uint32_t* m, int k) {
    uint32_t r = 0;
    for (int i = 0; i < k; ++i) r |= m[i];
    return r;
  };
  auto distinct = [](const uint32_t* m, int k) {
    uint32_t r = 0;
    for (int i = 0; i < k; ++i) {
      if (__builtin_popcount(m[i]) != 1 || (r & m[i])) return false;
      r |= m[i];
    }
    return true;
  };
  for (size_t k = 0; k < pds.size(); ++k) {
    const UnitPass& p = pds[k];
    const int nt = p.tb - 4;
    uint32_t slot[4];
    for (int b = 0; b < 4; ++b) slot[b] = p.j_g[1u << b];
    const uint32_t jm = bits_of(slot, 4), tm = bits_of(p.tid_g, nt), outer = bits_of(p.outer_bit, p.n_outer);
    const uint32_t tile = jm | tm;
    bool ok = p.tb == std::min(kTileMax, n) && distinct(slot, 4) && distinct(p.tid_g, nt) && (jm & tm) == 0 &&
              __builtin_popcount(tile) == p.tb && (tile & outer) == 0 && (tile | outer) == all &&
              distinct(p.outer_bit, p.n_outer);
    for (int j = 0; j < 16 && ok; ++j) {
      uint32_t g = 0;
      for (int b = 0; b < 4; ++b)
        if ((j >> b) & 1) g |= slot[b];
      ok = p.j_g[j] == g;
    }
    uint32_t UA = 0, UB = 0;
    for (int i = 0; i < p.la; ++i)
      for (int l = 0; l < p.aw[i]; ++l) UA |= p.aq[i][l];
    for (int i = 0; i < p.lb; ++i)
      for (int l = 0; l < p.bw[i]; ++l) UB |= p.bq[i][l];
    if (p.akind == U_X && !p.amix)  // WHT over the register slots
      for (int l = 0; l < p.wa && ok; ++l) ok = slot[l] == p.aq[0][l];
    if ((p.akind == U_X || p.akind == U_XP) && p.amix) {
      // A's qubits: lane bits among the thread's lowest four index bits, or
      // the lowest amix_r register slots; the local index tables match
      uint32_t seen = 0;
      for (int i = 0; i < nt && ok; ++i)
        if (p.a_tx[i]) {
          ok = i < 4 && ((p.amix_lanes >> i) & 1) && p.tid_g[i] == p.aq[0][__builtin_ctz(p.a_tx[i])];
          seen |= p.a_tx[i];
        }
      for (int b = 0; b < 4 && ok; ++b) {
        const uint32_t x = p.a_jx[1u << b];
        ok = b < p.amix_r ? (x != 0 && p.aq[0][__builtin_ctz(x)] == slot[b]) : x == 0;
        seen |= x;
      }
      ok = ok && seen == (1u << p.wa) - 1 && (tm & 0xFu) == 0xFu;
    }
    if (p.akind == U_Z && p.amode == 1) ok = ok && (jm & UA) == 0;
    if (p.bkind == U_Z && p.bmode == 1) ok = ok && (jm & UB) == 0;
    if (p.bmode == 2) {
      const uint32_t t2 = bits_of(p.b_tid_g, nt);
      ok = ok && distinct(p.b_tid_g, nt) && (t2 & ~tile) == 0;
      if (p.bkind == U_Z) ok = ok && ((tile & ~t2) & UB) == 0;
    }
    if (p.bkind == U_X && p.bmode == 1)
      for (int l = 0; l < p.wb && ok; ++l) ok = slot[l] == p.bq[0][l];
    const bool apair = p.akind == U_XP, bpair = p.bkind == U_XP;
    // a pair: whole tiles of 2^12 amplitudes, members of weight 2 or 4, and
    // each regrouped layout holds its member's qubits on the lowest slots
    if (apair || bpair) ok = ok && p.tb == kTileMax;
    auto member_slots = [&](const uint32_t* jg, const uint32_t* q, int w) {
      bool good = w == 2 || w == 4;
      for (int l = 0; l < w && good; ++l) good = jg[1u << l] == q[l];
      return good;
    };
    if (apair && ok) {
      ok = p.la == 2 && (p.amix || member_slots(p.j_g, p.aq[0], p.aw[0])) &&
           member_slots(p.p_j_g[0], p.aq[1], p.aw[1]);
      if (p.amix) ok = ok && p.aw[0] >= 2 && p.aw[0] <= 4;
    }
    if (bpair && ok)
      ok = p.lb == 2 && p.bmode == 2 && member_slots(p.b_j_g, p.bq[0], p.bw[0]) &&
           member_slots(p.p_j_g[1], p.bq[1], p.bw[1]);
    if ((p.bmode == 2 || apair || bpair) && ok) {
      // every layout puts every tile element in the same LDS slot, one each
      std::map<uint32_t, uint32_t> at;  // global index -> slot (layout 1)
      std::vector<uint8_t> used((size_t)1 << p.tb, 0);
      for (int t = 0; t < (1 << nt) && ok; ++t)
        for (int j = 0; j < 16 && ok; ++j) {
          uint32_t g = p.j_g[j], l = p.j_l[j];
          for (int i = 0; i < nt; ++i)
            if ((t >> i) & 1) { g |= p.tid_g[i]; l ^= p.tid_l[i]; }
          ok = l < used.size() && !used[l];
          if (ok) { used[l] = 1; at[g] = l; }
        }
      auto same = [&](const uint32_t* tg, const uint32_t* tl, const uint32_t* jg, const uint32_t* jl) {
        bool good = distinct(tg, nt);
        for (int t = 0; t < (1 << nt) && good; ++t)
          for (int j = 0; j < 16 && good; ++j) {
            uint32_t g = jg[j], l = jl[j];
            for (int i = 0; i < nt; ++i)
              if ((t >> i) & 1) { g |= tg[i]; l ^= tl[i]; }
            const auto it = at.find(g);
            good = it != at.end() && it->second == l;
          }
        return good;
      };
      if (p.bmode == 2) ok = ok && same(p.b_tid_g, p.b_tid_l, p.b_j_g, p.b_j_l);
      if (apair) ok = ok && same(p.p_tid_g[0], p.p_tid_l[0], p.p_j_g[0], p.p_j_l[0]);
      if (bpair) ok = ok && same(p.p_tid_g[1], p.p_tid_l[1], p.p_j_g[1], p.p_j_l[1]);
    }
    if (!ok) return fail(SV_EINVAL, "pass %zu: inconsistent layout", k);
  }
  // layouts of the LDS-resident batched kernel (d <= 3), for 1, 2 and 4
  // waves per trajectory: register and thread bits partition the register,
  // the check's first qubits are register bits and the rest the lowest
  // thread bits (lane bits of one wave)
  if (n <= kSmallBits) {
    for (int nw : {1, 2, 4}) {
      const int rb = nw == 1 ? 3 : nw == 2 ? 2 : 1;
      const std::vector<SmallDesc> sds = make_small_descs(n, tp, nw);
      for (size_t i = 0; i < sds.size(); ++i) {
        const SmallDesc& sd = sds[i];
        const TBlock& b = tp.blocks[i];
        uint32_t reg[3] = {0, 0, 0};
        for (int k = 0; k < rb; ++k) reg[k] = sd.j_off[1u << k];
        bool ok = sd.n_lane_bits == n - rb && sd.n_lane_bits <= 8 && distinct(reg, rb) &&
                  distinct(sd.lane_bit, sd.n_lane_bits) &&
                  (bits_of(reg, rb) & bits_of(sd.lane_bit, sd.n_lane_bits)) == 0 &&
                  (bits_of(reg, rb) | bits_of(sd.lane_bit, sd.n_lane_bits)) == all &&
                  sd.xreg + sd.xlanes == b.w && sd.xlanes <= 3 && sd.xmask == (1u << sd.xreg) - 1u;
        for (int j = 0; j < (1 << rb) && ok; ++j) {
          uint32_t g = 0;
          for (int k = 0; k < rb; ++k)
            if ((j >> k) & 1) g |= reg[k];
          ok = sd.j_off[j] == g;
        }
        for (int l = 0; l < b.w && ok; ++l) {
          const uint32_t q = 1u << b.qubit[l];
          ok = sd.q_bit[l] == q && (l < sd.xreg ? reg[l] == q : sd.lane_bit[l - sd.xreg] == q);
        }
        if (!ok) return fail(SV_EINVAL, "batched layout of block %zu (%d waves): inconsistent", i, nw);
      }
    }
  }
  if (n_passes) *n_passes = (int)pds.size();
  return SV_OK;
}

double sv_uniform(uint64_t seed, uint64_t t, uint64_t k) { return qec::uniform(seed, t, k); }

sv_status sv_block_kraus(int d, int gateset, int stab, int round, uint64_t seed, uint64_t t,
                         double p, double eps, const double* eps_site, double* D, uint32_t* F,
                         double* u, int* type, int* w, int* qubits) {
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (gateset != SV_GATESET_CR && gateset != SV_GATESET_TEXTBOOK) return fail(SV_EINVAL, "bad gateset");
  if (!D || !F || !u || !type || !w || !qubits) return fail(SV_EINVAL, "NULL output");
  const Template tp = build_template(d, gateset);
  if (stab < 0 || stab >= (int)tp.blocks.size() || round < 0) return fail(SV_EINVAL, "bad block");
  std::vector<double> es(std::max(1, tp.n_sites), eps);
  if (eps_site)
    for (int i = 0; i < tp.n_sites; ++i) es[i] = eps_site[i];
  const TBlock& b = tp.blocks[stab];
  uint8_t pauli[kMaxOps];
  BlockRT rt;
  const uint64_t k0 = (uint64_t)round * (uint64_t)tp.n_draws + (uint64_t)b.draw_off;
  draw_block(b, seed, t, k0, p, pauli, &rt.u);
  if (!build_block(b, es.data(), pauli, rt)) return fail(SV_EINVAL, "block is not monomial");
  std::memcpy(D, rt.D, sizeof rt.D);
  *F = rt.F;
  *u = rt.u;
  *type = b.type;
  *w = b.w;
  for (int l = 0; l < b.w; ++l) qubits[l] = b.qubit[l];
  return SV_OK;
}

static sv_status run_rounds_entry(const sv_job* job, sv_result* res, hipEvent_t done) {
  if (!job || !res) return fail(SV_EINVAL, "NULL job or result");
  if (job->d < 2 || job->d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", job->d);
  if (job->gateset != SV_GATESET_CR && job->gateset != SV_GATESET_TEXTBOOK)
    return fail(SV_EINVAL, "bad gateset %d", job->gateset);
  if (job->rounds < 1 || job->rounds > 100000) return fail(SV_EINVAL, "rounds=%d", job->rounds);
  if (job->dtype != SV_C64 && job->dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  if (job->n_traj < 0) return fail(SV_EINVAL, "n_traj < 0");
  if (job->flags & ~(SV_RUN_GRAPH | SV_RUN_TWIRL | SV_RUN_XBASIS | SV_RUN_VIRTUAL_Z | SV_RUN_IDLE_NOISE |
                     SV_RUN_ZZ_PLAQUETTE))
    return fail(SV_EINVAL, "unknown flags 0x%x", job->flags);
  if (!(job->p >= 0.0 && job->p <= 1.0)) return fail(SV_EINVAL, "p out of [0, 1]");
  if (!std::isfinite(job->eps) || !std::isfinite(job->zeta)) return fail(SV_EINVAL, "non-finite eps/zeta");
  if (job->n_traj > 0 && (!res->records || !res->final_bits))
    return fail(SV_EINVAL, "records and final_bits are required");
  if ((job->flags & SV_RUN_GRAPH) && res->final_states)
    return fail(SV_EINVAL, "final_states cannot be returned with SV_RUN_GRAPH");
  if (done && (job->flags & SV_RUN_GRAPH))
    return fail(SV_EINVAL, "the asynchronous run does not replay graphs");
  if (done && res->final_states) return fail(SV_EINVAL, "the asynchronous run returns no final states");
  const Template tp = build_template(job->d, job->gateset, (job->flags & SV_RUN_TWIRL) != 0,
                                     (job->flags & SV_RUN_VIRTUAL_Z) != 0,
                                     (job->flags & SV_RUN_IDLE_NOISE) != 0,
                                     (job->flags & SV_RUN_ZZ_PLAQUETTE) != 0 && job->zeta != 0.0);
  if (job->eps_site)
    for (int i = 0; i < tp.n_sites; ++i)
      if (!std::isfinite(job->eps_site[i])) return fail(SV_EINVAL, "non-finite eps_site[%d]", i);
  res->gpu_ms = done ? -1.0 : 0.0;
  res->pass_ms = done ? -1.0 : 0.0;
  res->passes_per_round = 0;
  if (job->n_traj == 0) {
    if (done) HIP_OK(hipEventRecord(done, (hipStream_t)job->hip_stream));
    return SV_OK;
  }
  if (job->dtype == SV_C128) return run_rounds_t<double>(job, res, tp, nullptr, done);
  return run_rounds_t<float>(job, res, tp, nullptr, done);
}

sv_status sv_run_rounds(const sv_job* job, sv_result* res) { return run_rounds_entry(job, res, nullptr); }

sv_status sv_run_rounds_async(const sv_job* job, sv_result* res, void* done_event) {
  if (!done_event) return fail(SV_EINVAL, "NULL event");
  return run_rounds_entry(job, res, (hipEvent_t)done_event);
}

static sv_status check_batch_job(const sv_batch_job* job, const sv_batch_result* res) {
  if (!job || !res) return fail(SV_EINVAL, "NULL job or result");
  if (job->d < 2 || job->d > 4) return fail(SV_EINVAL, "d=%d out of 2..4", job->d);
  if (job->gateset != SV_GATESET_CR && job->gateset != SV_GATESET_TEXTBOOK)
    return fail(SV_EINVAL, "bad gateset %d", job->gateset);
  if (job->dtype != SV_C64 && job->dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  if (job->n_traj < 0 || job->max_rounds < 1) return fail(SV_EINVAL, "bad n_traj / max_rounds");
  if (job->flags != 0) return fail(SV_EINVAL, "flags must be 0");
  if (!job->rounds || !job->p) return fail(SV_EINVAL, "rounds and p are required");
  if (!res->records || !res->final_bits) return fail(SV_EINVAL, "records and final_bits are required");
  if (!std::isfinite(job->eps) || !std::isfinite(job->zeta)) return fail(SV_EINVAL, "non-finite eps/zeta");
  for (int i = 0; i < job->n_traj; ++i) {
    if (job->rounds[i] < 1 || job->rounds[i] > job->max_rounds)
      return fail(SV_EINVAL, "rounds[%d]=%d out of 1..%d", i, job->rounds[i], job->max_rounds);
    if (!(job->p[i] >= 0.0 && job->p[i] <= 1.0)) return fail(SV_EINVAL, "p[%d] out of [0, 1]", i);
  }
  const int n_sites = build_template(job->d, job->gateset).n_sites;
  if (job->eps_site)
    for (size_t i = 0; i < (size_t)job->n_traj * n_sites; ++i)
      if (!std::isfinite(job->eps_site[i])) return fail(SV_EINVAL, "non-finite eps_site");
  return SV_OK;
}

// Per-trajectory seeds and draw streams of a batched job, and the inputs of
// the batched kernels.
struct BatchHost {
  std::vector<uint64_t> seeds, streams;
  std::vector<double> epsv;
  BatchInputs in;
  BatchHost(const sv_batch_job* job, sv_batch_result* res, const Template& tp)
      : seeds((size_t)job->n_traj, job->seed), streams((size_t)job->n_traj) {
    for (int i = 0; i < job->n_traj; ++i) streams[i] = job->traj0 + (uint64_t)i;
    if (!job->eps_site) epsv.assign(std::max(1, tp.n_sites), job->eps);
    in = BatchInputs{job->d, job->gateset, job->n_traj, job->max_rounds, job->zeta, seeds.data(),
                     streams.data(), job->rounds, job->p, job->eps_site ? job->eps_site : epsv.data(),
                     job->eps_site ? tp.n_sites : 0, res->records, res->final_bits,
                     (hipStream_t)job->hip_stream, 0.0};
  }
};

sv_status sv_run_batch(const sv_batch_job* job, sv_batch_result* res) {
  SV_OK_OR_RETURN(check_batch_job(job, res));
  res->gpu_ms = 0.0;
  if (job->n_traj == 0) return SV_OK;
  const Template tp = build_template(job->d, job->gateset);
  BatchHost h(job, res, tp);
  const sv_status st =
      job->dtype == SV_C128 ? run_batch_core<double>(h.in, tp) : run_batch_core<float>(h.in, tp);
  res->gpu_ms = h.in.gpu_ms;
  res->passes_per_round = h.in.passes_per_round;
  res->redo_passes = h.in.redo_passes;
  return st;
}

}  // extern "C"

// ------------------------------------------------ no-allocation batched run
// Every device buffer of sv_run_batch_noalloc comes from this array: each GPU
// the library runs on holds one copy of it until the process ends.  In host
// code its name is only a host-side stand-in; the device address of a GPU's
// copy comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is handed to kernels and copies.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
struct NoAllocDevice {
  std::once_flag once;
  sv_status init_status = SV_OK;
  std::string init_err;
  void* ptr = nullptr;                    // this device's copy of `scratch`
  hipEvent_t ev_a = nullptr, ev_b = nullptr;  // timing of the launch
  std::mutex mu;                          // one call at a time per device
};
NoAllocDevice g_noalloc[64];
}  // namespace

extern "C" {

sv_status sv_run_batch_noalloc(const sv_batch_job* job, sv_batch_result* res) {
  SV_OK_OR_RETURN(check_batch_job(job, res));
  if (job->d > 3) return fail(SV_EINVAL, "the no-allocation batch covers d <= 3 (d=%d)", job->d);
  const Template tp = build_template(job->d, job->gateset);
  if (!batch_template_fits(tp) || !batch_is_small(tp, job->d))
    return fail(SV_EINVAL, "block template too large for the batched path");
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SV_EINVAL, "device %d out of range", dev);
  NoAllocDevice& nd = g_noalloc[dev];
  std::call_once(nd.once, [&nd] {
    // this thread's current device is the one being set up
    hipError_t e = hipGetSymbolAddress(&nd.ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) e = hipEventCreate(&nd.ev_a);
    if (e == hipSuccess) e = hipEventCreate(&nd.ev_b);
    if (e != hipSuccess || !nd.ptr) {
      nd.init_status = SV_EDEVICE;
      nd.init_err = std::string("no-allocation scratch set-up: ") + hipGetErrorString(e);
    }
  });
  if (nd.init_status != SV_OK) return fail(nd.init_status, "%s", nd.init_err.c_str());
  res->gpu_ms = 0.0;
  if (job->n_traj == 0) return SV_OK;
  std::lock_guard<std::mutex> lk(nd.mu);
  BatchHost h(job, res, tp);
  Arena A{static_cast<char*>(nd.ptr), kNoAllocScratchBytes, 0, false};
  const sv_status st = job->dtype == SV_C128 ? run_batch_small<double>(h.in, tp, A, nd.ev_a, nd.ev_b)
                                             : run_batch_small<float>(h.in, tp, A, nd.ev_a, nd.ev_b);
  if (A.overflow)
    return fail(SV_ENOMEM, "the job needs more than the %zu MiB no-allocation scratch",
                kNoAllocScratchBytes >> 20);
  res->gpu_ms = h.in.gpu_ms;
  res->passes_per_round = h.in.passes_per_round;
  res->redo_passes = h.in.redo_passes;
  return st;
}

sv_status sv_tuning_get(int d, int dtype, sv_tuning* out) {
  if (!out) return fail(SV_EINVAL, "NULL output");
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  *out = tuning_for(d, dtype);
  return SV_OK;
}

sv_status sv_tuning_set(int d, int dtype, const sv_tuning* in) {
  if (!in) return fail(SV_EINVAL, "NULL tuning");
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  SV_OK_OR_RETURN(check_tuning(*in));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[TuneKey{current_device(), d, dtype}] = *in;
  return SV_OK;
}

sv_status sv_autotune(int d, int dtype, int gateset, sv_tuning* best, double* best_ms) {
  if (d < 2 || d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", d);
  if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  if (gateset != SV_GATESET_CR && gateset != SV_GATESET_TEXTBOOK) return fail(SV_EINVAL, "bad gateset");
  const Template tp = build_template(d, gateset);
  const TuneKey key{current_device(), d, dtype};
  sv_tuning base = default_tuning();
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it != g_tune.end()) base = it->second;
  }
  std::vector<sv_tuning> cands;
  if (d == 5) {
    for (int xp = 0; xp <= 1; ++xp)
      for (int z = 2; z <= kChainMax; ++z)
        for (int sn = 0; sn <= 1; ++sn)
          for (int wpc : {0, 3, 4, 6, 8, 12, 16}) {  // multiples of 2 and 3 resident workgroups
            sv_tuning c = base;
            c.xpair = xp;
            c.zchain = z;
            c.snake = sn;
            c.pass_wgs_per_cu = wpc;
            cands.push_back(c);
          }
  } else if (d == 4) {
    for (int xp = 0; xp <= 1; ++xp)
      for (int z = 2; z <= kChainMax; ++z)
        for (int mib : {256, 1024, 4096}) {
          sv_tuning c = base;
          c.xpair = xp;
          c.zchain = z;
          c.lockstep_mib = mib;
          cands.push_back(c);
        }
  } else {
    for (int w : {2, 4, 8, 12, 16}) {
      sv_tuning c = base;
      c.batch_waves_per_cu = w;
      cands.push_back(c);
    }
  }
  // synthetic trials of the tuned shape
  const int n = d * d, ns = (int)tp.blocks.size();
  // d = 4: as many trajectories as the batched workload, so that the group
  // memory (how many registers run in lockstep) is tested at its real size
  const int nt = d == 5 ? 1 : (d == 4 ? 4096 : 16384);
  const int R = d == 5 ? 1 : 3;
  std::vector<uint8_t> rec((size_t)nt * R * ns), bits((size_t)nt * n);
  std::vector<int> rounds(nt, R);
  std::vector<double> pv(nt, 2e-3), eps(std::max(1, tp.n_sites), 0.0125);
  std::vector<uint64_t> seeds(nt, 0x7E57), streams(nt);
  for (int i = 0; i < nt; ++i) streams[i] = (uint64_t)i;
  auto trial = [&](const sv_tuning& c, double* ms) -> sv_status {
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = c;
    }
    if (d == 5) {
      sv_job job{};
      job.d = d;
      job.gateset = gateset;
      job.rounds = R;
      job.dtype = dtype;
      job.n_traj = nt;
      job.seed = 0x7E57;
      job.p = 2e-3;
      job.eps = 0.0125;
      job.zeta = 0.01;
      sv_result res{};
      res.records = rec.data();
      res.final_bits = bits.data();
      SV_OK_OR_RETURN(dtype == SV_C128 ? run_rounds_t<double>(&job, &res, tp)
                                       : run_rounds_t<float>(&job, &res, tp));
      *ms = res.gpu_ms;
    } else {
      BatchInputs in{d, gateset, nt, R, 0.0, seeds.data(), streams.data(), rounds.data(), pv.data(),
                     eps.data(), 0, rec.data(), bits.data(), (hipStream_t)nullptr, 0.0};
      SV_OK_OR_RETURN(dtype == SV_C128 ? run_batch_core<double>(in, tp) : run_batch_core<float>(in, tp));
      *ms = in.gpu_ms;
    }
    return SV_OK;
  };
  double warm = 0.0;
  sv_status st = trial(base, &warm);
  int win = -1;
  double win_ms = 0.0;
  for (size_t i = 0; i < cands.size() && st == SV_OK; ++i) {
    double a = 0.0, b = 0.0;
    st = trial(cands[i], &a);
    if (st == SV_OK) st = trial(cands[i], &b);
    const double t = std::min(a, b);
    if (st == SV_OK && (win < 0 || t < win_ms)) {
      win = (int)i;
      win_ms = t;
    }
  }
  const sv_tuning chosen = (st == SV_OK && win >= 0) ? cands[win] : base;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = chosen;
  }
  if (st != SV_OK) return st;
  if (best) *best = chosen;
  if (best_ms) *best_ms = win_ms;
  return SV_OK;
}

static std::string device_arch() {
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, current_device()) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

sv_status sv_tuning_save(const char* path) {
  if (!path) return fail(SV_EINVAL, "NULL path");
  const std::string arch = device_arch();
  const int dev = current_device();
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(SV_EINVAL, "cannot write %s", path);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune)
      if (kv.first.dev == dev)
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d\n", arch.c_str(), kv.first.d, kv.first.dtype,
                     kv.second.zchain, kv.second.snake, kv.second.batch_waves_per_cu, kv.second.lockstep_mib,
                     kv.second.pass_wgs_per_cu, kv.second.xpair);
  }
  return std::fclose(f) == 0 ? SV_OK : fail(SV_EINVAL, "cannot write %s", path);
}

sv_status sv_tuning_load(const char* path) {
  if (!path) return fail(SV_EINVAL, "NULL path");
  const std::string arch = device_arch();
  const int dev = current_device();
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(SV_EINVAL, "cannot read %s", path);
  char line[512], a[128];
  int d, dt;
  std::vector<std::pair<TuneKey, sv_tuning>> got;
  bool bad = false;
  // lines of eight fields (no xpair: 0) or nine
  while (!bad && std::fgets(line, sizeof line, f)) {
    sv_tuning t = default_tuning();
    char extra[8];
    const int k = std::sscanf(line, "%127s %d %d %d %d %d %d %d %d %7s", a, &d, &dt, &t.zchain, &t.snake,
                              &t.batch_waves_per_cu, &t.lockstep_mib, &t.pass_wgs_per_cu, &t.xpair, extra);
    if (k <= 0) continue;  // blank line
    if (k == 8) t.xpair = 0;
    if (k != 8 && k != 9) {
      bad = true;
      break;
    }
    if (arch != a) continue;
    if (d < 2 || d > 5 || (dt != SV_C64 && dt != SV_C128) || check_tuning(t) != SV_OK) {
      std::fclose(f);
      return fail(SV_EINVAL, "bad tuning line in %s", path);
    }
    got.push_back({TuneKey{dev, d, dt}, t});
  }
  const bool eof = std::feof(f) != 0;
  std::fclose(f);
  if (bad || !eof) return fail(SV_EINVAL, "cannot parse %s", path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : got) g_tune[kv.first] = kv.second;
  return SV_OK;
}

}  // extern "C"

#include "decoder.hip"
#include "server.hip"
