// Batched trajectories for small distances (d = 2, 3: at most 2^9 data
// amplitudes).  One persistent launch runs thousands of trajectories with
// their own round counts, depolarizing probabilities and over-rotation
// angles.  The whole data register of a trajectory lives in LDS and a
// workgroup of NW waves runs it (NW = 1: 8 amplitudes per lane; 2: 4; 4: 2);
// a workgroup takes trajectories from a static list (sorted longest-first by
// the host) until the list is exhausted, so every wave reaches the exit.
//
// Per trajectory (set-up): cos/sin of every gate site's angle, the channel
// thresholds j p / 3 and j p / 15, and the noise-free Kraus pair of every
// stabilizer template are tabulated in LDS (angles common to the launch: the
// angle table and Kraus pairs come precomputed and are only copied).
// Per round: one thread per random draw evaluates Philox for the whole round
// (noise locations and measurements), and a wave vote per draw tells which
// noise locations picked a Pauli.
// Per stabilizer circuit (Sec. II.B: one circuit at a time, ancilla measured
// and reset):
//   1. if a location of the circuit drew a Pauli, one lane of wave 0 per
//      block-basis label runs the circuit's ops with the drawn Paulis on the
//      ancilla 2-vector (track_ops); otherwise the tabulated noise-free pair
//      is used;
//   2. each thread loads its amplitudes: the check's first qubits index the
//      thread's registers, its others are the lowest lane bits (their
//      Walsh-Hadamard stages pair lanes through DPP); the thread transforms
//      them to the check basis and accumulates S_0, S_1; wave reductions (and
//      for NW > 1 the waves' totals in wave order) give p1 and the outcome on
//      the device; the thread then applies D_m, transforms back, applies the
//      ZZ layer and 1/sqrt(S_m) and writes the amplitudes back.
// After the last round wave 0 measures the data qubits one by one from the
// highest label down (two-level descent: lane sums, then within one lane).
#include "qec_common.h"

namespace qec {

static_assert(sizeof(TOp) == 12 && offsetof(TBlock, ops) % 4 == 0,
              "an op is read as three 32-bit words");

constexpr int kSmallBits = 9;
constexpr int kSmallAmps = 1 << kSmallBits;
constexpr int kSmallStab = 8;     // d <= 3
constexpr int kSmallSites = 64;   // gate sites per round, d <= 3
constexpr int kSmallDraws = 128;  // random draws per round, d <= 3

// Per block template, for a trajectory run by NW waves (2^RB amplitudes per
// lane, RB = 3, 2, 1 for NW = 1, 2, 4): where each of a lane's amplitudes and
// each bit of the thread index sit in the register (bit values).  The check's
// first xreg qubits are register bits 0 .. xreg-1, the next xlanes ones are
// thread-index bits 0 .. xlanes-1: local check index of register j on thread
// t = (j & xmask) | (t & (2^xlanes - 1)) << xreg.
struct SmallDesc {
  uint32_t j_off[8];
  uint32_t lane_bit[8];
  uint32_t q_bit[4];
  int n_lane_bits;
  int xlanes;
  uint32_t xmask;
  int xreg;
};

template <typename T>
struct SmallSlot {
  C2<T> psi[kSmallAmps];
  C2<T> Dc[kSmallStab][2][16];  // noise-free Kraus diagonals per template
  double Wc[kSmallStab][2][16];
  C2<T> D[2][16];               // current block when a Pauli was drawn
  double W[2][16];
  double cs[2 * kSmallSites];   // cos, sin of each site's angle
  double t1[3], t2[15];         // channel thresholds
  double u[kSmallDraws];        // draws of the current round
  uint32_t F;
  int pad;
};

// Angle table and noise-free Kraus pairs of a launch whose over-rotation
// angles are common to every trajectory: computed once on the host and
// copied into each trajectory's slot instead of being rebuilt per trajectory.
template <typename T>
struct SmallShared {
  double cs[2 * kSmallSites];
  C2<T> Dc[kSmallStab][2][16];
  double Wc[kSmallStab][2][16];
};

__device__ __forceinline__ uint32_t sslot(uint32_t i) { return i ^ (((i >> 4) ^ (i >> 8)) & 15u); }

// Move of a double between lanes by a DPP pattern (all lanes active).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double lane_value(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// v of the last lane of the row before (row_bcast:15, rows in row_mask 0xA)
// or of lane 31 (row_bcast:31, rows in 0xC); 0 in the other rows.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_bcast(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sums over the 64 lanes of the wave of two values (every lane gets the same
// totals; called with every lane active): lane pairs, quads, eights and rows
// of 16 through DPP; then rows 1 and 3 add the sums of rows 0 and 2, and row
// 3 adds that of rows 0 + 1, so lane 63 holds (S3 + S2) + (S1 + S0), a fixed
// order.  The two reductions' steps are interleaved (two independent chains
// between dependent DPP moves).
__device__ __forceinline__ void wave_total2(double& a, double& b) {
  a += dpp_double<0xB1>(a);
  b += dpp_double<0xB1>(b);
  a += dpp_double<0x4E>(a);
  b += dpp_double<0x4E>(b);
  a += dpp_double<0x141>(a);
  b += dpp_double<0x141>(b);
  a += dpp_double<0x140>(a);
  b += dpp_double<0x140>(b);
  a += dpp_bcast<0x142, 0xA>(a);
  b += dpp_bcast<0x142, 0xA>(b);
  a += dpp_bcast<0x143, 0xC>(a);
  b += dpp_bcast<0x143, 0xC>(b);
  a = lane_value(a, 63);
  b = lane_value(b, 63);
}

// Any set bit in [off, off + len) of the 128-bit mask h1:h0 (len <= 16).
__device__ __forceinline__ bool any_in_window(uint64_t h0, uint64_t h1, int off, int len) {
  uint64_t w;
  if (off >= 64) w = h1 >> (off - 64);
  else if (off == 0) w = h0;
  else w = (h0 >> off) | (h1 << (64 - off));
  return (w & ((1ull << len) - 1)) != 0;
}

// Walsh-Hadamard stage over thread-index bit B (B < 3: lanes of one wave,
// exchanged through DPP) for a thread's NA amplitudes.
template <int B, typename T, int NA>
__device__ __forceinline__ void small_wht_lane_n(C2<T>* v, int tid) {
  const bool upper = (tid >> B) & 1;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const C2<T> o{lane_partner<B>(v[j].re, upper), lane_partner<B>(v[j].im, upper)};
    v[j] = upper ? C2<T>{o.re - v[j].re, o.im - v[j].im} : C2<T>{v[j].re + o.re, v[j].im + o.im};
  }
}

// Op source of track_ops for a block whose op i, Pauli code and angle sit in
// lane i: the walk reads them with readlane (op index uniform over the wave).
struct LaneOps {
  uint32_t w0, w1, w2;  // the TOp's three words
  uint32_t c;           // Pauli code
  double cos, sin;      // angle of a rotation op
  __device__ __forceinline__ TOp op_here() const {
    const uint32_t w[3] = {w0, w1, w2};
    TOp o;
    __builtin_memcpy(&o, w, sizeof(TOp));
    return o;
  }
  __device__ __forceinline__ TOp op(int i) const {
    const uint32_t w[3] = {(uint32_t)__builtin_amdgcn_readlane((int)w0, i),
                           (uint32_t)__builtin_amdgcn_readlane((int)w1, i),
                           (uint32_t)__builtin_amdgcn_readlane((int)w2, i)};
    TOp o;
    __builtin_memcpy(&o, w, sizeof(TOp));
    return o;
  }
  __device__ __forceinline__ int code(int i) const { return __builtin_amdgcn_readlane((int)c, i); }
  __device__ __forceinline__ cd angle(int i, const TOp&) const {
    return cd{lane_value(cos, i), lane_value(sin, i)};
  }
};

// Tables of a new trajectory: site angles, thresholds, logical |0>.  sites:
// the op of every gate site of the round template (index = site).
// (tid, nl: thread index and threads of the trajectory's workgroup)
template <typename T>
__device__ void small_setup_tables(SmallSlot<T>& S, int tid, int nl, int n, const TOp* sites,
                                   int n_sites, const uint32_t* init_mask, T amp0, const double* eps,
                                   double p, const SmallShared<T>* shared) {
  // cos / sin of every site's angle
  if (shared) {
    for (int k = tid; k < 2 * n_sites; k += nl) S.cs[k] = shared->cs[k];
  } else {
    for (int k = tid; k < n_sites; k += nl) {
      const double beta = op_angle(sites[k], eps);
      S.cs[2 * k] = cos(beta);
      S.cs[2 * k + 1] = sin(beta);
    }
  }
  if (tid < 3) S.t1[tid] = (double)(tid + 1) * p / 3.0;
  if (tid < 15) S.t2[tid] = (double)(tid + 1) * p / 15.0;
  // logical |0>: bit x of init_mask marks the X-stabilizer orbit of 0; thread
  // g writes amplitudes 8 g .. 8 g + 7
  for (int g = tid; g < (1 << (n - 3)); g += nl) {
    const uint32_t bits8 = (init_mask[g >> 2] >> ((g & 3) * 8)) & 0xFFu;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      S.psi[sslot((uint32_t)(g * 8 + k))] = C2<T>{((bits8 >> k) & 1) ? amp0 : (T)0, (T)0};
  }
}

// Noise-free Kraus pair of every template (needs the angle table).
template <typename T>
__device__ void small_setup_kraus(SmallSlot<T>& S, int tid, int nl, int ns, const TBlock* blocks,
                                  int* err, const SmallShared<T>* shared) {
  if (shared) {
    for (int i = tid; i < ns * 32; i += nl) {
      const int s = i >> 5, m = (i >> 4) & 1, x = i & 15;
      S.Dc[s][m][x] = shared->Dc[s][m][x];
      S.Wc[s][m][x] = shared->Wc[s][m][x];
    }
    return;
  }
  const uint8_t none[kMaxOpsBatch] = {};
  for (int i = tid; i < ns * 16; i += nl) {
    const int s = i >> 4, x = i & 15;
    const TBlock& b = blocks[s];
    if (x >= (1 << b.w)) continue;
    cd v0, v1;
    uint32_t cur = 0;
    if (!track_column(b, CsFromTable{S.cs}, none, x, v0, v1, &cur)) atomicOr(err, 1);
    const double norm = b.type == 0 ? 1.0 / (double)(1 << b.w) : 1.0;
    S.Dc[s][0][x] = C2<T>{(T)(v0.re * norm), (T)(v0.im * norm)};
    S.Dc[s][1][x] = C2<T>{(T)(v1.re * norm), (T)(v1.im * norm)};
    S.Wc[s][0][x] = (v0.re * v0.re + v0.im * v0.im) * norm;
    S.Wc[s][1][x] = (v1.re * v1.re + v1.im * v1.im) * norm;
  }
}

// Walsh-Hadamard transform of a thread's NA registers over the check's
// qubits: register bits 0 .. xreg-1, then thread-index bits 0 .. xlanes-1
// (lane pairs through DPP; every lane of the wave takes part).
template <typename T, int NA>
__device__ __forceinline__ void small_wht(C2<T>* v, int xreg, int xlanes, int tid) {
#pragma unroll
  for (int hb = 1; hb < NA; hb <<= 1) {
    if (hb < (1 << xreg)) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        if (i & hb) continue;
        const C2<T> a = v[i], b = v[i | hb];
        v[i] = {a.re + b.re, a.im + b.im};
        v[i | hb] = {a.re - b.re, a.im - b.im};
      }
    }
  }
  if (xlanes > 0) small_wht_lane_n<0, T, NA>(v, tid);
  if (xlanes > 1) small_wht_lane_n<1, T, NA>(v, tid);
  if (xlanes > 2) small_wht_lane_n<2, T, NA>(v, tid);
}

// NW waves (64 NW threads) run one trajectory at a time; lane bits and the
// wave index together form the thread-index bits of the register layout.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_batch_small(
    const TBlock* __restrict__ blocks, const SmallDesc* __restrict__ sdesc, int ns, int n,
    int draws_round, const JobConst* __restrict__ jc, const uint64_t* __restrict__ tseed,
    const uint64_t* __restrict__ tstream,
    const int* __restrict__ order, int n_traj, const int* __restrict__ rounds,
    const double* __restrict__ pvec, const double* __restrict__ eps, int eps_stride,
    uint8_t* __restrict__ rec, int max_rounds, uint8_t* __restrict__ bits, int* __restrict__ err,
    const TOp* __restrict__ sites, int n_sites, const SmallShared<T>* __restrict__ shared,
    const uint32_t* __restrict__ init_mask, const uint8_t* __restrict__ draw_kind) {
  static_assert(NW == 1 || NW == 2 || NW == 4, "one, two or four waves per trajectory");
  constexpr int NL = 64 * NW;                       // threads of a trajectory
  constexpr int NA = NW == 1 ? 8 : NW == 2 ? 4 : 2;  // amplitudes per thread
  constexpr int DR = (kSmallDraws + NL - 1) / NL;   // draws per thread and round
  __shared__ SmallSlot<T> S;
  // ZZ phases are read per amplitude: keep them in LDS (the round template
  // stays in global memory: more LDS per workgroup would cost occupancy)
  __shared__ C2<T> lzz[kSmallBits * 2 + 1];
  __shared__ uint64_t lhits[2];       // noise hits of the round (draws 0..63, 64..127)
  __shared__ double lsum[2][NW];      // per-wave S_0, S_1 of the current circuit
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i <= jc->n_edges && i <= 2 * kSmallBits; i += NL)
    lzz[i] = C2<T>{(T)jc->zz[2 * i], (T)jc->zz[2 * i + 1]};
  const int use_zz = jc->use_zz, zd = jc->d;
  const uint32_t hmask = jc->hmask, vmask = jc->vmask;
  const T amp0 = (T)jc->amp0;
  const int groups = 1 << (n - 3);
  __syncthreads();

  for (int qi = blockIdx.x; qi < n_traj; qi += gridDim.x) {
    const int t = order[qi];
    const int R = rounds[t];
    const double p = pvec[t];
    const uint64_t tg = tstream[t], seed = tseed[t];  // draw stream of this trajectory
    small_setup_tables(S, tid, NL, n, sites, n_sites, init_mask, amp0, eps + (size_t)t * eps_stride, p,
                       shared);
    __syncthreads();
    small_setup_kraus(S, tid, NL, ns, blocks, err, shared);
    __syncthreads();
    for (int r = 0; r < R; ++r) {
      // every draw of the round; hit: a noise location that picked a Pauli
#pragma unroll
      for (int c = 0; c < DR; ++c) {
        const int k = tid + NL * c;
        bool hit = false;
        if (k < draws_round) {
          const double u = uniform(seed, tg, (uint64_t)r * (uint64_t)draws_round + (uint64_t)k);
          S.u[k] = u;
          const int kind = draw_kind[k];
          hit = kind < 2 && u < (kind ? S.t2[14] : S.t1[2]);
        }
        const uint64_t h = __ballot(hit);
        const int chunk = wave + NW * c;
        if (lane == 0 && chunk < 2) lhits[chunk] = h;
      }
      __syncthreads();
      const uint64_t hits0 = lhits[0], hits1 = lhits[1];
      for (int s = 0; s < ns; ++s) {
        const TBlock& b = blocks[s];
        const SmallDesc& sd = sdesc[s];
        const int off = b.draw_off, nnoise = b.n_draws - 1;
        // noise draws off .. off + nnoise - 1 (at most 15, within 128)
        const bool noisy = any_in_window(hits0, hits1, off, nnoise);
        // 1. Kraus pair of this block instance
        const int nx = 1 << b.w;
        if (noisy) {
          // (wave 0) op i of the block, its Pauli code and its angle's
          // (cos, sin) go to lane i (one load and one table lookup in
          // parallel); the lanes of the block-basis labels then walk the
          // ops reading them with readlane
          if (wave == 0) {
            const int nops = b.n_ops;
            LaneOps lo{};
            if (lane < nops) {
              const uint32_t* w = reinterpret_cast<const uint32_t*>(&b.ops[lane]);
              lo.w0 = w[0];
              lo.w1 = w[1];
              lo.w2 = w[2];
              const TOp op = lo.op_here();
              int c = 0;
              if (op.draw >= 0) {
                const double u = S.u[off + op.draw];
                // first threshold above u (thresholds increase with j)
                if (op.kind == OP_N1_ANC || op.kind == OP_N1_DATA) {
                  if (u < S.t1[2]) c = 1 + (u >= S.t1[0]) + (u >= S.t1[1]);
                } else if (u < S.t2[14]) {
                  c = 1;
#pragma unroll
                  for (int j = 0; j < 14; ++j) c += u >= S.t2[j];
                }
              }
              lo.c = (uint32_t)c;
              if (is_rotation(op.kind)) {
                lo.cos = S.cs[2 * op.site];
                lo.sin = S.cs[2 * op.site + 1];
              }
            }
            if (lane < nx) {
              cd v0, v1;
              uint32_t cur = 0;
              if (!track_ops(b.type == 0, nops, lo, lane, v0, v1, &cur)) atomicOr(err, 1);
              const double norm = b.type == 0 ? 1.0 / (double)nx : 1.0;
              S.D[0][lane] = C2<T>{(T)(v0.re * norm), (T)(v0.im * norm)};
              S.D[1][lane] = C2<T>{(T)(v1.re * norm), (T)(v1.im * norm)};
              S.W[0][lane] = (v0.re * v0.re + v0.im * v0.im) * norm;
              S.W[1][lane] = (v1.re * v1.re + v1.im * v1.im) * norm;
              if (lane == 0) S.F = cur;  // label 0 maps to F
            }
          }
          __syncthreads();
        }
        const C2<T>(*D)[16] = noisy ? S.D : S.Dc[s];
        const double(*W)[16] = noisy ? S.W : S.Wc[s];
        const uint32_t F = noisy ? S.F : 0u;
        // 2. measure and apply
        const bool g_on = tid < (1 << sd.n_lane_bits);
        uint32_t lb = 0;
        for (int i = 0; i < sd.n_lane_bits; ++i)
          if ((tid >> i) & 1) lb |= sd.lane_bit[i];
        const uint32_t xm = sd.xmask;
        const int xreg = sd.xreg, xlanes = sd.xlanes;
        const uint32_t xhi = (uint32_t)(tid & ((1 << xlanes) - 1)) << xreg;  // local bits from the thread
        C2<T> v[NA];
#pragma unroll
        for (int j = 0; j < NA; ++j) v[j] = C2<T>{(T)0, (T)0};
        double s0 = 0.0, s1 = 0.0;
        const bool xb = b.type == 0;
        if (g_on) {
#pragma unroll
          for (int j = 0; j < NA; ++j) v[j] = S.psi[sslot(lb | sd.j_off[j])];
        }
        if (xb) small_wht<T, NA>(v, xreg, xlanes, tid);  // every lane joins the lane exchange
        if (g_on) {
#pragma unroll
          for (int j = 0; j < NA; ++j) {
            const uint32_t x = ((uint32_t)j & xm) | xhi;
            const double re = (double)v[j].re, im = (double)v[j].im, a2 = re * re + im * im;
            s0 += W[0][x] * a2;
            s1 += W[1][x] * a2;
          }
        }
        wave_total2(s0, s1);
        if constexpr (NW > 1) {
          // the waves' totals in wave order (the same sum on every wave)
          if (lane == 0) {
            lsum[0][wave] = s0;
            lsum[1][wave] = s1;
          }
          __syncthreads();
          s0 = lsum[0][0];
          s1 = lsum[1][0];
#pragma unroll
          for (int w = 1; w < NW; ++w) {
            s0 += lsum[0][w];
            s1 += lsum[1][w];
          }
        }
        // both renormalisations alongside p1 (the kept one has S_m > 0)
        const double r0 = rsqrt(s0), r1 = rsqrt(s1);
        const double p1 = clamp_p1(s1 / (s0 + s1));
        const int m = (S.u[off + nnoise] < p1) ? 1 : 0;
        if (tid == 0) rec[((size_t)t * max_rounds + r) * ns + s] = (uint8_t)m;
        const double scale = m ? r1 : r0;
        if (g_on) {
#pragma unroll
          for (int j = 0; j < NA; ++j) {
            const uint32_t x = ((uint32_t)j & xm) | xhi;
            v[j] = mulc(v[j], D[m][x].re, D[m][x].im);
          }
        }
        if (xb) small_wht<T, NA>(v, xreg, xlanes, tid);
        if (g_on) {
          uint32_t fo = 0;
          if (!xb)
            for (int l = 0; l < b.w; ++l)
              if ((F >> l) & 1) fo |= sd.q_bit[l];
          const T sc = (T)scale;
#pragma unroll
          for (int j = 0; j < NA; ++j) {
            C2<T> o = v[j];
            const uint32_t x = ((uint32_t)j & xm) | xhi;
            if (xb && (__popc(x & F) & 1)) o = {-o.re, -o.im};
            const uint32_t g = (lb | sd.j_off[j]) ^ fo;
            if (use_zz) {
              const int k = __popc((g ^ (g >> 1)) & hmask) + __popc((g ^ (g >> zd)) & vmask);
              o = mulc(o, lzz[k].re, lzz[k].im);
            }
            o.re *= sc;
            o.im *= sc;
            S.psi[sslot(g)] = o;
          }
        }
        __syncthreads();
      }
    }
    // final Z measurement of the data register, highest label first, by wave
    // 0: lane l holds amplitudes 8 l .. 8 l + 7
    if (wave == 0) {
      const bool g_on = lane < groups;
      double L = 0.0;
      if (g_on) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const C2<T> a = S.psi[sslot((uint32_t)(lane * 8 + k))];
          L += (double)a.re * (double)a.re + (double)a.im * (double)a.im;
        }
      }
      const uint64_t kf = (uint64_t)R * (uint64_t)draws_round;
      const double uf = lane < n ? uniform(seed, tg, kf + (uint64_t)lane) : 0.0;
      int lo = 0, size = groups, level = 0;
      for (; level < n - 3; ++level) {
        const int half = size >> 1;
        const bool in0 = lane >= lo && lane < lo + half;
        const bool in1 = lane >= lo + half && lane < lo + size;
        double S0 = in0 ? L : 0.0, S1 = in1 ? L : 0.0;
        wave_total2(S0, S1);
        const double pf = clamp_p1(S1 / (S0 + S1));
        const double u = lane_value(uf, level);
        const int bit = (u < pf) ? 1 : 0;
        if (lane == 0) bits[(size_t)t * n + (n - 1 - level)] = (uint8_t)bit;
        if (bit) lo += half;
        size = half;
      }
      // within the selected lane's 8: every lane reads the same amplitudes
      int lo2 = 0, size2 = 8;
      for (; level < n; ++level) {
        const int half = size2 >> 1;
        double S0 = 0.0, S1 = 0.0;
        for (int k = 0; k < size2; ++k) {
          const C2<T> a = S.psi[sslot((uint32_t)(lo * 8 + lo2 + k))];
          const double w = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
          if (k < half) S0 += w; else S1 += w;
        }
        const double pf = clamp_p1(S1 / (S0 + S1));
        const double u = lane_value(uf, level);
        const int bit = (u < pf) ? 1 : 0;
        if (lane == 0) bits[(size_t)t * n + (n - 1 - level)] = (uint8_t)bit;
        if (bit) lo2 += half;
        size2 = half;
      }
    }
    __syncthreads();  // the slot is rewritten by the next trajectory
  }
}

}  // namespace qec
