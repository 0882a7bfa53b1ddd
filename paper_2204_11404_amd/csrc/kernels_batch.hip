// Batched trajectories for small distances (d = 2, 3: at most 2^9 data
// amplitudes).  One persistent launch runs thousands of trajectories with
// their own round counts, depolarizing probabilities and over-rotation
// angles.  The whole data register of a trajectory lives in LDS; a wave runs
// two trajectories, one per half-wave, in lockstep over the stabilizer
// template; each half-wave takes trajectories from a static list (sorted
// longest-first by the host) until the list is exhausted, so every wave
// reaches the exit.
//
// Per trajectory (set-up): cos/sin of every gate site's angle, the channel
// thresholds j p / 3 and j p / 15, and the noise-free Kraus pair of every
// stabilizer template are tabulated in LDS.
// Per stabilizer circuit (Sec. II.B: one circuit at a time, ancilla measured
// and reset):
//   1. one lane per random draw evaluates Philox (noise locations, then the
//      measurement draw); a half-wave vote tells whether any location drew a
//      Pauli;
//   2. only then, one lane per block-basis label runs the circuit's ops with
//      the drawn Paulis on the ancilla 2-vector (track_column); otherwise the
//      tabulated noise-free pair is used;
//   3. each lane loads a group of 16 amplitudes spanning the check's qubits,
//      transforms them to the check basis, and accumulates S_0, S_1; a
//      half-wave reduction gives p1 and the outcome on the device; the lane
//      then applies D_m, transforms back, applies the ZZ layer and 1/sqrt(S_m)
//      and writes the group back.
// After the last round the data qubits are measured one by one from the
// highest label down (two-level descent: lane sums, then within one lane).
#include "qec_common.h"

namespace qec {

constexpr int kSmallBits = 9;
constexpr int kSmallAmps = 1 << kSmallBits;
constexpr int kSmallStab = 8;     // d <= 3
constexpr int kSmallSites = 64;   // gate sites per round, d <= 3

// Per block template: where each of a lane's 16 amplitudes and each lane bit
// sit in the register (bit values).
struct SmallDesc {
  uint32_t j_off[16];
  uint32_t lane_bit[8];
  uint32_t q_bit[4];
  int n_lane_bits;
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
  double u[32];                 // draws of the current block
  uint32_t F;
  int pad;
};

__device__ __forceinline__ uint32_t sslot(uint32_t i) { return i ^ (((i >> 4) ^ (i >> 8)) & 15u); }

// Sum over the 32 lanes of this half-wave (every lane gets the same total).
__device__ __forceinline__ double half_sum(double v) {
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Tables of a new trajectory: site angles, thresholds, logical |0>.
template <typename T>
__device__ void small_setup_tables(SmallSlot<T>& S, int lane, int n, int ns, const TBlock* blocks,
                                   const JobConst* jc, const double* eps, double p) {
  // cos / sin of every site's angle
  for (int s = 0; s < ns; ++s) {
    const TBlock& b = blocks[s];
    for (int i = lane; i < b.n_ops; i += 32) {
      const TOp& op = b.ops[i];
      if (op.site < 0) continue;
      const double beta = op_angle(op, eps);
      S.cs[2 * op.site] = cos(beta);
      S.cs[2 * op.site + 1] = sin(beta);
    }
  }
  if (lane < 3) S.t1[lane] = (double)(lane + 1) * p / 3.0;
  if (lane < 15) S.t2[lane] = (double)(lane + 1) * p / 15.0;
  // logical |0>
  const int groups = 1 << (n - 4);
  if (lane < groups) {
    for (int k = 0; k < 16; ++k) {
      uint32_t x = (uint32_t)(lane * 16 + k);
      const uint32_t idx = x;
      for (int i = 0; i < jc->n_x; ++i)
        if (x & jc->span_piv[i]) x ^= jc->span_vec[i];
      S.psi[sslot(idx)] = C2<T>{x == 0 ? (T)jc->amp0 : (T)0, (T)0};
    }
  }
}

// Noise-free Kraus pair of every template (needs the angle table).
template <typename T>
__device__ void small_setup_kraus(SmallSlot<T>& S, int lane, int ns, const TBlock* blocks, int* err) {
  const uint8_t none[kMaxOps] = {};
  for (int i = lane; i < ns * 16; i += 32) {
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

template <typename T>
__global__ __launch_bounds__(64) void k_batch_small(
    const TBlock* __restrict__ blocks, const SmallDesc* __restrict__ sdesc, int ns, int n,
    int draws_round, const JobConst* __restrict__ jc, const uint64_t* __restrict__ tseed,
    const uint64_t* __restrict__ tstream,
    const int* __restrict__ order, int n_traj, const int* __restrict__ rounds,
    const double* __restrict__ pvec, const double* __restrict__ eps, int eps_stride,
    uint8_t* __restrict__ rec, int max_rounds, uint8_t* __restrict__ bits, int* __restrict__ err) {
  __shared__ SmallSlot<T> slots[2];
  // ZZ phases are read per amplitude: keep them in LDS (the round template
  // stays in global memory: more LDS per workgroup would cost occupancy)
  __shared__ C2<T> lzz[kSmallBits * 2 + 1];
  for (int i = threadIdx.x; i <= jc->n_edges && i <= 2 * kSmallBits; i += blockDim.x)
    lzz[i] = C2<T>{(T)jc->zz[2 * i], (T)jc->zz[2 * i + 1]};
  __syncthreads();
  const int use_zz = jc->use_zz, zd = jc->d;
  const uint32_t hmask = jc->hmask, vmask = jc->vmask;

  const int h = threadIdx.x >> 5;
  const int lane = threadIdx.x & 31;
  SmallSlot<T>& S = slots[h];
  const int n_slots = gridDim.x * 2;
  const int groups = 1 << (n - 4);
  const uint64_t half_mask = 0xFFFFFFFFull << (32 * h);

  int qi = blockIdx.x * 2 + h;
  bool active = qi < n_traj;
  int t = active ? order[qi] : 0;
  int R = active ? rounds[t] : 0;
  int r = 0;
  double p = active ? pvec[t] : 0.0;
  uint64_t tg = tstream[t], seed = tseed[t];  // draw stream of the current trajectory
  small_setup_tables(S, lane, n, ns, blocks, jc, eps + (size_t)t * eps_stride, p);
  __syncthreads();
  small_setup_kraus(S, lane, ns, blocks, err);
  __syncthreads();

  while (__any(active)) {
    for (int s = 0; s < ns; ++s) {
      const TBlock& b = blocks[s];
      const SmallDesc& sd = sdesc[s];
      const uint64_t k0 = (uint64_t)r * (uint64_t)draws_round + (uint64_t)b.draw_off;
      // 1. draws; did any noise location pick a Pauli?
      bool hit = false;
      if (lane < b.n_draws) {
        const double u = uniform(seed, tg, k0 + (uint64_t)lane);
        S.u[lane] = u;
        if (lane < b.n_draws - 1) hit = u < (((b.n2mask >> lane) & 1) ? S.t2[14] : S.t1[2]);
      }
      const bool noisy = (__ballot(hit) & half_mask) != 0;
      __syncthreads();
      // 2. Kraus pair of this block instance
      const int nx = 1 << b.w;
      if (noisy && lane < nx) {
        uint8_t pauli[kMaxOps];
        for (int i = 0; i < b.n_ops; ++i) {
          const TOp& op = b.ops[i];
          uint8_t c = 0;
          if (op.draw >= 0) {
            const double u = S.u[op.draw];
            if (op.kind == OP_N1_ANC || op.kind == OP_N1_DATA) {
              for (int j = 0; j < 3 && !c; ++j)
                if (u < S.t1[j]) c = (uint8_t)(j + 1);
            } else {
              for (int j = 0; j < 15 && !c; ++j)
                if (u < S.t2[j]) c = (uint8_t)(j + 1);
            }
          }
          pauli[i] = c;
        }
        cd v0, v1;
        uint32_t cur = 0;
        if (!track_column(b, CsFromTable{S.cs}, pauli, lane, v0, v1, &cur) && active) atomicOr(err, 1);
        const double norm = b.type == 0 ? 1.0 / (double)nx : 1.0;
        S.D[0][lane] = C2<T>{(T)(v0.re * norm), (T)(v0.im * norm)};
        S.D[1][lane] = C2<T>{(T)(v1.re * norm), (T)(v1.im * norm)};
        S.W[0][lane] = (v0.re * v0.re + v0.im * v0.im) * norm;
        S.W[1][lane] = (v1.re * v1.re + v1.im * v1.im) * norm;
        if (lane == 0) S.F = cur;  // label 0 maps to F
      }
      __syncthreads();
      const C2<T>(*D)[16] = noisy ? S.D : S.Dc[s];
      const double(*W)[16] = noisy ? S.W : S.Wc[s];
      const uint32_t F = noisy ? S.F : 0u;
      // 3. measure and apply
      uint32_t lb = 0;
      for (int i = 0; i < sd.n_lane_bits; ++i)
        if ((lane >> i) & 1) lb |= sd.lane_bit[i];
      const bool g_on = lane < groups;
      C2<T> v[16];
      double s0 = 0.0, s1 = 0.0;
      const bool xb = b.type == 0;
      if (g_on) {
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = S.psi[sslot(lb | sd.j_off[j])];
        if (b.w == 4) {
          if (xb) wht<T, 4>(v);
#pragma unroll
          for (int x = 0; x < 16; ++x) {
            const double re = (double)v[x].re, im = (double)v[x].im, a2 = re * re + im * im;
            s0 += W[0][x] * a2;
            s1 += W[1][x] * a2;
          }
        } else {
#pragma unroll
          for (int hi = 0; hi < 16; hi += 4) {
            if (xb) wht<T, 2>(v + hi);
#pragma unroll
            for (int x = 0; x < 4; ++x) {
              const double re = (double)v[hi + x].re, im = (double)v[hi + x].im, a2 = re * re + im * im;
              s0 += W[0][x] * a2;
              s1 += W[1][x] * a2;
            }
          }
        }
      }
      s0 = half_sum(s0);
      s1 = half_sum(s1);
      const double p1 = clamp_p1(s1 / (s0 + s1));
      const int m = (S.u[b.n_draws - 1] < p1) ? 1 : 0;
      if (active && lane == 0) rec[((size_t)t * max_rounds + r) * ns + s] = (uint8_t)m;
      const double scale = 1.0 / sqrt(m ? s1 : s0);
      if (g_on) {
        const int wmask = nx - 1;
        if (b.w == 4) {
#pragma unroll
          for (int x = 0; x < 16; ++x) v[x] = mulc(v[x], D[m][x].re, D[m][x].im);
          if (xb) wht<T, 4>(v);
        } else {
#pragma unroll
          for (int hi = 0; hi < 16; hi += 4) {
#pragma unroll
            for (int x = 0; x < 4; ++x) v[hi + x] = mulc(v[hi + x], D[m][x].re, D[m][x].im);
            if (xb) wht<T, 2>(v + hi);
          }
        }
        uint32_t fo = 0;
        if (!xb)
          for (int l = 0; l < b.w; ++l)
            if ((F >> l) & 1) fo |= sd.q_bit[l];
        const T sc = (T)scale;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          C2<T> o = v[j];
          if (xb && (__popc((uint32_t)(j & wmask) & F) & 1)) o = {-o.re, -o.im};
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
    // round boundary
    ++r;
    const bool done = active && (r == R);
    if (__any(done)) {
      // final Z measurement of the data register, highest label first
      double L = 0.0;
      if (lane < groups) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const C2<T> a = S.psi[sslot((uint32_t)(lane * 16 + k))];
          L += (double)a.re * (double)a.re + (double)a.im * (double)a.im;
        }
      }
      const uint64_t kf = (uint64_t)R * (uint64_t)draws_round;
      const double uf = lane < n ? uniform(seed, tg, kf + (uint64_t)lane) : 0.0;
      int lo = 0, size = groups, level = 0;
      for (; level < n - 4; ++level) {
        const int half = size >> 1;
        const bool in0 = lane >= lo && lane < lo + half;
        const bool in1 = lane >= lo + half && lane < lo + size;
        const double S0 = half_sum(in0 ? L : 0.0);
        const double S1 = half_sum(in1 ? L : 0.0);
        const double pf = clamp_p1(S1 / (S0 + S1));
        const double u = __shfl(uf, (h << 5) + level, 64);
        const int bit = (u < pf) ? 1 : 0;
        if (done && lane == 0) bits[(size_t)t * n + (n - 1 - level)] = (uint8_t)bit;
        if (bit) lo += half;
        size = half;
      }
      // within the selected group of 16: every lane reads the same amplitudes
      int lo2 = 0, size2 = 16;
      for (; level < n; ++level) {
        const int half = size2 >> 1;
        double S0 = 0.0, S1 = 0.0;
        for (int k = 0; k < size2; ++k) {
          const C2<T> a = S.psi[sslot((uint32_t)(lo * 16 + lo2 + k))];
          const double w = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
          if (k < half) S0 += w; else S1 += w;
        }
        const double pf = clamp_p1(S1 / (S0 + S1));
        const double u = __shfl(uf, (h << 5) + level, 64);
        const int bit = (u < pf) ? 1 : 0;
        if (done && lane == 0) bits[(size_t)t * n + (n - 1 - level)] = (uint8_t)bit;
        if (bit) lo2 += half;
        size2 = half;
      }
      __syncthreads();
      if (done) {
        qi += n_slots;
        active = qi < n_traj;
        if (active) {
          t = order[qi];
          R = rounds[t];
          p = pvec[t];
          r = 0;
          tg = tstream[t];
          seed = tseed[t];
        }
      }
      // set-up of the next trajectory (barriers in wave-uniform control flow;
      // only halves that switched write their slot)
      const bool fresh = done && active;
      if (__any(fresh)) {
        if (fresh) small_setup_tables(S, lane, n, ns, blocks, jc, eps + (size_t)t * eps_stride, p);
        __syncthreads();
        if (fresh) small_setup_kraus(S, lane, ns, blocks, err);
      }
      __syncthreads();
    }
  }
}

}  // namespace qec
