// Batched trajectories whose data register does not fit in LDS (d = 4: 2^16
// amplitudes).  A persistent launch gives each 256-thread workgroup one
// trajectory at a time (static list, longest first); the workgroup keeps the
// register in its own HBM slice and streams it in tiles of 2^12 amplitudes.
// Each stabilizer circuit costs one read and one write of the register: the
// pass applies the previous circuit's Kraus operator (outcome already decided)
// and accumulates S_0, S_1 of the next one; the workgroup reduces them and
// decides the outcome itself, so no other workgroup is involved.  Kraus
// pairs, angle tables and thresholds live in LDS (noise-free pairs cached per
// template; a circuit whose draws hit a Pauli is rebuilt by one wave).
#include "qec_common.h"

namespace qec {

constexpr int kTiledStab = 15;    // d = 4
constexpr int kTiledSites = 128;  // gate sites per round, d = 4

template <typename T>
struct KrausBuf {
  C2<T> D[2][16];
  double W[2][16];
  double u_meas;
  uint32_t F;
  int pad;
};

template <typename T>
struct TiledLds {
  C2<T> tbuf[1 << kTileMax];
  C2<T> Dc[kTiledStab][2][16];
  double Wc[kTiledStab][2][16];
  KrausBuf<T> kb[2];
  double cs[2 * kTiledSites];
  double t1[3], t2[15];
  double u[32];
  C2<T> zzt[64];
  double red[16];
  double sm;
  int m;
  int pad;
};

// Kraus pair of block instance (round r, template s) into kb[slot].
template <typename T>
__device__ void tiled_kraus(TiledLds<T>& L, int slot, const TBlock& b, int s, int r,
                            int draws_round, uint64_t seed, uint64_t tg, int* err) {
  const int tid = threadIdx.x;
  const uint64_t k0 = (uint64_t)r * (uint64_t)draws_round + (uint64_t)b.draw_off;
  bool hit = false;
  if (tid < b.n_draws) {
    const double u = uniform(seed, tg, k0 + (uint64_t)tid);
    L.u[tid] = u;
    if (tid < b.n_draws - 1) hit = u < (((b.n2mask >> tid) & 1) ? L.t2[14] : L.t1[2]);
  }
  const int noisy = __syncthreads_or(hit);
  KrausBuf<T>& K = L.kb[slot];
  const int nx = 1 << b.w;
  if (noisy) {
    if (tid < nx) {
      uint8_t pauli[kMaxOps];
      for (int i = 0; i < b.n_ops; ++i) {
        const TOp& op = b.ops[i];
        uint8_t c = 0;
        if (op.draw >= 0) {
          const double u = L.u[op.draw];
          if (op.kind == OP_N1_ANC || op.kind == OP_N1_DATA) {
            for (int j = 0; j < 3 && !c; ++j)
              if (u < L.t1[j]) c = (uint8_t)(j + 1);
          } else {
            for (int j = 0; j < 15 && !c; ++j)
              if (u < L.t2[j]) c = (uint8_t)(j + 1);
          }
        }
        pauli[i] = c;
      }
      cd v0, v1;
      uint32_t cur = 0;
      if (!track_column(b, CsFromTable{L.cs}, pauli, tid, v0, v1, &cur)) atomicOr(err, 1);
      const double norm = b.type == 0 ? 1.0 / (double)nx : 1.0;
      K.D[0][tid] = C2<T>{(T)(v0.re * norm), (T)(v0.im * norm)};
      K.D[1][tid] = C2<T>{(T)(v1.re * norm), (T)(v1.im * norm)};
      K.W[0][tid] = (v0.re * v0.re + v0.im * v0.im) * norm;
      K.W[1][tid] = (v1.re * v1.re + v1.im * v1.im) * norm;
      if (tid == 0) K.F = cur;
    }
  } else if (tid < 2 * nx) {
    const int m = tid / nx, x = tid % nx;
    K.D[m][x] = L.Dc[s][m][x];
    K.W[m][x] = L.Wc[s][m][x];
    if (tid == 0) K.F = 0;
  }
  if (tid == 0) K.u_meas = L.u[b.n_draws - 1];
  __syncthreads();
}

// One pass over the register: apply kb[ka] (outcome L.m, norm L.sm) of a
// block with WA qubits (WA == 0: write logical |0>), accumulate S of kb[kbi].
template <typename T, int WA, int WB, int BMODE>
__device__ void tiled_pass(TiledLds<T>& L, T* st, const PassDesc* pd, const JobConst* jc, int ka,
                           int kbi, double& s0, double& s1) {
  const int tid = threadIdx.x;
  const int tb = pd->tb;
  uint32_t gt = 0, lt = 0, lbt = 0;
  for (int i = 0; i < tb - 4; ++i)
    if ((tid >> i) & 1) {
      gt |= pd->a_tid_g[i];
      lt |= pd->a_tid_l[i];
      lbt |= pd->a_tid_lb[i];
    }
  uint32_t blt = 0;
  for (int i = 0; i < tb - 4; ++i)
    if ((tid >> i) & 1) blt |= pd->b_tid_l[i];
  int m = 0;
  double scale = 1.0;
  uint32_t F = 0, fg = 0, fl = 0, lbf = 0;
  if constexpr (WA != 0) {
    m = L.m;
    scale = 1.0 / sqrt(L.sm);
    F = L.kb[ka].F;
    if (pd->typea != 0)
      for (int l = 0; l < WA; ++l)
        if ((F >> l) & 1) {
          fg |= pd->a_q_g[l];
          fl |= pd->a_q_l[l];
          lbf ^= pd->a_q_lb[l];
        }
  }
  const C2<T>* D = L.kb[ka].D[m];
  const double* W0 = L.kb[kbi].W[0];
  const double* W1 = L.kb[kbi].W[1];
  const int use_zz = (WA != 0) && jc->use_zz;
  const int d = jc->d;
  const uint32_t hm = jc->hmask, vm = jc->vmask;
  const int n_tiles = 1 << pd->n_outer;
  for (int tile = 0; tile < n_tiles; ++tile) {
    uint32_t base = 0;
    for (int i = 0; i < pd->n_outer; ++i)
      if ((tile >> i) & 1) base |= pd->outer_bit[i];
    C2<T> o[16];
    if constexpr (WA == 0) {
      const T amp = (T)jc->amp0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t g = base | gt | pd->a_j_g[j];
        uint32_t x = g;
        for (int i = 0; i < jc->n_x; ++i)
          if (x & jc->span_piv[i]) x ^= jc->span_vec[i];
        o[j] = {x == 0 ? amp : (T)0, (T)0};
        st2(st, g, o[j]);
      }
    } else {
      C2<T> v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = ld2(st, base | gt | pd->a_j_g[j]);
      constexpr int NA = 1 << WA;
      if (pd->typea == 0) {
#pragma unroll
        for (int hi = 0; hi < 16; hi += NA) {
          wht<T, WA>(v + hi);
#pragma unroll
          for (int x = 0; x < NA; ++x) v[hi + x] = mulc(v[hi + x], D[x].re, D[x].im);
          wht<T, WA>(v + hi);
#pragma unroll
          for (int x = 0; x < NA; ++x)
            if (__popc((uint32_t)x & F) & 1) v[hi + x] = {-v[hi + x].re, -v[hi + x].im};
        }
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = mulc(v[j], D[j & (NA - 1)].re, D[j & (NA - 1)].im);
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t g = (base | gt | pd->a_j_g[j]) ^ fg;
        C2<T> r = v[j];
        if (use_zz) {
          const int k = __popc((g ^ (g >> 1)) & hm) + __popc((g ^ (g >> d)) & vm);
          const C2<T> z = L.zzt[k];
          r = mulc(r, z.re, z.im);
        }
        if constexpr (sizeof(T) == 8) {
          r.re *= scale;
          r.im *= scale;
        } else {
          r.re = (T)((double)r.re * scale);
          r.im = (T)((double)r.im * scale);
        }
        st2(st, g, r);
        o[j] = r;
      }
    }
    if constexpr (BMODE == B_ZCHECK) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t x = (lbt | pd->a_j_lb[j]) ^ lbf;
        const double re = (double)o[j].re, im = (double)o[j].im, a2 = re * re + im * im;
        s0 += W0[x] * a2;
        s1 += W1[x] * a2;
      }
    }
    if constexpr (BMODE == B_XCHECK) {
#pragma unroll
      for (int j = 0; j < 16; ++j) L.tbuf[lslot((lt | pd->a_j_l[j]) ^ fl)] = o[j];
      __syncthreads();
      C2<T> v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = L.tbuf[lslot(blt | pd->b_j_l[j])];
      constexpr int NB = 1 << WB;
#pragma unroll
      for (int hi = 0; hi < 16; hi += NB) {
        wht<T, WB>(v + hi);
#pragma unroll
        for (int x = 0; x < NB; ++x) {
          const double re = (double)v[hi + x].re, im = (double)v[hi + x].im, a2 = re * re + im * im;
          s0 += W0[x] * a2;
          s1 += W1[x] * a2;
        }
      }
      __syncthreads();
    }
  }
}

template <typename T>
__device__ void tiled_pass_dispatch(int wa, int wb, int bmode, TiledLds<T>& L, T* st,
                                    const PassDesc* pd, const JobConst* jc, int ka, int kbi,
                                    double& s0, double& s1) {
#define QEC_TP(A, B, M)                                               \
  if (wa == A && wb == B && bmode == M) {                             \
    tiled_pass<T, A, B, M>(L, st, pd, jc, ka, kbi, s0, s1);           \
    return;                                                           \
  }
  QEC_TP(0, 2, B_XCHECK) QEC_TP(0, 4, B_XCHECK) QEC_TP(0, 2, B_ZCHECK) QEC_TP(0, 4, B_ZCHECK)
  QEC_TP(2, 0, B_NONE) QEC_TP(4, 0, B_NONE)
  QEC_TP(2, 2, B_XCHECK) QEC_TP(2, 4, B_XCHECK) QEC_TP(4, 2, B_XCHECK) QEC_TP(4, 4, B_XCHECK)
  QEC_TP(2, 2, B_ZCHECK) QEC_TP(2, 4, B_ZCHECK) QEC_TP(4, 2, B_ZCHECK) QEC_TP(4, 4, B_ZCHECK)
#undef QEC_TP
}

// Outcome of the block measured by the last pass; broadcast through LDS.
template <typename T>
__device__ void tiled_decide(TiledLds<T>& L, int kbi, double s0, double s1, uint8_t* rec_at) {
  block_sum2(s0, s1, L.red);
  if (threadIdx.x == 0) {
    const double p1 = clamp_p1(s1 / (s0 + s1));
    const int m = (L.kb[kbi].u_meas < p1) ? 1 : 0;
    L.m = m;
    L.sm = m ? s1 : s0;
    if (rec_at) *rec_at = (uint8_t)m;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_batch_tiled(
    const TBlock* __restrict__ blocks, const PassDesc* __restrict__ pds, int ns, int n,
    int draws_round, const JobConst* __restrict__ jc, const uint64_t* __restrict__ tseed,
    const uint64_t* __restrict__ tstream,
    const int* __restrict__ order, int n_traj, const int* __restrict__ rounds,
    const double* __restrict__ pvec, const double* __restrict__ eps, int eps_stride,
    uint8_t* __restrict__ rec, int max_rounds, uint8_t* __restrict__ bits, T* __restrict__ work,
    int* __restrict__ err) {
  __shared__ TiledLds<T> L;
  const int tid = threadIdx.x;
  T* st = work + ((size_t)blockIdx.x << n) * 2;
  if (jc->use_zz && tid <= jc->n_edges)
    L.zzt[tid] = C2<T>{(T)jc->zz[2 * tid], (T)jc->zz[2 * tid + 1]};
  for (int qi = blockIdx.x; qi < n_traj; qi += gridDim.x) {
    const int t = order[qi];
    const int R = rounds[t];
    const double p = pvec[t];
    const double* ep = eps + (size_t)t * eps_stride;
    const uint64_t tg = tstream[t], seed = tseed[t];
    // tables
    for (int s = 0; s < ns; ++s) {
      const TBlock& b = blocks[s];
      if (tid < b.n_ops && b.ops[tid].site >= 0) {
        const TOp& op = b.ops[tid];
        const double beta = op_angle(op, ep);
        L.cs[2 * op.site] = cos(beta);
        L.cs[2 * op.site + 1] = sin(beta);
      }
    }
    if (tid < 3) L.t1[tid] = (double)(tid + 1) * p / 3.0;
    if (tid < 15) L.t2[tid] = (double)(tid + 1) * p / 15.0;
    __syncthreads();
    if (tid < ns * 16) {
      const int s = tid >> 4, x = tid & 15;
      const TBlock& b = blocks[s];
      if (x < (1 << b.w)) {
        const uint8_t none[kMaxOps] = {};
        cd v0, v1;
        uint32_t cur = 0;
        if (!track_column(b, CsFromTable{L.cs}, none, x, v0, v1, &cur)) atomicOr(err, 1);
        const double norm = b.type == 0 ? 1.0 / (double)(1 << b.w) : 1.0;
        L.Dc[s][0][x] = C2<T>{(T)(v0.re * norm), (T)(v0.im * norm)};
        L.Dc[s][1][x] = C2<T>{(T)(v1.re * norm), (T)(v1.im * norm)};
        L.Wc[s][0][x] = (v0.re * v0.re + v0.im * v0.im) * norm;
        L.Wc[s][1][x] = (v1.re * v1.re + v1.im * v1.im) * norm;
      }
    }
    __syncthreads();
    uint8_t* rt = rec + (size_t)t * max_rounds * ns;
    // logical |0> and the first measurement
    tiled_kraus(L, 0, blocks[0], 0, 0, draws_round, seed, tg, err);
    {
      double s0 = 0.0, s1 = 0.0;
      tiled_pass_dispatch<T>(0, blocks[0].w, blocks[0].type == 0 ? B_XCHECK : B_ZCHECK, L, st,
                             &pds[0], jc, 0, 0, s0, s1);
      tiled_decide(L, 0, s0, s1, rt);
    }
    const int total = R * ns;
    for (int bi = 0; bi < total; ++bi) {
      const int sa = bi % ns;
      const bool last = (bi == total - 1);
      const int ka = bi & 1, kbi = (bi + 1) & 1;
      int wb = 0, bmode = B_NONE;
      if (!last) {
        const int sb = (bi + 1) % ns;
        tiled_kraus(L, kbi, blocks[sb], sb, (bi + 1) / ns, draws_round, seed, tg, err);
        wb = blocks[sb].w;
        bmode = blocks[sb].type == 0 ? B_XCHECK : B_ZCHECK;
      }
      double s0 = 0.0, s1 = 0.0;
      tiled_pass_dispatch<T>(blocks[sa].w, wb, bmode, L, st, &pds[last ? ns + 1 : 1 + sa], jc, ka,
                             kbi, s0, s1);
      __syncthreads();
      if (!last) tiled_decide(L, kbi, s0, s1, rt + bi + 1);
    }
    // final Z measurement, highest label first: tile sums, then the chosen tile
    {
      const int cb = kTileMax < n ? kTileMax : n;
      const int hb = n - cb;
      const uint64_t kf = (uint64_t)R * (uint64_t)draws_round;
      double* buf = reinterpret_cast<double*>(L.tbuf);  // >= 2^cb doubles for complex64 and 128
      int lo = 0;
      int level = 0;
      if (hb > 0) {
        // sums of the 2^hb contiguous chunks
        for (int c = 0; c < (1 << hb); ++c) {
          double sacc = 0.0, dummy = 0.0;
          for (int i = tid; i < (1 << cb); i += blockDim.x) {
            const C2<T> a = ld2(st, ((uint64_t)c << cb) + i);
            sacc += (double)a.re * (double)a.re + (double)a.im * (double)a.im;
          }
          block_sum2(sacc, dummy, L.red);
          if (tid == 0) L.u[c] = sacc;
          __syncthreads();
        }
        int size = 1 << hb;
        for (; level < hb; ++level) {
          const int half = size >> 1;
          double S0 = 0.0, S1 = 0.0;
          for (int c = 0; c < half; ++c) {
            S0 += L.u[lo + c];
            S1 += L.u[lo + half + c];
          }
          const double pf = clamp_p1(S1 / (S0 + S1));
          const int bit = (uniform(seed, tg, kf + (uint64_t)level) < pf) ? 1 : 0;
          if (tid == 0) bits[(size_t)t * n + (n - 1 - level)] = (uint8_t)bit;
          if (bit) lo += half;
          size = half;
        }
      }
      __syncthreads();
      for (int i = tid; i < (1 << cb); i += blockDim.x) {
        const C2<T> a = ld2(st, ((uint64_t)lo << cb) + i);
        buf[i] = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
      }
      __syncthreads();
      int lo2 = 0, size2 = 1 << cb;
      for (; level < n; ++level) {
        const int half = size2 >> 1;
        double S0 = 0.0, S1 = 0.0;
        for (int i = tid; i < half; i += blockDim.x) {
          S0 += buf[lo2 + i];
          S1 += buf[lo2 + half + i];
        }
        block_sum2(S0, S1, L.red);
        if (tid == 0) {
          const double pf = clamp_p1(S1 / (S0 + S1));
          const int bit = (uniform(seed, tg, kf + (uint64_t)level) < pf) ? 1 : 0;
          bits[(size_t)t * n + (n - 1 - level)] = (uint8_t)bit;
          L.m = bit;
        }
        __syncthreads();
        if (L.m) lo2 += half;
        size2 = half;
        __syncthreads();
      }
    }
  }
}

}  // namespace qec
