// HIP kernels for gfx950 (CDNA4, wave64).
//
// Trajectory engine (the delayed-measurement loop of Sec. II.B):
//   k_prepare      per (trajectory, block instance): draw the block's noise
//                  and measurement uniforms, build its two Kraus operators.
//   k_pass         one HBM pass per stabilizer circuit: apply the decided
//                  Kraus operator of block a, the ZZ layer and the
//                  renormalisation, and accumulate S_0, S_1 of block b; the
//                  last workgroup reduces the partial sums in a fixed order and
//                  decides block b's outcome on the device.
//   k_final_sums / k_final_measure   sequential Z measurement of the data
//                  register (highest label first) from a two-level sum tree.
// General register ops behind sv_apply_gate / sv_apply_diag / sv_apply_fused /
// sv_measure_reset_ancilla.
#include "qec_common.h"

namespace qec {

template <typename T> struct C2 { T re, im; };

template <typename T>
__device__ __forceinline__ C2<T> ld2(const T* p, uint64_t i) {
  if constexpr (sizeof(T) == 8) {
    const double2 v = reinterpret_cast<const double2*>(p)[i];
    return {v.x, v.y};
  } else {
    const float2 v = reinterpret_cast<const float2*>(p)[i];
    return {v.x, v.y};
  }
}
template <typename T>
__device__ __forceinline__ void st2(T* p, uint64_t i, C2<T> v) {
  if constexpr (sizeof(T) == 8) {
    reinterpret_cast<double2*>(p)[i] = make_double2(v.re, v.im);
  } else {
    reinterpret_cast<float2*>(p)[i] = make_float2(v.re, v.im);
  }
}

template <typename T>
__device__ __forceinline__ C2<T> mulc(C2<T> a, T br, T bi) {
  return {a.re * br - a.im * bi, a.re * bi + a.im * br};
}

// In-register Walsh-Hadamard transform (no normalisation) over the low W bits
// of v[base .. base + 2^W).
template <typename T, int W>
__device__ __forceinline__ void wht(C2<T>* v) {
#pragma unroll
  for (int h = 1; h < (1 << W); h <<= 1) {
#pragma unroll
    for (int i = 0; i < (1 << W); ++i) {
      if (i & h) continue;
      const C2<T> a = v[i], b = v[i | h];
      v[i] = {a.re + b.re, a.im + b.im};
      v[i | h] = {a.re - b.re, a.im - b.im};
    }
  }
}

// LDS slot of compressed tile index l: XOR-swizzle of the low 4 bits with
// higher bits so strided lane patterns spread over the banks.
__device__ __forceinline__ uint32_t lslot(uint32_t l) { return l ^ (((l >> 4) ^ (l >> 8)) & 15u); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block reduction of two doubles (fixed order).  `scratch`
// holds 2 * (blockDim/64) doubles.  Result valid in thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* scratch) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wid] = a;
    scratch[2 * wid + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < nw; ++w) {
      sa += scratch[2 * w];
      sb += scratch[2 * w + 1];
    }
    a = sa;
    b = sb;
  }
}

__device__ __forceinline__ double clamp_p1(double p1) {
  if (p1 < 1e-10) return 0.0;
  if (p1 > 1.0 - 1e-10) return 1.0;
  return p1;
}

// ---------------------------------------------------------------- prepare --
__global__ void k_prepare(const TBlock* __restrict__ blocks, int n_stab, int rounds,
                          int draws_per_round, uint64_t seed, uint64_t traj0, int n_traj,
                          double p, const double* __restrict__ eps_site,
                          BlockRT* __restrict__ out, int* __restrict__ err) {
  const int per_traj = rounds * n_stab;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)per_traj * n_traj) return;
  const int ti = (int)(gid / per_traj);
  const int bi = (int)(gid % per_traj);
  const int r = bi / n_stab, s = bi % n_stab;
  const TBlock& b = blocks[s];
  uint8_t pauli[kMaxOps];
  BlockRT rt;
  const uint64_t k0 = (uint64_t)r * (uint64_t)draws_per_round + (uint64_t)b.draw_off;
  draw_block(b, seed, traj0 + (uint64_t)ti, k0, p, pauli, &rt.u);
  if (!build_block(b, eps_site, pauli, rt)) atomicOr(err, 1);
  rt.pad = 0;
  out[gid] = rt;
}

// -------------------------------------------------------------------- pass --
constexpr int kTileMax = 12;  // 4096 amplitudes per tile

template <typename T>
struct PassLds {
  T v[2 << kTileMax];
};

template <typename T, int WA, int WB>
__global__ __launch_bounds__(256) void k_pass(
    T* __restrict__ st, const PassDesc* __restrict__ pd, const JobConst* __restrict__ jc,
    const BlockRT* __restrict__ rta, const BlockRT* __restrict__ rtb,
    const Decision* __restrict__ dec_a, Decision* __restrict__ dec_b,
    double2* __restrict__ partials, unsigned* __restrict__ counter,
    uint8_t* __restrict__ rec_b, double* __restrict__ p1_b) {
  __shared__ PassLds<T> sh;
  __shared__ double red[16];
  __shared__ int is_last;
  const int tid = threadIdx.x;
  const int tb = pd->tb;
  const int nt = 1 << (tb - 4);
  const bool active = tid < nt;

  uint32_t base = 0;
  for (int i = 0; i < pd->n_outer; ++i)
    if ((blockIdx.x >> i) & 1u) base |= pd->outer_bit[i];

  // ---------------- phase 1: apply block a (or write logical |0>) ----------
  if (active) {
    uint32_t gt = 0, lt = 0;
    for (int i = 0; i < tb - 4; ++i)
      if ((tid >> i) & 1) {
        gt |= pd->a_tid_g[i];
        lt |= pd->a_tid_l[i];
      }
    C2<T> v[16];
    if constexpr (WA == 0) {
      const T amp = (T)jc->amp0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        uint32_t x = base | gt | pd->a_j_g[j];
        for (int i = 0; i < jc->n_x; ++i)
          if (x & jc->span_piv[i]) x ^= jc->span_vec[i];
        v[j] = {x == 0 ? amp : (T)0, (T)0};
        const uint32_t g = base | gt | pd->a_j_g[j];
        st2(st, g, v[j]);
        st2(sh.v, lslot(lt | pd->a_j_l[j]), v[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = ld2(st, base | gt | pd->a_j_g[j]);
      const int m = dec_a->m;
      const double scale = 1.0 / sqrt(dec_a->Sm);
      const uint32_t F = rta->F;
      const double* D = &rta->D[m][0][0];
      constexpr int NA = 1 << WA;
      if (pd->typea == 0) {
#pragma unroll
        for (int hi = 0; hi < 16; hi += NA) {
          wht<T, WA>(v + hi);
#pragma unroll
          for (int x = 0; x < NA; ++x) v[hi + x] = mulc(v[hi + x], (T)D[2 * x], (T)D[2 * x + 1]);
          wht<T, WA>(v + hi);
#pragma unroll
          for (int x = 0; x < NA; ++x)
            if (__popc((uint32_t)x & F) & 1) v[hi + x] = {-v[hi + x].re, -v[hi + x].im};
        }
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int x = j & (NA - 1);
          v[j] = mulc(v[j], (T)D[2 * x], (T)D[2 * x + 1]);
        }
      }
      // destination: XOR permutation of block a's bits for Z checks
      uint32_t fg = 0, fl = 0;
      if (pd->typea != 0) {
#pragma unroll
        for (int l = 0; l < WA; ++l)
          if ((F >> l) & 1) {
            fg |= pd->a_q_g[l];
            fl |= pd->a_q_l[l];
          }
      }
      const int use_zz = jc->use_zz;
      const int d = jc->d;
      const uint32_t hm = jc->hmask, vm = jc->vmask;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t g = (base | gt | pd->a_j_g[j]) ^ fg;
        C2<T> o = v[j];
        if (use_zz) {
          const int k = __popc((g ^ (g >> 1)) & hm) + __popc((g ^ (g >> d)) & vm);
          o = mulc(o, (T)jc->zz[2 * k], (T)jc->zz[2 * k + 1]);
        }
        if constexpr (sizeof(T) == 8) {
          o.re *= scale;
          o.im *= scale;
        } else {
          o.re = (T)((double)o.re * scale);
          o.im = (T)((double)o.im * scale);
        }
        st2(st, g, o);
        if constexpr (WB != 0) st2(sh.v, lslot((lt | pd->a_j_l[j]) ^ fl), o);
      }
    }
  }
  if constexpr (WB == 0) return;

  __syncthreads();
  // ---------------- phase 2: S_0, S_1 of block b ----------------------------
  double s0 = 0.0, s1 = 0.0;
  if (active) {
    uint32_t lt = 0;
    for (int i = 0; i < tb - 4; ++i)
      if ((tid >> i) & 1) lt |= pd->b_tid_l[i];
    C2<T> v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = ld2(sh.v, lslot(lt | pd->b_j_l[j]));
    constexpr int NB = (WB == 0) ? 1 : (1 << WB);
    const double* W0 = rtb->W[0];
    const double* W1 = rtb->W[1];
#pragma unroll
    for (int hi = 0; hi < 16; hi += NB) {
      if (pd->typeb == 0) wht<T, WB>(v + hi);
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        const double re = (double)v[hi + x].re, im = (double)v[hi + x].im;
        const double a2 = re * re + im * im;
        s0 += W0[x] * a2;
        s1 += W1[x] * a2;
      }
    }
  }
  block_sum2(s0, s1, red);
  if (tid == 0) {
    __hip_atomic_store(&partials[blockIdx.x].x, s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&partials[blockIdx.x].y, s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    is_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double a0 = 0.0, a1 = 0.0;
  for (unsigned i = tid; i < gridDim.x; i += blockDim.x) {
    a0 += __hip_atomic_load(&partials[i].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a1 += __hip_atomic_load(&partials[i].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum2(a0, a1, red);
  if (tid == 0) {
    const double p1 = clamp_p1(a1 / (a0 + a1));
    const int m = (rtb->u < p1) ? 1 : 0;
    dec_b->m = m;
    dec_b->Sm = m ? a1 : a0;
    *rec_b = (uint8_t)m;
    if (p1_b) *p1_b = p1;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------ final measurement --
// Sums of |psi|^2 over contiguous chunks of 2^cb amplitudes.
template <typename T>
__global__ __launch_bounds__(256) void k_final_sums(const T* __restrict__ st, int cb,
                                                     double* __restrict__ sums) {
  __shared__ double red[16];
  const uint64_t base = (uint64_t)blockIdx.x << cb;
  const int len = 1 << cb;
  double s = 0.0, dummy = 0.0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const C2<T> a = ld2(st, base + i);
    const double re = (double)a.re, im = (double)a.im;
    s += re * re + im * im;
  }
  block_sum2(s, dummy, red);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__device__ double range_sum(const double* buf, int lo, int len, double* red) {
  double s = 0.0, dummy = 0.0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) s += buf[lo + i];
  block_sum2(s, dummy, red);
  __shared__ double bcast;
  if (threadIdx.x == 0) bcast = s;
  __syncthreads();
  const double r = bcast;
  __syncthreads();
  return r;
}

// Sequential measurement of data qubits n-1 .. 0 (labels n .. 1) using the
// chunk sums for the high n - cb bits and the selected chunk for the rest.
template <typename T>
__global__ __launch_bounds__(1024) void k_final_measure(const T* __restrict__ st, int n, int cb,
                                                         const double* __restrict__ sums,
                                                         uint64_t seed, uint64_t t, uint64_t k0,
                                                         uint8_t* __restrict__ bits) {
  __shared__ double buf[8192];
  __shared__ double red[32];
  const int hb = n - cb;  // bits resolved by chunk sums
  const int nchunk = 1 << hb;
  for (int i = threadIdx.x; i < nchunk; i += blockDim.x) buf[i] = sums[i];
  __syncthreads();
  int lo = 0, size = nchunk;
  int level = 0;
  for (; level < hb; ++level) {
    const int half = size >> 1;
    const double S0 = range_sum(buf, lo, half, red);
    const double S1 = range_sum(buf, lo + half, half, red);
    const double p1 = clamp_p1(S1 / (S0 + S1));
    const double u = uniform(seed, t, k0 + (uint64_t)level);
    const int b = (u < p1) ? 1 : 0;
    if (threadIdx.x == 0) bits[n - 1 - level] = (uint8_t)b;
    if (b) lo += half;
    size = half;
  }
  const uint64_t cbase = (uint64_t)lo << cb;
  const int len = 1 << cb;
  __syncthreads();
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const C2<T> a = ld2(st, cbase + i);
    const double re = (double)a.re, im = (double)a.im;
    buf[i] = re * re + im * im;
  }
  __syncthreads();
  lo = 0;
  size = len;
  for (; level < n; ++level) {
    const int half = size >> 1;
    const double S0 = range_sum(buf, lo, half, red);
    const double S1 = range_sum(buf, lo + half, half, red);
    const double p1 = clamp_p1(S1 / (S0 + S1));
    const double u = uniform(seed, t, k0 + (uint64_t)level);
    const int b = (u < p1) ? 1 : 0;
    if (threadIdx.x == 0) bits[n - 1 - level] = (uint8_t)b;
    if (b) lo += half;
    size = half;
  }
}

// --------------------------------------------------------- register ops --
struct Mat2 { double m[8]; };
struct Mat4 { double m[32]; };
struct Diag32 { double ph[64]; };

template <typename T>
__global__ void k_fill_basis(T* __restrict__ st, uint64_t n_amp, uint64_t idx) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_amp) return;
  st2(st, i, C2<T>{(T)(i == idx ? 1 : 0), (T)0});
}

template <typename T>
__global__ void k_logical0(T* __restrict__ st, uint64_t n_amp, const JobConst* __restrict__ jc) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_amp) return;
  bool in = (i >> jc->n) == 0;
  uint32_t x = (uint32_t)(i & ((1ull << jc->n) - 1));
  for (int k = 0; k < jc->n_x; ++k)
    if (x & jc->span_piv[k]) x ^= jc->span_vec[k];
  in = in && (x == 0);
  st2(st, i, C2<T>{in ? (T)jc->amp0 : (T)0, (T)0});
}

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int q) {
  const uint64_t lo = x & ((1ull << q) - 1);
  return ((x >> q) << (q + 1)) | lo;
}

template <typename T>
__global__ void k_gate1(T* __restrict__ st, uint64_t n_pairs, int q, Mat2 M) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const uint64_t i0 = insert_zero(p, q), i1 = i0 | (1ull << q);
  const C2<T> a = ld2(st, i0), b = ld2(st, i1);
  C2<T> o0, o1;
  o0.re = (T)M.m[0] * a.re - (T)M.m[1] * a.im + (T)M.m[2] * b.re - (T)M.m[3] * b.im;
  o0.im = (T)M.m[0] * a.im + (T)M.m[1] * a.re + (T)M.m[2] * b.im + (T)M.m[3] * b.re;
  o1.re = (T)M.m[4] * a.re - (T)M.m[5] * a.im + (T)M.m[6] * b.re - (T)M.m[7] * b.im;
  o1.im = (T)M.m[4] * a.im + (T)M.m[5] * a.re + (T)M.m[6] * b.im + (T)M.m[7] * b.re;
  st2(st, i0, o0);
  st2(st, i1, o1);
}

// qlo < qhi; local index bit 0 = q0 (first listed), bit 1 = q1.
template <typename T>
__global__ void k_gate2(T* __restrict__ st, uint64_t n_quads, int q0, int q1, Mat4 M) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_quads) return;
  const int qlo = q0 < q1 ? q0 : q1, qhi = q0 < q1 ? q1 : q0;
  const uint64_t i00 = insert_zero(insert_zero(p, qlo), qhi);
  const uint64_t b0 = 1ull << q0, b1 = 1ull << q1;
  const uint64_t idx[4] = {i00, i00 | b0, i00 | b1, i00 | b0 | b1};
  C2<T> v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = ld2(st, idx[r]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    T re = 0, im = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T mr = (T)M.m[8 * r + 2 * c], mi = (T)M.m[8 * r + 2 * c + 1];
      re += mr * v[c].re - mi * v[c].im;
      im += mr * v[c].im + mi * v[c].re;
    }
    st2(st, idx[r], C2<T>{re, im});
  }
}

template <typename T>
__global__ void k_diag(T* __restrict__ st, uint64_t n_amp, int k, int q0, int q1, int q2, int q3, int q4, Diag32 D) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_amp) return;
  const int qs[5] = {q0, q1, q2, q3, q4};
  int loc = 0;
  for (int j = 0; j < k; ++j) loc |= (int)((i >> qs[j]) & 1) << j;
  const C2<T> a = ld2(st, i);
  st2(st, i, mulc(a, (T)D.ph[2 * loc], (T)D.ph[2 * loc + 1]));
}

// Dense K-qubit matrix on sorted-insert groups; matrix staged in LDS.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_fused(T* __restrict__ st, uint64_t n_groups,
                                               const double* __restrict__ mat, int q0, int q1,
                                               int q2, int q3, int q4) {
  constexpr int N = 1 << K;
  __shared__ T sm[2 * N * N];
  for (int i = threadIdx.x; i < 2 * N * N; i += blockDim.x) sm[i] = (T)mat[i];
  __syncthreads();
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const int qs[5] = {q0, q1, q2, q3, q4};
  // insert zeros at the sorted qubit positions
  int sorted[5];
  for (int j = 0; j < K; ++j) sorted[j] = qs[j];
  for (int a = 1; a < K; ++a)
    for (int b = a; b > 0 && sorted[b - 1] > sorted[b]; --b) {
      const int t = sorted[b]; sorted[b] = sorted[b - 1]; sorted[b - 1] = t;
    }
  uint64_t base = g;
  for (int j = 0; j < K; ++j) base = insert_zero(base, sorted[j]);
  uint64_t off[N];
  C2<T> v[N];
#pragma unroll
  for (int x = 0; x < N; ++x) {
    uint64_t o = base;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if ((x >> j) & 1) o |= 1ull << qs[j];
    off[x] = o;
    v[x] = ld2(st, o);
  }
#pragma unroll
  for (int r = 0; r < N; ++r) {
    T re = 0, im = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const T mr = sm[2 * (N * r + c)], mi = sm[2 * (N * r + c) + 1];
      re += mr * v[c].re - mi * v[c].im;
      im += mr * v[c].im + mi * v[c].re;
    }
    st2(st, off[r], C2<T>{re, im});
  }
}

// S0 / S1 over bit q; last workgroup decides (forced >= 0 overrides u).
struct MeasOut {
  double S0, S1, p1;
  int m;
  int pad;
};

template <typename T>
__global__ __launch_bounds__(256) void k_measure_sums(const T* __restrict__ st, uint64_t n_amp, int q,
                                                      double u, int forced,
                                                      double2* __restrict__ partials,
                                                      unsigned* __restrict__ counter,
                                                      MeasOut* __restrict__ out) {
  __shared__ double red[16];
  __shared__ int is_last;
  double s0 = 0.0, s1 = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_amp; i += stride) {
    const C2<T> a = ld2(st, i);
    const double w = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
    if ((i >> q) & 1) s1 += w; else s0 += w;
  }
  block_sum2(s0, s1, red);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&partials[blockIdx.x].x, s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&partials[blockIdx.x].y, s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    is_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double a0 = 0.0, a1 = 0.0;
  for (unsigned i = threadIdx.x; i < gridDim.x; i += blockDim.x) {
    a0 += __hip_atomic_load(&partials[i].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a1 += __hip_atomic_load(&partials[i].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum2(a0, a1, red);
  if (threadIdx.x == 0) {
    const double p1 = clamp_p1(a1 / (a0 + a1));
    out->S0 = a0;
    out->S1 = a1;
    out->p1 = p1;
    out->m = forced >= 0 ? forced : ((u < p1) ? 1 : 0);
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T>
__global__ void k_project(T* __restrict__ st, uint64_t n_pairs, int q, const MeasOut* __restrict__ mo) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const int m = mo->m;
  const double Sm = m ? mo->S1 : mo->S0;
  const double scale = 1.0 / sqrt(Sm);
  const uint64_t i0 = insert_zero(p, q), i1 = i0 | (1ull << q);
  C2<T> a = ld2(st, m ? i1 : i0);
  a.re = (T)((double)a.re * scale);
  a.im = (T)((double)a.im * scale);
  st2(st, i0, a);
  st2(st, i1, C2<T>{(T)0, (T)0});
}

}  // namespace qec
