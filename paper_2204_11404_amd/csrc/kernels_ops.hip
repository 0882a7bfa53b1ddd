// HIP kernels for gfx950: the general register operations behind the C ABI
// (copy, basis states, logical |0>, one- and two-qubit gates, diagonal phase
// layers, dense fused k-qubit gates, Walsh-Hadamard layers for the X-basis
// readout, and the ancilla measure-and-reset of sv_measure_reset_ancilla).
// They share the register helpers of kernels.hip.
#include "qec_common.h"

namespace qec {

// --------------------------------------------------------- register ops --
// Plain streaming copy, 16-byte elements, four per thread per iteration.
__global__ __launch_bounds__(256) void k_copy16(double2* __restrict__ dst,
                                                const double2* __restrict__ src, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 4;
  for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x) * 4 + threadIdx.x; i < n; i += stride) {
    double2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i + (uint64_t)k * blockDim.x < n) v[k] = src[i + (uint64_t)k * blockDim.x];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i + (uint64_t)k * blockDim.x < n) dst[i + (uint64_t)k * blockDim.x] = v[k];
  }
}

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

// Two-qubit gate on qubits 0 and 1: thread i holds amplitude i (every load
// and store is one contiguous wave-wide access); the other three amplitudes
// of its quadruple are in the lanes of its DPP quad (quad_perm xor 1, 2, 3).
// Lane i computes row r(i) of M, read from LDS.  Needs whole 256-thread
// blocks.  swap: qubits listed as (1, 0).
template <typename T>
__device__ __forceinline__ T quad_xor(T v, int d) {  // lane ^ d within the quad
  return d == 1 ? dpp_mv<0xB1>(v) : d == 2 ? dpp_mv<0x4E>(v) : dpp_mv<0x1B>(v);
}
template <typename T>
__global__ __launch_bounds__(256) void k_gate2_quad(T* __restrict__ st, int swap, Mat4 M) {
  __shared__ T sm[32];
  if (threadIdx.x < 32) sm[threadIdx.x] = (T)M.m[threadIdx.x];
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const C2<T> a = ld2(st, i);
  const int x = (int)(i & 3);                               // address bits 0, 1
  auto local = [&](int y) { return swap ? ((y >> 1) & 1) | ((y & 1) << 1) : y; };
  const int r = local(x);
  T re = 0, im = 0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const C2<T> v = d == 0 ? a : C2<T>{quad_xor(a.re, d), quad_xor(a.im, d)};
    const int c = local(x ^ d);
    const T mr = sm[2 * (4 * r + c)], mi = sm[2 * (4 * r + c) + 1];
    re += mr * v.re - mi * v.im;
    im += mr * v.im + mi * v.re;
  }
  st2(st, i, C2<T>{re, im});
}

// The same gate for complex64 registers: thread i holds amplitudes 2 i and
// 2 i + 1 (one 16-byte access), its pair lane i ^ 1 the other half of the
// quadruple (DPP quad_perm xor 1); each thread computes its two rows.
__global__ __launch_bounds__(256) void k_gate2_pair_f32(float* __restrict__ st, int swap, Mat4 M) {
  __shared__ float sm[32];
  if (threadIdx.x < 32) sm[threadIdx.x] = (float)M.m[threadIdx.x];
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float4 a = reinterpret_cast<const float4*>(st)[i];
  const float4 b{dpp_mv<0xB1>(a.x), dpp_mv<0xB1>(a.y), dpp_mv<0xB1>(a.z), dpp_mv<0xB1>(a.w)};
  const int hi = (int)(i & 1);  // address bit 1 of this thread's pair
  // address-local amplitudes 0..3 of the quadruple
  C2<float> v[4];
  v[2 * hi] = {a.x, a.y};
  v[2 * hi + 1] = {a.z, a.w};
  v[2 * (1 - hi)] = {b.x, b.y};
  v[2 * (1 - hi) + 1] = {b.z, b.w};
  auto local = [&](int y) { return swap ? ((y >> 1) & 1) | ((y & 1) << 1) : y; };
  C2<float> out[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = local(2 * hi + k);
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int c = local(x);
      const float mr = sm[2 * (4 * r + c)], mi = sm[2 * (4 * r + c) + 1];
      re += mr * v[x].re - mi * v[x].im;
      im += mr * v[x].im + mi * v[x].re;
    }
    out[k] = {re, im};
  }
  reinterpret_cast<float4*>(st)[i] = make_float4(out[0].re, out[0].im, out[1].re, out[1].im);
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

// Dense K-qubit matrix (K = 4 or 5) on the matrix cores: for every group of
// 2^K amplitudes (the groups are the columns of V), Y = M V as 16x16x4 MFMA
// tiles, FP64 for complex128 and FP32 for complex64.  The real and imaginary
// parts are separate products: Yr = Mr Vr - Mi Vi, Yi = Mr Vi + Mi Vr.
//
// One wave owns 16 groups at a time (the 16 columns of a B/D tile), with the
// operand layouts of Mfma16: lane (c, q) = (lane % 16, lane / 16) loads
// element 4 s + q of group c for K step s, and for FP32 the rows of M are
// permuted (row 16 t + 4 q + r holds element 16 t + 4 r + q), so that for
// either type register r of row tile t holds element 16 t + 4 r + q: a store
// writes the same bit pattern a load reads.  The matrix stays in registers
// for the whole (persistent) launch.
template <typename T, int K, bool PF>
__global__ __launch_bounds__(256) void k_fused_mfma(T* __restrict__ st, uint64_t n_tiles,
                                                    const double* __restrict__ mat, int q0, int q1,
                                                    int q2, int q3, int q4) {
  static_assert(K == 4 || K == 5, "MFMA tiles need 16 or 32 rows");
  constexpr int N = 1 << K, RT = N / 16, KS = N / 4;
  using V4 = typename Mfma16<T>::V4;
  const int lane = threadIdx.x & 63, c = lane & 15, q = lane >> 4;
  const int qs[5] = {q0, q1, q2, q3, q4};
  int sorted[5];
#pragma unroll
  for (int j = 0; j < K; ++j) sorted[j] = qs[j];
#pragma unroll
  for (int a = 1; a < K; ++a)
#pragma unroll
    for (int b = a; b > 0; --b)
      if (sorted[b - 1] > sorted[b]) {
        const int t = sorted[b]; sorted[b] = sorted[b - 1]; sorted[b - 1] = t;
      }
  // register offset of local element bits 0,1 (this lane's q) and of bits
  // 2.. (K step s, or 4 t + r on the store side)
  const uint64_t xq = ((q & 1) ? 1ull << q0 : 0) | ((q & 2) ? 1ull << q1 : 0);
  uint64_t xh[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    uint64_t o = 0;
#pragma unroll
    for (int j = 2; j < K; ++j)
      if ((s >> (j - 2)) & 1) o |= 1ull << qs[j];
    xh[s] = o;
  }
  T ar[RT][KS], ai[RT][KS];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int row = 16 * t + (Mfma16<T>::kPermuteRows ? 4 * (c & 3) + (c >> 2) : c);
      const int col = 4 * s + q;
      ar[t][s] = (T)mat[2 * (N * row + col)];
      ai[t][s] = (T)mat[2 * (N * row + col) + 1];
    }
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t n_waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  auto tile_base = [&](uint64_t tl) {
    uint64_t b = tl * 16 + c;
#pragma unroll
    for (int j = 0; j < K; ++j) b = insert_zero(b, sorted[j]);
    return b | xq;
  };
  // PF: the next tile's loads are issued before this tile's products
  C2<T> v[KS];
  uint64_t tl = wave, base = 0;
  if (PF && tl < n_tiles) {
    base = tile_base(tl);
#pragma unroll
    for (int s = 0; s < KS; ++s) v[s] = ld2(st, base | xh[s]);
  }
  for (; tl < n_tiles; tl += n_waves) {
    if (!PF) {
      base = tile_base(tl);
#pragma unroll
      for (int s = 0; s < KS; ++s) v[s] = ld2(st, base | xh[s]);
    }
    C2<T> vn[PF ? KS : 1];
    uint64_t base_n = 0;
    if (PF && tl + n_waves < n_tiles) {
      base_n = tile_base(tl + n_waves);
#pragma unroll
      for (int s = 0; s < (PF ? KS : 1); ++s) vn[s] = ld2(st, base_n | xh[s]);
    }
    V4 yr[RT], yi[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      yr[t] = V4{0, 0, 0, 0};
      yi[t] = V4{0, 0, 0, 0};
    }
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        yr[t] = Mfma16<T>::op(ar[t][s], v[s].re, yr[t]);
        yi[t] = Mfma16<T>::op(ar[t][s], v[s].im, yi[t]);
        yi[t] = Mfma16<T>::op(ai[t][s], v[s].re, yi[t]);
        yr[t] = Mfma16<T>::op(ai[t][s], -v[s].im, yr[t]);
      }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) st2(st, base | xh[4 * t + r], C2<T>{yr[t][r], yi[t][r]});
    if (PF) {
#pragma unroll
      for (int s = 0; s < (PF ? KS : 1); ++s) v[s] = vn[s];
      base = base_n;
    }
  }
}

// The same product when the K target qubits are the register's K lowest bits
// (in any order): the 16 groups of a wave tile are 16 N consecutive
// amplitudes, so the wave moves them with 16-byte loads and stores that each
// cover a contiguous block, and regroups them through its own LDS region
// (rows of N + 1 amplitudes, so that the 16 groups of an MFMA operand fall
// on different banks).  q[j]: register bit of local bit j.  The library runs
// it for complex64 registers, whose 8-byte amplitudes the direct kernel
// reads in 32-byte pieces on these bits.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_fused_mfma_low(T* __restrict__ st, uint64_t n_tiles,
                                                        const double* __restrict__ mat, int q0,
                                                        int q1, int q2, int q3, int q4) {
  static_assert(K == 4 || K == 5, "MFMA tiles need 16 or 32 rows");
  constexpr int N = 1 << K, RT = N / 16, KS = N / 4, P = N + 1;
  constexpr int AMPS = 16 * N;                          // amplitudes of a wave tile
  constexpr int PER16 = 16 / (2 * sizeof(T));           // amplitudes per 16-byte access
  constexpr int ACC = AMPS / (64 * PER16);              // 16-byte accesses per lane
  using V4 = typename Mfma16<T>::V4;
  __shared__ C2<T> lds[4][16 * P];
  const int lane = threadIdx.x & 63, c = lane & 15, q = lane >> 4, w = threadIdx.x >> 6;
  C2<T>* reg = lds[w];
  const int qs[5] = {q0, q1, q2, q3, q4};
  auto perm = [&](int x) {
    int o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if ((x >> j) & 1) o |= 1 << qs[j];
    return o;
  };
  int xo[KS];  // in-group offset of element 4 s + q (bits 0, 1 from q)
#pragma unroll
  for (int s = 0; s < KS; ++s) xo[s] = perm(4 * s + q);
  T ar[RT][KS], ai[RT][KS];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int row = 16 * t + (Mfma16<T>::kPermuteRows ? 4 * (c & 3) + (c >> 2) : c);
      const int col = 4 * s + q;
      ar[t][s] = (T)mat[2 * (N * row + col)];
      ai[t][s] = (T)mat[2 * (N * row + col) + 1];
    }
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + w;
  const uint64_t n_waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t tl = wave; tl < n_tiles; tl += n_waves) {
    const uint64_t base = tl * AMPS;
    // contiguous 16-byte loads into the padded rows
#pragma unroll
    for (int a = 0; a < ACC; ++a) {
      const int e = (a * 64 + lane) * PER16;  // first amplitude of this access
      C2<T> v[PER16];
      if constexpr (sizeof(T) == 8) {
        const double2 d = reinterpret_cast<const double2*>(st)[base + e];
        v[0] = {d.x, d.y};
      } else {
        const float4 f = reinterpret_cast<const float4*>(st)[(base + e) >> 1];
        v[0] = {f.x, f.y};
        v[PER16 - 1] = {f.z, f.w};
      }
#pragma unroll
      for (int i = 0; i < PER16; ++i) reg[((e + i) >> K) * P + ((e + i) & (N - 1))] = v[i];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the wave's LDS writes are done
    V4 yr[RT], yi[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      yr[t] = V4{0, 0, 0, 0};
      yi[t] = V4{0, 0, 0, 0};
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const C2<T> x = reg[c * P + xo[s]];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        yr[t] = Mfma16<T>::op(ar[t][s], x.re, yr[t]);
        yi[t] = Mfma16<T>::op(ar[t][s], x.im, yi[t]);
        yi[t] = Mfma16<T>::op(ai[t][s], x.re, yi[t]);
        yr[t] = Mfma16<T>::op(ai[t][s], -x.im, yr[t]);
      }
    }
    __builtin_amdgcn_wave_barrier();  // every lane has read its operands
    // register r of row tile t holds element 16 t + 4 r + q of group c
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) reg[c * P + perm(16 * t + 4 * r + q)] = C2<T>{yr[t][r], yi[t][r]};
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
#pragma unroll
    for (int a = 0; a < ACC; ++a) {
      const int e = (a * 64 + lane) * PER16;
      C2<T> v[PER16];
#pragma unroll
      for (int i = 0; i < PER16; ++i) v[i] = reg[((e + i) >> K) * P + ((e + i) & (N - 1))];
      if constexpr (sizeof(T) == 8) {
        reinterpret_cast<double2*>(st)[base + e] = make_double2(v[0].re, v[0].im);
      } else {
        reinterpret_cast<float4*>(st)[(base + e) >> 1] =
            make_float4(v[0].re, v[0].im, v[PER16 - 1].re, v[PER16 - 1].im);
      }
    }
    __builtin_amdgcn_wave_barrier();  // the next tile overwrites the rows
  }
}

// Walsh-Hadamard transform over K qubits (bits q[0..K)) of the register, one
// group of 2^K amplitudes per thread, times `scale` (the X-basis readout
// applies H to every data qubit as ceil(n / 5) such passes).
template <typename T, int K>
__global__ __launch_bounds__(256) void k_wht_group(T* __restrict__ st, uint64_t n_groups, int q0,
                                                   int q1, int q2, int q3, int q4, double scale) {
  constexpr int N = 1 << K;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const int qs[5] = {q0, q1, q2, q3, q4};
  int sorted[5];
  for (int j = 0; j < K; ++j) sorted[j] = qs[j];
  for (int a = 1; a < K; ++a)
    for (int b = a; b > 0 && sorted[b - 1] > sorted[b]; --b) {
      const int t = sorted[b];
      sorted[b] = sorted[b - 1];
      sorted[b - 1] = t;
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
  wht<T, K>(v);
#pragma unroll
  for (int x = 0; x < N; ++x)
    st2(st, off[x], C2<T>{(T)((double)v[x].re * scale), (T)((double)v[x].im * scale)});
}

// S0 / S1 over bit q: per-workgroup partial sums (fixed order).
struct MeasOut {
  double S0, S1, p1;
  int m;
  int pad;
};

template <typename T>
__global__ __launch_bounds__(256) void k_measure_sums(const T* __restrict__ st, uint64_t n_amp, int q,
                                                      double2* __restrict__ partials) {
  __shared__ double red[16];
  double s0 = 0.0, s1 = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_amp; i += stride) {
    const C2<T> a = ld2(st, i);
    const double w = (double)a.re * (double)a.re + (double)a.im * (double)a.im;
    if ((i >> q) & 1) s1 += w; else s0 += w;
  }
  block_sum2(s0, s1, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(s0, s1);
}

// Reduce the partials in a fixed order and decide (forced >= 0 overrides u).
__global__ __launch_bounds__(256) void k_measure_decide(const double2* __restrict__ partials, int n,
                                                        double u, int forced,
                                                        MeasOut* __restrict__ out) {
  __shared__ double red[16];
  double a0 = 0.0, a1 = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double2 v = partials[i];
    a0 += v.x;
    a1 += v.y;
  }
  block_sum2(a0, a1, red);
  if (threadIdx.x == 0) {
    const double p1 = clamp_p1(a1 / (a0 + a1));
    out->S0 = a0;
    out->S1 = a1;
    out->p1 = p1;
    out->m = forced >= 0 ? forced : ((u < p1) ? 1 : 0);
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
