// HIP kernels for gfx950 (CDNA4, wave64).
//
// Trajectory engine (the delayed-measurement loop of Sec. II.B):
//   k_prepare      per (trajectory, block instance): draw the block's noise
//                  and measurement uniforms, build its two Kraus operators.
//   k_upass        one HBM pass per unit (an X check, or a chain of Z
//                  checks): apply the decided Kraus operators of unit A, the
//                  ZZ layers and the renormalisation, and accumulate the
//                  outcome sums of unit B.
//   k_udecide      fixed-order reduction of the per-workgroup sums and the
//                  outcomes of unit B's checks, on the device.
//   k_final_sums / k_final_measure   sequential Z measurement of the data
//                  register (highest label first) from a two-level sum tree.
//   k_commit       staged results of a replayed (graph) trajectory.
// General register ops are in kernels_ops.hip.
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

// The register through a buffer resource: an amplitude's byte offset is a
// per-thread part (VGPR) plus a per-slot part shared by the wave (SGPR), so
// a pass's 16 loads and stores per thread need no per-amplitude address
// arithmetic.  Offsets past `bytes` read 0 and drop stores.
template <typename T>
struct RegBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ RegBuf(T* p, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)bytes, 0x00020000)) {}  // raw dwords (gfx9)
  __device__ C2<T> ld(uint32_t voff, uint32_t soff) const {
    if constexpr (sizeof(T) == 8) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
      return {__hiloint2double((int)v[1], (int)v[0]), __hiloint2double((int)v[3], (int)v[2])};
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
      return {__uint_as_float(v[0]), __uint_as_float(v[1])};
    }
  }
  __device__ void st(uint32_t voff, uint32_t soff, C2<T> a) const {
    if constexpr (sizeof(T) == 8) {
      const unsigned long long x = __double_as_longlong(a.re), y = __double_as_longlong(a.im);
      __attribute__((ext_vector_type(4))) unsigned v = {(unsigned)x, (unsigned)(x >> 32), (unsigned)y,
                                                        (unsigned)(y >> 32)};
      __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, 0);
    } else {
      __attribute__((ext_vector_type(2))) unsigned v = {__float_as_uint(a.re), __float_as_uint(a.im)};
      __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
    }
  }
};

// LDS slot offsets in bytes: a thread's part (kept opaque, so the compiler
// does not fold the XOR back into a shift per access) XOR a slot's part
// (uniform: shifted on the scalar unit); one vector XOR per access.
template <typename E>
__device__ __forceinline__ uint32_t lds_bytes(uint32_t thread_slot) {
  uint32_t b = thread_slot * (uint32_t)sizeof(E);
  asm volatile("" : "+v"(b));
  return b;
}
template <typename E>
__device__ __forceinline__ E& lds_at(E* buf, uint32_t thread_bytes, uint32_t slot) {
  return *reinterpret_cast<E*>(reinterpret_cast<char*>(buf) + (thread_bytes ^ (slot * (uint32_t)sizeof(E))));
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


// Lane exchanges by DPP (every lane of the row of 16 active).
template <int CTRL>
__device__ __forceinline__ double dpp_mv(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mv(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
// Value of lane l ^ (1 << B), B = 0..3; upper: bit B of l is set.
template <int B, typename T>
__device__ __forceinline__ T lane_partner(T v, bool upper) {
  if constexpr (B == 0) {
    return dpp_mv<0xB1>(v);  // quad_perm 1,0,3,2
  } else if constexpr (B == 1) {
    return dpp_mv<0x4E>(v);  // quad_perm 2,3,0,1
  } else {
    const T from_above = dpp_mv<0x100 + (1 << B)>(v);  // row_shl: lane l reads l + 2^B
    const T from_below = dpp_mv<0x110 + (1 << B)>(v);  // row_shr: lane l reads l - 2^B
    return upper ? from_below : from_above;
  }
}

// Walsh-Hadamard stage over lane bit B for the thread's 16 amplitudes.
template <int B, typename T>
__device__ __forceinline__ void wht_lane(C2<T>* v, int tid) {
  const bool upper = (tid >> B) & 1;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const C2<T> o{lane_partner<B>(v[j].re, upper), lane_partner<B>(v[j].im, upper)};
    v[j] = upper ? C2<T>{o.re - v[j].re, o.im - v[j].im} : C2<T>{v[j].re + o.re, v[j].im + o.im};
  }
}

// Walsh-Hadamard transform of an X check A held partly on lane bits 0..3
// (mask lanes) and partly on the lowest r register slots.
template <int H, typename T>
__device__ __forceinline__ void wht_reg_stage(C2<T>* v) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i & H) continue;
    const C2<T> a = v[i], b = v[i | H];
    v[i] = {a.re + b.re, a.im + b.im};
    v[i | H] = {a.re - b.re, a.im - b.im};
  }
}
template <typename T>
__device__ __forceinline__ void wht_mixed(C2<T>* v, int r, int lanes, int tid) {
  if (r > 0) wht_reg_stage<1>(v);
  if (r > 1) wht_reg_stage<2>(v);
  if (r > 2) wht_reg_stage<4>(v);
  if (r > 3) wht_reg_stage<8>(v);
  if (lanes & 1) wht_lane<0>(v, tid);
  if (lanes & 2) wht_lane<1>(v, tid);
  if (lanes & 4) wht_lane<2>(v, tid);
  if (lanes & 8) wht_lane<3>(v, tid);
}

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
// Draws and Kraus pairs of every block instance of n_traj trajectories
// (draw streams traj0 + i, or *stream for a single trajectory when given);
// twirl_thr: per-site sin^2 eps of the Pauli-twirled model, or null.
__global__ void k_prepare(const TBlock* __restrict__ blocks, int n_stab, int rounds,
                          int draws_per_round, uint64_t seed, uint64_t traj0, int n_traj,
                          double p, const double* __restrict__ eps_site,
                          BlockRT* __restrict__ out, int* __restrict__ err,
                          const uint64_t* __restrict__ stream,
                          const double* __restrict__ twirl_thr) {
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
  const uint64_t t = stream ? *stream : traj0 + (uint64_t)ti;
  draw_block(b, seed, t, k0, p, pauli, &rt.u, twirl_thr);
  if (b.dense) {  // the Kraus pair comes from k_prepare_dense
    for (int m = 0; m < 2; ++m)
      for (int x = 0; x < 16; ++x) {
        rt.D[m][x][0] = rt.D[m][x][1] = 0.0;
        rt.W[m][x] = 0.0;
      }
    rt.F = 0;
  } else if (!build_block(b, eps_site, pauli, rt)) {
    atomicOr(err, 1);
  }
  rt.pad = 0;
  out[gid] = rt;
}

// Dense Kraus pairs of the blocks that are not monomial in their basis: one
// thread per (trajectory, block instance, input label x) runs the circuit on
// |anc 0, data x> with the instance's drawn Paulis and writes column x of K_0
// and K_1 (the same draws as k_prepare).
__global__ __launch_bounds__(128) void k_prepare_dense(
    const TBlock* __restrict__ blocks, int n_stab, int rounds, int draws_per_round, uint64_t seed,
    uint64_t traj0, int n_traj, double p, const double* __restrict__ eps_site,
    BlockDense* __restrict__ out, int* __restrict__ err, const uint64_t* __restrict__ stream,
    const double* __restrict__ twirl_thr) {
  const int per_traj = rounds * n_stab;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)per_traj * n_traj * 16) return;
  const int x = (int)(gid & 15);
  const int64_t inst = gid >> 4;
  const int ti = (int)(inst / per_traj);
  const int bi = (int)(inst % per_traj);
  const int r = bi / n_stab, s = bi % n_stab;
  const TBlock& b = blocks[s];
  if (!b.dense) return;
  BlockDense& o = out[inst];
  if (x >= (1 << b.w)) {
    for (int m = 0; m < 2; ++m)
      for (int i = 0; i < 16; ++i) o.K[m][i][x][0] = o.K[m][i][x][1] = 0.0;
    return;
  }
  uint8_t pauli[kMaxOps];
  double u;
  const uint64_t k0 = (uint64_t)r * (uint64_t)draws_per_round + (uint64_t)b.draw_off;
  const uint64_t t = stream ? *stream : traj0 + (uint64_t)ti;
  draw_block(b, seed, t, k0, p, pauli, &u, twirl_thr);
  cd psi[32];
  if (!dense_column(b, CsFromEps{eps_site}, pauli, x, psi)) atomicOr(err, 1);
  for (int m = 0; m < 2; ++m)
    for (int i = 0; i < 16; ++i) {
      const cd v = i < (1 << b.w) ? psi[(m << 4) | i] : cd{0.0, 0.0};
      o.K[m][i][x][0] = v.re;
      o.K[m][i][x][1] = v.im;
    }
}

// cos / sin of every gate site's angle for each trajectory slot (one thread
// per slot and op of the round template).
__global__ void k_site_cs(const TBlock* __restrict__ blocks, int n_stab,
                          const double* __restrict__ eps, int eps_stride, int n_sites, int slots,
                          double* __restrict__ cs) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)slots * n_stab * kMaxOps) return;
  const int slot = (int)(gid / (n_stab * kMaxOps));
  const int rem = (int)(gid % (n_stab * kMaxOps));
  const TBlock& b = blocks[rem / kMaxOps];
  const int i = rem % kMaxOps;
  if (i >= b.n_ops || b.ops[i].site < 0) return;
  const TOp& op = b.ops[i];
  const double beta = op_angle(op, eps + (size_t)slot * eps_stride);
  cs[((size_t)slot * n_sites + op.site) * 2] = cos(beta);
  cs[((size_t)slot * n_sites + op.site) * 2 + 1] = sin(beta);
}

// Kraus pairs of round r for `slots` trajectories with their own seed, draw
// stream and p: 16 lanes per block instance, lane x evaluates draw x (shared
// with the group by shuffles) and then the circuit's column x.
__global__ __launch_bounds__(256) void k_prepare_round(
    const TBlock* __restrict__ blocks, int n_stab, int r, int draws_round,
    const uint64_t* __restrict__ seeds, const uint64_t* __restrict__ streams,
    const double* __restrict__ pvec, const double* __restrict__ cs, int n_sites, int slots,
    BlockRT* __restrict__ out, int* __restrict__ err) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t inst = gid >> 4;  // (slot, stabilizer)
  const int x = (int)(gid & 15);
  const bool valid = inst < (int64_t)slots * n_stab;
  const int slot = valid ? (int)(inst / n_stab) : 0;
  const int s = valid ? (int)(inst % n_stab) : 0;
  const TBlock& b = blocks[s];
  const double p = pvec[slot];
  const uint64_t k0 = (uint64_t)r * (uint64_t)draws_round + (uint64_t)b.draw_off;
  const double u = (valid && x < b.n_draws) ? uniform(seeds[slot], streams[slot], k0 + (uint64_t)x) : 1.0;
  // every lane runs every shuffle (the op count differs between groups); the
  // host admits templates of at most kMaxOpsBatch ops and 16 draws here
  uint8_t pauli[kMaxOpsBatch];
  for (int i = 0; i < kMaxOpsBatch; ++i) {
    const TOp& op = b.ops[i];
    const bool drawn = i < b.n_ops && op.draw >= 0;
    const double ui = __shfl(u, drawn ? op.draw : 0, 16);
    pauli[i] = 0;
    if (drawn)
      pauli[i] = (uint8_t)((op.kind == OP_N1_ANC || op.kind == OP_N1_DATA) ? pick_pauli1(ui, p)
                                                                            : pick_pauli2(ui, p));
  }
  const double um = __shfl(u, b.n_draws - 1, 16);
  if (!valid) return;
  BlockRT& o = out[inst];
  const int nx = 1 << b.w;
  const double norm = b.type == 0 ? 1.0 / (double)nx : 1.0;
  if (x < nx) {
    cd v0, v1;
    uint32_t cur = 0;
    if (!track_column(b, CsFromTable{cs + (size_t)slot * n_sites * 2}, pauli, x, v0, v1, &cur))
      atomicOr(err, 1);
    o.D[0][x][0] = v0.re * norm;
    o.D[0][x][1] = v0.im * norm;
    o.D[1][x][0] = v1.re * norm;
    o.D[1][x][1] = v1.im * norm;
    o.W[0][x] = (v0.re * v0.re + v0.im * v0.im) * norm;
    o.W[1][x] = (v1.re * v1.re + v1.im * v1.im) * norm;
    if (x == 0) {
      o.F = cur;
      o.u = um;
      o.pad = 0;
    }
  } else {
    o.D[0][x][0] = o.D[0][x][1] = o.D[1][x][0] = o.D[1][x][1] = 0.0;
    o.W[0][x] = o.W[1][x] = 0.0;
  }
}

// -------------------------------------------------------------------- pass --
constexpr int kTileMax = 12;  // 4096 amplitudes per tile
constexpr int kMaxEdges = 40;  // ZZ neighbour pairs of the largest layout (d = 5)

// Several trajectories in one launch: blockIdx.y selects a trajectory slot;
// its register, Kraus tables and decisions sit at these strides (all zero for
// a single trajectory).
struct SlotStrides {
  size_t st;     // elements of T between registers
  size_t rt;     // BlockRT entries between slots
  size_t dec;    // Decision entries between slots
};

// Local index on a check's qubits (global bits q[0..w)) of global index g,
// and the global bits of a local pattern F.
__device__ __forceinline__ uint32_t gather_loc(uint32_t g, const uint32_t* q, int w) {
  uint32_t x = 0;
  for (int l = 0; l < w; ++l)
    if (g & q[l]) x |= 1u << l;
  return x;
}
__device__ __forceinline__ uint32_t scatter_loc(uint32_t F, const uint32_t* q, int w) {
  uint32_t g = 0;
  for (int l = 0; l < w; ++l)
    if ((F >> l) & 1) g |= q[l];
  return g;
}

// 16x16x4 matrix-core products (FP64 for complex128 registers, FP32 for
// complex64).  Operand layout: A[i][k] in lane (i + 16 k), B[k][j] in lane
// (j + 16 k); the result D[i][j] sits in lane (j + 16 (i % 4)), register i / 4
// for FP64 and in lane (j + 16 (i / 4)), register i % 4 for FP32 (both
// checked on gfx950).  kPermuteRows: the FP32 users permute A's rows so that
// register r of lane row q holds output 4 r + q for either type.
template <typename T> struct Mfma16;
template <> struct Mfma16<double> {
  static constexpr bool kPermuteRows = false;
  typedef double V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma16<float> {
  static constexpr bool kPermuteRows = true;
  typedef float V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Lane transpose for the matrix cores.  Lane l = 16 R + c holds the 16
// amplitudes v[0..15] of its own group; afterwards v[4 s + b] of lane
// 16 q + c holds element 4 s + q of the group of lane 16 b + c -- the B
// operand of K step s for the tile of row b's groups.  Two 2x2 exchanges of
// (row bit, register bit): lanes 32..63 <-> 0..31 for bit 1, odd <-> even
// 16-lane rows for bit 0.  Applying it twice restores the layout.
__device__ __forceinline__ void swap_rows32(uint32_t& x, uint32_t& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}
__device__ __forceinline__ void swap_rows16(uint32_t& x, uint32_t& y) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}
// The same swaps for doubles (two dwords each).
template <bool B32>
__device__ __forceinline__ void swap_d(double& a, double& b) {
  uint32_t x[2], y[2];
  __builtin_memcpy(x, &a, 8);
  __builtin_memcpy(y, &b, 8);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if constexpr (B32) swap_rows32(x[i], y[i]);
    else swap_rows16(x[i], y[i]);
  }
  __builtin_memcpy(&a, x, 8);
  __builtin_memcpy(&b, y, 8);
}

// Wave totals of 16 per-lane values in a fixed order: afterwards lane l
// holds the total of value (l >> 2) & 15.  A reduce-scatter: over lane bit 5
// and bit 4 each pair of values is swapped between the halves (rows) with a
// permlane swap and added (the lanes with the bit clear keep the lower
// values), over bits 3 and 2 the value to hand over is picked and moved by
// DPP; then butterflies over bits 1 and 0.  No LDS.
__device__ __forceinline__ double wave_reduce16(double (&v)[16]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    swap_d<true>(v[i], v[8 + i]);
    v[i] += v[8 + i];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    swap_d<false>(v[i], v[4 + i]);
    v[i] += v[4 + i];
  }
  const int lane = threadIdx.x & 63;
  const bool u3 = (lane >> 3) & 1, u2 = (lane >> 2) & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = u3 ? v[i] : v[2 + i], keep = u3 ? v[2 + i] : v[i];
    v[i] = keep + dpp_mv<0x128>(send);  // row_ror:8 within the row of 16: lane l ^ 8
  }
  {
    const double send = u2 ? v[0] : v[1], keep = u2 ? v[1] : v[0];
    v[0] = keep + lane_partner<2>(send, u2);
  }
  const double r = v[0] + dpp_mv<0x4E>(v[0]);  // quad_perm 2,3,0,1: lane l ^ 2
  return r + dpp_mv<0xB1>(r);                 // quad_perm 1,0,3,2: lane l ^ 1
}
template <typename T, bool B32>
__device__ __forceinline__ void swap_c2(C2<T>& a, C2<T>& b) {
  constexpr int W = sizeof(C2<T>) / 4;
  uint32_t x[W], y[W];
  __builtin_memcpy(x, &a, sizeof(x));
  __builtin_memcpy(y, &b, sizeof(y));
#pragma unroll
  for (int i = 0; i < W; ++i) {
    if constexpr (B32) swap_rows32(x[i], y[i]);
    else swap_rows16(x[i], y[i]);
  }
  __builtin_memcpy(&a, x, sizeof(x));
  __builtin_memcpy(&b, y, sizeof(y));
}
template <typename T>
__device__ __forceinline__ void xpose_rows(C2<T>* v) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    swap_c2<T, true>(v[4 * s + 0], v[4 * s + 2]);
    swap_c2<T, true>(v[4 * s + 1], v[4 * s + 3]);
    swap_c2<T, false>(v[4 * s + 0], v[4 * s + 1]);
    swap_c2<T, false>(v[4 * s + 2], v[4 * s + 3]);
  }
}

// y_b = K x_b for the four 16-group tiles of a transposed wave (xpose_rows):
// real and imaginary parts as four real products per K step; the result of
// tile b lands in v[4 r + b], the layout it was read from.  K: 16 x 16 in
// LDS.  Every lane of the wave must take part.
template <typename T>
__device__ __forceinline__ void mfma_tiles(C2<T>* v, const C2<T> (*K)[16], bool store,
                                           double& ssq) {
  using V4 = typename Mfma16<T>::V4;
  const int lane = threadIdx.x & 63, c = lane & 15, q = lane >> 4;
  const int row = Mfma16<T>::kPermuteRows ? 4 * (c & 3) + (c >> 2) : c;
  T ar[4], ai[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const C2<T> k = K[row][4 * s + q];
    ar[s] = k.re;
    ai[s] = k.im;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    V4 yr = V4{0, 0, 0, 0}, yi = V4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const C2<T> x = v[4 * s + b];
      yr = Mfma16<T>::op(ar[s], x.re, yr);
      yi = Mfma16<T>::op(ar[s], x.im, yi);
      yi = Mfma16<T>::op(ai[s], x.re, yi);
      yr = Mfma16<T>::op(ai[s], -x.im, yr);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (store) v[4 * r + b] = C2<T>{yr[r], yi[r]};
      ssq += (double)yr[r] * (double)yr[r] + (double)yi[r] * (double)yi[r];
    }
  }
}

// Dense Kraus operator on the matrix cores: v <- K v for each lane's 16
// amplitudes (the whole wave).
template <typename T>
__device__ __forceinline__ void mfma_dense_apply(C2<T>* v, const C2<T> (*K)[16]) {
  double unused = 0.0;
  xpose_rows(v);
  mfma_tiles(v, K, true, unused);
  xpose_rows(v);
}

// S_0, S_1 contributions of the wave's groups on the matrix cores (this
// lane's share of the sum over the wave; v is left unchanged).
template <typename T>
__device__ __forceinline__ void mfma_dense_sums(const C2<T>* v, const C2<T> (*K0)[16],
                                                const C2<T> (*K1)[16], double& s0, double& s1) {
  C2<T> w[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) w[j] = v[j];
  xpose_rows(w);
  double a = 0.0, b = 0.0;
  mfma_tiles(w, K0, false, a);
  mfma_tiles(w, K1, false, b);
  s0 += a;
  s1 += b;
}

// Dense Kraus pairs in the register's frame: with f the Pauli-X frame on the
// check's qubits, the physical operator is X^f K X^f, entry K[r ^ f][c ^ f];
// the pass stages those entries in LDS once per workgroup, in the register's
// precision (complex64 registers: products in FP32, each |K v|^2 summed in
// FP64; every amplitude read broadcasts one entry to the whole wave, so the
// LDS bytes per entry set the pass time).
template <typename T, int W>
__device__ __forceinline__ void dense_sums(const C2<T>* v, const C2<T> (*K0)[16],
                                           const C2<T> (*K1)[16], double& s0, double& s1) {
  constexpr int N = 1 << W;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const C2<T>(*K)[16] = m ? K1 : K0;
    double s = 0.0;
#pragma unroll 1
    for (int r = 0; r < N; ++r) {  // one row at a time: few live registers
      T yr = 0, yi = 0;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const C2<T> k = K[r][c];
        yr += k.re * v[c].re - k.im * v[c].im;
        yi += k.re * v[c].im + k.im * v[c].re;
      }
      s += (double)yr * (double)yr + (double)yi * (double)yi;
    }
    if (m == 0) s0 += s; else s1 += s;
  }
}

// LDS for the staged dense Kraus pairs (A's decided one, B's two); only the
// dense instantiation of the pass kernel allocates it.
template <typename T, bool DN>
__device__ __forceinline__ C2<T> (*dense_lds())[16][16] {
  if constexpr (DN) {
    __shared__ C2<T> k[3][16][16];
    return k;
  } else {
    return nullptr;
  }
}

// v <- K v for one group of 2^W amplitudes.
template <typename T, int W>
__device__ __forceinline__ void dense_apply(C2<T>* v, const C2<T> (*K)[16]) {
  constexpr int N = 1 << W;
  C2<T> y[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    T yr = 0, yi = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const C2<T> k = K[r][c];
      yr += k.re * v[c].re - k.im * v[c].im;
      yi += k.re * v[c].im + k.im * v[c].re;
    }
    y[r] = C2<T>{yr, yi};
  }
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] = y[r];
}

// Sums of an X check from a tile held in layout 1: regroup it through LDS
// into layout 2, where a lane holds the 16 amplitudes spanning the check's
// qubits.
template <typename T, int WB, bool DN>
__device__ __forceinline__ void xpose_xsums(const C2<T>* o, uint32_t lt_a, const UnitPass* pd,
                                            const double* w0, const double* w1, bool active,
                                            double& s0, double& s1, const C2<T> (*K0)[16],
                                            const C2<T> (*K1)[16], T* buf) {
  // real parts, then imaginary parts, through one buffer of a tile's size
  // (half the LDS of a complex buffer: one more workgroup fits per CU)
  uint32_t lt = 0;
  for (int i = 0; i < pd->tb - 4; ++i)
    if ((threadIdx.x >> i) & 1) lt ^= pd->b_tid_l[i];
  C2<T> v[16];
  const uint32_t wa = lds_bytes<T>(lt_a), rb = lds_bytes<T>(lt);
  if (active) {
#pragma unroll
    for (int j = 0; j < 16; ++j) lds_at(buf, wa, pd->j_l[j]) = o[j].re;
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j].re = lds_at(buf, rb, pd->b_j_l[j]);
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int j = 0; j < 16; ++j) lds_at(buf, wa, pd->j_l[j]) = o[j].im;
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j].im = lds_at(buf, rb, pd->b_j_l[j]);
    constexpr int NB = 1 << WB;
    if constexpr (DN) {
      if (K0) {
        if constexpr (WB == 4) {
          if (pd->tb >= 10) {  // whole waves of lanes: the matrix cores
            mfma_dense_sums<T>(v, K0, K1, s0, s1);
            return;
          }
        }
#pragma unroll
        for (int hi = 0; hi < 16; hi += NB) dense_sums<T, WB>(v + hi, K0, K1, s0, s1);
        return;
      }
    }
#pragma unroll
    for (int hi = 0; hi < 16; hi += NB) {
      wht<T, WB>(v + hi);
#pragma unroll
      for (int x = 0; x < NB; ++x) {
        const double re = (double)v[hi + x].re, im = (double)v[hi + x].im;
        const double a2 = re * re + im * im;
        s0 += w0[x] * a2;
        s1 += w1[x] * a2;
      }
    }
  }
}

// Sum of |amplitude|^2 over the 16 layout-2 slots of this thread, from a tile
// held in layout 1 (regrouped through LDS).
__device__ __forceinline__ double xpose_norms(const double* a2, uint32_t lt_a, const UnitPass* pd,
                                              bool active, double* buf) {
  if (active) {
    const uint32_t wa = lds_bytes<double>(lt_a);
#pragma unroll
    for (int j = 0; j < 16; ++j) lds_at(buf, wa, pd->j_l[j]) = a2[j];
  }
  __syncthreads();
  double s = 0.0;
  if (active) {
    uint32_t lt = 0;
    for (int i = 0; i < pd->tb - 4; ++i)
      if ((threadIdx.x >> i) & 1) lt ^= pd->b_tid_l[i];
    const uint32_t rb = lds_bytes<double>(lt);
#pragma unroll
    for (int j = 0; j < 16; ++j) s += lds_at(buf, rb, pd->b_j_l[j]);
  }
  return s;
}

// Regroup of a tile through LDS, real parts then imaginary parts through one
// buffer of a tile's size: this thread's values src of one layout (LDS slot
// lt_s ^ jl_s[j]) are written and those of another layout read into dst
// (slot lt_d ^ jl_d[j]); src and dst may be the same array.  Every thread of
// the workgroup takes part; it starts with a barrier, as the buffer may still
// be read by an earlier regroup.
template <typename T>
__device__ __forceinline__ void regroup(const C2<T>* src, uint32_t lt_s, const uint32_t* jl_s, C2<T>* dst,
                                        uint32_t lt_d, const uint32_t* jl_d, T* buf) {
  const uint32_t ws = lds_bytes<T>(lt_s), rd = lds_bytes<T>(lt_d);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) lds_at(buf, ws, jl_s[j]) = src[j].re;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) dst[j].re = lds_at(buf, rd, jl_d[j]);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) lds_at(buf, ws, jl_s[j]) = src[j].im;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) dst[j].im = lds_at(buf, rd, jl_d[j]);
}

// LDS of the X-pair code (passes with a pair only): the first B member's
// diagonals for both outcomes and the unscaled one-layer ZZ phase table.
template <typename T, bool P>
struct PairLds {
  C2<T> (*db)[16];
  C2<T>* zzu;
};
template <typename T, bool P>
__device__ __forceinline__ PairLds<T, P> pair_lds() {
  if constexpr (P) {
    __shared__ C2<T> db[2][16];
    __shared__ C2<T> zzu[kMaxEdges + 1];
    return {db, zzu};
  } else {
    return {nullptr, nullptr};
  }
}

// Entry x of a member table over 16 register-slot indices: a weight-w member
// sits on the lowest w slots, so entry x is its table at x mod 2^w divided by
// 2^(4 - w) (the unnormalised transforms over the other 4 - w slots square to
// 2^(4 - w) times the identity).
__device__ __forceinline__ double padded(const double* t, int stride, int w, int x) {
  return t[(x & ((1 << w) - 1)) * stride] * (w == 4 ? 1.0 : (w == 3 ? 0.5 : (w == 2 ? 0.25 : 0.125)));
}

// Hypothesis-tree sums of a Z chain for one weight a2 whose local indices on
// the members are x[0..lb): S[l][h] += a2 * prod_{i <= l} W_i[h_i](x_i).
template <int LB>
__device__ __forceinline__ void chain_tree(double a2, const uint32_t* x,
                                           const double (*wt)[2][16], double* acc) {
  double pre[8];
  pre[0] = a2;
#pragma unroll
  for (int l = 0; l < kChainMax; ++l) {
    if (l < LB) {
      const double w0 = wt[l][0][x[l]], w1 = wt[l][1][x[l]];
      const int off = (2 << l) - 2;
#pragma unroll
      for (int h = 0; h < (1 << l); ++h) {
        const double p0 = pre[h] * w0, p1 = pre[h] * w1;
        acc[off + h] += p0;
        acc[off + h + (1 << l)] += p1;
        if (l + 1 < kChainMax) {
          pre[h] = p0;
          pre[h + (1 << l)] = p1;
        }
      }
    }
  }
}

// Levels L0..L1-1 of the same tree: sum (l, h) goes to out[2^(l+1) - 2^(L0+1)
// + h] (the prefix products of the lower levels are formed again).
template <int L0, int L1>
__device__ __forceinline__ void chain_levels(double a2, const uint32_t* x, const double (*wt)[2][16],
                                             double* out) {
  double pre[8];
  pre[0] = a2;
#pragma unroll
  for (int l = 0; l < L1; ++l) {
    const double w0 = wt[l][0][x[l]], w1 = wt[l][1][x[l]];
    const int off = (2 << l) - (2 << L0);
#pragma unroll
    for (int h = 0; h < (1 << l); ++h) {
      const double p0 = pre[h] * w0, p1 = pre[h] * w1;
      if (l >= L0) {
        out[off + h] += p0;
        out[off + h + (1 << l)] += p1;
      }
      if (l + 1 < L1) {
        pre[h] = p0;
        pre[h + (1 << l)] = p1;
      }
    }
  }
}

// A chain of LB >= 3 members is summed at its last level only: S[h] for every
// outcome string h of all LB members (2^LB sums).  The sums of the shorter
// prefixes are its marginals, since every member's two outcome weights add up
// to one (a complete Kraus pair), and the decision forms them.  The last level
// goes in groups of 16: group G holds h = 16 G + i (members 0..3 take i's
// bits, member l >= 4 the bit (G >> (l - 4)) & 1 of G).
template <int LB>
struct ChainGroups {
  static constexpr int value = LB <= 4 ? 1 : (1 << (LB - 4));
};
// Products of the first min(LB, 4) members' weights for every outcome string
// of them, times a2.
template <int LB>
__device__ __forceinline__ void chain_prefix(double a2, const uint32_t* x, const double (*wt)[2][16],
                                             double* p) {
  constexpr int LO = LB < 4 ? LB : 4;
  p[0] = a2;
#pragma unroll
  for (int l = 0; l < LO; ++l) {
    const double w0 = wt[l][0][x[l]], w1 = wt[l][1][x[l]];
#pragma unroll
    for (int h = 0; h < (1 << l); ++h) {
      p[h + (1 << l)] = p[h] * w1;
      p[h] *= w0;
    }
  }
}
// The factor of group G: the weights of members 4.. for G's outcome bits.
template <int LB, int G>
__device__ __forceinline__ double chain_group_factor(const uint32_t* x, const double (*wt)[2][16]) {
  double f = 1.0;
#pragma unroll
  for (int l = 4; l < LB; ++l) f *= wt[l][(G >> (l - 4)) & 1][x[l]];
  return f;
}

// One pass over the register: apply unit A with its decided outcomes (or
// write logical |0> when A is U_INIT), each member's ZZ layer and the
// renormalisation 1/sqrt(S_m); accumulate the sums of unit B from the values
// still on chip.  B an X check: S_0, S_1 over the check's Hadamard basis.
// B a chain of L Z checks: S[l][h] for l < L and every outcome string h of
// members 0..l (bit i = outcome of member i), at index 2^(l+1) - 2 + h.
// Tiles are taken grid-stride; `reverse` walks them backwards (consecutive
// passes alternate, so a pass starts on the lines its predecessor wrote
// last).  Workgroup 0 records the frame after A in dec_b.
// AP: weight of an X check A, or the length of a Z chain A (BP likewise).
// DN: the instantiation that also handles dense Kraus pairs (kept apart so
// that the dense code does not weigh on the other passes' registers).
// Occupancy of a pass kernel: passes other than the dense ones and those
// summing a Z chain amplitude by amplitude are held to 168 registers, i.e.
// three waves per SIMD (measured on d=5: complex128 X-check passes
// 200 -> 186 us); those keep the registers they need.
// BM0: the instantiation that sums a Z chain B amplitude by amplitude (bmode
// 0: registers too small for four slot bits outside the chain's qubits, d <=
// 3); the others sum it once per thread (bmode 1, 2), which keeps a chain of
// four within three waves per SIMD in complex128.  Passes summing an X pair
// hold two copies of the tile (the first member's transform and one branch)
// and keep the registers they need.
template <typename T, int BK, int BP, bool DN, bool BM0>
struct UpassWaves {
  static constexpr int value = (!DN && !BM0 && BK != U_XP) ? 3 : 1;
};

// Speculative passes (SP = 1: prediction, SP = 2: redo): the register they
// write, the unit instance's control record, the predicted outcome of each
// member (prediction pass), a counter of the redos that ran; lockstep
// launches: per trajectory slot the register moves by the slot stride of st,
// the record by ctl_stride, the predictions by pred_stride.
struct SpecArgs {
  void* out;
  SpecCtl* ctl;
  const uint8_t* pred;
  int* redos;
  size_t ctl_stride, pred_stride;
};

template <typename T, int AK, int AP, int BK, int BP, bool DN, bool BM0, int SP>
__device__ __forceinline__ void upass_body(
    T* __restrict__ st, const UnitPass* __restrict__ pd, const JobConst* __restrict__ jc,
    const BlockRT* __restrict__ rta, const BlockRT* __restrict__ rtb,
    const Decision* __restrict__ dec_a, Decision* __restrict__ dec_b,
    double* __restrict__ partials, int reverse, SlotStrides ss,
    const BlockDense* __restrict__ dna, const BlockDense* __restrict__ dnb, SpecArgs sa) {
  // speculative unit: A (an X check or pair, summed along its applied
  // outcomes), or B (a Z chain after the pending renormalisation)
  constexpr bool kSpecA = SP != 0 && (AK == U_X || AK == U_XP);
  constexpr bool kSpecB = SP != 0 && BK == U_Z;
  static_assert(SP == 0 || (kSpecA && BK == U_NONE) || (kSpecB && AK == U_SC), "speculative unit kinds");
  // trajectory slot (lockstep launches): walked backwards with the tiles, so
  // that a pass starts on the registers its predecessor wrote last
  const size_t slot = reverse ? gridDim.y - 1 - blockIdx.y : blockIdx.y;
  int sm = 0;  // outcome bits applied to the speculative unit
  if constexpr (SP == 2) {
    SpecCtl* const ctl = sa.ctl + slot * sa.ctl_stride;
    if (!ctl->run) return;  // nothing to redo
    sm = ctl->m;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(sa.redos, 1);
  } else if constexpr (SP == 1) {
    constexpr int kLen = kSpecA ? (AK == U_XP ? 2 : 1) : BP;
    const uint8_t* const pred = sa.pred + slot * sa.pred_stride;
#pragma unroll
    for (int l = 0; l < kLen; ++l) sm |= (pred[l] & 1) << l;
    // (byte loads go through the vector unit: the bits are uniform, and the
    // tables they select must stay scalar loads)
    sm = __builtin_amdgcn_readfirstlane(sm);
    if (blockIdx.x == 0 && threadIdx.x == 0) sa.ctl[slot * sa.ctl_stride] = SpecCtl{sm, 0, 1, 0};
  }
  st += slot * ss.st;
  constexpr uint32_t kAmp = 2 * sizeof(T);  // bytes per amplitude
  const RegBuf<T> reg(st, (uint32_t)(kAmp << (pd->tb + pd->n_outer)));
  // speculative passes write the other register buffer (the redo reads the
  // pass's input again)
  const RegBuf<T> regw(SP != 0 ? static_cast<T*>(sa.out) + slot * ss.st : st,
                       (uint32_t)(kAmp << (pd->tb + pd->n_outer)));
  if (rta) rta += slot * ss.rt;
  if (rtb) rtb += slot * ss.rt;
  if (dna) dna += slot * ss.rt;
  if (dnb) dnb += slot * ss.rt;
  if (dec_a) dec_a += slot * ss.dec;
  dec_b += slot * ss.dec;
  const int n_tiles = 1 << pd->n_outer;
  // one partial sum per workgroup (over its tiles, in tile order): [acc][gridDim.x]
  partials += slot * kChainAcc * gridDim.x;
  __shared__ C2<T> da[kChainMax][16];
  __shared__ double wt[kChainMax][2][16];
  // phase table of A's ZZ layers and the per-wave sums of B, sized for the
  // units of this instantiation
  constexpr int kLayers = AK == U_Z ? AP : (kSpecB ? BP : 1);
  constexpr int kSums = kSpecA ? (AK == U_XP ? 4 : 2) : (BK == U_Z ? unit_sums(BP) : (BK == U_XP ? 6 : 2));
  __shared__ C2<T> zzt[kLayers * kMaxEdges + 1];
  __shared__ double red[kSums][4];
  const int tid = threadIdx.x;
  const int tb = pd->tb;
  const int nt = 1 << (tb - 4);
  // passes with an X pair run whole tiles of 2^12 amplitudes (every thread
  // active; the regroups between the members synchronise the workgroup)
  constexpr bool kPair = AK == U_XP || BK == U_XP;
  const bool active = kPair || tid < nt;
  constexpr int WA = AK == U_X ? AP : 0;
  constexpr int WB = BK == U_X ? BP : 0;
  constexpr int la = AK == U_Z ? AP : (AK == U_X ? 1 : (AK == U_XP ? 2 : 0));
  constexpr int lb = BK == U_Z ? BP : (BK == U_X ? 1 : (BK == U_XP ? 2 : 0));
  constexpr int LB = lb;
  // one LDS buffer of a tile's size for every regroup of the pass
  using XB = std::conditional_t<BK == U_Z, double, T>;
  __shared__ XB xbuf[1 << kTileMax];
  T* const tbuf = reinterpret_cast<T*>(xbuf);
  const PairLds<T, kPair> pl = pair_lds<T, kPair>();

  // frame and decided outcomes of A; frame-dependent offsets
  uint32_t phi = 0;
  int mbits = 0;
  double scale = 1.0;
  if constexpr (AK != U_INIT) {
    phi = dec_a->phi;
    mbits = kSpecA ? sm : dec_a->m;
    scale = 1.0 / sqrt(dec_a->Sm);
  }
  uint32_t M[kChainMax];   // logical-index masks of A's ZZ layers
  uint32_t ca[kChainMax];  // member-local input offsets
#pragma unroll
  for (int i = 0; i < kChainMax; ++i) {
    M[i] = phi;
    ca[i] = 0;
  }
  uint32_t phi_new = phi;
  uint32_t Fa = 0, Fa1 = 0;
  if constexpr (AK == U_X) {
    Fa = rta->F;
    if (__popc(gather_loc(phi, pd->aq[0], WA) & Fa) & 1) scale = -scale;
  }
  if constexpr (AK == U_XP) {  // both members' frame signs
    Fa = rta[0].F;
    Fa1 = rta[1].F;
    if ((__popc(gather_loc(phi, pd->aq[0], pd->aw[0]) & Fa) + __popc(gather_loc(phi, pd->aq[1], pd->aw[1]) & Fa1)) & 1)
      scale = -scale;
  }
  if constexpr (AK == U_Z) {
    uint32_t G = 0;
#pragma unroll
    for (int i = 0; i < kChainMax; ++i)
      if (i < la) {
        ca[i] = gather_loc(phi ^ G, pd->aq[i], pd->aw[i]);
        G ^= scatter_loc(rta[i].F, pd->aq[i], pd->aw[i]);
        M[i] = phi ^ G;
      }
    phi_new = phi ^ G;
  }
  uint32_t cb[kChainMax];
  uint32_t Mb[kChainMax];  // frames of a speculative chain B's ZZ layers
#pragma unroll
  for (int i = 0; i < kChainMax; ++i) cb[i] = Mb[i] = 0;
  uint32_t Gb = 0;
  if constexpr (BK == U_Z) {
#pragma unroll
    for (int i = 0; i < kChainMax; ++i)
      if (i < lb) {
        cb[i] = gather_loc(phi_new ^ Gb, pd->bq[i], pd->bw[i]);
        Gb ^= scatter_loc(rtb[i].F, pd->bq[i], pd->bw[i]);
        Mb[i] = phi_new ^ Gb;
      }
  }
  // frame after this pass's writes (a speculative chain B is applied here)
  if (blockIdx.x == 0 && tid == 0) dec_b->phi = kSpecB ? phi_new ^ Gb : phi_new;

  // tables (the workgroup may have only 64 threads)
  // an X check A's decided diagonal: in LDS for the lane-mixed layout, and
  // in complex64 (converted once per workgroup rather than per tile)
  // (speculative passes too: their second register's resource and the
  // control arguments leave no scalar registers for the table)
  if constexpr (AK == U_X) {
    if ((pd->amix || sizeof(T) == 4 || kSpecA) && tid < 16)
      da[0][tid] = C2<T>{(T)rta->D[mbits][tid][0], (T)rta->D[mbits][tid][1]};
  }
  if constexpr (AK == U_XP) {  // members' decided diagonals over 16 register slots
    if (tid < 32) {
      const int i = tid >> 4, x = tid & 15, m = (mbits >> i) & 1, w = pd->aw[i];
      if (i == 0 && pd->amix)  // first member partly on lanes: its own local index
        da[0][x] = C2<T>{(T)rta[0].D[m][x][0], (T)rta[0].D[m][x][1]};
      else
        da[i][x] = C2<T>{(T)padded(&rta[i].D[m][0][0], 2, w, x), (T)padded(&rta[i].D[m][0][1], 2, w, x)};
    }
  }
  if constexpr (BK == U_XP) {  // both members' weights, the first member's diagonals
    if (tid < 64) {
      const int i = tid >> 5, m = (tid >> 4) & 1, x = tid & 15;
      wt[i][m][x] = padded(&rtb[i].W[m][0], 1, pd->bw[i], x);
    }
    if (tid < 32) {
      const int m = tid >> 4, x = tid & 15, w = pd->bw[0];
      pl.db[m][x] = C2<T>{(T)padded(&rtb[0].D[m][0][0], 2, w, x), (T)padded(&rtb[0].D[m][0][1], 2, w, x)};
    }
  }
  if constexpr (kPair) {  // one unscaled ZZ layer (inside a pair)
    if (jc->use_zz)
      for (int k = tid; k <= jc->n_edges; k += blockDim.x)
        pl.zzu[k] = C2<T>{(T)jc->zzl[0][2 * k], (T)jc->zzl[0][2 * k + 1]};
  }
  // dense Kraus pairs in the register's frame (passes with a dense unit)
  C2<T>(*kdn)[16][16] = dense_lds<T, DN>();
  if constexpr (DN) {
    if (pd->adense) {
      const uint32_t fa = gather_loc(phi, pd->aq[0], WA);
      for (int k = tid; k < 256; k += blockDim.x) {
        const int r = k >> 4, c = k & 15;
        kdn[0][r][c] = C2<T>{(T)dna->K[mbits & 1][r ^ fa][c ^ fa][0], (T)dna->K[mbits & 1][r ^ fa][c ^ fa][1]};
      }
    }
    if (pd->bdense) {
      const uint32_t fb = gather_loc(phi_new, pd->bq[0], WB);
      for (int k = tid; k < 512; k += blockDim.x) {
        const int m = k >> 8, r = (k >> 4) & 15, c = k & 15;
        kdn[1 + m][r][c] = C2<T>{(T)dnb->K[m][r ^ fb][c ^ fb][0], (T)dnb->K[m][r ^ fb][c ^ fb][1]};
      }
    }
  }
  if constexpr (AK == U_Z) {
    for (int k = tid; k < kChainMax * 16; k += blockDim.x) {
      const int i = k >> 4, x = k & 15;
      if (i < la) {
        const int m = (mbits >> i) & 1;
        da[i][x] = C2<T>{(T)rta[i].D[m][x][0], (T)rta[i].D[m][x][1]};
      }
    }
  }
  if constexpr (BK == U_Z) {
    for (int k = tid; k < kChainMax * 32; k += blockDim.x) {
      const int i = k >> 5, m = (k >> 4) & 1, x = k & 15;
      if (i < lb) wt[i][m][x] = rtb[i].W[m][x];
    }
  }
  if constexpr (BK == U_X) {
    if (tid < 32) wt[0][tid >> 4][tid & 15] = rtb->W[tid >> 4][tid & 15];
  }
  if constexpr (kSpecA && AK == U_X) {  // the check's weights over its local index
    if (tid < 32) wt[0][tid >> 4][tid & 15] = rta->W[tid >> 4][tid & 15];
  }
  if constexpr (kSpecA && AK == U_XP) {  // members' weights as their diagonals are laid out
    if (tid < 64) {
      const int i = tid >> 5, m = (tid >> 4) & 1, x = tid & 15;
      wt[i][m][x] = (i == 0 && pd->amix) ? rta[0].W[m][x] : padded(&rta[i].W[m][0], 1, pd->aw[i], x);
    }
  }
  if constexpr (kSpecB) {  // the chain's diagonals for its applied outcomes
    for (int k = tid; k < kChainMax * 16; k += blockDim.x) {
      const int i = k >> 4, x = k & 15;
      if (i < lb) {
        const int m = (sm >> i) & 1;
        da[i][x] = C2<T>{(T)rtb[i].D[m][x][0], (T)rtb[i].D[m][x][1]};
      }
    }
    if (jc->use_zz)  // B's layers, unscaled (the renormalisation comes first)
      for (int k = tid; k <= lb * jc->n_edges; k += blockDim.x)
        zzt[k] = C2<T>{(T)jc->zzl[lb - 1][2 * k], (T)jc->zzl[lb - 1][2 * k + 1]};
  }
  constexpr int nl = AK == U_Z ? la : 1;
  const int use_zz = (AK != U_INIT && AK != U_SC) && jc->use_zz;
  // the phase table carries the renormalisation (and the sign of an X check
  // A's frame), formed in FP64: one complex product per amplitude does both
  if (use_zz)
    for (int k = tid; k <= nl * jc->n_edges; k += blockDim.x)
      zzt[k] = C2<T>{(T)(jc->zzl[nl - 1][2 * k] * scale), (T)(jc->zzl[nl - 1][2 * k + 1] * scale)};
  __syncthreads();

  const int d = jc->d;
  const uint32_t hm = jc->hmask, vm = jc->vmask;
  uint32_t eM[kChainMax], vM[kChainMax];
  bool zz_same = true;
#pragma unroll
  for (int i = 0; i < kChainMax; ++i) {
    eM[i] = M[i] ^ (M[i] >> 1);
    vM[i] = M[i] ^ (M[i] >> d);
    if (i > 0 && i < nl && M[i] != M[0]) zz_same = false;
  }

  uint32_t gt = 0, lt = 0;
  for (int i = 0; i < tb - 4; ++i)
    if ((tid >> i) & 1) {
      gt |= pd->tid_g[i];
      lt ^= pd->tid_l[i];
    }
  // X pairs: this thread's part of layouts 2, p[0] and p[1]; the ZZ layer
  // inside a pair (frame after A for a B pair)
  uint32_t lt2 = 0, gt2 = 0, ltp0 = 0, ltp1 = 0;
  if constexpr (kPair) {
    for (int i = 0; i < tb - 4; ++i)
      if ((tid >> i) & 1) {
        lt2 ^= pd->b_tid_l[i];
        gt2 |= pd->b_tid_g[i];
        ltp0 ^= pd->p_tid_l[0][i];
        ltp1 ^= pd->p_tid_l[1][i];
      }
  }
  const int zz_on = jc->use_zz;
  const uint32_t eMb = phi_new ^ (phi_new >> 1), vMb = phi_new ^ (phi_new >> d);
  uint32_t Fb0 = 0;
  if constexpr (BK == U_XP) Fb0 = rtb[0].F;
  // one unscaled ZZ layer (frame masks eMx, vMx) on 16 values whose global
  // indices are gbase | jg[j] (edge maps split as in `finish` below)
  auto zz_layer = [&](C2<T>* w, uint32_t gbase, const uint32_t* jg, uint32_t eMx, uint32_t vMx) {
    const uint32_t Et = ((gbase ^ (gbase >> 1)) ^ eMx) & hm, Vt = ((gbase ^ (gbase >> d)) ^ vMx) & vm;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t x = jg[j];
      const int K = __popc(Et ^ ((x ^ (x >> 1)) & hm)) + __popc(Vt ^ ((x ^ (x >> d)) & vm));
      const C2<T> z = pl.zzu[K];
      w[j] = mulc(w[j], z.re, z.im);
    }
  };
  // Kraus operator of an X check on the register slots: transform, diagonal
  // (16-slot table in LDS), transform, frame signs
  // (a speculative A: the member's sums over the transformed values first,
  // weights ws)
  auto x_slots = [&](C2<T>* w, const C2<T>* dg, uint32_t F, const double (*ws)[16], double* sp) {
    wht<T, 4>(w);
    if constexpr (kSpecA) {
      // weights read per tile (an opaque offset keeps them out of registers
      // across the tile loop)
      const uint32_t wz = lds_bytes<double>(0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double re = (double)w[j].re, im = (double)w[j].im;
        const double a2 = re * re + im * im;
        sp[0] += lds_at(const_cast<double*>(ws[0]), wz, j) * a2;
        sp[1] += lds_at(const_cast<double*>(ws[1]), wz, j) * a2;
        if ((j & 3) == 3) asm volatile("" : "+v"(sp[0]), "+v"(sp[1]) : : "memory");
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) w[j] = mulc(w[j], dg[j].re, dg[j].im);
    wht<T, 4>(w);
    if (F) {
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (__popc((uint32_t)j & F) & 1) w[j] = {-w[j].re, -w[j].im};
    }
  };
  // a speculative X check A partly on the lanes: its sums over the values
  // after the first transform (local index xl ^ a_jx[j])
  // (in groups of four values whose products are added at once: neither the
  // weights nor the squared magnitudes stay live across the rest of the tile)
  auto spec_mixed_sums = [&](const C2<T>* w, uint32_t xl, double& s0, double& s1) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t x = xl ^ pd->a_jx[j];
      const double re = (double)w[j].re, im = (double)w[j].im;
      const double a2 = re * re + im * im;
      s0 += wt[0][0][x] * a2;
      s1 += wt[0][1][x] * a2;
      if ((j & 3) == 3) asm volatile("" : "+v"(s0), "+v"(s1) : : "memory");
    }
  };
  // grid-stride over the tiles (one tile per workgroup when the grid covers
  // them all); the tables above are loaded once per workgroup, the sums of B
  // accumulate over the workgroup's tiles
  // Z chains of three to six checks: the tile's last-level sums (8 to 64) are
  // formed and reduced across the wave one 16-value group at a time; each
  // lane keeps one running total per group (lane l: sum (l >> 2) & 15 of the
  // group), so neither the accumulators of every sum nor a whole tree stays
  // live
  constexpr bool kWaveAcc = BK == U_Z && LB >= 3;
  constexpr int kAcc = kWaveAcc ? ChainGroups<LB>::value : 32;
  double acc[kAcc];
#pragma unroll
  for (int a = 0; a < kAcc; ++a) acc[a] = 0.0;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
  const int wg = reverse ? n_tiles - 1 - tile : tile;
  uint32_t base = 0;
  for (int i = 0; i < pd->n_outer; ++i)
    if ((wg >> i) & 1) base |= pd->outer_bit[i];
  const uint32_t gb = base | gt;
  // the LDS slot offsets of the regroups are formed per tile, not kept in
  // registers over the tile loop
  if constexpr (kPair) asm volatile("" : "+v"(lt), "+v"(ltp0), "+v"(ltp1), "+v"(lt2));

  C2<T> o[16];
  if (active) {
    if constexpr (AK == U_INIT) {
      // logical |0>: g is in the X-stabilizer orbit of 0 iff its reduction
      // against the echelon basis vanishes; logical |+>: g has even parity on
      // every Z check.  Both tests are linear in g, so they split into the
      // thread's part and the slot's part.
      const T amp = (T)jc->amp0;
      auto reduce = [&](uint32_t x) {
        if (jc->init_plus) {
          uint32_t syn = 0;
          for (int i = 0; i < jc->n_zc; ++i) syn |= (uint32_t)(__popc(x & jc->zc_mask[i]) & 1) << i;
          return syn;
        }
        for (int i = 0; i < jc->n_x; ++i)
          if (x & jc->span_piv[i]) x ^= jc->span_vec[i];
        return x;
      };
      const uint32_t rb = reduce(gb);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        o[j] = {(rb ^ reduce(pd->j_g[j])) == 0 ? amp : (T)0, (T)0};
        reg.st(gb * kAmp, pd->j_g[j] * kAmp, o[j]);
      }
    } else {
      C2<T> v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = reg.ld(gb * kAmp, pd->j_g[j] * kAmp);
      if constexpr (AK == U_X) {
        if (DN && pd->adense) {  // dense Kraus pair (crosstalk inside the check)
          if constexpr (DN) {
            constexpr int NA = 1 << WA;
            if (WA == 4 && tb >= 10) {  // whole waves of lanes: the matrix cores
              mfma_dense_apply<T>(v, kdn[0]);
            } else {
#pragma unroll
              for (int hi = 0; hi < 16; hi += NA) dense_apply<T, WA>(v + hi, kdn[0]);
            }
          }
        } else if (pd->amix) {
          uint32_t xl = 0;  // A's local index bits carried by this thread's lanes
          for (int i = 0; i < 4; ++i)
            if ((tid >> i) & 1) xl |= pd->a_tx[i];
          wht_mixed(v, pd->amix_r, pd->amix_lanes, tid);
          if constexpr (kSpecA) spec_mixed_sums(v, xl, acc[0], acc[1]);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const C2<T> e = da[0][xl ^ pd->a_jx[j]];
            v[j] = mulc(v[j], e.re, e.im);
          }
          wht_mixed(v, pd->amix_r, pd->amix_lanes, tid);
          if (Fa) {  // frame signs (a Z-type Pauli on the check's qubits; rare)
#pragma unroll
            for (int j = 0; j < 16; ++j)
              if (__popc((xl ^ pd->a_jx[j]) & Fa) & 1) v[j] = {-v[j].re, -v[j].im};
          }
        } else {
          const double* D = &rta->D[mbits][0][0];
          constexpr int NA = 1 << WA;
#pragma unroll
          for (int hi = 0; hi < 16; hi += NA) {
            wht<T, WA>(v + hi);
            if constexpr (kSpecA) {
              const uint32_t wz = lds_bytes<double>(0);
#pragma unroll
              for (int x = 0; x < NA; ++x) {
                const double re = (double)v[hi + x].re, im = (double)v[hi + x].im;
                const double a2 = re * re + im * im;
                acc[0] += lds_at(&wt[0][0][0], wz, x) * a2;
                acc[1] += lds_at(&wt[0][1][0], wz, x) * a2;
                if ((x & 3) == 3) asm volatile("" : "+v"(acc[0]), "+v"(acc[1]) : : "memory");
              }
            }
#pragma unroll
            for (int x = 0; x < NA; ++x) {
              if constexpr (sizeof(T) == 4 || kSpecA) {
                const C2<T> e = da[0][x];
                v[hi + x] = mulc(v[hi + x], e.re, e.im);
              } else {
                v[hi + x] = mulc(v[hi + x], D[2 * x], D[2 * x + 1]);
              }
            }
            wht<T, WA>(v + hi);
            if (Fa) {
#pragma unroll
              for (int x = 0; x < NA; ++x)
                if (__popc((uint32_t)x & Fa) & 1) v[hi + x] = {-v[hi + x].re, -v[hi + x].im};
            }
          }
        }
      } else if constexpr (AK == U_XP) {
        // first member in layout 1: its qubits on register slots, or partly
        // on the lowest lanes (then its own local index)
        if (pd->amix) {
          uint32_t xl = 0;
          for (int i = 0; i < 4; ++i)
            if ((tid >> i) & 1) xl |= pd->a_tx[i];
          wht_mixed(v, pd->amix_r, pd->amix_lanes, tid);
          if constexpr (kSpecA) spec_mixed_sums(v, xl, acc[0], acc[1]);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const C2<T> e = da[0][xl ^ pd->a_jx[j]];
            v[j] = mulc(v[j], e.re, e.im);
          }
          wht_mixed(v, pd->amix_r, pd->amix_lanes, tid);
          if (Fa) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
              if (__popc((xl ^ pd->a_jx[j]) & Fa) & 1) v[j] = {-v[j].re, -v[j].im};
          }
        } else if constexpr (kSpecA) {
          x_slots(v, da[0], Fa, wt[0], &acc[0]);
        } else {
          x_slots(v, da[0], Fa, wt[0], nullptr);
        }
        if (zz_on) zz_layer(v, gb, pd->j_g, eM[0], vM[0]);
        // second member on the register slots of layout p[0], then back
        regroup<T>(v, lt, pd->j_l, v, ltp0, pd->p_j_l[0], tbuf);
        if constexpr (kSpecA)
          x_slots(v, da[1], Fa1, wt[1], &acc[2]);
        else
          x_slots(v, da[1], Fa1, wt[1], nullptr);
        if (!pd->pstore) regroup<T>(v, ltp0, pd->p_j_l[0], v, lt, pd->j_l, tbuf);
      } else if constexpr (AK == U_Z) {
        uint32_t oa[kChainMax];
#pragma unroll
        for (int i = 0; i < kChainMax; ++i)
          oa[i] = i < la ? gather_loc(gb, pd->aq[i], pd->aw[i]) ^ ca[i] : 0u;
        if (pd->amode) {  // the chain's factor is shared by the thread's 16 amplitudes
          C2<T> f = da[0][oa[0]];
#pragma unroll
          for (int i = 1; i < kChainMax; ++i)
            if (i < la) {
              const C2<T> e = da[i][oa[i]];
              f = mulc(f, e.re, e.im);
            }
#pragma unroll
          for (int j = 0; j < 16; ++j) v[j] = mulc(v[j], f.re, f.im);
        } else {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            C2<T> f = da[0][oa[0] ^ pd->a_j_loc[0][j]];
#pragma unroll
            for (int i = 1; i < kChainMax; ++i)
              if (i < la) {
                const C2<T> e = da[i][oa[i] ^ pd->a_j_loc[i][j]];
                f = mulc(f, e.re, e.im);
              }
            v[j] = mulc(v[j], f.re, f.im);
          }
        }
      }
      // ZZ phase index: anti-aligned neighbour pairs summed over A's layers
      // (one popcount pair when every layer sees the same frame).  The edge
      // maps g ^ (g >> 1) and g ^ (g >> d) are linear over XOR and a slot's
      // bits are disjoint from the thread's, so the thread's part of each
      // masked map is formed once per tile and a slot adds its own part.
      // (an X pair A stored from layout p[0]: that layout's base and slots)
      uint32_t fgb = gb;
      const uint32_t* fjg = pd->j_g;
      if constexpr (AK == U_XP) {
        if (pd->pstore) {
          fgb = base;
          for (int i = 0; i < tb - 4; ++i)
            if ((tid >> i) & 1) fgb |= pd->p_tid_g[0][i];
          fjg = pd->p_j_g[0];
        }
      }
      auto finish = [&](auto layers) {
        constexpr int NZ = decltype(layers)::value;
        constexpr int NE = NZ == 0 ? 1 : NZ;
        uint32_t Et[NE], Vt[NE];
        const uint32_t eb = fgb ^ (fgb >> 1), wb = fgb ^ (fgb >> d);
#pragma unroll
        for (int i = 0; i < NE; ++i) {
          Et[i] = (eb ^ eM[i]) & hm;
          Vt[i] = (wb ^ vM[i]) & vm;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const uint32_t jg = fjg[j];
          C2<T> r = v[j];
          if (use_zz) {
            const uint32_t je = (jg ^ (jg >> 1)) & hm, jw = (jg ^ (jg >> d)) & vm;
            int K = 0;
#pragma unroll
            for (int i = 0; i < NE; ++i) K += __popc(Et[i] ^ je) + __popc(Vt[i] ^ jw);
            if constexpr (NZ == 0) K *= nl;
            const C2<T> z = zzt[K];
            r = mulc(r, z.re, z.im);
          } else if constexpr (sizeof(T) == 8) {
            r.re *= scale;
            r.im *= scale;
          } else {
            r.re = (T)((double)r.re * scale);
            r.im = (T)((double)r.im * scale);
          }
          if constexpr (!kSpecB) regw.st(fgb * kAmp, jg * kAmp, r);
          o[j] = r;
        }
      };
      if (nl == 1 || zz_same)
        finish(std::integral_constant<int, 0>{});
      else
        finish(std::integral_constant<int, nl>{});
    }
  }
  if constexpr (BK == U_X) {
    const bool bd = DN && pd->bdense;
    const C2<T>(*K0p)[16] = nullptr;
    const C2<T>(*K1p)[16] = nullptr;
    if constexpr (DN) {
      if (bd) {
        K0p = kdn[1];
        K1p = kdn[2];
      }
    }
    if (pd->bmode == 2) {
      xpose_xsums<T, WB, DN>(o, lt, pd, wt[0][0], wt[0][1], active, acc[0], acc[1], K0p, K1p, tbuf);
    } else if (active && bd) {
      if constexpr (DN) {
        constexpr int NB = 1 << WB;
        if (WB == 4 && tb >= 10) {  // whole waves of lanes: the matrix cores
          mfma_dense_sums<T>(o, kdn[1], kdn[2], acc[0], acc[1]);
        } else {
#pragma unroll
          for (int hi = 0; hi < 16; hi += NB) dense_sums<T, WB>(o + hi, kdn[1], kdn[2], acc[0], acc[1]);
        }
      }
    } else if (active) {
      constexpr int NB = 1 << WB;
#pragma unroll
      for (int hi = 0; hi < 16; hi += NB) {
        C2<T> v[NB];
#pragma unroll
        for (int x = 0; x < NB; ++x) v[x] = o[hi + x];
        wht<T, WB>(v);
#pragma unroll
        for (int x = 0; x < NB; ++x) {
          const double re = (double)v[x].re, im = (double)v[x].im;
          const double a2 = re * re + im * im;
          acc[0] += wt[0][0][x] * a2;
          acc[1] += wt[0][1][x] * a2;
        }
      }
    }
  }
  if constexpr (BK == U_Z) {
    double a2[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double re = (double)o[j].re, im = (double)o[j].im;
      a2[j] = active ? re * re + im * im : 0.0;
    }
    // the chain's local indices of each amplitude (bmode 0), or of the
    // thread's 16 amplitudes together with their norm (bmode 1, 2)
    double s = 0.0;
    uint32_t g2 = gb;
    if constexpr (!BM0) {
      if (pd->bmode == 1) {
#pragma unroll
        for (int j = 0; j < 16; ++j) s += a2[j];
      } else {
        s = xpose_norms(a2, lt, pd, active, reinterpret_cast<double*>(xbuf));
        g2 = base;
        for (int i = 0; i < tb - 4; ++i)
          if ((tid >> i) & 1) g2 |= pd->b_tid_g[i];
      }
    }
    uint32_t ob[kChainMax];
#pragma unroll
    for (int i = 0; i < kChainMax; ++i) ob[i] = i < lb ? gather_loc(g2, pd->bq[i], pd->bw[i]) ^ cb[i] : 0u;
    // sums of levels L0..L1-1 into t
    auto tree = [&](auto l0, auto l1, double* t) {
      constexpr int L0 = decltype(l0)::value, L1 = decltype(l1)::value;
      if (!active) return;
      if constexpr (BM0) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          uint32_t x[kChainMax];
#pragma unroll
          for (int i = 0; i < kChainMax; ++i) x[i] = ob[i] ^ pd->b_j_loc[i][j];
          chain_levels<L0, L1>(a2[j], x, wt, t);
        }
      } else {
        chain_levels<L0, L1>(s, ob, wt, t);
      }
    };
    if constexpr (kWaveAcc) {
      constexpr int kGroups = ChainGroups<LB>::value;
      double t[16];
      if constexpr (BM0) {
        // amplitude by amplitude: each group's products formed anew
        auto one = [&](auto gv) {
          constexpr int G = decltype(gv)::value;
#pragma unroll
          for (int a = 0; a < 16; ++a) t[a] = 0.0;
          if (active) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
              uint32_t x[kChainMax];
#pragma unroll
              for (int i = 0; i < kChainMax; ++i) x[i] = ob[i] ^ pd->b_j_loc[i][j];
              double p[16];
              chain_prefix<LB>(a2[j], x, wt, p);
              const double f = chain_group_factor<LB, G>(x, wt);
#pragma unroll
              for (int a = 0; a < (LB < 4 ? (1 << LB) : 16); ++a) t[a] += p[a] * f;
            }
          }
          acc[G] += wave_reduce16(t);
        };
        one(std::integral_constant<int, 0>{});
        if constexpr (kGroups > 1) one(std::integral_constant<int, 1>{});
        if constexpr (kGroups > 2) {
          one(std::integral_constant<int, 2>{});
          one(std::integral_constant<int, 3>{});
        }
        static_assert(kGroups <= 4, "chains of at most six checks");
      } else {
        // once per thread: the first members' products shared by the groups
        double p[16];
#pragma unroll
        for (int a = 0; a < 16; ++a) p[a] = 0.0;
        if (active) chain_prefix<LB>(s, ob, wt, p);
        auto one = [&](auto gv) {
          constexpr int G = decltype(gv)::value;
          const double f = active ? chain_group_factor<LB, G>(ob, wt) : 0.0;
#pragma unroll
          for (int a = 0; a < 16; ++a) t[a] = p[a] * f;
          acc[G] += wave_reduce16(t);
        };
        one(std::integral_constant<int, 0>{});
        if constexpr (kGroups > 1) one(std::integral_constant<int, 1>{});
        if constexpr (kGroups > 2) {
          one(std::integral_constant<int, 2>{});
          one(std::integral_constant<int, 3>{});
        }
        static_assert(kGroups <= 4, "chains of at most six checks");
      }
    } else {
      tree(std::integral_constant<int, 0>{}, std::integral_constant<int, LB>{}, acc);
    }
  }
  if constexpr (kSpecB) {
    // the speculative chain applied after its sums: its diagonals for the
    // applied outcomes (layout 1, the frame offsets of the sums), then one ZZ
    // layer per member in the frame after that member, then the store
    if (active) {
      uint32_t o1[kChainMax];
#pragma unroll
      for (int i = 0; i < kChainMax; ++i) o1[i] = i < lb ? gather_loc(gb, pd->bq[i], pd->bw[i]) ^ cb[i] : 0u;
      if (pd->bmode == 1) {  // no chain qubit on the register slots
        C2<T> f = da[0][o1[0]];
#pragma unroll
        for (int i = 1; i < kChainMax; ++i)
          if (i < lb) {
            const C2<T> e = da[i][o1[i]];
            f = mulc(f, e.re, e.im);
          }
#pragma unroll
        for (int j = 0; j < 16; ++j) o[j] = mulc(o[j], f.re, f.im);
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          C2<T> f = da[0][o1[0] ^ pd->b_j_loc[0][j]];
#pragma unroll
          for (int i = 1; i < kChainMax; ++i)
            if (i < lb) {
              const C2<T> e = da[i][o1[i] ^ pd->b_j_loc[i][j]];
              f = mulc(f, e.re, e.im);
            }
          o[j] = mulc(o[j], f.re, f.im);
        }
      }
      bool same = true;
#pragma unroll
      for (int i = 1; i < kChainMax; ++i)
        if (i < lb && Mb[i] != Mb[0]) same = false;
      const uint32_t eb = gb ^ (gb >> 1), wb = gb ^ (gb >> d);
      const int nz = same ? 1 : lb;  // layers with distinct frames
      uint32_t Et[kChainMax], Vt[kChainMax];
#pragma unroll
      for (int i = 0; i < kChainMax; ++i) {
        Et[i] = (eb ^ Mb[i] ^ (Mb[i] >> 1)) & hm;
        Vt[i] = (wb ^ Mb[i] ^ (Mb[i] >> d)) & vm;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t jg = pd->j_g[j];
        C2<T> r = o[j];
        if (zz_on) {
          const uint32_t je = (jg ^ (jg >> 1)) & hm, jw = (jg ^ (jg >> d)) & vm;
          int K = 0;
#pragma unroll
          for (int i = 0; i < kChainMax; ++i)
            if (i < nz) K += __popc(Et[i] ^ je) + __popc(Vt[i] ^ jw);
          if (same) K *= lb;
          const C2<T> z = zzt[K];
          r = mulc(r, z.re, z.im);
        }
        regw.st(gb * kAmp, jg * kAmp, r);
      }
    }
  }
  if constexpr (BK == U_XP) {
    // first member on the register slots of layout 2: its sums; then for each
    // of its outcomes m0 the second member's sums (register slots of layout
    // p[1]) after the first member's Kraus operator for m0 and its ZZ layer
    C2<T> w[16];
    regroup<T>(o, lt, pd->j_l, w, lt2, pd->b_j_l, tbuf);
    wht<T, 4>(w);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double re = (double)w[j].re, im = (double)w[j].im;
      const double a2 = re * re + im * im;
      acc[0] += wt[0][0][j] * a2;
      acc[1] += wt[0][1][j] * a2;
    }
#pragma unroll 1
    for (int m0 = 0; m0 < 2; ++m0) {
      // tables and slot offsets are read per outcome, not held over the loop
      asm volatile("" : "+v"(lt2), "+v"(ltp1) : : "memory");
      C2<T> u[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const C2<T> e = pl.db[m0][j];
        u[j] = mulc(w[j], e.re, e.im);
      }
      wht<T, 4>(u);
      if (Fb0) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (__popc((uint32_t)j & Fb0) & 1) u[j] = {-u[j].re, -u[j].im};
      }
      if (zz_on) zz_layer(u, base | gt2, pd->b_j_g, eMb, vMb);
      regroup<T>(u, lt2, pd->b_j_l, u, ltp1, pd->p_j_l[1], tbuf);
      wht<T, 4>(u);
      double t0 = 0.0, t1 = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double re = (double)u[j].re, im = (double)u[j].im;
        const double a2 = re * re + im * im;
        t0 += wt[1][0][j] * a2;
        t1 += wt[1][1][j] * a2;
      }
      if (m0) {
        acc[3] += t0;
        acc[5] += t1;
      } else {
        acc[2] += t0;
        acc[4] += t1;
      }
    }
  }
  __syncthreads();  // LDS buffers are reused by the next tile
  }
  if constexpr (BK != U_NONE || kSpecA) {
    constexpr int nacc = kSpecA ? kSums : unit_sums(lb);
    const int lane = tid & 63, wid = tid >> 6;
    const int nw = (int)(blockDim.x + 63) >> 6;
    if constexpr (nacc <= 6) {
#pragma unroll
      for (int a = 0; a < nacc; ++a) {
        const double s = wave_sum(acc[a]);
        if (lane == 0) red[a][wid] = s;
      }
    } else {
      static_assert(kWaveAcc, "more than six sums come from a chain of three or more");
      if ((lane & 3) == 0) {
        const int a = lane >> 2;
#pragma unroll
        for (int k = 0; k < kAcc; ++k)
          if (16 * k + a < nacc) red[16 * k + a][wid] = acc[k];
      }
    }
    __syncthreads();
    if (tid < nacc) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[tid][w];
      partials[(size_t)tid * gridDim.x + blockIdx.x] = s;
    }
  }
}

// The pass kernel (SP = 0; SP = 1: a speculative unit's prediction pass) and
// the redo of a speculative unit, under its own name (it mostly finds nothing
// to do and returns at once).
template <typename T, int AK, int AP, int BK, int BP, bool DN, bool BM0, int SP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UpassWaves<T, BK, BP, DN, BM0>::value))) void k_upass(
    T* __restrict__ st, const UnitPass* __restrict__ pd, const JobConst* __restrict__ jc,
    const BlockRT* __restrict__ rta, const BlockRT* __restrict__ rtb,
    const Decision* __restrict__ dec_a, Decision* __restrict__ dec_b,
    double* __restrict__ partials, int reverse, SlotStrides ss,
    const BlockDense* __restrict__ dna, const BlockDense* __restrict__ dnb, SpecArgs sa) {
  upass_body<T, AK, AP, BK, BP, DN, BM0, SP>(st, pd, jc, rta, rtb, dec_a, dec_b, partials, reverse, ss, dna, dnb, sa);
}
template <typename T, int AK, int AP, int BK, int BP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UpassWaves<T, BK, BP, false, false>::value))) void k_uredo(
    T* __restrict__ st, const UnitPass* __restrict__ pd, const JobConst* __restrict__ jc,
    const BlockRT* __restrict__ rta, const BlockRT* __restrict__ rtb,
    const Decision* __restrict__ dec_a, Decision* __restrict__ dec_b,
    double* __restrict__ partials, int reverse, SlotStrides ss,
    const BlockDense* __restrict__ dna, const BlockDense* __restrict__ dnb, SpecArgs sa) {
  upass_body<T, AK, AP, BK, BP, false, false, 2>(st, pd, jc, rta, rtb, dec_a, dec_b, partials, reverse, ss, dna, dnb, sa);
}

// Member-by-member outcomes of unit B from its sums S (see k_upass): each
// member l is decided from the two sums that follow the outcomes already
// drawn, p1 = S[l][h | 1 << l] / (S[l][h] + S[l][h | 1 << l]), clamped, against
// its measurement draw.
__device__ void decide_chain(const volatile double* S, int lb, const BlockRT* rtb, Decision* dec_b,
                             uint8_t* rec_b, double* p1_b) {
  int h = 0;
  double Sm = 0.0;
  for (int l = 0; l < lb; ++l) {
    const int off = (2 << l) - 2;
    const double s0 = S[off + h], s1 = S[off + (h | (1 << l))];
    const double p1 = clamp_p1(s1 / (s0 + s1));
    const int m = (rtb[l].u < p1) ? 1 : 0;
    rec_b[l] = (uint8_t)m;
    if (p1_b) p1_b[l] = p1;
    h |= m << l;
    Sm = m ? s1 : s0;
  }
  dec_b->m = h;
  dec_b->Sm = Sm;
}

// The full tree of prefix sums (index (2 << l) - 2 + h) in LDS from a unit's
// sums v(a), a < unit_sums(lb): as they are for lb <= 2; for a longer chain
// they are the last level, and each lower level is formed from the one above
// as S[l][h] = S[l + 1][h] + S[l + 1][h | 1 << (l + 1)] (the later member's
// two outcome weights add up to one).  Every thread of the workgroup takes
// part.
template <typename V>
__device__ __forceinline__ void chain_tree_lds(int lb, V v, double* full) {
  const int nacc = unit_sums(lb);
  const int base = lb >= 3 ? (2 << (lb - 1)) - 2 : 0;
  for (int a = threadIdx.x; a < nacc; a += blockDim.x) full[base + a] = v(a);
  for (int l = lb - 2; l >= 0 && lb >= 3; --l) {
    __syncthreads();
    const int up = (2 << (l + 1)) - 2, off = (2 << l) - 2;
    for (int h = threadIdx.x; h < (2 << l); h += blockDim.x)
      full[off + h] = full[up + h] + full[up + h + (2 << l)];
  }
  __syncthreads();
}

// Outcomes of unit B (a chain of lb checks; lb = 1 for an X check), reducing
// each sum over the n per-workgroup partials in a fixed order.
// split = 1, grid (nacc, slots): workgroup a reduces sum a; the last
// workgroup of a slot to finish (ticket counter, reset for the next use)
// decides.  split = 0, grid (slots): one workgroup per slot, thread a sums
// sum a serially (few partials: many small registers side by side).
__global__ __launch_bounds__(256) void k_udecide(const double* __restrict__ partials, int n,
                                                 int lb, const BlockRT* __restrict__ rtb,
                                                 Decision* __restrict__ dec_b,
                                                 uint8_t* __restrict__ rec_b,
                                                 double* __restrict__ p1_b, SlotStrides ss,
                                                 size_t rec_stride, double* __restrict__ sums,
                                                 unsigned* __restrict__ tickets, int split) {
  const int nacc = unit_sums(lb);
  const int slot = split ? (int)blockIdx.y : (int)blockIdx.x;
  partials += (size_t)slot * kChainAcc * n;
  rtb += (size_t)slot * ss.rt;
  dec_b += (size_t)slot * ss.dec;
  rec_b += (size_t)slot * rec_stride;
  if (p1_b) p1_b += (size_t)slot * rec_stride;
  __shared__ double full[kChainAcc];
  if (!split) {
    chain_tree_lds(lb, [&](int a) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += partials[(size_t)a * n + i];
      return s;
    }, full);
    if (threadIdx.x == 0) decide_chain(full, lb, rtb, dec_b, rec_b, p1_b);
    return;
  }
  const int a = blockIdx.x;
  partials += (size_t)a * n;
  sums += (size_t)slot * kChainAcc;
  __shared__ double red[8];
  __shared__ int last;
  double s = 0.0, dummy = 0.0;
  // up to 8 independent loads in flight per thread, summed in a fixed order
  for (int i0 = 0; i0 < n; i0 += 8 * (int)blockDim.x) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = i0 + k * (int)blockDim.x + (int)threadIdx.x;
      v[k] = i < n ? partials[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  block_sum2(s, dummy, red);
  if (threadIdx.x == 0) {
    sums[a] = s;
    __threadfence();
    last = atomicAdd(&tickets[slot], 1u) == (unsigned)(nacc - 1);
  }
  __syncthreads();
  if (!last) return;  // the slot's last workgroup decides
  __threadfence();
  const volatile double* vs = sums;
  chain_tree_lds(lb, [&](int b) { return vs[b]; }, full);
  if (threadIdx.x == 0) {
    decide_chain(full, lb, rtb, dec_b, rec_b, p1_b);
    tickets[slot] = 0u;
  }
}

// Decision of a speculative unit instance of len members after a prediction
// pass or a redo (the grid is set by `split`, below).  tree = 0: 2 len sums along the applied outcomes (S[2 l + m], taken before
// the pass applied the pending renormalisation of dec_a->Sm); each member from
// `known` on is decided as in a plain pass while the members before it match
// what was applied; at the first mismatch the outcome is fixed and a redo is
// due.  tree = 1: the chain's sums over every outcome string (after the
// renormalisation): every member is decided, and a redo re-applies them if
// any differs.  Once every member is decided, dec_b gets the outcome bits and
// S_m, the squared norm of the register the unit's pass writes (its
// renormalisation is applied by the next pass).  A redo that re-applied a
// decided unit leaves nothing to decide (run is cleared); after a redo that
// did not run the kernel returns at once.
// split = 1, grid (sums, slots): workgroup a reduces sum a, the last of a
// slot to finish (ticket) decides; split = 0, grid (slots): one workgroup
// per slot (lockstep launches: thousands of slots, each with few partials,
// and no fence per workgroup).  A slot's tables, records, control record,
// partials and ticket are found with the lockstep strides.
__global__ __launch_bounds__(256) void k_sdecide(const double* __restrict__ partials, int n, int len, int tree,
                                                 const BlockRT* __restrict__ rtb, const Decision* __restrict__ dec_a,
                                                 Decision* __restrict__ dec_b, uint8_t* __restrict__ rec_b,
                                                 double* __restrict__ p1_b, SpecCtl* __restrict__ ctl,
                                                 double* __restrict__ sums, unsigned* __restrict__ ticket,
                                                 SlotStrides ss, size_t rec_stride, size_t ctl_stride, int split) {
  const size_t slot = split ? blockIdx.y : blockIdx.x;
  partials += slot * kChainAcc * n;
  rtb += slot * ss.rt;
  dec_a += slot * ss.dec;
  dec_b += slot * ss.dec;
  rec_b += slot * rec_stride;
  if (p1_b) p1_b += slot * rec_stride;
  ctl += slot * ctl_stride;
  sums += slot * kChainAcc;
  ticket += slot;
  // the record as the workgroup sees it (workgroup 0 may clear run meanwhile)
  __shared__ int c_run, c_known;
  if (threadIdx.x == 0) {
    const volatile SpecCtl* vc = ctl;
    c_run = vc->run;
    c_known = vc->known;
  }
  __syncthreads();
  if (!c_run) return;
  if (c_known >= len) {
    if ((!split || blockIdx.x == 0) && threadIdx.x == 0) ctl->run = 0;
    return;
  }
  const int nacc = tree ? unit_sums(len) : 2 * len;
  __shared__ double full[kChainAcc];
  __shared__ double col[kChainAcc];
  const volatile double* vs = col;
  if (split) {
    const int a = blockIdx.x;
    if (a >= nacc) return;
    partials += (size_t)a * n;
    __shared__ double red[8];
    __shared__ int last;
    double s = 0.0, dummy = 0.0;
    for (int i0 = 0; i0 < n; i0 += 8 * (int)blockDim.x) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int i = i0 + k * (int)blockDim.x + (int)threadIdx.x;
        v[k] = i < n ? partials[i] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) s += v[k];
    }
    block_sum2(s, dummy, red);
    if (threadIdx.x == 0) {
      sums[a] = s;
      __threadfence();
      last = atomicAdd(ticket, 1u) == (unsigned)(nacc - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    vs = sums;
    if (threadIdx.x == 0) *ticket = 0u;
  } else {
    // one workgroup per slot (lockstep: few partials per sum): thread a
    // sums sum a serially, in the order of the partials
    for (int a = threadIdx.x; a < nacc; a += blockDim.x) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += partials[(size_t)a * n + i];
      col[a] = s;
    }
    __syncthreads();
  }
  if (tree) {
    chain_tree_lds(len, [&](int b) { return vs[b]; }, full);
    if (threadIdx.x == 0) {
      const int applied = ctl->m;
      decide_chain(full, len, rtb, dec_b, rec_b, p1_b);
      ctl->m = dec_b->m;
      ctl->known = len;
      ctl->run = dec_b->m != applied;
    }
    return;
  }
  if (threadIdx.x == 0) {
    const double sm_in = dec_a->Sm;
    int m = ctl->m;
    int l = ctl->known;
    bool redo = false;
    double Sm = 0.0;
    for (; l < len; ++l) {
      const double s0 = vs[2 * l], s1 = vs[2 * l + 1];
      const double p1 = clamp_p1(s1 / (s0 + s1));
      const int ml = (rtb[l].u < p1) ? 1 : 0;
      rec_b[l] = (uint8_t)ml;
      if (p1_b) p1_b[l] = p1;
      Sm = (ml ? s1 : s0) / sm_in;
      if (ml != ((m >> l) & 1)) {
        m ^= 1 << l;
        redo = true;
        ++l;
        break;
      }
    }
    ctl->m = m;
    ctl->known = l;
    ctl->run = redo;
    if (l == len) {
      dec_b->m = m;
      dec_b->Sm = Sm;
    }
  }
}

// Decision records of n trajectory slots (stride apart) for a register that
// logical |0> is written into: norm 1, frame 0.
__global__ void k_dec_init(Decision* __restrict__ d, int n, size_t stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[(size_t)i * stride] = Decision{1.0, 0, 0u};
}

// The pending renormalisation 1 / sqrt(d->Sm) applied to a whole register.
template <typename T>
__global__ __launch_bounds__(256) void k_renorm(T* __restrict__ st, uint64_t na, const Decision* __restrict__ d) {
  const double sc = 1.0 / sqrt(d->Sm);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += (uint64_t)gridDim.x * blockDim.x) {
    C2<T> a = ld2(st, i);
    a.re = (T)((double)a.re * sc);
    a.im = (T)((double)a.im * sc);
    st2(st, i, a);
  }
}

// ------------------------------------------------------ final measurement --
// Sums of |psi|^2 over contiguous chunks of 2^cb amplitudes.
template <typename T>
__global__ __launch_bounds__(256) void k_final_sums(const T* __restrict__ st, int cb,
                                                     double* __restrict__ sums, size_t st_stride) {
  st += (size_t)blockIdx.y * st_stride;
  sums += (size_t)blockIdx.y * gridDim.x;
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

// Sequential measurement of data qubits n-1 .. 0 (labels n .. 1) using the
// chunk sums for the high n - cb bits and the selected chunk for the rest;
// the register is read in the Pauli-X frame recorded in dfin (if given).
// Each phase builds the pairwise sum tree of its leaves (the chunk sums, then
// |psi|^2 over the selected chunk) in LDS, one level per step, and one thread
// walks it from the root: at each level the two child sums give p1, the
// qubit's draw picks a child.  The bottom level of leaves stays in memory.
// Slot blockIdx.x: its register at st + slot * st_stride, its draw stream
// (seed[slot], t[slot]) when the arrays are given, else (seed0, t0 + slot).
template <typename T>
__global__ __launch_bounds__(1024) void k_final_measure(const T* __restrict__ st, int n, int cb,
                                                         const double* __restrict__ sums,
                                                         uint64_t seed0, uint64_t t0, uint64_t k0,
                                                         uint8_t* __restrict__ bits, size_t st_stride,
                                                         const uint64_t* __restrict__ seeds,
                                                         const uint64_t* __restrict__ streams,
                                                         const int* __restrict__ rounds,
                                                         uint64_t draws_round,
                                                         const Decision* __restrict__ dfin,
                                                         size_t dfin_stride) {
  const int slot = blockIdx.x;
  // Pauli-X frame of the register: logical bit q = physical bit q ^ phi_q
  const uint32_t phi = dfin ? dfin[(size_t)slot * dfin_stride].phi : 0u;
  st += (size_t)slot * st_stride;
  sums += (size_t)slot << (n - cb);
  bits += (size_t)slot * n;
  const uint64_t seed = seeds ? seeds[slot] : seed0;
  const uint64_t t = streams ? streams[slot] : t0 + (uint64_t)slot;
  if (rounds) k0 = (uint64_t)rounds[slot] * draws_round;
  __shared__ double tree[8192];  // internal nodes of a tree of up to 2^13 leaves (node 1: root)
  __shared__ int sel;
  // qubits level0 .. level0 + h - 1 from a tree over the 2^h leaves leaf(i);
  // returns the chosen leaf
  auto descend = [&](int h, int level0, auto leaf) -> int {
    if (h == 0) return 0;
    const int N = 1 << h;
    __syncthreads();
    for (int k = N / 2 + (int)threadIdx.x; k < N; k += (int)blockDim.x) tree[k] = leaf(2 * k - N) + leaf(2 * k + 1 - N);
    for (int lev = h - 2; lev >= 0; --lev) {
      __syncthreads();
      for (int k = (1 << lev) + (int)threadIdx.x; k < (2 << lev); k += (int)blockDim.x)
        tree[k] = tree[2 * k] + tree[2 * k + 1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int c = 1;
      for (int i = 0; i < h; ++i) {
        const int level = level0 + i;
        const int fq = (phi >> (n - 1 - level)) & 1;
        const bool bottom = i == h - 1;
        const double P0 = bottom ? leaf(2 * c - N) : tree[2 * c];
        const double P1 = bottom ? leaf(2 * c + 1 - N) : tree[2 * c + 1];
        const double S0 = fq ? P1 : P0, S1 = fq ? P0 : P1;
        const double p1 = clamp_p1(S1 / (S0 + S1));
        const double u = uniform(seed, t, k0 + (uint64_t)level);
        const int b = (u < p1) ? 1 : 0;
        bits[n - 1 - level] = (uint8_t)b;
        c = 2 * c + (b ^ fq);
      }
      sel = c - N;
    }
    __syncthreads();
    return sel;
  };
  const int hb = n - cb;  // bits resolved by chunk sums
  const int chunk = descend(hb, 0, [&](int i) { return sums[i]; });
  const uint64_t cbase = (uint64_t)chunk << cb;
  descend(cb, hb, [&](int i) {
    const C2<T> a = ld2(st, cbase + (uint64_t)i);
    const double re = (double)a.re, im = (double)a.im;
    return re * re + im * im;
  });
}

// Replayed trajectories: copy the staged records, p1 trace and final bits of
// trajectory *cur to their slots, then advance *cur and its draw stream.
__global__ void k_commit(const uint8_t* __restrict__ rec_s, const double* __restrict__ p1_s,
                         const uint8_t* __restrict__ bits_s, uint8_t* __restrict__ rec,
                         double* __restrict__ p1, uint8_t* __restrict__ bits, int per_traj, int n,
                         uint64_t* __restrict__ cur, uint64_t* __restrict__ stream, uint64_t traj0) {
  const uint64_t c = *cur;
  for (int i = threadIdx.x; i < per_traj; i += blockDim.x) {
    rec[c * per_traj + i] = rec_s[i];
    if (p1) p1[c * per_traj + i] = p1_s[i];
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) bits[c * n + i] = bits_s[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    *cur = c + 1;
    *stream = traj0 + c + 1;
  }
}

}  // namespace qec
