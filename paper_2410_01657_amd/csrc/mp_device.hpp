// Device building blocks for the message-passing kernels (gfx950, wave64).
//
// Row-block layout.  A wave works on blocks of 16 rows (edges or nodes).
// Lane l handles row j = l % 16 of the block and lane group g = l / 16.  For
// a feature vector of width W (a multiple of 16) the lane holds W/4 values:
//   v[4*b + r]  <->  feature 16*b + 4*g + r      (b < W/16, r < 4)
// so the four lanes of a row together hold the whole row, each lane as W/16
// contiguous float4 chunks.  This is exactly the accumulator layout of the
// 16x16 MFMA instructions when the product is computed transposed
// (output features x rows), which lets the output of one Linear feed the
// next one with no data movement: the K ordering of each product is permuted
// to match, and the weight fragments are packed in that order.
//
// Weight fragments.  A product out[f][row] = sum_k A[f][k] in[k][row] with
// A of shape [M][K] is stored as
//   FP32 (v_mfma_f32_16x16x4f32):  frag[(mb*(K/4) + s)*64 + lane]
//        = A[16*mb + lane%16][16*(s/4) + 4*(lane/16) + s%4]
//   BF16 (v_mfma_f32_16x16x32_bf16): frag16[(mb*(K/32) + t)*64 + lane] =
//        8 values q = 0..7 of A[16*mb + lane%16][32*t + 16*(q/4) + 4*(lane/16) + q%4]
// and the input operand of step s (FP32) is in[s], of step t (BF16) is
// in[8t .. 8t+7], directly in the row-block layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// ------------------------------------------------------------------ loads

// Load the row-block slice of a W-wide row (ptr = start of the row).
// Lane (j, g) moves features 16b + 4g .. +3, so one instruction covers half
// of each 128-byte line of a row.  All row traffic uses ordinary cached
// loads and stores: L2 then merges the two halves of a line (non-temporal
// stores wrote about 40% more bytes than the arrays hold, and non-temporal
// loads measured slower as well).
template <int W>
__device__ __forceinline__ void load_row(const float* __restrict__ ptr, int g, float (&v)[W / 4]) {
#pragma unroll
  for (int b = 0; b < W / 16; ++b) {
    const float4 t = *reinterpret_cast<const float4*>(ptr + 16 * b + 4 * g);
    v[4 * b + 0] = t.x;
    v[4 * b + 1] = t.y;
    v[4 * b + 2] = t.z;
    v[4 * b + 3] = t.w;
  }
}

template <int W>
__device__ __forceinline__ void store_row(float* __restrict__ ptr, int g, const float (&v)[W / 4]) {
#pragma unroll
  for (int b = 0; b < W / 16; ++b)
    *reinterpret_cast<float4*>(ptr + 16 * b + 4 * g) =
        make_float4(v[4 * b + 0], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3]);
}

// BF16 storage of a row (round to nearest even) and its FP32 read-back.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
template <int W>
__device__ __forceinline__ void store_row_bf16(__bf16* __restrict__ ptr, int g, const float (&v)[W / 4]) {
#pragma unroll
  for (int b = 0; b < W / 16; ++b) {
    const v4bf t = {(__bf16)v[4 * b], (__bf16)v[4 * b + 1], (__bf16)v[4 * b + 2], (__bf16)v[4 * b + 3]};
    *reinterpret_cast<u32x2*>(ptr + 16 * b + 4 * g) = __builtin_bit_cast(u32x2, t);
  }
}
template <int W>
__device__ __forceinline__ void load_row_bf16(const __bf16* __restrict__ ptr, int g, float (&v)[W / 4]) {
#pragma unroll
  for (int b = 0; b < W / 16; ++b) {
    const v4bf t = __builtin_bit_cast(v4bf, *reinterpret_cast<const u32x2*>(ptr + 16 * b + 4 * g));
    v[4 * b + 0] = (float)t[0];
    v[4 * b + 1] = (float)t[1];
    v[4 * b + 2] = (float)t[2];
    v[4 * b + 3] = (float)t[3];
  }
}

// Row `row` of an [n][W] array stored as FP32 or (BF) BF16.
template <int W, bool BF>
__device__ __forceinline__ void store_row_t(void* __restrict__ base, int64_t row, int g, const float (&v)[W / 4]) {
  if constexpr (BF)
    store_row_bf16<W>(reinterpret_cast<__bf16*>(base) + row * W, g, v);
  else
    store_row<W>(reinterpret_cast<float*>(base) + row * W, g, v);
}
template <int W, bool BF>
__device__ __forceinline__ void load_row_t(const void* __restrict__ base, int64_t row, int g, float (&v)[W / 4]) {
  if constexpr (BF)
    load_row_bf16<W>(reinterpret_cast<const __bf16*>(base) + row * W, g, v);
  else
    load_row<W>(reinterpret_cast<const float*>(base) + row * W, g, v);
}

// Per-feature vector (bias, LayerNorm gain) in row-block layout.
template <int W>
__device__ __forceinline__ void load_vec(const float* __restrict__ p, int g, float (&v)[W / 4]) {
  load_row<W>(p, g, v);
}

// ------------------------------------------------------------- GEMMs

// acc[f] += sum_k A[f][k] in[k]  (A packed as FP32 fragments; MB = M/16,
// KB = K/16).  Independent output blocks are interleaved so consecutive
// MFMAs do not depend on each other.
// ROT: the fragments sit in LDS in the rotated layout of stage_frags_rot
// (element o of 64-float chunk c at c*64 + (o + c%4) % 64); chunk
// mb*4KB + s has c%4 = s%4.
template <int MB, int KB, bool ROT = false>
__device__ __forceinline__ void gemm_f32(const float* __restrict__ frag, const float (&in)[4 * KB],
                                         float (&acc)[4 * MB], int lane) {
  v4f c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) c[mb] = v4f{acc[4 * mb], acc[4 * mb + 1], acc[4 * mb + 2], acc[4 * mb + 3]};
#pragma unroll
  for (int s = 0; s < 4 * KB; ++s) {
    const int l = ROT ? ((lane + (s & 3)) & 63) : lane;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(frag[(mb * 4 * KB + s) * 64 + l], in[s], c[mb], 0, 0, 0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    acc[4 * mb] = c[mb][0];
    acc[4 * mb + 1] = c[mb][1];
    acc[4 * mb + 2] = c[mb][2];
    acc[4 * mb + 3] = c[mb][3];
  }
}

// acc += W^T in for a square H x H matrix W stored as FP32 fragments (the
// layout gemm_f32 reads for W in).  Fragment element (mb, s, lane i + 16k)
// holds W[16 mb + i][f(s, k)] with f(s, k) = 16 (s/4) + 4k + s%4, the
// feature order of the row-block layout; W^T's element for step s, output
// block mb' and lane (i, k) is W[f(s, k)][16 mb' + i], found at fragment
// (s/4, 4 mb' + i%4, lane 4k + s%4 + 16 (i/4)).  One LDS read per MFMA as
// in gemm_f32, so the transposed matrix need not be stored.  In the packed
// layout the 64 lanes of one read reach only 16 LDS banks (lanes with equal
// i/4 and k but different i%4 read the same bank of four fragments); in the
// rotated layout (ROT) they reach 64 distinct banks.
template <int H, bool ROT = false>
__device__ __forceinline__ void gemm_f32_tr(const float* __restrict__ frag, const float (&in)[H / 4],
                                            float (&acc)[H / 4], int lane) {
  constexpr int MB = H / 16, S = H / 4;
  const int i = lane & 15, k = lane >> 4;
  v4f c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) c[mb] = v4f{acc[4 * mb], acc[4 * mb + 1], acc[4 * mb + 2], acc[4 * mb + 3]};
#pragma unroll
  for (int s = 0; s < S; ++s) {
    // fragment (s/4) S + 4 mb + i%4 (its chunk index is i%4 mod 4), element s%4 + 4k + 16 (i/4)
    const int o = (s & 3) + 4 * k + 16 * (i >> 2);
    const int lane_off = (i & 3) * 64 + (ROT ? ((o + (i & 3)) & 63) : o);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(frag[((s >> 2) * S + 4 * mb) * 64 + lane_off], in[s], c[mb], 0,
                                                   0, 0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    acc[4 * mb] = c[mb][0];
    acc[4 * mb + 1] = c[mb][1];
    acc[4 * mb + 2] = c[mb][2];
    acc[4 * mb + 3] = c[mb][3];
  }
}

// acc += W^T in for an M x K matrix W stored as FP32 fragments (the layout
// gemm_f32 reads for W in): in holds M features, acc K.  The same
// transposed addressing as gemm_f32_tr, with the fragment row-block
// stride of a K-wide matrix (gemm_f32_tr is the case M = K = H).
template <int M, int K, bool ROT = false>
__device__ __forceinline__ void gemm_f32_tr_mk(const float* __restrict__ frag, const float (&in)[M / 4],
                                               float (&acc)[K / 4], int lane) {
  constexpr int MB = K / 16, S = K / 4, STEPS = M / 4;
  const int i = lane & 15, k = lane >> 4;
  v4f c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) c[mb] = v4f{acc[4 * mb], acc[4 * mb + 1], acc[4 * mb + 2], acc[4 * mb + 3]};
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
    const int o = (s & 3) + 4 * k + 16 * (i >> 2);
    const int lane_off = (i & 3) * 64 + (ROT ? ((o + (i & 3)) & 63) : o);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(frag[((s >> 2) * S + 4 * mb) * 64 + lane_off], in[s], c[mb], 0,
                                                   0, 0);
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    acc[4 * mb] = c[mb][0];
    acc[4 * mb + 1] = c[mb][1];
    acc[4 * mb + 2] = c[mb][2];
    acc[4 * mb + 3] = c[mb][3];
  }
}

__device__ __forceinline__ v8bf to_bf8(const float* x) {
  v8bf r;
#pragma unroll
  for (int q = 0; q < 8; ++q) r[q] = (__bf16)x[q];  // round to nearest even
  return r;
}

template <int MB, int KB>
__device__ __forceinline__ void gemm_bf16(const uint4* __restrict__ frag, const float (&in)[4 * KB],
                                          float (&acc)[4 * MB], int lane) {
  static_assert(KB % 2 == 0, "BF16 products need K to be a multiple of 32");
  constexpr int T = KB / 2;
  v4f c[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) c[mb] = v4f{acc[4 * mb], acc[4 * mb + 1], acc[4 * mb + 2], acc[4 * mb + 3]};
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const v8bf b = to_bf8(&in[8 * t]);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const uint4 a = frag[(mb * T + t) * 64 + lane];
      c[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), b, c[mb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    acc[4 * mb] = c[mb][0];
    acc[4 * mb + 1] = c[mb][1];
    acc[4 * mb + 2] = c[mb][2];
    acc[4 * mb + 3] = c[mb][3];
  }
}

// Dispatch on the GEMM operand type.  frag points at the fragments of one
// matrix (FP32: M*K floats; BF16: M*K bf16 values).
template <bool BF, int MB, int KB, bool ROT = false>
__device__ __forceinline__ void gemm(const void* frag, const float (&in)[4 * KB], float (&acc)[4 * MB], int lane) {
  static_assert(!(BF && ROT), "the rotated layout is an FP32 fragment layout");
  if constexpr (BF)
    gemm_bf16<MB, KB>(reinterpret_cast<const uint4*>(frag), in, acc, lane);
  else
    gemm_f32<MB, KB, ROT>(reinterpret_cast<const float*>(frag), in, acc, lane);
}

// Bytes of the packed fragments of an M x K matrix.
__host__ __device__ constexpr size_t frag_bytes(int M, int K, bool bf) { return size_t(M) * K * (bf ? 2 : 4); }

// An opaque zero: adding it to an LDS offset inside a loop keeps the
// compiler from hoisting every weight-fragment read out of the loop (which
// would pin the whole matrix in registers and cut occupancy).
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+v"(z));
  return z;
}

// --------------------------------------------------- elementwise helpers

// ELU with alpha = 1.  The negative branch uses the hardware exponential
// (v_exp_f32 on a prescaled argument, a few ulp): exp(z) - 1 is then off by
// at most ~1e-7 in absolute terms for z <= 0, far below FP32 tolerances.
__device__ __forceinline__ float elu(float z) { return z > 0.f ? z : __expf(z) - 1.f; }
__device__ __forceinline__ float elu_deriv(float z) { return z > 0.f ? 1.f : __expf(z); }
// ELU'(h) from u = ELU(h): 1 for h > 0, else exp(h) = u + 1.  u > 0 exactly
// when h > 0, and then u + 1 >= 1, so min(u + 1, 1) is the same value in
// two instructions instead of four.
__device__ __forceinline__ float elu_deriv_from_value(float u) { return fminf(u + 1.f, 1.f); }

// Sum over the four lanes that share a row (lane groups g = 0..3), on the
// matrix unit: v_mfma_f32_16x16x4f32 with A = 1 and B[k][j] = the value of
// lane j + 16k gives D[i][j] = sum over k for every i, and lane j + 16g
// receives D[4g..4g+3][j].  One FP32 MFMA instead of two dependent LDS
// permutes; must be called with all lanes active.
__device__ __forceinline__ float row_sum(float s) {
  const v4f d = __builtin_amdgcn_mfma_f32_16x16x4f32(1.f, s, v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  return d[0];
}

// LayerNorm statistics (biased variance) of a W-wide row in row-block layout.
template <int W>
__device__ __forceinline__ void ln_stats(const float (&v)[W / 4], float eps, float& mean, float& rstd) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < W / 4; ++i) s += v[i];
  mean = row_sum(s) * (1.f / W);
  float q = 0.f;
#pragma unroll
  for (int i = 0; i < W / 4; ++i) {
    const float d = v[i] - mean;
    q += d * d;
  }
  const float var = row_sum(q) * (1.f / W);
  rstd = 1.f / sqrtf(var + eps);
}

// --------------------------------------------- small first/last Linears

// Stage W[rows][k] (k <= 4) into LDS as [rows][4], zero padded, with the
// whole block (callers synchronise afterwards).
__device__ __forceinline__ void stage_small(float* __restrict__ dst, const float* __restrict__ W, int rows, int k) {
  for (int t = threadIdx.x; t < rows * 4; t += blockDim.x) {
    const int r = t >> 2, c = t & 3;
    dst[t] = c < k ? W[r * k + c] : 0.f;
  }
}

// z[f] += sum_k W0[f][k] in[k] for the lane's features, W0 staged as [H][4].
template <int H>
__device__ __forceinline__ void small_in_linear(const float* __restrict__ w0s, const float (&in)[4], int g,
                                                float (&z)[H / 4]) {
#pragma unroll
  for (int i = 0; i < H / 4; ++i) {
    const int f = 16 * (i / 4) + 4 * g + (i % 4);
    const float4 w = *reinterpret_cast<const float4*>(w0s + 4 * f);
    z[i] += w.x * in[0] + w.y * in[1] + w.z * in[2] + w.w * in[3];
  }
}

// ------------------------------------------- segmented sums over 16 lanes

// DPP row_shr:n within each 16-lane row; lanes j < n read 0.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, true);
}
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_ROR1 = 0x121;  // lane j reads lane (j-1) mod 16

// Inclusive segmented scan over the 16 lanes j of each lane group.  key
// identifies the segment (equal keys are contiguous in j) and must be
// nonzero, because lanes shifted in from outside the row read key 0.
template <int N>
__device__ __forceinline__ void seg_scan16(float (&v)[N], int key) {
  // Each step adds the value `off` lanes back when that lane is in the same
  // segment, written as v += shifted * (0 or 1) so the shift folds into the
  // multiply-add as a DPP operand.  Steps 4 and 8 are skipped (uniformly for
  // the wave) when no segment in the block is that long.
#define MP_SEG_STEP(CTRL)                                     \
  {                                                           \
    const float same = dpp_i<CTRL>(key) == key ? 1.f : 0.f;   \
    _Pragma("unroll") for (int i = 0; i < N; ++i)             \
      v[i] = fmaf(dpp_f<CTRL>(v[i]), same, v[i]);             \
  }
  MP_SEG_STEP(DPP_ROW_SHR1)
  MP_SEG_STEP(DPP_ROW_SHR2)
  if (__ballot(dpp_i<DPP_ROW_SHR4>(key) == key) != 0) {
    MP_SEG_STEP(DPP_ROW_SHR4)
    if (__ballot(dpp_i<DPP_ROW_SHR8>(key) == key) != 0) MP_SEG_STEP(DPP_ROW_SHR8)
  }
#undef MP_SEG_STEP
}

// Value of the lane whose index j (within its 16-lane group) differs in
// bit M (M = 1, 2, 4, 8): DPP quad permutations for 1 and 2, a 16-lane
// rotation by 8 for 8, and a bitmask swizzle (xor 4) for 4.
template <int M>
__device__ __forceinline__ float lane_xor16(float x) {
  const int v = __builtin_bit_cast(int, x);
  if constexpr (M == 1)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false));  // [1,0,3,2]
  else if constexpr (M == 2)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false));  // [2,3,0,1]
  else if constexpr (M == 4)
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(v, 0x101F));  // and 0x1f, xor 4
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false));  // row_ror:8
}

// One halving step of a reduce-scatter over the 16 lanes j of a lane
// group: the lane keeps the half of its N values selected by bit M of j
// and adds the partner's copy of that half (the partner sends the half it
// does not keep).
template <int N, int M>
__device__ __forceinline__ void sum16_half(const float (&in)[N], float (&out)[N / 2], int j) {
  const bool hi = (j & M) != 0;
#pragma unroll
  for (int q = 0; q < N / 2; ++q) {
    const float lo_v = in[q], hi_v = in[q + N / 2];
    out[q] = (hi ? hi_v : lo_v) + lane_xor16<M>(hi ? lo_v : hi_v);
  }
}

// Sum over the 16 lanes of each lane group, scattered: on return lane j
// holds in out[c] the sum over the group's lanes of v[j * (N / 16) + c]
// (N a multiple of 16).  Four halving steps (bits 8, 4, 2, 1 of j), N - N/16
// exchanged values in all; the additions are in a fixed order, so the sums
// are bitwise reproducible.
template <int N>
__device__ __forceinline__ void sum16_scatter(const float (&v)[N], float (&out)[N / 16], int j) {
  static_assert(N % 16 == 0, "sum16_scatter needs a multiple of 16 values");
  float a8[N / 2], a4[N / 4], a2[N / 8];
  sum16_half<N, 8>(v, a8, j);
  sum16_half<N / 2, 4>(a8, a4, j);
  sum16_half<N / 4, 2>(a4, a2, j);
  sum16_half<N / 8, 1>(a2, out, j);
}

// Value of lane 15 of the same lane group, delivered to lane 0 (and lane
// j+1 receives lane j, which callers ignore).
__device__ __forceinline__ float from_prev_lane(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), DPP_ROW_ROR1, 0xf, 0xf, false));
}
__device__ __forceinline__ int from_prev_lane_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, DPP_ROW_ROR1, 0xf, 0xf, false);
}

// ----------------------------------------- static wave schedules over rows

// Split rows [0, n_rows) into n_parts contiguous ranges with about equal
// edge counts: part p starts at the first row whose first edge index is at
// least floor(p * E / n_parts); the last part ends at n_rows.
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* __restrict__ a, int64_t n, int64_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ void part_rows(const int32_t* __restrict__ rowptr, int64_t n_rows, int64_t n_parts,
                                          int64_t p, int64_t& r0, int64_t& r1) {
  const int64_t E = rowptr[n_rows];
  r0 = (p == 0) ? 0 : lower_bound_i32(rowptr, n_rows + 1, (p * E) / n_parts);
  r1 = (p + 1 >= n_parts) ? n_rows : lower_bound_i32(rowptr, n_rows + 1, ((p + 1) * E) / n_parts);
  if (r0 > n_rows) r0 = n_rows;
  if (r1 > n_rows) r1 = n_rows;
  if (r1 < r0) r1 = r0;
}

// Tiled schedule for the edge kernels.  The rows are cut into n_tiles
// row-aligned tiles of about equal edge count (tile boundaries precomputed by
// k_tiles).  Workgroups are dealt round robin to the 8 XCDs, so workgroup b
// runs on XCD b % 8; each XCD takes one contiguous eighth of the tiles, and
// inside it the XCD's waves take consecutive tiles in turn.  All waves of an
// XCD thus sweep a compact window of rows together, and a node row gathered
// by edges a few planes apart is still in that XCD's L2.
struct TileSched {
  int64_t t0, t1;    // this group's tile range
  int64_t rank, nr;  // block rank inside the group, blocks in the group
};
__device__ __forceinline__ TileSched tile_sched(int64_t n_tiles) {
  const int64_t G = gridDim.x, V = G < 8 ? G : 8;
  const int64_t vx = blockIdx.x % V;
  TileSched s;
  s.rank = blockIdx.x / V;
  s.nr = (G - vx + V - 1) / V;
  s.t0 = vx * n_tiles / V;
  s.t1 = (vx + 1) * n_tiles / V;
  return s;
}

// Dynamic tile order: the tiles are cut into V contiguous ranges (one per
// XCD, V = min(grid, 8), workgroup b on XCD b % V as in tile_sched); a wave
// takes the next tile of its XCD's range from an atomic counter, and once
// that range is empty moves on to the next XCD's range, and so on.
// Returns -1 when every range is exhausted.  Tiles are row aligned, so a
// tile's results do not depend on which wave computes it: the order is
// dynamic but the results stay bitwise reproducible.
__device__ __forceinline__ int64_t queue_next(int32_t* queue, int64_t n_tiles, int64_t V, int x0, int& q) {
  while (q < V) {
    const int x = (int)((x0 + q) % V);
    const int64_t t0 = x * n_tiles / V, t1 = (x + 1) * n_tiles / V;
    int old = 0;
    if ((threadIdx.x & 63) == 0) old = atomicAdd(queue + x, 1);
    old = __builtin_amdgcn_readfirstlane(old);
    const int64_t t = t0 + old;
    if (t < t1) return t;
    ++q;
  }
  return -1;
}

// XCD-aware block numbering: the dispatcher hands consecutive workgroups to
// the 8 XCDs in turn; renumber so that each XCD gets one contiguous eighth
// of the work (its L2 then sees neighbouring rows).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t per = (nb + 7) / 8;
  const int64_t x = b % 8, i = b / 8;
  const int64_t full = nb % 8 == 0 ? 8 : nb % 8;  // XCDs that get `per` blocks
  // blocks dealt round robin: XCD x receives per or per-1 blocks
  const int64_t start = x < full ? x * per : full * per + (x - full) * (per - 1);
  return start + i;
}

}  // namespace mp
