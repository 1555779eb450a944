// Backward (adjoint) kernels of the consistent message-passing layer and of
// the row MLPs.  Gradient consistency (Eq. 3) needs the exact adjoint of
// every forward step: the segment sum's adjoint is a gather scaled by
// 1/d_ij, the halo sum is symmetric and reuses the forward kernel, and the
// gathers of receiver/sender features become in-row sums (the sender part
// through the reverse-edge index, so no atomics are needed).
//
// Weight gradients are sums over all rows of outer products.  The NW waves
// of a workgroup (4 or 8) walk their rows in lock step: every wave stages
// one 16-row block of the two factors in LDS, transposed, then each wave
// accumulates its own subset of 16x16 gradient tiles over the 16*NW staged
// rows with MFMA.  Each workgroup writes one slab of partial gradients;
// launch_wreduce adds the slabs in workgroup order.  Where the fused form
// does not fit on chip (H = 128), a streaming kernel writes the per-row
// factors and k_row_dw forms the same sums from them.  Schedules are
// static, so every result is bitwise reproducible.
#include <algorithm>
#include <type_traits>

#include "mp_device.hpp"
#include "mp_kernels.hpp"

namespace mp {

constexpr size_t kLdsLimit = 160 * 1024 - 1024;
constexpr int kWaves = 4;  // waves per workgroup in the row-MLP lock-step kernels

// LDS staging of a ROWS-row block of a W-wide operand, transposed: element
// (row r, feature f) sits at tile[f * RS + r], so the MFMA operands of the
// weight-gradient products (rows along K) are contiguous 16-byte reads.
// Each feature row is padded (4 floats, or 8 bf16 values) to spread banks.
template <bool BF, int ROWS>
struct Stg {
  using T = typename std::conditional<BF, __bf16, float>::type;
  static constexpr int RS = ROWS + (BF ? 8 : 4);
};
template <int W, bool BF, int ROWS = 64>
constexpr size_t tile_bytes() { return size_t(W) * Stg<BF, ROWS>::RS * (BF ? 2 : 4); }

template <int W, bool BF, int ROWS = 64, bool PK = true>
__device__ __forceinline__ void stage_row(void* __restrict__ tile, int row, int g, const float (&v)[W / 4]) {
  constexpr int RS = Stg<BF, ROWS>::RS;
  if constexpr (BF && !PK) {
    // one conversion per value (fewer live registers than the packed form)
    __bf16* t = reinterpret_cast<__bf16*>(tile);
#pragma unroll
    for (int i = 0; i < W / 4; ++i) t[(16 * (i / 4) + 4 * g + (i % 4)) * RS + row] = (__bf16)v[i];
  } else if constexpr (BF) {
    // features f, f+1 (consecutive in the lane) are rounded as one pair and
    // written as the low and high halves of the packed value
    uint16_t* t = reinterpret_cast<uint16_t*>(tile);
#pragma unroll
    for (int i = 0; i < W / 4; i += 2) {
      const int f = 16 * (i / 4) + 4 * g + (i % 4);
      uint32_t pk = __builtin_bit_cast(uint32_t, v2bf{(__bf16)v[i], (__bf16)v[i + 1]});
      asm volatile("" : "+v"(pk));  // keep the pair packed (one conversion, two half stores)
      t[f * RS + row] = (uint16_t)pk;
      t[(f + 1) * RS + row] = (uint16_t)(pk >> 16);
    }
  } else {
    float* t = reinterpret_cast<float*>(tile);
#pragma unroll
    for (int i = 0; i < W / 4; ++i) t[(16 * (i / 4) + 4 * g + (i % 4)) * RS + row] = v[i];
  }
}

template <int GW, int AW, int NW = kWaves>
constexpr int dw_tiles_per_wave() { return ((GW / 16) * (AW / 16) + NW - 1) / NW; }

// acc[n] += sum over the 16*NW staged rows of G[f][row] * A[k][row] for the
// tiles t = wave + NW*n (t = fb * (AW/16) + kb) this wave owns.
// FP32: v_mfma_f32_16x16x4f32, lane (i, kk) covering rows kk*4NW + s;
// BF16: v_mfma_f32_16x16x32_bf16, lane (i, kk) covering rows 32t + 8kk + q.
template <int GW, int AW, bool BF, int NW = kWaves>
__device__ __forceinline__ void dw_tiles(const void* __restrict__ G, const void* __restrict__ A,
                                         v4f (&acc)[dw_tiles_per_wave<GW, AW, NW>()], int wave, int lane) {
  constexpr int NT = dw_tiles_per_wave<GW, AW, NW>(), NTILE = (GW / 16) * (AW / 16), KBN = AW / 16;
  constexpr int ROWS = 16 * NW, RS = Stg<BF, ROWS>::RS;
  const int li = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int t = wave + NW * n;
    if (t < NTILE) {
      const int fb = t / KBN, kb = t % KBN;
      if constexpr (BF) {
        const __bf16* g = reinterpret_cast<const __bf16*>(G) + (16 * fb + li) * RS + 8 * kk;
        const __bf16* a = reinterpret_cast<const __bf16*>(A) + (16 * kb + li) * RS + 8 * kk;
#pragma unroll
        for (int tt = 0; tt < ROWS / 32; ++tt) {
          const v8bf gv = *reinterpret_cast<const v8bf*>(g + 32 * tt);
          const v8bf av = *reinterpret_cast<const v8bf*>(a + 32 * tt);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gv, av, acc[n], 0, 0, 0);
        }
      } else {
        const float* g = reinterpret_cast<const float*>(G) + (16 * fb + li) * RS + (ROWS / 4) * kk;
        const float* a = reinterpret_cast<const float*>(A) + (16 * kb + li) * RS + (ROWS / 4) * kk;
#pragma unroll
        for (int q = 0; q < ROWS / 16; ++q) {
          const float4 gv = *reinterpret_cast<const float4*>(g + 4 * q);
          const float4 av = *reinterpret_cast<const float4*>(a + 4 * q);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.x, av.x, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.y, av.y, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.z, av.z, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.w, av.w, acc[n], 0, 0, 0);
        }
      }
    }
  }
}

// Column sums of a staged W-wide BF16 tile over its 16*NW rows, on MFMA:
// with a B operand of ones, D[f][c] = sum over the rows of T[f][r] for every
// column c.  Wave w covers feature block(s) fb and 32-row chunks:
//   W/16 <= NW: fb = w % (W/16), chunks w / (W/16) + k * NW / (W/16);
//   W/16 >  NW: fb = w + a * NW (a < W/16/NW), every chunk.
// Lanes 0, 16, 32, 48 then hold features 16 fb + 4 (lane / 16) + v.
template <int W, int NW>
struct ColSum {
  static constexpr int FBN = W / 16, CH = NW / 2;  // feature blocks, 32-row chunks
  static constexpr int NA = FBN > NW ? FBN / NW : 1;
  static constexpr int WPF = FBN >= NW ? 1 : NW / FBN;  // waves per feature block
  static constexpr int CPW = CH / WPF;                  // chunks per wave
  static_assert(CPW >= 1 && CH % WPF == 0 && (FBN <= NW || FBN % NW == 0), "column-sum layout");
  v4f acc[NA];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  __device__ __forceinline__ void add(const void* __restrict__ tile, int wave, int lane) {
    constexpr int RS = Stg<true, 16 * NW>::RS;
    const v8bf ones = __builtin_bit_cast(v8bf, uint4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u});
    const int li = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int fb = FBN > NW ? wave + q * NW : wave % FBN;
      const int c0 = FBN >= NW ? 0 : wave / FBN;
      const __bf16* t = reinterpret_cast<const __bf16*>(tile) + (16 * fb + li) * RS + 8 * kk;
#pragma unroll
      for (int k = 0; k < CPW; ++k) {
        const v8bf a = *reinterpret_cast<const v8bf*>(t + 32 * (c0 + k * WPF));
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, ones, acc[q], 0, 0, 0);
      }
    }
  }
  // Sum the waves' partials in a fixed order and write the W sums to dst.
  // `scratch` holds at least WPF * W floats of LDS; contains barriers.
  __device__ __forceinline__ void store(float* __restrict__ scratch, float* __restrict__ dst, int wave,
                                        int lane) const {
    __syncthreads();
    if ((lane & 15) == 0) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int fb = FBN > NW ? wave + q * NW : wave % FBN;
        const int slot = FBN >= NW ? 0 : wave / FBN;
#pragma unroll
        for (int v = 0; v < 4; ++v) scratch[slot * W + 16 * fb + 4 * (lane >> 4) + v] = acc[q][v];
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < W) {
      float sum = 0.f;
      for (int sl = 0; sl < WPF; ++sl) sum += scratch[sl * W + threadIdx.x];
      dst[threadIdx.x] = sum;
    }
    __syncthreads();
  }
};

// The same column sums on the vector ALU (one float per thread instead of
// MFMA accumulators, for kernels short of registers): thread t adds the
// rows of segment t / W of feature t % W; store() adds the segments in order.
template <int W, int NW>
struct ColSumValu {
  static constexpr int ROWS = 16 * NW, RS = Stg<true, ROWS>::RS, NSEG = 64 * NW / W, LEN = ROWS / NSEG;
  static_assert(NSEG >= 1 && LEN % 8 == 0, "segment layout");
  float acc;
  __device__ __forceinline__ void zero() { acc = 0.f; }
  __device__ __forceinline__ void add(const void* __restrict__ tile, int, int) {
    const int f = threadIdx.x % W, sg = threadIdx.x / W;
    const __bf16* p = reinterpret_cast<const __bf16*>(tile) + f * RS + sg * LEN;
#pragma unroll
    for (int r = 0; r < LEN; r += 8) {
      const v8bf q = *reinterpret_cast<const v8bf*>(p + r);
#pragma unroll
      for (int c = 0; c < 8; ++c) acc += (float)q[c];
    }
  }
  __device__ __forceinline__ void store(float* __restrict__ scratch, float* __restrict__ dst, int, int) const {
    __syncthreads();
    scratch[threadIdx.x] = acc;
    __syncthreads();
    if ((int)threadIdx.x < W) {
      float sum = 0.f;
      for (int sg = 0; sg < NSEG; ++sg) sum += scratch[sg * W + threadIdx.x];
      dst[threadIdx.x] = sum;
    }
    __syncthreads();
  }
};

// Write the owned tiles into a row-major [frows][kcols] block of the slab
// (kcols <= AW and frows <= GW drop padded columns and rows).
template <int GW, int AW, int NW = kWaves>
__device__ __forceinline__ void dw_store(const v4f (&acc)[dw_tiles_per_wave<GW, AW, NW>()], float* __restrict__ dst,
                                         int kcols, int wave, int lane, int frows = GW) {
  constexpr int NT = dw_tiles_per_wave<GW, AW, NW>(), NTILE = (GW / 16) * (AW / 16), KBN = AW / 16;
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int t = wave + NW * n;
    if (t < NTILE) {
      const int fb = t / KBN, kb = t % KBN;
      const int k = 16 * kb + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int f = 16 * fb + 4 * (lane >> 4) + v;
        if (k < kcols && f < frows) dst[f * kcols + k] = acc[n][v];
      }
    }
  }
}

// Sum a per-lane row-block vector over all 16*NW rows of the workgroup (16
// lanes x NW waves) in a fixed order and write the W sums to dst.  Uses
// `scratch` (at least 16*NW*W floats of LDS); contains barriers.
template <int W, int NW = kWaves>
__device__ __forceinline__ void block_sum_vec(const float (&v)[W / 4], float* __restrict__ scratch,
                                              float* __restrict__ dst, int wave, int lane) {
  const int j = lane & 15, g = lane >> 4;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < W / 4; ++i) scratch[(wave * 16 + j) * W + 16 * (i / 4) + 4 * g + (i % 4)] = v[i];
  __syncthreads();
  for (int t = threadIdx.x; t < W; t += blockDim.x) {
    float s = 0.f;
    for (int r = 0; r < 16 * NW; ++r) s += scratch[r * W + t];
    dst[t] = s;
  }
  __syncthreads();
}

// The same for a vector reduced across each 16-lane group by sum16_scatter
// at H = 64 (one value per lane: lane j of group g holds feature
// 16 (j / 4) + 4 g + j % 4): the lanes' values of all waves are added in
// wave order.  Uses `scratch` (64 * NW floats of LDS); contains barriers.
template <int W, int NW = kWaves>
__device__ __forceinline__ void block_sum_scattered(float v, float* __restrict__ scratch, float* __restrict__ dst,
                                                    int wave, int lane) {
  static_assert(W == 64, "one feature per lane");
  __syncthreads();
  scratch[wave * 64 + lane] = v;
  __syncthreads();
  for (int t = threadIdx.x; t < W; t += blockDim.x) {
    const int l = (4 * (t / 16) + t % 4) + 16 * ((t % 16) / 4);
    float sum = 0.f;
    for (int w = 0; w < NW; ++w) sum += scratch[w * 64 + l];
    dst[t] = sum;
  }
  __syncthreads();
}

__device__ __forceinline__ void stage_frags(uint4* __restrict__ dst, const void* __restrict__ src, size_t bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  for (size_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) dst[i] = s[i];
}
// FP32 fragments in the rotated LDS layout (gemm_f32 / gemm_f32_tr with
// ROT): element o of 64-float chunk c at c*64 + (o + c%4) % 64.
__device__ __forceinline__ void stage_frags_rot(void* __restrict__ dst, const void* __restrict__ src, size_t bytes) {
  const float* s = reinterpret_cast<const float*>(src);
  float* d = reinterpret_cast<float*>(dst);
  for (size_t e = threadIdx.x; e < bytes / 4; e += blockDim.x) {
    const size_t c = e >> 6;
    d[(c << 6) + ((e + (c & 3)) & 63)] = s[e];
  }
}

// ----------------------------------------------------------- edge adjoint


template <int H, bool BF, int NWQ = 0>
struct EdgeBwdCfg {
  // Default: BF16 eight waves per workgroup (128 staged rows) so the
  // fragments are shared by more waves; FP32 (MFMA-bound) and H=128: four
  // waves.  NWQ (4 or 8) overrides it (a schedule dimension).
  static constexpr int NW = NWQ ? NWQ : ((BF && H <= 64) ? 8 : 4);
  static constexpr int ROWS = 16 * NW;
  // TP (FP32 at H = 64): two workgroups per CU, so two waves per SIMD (one
  // wave's memory and LDS waits and barriers are covered by the other
  // wave's work; FP32 matrix instructions do not issue beside VALU ones, so
  // the gain is in the waits): the weight-gradient factors are staged in
  // two rounds through one pair of tiles, only W1c and W2 sit in LDS (the
  // transposed products read them at transposed addresses), db2 is a
  // column sum of the staged gm tile and the LayerNorm-parameter sums are
  // reduced across the block's lanes (sum16_scatter) into one register per
  // lane, which brings the kernel to 245 VGPRs and 68 KB of LDS.  Measured on C4: 45.4 ->
  // 40.6 ms per launch (one wave per SIMD with the next block's rows
  // loaded ahead had given 47.7 -> 45.4); W1c / W2 in the rotated LDS
  // layout (stage_frags_rot, no bank conflicts in the transposed reads):
  // 40.1 -> 37.2 ms.
  static constexpr bool TP = !BF && H == 64;
  static constexpr int MINB = TP ? 2 : 1;
  // BF16: bias / LayerNorm gradients are column sums of staged tiles instead
  // of per-lane accumulators (frees registers); FP32 keeps them per lane.
  static constexpr bool VEC = BF;
  static constexpr int NTILES = TP ? 2 : (VEC ? 6 : 4);
  static constexpr int NFRAG = TP ? 2 : 4;
  static constexpr size_t FB = frag_bytes(H, H, BF);
  static constexpr size_t TB = tile_bytes<H, BF, ROWS>();
  static constexpr size_t STAGE = NTILES * TB;
  static constexpr bool LDS_FRAG = NFRAG * FB + STAGE <= kLdsLimit;
  static constexpr size_t VECS = 2 * H * sizeof(float);  // b2 and the LayerNorm gain
  static constexpr size_t CARRY = NW * H * sizeof(float);  // per-wave open-row sums between blocks
  static constexpr size_t LDS = STAGE + (LDS_FRAG ? NFRAG * FB : 0) + CARRY + VECS;
};

// The rows one 16-edge block of the edge adjoint reads: e_k, P_i, Q_j,
// g_a_i and g_e'_k (zero when absent); ES: e and g_e' stored as BF16.
template <int H, bool ES>
struct EdgeBwdRows {
  static constexpr int NF = H / 4;
  float ev[NF], u[NF], t[NF], gE[NF], go[NF];
  __device__ __forceinline__ void load(const EdgeBwdArgs& a, int64_t kk, int ri, int sj, int g) {
    load_row_t<H, ES>(a.e_in, kk, g, ev);
    load_row<H>(a.P + (int64_t)ri * H, g, u);
    load_row<H>(a.Q + (int64_t)sj * H, g, t);
    load_row<H>(a.g_a + (int64_t)ri * H, g, gE);
    if (a.g_e_out) {
      load_row_t<H, ES>(a.g_e_out, kk, g, go);
    } else {
#pragma unroll
      for (int i = 0; i < NF; ++i) go[i] = 0.f;
    }
  }
};

// Per edge k (receiver i, sender j), with the forward recomputed:
//   gE   = g_e_out[k] + g_a[i] / d_k         (adjoint of Eq. 4b plus the
//                                             gradient reaching e' directly)
//   gm   = LayerNorm adjoint of gE; db2 += gm; dW2 += gm u^T
//   gh   = (W2^T gm) * ELU'(h);   dW1c += gh e^T
//   g_e  = gE + W1c^T gh                     (residual + first Linear)
//   g_P[i] = sum of gh over i's incoming edges (segmented scan, as forward)
//   g_h[k] = gh, summed per sender by k_gq through the reverse edges.
// AM: the forward aggregated the MLP output, so the residual path carries
// only the next layer's gradient (not Eq. 4b's).
// ES: edge states and their gradients (e, g_e', g_e) stored as BF16.
template <int H, bool BF, bool AM, int NWQ, bool ES>
__global__ __launch_bounds__((64 * EdgeBwdCfg<H, BF, NWQ>::NW), (EdgeBwdCfg<H, BF, NWQ>::MINB)) void k_edge_bwd(EdgeBwdArgs a) {
  using C = EdgeBwdCfg<H, BF, NWQ>;
  constexpr int NF = H / 4, MB = H / 16, NW = C::NW, ROWS = C::ROWS, NT = dw_tiles_per_wave<H, H, NW>();
  constexpr bool TP = C::TP;
  extern __shared__ uint4 smem[];
  char* tG2 = reinterpret_cast<char*>(smem);
  char* tA2 = tG2 + C::TB;
  char* tG1 = TP ? tG2 : tA2 + C::TB;   // TP: the second round reuses the first round's tiles
  char* tA1 = TP ? tA2 : tG1 + C::TB;
  char* tGE = tA1 + C::TB;   // VEC: gE and gE * LN-normalised m, for dbeta / dgamma
  char* tGM = tGE + C::TB;
  const char* fr;
  // TP's transposed products read W1c / W2 in the rotated layout
  constexpr bool ROT = TP && C::LDS_FRAG;
  if constexpr (C::LDS_FRAG) {
    uint4* fl = smem + C::STAGE / 16;
    if constexpr (ROT)
      stage_frags_rot(fl, a.frag, C::NFRAG * C::FB);
    else
      stage_frags(fl, a.frag, C::NFRAG * C::FB);
    fr = reinterpret_cast<const char*>(fl);
  } else {
    fr = reinterpret_cast<const char*>(a.frag);
  }
  float* vecs = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + C::LDS - C::VECS);
  // the open row's partial g_P sum, handed from lane 15 of one block to lane
  // 0 of the next through LDS (same wave, so no barrier is needed)
  float* carry = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + C::LDS - C::VECS - C::CARRY) +
                 (threadIdx.x / 64) * H + (threadIdx.x / 16 % 4) * (H / 4);
  for (int t = threadIdx.x; t < 2 * H; t += blockDim.x) vecs[t] = t < H ? a.b2[t] : (a.ln ? a.lng[t - H] : 0.f);
  __syncthreads();

  const DevGraph& gr = a.g;
  const int lane = lane_id(), j = lane & 15, g = lane >> 4, wave = threadIdx.x / 64;
  const TileSched ts = tile_sched(gr.n_tiles);
  v4f acc2[NT], acc1[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n) acc2[n] = acc1[n] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int NV = (C::VEC || TP) ? 1 : NF;  // per-lane vector accumulators (FP32 path)
  float db2[NV], dga[NV], dbe[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) db2[i] = dga[i] = dbe[i] = 0.f;
  ColSum<H, NW> cs_b2, cs_ga, cs_be;  // BF16: MFMA column sums of the staged tiles
  cs_b2.zero();
  cs_ga.zero();
  cs_be.zero();

  // groups of NW consecutive tiles, one per wave, processed in lock step
  for (int64_t tg = ts.t0 + ts.rank * NW; tg < ts.t1; tg += ts.nr * NW) {
    // Tile bounds, clamped to the range end (a wave past it gets an empty
    // tile); all loads are independent so they share one round trip.
    const int64_t tile = tg + wave;
    const int64_t tc0 = std::min<int64_t>(tile, ts.t1), tc1 = std::min<int64_t>(tile + 1, ts.t1);
    const int64_t r0 = gr.tile_r[tc0], r1 = gr.tile_r[tc1];
    const int64_t e0 = gr.tile_e[tc0], e1 = gr.tile_e[tc1];
    // lock-step trip count: the most 16-edge blocks of any tile of the
    // group; lane w < NW reads the bounds of tile tg + w
    const int wl = lane < NW ? lane : 0;
    const int32_t eb0 = gr.tile_e[std::min<int64_t>(tg + wl, ts.t1)];
    const int32_t eb1 = gr.tile_e[std::min<int64_t>(tg + wl + 1, ts.t1)];
    int nb = lane < NW ? (eb1 - eb0 + 15) / 16 : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) nb = std::max(nb, __shfl_xor(nb, off));
    const int64_t n_iter = __builtin_amdgcn_readfirstlane(nb);  // the same in every lane and wave
    int carry_key = 0;  // no open row at the start of a tile

    // Index loads run one block ahead, so each block waits on a single
    // round trip to memory (its rows), not on indices and then rows.
    const int64_t e_last = e1 > e0 ? e1 - 1 : 0;  // in-bounds stand-in for absent edges
    int ri_n, sj_n, md_n, nx_n;
    {
      const int64_t k = e0 + j, kk = k < e1 ? k : e_last;
      ri_n = gr.recv[kk];
      sj_n = gr.col[kk];
      md_n = gr.mult[kk];
      nx_n = (k + 1 < e1) ? gr.recv[k + 1] : -1;
      // complete these loads here, so that the loop's entry state holds no
      // pending loads (else the compiler's wait at the loop head, merged
      // with the back edge, also drains the previous block's stores)
      asm volatile("" : "+v"(ri_n), "+v"(sj_n), "+v"(md_n), "+v"(nx_n));
    }

    for (int64_t it = 0; it < n_iter; ++it) {
      const char* frb = fr + opaque_zero();  // re-read the fragments each block
      const char* fW1c = frb;
      const char* fW2 = frb + C::FB;
      const char* fW2t = frb + 2 * C::FB;
      const char* fW1ct = frb + 3 * C::FB;
      const int srow = wave * 16 + j;
      const int64_t k = e0 + it * 16 + j;
      const bool valid = k < e1;
      const int64_t kk = valid ? k : e_last;
      const int ri = ri_n;
      const int sj = sj_n;
      const float inv_d = 1.f / (float)md_n;
      const int next = nx_n;
      const bool last = valid && next != ri;
      const int key = valid ? ri + 1 : -1;

      // next block's indices first (the only loads issued before this
      // block's stores that the next block waits on), then every row this
      // block reads, issued together
      {
        const int64_t k2 = k + 16, kk2 = k2 < e1 ? k2 : e_last;
        ri_n = gr.recv[kk2];
        sj_n = gr.col[kk2];
        md_n = gr.mult[kk2];
        nx_n = (k2 + 1 < e1) ? gr.recv[k2 + 1] : -1;
      }
      EdgeBwdRows<H, ES> cur;
      cur.load(a, kk, ri, sj, g);
      float (&ev)[NF] = cur.ev;
      float (&u)[NF] = cur.u;
      float (&t)[NF] = cur.t;
      float (&gE)[NF] = cur.gE;
      float (&go)[NF] = cur.go;
      __builtin_amdgcn_sched_barrier(0);  // all row loads issue before any use

      // recompute the forward
#pragma unroll
      for (int i = 0; i < NF; ++i) u[i] += t[i];
      gemm<BF, MB, MB, ROT>(fW1c, ev, u, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) u[i] = elu(u[i]);
      float mp[NF];
      const float* vb = vecs + opaque_zero();
      load_vec<H>(vb, g, mp);
      gemm<BF, MB, MB, ROT>(fW2, u, mp, lane);

      // gradient reaching e'
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const float v = gE[i] * inv_d + go[i];
        gE[i] = valid ? v : 0.f;
      }
      // LayerNorm adjoint (mp becomes the pre-LN gradient gm)
      if (a.ln) {
        float mean, rstd, gam[NF];
        ln_stats<H>(mp, a.eps, mean, rstd);
        load_vec<H>(vb + H, g, gam);
        float s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          const float xh = (mp[i] - mean) * rstd;
          if constexpr (!C::VEC && !TP) {
            dga[i] += gE[i] * xh;
            dbe[i] += gE[i];
          } else {
            t[i] = gE[i] * xh;
          }
          const float gx = gE[i] * gam[i];
          s1 += gx;
          s2 += gx * xh;
          mp[i] = xh;
        }
        if constexpr (C::VEC) {
          stage_row<H, BF, ROWS>(tGE, srow, g, gE);
          stage_row<H, BF, ROWS>(tGM, srow, g, t);
        }
        if constexpr (TP) {  // dbeta += sum of gE, dgamma += sum of gE * x^ over the block's rows
          float rs[1];
          sum16_scatter<NF>(gE, rs, j);
          dbe[0] += rs[0];
          sum16_scatter<NF>(t, rs, j);
          dga[0] += rs[0];
        }
        s1 = row_sum(s1) * (1.f / H);
        s2 = row_sum(s2) * (1.f / H);
        // rstd (gE gam - s1 - x^ s2) as two multiply-adds per feature
        const float c1 = -rstd * s1, c2 = -rstd * s2;
#pragma unroll
        for (int i = 0; i < NF; ++i) mp[i] = fmaf(mp[i], c2, fmaf(gE[i] * gam[i], rstd, c1));
      } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) mp[i] = gE[i];
      }
      if constexpr (TP) {
        // db2: column sums of the staged gm tile after the first barrier
      } else if constexpr (!C::VEC) {
#pragma unroll
        for (int i = 0; i < NF; ++i) db2[i] += mp[i];
      }
      stage_row<H, BF, ROWS>(tG2, srow, g, mp);
      stage_row<H, BF, ROWS>(tA2, srow, g, u);
      // gh = (W2^T gm) * ELU'(h); ELU'(h) = 1 for h > 0 else exp(h) = u + 1
#pragma unroll
      for (int i = 0; i < NF; ++i) t[i] = 0.f;
      if constexpr (TP)
        gemm_f32_tr<H, ROT>(reinterpret_cast<const float*>(fW2), mp, t, lane);
      else
        gemm<BF, MB, MB>(fW2t, mp, t, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) t[i] *= elu_deriv_from_value(u[i]);
      if constexpr (!TP) {
        stage_row<H, BF, ROWS>(tG1, srow, g, t);
        stage_row<H, BF, ROWS>(tA1, srow, g, ev);
      }
      if constexpr (AM) {
        if (a.g_e_out) {
          load_row_t<H, ES>(a.g_e_out, kk, g, gE);
        } else {
#pragma unroll
          for (int i = 0; i < NF; ++i) gE[i] = 0.f;
        }
      }
      // g_e = gE + W1c^T gh
      if constexpr (TP)
        gemm_f32_tr<H, ROT>(reinterpret_cast<const float*>(fW1c), t, gE, lane);
      else
        gemm<BF, MB, MB>(fW1ct, t, gE, lane);
      if (valid) {
        store_row_t<H, ES>(a.g_e_in, k, g, gE);
        if constexpr (BF)
          store_row_bf16<H>(reinterpret_cast<__bf16*>(a.g_h) + k * H, g, t);
        else
          store_row<H>(reinterpret_cast<float*>(a.g_h) + k * H, g, t);
      }
      if constexpr (TP) {
        // round 1: dW2 and db2 from the staged (gm, u); then the same tiles
        // take (gh, e).  db2: lane = feature (H = 64), wave w adds the staged
        // rows 16w .. 16w+15 (four 16-byte LDS reads, conflict-free).
        __syncthreads();
        dw_tiles<H, H, BF, NW>(tG2, tA2, acc2, wave, lane);
        {
          const float* col = reinterpret_cast<const float*>(tG2) + lane * Stg<BF, ROWS>::RS + 16 * wave;
          float s = 0.f;
#pragma unroll
          for (int r = 0; r < 16; r += 4) {
            const float4 q = *reinterpret_cast<const float4*>(col + r);
            s += ((q.x + q.y) + q.z) + q.w;
          }
          db2[0] += s;
        }
        __syncthreads();
        stage_row<H, BF, ROWS>(tG1, srow, g, t);
        stage_row<H, BF, ROWS>(tA1, srow, g, ev);
      }
      // g_P: segmented sum of gh per receiver.  Lanes past the tile's last
      // edge hold gh = 0 (their gE is zeroed, so are gm and W2^T gm) and a
      // key of their own, so they add nothing to any row's sum.
      if (j == 0 && key == carry_key) {
#pragma unroll
        for (int i = 0; i < NF; i += 4) {
          const float4 c = *reinterpret_cast<const float4*>(carry + i);
          t[i] += c.x;
          t[i + 1] += c.y;
          t[i + 2] += c.z;
          t[i + 3] += c.w;
        }
      }
      seg_scan16<NF>(t, key);
      if (last) store_row<H>(a.g_P + (int64_t)ri * H, g, t);
      if (j == 15) {
#pragma unroll
        for (int i = 0; i < NF; i += 4) *reinterpret_cast<float4*>(carry + i) = make_float4(t[i], t[i + 1], t[i + 2], t[i + 3]);
      }
      carry_key = from_prev_lane_i(key);

      __syncthreads();
      if constexpr (!TP) dw_tiles<H, H, BF, NW>(tG2, tA2, acc2, wave, lane);
      dw_tiles<H, H, BF, NW>(tG1, tA1, acc1, wave, lane);
      if constexpr (C::VEC) {
        cs_b2.add(tG2, wave, lane);
        if (a.ln) {
          cs_be.add(tGE, wave, lane);
          cs_ga.add(tGM, wave, lane);
        }
      }
      __syncthreads();
    }
    for (int64_t r = r0 + (lane >> 2); r < r1; r += 16) {
      if (gr.rowptr[r] == gr.rowptr[r + 1]) {
        float* dst = a.g_P + r * H;
        for (int c = (lane & 3) * 4; c < H; c += 16) *reinterpret_cast<float4*>(dst + c) = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }
  float* slab = a.part + blockIdx.x * a.slab;
  dw_store<H, H, NW>(acc1, slab, H, wave, lane);
  dw_store<H, H, NW>(acc2, slab + H * H, H, wave, lane);
  float* scratch = reinterpret_cast<float*>(tG2);
  if constexpr (C::VEC) {
    cs_b2.store(scratch, slab + 2 * H * H, wave, lane);
    cs_ga.store(scratch, slab + 2 * H * H + H, wave, lane);
    cs_be.store(scratch, slab + 2 * H * H + 2 * H, wave, lane);
  } else if constexpr (TP) {
    // db2: lane l holds feature l (column sums of the staged gm); dgamma,
    // dbeta: lane j of group g holds feature 16 (j / 4) + 4 g + j % 4 (H =
    // 64: one value per lane after the reduce-scatter); waves added in order
    __syncthreads();
    scratch[(wave * 64 + lane) * 3 + 0] = db2[0];
    scratch[(wave * 64 + lane) * 3 + 1] = dga[0];
    scratch[(wave * 64 + lane) * 3 + 2] = dbe[0];
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * H; t += blockDim.x) {
      const int v = t / H, f = t % H;
      const int l = v == 0 ? f : (4 * (f / 16) + f % 4) + 16 * ((f % 16) / 4);
      float sum = 0.f;
      for (int w = 0; w < NW; ++w) sum += scratch[(w * 64 + l) * 3 + v];
      slab[2 * H * H + v * H + f] = sum;
    }
  } else {
    block_sum_vec<H>(db2, scratch, slab + 2 * H * H, wave, lane);
    block_sum_vec<H>(dga, scratch, slab + 2 * H * H + H, wave, lane);
    block_sum_vec<H>(dbe, scratch, slab + 2 * H * H + 2 * H, wave, lane);
  }
}

template <int H, bool BF, bool AM, int NWQ, bool ES>
static hipError_t launch_edge_bwd_es(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  using C = EdgeBwdCfg<H, BF, NWQ>;
  (void)hipFuncSetAttribute((const void*)k_edge_bwd<H, BF, AM, NWQ, ES>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)C::LDS);
  hipLaunchKernelGGL((k_edge_bwd<H, BF, AM, NWQ, ES>), dim3(grid), dim3(64 * C::NW), C::LDS, s, a);
  return hipGetLastError();
}
template <int H, bool BF, bool AM, int NWQ>
static hipError_t launch_edge_bwd_am(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  if constexpr (BF) {
    if (a.es) return launch_edge_bwd_es<H, BF, AM, NWQ, true>(a, grid, s);
  }
  return launch_edge_bwd_es<H, BF, AM, NWQ, false>(a, grid, s);
}
// Waves per workgroup: the default, or 4 (any width and type), or 8 (the
// BF16 kernel at H <= 64, whose default it is); the C ABI validates it.
template <int H, bool BF>
static hipError_t launch_edge_bwd_t(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  if constexpr (BF && H <= 64) {
    if (a.waves == 4)
      return a.am ? launch_edge_bwd_am<H, BF, true, 4>(a, grid, s) : launch_edge_bwd_am<H, BF, false, 4>(a, grid, s);
  }
  return a.am ? launch_edge_bwd_am<H, BF, true, 0>(a, grid, s) : launch_edge_bwd_am<H, BF, false, 0>(a, grid, s);
}

hipError_t launch_edge_bwd(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  if (a.es && !a.bf) return hipErrorInvalidValue;
#define MP_CASE(HH) \
  if (a.H == HH) return a.bf ? launch_edge_bwd_t<HH, true>(a, grid, s) : launch_edge_bwd_t<HH, false>(a, grid, s);
  MP_CASE(32) MP_CASE(64) MP_CASE(128)
#undef MP_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------------- split edge adjoint (wide H)


template <int H, bool BF, int NWQ>
struct EdgeBwdSplitCfg {
  // NWQ independent waves sharing the LDS weight fragments: 8 (two per
  // SIMD, 256 registers each), or 4 (one per SIMD with up to 512: the
  // per-edge adjoint at H = 128 wants about 320, and at 256 the compiler
  // spills).  Measured on C3 (one launch, same box): BF16 7.30 ms at 8
  // waves, 7.04 at 4; FP32, whose products keep the matrix unit busy, 14.3
  // at 8 and 15.6 at 4.
  static_assert(NWQ == 4 || NWQ == 8, "4 or 8 waves per workgroup");
  static constexpr int NW = NWQ;
  static constexpr size_t FB = frag_bytes(H, H, BF);
  // BF16 keeps W1c, W2, W2^T, W1c^T; FP32 only W1c and W2 (the transposed
  // products read them at transposed addresses, gemm_f32_tr)
  static constexpr int NFR = BF ? 4 : 2;
  static constexpr size_t VECS = 2 * H * sizeof(float);
  static constexpr size_t CARRY = NW * H * sizeof(float);
  // per-lane LayerNorm-parameter sums of every wave, added up at the end
  static constexpr int NS = H / 64;  // values per lane after the 16-lane reduce-scatter
  static constexpr size_t RED = NW * 64 * 2 * NS * sizeof(float);
  static constexpr bool LDS_FRAG = NFR * FB + VECS + CARRY + RED <= kLdsLimit;
  static constexpr size_t RED_OFF = LDS_FRAG ? NFR * FB : 0;
  static constexpr size_t LDS = RED_OFF + RED + CARRY + VECS;
};

// The edge adjoint without its matrix weight gradients, for widths where
// the fused kernel's staging tiles and accumulators do not fit next to the
// weights.  Per edge it computes what k_edge_bwd computes (g_e, g_h, the
// segmented g_P) and writes the factors of the weight gradients instead of
// accumulating them: gm and u (dW2 = sum gm u^T, db2 = sum gm); dW1c =
// sum g_h e^T is formed from g_h and e.  The LayerNorm-parameter gradients
// (dbeta = sum gE, dgamma = sum gE * normalised m) are summed here: each
// block's 16 rows are reduced across lanes (sum16_scatter, so a lane keeps
// H/64 features), accumulated per lane, and the waves' sums are added in
// wave order into the workgroup's slab at the end.  Waves walk their tiles
// independently (no barriers in the loop).
template <int H, bool BF, bool AM, bool ES, int NWQ>
__global__ __launch_bounds__((64 * EdgeBwdSplitCfg<H, BF, NWQ>::NW)) void k_edge_bwd_split(EdgeBwdArgs a) {
  using C = EdgeBwdSplitCfg<H, BF, NWQ>;
  constexpr int NF = H / 4, MB = H / 16, NW = C::NW;
  // FP32: the transposed products read W1c / W2 in the rotated layout
  constexpr bool ROT = !BF && C::LDS_FRAG;
  extern __shared__ uint4 smem[];
  const char* fr;
  if constexpr (C::LDS_FRAG) {
    if constexpr (ROT)
      stage_frags_rot(smem, a.frag, C::NFR * C::FB);
    else
      stage_frags(smem, a.frag, C::NFR * C::FB);
    fr = reinterpret_cast<const char*>(smem);
  } else {
    fr = reinterpret_cast<const char*>(a.frag);
  }
  float* vecs = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + C::LDS - C::VECS);
  float* carry = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + C::LDS - C::VECS - C::CARRY) +
                 (threadIdx.x / 64) * H + (threadIdx.x / 16 % 4) * (H / 4);
  for (int t = threadIdx.x; t < 2 * H; t += blockDim.x) vecs[t] = t < H ? a.b2[t] : (a.ln ? a.lng[t - H] : 0.f);
  __syncthreads();

  const DevGraph& gr = a.g;
  const int lane = lane_id(), j = lane & 15, g0 = lane >> 4, wave = threadIdx.x / 64;
  const TileSched ts = tile_sched(gr.n_tiles);
  constexpr int NS = C::NS;
  float sbe[NS], sga[NS];  // this lane's share of dbeta, dgamma
#pragma unroll
  for (int c = 0; c < NS; ++c) sbe[c] = sga[c] = 0.f;
  for (int64_t tile = ts.t0 + ts.rank * NW + wave; tile < ts.t1; tile += ts.nr * NW) {
    const int64_t r0 = gr.tile_r[tile], r1 = gr.tile_r[tile + 1];
    const int64_t e0 = gr.tile_e[tile], e1 = gr.tile_e[tile + 1];
    int carry_key = 0;  // no open row at the start of a tile
    const int64_t e_last = e1 > e0 ? e1 - 1 : 0;
    int ri_n, sj_n, md_n, nx_n;  // next block's indices, one block ahead
    {
      const int64_t k = e0 + j, kk = k < e1 ? k : e_last;
      ri_n = gr.recv[kk];
      sj_n = gr.col[kk];
      md_n = gr.mult[kk];
      nx_n = (k + 1 < e1) ? gr.recv[k + 1] : -1;
      asm volatile("" : "+v"(ri_n), "+v"(sj_n), "+v"(md_n), "+v"(nx_n));
    }
    for (int64_t base = e0; base < e1; base += 16) {
      const char* frb = fr + opaque_zero();
      const char* fW1c = frb;
      const char* fW2 = frb + C::FB;
      const char* fW2t = frb + 2 * C::FB;
      const char* fW1ct = frb + 3 * C::FB;
      const int64_t k = base + j;
      const bool valid = k < e1;
      const int64_t kk = valid ? k : e_last;
      const int ri = ri_n, sj = sj_n;
      // the lane's feature offset, recomputed per block: hoisted out of the
      // loop, every array's 64-bit base plus offset would be held in
      // registers (at eight waves they spilled, and their reloads
      // serialised the block's row loads; C3: BF16 7.9 -> 7.3 ms, FP32
      // 14.8 -> 14.3 ms per launch at eight waves)
      const int g = g0 + opaque_zero();
      const float inv_d = 1.f / (float)md_n;
      const bool last = valid && nx_n != ri;
      const int key = valid ? ri + 1 : -1;
      {
        const int64_t k2 = k + 16, kk2 = k2 < e1 ? k2 : e_last;
        ri_n = gr.recv[kk2];
        sj_n = gr.col[kk2];
        md_n = gr.mult[kk2];
        nx_n = (k2 + 1 < e1) ? gr.recv[k2 + 1] : -1;
      }
      float ev[NF], u[NF], t[NF], gE[NF];
      load_row_t<H, ES>(a.e_in, kk, g, ev);
      load_row<H>(a.P + (int64_t)ri * H, g, u);
      load_row<H>(a.Q + (int64_t)sj * H, g, t);
      load_row<H>(a.g_a + (int64_t)ri * H, g, gE);
      __builtin_amdgcn_sched_barrier(0);
      // recompute the forward
#pragma unroll
      for (int i = 0; i < NF; ++i) u[i] += t[i];
      gemm<BF, MB, MB, ROT>(fW1c, ev, u, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) u[i] = elu(u[i]);
      if (valid) store_row_t<H, BF>(a.u, k, g, u);
      float mp[NF];
      const float* vb = vecs + opaque_zero();
      load_vec<H>(vb, g, mp);
      gemm<BF, MB, MB, ROT>(fW2, u, mp, lane);
      // gradient reaching e'
      if (a.g_e_out) {
        load_row_t<H, ES>(a.g_e_out, kk, g, t);
#pragma unroll
        for (int i = 0; i < NF; ++i) gE[i] = gE[i] * inv_d + t[i];
      } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) gE[i] *= inv_d;
      }
#pragma unroll
      for (int i = 0; i < NF; ++i) gE[i] = valid ? gE[i] : 0.f;
      if (a.ln) {
        float mean, rstd, gam[NF];
        ln_stats<H>(mp, a.eps, mean, rstd);
        load_vec<H>(vb + H, g, gam);
        float s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          const float xh = (mp[i] - mean) * rstd;
          t[i] = gE[i] * xh;
          const float gx = gE[i] * gam[i];
          s1 += gx;
          s2 += gx * xh;
          mp[i] = xh;
        }
        {
          float rs[NS];  // gE and t are zero on lanes past the tile's last edge
          sum16_scatter<NF>(gE, rs, j);
#pragma unroll
          for (int c = 0; c < NS; ++c) sbe[c] += rs[c];
          sum16_scatter<NF>(t, rs, j);
#pragma unroll
          for (int c = 0; c < NS; ++c) sga[c] += rs[c];
        }
        s1 = row_sum(s1) * (1.f / H);
        s2 = row_sum(s2) * (1.f / H);
        // rstd (gE gam - s1 - x^ s2) as two multiply-adds per feature
        const float c1 = -rstd * s1, c2 = -rstd * s2;
#pragma unroll
        for (int i = 0; i < NF; ++i) mp[i] = fmaf(mp[i], c2, fmaf(gE[i] * gam[i], rstd, c1));
      } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) mp[i] = gE[i];
      }
      if (valid) store_row_t<H, BF>(a.gm, k, g, mp);
      // gh = (W2^T gm) * ELU'(h); ELU'(h) = 1 for h > 0 else exp(h) = u + 1
#pragma unroll
      for (int i = 0; i < NF; ++i) t[i] = 0.f;
      if constexpr (!BF && C::LDS_FRAG)
        gemm_f32_tr<H, ROT>(reinterpret_cast<const float*>(fW2), mp, t, lane);
      else
        gemm<BF, MB, MB>(fW2t, mp, t, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) t[i] *= elu_deriv_from_value(u[i]);
      if constexpr (AM) {  // residual path: the next layer's gradient only
        if (a.g_e_out) {
          load_row_t<H, ES>(a.g_e_out, kk, g, gE);
        } else {
#pragma unroll
          for (int i = 0; i < NF; ++i) gE[i] = 0.f;
        }
      }
      // g_e = gE + W1c^T gh
      if constexpr (!BF && C::LDS_FRAG)
        gemm_f32_tr<H, ROT>(reinterpret_cast<const float*>(fW1c), t, gE, lane);
      else
        gemm<BF, MB, MB>(fW1ct, t, gE, lane);
      if (valid) {
        store_row_t<H, ES>(a.g_e_in, k, g, gE);
        store_row_t<H, BF>(a.g_h, k, g, t);
      }
      // g_P: segmented sum of gh per receiver (carry through LDS); lanes
      // past the tile's last edge hold gh = 0 (gE zeroed) and a key of their own
      if (j == 0 && key == carry_key) {
#pragma unroll
        for (int i = 0; i < NF; i += 4) {
          const float4 c = *reinterpret_cast<const float4*>(carry + i);
          t[i] += c.x;
          t[i + 1] += c.y;
          t[i + 2] += c.z;
          t[i + 3] += c.w;
        }
      }
      seg_scan16<NF>(t, key);
      if (last) store_row<H>(a.g_P + (int64_t)ri * H, g, t);
      if (j == 15) {
#pragma unroll
        for (int i = 0; i < NF; i += 4) *reinterpret_cast<float4*>(carry + i) = make_float4(t[i], t[i + 1], t[i + 2], t[i + 3]);
      }
      carry_key = from_prev_lane_i(key);
    }
    for (int64_t r = r0 + (lane >> 2); r < r1; r += 16) {
      if (gr.rowptr[r] == gr.rowptr[r + 1]) {
        float* dst = a.g_P + r * H;
        for (int c = (lane & 3) * 4; c < H; c += 16) *reinterpret_cast<float4*>(dst + c) = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }
  if (a.ln) {
    // lane j of group g holds value indices q = j*NS + c of the row-block
    // layout, i.e. feature 16 (q / 4) + 4 g + q % 4; add the waves in order
    float* red = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + C::RED_OFF);
#pragma unroll
    for (int c = 0; c < NS; ++c) {
      red[((wave * 64 + lane) * 2 + 0) * NS + c] = sbe[c];
      red[((wave * 64 + lane) * 2 + 1) * NS + c] = sga[c];
    }
    __syncthreads();
    float* slab = a.part + blockIdx.x * a.slab;
    for (int t = threadIdx.x; t < 2 * H; t += blockDim.x) {
      const int v = t / H, f = t % H;
      const int q = 4 * (f / 16) + f % 4, gg = (f % 16) / 4;
      const int l = q / NS + 16 * gg, c = q % NS;
      float sum = 0.f;
      for (int w = 0; w < NW; ++w) sum += red[((w * 64 + l) * 2 + v) * NS + c];
      slab[(v == 0 ? 2 * (int64_t)H * H + 2 * H : 2 * (int64_t)H * H + H) + f] = sum;  // dbeta, dgamma
    }
  }
}

template <int H, bool BF, bool AM, bool ES, int NWQ>
static hipError_t launch_edge_bwd_split_es(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  using C = EdgeBwdSplitCfg<H, BF, NWQ>;
  (void)hipFuncSetAttribute((const void*)k_edge_bwd_split<H, BF, AM, ES, NWQ>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
  hipLaunchKernelGGL((k_edge_bwd_split<H, BF, AM, ES, NWQ>), dim3(grid), dim3(64 * C::NW), C::LDS, s, a);
  return hipGetLastError();
}
template <int H, bool BF, bool AM, int NWQ>
static hipError_t launch_edge_bwd_split_am(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  if constexpr (BF) {
    if (a.es) return launch_edge_bwd_split_es<H, BF, AM, true, NWQ>(a, grid, s);
  }
  return launch_edge_bwd_split_es<H, BF, AM, false, NWQ>(a, grid, s);
}

// Waves per workgroup: 4 or 8; the default is 4 with BF16 GEMMs and 8 in
// FP32 (the C ABI validates the field).
template <int H, bool BF>
static hipError_t launch_edge_bwd_split_t(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  const int nw = a.waves ? a.waves : (BF ? 4 : 8);
  if (nw == 4)
    return a.am ? launch_edge_bwd_split_am<H, BF, true, 4>(a, grid, s) : launch_edge_bwd_split_am<H, BF, false, 4>(a, grid, s);
  return a.am ? launch_edge_bwd_split_am<H, BF, true, 8>(a, grid, s) : launch_edge_bwd_split_am<H, BF, false, 8>(a, grid, s);
}

hipError_t launch_edge_bwd_split(const EdgeBwdArgs& a, int grid, hipStream_t s) {
  if (a.es && !a.bf) return hipErrorInvalidValue;
  if (a.H == 128) return a.bf ? launch_edge_bwd_split_t<128, true>(a, grid, s) : launch_edge_bwd_split_t<128, false>(a, grid, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------- weight gradients from row pairs

template <int GW, int AW, bool BF>
struct RowDwCfg {
  static constexpr int NW = BF ? 8 : 4;
  static constexpr int ROWS = 16 * NW;
  static constexpr size_t TG = tile_bytes<GW, BF, ROWS>(), TA = tile_bytes<AW, BF, ROWS>();
  // the column-sum scratch (FP32 path: 16 NW x GW floats) reuses the A tile
  static constexpr size_t LDS = TG + TA;
  static_assert(BF || TA >= 16 * NW * GW * sizeof(float), "column-sum scratch");
};

// dst[GW][AW] = sum over rows of G[r] (x) A[r], lock-step waves staging
// 16-row blocks in LDS as the fused kernels do (same rounding of the
// operands to BF16 on the BF16 path); column sums of G from the staged tile.
// A2: the A row is the concatenation [A[r], A2[r]] of two AW/2-wide rows.
template <int GW, int AW, bool BF, bool GBF, bool ABF, bool A2>
__global__ __launch_bounds__((64 * RowDwCfg<GW, AW, BF>::NW)) void k_row_dw(RowDwArgs a) {
  using C = RowDwCfg<GW, AW, BF>;
  constexpr int NW = C::NW, ROWS = C::ROWS, NT = dw_tiles_per_wave<GW, AW, NW>();
  extern __shared__ uint4 smem[];
  char* tG = reinterpret_cast<char*>(smem);
  char* tA = tG + C::TG;
  const int lane = lane_id(), j = lane & 15, g = lane >> 4, wave = threadIdx.x / 64;
  const int srow = wave * 16 + j;
  const int64_t n = a.n_rows, nblk = (n + 15) / 16;
  const int64_t per = (nblk + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = blockIdx.x * per, b1 = std::min(nblk, b0 + per);
  const int64_t n_iter = (b1 - b0 + NW - 1) / NW;
  v4f acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  ColSum<GW, NW> cs;  // BF16 tiles
  cs.zero();
  float csf[GW / 4];  // FP32 tiles: per-lane sums
#pragma unroll
  for (int i = 0; i < GW / 4; ++i) csf[i] = 0.f;
  const bool want_cs = a.colsum_off >= 0;
  // one block ahead
  float gn[GW / 4], an[AW / 4];
  auto load_a = [&](int64_t row) {
    if constexpr (A2) {  // the two halves land directly in an[0, AW/8) and an[AW/8, AW/4)
      load_row_t<AW / 2, ABF>(a.A, row, g, *reinterpret_cast<float(*)[AW / 8]>(an));
      load_row_t<AW / 2, ABF>(a.A2, row, g, *reinterpret_cast<float(*)[AW / 8]>(an + AW / 8));
    } else {
      load_row_t<AW, ABF>(a.A, row, g, an);
    }
  };
  {
    const int64_t row = std::min<int64_t>((b0 + wave) * 16 + j, n - 1);
    load_row_t<GW, GBF>(a.G, row, g, gn);
    load_a(row);
#pragma unroll
    for (int i = 0; i < GW / 4; ++i) asm volatile("" : "+v"(gn[i]));
#pragma unroll
    for (int i = 0; i < AW / 4; ++i) asm volatile("" : "+v"(an[i]));
  }
  for (int64_t it = 0; it < n_iter; ++it) {
    const int64_t bk = b0 + it * NW + wave;
    const int64_t row = bk * 16 + j;
    const bool valid = bk < b1 && row < n;
    // stage this block's rows, then reuse their registers for the next
    // block's loads (their latency overlaps the barrier and the products)
#pragma unroll
    for (int i = 0; i < GW / 4; ++i) gn[i] = valid ? gn[i] : 0.f;
    if constexpr (!BF) {
#pragma unroll
      for (int i = 0; i < GW / 4; ++i) csf[i] += gn[i];
    }
    stage_row<GW, BF, ROWS>(tG, srow, g, gn);
    stage_row<AW, BF, ROWS>(tA, srow, g, an);
    {
      const int64_t bk2 = bk + NW, row2 = std::min<int64_t>(bk2 * 16 + j, n - 1);
      load_row_t<GW, GBF>(a.G, row2, g, gn);
      load_a(row2);
    }
    __syncthreads();
    dw_tiles<GW, AW, BF, NW>(tG, tA, acc, wave, lane);
    if constexpr (BF) {
      if (want_cs) cs.add(tG, wave, lane);
    }
    __syncthreads();
  }
  float* slab = a.part + blockIdx.x * a.slab;
  dw_store<GW, AW, NW>(acc, slab + a.off, AW, wave, lane);
  if (want_cs) {
    float* scratch = reinterpret_cast<float*>(tA);
    if constexpr (BF)
      cs.store(scratch, slab + a.colsum_off, wave, lane);
    else
      block_sum_vec<GW, NW>(csf, scratch, slab + a.colsum_off, wave, lane);
  }
}

template <int GW, int AW, bool BF, bool GBF, bool ABF, bool A2>
static hipError_t launch_row_dw_t(const RowDwArgs& a, int grid, hipStream_t s) {
  using C = RowDwCfg<GW, AW, BF>;
  (void)hipFuncSetAttribute((const void*)k_row_dw<GW, AW, BF, GBF, ABF, A2>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
  hipLaunchKernelGGL((k_row_dw<GW, AW, BF, GBF, ABF, A2>), dim3(grid), dim3(64 * C::NW), C::LDS, s, a);
  return hipGetLastError();
}

hipError_t launch_row_dw(const RowDwArgs& a, int grid, hipStream_t s) {
  // forms in use: 128 x 128 (edge adjoint: G BF16/FP32, A BF16/FP32) and
  // 128 x [128 | 128] (node update: A = [a*, x], FP32)
  if (a.GW != 128) return hipErrorInvalidValue;
  if (a.AW == 128 && !a.A2) {
    // BF16 products take BF16 or FP32 operands; FP32 products FP32 operands
    if (a.bf) {
      if (a.g_bf && a.a_bf) return launch_row_dw_t<128, 128, true, true, true, false>(a, grid, s);
      if (a.g_bf && !a.a_bf) return launch_row_dw_t<128, 128, true, true, false, false>(a, grid, s);
      return hipErrorInvalidValue;
    }
    if (!a.g_bf && !a.a_bf) return launch_row_dw_t<128, 128, false, false, false, false>(a, grid, s);
    return hipErrorInvalidValue;
  }
  if (a.AW == 256 && a.A2 && !a.a_bf) {
    if (a.bf && a.g_bf) return launch_row_dw_t<128, 256, true, true, false, true>(a, grid, s);
    if (!a.bf && !a.g_bf) return launch_row_dw_t<128, 256, false, false, false, true>(a, grid, s);
  }
  return hipErrorInvalidValue;
}

template <bool BF>
__device__ __forceinline__ float4 load4(const void* __restrict__ p, int64_t off) {
  if constexpr (BF) {
    const v4bf b = __builtin_bit_cast(v4bf, *reinterpret_cast<const u32x2*>(reinterpret_cast<const __bf16*>(p) + off));
    return make_float4((float)b[0], (float)b[1], (float)b[2], (float)b[3]);
  } else {
    return *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(p) + off);
  }
}

// Column sums of two [R][W] arrays: thread t sums feature group t % (W/4)
// (4 features) over rows t / (W/4), + P, + 2P, ... of the workgroup's
// range, then the row phases are added in order.
template <int W, bool XBF, bool YBF>
__global__ __launch_bounds__(256) void k_colsum2(int64_t n_rows, const void* __restrict__ X,
                                                 const void* __restrict__ Y, float* __restrict__ part,
                                                 int64_t slab, int64_t offx, int64_t offy) {
  constexpr int FG = W / 4, P = 256 / FG;
  __shared__ float4 sx[256], sy[256];
  const int fg = threadIdx.x % FG, ph = threadIdx.x / FG;
  const int64_t per = (n_rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per, r1 = std::min(n_rows, r0 + per);
  float4 ax = make_float4(0.f, 0.f, 0.f, 0.f), ay = ax;
  for (int64_t r = r0 + ph; r < r1; r += P) {
    const float4 x = load4<XBF>(X, r * W + 4 * fg), y = load4<YBF>(Y, r * W + 4 * fg);
    ax.x += x.x; ax.y += x.y; ax.z += x.z; ax.w += x.w;
    ay.x += y.x; ay.y += y.y; ay.z += y.z; ay.w += y.w;
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  if ((int)threadIdx.x < FG) {
    float4 tx = make_float4(0.f, 0.f, 0.f, 0.f), ty = tx;
    for (int q = 0; q < P; ++q) {
      const float4 u = sx[q * FG + threadIdx.x], v = sy[q * FG + threadIdx.x];
      tx.x += u.x; tx.y += u.y; tx.z += u.z; tx.w += u.w;
      ty.x += v.x; ty.y += v.y; ty.z += v.z; ty.w += v.w;
    }
    float* sl = part + blockIdx.x * slab;
    *reinterpret_cast<float4*>(sl + offx + 4 * threadIdx.x) = tx;
    *reinterpret_cast<float4*>(sl + offy + 4 * threadIdx.x) = ty;
  }
}

hipError_t launch_colsum2(int64_t n_rows, int W, int x_bf, int y_bf, const void* X, const void* Y, float* part,
                          int64_t slab, int64_t offx, int64_t offy, int grid, hipStream_t s) {
  if (W != 128) return hipErrorInvalidValue;
#define MP_CS(XB, YB)                                                                                          \
  if (!!x_bf == XB && !!y_bf == YB) {                                                                          \
    hipLaunchKernelGGL((k_colsum2<128, XB, YB>), dim3(grid), dim3(256), 0, s, n_rows, X, Y, part, slab, offx, offy); \
    return hipGetLastError();                                                                                  \
  }
  MP_CS(true, true) MP_CS(false, false) MP_CS(true, false)
#undef MP_CS
  return hipErrorInvalidValue;
}

// ------------------------------------------------- sender-side gradients


// One gathered row of g_h as loaded (BF16 pairs or FP32), converted to
// FP32 only when added; lane (j, g) holds features 16b + 4g + r.
template <int H, bool BF>
struct GqRaw {
  static constexpr int NB = H / 16;
  typename std::conditional<BF, u32x2, float4>::type v[NB];
  __device__ __forceinline__ void load(const void* __restrict__ base, int64_t r, int g) {
    if constexpr (BF) {
      const __bf16* p = reinterpret_cast<const __bf16*>(base) + r * H + 4 * g;
#pragma unroll
      for (int b = 0; b < NB; ++b) v[b] = *reinterpret_cast<const u32x2*>(p + 16 * b);
    } else {
      const float* p = reinterpret_cast<const float*>(base) + r * H + 4 * g;
#pragma unroll
      for (int b = 0; b < NB; ++b) v[b] = *reinterpret_cast<const float4*>(p + 16 * b);
    }
  }
  __device__ __forceinline__ void add_to(float* __restrict__ s) const {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if constexpr (BF) {
        const v4bf t = __builtin_bit_cast(v4bf, v[b]);
#pragma unroll
        for (int r = 0; r < 4; ++r) s[4 * b + r] += (float)t[r];
      } else {
        s[4 * b + 0] += v[b].x;
        s[4 * b + 1] += v[b].y;
        s[4 * b + 2] += v[b].z;
        s[4 * b + 3] += v[b].w;
      }
    }
  }
};

template <int H, bool BF>
struct GqCfg {
  // FP32 at H = 64: the staging tiles and fragments (84 KB at four waves)
  // leave room for one workgroup per CU, so it has eight waves (two per
  // SIMD, 133 KB); otherwise four waves and two workgroups per CU at H <= 64
  static constexpr int NW = (!BF && H == 64) ? 8 : 4;
  static constexpr int ROWS = 16 * NW;
  static constexpr int MINB = NW == 8 ? 1 : (H <= 64 ? 2 : 1);
  static constexpr size_t FB = frag_bytes(H, 2 * H, BF);
  // FP32 at H = 128: the weight-gradient tiles and accumulators do not fit
  // beside the gather; the kernel writes g_Q per node instead and the weight
  // gradients are summed from g_P, g_Q and x by launch_row_dw.
  static constexpr bool SPLIT = gq_split(H, BF);
  static constexpr size_t STAGE = SPLIT ? 0 : tile_bytes<2 * H, BF, ROWS>() + tile_bytes<H, BF, ROWS>();
  static constexpr bool LDS_FRAG = FB + STAGE <= kLdsLimit;
  static constexpr size_t LDS = STAGE + (LDS_FRAG ? FB : 0);
};

// Per node j: g_Q[j] = sum of g_h over j's outgoing edges, read as the
// reverse edges of j's incoming edges (in ascending order), then
//   g_x[j] += W1a^T g_P[j] + W1b^T g_Q[j]
//   dW1a += g_P x^T, dW1b += g_Q x^T, db1 += g_P.
template <int H, bool BF>
__global__ __launch_bounds__((64 * GqCfg<H, BF>::NW), (GqCfg<H, BF>::MINB)) void k_gq(GqArgs a) {
  using C = GqCfg<H, BF>;
  constexpr int NF = H / 4, MB = H / 16, NW = C::NW, ROWS = C::ROWS, NT = dw_tiles_per_wave<2 * H, H, NW>();
  // edges gathered per round trip: as many raw rows as fit in 48 registers
  // (6 at H=64 in BF16, the lattice's largest degree), at least 2, at most 8
  constexpr int RAWREG = BF ? H / 8 : H / 4;
  constexpr int RAWBUD = (!BF && H == 64) ? 96 : 48;
  constexpr int GQ_CH = RAWBUD / RAWREG < 2 ? 2 : (RAWBUD / RAWREG > 8 ? 8 : RAWBUD / RAWREG);
  extern __shared__ uint4 smem[];
  char* tG = reinterpret_cast<char*>(smem);
  char* tA = tG + (C::SPLIT ? 0 : tile_bytes<2 * H, BF, ROWS>());
  const char* fr;
  if constexpr (C::LDS_FRAG) {
    uint4* fl = smem + C::STAGE / 16;
    stage_frags(fl, a.frag_abt, C::FB);
    fr = reinterpret_cast<const char*>(fl);
  } else {
    fr = reinterpret_cast<const char*>(a.frag_abt);
  }
  __syncthreads();
  const DevGraph& gr = a.g;
  const int lane = lane_id(), j = lane & 15, g = lane >> 4, wave = threadIdx.x / 64;
  const int64_t n = gr.n_rows, nblk = (n + 15) / 16;
  // contiguous row blocks per workgroup, NW blocks (one per wave) per step
  const int64_t per = (nblk + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = blockIdx.x * per, b1 = std::min(nblk, b0 + per);
  const int64_t n_iter = (b1 - b0 + NW - 1) / NW;
  v4f acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  float db1[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) db1[i] = 0.f;

  // CSR bounds run one block ahead; completed before the loop so that its
  // entry state holds no pending loads
  const int64_t E = gr.n_edges;
  int p0_n, p1_n;
  {
    const int64_t bk = b0 + wave, row = bk * 16 + j;
    const int64_t rr = (bk < b1 && row < n) ? row : n - 1;
    p0_n = gr.rowptr[rr];
    p1_n = gr.rowptr[rr + 1];
    asm volatile("" : "+v"(p0_n), "+v"(p1_n));
  }

  for (int64_t it = 0; it < n_iter; ++it) {
    const int64_t bk = b0 + it * NW + wave;
    const int64_t row = bk * 16 + j;
    const bool valid = bk < b1 && row < n;
    const int64_t rr = valid ? row : n - 1;
    const int p0 = p0_n, deg = p1_n - p0_n;
    {
      const int64_t bk2 = bk + NW, row2 = bk2 * 16 + j;
      const int64_t rr2 = (bk2 < b1 && row2 < n) ? row2 : n - 1;
      p0_n = gr.rowptr[rr2];
      p1_n = gr.rowptr[rr2 + 1];
    }
    // reverse-edge indices of the first GQ_CH incoming edges (positions past
    // the row's end read an in-bounds index whose row is loaded, not added),
    // and the node rows, all in one round trip
    int rv[GQ_CH];
#pragma unroll
    for (int q = 0; q < GQ_CH; ++q) rv[q] = gr.rev[std::min<int64_t>(p0 + q, E - 1)];
    float in[2 * NF], gp[NF], xv[NF], gx[NF];
    load_row<H>(a.g_P + rr * H, g, gp);
    load_row<H>(a.x + rr * H, g, xv);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      in[i] = gp[i];
      in[NF + i] = 0.f;
    }
    // g_Q = sum of g_h over the reverse edges, added in ascending edge order
    for (int c = 0;;) {
      GqRaw<H, BF> t[GQ_CH];
#pragma unroll
      for (int q = 0; q < GQ_CH; ++q) t[q].load(a.g_h, rv[q], g);
      if (c == 0) load_row<H>(a.g_x + rr * H, g, gx);  // in flight with the gathers
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < GQ_CH; ++q)
        if (c + q < deg) t[q].add_to(in + NF);
      c += GQ_CH;
      if (__ballot(c < deg) == 0) break;
#pragma unroll
      for (int q = 0; q < GQ_CH; ++q) rv[q] = gr.rev[std::min<int64_t>(p0 + c + q, E - 1)];
    }
    if (!valid) {
#pragma unroll
      for (int i = 0; i < 2 * NF; ++i) in[i] = 0.f;
    }
    if constexpr (C::SPLIT) {
      if (valid) store_row<H>(a.gq_out + row * H, g, *reinterpret_cast<float(*)[NF]>(in + NF));
      gemm<BF, MB, 2 * MB>(fr, in, gx, lane);
      if (valid) store_row<H>(a.g_x + row * H, g, gx);
      continue;
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) db1[i] += in[i];
    stage_row<2 * H, BF, ROWS>(tG, wave * 16 + j, g, in);
    stage_row<H, BF, ROWS>(tA, wave * 16 + j, g, xv);
    gemm<BF, MB, 2 * MB>(fr, in, gx, lane);
    if (valid) store_row<H>(a.g_x + row * H, g, gx);
    __syncthreads();
    dw_tiles<2 * H, H, BF, NW>(tG, tA, acc, wave, lane);
    __syncthreads();
  }
  if constexpr (!C::SPLIT) {
    float* slab = a.part + blockIdx.x * a.slab;
    dw_store<2 * H, H, NW>(acc, slab, H, wave, lane);
    block_sum_vec<H, NW>(db1, reinterpret_cast<float*>(tG), slab + 2 * H * H, wave, lane);
  }
}

template <int H, bool BF>
static hipError_t launch_gq_t(const GqArgs& a, int grid, hipStream_t s) {
  using C = GqCfg<H, BF>;
  (void)hipFuncSetAttribute((const void*)k_gq<H, BF>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
  hipLaunchKernelGGL((k_gq<H, BF>), dim3(grid), dim3(64 * C::NW), C::LDS, s, a);
  return hipGetLastError();
}

hipError_t launch_gq(const GqArgs& a, int grid, hipStream_t s) {
#define MP_CASE(HH) if (a.H == HH) return a.bf ? launch_gq_t<HH, true>(a, grid, s) : launch_gq_t<HH, false>(a, grid, s);
  MP_CASE(32) MP_CASE(64) MP_CASE(128)
#undef MP_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------------------------- row MLP adjoint


template <int H, int KIN, bool TIN, bool TOUT, bool BF>
struct MlpBwdCfg {
  // TP (the FP32 node-update and encoder adjoints at H = 64): eight waves
  // in one workgroup, two per SIMD, in 256 registers: the transposed
  // products read W1 and W0 at transposed addresses (only W0 and W1 sit in
  // LDS), the next block's rows are not loaded ahead, and the bias /
  // LayerNorm sums are reduced across the block's lanes into one register
  // per lane.  Measured on C4: node update 11.4 -> 10.1 ms per launch.
  static constexpr bool TP = !BF && H == 64 && !TOUT && (KIN == 2 * H || TIN);
  static constexpr int NW = (TP || (BF && H <= 64)) ? 8 : 4;  // waves per workgroup
  static constexpr int ROWS = 16 * NW;
  // BF16: bias / LayerNorm gradients are column sums of staged tiles
  static constexpr bool VEC = BF && !TOUT;
  static constexpr int AW0 = TIN ? 16 : KIN;  // staged input width
  static constexpr size_t F0 = TIN ? 0 : frag_bytes(H, KIN, BF);
  static constexpr size_t F1 = TOUT ? 0 : frag_bytes(H, H, BF);
  // FP32 at H = 128: the square transposed products read the forward
  // matrix's own fragments (gemm_f32_tr), so W1^T / W0^T need no copy and
  // the remaining fragments fit in LDS beside the tiles
  static constexpr bool TR1 = (!BF && H == 128 && !TOUT) || TP;
  static constexpr bool TR0 = (!BF && H == 128 && !TIN && KIN == H) || TP;
  static constexpr size_t F1T = TR1 ? 0 : F1;
  // fragments: W0, W1, W1^T, W0^T
  static constexpr size_t FRAG = 2 * F0 + F1 + F1T - (TR0 ? F0 : 0);
  static constexpr size_t TB = tile_bytes<H, BF, ROWS>();
  // phase 1: [g_y, u (, g_out, g_out * normalised y)]; small output: [g_out (16 wide), u];
  // phase 0 reuses the first tile for g_z.  The input tile has its own
  // region, staged as soon as the block's input has been used.
  static constexpr size_t STAGE1 = (VEC ? 4 : 2) * TB;
  static constexpr size_t TA0 = tile_bytes<AW0, BF, ROWS>();
  static constexpr size_t SMALL_ = (TIN || TOUT) ? 16 * H : 0;
  // a separate input tile when everything (with the fragments) still fits;
  // otherwise phase 0 stages the input into the second phase-1 tile
  static constexpr bool SEP_A0 = STAGE1 + TA0 + 2 * F0 + 2 * F1 + SMALL_ + 3 * H * sizeof(float) <= kLdsLimit;
  static constexpr size_t STAGE0 = TB + TA0;
  // one staging round per block (both phases' tiles at once, two barriers
  // instead of four) when g_z has a tile of its own as well
  static constexpr bool ONE = SEP_A0 && STAGE1 + TA0 + TB + 2 * F0 + 2 * F1 + SMALL_ + 3 * H * sizeof(float) <= kLdsLimit;
  static constexpr size_t STAGE = ONE ? STAGE1 + TA0 + TB : SEP_A0 ? STAGE1 + TA0 : (STAGE0 > STAGE1 ? STAGE0 : STAGE1);
  static constexpr size_t SMALL = (TIN || TOUT) ? 16 * H : 0;  // small W0 / W1, [.][4] or [4][H]
  static constexpr size_t VECS = 3 * H * sizeof(float);         // b0, b1, LayerNorm gain
  static constexpr bool LDS_FRAG = FRAG + STAGE + SMALL + VECS <= kLdsLimit;
  static constexpr size_t LDS = STAGE + (LDS_FRAG ? FRAG : 0) + SMALL + VECS;
};

// The rows one 16-row block of k_mlp_bwd reads: its inputs and the
// gradient at its output.
template <int H, int KIN, bool TIN, bool TOUT, bool GB = false>
struct MlpBwdIn {
  static constexpr int NF = H / 4, NIN = TIN ? 4 : KIN / 4, NGO = TOUT ? 4 : H / 4;
  float in[NIN];
  float go[NGO];
  __device__ __forceinline__ void load(const MlpBwdArgs& a, int64_t rr, int g) {
    if constexpr (TIN) {
      // k0 <= 4 features per row; columns past k0 read column k0-1, then 0
#pragma unroll
      for (int k = 0; k < 4; ++k) in[k] = a.src0[rr * a.k0 + (k < a.k0 ? k : a.k0 - 1)];
#pragma unroll
      for (int k = 0; k < 4; ++k) in[k] = k < a.k0 ? in[k] : 0.f;
    } else if constexpr (KIN == 2 * H) {
      float t0[NF], t1[NF];
      load_row<H>(a.src0 + rr * H, g, t0);
      load_row<H>(a.src1 + rr * H, g, t1);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        in[i] = t0[i];
        in[NF + i] = t1[i];
      }
    } else {
      load_row<KIN>(a.src0 + rr * KIN, g, in);
    }
    if constexpr (TOUT) {
      // n_out <= 4 outputs; the same clamp-then-zero as the inputs
#pragma unroll
      for (int o = 0; o < 4; ++o)
        go[o] = reinterpret_cast<const float*>(a.g_out)[rr * a.n_out + (o < a.n_out ? o : a.n_out - 1)];
#pragma unroll
      for (int o = 0; o < 4; ++o) go[o] = o < a.n_out ? go[o] : 0.f;
    } else {
      load_row_t<H, GB>(a.g_out, rr, g, go);
    }
  }
  __device__ __forceinline__ void settle() {
#pragma unroll
    for (int i = 0; i < NIN; ++i) asm volatile("" : "+v"(in[i]));
#pragma unroll
    for (int i = 0; i < NGO; ++i) asm volatile("" : "+v"(go[i]));
  }
};

// Adjoint of k_mlp_fwd, forward recomputed per row block:
//   z = W0 in + b0, u = ELU(z), y = W1 u + b1, out = [resid +] LN(y)
// Two staging phases per step (dW1 with its bias / LayerNorm sums, then
// dW0 and db0) share the same LDS.  The next block's rows are loaded while
// the current one is processed (one block ahead, as in k_mlp_fwd).
// GB: the H-wide output gradient is stored as BF16 (the edge encoder's, an
// edge-state gradient, when edge states are BF16).
template <int H, int KIN, bool TIN, bool TOUT, bool BF, bool GB>
__global__ __launch_bounds__((64 * MlpBwdCfg<H, KIN, TIN, TOUT, BF>::NW)) void k_mlp_bwd(MlpBwdArgs a) {
  using C = MlpBwdCfg<H, KIN, TIN, TOUT, BF>;
  using In = MlpBwdIn<H, KIN, TIN, TOUT, GB>;
  constexpr bool PK = KIN != 2 * H;  // packed BF16 staging, except where registers are short
  constexpr int NF = H / 4, MB = H / 16, KB = TIN ? 1 : KIN / 16, AW0 = C::AW0, NW = C::NW, ROWS = C::ROWS;
  constexpr int NT1 = TOUT ? dw_tiles_per_wave<16, H, NW>() : dw_tiles_per_wave<H, H, NW>();
  constexpr int NT0 = dw_tiles_per_wave<H, AW0, NW>();
  // FP32 transposed products (TR1 / TR0) read W0 / W1 in the rotated
  // layout; W1^T / W0^T copies, where staged, keep the packed one
  constexpr bool ROT = !BF && (C::TR1 || C::TR0) && C::LDS_FRAG;
  extern __shared__ uint4 smem[];
  char* tG = reinterpret_cast<char*>(smem);
  char* tA = tG + C::TB;
  char* tGE = tA + C::TB;  // phase 1, VEC: g_out and g_out * normalised y
  char* tGM = tGE + C::TB;
  char* tA0 = C::SEP_A0 ? tG + C::STAGE1 : tA;            // phase 0: the input rows
  char* tG0 = C::ONE ? tG + C::STAGE1 + C::TA0 : tG;      // phase 0: g_z
  const char* fr;
  if constexpr (C::LDS_FRAG) {
    uint4* fl = smem + C::STAGE / 16;
    if constexpr (ROT) {
      stage_frags_rot(fl, a.frag0, C::F0);
      stage_frags_rot(fl + C::F0 / 16, a.frag1, C::F1);
    } else {
      stage_frags(fl, a.frag0, C::F0);
      stage_frags(fl + C::F0 / 16, a.frag1, C::F1);
    }
    if constexpr (!C::TR1) stage_frags(fl + (C::F0 + C::F1) / 16, a.frag1t, C::F1);
    if constexpr (!C::TR0)
      if (a.frag0t) stage_frags(fl + (C::F0 + C::F1 + C::F1T) / 16, a.frag0t, C::F0);
    fr = reinterpret_cast<const char*>(fl);
  } else {
    fr = nullptr;
  }
  float* small = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + C::STAGE + (C::LDS_FRAG ? C::FRAG : 0));
  float* vecs = small + C::SMALL / 4;
  if constexpr (TIN) stage_small(small, a.W0, H, a.k0);
  if constexpr (TOUT)
    for (int t = threadIdx.x; t < 4 * H; t += blockDim.x) small[t] = (t / H) < a.n_out ? a.W1[t] : 0.f;
  for (int t = threadIdx.x; t < 3 * H; t += blockDim.x)
    vecs[t] = t < H ? a.b0[t] : (t < 2 * H ? (TOUT ? 0.f : a.b1[t - H]) : (a.ln ? a.lng[t - 2 * H] : 0.f));
  __syncthreads();
  const bool want_gin = (a.g_src0 || a.g_src1) && !TIN;
  // the residual path's gradient is usually g_out itself (node update)
  const bool add1_is_gout = a.g_add1 != nullptr && static_cast<const void*>(a.g_add1) == a.g_out;

  const int lane = lane_id(), j = lane & 15, g = lane >> 4, wave = threadIdx.x / 64;
  const int srow = wave * 16 + j;
  const int64_t n = a.n_rows, nblk = (n + 15) / 16;
  const int64_t per = (nblk + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = blockIdx.x * per, b1 = std::min(nblk, b0 + per);
  const int64_t n_iter = (b1 - b0 + NW - 1) / NW;
  const int NO = TOUT ? a.n_out : H;

  v4f acc1[NT1], acc0[NT0];
#pragma unroll
  for (int t = 0; t < NT1; ++t) acc1[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < NT0; ++t) acc0[t] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int NV = (C::VEC || C::TP) ? 1 : NF;  // per-lane vector accumulators (FP32 path)
  float db0[NV], db1[NV], dga[NV], dbe[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) db0[i] = db1[i] = dga[i] = dbe[i] = 0.f;
  // BF16: column sums of the staged tiles (MFMA, or the vector ALU for the
  // node update, whose registers are fully used)
  using CS = typename std::conditional<KIN == 2 * H, ColSumValu<H, NW>, ColSum<H, NW>>::type;
  CS cs_b0, cs_b1, cs_ga, cs_be;
  // dW1 (and its bias / LayerNorm column sums) from the phase-1 tiles
  auto phase1_products = [&]() {
    if constexpr (TOUT) {
      dw_tiles<16, H, BF, NW>(tG, tA, acc1, wave, lane);
    } else {
      dw_tiles<H, H, BF, NW>(tG, tA, acc1, wave, lane);
      if constexpr (C::VEC) {
        cs_b1.add(tG, wave, lane);
        if (a.ln) {
          cs_be.add(tGE, wave, lane);
          cs_ga.add(tGM, wave, lane);
        }
      }
    }
  };
  cs_b0.zero();
  cs_b1.zero();
  cs_ga.zero();
  cs_be.zero();
  float db1s[4] = {0.f, 0.f, 0.f, 0.f};  // small-output db1 (lane group 0)

  // one-block-ahead loads where registers allow (H <= 64)
  constexpr bool PF = H <= 64 && !C::TP;
  In nx;
  if constexpr (PF) {
    const int64_t row = b0 * 16 + wave * 16 + j;
    nx.load(a, (b0 + wave < b1 && row < n) ? row : n - 1, g);
    nx.settle();  // the loop's entry state holds no pending loads
  }
  for (int64_t it = 0; it < n_iter; ++it) {
    const int oz = opaque_zero();  // re-read fragments and vectors each block
    const char* f0 = (C::LDS_FRAG ? fr : reinterpret_cast<const char*>(a.frag0)) + oz;
    const char* f1 = (C::LDS_FRAG ? fr + C::F0 : reinterpret_cast<const char*>(a.frag1)) + oz;
    const char* f1t = (C::LDS_FRAG ? fr + C::F0 + C::F1 : reinterpret_cast<const char*>(a.frag1t)) + oz;
    const char* f0t = (C::LDS_FRAG ? fr + C::F0 + C::F1 + C::F1T : reinterpret_cast<const char*>(a.frag0t)) + oz;
    const float* vb = vecs + oz;
    const int64_t bk = b0 + it * NW + wave;
    const int64_t row = bk * 16 + j;
    const bool valid = bk < b1 && row < n;
    const int64_t rr = valid ? row : n - 1;
    In cur;
    if constexpr (PF) {
      cur = nx;
      const int64_t bk2 = bk + NW, row2 = bk2 * 16 + j;
      nx.load(a, (bk2 < b1 && row2 < n) ? row2 : n - 1, g);
    } else {
      cur.load(a, rr, g);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (!valid) {
#pragma unroll
      for (int i = 0; i < In::NGO; ++i) cur.go[i] = 0.f;
    }
    // ---- recompute
    float z[NF];
    load_vec<H>(vb, g, z);
    if constexpr (TIN) {
      small_in_linear<H>(small + oz, cur.in, g, z);
    } else {
      gemm<BF, MB, KB, ROT>(f0, cur.in, z, lane);
    }
    // the input tile for dW0: staged now when it has its own region
    auto stage_in = [&]() {
      if constexpr (TIN) {
        float in16[4];  // lane group g holds input features 4g..4g+3
#pragma unroll
        for (int k = 0; k < 4; ++k) in16[k] = g == 0 ? cur.in[k] : 0.f;
        stage_row<16, BF, ROWS, PK>(tA0, srow, g, in16);
      } else {
        stage_row<KIN, BF, ROWS, PK>(tA0, srow, g, cur.in);
      }
    };
    if constexpr (C::SEP_A0) stage_in();
    float u[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) u[i] = elu(z[i]);
    // ---- gradient at u, and phase 1: dW1 (with its bias / LayerNorm sums)
    float gu[NF];
    if constexpr (TOUT) {
#pragma unroll
      for (int i = 0; i < NF; ++i) gu[i] = 0.f;
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        float w[NF];
        load_vec<H>(small + oz + o * H, g, w);
#pragma unroll
        for (int i = 0; i < NF; ++i) gu[i] += w[i] * cur.go[o];
      }
      // db1 (n_out values): one copy per row, in lane group 0
      if (g == 0) {
#pragma unroll
        for (int o = 0; o < 4; ++o) db1s[o] += cur.go[o];
      }
      // dW1 += g_out u^T: g_out staged 16 wide (lane group 0 holds outputs 0..3)
      float go16[4];
#pragma unroll
      for (int o = 0; o < 4; ++o) go16[o] = g == 0 ? cur.go[o] : 0.f;
      stage_row<16, BF, ROWS, PK>(tG, srow, g, go16);
      stage_row<H, BF, ROWS, PK>(tA, srow, g, u);
      if constexpr (!C::ONE) {
        __syncthreads();
        phase1_products();
        __syncthreads();
      }
    } else {
      float y[NF];
      load_vec<H>(vb + H, g, y);
      gemm<BF, MB, MB, ROT>(f1, u, y, lane);
      const float* go = cur.go;
      if (a.ln) {
        float mean, rstd, s1 = 0.f, s2 = 0.f, gam[NF];
        ln_stats<H>(y, a.eps, mean, rstd);
        load_vec<H>(vb + 2 * H, g, gam);
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          const float xh = (y[i] - mean) * rstd;
          if constexpr (!C::VEC && !C::TP) {
            dga[i] += go[i] * xh;
            dbe[i] += go[i];
          }
          const float gx = go[i] * gam[i];
          s1 += gx;
          s2 += gx * xh;
          y[i] = xh;
        }
        if constexpr (C::VEC) {
          float t[NF];
#pragma unroll
          for (int i = 0; i < NF; ++i) t[i] = go[i] * y[i];
          stage_row<H, BF, ROWS, PK>(tGE, srow, g, cur.go);
          stage_row<H, BF, ROWS, PK>(tGM, srow, g, t);
        }
        if constexpr (C::TP) {  // rows past n carry go = 0
          float t[NF], rs[1];
#pragma unroll
          for (int i = 0; i < NF; ++i) t[i] = go[i] * y[i];
          sum16_scatter<NF>(t, rs, j);
          dga[0] += rs[0];
          sum16_scatter<NF>(cur.go, rs, j);
          dbe[0] += rs[0];
        }
        s1 = row_sum(s1) * (1.f / H);
        s2 = row_sum(s2) * (1.f / H);
        const float c1 = -rstd * s1, c2 = -rstd * s2;
#pragma unroll
        for (int i = 0; i < NF; ++i) y[i] = fmaf(y[i], c2, fmaf(go[i] * gam[i], rstd, c1));
      } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) y[i] = go[i];
      }
      if constexpr (C::TP) {
        float rs[1];
        sum16_scatter<NF>(y, rs, j);
        db1[0] += rs[0];
      } else if constexpr (!C::VEC) {
#pragma unroll
        for (int i = 0; i < NF; ++i) db1[i] += y[i];
      }
      stage_row<H, BF, ROWS, PK>(tG, srow, g, y);
      stage_row<H, BF, ROWS, PK>(tA, srow, g, u);
      if constexpr (!C::ONE) {
        __syncthreads();
        phase1_products();
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < NF; ++i) gu[i] = 0.f;
      if constexpr (C::TR1)
        gemm_f32_tr<H, ROT>(reinterpret_cast<const float*>(f1), y, gu, lane);
      else
        gemm<BF, MB, MB>(f1t, y, gu, lane);
    }
    // ---- gradient at z; phase 0: dW0, db0
#pragma unroll
    for (int i = 0; i < NF; ++i) gu[i] *= elu_deriv_from_value(u[i]);
    if constexpr (C::TP) {
      float rs[1];  // rows past n: go = 0, so gu = 0
      sum16_scatter<NF>(gu, rs, j);
      db0[0] += rs[0];
    } else if constexpr (!C::VEC) {
#pragma unroll
      for (int i = 0; i < NF; ++i) db0[i] += gu[i];
    }
    stage_row<H, BF, ROWS, PK>(tG0, srow, g, gu);
    if constexpr (!C::SEP_A0) stage_in();
    __syncthreads();
    if constexpr (C::ONE) phase1_products();
    dw_tiles<H, AW0, BF, NW>(tG0, tA0, acc0, wave, lane);
    if constexpr (C::VEC) cs_b0.add(tG0, wave, lane);
    __syncthreads();
    // ---- input gradient
    if constexpr (!TIN) {
      if (want_gin) {
        float gi[KIN / 4];
#pragma unroll
        for (int i = 0; i < KIN / 4; ++i) gi[i] = 0.f;
        if constexpr (C::TR0)
          gemm_f32_tr_mk<H, KIN, ROT>(reinterpret_cast<const float*>(f0), gu, gi, lane);
        else
          gemm<BF, KIN / 16, MB>(f0t, gu, gi, lane);
        if constexpr (KIN == 2 * H) {
          float t0[NF], t1[NF];
#pragma unroll
          for (int i = 0; i < NF; ++i) {
            t0[i] = gi[i];
            t1[i] = gi[NF + i];
          }
          if (add1_is_gout) {
#pragma unroll
            for (int i = 0; i < NF; ++i) t1[i] += cur.go[i];
          } else if (a.g_add1) {
            float r[NF];
            load_row<H>(a.g_add1 + rr * H, g, r);
#pragma unroll
            for (int i = 0; i < NF; ++i) t1[i] += r[i];
          }
          if constexpr (PF) nx.settle();  // next block's loads complete before this block's stores
          if (valid && a.g_src0) store_row<H>(a.g_src0 + row * H, g, t0);
          if (valid && a.g_src1) store_row<H>(a.g_src1 + row * H, g, t1);
        } else {
          if constexpr (PF) nx.settle();
          if (valid && a.g_src0) store_row<KIN>(a.g_src0 + row * KIN, g, gi);
        }
      }
    }
  }
  // ---- write the slab: [dW0 | db0 | dW1 | db1 | dgamma | dbeta]
  float* slab = a.part + blockIdx.x * a.slab;
  const int k0w = TIN ? a.k0 : KIN;
  dw_store<H, AW0, NW>(acc0, slab, k0w, wave, lane);
  float* scratch = reinterpret_cast<float*>(tG);
  if constexpr (C::VEC)
    cs_b0.store(scratch, slab + H * k0w, wave, lane);
  else if constexpr (C::TP)
    block_sum_scattered<H, NW>(db0[0], scratch, slab + H * k0w, wave, lane);
  else
    block_sum_vec<H, NW>(db0, scratch, slab + H * k0w, wave, lane);
  float* s1 = slab + H * k0w + H;
  if constexpr (TOUT) {
    dw_store<16, H, NW>(acc1, s1, H, wave, lane, NO);
    // db1: summed over the workgroup's lanes in a fixed order
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 4; ++o) scratch[threadIdx.x * 4 + o] = (g == 0) ? db1s[o] : 0.f;
    __syncthreads();
    if ((int)threadIdx.x < NO) {
      float sum = 0.f;
      for (int t = 0; t < (int)blockDim.x; ++t) sum += scratch[t * 4 + threadIdx.x];
      s1[NO * H + threadIdx.x] = sum;
    }
    __syncthreads();
  } else {
    dw_store<H, H, NW>(acc1, s1, H, wave, lane);
    if constexpr (C::VEC) {
      cs_b1.store(scratch, s1 + H * H, wave, lane);
      if (a.ln) {
        cs_ga.store(scratch, s1 + H * H + H, wave, lane);
        cs_be.store(scratch, s1 + H * H + 2 * H, wave, lane);
      }
    } else if constexpr (C::TP) {
      block_sum_scattered<H, NW>(db1[0], scratch, s1 + H * H, wave, lane);
      if (a.ln) {
        block_sum_scattered<H, NW>(dga[0], scratch, s1 + H * H + H, wave, lane);
        block_sum_scattered<H, NW>(dbe[0], scratch, s1 + H * H + 2 * H, wave, lane);
      }
    } else {
      block_sum_vec<H, NW>(db1, scratch, s1 + H * H, wave, lane);
      if (a.ln) {
        block_sum_vec<H, NW>(dga, scratch, s1 + H * H + H, wave, lane);
        block_sum_vec<H, NW>(dbe, scratch, s1 + H * H + 2 * H, wave, lane);
      }
    }
  }
}

template <int H, int KIN, bool TIN, bool TOUT, bool BF, bool GB = false>
static hipError_t launch_mlp_bwd_t(const MlpBwdArgs& a, int grid, hipStream_t s) {
  using C = MlpBwdCfg<H, KIN, TIN, TOUT, BF>;
  const size_t lds = C::LDS;
  (void)hipFuncSetAttribute((const void*)k_mlp_bwd<H, KIN, TIN, TOUT, BF, GB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_mlp_bwd<H, KIN, TIN, TOUT, BF, GB>), dim3(grid), dim3(64 * C::NW), lds, s, a);
  return hipGetLastError();
}

template <int H, bool BF>
static hipError_t launch_mlp_bwd_h(const MlpBwdArgs& a, int grid, hipStream_t s) {
  const bool tin = a.k0 <= 4, tout = a.n_out < 16;
  const int kin = a.k0 + a.k1;
  if (a.gout_bf && !(tin && !tout && BF)) return hipErrorInvalidValue;
  if constexpr (BF) {
    if (tin && !tout && a.gout_bf) return launch_mlp_bwd_t<H, 4, true, false, BF, true>(a, grid, s);
  }
  if (tin && !tout) return launch_mlp_bwd_t<H, 4, true, false, BF>(a, grid, s);
  if (!tin && kin == H && tout) return launch_mlp_bwd_t<H, H, false, true, BF>(a, grid, s);
  if (!tin && kin == H && !tout) return launch_mlp_bwd_t<H, H, false, false, BF>(a, grid, s);
  if (!tin && kin == 2 * H && !tout) return launch_mlp_bwd_t<H, 2 * H, false, false, BF>(a, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_bwd(const MlpBwdArgs& a, int grid, hipStream_t s) {
#define MP_CASE(HH) \
  if (a.H == HH) return a.bf ? launch_mlp_bwd_h<HH, true>(a, grid, s) : launch_mlp_bwd_h<HH, false>(a, grid, s);
  MP_CASE(32) MP_CASE(64) MP_CASE(128)
#undef MP_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------ split node-update adjoint (wide H)

template <int H, bool BF>
struct NodeBwdSplitCfg {
  static constexpr int NW = 8;  // independent waves sharing the LDS weights
  static constexpr size_t F0 = frag_bytes(H, 2 * H, BF), F1 = frag_bytes(H, H, BF);
  static constexpr size_t VECS = 3 * H * sizeof(float);  // b0, b1, LayerNorm gain
  // BF16: pass 1 holds W0, W1 and W1^T.  FP32 (twice the bytes): pass 1 is
  // cut after u = ELU(W0 [a*, x] + b0) (W0 only), and pass 1b continues
  // from the stored u with W1 and W1^T.
  static constexpr bool CUT = F0 + 2 * F1 + VECS > kLdsLimit;
  static constexpr size_t LDS1 = CUT ? F0 + VECS : F0 + 2 * F1 + VECS;
  static constexpr size_t LDS1B = 2 * F1 + VECS;
  static constexpr size_t LDS2 = F0;  // pass 2: W0^T
  static_assert(LDS1 <= kLdsLimit && (!CUT || LDS1B <= kLdsLimit) && LDS2 <= kLdsLimit,
                "split node adjoint: weights must fit in LDS");
};

// Adjoint of the node update x' = x + LN(W1 ELU(W0 [a*, x] + b0) + b1)
// without its weight gradients (the fused kernel's tiles, accumulators and
// all four weight matrices do not fit at this width), in two passes whose
// weights each fit in LDS.  Pass 1 writes per row the factors u, g_y
// (dW1 = sum g_y u^T, db1), g_z (dW0 = sum g_z [a*, x]^T, db0) and
// g_out * normalised y (dgamma; dbeta sums g_out itself).
// PH: 0 the whole pass; 1 only up to u (stored); 2 from the stored u on.
template <int H, bool BF, int PH>
__global__ __launch_bounds__((64 * NodeBwdSplitCfg<H, BF>::NW)) void k_node_bwd_split(MlpBwdArgs a, void* u_out,
                                                                                      void* gy_out, void* gz_out,
                                                                                      void* goxh_out) {
  using C = NodeBwdSplitCfg<H, BF>;
  constexpr int NF = H / 4, MB = H / 16, KB = 2 * H / 16, NW = C::NW;
  constexpr size_t F0 = PH == 2 ? 0 : C::F0;                   // W0 present
  constexpr size_t F1 = PH == 1 ? 0 : C::F1;                   // W1, W1^T present
  constexpr size_t LDS = F0 + 2 * F1 + C::VECS;
  extern __shared__ uint4 smem[];
  if constexpr (PH != 2) stage_frags(smem, a.frag0, C::F0);
  if constexpr (PH != 1) {
    stage_frags(smem + F0 / 16, a.frag1, C::F1);
    stage_frags(smem + (F0 + C::F1) / 16, a.frag1t, C::F1);
  }
  const char* f0 = reinterpret_cast<const char*>(smem);
  const char* f1 = f0 + F0;
  const char* f1t = f1 + F1;
  float* vecs = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + LDS - C::VECS);
  for (int t = threadIdx.x; t < 3 * H; t += blockDim.x)
    vecs[t] = t < H ? a.b0[t] : (t < 2 * H ? a.b1[t - H] : (a.ln ? a.lng[t - 2 * H] : 0.f));
  __syncthreads();
  const int lane = lane_id(), j = lane & 15, g = lane >> 4, wave = threadIdx.x / 64;
  const int64_t n = a.n_rows, nblk = (n + 15) / 16;
  for (int64_t blk = (int64_t)blockIdx.x * NW + wave; blk < nblk; blk += (int64_t)gridDim.x * NW) {
    const int oz = opaque_zero();
    const float* vb = vecs + oz;
    const int64_t row = blk * 16 + j;
    const bool valid = row < n;
    const int64_t rr = valid ? row : n - 1;
    float u[NF], go[NF];
    if constexpr (PH != 2) {
      float in[2 * NF];
      load_row<H>(a.src0 + rr * H, g, *reinterpret_cast<float(*)[NF]>(in));
      load_row<H>(a.src1 + rr * H, g, *reinterpret_cast<float(*)[NF]>(in + NF));
      if constexpr (PH == 0) load_row<H>(reinterpret_cast<const float*>(a.g_out) + rr * H, g, go);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (PH == 0) {
        if (!valid) {
#pragma unroll
          for (int i = 0; i < NF; ++i) go[i] = 0.f;
        }
      }
      load_vec<H>(vb, g, u);
      gemm<BF, MB, KB>(f0 + oz, in, u, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) u[i] = elu(u[i]);
      if (valid) store_row_t<H, BF>(u_out, row, g, u);
      if constexpr (PH == 1) continue;
    } else {
      load_row_t<H, BF>(u_out, rr, g, u);
      load_row<H>(reinterpret_cast<const float*>(a.g_out) + rr * H, g, go);
      if (!valid) {
#pragma unroll
        for (int i = 0; i < NF; ++i) go[i] = 0.f;
      }
    }
    float y[NF];
    load_vec<H>(vb + H, g, y);
    gemm<BF, MB, MB>(f1 + oz, u, y, lane);
    if (a.ln) {
      float mean, rstd, s1 = 0.f, s2 = 0.f, gam[NF], t[NF];
      ln_stats<H>(y, a.eps, mean, rstd);
      load_vec<H>(vb + 2 * H, g, gam);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        const float xh = (y[i] - mean) * rstd;
        t[i] = go[i] * xh;
        const float gx = go[i] * gam[i];
        s1 += gx;
        s2 += gx * xh;
        y[i] = xh;
      }
      if (valid) store_row_t<H, BF>(goxh_out, row, g, t);
      s1 = row_sum(s1) * (1.f / H);
      s2 = row_sum(s2) * (1.f / H);
      const float c1 = -rstd * s1, c2 = -rstd * s2;
#pragma unroll
      for (int i = 0; i < NF; ++i) y[i] = fmaf(y[i], c2, fmaf(go[i] * gam[i], rstd, c1));
    } else {
#pragma unroll
      for (int i = 0; i < NF; ++i) y[i] = go[i];
    }
    if (valid) store_row_t<H, BF>(gy_out, row, g, y);
    float gu[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) gu[i] = 0.f;
    gemm<BF, MB, MB>(f1t + oz, y, gu, lane);
#pragma unroll
    for (int i = 0; i < NF; ++i) gu[i] *= elu_deriv_from_value(u[i]);
    if (valid) store_row_t<H, BF>(gz_out, row, g, gu);
  }
}

// Pass 2: [g_a*, g_x] = W0^T g_z, plus the residual path's gradient
// (g_add1, normally g_out) on g_x.
template <int H, bool BF>
__global__ __launch_bounds__((64 * NodeBwdSplitCfg<H, BF>::NW)) void k_node_gin(MlpBwdArgs a, const void* gz) {
  using C = NodeBwdSplitCfg<H, BF>;
  constexpr int NF = H / 4, MB = H / 16, NW = C::NW;
  extern __shared__ uint4 smem[];
  stage_frags(smem, a.frag0t, C::F0);
  const char* f0t = reinterpret_cast<const char*>(smem);
  __syncthreads();
  const int lane = lane_id(), j = lane & 15, g = lane >> 4, wave = threadIdx.x / 64;
  const int64_t n = a.n_rows, nblk = (n + 15) / 16;
  for (int64_t blk = (int64_t)blockIdx.x * NW + wave; blk < nblk; blk += (int64_t)gridDim.x * NW) {
    const int oz = opaque_zero();
    const int64_t row = blk * 16 + j;
    const bool valid = row < n;
    const int64_t rr = valid ? row : n - 1;
    float gu[NF], gi[2 * NF];
    load_row_t<H, BF>(gz, rr, g, gu);
#pragma unroll
    for (int i = 0; i < NF; ++i) gi[i] = 0.f;
    if (a.g_add1) {
      load_row<H>(a.g_add1 + rr * H, g, *reinterpret_cast<float(*)[NF]>(gi + NF));
    } else {
#pragma unroll
      for (int i = 0; i < NF; ++i) gi[NF + i] = 0.f;
    }
    gemm<BF, 2 * MB, MB>(f0t + oz, gu, gi, lane);
    if (valid) {
      if (a.g_src0) store_row<H>(a.g_src0 + row * H, g, *reinterpret_cast<float(*)[NF]>(gi));
      if (a.g_src1) store_row<H>(a.g_src1 + row * H, g, *reinterpret_cast<float(*)[NF]>(gi + NF));
    }
  }
}

template <int H, bool BF, int PH>
static hipError_t launch_node_pass1(const MlpBwdArgs& a, void* u, void* gy, void* gz, void* goxh, int grid,
                                    size_t lds, hipStream_t s) {
  using C = NodeBwdSplitCfg<H, BF>;
  (void)hipFuncSetAttribute((const void*)k_node_bwd_split<H, BF, PH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL((k_node_bwd_split<H, BF, PH>), dim3(grid), dim3(64 * C::NW), lds, s, a, u, gy, gz, goxh);
  return hipGetLastError();
}

template <int H, bool BF>
static hipError_t launch_node_bwd_split_t(const MlpBwdArgs& a, void* u, void* gy, void* gz, void* goxh, int grid,
                                          hipStream_t s) {
  using C = NodeBwdSplitCfg<H, BF>;
  hipError_t e;
  if constexpr (C::CUT) {
    e = launch_node_pass1<H, BF, 1>(a, u, gy, gz, goxh, grid, C::LDS1, s);
    if (e == hipSuccess) e = launch_node_pass1<H, BF, 2>(a, u, gy, gz, goxh, grid, C::LDS1B, s);
  } else {
    e = launch_node_pass1<H, BF, 0>(a, u, gy, gz, goxh, grid, C::LDS1, s);
  }
  if (e != hipSuccess) return e;
  (void)hipFuncSetAttribute((const void*)k_node_gin<H, BF>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS2);
  hipLaunchKernelGGL((k_node_gin<H, BF>), dim3(grid), dim3(64 * C::NW), C::LDS2, s, a, (const void*)gz);
  return hipGetLastError();
}

hipError_t launch_node_bwd_split(const MlpBwdArgs& a, void* u, void* gy, void* gz, void* goxh, int grid,
                                 hipStream_t s) {
  if (a.H != 128 || a.k0 != a.H || a.k1 != a.H || a.n_out != a.H) return hipErrorInvalidValue;
  return a.bf ? launch_node_bwd_split_t<128, true>(a, u, gy, gz, goxh, grid, s)
              : launch_node_bwd_split_t<128, false>(a, u, gy, gz, goxh, grid, s);
}

// ------------------------------------------------------ slab reduction

// dst[r][col0 + c] = sum over slabs of slab[src_off + r*cols + c].  A block
// covers 32 consecutive elements with 8 slab groups: thread (t, q) sums slabs
// q, q+8, q+16, ... of element t (4 loads in flight), then the 8 group sums
// are added in group order.  The order is fixed, so the result is bitwise
// reproducible.
__global__ __launch_bounds__(256) void k_wreduce(ReduceSegs segs) {
  __shared__ float part[8][33];
  const ReduceSeg S = segs.seg[blockIdx.y];
  const int64_t n = (int64_t)S.rows * S.cols;
  const int t = threadIdx.x & 31, q = threadIdx.x >> 5;
  for (int64_t e0 = (int64_t)blockIdx.x * 32; e0 < n; e0 += (int64_t)gridDim.x * 32) {
    const int64_t e = e0 + t;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (e < n) {
      const float* p = S.part + S.src_off + e;
      int b = q;
      for (; b + 24 < S.n_slabs; b += 32) {
        s0 += p[(int64_t)b * S.slab];
        s1 += p[(int64_t)(b + 8) * S.slab];
        s2 += p[(int64_t)(b + 16) * S.slab];
        s3 += p[(int64_t)(b + 24) * S.slab];
      }
      for (; b < S.n_slabs; b += 8) s0 += p[(int64_t)b * S.slab];
    }
    part[q][t] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (q == 0 && e < n) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < 8; ++k) s += part[k][t];
      const int64_t r = e / S.cols, c = e % S.cols;
      S.dst[r * S.ld + S.col0 + c] = s;
    }
    __syncthreads();
  }
}

hipError_t launch_wreduce(const ReduceSegs& segs, hipStream_t s) {
  if (segs.n <= 0) return hipSuccess;
  int64_t mx = 0;
  for (int i = 0; i < segs.n; ++i) mx = std::max<int64_t>(mx, (int64_t)segs.seg[i].rows * segs.seg[i].cols);
  const int grid = (int)std::min<int64_t>((mx + 31) / 32, 1024);
  hipLaunchKernelGGL(k_wreduce, dim3(grid, segs.n), dim3(256), 0, s, segs);
  return hipGetLastError();
}

}  // namespace mp
