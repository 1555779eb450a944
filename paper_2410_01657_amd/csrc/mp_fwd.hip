// Forward kernels of the consistent message-passing layer and its model
// wrapper: weight packing, node projections, the fused edge update with the
// 1/d-weighted aggregation (Eq. 4a-b), the in-device halo sum (Eq. 4c-d),
// row MLPs (node update Eq. 4e, encoders, decoder), edge inputs and loss
// (Eq. 5-6).
#include <algorithm>

#include "mp_device.hpp"
#include "mp_kernels.hpp"

namespace mp {

constexpr size_t kRowMlpLdsBudget = 100 * 1024;
constexpr size_t kRowMlpLdsMax = 150 * 1024;  // one workgroup per CU
constexpr size_t kEdgeLdsBudget = 128 * 1024;
// the projection kernel keeps nothing else in LDS: both FP32 128 x 128
// matrices (128 KB) still fit
constexpr size_t kProjLdsBudget = 128 * 1024;

// --------------------------------------------------------------- packing

__device__ __forceinline__ float view_elem(const PackView& v, int r, int c) {
  return v.trans ? v.p[(int64_t)c * v.ld + v.off + r] : v.p[(int64_t)r * v.ld + v.off + c];
}

__global__ void k_pack(PackJobs jobs, char* __restrict__ dst) {
  const PackJob J = jobs.job[blockIdx.y];
  const int64_t n = (int64_t)J.rows * J.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int row, col;
    if (!jobs.bf) {
      const int S = J.cols / 4;
      const int lane = (int)(e % 64);
      const int64_t t = e / 64;
      const int s = (int)(t % S), mb = (int)(t / S);
      row = 16 * mb + lane % 16;
      col = 16 * (s / 4) + 4 * (lane / 16) + s % 4;
    } else {
      const int T = J.cols / 32;
      const int q = (int)(e % 8);
      int64_t t = e / 8;
      const int lane = (int)(t % 64);
      t /= 64;
      const int tt = (int)(t % T), mb = (int)(t / T);
      row = 16 * mb + lane % 16;
      col = 32 * tt + 16 * (q / 4) + 4 * (lane / 16) + q % 4;
    }
    const float v = col < J.split ? view_elem(J.a, row, col) : view_elem(J.b, row, col - J.split);
    if (!jobs.bf)
      reinterpret_cast<float*>(dst + J.dst_off)[e] = v;
    else
      reinterpret_cast<__bf16*>(dst + J.dst_off)[e] = (__bf16)v;
  }
}

hipError_t launch_pack(const PackJobs& jobs, void* dst, hipStream_t s) {
  if (jobs.n <= 0) return hipSuccess;
  int64_t mx = 0;
  for (int i = 0; i < jobs.n; ++i) mx = std::max<int64_t>(mx, (int64_t)jobs.job[i].rows * jobs.job[i].cols);
  const int grid = (int)std::min<int64_t>((mx + 255) / 256, 1024);
  hipLaunchKernelGGL(k_pack, dim3(grid, jobs.n), dim3(256), 0, s, jobs, reinterpret_cast<char*>(dst));
  return hipGetLastError();
}

// Copy `bytes` (a multiple of 16) from global to LDS with the whole block.
__device__ __forceinline__ void stage_to_lds(uint4* __restrict__ dst, const void* __restrict__ src, size_t bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  for (size_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) dst[i] = s[i];
}

// ------------------------------------------------------------ projections

// P = W1a x + b1, Q = W1b x: the receiver and sender parts of the first
// edge-MLP Linear applied once per node instead of once per edge.  This
// splits the Linear of Eq. 4a over its concatenated input; the products
// are the same, only the summation grouping differs.
template <int H, bool BF>
__global__ __launch_bounds__(256, (H <= 64 ? 4 : 1)) void k_proj(int64_t n_rows, const float* __restrict__ x,
                                              const void* __restrict__ frag, const float* __restrict__ b1,
                                              float* __restrict__ P, float* __restrict__ Q) {
  constexpr int NF = H / 4, MB = H / 16;
  constexpr size_t FB = frag_bytes(H, H, BF);
  constexpr bool LDS = 2 * FB <= kProjLdsBudget;
  extern __shared__ uint4 smem[];
  const char* fr;
  if constexpr (LDS) {
    stage_to_lds(smem, frag, 2 * FB);
    __syncthreads();
    fr = reinterpret_cast<const char*>(smem);
  } else {
    fr = reinterpret_cast<const char*>(frag);
  }
  const int lane = lane_id(), j = lane & 15, g = lane >> 4;
  const int nw = blockDim.x / 64;
  const int64_t nblk = (n_rows + 15) / 16, stride = (int64_t)gridDim.x * nw;
  // one block ahead: the next block's x row loads before this block computes
  int64_t blk = (int64_t)blockIdx.x * nw + threadIdx.x / 64;
  float xn[NF];
  load_row<H>(x + std::min<int64_t>(blk * 16 + j, n_rows - 1) * H, g, xn);
#pragma unroll
  for (int i = 0; i < NF; ++i) asm volatile("" : "+v"(xn[i]));  // no pending loads at the loop entry
  for (; blk < nblk; blk += stride) {
    const int64_t row = blk * 16 + j;
    const bool valid = row < n_rows;
    float xv[NF], p[NF], q[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) xv[i] = xn[i];
    load_row<H>(x + std::min<int64_t>((blk + stride) * 16 + j, n_rows - 1) * H, g, xn);
    __builtin_amdgcn_sched_barrier(0);
    load_vec<H>(b1, g, p);
#pragma unroll
    for (int i = 0; i < NF; ++i) q[i] = 0.f;
    gemm<BF, MB, MB>(fr, xv, p, lane);
    gemm<BF, MB, MB>(fr + FB, xv, q, lane);
#pragma unroll
    for (int i = 0; i < NF; ++i) asm volatile("" : "+v"(xn[i]));  // before this block's stores
    if (valid) {
      store_row<H>(P + row * H, g, p);
      store_row<H>(Q + row * H, g, q);
    }
  }
}

template <int H, bool BF>
static hipError_t launch_proj_t(const DevGraph& gr, const float* x, const void* frag, const float* b1,
                                float* P, float* Q, int grid, hipStream_t s) {
  constexpr size_t FB = frag_bytes(H, H, BF);
  const size_t lds = (2 * FB <= kProjLdsBudget) ? 2 * FB : 0;
  if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)k_proj<H, BF>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_proj<H, BF>), dim3(grid), dim3(256), lds, s, gr.n_rows, x, frag, b1, P, Q);
  return hipGetLastError();
}

hipError_t launch_proj(int H, bool bf, const DevGraph& g, const float* x, const void* frag, const float* b1,
                       float* P, float* Q, int grid, hipStream_t s) {
#define MP_CASE(HH)                                                            \
  if (H == HH) return bf ? launch_proj_t<HH, true>(g, x, frag, b1, P, Q, grid, s) \
                         : launch_proj_t<HH, false>(g, x, frag, b1, P, Q, grid, s);
  MP_CASE(32) MP_CASE(64) MP_CASE(128)
#undef MP_CASE
  return hipErrorInvalidValue;
}

// --------------------------------------------- edge update + aggregation

// Row-aligned tiles of about kTileEdges edges: tile t starts at the first
// row whose first edge index is at least floor(t * E / T); the last tile
// ends at n_rows.  One thread per boundary.
__global__ __launch_bounds__(256) void k_tiles(const int32_t* __restrict__ rowptr, int64_t n_rows, int64_t T,
                                               int32_t* __restrict__ tile_r, int32_t* __restrict__ tile_e,
                                               int32_t* __restrict__ queue) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (queue && t < 8) queue[t] = 0;
  if (t > T) return;
  const int64_t E = rowptr[n_rows];
  int64_t r = (t == 0) ? 0 : (t == T ? n_rows : lower_bound_i32(rowptr, n_rows + 1, (t * E) / T));
  if (r > n_rows) r = n_rows;
  tile_r[t] = (int32_t)r;
  tile_e[t] = rowptr[r];
}

hipError_t launch_tiles(const DevGraph& g, int32_t* tile_r, int32_t* tile_e, int32_t* queue, hipStream_t s) {
  const int grid = (int)((g.n_tiles + 1 + 255) / 256);
  hipLaunchKernelGGL(k_tiles, dim3(grid), dim3(256), 0, s, g.rowptr, g.n_rows, g.n_tiles, tile_r, tile_e, queue);
  return hipGetLastError();
}

// Eq. 4a-b, one row-aligned tile at a time per wave (schedule: tile_sched).
// For every directed edge k (receiver i, sender j):
//   h  = P_i + Q_j + W1c e_k             (first Linear of the edge MLP)
//   m  = W2 ELU(h) + b2  [-> LayerNorm]  (second Linear)
//   e'_k = e_k + m                        (residual edge update)
// and a_i = sum_k e'_k / d_k over the receiver's edges, formed by a
// segmented scan across the 16 edges of each block with the open row
// carried into the next block.  Every row's sum is written once by the lane
// holding its last edge; no atomics, so results are bitwise reproducible.
// AM: aggregate the MLP output (message) instead of the updated state.
// DQ: take tiles from the per-XCD atomic counters (queue_next) instead of
// the fixed round robin of tile_sched.  ES: e_in and e_out hold BF16 (the
// update and the aggregation run in FP32; e' is rounded where it is stored).
template <int H, bool BF, bool AM, bool DQ, bool ES>
__global__ __launch_bounds__(256, (H <= 64 ? 4 : 2)) void k_edge_fwd(DevGraph gr, const float* __restrict__ P,
                                                  const float* __restrict__ Q, const void* __restrict__ e_in,
                                                  const void* __restrict__ frag, const float* __restrict__ b2,
                                                  const float* __restrict__ lng, const float* __restrict__ lnb,
                                                  int ln, float eps, void* __restrict__ e_out,
                                                  float* __restrict__ a_out) {
  constexpr int NF = H / 4, MB = H / 16;
  constexpr size_t FB = frag_bytes(H, H, BF);
  constexpr bool LDS = 2 * FB <= kEdgeLdsBudget;
  extern __shared__ uint4 smem[];
  const char* fr;
  // per-feature vectors (b2, LayerNorm gain and shift) live in LDS after the
  // fragments and are re-read per block rather than held in registers
  float* vecs = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + (LDS ? 2 * FB : 0));
  // the open row's partial sum, handed from lane 15 of one block to lane 0
  // of the next through LDS (same wave, so no barrier is needed)
  float* carry = vecs + 3 * H + (threadIdx.x / 64) * H + (threadIdx.x / 16 % 4) * (H / 4);
  for (int t = threadIdx.x; t < 3 * H; t += blockDim.x)
    vecs[t] = t < H ? b2[t] : (ln ? (t < 2 * H ? lng[t - H] : lnb[t - 2 * H]) : 0.f);
  if constexpr (LDS) {
    stage_to_lds(smem, frag, 2 * FB);
    fr = reinterpret_cast<const char*>(smem);
  } else {
    fr = reinterpret_cast<const char*>(frag);
  }
  __syncthreads();
  const int lane = lane_id(), j = lane & 15, g = lane >> 4;
  const int nw = blockDim.x / 64;
  const TileSched ts = tile_sched(gr.n_tiles);
  const int64_t V = gridDim.x < 8 ? gridDim.x : 8;
  const int x0 = (int)(blockIdx.x % V);
  int qi = 0;

  for (int64_t tile = DQ ? queue_next(gr.queue, gr.n_tiles, V, x0, qi) : ts.t0 + ts.rank * nw + threadIdx.x / 64;
       DQ ? tile >= 0 : tile < ts.t1;
       tile = DQ ? queue_next(gr.queue, gr.n_tiles, V, x0, qi) : tile + ts.nr * nw) {
    const int64_t r0 = gr.tile_r[tile], r1 = gr.tile_r[tile + 1];
    const int64_t e0 = gr.tile_e[tile], e1 = gr.tile_e[tile + 1];
    int carry_key = 0;  // no open row at the start of a tile

    // Index loads run one block ahead (issued before the block's row
    // loads), so each block waits on one round trip to memory, for its rows.
    const int64_t e_last = e1 > e0 ? e1 - 1 : 0;  // in-bounds stand-in for absent edges
    int ri_n, sj_n, md_n, nx_n;
    {
      const int64_t k = e0 + j, kk = k < e1 ? k : e_last;
      ri_n = gr.recv[kk];
      sj_n = gr.col[kk];
      md_n = gr.mult[kk];
      nx_n = (k + 1 < e1) ? gr.recv[k + 1] : -1;
      // complete these here: the loop's entry state then holds no pending
      // loads, so the compiler's wait at the loop head (merged with the
      // back edge) does not also drain the previous block's stores
      asm volatile("" : "+v"(ri_n), "+v"(sj_n), "+v"(md_n), "+v"(nx_n));
    }

    for (int64_t base = e0; base < e1; base += 16) {
      const char* frb = fr + opaque_zero();  // re-read the fragments each block
      const int64_t k = base + j;
      const bool valid = k < e1;
      const int64_t kk = valid ? k : e_last;
      const int ri = ri_n;
      const int sj = sj_n;
      const float inv_d = 1.f / (float)md_n;
      const int next = nx_n;
      const bool last = valid && next != ri;
      const int key = valid ? ri + 1 : -1;
      {
        const int64_t k2 = k + 16, kk2 = k2 < e1 ? k2 : e_last;
        ri_n = gr.recv[kk2];
        sj_n = gr.col[kk2];
        md_n = gr.mult[kk2];
        nx_n = (k2 + 1 < e1) ? gr.recv[k2 + 1] : -1;
      }

      float ev[NF], h[NF], q[NF];
      load_row_t<H, ES>(e_in, kk, g, ev);
      load_row<H>(P + (int64_t)ri * H, g, h);
      load_row<H>(Q + (int64_t)sj * H, g, q);
      __builtin_amdgcn_sched_barrier(0);  // all row loads issue before any use
#pragma unroll
      for (int i = 0; i < NF; ++i) h[i] += q[i];
      gemm<BF, MB, MB>(frb, ev, h, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) h[i] = elu(h[i]);
      float m[NF];
      const float* vb = vecs + opaque_zero();
      load_vec<H>(vb, g, m);
      gemm<BF, MB, MB>(frb + FB, h, m, lane);
      if (ln) {
        float mean, rstd, gam[NF], bet[NF];
        ln_stats<H>(m, eps, mean, rstd);
        load_vec<H>(vb + H, g, gam);
        load_vec<H>(vb + 2 * H, g, bet);
#pragma unroll
        for (int i = 0; i < NF; ++i) m[i] = (m[i] - mean) * rstd * gam[i] + bet[i];
      }
#pragma unroll
      for (int i = 0; i < NF; ++i) ev[i] += m[i];
      if (valid && e_out) store_row_t<H, ES>(e_out, k, g, ev);  // no e' for a last layer

      // aggregation: segmented scan of e'/d across the block, plus carry.
      // Lanes past the tile's last edge (finite values from an in-bounds
      // edge, a key of their own) add nothing to any row's sum.
#pragma unroll
      for (int i = 0; i < NF; ++i) ev[i] = (AM ? m[i] : ev[i]) * inv_d;
      if (j == 0 && key == carry_key) {
#pragma unroll
        for (int i = 0; i < NF; i += 4) {
          const float4 c = *reinterpret_cast<const float4*>(carry + i);
          ev[i] += c.x;
          ev[i + 1] += c.y;
          ev[i + 2] += c.z;
          ev[i + 3] += c.w;
        }
      }
      seg_scan16<NF>(ev, key);
      if (last) store_row<H>(a_out + (int64_t)ri * H, g, ev);
      if (j == 15) {
#pragma unroll
        for (int i = 0; i < NF; i += 4) *reinterpret_cast<float4*>(carry + i) = make_float4(ev[i], ev[i + 1], ev[i + 2], ev[i + 3]);
      }
      carry_key = from_prev_lane_i(key);
    }
    // rows without incoming edges aggregate to zero
    for (int64_t r = r0 + (lane >> 2); r < r1; r += 16) {
      if (gr.rowptr[r] == gr.rowptr[r + 1]) {
        float* dst = a_out + r * H;
        for (int c = (lane & 3) * 4; c < H; c += 16) *reinterpret_cast<float4*>(dst + c) = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }
}

template <int H, bool BF, bool AM, bool DQ, bool ES>
static hipError_t launch_edge_fwd_t(const DevGraph& g, const float* P, const float* Q, const void* e_in,
                                    const void* frag, const float* b2, const float* lng, const float* lnb, int ln,
                                    float eps, void* e_out, float* a_out, int grid, hipStream_t s) {
  constexpr size_t FB = frag_bytes(H, H, BF);
  // fragments, 3 per-feature vectors, per-wave carries (4 waves)
  const size_t lds = ((2 * FB <= kEdgeLdsBudget) ? 2 * FB : 0) + 3 * H * sizeof(float) + 4 * H * sizeof(float);
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_edge_fwd<H, BF, AM, DQ, ES>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL((k_edge_fwd<H, BF, AM, DQ, ES>), dim3(grid), dim3(256), lds, s, g, P, Q, e_in, frag, b2, lng, lnb,
                     ln, eps, e_out, a_out);
  return hipGetLastError();
}

template <int H, bool BF, bool ES>
static hipError_t launch_edge_fwd_am(bool am, bool dq, const DevGraph& g, const float* P, const float* Q,
                                     const void* e_in, const void* frag, const float* b2, const float* lng,
                                     const float* lnb, int ln, float eps, void* e_out, float* a_out, int grid,
                                     hipStream_t s) {
#define MP_EFWD(AMV, DQV) \
  launch_edge_fwd_t<H, BF, AMV, DQV, ES>(g, P, Q, e_in, frag, b2, lng, lnb, ln, eps, e_out, a_out, grid, s)
  if (dq) return am ? MP_EFWD(true, true) : MP_EFWD(false, true);
  return am ? MP_EFWD(true, false) : MP_EFWD(false, false);
#undef MP_EFWD
}

hipError_t launch_edge_fwd(int H, bool ln, bool bf, bool am, bool dq, bool es, const DevGraph& g, const float* P,
                           const float* Q, const void* e_in, const void* frag, const float* b2, const float* lng,
                           const float* lnb, float eps, void* e_out, float* a_out, int grid, hipStream_t s) {
  if (es && !bf) return hipErrorInvalidValue;  // BF16 edge states go with BF16 products
#define MP_CASE(HH)                                                                                              \
  if (H == HH) {                                                                                                 \
    if (bf && es)                                                                                                \
      return launch_edge_fwd_am<HH, true, true>(am, dq, g, P, Q, e_in, frag, b2, lng, lnb, ln, eps, e_out, a_out, \
                                                grid, s);                                                        \
    return bf ? launch_edge_fwd_am<HH, true, false>(am, dq, g, P, Q, e_in, frag, b2, lng, lnb, ln, eps, e_out,    \
                                                    a_out, grid, s)                                              \
              : launch_edge_fwd_am<HH, false, false>(am, dq, g, P, Q, e_in, frag, b2, lng, lnb, ln, eps, e_out,   \
                                                     a_out, grid, s);                                            \
  }
  MP_CASE(32) MP_CASE(64) MP_CASE(128)
#undef MP_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------- halo sum

// Eq. 4c-d on one GPU: every group lists the rows (one per sub-graph) that
// hold one global id.  Each copy receives the sum of all copies' local
// aggregates, added in ascending row order; rows in no group keep a.
// One thread per (group, 4 features); groups are disjoint, so the update
// in place is race free.
template <int H>
__global__ __launch_bounds__(256) void k_halo(int64_t n_groups, const int32_t* __restrict__ gptr,
                                              const int32_t* __restrict__ member, float* __restrict__ a) {
  constexpr int C = H / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t grp = t / C;
  if (grp >= n_groups) return;
  const int c = (int)(t % C) * 4;
  const int m0 = gptr[grp], m1 = gptr[grp + 1];
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int m = m0; m < m1; ++m) {
    const float4 v = *reinterpret_cast<const float4*>(a + (int64_t)member[m] * H + c);
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
    s.w += v.w;
  }
  for (int m = m0; m < m1; ++m) *reinterpret_cast<float4*>(a + (int64_t)member[m] * H + c) = s;
}

hipError_t launch_halo(int H, const DevGraph& g, float* a, hipStream_t s) {
  if (g.n_groups == 0) return hipSuccess;
  const int64_t threads = g.n_groups * (H / 4);
  const int grid = (int)((threads + 255) / 256);
  if (H == 8) hipLaunchKernelGGL(k_halo<8>, dim3(grid), dim3(256), 0, s, g.n_groups, g.group_ptr, g.member, a);
  else if (H == 16) hipLaunchKernelGGL(k_halo<16>, dim3(grid), dim3(256), 0, s, g.n_groups, g.group_ptr, g.member, a);
  else if (H == 32) hipLaunchKernelGGL(k_halo<32>, dim3(grid), dim3(256), 0, s, g.n_groups, g.group_ptr, g.member, a);
  else if (H == 64) hipLaunchKernelGGL(k_halo<64>, dim3(grid), dim3(256), 0, s, g.n_groups, g.group_ptr, g.member, a);
  else if (H == 128) hipLaunchKernelGGL(k_halo<128>, dim3(grid), dim3(256), 0, s, g.n_groups, g.group_ptr, g.member, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------- row MLPs

// out = [resid +] [LN] (W1 ELU(W0 in + b0) + b1), in = [src0, src1].
// TIN: in has k0 <= 4 features; the first Linear is done with FMAs from
// the raw weights.  TOUT: n_out < 16 outputs; the second Linear is done
// with FMAs and a reduction over the four lanes of each row.
//
// Each wave walks its 16-row blocks software-pipelined: the next block's
// inputs are loaded before this block is computed and stored, so a block
// waits on memory only for loads issued one block earlier.  Per-feature
// vectors (b0, b1, LayerNorm gain and shift) and small weights sit in LDS.
template <int H, int KIN, bool TIN, bool TOUT>
struct MlpFwdIn {
  static constexpr int NF = H / 4, NIN = TIN ? 4 : KIN / 4;
  float in[NIN];
  float r[(KIN == 2 * H || TIN || TOUT) ? 1 : NF];  // residual row when it is not src1
  __device__ __forceinline__ void load(const MlpFwdArgs& a, int64_t rr, int g, bool sep_resid) {
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
      if constexpr (!TOUT) {
        if (sep_resid) load_row<H>(a.resid + rr * H, g, r);
      }
    }
  }
  __device__ __forceinline__ void settle() {
#pragma unroll
    for (int i = 0; i < NIN; ++i) asm volatile("" : "+v"(in[i]));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(r) / sizeof(float)); ++i) asm volatile("" : "+v"(r[i]));
  }
};

template <int H, int KIN, bool TIN, bool TOUT, bool BF>
struct MlpFwdCfg {
  static constexpr size_t F0 = TIN ? 0 : frag_bytes(H, KIN, BF);
  static constexpr size_t F1 = TOUT ? 0 : frag_bytes(H, H, BF);
  static constexpr bool LDS_FRAG = (F0 + F1) <= kRowMlpLdsBudget;
  static constexpr size_t SMALL = (TIN || TOUT) ? 16 * H : 0;  // small W0 [H][4] or W1 [4][H]
  static constexpr size_t VECS = 4 * H * sizeof(float);        // b0, b1, LayerNorm gain, shift
  // when both do not fit (FP32, H = 128, 2H inputs), W0 alone may: the larger
  // matrix is then read from LDS and only W1 from L2
  static constexpr bool LDS_F0 = !LDS_FRAG && F0 > 0 && F0 + SMALL + VECS <= kRowMlpLdsMax;
  static constexpr size_t FRAG_LDS = LDS_FRAG ? F0 + F1 : (LDS_F0 ? F0 : 0);
  static constexpr size_t LDS = FRAG_LDS + SMALL + VECS;
};

// OB: the H-wide output is stored as BF16 (the edge encoder's output, an
// edge state, when edge states are BF16).
template <int H, int KIN, bool TIN, bool TOUT, bool BF, bool OB>
__global__ __launch_bounds__(256, (H <= 64 ? 4 : 1)) void k_mlp_fwd(MlpFwdArgs a) {
  using C = MlpFwdCfg<H, KIN, TIN, TOUT, BF>;
  constexpr int NF = H / 4, MB = H / 16, KB = TIN ? 1 : KIN / 16;
  extern __shared__ uint4 smem[];
  const char* f0;
  const char* f1;
  float* small = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + C::FRAG_LDS);
  float* vecs = small + C::SMALL / 4;
  if constexpr (TIN) stage_small(small, a.W0, H, a.k0);
  if constexpr (TOUT)
    for (int t = threadIdx.x; t < 4 * H; t += blockDim.x) small[t] = (t / H) < a.n_out ? a.W1[t] : 0.f;
  for (int t = threadIdx.x; t < 4 * H; t += blockDim.x) {
    const int q = t / H, f = t % H;
    vecs[t] = q == 0 ? a.b0[f] : q == 1 ? (TOUT ? 0.f : a.b1[f]) : q == 2 ? (a.ln ? a.lng[f] : 0.f) : (a.ln ? a.lnb[f] : 0.f);
  }
  if constexpr (C::LDS_FRAG) {
    if (C::F0) stage_to_lds(smem, a.frag0, C::F0);
    if (C::F1) stage_to_lds(smem + C::F0 / 16, a.frag1, C::F1);
    f0 = reinterpret_cast<const char*>(smem);
    f1 = f0 + C::F0;
  } else if constexpr (C::LDS_F0) {
    stage_to_lds(smem, a.frag0, C::F0);
    f0 = reinterpret_cast<const char*>(smem);
    f1 = reinterpret_cast<const char*>(a.frag1);
  } else {
    f0 = reinterpret_cast<const char*>(a.frag0);
    f1 = reinterpret_cast<const char*>(a.frag1);
  }
  __syncthreads();
  const int lane = lane_id(), j = lane & 15, g = lane >> 4;
  const int nw = blockDim.x / 64;
  const int64_t n = a.n_rows, nblk = (n + 15) / 16, stride = (int64_t)gridDim.x * nw;
  // the residual is src1 for the node update; otherwise it is a row of its own
  const bool sep_resid = !TOUT && a.resid != nullptr && !(KIN == 2 * H && a.resid == a.src1);
  const bool has_resid = !TOUT && a.resid != nullptr;

  int64_t blk = (int64_t)blockIdx.x * nw + threadIdx.x / 64;
  MlpFwdIn<H, KIN, TIN, TOUT> nx;
  nx.load(a, std::min<int64_t>(blk * 16 + j, n - 1), g, sep_resid);
  nx.settle();  // the loop's entry state holds no pending loads
  for (; blk < nblk; blk += stride) {
    const int64_t row = blk * 16 + j;
    const bool valid = row < n;
    const MlpFwdIn<H, KIN, TIN, TOUT> cur = nx;
    nx.load(a, std::min<int64_t>((blk + stride) * 16 + j, n - 1), g, sep_resid);
    __builtin_amdgcn_sched_barrier(0);

    const float* vb = vecs + opaque_zero();  // re-read the vectors each block
    float z[NF];
    load_vec<H>(vb, g, z);
    if constexpr (TIN) {
      small_in_linear<H>(small + opaque_zero(), cur.in, g, z);
    } else {
      gemm<BF, MB, KB>(f0 + opaque_zero(), cur.in, z, lane);
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) z[i] = elu(z[i]);
    if constexpr (TOUT) {
      float p[4];
      for (int o = 0; o < 4; ++o) {
        float w[NF];
        load_vec<H>(small + o * H, g, w);
        float t = 0.f;
#pragma unroll
        for (int i = 0; i < NF; ++i) t += w[i] * z[i];
        p[o] = row_sum(t);
      }
      nx.settle();  // next block's loads complete before this block's stores
      for (int o = 0; o < a.n_out; ++o)
        if (valid && g == 0) reinterpret_cast<float*>(a.out)[row * a.n_out + o] = p[o] + a.b1[o];
    } else {
      float y[NF];
      load_vec<H>(vb + H, g, y);
      gemm<BF, MB, MB>(f1 + opaque_zero(), z, y, lane);
      if (a.ln) {
        float mean, rstd, gm[NF], bt[NF];
        load_vec<H>(vb + 2 * H, g, gm);
        load_vec<H>(vb + 3 * H, g, bt);
        ln_stats<H>(y, a.eps, mean, rstd);
#pragma unroll
        for (int i = 0; i < NF; ++i) y[i] = (y[i] - mean) * rstd * gm[i] + bt[i];
      }
      if (has_resid) {
        if constexpr (KIN == 2 * H) {
          if (!sep_resid) {
#pragma unroll
            for (int i = 0; i < NF; ++i) y[i] += cur.in[NF + i];
          }
        } else if constexpr (!TIN) {
#pragma unroll
          for (int i = 0; i < NF; ++i) y[i] += cur.r[i];
        }
      }
      nx.settle();  // next block's loads complete before this block's stores
      if (valid) store_row_t<H, OB>(a.out, row, g, y);
    }
  }
}

template <int H, int KIN, bool TIN, bool TOUT, bool BF, bool OB = false>
static hipError_t launch_mlp_fwd_t(const MlpFwdArgs& a, int grid, hipStream_t s) {
  using C = MlpFwdCfg<H, KIN, TIN, TOUT, BF>;
  // residual rows other than src1 exist only for the H-input form
  if (a.resid && !(KIN == H && !TIN && !TOUT) && !(KIN == 2 * H && a.resid == a.src1)) return hipErrorInvalidValue;
  if (C::LDS > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_mlp_fwd<H, KIN, TIN, TOUT, BF, OB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
  hipLaunchKernelGGL((k_mlp_fwd<H, KIN, TIN, TOUT, BF, OB>), dim3(grid), dim3(256), C::LDS, s, a);
  return hipGetLastError();
}

template <int H, bool BF>
static hipError_t launch_mlp_fwd_h(const MlpFwdArgs& a, int grid, hipStream_t s) {
  const bool tin = a.k0 <= 4, tout = a.n_out < 16;
  const int kin = a.k0 + a.k1;
  if (a.out_bf && !(tin && !tout && BF)) return hipErrorInvalidValue;
  if constexpr (BF) {
    if (tin && !tout && a.out_bf) return launch_mlp_fwd_t<H, 4, true, false, BF, true>(a, grid, s);
  }
  if (tin && !tout) return launch_mlp_fwd_t<H, 4, true, false, BF>(a, grid, s);
  if (!tin && kin == H && tout) return launch_mlp_fwd_t<H, H, false, true, BF>(a, grid, s);
  if (!tin && kin == H && !tout) return launch_mlp_fwd_t<H, H, false, false, BF>(a, grid, s);
  if (!tin && kin == 2 * H && !tout) return launch_mlp_fwd_t<H, 2 * H, false, false, BF>(a, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_fwd(const MlpFwdArgs& a, int grid, hipStream_t s) {
#define MP_CASE(HH) \
  if (a.H == HH) return a.bf ? launch_mlp_fwd_h<HH, true>(a, grid, s) : launch_mlp_fwd_h<HH, false>(a, grid, s);
  MP_CASE(32) MP_CASE(64) MP_CASE(128)
#undef MP_CASE
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------- edge inputs

// Edge features of Sec. III: (p_j - p_i, |p_j - p_i|) with i the receiver
// and j the sender, differences in FP64, rounded once to FP32.  On an axis
// with period L > 0 the difference is taken to the nearest image of p_j.
__device__ inline double nearest_image(double d, double L) { return L > 0.0 ? d - L * rint(d / L) : d; }

// With a node field u, three more channels: u_j - u_i (the relative
// velocity of the edge features Sec. III lists), an FP32 difference.
__global__ __launch_bounds__(256) void k_edge_inputs(int64_t n_edges, const int32_t* __restrict__ recv,
                                                     const int32_t* __restrict__ col, const double* __restrict__ pos,
                                                     double Lx, double Ly, double Lz, const float* __restrict__ u,
                                                     float* __restrict__ e0) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_edges) return;
  const int64_t i = recv[k], jj = col[k];
  const double dx = nearest_image(pos[3 * jj] - pos[3 * i], Lx);
  const double dy = nearest_image(pos[3 * jj + 1] - pos[3 * i + 1], Ly);
  const double dz = nearest_image(pos[3 * jj + 2] - pos[3 * i + 2], Lz);
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (!u) {
    *reinterpret_cast<float4*>(e0 + 4 * k) = make_float4((float)dx, (float)dy, (float)dz, (float)r);
    return;
  }
  float* o = e0 + 7 * k;
  o[0] = (float)dx;
  o[1] = (float)dy;
  o[2] = (float)dz;
  o[3] = (float)r;
  o[4] = u[3 * jj] - u[3 * i];
  o[5] = u[3 * jj + 1] - u[3 * i + 1];
  o[6] = u[3 * jj + 2] - u[3 * i + 2];
}

hipError_t launch_edge_inputs(const DevGraph& g, const double* pos, const double period[3], const float* u,
                              float* e0, hipStream_t s) {
  if (g.n_edges == 0) return hipSuccess;
  const int grid = (int)((g.n_edges + 255) / 256);
  hipLaunchKernelGGL(k_edge_inputs, dim3(grid), dim3(256), 0, s, g.n_edges, g.recv, g.col, pos, period[0],
                     period[1], period[2], u, e0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ loss

// Eq. 6: per block, FP64 partial sums over a fixed row range of
// S = sum (1/d_i)(Y - T)^2 and N = sum 1/d_i; block tree in fixed order.
__global__ __launch_bounds__(256) void k_loss_part(int64_t n_rows, int F, const float* __restrict__ Y,
                                                   const float* __restrict__ T, const uint8_t* __restrict__ mult,
                                                   double* __restrict__ part) {
  __shared__ double sS[256], sN[256];
  const int64_t per = (n_rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n_rows, r0 + per);
  double S = 0.0, N = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const double w = 1.0 / (double)mult[r];
    double e = 0.0;
    for (int f = 0; f < F; ++f) {
      const double d = (double)Y[r * F + f] - (double)T[r * F + f];
      e += d * d;
    }
    S += w * e;
    N += w;
  }
  sS[threadIdx.x] = S;
  sN[threadIdx.x] = N;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sS[threadIdx.x] += sS[threadIdx.x + o];
      sN[threadIdx.x] += sN[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sS[0];
    part[2 * blockIdx.x + 1] = sN[0];
  }
}

// Sum the block partials in block order (single thread: a few hundred
// values) and publish loss and N_eff.
__global__ void k_loss_final(int n_part, int F, const double* __restrict__ part, double* __restrict__ tot,
                             float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double S = 0.0, N = 0.0;
  for (int b = 0; b < n_part; ++b) {
    S += part[2 * b];
    N += part[2 * b + 1];
  }
  tot[0] = S;
  tot[1] = N;
  *loss = (float)(S / (N * F));
}

__global__ __launch_bounds__(256) void k_loss_grad(int64_t n, int F, const float* __restrict__ Y,
                                                   const float* __restrict__ T, const uint8_t* __restrict__ mult,
                                                   const double* __restrict__ tot, float* __restrict__ gY) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t r = t / F;
  const double c = 2.0 / (tot[1] * F * (double)mult[r]);
  gY[t] = (float)(c * ((double)Y[t] - (double)T[t]));
}

hipError_t launch_loss(int64_t n_rows, int F, const float* Y, const float* T, const uint8_t* mult, double* part,
                       int n_part, float* loss, float* gY, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_part, dim3(n_part), dim3(256), 0, s, n_rows, F, Y, T, mult, part);
  double* tot = part + 2 * n_part;
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, n_part, F, part, tot, loss);
  if (gY) {
    const int grid = (int)((n_rows * F + 255) / 256);
    hipLaunchKernelGGL(k_loss_grad, dim3(grid), dim3(256), 0, s, n_rows, F, Y, T, mult, tot, gY);
  }
  return hipGetLastError();
}

}  // namespace mp
