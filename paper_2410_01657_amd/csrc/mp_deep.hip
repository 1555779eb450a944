// Narrow deep MLPs: the paper's own models (Table I: hidden width 8 or 32,
// two or five extra H -> H layers in every MLP), for the consistent layer
// (Eq. 4a-e), the encoders and the decoder.
//
// At these widths a 16 x 16 matrix-core tile is mostly padding (H = 8) and
// the products are small, so one thread owns one row (a node, or a
// receiver with its incoming edges) and runs the whole MLP in registers
// with FP32 FMAs.  The MLP's weights sit in LDS in the order the products
// read them: every lane of a wave reads the same address (an LDS
// broadcast), four weights per read.
//
// Forward: k_deep_edge_fwd walks each receiver's incoming edges in CSR
// order, updates every edge (Eq. 4a, residual) and sums e'/d_ij into the
// receiver (Eq. 4b) in that order, so no scan or atomic is needed.  The
// halo sum (Eq. 4c-d) is the shared k_halo; k_deep_row_fwd is the node
// update (Eq. 4e), the encoders and the decoder.
//
// Adjoint (Eq. 3): each row recomputes its MLP and writes, to a per-row
// record in the workspace, the MLP input, every hidden activation, every
// pre-activation gradient and the LayerNorm terms; input gradients leave
// the row kernels directly.  The records are stored column by column in
// blocks of 64 rows, so a wave's store of one column is one contiguous run
// of memory and no cache line is left half written.  The edge adjoint runs
// one thread per edge.  Weight gradients are then sums over rows of
// outer products of record columns, formed per chunk of rows on the matrix
// unit by k_outer_sum and added chunk by chunk in a fixed order
// (k_wreduce), so results are bitwise reproducible.  The sender-side input gradient of
// each edge is written per edge and gathered at the sender through the
// reverse-edge index (k_deep_gather), in CSR order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mp_device.hpp"
#include "mp_kernels.hpp"

namespace mp {

// LDS image of one MLP, zero padded to compile-time widths: input KM
// columns, output OM rows.  Layout (floats): W0[H][KM] b0[H],
// NH x (W[H][H] b[H]), Wo[OM][H] bo[OM] gamma[OM] beta[OM].
template <int H, int KM, int OM>
struct DeepLds {
  int NH;
  __host__ __device__ static constexpr int w0() { return 0; }
  __host__ __device__ static constexpr int b0() { return H * KM; }
  __host__ __device__ int wh(int l) const { return H * KM + H + l * (H * H + H); }
  __host__ __device__ int bh(int l) const { return wh(l) + H * H; }
  __host__ __device__ int wo() const { return wh(NH); }
  __host__ __device__ int bo() const { return wo() + OM * H; }
  __host__ __device__ int lg() const { return bo() + OM; }
  __host__ __device__ int lb() const { return lg() + OM; }
  __host__ __device__ int size() const { return lb() + OM; }
};

// Per-row record columns: in[KM], h_0..h_NH [H each], d_0..d_NH [H each]
// (gradients at the pre-activations), d_out[OM], then with LayerNorm
// (g_y * y_hat)[OM] and g_y[OM].
template <int H, int KM, int OM>
struct DeepRec {
  int NH, ln;
  __host__ __device__ static constexpr int in() { return 0; }
  __host__ __device__ static constexpr int h(int l) { return KM + l * H; }
  __host__ __device__ int d(int l) const { return KM + (NH + 1) * H + l * H; }
  __host__ __device__ int dout() const { return KM + 2 * (NH + 1) * H; }
  __host__ __device__ int lnr() const { return dout() + OM; }
  __host__ __device__ int size() const { return lnr() + (ln ? 2 * OM : 0); }
};

// Copy the flat parameter array (torch.nn.Linear order) into the LDS image.
// The MLP's input is [src_a (ka features, padded to KAM), src_b (KM - KAM)].
template <int H, int KM, int OM>
__device__ void stage_deep(float* __restrict__ L, const float* __restrict__ theta, const DeepLds<H, KM, OM>& m,
                           int ka, int kam, int O, int ln) {
  const int K = ka + (KM - kam);  // the parameter array's input width
  for (int t = threadIdx.x; t < H * KM; t += blockDim.x) {
    const int r = t / KM, c = t % KM;
    const int sc = c < kam ? (c < ka ? c : -1) : ka + (c - kam);
    L[t] = sc >= 0 ? theta[(int64_t)r * K + sc] : 0.f;
  }
  const float* tb0 = theta + (int64_t)H * K;
  for (int t = threadIdx.x; t < H; t += blockDim.x) L[m.b0() + t] = tb0[t];
  const float* th = tb0 + H;  // hidden layers, same layout in both
  for (int t = threadIdx.x; t < m.NH * (H * H + H); t += blockDim.x) L[m.wh(0) + t] = th[t];
  const float* two = th + (int64_t)m.NH * (H * H + H);
  for (int t = threadIdx.x; t < OM * H; t += blockDim.x) L[m.wo() + t] = t / H < O ? two[t] : 0.f;
  const float* tbo = two + (int64_t)O * H;
  for (int t = threadIdx.x; t < OM; t += blockDim.x) {
    L[m.bo() + t] = t < O ? tbo[t] : 0.f;
    L[m.lg() + t] = (ln && t < O) ? tbo[O + t] : 0.f;
    L[m.lb() + t] = (ln && t < O) ? tbo[2 * O + t] : 0.f;
  }
}

// An opaque zero that is only available once `dep` is: an LDS address
// built from it cannot be read before dep has been computed.
__device__ __forceinline__ int opaque_zero_after(float dep) {
  int z = 0;
  asm volatile("" : "+v"(z) : "v"(dep));
  return z;
}

__device__ __forceinline__ int opaque_zero_after4(float d0, float d1, float d2, float d3) {
  int z = 0;
  asm volatile("" : "+v"(z) : "v"(d0), "v"(d1), "v"(d2), "v"(d3));
  return z;
}

// z = W x + b, W [N][M] row-major in LDS.
// Each block of four rows reads through a base that depends on the
// previous block's result, so the compiler cannot issue the whole matrix's
// reads up front (which would hold the matrix in registers and spill).
template <int N, int M>
__device__ __forceinline__ void dlin(const float* __restrict__ W, const float* __restrict__ b, const float (&x)[M],
                                     float (&z)[N]) {
  constexpr int RB = M >= 32 ? 1 : (M >= 16 ? 2 : 4);  // rows per block: at most 96 weights in flight
  const float* Wb = W;
#pragma unroll
  for (int o = 0; o < N; ++o) {
    if (o % RB == 0) Wb = W + (o ? opaque_zero_after(z[o - 1]) : opaque_zero());
    float s = b[o];
#pragma unroll
    for (int c = 0; c < M; c += 4) {
      const float4 w = *reinterpret_cast<const float4*>(Wb + o * M + c);
      s = fmaf(w.x, x[c], s);
      s = fmaf(w.y, x[c + 1], s);
      s = fmaf(w.z, x[c + 2], s);
      s = fmaf(w.w, x[c + 3], s);
    }
    z[o] = s;
    if (o % RB == RB - 1) __builtin_amdgcn_sched_barrier(0);  // bound the reads in flight
  }
}

// gx[c] = sum_o W[o][C0 + c] gz[o] for c < MW (a column block of W^T gz).
// Column blocks of four outermost, each reading through a base that depends
// on all four of the previous block's sums (as in dlin).
template <int N, int M, int C0, int MW>
__device__ __forceinline__ void dlin_t(const float* __restrict__ W, const float (&gz)[N], float (&gx)[MW]) {
#pragma unroll
  for (int c = 0; c < MW; c += 4) {
    const float* Wb = W + (c ? opaque_zero_after4(gx[c - 4], gx[c - 3], gx[c - 2], gx[c - 1]) : opaque_zero());
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
    for (int o = 0; o < N; ++o) {
      // eight rows in flight; all four sums gate the next reads (gating on
      // one would let the other three hold their weights in registers)
      if (o > 0 && o % 8 == 0) Wb = W + opaque_zero_after4(s0, s1, s2, s3);
      const float4 w = *reinterpret_cast<const float4*>(Wb + o * M + C0 + c);
      s0 = fmaf(w.x, gz[o], s0);
      s1 = fmaf(w.y, gz[o], s1);
      s2 = fmaf(w.z, gz[o], s2);
      s3 = fmaf(w.w, gz[o], s3);
    }
    gx[c] = s0;
    gx[c + 1] = s1;
    gx[c + 2] = s2;
    gx[c + 3] = s3;
    __builtin_amdgcn_sched_barrier(0);  // bound the reads in flight
  }
}

// Keep the scheduler from interleaving consecutive products (which would
// hold both products' weight reads in registers at once).
__device__ __forceinline__ void phase_fence() { __builtin_amdgcn_sched_barrier(0); }

// One row's record: column c at p[c * kRecRows] (p = rec + deep_rec_at(r, 0, rs)).
struct RecRef {
  float* p;
};
// NT: a column no kernel reads back before the weight-gradient pass, stored
// non-temporally so it does not displace the node rows the kernel gathers.
template <int W, bool NT = false>
__device__ __forceinline__ void rstore(const RecRef& r, int c0, const float (&v)[W]) {
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if constexpr (NT)
      __builtin_nontemporal_store(v[c], r.p + (c0 + c) * kRecRows);
    else
      r.p[(c0 + c) * kRecRows] = v[c];
  }
}
template <int W>
__device__ __forceinline__ void rload(const RecRef& r, int c0, float (&v)[W]) {
#pragma unroll
  for (int c = 0; c < W; ++c) v[c] = r.p[(c0 + c) * kRecRows];
}

template <int W>
__device__ __forceinline__ void vload(const float* __restrict__ p, float (&v)[W]) {
#pragma unroll
  for (int c = 0; c < W; c += 4) {
    const float4 t = *reinterpret_cast<const float4*>(p + c);
    v[c] = t.x;
    v[c + 1] = t.y;
    v[c + 2] = t.z;
    v[c + 3] = t.w;
  }
}
template <int W>
__device__ __forceinline__ void vstore(float* __restrict__ p, const float (&v)[W]) {
#pragma unroll
  for (int c = 0; c < W; c += 4) *reinterpret_cast<float4*>(p + c) = make_float4(v[c], v[c + 1], v[c + 2], v[c + 3]);
}

// MLP forward up to the last Linear's output u (before LayerNorm).  With
// REC, the hidden activations go to the row's record.
template <int H, int KM, int OM, bool REC>
__device__ __forceinline__ void deep_fwd(const float* __restrict__ L, const DeepLds<H, KM, OM>& m,
                                         const float (&in)[KM], float (&u)[OM], const RecRef& rec) {
  using R = DeepRec<H, KM, OM>;
  float h[H];
  dlin<H, KM>(L + m.w0(), L + m.b0(), in, h);
#pragma unroll
  for (int c = 0; c < H; ++c) h[c] = elu(h[c]);
  if constexpr (REC) rstore<H>(rec, R::h(0), h);
  phase_fence();
  for (int l = 0; l < m.NH; ++l) {
    float z[H];
    dlin<H, H>(L + m.wh(l), L + m.bh(l), h, z);
#pragma unroll
    for (int c = 0; c < H; ++c) h[c] = elu(z[c]);
    if constexpr (REC) rstore<H>(rec, R::h(l + 1), h);
    phase_fence();
  }
  dlin<OM, H>(L + m.wo(), L + m.bo(), h, u);
  phase_fence();
}

// LayerNorm over the OM features of one row (biased variance), in place.
template <int OM>
__device__ __forceinline__ void dln_stats(const float (&u)[OM], float eps, float& mean, float& rstd) {
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < OM; ++c) s += u[c];
  mean = s * (1.f / OM);
  float q = 0.f;
#pragma unroll
  for (int c = 0; c < OM; ++c) q += (u[c] - mean) * (u[c] - mean);
  rstd = 1.f / sqrtf(q * (1.f / OM) + eps);
}

template <int OM>
__device__ __forceinline__ void dln_fwd(const float* __restrict__ g, const float* __restrict__ b, float eps,
                                        float (&u)[OM]) {
  float mean, rstd;
  dln_stats<OM>(u, eps, mean, rstd);
#pragma unroll
  for (int c = 0; c < OM; ++c) u[c] = (u[c] - mean) * rstd * g[c] + b[c];
}

// Adjoint of LayerNorm: g_y -> g_u (in gy), recording g_y * y_hat and g_y.
template <int OM>
__device__ __forceinline__ void dln_bwd(const float* __restrict__ g, float eps, const float (&u)[OM], float (&gy)[OM],
                                        const RecRef& rec, int c_ln) {
  float mean, rstd;
  dln_stats<OM>(u, eps, mean, rstd);
  float yh[OM], gyh[OM], m1 = 0.f, m2 = 0.f;
#pragma unroll
  for (int c = 0; c < OM; ++c) {
    yh[c] = (u[c] - mean) * rstd;
    gyh[c] = gy[c] * g[c];
    m1 += gyh[c];
    m2 += gyh[c] * yh[c];
  }
  m1 *= 1.f / OM;
  m2 *= 1.f / OM;
  float t[OM];
#pragma unroll
  for (int c = 0; c < OM; ++c) t[c] = gy[c] * yh[c];
  rstore<OM, true>(rec, c_ln, t);
  rstore<OM, true>(rec, c_ln + OM, gy);
#pragma unroll
  for (int c = 0; c < OM; ++c) gy[c] = rstd * (gyh[c] - m1 - yh[c] * m2);
}

// Back through the Linears given g_u (the gradient at the last Linear's
// output): records every pre-activation gradient and returns the first
// Linear's in d0.
template <int H, int KM, int OM>
__device__ __forceinline__ void deep_bwd(const float* __restrict__ L, const DeepLds<H, KM, OM>& m,
                                         const DeepRec<H, KM, OM>& rr, const float (&gu)[OM],
                                         const RecRef& rec, float (&d0)[H]) {
  rstore<OM, true>(rec, rr.dout(), gu);
  float gh[H];
  dlin_t<OM, H, 0, H>(L + m.wo(), gu, gh);
  phase_fence();
  for (int l = m.NH; l >= 0; --l) {
    float hl[H];
    rload<H>(rec, rr.h(l), hl);
#pragma unroll
    for (int c = 0; c < H; ++c) d0[c] = gh[c] * (hl[c] > 0.f ? 1.f : hl[c] + 1.f);  // ELU' from ELU's value
    rstore<H, true>(rec, rr.d(l), d0);
    if (l > 0) dlin_t<H, H, 0, H>(L + m.wh(l - 1), d0, gh);
    phase_fence();
  }
}

// ------------------------------------------------------------- row MLPs

// Input [src_a (ka <= KAM features), src_b (KB features)]; output O <= OM.
// SI: src_a is a narrow input (rows of ka floats, not 16-byte aligned).
template <int H, int KAM, int KB, int OM, bool SI>
struct DeepRowK {
  static constexpr int KM = KAM + KB;
  static __device__ __forceinline__ void load_in(const DeepRowArgs& a, int64_t r, float (&in)[KM]) {
    if constexpr (SI) {
#pragma unroll
      for (int c = 0; c < KAM; ++c) in[c] = c < a.ka ? a.src_a[r * a.ka + c] : 0.f;
    } else {
      float t[KAM];
      vload<KAM>(a.src_a + r * KAM, t);
#pragma unroll
      for (int c = 0; c < KAM; ++c) in[c] = t[c];
    }
    if constexpr (KB > 0) {
      float t[KB];
      vload<KB>(a.src_b + r * KB, t);
#pragma unroll
      for (int c = 0; c < KB; ++c) in[KAM + c] = t[c];
    }
  }
};

template <int H, int KAM, int KB, int OM, bool SI>
__global__ __launch_bounds__(256) void k_deep_row_fwd(DeepRowArgs a) {
  extern __shared__ float L[];
  using K = DeepRowK<H, KAM, KB, OM, SI>;
  const DeepLds<H, K::KM, OM> m{a.NH};
  stage_deep<H, K::KM, OM>(L, a.theta, m, a.ka, KAM, a.O, a.ln);
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n_rows) return;
  float in[K::KM];
  K::load_in(a, r, in);
  float u[OM];
  deep_fwd<H, K::KM, OM, false>(L, m, in, u, RecRef{nullptr});
  if (a.ln) dln_fwd<OM>(L + m.lg(), L + m.lb(), a.eps, u);
  if constexpr (OM < 8) {
#pragma unroll
    for (int c = 0; c < OM; ++c)
      if (c < a.O) a.out[r * a.O + c] = u[c];
  } else {
    if constexpr (KB == OM) {
      if (a.resid) {
#pragma unroll
        for (int c = 0; c < OM; ++c) u[c] += in[KAM + c];
      }
    }
    vstore<OM>(a.out + r * OM, u);
  }
}

template <int H, int KAM, int KB, int OM, bool SI>
__global__ __launch_bounds__(256) void k_deep_row_bwd(DeepRowArgs a) {
  extern __shared__ float L[];
  using K = DeepRowK<H, KAM, KB, OM, SI>;
  const DeepLds<H, K::KM, OM> m{a.NH};
  const DeepRec<H, K::KM, OM> rr{a.NH, a.ln};
  stage_deep<H, K::KM, OM>(L, a.theta, m, a.ka, KAM, a.O, a.ln);
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n_rows) return;
  const RecRef rec{a.rec + deep_rec_at(r, 0, a.rs)};
  float d0[H];
  {
    float gy[OM];
    float in[K::KM];
    K::load_in(a, r, in);
    rstore<K::KM, true>(rec, rr.in(), in);
    float u[OM];
    deep_fwd<H, K::KM, OM, true>(L, m, in, u, rec);
    if constexpr (OM < 8) {
#pragma unroll
      for (int c = 0; c < OM; ++c) gy[c] = c < a.O ? a.g_out[r * a.O + c] : 0.f;
    } else {
      vload<OM>(a.g_out + r * OM, gy);
    }
    float gu[OM];
#pragma unroll
    for (int c = 0; c < OM; ++c) gu[c] = gy[c];
    // a fresh view of the weights: the forward's reads are not reused (they
    // would all stay live across the adjoint)
    const float* Lb = L + opaque_zero();
    if (a.ln) dln_bwd<OM>(Lb + m.lg(), a.eps, u, gu, rec, rr.lnr());
    deep_bwd<H, K::KM, OM>(Lb, m, rr, gu, rec, d0);
  }
  const float* Lb = L + opaque_zero();
  if (a.g_a) {
    float t[KAM];
    dlin_t<H, K::KM, 0, KAM>(Lb + m.w0(), d0, t);
    if constexpr (SI) {
#pragma unroll
      for (int c = 0; c < KAM; ++c)
        if (c < a.ka) a.g_a[r * a.ka + c] = t[c];
    } else {
      vstore<KAM>(a.g_a + r * KAM, t);
    }
  }
  if constexpr (KB > 0) {
    float t[KB];
    dlin_t<H, K::KM, KAM, KB>(Lb + m.w0(), d0, t);
    if constexpr (KB == OM) {
      if (a.resid) {
        float go[OM];
        vload<OM>(a.g_out + r * OM, go);  // re-read rather than kept live
#pragma unroll
        for (int c = 0; c < KB; ++c) t[c] += go[c];
      }
    }
    vstore<KB>(a.g_b + r * KB, t);
  }
}

// --------------------------------------------------------- edge update

template <int H>
__global__ __launch_bounds__(256) void k_deep_edge_fwd(DeepEdgeArgs a) {
  extern __shared__ float L[];
  constexpr int KM = 3 * H;
  const DeepLds<H, KM, H> m{a.NH};
  stage_deep<H, KM, H>(L, a.theta, m, KM, KM, H, a.ln);
  __syncthreads();
  // XCD-aware numbering: each XCD's L2 sees a compact window of receivers
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= a.g.n_rows) return;
  float in[KM], acc[H];
  {
    float t[H];
    vload<H>(a.x + i * H, t);
#pragma unroll
    for (int c = 0; c < H; ++c) {
      in[c] = t[c];
      acc[c] = 0.f;
    }
  }
  const int k0 = a.g.rowptr[i], k1 = a.g.rowptr[i + 1];
  // H = 8: the next edge's x_j and e are loaded before this edge's MLP
  // runs, so their round trips (index, then row) overlap the arithmetic
  // (at 16 and 32 the extra registers cost a wave per SIMD)
  constexpr bool PF = H == 8;
  float nxj[PF ? H : 1], ne[PF ? H : 1];
  if constexpr (PF) {
    if (k0 < k1) {
      vload<H>(a.x + (int64_t)a.g.col[k0] * H, nxj);
      vload<H>(a.e_in + (int64_t)k0 * H, ne);
    }
  }
  for (int k = k0; k < k1; ++k) {
    const float* Lk = L + opaque_zero();  // re-read the weights per edge
    if constexpr (PF) {
#pragma unroll
      for (int c = 0; c < H; ++c) {
        in[H + c] = nxj[c];
        in[2 * H + c] = ne[c];
      }
      if (k + 1 < k1) {
        vload<H>(a.x + (int64_t)a.g.col[k + 1] * H, nxj);
        vload<H>(a.e_in + (int64_t)(k + 1) * H, ne);
      }
    } else {
      float t[H];
      vload<H>(a.x + (int64_t)a.g.col[k] * H, t);
#pragma unroll
      for (int c = 0; c < H; ++c) in[H + c] = t[c];
      vload<H>(a.e_in + (int64_t)k * H, t);
#pragma unroll
      for (int c = 0; c < H; ++c) in[2 * H + c] = t[c];
    }
    float u[H];
    deep_fwd<H, KM, H, false>(Lk, m, in, u, RecRef{nullptr});
    if (a.ln) dln_fwd<H>(Lk + m.lg(), Lk + m.lb(), a.eps, u);
    const float inv_d = 1.f / (float)a.g.mult[k];
#pragma unroll
    for (int c = 0; c < H; ++c) {
      const float msg = u[c];
      u[c] += in[2 * H + c];                     // residual edge update (Eq. 4a)
      acc[c] += (a.am ? msg : u[c]) * inv_d;     // Eq. 4b (or the message variant)
    }
    vstore<H>(a.e_out + (int64_t)k * H, u);
  }
  vstore<H>(a.a_out + i * H, acc);
}

// The adjoint of one edge k: its record (at rec) and its per-edge outputs.
template <int H>
__device__ __forceinline__ void deep_edge_bwd_one(const DeepEdgeArgs& a, const float* __restrict__ L,
                                                  const DeepLds<H, 3 * H, H>& m, const DeepRec<H, 3 * H, H>& rr,
                                                  int64_t k, const RecRef& rec) {
  constexpr int KM = 3 * H;
  const int64_t i = a.g.recv[k];
  const float inv_d = 1.f / (float)a.g.mult[k];
  float gy[H], d0[H];
  {
    float in[KM];
    float t[H];
    vload<H>(a.x + i * H, t);
#pragma unroll
    for (int c = 0; c < H; ++c) in[c] = t[c];
    vload<H>(a.x + (int64_t)a.g.col[k] * H, t);
#pragma unroll
    for (int c = 0; c < H; ++c) in[H + c] = t[c];
    vload<H>(a.e_in + k * H, t);
#pragma unroll
    for (int c = 0; c < H; ++c) in[2 * H + c] = t[c];
    rstore<KM, true>(rec, rr.in(), in);
    float u[H];
    deep_fwd<H, KM, H, true>(L, m, in, u, rec);
    // gradient of e' = e + MLP(...): the next layer's, plus Eq. 4b's adjoint
    if (a.g_e_out) {
      vload<H>(a.g_e_out + k * H, gy);
    } else {
#pragma unroll
      for (int c = 0; c < H; ++c) gy[c] = 0.f;
    }
    vload<H>(a.g_a + i * H, t);
#pragma unroll
    for (int c = 0; c < H; ++c) gy[c] += t[c] * inv_d;
    float gu[H];
#pragma unroll
    for (int c = 0; c < H; ++c) gu[c] = gy[c];
    const float* Lb = L + opaque_zero();  // see k_deep_row_bwd
    if (a.ln) dln_bwd<H>(Lb + m.lg(), a.eps, u, gu, rec, rr.lnr());
    deep_bwd<H, KM, H>(Lb, m, rr, gu, rec, d0);
  }
  const float* Lk = L + opaque_zero();
  float t[H];
  dlin_t<H, KM, 0, H>(Lk + m.w0(), d0, t);  // receiver part, summed by k_deep_gather
  vstore<H>(a.gxi + k * H, t);
  phase_fence();
  dlin_t<H, KM, H, H>(Lk + m.w0(), d0, t);  // sender part, gathered through rev
  vstore<H>(a.gxj + k * H, t);
  phase_fence();
  dlin_t<H, KM, 2 * H, H>(Lk + m.w0(), d0, t);  // edge-state part + residual
  if (a.am) {  // message aggregation: the residual carries the next layer's gradient only
    if (a.g_e_out) {
      vload<H>(a.g_e_out + k * H, gy);
    } else {
#pragma unroll
      for (int c = 0; c < H; ++c) gy[c] = 0.f;
    }
  }
#pragma unroll
  for (int c = 0; c < H; ++c) t[c] += gy[c];
  vstore<H>(a.g_e_in + k * H, t);
}

template <int H>
__global__ __launch_bounds__(256) void k_deep_edge_bwd(DeepEdgeArgs a) {
  extern __shared__ float L[];
  constexpr int KM = 3 * H;
  const DeepLds<H, KM, H> m{a.NH};
  const DeepRec<H, KM, H> rr{a.NH, a.ln};
  stage_deep<H, KM, H>(L, a.theta, m, KM, KM, H, a.ln);
  __syncthreads();
  // one thread per edge: every output is per edge (the receiver's and the
  // sender's input gradients are summed afterwards by k_deep_gather)
  const int64_t k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (k >= a.g.n_edges) return;
  deep_edge_bwd_one<H>(a, L, m, rr, k, RecRef{a.rec + deep_rec_at(k, 0, a.rs)});
}

// g_x[j] = g_x_node[j] + the input gradients of j's incoming edges (their
// receiver parts) and of j's outgoing edges (the reverses of its incoming
// edges; their sender parts), in CSR order.
template <int H>
__global__ __launch_bounds__(256) void k_deep_gather(DevGraph g, const float* __restrict__ gxn,
                                                     const float* __restrict__ gxi, const float* __restrict__ gxj,
                                                     float* __restrict__ gx) {
  const int64_t j = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= g.n_rows) return;
  float s[H];
  vload<H>(gxn + j * H, s);
  const int k0 = g.rowptr[j], k1 = g.rowptr[j + 1];
  // a few edges at a time (4 at H = 8, else 2): their reverse indices
  // first, then all their rows, so the dependent loads cost one round trip
  // per group; the sums stay in edge order
  constexpr int B = H == 8 ? 4 : 2;
  for (int kb = k0; kb < k1; kb += B) {
    int rv[B];
#pragma unroll
    for (int q = 0; q < B; ++q) rv[q] = kb + q < k1 ? g.rev[kb + q] : 0;
    float ti[B][H], tj[B][H];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (kb + q < k1) {
        vload<H>(gxi + (int64_t)(kb + q) * H, ti[q]);
        vload<H>(gxj + (int64_t)rv[q] * H, tj[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (kb + q < k1) {
#pragma unroll
        for (int c = 0; c < H; ++c) s[c] += ti[q][c];
#pragma unroll
        for (int c = 0; c < H; ++c) s[c] += tj[q][c];
      }
    }
  }
  vstore<H>(gx + j * H, s);
}

// ------------------------------------------------ weight-gradient sums

// Partial sums over one chunk of rows, for every weight block of one MLP:
// part[chunk][dst_w + o*aw + c] = sum_r G[r][o] A[r][c] and
// part[chunk][dst_b + o] = sum_r G[r][o] (blocks without A: only the latter).
//
// One workgroup per chunk (whole record blocks); its four waves split the
// 16 x 16 tiles (to, tc) of G^T A of all blocks between them, numbered block
// by block, strip (to) by strip, a contiguous range per wave.  The products
// run on the matrix unit with the rows as the reduction dimension, 16 rows
// per step: lane l = 16 k + i loads, as one 16-byte piece, rows 4k .. 4k+3 of
// record column G[16 to + i] (and of A[16 tc + i]) -- the column-by-column
// record blocks make that piece contiguous -- and step v of four takes
// component v of both pieces as the A and B operands of
// v_mfma_f32_16x16x4f32, so the instruction's four k slots hold rows
// 4k + v.  Lane l then holds rows 4 (l/16) .. 4 (l/16) + 3, column l%16 of
// the tile.  The column sums of G are plain adds of the same G values per
// lane, combined over the four k at the end.  Lanes past a block's width
// read its last column: their products land in rows and columns of the
// tile that are never stored.  Rows are added in a fixed order, so the
// partial sums are reproducible.
constexpr int kOuterMaxMT = 16;  // tiles per wave
constexpr int kOuterNW = 4;      // waves per workgroup

struct OuterTile {
  int to, tc;  // G strip, A tile; tc < 0: column sums only
  OuterMat M;  // its weight block (M.gw == 0: no tile)
};

__host__ __device__ inline int outer_strips(const OuterMat& M) { return (M.gw + 15) / 16; }
__host__ __device__ inline int outer_tiles_per_strip(const OuterMat& M) {
  return M.a_off >= 0 && M.aw > 0 ? (M.aw + 15) / 16 : 1;
}

// Tile id of the block list; the blocks are visited with constant indices
// (a dynamic index into the kernel's argument block would copy it to
// scratch memory).
__device__ __forceinline__ OuterTile outer_tile(const OuterArgs& a, int id) {
  OuterTile r{0, 0, OuterMat{0, 0, -1, 0, 0, 0}};
  bool found = false;
#pragma unroll
  for (int m = 0; m < kMaxOuterMats; ++m) {
    if (m < a.n_mats && !found) {
      const OuterMat& M = a.m[m];
      const int per = outer_tiles_per_strip(M), n = outer_strips(M) * per;
      if (id < n) {
        const bool hasA = M.a_off >= 0 && M.aw > 0;
        r = OuterTile{id / per, hasA ? id % per : -1, M};
        found = true;
      } else {
        id -= n;
      }
    }
  }
  return r;
}

// MT tile slots of one wave: tiles t0 .. t0 + nt - 1.  Unused slots (and
// the A operand of column-sum-only tiles) read G's column again and are not
// stored, so a step has no branches and all its loads are issued before its
// products.
template <int MT>
struct OuterAcc {
  int og[MT], ob[MT];  // offsets (from a step's first row) of this lane's G and A pieces
  v4f acc[MT];
  float gs[MT];

  __device__ __forceinline__ void init(const OuterArgs& a, int t0, int nt, int lane) {
    const int k = lane >> 4, col = lane & 15;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const OuterTile d = outer_tile(a, t < nt ? t0 + t : 1 << 30);
      const OuterMat& M = d.M;
      int cg = 0, cb = 0;
      if (M.gw > 0) {
        cg = M.g_off + std::min(16 * d.to + col, M.gw - 1);
        cb = d.tc >= 0 ? M.a_off + std::min(16 * d.tc + col, M.aw - 1) : cg;
      }
      og[t] = cg * kRecRows + 4 * k;
      ob[t] = cb * kRecRows + 4 * k;
      acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
      gs[t] = 0.f;
    }
  }

  // Sixteen rows rb .. rb + 15 whose record pieces start at base; rows from
  // r1 on add nothing.
  // (More than eight tiles go in two halves, loads then products, to bound
  // the registers the loads hold.)
  __device__ __forceinline__ void step(const float* __restrict__ base, int64_t rb, int64_t r1, int lane) {
    constexpr int HB = MT > 8 ? (MT + 1) / 2 : MT;
    const int64_t rr = rb + 4 * (lane >> 4);
#pragma unroll
    for (int h0 = 0; h0 < MT; h0 += HB) {
      float4 gv[HB], bv[HB];
#pragma unroll
      for (int j = 0; j < HB; ++j) {
        if (h0 + j < MT) {
          gv[j] = *reinterpret_cast<const float4*>(base + og[h0 + j]);
          bv[j] = *reinterpret_cast<const float4*>(base + ob[h0 + j]);
        }
      }
      if (rb + 16 > r1) {  // past the last row the block holds no data: zero both operands
#pragma unroll
        for (int j = 0; j < HB; ++j) {
          if (rr >= r1) gv[j].x = bv[j].x = 0.f;
          if (rr + 1 >= r1) gv[j].y = bv[j].y = 0.f;
          if (rr + 2 >= r1) gv[j].z = bv[j].z = 0.f;
          if (rr + 3 >= r1) gv[j].w = bv[j].w = 0.f;
        }
      }
#pragma unroll
      for (int j = 0; j < HB; ++j) {
        if (h0 + j >= MT) continue;
        const int t = h0 + j;
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[j].x, bv[j].x, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[j].y, bv[j].y, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[j].z, bv[j].z, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[j].w, bv[j].w, acc[t], 0, 0, 0);
        gs[t] += ((gv[j].x + gv[j].y) + gv[j].z) + gv[j].w;
      }
    }
  }

  __device__ __forceinline__ void store(const OuterArgs& a, int t0, int nt, int lane, float* __restrict__ dst) {
    const int k = lane >> 4, col = lane & 15;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (t >= nt) continue;
      const OuterTile d = outer_tile(a, t0 + t);
      const OuterMat& M = d.M;
      if (d.tc <= 0) {
        // column sums: the four k, added in a fixed order
        const float s1 = __shfl(gs[t], col + 16), s2 = __shfl(gs[t], col + 32), s3 = __shfl(gs[t], col + 48);
        const int o = 16 * d.to + col;
        if (k == 0 && o < M.gw) dst[M.dst_b + o] = ((gs[t] + s1) + s2) + s3;
      }
      if (d.tc >= 0) {
        const int c = 16 * d.tc + col;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = 16 * d.to + 4 * k + v;
          if (o < M.gw && c < M.aw) dst[M.dst_w + (int64_t)o * M.aw + c] = acc[t][v];
        }
      }
    }
  }
};

__device__ __forceinline__ int outer_ntiles(const OuterArgs& a) {
  int n = 0;
  for (int m = 0; m < a.n_mats; ++m) n += outer_strips(a.m[m]) * outer_tiles_per_strip(a.m[m]);
  return n;
}

template <int MT>
__global__ __launch_bounds__(64 * kOuterNW) void k_outer_sum(OuterArgs a) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ntiles = outer_ntiles(a);
  const int t0 = w * ntiles / kOuterNW, nt = (w + 1) * ntiles / kOuterNW - t0;
  OuterAcc<MT> s;
  s.init(a, t0, nt, lane);
  const int64_t r0 = (int64_t)blockIdx.x * a.ch, r1 = std::min<int64_t>(a.n_rows, r0 + a.ch);
  for (int64_t rb = r0; rb < r1; rb += 16)  // rb is a multiple of 16: one record block
    s.step(a.rec + deep_rec_at(rb, 0, a.rs), rb, r1, lane);
  s.store(a, t0, nt, lane, a.part + (int64_t)blockIdx.x * a.slab);
}

// ------------------------------------------------------------- launchers

template <int H, int KM, int OM>
static size_t deep_lds_bytes(int NH) {
  return (size_t)DeepLds<H, KM, OM>{NH}.size() * sizeof(float);
}

int deep_rec_floats(int H, int km, int om, int NH, int ln) {
  return km + 2 * (NH + 1) * H + om + (ln ? 2 * om : 0);
}

template <int H, int KAM, int KB, int OM, bool SI>
static hipError_t row_launch(const DeepRowArgs& a, bool bwd, hipStream_t s) {
  const int grid = (int)((a.n_rows + 255) / 256);
  const size_t lds = deep_lds_bytes<H, KAM + KB, OM>(a.NH);
  if (bwd)
    hipLaunchKernelGGL((k_deep_row_bwd<H, KAM, KB, OM, SI>), dim3(grid), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((k_deep_row_fwd<H, KAM, KB, OM, SI>), dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int H>
static hipError_t row_launch_h(const DeepRowArgs& a, DeepRowKind kind, bool bwd, hipStream_t s) {
  switch (kind) {
    case DeepRowKind::kSmallIn: return row_launch<H, 4, 0, H, true>(a, bwd, s);
    case DeepRowKind::kSmallIn8: return row_launch<H, 8, 0, H, true>(a, bwd, s);
    case DeepRowKind::kSmallOut: return row_launch<H, H, 0, 4, false>(a, bwd, s);
    case DeepRowKind::kWide: return row_launch<H, H, 0, H, false>(a, bwd, s);
    case DeepRowKind::kNode: return row_launch<H, H, H, H, false>(a, bwd, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_deep_row(const DeepRowArgs& a, int H, DeepRowKind kind, bool bwd, hipStream_t s) {
  if (a.n_rows == 0) return hipSuccess;
  if (H == 8) return row_launch_h<8>(a, kind, bwd, s);
  if (H == 16) return row_launch_h<16>(a, kind, bwd, s);
  if (H == 32) return row_launch_h<32>(a, kind, bwd, s);
  return hipErrorInvalidValue;
}

template <int H>
static hipError_t edge_launch(const DeepEdgeArgs& a, bool bwd, hipStream_t s) {
  const size_t lds = deep_lds_bytes<H, 3 * H, H>(a.NH);
  if (bwd)
    hipLaunchKernelGGL(k_deep_edge_bwd<H>, dim3((unsigned)((a.g.n_edges + 255) / 256)), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL(k_deep_edge_fwd<H>, dim3((unsigned)((a.g.n_rows + 255) / 256)), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_deep_edge(const DeepEdgeArgs& a, int H, bool bwd, hipStream_t s) {
  if (H == 8) return edge_launch<8>(a, bwd, s);
  if (H == 16) return edge_launch<16>(a, bwd, s);
  if (H == 32) return edge_launch<32>(a, bwd, s);
  return hipErrorInvalidValue;
}

hipError_t launch_deep_gather(int H, const DevGraph& g, const float* gxn, const float* gxi, const float* gxj,
                              float* gx, hipStream_t s) {
  const int grid = (int)((g.n_rows + 255) / 256);
  if (H == 8) hipLaunchKernelGGL(k_deep_gather<8>, dim3(grid), dim3(256), 0, s, g, gxn, gxi, gxj, gx);
  else if (H == 16) hipLaunchKernelGGL(k_deep_gather<16>, dim3(grid), dim3(256), 0, s, g, gxn, gxi, gxj, gx);
  else if (H == 32) hipLaunchKernelGGL(k_deep_gather<32>, dim3(grid), dim3(256), 0, s, g, gxn, gxi, gxj, gx);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

int outer_tiles(const OuterMat* m, int n_mats) {
  if (n_mats <= 0 || n_mats > kMaxOuterMats) return 0;
  int n = 0;
  for (int i = 0; i < n_mats; ++i) {
    if (m[i].gw < 1 || (m[i].a_off >= 0 && m[i].aw < 0)) return 0;
    n += outer_strips(m[i]) * outer_tiles_per_strip(m[i]);
  }
  return n;
}

bool outer_fits(const OuterMat* m, int n_mats) {
  const int n = outer_tiles(m, n_mats);
  return n >= 1 && n <= kOuterNW * kOuterMaxMT;
}

hipError_t launch_outer_sum(const OuterArgs& args, int n_mats, int64_t n_chunks, hipStream_t s) {
  if (n_chunks <= 0 || !outer_fits(args.m, n_mats) || args.rs < 1) return hipErrorInvalidValue;
  if (args.ch % kRecRows) return hipErrorInvalidValue;  // chunks of whole record blocks
  OuterArgs a = args;
  a.n_mats = n_mats;
  const int per_wave = (outer_tiles(a.m, n_mats) + kOuterNW - 1) / kOuterNW;
  const dim3 grid((unsigned)n_chunks), block(64 * kOuterNW);
  if (per_wave <= 1) hipLaunchKernelGGL(k_outer_sum<1>, grid, block, 0, s, a);
  else if (per_wave <= 2) hipLaunchKernelGGL(k_outer_sum<2>, grid, block, 0, s, a);
  else if (per_wave <= 4) hipLaunchKernelGGL(k_outer_sum<4>, grid, block, 0, s, a);
  else if (per_wave <= 8) hipLaunchKernelGGL(k_outer_sum<8>, grid, block, 0, s, a);
  else if (per_wave <= 12) hipLaunchKernelGGL(k_outer_sum<12>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(k_outer_sum<16>, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace mp
