// Kernel declarations and launch-side structures shared by the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mp {

// One matrix to pack into MFMA fragments: element (r, c) of the packed
// [rows][cols] matrix is  c < split ? A(r, c) : B(r, c - split)  where a
// view X(r, c) = trans ? p[c*ld + off + r] : p[r*ld + off + c].
struct PackView {
  const float* p;
  int ld, off, trans;
};
struct PackJob {
  PackView a, b;
  int rows, cols, split;
  int64_t dst_off;  // byte offset of the fragments in the packed buffer
};
constexpr int kMaxPackJobs = 12;
struct PackJobs {
  PackJob job[kMaxPackJobs];
  int n;
  int bf;  // 1: BF16 fragments
};

// Device graph arrays (see mp_dev_graph).
struct DevGraph {
  int64_t n_rows, n_edges, n_groups;
  const int32_t* rowptr;
  const int32_t* recv;
  const int32_t* col;
  const int32_t* rev;
  const uint8_t* mult;
  const int32_t* group_ptr;
  const int32_t* member;
  // row-aligned tiles of about equal edge count (built by launch_tiles):
  // tile t = rows [tile_r[t], tile_r[t+1]) = edges [tile_e[t], tile_e[t+1])
  int64_t n_tiles;
  const int32_t* tile_r;
  const int32_t* tile_e;
  // dynamic tile order (edge forward, queue = 1): one tile counter per XCD
  // range, zeroed by launch_tiles
  int32_t* queue;
};

// Edges per tile of the edge kernels' schedule.
constexpr int kTileEdges = 128;
// Also zeroes queue[0..7] when queue is not null.
hipError_t launch_tiles(const DevGraph& g, int32_t* tile_r, int32_t* tile_e, int32_t* queue, hipStream_t s);

// Launch helpers; each returns the hipError_t of the launch.
hipError_t launch_pack(const PackJobs& jobs, void* dst, hipStream_t s);

hipError_t launch_proj(int H, bool bf, const DevGraph& g, const float* x, const void* frag_ab,
                       const float* b1, float* P, float* Q, int grid, hipStream_t s);

// am: aggregate the edge MLP's output (message) instead of the updated state;
// dq: waves take tiles from per-XCD atomic counters (g.queue) instead of a
// fixed round robin; es: edge states e_in / e_out stored as BF16 (with bf only)
hipError_t launch_edge_fwd(int H, bool ln, bool bf, bool am, bool dq, bool es, const DevGraph& g, const float* P,
                           const float* Q, const void* e_in, const void* frag_c2, const float* b2,
                           const float* lng, const float* lnb, float eps, void* e_out, float* a_out, int grid,
                           hipStream_t s);

hipError_t launch_halo(int H, const DevGraph& g, float* a, hipStream_t s);

// Row MLP: out = [resid +] [LN] (W1 . ELU(W0 . in + b0) + b1) with
// in = [src0 (k0 features), src1 (k1 features)]; k0 in {3, 4} is the
// small-input form (first Linear by FMA, W0 read directly); n_out < 16 is
// the small-output form (second Linear by FMA, no LayerNorm).
struct MlpFwdArgs {
  int64_t n_rows;
  const float* src0;
  const float* src1;
  const float* resid;
  int k0, k1, H, n_out, ln, bf;
  const float* W0;  // raw weights (small-input form)
  const float* b0;
  const float* W1;  // raw weights (small-output form)
  const float* b1;
  const float* lng;
  const float* lnb;
  float eps;
  const void* frag0;  // packed W0 (when k0 >= 16)
  const void* frag1;  // packed W1 (when n_out == H)
  void* out;          // [n][n_out], FP32, or BF16 with out_bf
  int out_bf;         // small-input form with BF16 GEMMs and n_out == H only
};
hipError_t launch_mlp_fwd(const MlpFwdArgs& a, int grid, hipStream_t s);

// u (nullable): FP32 [N][3] node field; with it e0 is [E][7] and its last
// three channels are u_j - u_i.
hipError_t launch_edge_inputs(const DevGraph& g, const double* pos, const double period[3], const float* u,
                              float* e0, hipStream_t s);

hipError_t launch_loss(int64_t n_rows, int F, const float* Y, const float* T, const uint8_t* mult,
                       double* part, int n_part, float* loss, float* gY, hipStream_t s);

// ---------------------------------------------------------------- backward

// Floats per workgroup slab of partial weight gradients.
// edge adjoint: [dW1c H*H][dW2 H*H][db2 H][dgamma H][dbeta H]
__host__ __device__ constexpr int64_t edge_slab(int H) { return 2 * (int64_t)H * H + 3 * H; }
// sender-side pass: [dW1a H*H][dW1b H*H][db1 H]
__host__ __device__ constexpr int64_t gq_slab(int H) { return 2 * (int64_t)H * H + H; }
// row MLP adjoint: [dW0 H*kin][db0 H][dW1 n_out*H][db1 n_out][dgamma H][dbeta H]
__host__ __device__ constexpr int64_t mlp_slab(int H, int kin, int n_out) {
  return (int64_t)H * kin + H + (int64_t)n_out * H + n_out + 2 * H;
}

// Partial weight gradients: one slab of `slab` floats per workgroup of the
// producing kernel; launch_wreduce sums the slabs in workgroup order.
struct ReduceSeg {
  const float* part;  // first slab
  int n_slabs;
  int64_t slab;       // floats per slab
  int64_t src_off;    // float offset of this block inside a slab
  int rows, cols;     // gradient block shape (row-major inside the slab)
  float* dst;         // destination, leading dimension ld, first column col0
  int ld, col0;
};
constexpr int kMaxReduceSegs = 16;
struct ReduceSegs {
  ReduceSeg seg[kMaxReduceSegs];
  int n;
};
hipError_t launch_wreduce(const ReduceSegs& segs, hipStream_t s);

struct EdgeBwdArgs {
  DevGraph g;
  int H, ln, bf;
  int am;  // the forward aggregated the MLP output (message), not e'
  int waves;  // waves per workgroup: 0 (default), 4, or 8 (fused kernel: BF16, H <= 64; split kernel: any)
  int es;     // edge states and their gradients (e_in, g_e_out, g_e_in) stored as BF16 (with bf only)

  const float* P;
  const float* Q;
  const void* e_in;
  const void* g_e_out;   // may be null
  const float* g_a;      // gradient of a (after the adjoint halo sum)
  const void* frag;      // W1c, W2, W2^T, W1c^T fragments, consecutive
  const float* b2;
  const float* lng;
  const float* lnb;
  float eps;
  void* g_e_in;
  void* g_h;             // [E][H] gradient of the first pre-activation (BF16 on the BF16 path)
  float* g_P;            // [N][H] sum of g_h over each row's incoming edges
  float* part;           // partial weight gradients, slab per workgroup
  int64_t slab;
  // split form (edge_bwd_split): per-edge factors of the matrix weight
  // gradients, [E][H] each, BF16 on the BF16 path: gm (pre-LayerNorm
  // gradient) and u (ELU output)
  void* gm;
  void* u;
};
hipError_t launch_edge_bwd(const EdgeBwdArgs& a, int grid, hipStream_t s);
// Whether layers of width H use the split edge adjoint (the fused kernel's
// weight-gradient tiles and all four weight matrices do not fit on chip).
constexpr bool edge_bwd_split(int H) { return H > 64; }
hipError_t launch_edge_bwd_split(const EdgeBwdArgs& a, int grid, hipStream_t s);
// dst slab block [GW][AW] += sum over rows r of G[r] (x) A[r]  (G: [R][GW],
// A: [R][AW]; BF16 or FP32 as `g_bf` / `a_bf`), one slab per workgroup at
// part + blockIdx.x * slab + off; with colsum_off >= 0 also the column sums
// of G at colsum_off.  Rows split in contiguous ranges per workgroup.
struct RowDwArgs {
  int64_t n_rows;
  int GW, AW, bf;       // bf: staging and products in BF16
  const void* G;
  int g_bf;             // G stored as BF16
  const void* A;        // [R][AW], or with A2: the first AW/2 columns
  const void* A2;       // optional second half of A ([R][AW/2], same type)
  int a_bf;             // A stored as BF16
  float* part;
  int64_t slab, off, colsum_off;
};
hipError_t launch_row_dw(const RowDwArgs& a, int grid, hipStream_t s);
// Column sums of X[R][W] and Y[R][W] (each BF16 or FP32: x_bf, y_bf) into
// slab offsets offx / offy per workgroup, rows split as in launch_row_dw.
hipError_t launch_colsum2(int64_t n_rows, int W, int x_bf, int y_bf, const void* X, const void* Y, float* part,
                          int64_t slab, int64_t offx, int64_t offy, int grid, hipStream_t s);

struct MlpBwdArgs {
  int64_t n_rows;
  const float* src0;
  const float* src1;
  int k0, k1, H, n_out, ln, bf, resid;
  const float* W0;
  const float* b0;
  const float* W1;
  const float* b1;
  const float* lng;
  const float* lnb;
  float eps;
  const void* frag0;   // W0 (k0 >= 16)
  const void* frag1;   // W1 (n_out == H)
  const void* frag1t;  // W1^T (n_out == H)
  const void* frag0t;  // W0^T (k0 >= 16 and an input gradient is wanted)
  const void* g_out;   // [n][n_out], FP32, or BF16 with gout_bf
  int gout_bf;         // small-input form with BF16 GEMMs and n_out == H only
  float* g_src0;       // may be null
  float* g_src1;       // may be null
  const float* g_add1; // added to g_src1 (residual path); may be null
  float* part;
  int64_t slab;
};
hipError_t launch_mlp_bwd(const MlpBwdArgs& a, int grid, hipStream_t s);
// Whether the node update's adjoint (2H input) at width H uses the split
// form (both product types; FP32 cuts its first pass in two so that each
// pass's weights fit in LDS).
constexpr bool node_bwd_split(int H, bool /*bf*/) { return H > 64; }
hipError_t launch_node_bwd_split(const MlpBwdArgs& a, void* u, void* gy, void* gz, void* goxh, int grid, hipStream_t s);

struct GqArgs {
  DevGraph g;
  int H, bf;
  const float* x;
  const float* g_P;
  const void* g_h;       // [E][H], FP32 or (BF16 path) BF16
  const void* frag_abt;  // [W1a | W1b]^T as an H x 2H matrix
  float* g_x;            // accumulated: g_x += W1a^T g_P + W1b^T g_Q
  float* part;
  int64_t slab;
  float* gq_out;         // split form only: g_Q [N][H] (FP32)
};
// Whether the sender-side pass leaves its weight gradients to launch_row_dw
// (FP32 at H = 128, where its tiles and accumulators do not fit).
constexpr bool gq_split(int H, bool bf) { return H > 64 && !bf; }
hipError_t launch_gq(const GqArgs& a, int grid, hipStream_t s);

// ------------------------------------------------ narrow deep MLPs
// (hidden width 8, 16 or 32; n_hidden extra H -> H layers; FP32; one
// thread per row).  Parameters of one MLP are one flat FP32 array in
// torch.nn.Linear order: W0[H][K] b0[H], n_hidden x (W[H][H] b[H]),
// Wo[O][H] bo[O], then LayerNorm gain[O] and shift[O].
__host__ __device__ constexpr int64_t deep_theta_floats(int K, int H, int NH, int O, int ln) {
  return (int64_t)H * K + H + (int64_t)NH * (H * H + H) + (int64_t)O * H + O + (ln ? 2 * O : 0);
}
// floats of one row's adjoint record (padded input width km, output om)
int deep_rec_floats(int H, int km, int om, int NH, int ln);

enum class DeepRowKind { kSmallIn, kSmallIn8, kSmallOut, kWide, kNode };
// kSmallIn: in = src_a (1..4 features) -> H;  kSmallIn8: 5..8 features -> H;
// kSmallOut: H -> 1..4;
// kWide: H -> H;  kNode: [src_a (H), src_b (H)] -> H, optionally residual.
struct DeepRowArgs {
  int64_t n_rows;
  const float* theta;
  int NH, ka, O, ln;
  float eps;
  const float* src_a;
  const float* src_b;
  int resid;           // out = src_b + MLP (kNode only)
  float* out;
  const float* g_out;  // adjoint: [n][O]
  float* g_a;          // [n][ka] or NULL
  float* g_b;          // [n][H] (kNode), includes g_out when resid
  float* rec;          // per-row records (deep_rec_at), rs columns
  int rs;
};
hipError_t launch_deep_row(const DeepRowArgs& a, int H, DeepRowKind kind, bool bwd, hipStream_t s);

struct DeepEdgeArgs {
  DevGraph g;
  const float* theta;
  int NH, ln;
  int am;              // aggregate the MLP output (message), not e'

  float eps;
  const float* x;      // [N][H]
  const float* e_in;   // [E][H]
  float* e_out;        // forward: [E][H]
  float* a_out;        // forward: [N][H]
  const float* g_a;    // adjoint: gradient of the aggregate after the halo adjoint
  const float* g_e_out;  // [E][H] or NULL
  float* g_e_in;       // [E][H]
  float* gxi;          // [E][H] receiver-side input gradient per edge
  float* gxj;          // [E][H] sender-side input gradient per edge
  float* rec;          // per-edge records (deep_rec_at), rs columns
  int rs;
};
hipError_t launch_deep_edge(const DeepEdgeArgs& a, int H, bool bwd, hipStream_t s);
hipError_t launch_deep_gather(int H, const DevGraph& g, const float* gxn, const float* gxi, const float* gxj,
                              float* gx, hipStream_t s);

// Per-row records of rs columns are stored in blocks of kRecRows rows,
// column by column inside a block: column c of row r is at
// deep_rec_at(r, c, rs).  A wave's store of one column of 64 consecutive
// rows is one contiguous 256-byte run, and a block is one contiguous range.
constexpr int kRecRows = 64;
__host__ __device__ constexpr int64_t deep_rec_at(int64_t r, int c, int rs) {
  return (r / kRecRows) * kRecRows * rs + (int64_t)c * kRecRows + r % kRecRows;
}
constexpr int64_t deep_rec_size(int64_t n, int rs) { return (n + kRecRows - 1) / kRecRows * kRecRows * rs; }

// Weight-gradient partial sums over chunks of record rows.
struct OuterMat {
  int g_off, gw;     // G block: record columns [g_off, g_off + gw)
  int a_off, aw;     // A block (a_off < 0: none)
  int64_t dst_w, dst_b;  // offsets in the flat gradient of sum G^T A and sum G
};
constexpr int kMaxOuterMats = 12;
struct OuterArgs {
  const float* rec;  // records (deep_rec_at)
  int64_t n_rows;
  int rs;            // columns
  int64_t ch;        // rows per chunk
  float* part;       // [n_chunks][slab]
  int64_t slab;
  OuterMat m[kMaxOuterMats];
  int n_mats;        // set by launch_outer_sum
};
// Matrix-unit tiles of one set of weight blocks; 0 if a block is malformed.
int outer_tiles(const OuterMat* m, int n_mats);
bool outer_fits(const OuterMat* m, int n_mats);
hipError_t launch_outer_sum(const OuterArgs& a, int n_mats, int64_t n_chunks, hipStream_t s);

}  // namespace mp
