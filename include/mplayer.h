/*
 * mplayer.h - C ABI of the consistent neural message-passing layer on gfx950.
 *
 * The layer is the paper's consistent NMP layer (Eq. 4a-e of
 * "Scalable and Consistent Graph Neural Networks for Distributed Mesh-based
 * Data-driven Modeling"): an edge MLP on every directed edge, a 1/d_ij
 * weighted sum of edge states into receivers, a halo exchange that sums the
 * partial aggregates of every global node held by several sub-graphs, and a
 * residual node MLP.  All R sub-graphs of a partition live on one GPU as
 * row ranges of one set of buffers; the halo exchange is an in-device
 * gather/scatter over groups of rows that share a global id.
 *
 * Conventions (every entry point):
 *  - Every function returns MP_OK (0) or a positive error code; on error
 *    mp_last_error() returns a thread-local message.  Nothing throws across
 *    the ABI and nothing calls exit().
 *  - Validation happens before any launch: on an error return no kernel was
 *    launched and no output was written.
 *  - The caller owns every buffer.  The library owns only the opaque host
 *    objects mp_graph and mp_halo_plan, released by their *_destroy call.
 *  - Device entry points never allocate device memory; scratch comes from a
 *    caller workspace sized by the matching *_workspace_size call.
 *  - Device entry points are asynchronous on the given HIP stream (NULL is
 *    the default stream).  Inputs must stay alive until the stream reaches
 *    the work.
 *  - Matrices are row-major with features contiguous.  Weights follow the
 *    nn.Linear layout W[out][in].  Device pointers must be 16-byte aligned.
 *  - Reductions use fixed orders and no floating-point atomics, so every
 *    device result is bitwise reproducible run to run.
 */
#ifndef MPLAYER_H
#define MPLAYER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MP_ABI_VERSION 4

enum {
  MP_OK = 0,
  MP_EINVAL = 1, /* bad pointer, size, width, dtype or aliasing */
  MP_EPLAN = 2,  /* graph / plan descriptor inconsistent */
  MP_ENOMEM = 3, /* host allocation failed, or workspace too small */
  MP_EHIP = 4    /* HIP runtime or launch error */
};

enum { MP_F32 = 0, MP_BF16 = 1 }; /* arithmetic type of the MLP GEMM operands */
enum { MP_AGG_STATE = 0, MP_AGG_MESSAGE = 1 }; /* what Eq. 4b sums (mp_layer_cfg.aggregate) */

typedef struct ihipStream_t* mp_stream_t; /* the same type as hipStream_t */

int mp_abi_version(void);
const char* mp_last_error(void);

/* ---------------------------------------------------------------------
 * Host: distributed graph generation (Sec. II-A, Figs. 2-4).
 * ------------------------------------------------------------------- */

/* Element-local graph links of a hexahedral element of order P (Sec. II-A,
 * Fig. 2): undirected pairs of neighbouring GLL points, in local point
 * numbering a + (P+1)*(b + (P+1)*c).  With links == NULL only *n_links is
 * written ((P+1)^2 * P * 3 pairs).  links is [n_links][2], host memory. */
int mp_hex_links(int32_t P, int32_t* links, int32_t* n_links);

typedef struct mp_graph mp_graph;

/* Build the reduced distributed graph (Sec. II-A, Fig. 3c) of an element
 * partition.  Inputs (host memory, read only):
 *   elem_gid [n_elem][npe]  global node id of every element-local point;
 *   links    [n_links][2]   element-local point pairs joined by an edge;
 *   elem_part[n_elem]       sub-graph of every element, in [0, R).
 * Sub-graph r holds the distinct global ids of its elements' points as rows
 * (local coincident nodes collapsed), in ascending global id, and both
 * directions of every distinct link of its elements.  The R sub-graphs are
 * concatenated in r order.  Edges are sorted by (receiver row, sender row).
 * edge_mult d_ij = number of sub-graphs holding the link (the edge degree
 * under Eq. 4b); node_mult d_i = number of sub-graphs holding the node
 * (Eq. 6b-c).  Errors: MP_EINVAL for bad sizes, ids out of range, parts
 * out of range, self-links, empty sub-graphs or more than 2^31-1 rows or
 * edges; MP_ENOMEM on host allocation failure. */
int graph_partition(int64_t n_elem, int32_t npe, const int64_t* elem_gid,
                    int32_t n_links, const int32_t* links,
                    const int32_t* elem_part, int32_t R, mp_graph** out);

/* Renumber the rows of every sub-graph of g, in place, in reverse
 * Cuthill-McKee order (breadth-first levels from a pseudo-peripheral row,
 * neighbours in ascending degree, reversed; ties to the lower row): the
 * rows an edge joins end up close in memory, so a kernel sweeping the rows
 * finds the rows it gathers still in cache.  Sub-graphs keep their rows and
 * their place in the concatenation; edges stay sorted by (receiver row,
 * sender row) in the new numbering, with rev, recv, col, edge_mult,
 * node_mult and row_gid carried along.  The order is a function of the
 * graph alone.  Call before halo_plan_build.  Errors: MP_EINVAL for a NULL
 * graph, MP_ENOMEM on host allocation failure (g is then unchanged only
 * up to the sub-graphs already renumbered). */
int graph_order_rows(mp_graph* g);

int mp_graph_sizes(const mp_graph* g, int64_t* n_rows, int64_t* n_edges, int32_t* R);

/* Copy the graph out (host memory, sizes from mp_graph_sizes; any pointer
 * may be NULL to skip that array):
 *   row_off[R+1], edge_off[R+1]  row / edge range of each sub-graph;
 *   row_gid[N]                   global id of every row;
 *   rowptr[N+1]                  CSR offsets of each row's incoming edges;
 *   recv[E], col[E]              receiver and sender row of every edge;
 *   rev[E]                       index of the edge's reverse (j->i for i->j);
 *   edge_mult[E], node_mult[N]   degrees d_ij and d_i. */
int mp_graph_export(const mp_graph* g, int64_t* row_off, int64_t* edge_off,
                    int64_t* row_gid, int32_t* rowptr, int32_t* recv, int32_t* col,
                    int32_t* rev, uint8_t* edge_mult, uint8_t* node_mult);
/* Content checksum of the graph's device-side arrays (rowptr, recv, col,
 * rev, edge_mult, in that order), computed by graph_partition and again by
 * graph_order_rows.  Two graphs whose arrays differ anywhere (for instance
 * one mesh in ascending-id and in locality row order, which have the same
 * sizes) get different checksums with overwhelming probability. */
int mp_graph_checksum(const mp_graph* g, uint64_t* checksum);
int mp_graph_destroy(mp_graph* g);

typedef struct mp_halo_plan mp_halo_plan;

/* Halo plan of a graph (Eq. 4c-d, Fig. 4).  One-GPU form: groups of rows
 * that hold the same global id (only ids held by two or more sub-graphs),
 * members in ascending row order, groups in ascending global id.
 * Multi-GPU form (exported for a distributed runtime): for every ordered
 * pair (r, s) of sub-graphs sharing ids, the rows of r to send to s (r's
 * send mask) and the matching rows of s (where s's halo rows sum into),
 * in ascending global id; plus per-sub-graph halo-row and neighbour
 * counts (the columns of Table II). */
int halo_plan_build(const mp_graph* g, mp_halo_plan** out);
int mp_halo_plan_sizes(const mp_halo_plan* p, int64_t* n_groups, int64_t* n_members,
                       int64_t* n_pairs, int64_t* n_pair_rows);
/* Host arrays, any may be NULL: group_ptr[n_groups+1], member[n_members],
 * pair_r[n_pairs], pair_s[n_pairs], pair_ptr[n_pairs+1],
 * pair_rows_r[n_pair_rows], pair_rows_s[n_pair_rows] (global row indices),
 * halo_rows[R], neighbours[R]. */
int mp_halo_plan_export(const mp_halo_plan* p, int32_t* group_ptr, int32_t* member,
                        int32_t* pair_r, int32_t* pair_s, int64_t* pair_ptr,
                        int32_t* pair_rows_r, int32_t* pair_rows_s,
                        int64_t* halo_rows, int32_t* neighbours);
/* checksum: content checksum of group_ptr and member, chained to the
 * checksum of the graph the plan was built on; graph_checksum: that graph's
 * mp_graph_checksum at build time.  A plan is valid only beside the graph
 * whose checksum equals its graph_checksum. */
int mp_halo_plan_checksum(const mp_halo_plan* p, uint64_t* checksum, uint64_t* graph_checksum);
int mp_halo_plan_destroy(mp_halo_plan* p);

/* ---------------------------------------------------------------------
 * Device graph descriptor (the reduced graph of Sec. II-A and the halo plan
 * of Eq. 4c-d).  All arrays are device memory holding copies of what
 * mp_graph_export / mp_halo_plan_export return; the caller keeps them
 * alive.  graph_checksum is mp_graph_checksum of the graph exported;
 * plan_checksum and plan_graph_checksum are the two values
 * mp_halo_plan_checksum returns for the plan exported.  seal is written by
 * mp_dev_graph_seal; every device entry point recomputes it from the
 * descriptor's sizes, pointers and checksums and rejects a descriptor that
 * is unsealed, was changed after sealing, or pairs a graph with a plan
 * built for another graph (MP_EPLAN, before any launch).
 * ------------------------------------------------------------------- */
typedef struct {
  int64_t n_rows, n_edges, n_groups, n_members;
  const int32_t* rowptr;    /* [n_rows+1] */
  const int32_t* recv;      /* [n_edges] receiver row */
  const int32_t* col;       /* [n_edges] sender row */
  const int32_t* rev;       /* [n_edges] reverse edge */
  const uint8_t* edge_mult; /* [n_edges] d_ij >= 1 */
  const int32_t* group_ptr; /* [n_groups+1] */
  const int32_t* member;    /* [n_members] (may be NULL when n_members = 0) */
  uint64_t graph_checksum;
  uint64_t plan_checksum;
  uint64_t plan_graph_checksum;
  uint64_t seal;
} mp_dev_graph;

/* Seal a filled descriptor (a set-up call, not asynchronous).  Checks the
 * sizes and pointers, and that the plan was built for this graph
 * (plan_graph_checksum == graph_checksum); with verify_device != 0 it also
 * reads every array back from the device (synchronous copies; host memory
 * for the largest array is allocated and freed) and recomputes both content
 * checksums, so arrays uploaded from another graph or plan, or changed on
 * the device, are refused.  Errors: MP_EINVAL (NULL descriptor or array,
 * bad sizes), MP_EPLAN (checksum mismatch), MP_EHIP (a copy failed).  On
 * error seal is left 0. */
int mp_dev_graph_seal(mp_dev_graph* g, int verify_device);

/* ---------------------------------------------------------------------
 * One consistent NMP layer (Eq. 4a-e) on all sub-graphs at once.
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t H;          /* hidden width: 32, 64 or 128 */
  int32_t layernorm;  /* 1: LayerNorm on the output of both MLPs */
  int32_t halo;       /* 1: consistent (Eq. 4c-d); 0: "None" mode, halo skipped */
  int32_t gemm_dtype; /* MP_F32 or MP_BF16 (operands rounded to nearest even) */
  float ln_eps;
  /* Schedule (0 = library default): edges per row-aligned tile of the edge
   * kernels (16..4096), and the persistent workgroup counts of the forward
   * and adjoint edge kernels (1..65536).  Results are bitwise reproducible
   * for a fixed schedule; another schedule only regroups floating-point
   * sums (block boundaries of the aggregation scan, weight-gradient slabs). */
  int32_t tile_edges;
  int32_t edge_grid;
  int32_t edge_bwd_grid;
  /* What Eq. 4b sums: MP_AGG_STATE (0) the updated edge state e' = e + MLP
   * (the equations as written), or MP_AGG_MESSAGE (1) the MLP output alone
   * (a variant; the edge-state update is unchanged). */
  int32_t aggregate;
  /* More schedule dimensions (0 = library default; the results of every
   * choice are bitwise reproducible, and equal up to the grouping of the
   * weight-gradient sums): waves per workgroup of the edge adjoint (4, or
   * 8 for BF16 GEMMs at H <= 64, which stage 16 x waves edges per
   * weight-gradient round, and at H > 64, whose split adjoint then runs
   * two waves per SIMD instead of one), and the tile order of the edge
   * forward (0: a
   * fixed round robin over each XCD's range of tiles; 1: waves take the
   * next tile of their XCD's range from an atomic counter and move on to
   * the other ranges when theirs is empty; tiles are row aligned, so the
   * results are bitwise those of the fixed order). */
  int32_t edge_bwd_waves;
  int32_t edge_fwd_queue;
  /* Storage type of the edge states and their gradients (e_in, e_out,
   * g_e_out, g_e_in of the entry points below): MP_F32, or MP_BF16 (with
   * gemm_dtype = MP_BF16 only; rounded to nearest even where stored, while
   * the edge update, the aggregation of Eq. 4b and the adjoint still run
   * in FP32 registers).  Halves the edge-state traffic at the cost of
   * BF16-rounded states between layers. */
  int32_t estate_dtype;
} mp_layer_cfg;

/* Parameters of one layer, device FP32.  Edge MLP: Linear(3H->H), ELU,
 * Linear(H->H) [, LayerNorm]; the input is [x_i (receiver), x_j (sender),
 * e_ij] (Eq. 4a).  Node MLP: Linear(2H->H), ELU, Linear(H->H)
 * [, LayerNorm] on [a*_i, x_i] (Eq. 4e).  Both updates are residual. */
typedef struct {
  const float *We1, *be1; /* [H][3H], [H] */
  const float *We2, *be2; /* [H][H],  [H] */
  const float *ge, *bge;  /* LayerNorm gain/shift [H] (unused without LN) */
  const float *Wn1, *bn1; /* [H][2H], [H] */
  const float *Wn2, *bn2; /* [H][H],  [H] */
  const float *gn, *bgn;  /* [H] */
} mp_layer_params;

/* Gradients, same shapes; overwritten (not accumulated) by the backward. */
typedef struct {
  float *We1, *be1, *We2, *be2, *ge, *bge;
  float *Wn1, *bn1, *Wn2, *bn2, *gn, *bgn;
} mp_layer_grads;

int mp_layer_workspace_size(const mp_layer_cfg* cfg, const mp_dev_graph* g,
                            int backward, size_t* bytes);

/* Forward.  x_in[N][H], e_in[E][H] -> x_out[N][H], e_out[E][H] (edge
 * states FP32, or BF16 with estate_dtype = MP_BF16; node arrays FP32).
 * e_out may be NULL: the updated edge state is then not written (a model's
 * last layer, whose e' nothing reads; Eq. 4b still sums it into a).
 * a_star_out[N][H] receives the synchronised aggregate a* (needed by the
 * backward); it may be NULL.  pq_out[2][N][H], if not NULL, receives the
 * node projections of the first edge-MLP Linear (Eq. 4a split over its
 * input): P = W1a x_in + b1, then Q = W1b x_in; handing them to the
 * backward saves recomputing them.  Outputs must not alias inputs.
 * ws_bytes must be at least mp_layer_workspace_size(cfg, g, 0); when both
 * a_star_out and pq_out are given, only a prefix of that layout is used
 * (the packed weights and the edge tile bounds), and a workspace of that
 * prefix's size is accepted. */
int mp_layer_forward(const mp_layer_cfg* cfg, const mp_layer_params* p,
                     const mp_dev_graph* g, const float* x_in, const void* e_in,
                     float* x_out, void* e_out, float* a_star_out, float* pq_out,
                     void* ws, size_t ws_bytes, mp_stream_t stream);

/* The same forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid it): no
 * workspace argument, and no device or host allocation in the call.  Its
 * scratch (the packed weights and the edge tile bounds) is a module array
 * of mp_layer_forward_noalloc_max_scratch() bytes (32 MiB) that every GPU
 * the library runs on holds until the process ends; its device address is
 * looked up once per device on the first call there.  a_star_out and
 * pq_out are required (so no node-sized scratch is needed); all other
 * arguments and the results are those of mp_layer_forward, bit for bit.
 * Errors: as mp_layer_forward, plus MP_EINVAL when a_star_out or pq_out is
 * NULL, when the scratch needed (weights plus 8 bytes per edge tile)
 * exceeds the maximum, or when the stream belongs to another device than
 * the current one; MP_EHIP if the scratch address cannot be obtained.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on
 * one GPU (two streams, two threads) race.  Nothing in the scratch needs
 * to start at zero (each call writes what it reads).  Launches of this
 * entry point are not recorded by mp_profile_enable. */
int mp_layer_forward_noalloc(const mp_layer_cfg* cfg, const mp_layer_params* p,
                             const mp_dev_graph* g, const float* x_in, const void* e_in,
                             float* x_out, void* e_out, float* a_star_out, float* pq_out,
                             mp_stream_t stream);
size_t mp_layer_forward_noalloc_max_scratch(void);

/* Backward (adjoint of the forward, Eq. 3): given the forward inputs, the
 * saved a*, and the gradients of the loss with respect to x_out and e_out,
 * write the gradients with respect to x_in and e_in and every parameter.
 * Edge-MLP activations are recomputed from (x_in, e_in), not stored.  The
 * halo sum is its own adjoint and is applied to the a* gradient.  g_e_out
 * may be NULL (zero).  pq is the forward's pq_out for the same inputs and
 * parameters, or NULL (then P and Q are recomputed).  e_in, g_e_out and
 * g_e_in are [E][H] in cfg->estate_dtype (FP32 or BF16); everything else
 * FP32. */
int mp_layer_backward(const mp_layer_cfg* cfg, const mp_layer_params* p,
                      const mp_dev_graph* g, const float* x_in, const void* e_in,
                      const float* a_star, const float* pq, const float* g_x_out, const void* g_e_out,
                      float* g_x_in, void* g_e_in, const mp_layer_grads* grads,
                      void* ws, size_t ws_bytes, mp_stream_t stream);

/* ---------------------------------------------------------------------
 * Encoder / decoder MLPs, edge inputs and loss (Sec. III, Eq. 5-6).
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t n_in;       /* input features: 3, 4, or a multiple of 16 up to 128 */
  int32_t H;          /* hidden width: 32, 64 or 128 */
  int32_t n_out;      /* output features: H, or 1..4 (decoder) */
  int32_t layernorm;  /* LayerNorm on the output (requires n_out == H) */
  int32_t gemm_dtype; /* MP_F32 or MP_BF16 for the H x H products */
  float ln_eps;
  /* Storage type of `out` (forward) and `g_out` (backward): MP_F32, or
   * MP_BF16 for the edge encoder of a model with BF16 edge states (n_in
   * <= 4, n_out == H, BF16 GEMMs only). */
  int32_t out_dtype;
} mp_mlp_cfg;

/* Linear(n_in->H), ELU, Linear(H->n_out) [, LayerNorm]. */
typedef struct {
  const float *W0, *b0, *W1, *b1, *ln_g, *ln_b;
} mp_mlp_params;
typedef struct {
  float *W0, *b0, *W1, *b1, *ln_g, *ln_b;
} mp_mlp_grads;

int mp_mlp_workspace_size(const mp_mlp_cfg* cfg, int64_t n_rows, int backward, size_t* bytes);
int mp_mlp_forward(const mp_mlp_cfg* cfg, const mp_mlp_params* p, int64_t n_rows,
                   const float* in, void* out, void* ws, size_t ws_bytes,
                   mp_stream_t stream);
/* g_in may be NULL (input gradient not needed). */
int mp_mlp_backward(const mp_mlp_cfg* cfg, const mp_mlp_params* p, int64_t n_rows,
                    const float* in, const void* g_out, float* g_in,
                    const mp_mlp_grads* grads, void* ws, size_t ws_bytes,
                    mp_stream_t stream);

/* ---------------------------------------------------------------------
 * Narrow deep MLPs: the paper's own models (Table I: H = 8 with two and
 * H = 32 with five extra hidden layers per MLP), FP32, hidden width 8, 16
 * or 32.  Every MLP is Linear(in->H), ELU, n_hidden x (Linear(H->H), ELU),
 * Linear(H->out) [, LayerNorm] (Sec. III), and its parameters are ONE
 * flat device FP32 array in torch.nn.Linear order:
 *   W0[H][in] b0[H], n_hidden x (W[H][H] b[H]), Wo[out][H] bo[out],
 *   then with LayerNorm gain[out] and shift[out].
 * Gradients use the same layout and are overwritten, not accumulated.
 * Results are bitwise reproducible run to run (fixed-order sums).
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t H;          /* 8, 16 or 32 */
  int32_t n_hidden;   /* 0..8 */
  int32_t layernorm;  /* LayerNorm on both MLPs' outputs */
  int32_t halo;       /* 1: consistent (Eq. 4c-d); 0: "None" mode */
  float ln_eps;
  int32_t aggregate;  /* MP_AGG_STATE or MP_AGG_MESSAGE, as in mp_layer_cfg */
} mp_deep_layer_cfg;

/* Floats in the flat parameter array of one MLP. */
int mp_deep_theta_size(int32_t n_in, int32_t H, int32_t n_hidden, int32_t n_out, int32_t layernorm,
                       int64_t* floats);

/* Workspace bytes (0 for the forward). */
int mp_deep_layer_workspace_size(const mp_deep_layer_cfg* cfg, const mp_dev_graph* g,
                                 int backward, size_t* bytes);

/* One consistent NMP layer (Eq. 4a-e) with deep MLPs: theta_edge is the
 * edge MLP (input [x_i, x_j, e_ij], 3H -> H), theta_node the node MLP
 * (input [a*_i, x_i], 2H -> H); both updates residual.  x_in[N][H],
 * e_in[E][H] -> x_out[N][H], e_out[E][H]; a_star_out[N][H] (required)
 * receives the synchronised aggregate for the backward.  Outputs must not
 * alias inputs.  Errors: MP_EINVAL for a bad configuration (H not 8, 16 or
 * 32, n_hidden outside [0, 8], a non-positive ln_eps with LayerNorm, an
 * unknown aggregate), NULL, unaligned or aliasing buffers; MP_EPLAN for a
 * graph descriptor that is unsealed, changed after sealing, or pairs a
 * graph with another graph's halo plan. */
int mp_deep_layer_forward(const mp_deep_layer_cfg* cfg, const float* theta_edge,
                          const float* theta_node, const mp_dev_graph* g, const float* x_in,
                          const float* e_in, float* x_out, float* e_out, float* a_star_out,
                          mp_stream_t stream);

/* Adjoint (Eq. 3) of mp_deep_layer_forward for the same inputs and a*:
 * gradients of x_in, e_in and both parameter arrays.  MLP activations are
 * recomputed; the workspace (mp_deep_layer_workspace_size) holds per-row
 * records of them.  g_e_out may be NULL (zero).  The graph needs its
 * reverse-edge array.  Errors: as mp_deep_layer_forward, plus MP_EINVAL
 * for a missing reverse-edge array or gradient outputs aliasing inputs and
 * MP_ENOMEM for ws_bytes below mp_deep_layer_workspace_size. */
int mp_deep_layer_backward(const mp_deep_layer_cfg* cfg, const float* theta_edge,
                           const float* theta_node, const mp_dev_graph* g, const float* x_in,
                           const float* e_in, const float* a_star, const float* g_x_out,
                           const float* g_e_out, float* g_x_in, float* g_e_in,
                           float* g_theta_edge, float* g_theta_node, void* ws, size_t ws_bytes,
                           mp_stream_t stream);

/* Encoder / decoder with deep MLPs (Sec. III).  (n_in, n_out) is
 * (1..8, H), (H, 1..4) or (H, H); LayerNorm needs n_out == H. */
typedef struct {
  int32_t n_in, H, n_hidden, n_out, layernorm;
  float ln_eps;
} mp_deep_mlp_cfg;

int mp_deep_mlp_workspace_size(const mp_deep_mlp_cfg* cfg, int64_t n_rows, int backward, size_t* bytes);
/* in[n_rows][n_in] -> out[n_rows][n_out], device FP32. */
int mp_deep_mlp_forward(const mp_deep_mlp_cfg* cfg, const float* theta, int64_t n_rows,
                        const float* in, float* out, mp_stream_t stream);
/* g_in[n_rows][n_in] may be NULL (input gradient not needed). */
int mp_deep_mlp_backward(const mp_deep_mlp_cfg* cfg, const float* theta, int64_t n_rows,
                         const float* in, const float* g_out, float* g_in, float* g_theta,
                         void* ws, size_t ws_bytes, mp_stream_t stream);

/* Edge input features of Sec. III: e0[k] = (p_j - p_i, |p_j - p_i|) for
 * edge k with receiver i and sender j; row_pos[N][3] in FP64 (device), the
 * difference taken in FP64 and rounded once to FP32.  e0 is [E][4] (device).
 * period (host, 3 doubles, or NULL for none): on an axis with period L > 0
 * the difference is taken to the nearest periodic image of p_j, so a link
 * across a periodic boundary gets its element-local difference.  Errors:
 * row_u (device FP32 [N][3], or NULL): a node field; with it e0 is [E][7]
 * and channels 4..6 are u_j - u_i (the relative velocity of the edge
 * features Sec. III lists; the models of Table I use the first four), an
 * FP32 difference.  Errors: MP_EINVAL for NULL buffers, a 4-channel e0 not
 * 16-byte aligned, or a negative or non-finite period. */
int mp_edge_inputs(const mp_dev_graph* g, const double* row_pos, const double* period,
                   const float* row_u, float* e0, mp_stream_t stream);

/* Consistent MSE (Eq. 6a-c): loss = sum_i sum_f (1/d_i)(Y-T)^2 / (N_eff F)
 * with N_eff = sum_i 1/d_i, over all rows of all sub-graphs; for R=1
 * (every d_i = 1) this is the MSE of Eq. 5.  Y, T are [N][F] FP32,
 * node_mult[N] the degrees d_i; writes loss[1] (FP32, summed in FP64 in a
 * fixed order) and gY[N][F] = dloss/dY.  gY may be NULL. */
int mp_consistent_mse(int64_t n_rows, int32_t F, const float* Y, const float* T,
                      const uint8_t* node_mult, float* loss, float* gY,
                      void* ws, size_t ws_bytes, mp_stream_t stream);
int mp_consistent_mse_workspace_size(int64_t n_rows, size_t* bytes);

/* ---------------------------------------------------------------------
 * Measurement hooks.  While profiling is on, every kernel launch made by
 * the entry points above is bracketed by two HIP events recorded on the
 * launch's own stream.  mp_profile_enable clears the records (and turns
 * recording on or off); mp_profile_read waits for and sums the elapsed
 * times of one kernel's launches recorded since then.  Kernel names:
 * tiles, pack, proj, edge_fwd, halo, halo_adj, node_fwd, node_bwd, edge_bwd,
 * edge_dw, node_dw, gq_dw (weight gradients of the split adjoints, H = 128), gq,
 * wreduce, mlp_fwd, mlp_bwd, edge_inputs, loss; for the deep MLPs deep_edge_fwd,
 * deep_node_fwd, deep_node_bwd, deep_edge_bwd, deep_gather, deep_node_dw, deep_edge_dw,
 * deep_mlp_fwd, deep_mlp_bwd, deep_mlp_dw.
 * ------------------------------------------------------------------- */
int mp_profile_enable(int on);
int mp_profile_read(const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* MPLAYER_H */
