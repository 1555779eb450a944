// C ABI entry points: validation, workspace layout and launch sequences.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mp_internal.hpp"
#include "mp_device.hpp"
#include "mp_kernels.hpp"

using namespace mp;

static thread_local char g_err[512] = "";

int mp_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

extern "C" int mp_abi_version(void) { return MP_ABI_VERSION; }
extern "C" const char* mp_last_error(void) { return g_err; }

namespace {

// The value a sealed descriptor carries: a hash of its sizes, array
// pointers and checksums, so a descriptor edited after sealing is refused.
uint64_t seal_value(const mp_dev_graph* g) {
  const uint64_t v[14] = {(uint64_t)g->n_rows, (uint64_t)g->n_edges, (uint64_t)g->n_groups,
                          (uint64_t)g->n_members, (uint64_t)(uintptr_t)g->rowptr, (uint64_t)(uintptr_t)g->recv,
                          (uint64_t)(uintptr_t)g->col, (uint64_t)(uintptr_t)g->rev,
                          (uint64_t)(uintptr_t)g->edge_mult, (uint64_t)(uintptr_t)g->group_ptr,
                          (uint64_t)(uintptr_t)g->member, g->graph_checksum, g->plan_checksum,
                          g->plan_graph_checksum};
  return mp::hash_bytes(v, sizeof(v), 0x6d707365616cull) | 1u;  // never 0: 0 means "not sealed"
}

}  // namespace

extern "C" int mp_dev_graph_seal(mp_dev_graph* g, int verify_device) {
  if (!g) return mp_fail(MP_EINVAL, "mp_dev_graph_seal: descriptor is NULL");
  g->seal = 0;
  if (g->n_rows <= 0 || g->n_edges <= 0 || g->n_groups < 0 || g->n_members < 0)
    return mp_fail(MP_EINVAL, "mp_dev_graph_seal: sizes must be positive (rows %lld, edges %lld)",
                   (long long)g->n_rows, (long long)g->n_edges);
  if (!g->rowptr || !g->recv || !g->col || !g->rev || !g->edge_mult || !g->group_ptr ||
      (g->n_members > 0 && !g->member))
    return mp_fail(MP_EINVAL, "mp_dev_graph_seal: an array pointer is NULL");
  if (g->plan_graph_checksum != g->graph_checksum)
    return mp_fail(MP_EPLAN, "mp_dev_graph_seal: the halo plan was built for another graph "
                   "(plan's graph checksum %016llx, graph checksum %016llx)",
                   (unsigned long long)g->plan_graph_checksum, (unsigned long long)g->graph_checksum);
  if (verify_device) {
    // Read every array back and recompute both checksums.
    std::vector<unsigned char> buf;
    hipError_t err = hipSuccess;
    auto fetch = [&](const void* p, size_t bytes) -> const void* {
      try {
        buf.resize(bytes);
      } catch (...) {
        err = hipErrorOutOfMemory;
        return nullptr;
      }
      if (bytes == 0) return buf.data();
      err = hipMemcpy(buf.data(), p, bytes, hipMemcpyDeviceToHost);
      return err == hipSuccess ? buf.data() : nullptr;
    };
    const uint64_t gcs = mp::graph_checksum_of(g->n_rows, g->n_edges, g->rowptr, g->recv, g->col, g->rev,
                                               g->edge_mult, fetch);
    if (err != hipSuccess) return mp_fail(MP_EHIP, "mp_dev_graph_seal: reading the graph arrays: %s", hipGetErrorString(err));
    if (gcs != g->graph_checksum)
      return mp_fail(MP_EPLAN, "mp_dev_graph_seal: the device graph arrays do not match the graph checksum");
    const uint64_t pcs = mp::plan_checksum_of(g->graph_checksum, g->n_groups, g->n_members, g->group_ptr,
                                              g->member, fetch);
    if (err != hipSuccess) return mp_fail(MP_EHIP, "mp_dev_graph_seal: reading the halo plan: %s", hipGetErrorString(err));
    if (pcs != g->plan_checksum)
      return mp_fail(MP_EPLAN, "mp_dev_graph_seal: the device halo plan does not match the plan checksum "
                     "(or was built for another graph)");
  }
  g->seal = seal_value(g);
  return MP_OK;
}

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int hip_check(hipError_t e, const char* where) {
  if (e == hipSuccess) return MP_OK;
  return mp_fail(MP_EHIP, "%s: %s", where, hipGetErrorString(e));
}

int check_graph(const mp_dev_graph* g, bool need_rev) {
  if (!g) return mp_fail(MP_EINVAL, "graph descriptor is NULL");
  if (g->n_rows <= 0 || g->n_edges <= 0 || g->n_groups < 0 || g->n_members < 0)
    return mp_fail(MP_EINVAL, "graph sizes must be positive (rows %lld, edges %lld)", (long long)g->n_rows,
                   (long long)g->n_edges);
  if (g->n_rows >= (int64_t(1) << 31) - 1 || g->n_edges >= (int64_t(1) << 31) - 1)
    return mp_fail(MP_EINVAL, "graph has 2^31-1 or more rows or edges");
  if (!g->rowptr || !g->recv || !g->col || !g->edge_mult || (need_rev && !g->rev))
    return mp_fail(MP_EINVAL, "graph array is NULL");
  if (g->n_groups > 0 && (!g->group_ptr || !g->member)) return mp_fail(MP_EINVAL, "halo plan array is NULL");
  if (g->plan_graph_checksum != g->graph_checksum)
    return mp_fail(MP_EPLAN, "graph descriptor pairs a graph with a halo plan built for another graph");
  if (g->seal == 0 || g->seal != seal_value(g))
    return mp_fail(MP_EPLAN, "graph descriptor is not sealed, or was changed after mp_dev_graph_seal");
  return MP_OK;
}

DevGraph dev_graph(const mp_dev_graph* g) {
  DevGraph d;
  d.n_rows = g->n_rows;
  d.n_edges = g->n_edges;
  d.n_groups = g->n_groups;
  d.rowptr = g->rowptr;
  d.recv = g->recv;
  d.col = g->col;
  d.rev = g->rev;
  d.mult = g->edge_mult;
  d.group_ptr = g->group_ptr;
  d.member = g->member;
  d.n_tiles = 0;
  d.tile_r = d.tile_e = nullptr;
  d.queue = nullptr;
  return d;
}

int64_t n_tiles_for(int64_t E, int tile_edges) {
  const int64_t te = tile_edges > 0 ? tile_edges : kTileEdges;
  return std::max<int64_t>(1, (E + te - 1) / te);
}

int check_cfg(const mp_layer_cfg* c) {
  if (!c) return mp_fail(MP_EINVAL, "layer config is NULL");
  if (c->H != 32 && c->H != 64 && c->H != 128) return mp_fail(MP_EINVAL, "H must be 32, 64 or 128 (got %d)", c->H);
  if (c->gemm_dtype != MP_F32 && c->gemm_dtype != MP_BF16) return mp_fail(MP_EINVAL, "gemm_dtype must be MP_F32 or MP_BF16");
  if (c->layernorm && !(c->ln_eps > 0.f)) return mp_fail(MP_EINVAL, "ln_eps must be positive");
  if (c->tile_edges != 0 && (c->tile_edges < 16 || c->tile_edges > 4096))
    return mp_fail(MP_EINVAL, "tile_edges must be 0 or in [16, 4096] (got %d)", c->tile_edges);
  if (c->edge_grid < 0 || c->edge_grid > 65536 || c->edge_bwd_grid < 0 || c->edge_bwd_grid > 65536)
    return mp_fail(MP_EINVAL, "edge grids must be 0 or in [1, 65536]");
  if (c->aggregate != MP_AGG_STATE && c->aggregate != MP_AGG_MESSAGE)
    return mp_fail(MP_EINVAL, "aggregate must be MP_AGG_STATE or MP_AGG_MESSAGE");
  if (c->edge_bwd_waves != 0 && c->edge_bwd_waves != 4 &&
      !(c->edge_bwd_waves == 8 && ((c->gemm_dtype == MP_BF16 && c->H <= 64) || c->H > 64)))
    return mp_fail(MP_EINVAL, "edge_bwd_waves must be 0, 4, or 8 (BF16 GEMMs at H <= 64, or H > 64; got %d)",
                   c->edge_bwd_waves);
  if (c->edge_fwd_queue != 0 && c->edge_fwd_queue != 1)
    return mp_fail(MP_EINVAL, "edge_fwd_queue must be 0 or 1 (got %d)", c->edge_fwd_queue);
  if (c->estate_dtype != MP_F32 && c->estate_dtype != MP_BF16)
    return mp_fail(MP_EINVAL, "estate_dtype must be MP_F32 or MP_BF16");
  if (c->estate_dtype == MP_BF16 && c->gemm_dtype != MP_BF16)
    return mp_fail(MP_EINVAL, "BF16 edge states need BF16 GEMMs (gemm_dtype = MP_BF16)");
  return MP_OK;
}

// Grid sizes: persistent edge kernels give every wave at least ~64 edges.
int edge_grid(int64_t E) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, E / 256)); }
int edge_bwd_grid(int64_t E) { return (int)std::max<int64_t>(1, std::min<int64_t>(512, E / 256)); }
int row_grid(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (N + 63) / 64)); }
int row_bwd_grid(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(512, (N + 255) / 256)); }

// Packed fragments of one layer, in this order:
// W1a W1b | W1c W2 W2^T W1c^T | Wn1 Wn2 Wn2^T Wn1^T | [W1a|W1b]^T
struct LayerFrags {
  size_t f1, f2;  // bytes of an H x H and an H x 2H matrix
  size_t proj, edge, node, gq, total;
  LayerFrags(int H, bool bf) {
    f1 = frag_bytes(H, H, bf);
    f2 = frag_bytes(H, 2 * H, bf);
    proj = 0;
    edge = proj + 2 * f1;
    node = edge + 4 * f1;
    gq = node + 2 * f2 + 2 * f1;
    total = align_up(gq + f2);
  }
};

struct LayerWs {
  LayerFrags fr;
  size_t P, Q, a, gP, gh, gQ, part_e, part_n, part_q, tile_r, tile_e, queue, total;
  size_t sgm, su;  // split edge adjoint: per-edge weight-gradient factors
  size_t nu, ngy, ngz, ngx;   // split node adjoint: per-row weight-gradient factors
  int ge, gbe, gn, gbn;
  int64_t n_tiles;
  LayerWs(const mp_layer_cfg* c, const mp_dev_graph* g, bool bwd) : fr(c->H, c->gemm_dtype == MP_BF16) {
    const size_t H = c->H, N = g->n_rows, E = g->n_edges;
    ge = c->edge_grid > 0 ? c->edge_grid : edge_grid(E);
    gbe = c->edge_bwd_grid > 0 ? c->edge_bwd_grid : edge_bwd_grid(E);
    gn = row_grid(N);
    gbn = row_bwd_grid(N);
    n_tiles = n_tiles_for(E, c->tile_edges);
    size_t o = fr.total;
    tile_r = o; o = align_up(o + (size_t)(n_tiles + 1) * 4);
    tile_e = o; o = align_up(o + (size_t)(n_tiles + 1) * 4);
    queue = o; o = align_up(o + 8 * 4);
    P = o; o = align_up(o + N * H * 4);
    Q = o; o = align_up(o + N * H * 4);
    a = o; o = align_up(o + N * H * 4);
    gP = gh = gQ = part_e = part_n = part_q = 0;
    sgm = su = 0;
    nu = ngy = ngz = ngx = 0;
    if (bwd) {
      const size_t eb = E * H * (c->gemm_dtype == MP_BF16 ? 2 : 4);
      gP = o; o = align_up(o + N * H * 4);
      if (gq_split(c->H, c->gemm_dtype == MP_BF16)) {
        gQ = o;
        o = align_up(o + N * H * 4);
      }
      gh = o; o = align_up(o + eb);
      if (edge_bwd_split(c->H)) {
        sgm = o; o = align_up(o + eb);
        su = o; o = align_up(o + eb);
      }
      if (node_bwd_split(c->H, c->gemm_dtype == MP_BF16)) {
        const size_t nb = N * H * (c->gemm_dtype == MP_BF16 ? 2 : 4);  // factors in the product type
        nu = o; o = align_up(o + nb);
        ngy = o; o = align_up(o + nb);
        ngz = o; o = align_up(o + nb);
        ngx = o; o = align_up(o + nb);
      }
      part_e = o; o = align_up(o + (size_t)gbe * edge_slab(c->H) * 4);
      part_n = o; o = align_up(o + (size_t)gbn * mlp_slab(c->H, 2 * c->H, c->H) * 4);
      part_q = o; o = align_up(o + (size_t)gbn * gq_slab(c->H) * 4);
    }
    total = o;
  }
};

PackView view(const float* p, int ld, int off, int trans) { return PackView{p, ld, off, trans}; }

void add_job(PackJobs& J, int rows, int cols, PackView a, size_t dst, PackView b = PackView{nullptr, 0, 0, 0},
             int split = -1) {
  PackJob& j = J.job[J.n++];
  j.a = a;
  j.b = b.p ? b : a;
  j.rows = rows;
  j.cols = cols;
  j.split = split < 0 ? cols : split;
  j.dst_off = (int64_t)dst;
}

// Jobs for the layer fragments; the transposed ones only for the backward.
PackJobs layer_jobs(const mp_layer_cfg* c, const mp_layer_params* p, const LayerFrags& F, bool bwd) {
  const int H = c->H;
  PackJobs J;
  J.n = 0;
  J.bf = c->gemm_dtype == MP_BF16;
  add_job(J, H, H, view(p->We1, 3 * H, 0, 0), F.proj);                     // W1a
  add_job(J, H, H, view(p->We1, 3 * H, H, 0), F.proj + F.f1);              // W1b
  add_job(J, H, H, view(p->We1, 3 * H, 2 * H, 0), F.edge);                 // W1c
  add_job(J, H, H, view(p->We2, H, 0, 0), F.edge + F.f1);                  // W2
  add_job(J, H, 2 * H, view(p->Wn1, 2 * H, 0, 0), F.node);                 // Wn1
  add_job(J, H, H, view(p->Wn2, H, 0, 0), F.node + F.f2);                  // Wn2
  if (bwd) {
    add_job(J, H, H, view(p->We2, H, 0, 1), F.edge + 2 * F.f1);            // W2^T
    add_job(J, H, H, view(p->We1, 3 * H, 2 * H, 1), F.edge + 3 * F.f1);    // W1c^T
    add_job(J, H, H, view(p->Wn2, H, 0, 1), F.node + F.f2 + F.f1);         // Wn2^T
    add_job(J, 2 * H, H, view(p->Wn1, 2 * H, 0, 1), F.node + F.f2 + 2 * F.f1);  // Wn1^T
    // [W1a | W1b]^T: element (k, c) = c < H ? We1[c][k] : We1[c-H][H+k]
    add_job(J, H, 2 * H, view(p->We1, 3 * H, 0, 1), F.gq, view(p->We1, 3 * H, H, 1), H);
  }
  return J;
}

int check_layer_params(const mp_layer_cfg* c, const mp_layer_params* p) {
  if (!p) return mp_fail(MP_EINVAL, "layer parameters are NULL");
  const void* req[] = {p->We1, p->be1, p->We2, p->be2, p->Wn1, p->bn1, p->Wn2, p->bn2};
  for (const void* q : req)
    if (!q || !aligned16(q)) return mp_fail(MP_EINVAL, "a layer parameter is NULL or not 16-byte aligned");
  if (c->layernorm) {
    const void* lq[] = {p->ge, p->bge, p->gn, p->bgn};
    for (const void* q : lq)
      if (!q || !aligned16(q)) return mp_fail(MP_EINVAL, "a LayerNorm parameter is NULL or not 16-byte aligned");
  }
  return MP_OK;
}

char* ws_at(void* ws, size_t off) { return reinterpret_cast<char*>(ws) + off; }
float* wsf(void* ws, size_t off) { return reinterpret_cast<float*>(ws_at(ws, off)); }

}  // namespace

// ------------------------------------------------------- launch profiling
// Optional per-kernel timing: when enabled, every launch is bracketed by
// two HIP events recorded on the launch's own stream.
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
  hipEvent_t e = nullptr;
  if (!g_prof_pool.empty()) {
    e = g_prof_pool.back();
    g_prof_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// Set while an entry point that must not create anything runs (the
// allocation-free forward): its launches are not bracketed by events.
thread_local bool t_no_prof = false;

long prof_begin(const char* name, hipStream_t s) {
  if (t_no_prof) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return -1;
  ProfRec r{name, prof_event(), prof_event()};
  if (!r.a || !r.b) return -1;
  (void)hipEventRecord(r.a, s);
  g_prof.push_back(r);
  return (long)g_prof.size() - 1;
}

void prof_end(long idx, hipStream_t s) {
  if (idx < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (idx < (long)g_prof.size()) (void)hipEventRecord(g_prof[idx].b, s);
}

template <class F>
int run(const char* name, hipStream_t s, F&& f) {
  const long slot = prof_begin(name, s);
  const hipError_t e = f();
  prof_end(slot, s);
  return hip_check(e, name);
}
}  // namespace

extern "C" int mp_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof) {
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof.clear();
  g_prof_on = on != 0;
  return MP_OK;
}

extern "C" int mp_profile_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return mp_fail(MP_EINVAL, "mp_profile_read: NULL argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double t = 0.0;
  int64_t n = 0;
  for (auto& r : g_prof) {
    if (r.name != kernel) continue;
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      return mp_fail(MP_EHIP, "mp_profile_read: event query failed");
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return MP_OK;
}

extern "C" int mp_layer_workspace_size(const mp_layer_cfg* cfg, const mp_dev_graph* g, int backward, size_t* bytes) {
  int rc;
  if ((rc = check_cfg(cfg)) || (rc = check_graph(g, false))) return rc;
  if (!bytes) return mp_fail(MP_EINVAL, "bytes is NULL");
  *bytes = LayerWs(cfg, g, backward != 0).total;
  return MP_OK;
}

namespace {

// Validation of the forward's arguments (everything but the workspace).
int check_layer_forward(const mp_layer_cfg* cfg, const mp_layer_params* p, const mp_dev_graph* g,
                        const float* x_in, const void* e_in, const float* x_out, const void* e_out,
                        const float* a_star_out, const float* pq_out) {
  int rc;
  if ((rc = check_cfg(cfg)) || (rc = check_graph(g, false)) || (rc = check_layer_params(cfg, p))) return rc;
  if (!x_in || !e_in || !x_out) return mp_fail(MP_EINVAL, "mp_layer_forward: NULL buffer");
  if (!aligned16(x_in) || !aligned16(e_in) || !aligned16(x_out) || (e_out && !aligned16(e_out)) ||
      (a_star_out && !aligned16(a_star_out)) || (pq_out && !aligned16(pq_out)))
    return mp_fail(MP_EINVAL, "mp_layer_forward: buffers must be 16-byte aligned");
  if (x_out == x_in || (e_out && (e_out == e_in || e_out == (const void*)x_in)) ||
      (const void*)x_out == e_in || (pq_out && ((const float*)pq_out == x_in || (const void*)pq_out == e_in)))
    return mp_fail(MP_EINVAL, "mp_layer_forward: outputs must not alias inputs");
  return MP_OK;
}

// Bytes of the forward workspace actually used: the whole layout, or only
// its prefix (packed weights and tile bounds) when the caller supplies the
// node projections and the aggregate.
size_t layer_forward_ws_need(const LayerWs& W, const float* a_star_out, const float* pq_out) {
  return (a_star_out && pq_out) ? W.P : W.total;
}

// The forward's launch sequence (arguments validated, workspace checked).
int layer_forward_launch(const mp_layer_cfg* cfg, const mp_layer_params* p, const mp_dev_graph* g,
                         const float* x_in, const void* e_in, float* x_out, void* e_out, float* a_star_out,
                         float* pq_out, void* ws, const LayerWs& W, mp_stream_t stream) {
  int rc;
  const int H = cfg->H;
  const bool bf = cfg->gemm_dtype == MP_BF16;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  DevGraph d = dev_graph(g);
  d.n_tiles = W.n_tiles;
  d.tile_r = reinterpret_cast<const int32_t*>(ws_at(ws, W.tile_r));
  d.tile_e = reinterpret_cast<const int32_t*>(ws_at(ws, W.tile_e));
  d.queue = reinterpret_cast<int32_t*>(ws_at(ws, W.queue));
  float* P = pq_out ? pq_out : wsf(ws, W.P);
  float* Q = pq_out ? pq_out + (size_t)g->n_rows * cfg->H : wsf(ws, W.Q);
  float* a = a_star_out ? a_star_out : wsf(ws, W.a);
  if ((rc = run("tiles", s, [&] {
         return launch_tiles(d, reinterpret_cast<int32_t*>(ws_at(ws, W.tile_r)),
                             reinterpret_cast<int32_t*>(ws_at(ws, W.tile_e)), d.queue, s);
       })))
    return rc;
  if ((rc = run("pack", s, [&] { return launch_pack(layer_jobs(cfg, p, W.fr, false), ws, s); }))) return rc;
  if ((rc = run("proj", s, [&] { return launch_proj(H, bf, d, x_in, ws_at(ws, W.fr.proj), p->be1, P, Q, W.gn, s); }))) return rc;
  const bool es = cfg->estate_dtype == MP_BF16;
  if ((rc = run("edge_fwd", s, [&] {
         return launch_edge_fwd(H, cfg->layernorm != 0, bf, cfg->aggregate != 0, cfg->edge_fwd_queue != 0, es, d, P,
                                Q, e_in, ws_at(ws, W.fr.edge), p->be2, p->ge, p->bge, cfg->ln_eps, e_out, a, W.ge, s);
       })))
    return rc;
  if (cfg->halo && (rc = run("halo", s, [&] { return launch_halo(H, d, a, s); }))) return rc;
  MlpFwdArgs m{};
  m.n_rows = g->n_rows;
  m.src0 = a;
  m.src1 = x_in;
  m.resid = x_in;
  m.k0 = H;
  m.k1 = H;
  m.H = H;
  m.n_out = H;
  m.ln = cfg->layernorm;
  m.bf = bf;
  m.b0 = p->bn1;
  m.b1 = p->bn2;
  m.lng = p->gn;
  m.lnb = p->bgn;
  m.eps = cfg->ln_eps;
  m.frag0 = ws_at(ws, W.fr.node);
  m.frag1 = ws_at(ws, W.fr.node + W.fr.f2);
  m.out = x_out;
  return run("node_fwd", s, [&] { return launch_mlp_fwd(m, W.gn, s); });
}

}  // namespace

extern "C" int mp_layer_forward(const mp_layer_cfg* cfg, const mp_layer_params* p, const mp_dev_graph* g,
                                const float* x_in, const void* e_in, float* x_out, void* e_out, float* a_star_out,
                                float* pq_out, void* ws, size_t ws_bytes, mp_stream_t stream) {
  int rc;
  if ((rc = check_layer_forward(cfg, p, g, x_in, e_in, x_out, e_out, a_star_out, pq_out))) return rc;
  if (!ws) return mp_fail(MP_EINVAL, "mp_layer_forward: NULL workspace");
  if (!aligned16(ws)) return mp_fail(MP_EINVAL, "mp_layer_forward: workspace must be 16-byte aligned");
  const LayerWs W(cfg, g, false);
  const size_t need = layer_forward_ws_need(W, a_star_out, pq_out);
  if (ws_bytes < need) return mp_fail(MP_ENOMEM, "mp_layer_forward: workspace %zu < %zu bytes", ws_bytes, need);
  return layer_forward_launch(cfg, p, g, x_in, e_in, x_out, e_out, a_star_out, pq_out, ws, W, stream);
}

// ----------------------------------------- allocation-free layer forward
// Scratch of mp_layer_forward_noalloc: the packed weights and the edge
// tile bounds, in a module array that every GPU the library runs on holds
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in); it uses the device address
// hipGetSymbolAddress returns, looked up once per device.
constexpr size_t kNoallocScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(hipStream_t s, void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return mp_fail(MP_EHIP, "mp_layer_forward_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return mp_fail(MP_EINVAL, "mp_layer_forward_noalloc: device %d out of range", dev);
  if (s) {
    hipDevice_t sd = -1;
    e = hipStreamGetDevice(s, &sd);
    if (e != hipSuccess)
      return mp_fail(MP_EHIP, "mp_layer_forward_noalloc: hipStreamGetDevice: %s", hipGetErrorString(e));
    if (sd != dev)
      return mp_fail(MP_EINVAL, "mp_layer_forward_noalloc: the stream belongs to device %d, the current device is %d",
                     (int)sd, dev);
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return mp_fail(MP_EHIP, "mp_layer_forward_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MP_OK;
}

struct NoProfile {
  NoProfile() { t_no_prof = true; }
  ~NoProfile() { t_no_prof = false; }
};
}  // namespace

extern "C" size_t mp_layer_forward_noalloc_max_scratch(void) { return kNoallocScratchBytes; }

extern "C" int mp_layer_forward_noalloc(const mp_layer_cfg* cfg, const mp_layer_params* p, const mp_dev_graph* g,
                                        const float* x_in, const void* e_in, float* x_out, void* e_out,
                                        float* a_star_out, float* pq_out, mp_stream_t stream) {
  int rc;
  if ((rc = check_layer_forward(cfg, p, g, x_in, e_in, x_out, e_out, a_star_out, pq_out))) return rc;
  if (!a_star_out || !pq_out)
    return mp_fail(MP_EINVAL, "mp_layer_forward_noalloc: a_star_out and pq_out are required");
  const LayerWs W(cfg, g, false);
  const size_t need = layer_forward_ws_need(W, a_star_out, pq_out);
  if (need > kNoallocScratchBytes)
    return mp_fail(MP_EINVAL, "mp_layer_forward_noalloc: needs %zu bytes of scratch, the maximum is %zu "
                   "(fewer edges or larger tiles)", need, kNoallocScratchBytes);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* ws = nullptr;
  if ((rc = noalloc_scratch(s, &ws))) return rc;
  NoProfile np;
  return layer_forward_launch(cfg, p, g, x_in, e_in, x_out, e_out, a_star_out, pq_out, ws, W, stream);
}

extern "C" int mp_layer_backward(const mp_layer_cfg* cfg, const mp_layer_params* p, const mp_dev_graph* g,
                                 const float* x_in, const void* e_in, const float* a_star, const float* pq,
                                 const float* g_x_out, const void* g_e_out, float* g_x_in, void* g_e_in,
                                 const mp_layer_grads* gr,
                                 void* ws, size_t ws_bytes, mp_stream_t stream) {
  int rc;
  if ((rc = check_cfg(cfg)) || (rc = check_graph(g, true)) || (rc = check_layer_params(cfg, p))) return rc;
  if (!x_in || !e_in || !a_star || !g_x_out || !g_x_in || !g_e_in || !gr || !ws)
    return mp_fail(MP_EINVAL, "mp_layer_backward: NULL buffer");
  const void* al[] = {x_in, e_in, a_star, g_x_out, g_x_in, g_e_in, ws};
  for (const void* q : al)
    if (!aligned16(q)) return mp_fail(MP_EINVAL, "mp_layer_backward: buffers must be 16-byte aligned");
  if (g_e_out && !aligned16(g_e_out)) return mp_fail(MP_EINVAL, "mp_layer_backward: g_e_out not aligned");
  if (pq && !aligned16(pq)) return mp_fail(MP_EINVAL, "mp_layer_backward: pq not aligned");
  float* gw[] = {gr->We1, gr->be1, gr->We2, gr->be2, gr->Wn1, gr->bn1, gr->Wn2, gr->bn2};
  for (float* q : gw)
    if (!q) return mp_fail(MP_EINVAL, "mp_layer_backward: a gradient buffer is NULL");
  if (cfg->layernorm && (!gr->ge || !gr->bge || !gr->gn || !gr->bgn))
    return mp_fail(MP_EINVAL, "mp_layer_backward: a LayerNorm gradient buffer is NULL");
  if ((const float*)g_x_in == g_x_out || (const void*)g_e_in == g_e_out || (const void*)g_e_in == e_in ||
      (const float*)g_x_in == x_in)
    return mp_fail(MP_EINVAL, "mp_layer_backward: gradient outputs must not alias inputs");
  const LayerWs W(cfg, g, true);
  if (ws_bytes < W.total) return mp_fail(MP_ENOMEM, "mp_layer_backward: workspace %zu < %zu bytes", ws_bytes, W.total);
  const int H = cfg->H;
  const bool bf = cfg->gemm_dtype == MP_BF16;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  DevGraph d = dev_graph(g);
  d.n_tiles = W.n_tiles;
  d.tile_r = reinterpret_cast<const int32_t*>(ws_at(ws, W.tile_r));
  d.tile_e = reinterpret_cast<const int32_t*>(ws_at(ws, W.tile_e));
  d.queue = reinterpret_cast<int32_t*>(ws_at(ws, W.queue));
  const float* P = pq ? pq : wsf(ws, W.P);
  const float* Q = pq ? pq + (size_t)g->n_rows * H : wsf(ws, W.Q);
  float* ga = wsf(ws, W.a);
  if ((rc = run("tiles", s, [&] {
         return launch_tiles(d, reinterpret_cast<int32_t*>(ws_at(ws, W.tile_r)),
                             reinterpret_cast<int32_t*>(ws_at(ws, W.tile_e)), d.queue, s);
       })))
    return rc;
  float* gP = wsf(ws, W.gP);
  void* gh = ws_at(ws, W.gh);
  if ((rc = run("pack", s, [&] { return launch_pack(layer_jobs(cfg, p, W.fr, true), ws, s); }))) return rc;
  if (!pq && (rc = run("proj", s, [&] {
                return launch_proj(H, bf, d, x_in, ws_at(ws, W.fr.proj), p->be1, wsf(ws, W.P), wsf(ws, W.Q), W.gn, s);
              })))
    return rc;
  // node MLP adjoint: g_a* and g_x (residual + node-MLP part)
  MlpBwdArgs m{};
  m.n_rows = g->n_rows;
  m.src0 = a_star;
  m.src1 = x_in;
  m.k0 = H;
  m.k1 = H;
  m.H = H;
  m.n_out = H;
  m.ln = cfg->layernorm;
  m.bf = bf;
  m.resid = 1;
  m.b0 = p->bn1;
  m.b1 = p->bn2;
  m.lng = p->gn;
  m.lnb = p->bgn;
  m.eps = cfg->ln_eps;
  m.frag0 = ws_at(ws, W.fr.node);
  m.frag1 = ws_at(ws, W.fr.node + W.fr.f2);
  m.frag1t = ws_at(ws, W.fr.node + W.fr.f2 + W.fr.f1);
  m.frag0t = ws_at(ws, W.fr.node + W.fr.f2 + 2 * W.fr.f1);
  m.g_out = g_x_out;
  m.g_src0 = ga;
  m.g_src1 = g_x_in;
  m.g_add1 = g_x_out;
  m.part = wsf(ws, W.part_n);
  m.slab = mlp_slab(H, 2 * H, H);
  if (node_bwd_split(H, bf)) {
    // wide layers: the adjoint writes per-row factors, then the weight
    // gradients are summed from them into the fused kernel's slab layout
    void* nu = ws_at(ws, W.nu);
    void* ngy = ws_at(ws, W.ngy);
    void* ngz = ws_at(ws, W.ngz);
    void* ngx = ws_at(ws, W.ngx);
    if ((rc = run("node_bwd", s, [&] { return launch_node_bwd_split(m, nu, ngy, ngz, ngx, W.gbn, s); }))) return rc;
    const int64_t s1 = 2 * (int64_t)H * H + H;  // dW1 block of the slab
    RowDwArgs rd{};
    rd.n_rows = g->n_rows;
    rd.GW = H;
    rd.bf = bf;
    rd.part = m.part;
    rd.slab = m.slab;
    rd.AW = H;  // dW1 = sum g_y u^T, db1 = sum g_y
    rd.G = ngy;
    rd.g_bf = bf;
    rd.A = nu;
    rd.a_bf = bf;
    rd.off = s1;
    rd.colsum_off = s1 + (int64_t)H * H;
    if ((rc = run("node_dw", s, [&] { return launch_row_dw(rd, W.gbn, s); }))) return rc;
    rd.AW = 2 * H;  // dW0 = sum g_z [a*, x]^T, db0 = sum g_z
    rd.G = ngz;
    rd.A = a_star;
    rd.A2 = x_in;
    rd.a_bf = 0;
    rd.off = 0;
    rd.colsum_off = 2 * (int64_t)H * H;
    if ((rc = run("node_dw", s, [&] { return launch_row_dw(rd, W.gbn, s); }))) return rc;
    if (cfg->layernorm &&
        (rc = run("node_dw", s, [&] {
           return launch_colsum2(g->n_rows, H, bf, 0, ngx, g_x_out, m.part, m.slab, s1 + (int64_t)H * H + H,
                                 s1 + (int64_t)H * H + 2 * H, W.gbn, s);
         })))
      return rc;
  } else if ((rc = run("node_bwd", s, [&] { return launch_mlp_bwd(m, W.gbn, s); }))) {
    return rc;
  }
  // the halo sum is symmetric: its adjoint is the same group sum
  if (cfg->halo && (rc = run("halo_adj", s, [&] { return launch_halo(H, d, ga, s); }))) return rc;
  EdgeBwdArgs eb{};
  eb.g = d;
  eb.H = H;
  eb.ln = cfg->layernorm;
  eb.bf = bf;
  eb.am = cfg->aggregate;
  eb.waves = cfg->edge_bwd_waves;
  eb.es = cfg->estate_dtype == MP_BF16;
  eb.P = P;
  eb.Q = Q;
  eb.e_in = e_in;
  eb.g_e_out = g_e_out;
  eb.g_a = ga;
  eb.frag = ws_at(ws, W.fr.edge);
  eb.b2 = p->be2;
  eb.lng = p->ge;
  eb.lnb = p->bge;
  eb.eps = cfg->ln_eps;
  eb.g_e_in = g_e_in;
  eb.g_h = gh;
  eb.g_P = gP;
  eb.part = wsf(ws, W.part_e);
  eb.slab = edge_slab(H);
  if (edge_bwd_split(H)) {
    // wide layers: the adjoint writes the per-edge factors, then the weight
    // gradients are summed from them (same slab layout as the fused kernel)
    eb.gm = ws_at(ws, W.sgm);
    eb.u = ws_at(ws, W.su);
    if ((rc = run("edge_bwd", s, [&] { return launch_edge_bwd_split(eb, W.gbe, s); }))) return rc;
    RowDwArgs rd{};
    rd.n_rows = g->n_edges;
    rd.GW = rd.AW = H;
    rd.bf = bf;
    rd.part = eb.part;
    rd.slab = eb.slab;
    rd.G = gh;  // dW1c = sum g_h e^T
    rd.g_bf = bf;
    rd.A = e_in;
    rd.a_bf = eb.es;
    rd.off = 0;
    rd.colsum_off = -1;
    if ((rc = run("edge_dw", s, [&] { return launch_row_dw(rd, W.gbe, s); }))) return rc;
    rd.G = eb.gm;  // dW2 = sum gm u^T, db2 = sum gm
    rd.A = eb.u;
    rd.a_bf = bf;
    rd.off = (int64_t)H * H;
    rd.colsum_off = 2 * (int64_t)H * H;
    if ((rc = run("edge_dw", s, [&] { return launch_row_dw(rd, W.gbe, s); }))) return rc;
  } else if ((rc = run("edge_bwd", s, [&] { return launch_edge_bwd(eb, W.gbe, s); }))) {
    return rc;
  }
  GqArgs q{};
  q.g = d;
  q.H = H;
  q.bf = bf;
  q.x = x_in;
  q.g_P = gP;
  q.g_h = gh;
  q.frag_abt = ws_at(ws, W.fr.gq);
  q.g_x = g_x_in;
  q.part = wsf(ws, W.part_q);
  q.slab = gq_slab(H);
  q.gq_out = gq_split(H, bf) ? wsf(ws, W.gQ) : nullptr;
  if ((rc = run("gq", s, [&] { return launch_gq(q, W.gbn, s); }))) return rc;
  if (gq_split(H, bf)) {
    // dW1a = sum g_P x^T with db1 = sum g_P, dW1b = sum g_Q x^T, into the
    // slab layout of the fused form
    RowDwArgs rq{};
    rq.n_rows = g->n_rows;
    rq.GW = H;
    rq.AW = H;
    rq.part = q.part;
    rq.slab = q.slab;
    rq.G = gP;
    rq.A = x_in;
    rq.off = 0;
    rq.colsum_off = 2 * (int64_t)H * H;
    if ((rc = run("gq_dw", s, [&] { return launch_row_dw(rq, W.gbn, s); }))) return rc;
    rq.G = q.gq_out;
    rq.off = (int64_t)H * H;
    rq.colsum_off = -1;
    if ((rc = run("gq_dw", s, [&] { return launch_row_dw(rq, W.gbn, s); }))) return rc;
  }
  // weight gradients: fixed-order sums of the workgroup slabs
  ReduceSegs R;
  R.n = 0;
  auto seg = [&](const float* part, int n_slabs, int64_t slab, int64_t off, int rows, int cols, float* dst, int ld,
                 int col0) { R.seg[R.n++] = ReduceSeg{part, n_slabs, slab, off, rows, cols, dst, ld, col0}; };
  const float* pn = wsf(ws, W.part_n);
  const int64_t sn = mlp_slab(H, 2 * H, H);
  seg(pn, W.gbn, sn, 0, H, 2 * H, gr->Wn1, 2 * H, 0);
  seg(pn, W.gbn, sn, 2 * H * H, 1, H, gr->bn1, H, 0);
  seg(pn, W.gbn, sn, 2 * H * H + H, H, H, gr->Wn2, H, 0);
  seg(pn, W.gbn, sn, 3 * H * H + H, 1, H, gr->bn2, H, 0);
  if (cfg->layernorm) {
    seg(pn, W.gbn, sn, 3 * H * H + 2 * H, 1, H, gr->gn, H, 0);
    seg(pn, W.gbn, sn, 3 * H * H + 3 * H, 1, H, gr->bgn, H, 0);
  }
  const float* pe = wsf(ws, W.part_e);
  const int64_t se = edge_slab(H);
  seg(pe, W.gbe, se, 0, H, H, gr->We1, 3 * H, 2 * H);
  seg(pe, W.gbe, se, H * H, H, H, gr->We2, H, 0);
  seg(pe, W.gbe, se, 2 * H * H, 1, H, gr->be2, H, 0);
  if (cfg->layernorm) {
    seg(pe, W.gbe, se, 2 * H * H + H, 1, H, gr->ge, H, 0);
    seg(pe, W.gbe, se, 2 * H * H + 2 * H, 1, H, gr->bge, H, 0);
  }
  const float* pgq = wsf(ws, W.part_q);
  const int64_t sq = gq_slab(H);
  seg(pgq, W.gbn, sq, 0, H, H, gr->We1, 3 * H, 0);
  seg(pgq, W.gbn, sq, H * H, H, H, gr->We1, 3 * H, H);
  seg(pgq, W.gbn, sq, 2 * H * H, 1, H, gr->be1, H, 0);
  return run("wreduce", s, [&] { return launch_wreduce(R, s); });
}

// ------------------------------------------------------------ row MLPs

namespace {

int check_mlp_cfg(const mp_mlp_cfg* c) {
  if (!c) return mp_fail(MP_EINVAL, "mlp config is NULL");
  if (c->H != 32 && c->H != 64 && c->H != 128) return mp_fail(MP_EINVAL, "H must be 32, 64 or 128 (got %d)", c->H);
  if (!((c->n_in >= 1 && c->n_in <= 4) || c->n_in == c->H))
    return mp_fail(MP_EINVAL, "n_in must be 1..4 or H (got %d)", c->n_in);
  if (!((c->n_out >= 1 && c->n_out <= 4) || c->n_out == c->H))
    return mp_fail(MP_EINVAL, "n_out must be 1..4 or H (got %d)", c->n_out);
  if (c->n_in <= 4 && c->n_out <= 4) return mp_fail(MP_EINVAL, "small input and small output together are not supported");
  if (c->layernorm && c->n_out != c->H) return mp_fail(MP_EINVAL, "LayerNorm needs n_out == H");
  if (c->layernorm && !(c->ln_eps > 0.f)) return mp_fail(MP_EINVAL, "ln_eps must be positive");
  if (c->gemm_dtype != MP_F32 && c->gemm_dtype != MP_BF16) return mp_fail(MP_EINVAL, "bad gemm_dtype");
  if (c->out_dtype != MP_F32 && c->out_dtype != MP_BF16) return mp_fail(MP_EINVAL, "bad out_dtype");
  if (c->out_dtype == MP_BF16 && !(c->n_in <= 4 && c->n_out == c->H && c->gemm_dtype == MP_BF16))
    return mp_fail(MP_EINVAL, "a BF16 output needs n_in <= 4, n_out == H and BF16 GEMMs (the edge encoder)");
  return MP_OK;
}

struct MlpWs {
  size_t f0, f1, fr0, fr1, fr1t, fr0t, part, total;
  int grid, gridb;
  MlpWs(const mp_mlp_cfg* c, int64_t n, bool bwd) {
    const bool bf = c->gemm_dtype == MP_BF16;
    f0 = c->n_in > 4 ? frag_bytes(c->H, c->n_in, bf) : 0;
    f1 = c->n_out > 4 ? frag_bytes(c->H, c->H, bf) : 0;
    size_t o = 0;
    fr0 = o; o = align_up(o + f0);
    fr1 = o; o = align_up(o + f1);
    fr1t = o; o = align_up(o + (bwd ? f1 : 0));
    fr0t = o; o = align_up(o + (bwd ? f0 : 0));
    grid = row_grid(n);
    gridb = row_bwd_grid(n);
    part = o;
    if (bwd) o = align_up(o + (size_t)gridb * mlp_slab(c->H, c->n_in, c->n_out) * 4);
    total = std::max<size_t>(o, kAlign);
  }
};

PackJobs mlp_jobs(const mp_mlp_cfg* c, const mp_mlp_params* p, const MlpWs& W, bool bwd) {
  PackJobs J;
  J.n = 0;
  J.bf = c->gemm_dtype == MP_BF16;
  const int H = c->H;
  if (W.f0) add_job(J, H, c->n_in, view(p->W0, c->n_in, 0, 0), W.fr0);
  if (W.f1) add_job(J, H, H, view(p->W1, H, 0, 0), W.fr1);
  if (bwd && W.f1) add_job(J, H, H, view(p->W1, H, 0, 1), W.fr1t);
  if (bwd && W.f0) add_job(J, c->n_in, H, view(p->W0, c->n_in, 0, 1), W.fr0t);
  return J;
}

int check_mlp_params(const mp_mlp_cfg* c, const mp_mlp_params* p) {
  if (!p || !p->W0 || !p->b0 || !p->W1 || !p->b1) return mp_fail(MP_EINVAL, "mlp parameter is NULL");
  if (!aligned16(p->b0) || !aligned16(p->W1) || !aligned16(p->W0) || !aligned16(p->b1))
    return mp_fail(MP_EINVAL, "mlp parameters must be 16-byte aligned");
  if (c->layernorm && (!p->ln_g || !p->ln_b || !aligned16(p->ln_g) || !aligned16(p->ln_b)))
    return mp_fail(MP_EINVAL, "LayerNorm parameter is NULL or unaligned");
  return MP_OK;
}

}  // namespace

extern "C" int mp_mlp_workspace_size(const mp_mlp_cfg* cfg, int64_t n_rows, int backward, size_t* bytes) {
  int rc;
  if ((rc = check_mlp_cfg(cfg))) return rc;
  if (n_rows <= 0 || !bytes) return mp_fail(MP_EINVAL, "mp_mlp_workspace_size: bad n_rows or bytes");
  *bytes = MlpWs(cfg, n_rows, backward != 0).total;
  return MP_OK;
}

extern "C" int mp_mlp_forward(const mp_mlp_cfg* cfg, const mp_mlp_params* p, int64_t n_rows, const float* in,
                              void* out, void* ws, size_t ws_bytes, mp_stream_t stream) {
  int rc;
  if ((rc = check_mlp_cfg(cfg)) || (rc = check_mlp_params(cfg, p))) return rc;
  if (n_rows <= 0 || !in || !out || !ws) return mp_fail(MP_EINVAL, "mp_mlp_forward: bad size or NULL buffer");
  if (!aligned16(in) || !aligned16(out) || !aligned16(ws)) return mp_fail(MP_EINVAL, "mp_mlp_forward: unaligned buffer");
  if (out == (const void*)in) return mp_fail(MP_EINVAL, "mp_mlp_forward: out must not alias in");
  const MlpWs W(cfg, n_rows, false);
  if (ws_bytes < W.total) return mp_fail(MP_ENOMEM, "mp_mlp_forward: workspace %zu < %zu bytes", ws_bytes, W.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = run("pack", s, [&] { return launch_pack(mlp_jobs(cfg, p, W, false), ws, s); }))) return rc;
  MlpFwdArgs m{};
  m.n_rows = n_rows;
  m.src0 = in;
  m.k0 = cfg->n_in;
  m.k1 = 0;
  m.H = cfg->H;
  m.n_out = cfg->n_out;
  m.ln = cfg->layernorm;
  m.bf = cfg->gemm_dtype == MP_BF16;
  m.W0 = p->W0;
  m.b0 = p->b0;
  m.W1 = p->W1;
  m.b1 = p->b1;
  m.lng = p->ln_g;
  m.lnb = p->ln_b;
  m.eps = cfg->ln_eps;
  m.frag0 = ws_at(ws, W.fr0);
  m.frag1 = ws_at(ws, W.fr1);
  m.out = out;
  m.out_bf = cfg->out_dtype == MP_BF16;
  return run("mlp_fwd", s, [&] { return launch_mlp_fwd(m, W.grid, s); });
}

extern "C" int mp_mlp_backward(const mp_mlp_cfg* cfg, const mp_mlp_params* p, int64_t n_rows, const float* in,
                               const void* g_out, float* g_in, const mp_mlp_grads* gr, void* ws, size_t ws_bytes,
                               mp_stream_t stream) {
  int rc;
  if ((rc = check_mlp_cfg(cfg)) || (rc = check_mlp_params(cfg, p))) return rc;
  if (n_rows <= 0 || !in || !g_out || !gr || !ws) return mp_fail(MP_EINVAL, "mp_mlp_backward: bad size or NULL buffer");
  if (!gr->W0 || !gr->b0 || !gr->W1 || !gr->b1 || (cfg->layernorm && (!gr->ln_g || !gr->ln_b)))
    return mp_fail(MP_EINVAL, "mp_mlp_backward: a gradient buffer is NULL");
  if (!aligned16(in) || !aligned16(g_out) || !aligned16(ws) || (g_in && !aligned16(g_in)))
    return mp_fail(MP_EINVAL, "mp_mlp_backward: unaligned buffer");
  if (g_in && cfg->n_in <= 4) return mp_fail(MP_EINVAL, "mp_mlp_backward: no input gradient for n_in <= 4");
  if (g_in && ((const void*)g_in == g_out || (const float*)g_in == in))
    return mp_fail(MP_EINVAL, "mp_mlp_backward: g_in must not alias inputs");
  const MlpWs W(cfg, n_rows, true);
  if (ws_bytes < W.total) return mp_fail(MP_ENOMEM, "mp_mlp_backward: workspace %zu < %zu bytes", ws_bytes, W.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = run("pack", s, [&] { return launch_pack(mlp_jobs(cfg, p, W, true), ws, s); }))) return rc;
  const int H = cfg->H;
  MlpBwdArgs m{};
  m.n_rows = n_rows;
  m.src0 = in;
  m.k0 = cfg->n_in;
  m.k1 = 0;
  m.H = H;
  m.n_out = cfg->n_out;
  m.ln = cfg->layernorm;
  m.bf = cfg->gemm_dtype == MP_BF16;
  m.W0 = p->W0;
  m.b0 = p->b0;
  m.W1 = p->W1;
  m.b1 = p->b1;
  m.lng = p->ln_g;
  m.lnb = p->ln_b;
  m.eps = cfg->ln_eps;
  m.frag0 = ws_at(ws, W.fr0);
  m.frag1 = ws_at(ws, W.fr1);
  m.frag1t = ws_at(ws, W.fr1t);
  m.frag0t = g_in ? ws_at(ws, W.fr0t) : nullptr;
  m.g_out = g_out;
  m.gout_bf = cfg->out_dtype == MP_BF16;
  m.g_src0 = g_in;
  m.part = wsf(ws, W.part);
  m.slab = mlp_slab(H, cfg->n_in, cfg->n_out);
  if ((rc = run("mlp_bwd", s, [&] { return launch_mlp_bwd(m, W.gridb, s); }))) return rc;
  ReduceSegs R;
  R.n = 0;
  const float* pp = wsf(ws, W.part);
  const int kin = cfg->n_in, no = cfg->n_out;
  const int64_t sl = m.slab;
  R.seg[R.n++] = ReduceSeg{pp, W.gridb, sl, 0, H, kin, gr->W0, kin, 0};
  R.seg[R.n++] = ReduceSeg{pp, W.gridb, sl, (int64_t)H * kin, 1, H, gr->b0, H, 0};
  R.seg[R.n++] = ReduceSeg{pp, W.gridb, sl, (int64_t)H * kin + H, no, H, gr->W1, H, 0};
  R.seg[R.n++] = ReduceSeg{pp, W.gridb, sl, (int64_t)H * kin + H + (int64_t)no * H, 1, no, gr->b1, no, 0};
  if (cfg->layernorm) {
    const int64_t o = (int64_t)H * kin + H + (int64_t)no * H + no;
    R.seg[R.n++] = ReduceSeg{pp, W.gridb, sl, o, 1, H, gr->ln_g, H, 0};
    R.seg[R.n++] = ReduceSeg{pp, W.gridb, sl, o + H, 1, H, gr->ln_b, H, 0};
  }
  return run("wreduce", s, [&] { return launch_wreduce(R, s); });
}

// ------------------------------------------------ narrow deep MLPs

namespace {

constexpr int kDeepMaxHidden = 8;

bool deep_width_ok(int H) { return H == 8 || H == 16 || H == 32; }

int check_deep_layer_cfg(const mp_deep_layer_cfg* c) {
  if (!c) return mp_fail(MP_EINVAL, "deep layer config is NULL");
  if (!deep_width_ok(c->H)) return mp_fail(MP_EINVAL, "deep layers: H must be 8, 16 or 32 (got %d)", c->H);
  if (c->n_hidden < 0 || c->n_hidden > kDeepMaxHidden)
    return mp_fail(MP_EINVAL, "n_hidden must be in [0, %d] (got %d)", kDeepMaxHidden, c->n_hidden);
  if (c->layernorm && !(c->ln_eps > 0.f)) return mp_fail(MP_EINVAL, "ln_eps must be positive");
  if (c->aggregate != MP_AGG_STATE && c->aggregate != MP_AGG_MESSAGE)
    return mp_fail(MP_EINVAL, "aggregate must be MP_AGG_STATE or MP_AGG_MESSAGE");
  return MP_OK;
}

// Rows per weight-gradient chunk: at most 2048 chunks, at least 256 rows,
// whole record blocks.
int64_t deep_chunk(int64_t n) {
  int64_t ch = std::max<int64_t>(256, (n + 2047) / 2048);
  return (ch + kRecRows - 1) / kRecRows * kRecRows;
}
int64_t deep_chunks(int64_t n) { return (n + deep_chunk(n) - 1) / deep_chunk(n); }

// One MLP's weight-gradient blocks over its records (K input features in
// columns [0, K) of the record, padded widths km, om).
int deep_outer_mats(OuterArgs& oa, int K, int H, int NH, int O, int ln, int km, int om) {
  auto h = [&](int l) { return km + l * H; };
  auto d = [&](int l) { return km + (NH + 1) * H + l * H; };
  const int dout = km + 2 * (NH + 1) * H, lnr = dout + om;
  auto wh = [&](int l) { return (int64_t)H * K + H + (int64_t)l * (H * H + H); };
  const int64_t wo = wh(NH), bo = wo + (int64_t)O * H, lg = bo + O;
  int n = 0;
  oa.m[n++] = OuterMat{d(0), H, 0, K, 0, (int64_t)H * K};
  for (int l = 1; l <= NH; ++l) oa.m[n++] = OuterMat{d(l), H, h(l - 1), H, wh(l - 1), wh(l - 1) + (int64_t)H * H};
  oa.m[n++] = OuterMat{dout, O, h(NH), H, wo, bo};
  if (ln) oa.m[n++] = OuterMat{lnr, 2 * O, -1, 0, 0, lg};
  return n;
}

// Sum the chunk partials of one MLP into its flat gradient.
int deep_grad_sums(const char* name, const float* rec, int64_t n_rows, int rs, int K, int H, int NH, int O, int ln,
                   int km, int om, float* part, float* g_theta, hipStream_t s) {
  OuterArgs oa{};
  oa.rec = rec;
  oa.n_rows = n_rows;
  oa.rs = rs;
  oa.ch = deep_chunk(n_rows);
  oa.part = part;
  oa.slab = deep_theta_floats(K, H, NH, O, ln);
  const int nm = deep_outer_mats(oa, K, H, NH, O, ln, km, om);
  if (!outer_fits(oa.m, nm)) return mp_fail(MP_EINVAL, "%s: weight blocks too large for one workgroup", name);
  const int64_t nc = deep_chunks(n_rows);
  int rc;
  if ((rc = run(name, s, [&] { return launch_outer_sum(oa, nm, nc, s); }))) return rc;
  ReduceSegs R;
  R.n = 1;
  R.seg[0] = ReduceSeg{part, (int)nc, oa.slab, 0, 1, (int)oa.slab, g_theta, (int)oa.slab, 0};
  return run("wreduce", s, [&] { return launch_wreduce(R, s); });
}

struct DeepLayerWs {
  size_t recN = 0, recE = 0, ga = 0, gxn = 0, gxi = 0, gxj = 0, partN = 0, partE = 0, total = 0;
  int rsN = 0, rsE = 0;
  DeepLayerWs(const mp_deep_layer_cfg* c, const mp_dev_graph* g) {
    const int H = c->H, NH = c->n_hidden, ln = c->layernorm != 0;
    const int64_t N = g->n_rows, E = g->n_edges;
    rsN = deep_rec_floats(H, 2 * H, H, NH, ln);
    rsE = deep_rec_floats(H, 3 * H, H, NH, ln);
    size_t o = 0;
    auto take = [&](size_t& slot, size_t floats) {
      slot = o;
      o = align_up(o + floats * sizeof(float));
    };
    take(recN, (size_t)deep_rec_size(N, rsN));
    take(recE, (size_t)deep_rec_size(E, rsE));
    take(ga, (size_t)N * H);
    take(gxn, (size_t)N * H);
    take(gxi, (size_t)E * H);
    take(gxj, (size_t)E * H);
    take(partN, (size_t)deep_chunks(N) * deep_theta_floats(2 * H, H, NH, H, ln));
    take(partE, (size_t)deep_chunks(E) * deep_theta_floats(3 * H, H, NH, H, ln));
    total = o;
  }
};

int deep_mlp_kind(const mp_deep_mlp_cfg* c, DeepRowKind& kind, int& km, int& om) {
  if (!c) return mp_fail(MP_EINVAL, "deep mlp config is NULL");
  if (!deep_width_ok(c->H)) return mp_fail(MP_EINVAL, "deep MLPs: H must be 8, 16 or 32 (got %d)", c->H);
  if (c->n_hidden < 0 || c->n_hidden > kDeepMaxHidden)
    return mp_fail(MP_EINVAL, "n_hidden must be in [0, %d] (got %d)", kDeepMaxHidden, c->n_hidden);
  if (c->layernorm && (c->n_out != c->H || !(c->ln_eps > 0.f)))
    return mp_fail(MP_EINVAL, "LayerNorm needs n_out == H and a positive ln_eps");
  const int H = c->H;
  if (c->n_in >= 1 && c->n_in <= 4 && c->n_out == H) {
    kind = DeepRowKind::kSmallIn, km = 4, om = H;
  } else if (c->n_in >= 5 && c->n_in <= 8 && c->n_in != H && c->n_out == H) {
    kind = DeepRowKind::kSmallIn8, km = 8, om = H;
  } else if (c->n_in == H && c->n_out >= 1 && c->n_out <= 4) {
    kind = DeepRowKind::kSmallOut, km = H, om = 4;
  } else if (c->n_in == H && c->n_out == H) {
    kind = DeepRowKind::kWide, km = H, om = H;
  } else {
    return mp_fail(MP_EINVAL, "deep MLPs: (n_in, n_out) must be (1..8, H), (H, 1..4) or (H, H); got (%d, %d)",
                   c->n_in, c->n_out);
  }
  return MP_OK;
}

}  // namespace

extern "C" int mp_deep_theta_size(int32_t n_in, int32_t H, int32_t n_hidden, int32_t n_out, int32_t layernorm,
                                  int64_t* floats) {
  if (!floats || n_in <= 0 || H <= 0 || n_hidden < 0 || n_out <= 0)
    return mp_fail(MP_EINVAL, "mp_deep_theta_size: bad argument");
  *floats = deep_theta_floats(n_in, H, n_hidden, n_out, layernorm != 0);
  return MP_OK;
}

extern "C" int mp_deep_layer_workspace_size(const mp_deep_layer_cfg* cfg, const mp_dev_graph* g, int backward,
                                            size_t* bytes) {
  int rc;
  if ((rc = check_deep_layer_cfg(cfg)) || (rc = check_graph(g, false))) return rc;
  if (!bytes) return mp_fail(MP_EINVAL, "bytes is NULL");
  *bytes = backward ? DeepLayerWs(cfg, g).total : 0;
  return MP_OK;
}

extern "C" int mp_deep_layer_forward(const mp_deep_layer_cfg* cfg, const float* theta_edge,
                                     const float* theta_node, const mp_dev_graph* g, const float* x_in,
                                     const float* e_in, float* x_out, float* e_out, float* a_star_out,
                                     mp_stream_t stream) {
  int rc;
  if ((rc = check_deep_layer_cfg(cfg)) || (rc = check_graph(g, false))) return rc;
  if (!theta_edge || !theta_node || !x_in || !e_in || !x_out || !e_out || !a_star_out)
    return mp_fail(MP_EINVAL, "mp_deep_layer_forward: NULL buffer");
  if (!aligned16(x_in) || !aligned16(e_in) || !aligned16(x_out) || !aligned16(e_out) || !aligned16(a_star_out))
    return mp_fail(MP_EINVAL, "mp_deep_layer_forward: buffers must be 16-byte aligned");
  if (x_out == x_in || e_out == e_in || a_star_out == x_in || a_star_out == x_out)
    return mp_fail(MP_EINVAL, "mp_deep_layer_forward: outputs must not alias inputs");
  const int H = cfg->H;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const DevGraph d = dev_graph(g);
  DeepEdgeArgs ea{};
  ea.g = d;
  ea.theta = theta_edge;
  ea.NH = cfg->n_hidden;
  ea.ln = cfg->layernorm != 0;
  ea.am = cfg->aggregate != 0;
  ea.eps = cfg->ln_eps;
  ea.x = x_in;
  ea.e_in = e_in;
  ea.e_out = e_out;
  ea.a_out = a_star_out;
  if ((rc = run("deep_edge_fwd", s, [&] { return launch_deep_edge(ea, H, false, s); }))) return rc;
  if (cfg->halo && (rc = run("halo", s, [&] { return launch_halo(H, d, a_star_out, s); }))) return rc;
  DeepRowArgs na{};
  na.n_rows = g->n_rows;
  na.theta = theta_node;
  na.NH = cfg->n_hidden;
  na.ka = H;
  na.O = H;
  na.ln = cfg->layernorm != 0;
  na.eps = cfg->ln_eps;
  na.src_a = a_star_out;
  na.src_b = x_in;
  na.resid = 1;
  na.out = x_out;
  return run("deep_node_fwd", s, [&] { return launch_deep_row(na, H, DeepRowKind::kNode, false, s); });
}

extern "C" int mp_deep_layer_backward(const mp_deep_layer_cfg* cfg, const float* theta_edge,
                                      const float* theta_node, const mp_dev_graph* g, const float* x_in,
                                      const float* e_in, const float* a_star, const float* g_x_out,
                                      const float* g_e_out, float* g_x_in, float* g_e_in, float* g_theta_edge,
                                      float* g_theta_node, void* ws, size_t ws_bytes, mp_stream_t stream) {
  int rc;
  if ((rc = check_deep_layer_cfg(cfg)) || (rc = check_graph(g, true))) return rc;
  if (!theta_edge || !theta_node || !x_in || !e_in || !a_star || !g_x_out || !g_x_in || !g_e_in ||
      !g_theta_edge || !g_theta_node || !ws)
    return mp_fail(MP_EINVAL, "mp_deep_layer_backward: NULL buffer");
  const void* al[] = {x_in, e_in, a_star, g_x_out, g_x_in, g_e_in, ws};
  for (const void* q : al)
    if (!aligned16(q)) return mp_fail(MP_EINVAL, "mp_deep_layer_backward: buffers must be 16-byte aligned");
  if (g_e_out && !aligned16(g_e_out)) return mp_fail(MP_EINVAL, "mp_deep_layer_backward: g_e_out not aligned");
  if (g_x_in == g_x_out || (const float*)g_e_in == g_e_out || g_x_in == x_in || g_e_in == e_in)
    return mp_fail(MP_EINVAL, "mp_deep_layer_backward: gradient outputs must not alias inputs");
  const DeepLayerWs W(cfg, g);
  if (ws_bytes < W.total)
    return mp_fail(MP_ENOMEM, "mp_deep_layer_backward: workspace %zu < %zu bytes", ws_bytes, W.total);
  const int H = cfg->H, NH = cfg->n_hidden, ln = cfg->layernorm != 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const DevGraph d = dev_graph(g);
  float* ga = wsf(ws, W.ga);
  float* gxn = wsf(ws, W.gxn);
  // node update adjoint: gradient at a* (into ga) and at x (into gxn)
  DeepRowArgs na{};
  na.n_rows = g->n_rows;
  na.theta = theta_node;
  na.NH = NH;
  na.ka = H;
  na.O = H;
  na.ln = ln;
  na.eps = cfg->ln_eps;
  na.src_a = a_star;
  na.src_b = x_in;
  na.resid = 1;
  na.g_out = g_x_out;
  na.g_a = ga;
  na.g_b = gxn;
  na.rec = wsf(ws, W.recN);
  na.rs = W.rsN;
  if ((rc = run("deep_node_bwd", s, [&] { return launch_deep_row(na, H, DeepRowKind::kNode, true, s); }))) return rc;
  if (cfg->halo && (rc = run("halo_adj", s, [&] { return launch_halo(H, d, ga, s); }))) return rc;
  DeepEdgeArgs ea{};
  ea.g = d;
  ea.theta = theta_edge;
  ea.NH = NH;
  ea.ln = ln;
  ea.am = cfg->aggregate != 0;
  ea.eps = cfg->ln_eps;
  ea.x = x_in;
  ea.e_in = e_in;
  ea.g_a = ga;
  ea.g_e_out = g_e_out;
  ea.g_e_in = g_e_in;
  ea.gxi = wsf(ws, W.gxi);
  ea.gxj = wsf(ws, W.gxj);
  ea.rec = wsf(ws, W.recE);
  ea.rs = W.rsE;
  if ((rc = run("deep_edge_bwd", s, [&] { return launch_deep_edge(ea, H, true, s); }))) return rc;
  if ((rc = run("deep_gather", s, [&] { return launch_deep_gather(H, d, gxn, ea.gxi, ea.gxj, g_x_in, s); })))
    return rc;
  if ((rc = deep_grad_sums("deep_node_dw", na.rec, g->n_rows, W.rsN, 2 * H, H, NH, H, ln, 2 * H, H,
                           wsf(ws, W.partN), g_theta_node, s)))
    return rc;
  return deep_grad_sums("deep_edge_dw", ea.rec, g->n_edges, W.rsE, 3 * H, H, NH, H, ln, 3 * H, H,
                        wsf(ws, W.partE), g_theta_edge, s);
}

extern "C" int mp_deep_mlp_workspace_size(const mp_deep_mlp_cfg* cfg, int64_t n_rows, int backward,
                                          size_t* bytes) {
  int rc, km, om;
  DeepRowKind kind;
  if ((rc = deep_mlp_kind(cfg, kind, km, om))) return rc;
  if (n_rows <= 0 || !bytes) return mp_fail(MP_EINVAL, "mp_deep_mlp_workspace_size: bad n_rows or bytes");
  if (!backward) {
    *bytes = 0;
    return MP_OK;
  }
  const int rs = deep_rec_floats(cfg->H, km, om, cfg->n_hidden, cfg->layernorm != 0);
  *bytes = align_up((size_t)deep_rec_size(n_rows, rs) * sizeof(float)) +
           align_up((size_t)deep_chunks(n_rows) *
                    deep_theta_floats(cfg->n_in, cfg->H, cfg->n_hidden, cfg->n_out, cfg->layernorm != 0) *
                    sizeof(float));
  return MP_OK;
}

extern "C" int mp_deep_mlp_forward(const mp_deep_mlp_cfg* cfg, const float* theta, int64_t n_rows,
                                   const float* in, float* out, mp_stream_t stream) {
  int rc, km, om;
  DeepRowKind kind;
  if ((rc = deep_mlp_kind(cfg, kind, km, om))) return rc;
  if (n_rows <= 0 || !theta || !in || !out) return mp_fail(MP_EINVAL, "mp_deep_mlp_forward: bad size or NULL buffer");
  if (!aligned16(in) || !aligned16(out)) return mp_fail(MP_EINVAL, "mp_deep_mlp_forward: unaligned buffer");
  if ((const float*)out == in) return mp_fail(MP_EINVAL, "mp_deep_mlp_forward: out must not alias in");
  DeepRowArgs a{};
  a.n_rows = n_rows;
  a.theta = theta;
  a.NH = cfg->n_hidden;
  a.ka = cfg->n_in;
  a.O = cfg->n_out;
  a.ln = cfg->layernorm != 0;
  a.eps = cfg->ln_eps;
  a.src_a = in;
  a.out = out;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return run("deep_mlp_fwd", s, [&] { return launch_deep_row(a, cfg->H, kind, false, s); });
}

extern "C" int mp_deep_mlp_backward(const mp_deep_mlp_cfg* cfg, const float* theta, int64_t n_rows,
                                    const float* in, const float* g_out, float* g_in, float* g_theta, void* ws,
                                    size_t ws_bytes, mp_stream_t stream) {
  int rc, km, om;
  DeepRowKind kind;
  if ((rc = deep_mlp_kind(cfg, kind, km, om))) return rc;
  if (n_rows <= 0 || !theta || !in || !g_out || !g_theta || !ws)
    return mp_fail(MP_EINVAL, "mp_deep_mlp_backward: bad size or NULL buffer");
  if (!aligned16(in) || !aligned16(g_out) || !aligned16(ws) || (g_in && !aligned16(g_in)))
    return mp_fail(MP_EINVAL, "mp_deep_mlp_backward: unaligned buffer");
  if (g_in && ((const float*)g_in == g_out || (const float*)g_in == in))
    return mp_fail(MP_EINVAL, "mp_deep_mlp_backward: g_in must not alias inputs");
  size_t need = 0;
  mp_deep_mlp_workspace_size(cfg, n_rows, 1, &need);
  if (ws_bytes < need) return mp_fail(MP_ENOMEM, "mp_deep_mlp_backward: workspace %zu < %zu bytes", ws_bytes, need);
  const int H = cfg->H, NH = cfg->n_hidden, ln = cfg->layernorm != 0;
  const int rs = deep_rec_floats(H, km, om, NH, ln);
  DeepRowArgs a{};
  a.n_rows = n_rows;
  a.theta = theta;
  a.NH = NH;
  a.ka = cfg->n_in;
  a.O = cfg->n_out;
  a.ln = ln;
  a.eps = cfg->ln_eps;
  a.src_a = in;
  a.g_out = g_out;
  a.g_a = g_in;
  a.rec = reinterpret_cast<float*>(ws);
  a.rs = rs;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = run("deep_mlp_bwd", s, [&] { return launch_deep_row(a, H, kind, true, s); }))) return rc;
  float* part = wsf(ws, align_up((size_t)deep_rec_size(n_rows, rs) * sizeof(float)));
  return deep_grad_sums("deep_mlp_dw", a.rec, n_rows, rs, cfg->n_in, H, NH, cfg->n_out, ln, km, om, part, g_theta,
                        s);
}

// ------------------------------------------------------- edge inputs, loss

extern "C" int mp_edge_inputs(const mp_dev_graph* g, const double* row_pos, const double* period,
                              const float* row_u, float* e0, mp_stream_t stream) {
  int rc;
  if ((rc = check_graph(g, false))) return rc;
  if (!row_pos || !e0 || (!row_u && !aligned16(e0)))
    return mp_fail(MP_EINVAL, "mp_edge_inputs: NULL or unaligned buffer");
  double L[3] = {0.0, 0.0, 0.0};
  for (int a = 0; period && a < 3; ++a) {
    if (!(period[a] >= 0.0) || std::isinf(period[a]))
      return mp_fail(MP_EINVAL, "mp_edge_inputs: period[%d] must be finite and >= 0", a);
    L[a] = period[a];
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return run("edge_inputs", s, [&] { return launch_edge_inputs(dev_graph(g), row_pos, L, row_u, e0, s); });
}

static int loss_parts(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, (n + 4095) / 4096)); }

extern "C" int mp_consistent_mse_workspace_size(int64_t n_rows, size_t* bytes) {
  if (n_rows <= 0 || !bytes) return mp_fail(MP_EINVAL, "mp_consistent_mse_workspace_size: bad arguments");
  *bytes = align_up((size_t)(2 * loss_parts(n_rows) + 2) * sizeof(double));
  return MP_OK;
}

extern "C" int mp_consistent_mse(int64_t n_rows, int32_t F, const float* Y, const float* T, const uint8_t* node_mult,
                                 float* loss, float* gY, void* ws, size_t ws_bytes, mp_stream_t stream) {
  if (n_rows <= 0 || F <= 0 || F > 64 || !Y || !T || !node_mult || !loss || !ws)
    return mp_fail(MP_EINVAL, "mp_consistent_mse: bad size or NULL buffer");
  size_t need;
  mp_consistent_mse_workspace_size(n_rows, &need);
  if (ws_bytes < need) return mp_fail(MP_ENOMEM, "mp_consistent_mse: workspace %zu < %zu bytes", ws_bytes, need);
  if ((reinterpret_cast<uintptr_t>(ws) & 7) != 0) return mp_fail(MP_EINVAL, "mp_consistent_mse: workspace unaligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return run("loss", s, [&] {
    return launch_loss(n_rows, F, Y, T, node_mult, reinterpret_cast<double*>(ws), loss_parts(n_rows), loss, gY, s);
  });
}
