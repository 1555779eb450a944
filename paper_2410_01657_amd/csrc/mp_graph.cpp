// Host-side distributed graph generation (Sec. II-A, Figs. 2-4) and the halo
// plan (Eq. 4c-d, Fig. 4).  Deterministic; parallel over sub-graphs.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "mp_internal.hpp"

struct mp_graph {
  int32_t R = 0;
  std::vector<int64_t> row_off, edge_off;  // [R+1]
  std::vector<int64_t> row_gid;            // [N]
  std::vector<int32_t> rowptr;             // [N+1]
  std::vector<int32_t> recv, col, rev;     // [E]
  std::vector<uint8_t> edge_mult;          // [E]
  std::vector<uint8_t> node_mult;          // [N]
  uint64_t checksum = 0;                   // of rowptr, recv, col, rev, edge_mult
  void seal() {
    checksum = mp::graph_checksum_of(row_off.back(), edge_off.back(), rowptr.data(), recv.data(), col.data(),
                                     rev.data(), edge_mult.data(), mp::host_fetch);
  }
};

struct mp_halo_plan {
  int32_t R = 0;
  std::vector<int32_t> group_ptr, member;
  std::vector<int32_t> pair_r, pair_s;
  std::vector<int64_t> pair_ptr;
  std::vector<int32_t> pair_rows_r, pair_rows_s;
  std::vector<int64_t> halo_rows;
  std::vector<int32_t> neighbours;
  uint64_t graph_checksum = 0;  // checksum of the graph the plan was built on
  uint64_t checksum = 0;        // of group_ptr, member, chained to graph_checksum
};

namespace {

// Runs f(0..n-1) on up to 16 threads.  An exception thrown by f (a failed
// allocation) stops the worker that threw it; after every thread has joined
// the first one is rethrown on the calling thread, where the entry point
// turns it into an error code.  If a thread cannot be started, its share of
// the work runs on the calling thread.
template <class F>
void parallel_for(int n, F&& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = std::max(1, std::min<int>(n, std::min<unsigned>(hw ? hw : 1, 16u)));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::mutex mu;
  std::exception_ptr first;
  auto work = [&](int t) {
    try {
      for (int i = t; i < n; i += nt) f(i);
    } catch (...) {
      std::lock_guard<std::mutex> lk(mu);
      if (!first) first = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  int started = 0;
  try {
    th.reserve(nt);
    for (; started < nt; ++started) th.emplace_back(work, started);
  } catch (...) {
  }
  for (int t = started; t < nt; ++t) work(t);
  for (auto& x : th) x.join();
  if (first) std::rethrow_exception(first);
}

struct SubGraphBuild {
  std::vector<int64_t> gid;      // rows, ascending
  std::vector<uint64_t> edges;   // (recv << 32) | send, local, sorted unique
};

}  // namespace

extern "C" int mp_hex_links(int32_t P, int32_t* links, int32_t* n_links) {
  if (P < 1 || P > 32 || !n_links) return mp_fail(MP_EINVAL, "mp_hex_links: need 1 <= P <= 32 and n_links");
  const int q = P + 1;
  int32_t n = 0;
  for (int c = 0; c < q; ++c)
    for (int b = 0; b < q; ++b)
      for (int a = 0; a < q; ++a) {
        const int i = a + q * (b + q * c);
        const int nb[3] = {a + 1 < q ? i + 1 : -1, b + 1 < q ? i + q : -1, c + 1 < q ? i + q * q : -1};
        for (int t = 0; t < 3; ++t)
          if (nb[t] >= 0) {
            if (links) {
              links[2 * n] = i;
              links[2 * n + 1] = nb[t];
            }
            ++n;
          }
      }
  *n_links = n;
  return MP_OK;
}

extern "C" int graph_partition(int64_t n_elem, int32_t npe, const int64_t* elem_gid,
                               int32_t n_links, const int32_t* links,
                               const int32_t* elem_part, int32_t R, mp_graph** out) {
  if (!out) return mp_fail(MP_EINVAL, "graph_partition: out is NULL");
  *out = nullptr;
  if (n_elem <= 0 || npe <= 0 || n_links <= 0 || R <= 0 || R > 65535)
    return mp_fail(MP_EINVAL, "graph_partition: need n_elem, npe, n_links > 0 and 0 < R <= 65535");
  if (!elem_gid || !links || !elem_part) return mp_fail(MP_EINVAL, "graph_partition: NULL input array");
  for (int32_t l = 0; l < n_links; ++l) {
    const int32_t a = links[2 * l], b = links[2 * l + 1];
    if (a < 0 || b < 0 || a >= npe || b >= npe || a == b)
      return mp_fail(MP_EINVAL, "graph_partition: link %d = (%d, %d) is out of range or a self-link", l, a, b);
  }
  int64_t max_gid = -1;
  for (int64_t k = 0; k < n_elem * npe; ++k) {
    if (elem_gid[k] < 0) return mp_fail(MP_EINVAL, "graph_partition: negative global id at %lld", (long long)k);
    max_gid = std::max(max_gid, elem_gid[k]);
  }
  const int64_t n_gid = max_gid + 1;
  if (n_gid >= (int64_t(1) << 31)) return mp_fail(MP_EINVAL, "graph_partition: more than 2^31 global ids");
  std::vector<std::vector<int64_t>> elems(R);
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t p = elem_part[e];
    if (p < 0 || p >= R) return mp_fail(MP_EINVAL, "graph_partition: element %lld has part %d outside [0, %d)", (long long)e, p, R);
    elems[p].push_back(e);
  }
  for (int r = 0; r < R; ++r)
    if (elems[r].empty()) return mp_fail(MP_EINVAL, "graph_partition: sub-graph %d has no element", r);

  std::unique_ptr<mp_graph> G;
  try {
    G.reset(new mp_graph());
    std::vector<SubGraphBuild> sub(R);
    std::vector<int> self_loop(R, 0);
    // rows: distinct global ids of each sub-graph's points (Fig. 3c collapse);
    // edges: distinct local (receiver, sender) pairs of each element link
    parallel_for(R, [&](int r) {
      SubGraphBuild& S = sub[r];
      const auto& el = elems[r];
      S.gid.reserve(el.size() * npe);
      for (int64_t e : el)
        for (int32_t k = 0; k < npe; ++k) S.gid.push_back(elem_gid[e * npe + k]);
      std::sort(S.gid.begin(), S.gid.end());
      S.gid.erase(std::unique(S.gid.begin(), S.gid.end()), S.gid.end());
      std::vector<uint32_t> loc(npe);
      S.edges.reserve(el.size() * n_links * 2);
      for (int64_t e : el) {
        for (int32_t k = 0; k < npe; ++k)
          loc[k] = (uint32_t)(std::lower_bound(S.gid.begin(), S.gid.end(), elem_gid[e * npe + k]) - S.gid.begin());
        for (int32_t l = 0; l < n_links; ++l) {
          const uint32_t a = loc[links[2 * l]], b = loc[links[2 * l + 1]];
          if (a == b) {
            self_loop[r] = 1;
            continue;
          }
          S.edges.push_back((uint64_t(a) << 32) | b);
          S.edges.push_back((uint64_t(b) << 32) | a);
        }
      }
      std::sort(S.edges.begin(), S.edges.end());
      S.edges.erase(std::unique(S.edges.begin(), S.edges.end()), S.edges.end());
    });
    for (int r = 0; r < R; ++r)
      if (self_loop[r]) return mp_fail(MP_EINVAL, "graph_partition: an element link joins a global id to itself (sub-graph %d)", r);

    // node degree d_i: number of sub-graphs holding the global id
    std::vector<uint8_t> ncount(n_gid, 0);
    for (int r = 0; r < R; ++r)
      for (int64_t g : sub[r].gid) {
        if (ncount[g] == 255) return mp_fail(MP_EINVAL, "graph_partition: a node is held by more than 255 sub-graphs");
        ++ncount[g];
      }
    // edge degree d_ij: number of sub-graphs holding the link.  Only links
    // whose two end points are both shared can be held more than once.
    std::vector<std::vector<uint64_t>> cand(R);
    parallel_for(R, [&](int r) {
      const SubGraphBuild& S = sub[r];
      for (uint64_t k : S.edges) {
        const int64_t gi = S.gid[k >> 32], gj = S.gid[k & 0xffffffffu];
        if (gi < gj && ncount[gi] > 1 && ncount[gj] > 1) cand[r].push_back(uint64_t(gi) * uint64_t(n_gid) + uint64_t(gj));
      }
    });
    std::vector<uint64_t> allc;
    for (int r = 0; r < R; ++r) allc.insert(allc.end(), cand[r].begin(), cand[r].end());
    std::sort(allc.begin(), allc.end());

    int64_t N = 0, E = 0;
    G->R = R;
    G->row_off.assign(R + 1, 0);
    G->edge_off.assign(R + 1, 0);
    for (int r = 0; r < R; ++r) {
      G->row_off[r + 1] = G->row_off[r] + (int64_t)sub[r].gid.size();
      G->edge_off[r + 1] = G->edge_off[r] + (int64_t)sub[r].edges.size();
    }
    N = G->row_off[R];
    E = G->edge_off[R];
    if (N >= (int64_t(1) << 31) || E >= (int64_t(1) << 31))
      return mp_fail(MP_EINVAL, "graph_partition: more than 2^31-1 rows or edges");
    G->row_gid.resize(N);
    G->node_mult.resize(N);
    G->rowptr.resize(N + 1);
    G->recv.resize(E);
    G->col.resize(E);
    G->rev.resize(E);
    G->edge_mult.resize(E);
    int bad_mult = 0;
    parallel_for(R, [&](int r) {
      const SubGraphBuild& S = sub[r];
      const int64_t r0 = G->row_off[r], e0 = G->edge_off[r];
      const int64_t n = (int64_t)S.gid.size(), ne = (int64_t)S.edges.size();
      for (int64_t i = 0; i < n; ++i) {
        G->row_gid[r0 + i] = S.gid[i];
        G->node_mult[r0 + i] = ncount[S.gid[i]];
      }
      int64_t k = 0;
      for (int64_t i = 0; i < n; ++i) {
        G->rowptr[r0 + i] = (int32_t)(e0 + k);
        while (k < ne && (int64_t)(S.edges[k] >> 32) == i) ++k;
      }
      if (r == R - 1) G->rowptr[N] = (int32_t)E;
      for (int64_t t = 0; t < ne; ++t) {
        const uint32_t i = uint32_t(S.edges[t] >> 32), j = uint32_t(S.edges[t] & 0xffffffffu);
        G->recv[e0 + t] = (int32_t)(r0 + i);
        G->col[e0 + t] = (int32_t)(r0 + j);
        // reverse edge j -> i sits in row j, found by its sender i
        const uint64_t key = (uint64_t(j) << 32) | i;
        const int64_t pos = std::lower_bound(S.edges.begin(), S.edges.end(), key) - S.edges.begin();
        G->rev[e0 + t] = (int32_t)(e0 + pos);
        int64_t gi = S.gid[i], gj = S.gid[j];
        if (gi > gj) std::swap(gi, gj);
        int m = 1;
        if (ncount[gi] > 1 && ncount[gj] > 1) {
          const uint64_t ck = uint64_t(gi) * uint64_t(n_gid) + uint64_t(gj);
          auto lo = std::lower_bound(allc.begin(), allc.end(), ck);
          auto hi = std::upper_bound(lo, allc.end(), ck);
          m = (int)(hi - lo);
          if (m < 1 || m > 255) bad_mult = 1;
        }
        G->edge_mult[e0 + t] = (uint8_t)std::max(1, std::min(m, 255));
      }
    });
    if (bad_mult) return mp_fail(MP_EINVAL, "graph_partition: edge degree outside [1, 255]");
    G->seal();
  } catch (const std::bad_alloc&) {
    return mp_fail(MP_ENOMEM, "graph_partition: host allocation failed");
  } catch (...) {
    return mp_fail(MP_ENOMEM, "graph_partition: host resources (memory or threads) exhausted");
  }
  *out = G.release();
  return MP_OK;
}

namespace {

// Reverse Cuthill-McKee order of one sub-graph (n rows, CSR rowptr/col with
// local indices): breadth-first levels from a pseudo-peripheral row of
// least degree, neighbours taken in ascending degree, the whole order
// reversed.  ord[new] = old.  Ties go to the lower index, so the order is a
// function of the graph alone.
std::vector<int32_t> rcm_order(int32_t n, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col) {
  auto deg = [&](int32_t i) { return rowptr[i + 1] - rowptr[i]; };
  std::vector<int32_t> ord;
  ord.reserve(n);
  std::vector<int32_t> level(n, -1), nb;
  std::vector<char> done(n, 0);
  // last level of a breadth-first sweep from s over s's component (level
  // marks are reset afterwards)
  auto far_row = [&](int32_t s) {
    std::vector<int32_t> q{s};
    level[s] = 0;
    for (size_t h = 0; h < q.size(); ++h)
      for (int32_t k = rowptr[q[h]]; k < rowptr[q[h] + 1]; ++k)
        if (level[col[k]] < 0) {
          level[col[k]] = level[q[h]] + 1;
          q.push_back(col[k]);
        }
    int32_t best = q.back();
    for (int32_t v : q)
      if (level[v] == level[q.back()] && (deg(v) < deg(best) || (deg(v) == deg(best) && v < best))) best = v;
    const int32_t depth = level[q.back()];
    for (int32_t v : q) level[v] = -1;
    return std::make_pair(best, depth);
  };
  for (int32_t s0 = 0; s0 < n; ++s0) {
    if (done[s0]) continue;
    // start: the least-degree row of the component, moved to the far end
    // of its sweeps while that lengthens them (two sweeps at most)
    int32_t s = s0;
    {
      std::vector<int32_t> q{s0};
      level[s0] = 0;
      for (size_t h = 0; h < q.size(); ++h)
        for (int32_t k = rowptr[q[h]]; k < rowptr[q[h] + 1]; ++k)
          if (level[col[k]] < 0) {
            level[col[k]] = 0;
            q.push_back(col[k]);
          }
      for (int32_t v : q) {
        if (deg(v) < deg(s) || (deg(v) == deg(s) && v < s)) s = v;
        level[v] = -1;
      }
    }
    auto fr = far_row(s);
    for (int it = 0; it < 2; ++it) {
      auto nx = far_row(fr.first);
      if (nx.second <= fr.second) break;
      s = fr.first;
      fr = nx;
    }
    const size_t base = ord.size();
    ord.push_back(s);
    done[s] = 1;
    for (size_t h = base; h < ord.size(); ++h) {
      const int32_t v = ord[h];
      nb.clear();
      for (int32_t k = rowptr[v]; k < rowptr[v + 1]; ++k)
        if (!done[col[k]]) {
          done[col[k]] = 1;
          nb.push_back(col[k]);
        }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; });
      ord.insert(ord.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(ord.begin(), ord.end());
  return ord;
}

}  // namespace

extern "C" int graph_order_rows(mp_graph* g) {
  if (!g) return mp_fail(MP_EINVAL, "graph_order_rows: graph is NULL");
  try {
    const int R = g->R;
    mp_graph& G = *g;
    parallel_for(R, [&](int r) {
      const int64_t r0 = G.row_off[r], e0 = G.edge_off[r];
      const int32_t n = (int32_t)(G.row_off[r + 1] - r0);
      const int64_t ne = G.edge_off[r + 1] - e0;
      std::vector<int32_t> rp(n + 1), cl(ne);
      for (int32_t i = 0; i <= n; ++i) rp[i] = (int32_t)(G.rowptr[r0 + i] - e0);
      for (int64_t k = 0; k < ne; ++k) cl[k] = (int32_t)(G.col[e0 + k] - r0);
      const std::vector<int32_t> ord = rcm_order(n, rp, cl);
      std::vector<int32_t> inv(n);
      for (int32_t i = 0; i < n; ++i) inv[ord[i]] = i;
      std::vector<int64_t> gid(n);
      std::vector<uint8_t> nm(n), em(ne);
      std::vector<int32_t> nrp(n + 1), ncl(ne);
      std::vector<std::pair<int32_t, uint8_t>> row;
      int64_t k = 0;
      for (int32_t i = 0; i < n; ++i) {
        const int32_t o = ord[i];
        gid[i] = G.row_gid[r0 + o];
        nm[i] = G.node_mult[r0 + o];
        nrp[i] = (int32_t)k;
        row.clear();
        for (int32_t t = rp[o]; t < rp[o + 1]; ++t) row.emplace_back(inv[cl[t]], G.edge_mult[e0 + t]);
        std::sort(row.begin(), row.end());
        for (const auto& x : row) {
          ncl[k] = x.first;
          em[k] = x.second;
          ++k;
        }
      }
      nrp[n] = (int32_t)k;
      for (int32_t i = 0; i < n; ++i) {
        G.row_gid[r0 + i] = gid[i];
        G.node_mult[r0 + i] = nm[i];
        G.rowptr[r0 + i] = (int32_t)(e0 + nrp[i]);
        for (int32_t t = nrp[i]; t < nrp[i + 1]; ++t) {
          G.recv[e0 + t] = (int32_t)(r0 + i);
          G.col[e0 + t] = (int32_t)(r0 + ncl[t]);
          G.edge_mult[e0 + t] = em[t];
          // reverse edge: in the sender's row, found by its sender i
          const int32_t j = ncl[t];
          const int32_t pos = (int32_t)(std::lower_bound(ncl.begin() + nrp[j], ncl.begin() + nrp[j + 1], i) -
                                        ncl.begin());
          G.rev[e0 + t] = (int32_t)(e0 + pos);
        }
      }
    });
  } catch (const std::bad_alloc&) {
    g->seal();
    return mp_fail(MP_ENOMEM, "graph_order_rows: host allocation failed");
  } catch (...) {
    g->seal();
    return mp_fail(MP_ENOMEM, "graph_order_rows: host resources (memory or threads) exhausted");
  }
  g->seal();
  return MP_OK;
}

extern "C" int mp_graph_sizes(const mp_graph* g, int64_t* n_rows, int64_t* n_edges, int32_t* R) {
  if (!g) return mp_fail(MP_EINVAL, "mp_graph_sizes: graph is NULL");
  if (n_rows) *n_rows = g->row_off.back();
  if (n_edges) *n_edges = g->edge_off.back();
  if (R) *R = g->R;
  return MP_OK;
}

template <class T>
static void copy_out(T* dst, const std::vector<T>& src) {
  if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(T));
}

extern "C" int mp_graph_export(const mp_graph* g, int64_t* row_off, int64_t* edge_off,
                               int64_t* row_gid, int32_t* rowptr, int32_t* recv, int32_t* col,
                               int32_t* rev, uint8_t* edge_mult, uint8_t* node_mult) {
  if (!g) return mp_fail(MP_EINVAL, "mp_graph_export: graph is NULL");
  copy_out(row_off, g->row_off);
  copy_out(edge_off, g->edge_off);
  copy_out(row_gid, g->row_gid);
  copy_out(rowptr, g->rowptr);
  copy_out(recv, g->recv);
  copy_out(col, g->col);
  copy_out(rev, g->rev);
  copy_out(edge_mult, g->edge_mult);
  copy_out(node_mult, g->node_mult);
  return MP_OK;
}

extern "C" int mp_graph_checksum(const mp_graph* g, uint64_t* checksum) {
  if (!g || !checksum) return mp_fail(MP_EINVAL, "mp_graph_checksum: NULL argument");
  *checksum = g->checksum;
  return MP_OK;
}

extern "C" int mp_graph_destroy(mp_graph* g) {
  delete g;
  return MP_OK;
}

extern "C" int halo_plan_build(const mp_graph* g, mp_halo_plan** out) {
  if (!out) return mp_fail(MP_EINVAL, "halo_plan_build: out is NULL");
  *out = nullptr;
  if (!g) return mp_fail(MP_EINVAL, "halo_plan_build: graph is NULL");
  std::unique_ptr<mp_halo_plan> P;
  try {
    P.reset(new mp_halo_plan());
    const int64_t N = g->row_off.back();
    const int R = g->R;
    P->R = R;
    // (gid, row) of every row held by two or more sub-graphs; rows ascend
    // within a gid because sub-graphs are concatenated in r order
    std::vector<std::pair<int64_t, int32_t>> sh;
    for (int64_t i = 0; i < N; ++i)
      if (g->node_mult[i] > 1) sh.emplace_back(g->row_gid[i], (int32_t)i);
    std::sort(sh.begin(), sh.end());
    std::vector<int32_t> row_part(N);
    for (int r = 0; r < R; ++r)
      for (int64_t i = g->row_off[r]; i < g->row_off[r + 1]; ++i) row_part[i] = r;
    P->group_ptr.push_back(0);
    struct PairEntry {
      int32_t r, s;
      int64_t gid;
      int32_t rr, rs;
      bool operator<(const PairEntry& o) const {
        if (r != o.r) return r < o.r;
        if (s != o.s) return s < o.s;
        return gid < o.gid;
      }
    };
    std::vector<PairEntry> pe;
    P->halo_rows.assign(R, 0);
    size_t a = 0;
    while (a < sh.size()) {
      size_t b = a;
      while (b < sh.size() && sh[b].first == sh[a].first) ++b;
      if (b - a < 2) return mp_fail(MP_EPLAN, "halo_plan_build: shared id with a single copy");
      for (size_t t = a; t < b; ++t) P->member.push_back(sh[t].second);
      P->group_ptr.push_back((int32_t)P->member.size());
      for (size_t t = a; t < b; ++t) {
        const int32_t r = row_part[sh[t].second];
        P->halo_rows[r] += (int64_t)(b - a - 1);
        for (size_t u = a; u < b; ++u)
          if (u != t) {
            const int32_t s = row_part[sh[u].second];
            pe.push_back({r, s, sh[t].first, sh[t].second, sh[u].second});
          }
      }
      a = b;
    }
    std::sort(pe.begin(), pe.end());
    size_t c = 0;
    P->pair_ptr.push_back(0);
    while (c < pe.size()) {
      size_t d = c;
      while (d < pe.size() && pe[d].r == pe[c].r && pe[d].s == pe[c].s) {
        P->pair_rows_r.push_back(pe[d].rr);
        P->pair_rows_s.push_back(pe[d].rs);
        ++d;
      }
      P->pair_r.push_back(pe[c].r);
      P->pair_s.push_back(pe[c].s);
      P->pair_ptr.push_back((int64_t)P->pair_rows_r.size());
      c = d;
    }
    // pairs are sorted by (r, s): each listed pair is one neighbour of r
    P->neighbours.assign(R, 0);
    for (int32_t r : P->pair_r) ++P->neighbours[r];
    P->graph_checksum = g->checksum;
    P->checksum = mp::plan_checksum_of(g->checksum, (int64_t)P->group_ptr.size() - 1, (int64_t)P->member.size(),
                                       P->group_ptr.data(), P->member.data(), mp::host_fetch);
  } catch (...) {
    return mp_fail(MP_ENOMEM, "halo_plan_build: host allocation failed");
  }
  *out = P.release();
  return MP_OK;
}

extern "C" int mp_halo_plan_sizes(const mp_halo_plan* p, int64_t* n_groups, int64_t* n_members,
                                  int64_t* n_pairs, int64_t* n_pair_rows) {
  if (!p) return mp_fail(MP_EINVAL, "mp_halo_plan_sizes: plan is NULL");
  if (n_groups) *n_groups = (int64_t)p->group_ptr.size() - 1;
  if (n_members) *n_members = (int64_t)p->member.size();
  if (n_pairs) *n_pairs = (int64_t)p->pair_r.size();
  if (n_pair_rows) *n_pair_rows = (int64_t)p->pair_rows_r.size();
  return MP_OK;
}

extern "C" int mp_halo_plan_export(const mp_halo_plan* p, int32_t* group_ptr, int32_t* member,
                                   int32_t* pair_r, int32_t* pair_s, int64_t* pair_ptr,
                                   int32_t* pair_rows_r, int32_t* pair_rows_s,
                                   int64_t* halo_rows, int32_t* neighbours) {
  if (!p) return mp_fail(MP_EINVAL, "mp_halo_plan_export: plan is NULL");
  copy_out(group_ptr, p->group_ptr);
  copy_out(member, p->member);
  copy_out(pair_r, p->pair_r);
  copy_out(pair_s, p->pair_s);
  copy_out(pair_ptr, p->pair_ptr);
  copy_out(pair_rows_r, p->pair_rows_r);
  copy_out(pair_rows_s, p->pair_rows_s);
  copy_out(halo_rows, p->halo_rows);
  copy_out(neighbours, p->neighbours);
  return MP_OK;
}

extern "C" int mp_halo_plan_checksum(const mp_halo_plan* p, uint64_t* checksum, uint64_t* graph_checksum) {
  if (!p || !checksum || !graph_checksum) return mp_fail(MP_EINVAL, "mp_halo_plan_checksum: NULL argument");
  *checksum = p->checksum;
  *graph_checksum = p->graph_checksum;
  return MP_OK;
}

extern "C" int mp_halo_plan_destroy(mp_halo_plan* p) {
  delete p;
  return MP_OK;
}
