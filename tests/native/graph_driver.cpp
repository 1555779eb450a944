// Host-only driver for the graph builder (graph_partition, graph_order_rows,
// halo_plan_build), built with g++ from the library's own mp_graph.cpp under
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_graph_sanitize.py.
//
// Input file (little-endian): int64 n_elem, int32 npe, int32 n_links,
// int32 R, int32 order (1: reverse Cuthill-McKee rows); then
// elem_gid[n_elem*npe] int64, links[n_links*2] int32, elem_part[n_elem] int32.
// Output file: every exported array of the graph and its halo plan, in the
// order of mp_graph_export / mp_halo_plan_export, each preceded by its byte
// count (int64), then the three checksums.  Exit status: 0, or the error
// code of the first failing call (its message on stderr).
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/mplayer.h"

// The library defines mp_fail beside its device code; the host-only build
// needs its own.
int mp_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vfprintf(stderr, fmt, ap);
  va_end(ap);
  std::fputc('\n', stderr);
  return code;
}

template <class T>
static bool rd(std::FILE* f, T* p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}
template <class T>
static void wr(std::FILE* f, const std::vector<T>& v) {
  const int64_t bytes = (int64_t)(v.size() * sizeof(T));
  std::fwrite(&bytes, sizeof bytes, 1, f);
  if (!v.empty()) std::fwrite(v.data(), sizeof(T), v.size(), f);
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  std::FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t n_elem = 0;
  int32_t npe = 0, n_links = 0, R = 0, order = 0;
  if (!rd(in, &n_elem, 1) || !rd(in, &npe, 1) || !rd(in, &n_links, 1) || !rd(in, &R, 1) || !rd(in, &order, 1))
    return 2;
  std::vector<int64_t> gid((size_t)(n_elem * npe));
  std::vector<int32_t> links((size_t)n_links * 2), part((size_t)n_elem);
  if (!rd(in, gid.data(), gid.size()) || !rd(in, links.data(), links.size()) || !rd(in, part.data(), part.size()))
    return 2;
  std::fclose(in);

  mp_graph* g = nullptr;
  int rc = graph_partition(n_elem, npe, gid.data(), n_links, links.data(), part.data(), R, &g);
  if (rc) return rc;
  if (order && (rc = graph_order_rows(g))) return rc;
  int64_t N = 0, E = 0;
  int32_t RR = 0;
  if ((rc = mp_graph_sizes(g, &N, &E, &RR))) return rc;
  std::vector<int64_t> row_off(RR + 1), edge_off(RR + 1), row_gid(N);
  std::vector<int32_t> rowptr(N + 1), recv(E), col(E), rev(E);
  std::vector<uint8_t> emult(E), nmult(N);
  if ((rc = mp_graph_export(g, row_off.data(), edge_off.data(), row_gid.data(), rowptr.data(), recv.data(),
                            col.data(), rev.data(), emult.data(), nmult.data())))
    return rc;
  uint64_t gcs = 0;
  if ((rc = mp_graph_checksum(g, &gcs))) return rc;
  mp_halo_plan* h = nullptr;
  if ((rc = halo_plan_build(g, &h))) return rc;
  int64_t G = 0, M = 0, NP = 0, NPR = 0;
  if ((rc = mp_halo_plan_sizes(h, &G, &M, &NP, &NPR))) return rc;
  std::vector<int32_t> gptr(G + 1), member(M), pr(NP), ps(NP), rows_r(NPR), rows_s(NPR), nb(RR);
  std::vector<int64_t> pptr(NP + 1), halo_rows(RR);
  if ((rc = mp_halo_plan_export(h, gptr.data(), member.data(), pr.data(), ps.data(), pptr.data(), rows_r.data(),
                                rows_s.data(), halo_rows.data(), nb.data())))
    return rc;
  uint64_t pcs = 0, pgcs = 0;
  if ((rc = mp_halo_plan_checksum(h, &pcs, &pgcs))) return rc;

  std::FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  wr(out, row_off); wr(out, edge_off); wr(out, row_gid); wr(out, rowptr); wr(out, recv); wr(out, col);
  wr(out, rev); wr(out, emult); wr(out, nmult);
  wr(out, gptr); wr(out, member); wr(out, pr); wr(out, ps); wr(out, pptr); wr(out, rows_r); wr(out, rows_s);
  wr(out, halo_rows); wr(out, nb);
  wr(out, std::vector<uint64_t>{gcs, pcs, pgcs});
  std::fclose(out);
  mp_halo_plan_destroy(h);
  mp_graph_destroy(g);
  return 0;
}
