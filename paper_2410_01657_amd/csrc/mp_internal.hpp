// Internal helpers shared by the library's translation units.
#pragma once
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/mplayer.h"

// Record a thread-local error message (read back by mp_last_error) and
// return the code, so call sites read `return mp_fail(MP_EINVAL, "...")`.
int mp_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

namespace mp {

// Content hash of the graph and halo-plan arrays.  Four independent
// multiply-rotate lanes over 8-byte words (so a core keeps several
// multiplies in flight), the tail packed into one word, the byte count and
// the seed mixed in, and a final avalanche.  Chaining arrays through the
// seed makes the result depend on their order.  Not cryptographic: it
// detects a descriptor paired with the arrays of another graph or plan.
inline uint64_t hash_rotl(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }
inline uint64_t hash_fmix(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}
inline uint64_t hash_bytes(const void* data, size_t n, uint64_t seed) {
  constexpr uint64_t K1 = 0x9e3779b97f4a7c15ull, K2 = 0xc2b2ae3d27d4eb4full;
  const unsigned char* p = static_cast<const unsigned char*>(data);
  uint64_t s0 = seed ^ K1, s1 = seed ^ K2, s2 = hash_rotl(seed, 17) ^ K1, s3 = hash_rotl(seed, 41) ^ K2;
  size_t i = 0;
  for (; i + 32 <= n; i += 32) {
    uint64_t w[4];
    std::memcpy(w, p + i, 32);
    s0 = hash_rotl(s0 ^ (w[0] * K2), 31) * K1;
    s1 = hash_rotl(s1 ^ (w[1] * K2), 31) * K1;
    s2 = hash_rotl(s2 ^ (w[2] * K2), 31) * K1;
    s3 = hash_rotl(s3 ^ (w[3] * K2), 31) * K1;
  }
  uint64_t h = hash_fmix(s0) ^ hash_rotl(hash_fmix(s1), 16) ^ hash_rotl(hash_fmix(s2), 32) ^
               hash_rotl(hash_fmix(s3), 48);
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    std::memcpy(&w, p + i, 8);
    h = hash_rotl(h ^ (w * K2), 27) * K1 + 0x52dce729u;
  }
  if (i < n) {
    uint64_t w = 0;
    std::memcpy(&w, p + i, n - i);
    h = hash_rotl(h ^ (w * K2), 27) * K1 + 0x38495ab5u;
  }
  return hash_fmix(h ^ (uint64_t)n);
}

// Checksum of a graph's device-side arrays (rowptr, recv, col, rev,
// edge_mult), and of a halo plan's arrays (group_ptr, member) chained to the
// checksum of the graph the plan was built on.  `fetch(ptr, bytes)` returns
// a host pointer to an array's content: the array itself on the host, a
// copy read back from the device when a descriptor is verified.
template <class Fetch>
uint64_t graph_checksum_of(int64_t N, int64_t E, const int32_t* rowptr, const int32_t* recv, const int32_t* col,
                           const int32_t* rev, const uint8_t* edge_mult, Fetch fetch) {
  const void* arr[5] = {rowptr, recv, col, rev, edge_mult};
  const size_t bytes[5] = {(size_t)(N + 1) * 4, (size_t)E * 4, (size_t)E * 4, (size_t)E * 4, (size_t)E};
  uint64_t h = hash_fmix(0x6d706772617068ull ^ (uint64_t)N ^ hash_rotl((uint64_t)E, 32));
  for (int k = 0; k < 5; ++k) {
    const void* hp = fetch(arr[k], bytes[k]);
    if (!hp) return 0;
    h = hash_bytes(hp, bytes[k], h);
  }
  return h;
}
template <class Fetch>
uint64_t plan_checksum_of(uint64_t graph_cs, int64_t G, int64_t M, const int32_t* group_ptr, const int32_t* member,
                          Fetch fetch) {
  uint64_t h = hash_fmix(graph_cs ^ 0x6d70706c616eull ^ (uint64_t)G ^ hash_rotl((uint64_t)M, 32));
  const void* gp = fetch(group_ptr, (size_t)(G + 1) * 4);
  if (!gp) return 0;
  h = hash_bytes(gp, (size_t)(G + 1) * 4, h);
  if (M == 0) return hash_bytes(nullptr, 0, h);
  const void* mp = fetch(member, (size_t)M * 4);
  if (!mp) return 0;
  return hash_bytes(mp, (size_t)M * 4, h);
}
inline const void* host_fetch(const void* p, size_t) { return p; }

}  // namespace mp
