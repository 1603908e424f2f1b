// Serial CPU oracle for mesh re-indexing with duplicate- and unused-vertex
// removal (Wald, "GPGPU-Parallel Re-indexing of Triangle Meshes with
// Duplicate-Vertex and Unused-Vertex Removal").
//
// TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
// definition that the GPU path is checked against. Only the tests, the smoke
// entry point and the benchmark's CPU-baseline leg may load it. It shares no
// code, header, table or helper with the HIP library.
//
// What it computes (Section 1's std::map re-mesher, with the output order and
// tie rule of the parallel method of Section 2):
//   * key(i): vertex record i read as little-endian uint32 words w0..w{K-1};
//     two vertices are duplicates iff all words are equal (bitwise equality,
//     Section 2: "exact duplicates"); keys are ordered lexicographically with
//     w0 most significant, words compared unsigned (the "obvious ordering"
//     the method sorts by, Section 2 Step 2).
//   * the representative of a set of duplicates is the one with the smallest
//     original id (any copy is allowed by Section 2 Step 2; a stable sort of
//     (key, original id) yields the first one).
//   * a value is used iff any of its copies is referenced by an index entry
//     (Section 2 Step 1 turns unused vertices into duplicates so that they
//     disappear; only referenced values survive).
//   * output vertices are the used values in ascending key order (Section 2
//     Step 3: the compacted array follows the sorted array), new ids are
//     their positions, indices are remapped through old -> new (Section 2
//     Step 4), and vertices whose value is not used map to -1.
//
// Parity: pinned by the tests against the paper's worked example (Section 2,
// "Checking our Example"), a paper-order re-enactment of Steps 1-4, an O(n^2)
// brute force, numpy.unique, and closed-form vertex counts.
#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

namespace {

constexpr int kMaxWords = 16;  // records of 4..64 bytes

using Key = std::array<uint32_t, kMaxWords>;  // unused tail words stay 0

Key key_of(const uint32_t* vtx, int64_t i, int32_t words) {
  Key k{};
  for (int32_t w = 0; w < words; ++w) k[w] = vtx[i * words + w];
  return k;  // std::array's operator< is lexicographic over uint32_t: w0 first, unsigned
}

}  // namespace

extern "C" {

// Status codes match the library's public ones for the cases the oracle has.
enum { ORACLE_OK = 0, ORACLE_INVALID_ARGUMENT = 1, ORACLE_INDEX_OUT_OF_RANGE = 3 };

// vtx       [num_vtx * words] uint32, record i at vtx[i*words .. i*words+words)
// idx       [num_idx] int32 (all index entries of all elements, flattened)
// out_vtx   capacity num_vtx * words; out_idx [num_idx]; old2new [num_vtx];
// new2old   capacity num_vtx; *out_num_vtx receives U.
// On an out-of-range index, *bad_pos receives the first offending position.
int oracle_reindex(const uint32_t* vtx, int64_t num_vtx, int32_t words,
                   const int32_t* idx, int64_t num_idx,
                   uint32_t* out_vtx, int32_t* out_idx, int32_t* old2new,
                   int32_t* new2old, int64_t* out_num_vtx, int64_t* bad_pos) {
  if (words < 1 || words > kMaxWords || num_vtx < 0 || num_idx < 0 ||
      num_vtx > INT32_MAX)
    return ORACLE_INVALID_ARGUMENT;
  *out_num_vtx = 0;
  *bad_pos = -1;
  for (int64_t k = 0; k < num_idx; ++k) {
    if (idx[k] < 0 || idx[k] >= num_vtx) {
      *bad_pos = k;
      return ORACLE_INDEX_OUT_OF_RANGE;
    }
  }

  // One entry per distinct value, keyed (and therefore iterated) in key order.
  struct Group {
    int32_t rep;     // smallest original id holding this value
    bool used;       // referenced through any of its copies
    int32_t new_id;  // position among used values, -1 if unused
  };
  std::map<Key, Group> groups;

  // 1. representative: first occurrence in original-id order.
  for (int64_t i = 0; i < num_vtx; ++i) groups.emplace(key_of(vtx, i, words), Group{(int32_t)i, false, -1});

  // 2. a value is used iff any copy of it is referenced.
  for (int64_t k = 0; k < num_idx; ++k) groups.at(key_of(vtx, idx[k], words)).used = true;

  // 3. used values in ascending key order get consecutive new ids.
  int64_t u = 0;
  for (auto& kv : groups) {
    Group& g = kv.second;
    if (!g.used) continue;
    g.new_id = (int32_t)u;
    std::memcpy(out_vtx + u * words, vtx + (int64_t)g.rep * words, sizeof(uint32_t) * words);
    new2old[u] = g.rep;
    ++u;
  }

  // 4. old -> new for every original vertex (-1: its value is not used).
  for (int64_t i = 0; i < num_vtx; ++i) old2new[i] = groups.at(key_of(vtx, i, words)).new_id;

  // 5. remap every index entry.
  for (int64_t k = 0; k < num_idx; ++k) out_idx[k] = old2new[idx[k]];

  *out_num_vtx = u;
  return ORACLE_OK;
}

}  // extern "C"
