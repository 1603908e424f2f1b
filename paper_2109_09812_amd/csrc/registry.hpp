// Host-side table of compiled sort variants (one object file per record width).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "band_kernels.hpp"
#include "group_kernels.hpp"
#include "scan_kernels.hpp"
#include "sort_kernels.hpp"

namespace mrx {

// Shape of the flag-scan and compaction tiles (independent of the sort tuning).
constexpr int kScanBlock = 256;
constexpr int kScanIpt = 16;
constexpr int kScanTile = kScanBlock * kScanIpt;

// Step 1 and the digit histograms of Step 2 as one launch. The two read
// different arrays and are held up by different units (scattered byte
// stores for the marking, LDS atomics for the histograms), so their tiles are
// spread evenly over one grid and run side by side. With H histogram tiles
// and M marking tiles, h(b) = floor(b * H / (H + M)) counts the histogram
// tiles before block b: block b is histogram tile h(b) if h(b + 1) > h(b),
// else marking tile b - h(b). DG chooses the digits: every key pass of the
// LSD sort, or the hash passes of the hash grouping.
template <class DG, int K, int D, int BLOCK, int GROUPS, bool BATCHED>
__global__ __launch_bounds__(BLOCK) void k_mark_histogram(MarkArgs ma, const uint32_t* __restrict__ vtx,
                                                          int64_t n, uint32_t* __restrict__ hist,
                                                          int64_t hist_tiles, int64_t mark_tiles) {
  static_assert(BLOCK == kRandBlock, "both halves use the marking block shape");
  constexpr int WORDS = DG::kPasses << D;
  __shared__ uint32_t s_h[WORDS];
  const int64_t total = hist_tiles + mark_tiles;
  const int64_t b = blockIdx.x;
  const int64_t h0 = b * hist_tiles / total;
  const int64_t h1 = (b + 1) * hist_tiles / total;
  if (h1 > h0) {
    zero_histograms<WORDS, BLOCK>(s_h);
    histogram_chunk<DG, K, D, K, BLOCK, GROUPS>(vtx, n, s_h, h0);
    flush_histograms<WORDS, BLOCK>(s_h, hist);
  } else {
    mark_used_tile<BATCHED>(ma, b - h0);
  }
}

struct SortVariant {
  int K = 0, D = 0, block = 0, ipt = 0;
  // one LSD pass over `grid` tiles; `wide` selects 64-bit tagged look-back
  // words (needed once counts can reach 2^30), else 32-bit ones
  void (*pass)(const SortPassArgs&, int mode, bool wide, int64_t grid, hipStream_t) = nullptr;
  // digit histograms of all key passes
  void (*hist)(const uint32_t* vtx, int64_t n, uint32_t* hist, hipStream_t) = nullptr;
  // Step 1 fused with `hist` (k_mark_histogram), where mark_hist_applies:
  // there is something to mark and to sort, and the histograms are small
  // enough to share the CU with the marking waves
  bool (*mark_hist_applies)(int64_t n, int64_t m) = nullptr;
  void (*mark_hist)(const MarkArgs& mark, bool batched, const uint32_t* vtx, int64_t n, uint32_t* hist,
                    hipStream_t) = nullptr;
  // digit histograms of the mesh-id passes of a batch
  void (*mesh_hist)(const int64_t* off, int32_t nmesh, int32_t passes, uint32_t* hist,
                    hipStream_t) = nullptr;
  // per-pass exclusive scan of the histograms, and the passes whose digit
  // is the same for all min(n, *n_dev) elements (dead[p] = 1)
  void (*scan)(uint32_t* hist, int32_t passes, int64_t n, const int64_t* n_dev, uint32_t* dead,
               hipStream_t) = nullptr;
  // run-head flags + prefix sum + scatters over the sorted elements
  void (*flag_scan)(const FlagScanArgs&, bool batched, int64_t grid, hipStream_t) = nullptr;
  // hash grouping: key-digit histograms of sort elements (buffer and count
  // read on the device), hash-digit histograms of the records for `ph`
  // passes (with Step 1's marking when `mark` is given), the grouping kernel
  // and the finalisation after the key sort of the used groups
  void (*elem_hist)(const HistArgs&, hipStream_t) = nullptr;
  void (*hash_hist)(const MarkArgs* mark, const uint32_t* vtx, int64_t n, int ph, uint32_t* hist,
                    hipStream_t) = nullptr;
  // Step 1's band marking (small bands, 256-thread blocks) in one launch
  // with the hash-digit histograms
  void (*band_mark_hash_hist)(const BandArgs& ba, const uint32_t* vtx, int64_t n, int ph, uint32_t* hist,
                              hipStream_t) = nullptr;
  void (*group)(const GroupArgs&, int64_t grid, hipStream_t) = nullptr;
  // grouping path: dense copy of the used groups' elements + their key-digit
  // histograms
  void (*group_compact_hist)(const GroupCompactArgs&, hipStream_t) = nullptr;
  void (*finalize)(const FinalizeArgs&, int64_t grid, hipStream_t) = nullptr;
  int group_chunk = 0;           // sorted positions per grouping workgroup
  int group_target_bucket = 0;   // average bucket size the hash passes aim for
  // hash grouping of a batch: bucket-digit histograms of (mesh id,
  // record), the grouping by (mesh id, record), and the mesh-id digit
  // histograms of the key sort that follows (k_mesh_histogram_path)
  // (with Step 1's marking of the batch in the same launch when `mark` is given)
  void (*hash_mesh_hist)(const MarkArgs* mark, const uint32_t* vtx, int64_t n, const int64_t* off, int32_t nmesh,
                         const int32_t* tab, const uint2* mesh_buckets, int ph, uint32_t* hist,
                         hipStream_t) = nullptr;
  void (*group_mesh)(const GroupArgs&, int64_t grid, hipStream_t) = nullptr;
  void (*mesh_hist_path)(const int64_t* off_grouped, const int64_t* off_all, const Control* ctl, int32_t nmesh,
                         int32_t passes, uint32_t* hist, hipStream_t) = nullptr;
  int group_mesh_chunk = 0;
  int group_mesh_target_bucket = 0;

  int tile() const { return block * ipt; }
  int radix() const { return 1 << D; }
};

// Items per thread of the default variant for K key words (+1 id word):
// wider records hold fewer elements per thread to stay within registers.
constexpr int default_ipt(int K) {
  return (K + 1) <= 4 ? 16 : (K + 1) <= 6 ? 12 : (K + 1) <= 9 ? 8 : (K + 1) <= 12 ? 6 : 4;
}

void register_k1(std::vector<SortVariant>&);
void register_k2(std::vector<SortVariant>&);
void register_k3(std::vector<SortVariant>&);
void register_k4(std::vector<SortVariant>&);
void register_k5(std::vector<SortVariant>&);
void register_k6(std::vector<SortVariant>&);
void register_k7(std::vector<SortVariant>&);
void register_k8(std::vector<SortVariant>&);
void register_k9(std::vector<SortVariant>&);
void register_k10(std::vector<SortVariant>&);
void register_k11(std::vector<SortVariant>&);
void register_k12(std::vector<SortVariant>&);
void register_k13(std::vector<SortVariant>&);
void register_k14(std::vector<SortVariant>&);
void register_k15(std::vector<SortVariant>&);
void register_k16(std::vector<SortVariant>&);

}  // namespace mrx
