// Host-side table of compiled sort variants (one object file per record width).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "scan_kernels.hpp"
#include "sort_kernels.hpp"

namespace mrx {

// Shape of the flag-scan and compaction tiles (independent of the sort tuning).
constexpr int kScanBlock = 256;
constexpr int kScanIpt = 16;
constexpr int kScanTile = kScanBlock * kScanIpt;

struct SortVariant {
  int K = 0, D = 0, block = 0, ipt = 0;
  // one LSD pass over `grid` tiles; `wide` selects 64-bit tagged look-back
  // words (needed once counts can reach 2^30), else 32-bit ones
  void (*pass)(const SortPassArgs&, int mode, bool wide, int64_t grid, hipStream_t) = nullptr;
  // digit histograms of all key passes
  void (*hist)(const uint32_t* vtx, int64_t n, uint32_t* hist, hipStream_t) = nullptr;
  // digit histograms of the mesh-id passes of a batch
  void (*mesh_hist)(const int64_t* off, int32_t nmesh, int32_t passes, uint32_t* hist,
                    hipStream_t) = nullptr;
  // per-pass exclusive scan of the histograms
  void (*scan)(uint32_t* hist, int32_t passes, hipStream_t) = nullptr;
  // run-head flags + prefix sum + scatters over the sorted elements
  void (*flag_scan)(const FlagScanArgs&, bool batched, int64_t grid, hipStream_t) = nullptr;

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
