// Instantiates the sort and flag-scan kernels for one record width.
// Built once per K with -DMRX_INST_K=<K>.
#include <algorithm>

#include "group_kernels.hpp"
#include "registry.hpp"

#ifndef MRX_INST_K
#error "MRX_INST_K must be defined"
#endif

#define MRX_CAT2(a, b) a##b
#define MRX_CAT(a, b) MRX_CAT2(a, b)

namespace mrx {
namespace {

constexpr int K = MRX_INST_K;

template <int D, int BLOCK, int IPT, bool WIDE>
void launch_pass_w(const SortPassArgs& a, int mode, int64_t grid, hipStream_t s) {
  switch (mode) {
    case kPassFirst:
      hipLaunchKernelGGL((k_onesweep<K, D, BLOCK, IPT, kPassFirst, WIDE>), dim3(grid), dim3(BLOCK), 0, s, a);
      break;
    case kPassKey:
      hipLaunchKernelGGL((k_onesweep<K, D, BLOCK, IPT, kPassKey, WIDE>), dim3(grid), dim3(BLOCK), 0, s, a);
      break;
    case kPassFirstHash:
      hipLaunchKernelGGL((k_onesweep<K, D, BLOCK, IPT, kPassFirstHash, WIDE>), dim3(grid), dim3(BLOCK), 0, s, a);
      break;
    case kPassHash:
      hipLaunchKernelGGL((k_onesweep<K, D, BLOCK, IPT, kPassHash, WIDE>), dim3(grid), dim3(BLOCK), 0, s, a);
      break;
    case kPassFirstHashMesh:
      hipLaunchKernelGGL((k_onesweep<K, D, BLOCK, IPT, kPassFirstHashMesh, WIDE>), dim3(grid), dim3(BLOCK), 0, s,
                         a);
      break;
    case kPassHashMesh:
      hipLaunchKernelGGL((k_onesweep<K, D, BLOCK, IPT, kPassHashMesh, WIDE>), dim3(grid), dim3(BLOCK), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_onesweep<K, D, BLOCK, IPT, kPassMesh, WIDE>), dim3(grid), dim3(BLOCK), 0, s, a);
      break;
  }
}

template <int D, int BLOCK, int IPT>
void launch_pass(const SortPassArgs& a, int mode, bool wide, int64_t grid, hipStream_t s) {
  if (grid <= 0) return;
  if (wide)
    launch_pass_w<D, BLOCK, IPT, true>(a, mode, grid, s);
  else
    launch_pass_w<D, BLOCK, IPT, false>(a, mode, grid, s);
}

// Record groups per thread of a histogram workgroup (a chunk is 256 threads
// times this many groups).
constexpr int kHistGroups = 4;

template <int D>
void launch_hist(const uint32_t* vtx, int64_t n, uint32_t* hist, hipStream_t s) {
  constexpr int B = 256, GROUPS = kHistGroups;
  constexpr int R = items_per_group(K);
  const int64_t per_block = int64_t(B) * GROUPS * R;
  const int64_t grid = (n + per_block - 1) / per_block;
  const HistArgs a{{vtx, vtx}, nullptr, n, nullptr, hist};
  if (grid > 0)
    hipLaunchKernelGGL((k_histogram<KeyDigits<K, D>, K, D, K, B, GROUPS>), dim3(grid), dim3(B), 0, s, a);
}

// Key-digit histograms of sort elements (K + 1 words) whose buffer and count
// are read on the device. The grid covers a.n (the capacity), capped at two
// workgroups per CU: each workgroup then walks several chunks before it adds
// its LDS histograms to the global ones once (with one chunk per workgroup
// those additions, one per nonzero bin, cost more than the counting).
constexpr int64_t kElemHistGrid = 512;

template <int D>
void launch_elem_hist(const HistArgs& a, hipStream_t s) {
  constexpr int B = 256, GROUPS = kHistGroups;
  constexpr int R = items_per_group(K + 1);
  const int64_t per_block = int64_t(B) * GROUPS * R;
  const int64_t grid = std::min<int64_t>((a.n + per_block - 1) / per_block, kElemHistGrid);
  if (grid > 0)
    hipLaunchKernelGGL((k_histogram<KeyDigits<K, D>, K, D, K + 1, B, GROUPS>), dim3(grid), dim3(B), 0, s, a);
}

// Hash-digit histograms of the records for ph passes, with Step 1's marking
// in the same launch when there is something to mark.
template <int D, int PH>
void launch_hash_hist_ph(const MarkArgs* ma, const uint32_t* vtx, int64_t n, uint32_t* hist, hipStream_t s) {
  constexpr int B = kRandBlock, GROUPS = kHistGroups;
  constexpr int R = items_per_group(K);
  const int64_t per_block = int64_t(B) * GROUPS * R;
  const int64_t ht = (n + per_block - 1) / per_block;
  if (ma && ma->m > 0) {
    const int64_t mt = (ma->m + kRandBlock * kRandItems - 1) / (kRandBlock * kRandItems);
    hipLaunchKernelGGL((k_mark_histogram<HashDigits<K, D, PH>, K, D, B, GROUPS, false>), dim3(ht + mt), dim3(B),
                       0, s, *ma, vtx, n, hist, ht, mt);
  } else if (ht > 0) {
    // a few digits per record: the per-workgroup flush of every nonzero bin
    // outweighs the counting of one chunk, so workgroups walk several chunks
    const HistArgs a{{vtx, vtx}, nullptr, n, nullptr, hist};
    hipLaunchKernelGGL((k_histogram<HashDigits<K, D, PH>, K, D, K, B, GROUPS>), dim3(std::min(ht, kElemHistGrid)),
                       dim3(B), 0, s, a);
  }
}

// Step 1's band marking (one block per band) and the hash-digit histograms
// (hist_blocks blocks walking the record chunks) in one launch: the band
// blocks wait on short slice reads, the histogram blocks stream records and
// count in LDS, so spread evenly over the grid (block b is histogram block
// h(b) = floor(b * H / (H + nb)) when h steps at b, else band b - h(b)) they
// overlap on every CU.
template <int D, int PH>
__global__ __launch_bounds__(kRandBlock) void k_band_mark_hash_hist(BandArgs ba, HistArgs ha, int64_t hist_blocks) {
  constexpr int B = kRandBlock, GROUPS = kHistGroups;
  using DG = HashDigits<K, D, PH>;
  constexpr int WORDS = PH << D;
  constexpr int R = items_per_group(K);
  __shared__ uint32_t s_h[WORDS];
  extern __shared__ uint32_t s_bits[];
  const int64_t total = hist_blocks + ba.nb;
  const int64_t b = blockIdx.x;
  const int64_t h0 = b * hist_blocks / total;
  const int64_t h1 = (b + 1) * hist_blocks / total;
  if (h1 > h0) {
    const int64_t chunks = ((ha.n + R - 1) / R + B * GROUPS - 1) / (B * GROUPS);
    if (h0 >= chunks) return;  // the whole block
    zero_histograms<WORDS, B>(s_h);
    for (int64_t c = h0; c < chunks; c += hist_blocks) histogram_chunk<DG, K, D, K, B, GROUPS>(ha.src[0], ha.n, s_h, c);
    flush_histograms<WORDS, B>(s_h, ha.hist);
  } else {
    band_mark_body<B>(ba, b - h0, s_bits);
  }
}

template <int D, int PH>
void launch_band_mark_hash_hist_ph(const BandArgs& ba, const uint32_t* vtx, int64_t n, uint32_t* hist,
                                   hipStream_t s) {
  constexpr int B = kRandBlock, GROUPS = kHistGroups;
  constexpr int R = items_per_group(K);
  const int64_t per_block = int64_t(B) * GROUPS * R;
  const int64_t hb = std::min((n + per_block - 1) / per_block, kElemHistGrid);
  const HistArgs ha{{vtx, vtx}, nullptr, n, nullptr, hist};
  const size_t bits_lds = (size_t(1) << ba.shift) / 8;
  hipLaunchKernelGGL((k_band_mark_hash_hist<D, PH>), dim3(hb + ba.nb), dim3(B), bits_lds, s, ba, ha, hb);
}

template <int D>
void launch_band_mark_hash_hist(const BandArgs& ba, const uint32_t* vtx, int64_t n, int ph, uint32_t* hist,
                                hipStream_t s) {
  switch (ph) {
    case 1: launch_band_mark_hash_hist_ph<D, 1>(ba, vtx, n, hist, s); break;
    case 2: launch_band_mark_hash_hist_ph<D, 2>(ba, vtx, n, hist, s); break;
    default: launch_band_mark_hash_hist_ph<D, 3>(ba, vtx, n, hist, s); break;
  }
}

template <int D>
void launch_hash_hist(const MarkArgs* ma, const uint32_t* vtx, int64_t n, int ph, uint32_t* hist,
                      hipStream_t s) {
  switch (ph) {
    case 1: launch_hash_hist_ph<D, 1>(ma, vtx, n, hist, s); break;
    case 2: launch_hash_hist_ph<D, 2>(ma, vtx, n, hist, s); break;
    default: launch_hash_hist_ph<D, 3>(ma, vtx, n, hist, s); break;
  }
}

// Hash-digit histograms of a batch's records (hash of (mesh id, record)),
// on a capped grid of workgroups that each walk several chunks.
// Step 1's marking of a batch (mark_used_tile) and the bucket-digit
// histograms in one launch: the histogram workgroups (few, long, bound by
// the hash and LDS atomics) come first in the grid and the marking tiles
// (many, short, bound by scattered byte stores) fill the rest of the GPU
// beside them.
template <int D, int PH>
__global__ __launch_bounds__(kRandBlock) void k_mark_hash_mesh_hist(MarkArgs ma, const uint32_t* __restrict__ vtx,
                                                                    int64_t n, const int64_t* __restrict__ off,
                                                                    int32_t nmesh, const int32_t* __restrict__ tab,
                                                                    const uint2* __restrict__ mb,
                                                                    uint32_t* __restrict__ hist, int64_t hist_blocks) {
  __shared__ uint32_t s_h[PH << D];
  const int64_t b = blockIdx.x;
  if (b < hist_blocks)
    hash_mesh_hist_block<K, D, PH, kRandBlock, kHistGroups>(vtx, n, off, nmesh, tab, mb, hist, b, hist_blocks, s_h);
  else
    mark_used_tile<true>(ma, b - hist_blocks);
}

template <int D, int PH>
void launch_hash_mesh_hist_ph(const MarkArgs* ma, const uint32_t* vtx, int64_t n, const int64_t* off, int32_t nmesh,
                              const int32_t* tab, const uint2* mb, uint32_t* hist, hipStream_t s) {
  constexpr int B = kRandBlock, GROUPS = kHistGroups;
  const int64_t per_block = int64_t(B) * GROUPS;
  const int64_t grid = std::min((n + per_block - 1) / per_block, kElemHistGrid);
  if (ma && ma->m > 0) {
    const int64_t mt = (ma->m + kRandBlock * kRandItems - 1) / (kRandBlock * kRandItems);
    hipLaunchKernelGGL((k_mark_hash_mesh_hist<D, PH>), dim3(grid + mt), dim3(B), 0, s, *ma, vtx, n, off, nmesh, tab,
                       mb, hist, grid);
  } else if (grid > 0) {
    hipLaunchKernelGGL((k_hash_mesh_histogram<K, D, PH, B, GROUPS>), dim3(grid), dim3(B), 0, s, vtx, n, off, nmesh,
                       tab, mb, hist);
  }
}

template <int D>
void launch_hash_mesh_hist(const MarkArgs* ma, const uint32_t* vtx, int64_t n, const int64_t* off, int32_t nmesh,
                           const int32_t* tab, const uint2* mb, int ph, uint32_t* hist, hipStream_t s) {
  switch (ph) {
    case 1: launch_hash_mesh_hist_ph<D, 1>(ma, vtx, n, off, nmesh, tab, mb, hist, s); break;
    case 2: launch_hash_mesh_hist_ph<D, 2>(ma, vtx, n, off, nmesh, tab, mb, hist, s); break;
    default: launch_hash_mesh_hist_ph<D, 3>(ma, vtx, n, off, nmesh, tab, mb, hist, s); break;
  }
}

template <int D>
void launch_group_compact_hist(const GroupCompactArgs& a, hipStream_t s) {
  constexpr int B = 256;
  if (a.ranges > 0) hipLaunchKernelGGL((k_group_compact_hist<K, D, B>), dim3(a.ranges), dim3(B), 0, s, a);
}

void launch_group(const GroupArgs& a, int64_t grid, hipStream_t s) {
  if (grid > 0) hipLaunchKernelGGL((k_group<K, false>), dim3(grid), dim3(GroupShape<K>::BLOCK), 0, s, a);
}

// Grouping by (mesh id, record) for a batch (the shape of K + 1-word keys).
void launch_group_mesh(const GroupArgs& a, int64_t grid, hipStream_t s) {
  if (grid > 0) hipLaunchKernelGGL((k_group<K, true>), dim3(grid), dim3(GroupShape<K + 1>::BLOCK), 0, s, a);
}

// Mesh-id digit histograms of a batch's key sort after its hash grouping:
// per-mesh counts from the used values' offsets (grouping path) or the
// vertex offsets (everything sorted).
template <int D>
void launch_mesh_hist_path(const int64_t* off_grouped, const int64_t* off_all, const Control* ctl, int32_t nmesh,
                           int32_t passes, uint32_t* hist, hipStream_t s) {
  if (nmesh <= 0 || passes <= 0) return;
  hipLaunchKernelGGL((k_mesh_histogram_path<D>), dim3((nmesh + 255) / 256), dim3(256), 0, s, off_grouped, off_all,
                     ctl, nmesh, passes, hist);
}

void launch_finalize(const FinalizeArgs& a, int64_t grid, hipStream_t s) {
  if (grid > 0) hipLaunchKernelGGL((k_group_finalize<K>), dim3(grid), dim3(256), 0, s, a);
}

// Every block of the fused launch holds the histogram's LDS; beyond this size
// it would cut the number of marking waves a CU can hold.
constexpr int kFusedHistLds = 16 * 1024;

template <int D>
bool mark_hist_applies(int64_t n, int64_t m) {
  constexpr int P = (32 * K + D - 1) / D;
  if (P * (1 << D) * 4 > kFusedHistLds || n <= 0 || m <= 0) return false;
  constexpr int64_t per_block = int64_t(kRandBlock) * kHistGroups * items_per_group(K);
  const int64_t ht = (n + per_block - 1) / per_block;
  const int64_t mt = (m + kRandBlock * kRandItems - 1) / (kRandBlock * kRandItems);
  return ht + mt <= INT32_MAX;
}

template <int D>
void launch_mark_hist(const MarkArgs& ma, bool batched, const uint32_t* vtx, int64_t n, uint32_t* hist,
                      hipStream_t s) {
  constexpr int B = kRandBlock, GROUPS = kHistGroups;
  constexpr int P = (32 * K + D - 1) / D;
  if constexpr (P * (1 << D) * 4 <= kFusedHistLds) {
    if (!mark_hist_applies<D>(n, ma.m)) return;
    constexpr int R = items_per_group(K);
    const int64_t per_block = int64_t(B) * GROUPS * R;
    const int64_t ht = (n + per_block - 1) / per_block;
    const int64_t mt = (ma.m + kRandBlock * kRandItems - 1) / (kRandBlock * kRandItems);
    if (batched)
      hipLaunchKernelGGL((k_mark_histogram<KeyDigits<K, D>, K, D, B, GROUPS, true>), dim3(ht + mt), dim3(B), 0, s,
                         ma, vtx, n, hist, ht, mt);
    else
      hipLaunchKernelGGL((k_mark_histogram<KeyDigits<K, D>, K, D, B, GROUPS, false>), dim3(ht + mt), dim3(B), 0,
                         s, ma, vtx, n, hist, ht, mt);
  }
}

template <int D>
void launch_mesh_hist(const int64_t* off, int32_t nmesh, int32_t passes, uint32_t* hist, hipStream_t s) {
  if (nmesh <= 0 || passes <= 0) return;
  hipLaunchKernelGGL((k_mesh_histogram<D>), dim3((nmesh + 255) / 256), dim3(256), 0, s, off, nmesh,
                     passes, hist);
}

template <int D>
void launch_scan(uint32_t* hist, int32_t passes, int64_t n, const int64_t* n_dev, uint32_t* dead,
                 hipStream_t s) {
  if (passes > 0)
    hipLaunchKernelGGL((k_scan_buckets<D, 256>), dim3(passes), dim3(256), 0, s, hist, n, n_dev, dead);
}

void launch_flag_scan(const FlagScanArgs& a, bool batched, int64_t grid, hipStream_t s) {
  if (grid <= 0) return;
  if (batched)
    hipLaunchKernelGGL((k_flag_scan<K, kScanBlock, kScanIpt, true>), dim3(grid), dim3(kScanBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_flag_scan<K, kScanBlock, kScanIpt, false>), dim3(grid), dim3(kScanBlock), 0, s, a);
}

template <int D, int BLOCK, int IPT>
SortVariant make() {
  SortVariant v;
  v.K = K;
  v.D = D;
  v.block = BLOCK;
  v.ipt = IPT;
  v.pass = &launch_pass<D, BLOCK, IPT>;
  v.hist = &launch_hist<D>;
  v.mark_hist_applies = &mark_hist_applies<D>;
  v.mark_hist = &launch_mark_hist<D>;
  v.mesh_hist = &launch_mesh_hist<D>;
  v.scan = &launch_scan<D>;
  v.flag_scan = &launch_flag_scan;
  v.elem_hist = &launch_elem_hist<D>;
  v.hash_hist = &launch_hash_hist<D>;
  v.band_mark_hash_hist = &launch_band_mark_hash_hist<D>;
  v.group = &launch_group;
  v.group_compact_hist = &launch_group_compact_hist<D>;
  v.finalize = &launch_finalize;
  v.group_chunk = GroupShape<K>::CHUNK;
  v.group_target_bucket = GroupShape<K>::TARGET_BUCKET;
  v.hash_mesh_hist = &launch_hash_mesh_hist<D>;
  v.mesh_hist_path = &launch_mesh_hist_path<D>;
  v.group_mesh = &launch_group_mesh;
  v.group_mesh_chunk = GroupShape<K + 1>::CHUNK;
  v.group_mesh_target_bucket = GroupShape<K + 1>::TARGET_BUCKET;
  return v;
}

}  // namespace

void MRX_CAT(register_k, MRX_INST_K)(std::vector<SortVariant>& out) {
  out.push_back(make<8, 256, default_ipt(K)>());  // variant 0: default
#if MRX_INST_K != 2 && MRX_INST_K != 3 && MRX_INST_K != 8
  // every other width: larger tiles with half the items per thread, and
  // smaller workgroups
  out.push_back(make<8, 512, (default_ipt(K) / 2 > 2 ? default_ipt(K) / 2 : 2)>());
  out.push_back(make<8, 128, default_ipt(K)>());
#endif
#if MRX_INST_K == 2 || MRX_INST_K == 3
  out.push_back(make<8, 512, 16>());
  out.push_back(make<8, 256, 12>());
  out.push_back(make<8, 512, 8>());
  out.push_back(make<8, 1024, 8>());
  out.push_back(make<9, 256, 16>());
  out.push_back(make<9, 512, 8>());
#elif MRX_INST_K == 8
  out.push_back(make<8, 512, 8>());
  out.push_back(make<8, 256, 6>());
#endif
}

}  // namespace mrx
