// meshrx C ABI: argument validation, workspace layout and the launch
// sequence of the re-indexing pipeline (Section 2, Steps 1-4), plus the
// attribute gather and its backward.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/meshrx.h"
#include "band_kernels.hpp"
#include "edit_kernels.hpp"
#include "registry.hpp"

namespace mrx {

// Zero a 16-byte aligned byte range (the per-call control state) and the
// caller's status word.
__global__ void k_fill_zero(uint4* __restrict__ p, int64_t n16, int32_t* status, int64_t* count,
                            int64_t* count2) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (status) *status = 0;
    if (count) *count = 0;
    if (count2) *count2 = 0;
  }
}

// Batch epilogue: out_off[b] = number of used groups of meshes < b, read
// from cmap at the first sorted position of mesh b (a head, since heads
// break at mesh starts).
__global__ void k_batch_offsets(const int64_t* __restrict__ vtx_off, int32_t nmesh, SortBuffers bufs,
                                const uint2* pairs_in, const int32_t* __restrict__ cmap, const Control* ctl,
                                const int64_t* __restrict__ total_used, int64_t n, int32_t gate,
                                int64_t* __restrict__ out_off) {
  if (gate_closed(gate, ctl)) return;
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nmesh) return;
  const int64_t p = vtx_off[b];
  int64_t r = *total_used;
  if (b < nmesh && p >= 0 && p < n) {
    const uint2* pairs = pairs_in ? pairs_in : reinterpret_cast<const uint2*>(bufs.spare());
    const uint32_t g = pairs[p].x;
    if (int64_t(g) < ctl->num_groups) {
      const int32_t c = cmap[g];
      r = c >= 0 ? c : ~c;
    }
  }
  out_off[b] = r;
}

// Output offsets of a batch after its hash grouping: the used groups'
// elements (record, name), packed densely before the key sort, are in order
// of their names, the sorted positions of the groups' first copies, which
// lie in their mesh's vertex range; so mesh b's outputs start at the number
// of packed elements whose name is below vtx_off[b] (a binary search per
// mesh). The key sort by (mesh id, record) keeps the meshes in that order.
__global__ void k_batch_offsets_dense(const uint32_t* __restrict__ dense, int32_t stride, const Control* ctl,
                                      const int64_t* __restrict__ vtx_off, int32_t nmesh,
                                      int64_t* __restrict__ out_off) {
  if (gate_closed(kGateGrouped, ctl)) return;
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nmesh) return;
  const int64_t u = ctl->num_used;
  const int64_t start = vtx_off[b];
  int64_t lo = 0, hi = u;  // first packed position whose name is >= start
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(dense[mid * stride + stride - 1]) < start) lo = mid + 1; else hi = mid;
  }
  out_off[b] = lo;
}

// Hash buckets of a batch's meshes (mesh_bucket): mesh b gets the smallest
// power-of-two count of buckets that brings its vertices per bucket down to
// `target`, and the meshes' ranges follow each other in mesh order. One
// workgroup.
constexpr int kMeshBucketBlock = 1024;
__global__ __launch_bounds__(kMeshBucketBlock) void k_mesh_buckets(const int64_t* __restrict__ off, int32_t nmesh,
                                                                   int32_t target, uint2* __restrict__ mb) {
  __shared__ uint32_t s_wave[kMeshBucketBlock / kWave];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nmesh; b0 += kMeshBucketBlock) {
    const int64_t b = b0 + threadIdx.x;
    uint32_t cnt = 0;
    if (b < nmesh) {
      const int64_t nb = off[b + 1] - off[b];
      int k = 0;
      while (k < 30 && (nb >> k) > target) ++k;
      cnt = 1u << k;
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<kMeshBucketBlock>(cnt, s_wave, &total);
    if (b < nmesh) mb[b] = make_uint2(carry + ex, cnt - 1u);
    carry += total;
  }
}

__global__ void k_localize_new2old(int32_t* __restrict__ new2old, const int64_t* __restrict__ total_used,
                                   const int64_t* __restrict__ vtx_off, int32_t nmesh,
                                   const int32_t* __restrict__ vtx_tab) {
  const int64_t u = *total_used;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < u; j += stride) {
    const int32_t g = new2old[j];
    new2old[j] = g - int32_t(vtx_off[mesh_of(vtx_off, nmesh, g, vtx_tab)]);
  }
}

// tab[q] = mesh of packed id min(q << kMeshTabShift, total - 1), q in [0, nq),
// the bucket table that lets mesh_of search a handful of meshes.
__global__ void k_mesh_table(const int64_t* __restrict__ off, int32_t nmesh, int64_t total, int32_t* tab,
                             int64_t nq) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int64_t x = min(q << kMeshTabShift, total - 1);
  tab[q] = int32_t(mesh_of(off, nmesh, x));
}

// Workspace of mrx_reindex_mesh_noalloc: a fixed array in the library's code
// object, one copy per GPU the library runs on, kept until the process ends.
// In host code this name denotes a host-side stand-in, not device memory:
// host code only ever uses the device address that hipGetSymbolAddress
// returns for it (scratch_of_current_device).
static __device__ __align__(256) unsigned char scratch[MRX_NOALLOC_SCRATCH_BYTES];

namespace {

// ---------------------------------------------------------------- profiling
struct ProfRecord {
  const char* name;  // null: end of a call
  hipEvent_t event;
};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<ProfRecord> recs;

  hipEvent_t take() {
    if (next == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[next++];
  }
};

Profiler& profiler() {
  static Profiler p;
  return p;
}

// Records a timing event on the stream before a kernel launch (name != null)
// or after the last launch of a call (name == null). Kernel i of a call runs
// between its mark and the next one, since the stream executes in order.
void prof_mark(const char* name, hipStream_t s) {
  Profiler& p = profiler();
  if (!p.on) return;
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t e = p.take();
  if (!e) return;
  if (hipEventRecord(e, s) != hipSuccess) return;
  p.recs.push_back(ProfRecord{name, e});
}

constexpr int64_t kMaxCount = int64_t(INT32_MAX);  // ids and counts are int32
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

const std::vector<SortVariant>& variants_for(int K) {
  static std::vector<SortVariant> table[17];
  static std::once_flag once;
  std::call_once(once, [] {
    void (*reg[16])(std::vector<SortVariant>&) = {
        register_k1, register_k2, register_k3, register_k4, register_k5, register_k6,
        register_k7, register_k8, register_k9, register_k10, register_k11, register_k12,
        register_k13, register_k14, register_k15, register_k16};
    for (int k = 1; k <= 16; ++k) reg[k - 1](table[k]);
  });
  static const std::vector<SortVariant> empty;
  return (K >= 1 && K <= 16) ? table[K] : empty;
}

// Sort passes use 32-bit look-back words unless a count could reach 2^30
// (or the caller asks for the 64-bit words).
constexpr int64_t kCompactLookbackLimit = int64_t(1) << 30;
bool wide_lookback(int64_t n, const mrx_tuning* t) {
  return n >= kCompactLookbackLimit || (t && (t->flags & MRX_TUNING_WIDE_LOOKBACK));
}

// Picks the variant a tuning asks for; all-zero shape (or NULL) = variant 0.
// Unknown flag bits are rejected.
const SortVariant* pick_variant(int K, const mrx_tuning* t) {
  const auto& vs = variants_for(K);
  if (vs.empty()) return nullptr;
  constexpr int32_t known = MRX_TUNING_WIDE_LOOKBACK | MRX_TUNING_CLAIMED_TILES | MRX_TUNING_SORT_ALL |
                             MRX_TUNING_HASH_GROUPS | MRX_TUNING_BANDS;
  if (t && (t->flags & ~known) != 0) return nullptr;
  if (t && (t->flags & MRX_TUNING_SORT_ALL) && (t->flags & MRX_TUNING_HASH_GROUPS)) return nullptr;
  if (!t || (t->digit_bits == 0 && t->block_threads == 0 && t->items_per_thread == 0)) return &vs[0];
  for (const auto& v : vs)
    if (v.D == t->digit_bits && v.block == t->block_threads && v.ipt == t->items_per_thread) return &v;
  return nullptr;
}

int bits_for(int64_t x) {  // bits needed to represent values 0..x
  int b = 0;
  while (x > 0) { ++b; x >>= 1; }
  return b;
}

// Hash grouping for a single mesh of n vertices? Its look-back words hold
// counts below 2^30.
constexpr int64_t kHashMinDefault = int64_t(1) << 16;
bool use_hash_groups(int64_t n, int32_t nmesh, const mrx_tuning* t) {
  if (nmesh != 1 || n >= kCompactLookbackLimit) return false;
  if (t && (t->flags & MRX_TUNING_SORT_ALL)) return false;
  if (t && (t->flags & MRX_TUNING_HASH_GROUPS)) return true;
  return n >= kHashMinDefault;
}

// Hash grouping for a batch (key = (mesh id, record))? By default from 2^16
// vertices in all, as for single meshes.
bool use_batched_hash(int64_t n, int32_t nmesh, const mrx_tuning* t) {
  if (nmesh < 2 || n <= 0 || n >= kCompactLookbackLimit) return false;
  if (t && (t->flags & MRX_TUNING_SORT_ALL)) return false;
  if (t && (t->flags & MRX_TUNING_HASH_GROUPS)) return true;
  return n >= kHashMinDefault;
}

// Hash passes: enough D-bit hash digits that a bucket averages at most the
// grouping kernel's target size (1 to 3 passes).
int hash_passes(int64_t n, int D, int target_bucket) {
  int bits = 0;
  while ((n >> bits) > target_bucket) ++bits;
  return std::max(1, std::min(3, (bits + D - 1) / D));
}

// Steps 1 and 4 by vertex bands (band_kernels.hpp) for one mesh. kMarkOnly:
// the marking alone (the index partition in a sort buffer that is free until
// the marking is done: C on the hash-grouping path, B on the sort-all path);
// kMarkAndMap: the marking, old2new and the remap, with the index partition
// in out_idx (its slots become the remapped tiles) and the new ids of the
// entries in a free sort buffer (C, or the sort-all path's spare buffer once
// the pairs in it are partitioned). Chosen when there are enough entries to pay for the extra
// launches on the hash-grouping path (or MRX_TUNING_BANDS asks for it, on
// either path), at most kMaxBands bands of at
// most 2^kMaxMarkShift (marking) or 2^kMaxMapShift (map) vertices, and C
// holds m words. Below about 2^20 entries the five extra launches cost more
// than the scattered accesses they replace (a 390K-entry soup: 0.28 against
// 0.22 ms).
enum BandMode { kBandNone = 0, kMarkOnly = 1, kMarkAndMap = 2 };
constexpr int64_t kBandMinEntries = int64_t(1) << 20;
struct BandPlan {
  int mode = kBandNone;
  int shift = 0, nb = 0;
  int64_t itiles = 0, ptiles = 0;
  size_t words() const {  // index table + tile counts (+ pair table)
    if (mode == kBandNone) return 0;
    return size_t(nb) * size_t(itiles) + size_t(itiles) + (mode == kMarkAndMap ? size_t(nb) * size_t(ptiles) : 0);
  }
};
BandPlan band_plan(int64_t n, int64_t m, int s, bool force, bool automatic) {
  BandPlan b;
  if (n <= 0 || m <= 0 || (!force && (!automatic || m < kBandMinEntries)) || m > n * int64_t(s)) return b;
  int want = kMinBandShift;  // about 256 bands where the band size allows it
  while (((n - 1) >> want) + 1 > 256) ++want;
  for (int mode : {int(kMarkAndMap), int(kMarkOnly)}) {
    const int shift = std::min(want, mode == kMarkAndMap ? kMaxMapShift : kMaxMarkShift);
    const int64_t nb = ((n - 1) >> shift) + 1;
    if (nb > kMaxBands) continue;
    b.mode = mode;
    b.shift = shift;
    b.nb = int(nb);
    b.itiles = (m + kBandTile - 1) / kBandTile;
    b.ptiles = mode == kMarkAndMap ? (n + kPairTile - 1) / kPairTile : 0;
    return b;
  }
  return b;
}

struct Layout {
  int K = 0, S = 0, P_key = 0, P_mesh = 0, P_hash = 0;  // P_hash > 0: hash grouping
  BandPlan band;                                         // hash grouping only
  int64_t tiles_sort = 0, tiles_scan = 0, tiles_group = 0;
  bool mesh_hash = false;  // hash grouping of a batch (key = (mesh id, record))
  // zeroed region
  size_t ctl = 0, counters = 0, hist = 0, plan = 0, lookback = 0, scan_lookback = 0, elem_lookback = 0,
         used_v = 0, used_g = 0, hist_hash = 0, plan_hash = 0, dead_hash = 0, group_chunks = 0, group_ranges = 0,
         zero_end = 0;
  int64_t tiles_elem = 0;
  // scratch
  size_t buf_a = 0, buf_b = 0, buf_c = 0, uniq = 0, rep = 0, cmap = 0, vtx_tab = 0, elem_tab = 0, band_tab = 0,
         mesh_bk = 0, total = 0;
  int64_t vtx_tab_n = 0, elem_tab_n = 0;
};

// Element tiles of the sub-mesh selection (k_select_elements).
constexpr int kSelectBlock = 256;
constexpr int kSelectIpt = 16;
constexpr int kSelectTile = kSelectBlock * kSelectIpt;

// num_idx bounds the element count of a sub-mesh selection (arity >= 1).
Layout make_layout(int64_t n, int64_t num_idx, int K, int32_t nmesh, const SortVariant& v,
                   const mrx_tuning* tuning) {
  Layout L;
  L.K = K;
  L.S = K + 1;
  L.P_key = (32 * K + v.D - 1) / v.D;
  L.P_mesh = nmesh > 1 ? (bits_for(int64_t(nmesh) - 1) + v.D - 1) / v.D : 0;
  int ph_mesh = 0;
  if (use_batched_hash(n, nmesh, tuning)) {
    // every mesh's bucket count is at most 1 + 2 n_b / target (k_mesh_buckets)
    const int64_t buckets = int64_t(nmesh) + 2 * n / v.group_mesh_target_bucket + 1;
    ph_mesh = (bits_for(buckets) + v.D - 1) / v.D;
    L.mesh_hash = ph_mesh <= 3;  // more than 2^24 buckets: sort all
  }
  if (L.mesh_hash)
    L.P_hash = ph_mesh;
  else
    L.P_hash = use_hash_groups(n, nmesh, tuning) ? hash_passes(n, v.D, v.group_target_bucket) : 0;
  L.tiles_sort = (n + v.tile() - 1) / v.tile();
  L.tiles_scan = (n + kScanTile - 1) / kScanTile;
  const int group_chunk = L.mesh_hash ? v.group_mesh_chunk : v.group_chunk;
  L.tiles_group = L.P_hash ? (n + group_chunk - 1) / group_chunk : 0;
  const int P = L.P_key + L.P_mesh;
  size_t off = 0;
  L.ctl = off;      off = align_up(off + sizeof(Control));
  // tile counters of every look-back launch of a call (claimed tiles)
  L.counters = off; off = align_up(off + sizeof(uint32_t) * size_t(P + L.P_hash + 8));
  L.hist = off;     off = align_up(off + sizeof(uint32_t) * size_t(P) * size_t(v.radix()));
  L.plan = off;     off = align_up(off + sizeof(uint32_t) * size_t(2 * P + 1));  // SortBuffers::plan
  // sort look-back: tiles x radix 64-bit words, or two alternating buffers of
  // 32-bit words in the same bytes; flag scan and compaction have their own
  const int64_t lb_words = std::max<int64_t>(L.tiles_sort * v.radix(), 1);
  L.lookback = off; off = align_up(off + sizeof(uint64_t) * size_t(lb_words));
  L.scan_lookback = off; off = align_up(off + sizeof(uint64_t) * size_t(L.tiles_scan + 1));
  L.tiles_elem = (num_idx + kSelectTile - 1) / kSelectTile;
  L.elem_lookback = off; off = align_up(off + sizeof(uint64_t) * size_t(L.tiles_elem + 1));
  L.used_g = off;   off = align_up(off + size_t(n));
  if (L.P_hash) {
    L.hist_hash = off; off = align_up(off + sizeof(uint32_t) * size_t(L.P_hash) * size_t(v.radix()));
    L.plan_hash = off; off = align_up(off + sizeof(uint32_t) * size_t(2 * L.P_hash + 1));
    L.dead_hash = off; off = align_up(off + sizeof(uint32_t) * size_t(L.P_hash));
    L.group_chunks = off; off = align_up(off + sizeof(uint32_t) * 4 * size_t(L.tiles_group));
    L.group_ranges = off; off = align_up(off + sizeof(uint32_t) * 3 * size_t(group_compact_ranges(L.tiles_group)));
  }
  // last, so that a call whose Step 1 writes every flag (by bands) can leave
  // it out of the clearing
  L.used_v = off;   off = align_up(off + size_t(n));
  L.zero_end = off;
  L.buf_a = off;    off = align_up(off + sizeof(uint32_t) * size_t(n) * L.S);
  L.buf_b = off;    off = align_up(off + sizeof(uint32_t) * size_t(n) * L.S);
  if (L.P_hash) {
    L.buf_c = off;  off = align_up(off + sizeof(uint32_t) * size_t(n) * L.S);
  }
  if (nmesh == 1) {
    // by default only with hash grouping, the strategy for meshes whose
    // copies (and so index entries) are scattered; on the sort-all path,
    // which the autotuner keeps for meshes stored in order (the paper's quad
    // grid: 0.46 ms without bands, 0.75 ms with), only when asked for
    L.band = band_plan(n, num_idx, L.S, tuning && (tuning->flags & MRX_TUNING_BANDS), L.P_hash > 0);
    L.band_tab = off; off = align_up(off + sizeof(uint32_t) * L.band.words());
  }
  L.uniq = off;     off = align_up(off + sizeof(uint32_t) * size_t(n) * K);
  L.rep = off;      off = align_up(off + sizeof(int32_t) * size_t(n));
  L.cmap = off;     off = align_up(off + sizeof(int32_t) * size_t(n));
  // bucket tables of the element offsets (batch, merge) and vertex offsets
  // (batch) for mesh_of; the element table is small enough to always reserve
  L.elem_tab_n = (std::max<int64_t>(num_idx, 1) - 1) / (int64_t(1) << kMeshTabShift) + 2;
  L.elem_tab = off; off = align_up(off + sizeof(int32_t) * size_t(L.elem_tab_n));
  if (nmesh > 1) {
    L.vtx_tab_n = (std::max<int64_t>(n, 1) - 1) / (int64_t(1) << kMeshTabShift) + 2;
    L.vtx_tab = off;  off = align_up(off + sizeof(int32_t) * size_t(L.vtx_tab_n));
  }
  if (L.mesh_hash) {
    L.mesh_bk = off;  off = align_up(off + sizeof(uint2) * size_t(nmesh));
  }
  L.total = off;
  return L;
}

// True if [a, a+na) and [b, b+nb) overlap (empty ranges never do).
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

struct Buffer {
  const void* p;
  size_t bytes;
};

// No two listed buffers may overlap.
bool disjoint(std::initializer_list<Buffer> list) {
  std::vector<Buffer> v(list);
  for (size_t i = 0; i < v.size(); ++i)
    for (size_t j = i + 1; j < v.size(); ++j)
      if (overlaps(v[i].p, v[i].bytes, v[j].p, v[j].bytes)) return false;
  return true;
}

int64_t grid_for(int64_t work, int block, int64_t cap = 8192) {
  return std::max<int64_t>(1, std::min<int64_t>((work + block - 1) / block, cap));
}

// Digit location of LSD key bit `bit` (0 = least significant bit of the last
// word): word masks select the word holding it and the next more
// significant word.
void set_digit(SortPassArgs& a, int K, int bit) {
  a.lo_word = K - 1 - bit / 32;
  a.hi_word = a.lo_word - 1;  // -1: none
  a.shift = bit % 32;
}

int64_t rand_grid(int64_t work, int items = kRandItems) {
  return std::max<int64_t>(1, (work + kRandBlock * items - 1) / (kRandBlock * items));
}

mrx_status check_launch() {
  return hipGetLastError() == hipSuccess ? MRX_OK : MRX_ERR_HIP;
}

// Shared validation of the re-index calls (everything before any HIP call).
mrx_status validate_common(const void* vtx, int64_t num_vtx, int32_t vtx_bytes, const int32_t* idx,
                           int64_t num_elems, int32_t arity, const void* out_vtx,
                           const int32_t* out_idx, const int32_t* old2new, const void* workspace,
                           size_t workspace_bytes) {
  if (vtx_bytes < 4 || vtx_bytes > 64 || vtx_bytes % 4 != 0) return MRX_ERR_INVALID_ARGUMENT;
  if (arity < 1 || num_vtx < 0 || num_elems < 0) return MRX_ERR_INVALID_ARGUMENT;
  if (num_vtx > kMaxCount) return MRX_ERR_TOO_LARGE;
  if (num_elems > kMaxCount / arity) return MRX_ERR_TOO_LARGE;
  const int64_t m = num_elems * arity;
  if (num_vtx > 0 && (!vtx || !out_vtx || !old2new)) return MRX_ERR_INVALID_ARGUMENT;
  if (m > 0 && (!idx || !out_idx)) return MRX_ERR_INVALID_ARGUMENT;
  if (!aligned(vtx, 4) || !aligned(out_vtx, 4) || !aligned(idx, 4) || !aligned(out_idx, 4) ||
      !aligned(old2new, 4))
    return MRX_ERR_INVALID_ARGUMENT;
  if (workspace_bytes > 0 && (!workspace || !aligned(workspace, kAlign))) return MRX_ERR_INVALID_ARGUMENT;
  return MRX_OK;
}

// Checks shared by every single-mesh call; on success *layout describes the
// workspace. `extra` lists caller buffers of the call that must not overlap
// any of the others (NULL entries are ignored).
mrx_status validate_single(const void* vtx, int64_t num_vtx, int32_t vtx_bytes, const int32_t* idx,
                           int64_t num_elems, int32_t arity, const void* out_vtx, const int32_t* out_idx,
                           const int32_t* old2new, const int32_t* new2old, const int64_t* out_num_vtx,
                           const int32_t* dev_status, const void* workspace, size_t workspace_bytes,
                           const mrx_tuning* tuning, std::initializer_list<Buffer> extra,
                           const SortVariant** variant, Layout* layout) {
  mrx_status st = validate_common(vtx, num_vtx, vtx_bytes, idx, num_elems, arity, out_vtx, out_idx,
                                  old2new, workspace, workspace_bytes);
  if (st != MRX_OK) return st;
  // dev_status is required: it is the only channel for data errors and for
  // a cross-workgroup wait that gave up (results invalid)
  if (!out_num_vtx || !aligned(out_num_vtx, 8) || !aligned(new2old, 4) || !dev_status ||
      !aligned(dev_status, 4))
    return MRX_ERR_INVALID_ARGUMENT;
  const int K = vtx_bytes / 4;
  const SortVariant* vp = pick_variant(K, tuning);
  if (!vp) return MRX_ERR_UNSUPPORTED;
  const int64_t n = num_vtx, m = num_elems * arity;
  const Layout L = make_layout(n, m, K, 1, *vp, tuning);
  if (workspace_bytes < L.total) return MRX_ERR_WORKSPACE_TOO_SMALL;
  const size_t vb = size_t(n) * vtx_bytes, ib = size_t(m) * 4, nb = size_t(n) * 4;
  std::vector<Buffer> outs = {{out_idx, ib}, {vtx, vb}, {out_vtx, vb}, {old2new, nb},
                              {new2old, new2old ? nb : 0}, {out_num_vtx, 8},
                              {dev_status, 4u}, {workspace, L.total}};
  for (const Buffer& b : extra) outs.push_back(b);
  for (size_t i = 0; i < outs.size(); ++i)
    for (size_t j = i + 1; j < outs.size(); ++j)
      if (overlaps(outs[i].p, outs[i].bytes, outs[j].p, outs[j].bytes)) return MRX_ERR_INVALID_ARGUMENT;
  // idx may be out_idx itself, but may not overlap any other buffer
  if (idx != out_idx)
    for (size_t j = 0; j < outs.size(); ++j)
      if (overlaps(idx, ib, outs[j].p, outs[j].bytes)) return MRX_ERR_INVALID_ARGUMENT;
  *variant = vp;
  *layout = L;
  return MRX_OK;
}

// The hash-grouping launch sequence of one mesh (see group_kernels.hpp):
//   Step 1 (marking, by vertex bands or by scattered stores) with the
//   hash-digit histograms; stable sort of (record, id | used << 31) by
//   P_hash hash digits into X; grouping of each hash bucket in LDS (pairs
//   (group, id) into Y, one (record, group) element per used group into its
//   chunk's slots of C); the totals and, on the grouping path, the used
//   groups' elements packed into X with their key-digit histograms; key sort
//   of X (the used groups, or, if a bucket did not fit, all N hash-ordered
//   elements); then either the finalisation (output records,
//   representatives, group -> new id) or, on the fallback path, Section 2's
//   flag scan and compaction; Step 4 (old2new and the index remap, by
//   vertex bands or by scattered accesses) is shared.
// Buffers: A and B hold the hash passes (X = the last one written, Y = the
// other), C the used groups' slots (before the grouping: Step 1's index
// partition when only the marking goes by bands); the key sort alternates
// between X and C starting from X; by bands, Step 4 then partitions the
// pairs into X and puts the index entries' new ids in C.
mrx_status launch_hash(const SortVariant& v, const Layout& L, const void* vtx, int64_t num_vtx,
                       int32_t vtx_bytes, const int32_t* idx, int64_t num_elems, int32_t arity,
                       const int64_t* live_elems, void* out_vtx, int32_t* out_idx, int32_t* old2new,
                       int32_t* new2old, int64_t* out_num_vtx, int32_t* dev_status, void* workspace,
                       const mrx_tuning* tuning, void* stream_, bool state_zeroed) {
  const int K = vtx_bytes / 4;
  const int64_t n = num_vtx, m = num_elems * arity;
  const int ph = L.P_hash;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);
  Control* ctl = reinterpret_cast<Control*>(ws + L.ctl);
  uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  uint32_t* plan = reinterpret_cast<uint32_t*>(ws + L.plan);
  uint32_t* hist_hash = reinterpret_cast<uint32_t*>(ws + L.hist_hash);
  uint32_t* plan_hash = reinterpret_cast<uint32_t*>(ws + L.plan_hash);
  uint32_t* dead_hash = reinterpret_cast<uint32_t*>(ws + L.dead_hash);
  uint64_t* lookback = reinterpret_cast<uint64_t*>(ws + L.lookback);
  uint64_t* scan_lookback = reinterpret_cast<uint64_t*>(ws + L.scan_lookback);
  uint4* group_chunks = reinterpret_cast<uint4*>(ws + L.group_chunks);
  uint32_t* group_range_sums = reinterpret_cast<uint32_t*>(ws + L.group_ranges);
  const int64_t group_ranges = group_compact_ranges(L.tiles_group);
  const bool wide = wide_lookback(n, tuning);
  const bool claimed = tuning && (tuning->flags & MRX_TUNING_CLAIMED_TILES);
  uint32_t* const lb32[2] = {reinterpret_cast<uint32_t*>(lookback),
                             reinterpret_cast<uint32_t*>(lookback) + size_t(L.tiles_sort) * v.radix()};
  uint8_t* used_v = reinterpret_cast<uint8_t*>(ws + L.used_v);
  uint8_t* used_g = reinterpret_cast<uint8_t*>(ws + L.used_g);
  uint32_t* buf[3] = {reinterpret_cast<uint32_t*>(ws + L.buf_a), reinterpret_cast<uint32_t*>(ws + L.buf_b),
                      reinterpret_cast<uint32_t*>(ws + L.buf_c)};
  uint32_t* uniq = reinterpret_cast<uint32_t*>(ws + L.uniq);
  int32_t* rep = reinterpret_cast<int32_t*>(ws + L.rep);
  int32_t* cmap = reinterpret_cast<int32_t*>(ws + L.cmap);
  int32_t* status = dev_status;
  int counter = 0;  // next tile counter (claimed tiles)
  auto next_counter = [&]() { return claimed ? counters + counter++ : nullptr; };

  if (!state_zeroed) {
    // band marking writes every used flag: those need no clearing
    const int64_t words = int64_t((L.band.mode != kBandNone ? L.used_v : L.zero_end) / 16);
    prof_mark("fill_zero", s);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(words, 256, 4096)), dim3(256), 0, s,
                       reinterpret_cast<uint4*>(ws), words, dev_status, out_num_vtx,
                       static_cast<int64_t*>(nullptr));
  }
  // Step 1 and the hash-digit histograms: Step 1 by vertex bands (the index
  // partition in out_idx, or in C, which the grouping fills only later),
  // else scattered byte stores beside the histograms
  const BandPlan& bp = L.band;
  const MarkArgs mark{idx, m, arity, n, nullptr, nullptr, 0, nullptr, live_elems, used_v, status};
  uint32_t* band_tab = reinterpret_cast<uint32_t*>(ws + L.band_tab);
  uint32_t* ipart = bp.mode == kMarkAndMap ? reinterpret_cast<uint32_t*>(out_idx) : buf[2];
  uint32_t* itable = band_tab;
  uint32_t* itile_valid = itable + size_t(bp.nb) * size_t(bp.itiles);
  uint32_t* ptable = itile_valid + bp.itiles;
  if (bp.mode != kBandNone) {
    const BandArgs ba{idx, m, arity, n, live_elems, bp.shift, bp.nb, aligned(idx, 16) ? 1 : 0,
                      bp.mode == kMarkAndMap ? 1 : 0, bp.itiles, ipart, itable, itile_valid, used_v, status};
    prof_mark("band_partition", s);
    launch_band_partition(ba, s);
    if (bp.mode == kMarkAndMap) {
      prof_mark("band_mark_histogram", s);
      v.band_mark_hash_hist(ba, static_cast<const uint32_t*>(vtx), n, ph, hist_hash, s);
    } else {
      prof_mark("band_mark", s);
      launch_band_mark(ba, false, s);
    }
  }
  if (bp.mode != kMarkAndMap) {
    const bool fused_mark = m > 0 && bp.mode == kBandNone;
    prof_mark(fused_mark ? "mark_histogram" : "hash_histogram", s);
    v.hash_hist(fused_mark ? &mark : nullptr, static_cast<const uint32_t*>(vtx), n, ph, hist_hash, s);
  }
  if (n > 0) {
    // stable sort by the hash digits; every hash pass runs (dead flags go to
    // a word nobody reads), so the elements end in X = buf[(ph - 1) & 1]
    prof_mark("scan_buckets", s);
    v.scan(hist_hash, ph, n, nullptr, dead_hash, s);
    const SortBuffers sbh{{buf[0], buf[1]}, plan_hash, ph};
    int gp = 0;  // index of the pass in the call (look-back buffer parity, tag)
    for (int p = 0; p < ph; ++p, ++gp) {
      SortPassArgs a{};
      a.vtx = static_cast<const uint32_t*>(vtx);
      a.bufs = sbh;
      a.pass = p;
      a.used = used_v;
      a.bucket_base = hist_hash + size_t(p) * v.radix();
      a.lookback = wide ? static_cast<void*>(lookback) : static_cast<void*>(lb32[gp & 1]);
      a.lookback_next = lb32[(gp + 1) & 1];
      a.tile_counter = next_counter();
      a.ctl = ctl;
      a.status = status;
      a.n = n;
      a.lo_word = a.hi_word = -1;
      a.shift = p * v.D;
      a.tag = uint32_t(gp + 1);
      prof_mark(p == 0 ? "onesweep_hash_first" : "onesweep_hash", s);
      v.pass(a, p == 0 ? kPassFirstHash : kPassHash, wide, L.tiles_sort, s);
    }
    uint32_t* X = buf[(ph - 1) & 1];
    uint32_t* Y = buf[((ph - 1) & 1) ^ 1];
    uint2* pairs = reinterpret_cast<uint2*>(Y);

    // group each hash bucket
    GroupArgs g{};
    g.elems = X;
    g.n = n;
    g.bucket_mask = ph * v.D >= 32 ? 0xFFFFFFFFu : (1u << (ph * v.D)) - 1u;
    g.pairs = pairs;
    g.rep = rep;
    g.cmap = cmap;
    g.uelems = buf[2];
    g.chunks = group_chunks;
    g.range_sums = group_range_sums;
    g.ranges = group_ranges;
    g.status = status;
    prof_mark("group", s);
    v.group(g, L.tiles_group, s);

    // key sort of X: the used groups' elements packed from C (or, on the
    // fallback path, all N hash-ordered elements)
    const SortBuffers sbk{{X, buf[2]}, plan, L.P_key};
    const GroupCompactArgs gc{buf[2], group_chunks, group_range_sums, L.tiles_group, group_ranges, n, X, hist, ctl};
    prof_mark("compact_histogram", s);
    v.group_compact_hist(gc, s);
    const HistArgs ha{{X, X}, nullptr, n, &ctl->all_count, hist};
    prof_mark("histogram", s);
    v.elem_hist(ha, s);
    prof_mark("scan_buckets", s);
    v.scan(hist, L.P_key, n, &ctl->sort_count, plan + L.P_key + 1, s);
    prof_mark("sort_plan", s);
    hipLaunchKernelGGL(k_group_sort_plan, dim3(1), dim3(64), 0, s, sbk, static_cast<const Control*>(ctl));
    for (int p = 0; p < L.P_key; ++p, ++gp) {
      SortPassArgs a{};
      a.bufs = sbk;
      a.pass = p;
      a.bucket_base = hist + size_t(p) * v.radix();
      a.lookback = wide ? static_cast<void*>(lookback) : static_cast<void*>(lb32[gp & 1]);
      a.lookback_next = lb32[(gp + 1) & 1];
      a.tile_counter = next_counter();
      a.ctl = ctl;
      a.status = status;
      a.n = n;
      a.n_dev = &ctl->sort_count;
      set_digit(a, K, p * v.D);
      a.tag = uint32_t(gp + 1);
      prof_mark("onesweep", s);
      v.pass(a, kPassKey, wide, L.tiles_sort, s);
    }
    // grouping path: sorted position = new id
    FinalizeArgs fa{};
    fa.bufs = sbk;
    fa.rep = rep;
    fa.cmap = cmap;
    fa.out_vtx = static_cast<uint32_t*>(out_vtx);
    fa.new2old = new2old;
    fa.out_num = out_num_vtx;
    fa.cap = n;
    fa.ctl = ctl;
    fa.status = status;
    prof_mark("finalize", s);
    v.finalize(fa, grid_for(n, 256, 4096), s);
    // fallback path: Section 2's flags, scans and compaction over all of X
    FlagScanArgs f{};
    f.bufs = sbk;
    f.n = n;
    f.uniq = uniq;
    f.rep = rep;
    f.used_g = used_g;
    f.lookback = scan_lookback;
    f.tile_counter = next_counter();
    f.ctl = ctl;
    f.status = status;
    f.tag = uint32_t(gp + 1);
    f.pairs = pairs;
    f.gate = kGateSortAll;
    prof_mark("flag_scan", s);
    v.flag_scan(f, false, L.tiles_scan, s);
    CompactArgs c{};
    c.used_g = used_g;
    c.uniq = uniq;
    c.rep = rep;
    c.K = K;
    c.out_vtx = static_cast<uint32_t*>(out_vtx);
    c.new2old = new2old;
    c.cmap = cmap;
    c.out_num = out_num_vtx;
    c.cap = n;
    c.lookback = scan_lookback;
    c.tile_counter = next_counter();
    c.ctl = ctl;
    c.status = status;
    c.tag = uint32_t(gp + 2);
    c.gate = kGateSortAll;
    prof_mark("compact", s);
    hipLaunchKernelGGL((k_compact<kScanBlock, kScanIpt>), dim3(L.tiles_scan), dim3(kScanBlock), 0, s, c);
    // both paths: Step 4's map (and, by bands, the remap)
    if (bp.mode == kMarkAndMap) {
      // X and C are free again: X takes the partitioned pairs, C the new ids
      // of the index entries
      const PairPartArgs pa{static_cast<const uint2*>(pairs), cmap, n, bp.shift, bp.nb, bp.ptiles,
                            reinterpret_cast<uint2*>(X), ptable, status};
      prof_mark("pair_partition", s);
      launch_pair_partition(pa, s);
      const BandMapArgs ma{reinterpret_cast<const uint2*>(X), ptable, bp.ptiles, ipart, itable, bp.itiles, n,
                           bp.shift, old2new, reinterpret_cast<int32_t*>(buf[2])};
      prof_mark("band_map", s);
      launch_band_map(ma, bp.nb, s);
      const BandRemapArgs ra{ipart, reinterpret_cast<const int32_t*>(buf[2]), itile_valid, m, arity, live_elems,
                             out_idx};
      prof_mark("band_remap", s);
      launch_band_remap(ra, bp.itiles, s);
      prof_mark(nullptr, s);
      return check_launch();
    }
    prof_mark("old2new", s);
    hipLaunchKernelGGL((k_scatter_old2new<false>), dim3(rand_grid(n, kScatterItems)), dim3(kRandBlock), 0, s,
                       sbk, static_cast<const uint2*>(pairs), cmap, n, nullptr, nullptr, 0, nullptr, old2new);
  }
  // Step 4: remap the index array
  if (m > 0) {
    prof_mark("remap", s);
    hipLaunchKernelGGL((k_remap<false>), dim3(rand_grid(m)), dim3(kRandBlock), 0, s, idx, m, arity, n,
                       nullptr, nullptr, 0, nullptr, live_elems, old2new, out_idx);
  }
  prof_mark(nullptr, s);
  return check_launch();
}

// The single-mesh launch sequence (Section 2, Steps 1-4). live_elems
// (device, nullable) limits the index array to its first *live_elems
// elements; num_elems is then only a capacity.
mrx_status launch_single(const SortVariant& v, const Layout& L, const void* vtx, int64_t num_vtx,
                         int32_t vtx_bytes, const int32_t* idx, int64_t num_elems, int32_t arity,
                         const int64_t* live_elems, void* out_vtx, int32_t* out_idx, int32_t* old2new,
                         int32_t* new2old, int64_t* out_num_vtx, int32_t* dev_status, void* workspace,
                         const mrx_tuning* tuning, void* stream_, bool state_zeroed = false) {
  if (L.P_hash)
    return launch_hash(v, L, vtx, num_vtx, vtx_bytes, idx, num_elems, arity, live_elems, out_vtx, out_idx,
                       old2new, new2old, out_num_vtx, dev_status, workspace, tuning, stream_, state_zeroed);
  const int K = vtx_bytes / 4;
  const int64_t n = num_vtx, m = num_elems * arity;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);
  Control* ctl = reinterpret_cast<Control*>(ws + L.ctl);
  uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  uint32_t* plan = reinterpret_cast<uint32_t*>(ws + L.plan);
  uint64_t* lookback = reinterpret_cast<uint64_t*>(ws + L.lookback);
  uint64_t* scan_lookback = reinterpret_cast<uint64_t*>(ws + L.scan_lookback);
  const bool wide = wide_lookback(n, tuning);
  const bool claimed = tuning && (tuning->flags & MRX_TUNING_CLAIMED_TILES);
  uint32_t* const lb32[2] = {reinterpret_cast<uint32_t*>(lookback),
                             reinterpret_cast<uint32_t*>(lookback) + size_t(L.tiles_sort) * v.radix()};
  uint8_t* used_v = reinterpret_cast<uint8_t*>(ws + L.used_v);
  uint8_t* used_g = reinterpret_cast<uint8_t*>(ws + L.used_g);
  uint32_t* buf[2] = {reinterpret_cast<uint32_t*>(ws + L.buf_a), reinterpret_cast<uint32_t*>(ws + L.buf_b)};
  uint32_t* uniq = reinterpret_cast<uint32_t*>(ws + L.uniq);
  int32_t* rep = reinterpret_cast<int32_t*>(ws + L.rep);
  int32_t* cmap = reinterpret_cast<int32_t*>(ws + L.cmap);
  int32_t* status = dev_status;

  const BandPlan& bp = L.band;
  // per-call state: look-back words, tile counters, histograms, flags, G
  // (already cleared when a preceding step of the same call used it; band
  // marking writes every used flag, so those need no clearing)
  if (!state_zeroed) {
    const int64_t words = int64_t((bp.mode != kBandNone ? L.used_v : L.zero_end) / 16);
    prof_mark("fill_zero", s);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(words, 256, 4096)), dim3(256), 0, s,
                       reinterpret_cast<uint4*>(ws), words, dev_status, out_num_vtx,
                       static_cast<int64_t*>(nullptr));
  }
  // Step 1: mark referenced vertices (and report out-of-range entries): by
  // vertex bands (the index partition in out_idx, or in B, which the sort
  // first writes in its second pass), else with the digit histograms of
  // Step 2 in the same launch where it applies
  const MarkArgs mark{idx, m, arity, n, nullptr, nullptr, 0, nullptr, live_elems, used_v, status};
  uint32_t* band_tab = reinterpret_cast<uint32_t*>(ws + L.band_tab);
  uint32_t* ipart = bp.mode == kMarkAndMap ? reinterpret_cast<uint32_t*>(out_idx) : buf[1];
  uint32_t* itable = band_tab;
  uint32_t* itile_valid = itable + size_t(bp.nb) * size_t(bp.itiles);
  uint32_t* ptable = itile_valid + bp.itiles;
  const bool fused = bp.mode == kBandNone && v.mark_hist_applies(n, m);
  if (bp.mode != kBandNone) {
    const BandArgs ba{idx, m, arity, n, live_elems, bp.shift, bp.nb, aligned(idx, 16) ? 1 : 0,
                      bp.mode == kMarkAndMap ? 1 : 0, bp.itiles, ipart, itable, itile_valid, used_v, status};
    prof_mark("band_partition", s);
    launch_band_partition(ba, s);
    prof_mark("band_mark", s);
    launch_band_mark(ba, bp.mode == kMarkAndMap, s);
  } else if (fused) {
    prof_mark("mark_histogram", s);
    v.mark_hist(mark, false, static_cast<const uint32_t*>(vtx), n, hist, s);
  } else if (m > 0) {
    prof_mark("mark_used", s);
    hipLaunchKernelGGL((k_mark_used<false>), dim3(rand_grid(m)), dim3(kRandBlock), 0, s, mark);
  }
  if (n > 0) {
    // Step 2: stable LSD radix sort of (record, id | used << 31)
    if (!fused) {
      prof_mark("histogram", s);
      v.hist(static_cast<const uint32_t*>(vtx), n, hist, s);
    }
    prof_mark("scan_buckets", s);
    v.scan(hist, L.P_key, n, nullptr, plan + L.P_key + 1, s);
    const SortBuffers sb{{buf[0], buf[1]}, plan, L.P_key};
    for (int p = 0; p < L.P_key; ++p) {
      SortPassArgs a{};
      a.vtx = static_cast<const uint32_t*>(vtx);
      a.bufs = sb;
      a.pass = p;
      a.used = used_v;
      a.bucket_base = hist + size_t(p) * v.radix();
      a.lookback = wide ? static_cast<void*>(lookback) : static_cast<void*>(lb32[p & 1]);
      a.lookback_next = lb32[(p + 1) & 1];
      a.tile_counter = claimed ? counters + p : nullptr;
      a.ctl = ctl;
      a.status = status;
      a.n = n;
      set_digit(a, K, p * v.D);
      a.tag = uint32_t(p + 1);
      prof_mark(p == 0 ? "onesweep_first" : "onesweep", s);
      v.pass(a, p == 0 ? kPassFirst : kPassKey, wide, L.tiles_sort, s);
    }
    // Step 2 flags + prefix sum, Step 3/4 scatters
    FlagScanArgs f{};
    f.bufs = sb;
    f.n = n;
    f.uniq = uniq;
    f.rep = rep;
    f.used_g = used_g;
    f.lookback = scan_lookback;
    f.tile_counter = claimed ? counters + L.P_key : nullptr;
    f.ctl = ctl;
    f.status = status;
    f.tag = uint32_t(L.P_key + 1);
    prof_mark("flag_scan", s);
    v.flag_scan(f, false, L.tiles_scan, s);
    // Step 3 on used groups only: compaction
    CompactArgs c{};
    c.used_g = used_g;
    c.uniq = uniq;
    c.rep = rep;
    c.K = K;
    c.out_vtx = static_cast<uint32_t*>(out_vtx);
    c.new2old = new2old;
    c.cmap = cmap;
    c.out_num = out_num_vtx;
    c.cap = n;
    c.lookback = scan_lookback;
    c.tile_counter = claimed ? counters + L.P_key + 1 : nullptr;
    c.ctl = ctl;
    c.status = status;
    c.tag = uint32_t(L.P_key + 2);
    prof_mark("compact", s);
    hipLaunchKernelGGL((k_compact<kScanBlock, kScanIpt>), dim3(L.tiles_scan), dim3(kScanBlock), 0, s, c);
    if (bp.mode == kMarkAndMap) {
      // Step 4 by vertex bands: the pairs (in the spare buffer) partitioned
      // into the sorted buffer, the index entries' new ids into the spare one
      PairPartArgs pa{};
      pa.cmap = cmap;
      pa.n = n;
      pa.shift = bp.shift;
      pa.nb = bp.nb;
      pa.tiles = bp.ptiles;
      pa.table = ptable;
      pa.status = status;
      pa.sort = sb;
      pa.from_sort = 1;
      prof_mark("pair_partition", s);
      launch_pair_partition(pa, s);
      BandMapArgs ma{};
      ma.ptable = ptable;
      ma.ptiles = bp.ptiles;
      ma.ipart = ipart;
      ma.itable = itable;
      ma.itiles = bp.itiles;
      ma.n = n;
      ma.shift = bp.shift;
      ma.old2new = old2new;
      ma.sort = sb;
      ma.from_sort = 1;
      prof_mark("band_map", s);
      launch_band_map(ma, bp.nb, s);
      BandRemapArgs ra{};
      ra.ipart = ipart;
      ra.tile_valid = itile_valid;
      ra.m = m;
      ra.arity = arity;
      ra.live_elems = live_elems;
      ra.out_idx = out_idx;
      ra.sort = sb;
      ra.from_sort = 1;
      prof_mark("band_remap", s);
      launch_band_remap(ra, bp.itiles, s);
      prof_mark(nullptr, s);
      return check_launch();
    }
    prof_mark("old2new", s);
    hipLaunchKernelGGL((k_scatter_old2new<false>), dim3(rand_grid(n, kScatterItems)), dim3(kRandBlock), 0, s,
                       sb, static_cast<const uint2*>(nullptr), cmap, n, nullptr, nullptr, 0, nullptr, old2new);
  }
  // Step 4: remap the index array
  if (m > 0) {
    prof_mark("remap", s);
    hipLaunchKernelGGL((k_remap<false>), dim3(rand_grid(m)), dim3(kRandBlock), 0, s, idx, m, arity, n,
                       nullptr, nullptr, 0, nullptr, live_elems, old2new, out_idx);
  }
  prof_mark(nullptr, s);
  return check_launch();
}

// The hash-grouping launch sequence of a batch: launch_hash's, with
// vertices told apart by (mesh id, record). The hash digits are those of a
// bucket of the vertex's mesh (each mesh owns a range of buckets, in mesh
// order), so the hash-ordered elements are grouped by mesh; the grouping
// compares (mesh id, record) in LDS and names each group by the sorted
// position of its first copy, which lies in its mesh's vertex range. The
// packed used elements are thus in mesh order, which gives the output
// offsets, and the key sort of the used values adds the mesh-id passes of
// the batched sort-all path (the mesh of an element is that of its name).
// New ids are numbered over the whole batch and made mesh-local by the
// old2new scatter and the new2old pass. A bucket that does not fit makes the
// device sort all N hash-ordered elements by (mesh id, record) instead and
// finish with the batched flags, scans and compaction.
mrx_status launch_batched_hash(const SortVariant& v, const Layout& L, const void* vtx, const int64_t* vtx_offsets,
                               int64_t n, int32_t vtx_bytes, const int32_t* idx, const int64_t* elem_offsets,
                               int64_t total_elems, int32_t arity, int32_t num_meshes, void* out_vtx,
                               int64_t* out_vtx_offsets, int32_t* out_idx, int32_t* old2new, int32_t* new2old,
                               int32_t* dev_status, void* workspace, const mrx_tuning* tuning, void* stream_) {
  const int K = vtx_bytes / 4;
  const int64_t m = total_elems * arity;
  const int ph = L.P_hash;
  const int P = L.P_key + L.P_mesh;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);
  Control* ctl = reinterpret_cast<Control*>(ws + L.ctl);
  uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  uint32_t* plan = reinterpret_cast<uint32_t*>(ws + L.plan);
  uint32_t* hist_hash = reinterpret_cast<uint32_t*>(ws + L.hist_hash);
  uint32_t* plan_hash = reinterpret_cast<uint32_t*>(ws + L.plan_hash);
  uint32_t* dead_hash = reinterpret_cast<uint32_t*>(ws + L.dead_hash);
  uint64_t* lookback = reinterpret_cast<uint64_t*>(ws + L.lookback);
  uint64_t* scan_lookback = reinterpret_cast<uint64_t*>(ws + L.scan_lookback);
  uint4* group_chunks = reinterpret_cast<uint4*>(ws + L.group_chunks);
  uint32_t* group_range_sums = reinterpret_cast<uint32_t*>(ws + L.group_ranges);
  const int64_t group_ranges = group_compact_ranges(L.tiles_group);
  const bool wide = wide_lookback(n, tuning);
  const bool claimed = tuning && (tuning->flags & MRX_TUNING_CLAIMED_TILES);
  uint32_t* const lb32[2] = {reinterpret_cast<uint32_t*>(lookback),
                             reinterpret_cast<uint32_t*>(lookback) + size_t(L.tiles_sort) * v.radix()};
  uint8_t* used_v = reinterpret_cast<uint8_t*>(ws + L.used_v);
  uint8_t* used_g = reinterpret_cast<uint8_t*>(ws + L.used_g);
  uint32_t* buf[3] = {reinterpret_cast<uint32_t*>(ws + L.buf_a), reinterpret_cast<uint32_t*>(ws + L.buf_b),
                      reinterpret_cast<uint32_t*>(ws + L.buf_c)};
  uint32_t* uniq = reinterpret_cast<uint32_t*>(ws + L.uniq);
  int32_t* rep = reinterpret_cast<int32_t*>(ws + L.rep);
  int32_t* cmap = reinterpret_cast<int32_t*>(ws + L.cmap);
  int32_t* vtab = reinterpret_cast<int32_t*>(ws + L.vtx_tab);
  int32_t* etab = L.elem_tab_n ? reinterpret_cast<int32_t*>(ws + L.elem_tab) : nullptr;
  uint2* mbk = reinterpret_cast<uint2*>(ws + L.mesh_bk);
  int32_t* status = dev_status;
  int counter = 0;  // next tile counter (claimed tiles)
  auto next_counter = [&]() { return claimed ? counters + counter++ : nullptr; };

  prof_mark("fill_zero", s);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(int64_t(L.zero_end / 16), 256, 4096)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(ws), int64_t(L.zero_end / 16), dev_status,
                     static_cast<int64_t*>(nullptr), static_cast<int64_t*>(nullptr));
  // n > 0 and num_meshes > 1 here (use_batched_hash)
  prof_mark("mesh_tables", s);
  hipLaunchKernelGGL(k_mesh_table, dim3((L.vtx_tab_n + 255) / 256), dim3(256), 0, s, vtx_offsets, num_meshes, n,
                     vtab, L.vtx_tab_n);
  const int64_t num_e = total_elems;
  if (etab && num_e > 0) {
    const int64_t nq = (num_e - 1) / (int64_t(1) << kMeshTabShift) + 2;  // <= L.elem_tab_n
    hipLaunchKernelGGL(k_mesh_table, dim3((nq + 255) / 256), dim3(256), 0, s, elem_offsets, num_meshes, num_e,
                       etab, nq);
  } else {
    etab = nullptr;
  }
  prof_mark("mesh_buckets", s);
  hipLaunchKernelGGL(k_mesh_buckets, dim3(1), dim3(kMeshBucketBlock), 0, s, vtx_offsets, num_meshes,
                     int32_t(v.group_mesh_target_bucket), mbk);
  // Step 1 (scattered byte stores; reports out-of-range entries) beside the
  // bucket-digit histograms of the stable sort of (record, id | used << 31)
  // by the buckets of (mesh id, record)
  const MarkArgs mark{idx, m, arity, n, vtx_offsets, elem_offsets, num_meshes, etab, nullptr, used_v, status};
  prof_mark(m > 0 ? "mark_histogram" : "hash_histogram", s);
  v.hash_mesh_hist(m > 0 ? &mark : nullptr, static_cast<const uint32_t*>(vtx), n, vtx_offsets, num_meshes, vtab, mbk,
                   ph, hist_hash, s);
  prof_mark("scan_buckets", s);
  v.scan(hist_hash, ph, n, nullptr, dead_hash, s);
  const SortBuffers sbh{{buf[0], buf[1]}, plan_hash, ph};
  int gp = 0;  // index of the pass in the call (look-back buffer parity, tag)
  for (int p = 0; p < ph; ++p, ++gp) {
    SortPassArgs a{};
    a.vtx = static_cast<const uint32_t*>(vtx);
    a.bufs = sbh;
    a.pass = p;
    a.used = used_v;
    a.bucket_base = hist_hash + size_t(p) * v.radix();
    a.lookback = wide ? static_cast<void*>(lookback) : static_cast<void*>(lb32[gp & 1]);
    a.lookback_next = lb32[(gp + 1) & 1];
    a.tile_counter = next_counter();
    a.ctl = ctl;
    a.status = status;
    a.n = n;
    a.mesh_off = vtx_offsets;
    a.mesh_tab = vtab;
    a.mesh_buckets = mbk;
    a.nmesh = num_meshes;
    a.lo_word = a.hi_word = -1;
    a.shift = p * v.D;
    a.tag = uint32_t(gp + 1);
    prof_mark(p == 0 ? "onesweep_hash_first" : "onesweep_hash", s);
    v.pass(a, p == 0 ? kPassFirstHashMesh : kPassHashMesh, wide, L.tiles_sort, s);
  }
  uint32_t* X = buf[(ph - 1) & 1];
  uint32_t* Y = buf[((ph - 1) & 1) ^ 1];
  uint2* pairs = reinterpret_cast<uint2*>(Y);

  // group each bucket by (mesh id, record)
  GroupArgs g{};
  g.elems = X;
  g.n = n;
  g.pairs = pairs;
  g.rep = rep;
  g.cmap = cmap;
  g.uelems = buf[2];
  g.chunks = group_chunks;
  g.range_sums = group_range_sums;
  g.ranges = group_ranges;
  g.status = status;
  g.mesh_off = vtx_offsets;
  g.mesh_tab = vtab;
  g.mesh_buckets = mbk;
  g.nmesh = num_meshes;
  prof_mark("group", s);
  v.group_mesh(g, L.tiles_group, s);

  // key sort of X by (mesh id, record): the used groups' (record, name)
  // elements packed from C in name order (or, on the fallback path, all N
  // hash-ordered (record, id) elements)
  const SortBuffers sbk{{X, buf[2]}, plan, P};
  const GroupCompactArgs gc{buf[2], group_chunks, group_range_sums, L.tiles_group, group_ranges, n, X, hist, ctl};
  prof_mark("compact_histogram", s);
  v.group_compact_hist(gc, s);
  const HistArgs ha{{X, X}, nullptr, n, &ctl->all_count, hist};
  prof_mark("histogram", s);
  v.elem_hist(ha, s);
  prof_mark("batch_offsets", s);
  hipLaunchKernelGGL(k_batch_offsets_dense, dim3((num_meshes + 1 + 255) / 256), dim3(256), 0, s,
                     static_cast<const uint32_t*>(X), int32_t(K + 1), static_cast<const Control*>(ctl), vtx_offsets,
                     num_meshes, out_vtx_offsets);
  prof_mark("mesh_histogram", s);
  v.mesh_hist_path(out_vtx_offsets, vtx_offsets, ctl, num_meshes, L.P_mesh, hist + size_t(L.P_key) * v.radix(), s);
  prof_mark("scan_buckets", s);
  v.scan(hist, P, n, &ctl->sort_count, plan + P + 1, s);
  prof_mark("sort_plan", s);
  hipLaunchKernelGGL(k_group_sort_plan, dim3(1), dim3(64), 0, s, sbk, static_cast<const Control*>(ctl));
  for (int p = 0; p < P; ++p, ++gp) {
    SortPassArgs a{};
    a.bufs = sbk;
    a.pass = p;
    a.bucket_base = hist + size_t(p) * v.radix();
    a.lookback = wide ? static_cast<void*>(lookback) : static_cast<void*>(lb32[gp & 1]);
    a.lookback_next = lb32[(gp + 1) & 1];
    a.tile_counter = next_counter();
    a.ctl = ctl;
    a.status = status;
    a.n = n;
    a.n_dev = &ctl->sort_count;
    a.mesh_off = vtx_offsets;
    a.mesh_tab = vtab;
    a.nmesh = num_meshes;
    a.tag = uint32_t(gp + 1);
    int mode = kPassKey;
    if (p < L.P_key) {
      set_digit(a, K, p * v.D);
    } else {
      a.shift = (p - L.P_key) * v.D;
      mode = kPassMesh;
    }
    prof_mark(mode == kPassMesh ? "onesweep_mesh" : "onesweep", s);
    v.pass(a, mode, wide, L.tiles_sort, s);
  }
  // grouping path: sorted position = new id over the whole batch
  FinalizeArgs fa{};
  fa.bufs = sbk;
  fa.rep = rep;
  fa.cmap = cmap;
  fa.out_vtx = static_cast<uint32_t*>(out_vtx);
  fa.new2old = new2old;
  fa.out_num = nullptr;
  fa.cap = n;
  fa.ctl = ctl;
  fa.status = status;
  prof_mark("finalize", s);
  v.finalize(fa, grid_for(n, 256, 4096), s);
  // fallback path: the batched flags, scans and compaction over all of X
  FlagScanArgs f{};
  f.bufs = sbk;
  f.n = n;
  f.uniq = uniq;
  f.rep = rep;
  f.used_g = used_g;
  f.lookback = scan_lookback;
  f.tile_counter = next_counter();
  f.ctl = ctl;
  f.status = status;
  f.mesh_off = vtx_offsets;
  f.mesh_tab = vtab;
  f.nmesh = num_meshes;
  f.tag = uint32_t(gp + 1);
  f.pairs = pairs;
  f.gate = kGateSortAll;
  prof_mark("flag_scan", s);
  v.flag_scan(f, true, L.tiles_scan, s);
  CompactArgs c{};
  c.used_g = used_g;
  c.uniq = uniq;
  c.rep = rep;
  c.K = K;
  c.out_vtx = static_cast<uint32_t*>(out_vtx);
  c.new2old = new2old;
  c.cmap = cmap;
  c.out_num = &ctl->num_used;
  c.cap = n;
  c.lookback = scan_lookback;
  c.tile_counter = next_counter();
  c.ctl = ctl;
  c.status = status;
  c.tag = uint32_t(gp + 2);
  c.gate = kGateSortAll;
  prof_mark("compact", s);
  hipLaunchKernelGGL((k_compact<kScanBlock, kScanIpt>), dim3(L.tiles_scan), dim3(kScanBlock), 0, s, c);
  prof_mark("batch_offsets", s);
  hipLaunchKernelGGL(k_batch_offsets, dim3((num_meshes + 1 + 255) / 256), dim3(256), 0, s, vtx_offsets, num_meshes,
                     sbk, static_cast<const uint2*>(pairs), static_cast<const int32_t*>(cmap),
                     static_cast<const Control*>(ctl), static_cast<const int64_t*>(&ctl->num_used), n,
                     int32_t(kGateSortAll), out_vtx_offsets);

  // both paths: Step 4's map made mesh-local, new2old made mesh-local, remap
  prof_mark("old2new", s);
  hipLaunchKernelGGL((k_scatter_old2new<true>), dim3(rand_grid(n, kScatterItems)), dim3(kRandBlock), 0, s,
                     SortBuffers{{nullptr, nullptr}, nullptr, 0}, static_cast<const uint2*>(pairs), cmap, n,
                     vtx_offsets, static_cast<const int64_t*>(out_vtx_offsets), num_meshes,
                     static_cast<const int32_t*>(vtab), old2new);
  if (new2old) {
    prof_mark("localize_new2old", s);
    hipLaunchKernelGGL(k_localize_new2old, dim3(grid_for(n, 256)), dim3(256), 0, s, new2old, &ctl->num_used,
                       vtx_offsets, num_meshes, static_cast<const int32_t*>(vtab));
  }
  if (m > 0) {
    prof_mark("remap", s);
    hipLaunchKernelGGL((k_remap<true>), dim3(rand_grid(m)), dim3(kRandBlock), 0, s, idx, m, arity, n, vtx_offsets,
                       elem_offsets, num_meshes, static_cast<const int32_t*>(etab),
                       static_cast<const int64_t*>(nullptr), old2new, out_idx);
  }
  prof_mark(nullptr, s);
  return check_launch();
}

// Device address of `scratch` on the current device, looked up once per
// device (the first call on that device) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

mrx_status scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MRX_ERR_HIP;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MRX_ERR_HIP;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return MRX_OK;
}

}  // namespace
}  // namespace mrx

using namespace mrx;

extern "C" {

int32_t mrx_abi_version(void) { return MRX_ABI_VERSION; }

const char* mrx_status_string(int32_t s) {
  switch (s) {
    case MRX_OK: return "MRX_OK";
    case MRX_ERR_INVALID_ARGUMENT: return "MRX_ERR_INVALID_ARGUMENT";
    case MRX_ERR_WORKSPACE_TOO_SMALL: return "MRX_ERR_WORKSPACE_TOO_SMALL";
    case MRX_ERR_INDEX_OUT_OF_RANGE: return "MRX_ERR_INDEX_OUT_OF_RANGE";
    case MRX_ERR_TOO_LARGE: return "MRX_ERR_TOO_LARGE";
    case MRX_ERR_HIP: return "MRX_ERR_HIP";
    case MRX_ERR_UNSUPPORTED: return "MRX_ERR_UNSUPPORTED";
    case MRX_ERR_INTERNAL: return "MRX_ERR_INTERNAL";
    case MRX_ERR_NOALLOC_TOO_LARGE: return "MRX_ERR_NOALLOC_TOO_LARGE";
    default: return "MRX_UNKNOWN_STATUS";
  }
}

int32_t mrx_tuning_count(int32_t vtx_bytes) {
  if (vtx_bytes < 4 || vtx_bytes > 64 || vtx_bytes % 4) return 0;
  return int32_t(variants_for(vtx_bytes / 4).size());
}

mrx_status mrx_tuning_get(int32_t vtx_bytes, int32_t i, mrx_tuning* out) {
  if (!out || i < 0 || i >= mrx_tuning_count(vtx_bytes)) return MRX_ERR_INVALID_ARGUMENT;
  const SortVariant& v = variants_for(vtx_bytes / 4)[i];
  out->digit_bits = v.D;
  out->block_threads = v.block;
  out->items_per_thread = v.ipt;
  out->flags = 0;
  return MRX_OK;
}

mrx_status mrx_profile_enable(int32_t on) {
  Profiler& p = profiler();
  std::lock_guard<std::mutex> g(p.mu);
  if (on) {
    p.recs.clear();
    p.next = 0;
  }
  p.on = on != 0;
  return MRX_OK;
}

// Named marks, each followed by the mark that ends its kernel.
static std::vector<std::pair<size_t, size_t>> prof_pairs(const Profiler& p) {
  std::vector<std::pair<size_t, size_t>> out;
  for (size_t i = 0; i + 1 < p.recs.size(); ++i)
    if (p.recs[i].name) out.emplace_back(i, i + 1);
  return out;
}

int32_t mrx_profile_count(void) {
  Profiler& p = profiler();
  std::lock_guard<std::mutex> g(p.mu);
  return int32_t(prof_pairs(p).size());
}

mrx_status mrx_profile_get(int32_t i, const char** name, float* ms) {
  Profiler& p = profiler();
  ProfRecord a, b;
  {
    std::lock_guard<std::mutex> g(p.mu);
    const auto pairs = prof_pairs(p);
    if (i < 0 || size_t(i) >= pairs.size() || !ms) return MRX_ERR_INVALID_ARGUMENT;
    a = p.recs[pairs[size_t(i)].first];
    b = p.recs[pairs[size_t(i)].second];
  }
  if (name) *name = a.name;
  if (hipEventSynchronize(b.event) != hipSuccess) return MRX_ERR_HIP;
  return hipEventElapsedTime(ms, a.event, b.event) == hipSuccess ? MRX_OK : MRX_ERR_HIP;
}

mrx_status mrx_reindex_workspace_size(int64_t num_vtx, int32_t vtx_bytes, int64_t num_idx,
                                      int32_t num_meshes, const mrx_tuning* tuning, size_t* bytes) {
  if (!bytes) return MRX_ERR_INVALID_ARGUMENT;
  if (vtx_bytes < 4 || vtx_bytes > 64 || vtx_bytes % 4 != 0) return MRX_ERR_INVALID_ARGUMENT;
  if (num_vtx < 0 || num_idx < 0 || num_meshes < 1) return MRX_ERR_INVALID_ARGUMENT;
  if (num_vtx > kMaxCount || num_idx > kMaxCount) return MRX_ERR_TOO_LARGE;
  const SortVariant* v = pick_variant(vtx_bytes / 4, tuning);
  if (!v) return MRX_ERR_UNSUPPORTED;
  *bytes = make_layout(num_vtx, num_idx, vtx_bytes / 4, num_meshes, *v, tuning).total;
  return MRX_OK;
}


mrx_status mrx_reindex_mesh(const void* vtx, int64_t num_vtx, int32_t vtx_bytes, const int32_t* idx,
                            int64_t num_elems, int32_t arity, void* out_vtx, int32_t* out_idx,
                            int32_t* old2new, int32_t* new2old, int64_t* out_num_vtx,
                            int32_t* dev_status, void* workspace, size_t workspace_bytes,
                            const mrx_tuning* tuning, void* stream) {
  const SortVariant* v = nullptr;
  Layout L;
  mrx_status st = validate_single(vtx, num_vtx, vtx_bytes, idx, num_elems, arity, out_vtx, out_idx, old2new,
                                  new2old, out_num_vtx, dev_status, workspace, workspace_bytes, tuning, {},
                                  &v, &L);
  if (st != MRX_OK) return st;
  return launch_single(*v, L, vtx, num_vtx, vtx_bytes, idx, num_elems, arity, nullptr, out_vtx, out_idx,
                       old2new, new2old, out_num_vtx, dev_status, workspace, tuning, stream);
}

mrx_status mrx_reindex_mesh_noalloc(const void* vtx, int64_t num_vtx, int32_t vtx_bytes, const int32_t* idx,
                                    int64_t num_elems, int32_t arity, void* out_vtx, int32_t* out_idx,
                                    int32_t* old2new, int32_t* new2old, int64_t* out_num_vtx,
                                    int32_t* dev_status, const mrx_tuning* tuning, void* stream) {
  // the stream must belong to the current device: its kernels get that
  // device's copy of the array
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return MRX_ERR_HIP;
  if (stream) {
    hipDevice_t sd = -1;
    if (hipStreamGetDevice(reinterpret_cast<hipStream_t>(stream), &sd) != hipSuccess) return MRX_ERR_HIP;
    if (int(sd) != cur) return MRX_ERR_INVALID_ARGUMENT;
  }
  void* ws = nullptr;
  mrx_status st = scratch_of_current_device(&ws);
  if (st != MRX_OK) return st;
  const SortVariant* v = nullptr;
  Layout L;
  st = validate_single(vtx, num_vtx, vtx_bytes, idx, num_elems, arity, out_vtx, out_idx, old2new, new2old,
                       out_num_vtx, dev_status, ws, MRX_NOALLOC_SCRATCH_BYTES, tuning, {}, &v, &L);
  if (st == MRX_ERR_WORKSPACE_TOO_SMALL) return MRX_ERR_NOALLOC_TOO_LARGE;
  if (st != MRX_OK) return st;
  return launch_single(*v, L, vtx, num_vtx, vtx_bytes, idx, num_elems, arity, nullptr, out_vtx, out_idx,
                       old2new, new2old, out_num_vtx, dev_status, ws, tuning, stream);
}

mrx_status mrx_reindex_mesh_batched(const void* vtx, const int64_t* vtx_offsets, int64_t total_vtx,
                                    int32_t vtx_bytes, const int32_t* idx, const int64_t* elem_offsets,
                                    int64_t total_elems, int32_t arity, int32_t num_meshes,
                                    void* out_vtx, int64_t* out_vtx_offsets, int32_t* out_idx,
                                    int32_t* old2new, int32_t* new2old, int32_t* dev_status,
                                    void* workspace, size_t workspace_bytes,
                                    const mrx_tuning* tuning, void* stream_) {
  mrx_status st = validate_common(vtx, total_vtx, vtx_bytes, idx, total_elems, arity, out_vtx, out_idx,
                                  old2new, workspace, workspace_bytes);
  if (st != MRX_OK) return st;
  if (num_meshes < 1 || !vtx_offsets || !elem_offsets || !out_vtx_offsets ||
      !aligned(vtx_offsets, 8) || !aligned(elem_offsets, 8) || !aligned(out_vtx_offsets, 8) ||
      !aligned(new2old, 4) || !dev_status || !aligned(dev_status, 4))
    return MRX_ERR_INVALID_ARGUMENT;
  const int K = vtx_bytes / 4;
  const SortVariant* vp = pick_variant(K, tuning);
  if (!vp) return MRX_ERR_UNSUPPORTED;
  const SortVariant& v = *vp;
  const int64_t n = total_vtx, m = total_elems * arity;
  const Layout L = make_layout(n, m, K, num_meshes, v, tuning);
  if (workspace_bytes < L.total) return MRX_ERR_WORKSPACE_TOO_SMALL;
  const size_t vb = size_t(n) * vtx_bytes, ib = size_t(m) * 4, nb = size_t(n) * 4,
               ob = size_t(num_meshes + 1) * 8;
  if (!disjoint({{vtx, vb}, {out_vtx, vb}, {old2new, nb}, {new2old, new2old ? nb : 0},
                 {out_vtx_offsets, ob}, {dev_status, 4u}, {workspace, L.total},
                 {vtx_offsets, ob}, {elem_offsets, ob}, {idx == out_idx ? nullptr : idx, ib}}) ||
      !disjoint({{out_idx, ib}, {vtx, vb}, {out_vtx, vb}, {old2new, nb}, {new2old, new2old ? nb : 0},
                 {out_vtx_offsets, ob}, {dev_status, 4u}, {workspace, L.total},
                 {vtx_offsets, ob}, {elem_offsets, ob}}) ||
      (idx != out_idx && overlaps(idx, ib, out_idx, ib)))  // in place, or not at all
    return MRX_ERR_INVALID_ARGUMENT;

  if (L.mesh_hash)
    return launch_batched_hash(v, L, vtx, vtx_offsets, n, vtx_bytes, idx, elem_offsets, total_elems, arity,
                               num_meshes, out_vtx, out_vtx_offsets, out_idx, old2new, new2old, dev_status,
                               workspace, tuning, stream_);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
  char* ws = static_cast<char*>(workspace);
  Control* ctl = reinterpret_cast<Control*>(ws + L.ctl);
  uint32_t* counters = reinterpret_cast<uint32_t*>(ws + L.counters);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
  uint32_t* plan = reinterpret_cast<uint32_t*>(ws + L.plan);
  uint64_t* lookback = reinterpret_cast<uint64_t*>(ws + L.lookback);
  uint64_t* scan_lookback = reinterpret_cast<uint64_t*>(ws + L.scan_lookback);
  const bool wide = wide_lookback(n, tuning);
  const bool claimed = tuning && (tuning->flags & MRX_TUNING_CLAIMED_TILES);
  uint32_t* const lb32[2] = {reinterpret_cast<uint32_t*>(lookback),
                             reinterpret_cast<uint32_t*>(lookback) + size_t(L.tiles_sort) * v.radix()};
  uint8_t* used_v = reinterpret_cast<uint8_t*>(ws + L.used_v);
  uint8_t* used_g = reinterpret_cast<uint8_t*>(ws + L.used_g);
  uint32_t* buf[2] = {reinterpret_cast<uint32_t*>(ws + L.buf_a), reinterpret_cast<uint32_t*>(ws + L.buf_b)};
  uint32_t* uniq = reinterpret_cast<uint32_t*>(ws + L.uniq);
  int32_t* rep = reinterpret_cast<int32_t*>(ws + L.rep);
  int32_t* cmap = reinterpret_cast<int32_t*>(ws + L.cmap);
  int32_t* status = dev_status;
  const int P = L.P_key + L.P_mesh;
  int32_t* vtab = L.vtx_tab_n ? reinterpret_cast<int32_t*>(ws + L.vtx_tab) : nullptr;
  int32_t* etab = L.elem_tab_n ? reinterpret_cast<int32_t*>(ws + L.elem_tab) : nullptr;

  prof_mark("fill_zero", s);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(int64_t(L.zero_end / 16), 256, 4096)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(ws), int64_t(L.zero_end / 16), dev_status,
                     static_cast<int64_t*>(nullptr), static_cast<int64_t*>(nullptr));
  const int64_t num_e = total_elems;
  if (vtab && n > 0) {
    prof_mark("mesh_tables", s);
    hipLaunchKernelGGL(k_mesh_table, dim3((L.vtx_tab_n + 255) / 256), dim3(256), 0, s, vtx_offsets, num_meshes,
                       n, vtab, L.vtx_tab_n);
  } else {
    vtab = nullptr;
  }
  if (etab && num_e > 0) {
    const int64_t nq = (num_e - 1) / (int64_t(1) << kMeshTabShift) + 2;  // <= L.elem_tab_n
    hipLaunchKernelGGL(k_mesh_table, dim3((nq + 255) / 256), dim3(256), 0, s, elem_offsets, num_meshes, num_e,
                       etab, nq);
  } else {
    etab = nullptr;
  }
  const MarkArgs mark{idx, m, arity, n, vtx_offsets, elem_offsets, num_meshes, etab, nullptr, used_v, status};
  const bool fused = v.mark_hist_applies(n, m);
  if (fused) {
    prof_mark("mark_histogram", s);
    v.mark_hist(mark, true, static_cast<const uint32_t*>(vtx), n, hist, s);
  } else if (m > 0) {
    prof_mark("mark_used", s);
    hipLaunchKernelGGL((k_mark_used<true>), dim3(rand_grid(m)), dim3(kRandBlock), 0, s, mark);
  }
  if (n > 0) {
    if (!fused) {
      prof_mark("histogram", s);
      v.hist(static_cast<const uint32_t*>(vtx), n, hist, s);
    }
    prof_mark("mesh_histogram", s);
    v.mesh_hist(vtx_offsets, num_meshes, L.P_mesh, hist + size_t(L.P_key) * v.radix(), s);
    prof_mark("scan_buckets", s);
    v.scan(hist, P, n, nullptr, plan + P + 1, s);
    const SortBuffers sb{{buf[0], buf[1]}, plan, P};
    for (int p = 0; p < P; ++p) {
      SortPassArgs a{};
      a.vtx = static_cast<const uint32_t*>(vtx);
      a.bufs = sb;
      a.pass = p;
      a.used = used_v;
      a.bucket_base = hist + size_t(p) * v.radix();
      a.lookback = wide ? static_cast<void*>(lookback) : static_cast<void*>(lb32[p & 1]);
      a.lookback_next = lb32[(p + 1) & 1];
      a.tile_counter = claimed ? counters + p : nullptr;
      a.ctl = ctl;
      a.status = status;
      a.n = n;
      a.mesh_off = vtx_offsets;
      a.mesh_tab = vtab;
      a.nmesh = num_meshes;
      a.tag = uint32_t(p + 1);
      int mode = kPassKey;
      if (p < L.P_key) {
        set_digit(a, K, p * v.D);
        if (p == 0) mode = kPassFirst;
      } else {
        a.shift = (p - L.P_key) * v.D;
        mode = kPassMesh;
      }
      prof_mark(mode == kPassFirst ? "onesweep_first" : mode == kPassMesh ? "onesweep_mesh" : "onesweep", s);
      v.pass(a, mode, wide, L.tiles_sort, s);
    }
    FlagScanArgs f{};
    f.bufs = sb;
    f.n = n;
    f.uniq = uniq;
    f.rep = rep;
    f.used_g = used_g;
    f.lookback = scan_lookback;
    f.tile_counter = claimed ? counters + P : nullptr;
    f.ctl = ctl;
    f.status = status;
    f.mesh_off = vtx_offsets;
    f.mesh_tab = vtab;
    f.nmesh = num_meshes;
    f.tag = uint32_t(P + 1);
    prof_mark("flag_scan", s);
    v.flag_scan(f, true, L.tiles_scan, s);
    CompactArgs c{};
    c.used_g = used_g;
    c.uniq = uniq;
    c.rep = rep;
    c.K = K;
    c.out_vtx = static_cast<uint32_t*>(out_vtx);
    c.new2old = new2old;
    c.cmap = cmap;
    c.out_num = &ctl->num_used;
    c.cap = n;
    c.lookback = scan_lookback;
    c.tile_counter = claimed ? counters + P + 1 : nullptr;
    c.ctl = ctl;
    c.status = status;
    c.tag = uint32_t(P + 2);
    prof_mark("compact", s);
    hipLaunchKernelGGL((k_compact<kScanBlock, kScanIpt>), dim3(L.tiles_scan), dim3(kScanBlock), 0, s, c);
    prof_mark("batch_offsets", s);
    hipLaunchKernelGGL(k_batch_offsets, dim3((num_meshes + 1 + 255) / 256), dim3(256), 0, s, vtx_offsets,
                       num_meshes, sb, static_cast<const uint2*>(nullptr), static_cast<const int32_t*>(cmap),
                       static_cast<const Control*>(ctl), static_cast<const int64_t*>(&ctl->num_used), n,
                       int32_t(kGateAlways), out_vtx_offsets);
    prof_mark("old2new", s);
    hipLaunchKernelGGL((k_scatter_old2new<true>), dim3(rand_grid(n, kScatterItems)), dim3(kRandBlock), 0, s,
                       sb, static_cast<const uint2*>(nullptr), cmap, n, vtx_offsets, out_vtx_offsets, num_meshes,
                       static_cast<const int32_t*>(vtab), old2new);
    if (new2old) {
      prof_mark("localize_new2old", s);
      hipLaunchKernelGGL(k_localize_new2old, dim3(grid_for(n, 256)), dim3(256), 0, s, new2old,
                         &ctl->num_used, vtx_offsets, num_meshes, static_cast<const int32_t*>(vtab));
    }
  } else {
    prof_mark("batch_offsets", s);
    hipLaunchKernelGGL(k_batch_offsets, dim3((num_meshes + 1 + 255) / 256), dim3(256), 0, s, vtx_offsets,
                       num_meshes, SortBuffers{{nullptr, nullptr}, nullptr, 0}, static_cast<const uint2*>(nullptr),
                       static_cast<const int32_t*>(cmap), static_cast<const Control*>(ctl),
                       static_cast<const int64_t*>(&ctl->num_used), n, int32_t(kGateAlways), out_vtx_offsets);
  }
  if (m > 0) {
    prof_mark("remap", s);
    hipLaunchKernelGGL((k_remap<true>), dim3(rand_grid(m)), dim3(kRandBlock), 0, s, idx, m, arity, n,
                       vtx_offsets, elem_offsets, num_meshes, static_cast<const int32_t*>(etab),
                       static_cast<const int64_t*>(nullptr), old2new, out_idx);
  }
  prof_mark(nullptr, s);
  return check_launch();
}

mrx_status mrx_merge_meshes(const void* vtx, const int64_t* vtx_offsets, int64_t total_vtx, int32_t vtx_bytes,
                            const int32_t* idx, const int64_t* elem_offsets, int64_t total_elems,
                            int32_t arity, int32_t num_meshes, void* out_vtx, int32_t* out_idx,
                            int32_t* old2new, int32_t* new2old, int64_t* out_num_vtx, int32_t* dev_status,
                            void* workspace, size_t workspace_bytes, const mrx_tuning* tuning,
                            void* stream) {
  if (num_meshes < 1 || !vtx_offsets || !elem_offsets || !aligned(vtx_offsets, 8) ||
      !aligned(elem_offsets, 8))
    return MRX_ERR_INVALID_ARGUMENT;
  const size_t ob = sizeof(int64_t) * (size_t(num_meshes) + 1);
  const SortVariant* v = nullptr;
  Layout L;
  mrx_status st = validate_single(vtx, total_vtx, vtx_bytes, idx, total_elems, arity, out_vtx, out_idx,
                                  old2new, new2old, out_num_vtx, dev_status, workspace, workspace_bytes,
                                  tuning, {{vtx_offsets, ob}, {elem_offsets, ob}}, &v, &L);
  if (st != MRX_OK) return st;
  // the offsets must not overlap each other either
  if (overlaps(vtx_offsets, ob, elem_offsets, ob)) return MRX_ERR_INVALID_ARGUMENT;
  const int64_t m = total_elems * arity;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (m > 0) {
    int32_t* etab = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + L.elem_tab);
    const int64_t nq = (total_elems - 1) / (int64_t(1) << kMeshTabShift) + 2;  // <= L.elem_tab_n
    prof_mark("mesh_tables", s);
    hipLaunchKernelGGL(k_mesh_table, dim3((nq + 255) / 256), dim3(256), 0, s, elem_offsets, num_meshes,
                       total_elems, etab, nq);
    prof_mark("offset_indices", s);
    hipLaunchKernelGGL(k_offset_indices, dim3((m + 255) / 256), dim3(256), 0, s, idx, m, arity, vtx_offsets,
                       elem_offsets, num_meshes, static_cast<const int32_t*>(etab), out_idx);
  }
  return launch_single(*v, L, vtx, total_vtx, vtx_bytes, out_idx, total_elems, arity, nullptr, out_vtx,
                       out_idx, old2new, new2old, out_num_vtx, dev_status, workspace, tuning, stream);
}

mrx_status mrx_extract_submesh(const void* vtx, int64_t num_vtx, int32_t vtx_bytes, const int32_t* idx,
                               int64_t num_elems, int32_t arity, const uint8_t* keep, void* out_vtx,
                               int32_t* out_idx, int64_t* out_num_elems, int32_t* old2new, int32_t* new2old,
                               int64_t* out_num_vtx, int32_t* dev_status, void* workspace,
                               size_t workspace_bytes, const mrx_tuning* tuning, void* stream) {
  if (!out_num_elems || !aligned(out_num_elems, 8)) return MRX_ERR_INVALID_ARGUMENT;
  if (num_elems > 0 && (!keep || idx == out_idx)) return MRX_ERR_INVALID_ARGUMENT;
  const SortVariant* v = nullptr;
  Layout L;
  mrx_status st = validate_single(vtx, num_vtx, vtx_bytes, idx, num_elems, arity, out_vtx, out_idx, old2new,
                                  new2old, out_num_vtx, dev_status, workspace, workspace_bytes, tuning,
                                  {{keep, size_t(num_elems)}, {out_num_elems, 8}}, &v, &L);
  if (st != MRX_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  Control* ctl = reinterpret_cast<Control*>(ws + L.ctl);
  // per-call state for the selection and the re-index that follows it
  prof_mark("fill_zero", s);
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(int64_t(L.zero_end / 16), 256, 4096)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(ws), int64_t(L.zero_end / 16), dev_status, out_num_vtx,
                     out_num_elems);
  if (num_elems > 0) {
    SelectArgs a{};
    a.keep = keep;
    a.idx = idx;
    a.num_elems = num_elems;
    a.arity = arity;
    a.out = out_idx;
    a.out_count = out_num_elems;
    a.lookback = reinterpret_cast<uint64_t*>(ws + L.elem_lookback);
    a.tile_counter = (tuning && (tuning->flags & MRX_TUNING_CLAIMED_TILES))
                         ? reinterpret_cast<uint32_t*>(ws + L.counters) + L.P_key + L.P_mesh + L.P_hash + 7
                         : nullptr;
    a.ctl = ctl;
    a.status = dev_status;
    a.tag = 1;
    const int64_t tiles = (num_elems + kSelectTile - 1) / kSelectTile;
    prof_mark("select_elements", s);
    hipLaunchKernelGGL((k_select_elements<kSelectBlock, kSelectIpt>), dim3(tiles), dim3(kSelectBlock), 0, s, a);
  }
  return launch_single(*v, L, vtx, num_vtx, vtx_bytes, out_idx, num_elems, arity, out_num_elems, out_vtx,
                       out_idx, old2new, new2old, out_num_vtx, dev_status, workspace, tuning, stream,
                       /*state_zeroed=*/true);
}

}  // extern "C"
