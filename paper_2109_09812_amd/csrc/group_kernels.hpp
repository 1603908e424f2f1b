// Hash grouping: duplicate detection (Section 2, Steps 2-3) without sorting
// every vertex by its full key.
//
// Section 2 finds duplicates by sorting all N (record, id) pairs by the full
// record; the sort is the dominant cost. Grouping only needs equal records
// to be adjacent, so here the N pairs are first sorted by a few hash digits
// of the record (stable, so within a bucket of equal hash digits ids stay
// ascending). Equal records share their hash, so every group of duplicates
// lies inside one bucket, and buckets are small enough (a few hundred
// records) to be grouped in LDS: k_group numbers the groups of each bucket in
// order of their first copy, which is the smallest original id (Step 2's
// representative rule), and emits one element per *used* group. Only those U
// elements are then sorted by their full key (Step 3's output order), a
// fraction of the N the plain method sorts.
//
// A group is named by a position: each workgroup owns the buckets that start
// in its chunk, i.e. a span of sorted positions disjoint from every other
// chunk's, and its k-th group (in order of first copy) is called span start +
// k, its k-th used group's element goes to slot span start + k of the
// element buffer. Names stay below N and need no count of earlier chunks, so
// the chunks never wait for each other; the chunks' counts go to per-run
// sums, and k_group_compact_hist adds those up and packs the used groups'
// elements densely while counting their key digits.
//
// A batch groups by (mesh id, record): every mesh owns a range of buckets,
// so its vertices end up at the sorted positions of its own vertex range,
// and a group is named by the position of its first copy instead, which
// lies in that range (the name tells the group's mesh).
//
// A bucket that does not fit the LDS window (many copies of one value, or an
// unlucky hash) makes the call take the plain path instead: the same key
// sort then runs on all N hash-ordered elements, followed by Section 2's
// run-head flags and scans. Both paths give the identical result; which one
// runs is decided on the device (Control::path).
#pragma once

#include "device_common.hpp"
#include "sort_kernels.hpp"

namespace mrx {

// Shape of the grouping kernel for K-word records: a workgroup owns the
// buckets that start inside its chunk of CHUNK sorted positions and reads a
// window of WIN positions (the one before the chunk, the chunk, and room for
// its last bucket to end) into LDS.
template <int K>
struct GroupShape {
  static constexpr int S = K + 1;
  static constexpr int BLOCK = 512;
  static constexpr int WIN = S <= 4 ? 3072 : S <= 6 ? 2048 : S <= 9 ? 1024 : 512;
  static constexpr int CHUNK = WIN * 2 / 3;
  static constexpr int IPT = WIN / BLOCK;
  // open-addressing table of at least 4/3 WIN slots (a window holds at most
  // WIN - 2 distinct records, so probing always meets an empty slot)
  static constexpr int TB = WIN > 2048 ? 12 : WIN > 1024 ? 12 : WIN > 512 ? 11 : 10;
  static constexpr int TS = 1 << TB;
  // average bucket size the host aims for when it picks the hash passes
  static constexpr int TARGET_BUCKET = CHUNK / 4;
  // waves per SIMD the register budget is set for: three workgroups per CU
  // (LDS: keys of the window + the table, at most 53 KB each)
  static constexpr int MIN_WAVES_PER_SIMD = 3 * (BLOCK / 64) / 4;
  static_assert(WIN % BLOCK == 0, "window positions per thread");
  static_assert(TS * 3 >= WIN * 4, "table load");
};

// Per-chunk record of k_group: span start, used groups, groups, 1 if the
// chunk's last bucket did not fit the window.
struct GroupArgs {
  const uint32_t* elems;   // [n][K+1] elements in (hash bucket, id) order
  int64_t n;
  uint32_t bucket_mask;    // bucket of a record = hash & bucket_mask
  uint2* pairs;            // [n] (group name, original id) per position
  int32_t* rep;            // [n] smallest original id of each group, by name
  int32_t* cmap;           // [n] -1 for unused groups (used ones are set by the key sort's finalisation)
  uint32_t* uelems;        // [n][K+1] (record, group name) of every used group, in its span's slots
  uint4* chunks;           // [chunks] (span start, used groups, groups, overflow)
  uint32_t* range_sums;    // [3][ranges] zeroed: used groups, groups and overflow of each run of
                           // chunks k_group_compact_hist takes (spread over many addresses: atomics
                           // on one address from every chunk would serialise)
  int64_t ranges;          // that kernel's grid (group_compact_ranges)
  int32_t* status;
  // batches (k_group<K, true>): vertex offsets [nmesh+1] and their bucket
  // table; the grouping key is then (mesh id, record)
  const int64_t* mesh_off;
  const int32_t* mesh_tab;
  const uint2* mesh_buckets;  // each mesh's hash buckets (mesh_bucket)
  int32_t nmesh;
};

// Runs of consecutive chunks, one per workgroup of k_group_compact_hist: few
// (each flushes its digit histograms once), each of at most kCompactMaxChunks.
constexpr int kCompactMaxChunks = 2048;
constexpr int64_t kCompactMinRanges = 512;
__host__ __device__ inline int64_t group_compact_ranges(int64_t tiles) {
  const int64_t by_size = (tiles + kCompactMaxChunks - 1) / kCompactMaxChunks;
  return tiles < kCompactMinRanges ? tiles : (by_size > kCompactMinRanges ? by_size : kCompactMinRanges);
}
// First chunk of run w (of `ranges` runs over `tiles` chunks).
__host__ __device__ inline int64_t group_range_start(int64_t w, int64_t tiles, int64_t ranges) {
  return w * tiles / ranges;
}

template <int K>
__device__ __forceinline__ bool lds_keys_equal(const uint32_t* s_keys, int a, int b, int win) {
  bool eq = true;
#pragma unroll
  for (int w = 0; w < K; ++w) eq = eq && (s_keys[w * win + a] == s_keys[w * win + b]);
  return eq;
}

// MESH (batches): the elements are (record, id) as always, but records are
// told apart by (mesh of id, record): the key held in LDS, hashed and
// compared is KW = K + 1 words with the mesh id first, and the shape is that
// of KW-word records. Each mesh's vertices then occupy its own vertex range
// of sorted positions (its buckets come after those of the meshes before
// it), and a group is named by the sorted position of its first copy, which
// lies in that range: the mesh of a group is the mesh of its name.
// Waves per SIMD the grouping kernel's registers are budgeted for: the
// shape's, except for batches of 1- and 2-word records, whose mesh-id key
// word and lookups would otherwise spill to scratch at that budget.
template <int K, bool MESH>
constexpr int group_min_waves() {
  return MESH && K <= 2 ? GroupShape<K + 1>::MIN_WAVES_PER_SIMD - 1
                        : GroupShape<MESH ? K + 1 : K>::MIN_WAVES_PER_SIMD;
}

template <int K, bool MESH>
__global__ __launch_bounds__(GroupShape<MESH ? K + 1 : K>::BLOCK, (group_min_waves<K, MESH>())) void k_group(
    GroupArgs a) {
  constexpr int KW = MESH ? K + 1 : K;  // key words
  using SH = GroupShape<KW>;
  constexpr int S = K + 1;              // words of an input element
  constexpr int KO = MESH ? 1 : 0;      // first record word of a key
  constexpr int BLOCK = SH::BLOCK, WIN = SH::WIN, CHUNK = SH::CHUNK, IPT = SH::IPT;
  constexpr int TS = SH::TS, TB = SH::TB;
  constexpr int WAVES = BLOCK / kWave;
  constexpr uint32_t kEmpty = 0xFFFFFFFFu;
  constexpr uint32_t kUsedBit = 0x80000000u;
  constexpr int kScratch = WIN > TS ? WIN : TS;

  __shared__ uint32_t s_keys[KW * WIN];     // window keys, word-major
  __shared__ uint32_t s_scratch[kScratch];  // buckets of the window, then the table
  __shared__ uint32_t s_cnt[2][IPT][WAVES];
  __shared__ uint32_t s_sq, s_eq;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int64_t n = a.n;
  if (tid == 0) {
    s_sq = WIN;
    s_eq = WIN;
  }
  const uint32_t tile = blockIdx.x;
  const int64_t c0 = int64_t(tile) * CHUNK;
  const int64_t c1 = min(n, c0 + CHUNK);
  const int qc1 = int(c1 - c0) + 1;  // window slot of position c1

  // ---- window: positions c0 - 1 + q, q in [0, WIN). Each thread keeps, for
  // its own slots, the id (bit 31: referenced) and, until the table is
  // built, the record's hash in `slot`; everything else lives in LDS, so
  // that three workgroups fit on a CU.
  uint32_t ids[IPT], slot[IPT];
  // batches: mesh b's elements sit at sorted positions [mesh_off[b],
  // mesh_off[b+1]) (its buckets follow those of the meshes before it), so a
  // window inside one mesh needs one lookup, and otherwise a position's mesh
  // is looked up instead of its id's
  uint32_t win_mesh[2] = {0u, 1u};
  if constexpr (MESH) {
    const int64_t p0 = max(c0 - 1, int64_t(0)), p1 = min(c0 - 1 + WIN, n) - 1;
    if (p0 <= p1) {
      win_mesh[0] = __builtin_amdgcn_readfirstlane(mesh_of(a.mesh_off, a.nmesh, p0, a.mesh_tab));
      win_mesh[1] = __builtin_amdgcn_readfirstlane(mesh_of(a.mesh_off, a.nmesh, p1, a.mesh_tab));
    }
  }
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int q = i * BLOCK + tid;
    const int64_t pos = c0 - 1 + q;
    uint32_t e[S];
    if (pos >= 0 && pos < n) {
      load_words<S>(a.elems + pos * S, e);
    } else {
#pragma unroll
      for (int w = 0; w < S; ++w) e[w] = 0u;
    }
    uint32_t key[KW];
    if constexpr (MESH) {
      key[0] = (pos < 0 || pos >= n)            ? 0u
               : win_mesh[0] == win_mesh[1] ? win_mesh[0]
                                            : mesh_of(a.mesh_off, a.nmesh, pos, a.mesh_tab);
#pragma unroll
      for (int w = 0; w < K; ++w) key[w + 1] = e[w];
    } else {
#pragma unroll
      for (int w = 0; w < K; ++w) key[w] = e[w];
    }
#pragma unroll
    for (int w = 0; w < KW; ++w) s_keys[w * WIN + q] = key[w];
    ids[i] = e[K];
    slot[i] = hash_words<KW>(key);
    if constexpr (MESH)
      s_scratch[q] = mesh_bucket(a.mesh_buckets, key[0], slot[i]);
    else
      s_scratch[q] = slot[i] & a.bucket_mask;
  }
  __syncthreads();

  // ---- bucket starts: the first in the chunk (sq) and the first at or after
  // position c1 (eq; position n counts as one)
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int q = i * BLOCK + tid;
    const int64_t pos = c0 - 1 + q;
    if (q == 0 || pos > n) continue;
    const bool start = pos == 0 || pos == n || s_scratch[q] != s_scratch[q - 1];
    if (!start) continue;
    if (q < qc1) atomicMin(&s_sq, uint32_t(q));
    else atomicMin(&s_eq, uint32_t(q));
  }
  __syncthreads();
  const int sq = int(s_sq), eq = int(s_eq);
  const bool owns = sq < qc1;
  const bool over = owns && eq >= WIN;  // the chunk's last bucket runs past the window
  const bool active = owns && !over;
  for (int i = tid; i < TS; i += BLOCK) s_scratch[i] = kEmpty;  // buckets are no longer needed
  __syncthreads();

  // ---- one table entry per distinct record of the owned span [sq, eq):
  // the smallest window slot holding it (its first copy), bit 31 = used
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int q = i * BLOCK + tid;
    const uint32_t h = slot[i];
    slot[i] = kEmpty;
    if (!active || q < sq || q >= eq) continue;
    uint32_t sl = (h * 0x9E3779B1u) >> (32 - TB);
    for (int probe = 0; probe < TS; ++probe) {
      uint32_t cur = s_scratch[sl];
      if (cur == kEmpty) {
        cur = atomicCAS(&s_scratch[sl], kEmpty, uint32_t(q));
        if (cur == kEmpty) {
          slot[i] = sl;
          break;
        }
      }
      if (lds_keys_equal<KW>(s_keys, int(cur & 0xFFFFu), q, WIN)) {
        atomicMin(&s_scratch[sl], uint32_t(q));
        slot[i] = sl;
        break;
      }
      sl = (sl + 1) & (TS - 1);
    }
  }
  __syncthreads();
  uint32_t headm = 0;  // bit i: slot i of this thread holds its group's first copy
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int q = i * BLOCK + tid;
    if (slot[i] == kEmpty) continue;
    if ((s_scratch[slot[i]] & 0xFFFFu) == uint32_t(q)) headm |= 1u << i;
    if (ids[i] & kUsedBit) atomicOr(&s_scratch[slot[i]], kUsedBit);
  }
  __syncthreads();

  // ---- number the groups (and the used ones) in window order: slot q =
  // i * BLOCK + tid, so round i of every wave precedes round i + 1
  uint32_t uheadm = 0;  // bit i: a head whose group is used
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const bool h = (headm >> i) & 1u;
    const bool uh = h && (s_scratch[slot[i]] & kUsedBit) != 0u;
    uheadm |= uh ? (1u << i) : 0u;
    const uint64_t hm = ballot(h);
    const uint64_t um = ballot(uh);
    if (lane == 0) {
      s_cnt[0][i][wave] = uint32_t(popc64(hm));
      s_cnt[1][i][wave] = uint32_t(popc64(um));
    }
  }
  __syncthreads();
  uint32_t gt = 0, ut = 0;  // totals of the window
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    uint32_t gb = gt, ub = ut;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t cg = s_cnt[0][i][w], cu = s_cnt[1][i][w];
      if (w < wave) {
        gb += cg;
        ub += cu;
      }
      gt += cg;
      ut += cu;
    }
    const bool h = (headm >> i) & 1u;
    const uint64_t hm = ballot(h);
    const uint64_t um = ballot((uheadm >> i) & 1u);
    gb += uint32_t(popc64(hm & lanemask_lt()));
    ub += uint32_t(popc64(um & lanemask_lt()));
    // heads leave their group's rank (batches: their window slot) in the low
    // half and their used rank in the high half of the table entry for the
    // other copies; both are below WIN <= 2^16
    const uint32_t q = uint32_t(i * BLOCK + tid);
    if (h) s_scratch[slot[i]] = (MESH ? q : gb) | (ub << 16);
  }

  // ---- the chunk's record and its share of its run's sums; names start at
  // the span's first position (batches: the first copy's position)
  const uint32_t span0 = owns ? uint32_t(c0 - 1 + sq) : 0u;
  if (tid == 0) {
    const uint32_t u_own = active ? ut : 0u, g_own = active ? gt : 0u;
    a.chunks[tile] = make_uint4(span0, u_own, g_own, over ? 1u : 0u);
    // run of this chunk: the last w whose first chunk is at most `tile`
    const int64_t T = int64_t(gridDim.x);
    int64_t w = int64_t(tile) * a.ranges / T;
    while (w + 1 < a.ranges && group_range_start(w + 1, T, a.ranges) <= tile) ++w;
    while (w > 0 && group_range_start(w, T, a.ranges) > tile) --w;
    if (u_own) atomicAdd(&a.range_sums[w], u_own);
    if (g_own) atomicAdd(&a.range_sums[a.ranges + w], g_own);
    if (over) atomicOr(&a.range_sums[2 * a.ranges + w], 1u);
  }
  __syncthreads();  // the ranks the heads left in the table are read below
  if (!active) return;
  const uint32_t gpre = span0, upre = span0;

  // ---- outputs of the owned span
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    if (slot[i] == kEmpty) continue;
    const int q = i * BLOCK + tid;
    const int64_t pos = c0 - 1 + q;
    const uint32_t ranks = s_scratch[slot[i]];
    const uint32_t g = MESH ? uint32_t(c0 - 1) + (ranks & 0xFFFFu) : gpre + (ranks & 0xFFFFu);
    const uint32_t org = ids[i] & 0x7FFFFFFFu;
    if (int64_t(g) >= n || pos < 0 || pos >= n) {  // only after a failed wait
      atomicMax(a.status, 7 /* MRX_ERR_INTERNAL */);
      continue;
    }
    a.pairs[pos] = make_uint2(g, org);
    if (!((headm >> i) & 1u)) continue;
    a.rep[g] = int32_t(org);
    if ((uheadm >> i) & 1u) {
      const uint32_t u = upre + (ranks >> 16);
      if (int64_t(u) >= n) {
        atomicMax(a.status, 7 /* MRX_ERR_INTERNAL */);
        continue;
      }
      uint32_t e[S];
#pragma unroll
      for (int w = 0; w < K; ++w) e[w] = s_keys[(w + KO) * WIN + q];
      e[K] = g;
      store_words<S>(a.uelems + int64_t(u) * S, e);
    } else {
      a.cmap[g] = -1;
    }
  }
}

// Totals of the grouping (every workgroup adds up the runs' sums; workgroup 0
// stores them: U, G, Control::path = some bucket did not fit, and the
// element counts of the key sort). Then, on the grouping path, packs the used
// groups' elements (slots span start + k of each chunk) densely into `dense`
// at the chunk's used-group offset, and adds every key digit of them to the
// LDS histograms (flushed once per workgroup). A workgroup takes a run of consecutive chunks, whose elements
// are one contiguous stretch of `dense`; each thread maps its dense positions
// back to (chunk, slot) with a search over the run's offsets in LDS.
struct GroupCompactArgs {
  const uint32_t* sparse;     // [n][K+1]
  const uint4* chunks;
  const uint32_t* range_sums; // [3][ranges] (k_group)
  int64_t tiles;
  int64_t ranges;             // the grid
  int64_t n;
  uint32_t* dense;            // [U][K+1]
  uint32_t* hist;             // [P][2^D] global histograms
  Control* ctl;               // totals of the grouping, set here by workgroup 0
};

template <int K, int D, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_group_compact_hist(GroupCompactArgs a) {
  using DG = KeyDigits<K, D>;
  constexpr int S = K + 1;
  constexpr int P = DG::kPasses;
  constexpr int WORDS = P << D;
  // several items in flight per thread, but wide items one at a time: the
  // multi-item register layout of items wider than 4 words is the one that
  // miscounted histograms on the GPU (see items_per_group)
  constexpr int UNROLL = S <= 4 ? 4 : 1;
  constexpr int PER = kCompactMaxChunks / BLOCK;
  __shared__ uint32_t s_h[WORDS];
  __shared__ uint32_t s_base[kCompactMaxChunks + 1];
  __shared__ uint32_t s_span[kCompactMaxChunks];
  __shared__ uint32_t s_wave[BLOCK / kWave];
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  // totals, and the used groups of the runs before this one
  uint32_t used = 0, before = 0, groups = 0, over = 0;
  for (int64_t r = tid; r < a.ranges; r += BLOCK) {
    const uint32_t ur = a.range_sums[r];
    used += ur;
    before += r < w ? ur : 0u;
    groups += a.range_sums[a.ranges + r];
    over |= a.range_sums[2 * a.ranges + r];
  }
  uint32_t total_used, first, total_groups;
  (void)block_exclusive_scan<BLOCK>(used, s_wave, &total_used);
  (void)block_exclusive_scan<BLOCK>(before, s_wave, &first);
  (void)block_exclusive_scan<BLOCK>(groups, s_wave, &total_groups);
  const bool fallback = __syncthreads_or(over != 0u) != 0;
  if (w == 0 && tid == 0) {
    a.ctl->num_used = int64_t(total_used);
    a.ctl->num_groups = int64_t(total_groups);
    a.ctl->path = fallback ? 1 : 0;
    a.ctl->sort_count = fallback ? a.n : int64_t(total_used);
    a.ctl->all_count = fallback ? a.n : 0;
  }
  if (fallback) return;  // the same in every workgroup
  const int64_t t0 = group_range_start(w, a.tiles, a.ranges);
  const int64_t t1 = group_range_start(w + 1, a.tiles, a.ranges);
  const int nc = int(t1 - t0);  // <= kCompactMaxChunks (group_compact_ranges)
  // the run's chunks: offsets (exclusive prefix of their used counts) and span starts
  uint32_t cnt[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = tid * PER + j;
    uint4 c = make_uint4(0, 0, 0, 0);
    if (i < nc) c = a.chunks[t0 + i];
    cnt[j] = c.y;
    sum += c.y;
    if (i < nc) s_span[i] = c.x;
  }
  uint32_t run_total;
  const uint32_t ex = block_exclusive_scan<BLOCK>(sum, s_wave, &run_total);
  uint32_t acc = first + ex;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = tid * PER + j;
    if (i < nc) s_base[i] = acc;
    acc += cnt[j];
  }
  const uint32_t end = first + run_total;
  if (tid == 0) s_base[nc] = end;
  zero_histograms<WORDS, BLOCK>(s_h);  // synchronises
  uint32_t last[P], run[P];
#pragma unroll
  for (int p = 0; p < P; ++p) { last[p] = 0; run[p] = 0; }
  const uint32_t total = end - first;
  for (uint32_t j0 = 0; j0 < total; j0 += BLOCK * UNROLL) {
    uint32_t e[UNROLL][S];
    uint32_t pos[UNROLL];
#pragma unroll
    for (int r = 0; r < UNROLL; ++r) {
      const uint32_t j = j0 + uint32_t(r * BLOCK + tid);
      pos[r] = first + j;
      if (j < total) {
        // chunk of dense position first + j: the last c with s_base[c] <= it
        int lo = 0, hi = nc - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_base[mid] <= pos[r]) lo = mid; else hi = mid - 1;
        }
        const uint32_t slot = s_span[lo] + (pos[r] - s_base[lo]);
        load_words<S>(a.sparse + int64_t(slot) * S, e[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < UNROLL; ++r) {
      if (j0 + uint32_t(r * BLOCK + tid) >= total) continue;
      store_words<S>(a.dense + int64_t(pos[r]) * S, e[r]);
      hist_item<DG, D>(e[r], s_h, last, run);
    }
  }
#pragma unroll
  for (int p = 0; p < P; ++p)
    if (run[p]) atomicAdd(&s_h[p * (1 << D) + last[p]], run[p]);
  flush_histograms<WORDS, BLOCK>(s_h, a.hist);
}

// Plan of the key sort that follows the grouping: it reads buf[0], which
// holds the packed used groups' elements when the grouping succeeded, else
// all N hash-ordered elements; passes whose digit is the same for every
// element (dead, from the bucket scan) are skipped. One thread.
static __global__ void k_group_sort_plan(SortBuffers b, const Control* ctl) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  (void)ctl;
  const uint32_t* dead = b.plan + b.passes + 1;
  uint32_t in = 0u;
  for (int p = 0; p < b.passes; ++p) {
    const bool skip = dead[p] != 0u;
    b.plan[p] = in | (skip ? 2u : 0u);
    if (!skip) in ^= 1u;
  }
  b.plan[b.passes] = in;
}

// After the key sort of the used groups: sorted position c is output vertex
// c (Section 2, Step 3 compacts the sorted array). Writes the record, the
// representative, cmap[group] = c, and U. Runs only when the grouping
// succeeded.
struct FinalizeArgs {
  SortBuffers bufs;        // sorted(): [U][K+1] (record, group id)
  const int32_t* rep;      // [G]
  int32_t* cmap;           // [G]
  uint32_t* out_vtx;       // [U][K]
  int32_t* new2old;        // [U], nullable
  int64_t* out_num;        // nullable
  int64_t cap;             // n
  Control* ctl;
  int32_t* status;
};

template <int K>
__global__ __launch_bounds__(256) void k_group_finalize(FinalizeArgs a) {
  constexpr int S = K + 1;
  if (gate_closed(kGateGrouped, a.ctl)) return;
  const int64_t u = a.ctl->num_used;
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.out_num) *a.out_num = u;
  const uint32_t* sorted = a.bufs.sorted();
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < u && c < a.cap; c += stride) {
    uint32_t e[S];
    load_words<S>(sorted + c * S, e);
#pragma unroll
    for (int w = 0; w < K; ++w) a.out_vtx[c * K + w] = e[w];
    const uint32_t g = e[K];
    if (int64_t(g) >= a.cap) {
      atomicMax(a.status, 7 /* MRX_ERR_INTERNAL */);
      continue;
    }
    if (a.new2old) a.new2old[c] = a.rep[g];
    a.cmap[g] = int32_t(c);
  }
}

}  // namespace mrx
