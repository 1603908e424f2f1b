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
// A bucket that does not fit the LDS window (many copies of one value, or an
// unlucky hash) makes the call take the plain path instead: the same key
// sort then runs on all N hash-ordered elements, followed by Section 2's
// run-head flags and scans. Both paths give the identical result; which one
// runs is decided on the device (Control::path).
#pragma once

#include "device_common.hpp"

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

// Look-back word of the grouping kernel (one per chunk, zeroed per call):
// groups in bits 0..29, used groups in bits 30..59, bit 60 = some chunk up to
// here met a bucket that did not fit, status in bits 62..63.
struct GroupLb {
  static __device__ __forceinline__ uint64_t pack(uint32_t st, uint32_t g, uint32_t u, uint32_t over) {
    return (uint64_t(st) << 62) | (uint64_t(over & 1u) << 60) | (uint64_t(u & 0x3FFFFFFFu) << 30) |
           uint64_t(g & 0x3FFFFFFFu);
  }
  static __device__ __forceinline__ uint32_t status(uint64_t w) { return uint32_t(w >> 62); }
  static __device__ __forceinline__ uint32_t groups(uint64_t w) { return uint32_t(w) & 0x3FFFFFFFu; }
  static __device__ __forceinline__ uint32_t used(uint64_t w) { return uint32_t(w >> 30) & 0x3FFFFFFFu; }
  static __device__ __forceinline__ uint32_t over(uint64_t w) { return uint32_t(w >> 60) & 1u; }
};

struct GroupArgs {
  const uint32_t* elems;   // [n][K+1] elements in (hash bucket, id) order
  int64_t n;
  uint32_t bucket_mask;    // bucket of a record = hash & bucket_mask
  uint2* pairs;            // [n] (group id, original id) per position
  int32_t* rep;            // [G] smallest original id of each group
  int32_t* cmap;           // [G] -1 for unused groups (used ones are set by the key sort's finalisation)
  uint32_t* uelems;        // [U][K+1] (record, group id) of every used group, in group order
  uint64_t* lookback;      // [chunks] zeroed
  uint32_t* tile_counter;
  Control* ctl;
  int32_t* status;
};

template <int K>
__device__ __forceinline__ bool lds_keys_equal(const uint32_t* s_keys, int a, int b, int win) {
  bool eq = true;
#pragma unroll
  for (int w = 0; w < K; ++w) eq = eq && (s_keys[w * win + a] == s_keys[w * win + b]);
  return eq;
}

template <int K>
__global__ __launch_bounds__(GroupShape<K>::BLOCK, GroupShape<K>::MIN_WAVES_PER_SIMD) void k_group(GroupArgs a) {
  using SH = GroupShape<K>;
  constexpr int S = SH::S, BLOCK = SH::BLOCK, WIN = SH::WIN, CHUNK = SH::CHUNK, IPT = SH::IPT;
  constexpr int TS = SH::TS, TB = SH::TB;
  constexpr int WAVES = BLOCK / kWave;
  constexpr uint32_t kEmpty = 0xFFFFFFFFu;
  constexpr uint32_t kUsedBit = 0x80000000u;
  constexpr int kScratch = WIN > TS ? WIN : TS;

  __shared__ uint32_t s_keys[K * WIN];      // window records, word-major
  __shared__ uint32_t s_scratch[kScratch];  // buckets of the window, then the table
  __shared__ uint32_t s_cnt[2][IPT][WAVES];
  __shared__ uint32_t s_tile, s_sq, s_eq;
  __shared__ uint32_t s_gpre, s_upre;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int64_t n = a.n;
  if (tid == 0) {
    s_sq = WIN;
    s_eq = WIN;
  }
  const uint32_t tile = claim_tile(a.tile_counter, &s_tile);  // synchronises the block
  const int64_t c0 = int64_t(tile) * CHUNK;
  const int64_t c1 = min(n, c0 + CHUNK);
  const int qc1 = int(c1 - c0) + 1;  // window slot of position c1

  // ---- window: positions c0 - 1 + q, q in [0, WIN). Each thread keeps, for
  // its own slots, the id (bit 31: referenced) and, until the table is
  // built, the record's hash in `slot`; everything else lives in LDS, so
  // that three workgroups fit on a CU.
  uint32_t ids[IPT], slot[IPT];
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
#pragma unroll
    for (int w = 0; w < K; ++w) s_keys[w * WIN + q] = e[w];
    ids[i] = e[K];
    slot[i] = hash_words<K>(e);
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
      if (lds_keys_equal<K>(s_keys, int(cur & 0xFFFFu), q, WIN)) {
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
    // heads leave their group's rank (low half) and used rank (high half)
    // in the table for the other copies; both are below WIN <= 2^16
    if (h) s_scratch[slot[i]] = gb | (ub << 16);
  }

  // ---- look-back across chunks: groups and used groups before this chunk.
  // Wave 0 reads 64 predecessors' words per step (lane l: chunk hi - l), so a
  // walk over chunks that have only published their own counts takes one
  // round trip per 64 chunks.
  if (wave == 0) {
    const uint32_t g_own = active ? gt : 0u, u_own = active ? ut : 0u, o_own = over ? 1u : 0u;
    uint64_t* lb = a.lookback + tile;
    uint32_t gp = 0, up = 0, op = 0;
    if (tile == 0) {
      if (lane == 0) lb_store(lb, GroupLb::pack(kLbInclusive, g_own, u_own, o_own));
    } else {
      if (lane == 0) lb_store(lb, GroupLb::pack(kLbAggregate, g_own, u_own, o_own));
      int64_t hi = int64_t(tile) - 1;
      uint32_t spins = 0;
      while (true) {
        const int64_t t = hi - lane;
        // below chunk 0: a virtual inclusive prefix of zero
        const uint64_t w = t >= 0 ? lb_load(a.lookback + t) : GroupLb::pack(kLbInclusive, 0, 0, 0);
        const uint32_t st = GroupLb::status(w);
        const uint64_t incl = ballot(st == kLbInclusive);
        const uint64_t none = ballot(st == 0);
        // lanes up to and including the nearest inclusive prefix
        const int stop = incl ? __ffsll((unsigned long long)incl) - 1 : kWave - 1;
        const uint64_t upto = stop == kWave - 1 ? ~uint64_t(0) : ((uint64_t(1) << (stop + 1)) - 1);
        if (none & upto) {  // a predecessor that counts has not published yet
          if (++spins >= kSpinLimit || flag_load(&a.ctl->abort)) {
            if (lane == 0) {
              __hip_atomic_store(&a.ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              atomicMax(a.status, 7 /* MRX_ERR_INTERNAL */);
            }
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        const bool mine = (upto >> lane) & 1u;
        uint32_t g = mine ? GroupLb::groups(w) : 0u, u = mine ? GroupLb::used(w) : 0u;
        uint32_t o = mine ? GroupLb::over(w) : 0u;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
          g += __shfl_xor(g, off, kWave);
          u += __shfl_xor(u, off, kWave);
          o |= __shfl_xor(o, off, kWave);
        }
        gp += g;
        up += u;
        op |= o;
        if (incl) break;
        hi -= kWave;
      }
      if (lane == 0) lb_store(lb, GroupLb::pack(kLbInclusive, gp + g_own, up + u_own, op | o_own));
    }
    if (lane == 0) {
      s_gpre = gp;
      s_upre = up;
      if (tile == gridDim.x - 1) {
        const uint32_t any_over = op | o_own;
        a.ctl->num_groups = int64_t(gp) + g_own;
        a.ctl->num_used = int64_t(up) + u_own;
        a.ctl->path = int32_t(any_over);
        a.ctl->sort_count = any_over ? n : int64_t(up) + u_own;
      }
    }
  }
  __syncthreads();
  if (!active) return;
  const uint32_t gpre = s_gpre, upre = s_upre;

  // ---- outputs of the owned span
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    if (slot[i] == kEmpty) continue;
    const int q = i * BLOCK + tid;
    const int64_t pos = c0 - 1 + q;
    const uint32_t ranks = s_scratch[slot[i]];
    const uint32_t g = gpre + (ranks & 0xFFFFu);
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
      for (int w = 0; w < K; ++w) e[w] = s_keys[w * WIN + q];
      e[K] = g;
      store_words<S>(a.uelems + int64_t(u) * S, e);
    } else {
      a.cmap[g] = -1;
    }
  }
}

// Plan of the key sort that follows the grouping: it reads buf[1] (the used
// groups' elements) when the grouping succeeded, else buf[0] (all N
// hash-ordered elements); passes whose digit is the same for every element
// (dead, from the bucket scan) are skipped. One thread.
static __global__ void k_group_sort_plan(SortBuffers b, const Control* ctl) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const uint32_t* dead = b.plan + b.passes + 1;
  uint32_t in = ctl->path != 0 ? 0u : 1u;
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
  int64_t* out_num;
  int64_t cap;             // n
  Control* ctl;
  int32_t* status;
};

template <int K>
__global__ __launch_bounds__(256) void k_group_finalize(FinalizeArgs a) {
  constexpr int S = K + 1;
  if (gate_closed(kGateGrouped, a.ctl)) return;
  const int64_t u = a.ctl->num_used;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.out_num = u;
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
