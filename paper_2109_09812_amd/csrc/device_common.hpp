// Device-side building blocks shared by the meshrx kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrx {

constexpr int kWave = 64;

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (uint64_t(1) << lane_id()) - 1;  // lane 0 -> 0
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Inclusive scan of a 32-bit value across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    uint32_t t = __shfl_up(v, off, kWave);
    if (lane_id() >= off) v += t;
  }
  return v;
}

// Exclusive scan over all threads of a block (BLOCK threads, BLOCK % 64 == 0).
// `s_wave` must hold BLOCK/64 words of LDS. Returns the exclusive prefix and
// the block total in *total. Contains __syncthreads().
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave,
                                                         uint32_t* total) {
  constexpr int WAVES = BLOCK / kWave;
  const int wave = threadIdx.x / kWave;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane_id() == kWave - 1) s_wave[wave] = inc;
  __syncthreads();
  uint32_t wave_base = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    uint32_t t = s_wave[w];
    if (w < wave) wave_base += t;
    sum += t;
  }
  *total = sum;
  __syncthreads();  // s_wave may be reused by the caller afterwards
  return wave_base + inc - v;
}

// ---------------------------------------------------------------- look-back
//
// Decoupled look-back state: one word per (tile, bin) holding a status
// (0 = not published, 1 = tile aggregate only, 2 = inclusive prefix) and a
// count. The value travels inside the same atomic word as its status, so
// relaxed agent-scope atomics suffice: no other memory is published through
// it. Two word formats:
//   LbTagged  (64 bit): value bits 0..31, tag bits 32..47 (which launch of the
//             call wrote it), status bits 48..49. A word written by an earlier
//             launch of the same call carries another tag and reads as "not
//             published", so launches can share one zeroed buffer.
//   LbCompact (32 bit): value bits 0..29, status bits 30..31. No tag: each
//             launch needs a buffer cleared since the last launch that used
//             it. Half the polling traffic; values must stay below 2^30.

constexpr uint32_t kLbAggregate = 1;
constexpr uint32_t kLbInclusive = 2;

struct LbTagged {
  using Word = uint64_t;
  static __device__ __forceinline__ Word pack(uint32_t st, uint32_t tag, uint32_t value) {
    return (uint64_t(st) << 48) | (uint64_t(tag & 0xFFFFu) << 32) | uint64_t(value);
  }
  // status of a word for a reader of launch `tag` (0 if written by another launch)
  static __device__ __forceinline__ uint32_t status(Word w, uint32_t tag) {
    return (uint32_t(w >> 32) & 0xFFFFu) == (tag & 0xFFFFu) ? uint32_t(w >> 48) : 0u;
  }
  static __device__ __forceinline__ uint32_t value(Word w) { return uint32_t(w); }
};

struct LbCompact {
  using Word = uint32_t;
  static constexpr uint32_t kMaxValue = (1u << 30) - 1;
  static __device__ __forceinline__ Word pack(uint32_t st, uint32_t, uint32_t value) {
    return (st << 30) | value;
  }
  static __device__ __forceinline__ uint32_t status(Word w, uint32_t) { return w >> 30; }
  static __device__ __forceinline__ uint32_t value(Word w) { return w & kMaxValue; }
};

template <typename W>
__device__ __forceinline__ void lb_store(W* p, W v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename W>
__device__ __forceinline__ W lb_load(const W* p) {
  return __hip_atomic_load(const_cast<W*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t flag_load(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Upper bound on polls of one look-back word. A predecessor tile has already
// claimed its tile id and is running, so in a correct launch it publishes
// within microseconds; the bound only keeps a broken launch from hanging.
constexpr uint32_t kSpinLimit = 1u << 20;

// Control block kept in the (zeroed) workspace.
struct Control {
  int32_t abort;        // set once any wait exceeds kSpinLimit; all waits then give up
  int32_t path;         // hash grouping: 0 = groups found, 1 = a bucket did not fit, sort everything
  int32_t pad[2];
  int64_t num_groups;   // G: distinct values (per mesh, for a batch) among all vertices
  int64_t num_used;     // U of a batch (all meshes), or of the hash grouping
  int64_t sort_count;   // hash grouping: elements the key sort handles (U, or N after path = 1)
  int64_t all_count;    // hash grouping: N after path = 1, else 0 (histogram of all N elements)
};

// Which kernels of a launch sequence run, decided on the device (the host
// never reads device data): kGateAlways, or only while Control::path is 0
// (hash grouping succeeded) or 1 (it gave up).
enum Gate : int32_t { kGateAlways = 0, kGateGrouped = 1, kGateSortAll = 2 };

__device__ __forceinline__ bool gate_closed(int32_t gate, const Control* ctl) {
  if (gate == kGateAlways) return false;
  const int32_t path = __builtin_amdgcn_readfirstlane(ctl->path);
  return gate == kGateGrouped ? path != 0 : path == 0;
}

// ---------------------------------------------------------------- record hash
//
// 32-bit hash of a record's K words: the block and finalisation steps of
// MurmurHash3 (x86, 32-bit variant, by Austin Appleby). Equal records hash
// equally; the hash grouping only needs that and a good spread of distinct
// records over the buckets, never the order of the hashes.
__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

template <int K, int N>
__device__ __forceinline__ uint32_t hash_words(const uint32_t (&v)[N]) {
  static_assert(K <= N, "record words");
  uint32_t h = 0x21090981u;
#pragma unroll
  for (int w = 0; w < K; ++w) {
    uint32_t k = v[w] * 0xcc9e2d51u;
    k = rotl32(k, 15) * 0x1b873593u;
    h = rotl32(h ^ k, 13) * 5u + 0xe6546b64u;
  }
  h ^= uint32_t(4 * K);
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Hash of a batch's record: the (K+1)-word record (mesh id, record words),
// so that equal records of different meshes land in different buckets.
template <int K, int N>
__device__ __forceinline__ uint32_t hash_mesh_words(uint32_t mesh, const uint32_t (&v)[N]) {
  static_assert(K <= N, "record words");
  uint32_t x[K + 1];
  x[0] = mesh;
#pragma unroll
  for (int w = 0; w < K; ++w) x[w + 1] = v[w];
  return hash_words<K + 1>(x);
}

// Hash bucket of a batch's record: every mesh owns a contiguous range of
// buckets, mb[mesh] = (first bucket, bucket count - 1) with a power-of-two
// count sized to the mesh, so that the hash-ordered elements stay grouped by
// mesh (and the vertex ids of neighbouring elements close together).
__device__ __forceinline__ uint32_t mesh_bucket(const uint2* __restrict__ mb, uint32_t mesh, uint32_t h) {
  const uint2 e = mb[mesh];
  return e.x + (h & e.y);
}

template <int K>
__device__ __forceinline__ uint32_t hash_ptr(const uint32_t* w) {
  uint32_t v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = w[i];
  return hash_words<K>(v);
}

// The two element buffers of the LSD sort. A pass whose digit is the same
// for every element (read off the digit histograms) would not reorder
// anything and moves no data, so which buffer holds the elements before a
// pass depends on how many passes before it moved them. `plan` holds
// 2 * passes + 1 words: dead(p) = plan[passes + 1 + p] is 1 if one digit
// holds every element in pass p (written with the bucket offsets); the first
// pass, which reads the caller's records and always runs, then fills in
// plan[p], 1 <= p < passes: bit 0 = buffer that pass p reads (it writes the
// other), bit 1 = pass p is skipped; and plan[passes] = buffer holding the
// sorted elements.
struct SortBuffers {
  uint32_t* buf[2];
  uint32_t* plan;
  int32_t passes;

  // plan[p], the same for every lane (kept in scalar registers)
  __device__ __forceinline__ uint32_t entry(int p) const {
    return __builtin_amdgcn_readfirstlane(plan[p]);
  }
  __device__ __forceinline__ bool skipped(int p) const { return (entry(p) & 2u) != 0u; }
  __device__ __forceinline__ uint32_t* input_of(int p) const { return (entry(p) & 1u) ? buf[1] : buf[0]; }
  __device__ __forceinline__ uint32_t* output_of(int p) const { return (entry(p) & 1u) ? buf[0] : buf[1]; }
  // after the last pass: the sorted elements, and the other buffer
  __device__ __forceinline__ uint32_t* sorted() const { return input_of(passes); }
  __device__ __forceinline__ uint32_t* spare() const { return output_of(passes); }
};

// Fills in plan[1 .. passes] from the dead flags; one thread.
__device__ __forceinline__ void write_sort_plan(const SortBuffers& b) {
  const uint32_t* dead = b.plan + b.passes + 1;
  uint32_t in = 0;  // the first pass writes buf[0]
  for (int p = 1; p < b.passes; ++p) {
    const bool skip = dead[p] != 0u;
    b.plan[p] = in | (skip ? 2u : 0u);
    if (!skip) in ^= 1u;
  }
  b.plan[b.passes] = in;
}

// Exclusive prefix over tiles [0, tile) for one bin. The walk reads W
// predecessor words per step (tile-1 .. tile-W) with independent loads, adds
// aggregates until it meets an inclusive prefix, and re-polls from the first
// word that is not published yet. Reading a window per step matters on a
// multi-die GPU: each agent-scope poll costs a trip to the memory side, so a
// one-word-per-step walk would let the inclusive prefixes fall behind.
// `stride` is the distance in words between consecutive tiles' entries.
template <int W, typename C>
struct LookbackWindow {
  typename C::Word w[W];
  int64_t hi;  // tile of w[0]; w[i] belongs to tile hi - i
};

template <int W, typename C>
__device__ __forceinline__ void lookback_issue(LookbackWindow<W, C>& win, const typename C::Word* base,
                                               int64_t hi, int64_t stride, uint32_t tag) {
  win.hi = hi;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const int64_t t = hi - i;
    // below tile 0: a virtual inclusive prefix of 0
    win.w[i] = t >= 0 ? lb_load(base + t * stride) : C::pack(kLbInclusive, tag, 0);
  }
}

template <int W, typename C>
__device__ __forceinline__ uint32_t lookback_finish(LookbackWindow<W, C>& win, const typename C::Word* base,
                                                    int64_t stride, uint32_t tag, Control* ctl,
                                                    int32_t* status) {
  uint32_t excl = 0;
  uint32_t spins = 0;
  while (true) {
    int stall = -1;  // first window slot that is not published yet
    bool done = false;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      if (done || stall >= 0) continue;
      const uint32_t st = C::status(win.w[i], tag);
      if (st == 0) {
        stall = i;
        continue;
      }
      excl += C::value(win.w[i]);
      if (st == kLbInclusive) done = true;
    }
    if (done) return excl;
    int64_t next = win.hi - W;
    if (stall >= 0) {
      if (++spins >= kSpinLimit || flag_load(&ctl->abort)) {
        __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicMax(status, 7 /* MRX_ERR_INTERNAL */);
        return excl;
      }
      __builtin_amdgcn_s_sleep(1);
      next = win.hi - stall;
    }
    lookback_issue<W, C>(win, base, next, stride, tag);
  }
}

__device__ __forceinline__ uint32_t lookback_exclusive(const uint64_t* base, int64_t tile, int64_t stride,
                                                       uint32_t tag, Control* ctl, int32_t* status) {
  if (tile <= 0) return 0;
  LookbackWindow<1, LbTagged> win;
  lookback_issue<1, LbTagged>(win, base, tile - 1, stride, tag);
  return lookback_finish<1, LbTagged>(win, base, stride, tag, ctl, status);
}

// Tile of this workgroup in a launch whose tiles wait on their predecessors
// (decoupled look-back). Synchronises the block.
//  * counter == nullptr: the workgroup id. A tile then only waits on tiles of
//    smaller workgroup id; every die of the GPU dispatches its workgroups in
//    increasing id order and runs them to completion, so the smallest
//    unfinished tile is always running and the launch makes progress. No
//    round trip precedes the tile's loads.
//  * otherwise tiles are claimed from the counter in arrival order, so every
//    tile a claimant waits on has already started, whatever the dispatch
//    order; the claim's round trip delays every tile.
// Either way the waits are bounded (kSpinLimit) and end in MRX_ERR_INTERNAL
// rather than a hang.
__device__ __forceinline__ uint32_t claim_tile(uint32_t* counter, uint32_t* s_slot) {
  if (counter == nullptr) {
    __syncthreads();
    return blockIdx.x;
  }
  if (threadIdx.x == 0) *s_slot = atomicAdd(counter, 1u);
  __syncthreads();
  uint32_t t = *s_slot;
  return t;
}

// ---------------------------------------------------------------- streaming accesses
// Loads/stores of data touched exactly once. Plain accesses: non-temporal
// hints were measured and changed neither the request sizes nor the times
// of these kernels on gfx950.
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  return *p;
}

template <typename T>
__device__ __forceinline__ void stream_store(T* p, T v) {
  *p = v;
}

// ---------------------------------------------------------------- element I/O
//
// Sort elements are S = K + 1 uint32 words: K key words then the original
// vertex id (bit 31 = "some index entry references this vertex").

template <int S>
__device__ __forceinline__ void load_words(const uint32_t* __restrict__ p, uint32_t (&v)[S]) {
  if constexpr (S % 4 == 0) {
#pragma unroll
    for (int w = 0; w < S; w += 4) {
      uint4 x = *reinterpret_cast<const uint4*>(p + w);
      v[w] = x.x; v[w + 1] = x.y; v[w + 2] = x.z; v[w + 3] = x.w;
    }
  } else if constexpr (S % 2 == 0) {
#pragma unroll
    for (int w = 0; w < S; w += 2) {
      uint2 x = *reinterpret_cast<const uint2*>(p + w);
      v[w] = x.x; v[w + 1] = x.y;
    }
  } else {
#pragma unroll
    for (int w = 0; w < S; ++w) v[w] = p[w];
  }
}

template <int S>
__device__ __forceinline__ void store_words(uint32_t* __restrict__ p, const uint32_t (&v)[S]) {
  if constexpr (S % 4 == 0) {
#pragma unroll
    for (int w = 0; w < S; w += 4)
      *reinterpret_cast<uint4*>(p + w) = make_uint4(v[w], v[w + 1], v[w + 2], v[w + 3]);
  } else if constexpr (S % 2 == 0) {
#pragma unroll
    for (int w = 0; w < S; w += 2) *reinterpret_cast<uint2*>(p + w) = make_uint2(v[w], v[w + 1]);
  } else {
#pragma unroll
    for (int w = 0; w < S; ++w) p[w] = v[w];
  }
}

// Mesh of a packed id: the b with off[b] <= id < off[b+1] (binary search;
// off has nmesh+1 entries). With `tab` (tab[q] = mesh of id q << kMeshTabShift,
// clamped to the last id; see k_mesh_table) the search only spans the meshes
// that start inside id's bucket of 2^kMeshTabShift ids, a step or two
// instead of log2(nmesh) dependent loads.
constexpr int kMeshTabShift = 8;

__device__ __forceinline__ uint32_t mesh_of(const int64_t* __restrict__ off, int32_t nmesh,
                                            int64_t id, const int32_t* __restrict__ tab = nullptr) {
  int32_t lo = 0, hi = nmesh;  // invariant: off[lo] <= id < off[hi]
  if (tab) {
    const int64_t q = id >> kMeshTabShift;
    lo = max(0, min(tab[q], nmesh - 1));
    hi = min(nmesh, max(tab[q + 1] + 1, lo + 1));
  }
  while (hi - lo > 1) {
    int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= id) lo = mid; else hi = mid;
  }
  return uint32_t(lo);
}

}  // namespace mrx
