// LSD radix sort of (vertex record, original id) pairs — the key-value sort
// of Section 2, Step 2 — as one-sweep digit passes with decoupled look-back.
//
// Key order: record words w0..w{K-1} compared lexicographically, w0 most
// significant, unsigned. LSD pass p handles key bits [p*D, p*D + D) counted
// from the least significant bit of w{K-1}. Every pass is stable, so equal
// records end up in ascending original-id order: the first element of every
// run of equal records is the copy with the smallest original id.
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace mrx {

enum PassMode : int {
  kPassFirst = 0,      // reads the caller's records (+ referenced flags), digit from the key words
  kPassKey = 1,        // element to element, digit from the key words
  kPassMesh = 2,       // element to element, digit from the element's mesh id (batches)
  kPassFirstHash = 3,  // as kPassFirst, digit from the record's hash (hash grouping)
  kPassHash = 4,       // as kPassKey, digit from the record's hash
  kPassFirstHashMesh = 5,  // as kPassFirstHash, hash of (mesh id, record) (hash grouping of a batch)
  kPassHashMesh = 6,       // as kPassHash, hash of (mesh id, record)
};

struct SortPassArgs {
  const uint32_t* vtx;          // first passes: vertex records (K words)
  SortBuffers bufs;             // elements (K+1 words); the first pass writes buf[0] and the plan
  const uint8_t* used;          // first passes: 1 if some index entry references the vertex (nullable)
  const uint32_t* bucket_base;  // [RADIX] start of each digit's bucket in the output
  // Look-back words, [tiles][RADIX]: LbTagged words (wide launches), or
  // LbCompact words. Compact words alternate between two buffers of
  // tiles * RADIX words: each launch clears its rows of `lookback_next`,
  // the buffer the next pass uses.
  void* lookback;
  void* lookback_next;
  uint32_t* tile_counter;
  Control* ctl;
  int32_t* status;
  const int64_t* mesh_off;      // mesh and mesh-hash passes: [nmesh+1] vertex offsets
  const int32_t* mesh_tab;      // mesh passes: bucket table of mesh_off (mesh_of)
  const uint2* mesh_buckets;    // mesh-hash passes: each mesh's hash buckets (mesh_bucket)
  const int64_t* n_dev;         // non-null: the element count is min(n, *n_dev), read on the device
  int32_t nmesh;
  // Key passes: the digit is bits [shift, shift + D) of (w[hi_word]:w[lo_word])
  // (hi_word < 0: none). Hash passes: bits [shift, shift + D) of the hash
  // (mesh-hash passes: of the bucket of (mesh id, record)); mesh passes: of
  // the mesh id.
  int32_t lo_word, hi_word;
  int32_t shift;
  int64_t n;
  uint32_t tag;
  int32_t pass;                 // index of this pass in the plan
};
// Kept within 256 bytes: a larger argument block measurably raised the
// register count of the pass kernels on gfx950 (e.g. 125 -> 138 VGPRs for
// 512 x 16 tiles, one wave fewer per SIMD).
static_assert(sizeof(SortPassArgs) <= 256, "pass arguments outgrew 256 bytes");

// (word_hi:word_lo) >> shift, masked to D bits, with the words chosen by masks.
template <int D, int K, int N>
__device__ __forceinline__ uint32_t masked_digit(const uint32_t (&v)[N], const uint32_t* lo_mask,
                                                 const uint32_t* hi_mask, int shift) {
  uint32_t lo = 0;
#pragma unroll
  for (int w = 0; w < K; ++w) lo |= v[w] & lo_mask[w];
  uint32_t x = lo >> shift;
  if constexpr (32 % D != 0) {
    uint32_t hi = 0;
#pragma unroll
    for (int w = 0; w < K; ++w) hi |= v[w] & hi_mask[w];
    if (shift + D > 32) x |= hi << (32 - shift);  // digit spans two words
  }
  return x & ((1u << D) - 1u);
}

template <int D>
__device__ __forceinline__ uint32_t digit_of(uint32_t lo, uint32_t hi, int shift) {
  uint32_t x = lo >> shift;
  if constexpr (32 % D != 0) {
    if (shift + D > 32) x |= hi << (32 - shift);  // digit spans two words
  }
  return x & ((1u << D) - 1u);
}

// ----------------------------------------------------------------------------
// Digit histograms of every pass in one read of the items.
// hist[p * RADIX + b] += number of items whose pass-p digit is b.
//
// Item i's key words are src[i * STRIDE .. i * STRIDE + K): caller records
// (STRIDE = K) or sort elements (STRIDE = K + 1). Items are read in groups
// of R = 4 / gcd(STRIDE, 4) consecutive ones, i.e. R*STRIDE words = a whole
// number of 16-byte vectors, so a wave reads one contiguous stretch per load
// instruction (when src is 16-byte aligned; otherwise word by word).
constexpr int gcd4(int k) { return (k % 4 == 0) ? 4 : (k % 2 == 0) ? 2 : 1; }

// Digits of every LSD key pass of a K-word record.
template <int K, int D>
struct KeyDigits {
  static constexpr int kPasses = (32 * K + D - 1) / D;
  static __device__ __forceinline__ void digits(const uint32_t* w, uint32_t (&d)[kPasses]) {
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      const int bit = p * D;
      const int wi = K - 1 - bit / 32;
      const int hi = wi - 1;
      d[p] = digit_of<D>(w[wi], hi >= 0 ? w[hi >= 0 ? hi : 0] : 0u, bit % 32);
    }
  }
};

// Digits of the PH hash passes of a K-word record (hash grouping).
template <int K, int D, int PH>
struct HashDigits {
  static constexpr int kPasses = PH;
  static __device__ __forceinline__ void digits(const uint32_t* w, uint32_t (&d)[kPasses]) {
    const uint32_t h = hash_ptr<K>(w);
#pragma unroll
    for (int p = 0; p < PH; ++p) d[p] = (h >> (p * D)) & ((1u << D) - 1u);
  }
};

// Runs of equal digits are counted in registers first: skewed digits (the
// exponent byte of float coordinates) would otherwise serialise on one LDS
// address.
template <class DG, int D>
__device__ __forceinline__ void hist_item(const uint32_t* w, uint32_t* s_h, uint32_t (&last)[DG::kPasses],
                                          uint32_t (&run)[DG::kPasses]) {
  constexpr int RADIX = 1 << D;
  uint32_t d[DG::kPasses];
  DG::digits(w, d);
#pragma unroll
  for (int p = 0; p < DG::kPasses; ++p) {
    if (run[p] != 0 && d[p] == last[p]) {
      ++run[p];
    } else {
      if (run[p]) atomicAdd(&s_h[p * RADIX + last[p]], run[p]);
      last[p] = d[p];
      run[p] = 1;
    }
  }
}

// Items per load group: R consecutive items of STRIDE <= 4 words make a
// whole number of 16-byte vectors, so a wave reads one contiguous stretch per
// load instruction. Wider items are read one at a time: with several wide
// items per group (20 to 36 words in registers next to the per-pass run
// registers) the counts came out wrong on the GPU for 5- to 8-word keys,
// although the source computes them correctly (see the design notes).
constexpr int items_per_group(int stride) { return stride <= 4 ? 4 / gcd4(stride) : 1; }

// Adds chunk `chunk` (BLOCK * GROUPS item groups) of the n items to the
// block's LDS histograms `s_h` ([kPasses * RADIX], zeroed by the caller). The
// one body behind every histogram launch; it touches only LDS, the caller
// adds s_h to the global histograms once (flush_histograms).
template <class DG, int K, int D, int STRIDE, int BLOCK, int GROUPS>
__device__ __forceinline__ void histogram_chunk(const uint32_t* __restrict__ src, int64_t n, uint32_t* s_h,
                                                int64_t chunk) {
  constexpr int P = DG::kPasses;
  constexpr int R = items_per_group(STRIDE);
  constexpr int GW = R == 1 ? K : R * STRIDE;  // words held per group
  uint32_t last[P], run[P];
#pragma unroll
  for (int p = 0; p < P; ++p) { last[p] = 0; run[p] = 0; }
  const bool vec = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
  for (int it = 0; it < GROUPS; ++it) {
    const int64_t g = chunk * (BLOCK * GROUPS) + int64_t(it) * BLOCK + threadIdx.x;
    const int64_t r0 = g * R;
    if (r0 >= n) break;
    uint32_t w[GW];
    if constexpr (R == 1) {
#pragma unroll
      for (int q = 0; q < K; ++q) w[q] = src[r0 * STRIDE + q];
    } else {
      if (vec && r0 + R <= n) {
        const uint4* p4 = reinterpret_cast<const uint4*>(src + r0 * STRIDE);
#pragma unroll
        for (int q = 0; q < GW / 4; ++q) {
          const uint4 x = p4[q];
          w[4 * q] = x.x; w[4 * q + 1] = x.y; w[4 * q + 2] = x.z; w[4 * q + 3] = x.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < GW; ++q) w[q] = (r0 * STRIDE + q < n * STRIDE) ? src[r0 * STRIDE + q] : 0u;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r0 + r < n) hist_item<DG, D>(w + r * STRIDE, s_h, last, run);
  }
#pragma unroll
  for (int p = 0; p < P; ++p)
    if (run[p]) atomicAdd(&s_h[p * (1 << D) + last[p]], run[p]);
}

template <int WORDS, int BLOCK>
__device__ __forceinline__ void zero_histograms(uint32_t* s_h) {
  for (int i = threadIdx.x; i < WORDS; i += BLOCK) s_h[i] = 0;
  __syncthreads();
}

template <int WORDS, int BLOCK>
__device__ __forceinline__ void flush_histograms(const uint32_t* s_h, uint32_t* __restrict__ hist) {
  __syncthreads();
  for (int i = threadIdx.x; i < WORDS; i += BLOCK)
    if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// Histogram launch over items that may sit in one of two buffers: src[0],
// or src[1] when *sel is non-zero; the count is min(n, *n_dev) when n_dev is
// set (both read on the device: the key sort of the hash grouping learns its
// input only there).
struct HistArgs {
  const uint32_t* src[2];
  const int32_t* sel;
  int64_t n;
  const int64_t* n_dev;
  uint32_t* hist;
};

// Every chunk gets its own workgroup (fewer, longer-lived workgroups
// measured slower); the grid-stride loop only matters for capped grids.
template <class DG, int K, int D, int STRIDE, int BLOCK, int GROUPS>
__global__ __launch_bounds__(BLOCK) void k_histogram(HistArgs a) {
  constexpr int WORDS = DG::kPasses << D;
  __shared__ uint32_t s_h[WORDS];
  const int64_t n = a.n_dev ? min(a.n, int64_t(__builtin_amdgcn_readfirstlane(int32_t(*a.n_dev)))) : a.n;
  const uint32_t* src = (a.sel && __builtin_amdgcn_readfirstlane(*a.sel)) ? a.src[1] : a.src[0];
  constexpr int R = items_per_group(STRIDE);
  const int64_t chunks = ((n + R - 1) / R + BLOCK * GROUPS - 1) / (BLOCK * GROUPS);
  if (int64_t(blockIdx.x) >= chunks) return;  // whole block
  zero_histograms<WORDS, BLOCK>(s_h);
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x)
    histogram_chunk<DG, K, D, STRIDE, BLOCK, GROUPS>(src, n, s_h, c);
  flush_histograms<WORDS, BLOCK>(s_h, a.hist);
}

// Digits of the PH passes over one word (w[0]).
template <int D, int PH>
struct WordDigits {
  static constexpr int kPasses = PH;
  static __device__ __forceinline__ void digits(const uint32_t* w, uint32_t (&d)[kPasses]) {
#pragma unroll
    for (int p = 0; p < PH; ++p) d[p] = (w[0] >> (p * D)) & ((1u << D) - 1u);
  }
};

// Bucket-digit histograms of a batch's records for the PH hash passes of its
// hash grouping: record i is hashed together with its mesh id (the mesh
// whose vertex range holds i) and falls in one of that mesh's buckets, as in
// the hash passes and the grouping.
// One workgroup's share (block hb of nb, walking chunks hb, hb + nb, ...);
// s_h holds PH << D words of LDS.
template <int K, int D, int PH, int BLOCK, int GROUPS>
__device__ __forceinline__ void hash_mesh_hist_block(const uint32_t* __restrict__ vtx, int64_t n,
                                                     const int64_t* __restrict__ off, int32_t nmesh,
                                                     const int32_t* __restrict__ tab, const uint2* __restrict__ mb,
                                                     uint32_t* __restrict__ hist, int64_t hb, int64_t nb,
                                                     uint32_t* s_h) {
  using DG = WordDigits<D, PH>;
  constexpr int WORDS = PH << D;
  const int64_t chunks = (n + BLOCK * GROUPS - 1) / (BLOCK * GROUPS);
  if (hb >= chunks) return;  // whole block
  zero_histograms<WORDS, BLOCK>(s_h);
  uint32_t last[PH], run[PH];
#pragma unroll
  for (int p = 0; p < PH; ++p) { last[p] = 0; run[p] = 0; }
  for (int64_t c = hb; c < chunks; c += nb) {
    // a chunk inside one mesh (the usual case) needs one mesh lookup
    const int64_t c0 = c * (BLOCK * GROUPS);
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(mesh_of(off, nmesh, c0, tab));
    const uint32_t m1 = __builtin_amdgcn_readfirstlane(mesh_of(off, nmesh, min(c0 + BLOCK * GROUPS, n) - 1, tab));
    // every load first (positions past the end read the last record)
    uint32_t x[GROUPS][K];
#pragma unroll
    for (int it = 0; it < GROUPS; ++it) {
      const int64_t i = min(c0 + int64_t(it) * BLOCK + threadIdx.x, n - 1);
#pragma unroll
      for (int w = 0; w < K; ++w) x[it][w] = vtx[i * K + w];
    }
#pragma unroll
    for (int it = 0; it < GROUPS; ++it) {
      const int64_t i = c0 + int64_t(it) * BLOCK + threadIdx.x;
      if (i >= n) break;
      const uint32_t m = m0 == m1 ? m0 : mesh_of(off, nmesh, i, tab);
      const uint32_t bucket[1] = {mesh_bucket(mb, m, hash_mesh_words<K>(m, x[it]))};
      hist_item<DG, D>(bucket, s_h, last, run);
    }
  }
#pragma unroll
  for (int p = 0; p < PH; ++p)
    if (run[p]) atomicAdd(&s_h[p * (1 << D) + last[p]], run[p]);
  flush_histograms<WORDS, BLOCK>(s_h, hist);
}

template <int K, int D, int PH, int BLOCK, int GROUPS>
__global__ __launch_bounds__(BLOCK) void k_hash_mesh_histogram(const uint32_t* __restrict__ vtx, int64_t n,
                                                               const int64_t* __restrict__ off, int32_t nmesh,
                                                               const int32_t* __restrict__ tab,
                                                               const uint2* __restrict__ mb,
                                                               uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[PH << D];
  hash_mesh_hist_block<K, D, PH, BLOCK, GROUPS>(vtx, n, off, nmesh, tab, mb, hist, blockIdx.x, gridDim.x, s_h);
}

// Histograms of the mesh-id passes of a batch: mesh b contributes its vertex
// count to digit (b >> shift_q) of mesh pass q.
template <int D>
__global__ void k_mesh_histogram(const int64_t* __restrict__ off, int32_t nmesh, int32_t mesh_passes,
                                 uint32_t* __restrict__ hist) {
  constexpr int RADIX = 1 << D;
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nmesh) return;
  const uint32_t cnt = uint32_t(off[b + 1] - off[b]);
  if (cnt == 0) return;
  for (int q = 0; q < mesh_passes; ++q)
    atomicAdd(&hist[q * RADIX + ((uint32_t(b) >> (q * D)) & (RADIX - 1))], cnt);
}

// The same for the key sort of a batch after its hash grouping, which sorts
// the used values (grouping path: per-mesh counts from their offsets
// off_grouped) or every vertex (Control::path = 1: from off_all).
template <int D>
__global__ void k_mesh_histogram_path(const int64_t* __restrict__ off_grouped, const int64_t* __restrict__ off_all,
                                      const Control* ctl, int32_t nmesh, int32_t mesh_passes,
                                      uint32_t* __restrict__ hist) {
  constexpr int RADIX = 1 << D;
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nmesh) return;
  const int64_t* off = __builtin_amdgcn_readfirstlane(ctl->path) == 0 ? off_grouped : off_all;
  const uint32_t cnt = uint32_t(off[b + 1] - off[b]);
  if (cnt == 0) return;
  for (int q = 0; q < mesh_passes; ++q)
    atomicAdd(&hist[q * RADIX + ((uint32_t(b) >> (q * D)) & (RADIX - 1))], cnt);
}

// Exclusive scan of each pass's RADIX counts, in place (one block per pass),
// and dead[p] = 1 if one digit holds all n elements in pass p.
template <int D, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_scan_buckets(uint32_t* __restrict__ hist, int64_t n,
                                                        const int64_t* __restrict__ n_dev,
                                                        uint32_t* __restrict__ dead) {
  if (n_dev) n = min(n, *n_dev);
  constexpr int RADIX = 1 << D;
  constexpr int BPT = (RADIX + BLOCK - 1) / BLOCK;
  __shared__ uint32_t s_wave[BLOCK / kWave];
  uint32_t* h = hist + int64_t(blockIdx.x) * RADIX;
  uint32_t c[BPT];
  uint32_t sum = 0;
  int all = 0;
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int bin = threadIdx.x * BPT + k;
    c[k] = bin < RADIX ? h[bin] : 0u;
    sum += c[k];
    all |= int64_t(c[k]) == n;
  }
  all = __syncthreads_or(all);
  if (threadIdx.x == 0) dead[blockIdx.x] = all ? 1u : 0u;
  uint32_t total;
  uint32_t run = block_exclusive_scan<BLOCK>(sum, s_wave, &total);
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int bin = threadIdx.x * BPT + k;
    if (bin < RADIX) h[bin] = run;
    run += c[k];
  }
}

// ----------------------------------------------------------------------------
// One LSD digit pass.
//
// Tile layout: wave w of the block owns positions
//   tile*TILE + w*64*IPT + j*64 + lane,   j = 0..IPT-1,
// so every load instruction is coalesced and the (wave, j, lane) order is the
// input order. Ranking is stable: within a wave the D digit bits are matched
// with ballots, the lowest lane of each equal-digit group bumps a per-wave
// LDS counter by the group size, and every lane adds the number of peers on
// lower lanes. Wave counters are then turned into wave-exclusive offsets, a
// block scan gives each digit's start inside the tile, and a decoupled
// look-back over preceding tiles (one word per (tile, digit)) gives the
// digit's global offset. Elements are reordered through LDS into digit
// order, two 32-bit word planes (one 8-byte slot per element) at a time
// where LDS allows, so each thread writes runs of
// consecutive addresses.
template <int K, int D, int BLOCK, int IPT, int MODE, bool WIDE>
__global__ __launch_bounds__(BLOCK) void k_onesweep(SortPassArgs a) {
  using LB = typename std::conditional<WIDE, LbTagged, LbCompact>::type;
  using LbWord = typename LB::Word;
  LbWord* const lookback = static_cast<LbWord*>(a.lookback);
  constexpr int S = K + 1;
  constexpr int RADIX = 1 << D;
  constexpr uint32_t MASK = RADIX - 1;
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * IPT;
  constexpr int BPT = (RADIX + BLOCK - 1) / BLOCK;
  static_assert(D <= 16, "digits are staged as 16-bit values");

  // Word planes go through LDS double-buffered when two planes fit next to
  // the rest; big tiles use one plane and an extra barrier per word.
  constexpr int NBUF = (2 * TILE * 4 + TILE * 2 + WAVES * RADIX * 4 <= 64 * 1024) ? 2 : 1;
  __shared__ uint32_t s_hist[WAVES * RADIX];
  __shared__ uint32_t s_start[RADIX];
  __shared__ uint32_t s_base[RADIX];
  __shared__ __align__(16) uint32_t s_buf[NBUF][TILE];
  // Key passes recompute each element's digit from its reordered words;
  // mesh and hash passes (whose digit costs a lookup or a hash) stage it in
  // LDS.
  constexpr bool kFirst = MODE == kPassFirst || MODE == kPassFirstHash || MODE == kPassFirstHashMesh;
  constexpr bool kMeshHash = MODE == kPassFirstHashMesh || MODE == kPassHashMesh;
  constexpr bool kHash = MODE == kPassFirstHash || MODE == kPassHash || kMeshHash;
  constexpr bool kStageDigits = MODE == kPassMesh || kHash;
  __shared__ uint16_t s_dig[kStageDigits ? TILE : 1];
  __shared__ uint32_t s_wave[WAVES];
  __shared__ uint32_t s_tile;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  // This pass's plan entry is requested first and examined after the LDS
  // set-up and the block barrier below, so its latency is hidden.
  const uint32_t entry = kFirst ? 0u : a.bufs.entry(a.pass);
  // element count (read on the device for the key sort of the hash grouping)
  const int64_t n = a.n_dev ? min(a.n, int64_t(__builtin_amdgcn_readfirstlane(int32_t(*a.n_dev)))) : a.n;
  if constexpr (kFirst) {
    if (blockIdx.x == 0 && tid == 0) write_sort_plan(a.bufs);
  }
  for (int i = tid; i < WAVES * RADIX; i += BLOCK) s_hist[i] = 0;
  const uint32_t tile = claim_tile(a.tile_counter, &s_tile);  // synchronises the block
  // Tiles past the count have no elements: nobody waits on them, and the
  // next pass (same count) never reads their look-back rows.
  if (int64_t(tile) * TILE >= n) return;
  if constexpr (!kFirst) {
    // A pass with a single live digit would leave the order as it is: it
    // moves nothing, and only clears its row of the next pass's look-back
    // buffer.
    if (entry & 2u) {
      if constexpr (!WIDE)
        for (int bin = tid; bin < RADIX; bin += BLOCK)
          lb_store(static_cast<uint32_t*>(a.lookback_next) + int64_t(tile) * RADIX + bin, 0u);
      return;
    }
  }
  const uint32_t* const src = kFirst ? a.vtx : a.bufs.buf[entry & 1u];
  const int64_t tile_base = int64_t(tile) * TILE;
  // word masks of the key digit (all-ones for the chosen word), uniform
  uint32_t lo_mask[K], hi_mask[K];
#pragma unroll
  for (int w = 0; w < K; ++w) {
    lo_mask[w] = w == a.lo_word ? 0xFFFFFFFFu : 0u;
    hi_mask[w] = w == a.hi_word ? 0xFFFFFFFFu : 0u;
  }
  const int valid_count = int(min(int64_t(TILE), n - tile_base));

  // ---- load
  uint32_t v[IPT][S];
  const int64_t wave_base = tile_base + int64_t(wave) * (kWave * IPT) + lane;

  // First pass: the referenced flags of the wave's kWave*IPT consecutive
  // vertices are read as whole words (lane i takes bytes [i*IPT, i*IPT+IPT)
  // of the chunk) and handed to the lanes that own them through LDS, instead
  // of one byte load per element (the byte loads cost more than the rest of
  // the pass's reads together).
  const uint8_t* s_used = nullptr;
  if constexpr (kFirst && IPT % 4 == 0) {
    uint8_t* stage = reinterpret_cast<uint8_t*>(&s_buf[0][0]) + wave * (kWave * IPT);
    const int64_t chunk = tile_base + int64_t(wave) * (kWave * IPT);
    const int64_t mine = chunk + int64_t(lane) * IPT;
    uint32_t w[IPT / 4];
    if (!a.used) {
#pragma unroll
      for (int q = 0; q < IPT / 4; ++q) w[q] = 0u;
    } else if (mine + IPT <= n) {
#pragma unroll
      for (int q = 0; q < IPT / 4; ++q) w[q] = reinterpret_cast<const uint32_t*>(a.used + mine)[q];
    } else {
#pragma unroll
      for (int q = 0; q < IPT / 4; ++q) {
        uint32_t x = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int64_t p = mine + 4 * q + b;
          if (p < n) x |= uint32_t(a.used[p]) << (8 * b);
        }
        w[q] = x;
      }
    }
#pragma unroll
    for (int q = 0; q < IPT / 4; ++q) reinterpret_cast<uint32_t*>(stage + lane * IPT)[q] = w[q];
    __syncthreads();
    s_used = stage;
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t pos = wave_base + j * kWave;
    if (pos < n) {
      if constexpr (kFirst) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[j][k] = src[pos * K + k];
        const bool used = (IPT % 4 == 0) ? s_used[j * kWave + lane] != 0 : (a.used && a.used[pos] != 0);
        v[j][K] = uint32_t(pos) | (used ? 0x80000000u : 0u);
      } else {
        load_words<S>(src + pos * S, v[j]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < S; ++k) v[j][k] = 0;
    }
  }

  // ---- digits
  // first mesh-hash pass: the meshes of the tile's first and last vertex
  uint32_t tile_mesh[2] = {0u, 1u};
  if constexpr (kFirst && kMeshHash) {
    tile_mesh[0] = __builtin_amdgcn_readfirstlane(mesh_of(a.mesh_off, a.nmesh, tile_base, a.mesh_tab));
    tile_mesh[1] = __builtin_amdgcn_readfirstlane(
        mesh_of(a.mesh_off, a.nmesh, tile_base + valid_count - 1, a.mesh_tab));
  }
  uint32_t dig[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if constexpr (MODE == kPassMesh) {
      const int64_t pos = wave_base + j * kWave;
      const uint32_t m = pos < n ? mesh_of(a.mesh_off, a.nmesh, int64_t(v[j][K] & 0x7FFFFFFFu), a.mesh_tab) : 0u;
      dig[j] = (m >> a.shift) & MASK;
    } else {
      if constexpr (kMeshHash) {
        const int64_t pos = wave_base + j * kWave;
        uint32_t m = 0;
        if (kFirst && tile_mesh[0] == tile_mesh[1])
          m = tile_mesh[0];  // ids are positions; the whole tile is one mesh's
        else if (pos < n)
          m = mesh_of(a.mesh_off, a.nmesh, int64_t(v[j][K] & 0x7FFFFFFFu), a.mesh_tab);
        dig[j] = (mesh_bucket(a.mesh_buckets, m, hash_mesh_words<K>(m, v[j])) >> a.shift) & MASK;
      } else if constexpr (kHash)
        dig[j] = (hash_words<K>(v[j]) >> a.shift) & MASK;
      else
        dig[j] = masked_digit<D, K>(v[j], lo_mask, hi_mask, a.shift);
    }
  }

  // ---- stable rank inside the wave
  uint32_t* my_hist = s_hist + wave * RADIX;
  uint32_t rank[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const bool valid = (wave_base + j * kWave) < n;
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const bool bit = (dig[j] >> b) & 1u;
      const uint64_t m = ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int leader = peers ? (__ffsll((unsigned long long)peers) - 1) : lane;
    const uint32_t below = uint32_t(popc64(peers & lanemask_lt()));
    uint32_t base = 0;
    if (valid && lane == leader) base = atomicAdd(&my_hist[dig[j]], uint32_t(popc64(peers)));
    base = __shfl(base, leader, kWave);
    rank[j] = base + below;
  }
  __syncthreads();

  // ---- per-digit tile totals; wave counters become wave-exclusive offsets.
  // The tile's counts are published at once, and the first look-back window
  // (the predecessor tiles' words) is requested now but examined only after
  // the LDS reorder below, so its latency overlaps that work.
  constexpr int LBW = 4;  // look-back window: predecessor tiles read per poll
  // Digits that no element of the whole pass carries (the global histogram
  // says so) are skipped by every tile alike: nothing is published for them
  // and nobody waits on them.
  uint32_t tot[BPT], start_of[BPT];
  bool live[BPT];
  LookbackWindow<LBW, LB> probe[BPT];
  uint32_t my_sum = 0;
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int bin = tid * BPT + k;
    uint32_t run = 0;
    live[k] = false;
    if (bin < RADIX) {
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = s_hist[w * RADIX + bin];
        s_hist[w * RADIX + bin] = run;
        run += c;
      }
      if constexpr (!WIDE)
        lb_store(static_cast<uint32_t*>(a.lookback_next) + int64_t(tile) * RADIX + bin, 0u);
      const uint32_t gend = bin + 1 < RADIX ? a.bucket_base[bin + 1] : uint32_t(n);
      live[k] = gend != a.bucket_base[bin];
      if (live[k]) {
        lb_store(lookback + int64_t(tile) * RADIX + bin,
                 LB::pack(tile == 0 ? kLbInclusive : kLbAggregate, a.tag, run));
        if (tile != 0) lookback_issue<LBW, LB>(probe[k], lookback + bin, int64_t(tile) - 1, RADIX, a.tag);
      }
    }
    tot[k] = run;
    my_sum += run;
  }
  uint32_t tile_total;
  uint32_t start = block_exclusive_scan<BLOCK>(my_sum, s_wave, &tile_total);
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int bin = tid * BPT + k;
    if (bin < RADIX) s_start[bin] = start;
    start_of[k] = start;
    start += tot[k];
  }
  __syncthreads();

  // ---- positions inside the tile (digit-major, stable)
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if ((wave_base + j * kWave) < n) {
      rank[j] += s_start[dig[j]] + my_hist[dig[j]];
      if constexpr (kStageDigits) s_dig[rank[j]] = uint16_t(dig[j]);
    }
  }

  // ---- reorder through LDS: two word planes at a time (8-byte slots) when
  // two planes fit, else one plane at a time
  if constexpr (NBUF == 2) {
    uint2* buf2 = reinterpret_cast<uint2*>(&s_buf[0][0]);
#pragma unroll
    for (int w = 0; w + 1 < S; w += 2) {
      if (w > 0) __syncthreads();  // previous pair fully read
#pragma unroll
      for (int j = 0; j < IPT; ++j)
        if ((wave_base + j * kWave) < n) buf2[rank[j]] = make_uint2(v[j][w], v[j][w + 1]);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int q = r * BLOCK + tid;
        if (q < valid_count) {
          const uint2 x = buf2[q];
          v[r][w] = x.x;
          v[r][w + 1] = x.y;
        }
      }
    }
    if constexpr (S % 2 == 1) {
      uint32_t* buf = &s_buf[0][0];
      if constexpr (S > 1) __syncthreads();
#pragma unroll
      for (int j = 0; j < IPT; ++j)
        if ((wave_base + j * kWave) < n) buf[rank[j]] = v[j][S - 1];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int q = r * BLOCK + tid;
        if (q < valid_count) v[r][S - 1] = buf[q];
      }
    }
  } else {
#pragma unroll
    for (int w = 0; w < S; ++w) {
      uint32_t* buf = s_buf[0];
      if (w > 0) __syncthreads();  // previous plane fully read
#pragma unroll
      for (int j = 0; j < IPT; ++j)
        if ((wave_base + j * kWave) < n) buf[rank[j]] = v[j][w];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const int q = r * BLOCK + tid;
        if (q < valid_count) v[r][w] = buf[q];
      }
    }
  }

  // ---- finish the look-back: global start of each digit's run in this tile
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int bin = tid * BPT + k;
    if (bin < RADIX) {
      uint32_t prev = 0;
      if (tile != 0 && live[k]) {
        prev = lookback_finish<LBW, LB>(probe[k], lookback + bin, RADIX, a.tag, a.ctl, a.status);
        lb_store(lookback + int64_t(tile) * RADIX + bin, LB::pack(kLbInclusive, a.tag, prev + tot[k]));
      }
      s_base[bin] = a.bucket_base[bin] + prev - start_of[k];  // wraps; base + local position is exact
    }
  }
  __syncthreads();
  uint32_t opos[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int q = r * BLOCK + tid;
    uint32_t d;
    if constexpr (kStageDigits)
      d = s_dig[q < valid_count ? q : 0];
    else
      d = masked_digit<D, K>(v[r], lo_mask, hi_mask, a.shift);
    opos[r] = q < valid_count ? s_base[d] + uint32_t(q) : 0xFFFFFFFFu;
  }

  // ---- scatter: consecutive q of one digit go to consecutive addresses
  uint32_t* const out = a.bufs.buf[kFirst ? 0u : (entry & 1u) ^ 1u];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    if (int64_t(opos[r]) < n) store_words<S>(out + int64_t(opos[r]) * S, v[r]);
  }
}

}  // namespace mrx
