// Steps 1 and 4 of one mesh by vertex bands.
//
// The used marking (Section 2, Step 1), the old2new map and the index remap
// (Step 4) each touch one vertex-indexed table at scattered positions. On
// gfx950 every scattered store costs one fabric request however few bytes it
// writes, and every scattered load fetches a 128-byte line, so these steps
// run at the fabric's request rate. Here the vertex range is cut into bands
// of 2^shift vertices, each small enough that a workgroup holds the band's
// part of the table in LDS, and the index entries and the (group, vertex)
// pairs are first grouped by band:
//  * k_band_partition: a tile of kBandTile index entries groups its valid
//    entries by band in LDS and writes them, band after band, into its own
//    slot part[tile * kBandTile, ...); table[band][tile] = offset << 16 |
//    count within the slot. With positions kept, an entry is
//    pos << kPosShift | (vertex - band start), pos its place in the tile.
//  * k_band_mark: one workgroup per band sets the referenced vertices' bits
//    in an LDS bitmap and writes every flag of the band, 0 or 1, with
//    16-byte stores.
//  * k_pair_partition: the same grouping for the (group, vertex) pairs of
//    Step 3, each carrying the new id of its group: (new id, vertex - band
//    start).
//  * k_band_map: one workgroup per band builds the band's slice of old2new
//    in LDS from its pairs, writes it out whole, then looks up the new id of
//    every index entry of the band and stores it at the entry's slot.
//  * k_band_remap: one workgroup per index tile puts the new ids of its slot
//    back in entry order in LDS and writes its part of out_idx.
// All reads and writes of these kernels are whole runs of a tile slot or a
// band, except the per-(band, tile) slices of the partitions (tens of
// entries each on the meshes this is chosen for).
#pragma once

#include "device_common.hpp"

namespace mrx {

constexpr int kBandBlock = 1024;                    // k_band_map, k_band_remap
constexpr int kIdxPartBlock = 512;                  // index partition
constexpr int kIdxPartItems = 64;
constexpr int kBandTile = kIdxPartBlock * kIdxPartItems;  // 32768 entries: offsets and counts fit 16 bits
constexpr int kMaxBands = 1024;
constexpr int kPairBlock = 512;
constexpr int kPairItems = 32;
constexpr int kPairTile = kPairBlock * kPairItems;  // 16384 pairs (128 KB staged)
constexpr int kMinBandShift = 12;                   // bands start 16-byte aligned
constexpr int kMaxMarkShift = 19;                   // a band's bitmap: at most 64 KB
constexpr int kMaxMapShift = 15;                    // a band's old2new slice: 128 KB
constexpr int kPosShift = 17;                       // entry = pos << 17 | vertex - band start
constexpr int kBandErrIndex = 3;                    // MRX_ERR_INDEX_OUT_OF_RANGE
constexpr int kBandErrInternal = 7;                 // MRX_ERR_INTERNAL

struct BandArgs {
  const int32_t* idx;          // [m] index entries (may be the memory `part` points to)
  int64_t m;                   // capacity in entries (num_elems * arity)
  int32_t arity;
  int64_t n;                   // vertices
  const int64_t* live_elems;   // device, nullable: only the first *live_elems elements count
  int32_t shift;               // band of vertex v = v >> shift
  int32_t nb;                  // ceil(n / 2^shift) <= kMaxBands
  int32_t vec;                 // idx is 16-byte aligned
  int32_t keep_pos;            // entries carry their position in the tile (shift <= kPosShift)
  int64_t tiles;               // ceil(m / kBandTile)
  uint32_t* part;              // [m]
  uint32_t* table;             // [nb][tiles]
  uint32_t* tile_valid;        // [tiles], nullable: valid entries of each tile
  uint8_t* used;               // [n], 16-byte aligned
  int32_t* status;
};

__device__ __forceinline__ int64_t live_entries(const int64_t* live_elems, int64_t m, int32_t arity) {
  return live_elems ? min(m, *live_elems * arity) : m;
}

static __global__ __launch_bounds__(kIdxPartBlock) void k_band_partition(BandArgs a) {
  constexpr int B = kIdxPartBlock, ITEMS = kIdxPartItems;
  static_assert(ITEMS % 4 == 0, "entries are loaded four at a time");
  static_assert(kBandTile <= (1 << (32 - kPosShift)), "positions fit above the vertex offset");
  __shared__ uint32_t s_cnt[kMaxBands];
  __shared__ uint32_t s_off[kMaxBands];
  __shared__ uint32_t s_stage[kBandTile];
  __shared__ uint32_t s_wave[B / kWave];
  const int tid = threadIdx.x;
  for (int b = tid; b < kMaxBands; b += B) s_cnt[b] = 0;
  __syncthreads();
  const int64_t m = live_entries(a.live_elems, a.m, a.arity);
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kBandTile;
  // entry 4 * (i * B + tid) + c of the tile goes to v[4 * i + c]
  int32_t v[ITEMS];
  if (a.vec && base + kBandTile <= m) {
    const int4* p = reinterpret_cast<const int4*>(a.idx + base);
#pragma unroll
    for (int i = 0; i < ITEMS / 4; ++i) {
      const int4 q = stream_load(p + i * B + tid);
      v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < ITEMS / 4; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t k = base + 4 * (int64_t(i) * B + tid) + c;
        v[4 * i + c] = k < m ? stream_load(a.idx + k) : -1;
      }
  }
  bool bad = false;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int64_t k = base + 4 * (int64_t(i / 4) * B + tid) + (i % 4);
    if (k < m && (v[i] < 0 || int64_t(v[i]) >= a.n)) {
      bad = true;
      v[i] = -1;
    }
  }
  if (bad) atomicMax(a.status, kBandErrIndex);
  uint32_t r[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (v[i] >= 0) r[i] = atomicAdd(&s_cnt[v[i] >> a.shift], 1u);
  __syncthreads();
  constexpr int PER = kMaxBands / B;
  uint32_t loc[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    loc[j] = sum;
    sum += s_cnt[tid * PER + j];
  }
  uint32_t valid;
  const uint32_t ex = block_exclusive_scan<B>(sum, s_wave, &valid);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int b = tid * PER + j;
    s_off[b] = ex + loc[j];
    if (b < a.nb) a.table[size_t(b) * size_t(a.tiles) + size_t(tile)] = ((ex + loc[j]) << 16) | s_cnt[b];
  }
  if (tid == 0 && a.tile_valid) a.tile_valid[tile] = valid;
  __syncthreads();
  const uint32_t mask = (1u << a.shift) - 1u;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (v[i] >= 0) {
      const uint32_t pos = 4u * uint32_t((i / 4) * B + tid) + uint32_t(i % 4);
      const uint32_t local = uint32_t(v[i]) & mask;
      s_stage[s_off[uint32_t(v[i]) >> a.shift] + r[i]] = a.keep_pos ? (pos << kPosShift) | local : local;
    }
  __syncthreads();
  for (uint32_t j = tid; j < valid; j += B) stream_store(a.part + base + j, s_stage[j]);
}

__device__ __forceinline__ uint32_t spread_bits4(uint32_t x) {  // bit i -> byte i (i < 4)
  return (x & 1u) | ((x & 2u) << 7) | ((x & 4u) << 14) | ((x & 8u) << 21);
}

// Walks the band's row of a partition table: fn(entry) for every entry of
// the band, wave by wave, BATCH slices in flight per wave. Slices are
// `tile_size` apart; word positions fit 32 bits (fewer than 2^31 entries).
template <int BLOCK, int BATCH, class Load, class Fn>
__device__ __forceinline__ void for_band_entries(const uint32_t* __restrict__ row, int64_t tiles, int tile_size,
                                                 Load load, Fn fn) {
  constexpr int WAVES = BLOCK / kWave;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  for (int64_t t0 = int64_t(wave) * kWave; t0 < tiles; t0 += int64_t(WAVES) * kWave) {
    const uint32_t mine = t0 + lane < tiles ? row[t0 + lane] : 0u;
    for (int j0 = 0; j0 < kWave; j0 += BATCH) {
      uint32_t e[BATCH];
      decltype(load(0u)) x[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        e[u] = __shfl(mine, j0 + u, kWave);
        const uint32_t at = uint32_t(t0 + j0 + u) * uint32_t(tile_size) + (e[u] >> 16) + lane;
        if (uint32_t(lane) < (e[u] & 0xFFFFu)) x[u] = load(at);
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u)
        if (uint32_t(lane) < (e[u] & 0xFFFFu)) fn(x[u], uint32_t(t0 + j0 + u) * uint32_t(tile_size) + (e[u] >> 16) + lane);
      // slices longer than a wave
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const uint32_t at = uint32_t(t0 + j0 + u) * uint32_t(tile_size) + (e[u] >> 16);
        for (uint32_t k = lane + kWave; k < (e[u] & 0xFFFFu); k += kWave) fn(load(at + k), at + k);
      }
    }
  }
}

// One band of k_band_mark; s_bits holds (1 << shift) / 32 words of LDS.
template <int BLOCK>
__device__ __forceinline__ void band_mark_body(const BandArgs& a, int64_t band, uint32_t* s_bits) {
  const int tid = threadIdx.x;
  const int words = (1 << a.shift) / 32;
  for (int w = tid; w < words; w += BLOCK) s_bits[w] = 0;
  __syncthreads();
  const int64_t lo = band << a.shift;
  const uint32_t mask = (1u << a.shift) - 1u;
  const uint32_t* part = a.part;
  for_band_entries<BLOCK, 16>(
      a.table + size_t(band) * size_t(a.tiles), a.tiles, kBandTile,
      [&](uint32_t at) { return stream_load(part + at); },
      [&](uint32_t e, uint32_t) {
        const uint32_t l = e & mask;
        atomicOr(&s_bits[l >> 5], 1u << (l & 31));
      });
  __syncthreads();
  const int64_t hi = min(a.n, lo + (int64_t(1) << a.shift));
  for (int64_t q = lo + int64_t(tid) * 16; q < hi; q += int64_t(BLOCK) * 16) {
    const uint32_t w = (s_bits[(q - lo) >> 5] >> ((q - lo) & 31)) & 0xFFFFu;
    if (q + 16 <= hi) {
      const uint4 o = {spread_bits4(w), spread_bits4(w >> 4), spread_bits4(w >> 8), spread_bits4(w >> 12)};
      stream_store(reinterpret_cast<uint4*>(a.used + q), o);
    } else {
      for (int64_t t = q; t < hi; ++t) a.used[t] = uint8_t((w >> (t - q)) & 1u);
    }
  }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_band_mark(BandArgs a) {
  extern __shared__ uint32_t s_bits[];
  band_mark_body<BLOCK>(a, blockIdx.x, s_bits);
}

// Buffers of the sort-all path are decided on the device: with from_sort
// set, the pairs are read from sort.spare() and the partition is written
// into sort.sorted() (free once the flag scan has run) instead of the plain
// pointers.
struct PairPartArgs {
  const uint2* pairs;          // [n] (group, vertex) pairs of Step 3
  const int32_t* cmap;         // [G] new id of each group, negative if the group is unused
  int64_t n;
  int32_t shift;
  int32_t nb;
  int64_t tiles;               // ceil(n / kPairTile)
  uint2* part;                 // [n] (new id or -1, vertex - band start)
  uint32_t* table;             // [nb][tiles]
  int32_t* status;
  SortBuffers sort;
  int32_t from_sort;
};

// The group ids of a tile of pairs are clustered (sorted, or grouped by
// hash bucket), so the cmap reads hit cache lines other lanes fetched.
static __global__ __launch_bounds__(kPairBlock) void k_pair_partition(PairPartArgs a) {
  __shared__ uint32_t s_cnt[kMaxBands];
  __shared__ uint32_t s_off[kMaxBands];
  __shared__ uint2 s_stage[kPairTile];
  __shared__ uint32_t s_wave[kPairBlock / kWave];
  const int tid = threadIdx.x;
  for (int b = tid; b < kMaxBands; b += kPairBlock) s_cnt[b] = 0;
  __syncthreads();
  const uint2* pairs = a.from_sort ? reinterpret_cast<const uint2*>(a.sort.spare()) : a.pairs;
  uint2* out = a.from_sort ? reinterpret_cast<uint2*>(a.sort.sorted()) : a.part;
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kPairTile;
  // every load unconditional (clamped positions), so that all of them are
  // in flight at once: first the pairs, then the new ids of their groups
  const uint32_t last = uint32_t(a.n - 1);
  uint2 p[kPairItems];
#pragma unroll
  for (int i = 0; i < kPairItems; ++i)
    p[i] = stream_load(pairs + min(uint32_t(base + int64_t(i) * kPairBlock + tid), last));
  int32_t val[kPairItems];
#pragma unroll
  for (int i = 0; i < kPairItems; ++i) val[i] = a.cmap[min(p[i].x, last)];
  uint32_t vtx[kPairItems];
  bool bad = false;
#pragma unroll
  for (int i = 0; i < kPairItems; ++i) {
    const int64_t k = base + int64_t(i) * kPairBlock + tid;
    const bool ok = p[i].x <= last && p[i].y <= last;
    if (k < a.n && !ok) bad = true;  // only after a failed wait
    vtx[i] = k < a.n && ok ? p[i].y : 0xFFFFFFFFu;
  }
  if (bad) atomicMax(a.status, kBandErrInternal);
  uint32_t r[kPairItems];
#pragma unroll
  for (int i = 0; i < kPairItems; ++i)
    if (vtx[i] != 0xFFFFFFFFu) r[i] = atomicAdd(&s_cnt[vtx[i] >> a.shift], 1u);
  __syncthreads();
  constexpr int PER = kMaxBands / kPairBlock;
  uint32_t loc[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    loc[j] = sum;
    sum += s_cnt[tid * PER + j];
  }
  uint32_t valid;
  const uint32_t ex = block_exclusive_scan<kPairBlock>(sum, s_wave, &valid);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int b = tid * PER + j;
    s_off[b] = ex + loc[j];
    if (b < a.nb) a.table[size_t(b) * size_t(a.tiles) + size_t(tile)] = ((ex + loc[j]) << 16) | s_cnt[b];
  }
  __syncthreads();
  const uint32_t mask = (1u << a.shift) - 1u;
#pragma unroll
  for (int i = 0; i < kPairItems; ++i)
    if (vtx[i] != 0xFFFFFFFFu)
      s_stage[s_off[vtx[i] >> a.shift] + r[i]] = make_uint2(uint32_t(val[i] < 0 ? -1 : val[i]), vtx[i] & mask);
  __syncthreads();
  for (uint32_t j = tid; j < valid; j += kPairBlock) stream_store(out + base + j, s_stage[j]);
}

struct BandMapArgs {
  const uint2* ppart;          // pair partition
  const uint32_t* ptable;
  int64_t ptiles;
  const uint32_t* ipart;       // index partition (entries with positions)
  const uint32_t* itable;
  int64_t itiles;
  int64_t n;
  int32_t shift;               // <= kMaxMapShift
  int32_t* old2new;            // [n]
  int32_t* values;             // [m]: new id of the entry at the same place in ipart
  SortBuffers sort;            // with from_sort: ppart = sort.sorted(), values = sort.spare()
  int32_t from_sort;
};

static __global__ __launch_bounds__(kBandBlock) void k_band_map(BandMapArgs a) {
  __shared__ int32_t s_map[1 << kMaxMapShift];
  const int tid = threadIdx.x;
  const int64_t band = blockIdx.x;
  const int64_t lo = band << a.shift;
  const int64_t hi = min(a.n, lo + (int64_t(1) << a.shift));
  const int len = int(hi - lo);
  // vertices whose pair went missing (only after a failed wait) map to -1
  for (int i = tid; i < len; i += kBandBlock) s_map[i] = -1;
  __syncthreads();
  const uint2* ppart = a.from_sort ? reinterpret_cast<const uint2*>(a.sort.sorted()) : a.ppart;
  for_band_entries<kBandBlock, 8>(
      a.ptable + size_t(band) * size_t(a.ptiles), a.ptiles, kPairTile,
      [&](uint32_t at) { return stream_load(ppart + at); },
      [&](uint2 p, uint32_t) { s_map[p.y] = int32_t(p.x); });
  __syncthreads();
  int32_t* out = a.old2new + lo;
  if ((reinterpret_cast<uintptr_t>(out) & 15) == 0) {
    for (int i = 4 * tid; i < len; i += 4 * kBandBlock) {
      if (i + 4 <= len) {
        stream_store(reinterpret_cast<int4*>(out + i), make_int4(s_map[i], s_map[i + 1], s_map[i + 2], s_map[i + 3]));
      } else {
        for (int t = i; t < len; ++t) out[t] = s_map[t];
      }
    }
  } else {
    for (int i = tid; i < len; i += kBandBlock) out[i] = s_map[i];
  }
  const uint32_t mask = (1u << a.shift) - 1u;
  const uint32_t* ipart = a.ipart;
  int32_t* values = a.from_sort ? reinterpret_cast<int32_t*>(a.sort.spare()) : a.values;
  for_band_entries<kBandBlock, 8>(
      a.itable + size_t(band) * size_t(a.itiles), a.itiles, kBandTile,
      [&](uint32_t at) { return stream_load(ipart + at); },
      [&](uint32_t e, uint32_t at) { stream_store(values + at, s_map[e & mask]); });
}

struct BandRemapArgs {
  const uint32_t* ipart;       // index partition (may be out_idx itself)
  const int32_t* values;       // new ids in ipart's layout
  const uint32_t* tile_valid;  // [tiles]
  int64_t m;
  int32_t arity;
  const int64_t* live_elems;   // device, nullable
  int32_t* out_idx;            // [m]
  SortBuffers sort;            // with from_sort: values = sort.spare()
  int32_t from_sort;
};

// Entries dropped by the partition (out of range) come out as -1.
static __global__ __launch_bounds__(kBandBlock) void k_band_remap(BandRemapArgs a) {
  __shared__ int32_t s_out[kBandTile];
  const int tid = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kBandTile;
  for (int j = tid; j < kBandTile; j += kBandBlock) s_out[j] = -1;
  __syncthreads();
  const uint32_t valid = a.tile_valid[tile];
  const int32_t* values = a.from_sort ? reinterpret_cast<const int32_t*>(a.sort.spare()) : a.values;
  if (valid > 0) {
    // unconditional loads (clamped positions), all in flight at once
    constexpr int PER = kBandTile / kBandBlock;
    uint32_t e[PER];
    int32_t x[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t j = min(uint32_t(i * kBandBlock + tid), valid - 1);
      e[i] = a.ipart[base + j];
      x[i] = stream_load(values + base + j);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (uint32_t(i * kBandBlock + tid) < valid) s_out[e[i] >> kPosShift] = x[i];
  }
  __syncthreads();  // every read of this tile's slot precedes the writes below
  const int64_t m = live_entries(a.live_elems, a.m, a.arity);
  const int len = int(min(int64_t(kBandTile), m - base));
  for (int j = tid; j < len; j += kBandBlock) stream_store(a.out_idx + base + j, s_out[j]);
}

// Launches, each with the block shape its kernel is written for.
static inline void launch_band_partition(const BandArgs& a, hipStream_t s) {
  if (a.tiles > 0) hipLaunchKernelGGL(k_band_partition, dim3(a.tiles), dim3(kIdxPartBlock), 0, s, a);
}

// Small bands (Step 4 follows): many short workgroups; large bands: few,
// each reading many entries.
static inline void launch_band_mark(const BandArgs& a, bool small_bands, hipStream_t s) {
  const size_t bits_lds = (size_t(1) << a.shift) / 8;
  if (small_bands)
    hipLaunchKernelGGL(k_band_mark<256>, dim3(a.nb), dim3(256), bits_lds, s, a);
  else
    hipLaunchKernelGGL(k_band_mark<1024>, dim3(a.nb), dim3(1024), bits_lds, s, a);
}

static inline void launch_pair_partition(const PairPartArgs& a, hipStream_t s) {
  if (a.tiles > 0) hipLaunchKernelGGL(k_pair_partition, dim3(a.tiles), dim3(kPairBlock), 0, s, a);
}

static inline void launch_band_map(const BandMapArgs& a, int32_t nb, hipStream_t s) {
  hipLaunchKernelGGL(k_band_map, dim3(nb), dim3(kBandBlock), 0, s, a);
}

static inline void launch_band_remap(const BandRemapArgs& a, int64_t tiles, hipStream_t s) {
  if (tiles > 0) hipLaunchKernelGGL(k_band_remap, dim3(tiles), dim3(kBandBlock), 0, s, a);
}

}  // namespace mrx
