// Kernels around the sort: used-vertex marking (Section 2, Step 1), run-head
// flags + prefix sum + scatters (Step 2 / Step 3), compaction of the used
// values, and the index remap (Step 4).
#pragma once

#include "device_common.hpp"

namespace mrx {

constexpr int32_t kErrIndex = 3;     // MRX_ERR_INDEX_OUT_OF_RANGE
constexpr int32_t kErrInternal = 7;  // MRX_ERR_INTERNAL

// Random-access kernels: block size, and independent elements per thread
// (all loads are issued before any dependent access). Measured on a 26.4M-
// vertex soup: the old2new scatter needs many (pair load, id lookup, store)
// chains in flight per thread; the index kernels gain nothing beyond two.
constexpr int kRandBlock = 256;
constexpr int kRandItems = 2;        // k_mark_used, k_remap
constexpr int kScatterItems = 16;    // k_scatter_old2new

// Step 1: used[v] = 1 for every referenced vertex v. Batched meshes carry
// mesh-local indices; the element's mesh supplies the vertex offset.
struct MarkArgs {
  const int32_t* idx;          // [m] index entries
  int64_t m;                   // capacity in entries (num_elems * arity)
  int32_t arity;
  int64_t n;                   // vertices
  const int64_t* vtx_off;      // batched: [nmesh+1] vertex offsets
  const int64_t* elem_off;     // batched: [nmesh+1] element offsets
  int32_t nmesh;
  const int32_t* elem_tab;     // batched: bucket table of elem_off (mesh_of)
  const int64_t* live_elems;   // device, nullable: only the first *live_elems elements count
  uint8_t* used;               // [n], zeroed
  int32_t* status;
};

// One tile of kRandBlock * kRandItems entries (tile = the workgroup's share).
template <bool BATCHED>
__device__ __forceinline__ void mark_used_tile(const MarkArgs& a, int64_t tile) {
  const int64_t m = a.live_elems ? min(a.m, *a.live_elems * a.arity) : a.m;
  const int64_t base = tile * (kRandBlock * kRandItems) + threadIdx.x;
  int32_t v[kRandItems];
#pragma unroll
  for (int it = 0; it < kRandItems; ++it) {
    const int64_t k = base + it * kRandBlock;
    v[it] = k < m ? stream_load(a.idx + k) : 0;
  }
#pragma unroll
  for (int it = 0; it < kRandItems; ++it) {
    const int64_t k = base + it * kRandBlock;
    if (k >= m) break;
    int64_t lo = 0, cnt = a.n;
    if constexpr (BATCHED) {
      const uint32_t b = mesh_of(a.elem_off, a.nmesh, k / a.arity, a.elem_tab);
      lo = a.vtx_off[b];
      cnt = a.vtx_off[b + 1] - lo;
    }
    if (v[it] < 0 || v[it] >= cnt || lo < 0 || lo + v[it] >= a.n) {
      atomicMax(a.status, kErrIndex);
    } else {
      a.used[lo + v[it]] = 1;
    }
  }
}

template <bool BATCHED>
__global__ __launch_bounds__(kRandBlock) void k_mark_used(MarkArgs a) {
  mark_used_tile<BATCHED>(a, blockIdx.x);
}

// ----------------------------------------------------------------------------
// Step 2 (flags and prefix sum) fused with the scatter of Step 3.
// Over the sorted elements: head(i) = i == 0 || key(i) != key(i-1) (or, for a
// batch, i starts a mesh); gid(i) = inclusive_sum(head)(i) - 1. Heads write
// the group's record and representative id; every element writes the pair
// (gid(i), original id) at its sorted position and marks the group used if
// the vertex is referenced. The last tile stores G.
struct FlagScanArgs {
  SortBuffers bufs;        // sorted(): [n][K+1] elements; spare(): receives the
                           // [n] (group id, original id) pairs in sorted order
  int64_t n;
  uint32_t* uniq;          // [G][K] group records
  int32_t* rep;            // [G] smallest original id of the group
  uint8_t* used_g;         // [G] zeroed; 1 = some copy referenced
  uint64_t* lookback;
  uint32_t* tile_counter;
  Control* ctl;
  int32_t* status;
  const int64_t* mesh_off; // batched: [nmesh+1]; head also at every mesh start
  const int32_t* mesh_tab; // batched: bucket table of mesh_off (mesh_of)
  int32_t nmesh;
  uint32_t tag;
  uint2* pairs;            // nullable: receives the pairs instead of bufs.spare()
  int32_t gate;            // Gate: run always, or only on one path of the hash grouping
};

template <int K, int BLOCK, int IPT, bool BATCHED>
__global__ __launch_bounds__(BLOCK) void k_flag_scan(FlagScanArgs a) {
  constexpr int S = K + 1;
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * IPT;
  __shared__ uint32_t s_wave[WAVES];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_prefix;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  if (gate_closed(a.gate, a.ctl)) return;  // the same for every workgroup
  const uint32_t fin = a.bufs.entry(a.bufs.passes);  // requested before the barrier
  const uint32_t tile = claim_tile(a.tile_counter, &s_tile);
  const int64_t n = a.n;
  const int64_t wave_base = int64_t(tile) * TILE + int64_t(wave) * (kWave * IPT) + lane;
  const uint32_t* sorted = a.bufs.buf[fin & 1u];
  uint2* pairs = a.pairs ? a.pairs : reinterpret_cast<uint2*>(a.bufs.buf[(fin & 1u) ^ 1u]);

  uint32_t id[IPT];
  uint32_t incl[IPT];   // heads at or before this element within the wave's (j, lane) order
  bool head[IPT];
  uint32_t running = 0;
  // The element before this wave's first one (positions are consecutive
  // within the wave: item j, lane l is wave_base + 64 j + l).
  uint32_t carry[K];
  {
    const int64_t p0 = wave_base - lane - 1;
#pragma unroll
    for (int w = 0; w < K; ++w) carry[w] = (p0 >= 0 && p0 < n) ? sorted[p0 * S + w] : 0u;
  }
  uint32_t e[IPT][S];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t pos = wave_base + j * kWave;
    if (pos < n) load_words<S>(sorted + pos * S, e[j]);
    else {
#pragma unroll
      for (int w = 0; w < S; ++w) e[j][w] = 0;
    }
  }
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t pos = wave_base + j * kWave;
    const bool valid = pos < n;
    bool h = false;
    bool differs = false;
#pragma unroll
    for (int w = 0; w < K; ++w) {
      uint32_t pw = __shfl_up(e[j][w], 1, kWave);
      if (lane == 0) pw = carry[w];
      carry[w] = __shfl(e[j][w], kWave - 1, kWave);  // predecessor of lane 0 at item j + 1
      differs |= (pw != e[j][w]);
    }
    if (valid) {
      h = (pos == 0) || differs;
      if constexpr (BATCHED) {
        const uint32_t b = mesh_of(a.mesh_off, a.nmesh, pos, a.mesh_tab);
        h = h || (a.mesh_off[b] == pos);
      }
    }
    id[j] = e[j][K];
    const uint64_t hm = ballot(h);
    incl[j] = running + uint32_t(popc64(hm & lanemask_lt())) + (h ? 1u : 0u);
    running += uint32_t(popc64(hm));
    head[j] = h;
  }

  // wave totals -> block prefix -> look-back across tiles
  if (lane == 0) s_wave[wave] = running;
  __syncthreads();
  uint32_t wave_excl = 0, tile_total = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const uint32_t t = s_wave[w];
    if (w < wave) wave_excl += t;
    tile_total += t;
  }
  if (tid == 0) {
    uint64_t* lb = a.lookback + tile;
    if (tile == 0) {
      lb_store(lb, LbTagged::pack(kLbInclusive, a.tag, tile_total));
      s_prefix = 0;
    } else {
      lb_store(lb, LbTagged::pack(kLbAggregate, a.tag, tile_total));
      const uint32_t prev = lookback_exclusive(a.lookback, tile, 1, a.tag, a.ctl, a.status);
      lb_store(lb, LbTagged::pack(kLbInclusive, a.tag, prev + tile_total));
      s_prefix = prev;
    }
  }
  __syncthreads();
  const uint32_t base = s_prefix + wave_excl;

#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t pos = wave_base + j * kWave;
    if (pos >= n) continue;
    const uint32_t g = base + incl[j] - 1u;
    const uint32_t org = id[j] & 0x7FFFFFFFu;
    if (int64_t(g) >= n || int64_t(org) >= n) {  // only after a failed wait
      atomicMax(a.status, kErrInternal);
      continue;
    }
    if (head[j]) {
#pragma unroll
      for (int w = 0; w < K; ++w) a.uniq[int64_t(g) * K + w] = e[j][w];
      a.rep[g] = int32_t(org);
    }
    if (id[j] & 0x80000000u) a.used_g[g] = 1;
    pairs[pos] = make_uint2(g, org);
    if (pos == n - 1) a.ctl->num_groups = int64_t(g) + 1;
  }
}

// ----------------------------------------------------------------------------
// Step 3 restricted to used groups: cid(g) = number of used groups before g
// (exclusive prefix sum of used_g). Used groups copy their record and
// representative to the outputs; cmap[g] = cid for used groups and ~cid
// (negative) for unused ones, so that both the new id and the count of used
// groups before g can be recovered. The last tile stores U.
struct CompactArgs {
  const uint8_t* used_g;
  const uint32_t* uniq;
  const int32_t* rep;
  int32_t K;
  uint32_t* out_vtx;
  int32_t* new2old;        // may be null
  int32_t* cmap;
  int64_t* out_num;        // U
  int64_t cap;             // capacity (n) for bounds checks
  uint64_t* lookback;
  uint32_t* tile_counter;
  Control* ctl;
  int32_t* status;
  uint32_t tag;
  int32_t gate;            // Gate: run always, or only on one path of the hash grouping
};

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_compact(CompactArgs a) {
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * IPT;
  __shared__ uint32_t s_wave[WAVES];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_prefix;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  if (gate_closed(a.gate, a.ctl)) return;  // the same for every workgroup
  const uint32_t tile = claim_tile(a.tile_counter, &s_tile);
  const int64_t G = a.ctl->num_groups;
  if (int64_t(tile) * TILE >= G) return;  // whole block: tile is uniform
  const int64_t wave_base = int64_t(tile) * TILE + int64_t(wave) * (kWave * IPT) + lane;

  uint32_t excl[IPT];
  bool u[IPT];
  uint32_t running = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t g = wave_base + j * kWave;
    const bool used = g < G && a.used_g[g] != 0;
    const uint64_t m = ballot(used);
    excl[j] = running + uint32_t(popc64(m & lanemask_lt()));
    running += uint32_t(popc64(m));
    u[j] = used;
  }
  if (lane == 0) s_wave[wave] = running;
  __syncthreads();
  uint32_t wave_excl = 0, tile_total = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const uint32_t t = s_wave[w];
    if (w < wave) wave_excl += t;
    tile_total += t;
  }
  if (tid == 0) {
    uint64_t* lb = a.lookback + tile;
    if (tile == 0) {
      lb_store(lb, LbTagged::pack(kLbInclusive, a.tag, tile_total));
      s_prefix = 0;
    } else {
      lb_store(lb, LbTagged::pack(kLbAggregate, a.tag, tile_total));
      const uint32_t prev = lookback_exclusive(a.lookback, tile, 1, a.tag, a.ctl, a.status);
      lb_store(lb, LbTagged::pack(kLbInclusive, a.tag, prev + tile_total));
      s_prefix = prev;
    }
  }
  __syncthreads();
  const uint32_t base = s_prefix + wave_excl;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t g = wave_base + j * kWave;
    if (g >= G) continue;
    const uint32_t c = base + excl[j];
    if (int64_t(c) >= a.cap) {
      atomicMax(a.status, kErrInternal);
      continue;
    }
    if (u[j]) {
      for (int w = 0; w < a.K; ++w) a.out_vtx[int64_t(c) * a.K + w] = a.uniq[g * a.K + w];
      if (a.new2old) a.new2old[c] = a.rep[g];
    }
    a.cmap[g] = u[j] ? int32_t(c) : ~int32_t(c);
    if (g == G - 1) *a.out_num = int64_t(c) + (u[j] ? 1 : 0);
  }
}

// Step 4's map: old2new[org] = new id of the group of each sorted element
// (-1 if the group is unused), a scatter from the (group id, original id)
// pairs that the flag scan left in the spare sort buffer (or that the hash
// grouping left in `pairs_in`); the cmap reads follow the non-decreasing
// group ids. For a batch the new id is made mesh-local with the mesh's
// output offset. A batch's pairs are in mesh order, mesh b's at positions
// [vtx_off[b], vtx_off[b+1]) (sorted by (mesh id, record), or hash-ordered
// with per-mesh bucket ranges), so the mesh of an element is that of its
// position: one lookup for a tile inside one mesh.
template <bool BATCHED>
__global__ __launch_bounds__(kRandBlock) void k_scatter_old2new(SortBuffers bufs, const uint2* pairs_in,
                                                                const int32_t* __restrict__ cmap, int64_t n,
                                                                const int64_t* __restrict__ vtx_off,
                                                                const int64_t* __restrict__ out_off,
                                                                int32_t nmesh, const int32_t* __restrict__ vtx_tab,
                                                                int32_t* __restrict__ old2new) {
  constexpr int TILE = kRandBlock * kScatterItems;
  const uint2* __restrict__ pairs = pairs_in ? pairs_in : reinterpret_cast<const uint2*>(bufs.spare());
  __shared__ int32_t s_cmap[TILE];
  __shared__ uint32_t s_g[2];
  __shared__ uint32_t s_mesh[2];
  const int64_t t0 = int64_t(blockIdx.x) * TILE;
  const int64_t base = t0 + threadIdx.x;
  const int64_t t1 = min(t0 + TILE, n) - 1;  // last position of the tile
  // A tile's group ids are non-decreasing and grow by at most one per
  // position, so cmap[g_first .. g_last] (at most TILE entries) is staged in
  // LDS with coalesced loads instead of one gather per element.
  if (threadIdx.x == 0) {
    s_g[0] = pairs[t0].x;
    s_g[1] = pairs[t1].x;
    if constexpr (BATCHED) {
      s_mesh[0] = mesh_of(vtx_off, nmesh, t0, vtx_tab);
      s_mesh[1] = mesh_of(vtx_off, nmesh, t1, vtx_tab);
    }
  }
  uint2 p[kScatterItems];
  int32_t c[kScatterItems];
#pragma unroll
  for (int it = 0; it < kScatterItems; ++it) {
    const int64_t i = base + it * kRandBlock;
    if (i < n) {
      p[it] = pairs[i];  // one 8-byte load
    } else {
      p[it] = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
    }
  }
  __syncthreads();
  const uint32_t g0 = s_g[0];
  const int64_t span = min(int64_t(TILE), int64_t(s_g[1]) - int64_t(g0) + 1);
  for (int64_t i = threadIdx.x; i < span; i += kRandBlock)
    s_cmap[i] = (int64_t(g0) + i < n) ? cmap[int64_t(g0) + i] : -1;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kScatterItems; ++it) {
    const int64_t off = int64_t(p[it].x) - int64_t(g0);
    if (int64_t(p[it].x) >= n || int64_t(p[it].y) >= n) c[it] = -1;
    else c[it] = (off >= 0 && off < span) ? s_cmap[off] : cmap[p[it].x];  // outside: only after a failed wait
  }
  int64_t tile_off = 0;  // output offset of the tile's mesh, if it has one
  const bool one_mesh = BATCHED && s_mesh[0] == s_mesh[1];
  if constexpr (BATCHED) {
    if (one_mesh) tile_off = out_off[s_mesh[0]];
  }
#pragma unroll
  for (int it = 0; it < kScatterItems; ++it) {
    if (int64_t(p[it].x) >= n || int64_t(p[it].y) >= n) continue;  // past the end (or a failed wait)
    int32_t cc = c[it] < 0 ? -1 : c[it];
    if constexpr (BATCHED) {
      if (cc >= 0)
        cc -= int32_t(one_mesh ? tile_off : out_off[mesh_of(vtx_off, nmesh, base + it * kRandBlock, vtx_tab)]);
    }
    old2new[p[it].y] = cc;
  }
}

// Step 4: out_idx[k] = old2new[idx[k]] (-1 for an out-of-range entry).
template <bool BATCHED>
__global__ __launch_bounds__(kRandBlock) void k_remap(const int32_t* idx, int64_t m, int32_t arity, int64_t n,
                                                      const int64_t* __restrict__ vtx_off,
                                                      const int64_t* __restrict__ elem_off, int32_t nmesh,
                                                      const int32_t* __restrict__ elem_tab,
                                                      const int64_t* __restrict__ live_elems,
                                                      const int32_t* __restrict__ old2new, int32_t* out_idx) {
  if (live_elems) m = min(m, *live_elems * arity);  // see MarkArgs
  const int64_t base = int64_t(blockIdx.x) * (kRandBlock * kRandItems) + threadIdx.x;
  int64_t src[kRandItems];
#pragma unroll
  for (int it = 0; it < kRandItems; ++it) {
    const int64_t k = base + it * kRandBlock;
    src[it] = -1;
    if (k < m) {
      const int32_t v = stream_load(idx + k);
      int64_t lo = 0, cnt = n;
      if constexpr (BATCHED) {
        const uint32_t b = mesh_of(elem_off, nmesh, k / arity, elem_tab);
        lo = vtx_off[b];
        cnt = vtx_off[b + 1] - lo;
      }
      if (v >= 0 && v < cnt && lo >= 0 && lo + v < n) src[it] = lo + v;
    }
  }
  int32_t r[kRandItems];
#pragma unroll
  for (int it = 0; it < kRandItems; ++it) r[it] = src[it] >= 0 ? old2new[src[it]] : -1;
#pragma unroll
  for (int it = 0; it < kRandItems; ++it) {
    const int64_t k = base + it * kRandBlock;
    if (k < m) stream_store(out_idx + k, r[it]);
  }
}

}  // namespace mrx
