// Kernels around the sort: used-vertex marking (Section 2, Step 1), run-head
// flags + prefix sum + scatters (Step 2 / Step 3), compaction of the used
// values, and the index remap (Step 4).
#pragma once

#include "device_common.hpp"

namespace mrx {

constexpr int32_t kErrIndex = 3;     // MRX_ERR_INDEX_OUT_OF_RANGE
constexpr int32_t kErrInternal = 7;  // MRX_ERR_INTERNAL

// Step 1: used[v] = 1 for every referenced vertex v. Batched meshes carry
// mesh-local indices; the element's mesh supplies the vertex offset.
template <bool BATCHED>
__global__ void k_mark_used(const int32_t* __restrict__ idx, int64_t m, int32_t arity, int64_t n,
                            const int64_t* __restrict__ vtx_off, const int64_t* __restrict__ elem_off,
                            int32_t nmesh, uint8_t* __restrict__ used, int32_t* status) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < m; k += stride) {
    const int32_t v = idx[k];
    int64_t lo = 0, cnt = n;
    if constexpr (BATCHED) {
      const uint32_t b = mesh_of(elem_off, nmesh, k / arity);
      lo = vtx_off[b];
      cnt = vtx_off[b + 1] - lo;
    }
    if (v < 0 || v >= cnt || lo < 0 || lo + v >= n) {
      atomicMax(status, kErrIndex);
    } else {
      used[lo + v] = 1;
    }
  }
}

// ----------------------------------------------------------------------------
// Step 2 (flags and prefix sum) fused with the scatters of Steps 3 and 4.
// Over the sorted elements: head(i) = i == 0 || key(i) != key(i-1) (or, for a
// batch, i starts a mesh); gid(i) = inclusive_sum(head)(i) - 1. Heads write
// the group's record and representative id; every element writes its
// group id to the old -> group map and marks the group used if the vertex is
// referenced. The last tile stores G.
struct FlagScanArgs {
  const uint32_t* sorted;  // [n][K+1]
  int64_t n;
  int32_t* o2g;            // [n] original id -> group id
  uint32_t* uniq;          // [G][K] group records
  int32_t* rep;            // [G] smallest original id of the group
  uint8_t* used_g;         // [G] zeroed; 1 = some copy referenced
  uint64_t* lookback;
  uint32_t* tile_counter;
  Control* ctl;
  int32_t* status;
  const int64_t* mesh_off; // batched: [nmesh+1]; head also at every mesh start
  int32_t nmesh;
  uint32_t tag;
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
  const uint32_t tile = claim_tile(a.tile_counter, &s_tile);
  const int64_t n = a.n;
  const int64_t wave_base = int64_t(tile) * TILE + int64_t(wave) * (kWave * IPT) + lane;

  uint32_t id[IPT];
  uint32_t incl[IPT];   // heads at or before this element within the wave's (j, lane) order
  bool head[IPT];
  uint32_t running = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t pos = wave_base + j * kWave;
    const bool valid = pos < n;
    uint32_t e[S];
    if (valid) load_words<S>(a.sorted + pos * S, e);
    else {
#pragma unroll
      for (int w = 0; w < S; ++w) e[w] = 0;
    }
    bool h = false;
    bool differs = false;
#pragma unroll
    for (int w = 0; w < K; ++w) {
      uint32_t pw = __shfl_up(e[w], 1, kWave);
      if (lane == 0 && valid && pos > 0) pw = a.sorted[(pos - 1) * S + w];
      differs |= (pw != e[w]);
    }
    if (valid) {
      h = (pos == 0) || differs;
      if constexpr (BATCHED) {
        const uint32_t b = mesh_of(a.mesh_off, a.nmesh, pos);
        h = h || (a.mesh_off[b] == pos);
      }
    }
    id[j] = e[K];
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
      lb_store(lb, lb_pack(kLbInclusive, a.tag, tile_total));
      s_prefix = 0;
    } else {
      lb_store(lb, lb_pack(kLbAggregate, a.tag, tile_total));
      const uint32_t prev = lookback_exclusive(a.lookback, tile, 1, a.tag, a.ctl, a.status);
      lb_store(lb, lb_pack(kLbInclusive, a.tag, prev + tile_total));
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
    if (head[j]) {  // the record was loaded before the look-back; this re-read hits the cache
#pragma unroll
      for (int w = 0; w < K; ++w) a.uniq[int64_t(g) * K + w] = a.sorted[pos * S + w];
      a.rep[g] = int32_t(org);
    }
    if (id[j] & 0x80000000u) a.used_g[g] = 1;
    a.o2g[org] = int32_t(g);
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
};

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_compact(CompactArgs a) {
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * IPT;
  __shared__ uint32_t s_wave[WAVES];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_prefix;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
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
      lb_store(lb, lb_pack(kLbInclusive, a.tag, tile_total));
      s_prefix = 0;
    } else {
      lb_store(lb, lb_pack(kLbAggregate, a.tag, tile_total));
      const uint32_t prev = lookback_exclusive(a.lookback, tile, 1, a.tag, a.ctl, a.status);
      lb_store(lb, lb_pack(kLbInclusive, a.tag, prev + tile_total));
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

// old2new[i] = new id of vertex i's group, -1 if unused. For a batch the
// global new id is made mesh-local with the mesh's output offset.
template <bool BATCHED>
__global__ void k_old2new(const int32_t* __restrict__ o2g, const int32_t* __restrict__ cmap, int64_t n,
                          int64_t num_groups_cap, const int64_t* __restrict__ vtx_off,
                          const int64_t* __restrict__ out_off, int32_t nmesh,
                          int32_t* __restrict__ old2new) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t g = o2g[i];
    int32_t c = (g >= 0 && g < num_groups_cap) ? cmap[g] : -1;
    if (c < 0) c = -1;
    if constexpr (BATCHED) {
      if (c >= 0) c -= int32_t(out_off[mesh_of(vtx_off, nmesh, i)]);
    }
    old2new[i] = c;
  }
}

// Step 4: out_idx[k] = old2new[idx[k]] (-1 for an out-of-range entry).
template <bool BATCHED>
__global__ void k_remap(const int32_t* idx, int64_t m, int32_t arity, int64_t n,
                        const int64_t* __restrict__ vtx_off, const int64_t* __restrict__ elem_off,
                        int32_t nmesh, const int32_t* __restrict__ old2new, int32_t* out_idx) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < m; k += stride) {
    const int32_t v = idx[k];
    int64_t lo = 0, cnt = n;
    if constexpr (BATCHED) {
      const uint32_t b = mesh_of(elem_off, nmesh, k / arity);
      lo = vtx_off[b];
      cnt = vtx_off[b + 1] - lo;
    }
    out_idx[k] = (v >= 0 && v < cnt && lo >= 0 && lo + v < n) ? old2new[lo + v] : -1;
  }
}

}  // namespace mrx
