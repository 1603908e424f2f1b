// Kernels of the mesh edits that feed the re-index (paper Section 3, sample
// use cases): merging the meshes of a packed batch, and keeping a subset of
// a mesh's elements. Both produce a plain index array that the single-mesh
// launch sequence then re-indexes in place.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace mrx {

// Merging meshes: global[k] = local[k] + the first vertex of entry k's mesh.
// An entry outside its own mesh becomes -1, which the re-index reports as an
// index error. `out` may be `idx` itself.
__global__ __launch_bounds__(256) void k_offset_indices(const int32_t* idx, int64_t m, int32_t arity,
                                                        const int64_t* __restrict__ vtx_off,
                                                        const int64_t* __restrict__ elem_off, int32_t nmesh,
                                                        const int32_t* __restrict__ elem_tab, int32_t* out) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= m) return;
  const int32_t v = idx[k];
  const uint32_t b = mesh_of(elem_off, nmesh, k / arity, elem_tab);
  const int64_t lo = vtx_off[b], cnt = vtx_off[b + 1] - lo;
  out[k] = (v >= 0 && int64_t(v) < cnt && lo >= 0) ? int32_t(lo + v) : -1;
}

// Subset of a mesh: the elements e with keep[e] != 0, in order, are copied
// to the front of `out` (arity entries each) and their number is stored in
// *out_count. A stable stream compaction: each tile counts its kept elements
// (wave ballots, block scan) and takes its output offset from a decoupled
// look-back over the preceding tiles' counts.
struct SelectArgs {
  const uint8_t* keep;     // [num_elems]
  const int32_t* idx;      // [num_elems][arity]
  int64_t num_elems;
  int32_t arity;
  int32_t* out;            // [num_elems][arity] capacity; must not overlap idx
  int64_t* out_count;      // device
  uint64_t* lookback;      // [tiles + 1] zeroed LbTagged words
  uint32_t* tile_counter;  // nullptr: tiles by workgroup id
  Control* ctl;
  int32_t* status;
  uint32_t tag;
};

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void k_select_elements(SelectArgs a) {
  constexpr int WAVES = BLOCK / kWave;
  constexpr int TILE = BLOCK * IPT;
  __shared__ uint32_t s_wave[WAVES];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_prefix;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const uint32_t tile = claim_tile(a.tile_counter, &s_tile);
  const int64_t ntiles = (a.num_elems + TILE - 1) / TILE;
  const int64_t wave_base = int64_t(tile) * TILE + int64_t(wave) * (kWave * IPT) + lane;

  uint32_t excl[IPT];
  bool kept[IPT];
  uint32_t running = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const int64_t e = wave_base + j * kWave;
    const bool k = e < a.num_elems && a.keep[e] != 0;
    const uint64_t mask = ballot(k);
    excl[j] = running + uint32_t(popc64(mask & lanemask_lt()));
    running += uint32_t(popc64(mask));
    kept[j] = k;
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
    uint32_t prev = 0;
    if (tile == 0) {
      lb_store(lb, LbTagged::pack(kLbInclusive, a.tag, tile_total));
    } else {
      lb_store(lb, LbTagged::pack(kLbAggregate, a.tag, tile_total));
      prev = lookback_exclusive(a.lookback, tile, 1, a.tag, a.ctl, a.status);
      lb_store(lb, LbTagged::pack(kLbInclusive, a.tag, prev + tile_total));
    }
    s_prefix = prev;
    if (int64_t(tile) == ntiles - 1) *a.out_count = int64_t(prev) + tile_total;
  }
  __syncthreads();
  const int64_t base = int64_t(s_prefix) + wave_excl;
  const int32_t A = a.arity;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if (!kept[j]) continue;
    const int64_t e = wave_base + j * kWave;
    const int64_t o = base + excl[j];
    if (o >= a.num_elems) continue;  // only after a failed look-back wait
    for (int c = 0; c < A; ++c) a.out[o * A + c] = a.idx[e * A + c];
  }
}

}  // namespace mrx
