// Multi-threaded CPU re-indexer — TEST INFRASTRUCTURE (a host baseline).
//
// The paper's data-parallel formulation (Section 2, Steps 1-4) run on host
// threads, as its parallel-CPU column of Table 1 does: mark referenced
// vertices, stable LSD radix sort of (record words, id), run-head flags and
// a prefix sum into group ids, a scan over used groups, compaction, the
// old-to-new scatter and the index remap. Each step splits its range into
// one contiguous chunk per thread; scans combine per-chunk totals. Results
// are identical to the serial oracle (oracle.cpp); tests check that.
//
// It is timed beside the serial oracle as a stronger CPU baseline; it is
// not the oracle and shares no code with the GPU library.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

struct Pool {
  int threads;
  template <typename F>
  void run(F&& f) const {  // f(t) for t in [0, threads)
    std::vector<std::thread> ts;
    ts.reserve(size_t(threads));
    for (int t = 1; t < threads; ++t) ts.emplace_back([&f, t] { f(t); });
    f(0);
    for (auto& th : ts) th.join();
  }
  void chunk(int64_t n, int t, int64_t* lo, int64_t* hi) const {
    const int64_t per = (n + threads - 1) / threads;
    *lo = std::min<int64_t>(n, per * t);
    *hi = std::min<int64_t>(n, *lo + per);
  }
};

}  // namespace

extern "C" int cpu_parallel_reindex(const uint32_t* vtx, int64_t n, int32_t K, const int32_t* idx, int64_t m,
                                    int32_t threads, uint32_t* out_vtx, int32_t* out_idx, int32_t* old2new,
                                    int32_t* new2old, int64_t* out_u, int64_t* bad_pos) {
  if (K < 1 || K > 16 || n < 0 || m < 0 || n > INT32_MAX || threads < 1) return 1;
  const Pool pool{threads};
  const int S = K + 1;

  // validation: the first out-of-range index entry
  std::atomic<int64_t> bad{INT64_MAX};
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(m, t, &lo, &hi);
    for (int64_t k = lo; k < hi; ++k)
      if (idx[k] < 0 || idx[k] >= n) {
        int64_t cur = bad.load();
        while (k < cur && !bad.compare_exchange_weak(cur, k)) {
        }
        break;
      }
  });
  if (bad.load() != INT64_MAX) {
    *bad_pos = bad.load();
    return 3;
  }

  // Step 1: referenced vertices
  std::vector<std::atomic<uint8_t>> used(static_cast<size_t>(n));
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(n, t, &lo, &hi);
    for (int64_t i = lo; i < hi; ++i) used[size_t(i)].store(0, std::memory_order_relaxed);
  });
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(m, t, &lo, &hi);
    for (int64_t k = lo; k < hi; ++k) used[size_t(idx[k])].store(1, std::memory_order_relaxed);
  });

  // Step 2: stable LSD radix sort of elements (K words, id) by 8-bit digits,
  // least significant byte of the last word first
  std::vector<uint32_t> a(size_t(n) * S), b(size_t(n) * S);
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(n, t, &lo, &hi);
    for (int64_t i = lo; i < hi; ++i) {
      std::memcpy(&a[size_t(i) * S], &vtx[size_t(i) * K], sizeof(uint32_t) * K);
      a[size_t(i) * S + K] = uint32_t(i);
    }
  });
  std::vector<int64_t> counts(size_t(threads) * 256);
  for (int pass = 0; pass < 4 * K; ++pass) {
    const int word = K - 1 - pass / 4;
    const int shift = 8 * (pass % 4);
    pool.run([&](int t) {
      int64_t lo, hi;
      pool.chunk(n, t, &lo, &hi);
      int64_t* c = &counts[size_t(t) * 256];
      std::fill(c, c + 256, 0);
      for (int64_t i = lo; i < hi; ++i) ++c[(a[size_t(i) * S + word] >> shift) & 255u];
    });
    // exclusive offsets: digit-major, then thread order (keeps the sort stable)
    int64_t run = 0;
    for (int d = 0; d < 256; ++d)
      for (int t = 0; t < threads; ++t) {
        const int64_t c = counts[size_t(t) * 256 + d];
        counts[size_t(t) * 256 + d] = run;
        run += c;
      }
    pool.run([&](int t) {
      int64_t lo, hi;
      pool.chunk(n, t, &lo, &hi);
      int64_t* off = &counts[size_t(t) * 256];
      for (int64_t i = lo; i < hi; ++i) {
        const uint32_t d = (a[size_t(i) * S + word] >> shift) & 255u;
        std::memcpy(&b[size_t(off[d]++) * S], &a[size_t(i) * S], sizeof(uint32_t) * S);
      }
    });
    a.swap(b);
  }

  // Steps 2-3: run heads, group ids (inclusive scan of heads minus one),
  // group used flags, representatives
  std::vector<int64_t> tot(size_t(threads) + 1, 0);
  auto head = [&](int64_t i) {
    return i == 0 || std::memcmp(&a[size_t(i) * S], &a[size_t(i - 1) * S], sizeof(uint32_t) * K) != 0;
  };
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(n, t, &lo, &hi);
    int64_t c = 0;
    for (int64_t i = lo; i < hi; ++i) c += head(i);
    tot[size_t(t) + 1] = c;
  });
  for (int t = 0; t < threads; ++t) tot[size_t(t) + 1] += tot[size_t(t)];
  const int64_t G = tot[size_t(threads)];
  std::vector<int32_t> gid(static_cast<size_t>(n));
  std::vector<std::atomic<uint8_t>> gused(static_cast<size_t>(G));
  std::vector<int64_t> rep(static_cast<size_t>(G));
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(G, t, &lo, &hi);
    for (int64_t g = lo; g < hi; ++g) gused[size_t(g)].store(0, std::memory_order_relaxed);
  });
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(n, t, &lo, &hi);
    int64_t g = tot[size_t(t)] - 1;
    for (int64_t i = lo; i < hi; ++i) {
      if (head(i)) {
        ++g;
        rep[size_t(g)] = a[size_t(i) * S + K];
      }
      gid[size_t(i)] = int32_t(g);
      if (used[a[size_t(i) * S + K]].load(std::memory_order_relaxed))
        gused[size_t(g)].store(1, std::memory_order_relaxed);
    }
  });

  // Step 3 over used groups: compacted ids (exclusive scan), output vertices
  std::fill(tot.begin(), tot.end(), 0);
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(G, t, &lo, &hi);
    int64_t c = 0;
    for (int64_t g = lo; g < hi; ++g) c += gused[size_t(g)].load(std::memory_order_relaxed);
    tot[size_t(t) + 1] = c;
  });
  for (int t = 0; t < threads; ++t) tot[size_t(t) + 1] += tot[size_t(t)];
  const int64_t U = tot[size_t(threads)];
  std::vector<int32_t> cid(static_cast<size_t>(G));
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(G, t, &lo, &hi);
    int64_t c = tot[size_t(t)];
    for (int64_t g = lo; g < hi; ++g) {
      if (gused[size_t(g)].load(std::memory_order_relaxed)) {
        const int64_t r = rep[size_t(g)];
        std::memcpy(&out_vtx[size_t(c) * K], &vtx[size_t(r) * K], sizeof(uint32_t) * K);
        new2old[c] = int32_t(r);
        cid[size_t(g)] = int32_t(c++);
      } else {
        cid[size_t(g)] = -1;
      }
    }
  });

  // Step 4: old-to-new map over sorted positions, then the index remap
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(n, t, &lo, &hi);
    for (int64_t i = lo; i < hi; ++i) old2new[a[size_t(i) * S + K]] = cid[size_t(gid[size_t(i)])];
  });
  pool.run([&](int t) {
    int64_t lo, hi;
    pool.chunk(m, t, &lo, &hi);
    for (int64_t k = lo; k < hi; ++k) out_idx[k] = old2new[idx[k]];
  });
  *out_u = U;
  return 0;
}
