// Host driver that runs the serial oracle (oracle/oracle.cpp) and the
// multi-threaded CPU baseline (oracle/parallel_cpu.cpp) on seeded random
// meshes. The test suite builds it with AddressSanitizer and
// UndefinedBehaviorSanitizer, so every out-of-bounds access or undefined
// operation in either file aborts the run. Beyond that, it checks that both
// produce the same result and that the result satisfies the re-index
// identities (Section 2, "Checking our Example": every remapped index
// points at a record equal to the one it pointed at before).
//
// CPU only; shares nothing with the GPU library.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

extern "C" int oracle_reindex(const uint32_t* vtx, int64_t num_vtx, int32_t words, const int32_t* idx,
                              int64_t num_idx, uint32_t* out_vtx, int32_t* out_idx, int32_t* old2new,
                              int32_t* new2old, int64_t* out_num_vtx, int64_t* bad_pos);
extern "C" int cpu_parallel_reindex(const uint32_t* vtx, int64_t n, int32_t K, const int32_t* idx, int64_t m,
                                    int32_t threads, uint32_t* out_vtx, int32_t* out_idx, int32_t* old2new,
                                    int32_t* new2old, int64_t* out_u, int64_t* bad_pos);

namespace {

struct Rng {  // splitmix64
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int64_t below(int64_t n) { return n > 0 ? int64_t(next() % uint64_t(n)) : 0; }
};

struct Result {
  int rc = -1;
  int64_t u = 0, bad = -1;
  std::vector<uint32_t> out_vtx;
  std::vector<int32_t> out_idx, old2new, new2old;
};

Result run(bool parallel, int threads, const std::vector<uint32_t>& vtx, int64_t n, int k,
           const std::vector<int32_t>& idx) {
  Result r;
  // exact-size outputs (capacity n), so the sanitizer sees any overrun
  r.out_vtx.assign(size_t(n) * k, 0u);
  r.out_idx.assign(idx.size(), 0);
  r.old2new.assign(size_t(n), 0);
  r.new2old.assign(size_t(n), 0);
  uint32_t* ov = n ? r.out_vtx.data() : nullptr;
  int32_t* o2n = n ? r.old2new.data() : nullptr;
  int32_t* n2o = n ? r.new2old.data() : nullptr;
  int32_t* oi = idx.empty() ? nullptr : r.out_idx.data();
  const int32_t* ii = idx.empty() ? nullptr : idx.data();
  const uint32_t* vv = n ? vtx.data() : nullptr;
  if (parallel)
    r.rc = cpu_parallel_reindex(vv, n, k, ii, int64_t(idx.size()), threads, ov, oi, o2n, n2o, &r.u, &r.bad);
  else
    r.rc = oracle_reindex(vv, n, k, ii, int64_t(idx.size()), ov, oi, o2n, n2o, &r.u, &r.bad);
  return r;
}

bool same(const Result& a, const Result& b) {
  if (a.rc != b.rc) return false;
  if (a.rc != 0) return a.bad == b.bad;
  return a.u == b.u && a.out_vtx == b.out_vtx && a.out_idx == b.out_idx && a.old2new == b.old2new &&
         a.new2old == b.new2old;
}

bool identities(const Result& r, const std::vector<uint32_t>& vtx, int k, const std::vector<int32_t>& idx) {
  if (r.rc != 0) return true;
  for (size_t e = 0; e < idx.size(); ++e) {
    const int32_t j = r.out_idx[e];
    if (j < 0 || j >= r.u) return false;
    if (std::memcmp(&r.out_vtx[size_t(j) * k], &vtx[size_t(idx[e]) * k], 4u * k) != 0) return false;
  }
  for (int64_t j = 0; j < r.u; ++j) {
    const int32_t o = r.new2old[size_t(j)];
    if (r.old2new[size_t(o)] != j) return false;
  }
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  const int cases = argc > 1 ? std::atoi(argv[1]) : 300;
  int failures = 0;
  for (int c = 0; c < cases; ++c) {
    Rng rng{uint64_t(0x2109'09812ull) + uint64_t(c)};
    const int k = 1 + int(rng.below(16));
    const int64_t n = (c % 17 == 0) ? 0 : rng.below(700);
    const int arity = 1 + int(rng.below(4));
    const int64_t e = (c % 13 == 0) ? 0 : (n == 0 ? int64_t(c & 1) : rng.below(n + 1));
    const int64_t pool = 1 + rng.below(n + 1);
    // a pool of random records (any bit pattern: signed zeros, NaN payloads,
    // words with the top bit set), vertices drawn from it with repetition
    std::vector<uint32_t> recs(size_t(pool) * k);
    for (auto& w : recs) w = uint32_t(rng.next() >> ((rng.next() & 1) ? 0 : 28));
    std::vector<uint32_t> vtx(size_t(n) * k);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t p = rng.below(pool);
      std::memcpy(&vtx[size_t(i) * k], &recs[size_t(p) * k], 4u * k);
    }
    std::vector<int32_t> idx(size_t(e) * arity);
    for (auto& x : idx) x = int32_t(rng.below(n));
    if (!idx.empty() && c % 11 == 5) idx[size_t(rng.below(int64_t(idx.size())))] = (c & 1) ? -1 : int32_t(n);
    if (n == 0 && !idx.empty()) idx[0] = 0;  // an index into an empty vertex array
    const Result ref = run(false, 1, vtx, n, k, idx);
    bool ok = identities(ref, vtx, k, idx);
    for (int t : {1, 3, 8}) ok = ok && same(ref, run(true, t, vtx, n, k, idx));
    if (!ok) {
      std::fprintf(stderr, "case %d (n=%lld k=%d arity=%d e=%lld): mismatch\n", c, (long long)n, k, arity,
                   (long long)e);
      ++failures;
    }
  }
  std::printf("%d cases, %d failures\n", cases, failures);
  return failures ? 1 : 0;
}
