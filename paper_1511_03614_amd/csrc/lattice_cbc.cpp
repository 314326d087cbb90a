// Rank-1 lattice generating vectors by component-by-component (CBC) search.
//
// Criterion for N = 2^m points (Korobov space, smoothness 2, product weights
// gamma_j = 1/j^2): with the running products p_k = prod_{i<j}(1 + gamma_i
// 2 pi^2 B2({k z_i / N})), dimension j takes the candidate z minimising
//   E(z) = sum_{k<N} p_k (1 + gamma_j 2 pi^2 B2({k z / N})),  B2(t) = t^2 - t + 1/6,
// ties (relative 1e-12) going to the earlier candidate.  Candidates: every odd
// z < N when there are at most 64, else the 64 odd numbers
// 2 * ((k * 0x9E3779B97F4A7C15 mod 2^64) >> (65 - m)) + 1, k = 1..64.
// z_1 = 1.  Vectors are built for 16 dimensions once per m and cached; the
// vector for fewer dimensions is a prefix.
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "host.h"

namespace sdi {

static std::vector<uint32_t> candidates(int m) {
  const uint64_t N = 1ull << m;
  std::vector<uint32_t> c;
  if (N / 2 <= 64) {
    for (uint64_t k = 0; k < N / 2; ++k) c.push_back((uint32_t)(2 * k + 1));
    return c;
  }
  for (uint64_t k = 1; k <= 64; ++k) {
    const uint64_t h = k * 0x9E3779B97F4A7C15ull;
    c.push_back((uint32_t)(2 * (h >> (64 - (m - 1))) + 1));
  }
  return c;
}

static inline double omega(uint64_t kz, uint64_t N) {
  const double t = (double)(kz & (N - 1)) / (double)N;
  return 2.0 * M_PI * M_PI * (t * t - t + 1.0 / 6.0);
}

// Pairwise sum of p_k * (1 + g * omega(k z)) over k in [lo, hi).
static double crit_sum(const std::vector<double>& p, uint64_t z, uint64_t N, double g, uint64_t lo,
                       uint64_t hi) {
  if (hi - lo <= 128) {
    double s = 0.0;
    for (uint64_t k = lo; k < hi; ++k) s += p[k] * (1.0 + g * omega(k * z, N));
    return s;
  }
  const uint64_t mid = lo + (hi - lo) / 2;
  return crit_sum(p, z, N, g, lo, mid) + crit_sum(p, z, N, g, mid, hi);
}

static std::vector<uint32_t> build(int m, int dims) {
  const uint64_t N = 1ull << m;
  std::vector<double> p(N, 1.0);
  std::vector<uint32_t> z;
  const std::vector<uint32_t> cand = candidates(m);
  unsigned nth = std::thread::hardware_concurrency();
  if (nth == 0) nth = 1;
  if (nth > 16) nth = 16;
  for (int j = 1; j <= dims; ++j) {
    const double g = 1.0 / ((double)j * j);
    uint32_t best = 1;
    if (j > 1) {
      std::vector<double> e(cand.size());
      std::vector<std::thread> th;
      for (unsigned t = 0; t < nth; ++t)
        th.emplace_back([&, t]() {
          for (size_t c = t; c < cand.size(); c += nth) e[c] = crit_sum(p, cand[c], N, g, 0, N);
        });
      for (auto& x : th) x.join();
      double be = 0.0;
      for (size_t c = 0; c < cand.size(); ++c) {
        if (c == 0 || e[c] < be * (1.0 - 1e-12)) {
          best = cand[c];
          be = e[c];
        }
      }
    }
    for (uint64_t k = 0; k < N; ++k) p[k] *= 1.0 + g * omega(k * best, N);
    z.push_back(best);
  }
  return z;
}

const std::vector<uint32_t>& lattice_vector16(int m) {
  static std::mutex mu;
  static std::map<int, std::vector<uint32_t>> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(m);
  if (it != cache.end()) return it->second;
  return cache.emplace(m, build(m, MAXV)).first->second;
}

}  // namespace sdi
