// Host-only driver for the sanitizer test: runs the oracle and the seeded
// generators on tiny random inputs (empty inputs, duplicate keys, extreme
// values, sentinel-like keys) under AddressSanitizer and UBSan, and checks
// the join size and group totals against brute force. Exit status 0 and the
// line "sanitized ok" mean no report and no mismatch.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

extern "C" {
int64_t oracle_filter(int, const void* const*, const int*, int64_t, const uint32_t*, int64_t, int,
                      const int*, const int*, const int64_t*, const int64_t*, uint32_t*);
int64_t oracle_hash_join(const void*, const void*, int, int64_t, int64_t, uint32_t*, uint32_t*,
                         int64_t);
int64_t oracle_groupby(int, const void* const*, const int*, int, const void* const*, const int*,
                       int, const int*, const int*, int64_t, int64_t*, int64_t*, int64_t);
int64_t oracle_pipeline(int, const void* const*, const int*, int64_t, int, const int*, const int*,
                        const int64_t*, const int64_t*, int, const int*, const void* const*,
                        const int*, const int64_t*, const void* const*, const int*, int,
                        const int*, const int*, int, const int*, const int*, int64_t*, int64_t*,
                        int64_t);
uint64_t gen_splitmix64_at(uint64_t, uint64_t);
void gen_u64(uint64_t, uint64_t, int64_t, uint64_t*);
void gen_uniform(uint64_t, uint64_t, int64_t, int64_t, int64_t, void*, int);
void gen_permutation_i32(uint64_t, uint64_t, int64_t, int32_t*);
void gen_unique_i64(uint64_t, uint64_t, int64_t, int64_t, int64_t*);
void gen_map_ranks_i64(uint64_t, uint64_t, int64_t, int64_t, const int64_t*, int64_t*);
void gen_zipf(uint64_t, uint64_t, int64_t, double, int64_t, int64_t*);
}

static int fail(const char* what, int round) {
  std::printf("mismatch: %s (round %d)\n", what, round);
  return 1;
}

int main() {
  std::mt19937_64 rng(2508047010ULL);
  const int64_t extremes[] = {INT64_MIN, INT64_MAX, -1, 0, 1, INT32_MIN, INT32_MAX};
  for (int round = 0; round < 300; ++round) {
    const int64_t n = static_cast<int64_t>(rng() % 200), nb = static_cast<int64_t>(rng() % 40);
    std::vector<int64_t> a(n), b(nb), v(n);
    std::vector<int32_t> a32(n), b32(nb), g32(n);
    for (int64_t i = 0; i < n; ++i) {
      a[i] = (rng() % 8 == 0) ? extremes[rng() % 7] : static_cast<int64_t>(rng() % 16) - 4;
      a32[i] = static_cast<int32_t>(a[i]);
      v[i] = (rng() % 16 == 0) ? extremes[rng() % 7] : static_cast<int64_t>(rng() % 1000);
      g32[i] = static_cast<int32_t>(rng() % 5);
    }
    for (int64_t i = 0; i < nb; ++i) {
      b[i] = (rng() % 8 == 0) ? extremes[rng() % 7] : static_cast<int64_t>(rng() % 16) - 4;
      b32[i] = static_cast<int32_t>(b[i]);
    }
    // join: size against the nested loop (64-bit and 32-bit keys)
    int64_t brute = 0, brute32 = 0;
    for (int64_t p = 0; p < n; ++p)
      for (int64_t q = 0; q < nb; ++q) {
        brute += a[p] == b[q];
        brute32 += a32[p] == b32[q];
      }
    std::vector<uint32_t> ob(brute + 1), op(brute + 1);
    if (oracle_hash_join(b.data(), a.data(), 3, nb, n, ob.data(), op.data(), brute) != brute)
      return fail("join int64", round);
    std::vector<uint32_t> ob32(brute32 + 1), op32(brute32 + 1);
    if (oracle_hash_join(b32.data(), a32.data(), 2, nb, n, ob32.data(), op32.data(), brute32 / 2) !=
        brute32)
      return fail("join int32 (capped output)", round);
    // filter
    const void* cols[2] = {a.data(), v.data()};
    const int types[2] = {3, 3};
    const int tcol[1] = {0}, top[1] = {6};
    const int64_t tlo[1] = {-2}, thi[1] = {5};
    std::vector<uint32_t> ids(n + 1);
    const int64_t nf = oracle_filter(2, cols, types, n, nullptr, 0, 1, tcol, top, tlo, thi, ids.data());
    int64_t nf_brute = 0;
    for (int64_t i = 0; i < n; ++i) nf_brute += a[i] >= -2 && a[i] < 5;
    if (nf != nf_brute) return fail("filter", round);
    // group-by: COUNT sums to n (grouped by an int32 column)
    const void* keys[1] = {g32.data()};
    const int ktypes[1] = {2};
    const void* vals[1] = {v.data()};
    const int vtypes[1] = {3};
    const int ops[5] = {0, 1, 2, 3, 4}, acol[5] = {0, 0, 0, 0, 0};
    std::vector<int64_t> ok(8), oa(5 * 8);
    const int64_t ng = oracle_groupby(1, keys, ktypes, 1, vals, vtypes, 5, ops, acol, n, ok.data(),
                                      oa.data(), 8);
    int64_t cnt = 0;
    for (int64_t gi = 0; gi < ng && gi < 8; ++gi) cnt += oa[1 * 8 + gi];
    if (ng > 5 || cnt != n) return fail("group-by counts", round);
    // ungrouped: exactly one row even over no input
    std::vector<int64_t> ua(5);
    if (oracle_groupby(0, nullptr, nullptr, 1, vals, vtypes, 5, ops, acol, n, nullptr, ua.data(),
                       1) != 1)
      return fail("ungrouped", round);
    // pipeline: one dim (int64 keys with duplicates), key = dim payload
    const void* fact[3] = {a.data(), v.data(), g32.data()};
    const int ftypes[3] = {3, 3, 2};
    const int dfk[1] = {0};
    const void* dkey[1] = {b.data()};
    const int dktype[1] = {3};
    const int64_t dn[1] = {nb};
    std::vector<int32_t> pay(nb);
    for (int64_t i = 0; i < nb; ++i) pay[i] = static_cast<int32_t>(i % 3);
    const void* dpay[1] = {pay.data()};
    const int dptype[1] = {2};
    const int ksrc[2] = {1, 0}, kcol[2] = {0, 2};
    const int pops[2] = {1, 0}, pcol[2] = {1, 1};
    std::vector<int64_t> pk(2 * 64), pa(2 * 64);
    const int64_t npg = oracle_pipeline(3, fact, ftypes, n, 0, nullptr, nullptr, nullptr, nullptr,
                                        1, dfk, dkey, dktype, dn, dpay, dptype, 2, ksrc, kcol, 2,
                                        pops, pcol, pk.data(), pa.data(), 64);
    int64_t pcount = 0;
    for (int64_t gi = 0; gi < npg && gi < 64; ++gi) pcount += pa[gi];
    if (npg <= 64 && pcount != brute) return fail("pipeline count", round);
  }
  // generators on small sizes, including empty ones
  for (int64_t n : {0, 1, 7, 1000}) {
    std::vector<uint64_t> u(n + 1);
    gen_u64(1, 2, n, u.data());
    std::vector<int32_t> i32(n + 1);
    gen_uniform(1, 3, -5, 7, n, i32.data(), 4);
    gen_permutation_i32(1, 4, n, i32.data());
    std::vector<int64_t> i64(n + 1), r(n + 1), m(n + 1);
    gen_unique_i64(1, 5, 0, n, i64.data());
    gen_zipf(1, 6, 1000, 1.0, n, r.data());
    gen_map_ranks_i64(1, 7, 1000, n, r.data(), m.data());
    for (int64_t i = 0; i < n; ++i)
      if (r[i] < 1 || r[i] > 1000) return fail("zipf rank range", 0);
  }
  if (gen_splitmix64_at(1234567, 0) == 0) return fail("splitmix", 0);
  std::printf("sanitized ok\n");
  return 0;
}
