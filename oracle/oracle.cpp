// Plain, slow, single-threaded CPU oracle for the relational hot path of
// "Rethinking Analytical Processing in the GPU Era" (arXiv 2508.04701).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
// loads this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do. It shares no code, header, table or helper with the HIP
// path: its types, operator codes and hash maps are its own.
//
// What it computes is fixed by plain relational definitions, because the paper
// delegates every operator to a dataframe library and prints no algorithm of
// its own (Section 3.2.2, "Query Execution Engine"):
//   * filter        - the rows of a table that satisfy a conjunction of
//                     comparisons, reported as row ids (the late-materialised
//                     form of filter/join output, Section 3.2.2 and the row-id
//                     discussion of Section 3.2.3);
//   * hash join     - inner equi-join on one key column: every pair (b, p)
//                     with build[b] == probe[p], as row-id pairs;
//   * group-by      - per distinct key tuple: SUM, COUNT, MIN, MAX and AVG
//                     of 64-bit integer values;
//   * pipeline      - filter -> inner join against up to two dimension
//                     tables -> group-by, one fact row at a time, which is the
//                     "whole query plan on the GPU" path of Section 3.1;
//   * semi-join     - the probe rows that have at least one equal build key
//                     (what a Bloom-filter predicate transfer approximates
//                     from above, Section 3.4, "Performance Optimizations");
//   * gather        - late materialisation of a column by row ids
//                     (Section 3.2.2);
//   * top-N         - the first N rows of a result table in the order of one
//                     of its columns, ties broken by the key tuple (the
//                     order-by / top-N operators named among ClickBench's
//                     costs, Section 4.2);
//   * string group-by - group-by on a variable-length string key (Arrow
//                     offsets + bytes), optionally with one integer key
//                     beside it (group-by cost on string keys, Section 4.2).
// The join and group-by use std::unordered_map, as the operator semantics
// require nothing more. Output order: filter follows scan order; join pairs
// are emitted sorted by (probe row, build row); groups are emitted sorted by
// key tuple (signed, lexicographic). Parity tests compare against these
// canonical orders.
//
// Arithmetic: SUM wraps modulo 2^64 (two's complement), COUNT is exact,
// MIN/MAX are signed, AVG is one IEEE-754 binary64 division of the exact
// (int64) SUM by the exact COUNT, each converted to double with
// round-to-nearest-even. A grouped input yields no group with COUNT 0; an
// ungrouped aggregate (no keys) over zero rows yields one row with COUNT 0,
// SUM 0, MIN = INT64_MAX, MAX = INT64_MIN and AVG = the quiet NaN
// 0x7FF8000000000000.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <numeric>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

namespace {

// Column element types of the oracle's own interface.
enum OracleType { OT_I8 = 1, OT_I32 = 2, OT_I64 = 3 };
// Comparison operators; RANGE means lo <= v < hi, the others compare v to lo.
enum OracleCmp { OC_LT = 0, OC_LE = 1, OC_GT = 2, OC_GE = 3, OC_EQ = 4, OC_NE = 5, OC_RANGE = 6 };
// Aggregate operators.
enum OracleAgg { OA_SUM = 0, OA_COUNT = 1, OA_MIN = 2, OA_MAX = 3, OA_AVG = 4 };

const uint64_t kCanonicalNaN = 0x7FF8000000000000ULL;

int64_t read_value(const void* col, int type, int64_t i) {
  switch (type) {
    case OT_I8: return static_cast<const int8_t*>(col)[i];
    case OT_I32: return static_cast<const int32_t*>(col)[i];
    default: return static_cast<const int64_t*>(col)[i];
  }
}

bool comparison_holds(int op, int64_t v, int64_t lo, int64_t hi) {
  switch (op) {
    case OC_LT: return v < lo;
    case OC_LE: return v <= lo;
    case OC_GT: return v > lo;
    case OC_GE: return v >= lo;
    case OC_EQ: return v == lo;
    case OC_NE: return v != lo;
    default: return lo <= v && v < hi;
  }
}

struct Predicate {
  int nterms;
  const int* term_col;
  const int* term_op;
  const int64_t* term_lo;
  const int64_t* term_hi;

  bool holds(const void* const* cols, const int* types, int64_t row) const {
    for (int t = 0; t < nterms; ++t) {
      int c = term_col[t];
      if (!comparison_holds(term_op[t], read_value(cols[c], types[c], row), term_lo[t], term_hi[t]))
        return false;
    }
    return true;
  }
};

// Running state of one aggregate inside one group.
struct AggState {
  uint64_t sum = 0;  // wraps modulo 2^64
  int64_t count = 0;
  int64_t min = std::numeric_limits<int64_t>::max();
  int64_t max = std::numeric_limits<int64_t>::min();

  void add(int64_t v) {
    sum += static_cast<uint64_t>(v);
    count += 1;
    min = std::min(min, v);
    max = std::max(max, v);
  }

  // Final value of aggregate `op`, as the int64 bit pattern written out
  // (AVG is a binary64 stored bit for bit).
  int64_t result(int op) const {
    switch (op) {
      case OA_SUM: return static_cast<int64_t>(sum);
      case OA_COUNT: return count;
      case OA_MIN: return min;
      case OA_MAX: return max;
      default: {
        uint64_t bits = kCanonicalNaN;
        if (count > 0) {
          double avg = static_cast<double>(static_cast<int64_t>(sum)) / static_cast<double>(count);
          std::memcpy(&bits, &avg, sizeof bits);
        }
        return static_cast<int64_t>(bits);
      }
    }
  }
};

struct KeyTupleHash {
  size_t operator()(const std::vector<int64_t>& k) const {
    size_t h = 0;
    for (int64_t v : k) h = h * 1000003u ^ std::hash<int64_t>()(v);
    return h;
  }
};

using GroupMap = std::unordered_map<std::vector<int64_t>, std::vector<AggState>, KeyTupleHash>;

// Writes the groups of `groups` sorted by key tuple; returns the group count.
int64_t emit_groups(const GroupMap& groups, int nkeys, int naggs, const int* agg_op,
                    int64_t* out_keys, int64_t* out_aggs, int64_t cap) {
  std::vector<const std::vector<int64_t>*> order;
  order.reserve(groups.size());
  for (const auto& g : groups) order.push_back(&g.first);
  std::sort(order.begin(), order.end(),
            [](const std::vector<int64_t>* a, const std::vector<int64_t>* b) { return *a < *b; });
  int64_t ng = static_cast<int64_t>(order.size());
  for (int64_t g = 0; g < ng && g < cap; ++g) {
    const std::vector<int64_t>& key = *order[g];
    const std::vector<AggState>& st = groups.at(key);
    for (int k = 0; k < nkeys; ++k) out_keys[k * cap + g] = key[k];
    for (int a = 0; a < naggs; ++a) out_aggs[a * cap + g] = st[a].result(agg_op[a]);
  }
  return ng;
}

}  // namespace

extern "C" {

// Filter: scans rows sel[0..nsel) in the given order (or 0..n-1 when sel is
// NULL) and writes to out every row id whose row satisfies all terms.
// Returns the number of rows written; out must hold nsel (or n) entries.
int64_t oracle_filter(int ncols, const void* const* cols, const int* types, int64_t n,
                      const uint32_t* sel, int64_t nsel, int nterms, const int* term_col,
                      const int* term_op, const int64_t* term_lo, const int64_t* term_hi,
                      uint32_t* out) {
  (void)ncols;
  Predicate pred{nterms, term_col, term_op, term_lo, term_hi};
  int64_t written = 0;
  int64_t scan = sel ? nsel : n;
  for (int64_t i = 0; i < scan; ++i) {
    int64_t row = sel ? static_cast<int64_t>(sel[i]) : i;
    if (pred.holds(cols, types, row)) out[written++] = static_cast<uint32_t>(row);
  }
  return written;
}

// Inner equi-join: returns |{(b, p) : build[b] == probe[p]}| and writes the
// first `cap` pairs in (probe row, build row) order.
int64_t oracle_hash_join(const void* build, const void* probe, int key_type, int64_t nb,
                         int64_t np, uint32_t* out_build, uint32_t* out_probe, int64_t cap) {
  std::unordered_map<int64_t, std::vector<uint32_t>> table;
  for (int64_t b = 0; b < nb; ++b) table[read_value(build, key_type, b)].push_back(static_cast<uint32_t>(b));
  int64_t count = 0;
  for (int64_t p = 0; p < np; ++p) {
    auto it = table.find(read_value(probe, key_type, p));
    if (it == table.end()) continue;
    for (uint32_t b : it->second) {
      if (count < cap) {
        out_build[count] = b;
        out_probe[count] = static_cast<uint32_t>(p);
      }
      ++count;
    }
  }
  return count;
}

// Group-by over n rows: key columns keys[0..nkeys), value columns
// vals[0..nvals); aggregate a is agg_op[a] over vals[agg_col[a]] (COUNT
// ignores its column). Outputs are column-major with stride cap:
// out_keys[k*cap + g] and out_aggs[a*cap + g]. Returns the group count.
int64_t oracle_groupby(int nkeys, const void* const* keys, const int* key_types, int nvals,
                       const void* const* vals, const int* val_types, int naggs,
                       const int* agg_op, const int* agg_col, int64_t n, int64_t* out_keys,
                       int64_t* out_aggs, int64_t cap) {
  (void)nvals;
  GroupMap groups;
  if (nkeys == 0) groups[std::vector<int64_t>()].resize(naggs);
  std::vector<int64_t> key(nkeys);
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < nkeys; ++k) key[k] = read_value(keys[k], key_types[k], i);
    std::vector<AggState>& st = groups[key];
    if (st.empty()) st.resize(naggs);
    for (int a = 0; a < naggs; ++a) {
      int64_t v = agg_op[a] == OA_COUNT ? 0 : read_value(vals[agg_col[a]], val_types[agg_col[a]], i);
      st[a].add(v);
    }
  }
  return emit_groups(groups, nkeys, naggs, agg_op, out_keys, out_aggs, cap);
}

// Fused plan, one fact row at a time:
//   for each fact row i satisfying the predicate,
//     for each dim-0 row b0 with dim0_key[b0] == fact[dim_fk_col[0]][i]
//       for each dim-1 row b1 with dim1_key[b1] == fact[dim_fk_col[1]][i]
//         group key = (key 0, key 1), each read from a fact column or from
//                     the payload column of a dim row; accumulate the fact
//                     values of row i.
// A dim with no match drops the row (inner join); several matches repeat it.
// key_src[k] is 0 for fact column key_col[k], or 1 + d for the payload of dim d.
int64_t oracle_pipeline(int nfact, const void* const* fact, const int* fact_types, int64_t n,
                        int nterms, const int* term_col, const int* term_op,
                        const int64_t* term_lo, const int64_t* term_hi, int ndims,
                        const int* dim_fk_col, const void* const* dim_key,
                        const int* dim_key_type, const int64_t* dim_n,
                        const void* const* dim_payload, const int* dim_payload_type,
                        int nkeys, const int* key_src, const int* key_col, int naggs,
                        const int* agg_op, const int* agg_col, int64_t* out_keys,
                        int64_t* out_aggs, int64_t cap) {
  (void)nfact;
  Predicate pred{nterms, term_col, term_op, term_lo, term_hi};
  std::vector<std::unordered_map<int64_t, std::vector<uint32_t>>> dim_map(ndims);
  for (int d = 0; d < ndims; ++d)
    for (int64_t b = 0; b < dim_n[d]; ++b)
      dim_map[d][read_value(dim_key[d], dim_key_type[d], b)].push_back(static_cast<uint32_t>(b));

  GroupMap groups;
  if (nkeys == 0) groups[std::vector<int64_t>()].resize(naggs);
  const std::vector<uint32_t> no_dim(1, 0);  // stands in for an absent dim
  std::vector<int64_t> key(nkeys);
  for (int64_t i = 0; i < n; ++i) {
    if (!pred.holds(fact, fact_types, i)) continue;
    const std::vector<uint32_t>* match[2] = {&no_dim, &no_dim};
    bool dropped = false;
    for (int d = 0; d < ndims; ++d) {
      int c = dim_fk_col[d];
      auto it = dim_map[d].find(read_value(fact[c], fact_types[c], i));
      if (it == dim_map[d].end()) {
        dropped = true;
        break;
      }
      match[d] = &it->second;
    }
    if (dropped) continue;
    for (uint32_t b0 : *match[0]) {
      for (uint32_t b1 : *match[1]) {
        const uint32_t dim_row[2] = {b0, b1};
        for (int k = 0; k < nkeys; ++k) {
          if (key_src[k] == 0) {
            key[k] = read_value(fact[key_col[k]], fact_types[key_col[k]], i);
          } else {
            int d = key_src[k] - 1;
            key[k] = read_value(dim_payload[d], dim_payload_type[d], dim_row[d]);
          }
        }
        std::vector<AggState>& st = groups[key];
        if (st.empty()) st.resize(naggs);
        for (int a = 0; a < naggs; ++a) {
          int64_t v = agg_op[a] == OA_COUNT
                          ? 0
                          : read_value(fact[agg_col[a]], fact_types[agg_col[a]], i);
          st[a].add(v);
        }
      }
    }
  }
  return emit_groups(groups, nkeys, naggs, agg_op, out_keys, out_aggs, cap);
}

// Semi-join: writes the probe row ids p (ascending) for which some build
// row b has build[b] == probe[p]; returns their number (out holds np).
int64_t oracle_semi_join(const void* build, const void* probe, int key_type, int64_t nb,
                         int64_t np, uint32_t* out) {
  std::unordered_set<int64_t> keys;
  for (int64_t b = 0; b < nb; ++b) keys.insert(read_value(build, key_type, b));
  int64_t written = 0;
  for (int64_t p = 0; p < np; ++p)
    if (keys.count(read_value(probe, key_type, p))) out[written++] = static_cast<uint32_t>(p);
  return written;
}

// Late materialisation: out[i] = col[idx[i]] widened to int64, i < n.
void oracle_gather(const void* col, int type, const uint32_t* idx, int64_t n, int64_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = read_value(col, type, idx[i]);
}

// Order-by / top-N over a result table of n rows: row r has the order value
// order[r] (int64, or binary64 when order_is_double) and the key tuple
// (keys[0][r], ..., keys[nkeys-1][r]). Rows are sorted by the order value,
// descending when desc, ties by the key tuple ascending (signed,
// lexicographic); the first min(limit, n) row positions go to out. Returns
// that count.
int64_t oracle_topn(int64_t n, const void* order, int order_is_double, int desc, int nkeys,
                    const int64_t* const* keys, int64_t limit, uint32_t* out) {
  std::vector<uint32_t> rows(static_cast<size_t>(n));
  std::iota(rows.begin(), rows.end(), 0u);
  auto value_less = [&](uint32_t a, uint32_t b) {
    if (order_is_double) {
      const double x = static_cast<const double*>(order)[a], y = static_cast<const double*>(order)[b];
      return x < y;
    }
    return static_cast<const int64_t*>(order)[a] < static_cast<const int64_t*>(order)[b];
  };
  auto before = [&](uint32_t a, uint32_t b) {
    const bool lt = value_less(a, b), gt = value_less(b, a);
    if (lt || gt) return desc ? gt : lt;
    for (int k = 0; k < nkeys; ++k)
      if (keys[k][a] != keys[k][b]) return keys[k][a] < keys[k][b];
    return a < b;
  };
  std::sort(rows.begin(), rows.end(), before);
  const int64_t m = std::min<int64_t>(limit, n);
  for (int64_t i = 0; i < m; ++i) out[i] = rows[i];
  return m;
}

// Group-by on a string key, optionally with one integer key: row i's
// string is bytes[offsets[i] .. offsets[i+1]) (Arrow layout), its integer
// key ikey[i] when ikey_type != 0. Groups are ordered by (string, integer
// key), strings byte-wise as unsigned bytes (a prefix first). Per group:
// out_row = the smallest row id of the group, out_ikey = its integer key,
// out_aggs[a * cap + g] = aggregate a as in oracle_groupby. Returns the group
// count; writes the first cap groups.
int64_t oracle_groupby_str(int64_t n, const int64_t* offsets, const uint8_t* bytes,
                           const void* ikey, int ikey_type, int nvals, const void* const* vals,
                           const int* val_types, int naggs, const int* agg_op,
                           const int* agg_col, uint32_t* out_row, int64_t* out_ikey,
                           int64_t* out_aggs, int64_t cap) {
  (void)nvals;
  struct Group {
    uint32_t first;
    std::vector<AggState> acc;
  };
  std::map<std::pair<std::string, int64_t>, Group> groups;
  for (int64_t i = 0; i < n; ++i) {
    std::string key(reinterpret_cast<const char*>(bytes + offsets[i]),
                    static_cast<size_t>(offsets[i + 1] - offsets[i]));
    const int64_t k2 = ikey_type ? read_value(ikey, ikey_type, i) : 0;
    auto it = groups.find({key, k2});
    if (it == groups.end()) {
      Group g;
      g.first = static_cast<uint32_t>(i);
      g.acc.resize(naggs);
      it = groups.emplace(std::make_pair(key, k2), std::move(g)).first;
    }
    for (int a = 0; a < naggs; ++a) {
      const int64_t v = agg_op[a] == OA_COUNT ? 0 : read_value(vals[agg_col[a]], val_types[agg_col[a]], i);
      it->second.acc[a].add(v);
    }
  }
  int64_t g = 0;
  for (const auto& kv : groups) {
    if (g < cap) {
      out_row[g] = kv.second.first;
      out_ikey[g] = kv.first.second;
      for (int a = 0; a < naggs; ++a) out_aggs[a * cap + g] = kv.second.acc[a].result(agg_op[a]);
    }
    ++g;
  }
  return g;
}

}  // extern "C"
