// C-ABI entry points of librel.so (declared in include/rel.h).
//
// Every call validates its arguments on the host before touching the HIP
// runtime, so malformed requests fail without a GPU. It then carves the
// caller's workspace into the operator's hash tables and counters, and
// enqueues the kernels on the caller's stream. Nothing here allocates device
// memory and nothing here falls back to the CPU.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "rel.h"

namespace rel {

namespace {

thread_local std::string g_error;

rel_status fail(rel_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

}  // namespace

int set_last_error(int status, const char* msg) {
  g_error = msg ? msg : "";
  return status;
}

void clear_last_error() { g_error.clear(); }

namespace {

constexpr int64_t kMaxRows = 0xFFFFFFFELL;  // row ids must stay below the all-ones value

// Bloom filters: bits per key of the filter a join builds (about 0.1% false
// positives), and the bytes of a filter of n keys at `bits` per key: a
// power-of-two number of 32-byte blocks.
constexpr int kBloomBitsPerKey = 16;
size_t bloom_bytes(int64_t n, int bits) {
  uint64_t want = (static_cast<uint64_t>(n > 0 ? n : 1) * static_cast<uint64_t>(bits) + 255) / 256;
  uint64_t blocks = 1;
  while (blocks < want) blocks <<= 1;
  return static_cast<size_t>(blocks) * 32;
}
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Workspace of rel_filter (the bitmap path): per tile of kFilterTile rows its
// selection bitmap (kFilterTile / 32 words) and its count (padded to whole
// groups of kFilterGroupTiles), and per group its offset.
struct FilterLayout {
  int64_t tiles = 1;
  size_t bitmap_off = 0, count_off = 0, offset_off = 0, end = 0;
};

FilterLayout filter_layout(int64_t n) {
  FilterLayout L;
  L.tiles = n > 0 ? (n + kFilterTile - 1) / kFilterTile : 1;
  const size_t t = static_cast<size_t>(L.tiles);
  const size_t groups = (t + kFilterGroupTiles - 1) / kFilterGroupTiles;
  L.bitmap_off = 0;
  L.count_off = align_up(t * (kFilterTile / 32) * 4);
  L.offset_off = L.count_off + align_up(groups * kFilterGroupTiles * 4);
  L.end = L.offset_off + align_up(groups * 8);
  return L;
}

uint64_t next_pow2(uint64_t v) {
  uint64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

bool valid_type(int32_t t) { return t == REL_I8 || t == REL_I32 || t == REL_I64; }
int type_bits(int32_t t) { return t == REL_I8 ? 8 : (t == REL_I32 ? 32 : 64); }

float load_factor(const rel_tuning* t) {
  float lf = (t && t->load_factor > 0.0f) ? t->load_factor : 0.5f;
  return lf > 0.9f ? 0.9f : lf;
}

rel_status check_tuning(const rel_tuning* t) {
  if (!t) return REL_OK;
  if (t->load_factor < 0.0f || t->load_factor > 0.9f || std::isnan(t->load_factor))
    return fail(REL_EINVAL, "tuning.load_factor must be in (0, 0.9] (or 0 for the default)");
  if (t->block < 0 || t->block > 1024 || t->block % 64 != 0)
    return fail(REL_EINVAL, "tuning.block must be a multiple of 64 up to 1024 (or 0)");
  if (t->grid < 0) return fail(REL_EINVAL, "tuning.grid must be >= 0");
  if (t->lds_slots < -1 || (t->lds_slots > 0 && (t->lds_slots & (t->lds_slots - 1)) != 0))
    return fail(REL_EINVAL, "tuning.lds_slots must be -1, 0 or a power of two");
  if (t->flags & ~(REL_TUNE_NO_DIRECT | REL_TUNE_BLOOM))
    return fail(REL_EINVAL, "tuning.flags: unknown bits");
  if (t->chunk_tiles < 0) return fail(REL_EINVAL, "tuning.chunk_tiles must be >= 0");
  if (t->replicas < 0 || t->replicas > 256)
    return fail(REL_EINVAL, "tuning.replicas must be in [0, 256]");
  if (t->fanout < -1 || (t->fanout > 0 && (t->fanout < 4 || t->fanout > (1 << kPartMaxBits) ||
                                          (t->fanout & (t->fanout - 1)) != 0)))
    return fail(REL_EINVAL, "tuning.fanout must be -1, 0 or a power of two in [4, %d]",
                1 << kPartMaxBits);
  return REL_OK;
}

rel_status check_column(const rel_column* c, const char* what) {
  if (!c) return fail(REL_EINVAL, "%s: NULL column", what);
  if (!valid_type(c->type)) return fail(REL_EINVAL, "%s: invalid type %d", what, c->type);
  if (c->len < 0 || c->len > kMaxRows)
    return fail(REL_EUNSUPPORTED, "%s: length %lld outside [0, 2^32-2]", what, (long long)c->len);
  if (c->len > 0 && !c->data) return fail(REL_EINVAL, "%s: NULL data", what);
  return REL_OK;
}

rel_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (ws_bytes < need)
    return fail(REL_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if (!ws) return fail(REL_EINVAL, "NULL workspace");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
    return fail(REL_EINVAL, "workspace must be 256-byte aligned");
  return REL_OK;
}

bool debug_sync() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("REL_DEBUG_SYNC");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

rel_status after_launch(hipStream_t s, const char* what) {
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && debug_sync()) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(REL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return REL_OK;
}

// ---------------------------------------------------------- hash map sizes

struct MapLayout {
  uint64_t cap;
  size_t slot_bytes;
  bool compact;  // 16-byte buckets of 16-bit entries; cap counts buckets
  int rbits;
  uint64_t over_cap;  // compact: overflow set slots (at oob_vals_off)
  size_t slots_off, oob_count_off, oob_vals_off, end;
  uint64_t nkeys;
  uint64_t direct_cap;          // 0: none
  size_t dbits_off, dvals_off;  // dvals_off 0: no payload array
};

// Direct tables cover key ranges up to this many times the build size.
constexpr uint64_t kDirectSpan = 2;

// Reserves a direct table after layout m (int32 keys): a presence bitmap and,
// with a payload, 4 bytes per entry; the build uses it if the keys allow.
void add_direct(MapLayout& m, int64_t n, bool payload) {
  m.direct_cap = (kDirectSpan * static_cast<uint64_t>(n > 0 ? n : 1) + 63) / 64 * 64;
  m.dbits_off = m.end;
  m.end = align_up(m.dbits_off + m.direct_cap / 8);
  m.dvals_off = 0;
  if (payload) {
    m.dvals_off = m.end;
    m.end = align_up(m.dvals_off + m.direct_cap * 4);
  }
}

// Compact membership sets: eight 16-bit entries per 16-byte bucket, filled
// to at most this load factor; used when the remainder fits 14 bits.
constexpr double kCsetLoad = 0.75;
constexpr int kCsetMinBucketBits = 18;

MapLayout map_layout(int32_t key_type, int64_t n, float lf, size_t base, bool key_only = false,
                     bool allow_compact = false) {
  MapLayout m;
  m.compact = false;
  m.rbits = 0;
  m.over_cap = 0;
  m.nkeys = static_cast<uint64_t>(n > 0 ? n : 0);
  m.direct_cap = 0;
  m.dbits_off = m.dvals_off = 0;
  if (key_only && allow_compact && key_type == REL_I32) {
    const uint64_t buckets = next_pow2(static_cast<uint64_t>(std::ceil(n / (8 * kCsetLoad))));
    int bits = 0;
    while ((1ULL << bits) < buckets) ++bits;
    if (bits >= kCsetMinBucketBits && bits <= 31) {
      // buckets, then the header (overflow sentinel count, duplicate flag),
      // then the overflow set, sized so that even every key would fit
      m.compact = true;
      m.rbits = 32 - bits;
      m.cap = buckets;
      m.slot_bytes = 16;
      m.slots_off = base;
      m.oob_count_off = align_up(m.slots_off + m.cap * 16);
      m.over_cap = next_pow2(2 * static_cast<uint64_t>(n) + 64);
      m.oob_vals_off = m.oob_count_off + kAlign;
      m.end = align_up(m.oob_vals_off + m.over_cap * 4);
      return m;
    }
  }
  uint64_t want = static_cast<uint64_t>(std::ceil(static_cast<double>(n) / lf));
  m.cap = next_pow2(want < 64 ? 64 : want);
  if (m.cap <= static_cast<uint64_t>(n)) m.cap = next_pow2(static_cast<uint64_t>(n) + 1);
  size_t slot = key_type == REL_I64 ? 16 : (key_only ? 4 : 8);
  m.slot_bytes = slot;
  m.slots_off = base;
  m.oob_count_off = align_up(m.slots_off + m.cap * slot);
  m.oob_vals_off = m.oob_count_off + kAlign;
  m.end = align_up(m.oob_vals_off + static_cast<size_t>(n > 0 ? n : 1) * 4);
  return m;
}

MapDesc map_desc(const MapLayout& l, int32_t key_type, unsigned char* ws) {
  MapDesc d;
  d.key_type = key_type == REL_I64 ? kI64 : kI32;
  d.key_only = (key_type != REL_I64 && (l.slot_bytes == 4 || l.compact)) ? 1 : 0;
  d.compact = l.compact ? 1 : 0;
  d.rbits = l.rbits;
  d.over = l.compact ? reinterpret_cast<uint32_t*>(ws + l.oob_vals_off) : nullptr;
  d.over_cap = l.compact ? l.over_cap : 0;
  d.cap = l.cap;
  d.slots = ws + l.slots_off;
  d.oob_count = reinterpret_cast<unsigned long long*>(ws + l.oob_count_off);
  d.dup = reinterpret_cast<int32_t*>(ws + l.oob_count_off + 8);
  d.oob_vals = reinterpret_cast<uint32_t*>(ws + l.oob_vals_off);
  d.nkeys = l.nkeys;
  d.direct_cap = l.direct_cap;
  d.dstate = reinterpret_cast<int32_t*>(ws + l.oob_count_off + 16);
  d.dbits = l.direct_cap ? reinterpret_cast<uint32_t*>(ws + l.dbits_off) : nullptr;
  d.dvals = (l.direct_cap && l.dvals_off) ? static_cast<void*>(ws + l.dvals_off) : nullptr;
  return d;
}

// ---------------------------------------------------------- group tables

struct GroupPlan {
  GroupKeyPack kp;
  AccPlan ap;
  int32_t agg_acc[REL_MAX_AGGS];
  int32_t words;
};

int acc_index(AccPlan& ap, int32_t kind, int32_t col) {
  for (int a = 0; a < ap.nacc; ++a)
    if (ap.kind[a] == kind && ap.col[a] == col) return a;
  ap.kind[ap.nacc] = kind;
  ap.col[ap.nacc] = col;
  return ap.nacc++;
}

// Key types and aggregates -> packing and accumulators (validated already).
rel_status group_plan(int nkeys, const int32_t* key_types, int naggs, const rel_agg* aggs,
                      GroupPlan& gp) {
  std::memset(&gp, 0, sizeof gp);
  gp.kp.nkeys = nkeys;
  int bits = 0;
  for (int k = 0; k < nkeys; ++k) {
    gp.kp.type[k] = key_types[k];
    bits += type_bits(key_types[k]);
  }
  if (bits > 64)
    return fail(REL_EUNSUPPORTED, "group key tuple of %d bits; at most 64 are supported", bits);
  gp.kp.shift0 = nkeys == 2 ? type_bits(key_types[1]) : 0;
  for (int a = 0; a < naggs; ++a) {
    switch (aggs[a].op) {
      case REL_SUM:
      case REL_AVG: gp.agg_acc[a] = acc_index(gp.ap, kAccSum, aggs[a].col); break;
      case REL_MIN: gp.agg_acc[a] = acc_index(gp.ap, kAccMin, aggs[a].col); break;
      case REL_MAX: gp.agg_acc[a] = acc_index(gp.ap, kAccMax, aggs[a].col); break;
      default: gp.agg_acc[a] = -1; break;
    }
  }
  // Not rounded to an even count: tables stay 1/(words + 1) smaller (fewer
  // bytes to fill, scan and hold in LDS); an odd stride also spreads an LDS
  // table over more banks, which measured neutral on the fused kernel.
  gp.words = 2 + gp.ap.nacc;
  return REL_OK;
}

struct GroupLayout {
  uint64_t cap;
  int replicas;
  size_t slots_off, overflow_off, end;
};

// Replicas of the global group table: with few groups (all of them fit the
// per-workgroup LDS tables) merges are spread over kGroupReplicas copies.
constexpr int kGroupReplicas = 64;

// Default LDS bytes for dim tables in the fused pipeline.
constexpr size_t kDimLdsDefault = 32768;
// Largest LDS group table of the fused pipeline, and the group count (in
// multiples of its slots) beyond which the small default table is used.
constexpr size_t kGroupLdsMax = 131072;
constexpr int64_t kGroupLdsShare = 32;

GroupLayout group_layout(const GroupPlan& gp, int64_t max_groups, float lf, size_t base,
                         int replicas = 1) {
  GroupLayout g;
  uint64_t want = static_cast<uint64_t>(std::ceil(static_cast<double>(max_groups < 1 ? 1 : max_groups) / lf));
  g.cap = next_pow2(want < 64 ? 64 : want);
  g.replicas = replicas;
  g.slots_off = base;
  g.overflow_off = align_up(g.slots_off + replicas * (g.cap + 1) * gp.words * 8);
  g.end = g.overflow_off + kAlign;
  return g;
}

GroupDesc group_desc(const GroupPlan& gp, const GroupLayout& l, unsigned char* ws,
                     int64_t* d_groups) {
  GroupDesc g;
  g.kp = gp.kp;
  g.ap = gp.ap;
  g.cap = l.cap;
  g.words = gp.words;
  g.replicas = l.replicas;
  g.slots = reinterpret_cast<uint64_t*>(ws + l.slots_off);
  g.overflow = reinterpret_cast<int32_t*>(ws + l.overflow_off);
  g.d_groups = reinterpret_cast<unsigned long long*>(d_groups);
  return g;
}

rel_status check_aggs(const rel_agg* aggs, int naggs, int ncols, const char* what) {
  if (naggs < 1 || naggs > REL_MAX_AGGS)
    return fail(REL_EINVAL, "%s: 1..%d aggregates required", what, REL_MAX_AGGS);
  if (!aggs) return fail(REL_EINVAL, "%s: NULL aggregates", what);
  for (int a = 0; a < naggs; ++a) {
    if (aggs[a].op < REL_SUM || aggs[a].op > REL_AVG)
      return fail(REL_EINVAL, "%s: aggregate %d has invalid op %d", what, a, aggs[a].op);
    if (aggs[a].op != REL_COUNT && (aggs[a].col < 0 || aggs[a].col >= ncols))
      return fail(REL_EINVAL, "%s: aggregate %d reads column %d of %d", what, a, aggs[a].col, ncols);
  }
  return REL_OK;
}

int default_lds_slots(const rel_tuning* t, int64_t max_groups, int words, size_t budget) {
  if (t && t->lds_slots == -1) return 0;
  uint64_t max_by_lds = next_pow2(budget / (static_cast<size_t>(words) * 8) + 1) / 2;
  uint64_t want = (t && t->lds_slots > 0) ? static_cast<uint64_t>(t->lds_slots)
                                          : next_pow2(2 * static_cast<uint64_t>(max_groups < 32 ? 32 : max_groups));
  if (want > max_by_lds) want = max_by_lds;
  return static_cast<int>(want);
}

// Replicas of the global group table: a tuned count, else kGroupReplicas
// when every group fits the LDS tables (only their flushes reach the global
// table), else, for tables up to kSpillTableBytes, as many as keep the copies
// within kReplicaBytes (at most kSpillReplicas): rows that spill from LDS
// update the global table with device-scope atomics, which serialise per
// cache line, so copies spread the hot lines (workgroup w updates copy
// w mod replicas, and w mod 8 is its XCD). Larger tables already spread their
// atomics over many lines; copies would only add fill and merge traffic.
constexpr int kSpillReplicas = 32;
constexpr uint64_t kReplicaBytes = 256ull << 20;
constexpr uint64_t kSpillTableBytes = 1ull << 20;

int group_replicas(const rel_tuning* t, int64_t max_groups, int lds_slots, int words, float lf) {
  if (t && t->replicas > 0) return t->replicas;
  if (lds_slots > 0 && 2 * max_groups <= lds_slots) return kGroupReplicas;
  const uint64_t want = static_cast<uint64_t>(std::ceil(static_cast<double>(max_groups < 1 ? 1 : max_groups) / lf));
  const uint64_t table = next_pow2(want < 64 ? 64 : want) * static_cast<uint64_t>(words) * 8;
  int r = 1;
  if (table > kSpillTableBytes) return r;
  while (r < kSpillReplicas && 2 * r * table <= kReplicaBytes) r *= 2;
  return r;
}

int groupby_replicas(const rel_tuning* t, int64_t max_groups, const GroupPlan& gp) {
  return group_replicas(t, max_groups, default_lds_slots(t, max_groups, gp.words, 32768), gp.words,
                        load_factor(t));
}

FinalizeParams finalize_params(const GroupDesc& g, const GroupPlan& gp, const rel_agg* aggs,
                               int naggs, void* const* out_keys, const int32_t* key_types,
                               void* const* out_aggs, int64_t cap) {
  FinalizeParams f;
  std::memset(&f, 0, sizeof f);
  f.g = g;
  f.naggs = naggs;
  for (int a = 0; a < naggs; ++a) {
    f.op[a] = aggs[a].op;
    f.acc[a] = gp.agg_acc[a] < 0 ? 0 : gp.agg_acc[a];
    f.out_aggs[a] = out_aggs ? out_aggs[a] : nullptr;
  }
  for (int k = 0; k < gp.kp.nkeys; ++k) {
    f.out_keys[k] = out_keys ? out_keys[k] : nullptr;
    f.out_key_type[k] = key_types[k];
  }
  f.cap = cap;
  return f;
}

rel_status check_outputs(void* const* out_keys, int nkeys, void* const* out_aggs, int naggs,
                         int64_t cap, const void* d_groups) {
  if (cap < 0) return fail(REL_EINVAL, "negative output capacity");
  if (!d_groups) return fail(REL_EINVAL, "NULL group count");
  if (cap > 0) {
    if (nkeys > 0 && !out_keys) return fail(REL_EINVAL, "NULL key outputs");
    for (int k = 0; k < nkeys; ++k)
      if (!out_keys[k]) return fail(REL_EINVAL, "NULL output for key %d", k);
    if (!out_aggs) return fail(REL_EINVAL, "NULL aggregate outputs");
    for (int a = 0; a < naggs; ++a)
      if (!out_aggs[a]) return fail(REL_EINVAL, "NULL output for aggregate %d", a);
  }
  return REL_OK;
}

// ---------------------------------------------------------- pipeline plan

struct PipeLayout {
  MapLayout dim[REL_MAX_DIMS];
  GroupPlan gp;
  GroupLayout group;
  int32_t key_types[REL_MAX_KEYS];
  int lds_slots;
  size_t end;
};

rel_status check_pipeline(const rel_pipeline_desc* d) {
  if (!d) return fail(REL_EINVAL, "NULL pipeline description");
  if (d->n_fact < 1 || d->n_fact > REL_MAX_FACT_COLS || !d->fact)
    return fail(REL_EINVAL, "pipeline: 1..%d fact columns required", REL_MAX_FACT_COLS);
  for (int c = 0; c < d->n_fact; ++c) {
    rel_status st = check_column(&d->fact[c], "pipeline fact column");
    if (st) return st;
    if (d->fact[c].idx) return fail(REL_EUNSUPPORTED, "pipeline: fact columns take no idx");
    if (d->fact[c].len != d->fact[0].len)
      return fail(REL_EINVAL, "pipeline: fact columns differ in length");
  }
  if (d->n_preds < 0 || d->n_preds > REL_MAX_TERMS || (d->n_preds > 0 && !d->preds))
    return fail(REL_EINVAL, "pipeline: 0..%d predicate terms", REL_MAX_TERMS);
  for (int t = 0; t < d->n_preds; ++t) {
    if (d->preds[t].col < 0 || d->preds[t].col >= d->n_fact)
      return fail(REL_EINVAL, "pipeline: term %d reads column %d", t, d->preds[t].col);
    if (d->preds[t].op < REL_LT || d->preds[t].op > REL_RANGE)
      return fail(REL_EINVAL, "pipeline: term %d has invalid op %d", t, d->preds[t].op);
  }
  if (d->n_dims < 0 || d->n_dims > REL_MAX_DIMS || (d->n_dims > 0 && !d->dims))
    return fail(REL_EINVAL, "pipeline: 0..%d dims", REL_MAX_DIMS);
  for (int i = 0; i < d->n_dims; ++i) {
    const rel_dim& dm = d->dims[i];
    if (dm.fact_col < 0 || dm.fact_col >= d->n_fact)
      return fail(REL_EINVAL, "pipeline: dim %d foreign key column %d", i, dm.fact_col);
    rel_status st = check_column(&dm.key, "pipeline dim key");
    if (st) return st;
    if (dm.key.idx) return fail(REL_EUNSUPPORTED, "pipeline: dim columns take no idx");
    if (dm.key.type == REL_I8) return fail(REL_EUNSUPPORTED, "pipeline: int8 dim keys");
    int32_t fk = d->fact[dm.fact_col].type;
    if (!(fk == dm.key.type || (fk == REL_I8 && dm.key.type == REL_I32) ||
          (fk == REL_I8 && dm.key.type == REL_I64) || (fk == REL_I32 && dm.key.type == REL_I64)))
      return fail(REL_EINVAL, "pipeline: dim %d key type %d cannot hold foreign keys of type %d", i,
                  dm.key.type, fk);
    if (dm.has_payload) {
      st = check_column(&dm.payload, "pipeline dim payload");
      if (st) return st;
      if (dm.payload.idx) return fail(REL_EUNSUPPORTED, "pipeline: dim columns take no idx");
      if (dm.payload.type == REL_I64) return fail(REL_EUNSUPPORTED, "pipeline: int64 dim payloads");
      if (dm.payload.len != dm.key.len)
        return fail(REL_EINVAL, "pipeline: dim %d payload and key lengths differ", i);
    }
  }
  if (d->n_keys < 0 || d->n_keys > REL_MAX_KEYS || (d->n_keys > 0 && !d->keys))
    return fail(REL_EINVAL, "pipeline: 0..%d group keys", REL_MAX_KEYS);
  for (int k = 0; k < d->n_keys; ++k) {
    const rel_key_ref& kr = d->keys[k];
    if (kr.src == REL_KEY_FACT) {
      if (kr.col < 0 || kr.col >= d->n_fact) return fail(REL_EINVAL, "pipeline: key %d column", k);
    } else if (kr.src == REL_KEY_DIM) {
      if (kr.col < 0 || kr.col >= d->n_dims || !d->dims[kr.col].has_payload)
        return fail(REL_EINVAL, "pipeline: key %d needs a dim with a payload", k);
    } else {
      return fail(REL_EINVAL, "pipeline: key %d has invalid source %d", k, kr.src);
    }
  }
  rel_status st = check_aggs(d->aggs, d->n_aggs, d->n_fact, "pipeline");
  if (st) return st;
  if (d->max_groups < 0) return fail(REL_EINVAL, "pipeline: negative max_groups");
  return check_tuning(d->tuning);
}

// Workspace layout of plan d from byte offset `base`. Batched plans keep
// every dim in plain slot arrays (no compact sets), so that all instances of
// a shape share one kernel variant.
rel_status pipeline_layout(const rel_pipeline_desc* d, PipeLayout& L, bool batch = false,
                           size_t base = 0) {
  const float lf = load_factor(d->tuning);
  size_t off = base;
  for (int i = 0; i < d->n_dims; ++i) {
    // membership-only int32 dims keep keys alone (4-byte slots)
    const bool key_only = d->dims[i].key.type == REL_I32 && !d->dims[i].has_payload;
    // dims fill their tables to the tuning's load factor (default 0.5: at
    // 0.75 a third more probes meet a full first bucket, and the fused pass
    // measured 10% slower on 600M fact rows against 1.5M- and 10k-key dims)
    L.dim[i] = map_layout(d->dims[i].key.type, d->dims[i].key.len, lf, off, key_only, !batch);
    const bool no_direct = d->tuning && (d->tuning->flags & REL_TUNE_NO_DIRECT);
    if (d->dims[i].key.type == REL_I32 && !no_direct)
      add_direct(L.dim[i], d->dims[i].key.len, d->dims[i].has_payload != 0);
    off = L.dim[i].end;
  }
  for (int k = 0; k < d->n_keys; ++k) {
    const rel_key_ref& kr = d->keys[k];
    L.key_types[k] = kr.src == REL_KEY_FACT ? d->fact[kr.col].type : d->dims[kr.col].payload.type;
  }
  rel_status st = group_plan(d->n_keys, L.key_types, d->n_aggs, d->aggs, L.gp);
  if (st) return st;
  // Up to kGroupLdsMax: rows of groups beyond the LDS table pay device-scope
  // atomics in the global table, which costs more than the occupancy a large
  // table takes (measured on join + group-by instances of 1k-80k groups) -
  // while the table holds a useful share of the groups. Beyond
  // kGroupLdsShare times its slots (1M-group queries) the 16 KB table, at
  // full occupancy, is faster.
  L.lds_slots = default_lds_slots(d->tuning, d->max_groups, L.gp.words, kGroupLdsMax);
  if (!(d->tuning && d->tuning->lds_slots != 0) &&
      d->max_groups > kGroupLdsShare * static_cast<int64_t>(L.lds_slots))
    L.lds_slots = default_lds_slots(d->tuning, d->max_groups, L.gp.words, 16384);
  L.group = group_layout(L.gp, d->max_groups, lf, off,
                         group_replicas(d->tuning, d->max_groups, L.lds_slots, L.gp.words, lf));
  L.end = L.group.end;
  return REL_OK;
}

// Row spec of a single plan (see the fused kernels): the sources of its group
// keys and values when they fit a compile-time form, else 0 (generic). Dims
// must be int32 hash tables read from HBM, every accumulator must read one
// int64 fact column, and each group key must be a dim payload or an int8 or
// int32 fact column. The launcher falls back to the generic kernel for a
// spec it has not built.
int row_spec(const rel_pipeline_desc* d, const PipeLayout& L, PipelineParams& p) {
  for (int i = 0; i < d->n_dims; ++i) {
    const int c = d->dims[i].fact_col;
    if (d->dims[i].key.type != REL_I32 || p.dim[i].in_lds) return 0;
    if (d->fact[c].type != REL_I32 || !p.fact_vec[c]) return 0;
  }
  // at most one predicate term, on an aligned int32 column, as a range of
  // the widened value: [lo, hi) clamped to the int32 domain
  if (d->n_preds > 1) return 0;
  if (d->n_preds == 1) {
    const rel_pred& t = d->preds[0];
    if (d->fact[t.col].type != REL_I32 || !p.fact_vec[t.col]) return 0;
    const int64_t dmin = INT32_MIN, dend = static_cast<int64_t>(INT32_MAX) + 1;
    auto clamp = [&](int64_t v) { return v < dmin ? dmin : (v > dend ? dend : v); };
    int64_t lo = dmin, hi = dend;
    switch (t.op) {
      case REL_LT: hi = clamp(t.lo); break;
      case REL_LE: hi = t.lo >= INT32_MAX ? dend : clamp(t.lo + 1); break;
      case REL_GT: lo = t.lo >= INT32_MAX ? dend : clamp(t.lo + 1); break;
      case REL_GE: lo = clamp(t.lo); break;
      case REL_EQ:
        lo = clamp(t.lo);
        hi = (t.lo < dmin || t.lo > INT32_MAX) ? lo : lo + 1;
        break;
      case REL_RANGE: lo = clamp(t.lo); hi = clamp(t.hi); break;
      default: return 0;  // NE is no single range
    }
    if (hi < lo) hi = lo;
    p.spec_lo = lo;
    p.spec_span = static_cast<uint64_t>(hi - lo);
  }
  const AccPlan& ap = L.gp.ap;
  if (ap.nacc < 1) return 0;
  for (int a = 0; a < ap.nacc; ++a)
    if (ap.col[a] != ap.col[0]) return 0;
  if (d->fact[ap.col[0]].type != REL_I64) return 0;
  int k[REL_MAX_KEYS] = {0, 0};  // 0 none, 1 dim 0, 2 dim 1, 3 int8 fact, 4 int32 fact
  for (int j = 0; j < d->n_keys; ++j) {
    const rel_key_ref& kr = d->keys[j];
    if (kr.src == REL_KEY_DIM) {
      k[j] = 1 + kr.col;
    } else {
      const int32_t t = d->fact[kr.col].type;
      if (t == REL_I8) k[j] = 3;
      else if (t == REL_I32) k[j] = 4;
      else return 0;
      p.spec_key[j] = d->fact[kr.col].data;
    }
  }
  p.spec_val = static_cast<const int64_t*>(d->fact[ap.col[0]].data);
  return k[0] | (k[1] << 3) | (1 << 6);
}

// Kernel parameters of plan d (layout L) over workspace w, and the builds of
// its dims. Batched plans keep every dim in HBM.
void plan_params(const rel_pipeline_desc* d, const PipeLayout& L, unsigned char* w,
                 int64_t* d_groups, bool batch, PipelineParams& p,
                 MapBuildParams b[REL_MAX_DIMS]) {
  const DeviceInfo& di = device_info();
  const rel_tuning* t = d->tuning;
  std::memset(&p, 0, sizeof p);
  const int64_t n = d->fact[0].len;
  for (int c = 0; c < d->n_fact; ++c) {
    p.fact[c] = d->fact[c].data;
    p.fact_type[c] = d->fact[c].type;
    p.fact_vec[c] = (reinterpret_cast<uintptr_t>(d->fact[c].data) % 16) == 0;
  }
  p.n = n;
  p.nterms = d->n_preds;
  for (int i = 0; i < d->n_preds; ++i) {
    p.term_col[i] = d->preds[i].col;
    p.term_op[i] = d->preds[i].op;
    p.term_lo[i] = d->preds[i].lo;
    p.term_hi[i] = d->preds[i].hi;
  }
  p.g = group_desc(L.gp, L.group, w, d_groups);
  for (int k = 0; k < d->n_keys; ++k) {
    p.key_src[k] = d->keys[k].src == REL_KEY_FACT ? 0 : 1 + d->keys[k].col;
    p.key_col[k] = d->keys[k].src == REL_KEY_FACT ? d->keys[k].col : 0;
  }

  // LDS: the group table, the per-wave row queues, then dim tables that fit
  // (smaller dims first).
  const size_t budget = static_cast<size_t>(di.lds_per_block);
  p.lds_slots = L.lds_slots;
  uint32_t stride = 0;  // bytes of one wave's row queue
  {
    // queued row fields: width 8 for int64 columns, else 4
    bool present[kQueueFields] = {};
    bool wide[kQueueFields] = {};
    present[kQRow] = true;
    for (int i = 0; i < d->n_dims; ++i) {
      present[kQFk0 + i] = true;
      wide[kQFk0 + i] = d->dims[i].key.type == REL_I64;
      present[kQSt0 + i] = true;
    }
    // The first two distinct value columns are gathered with the probes.
    int early[2] = {-1, -1};
    for (int a = 0; a < L.gp.ap.nacc; ++a) {
      const int c = L.gp.ap.col[a];
      p.acc_col[a] = c;
      p.acc_src[a] = -1;
      for (int k = 0; k < 2; ++k) {
        if (early[k] == c || early[k] < 0) {
          early[k] = c;
          p.acc_src[a] = k;
          break;
        }
      }
    }
    for (int k = 0; k < 2; ++k) p.early_col[k] = early[k];
    for (int f = 0; f < kQueueFields; ++f) {
      p.field_offset[f] = stride;
      p.field_wide[f] = wide[f] ? 1 : 0;
      if (present[f]) stride += kPipeQueue * (wide[f] ? 8 : 4);
    }
  }
  const size_t queues = static_cast<size_t>(kPipeThreads / kWave) * stride;
  // A single plan's group table grows up to four slots per group while the
  // table and the queues stay within the LDS share of a workgroup at full
  // occupancy (four workgroups of eight waves per CU): shorter hash runs at
  // no cost in resident waves (75 groups in 512 instead of 256 slots: the
  // star-schema plan's fused pass 2.66 -> 2.51 ms; at 1024 slots only two
  // workgroups fit and it takes 3.6 ms). Batched plans keep their LDS
  // classes.
  constexpr int kFusedBlocksPerCu = 4;
  if (!batch && !(t && t->lds_slots != 0) && p.lds_slots > 0) {
    const size_t share = budget / kFusedBlocksPerCu;
    while (static_cast<int64_t>(p.lds_slots) * 2 <= 4 * d->max_groups &&
           static_cast<size_t>(p.lds_slots) * 2 * L.gp.words * 8 + queues <= share)
      p.lds_slots *= 2;
  }
  size_t lds = 0;
  p.lds_group_offset = 0;
  lds += static_cast<size_t>(p.lds_slots) * L.gp.words * 8;
  lds = (lds + 15) / 16 * 16;
  p.queue_offset = static_cast<uint32_t>(lds);
  p.queue_stride = stride;
  lds += queues;
  // Dim tables go to LDS only when small: a large LDS copy costs resident
  // workgroups, and occupancy is what hides the probe latency.
  const size_t avail = budget > lds ? budget - lds : 0;
  size_t dim_budget = kDimLdsDefault;
  if (t && t->dim_lds_bytes > 0) dim_budget = static_cast<size_t>(t->dim_lds_bytes);
  if (t && t->dim_lds_bytes < 0) dim_budget = 0;
  if (dim_budget > avail) dim_budget = avail;
  p.ndims = d->n_dims;
  int order[REL_MAX_DIMS] = {0, 1};
  if (d->n_dims == 2 && L.dim[1].cap * L.dim[1].slot_bytes < L.dim[0].cap * L.dim[0].slot_bytes) {
    order[0] = 1;
    order[1] = 0;
  }
  size_t dim_used = 0;
  for (int oi = 0; oi < d->n_dims; ++oi) {
    const int i = order[oi];
    const rel_dim& dm = d->dims[i];
    p.dim[i].map = map_desc(L.dim[i], dm.key.type, w);
    p.dim[i].fk_col = dm.fact_col;
    const size_t bytes = L.dim[i].cap * L.dim[i].slot_bytes;
    if (!batch && dm.key.type == REL_I32 && !L.dim[i].compact && dim_used + bytes <= dim_budget) {
      // the LDS copy is of the slot array, which must then always be built
      p.dim[i].map.direct_cap = 0;
      p.dim[i].in_lds = 1;
      p.dim[i].lds_offset = static_cast<uint32_t>(lds);
      lds += bytes;
      dim_used += bytes;
    }
  }
  p.lds_bytes = static_cast<uint32_t>(lds);
  p.ntiles = n > 0 ? (n + kPipeTile - 1) / kPipeTile : 0;
  p.directable = 1;
  for (int i = 0; i < d->n_dims; ++i)
    if (p.dim[i].map.direct_cap == 0) p.directable = 0;
  if (!batch) p.spec = row_spec(d, L, p);
  for (int i = 0; i < d->n_dims; ++i) {
    const rel_dim& dm = d->dims[i];
    std::memset(&b[i], 0, sizeof b[i]);
    b[i].map = p.dim[i].map;
    b[i].keys = dm.key.data;
    b[i].type = dm.key.type;
    b[i].n = dm.key.len;
    if (dm.has_payload) {
      b[i].val_col = dm.payload.data;
      b[i].val_type = dm.payload.type;
    }
  }
}

// ------------------------------------------------------------ batch layout

// Units per work item of the batched phases.
constexpr uint64_t kFillChunk = 32768;   // words

// Bits of a direct-table slice that one workgroup sets in LDS during a batch
// build: 2^20 (128 KB) when a workgroup may hold that much, else the largest
// power of two that fits.
// Parts of a dim's build rows that the workgroups of one direct-table slice
// split between them (at most 512k rows each).
uint64_t slice_parts(uint64_t rows) {
  const uint64_t per = uint64_t(1) << 19;
  const uint64_t parts = (rows + per - 1) / per;
  return parts < 1 ? 1 : parts;
}

uint32_t direct_slice_bits() {
  uint64_t bits = 1u << 20;
  const uint64_t lds_bits = static_cast<uint64_t>(device_info().lds_per_block) * 8;
  while (bits > 32 * 1024 && bits > lds_bits) bits >>= 1;
  return static_cast<uint32_t>(bits);
}
constexpr uint64_t kSlotChunk = 16384;   // group slots (a multiple of the finalize chunk, 2048)
#ifndef REL_MAXCHUNK
#define REL_MAXCHUNK 32
#endif
constexpr int kMaxChunkTiles = REL_MAXCHUNK;
constexpr int kMaxBatch = 1 << 16;

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Words of a dim's slot array.
uint64_t map_words(const MapLayout& m, int32_t key_type) {
  if (key_type == REL_I64) return 2 * m.cap;
  return m.slot_bytes == 4 ? m.cap / 2 : m.cap;
}

// Spilled-row records of one batched plan (see RecDesc): the partitions,
// the record and aggregation-table sizes, and the regions' offsets (from the
// end of the uploaded block).
struct RecLayout {
  uint32_t parts = 0;  // 0: no records
  uint32_t agg_parts = 0, words = 0, nitems = 0, agg_slots = 0, narrow = 0;
  size_t recs = 0, parted = 0, rkeys = 0, pkeys = 0, counts = 0, item_n = 0, part_begin = 0;
  size_t cursor = 0;
};

// Workspace bound of a batch's records: plans are given records in order
// while their regions fit; the spilled rows of the others use device-scope
// atomics. (Served batches of 200M-row queries with 5k and 1M groups need
// about 4.8 GB each; at twice the one-at-a-time capacity, continuous
// batching took p50 / p99 248 / 450 ms with 32 GiB, 175 / 324 ms with
// 60 GiB, against 217 / 407 ms one at a time.)
constexpr uint64_t kRecordBudget = 64ull << 30;

// The workspace of a batch: first a block uploaded from the host in one
// copy (the fused-pass counter, then the per-instance kernel parameters and
// the work-item lists), then each instance's dim and group tables, then the
// record regions and the aggregation pieces.
struct BatchLayout {
  std::vector<PipeLayout> L;
  std::vector<size_t> base;
  std::vector<RecLayout> rec;
  size_t off_plans, off_builds, off_fins, off_fill, off_build_items, off_tile_items;
  size_t off_merge_items, off_fin_items, off_slice_items, off_win_items, blob;
  size_t off_pieces;  // from the end of the uploaded block
  uint64_t nfill, nbuild, ntile, nmerge, nfin, nslice, nwin;
  // windowed direct-table builds (2 per plan: dim d of plan i at 2i + d):
  // windows (0: not windowed) and region offsets from the end of the block
  std::vector<uint32_t> win_n;
  std::vector<size_t> win_pairs, win_cursor, win_begin;
  uint64_t piece_cap;
  uint32_t rec_plans, agg_lds_bytes;
  uint32_t slice_bits;  // direct-table slice of the second build pass
  int chunk_tiles;
  size_t end;
};

// LDS group tables above this size leave room for one fused-pass workgroup
// per CU; a plan that needs one takes records instead (on the 256-instance
// batch, its plans of 1025-2048 groups: 4.4 ms at one workgroup per CU, the
// batch 1.4 ms faster with records).
constexpr uint64_t kRecTableBytes = 65536;

// Records for a batched plan when its rows would spill from the fused
// pass's LDS table (more groups than half its slots) or its table exceeds
// kRecTableBytes, its accumulators read
// at most two value columns (gathered with the probes), its group count
// needs at most kMaxRecParts partitions of an aggregation table and
// tuning.fanout is not -1. The aggregation table holds as many slots as fit
// kRecAggLds; an aggregation partition is sized for half of them (fanout > 0
// sets their count, clamped to [1, kMaxRecParts]). The fused pass and the
// scatter split each into partitions of their own up to kMinRecParts.
RecLayout rec_plan(const rel_pipeline_desc* d, const PipeLayout& L, int chunk_tiles) {
  RecLayout R;
  const rel_tuning* t = d->tuning;
  const int fan = t ? t->fanout : 0;
  if (fan < 0 || d->n_keys == 0 || d->max_groups < 1) return R;
  const bool spills = 2 * static_cast<uint64_t>(d->max_groups) > static_cast<uint64_t>(L.lds_slots);
  const bool one_per_cu = static_cast<uint64_t>(L.lds_slots) * L.gp.words * 8 > kRecTableBytes;
  if (!spills && !one_per_cu) return R;
  const uint64_t n = static_cast<uint64_t>(d->fact[0].len);
  if (n == 0 || n > (1ull << 31)) return R;
  int cols[2] = {-1, -1}, ncols = 0;
  for (int a = 0; a < L.gp.ap.nacc; ++a) {
    const int c = L.gp.ap.col[a];
    if (c == cols[0] || c == cols[1]) continue;
    if (ncols == 2) return R;
    cols[ncols++] = c;
  }
  uint32_t slots = 1;
  while (static_cast<uint64_t>(slots) * 2 * L.gp.words * 8 <= kRecAggLds) slots *= 2;
  uint64_t parts;
  if (fan > 0) {
    parts = static_cast<uint64_t>(fan) > kMaxRecParts ? kMaxRecParts : static_cast<uint64_t>(fan);
  } else {
    parts = next_pow2(ceil_div(2 * static_cast<uint64_t>(d->max_groups), slots));
    if (parts > kMaxRecParts) return R;
  }
  R.agg_parts = static_cast<uint32_t>(parts < 1 ? 1 : parts);
  R.parts = R.agg_parts < kMinRecParts ? kMinRecParts : R.agg_parts;
  R.words = 1 + ncols;
  // 12-byte records when the packed key fits 32 bits and one value column
  // is carried (see RecDesc)
  const GroupKeyPack& kp = L.gp.kp;
  auto bits = [](int32_t t) { return t == REL_I8 ? 8 : (t == REL_I32 ? 32 : 64); };
  if (R.words == 2) {
    if (kp.nkeys == 1 && bits(kp.type[0]) <= 32) R.narrow = 1;
    else if (kp.nkeys == 2 && bits(kp.type[0]) + bits(kp.type[1]) <= 32) R.narrow = 2;
  }
  R.nitems = static_cast<uint32_t>(ceil_div(ceil_div(n, kPipeTile), chunk_tiles));
  R.agg_slots = slots;
  return R;
}

// The description a plan with records is laid out with: unless its tuning
// sets one, no LDS group table in the fused pass (its groups are well
// beyond the table, so most rows would walk a full probe window and spill
// anyway, and the table costs resident workgroups: on the 256-instance
// batch's plans above 2048 groups, fused pass 27.0 -> 5.6 ms for 4.7 ->
// 11.9 ms of record passes), and one global table whatever the tuning
// (only the aggregation pass's merges reach it, once per key and piece, so
// copies would only add fill and merge work).
struct RecPlanDesc {
  rel_pipeline_desc d;
  rel_tuning t;
  explicit RecPlanDesc(const rel_pipeline_desc& src) : d(src) {
    std::memset(&t, 0, sizeof t);
    if (src.tuning) t = *src.tuning;
    if (t.lds_slots == 0) t.lds_slots = -1;
    t.replicas = 1;
    d.tuning = &t;
  }
};

// Record bytes of R over n fact rows: the fused pass's runs, the
// partitioned copy (each as 64-bit words, or for narrow records value words
// and 32-bit keys), the counts, the item sizes and the partition offsets.
uint64_t rec_bytes(const RecLayout& R, uint64_t n, int chunk_tiles) {
  const uint64_t item_rows = static_cast<uint64_t>(chunk_tiles) * kPipeTile;
  const uint64_t run = R.nitems * item_rows;
  const uint64_t words = R.narrow ? 1 : R.words;
  uint64_t b = align_up(run * words * 8) + align_up(n * words * 8);
  if (R.narrow) b += align_up(run * 4) + align_up(n * 4);
  return b + align_up(static_cast<uint64_t>(R.parts) * R.nitems * 4) + align_up(R.nitems * 4ull) +
         align_up((R.parts + 1) * 4ull) + align_up(R.parts * 4ull);
}

// Instances of one batch must share the kernel variant: the same number of
// dims, and per dim the same key type and payload presence.
rel_status check_batch(const rel_pipeline_desc* d, int n) {
  if (n < 1 || n > kMaxBatch) return fail(REL_EINVAL, "batch: 1..%d plans required", kMaxBatch);
  if (!d) return fail(REL_EINVAL, "batch: NULL descriptions");
  for (int i = 0; i < n; ++i) {
    rel_status st = check_pipeline(&d[i]);
    if (st) return fail(st, "batch plan %d: %s", i, g_error.c_str());
    if (d[i].n_dims != d[0].n_dims)
      return fail(REL_EINVAL, "batch plan %d joins %d dims, plan 0 joins %d", i, d[i].n_dims,
                  d[0].n_dims);
    for (int k = 0; k < d[0].n_dims; ++k) {
      if (d[i].dims[k].key.type != d[0].dims[k].key.type ||
          (d[i].dims[k].has_payload != 0) != (d[0].dims[k].has_payload != 0))
        return fail(REL_EINVAL, "batch plan %d: dim %d differs in key type or payload from plan 0",
                    i, k);
    }
  }
  return REL_OK;
}

rel_status batch_layout(const rel_pipeline_desc* d, int n, BatchLayout& B) {
  B.L.resize(n);
  B.base.resize(n);
  B.nfill = B.nbuild = B.ntile = B.nmerge = B.nfin = B.nslice = B.nwin = 0;
  B.win_n.assign(2 * static_cast<size_t>(n), 0);
  B.win_pairs.assign(2 * static_cast<size_t>(n), 0);
  B.win_cursor.assign(2 * static_cast<size_t>(n), 0);
  B.win_begin.assign(2 * static_cast<size_t>(n), 0);
  B.slice_bits = direct_slice_bits();
  uint64_t tiles = 0;
  for (int i = 0; i < n; ++i) tiles += ceil_div(static_cast<uint64_t>(d[i].fact[0].len), kPipeTile);
  const rel_tuning* t0 = d[0].tuning;
  if (t0 && t0->chunk_tiles > 0) {
    B.chunk_tiles = t0->chunk_tiles;
  } else {
    // about eight items per resident workgroup, at most kMaxChunkTiles tiles each
    const uint64_t want = static_cast<uint64_t>(device_info().cu_count) * 4 * 8;
    uint64_t c = tiles / (want ? want : 1);
    B.chunk_tiles = static_cast<int>(c < 1 ? 1 : (c > kMaxChunkTiles ? kMaxChunkTiles : c));
  }
  // instance tables after the uploaded block, whose size depends on the item
  // counts: lay the tables out from 0 first, count, then shift
  size_t off = 0;
  B.rec.assign(n, RecLayout());
  uint64_t rec_total = 0;
  for (int i = 0; i < n; ++i) {
    rel_status st = pipeline_layout(&d[i], B.L[i], true, off);
    if (st) return fail(st, "batch plan %d: %s", i, g_error.c_str());
    // records within kRecordBudget; such a plan is then laid out again
    // without the fused pass's LDS table and with one global table
    RecLayout R = rec_plan(&d[i], B.L[i], B.chunk_tiles);
    if (R.parts) {
      const uint64_t bytes = rec_bytes(R, static_cast<uint64_t>(d[i].fact[0].len), B.chunk_tiles);
      if (rec_total + bytes <= kRecordBudget) {
        rec_total += bytes;
        B.rec[i] = R;
        B.nfill += 1;  // the partition cursors
        RecPlanDesc rd(d[i]);
        st = pipeline_layout(&rd.d, B.L[i], true, off);
        if (st) return fail(st, "batch plan %d: %s", i, g_error.c_str());
      }
    }
    B.base[i] = off;
    off = B.L[i].end;
    for (int k = 0; k < d[i].n_dims; ++k) {
      B.nfill += ceil_div(map_words(B.L[i].dim[k], d[i].dims[k].key.type), kFillChunk) + 1;
      if (B.L[i].dim[k].direct_cap) {
        B.nfill += 1 + ceil_div(B.L[i].dim[k].direct_cap / 64, kFillChunk);
        // dims with payloads are built by windows when they have few enough
        const uint64_t wins = ceil_div(B.L[i].dim[k].direct_cap, kWinKeys);
        if (d[i].dims[k].has_payload && wins <= kMaxWins) {
          B.win_n[2 * i + k] = static_cast<uint32_t>(wins);
          B.nwin += wins;
          B.nfill += 1;  // the window cursors
        } else {
          B.nslice += ceil_div(B.L[i].dim[k].direct_cap, B.slice_bits) *
                      slice_parts(static_cast<uint64_t>(d[i].dims[k].key.len));
        }
      }
      B.nbuild += ceil_div(static_cast<uint64_t>(d[i].dims[k].key.len), kBuildChunk);
    }
    const GroupLayout& g = B.L[i].group;
    B.nfill += ceil_div(g.replicas * (g.cap + 1) * B.L[i].gp.words, kFillChunk) + 2;
    B.ntile += ceil_div(ceil_div(static_cast<uint64_t>(d[i].fact[0].len), kPipeTile),
                        B.chunk_tiles);
    if (g.replicas > 1) B.nmerge += ceil_div((g.replicas - 1) * (g.cap + 1), kSlotChunk);
    B.nfin += ceil_div(d[i].n_keys == 0 ? 1 : g.cap + 1, kSlotChunk);
  }
  // record regions after the tables
  B.rec_plans = 0;
  B.agg_lds_bytes = 0;
  B.piece_cap = 0;
  for (int i = 0; i < n; ++i) {
    RecLayout& R = B.rec[i];
    if (R.parts == 0) continue;
    const uint64_t rows = static_cast<uint64_t>(d[i].fact[0].len);
    off = align_up(off);
    const uint64_t item_rows = static_cast<uint64_t>(B.chunk_tiles) * kPipeTile;
    const uint64_t words = R.narrow ? 1 : R.words;
    R.recs = off;
    off += align_up(R.nitems * item_rows * words * 8);
    R.parted = off;
    off += align_up(rows * words * 8);
    if (R.narrow) {
      R.rkeys = off;
      off += align_up(R.nitems * item_rows * 4);
      R.pkeys = off;
      off += align_up(rows * 4);
    }
    R.counts = off;
    off += align_up(static_cast<uint64_t>(R.parts) * R.nitems * 4);
    R.item_n = off;
    off += align_up(R.nitems * 4ull);
    R.part_begin = off;
    off += align_up((R.parts + 1) * 4ull);
    R.cursor = off;
    off += align_up(R.parts * 4ull);
    ++B.rec_plans;
    const uint32_t agg = R.agg_slots * B.L[i].gp.words * 8;
    if (agg > B.agg_lds_bytes) B.agg_lds_bytes = agg;
    B.piece_cap += ceil_div(rows, kRecPiece) + R.agg_parts;
  }
  // window regions: the grouped pairs, the cursors, the offsets
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < d[i].n_dims; ++k) {
      const uint32_t wins = B.win_n[2 * i + k];
      if (wins == 0) continue;
      off = align_up(off);
      B.win_pairs[2 * i + k] = off;
      off += align_up(static_cast<uint64_t>(d[i].dims[k].key.len) * 8);
      B.win_cursor[2 * i + k] = off;
      off += align_up(wins * 4ull);
      B.win_begin[2 * i + k] = off;
      off += align_up((wins + 1) * 4ull);
    }
  }
  off = align_up(off);
  B.off_pieces = off;
  off += align_up(B.piece_cap * sizeof(RecPiece));
  if (B.piece_cap > 0xFFFFFFFFull) return fail(REL_EUNSUPPORTED, "batch: too many record pieces");
  const uint64_t most = 0xFFFFFFFFull;
  if (B.nfill > most || B.nbuild > most || B.ntile > most || B.nmerge > most || B.nfin > most ||
      B.nslice > most || B.nwin > most)
    return fail(REL_EUNSUPPORTED, "batch: more than 2^32 - 1 work items in a phase");
  size_t h = kAlign;  // the counter
  B.off_plans = h;
  h = align_up(h + n * sizeof(PipelineParams));
  B.off_builds = h;
  h = align_up(h + 2 * n * sizeof(MapBuildParams));
  B.off_fins = h;
  h = align_up(h + n * sizeof(FinalizeParams));
  B.off_fill = h;
  h = align_up(h + B.nfill * sizeof(FillItem));
  B.off_build_items = h;
  h = align_up(h + B.nbuild * sizeof(BatchItem));
  B.off_tile_items = h;
  h = align_up(h + B.ntile * sizeof(BatchItem));
  B.off_merge_items = h;
  h = align_up(h + B.nmerge * sizeof(BatchItem));
  B.off_fin_items = h;
  h = align_up(h + B.nfin * sizeof(BatchItem));
  B.off_slice_items = h;
  h = align_up(h + B.nslice * sizeof(BatchItem));
  B.off_win_items = h;
  h = align_up(h + B.nwin * sizeof(BatchItem));
  B.blob = h;
  for (int i = 0; i < n; ++i) {
    RecPlanDesc rd(d[i]);
    rel_status st = pipeline_layout(B.rec[i].parts ? &rd.d : &d[i], B.L[i], true, B.blob + B.base[i]);
    if (st) return st;
    B.base[i] += B.blob;
  }
  B.end = B.blob + off;
  return REL_OK;
}

// True when every plan scans the same fact columns.
bool shared_scan(const rel_pipeline_desc* d, int n) {
  for (int i = 1; i < n; ++i) {
    if (d[i].n_fact != d[0].n_fact) return false;
    for (int c = 0; c < d[0].n_fact; ++c)
      if (d[i].fact[c].data != d[0].fact[c].data || d[i].fact[c].len != d[0].fact[c].len)
        return false;
  }
  return n > 1;
}

void push_fill(std::vector<FillItem>& v, uint64_t* p, uint64_t words, int32_t kind,
               uint64_t pattern, uint32_t inst) {
  for (uint64_t b = 0; b < words; b += kFillChunk) {
    FillItem f;
    f.p = p;
    f.begin = b;
    f.end = b + kFillChunk < words ? b + kFillChunk : words;
    f.pattern = pattern;
    f.kind = kind;
    f.inst = inst;
    v.push_back(f);
  }
}

void push_items(std::vector<BatchItem>& v, uint32_t inst, uint32_t aux, uint64_t units,
                uint64_t chunk) {
  for (uint64_t b = 0; b < units; b += chunk) {
    BatchItem it;
    it.inst = inst;
    it.aux = aux;
    it.begin = b;
    it.end = b + chunk < units ? b + chunk : units;
    v.push_back(it);
  }
}

// Writes the uploaded block of batch B over workspace w into `host` (B.blob
// bytes), returns instance 0's plan in `shape` and the kernel arguments.
// The fused pass runs one persistent launch per class of LDS group-table
// size (up to 16, 32, 64 and 128 KB), so that instances with small tables
// keep the occupancy their LDS allows instead of the largest table's.
constexpr int kLdsClasses = 4;
constexpr uint32_t kClassGroupLds[kLdsClasses] = {16384, 32768, 65536, 1u << 30};

int lds_class(uint32_t group_lds) {
  int c = 0;
  while (group_lds > kClassGroupLds[c]) ++c;
  return c;
}

// Fills the uploaded block at `host`. `bp` covers every instance and the
// fused pass of class 0; fused[c] the fused pass of class c (fused[c].ntile
// = 0 when the class is empty; fused[0] = bp).
void batch_blob(const rel_pipeline_desc* d, int n, const rel_outputs* o, const BatchLayout& B,
                unsigned char* w, unsigned char* host, PipelineParams& shape, BatchParams& bp,
                BatchParams fused[kLdsClasses]) {
  std::memset(host, 0, B.blob);
  PipelineParams* plans = reinterpret_cast<PipelineParams*>(host + B.off_plans);
  MapBuildParams* builds = reinterpret_cast<MapBuildParams*>(host + B.off_builds);
  FinalizeParams* fins = reinterpret_cast<FinalizeParams*>(host + B.off_fins);
  std::vector<FillItem> fill;
  std::vector<BatchItem> build_items, tile_items, merge_items, fin_items, slice_items, win_items;
  fill.reserve(B.nfill);
  build_items.reserve(B.nbuild);
  tile_items.reserve(B.ntile);
  merge_items.reserve(B.nmerge);
  fin_items.reserve(B.nfin);
  slice_items.reserve(B.nslice);
  win_items.reserve(B.nwin);
  uint32_t group_lds[kLdsClasses] = {};
  std::vector<int> cls(n);
  for (int i = 0; i < n; ++i) {
    const PipeLayout& L = B.L[i];
    PipelineParams& p = plans[i];
    plan_params(&d[i], L, w, o[i].d_groups, true, p, &builds[2 * i]);
    const uint32_t gl = static_cast<uint32_t>((static_cast<size_t>(p.lds_slots) * L.gp.words * 8 + 15) / 16 * 16);
    cls[i] = lds_class(gl);
    if (gl > group_lds[cls[i]]) group_lds[cls[i]] = gl;
    fins[i] = finalize_params(p.g, L.gp, d[i].aggs, d[i].n_aggs, o[i].keys, L.key_types, o[i].aggs,
                              o[i].cap);
    for (int k = 0; k < d[i].n_dims; ++k) {
      const MapDesc& m = p.dim[k].map;
      const uint64_t words = map_words(L.dim[k], d[i].dims[k].key.type);
      if (d[i].dims[k].key.type == REL_I64)
        push_fill(fill, static_cast<uint64_t*>(m.slots), words, kFillPairs, 0, i);
      else if (m.key_only)
        push_fill(fill, static_cast<uint64_t*>(m.slots), words, kFillConst, 0x8000000080000000ULL, i);
      else
        push_fill(fill, static_cast<uint64_t*>(m.slots), words, kFillConst, kEmptySlot32, i);
      // the out-of-band count and the duplicate flag
      push_fill(fill, reinterpret_cast<uint64_t*>(m.oob_count), 2, kFillConst, 0, i);
      if (m.direct_cap) {
        push_fill(fill, reinterpret_cast<uint64_t*>(m.dstate), 2, kFillConst, kDirectStateInit, i);
        push_fill(fill, reinterpret_cast<uint64_t*>(m.dbits), m.direct_cap / 64, kFillConst, 0, i);
      }
      const uint32_t wins = B.win_n[2 * i + k];
      MapBuildParams& bw = builds[2 * i + k];
      bw.nwin = wins;
      if (wins) {
        unsigned char* tables = w + B.blob;
        bw.wpairs = reinterpret_cast<uint64_t*>(tables + B.win_pairs[2 * i + k]);
        bw.wcursor = reinterpret_cast<uint32_t*>(tables + B.win_cursor[2 * i + k]);
        bw.wbegin = reinterpret_cast<uint32_t*>(tables + B.win_begin[2 * i + k]);
        push_fill(fill, reinterpret_cast<uint64_t*>(bw.wcursor), (wins + 1) / 2, kFillConst, 0, i);
        for (uint32_t wi = 0; wi < wins; ++wi) {
          BatchItem it;
          it.inst = i;
          it.aux = k;
          it.begin = wi;
          it.end = wi + 1;
          win_items.push_back(it);
        }
      }
      if (m.direct_cap && !wins) {
        const uint64_t parts = slice_parts(static_cast<uint64_t>(d[i].dims[k].key.len));
        for (uint64_t lo = 0; lo < m.direct_cap; lo += B.slice_bits)
          for (uint64_t part = 0; part < parts; ++part) {
            BatchItem it;
            it.inst = i;
            it.aux = k;
            it.begin = lo;
            it.end = part << 32 | parts;  // part `part` of `parts` of the build rows
            slice_items.push_back(it);
          }
      }
      push_items(build_items, i, k, static_cast<uint64_t>(d[i].dims[k].key.len), kBuildChunk);
    }
    const GroupDesc& g = p.g;
    push_fill(fill, g.slots, g.replicas * (g.cap + 1) * g.words, kFillGroup, 0, i);
    push_fill(fill, reinterpret_cast<uint64_t*>(g.overflow), 1, kFillConst, 0, i);
    push_fill(fill, reinterpret_cast<uint64_t*>(g.d_groups), 1, kFillConst, 0, i);
    if (B.rec[i].parts)
      push_fill(fill, reinterpret_cast<uint64_t*>(w + B.blob + B.rec[i].cursor),
                (B.rec[i].parts + 1) / 2, kFillConst, 0, i);
    if (g.replicas > 1) push_items(merge_items, i, 0, (g.replicas - 1) * (g.cap + 1), kSlotChunk);
    push_items(fin_items, i, 0, d[i].n_keys == 0 ? 1 : g.cap + 1, kSlotChunk);
  }
  // the fused-pass items class by class
  size_t class_end[kLdsClasses] = {};
  for (int c = 0; c < kLdsClasses; ++c) {
    if (shared_scan(d, n)) {
      // plans over one fact table: tile range j of every plan, then range
      // j + 1, so that the plans' passes over a range run together and share
      // its columns through the caches
      const uint64_t ntiles = static_cast<uint64_t>(plans[0].ntiles);
      for (uint64_t b = 0; b < ntiles; b += B.chunk_tiles)
        for (int i = 0; i < n; ++i) {
          if (cls[i] != c) continue;
          BatchItem it;
          it.inst = i;
          it.aux = 0;
          it.begin = b;
          it.end = b + B.chunk_tiles < ntiles ? b + B.chunk_tiles : ntiles;
          tile_items.push_back(it);
        }
    } else {
      for (int i = 0; i < n; ++i)
        if (cls[i] == c)
          push_items(tile_items, i, 0, static_cast<uint64_t>(plans[i].ntiles), B.chunk_tiles);
    }
    class_end[c] = tile_items.size();
  }
  // one LDS layout per class: its largest group table, then the queues, then
  // (plans with records) the partition histogram
  uint32_t lds_bytes[kLdsClasses] = {};
  unsigned char* tables = w + B.blob;
  for (int i = 0; i < n; ++i) {
    plans[i].lds_group_offset = 0;
    plans[i].queue_offset = group_lds[cls[i]];
    plans[i].lds_bytes = group_lds[cls[i]] + (kPipeThreads / kWave) * plans[i].queue_stride;
    const RecLayout& R = B.rec[i];
    RecDesc& rd = plans[i].rec;
    std::memset(&rd, 0, sizeof rd);
    if (R.parts) {
      rd.recs = reinterpret_cast<uint64_t*>(tables + R.recs);
      rd.parted = reinterpret_cast<uint64_t*>(tables + R.parted);
      if (R.narrow) {
        rd.rkeys = reinterpret_cast<uint32_t*>(tables + R.rkeys);
        rd.pkeys = reinterpret_cast<uint32_t*>(tables + R.pkeys);
        rd.narrow = R.narrow;
      }
      rd.counts = reinterpret_cast<uint32_t*>(tables + R.counts);
      rd.item_n = reinterpret_cast<uint32_t*>(tables + R.item_n);
      rd.part_begin = reinterpret_cast<uint32_t*>(tables + R.part_begin);
      rd.cursor = reinterpret_cast<uint32_t*>(tables + R.cursor);
      rd.parts = R.parts;
      rd.agg_parts = R.agg_parts;
      rd.words = R.words;
      rd.nitems = R.nitems;
      rd.item_tiles = static_cast<uint32_t>(B.chunk_tiles);
      rd.agg_slots = R.agg_slots;
      rd.lds_offset = (plans[i].lds_bytes + 15) / 16 * 16;
      plans[i].lds_bytes = rd.lds_offset + (R.parts + 1) * 4;
    }
    if (plans[i].lds_bytes > lds_bytes[cls[i]]) lds_bytes[cls[i]] = plans[i].lds_bytes;
  }
  std::memcpy(host + B.off_fill, fill.data(), fill.size() * sizeof(FillItem));
  std::memcpy(host + B.off_build_items, build_items.data(), build_items.size() * sizeof(BatchItem));
  std::memcpy(host + B.off_tile_items, tile_items.data(), tile_items.size() * sizeof(BatchItem));
  std::memcpy(host + B.off_merge_items, merge_items.data(), merge_items.size() * sizeof(BatchItem));
  std::memcpy(host + B.off_fin_items, fin_items.data(), fin_items.size() * sizeof(BatchItem));
  std::memcpy(host + B.off_slice_items, slice_items.data(), slice_items.size() * sizeof(BatchItem));
  std::memcpy(host + B.off_win_items, win_items.data(), win_items.size() * sizeof(BatchItem));
  shape = plans[0];
  std::memset(&bp, 0, sizeof bp);
  bp.plans = reinterpret_cast<const PipelineParams*>(w + B.off_plans);
  bp.builds = reinterpret_cast<const MapBuildParams*>(w + B.off_builds);
  bp.fins = reinterpret_cast<const FinalizeParams*>(w + B.off_fins);
  bp.fill = reinterpret_cast<const FillItem*>(w + B.off_fill);
  bp.build_items = reinterpret_cast<const BatchItem*>(w + B.off_build_items);
  bp.tile_items = reinterpret_cast<const BatchItem*>(w + B.off_tile_items);
  bp.merge_items = reinterpret_cast<const BatchItem*>(w + B.off_merge_items);
  bp.fin_items = reinterpret_cast<const BatchItem*>(w + B.off_fin_items);
  bp.slice_items = reinterpret_cast<const BatchItem*>(w + B.off_slice_items);
  bp.win_items = reinterpret_cast<const BatchItem*>(w + B.off_win_items);
  bp.nfill = static_cast<uint32_t>(fill.size());
  bp.nbuild = static_cast<uint32_t>(build_items.size());
  bp.ntile = static_cast<uint32_t>(class_end[0]);
  bp.nmerge = static_cast<uint32_t>(merge_items.size());
  bp.nfin = static_cast<uint32_t>(fin_items.size());
  bp.nslice = static_cast<uint32_t>(slice_items.size());
  bp.nwin = static_cast<uint32_t>(win_items.size());
  bp.slice_bits = B.slice_bits;
  bp.lds_bytes = lds_bytes[0];
  bp.group_lds_bytes = group_lds[0];
  bp.counter = reinterpret_cast<unsigned long long*>(w);
  bp.nplans = static_cast<uint32_t>(n);
  bp.ntile_all = static_cast<uint32_t>(tile_items.size());
  bp.rec_plans = B.rec_plans;
  bp.agg_lds_bytes = B.agg_lds_bytes;
  bp.piece_cap = static_cast<uint32_t>(B.piece_cap);
  bp.pieces = reinterpret_cast<RecPiece*>(tables + B.off_pieces);
  // counters after the four fused-pass classes' in the zeroed first block
  bp.npieces = reinterpret_cast<unsigned long long*>(w) + kLdsClasses;
  bp.agg_counter = reinterpret_cast<unsigned long long*>(w) + kLdsClasses + 1;
  for (int c = 0; c < kLdsClasses; ++c) {
    const size_t begin = c == 0 ? 0 : class_end[c - 1];
    fused[c] = bp;
    fused[c].tile_items = bp.tile_items + begin;
    fused[c].ntile = static_cast<uint32_t>(class_end[c] - begin);
    fused[c].lds_bytes = lds_bytes[c];
    fused[c].group_lds_bytes = group_lds[c];
    // one counter per class, in the uploaded (zeroed) first block
    fused[c].counter = reinterpret_cast<unsigned long long*>(w) + c;
  }
}

// Enqueues the upload of the block at `host` and the six batch launches.
rel_status batch_enqueue(const BatchLayout& B, const BatchParams& bp,
                         const BatchParams fused[kLdsClasses], const PipelineParams& shape,
                         unsigned char* w, const void* host, int grid, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(w, host, B.blob, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(REL_EDEVICE, "batch: descriptor upload: %s", hipGetErrorString(e));
  launch_batch_fill(bp, s);
  launch_batch_build(bp, s);
  for (int c = 0; c < kLdsClasses; ++c) {
    if (fused[c].ntile == 0) continue;
    e = launch_batch_pipeline(fused[c], shape, grid, s);
    if (e != hipSuccess)
      return fail(REL_EDEVICE, "batch: fused kernel launch (%u bytes of LDS): %s",
                  fused[c].lds_bytes, hipGetErrorString(e));
  }
  launch_batch_records(bp, s);
  launch_batch_merge(bp, s);
  launch_batch_finalize(bp, s);
  return after_launch(s, "batch");
}

// Pinned host staging for the batch uploads: a small ring per thread; a
// slot is written again only once the copy that read it has completed. The
// buffers live until the process ends.
struct StagingSlot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
constexpr int kStagingSlots = 4;
thread_local StagingSlot g_staging[kStagingSlots];
thread_local int g_staging_next = 0;

rel_status staging_take(size_t bytes, StagingSlot*& out) {
  StagingSlot& sl = g_staging[g_staging_next];
  g_staging_next = (g_staging_next + 1) % kStagingSlots;
  if (sl.pending) {
    const hipError_t e = hipEventSynchronize(sl.done);
    if (e != hipSuccess) return fail(REL_EDEVICE, "batch: staging wait: %s", hipGetErrorString(e));
    sl.pending = false;
  }
  if (!sl.done) {
    const hipError_t e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      sl.done = nullptr;
      return fail(REL_EDEVICE, "batch: staging event: %s", hipGetErrorString(e));
    }
  }
  if (sl.cap < bytes) {
    if (sl.host) (void)hipHostFree(sl.host);
    sl.host = nullptr;
    sl.cap = 0;
    const size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    const hipError_t e = hipHostMalloc(&sl.host, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      sl.host = nullptr;
      return fail(REL_EDEVICE, "batch: %zu bytes of pinned staging: %s", want, hipGetErrorString(e));
    }
    sl.cap = want;
  }
  out = &sl;
  return REL_OK;
}

}  // namespace

const DeviceInfo& device_info() {
  static DeviceInfo info[64];
  static bool have[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (!have[dev]) {
    int cus = 0, lds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        lds <= 0)
      lds = 65536;
    info[dev].cu_count = cus;
    info[dev].lds_per_block = lds;
    have[dev] = true;
  }
  return info[dev];
}

// Radix-partitioned aggregation (see partition.hip): used by default when
// the groups do not fit the single pass's LDS table and there are at least
// kPartMinRows rows: the single pass then updates the global table with a
// device-scope atomic per row and accumulator (65-82 ms for 400M rows at
// 10k-3M uniform groups, against 10-13 ms partitioned). The partitioned map
// build is used for slot arrays above kPartTableBytes.
constexpr uint64_t kPartTableBytes = 64ull << 20;
constexpr int64_t kPartMinRows = 1000000;
constexpr size_t kPartAggLds = 128 * 1024;  // LDS of the aggregation pass
constexpr uint32_t kPartPiece = 65536;       // records per aggregation work item
constexpr double kPartFill = 0.6;            // target keys per LDS slot of a partition

struct PartPlan {
  bool on = false;
  int b1 = 0, b2 = 0, pre_slots = 0, agg_slots = 0;
  int ncols = 0, rw = 1;
  int cols[kMaxAcc] = {};  // value column (of the call) of each record column
  int src[kMaxAcc] = {};   // record column of each accumulator
  size_t ctl_off = 0, a_off = 0, b_off = 0;
};

int log2_ceil(uint64_t v) {
  int b = 0;
  while ((1ull << b) < v) ++b;
  return b;
}

// Layout of rel_groupby_agg over n rows: the group table, and with
// partitioning its control words and two record buffers of n records.
GroupLayout groupby_layout(const GroupPlan& gp, int64_t n, int64_t max_groups,
                           const rel_tuning* t, PartPlan& pp) {
  pp = PartPlan();
  const int fan = t ? t->fanout : 0;
  const float lf = load_factor(t);
  GroupLayout one = group_layout(gp, max_groups, lf, 0, 1);
  const int single_lds = default_lds_slots(t, max_groups, gp.words, 32768);
  const bool fits_lds = single_lds > 0 && 2 * max_groups <= single_lds;
  if (fan < 0 || gp.kp.nkeys == 0 || n <= 0 || (fan == 0 && (fits_lds || n < kPartMinRows)))
    return group_layout(gp, max_groups, lf, 0, groupby_replicas(t, max_groups, gp));
  pp.on = true;
  pp.agg_slots = static_cast<int>(next_pow2(kPartAggLds / (static_cast<size_t>(gp.words) * 8) + 1) / 2);
  int pb;
  if (fan > 0) {
    pb = log2_ceil(static_cast<uint64_t>(fan));
  } else {
    const double per = kPartFill * pp.agg_slots;
    pb = log2_ceil(static_cast<uint64_t>(std::ceil(static_cast<double>(max_groups) / per)));
  }
  if (pb < 2) pb = 2;
  if (pb > kPartMaxBits) pb = kPartMaxBits;
  pp.b1 = (pb + 1) / 2;
  pp.b2 = pb - pp.b1;
  pp.pre_slots = default_lds_slots(t, max_groups, gp.words, 32768);
  for (int a = 0; a < gp.ap.nacc; ++a) {
    int c = 0;
    while (c < pp.ncols && pp.cols[c] != gp.ap.col[a]) ++c;
    if (c == pp.ncols) pp.cols[pp.ncols++] = gp.ap.col[a];
    pp.src[a] = c;
  }
  pp.rw = 1 + pp.ncols;
  pp.ctl_off = one.end;
  pp.a_off = align_up(pp.ctl_off + kCtlWords * 8);
  pp.b_off = align_up(pp.a_off + static_cast<size_t>(n) * pp.rw * 8);
  one.end = align_up(pp.b_off + static_cast<size_t>(n) * pp.rw * 8);
  return one;
}

// Partitioned map build for rel_hash_join (see partition.hip): used by
// default when the slot array exceeds kPartTableBytes, where inserts would
// otherwise be random device-scope CAS into HBM. Ranges of kMapSpanBytes of
// slots are built in LDS; the slot array needs at least 4 of them.
constexpr size_t kMapSpanBytes = 128 * 1024;

struct JoinPart {
  bool on = false;
  int span_log2 = 0, sub = 1, b1 = 0, b2 = 0;
  size_t ctl_off = 0, a_off = 0, b_off = 0, end = 0;
};

JoinPart join_part(const MapLayout& L, int64_t n, const rel_tuning* t) {
  JoinPart jp;
  jp.end = L.end;
  const int fan = t ? t->fanout : 0;
  const uint64_t bytes = L.cap * L.slot_bytes;
  int span_log2 = 0;
  while ((static_cast<size_t>(1) << (span_log2 + 1)) * L.slot_bytes <= kMapSpanBytes) ++span_log2;
  if (L.compact || n <= 0 || fan < 0 || (fan == 0 && bytes < kPartTableBytes) ||
      L.cap < (4ULL << span_log2))
    return jp;
  int cap_log2 = 0;
  while ((1ULL << cap_log2) < L.cap) ++cap_log2;
  int pb = cap_log2 - span_log2;  // one partition per range
  if (fan > 0) {
    const int want = log2_ceil(static_cast<uint64_t>(fan));
    if (want < pb) pb = want;
  }
  if (pb > kPartMaxBits) pb = kPartMaxBits;
  jp.on = true;
  jp.span_log2 = span_log2;
  jp.sub = 1 << (cap_log2 - span_log2 - pb);
  jp.b1 = (pb + 1) / 2;
  jp.b2 = pb - jp.b1;
  jp.ctl_off = align_up(L.end);
  jp.a_off = align_up(jp.ctl_off + kCtlAll * 8);
  jp.b_off = align_up(jp.a_off + static_cast<size_t>(n) * 16);
  jp.end = align_up(jp.b_off + static_cast<size_t>(n) * 16);
  return jp;
}

}  // namespace rel

using namespace rel;

extern "C" {

const char* rel_status_str(rel_status s) {
  switch (s) {
    case REL_OK: return "ok";
    case REL_EINVAL: return "invalid argument";
    case REL_ENOMEM: return "workspace too small";
    case REL_ECAPACITY: return "capacity exceeded";
    case REL_EDEVICE: return "device error";
    case REL_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* rel_last_error(void) { return g_error.c_str(); }

int rel_version(void) { return REL_VERSION; }

// ----------------------------------------------------------- stream read

rel_status rel_stream_read(const void* data, int64_t bytes, uint64_t* d_xor, void* stream) {
  g_error.clear();
  if (bytes < 0) return fail(REL_EINVAL, "stream_read: negative size");
  if (bytes > 0 && !data) return fail(REL_EINVAL, "stream_read: NULL data");
  if (reinterpret_cast<uintptr_t>(data) % 16 != 0)
    return fail(REL_EINVAL, "stream_read: data must be 16-byte aligned");
  if (!d_xor || reinterpret_cast<uintptr_t>(d_xor) % 8 != 0)
    return fail(REL_EINVAL, "stream_read: NULL or misaligned result word");
  hipError_t e = launch_stream_read(data, static_cast<uint64_t>(bytes),
                                    reinterpret_cast<unsigned long long*>(d_xor),
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(REL_EDEVICE, "stream_read: %s", hipGetErrorString(e));
  return REL_OK;
}

// ------------------------------------------------------------------ filter

size_t rel_filter_ws(int64_t n) { return rel::filter_layout(n).end; }

}  // extern "C"

namespace rel {
namespace {

// Tile states of the single-pass (look-back) filter: the ticket's block and
// one word per tile (the allocation-free filter's static scratch).
size_t filter_state_bytes(int64_t n) {
  const int64_t tiles = n > 0 ? (n + kFilterTile - 1) / kFilterTile : 1;
  return align_up(kAlign + static_cast<size_t>(tiles) * 8);
}

// Points p at the bitmap path's workspace (filter_layout(p.n) bytes at w).
void filter_bind_marked(FilterParams& p, unsigned char* w) {
  const FilterLayout L = filter_layout(p.n);
  p.ntiles = L.tiles;
  p.bitmap = reinterpret_cast<uint32_t*>(w + L.bitmap_off);
  p.tile_count = reinterpret_cast<uint32_t*>(w + L.count_off);
  p.group_offset = reinterpret_cast<uint64_t*>(w + L.offset_off);
}

rel_status filter_check(const rel_column* cols, int ncols, const rel_pred* preds, int npreds,
                        rel_rowid* out, int64_t out_cap, int64_t* d_count) {
  if (!cols || ncols < 1 || ncols > REL_MAX_FACT_COLS)
    return fail(REL_EINVAL, "filter: 1..%d columns required", REL_MAX_FACT_COLS);
  for (int c = 0; c < ncols; ++c) {
    rel_status st = check_column(&cols[c], "filter column");
    if (st) return st;
    if (cols[c].len != cols[0].len) return fail(REL_EINVAL, "filter: columns differ in length");
    if (cols[c].idx != cols[0].idx) return fail(REL_EINVAL, "filter: columns must share one idx");
  }
  if (!preds || npreds < 1 || npreds > REL_MAX_TERMS)
    return fail(REL_EINVAL, "filter: 1..%d terms required", REL_MAX_TERMS);
  for (int t = 0; t < npreds; ++t) {
    if (preds[t].col < 0 || preds[t].col >= ncols)
      return fail(REL_EINVAL, "filter: term %d reads column %d of %d", t, preds[t].col, ncols);
    if (preds[t].op < REL_LT || preds[t].op > REL_RANGE)
      return fail(REL_EINVAL, "filter: term %d has invalid op %d", t, preds[t].op);
  }
  if (out_cap < 0 || (out_cap > 0 && !out)) return fail(REL_EINVAL, "filter: bad output");
  if (!d_count) return fail(REL_EINVAL, "filter: NULL count");
  return REL_OK;
}

// Enqueues the filter: with `marked`, the bitmap path over a workspace of
// rel_filter_ws(n) bytes at w; else the single pass with its tile states at
// w (filter_state_bytes(n) bytes).
rel_status filter_enqueue(const rel_column* cols, const rel_pred* preds, int npreds,
                          rel_rowid* out, int64_t out_cap, int64_t* d_count, unsigned char* w,
                          bool marked, hipStream_t s) {
  const int64_t n = cols[0].len;
  FilterParams p;
  std::memset(&p, 0, sizeof p);
  for (int t = 0; t < npreds; ++t) {
    const rel_column& c = cols[preds[t].col];
    p.term[t].data = c.data;
    p.term[t].type = c.type;
    p.term[t].op = preds[t].op;
    p.term[t].lo = preds[t].lo;
    p.term[t].hi = preds[t].hi;
    p.term[t].vec = (reinterpret_cast<uintptr_t>(c.data) % 16) == 0;
  }
  p.nterms = npreds;
  p.idx = cols[0].idx;
  p.n = n;
  p.out = out;
  p.cap = out_cap;
  p.d_count = reinterpret_cast<long long*>(d_count);
  if (marked) {
    filter_bind_marked(p, w);
    launch_filter_marked(p, s);
    return after_launch(s, "filter");
  }
  p.ticket = reinterpret_cast<uint32_t*>(w);
  p.tile_state = reinterpret_cast<uint64_t*>(w + kAlign);
  p.ntiles = n > 0 ? (n + kFilterTile - 1) / kFilterTile : 1;
  launch_fill64(reinterpret_cast<uint64_t*>(w), (kAlign + p.ntiles * 8) / 8, 0, s);
  launch_filter(p, s);
  return after_launch(s, "filter");
}

}  // namespace
}  // namespace rel

extern "C" {

rel_status rel_filter(const rel_column* cols, int ncols, const rel_pred* preds, int npreds,
                      rel_rowid* out, int64_t out_cap, int64_t* d_count, void* ws,
                      size_t ws_bytes, void* stream) {
  g_error.clear();
  rel_status st = filter_check(cols, ncols, preds, npreds, out, out_cap, d_count);
  if (st) return st;
  st = check_ws(ws, ws_bytes, rel_filter_ws(cols[0].len));
  if (st) return st;
  return filter_enqueue(cols, preds, npreds, out, out_cap, d_count,
                        static_cast<unsigned char*>(ws), true, static_cast<hipStream_t>(stream));
}

rel_status rel_filter_noalloc(const rel_column* cols, int ncols, const rel_pred* preds,
                              int npreds, rel_rowid* out, int64_t out_cap, int64_t* d_count,
                              void* stream) {
  g_error.clear();
  rel_status st = filter_check(cols, ncols, preds, npreds, out, out_cap, d_count);
  if (st) return st;
  const size_t need = filter_state_bytes(cols[0].len);
  if (need > kFilterScratchBytes)
    return fail(REL_ECAPACITY,
                "filter_noalloc: %lld rows need %zu bytes of tile state, the static scratch "
                "holds %zu (at most %lld rows)",
                static_cast<long long>(cols[0].len), need, kFilterScratchBytes,
                static_cast<long long>(kFilterNoallocMaxRows));
  void* scratch = nullptr;
  hipError_t e = filter_scratch(&scratch);
  if (e != hipSuccess) return fail(REL_EDEVICE, "filter_noalloc: %s", hipGetErrorString(e));
  return filter_enqueue(cols, preds, npreds, out, out_cap, d_count,
                        static_cast<unsigned char*>(scratch), false,
                        static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------- Bloom filters

size_t rel_bloom_bytes(int64_t n_keys, int32_t bits_per_key) {
  if (n_keys < 0 || n_keys > kMaxRows) return 0;
  if (bits_per_key == 0) bits_per_key = kBloomBitsPerKey;
  if (bits_per_key < 4 || bits_per_key > 64) return 0;
  return bloom_bytes(n_keys, bits_per_key);
}

}  // extern "C"

namespace rel {
namespace {

rel_status check_bloom(const void* filter, size_t filter_bytes, const char* what) {
  if (!filter) return fail(REL_EINVAL, "%s: NULL filter", what);
  if (reinterpret_cast<uintptr_t>(filter) % 32 != 0)
    return fail(REL_EINVAL, "%s: the filter must be 32-byte aligned", what);
  const size_t blocks = filter_bytes / 32;
  if (filter_bytes % 32 != 0 || blocks == 0 || (blocks & (blocks - 1)) != 0)
    return fail(REL_EINVAL, "%s: filter_bytes must be 32 times a power of two", what);
  return REL_OK;
}

}  // namespace
}  // namespace rel

extern "C" {

rel_status rel_bloom_build(const rel_column* keys, void* filter, size_t filter_bytes,
                           void* stream) {
  g_error.clear();
  rel_status st = check_column(keys, "bloom build keys");
  if (st) return st;
  st = check_bloom(filter, filter_bytes, "bloom build");
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  BloomBuildParams b;
  std::memset(&b, 0, sizeof b);
  b.words = static_cast<uint32_t*>(filter);
  b.bmask = filter_bytes / 32 - 1;
  b.keys = keys->data;
  b.idx = keys->idx;
  b.type = keys->type;
  b.n = keys->len;
  launch_bloom_build(b, s);
  return after_launch(s, "bloom build");
}

rel_status rel_bloom_filter(const rel_column* probe_keys, const void* filter, size_t filter_bytes,
                            rel_rowid* out, int64_t out_cap, int64_t* d_count, void* ws,
                            size_t ws_bytes, void* stream) {
  g_error.clear();
  rel_status st = check_column(probe_keys, "bloom filter keys");
  if (st) return st;
  st = check_bloom(filter, filter_bytes, "bloom filter");
  if (st) return st;
  if (out_cap < 0 || (out_cap > 0 && !out)) return fail(REL_EINVAL, "bloom filter: bad output");
  if (!d_count) return fail(REL_EINVAL, "bloom filter: NULL count");
  const int64_t n = probe_keys->len;
  st = check_ws(ws, ws_bytes, rel_filter_ws(n));
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  FilterParams p;
  std::memset(&p, 0, sizeof p);
  p.nterms = 0;
  p.idx = probe_keys->idx;
  p.n = n;
  p.out = out;
  p.cap = out_cap;
  p.d_count = reinterpret_cast<long long*>(d_count);
  p.bloom.words = static_cast<const uint32_t*>(filter);
  p.bloom.bmask = filter_bytes / 32 - 1;
  p.bloom_keys = probe_keys->data;
  p.bloom_type = probe_keys->type;
  p.bloom_vec = (reinterpret_cast<uintptr_t>(probe_keys->data) % 16) == 0;
  filter_bind_marked(p, w);
  launch_filter_marked(p, s);
  return after_launch(s, "bloom filter");
}

// ---------------------------------------------------- late materialisation

rel_status rel_gather(const rel_column* cols, int ncols, const rel_rowid* ids, int64_t n,
                      void* const* out, void* stream) {
  g_error.clear();
  if (!cols || ncols < 1 || ncols > 8) return fail(REL_EINVAL, "gather: 1..8 columns required");
  if (n < 0 || n > kMaxRows) return fail(REL_EINVAL, "gather: bad row count");
  if (n > 0 && (!ids || !out)) return fail(REL_EINVAL, "gather: NULL ids or outputs");
  GatherParams p;
  std::memset(&p, 0, sizeof p);
  for (int c = 0; c < ncols; ++c) {
    rel_status st = check_column(&cols[c], "gather column");
    if (st) return st;
    if (cols[c].idx) return fail(REL_EINVAL, "gather: columns take no idx (the ids select)");
    if (n > 0 && !out[c]) return fail(REL_EINVAL, "gather: NULL output %d", c);
    p.src[c] = cols[c].data;
    p.type[c] = cols[c].type;
    p.dst[c] = n > 0 ? out[c] : nullptr;
  }
  p.ncols = ncols;
  p.ids = ids;
  p.ids_vec = (reinterpret_cast<uintptr_t>(ids) % 16) == 0;
  p.n = n;
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_gather(p, s);
  return after_launch(s, "gather");
}

}  // extern "C"

namespace rel {
namespace {

struct TopLayout {
  int pow2 = 1, lists = 0;
  int64_t span = 0;
  size_t list_bytes = 0, end = 0;
};

TopLayout top_layout(int64_t n, int64_t limit) {
  TopLayout L;
  while (L.pow2 < limit) L.pow2 <<= 1;
  if (n <= 0) return L;
  int64_t lists = static_cast<int64_t>(device_info().cu_count) * 2;
  const int64_t chunks = (n + L.pow2 - 1) / L.pow2;
  if (lists > chunks) lists = chunks;
  int64_t per = (n + lists - 1) / lists;
  L.span = (per + L.pow2 - 1) / L.pow2 * L.pow2;
  L.lists = static_cast<int>((n + L.span - 1) / L.span);
  L.list_bytes = static_cast<size_t>(L.lists) * L.pow2;  // entries per buffer
  L.end = 2 * align_up(L.list_bytes * 8) * 3 + 2 * align_up(L.list_bytes * 4);
  return L;
}

}  // namespace
}  // namespace rel

extern "C" {

size_t rel_topn_ws(int64_t n, int64_t limit) {
  if (n < 0 || n > kMaxRows || limit < 0 || limit > kTopMax) return 0;
  return align_up(top_layout(n, limit).end + kAlign);
}

rel_status rel_topn(const void* order, int32_t order_type, int32_t desc, const rel_column* keys,
                    int nkeys, int64_t n, int64_t limit, rel_rowid* out, int64_t* d_count,
                    void* ws, size_t ws_bytes, void* stream) {
  g_error.clear();
  if (n < 0 || n > kMaxRows) return fail(REL_EINVAL, "top-N: bad row count");
  if (limit < 0 || limit > kTopMax) return fail(REL_EINVAL, "top-N: limit must be in [0, %d]", kTopMax);
  if (order_type != REL_I64 && order_type != REL_F64)
    return fail(REL_EINVAL, "top-N: the order column is int64 or binary64");
  if (n > 0 && !order) return fail(REL_EINVAL, "top-N: NULL order column");
  if (reinterpret_cast<uintptr_t>(order) % 8 != 0) return fail(REL_EINVAL, "top-N: misaligned order column");
  if (nkeys < 0 || nkeys > 2 || (nkeys > 0 && !keys)) return fail(REL_EINVAL, "top-N: 0..2 keys");
  for (int k = 0; k < nkeys; ++k) {
    rel_status st = check_column(&keys[k], "top-N key");
    if (st) return st;
    if (keys[k].idx || keys[k].len < n) return fail(REL_EINVAL, "top-N: key %d must cover the rows", k);
  }
  if (!d_count || (limit > 0 && n > 0 && !out)) return fail(REL_EINVAL, "top-N: NULL outputs");
  rel_status st = check_ws(ws, ws_bytes, rel_topn_ws(n, limit));
  if (st) return st;
  const TopLayout L = top_layout(n, limit);
  TopNParams p;
  std::memset(&p, 0, sizeof p);
  p.order = order;
  p.order_is_double = order_type == REL_F64;
  p.desc = desc != 0;
  for (int k = 0; k < nkeys; ++k) {
    p.keys[k] = keys[k].data;
    p.key_type[k] = keys[k].type;
  }
  p.nkeys = nkeys;
  p.pow2 = L.pow2;
  p.n = n;
  p.limit = limit;
  p.span = L.span;
  p.nlists = L.lists;
  unsigned char* w = static_cast<unsigned char*>(ws);
  size_t off = 0;
  for (int b = 0; b < 2; ++b) {
    p.buf[b].a = reinterpret_cast<uint64_t*>(w + off);
    off += align_up(L.list_bytes * 8);
    p.buf[b].b = reinterpret_cast<uint64_t*>(w + off);
    off += align_up(L.list_bytes * 8);
    p.buf[b].c = reinterpret_cast<uint64_t*>(w + off);
    off += align_up(L.list_bytes * 8);
    p.buf[b].row = reinterpret_cast<uint32_t*>(w + off);
    off += align_up(L.list_bytes * 4);
  }
  p.out = out;
  p.d_count = reinterpret_cast<long long*>(d_count);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const hipError_t e = launch_topn(p, s);
  if (e != hipSuccess) return fail(REL_EDEVICE, "top-N: %s", hipGetErrorString(e));
  return after_launch(s, "top-N");
}

// ------------------------------------------------------ string group-by

}  // extern "C"

namespace rel {
namespace {

struct StrLayout {
  uint64_t cap = 0, dict_cap = 0;
  int words = 0;
  size_t slots_off = 0, overflow_off = 0, dict_off = 0, canon_off = 0, slot_of_off = 0, end = 0;
};

// Group table of 2 x max_groups slots (at least 64); with a dictionary of
// n_dict entries, its string table (2 x n_dict claim words), the canonical
// id of every entry and the group slot of every entry.
StrLayout str_layout(int64_t max_groups, int64_t n_dict, int nacc) {
  StrLayout L;
  uint64_t want = static_cast<uint64_t>(max_groups > 0 ? max_groups : 1) * 2;
  L.cap = next_pow2(want < 64 ? 64 : want);
  L.words = 3 + nacc;
  L.slots_off = 0;
  L.overflow_off = align_up(L.cap * L.words * 8);
  L.dict_off = L.overflow_off + kAlign;
  L.end = L.dict_off;
  if (n_dict > 0) {
    const uint64_t dw = static_cast<uint64_t>(n_dict) * 2;
    L.dict_cap = next_pow2(dw < 64 ? 64 : dw);
    L.canon_off = align_up(L.dict_off + L.dict_cap * 8);
    L.slot_of_off = align_up(L.canon_off + static_cast<size_t>(n_dict) * 4);
    L.end = L.slot_of_off + static_cast<size_t>(n_dict) * 4;
  }
  return L;
}

// LDS pre-aggregation entries per workgroup: a power of two within a 32 KB
// table (16 + 8 x nacc bytes an entry), no more than the group table has
// slots, none when slot indices would not fit the table's 32-bit keys.
int32_t str_lds_slots(uint64_t cap, int nacc) {
  if (cap > (1ULL << 31)) return 0;
  uint64_t k = 2048;
  while (k > 256 && k * (16 + 8 * static_cast<uint64_t>(nacc)) > 32768) k >>= 1;
  if (k > cap) k = cap;
  return static_cast<int32_t>(k);
}

}  // namespace
}  // namespace rel

extern "C" {

size_t rel_groupby_str_ws(int64_t max_groups, int64_t n_dict, int naggs, const rel_agg* aggs) {
  if (max_groups < 0 || max_groups > kMaxRows || n_dict < 0 || n_dict > kMaxRows || naggs < 1 ||
      naggs > REL_MAX_AGGS || !aggs)
    return 0;
  GroupPlan gp;
  if (group_plan(0, nullptr, naggs, aggs, gp) != REL_OK) return 0;
  return align_up(str_layout(max_groups, n_dict, gp.ap.nacc).end);
}

rel_status rel_groupby_str(const rel_strings* key, const rel_column* ikey, const rel_column* vals,
                           int nvals, const rel_agg* aggs, int naggs, rel_rowid* out_rows,
                           void* out_ikey, void* const* out_aggs, int64_t out_cap,
                           int64_t* d_groups, int64_t max_groups, void* ws, size_t ws_bytes,
                           void* stream) {
  g_error.clear();
  if (!key) return fail(REL_EINVAL, "string group-by: NULL key");
  const int64_t n = key->len;
  if (n < 0 || n > kMaxRows) return fail(REL_EINVAL, "string group-by: bad row count");
  if (key->n_strings < 0 || (key->n_strings > 0 && (!key->offsets || !key->bytes)))
    return fail(REL_EINVAL, "string group-by: NULL offsets or bytes");
  if (!key->codes && key->n_strings != n)
    return fail(REL_EINVAL, "string group-by: without codes every row is one string");
  if (n > 0 && key->n_strings == 0)
    return fail(REL_EINVAL, "string group-by: rows without strings");
  if (ikey) {
    rel_status st = check_column(ikey, "string group-by int key");
    if (st) return st;
    if (ikey->idx || ikey->len != n) return fail(REL_EINVAL, "string group-by: int key length");
  }
  if (nvals < 0 || nvals > REL_MAX_FACT_COLS || (nvals > 0 && !vals))
    return fail(REL_EINVAL, "string group-by: 0..%d value columns", REL_MAX_FACT_COLS);
  for (int v = 0; v < nvals; ++v) {
    rel_status st = check_column(&vals[v], "string group-by value");
    if (st) return st;
    if (vals[v].idx || vals[v].len != n) return fail(REL_EINVAL, "string group-by: value length");
  }
  rel_status st = check_aggs(aggs, naggs, nvals, "string group-by");
  if (st) return st;
  if (max_groups < 0) return fail(REL_EINVAL, "string group-by: negative max_groups");
  if (!d_groups || out_cap < 0 || (out_cap > 0 && !out_rows))
    return fail(REL_EINVAL, "string group-by: bad outputs");
  for (int a = 0; a < naggs && out_cap > 0; ++a)
    if (!out_aggs || !out_aggs[a]) return fail(REL_EINVAL, "string group-by: NULL output %d", a);
  GroupPlan gp;
  st = group_plan(0, nullptr, naggs, aggs, gp);
  if (st) return st;
  if (key->n_strings > kMaxRows) return fail(REL_EINVAL, "string group-by: too many strings");
  const int64_t n_dict = key->codes ? key->n_strings : 0;
  const StrLayout L = str_layout(max_groups, n_dict, gp.ap.nacc);
  st = check_ws(ws, ws_bytes, align_up(L.end));
  if (st) return st;
  unsigned char* w = static_cast<unsigned char*>(ws);
  StrGroupParams p;
  std::memset(&p, 0, sizeof p);
  p.offsets = key->offsets;
  p.bytes = key->bytes;
  p.codes = key->codes;
  p.n = n;
  if (ikey) {
    p.ikey = ikey->data;
    p.ikey_type = ikey->type;
  }
  for (int v = 0; v < nvals; ++v) {
    p.val[v] = vals[v].data;
    p.val_type[v] = vals[v].type;
  }
  p.ap = gp.ap;
  p.slots = reinterpret_cast<uint64_t*>(w + L.slots_off);
  p.mask = L.cap - 1;
  p.words = L.words;
  p.overflow = reinterpret_cast<int32_t*>(w + L.overflow_off);
  p.n_dict = n_dict;
  if (n_dict > 0) {
    p.dict_slots = reinterpret_cast<uint64_t*>(w + L.dict_off);
    p.dict_mask = L.dict_cap - 1;
    p.canon = reinterpret_cast<uint32_t*>(w + L.canon_off);
    p.slot_of = reinterpret_cast<uint32_t*>(w + L.slot_of_off);
  }
  p.lds_slots = str_lds_slots(L.cap, gp.ap.nacc);
  p.naggs = naggs;
  for (int a = 0; a < naggs; ++a) {
    p.agg_op[a] = aggs[a].op;
    p.agg_acc[a] = gp.agg_acc[a];
    p.out_aggs[a] = out_cap > 0 ? out_aggs[a] : nullptr;
  }
  p.out_rows = out_rows;
  p.out_ikey = out_ikey;
  p.cap = out_cap;
  p.d_groups = reinterpret_cast<unsigned long long*>(d_groups);
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_groupby_str(p, s);
  return after_launch(s, "string group-by");
}

// --------------------------------------------------------------- hash join

size_t rel_hash_join_ws(int32_t key_type, int64_t n_build, const rel_tuning* t) {
  if ((key_type != REL_I32 && key_type != REL_I64) || n_build < 0 || n_build > kMaxRows) return 0;
  if (t && check_tuning(t) != REL_OK) return 0;
  const MapLayout L = map_layout(key_type, n_build, load_factor(t), 0);
  const size_t end = join_part(L, n_build, t).end;
  if (t && (t->flags & REL_TUNE_BLOOM)) return align_up(end) + bloom_bytes(n_build, kBloomBitsPerKey);
  return end;
}

rel_status rel_hash_join(const rel_column* build_keys, const rel_column* probe_keys,
                         rel_rowid* out_build, rel_rowid* out_probe, int64_t out_cap,
                         int64_t* d_count, const rel_tuning* t, void* ws, size_t ws_bytes,
                         void* stream) {
  g_error.clear();
  rel_status st = check_column(build_keys, "join build keys");
  if (st) return st;
  st = check_column(probe_keys, "join probe keys");
  if (st) return st;
  if (build_keys->type != probe_keys->type)
    return fail(REL_EINVAL, "join: build and probe key types differ");
  if (build_keys->type == REL_I8) return fail(REL_EUNSUPPORTED, "join: int8 keys");
  if (out_cap < 0 || (out_cap > 0 && (!out_build || !out_probe)))
    return fail(REL_EINVAL, "join: bad outputs");
  if (!d_count) return fail(REL_EINVAL, "join: NULL count");
  st = check_tuning(t);
  if (st) return st;
  const MapLayout L = map_layout(build_keys->type, build_keys->len, load_factor(t), 0);
  const JoinPart jp = join_part(L, build_keys->len, t);
  const bool bloom = t && (t->flags & REL_TUNE_BLOOM);
  const size_t bloom_off = align_up(jp.end);
  const size_t bloom_len = bloom ? bloom_bytes(build_keys->len, kBloomBitsPerKey) : 0;
  st = check_ws(ws, ws_bytes, bloom ? bloom_off + bloom_len : jp.end);
  if (st) return st;

  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  const MapDesc m = map_desc(L, build_keys->type, w);
  if (jp.on) {
    // every slot is written by the range builds: only the header starts at zero
    launch_fill64(reinterpret_cast<uint64_t*>(m.oob_count), 2, 0, s);
    PartParams p;
    std::memset(&p, 0, sizeof p);
    p.g.kp.nkeys = 1;
    p.g.kp.type[0] = build_keys->type;
    p.g.words = 2;
    p.g.replicas = 1;
    p.key_data[0] = build_keys->data;
    p.key_idx[0] = build_keys->idx;
    p.ncols = 1;
    p.rw = 2;
    p.value_row = 1;
    p.n = build_keys->len;
    p.b1 = jp.b1;
    p.b2 = jp.b2;
    p.piece = kPartPiece;
    p.ctl = reinterpret_cast<unsigned long long*>(w + jp.ctl_off);
    p.rec_a = reinterpret_cast<uint64_t*>(w + jp.a_off);
    p.rec_b = reinterpret_cast<uint64_t*>(w + jp.b_off);
    p.map_key = build_keys->type;
    p.oob_count = m.oob_count;
    p.oob_vals = m.oob_vals;
    p.dup = m.dup;
    if ((static_cast<size_t>(1) << jp.span_log2) * L.slot_bytes >
        static_cast<size_t>(device_info().lds_per_block))
      return fail(REL_EUNSUPPORTED, "join: the partitioned build exceeds the LDS of a workgroup");
    launch_fill64(reinterpret_cast<uint64_t*>(p.ctl), kCtlZero, 0, s);
    launch_fill64(reinterpret_cast<uint64_t*>(p.ctl + kCtlSpill), 1, 0, s);
    hipError_t e = launch_map_partitioned(p, m, jp.span_log2, jp.sub, s);
    if (e != hipSuccess) return fail(REL_EDEVICE, "join: %s", hipGetErrorString(e));
  } else {
    launch_map_init(m, s);
    MapBuildParams b;
    std::memset(&b, 0, sizeof b);
    b.map = m;
    b.keys = build_keys->data;
    b.idx = build_keys->idx;
    b.type = build_keys->type;
    b.n = build_keys->len;
    launch_map_build(b, s);
  }
  launch_fill64(reinterpret_cast<uint64_t*>(d_count), 1, 0, s);
  MapProbeParams p;
  std::memset(&p, 0, sizeof p);
  p.map = m;
  p.keys = probe_keys->data;
  p.idx = probe_keys->idx;
  p.type = probe_keys->type;
  p.n = probe_keys->len;
  p.out_build = out_build;
  p.out_probe = out_probe;
  p.cap = out_cap;
  p.d_count = reinterpret_cast<unsigned long long*>(d_count);
  if (bloom) {
    // the build side's keys also go into a Bloom filter that the probe
    // consults before walking the table
    BloomBuildParams bb;
    std::memset(&bb, 0, sizeof bb);
    bb.words = reinterpret_cast<uint32_t*>(w + bloom_off);
    bb.bmask = bloom_len / 32 - 1;
    bb.keys = build_keys->data;
    bb.idx = build_keys->idx;
    bb.type = build_keys->type;
    bb.n = build_keys->len;
    launch_bloom_build(bb, s);
    p.bloom.words = bb.words;
    p.bloom.bmask = bb.bmask;
  }
  const DeviceInfo& di = device_info();
  int64_t blocks = (p.n + 255) / 256;
  int64_t limit = (t && t->grid > 0) ? t->grid : static_cast<int64_t>(di.cu_count) * 16;
  if (blocks > limit) blocks = limit;
  launch_map_probe(p, static_cast<int>(blocks < 1 ? 1 : blocks), 256, s);
  return after_launch(s, "hash join");
}

// ---------------------------------------------------------------- group-by

size_t rel_groupby_ws(int nkeys, const int32_t* key_types, int naggs, const rel_agg* aggs,
                      int64_t n_rows, int64_t max_groups, const rel_tuning* t) {
  if (nkeys < 0 || nkeys > REL_MAX_KEYS || naggs < 1 || naggs > REL_MAX_AGGS || !aggs ||
      (nkeys > 0 && !key_types) || max_groups < 0 || n_rows < 0 || n_rows > kMaxRows)
    return 0;
  for (int k = 0; k < nkeys; ++k)
    if (!valid_type(key_types[k])) return 0;
  if (t && check_tuning(t) != REL_OK) return 0;
  GroupPlan gp;
  if (group_plan(nkeys, key_types, naggs, aggs, gp) != REL_OK) return 0;
  PartPlan pp;
  return groupby_layout(gp, n_rows, max_groups, t, pp).end;
}

rel_status rel_groupby_agg(const rel_column* keys, int nkeys, const rel_column* vals, int nvals,
                           const rel_agg* aggs, int naggs, void* const* out_keys,
                           void* const* out_aggs, int64_t out_cap, int64_t* d_groups,
                           int64_t max_groups, const rel_tuning* t, void* ws, size_t ws_bytes,
                           void* stream) {
  g_error.clear();
  if (nkeys < 0 || nkeys > REL_MAX_KEYS || (nkeys > 0 && !keys))
    return fail(REL_EINVAL, "groupby: 0..%d key columns", REL_MAX_KEYS);
  if (nvals < 0 || nvals > REL_MAX_AGGS || (nvals > 0 && !vals))
    return fail(REL_EINVAL, "groupby: 0..%d value columns", REL_MAX_AGGS);
  if (nkeys == 0 && nvals == 0) return fail(REL_EINVAL, "groupby: no input columns");
  const int64_t n = nkeys > 0 ? keys[0].len : vals[0].len;
  int32_t key_types[REL_MAX_KEYS] = {0, 0};
  for (int k = 0; k < nkeys; ++k) {
    rel_status st = check_column(&keys[k], "groupby key");
    if (st) return st;
    if (keys[k].len != n) return fail(REL_EINVAL, "groupby: columns differ in length");
    key_types[k] = keys[k].type;
  }
  for (int v = 0; v < nvals; ++v) {
    rel_status st = check_column(&vals[v], "groupby value");
    if (st) return st;
    if (vals[v].len != n) return fail(REL_EINVAL, "groupby: columns differ in length");
  }
  rel_status st = check_aggs(aggs, naggs, nvals, "groupby");
  if (st) return st;
  st = check_outputs(out_keys, nkeys, out_aggs, naggs, out_cap, d_groups);
  if (st) return st;
  if (max_groups < 0) return fail(REL_EINVAL, "groupby: negative max_groups");
  st = check_tuning(t);
  if (st) return st;
  GroupPlan gp;
  st = group_plan(nkeys, key_types, naggs, aggs, gp);
  if (st) return st;
  PartPlan pp;
  const GroupLayout L = groupby_layout(gp, n, max_groups, t, pp);
  st = check_ws(ws, ws_bytes, L.end);
  if (st) return st;

  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  const GroupDesc g = group_desc(gp, L, w, d_groups);
  launch_group_init(g, s);
  if (pp.on) {
    PartParams p;
    std::memset(&p, 0, sizeof p);
    p.g = g;
    for (int k = 0; k < nkeys; ++k) {
      p.key_data[k] = keys[k].data;
      p.key_idx[k] = keys[k].idx;
    }
    for (int c = 0; c < pp.ncols; ++c) {
      const rel_column& col = vals[pp.cols[c]];
      p.col_data[c] = col.data;
      p.col_idx[c] = col.idx;
      p.col_type[c] = col.type;
    }
    p.ncols = pp.ncols;
    for (int a = 0; a < gp.ap.nacc; ++a) p.src[a] = pp.src[a];
    p.rw = pp.rw;
    p.n = n;
    p.b1 = pp.b1;
    p.b2 = pp.b2;
    p.pre_slots = pp.pre_slots;
    p.agg_slots = pp.agg_slots;
    p.piece = kPartPiece;
    p.ctl = reinterpret_cast<unsigned long long*>(w + pp.ctl_off);
    p.rec_a = reinterpret_cast<uint64_t*>(w + pp.a_off);
    p.rec_b = reinterpret_cast<uint64_t*>(w + pp.b_off);
    const DeviceInfo& di = device_info();
    const size_t scatter_lds = static_cast<size_t>(p.pre_slots) * gp.words * 8 +
                               (sizeof(uint32_t) << (p.b1 + p.b2)) + 12 * (1u << kPartLevelBits);
    if (scatter_lds > static_cast<size_t>(di.lds_per_block) ||
        static_cast<size_t>(p.agg_slots) * gp.words * 8 > static_cast<size_t>(di.lds_per_block))
      return fail(REL_EUNSUPPORTED, "groupby: the partitioned tables exceed the LDS of a workgroup");
    launch_fill64(reinterpret_cast<uint64_t*>(p.ctl), kCtlZero, 0, s);
    hipError_t e = launch_group_partitioned(p, s);
    if (e != hipSuccess) return fail(REL_EDEVICE, "groupby: %s", hipGetErrorString(e));
  } else if (n > 0) {
    GroupAggParams p;
    std::memset(&p, 0, sizeof p);
    p.g = g;
    for (int k = 0; k < nkeys; ++k) {
      p.key_data[k] = keys[k].data;
      p.key_idx[k] = keys[k].idx;
    }
    for (int a = 0; a < gp.ap.nacc; ++a) {
      const rel_column& c = vals[gp.ap.col[a]];
      p.val_data[a] = c.data;
      p.val_idx[a] = c.idx;
      p.val_type[a] = c.type;
    }
    p.n = n;
    const DeviceInfo& di = device_info();
    const int block = (t && t->block > 0) ? (t->block > 256 ? 256 : t->block) : 256;
    p.lds_slots = default_lds_slots(t, max_groups, gp.words, 32768);
    int64_t blocks = (n + block - 1) / block;
    int64_t limit = (t && t->grid > 0) ? t->grid : static_cast<int64_t>(di.cu_count) * 4;
    if (blocks > limit) blocks = limit;
    launch_group_agg(p, static_cast<int>(blocks), block, s);
  }
  launch_group_merge(g, s);
  launch_group_finalize(
      finalize_params(g, gp, aggs, naggs, out_keys, key_types, out_aggs, out_cap), s);
  return after_launch(s, "groupby");
}

// ---------------------------------------------------------------- pipeline

size_t rel_pipeline_ws(const rel_pipeline_desc* d) {
  if (check_pipeline(d) != REL_OK) return 0;
  PipeLayout L;
  if (pipeline_layout(d, L) != REL_OK) return 0;
  return L.end;
}

rel_status rel_pipeline(const rel_pipeline_desc* d, const rel_outputs* o, void* ws,
                        size_t ws_bytes, void* stream) {
  g_error.clear();
  rel_status st = check_pipeline(d);
  if (st) return st;
  if (!o) return fail(REL_EINVAL, "pipeline: NULL outputs");
  st = check_outputs(o->keys, d->n_keys, o->aggs, d->n_aggs, o->cap, o->d_groups);
  if (st) return st;
  PipeLayout L;
  st = pipeline_layout(d, L);
  if (st) return st;
  st = check_ws(ws, ws_bytes, L.end);
  if (st) return st;

  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  const rel_tuning* t = d->tuning;
  PipelineParams p;
  MapBuildParams b[REL_MAX_DIMS];
  plan_params(d, L, w, o->d_groups, false, p, b);
  for (int i = 0; i < d->n_dims; ++i) {
    launch_map_init(p.dim[i].map, s);
    launch_map_build(b[i], s);
  }
  launch_group_init(p.g, s);
  if (p.ntiles > 0) {
    const hipError_t e = launch_pipeline(p, (t && t->grid > 0) ? t->grid : 0, s);
    if (e != hipSuccess)
      return fail(REL_EDEVICE, "pipeline: fused kernel launch (%u bytes of LDS): %s", p.lds_bytes,
                  hipGetErrorString(e));
  }
  launch_group_merge(p.g, s);
  launch_group_finalize(finalize_params(p.g, L.gp, d->aggs, d->n_aggs, o->keys, L.key_types,
                                        o->aggs, o->cap),
                        s);
  return after_launch(s, "pipeline");
}

// ---------------------------------------------------------- out of core

}  // extern "C"

namespace rel {
namespace {

int type_bytes(int32_t type) { return type == REL_I8 ? 1 : (type == REL_I32 ? 4 : 8); }

// Staging of the streamed plan: two slots, each one chunk of every fact
// column (each column's part 256-byte aligned), after the plan's workspace.
struct StreamLayout {
  PipeLayout pipe;
  size_t col_off[REL_MAX_FACT_COLS];
  size_t slot_bytes = 0, slots_off = 0, end = 0;
};

rel_status stream_layout(const rel_pipeline_desc* d, int64_t chunk, StreamLayout& S) {
  rel_status st = pipeline_layout(d, S.pipe);
  if (st) return st;
  size_t off = 0;
  for (int c = 0; c < d->n_fact; ++c) {
    S.col_off[c] = off;
    off = align_up(off + static_cast<size_t>(chunk) * type_bytes(d->fact[c].type));
  }
  S.slot_bytes = off;
  S.slots_off = align_up(S.pipe.end);
  S.end = S.slots_off + 2 * S.slot_bytes;
  return REL_OK;
}

// The copy stream and events of the calling thread (created on first use,
// default priority, kept until the process ends).
struct StreamState {
  hipStream_t copy = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr};
  hipEvent_t freed[2] = {nullptr, nullptr};
  int device = -1;
};
thread_local StreamState g_stream_state;

rel_status stream_state(StreamState*& out) {
  StreamState& ss = g_stream_state;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(REL_EDEVICE, "pipeline stream: %s", hipGetErrorString(e));
  if (ss.copy && ss.device != dev) {
    // a different device from the last call: new stream and events there
    ss = StreamState();
  }
  if (!ss.copy) {
    e = hipStreamCreateWithFlags(&ss.copy, hipStreamNonBlocking);
    for (int k = 0; e == hipSuccess && k < 2; ++k) {
      e = hipEventCreateWithFlags(&ss.copied[k], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.freed[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) return fail(REL_EDEVICE, "pipeline stream: %s", hipGetErrorString(e));
    ss.device = dev;
  }
  out = &ss;
  return REL_OK;
}

}  // namespace
}  // namespace rel

extern "C" {

size_t rel_pipeline_stream_ws(const rel_pipeline_desc* d, int64_t chunk_rows) {
  if (check_pipeline(d) != REL_OK || chunk_rows < kPipeTile || chunk_rows % kPipeTile != 0)
    return 0;
  StreamLayout S;
  if (stream_layout(d, chunk_rows, S) != REL_OK) return 0;
  return S.end;
}

rel_status rel_pipeline_stream(const rel_pipeline_desc* d, int64_t chunk_rows,
                               const rel_outputs* o, void* ws, size_t ws_bytes, void* stream) {
  g_error.clear();
  rel_status st = check_pipeline(d);
  if (st) return st;
  if (chunk_rows < kPipeTile || chunk_rows % kPipeTile != 0)
    return fail(REL_EINVAL, "pipeline stream: chunk_rows must be a positive multiple of %d",
                kPipeTile);
  if (!o) return fail(REL_EINVAL, "pipeline stream: NULL outputs");
  st = check_outputs(o->keys, d->n_keys, o->aggs, d->n_aggs, o->cap, o->d_groups);
  if (st) return st;
  StreamLayout S;
  st = stream_layout(d, chunk_rows, S);
  if (st) return st;
  st = check_ws(ws, ws_bytes, S.end);
  if (st) return st;
  StreamState* ss = nullptr;
  st = stream_state(ss);
  if (st) return st;

  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  const int64_t n = d->fact[0].len;
  // the plan over one chunk (fact columns in a staging slot): its layout
  // does not depend on the fact length, so one workspace serves every chunk
  rel_column cols[REL_MAX_FACT_COLS];
  rel_pipeline_desc cd = *d;
  cd.fact = cols;
  for (int c = 0; c < d->n_fact; ++c) {
    cols[c] = d->fact[c];
    cols[c].data = w + S.slots_off + S.col_off[c];
    cols[c].len = n < chunk_rows ? n : chunk_rows;
  }
  PipelineParams p;
  MapBuildParams b[REL_MAX_DIMS];
  plan_params(&cd, S.pipe, w, o->d_groups, false, p, b);
  for (int i = 0; i < d->n_dims; ++i) {
    launch_map_init(p.dim[i].map, s);
    launch_map_build(b[i], s);
  }
  launch_group_init(p.g, s);
  hipError_t e = hipSuccess;
  for (int64_t k = 0, r0 = 0; r0 < n && e == hipSuccess; ++k, r0 += chunk_rows) {
    const int slot = static_cast<int>(k & 1);
    const int64_t rows = n - r0 < chunk_rows ? n - r0 : chunk_rows;
    unsigned char* base = w + S.slots_off + slot * S.slot_bytes;
    // copy stream: wait until the kernels that read this slot two chunks
    // ago are done, then bring in the chunk
    if (k >= 2) e = hipStreamWaitEvent(ss->copy, ss->freed[slot], 0);
    for (int c = 0; e == hipSuccess && c < d->n_fact; ++c) {
      const int wbytes = type_bytes(d->fact[c].type);
      e = hipMemcpyAsync(base + S.col_off[c],
                         static_cast<const unsigned char*>(d->fact[c].data) + r0 * wbytes,
                         static_cast<size_t>(rows) * wbytes, hipMemcpyHostToDevice, ss->copy);
    }
    if (e == hipSuccess) e = hipEventRecord(ss->copied[slot], ss->copy);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ss->copied[slot], 0);
    if (e != hipSuccess) break;
    // compute stream: the fused pass over the chunk, into the same groups
    for (int c = 0; c < d->n_fact; ++c) {
      cols[c].data = base + S.col_off[c];
      cols[c].len = rows;
    }
    PipelineParams pk;
    MapBuildParams unused[REL_MAX_DIMS];
    plan_params(&cd, S.pipe, w, o->d_groups, false, pk, unused);
    e = launch_pipeline(pk, (d->tuning && d->tuning->grid > 0) ? d->tuning->grid : 0, s);
    if (e == hipSuccess) e = hipEventRecord(ss->freed[slot], s);
  }
  if (e != hipSuccess) return fail(REL_EDEVICE, "pipeline stream: %s", hipGetErrorString(e));
  launch_group_merge(p.g, s);
  launch_group_finalize(finalize_params(p.g, S.pipe.gp, d->aggs, d->n_aggs, o->keys,
                                        S.pipe.key_types, o->aggs, o->cap),
                        s);
  return after_launch(s, "pipeline stream");
}

// ------------------------------------------------------------------ batches

size_t rel_pipeline_batch_ws(const rel_pipeline_desc* d, int n) {
  if (check_batch(d, n) != REL_OK) return 0;
  BatchLayout B;
  if (batch_layout(d, n, B) != REL_OK) return 0;
  return B.end;
}

namespace {

rel_status batch_prepare(const rel_pipeline_desc* d, int n, const rel_outputs* o, void* ws,
                         size_t ws_bytes, BatchLayout& B) {
  g_error.clear();
  rel_status st = check_batch(d, n);
  if (st) return st;
  if (!o) return fail(REL_EINVAL, "batch: NULL outputs");
  for (int i = 0; i < n; ++i) {
    st = check_outputs(o[i].keys, d[i].n_keys, o[i].aggs, d[i].n_aggs, o[i].cap, o[i].d_groups);
    if (st) return fail(st, "batch plan %d: %s", i, g_error.c_str());
  }
  st = batch_layout(d, n, B);
  if (st) return st;
  return check_ws(ws, ws_bytes, B.end);
}

int batch_grid(const rel_pipeline_desc* d) {
  return (d[0].tuning && d[0].tuning->grid > 0) ? d[0].tuning->grid : 0;
}

}  // namespace

rel_status rel_pipeline_batch(const rel_pipeline_desc* d, int n, const rel_outputs* o, void* ws,
                              size_t ws_bytes, void* stream) {
  BatchLayout B;
  rel_status st = batch_prepare(d, n, o, ws, ws_bytes, B);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  StagingSlot* sl = nullptr;
  st = staging_take(B.blob, sl);
  if (st) return st;
  PipelineParams shape;
  BatchParams bp, fused[kLdsClasses];
  batch_blob(d, n, o, B, w, static_cast<unsigned char*>(sl->host), shape, bp, fused);
  st = batch_enqueue(B, bp, fused, shape, w, sl->host, batch_grid(d), s);
  // the slot is reused once the stream is past the upload (or at once when
  // nothing was enqueued)
  if (hipEventRecord(sl->done, s) == hipSuccess) sl->pending = true;
  return st;
}

struct rel_graph {
  void* host;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

rel_status rel_pipeline_batch_graph(const rel_pipeline_desc* d, int n, const rel_outputs* o,
                                    void* ws, size_t ws_bytes, rel_graph** out) {
  if (!out) return fail(REL_EINVAL, "batch graph: NULL result pointer");
  *out = nullptr;
  BatchLayout B;
  rel_status st = batch_prepare(d, n, o, ws, ws_bytes, B);
  if (st) return st;
  unsigned char* w = static_cast<unsigned char*>(ws);
  rel_graph* g = new rel_graph{nullptr, nullptr, nullptr};
  hipStream_t cs = nullptr;
  auto bail = [&](rel_status code, const char* what, hipError_t e) {
    if (cs) (void)hipStreamDestroy(cs);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->host) (void)hipHostFree(g->host);
    delete g;
    return code == REL_EDEVICE ? fail(code, "batch graph: %s: %s", what, hipGetErrorString(e))
                               : code;
  };
  hipError_t e = hipHostMalloc(&g->host, B.blob, hipHostMallocDefault);
  if (e != hipSuccess) return bail(REL_EDEVICE, "pinned descriptor block", e);
  PipelineParams shape;
  BatchParams bp, fused[kLdsClasses];
  batch_blob(d, n, o, B, w, static_cast<unsigned char*>(g->host), shape, bp, fused);
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(REL_EDEVICE, "capture stream", e);
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return bail(REL_EDEVICE, "begin capture", e);
  g_capturing = true;
  st = batch_enqueue(B, bp, fused, shape, w, g->host, batch_grid(d), cs);
  g_capturing = false;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  g->graph = graph;
  if (st) return bail(st, nullptr, hipSuccess);
  if (e != hipSuccess) return bail(REL_EDEVICE, "end capture", e);
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(REL_EDEVICE, "instantiate", e);
  (void)hipStreamDestroy(cs);
  *out = g;
  return REL_OK;
}

rel_status rel_graph_launch(rel_graph* g, void* stream) {
  g_error.clear();
  if (!g || !g->exec) return fail(REL_EINVAL, "graph launch: NULL graph");
  const hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(REL_EDEVICE, "graph launch: %s", hipGetErrorString(e));
  return REL_OK;
}

void rel_graph_destroy(rel_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->host) (void)hipHostFree(g->host);
  delete g;
}

// ------------------------------------------------------- synchronous forms

}  // extern "C"

namespace rel {
namespace {

// Waits for `stream` and reads the device int64 at d_count into *count;
// REL_ECAPACITY when it exceeds cap (or, for group counts, is -1).
rel_status read_count(rel_status st, const int64_t* d_count, int64_t cap, void* stream,
                      int64_t* count, const char* what) {
  if (st != REL_OK) return st;
  int64_t host = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&host, d_count, sizeof host, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(REL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  if (count) *count = host;
  if (host < 0) return fail(REL_ECAPACITY, "%s: more groups than max_groups", what);
  if (host > cap)
    return fail(REL_ECAPACITY, "%s: %lld results exceed the output capacity %lld", what,
                static_cast<long long>(host), static_cast<long long>(cap));
  return REL_OK;
}

}  // namespace
}  // namespace rel

extern "C" {

rel_status rel_filter_sync(const rel_column* cols, int ncols, const rel_pred* preds, int npreds,
                           rel_rowid* out, int64_t out_cap, int64_t* d_count, void* ws,
                           size_t ws_bytes, void* stream, int64_t* count) {
  return read_count(rel_filter(cols, ncols, preds, npreds, out, out_cap, d_count, ws, ws_bytes,
                               stream),
                    d_count, out_cap, stream, count, "filter");
}

rel_status rel_hash_join_sync(const rel_column* build_keys, const rel_column* probe_keys,
                              rel_rowid* out_build, rel_rowid* out_probe, int64_t out_cap,
                              int64_t* d_count, const rel_tuning* t, void* ws, size_t ws_bytes,
                              void* stream, int64_t* count) {
  return read_count(rel_hash_join(build_keys, probe_keys, out_build, out_probe, out_cap, d_count, t,
                                  ws, ws_bytes, stream),
                    d_count, out_cap, stream, count, "hash join");
}

rel_status rel_groupby_agg_sync(const rel_column* keys, int nkeys, const rel_column* vals,
                                int nvals, const rel_agg* aggs, int naggs, void* const* out_keys,
                                void* const* out_aggs, int64_t out_cap, int64_t* d_groups,
                                int64_t max_groups, const rel_tuning* t, void* ws,
                                size_t ws_bytes, void* stream, int64_t* groups) {
  return read_count(rel_groupby_agg(keys, nkeys, vals, nvals, aggs, naggs, out_keys, out_aggs,
                                    out_cap, d_groups, max_groups, t, ws, ws_bytes, stream),
                    d_groups, out_cap, stream, groups, "group-by");
}

rel_status rel_pipeline_sync(const rel_pipeline_desc* d, const rel_outputs* o, void* ws,
                             size_t ws_bytes, void* stream, int64_t* groups) {
  if (!o) return fail(REL_EINVAL, "pipeline: NULL outputs");
  return read_count(rel_pipeline(d, o, ws, ws_bytes, stream), o->d_groups, o->cap, stream, groups,
                    "pipeline");
}

}  // extern "C"
