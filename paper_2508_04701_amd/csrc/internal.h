// Host <-> kernel interface of the library: launch parameter blocks and the
// launcher entry points implemented next to each kernel. The public C-ABI in
// api.cpp validates arguments, carves the workspace and calls these.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace rel {

// ------------------------------------------------------------------ common

struct DeviceInfo {
  int cu_count;
  int lds_per_block;  // bytes of LDS one workgroup may use
};
const DeviceInfo& device_info();

// Per-kernel timing: when enabled, launch sites bracket each kernel with a
// pair of events on the launch stream (kernel classes as in rel.h).
enum KernelClass : int {
  kKFill = 0, kKFilter, kKMapBuild, kKMapProbe, kKGroupAgg, kKPipeline, kKFinalize,
  kKGroupPartition, kKStream, kKBloom, kKGather, kKTopN, kKCount
};
struct ProfileScope {
  ProfileScope(int kclass, hipStream_t s);
  ~ProfileScope();
  int k;
  hipStream_t s;
  void* start;
};

// The calling thread's rel_last_error() message: set_last_error stores msg
// and returns status; clear_last_error empties it (api.cpp).
int set_last_error(int status, const char* msg);
void clear_last_error();

// Fills n 64-bit words with `pattern` (graph-safe replacement for memset).
void launch_fill64(uint64_t* p, uint64_t n, uint64_t pattern, hipStream_t s);

// Reads `bytes` bytes at `data` (16-byte aligned) once; *out = XOR of its
// zero-padded 64-bit words.
hipError_t launch_stream_read(const void* data, uint64_t bytes, unsigned long long* out,
                              hipStream_t s);

// --------------------------------------------------------------- filter

constexpr int kFilterThreads = 512;
constexpr int kFilterChunks = 8;                               // chunks of 4 rows per thread
constexpr int kFilterTile = kFilterThreads * 4 * kFilterChunks;  // rows per tile
constexpr int kFilterGroupTiles = 64;  // tiles per offset group of the bitmap path

struct FilterTerm {
  const void* data;
  int32_t type;
  int32_t op;
  int64_t lo, hi;
  int32_t vec;  // data is 16-byte aligned
};

struct FilterParams {
  FilterTerm term[4];
  int32_t nterms;
  const uint32_t* idx;  // optional gather
  int64_t n;
  uint32_t* out;
  int64_t cap;
  long long* d_count;
  uint64_t* tile_state;  // one word per tile, zeroed (look-back path)
  uint32_t* ticket;      // zeroed (look-back path)
  int64_t ntiles;
  uint32_t* bitmap;        // bitmap path: kFilterTile / 32 words per tile
  uint32_t* tile_count;    // bitmap path: passing rows per tile
  uint64_t* group_offset;  // bitmap path: exclusive prefix per kFilterGroupTiles tiles
  // Optional semi-join reduction: a row also needs its key (bloom_keys,
  // gathered through idx like the terms' columns) to pass the Bloom filter.
  BloomDesc bloom;       // words == NULL: none
  const void* bloom_keys;
  int32_t bloom_type;
  int32_t bloom_vec;     // bloom_keys is 16-byte aligned
};

// Single pass with a decoupled look-back over ticketed tiles (tile_state,
// ticket): the allocation-free filter's path.
void launch_filter(const FilterParams& p, hipStream_t s);
// Selection bitmap, tile counts and offsets (bitmap, tile_count,
// tile_offset): mark, scan and expand passes.
void launch_filter_marked(const FilterParams& p, hipStream_t s);

// Static scratch of the allocation-free filter: the ticket word's 256-byte
// block plus one tile-state word per 16384-row tile. 1 MiB holds the states
// of 131040 tiles, i.e. up to 2,146,959,360 rows.
constexpr size_t kFilterScratchBytes = size_t(1) << 20;
constexpr int64_t kFilterNoallocMaxRows =
    static_cast<int64_t>((kFilterScratchBytes - 256) / 8) * kFilterTile;

// Device address of the calling thread's current device's copy of the
// filter scratch, looked up once per device.
hipError_t filter_scratch(void** ptr);

// ------------------------------------------------- late materialisation

// out dst[c][i] = src[c][ids[i]] (element type type[c]) for i < n.
struct GatherParams {
  const void* src[8];
  int32_t type[8];
  void* dst[8];
  int32_t ncols;
  int32_t ids_vec;  // ids is 16-byte aligned
  const uint32_t* ids;
  int64_t n;
};
void launch_gather(const GatherParams& p, hipStream_t s);

// Top-N: composite sort keys (a, b, c, row) in two candidate buffers of
// lists of `pow2` entries each.
constexpr int kTopMax = 1024;   // largest N
constexpr int kTopFanIn = 16;   // lists folded per workgroup in a merge round
struct TopBuf {
  uint64_t* a;
  uint64_t* b;
  uint64_t* c;
  uint32_t* row;
};
struct TopNParams {
  const void* order;        // int64 values or binary64 bit patterns
  int32_t order_is_double;
  int32_t desc;
  const void* keys[2];
  int32_t key_type[2];
  int32_t nkeys;
  int32_t pow2;             // power of two >= limit, <= kTopMax
  int64_t n;
  int64_t limit;
  int64_t span;             // rows per workgroup of the first phase
  int32_t nlists;           // workgroups of the first phase (0 when n == 0)
  TopBuf buf[2];
  uint32_t* out;
  long long* d_count;
};
hipError_t launch_topn(const TopNParams& p, hipStream_t s);

// ------------------------------------------------------ string group-by

// Group-by on a string key (Arrow offsets/bytes, optionally through
// dictionary codes) and an optional integer key; slots of `words` words:
// claim word, COUNT, first row, accumulators.
struct StrGroupParams {
  const int64_t* offsets;
  const uint8_t* bytes;
  const int32_t* codes;  // NULL: row i is string i
  int64_t n;
  int64_t n_dict;         // dictionary entries (codes only)
  uint64_t* dict_slots;   // claim words of the dictionary's string table
  uint64_t dict_mask;
  uint32_t* canon;        // canonical id of each dictionary entry
  uint32_t* slot_of;      // group slot of each dictionary entry (no integer key)
  int32_t lds_slots;      // LDS pre-aggregation entries (0 or a power of two)
  const void* ikey;      // NULL: no integer key
  int32_t ikey_type;
  const void* val[8];
  int32_t val_type[8];
  AccPlan ap;
  uint64_t* slots;
  uint64_t mask;
  int32_t words;
  int32_t* overflow;
  int32_t naggs;
  int32_t agg_op[8];
  int32_t agg_acc[8];
  uint32_t* out_rows;
  void* out_ikey;
  void* out_aggs[8];
  int64_t cap;
  unsigned long long* d_groups;
};
void launch_groupby_str(const StrGroupParams& p, hipStream_t s);

// ------------------------------------------------------------- hash maps

// Geometry of one multimap in the workspace.
struct MapDesc {
  int32_t key_type;   // kI32 or kI64
  int32_t key_only;   // int32 keys without values (membership): 4-byte slots
  int32_t compact;    // membership set in 16-bit entries (CsetDesc layout)
  int32_t rbits;      // compact: remainder bits
  uint64_t cap;       // slots (power of two)
  void* slots;        // cap * 4 (key-only), 8 (int32 keys) or 16 (int64 keys) bytes
  unsigned long long* oob_count;
  uint32_t* oob_vals;  // n entries
  int32_t* dup;        // set by the build when a key occurs twice
  uint32_t* over;      // compact: overflow key-only set
  uint64_t over_cap;   // compact: its slots (power of two)
  // Dense keys (int32 only): when the build keys span at most direct_cap
  // values and none repeats, key k is held at index k - kmin of a presence
  // bitmap and, with a payload, of a payload array, instead of the slot
  // array. The build decides on the device; see DirectState.
  uint64_t direct_cap;   // 0: no direct table reserved
  uint64_t nkeys;        // build keys
  uint32_t* dbits;       // direct_cap bits
  void* dvals;           // direct_cap payload entries (1, 2 or 4 bytes each), or NULL
  int32_t* dstate;       // DirectState
};

// Key and payload ranges of a build (device, reduced by the first build
// pass; kmin/pmin start at INT32_MAX, kmax/pmax at INT32_MIN).
enum DirectState : int { kDKmin = 0, kDKmax = 1, kDPmin = 2, kDPmax = 3 };
// Two 64-bit words that initialise a DirectState: (INT32_MAX, INT32_MIN) twice.
constexpr uint64_t kDirectStateInit = 0x800000007FFFFFFFULL;

// A direct table as its readers see it (uniform values). Payload entries
// hold payload - pmin in the fewest bytes (1, 2 or 4) that cover the range.
// mode: 0 = not in use (the dim's slot array holds the keys); otherwise
// kDirectOn | (keys fill [kmin, kmin + range) ? kDirectFull : 0) | width << 2.
constexpr uint32_t kDirectOn = 1, kDirectFull = 2;
struct DirectView {
  uint32_t mode;
  int32_t kmin, pmin;
  uint32_t range;
  const uint32_t* bits;
  const void* vals;
};

__device__ __forceinline__ int direct_width(int32_t pmin, int32_t pmax) {
  const int64_t span = static_cast<int64_t>(pmax) - pmin;
  return span < 256 ? 1 : (span < 65536 ? 2 : 4);
}

// The key range of a build once its range pass is done (0: no keys), and
// whether it fits the reserved table.
__device__ __forceinline__ uint64_t direct_range(const MapDesc& m) {
  const int32_t kmin = m.dstate[kDKmin], kmax = m.dstate[kDKmax];
  if (kmax < kmin) return 0;
  return static_cast<uint64_t>(static_cast<int64_t>(kmax) - kmin + 1);
}

// Valid after the build: duplicates send the dim back to its slot array.
// (A direct table needs its range below 2^32, which a build of fewer than
// 2^31 keys guarantees; larger ranges keep the slot array.)
__device__ __forceinline__ DirectView direct_view(const MapDesc& m) {
  DirectView v;
  v.mode = 0;
  v.kmin = 0;
  v.pmin = 0;
  v.range = 0;
  v.bits = m.dbits;
  v.vals = m.dvals;
  if (m.direct_cap == 0) return v;
  const uint64_t range = direct_range(m);
  if (range == 0 || range > m.direct_cap || range >= (1ull << 32) || *m.dup) return v;
  v.range = static_cast<uint32_t>(range);
  v.kmin = m.dstate[kDKmin];
  v.mode = kDirectOn | (range == m.nkeys ? kDirectFull : 0u);
  if (m.dvals) {
    v.pmin = m.dstate[kDPmin];
    v.mode |= static_cast<uint32_t>(direct_width(v.pmin, m.dstate[kDPmax])) << 2;
  }
  return v;
}

// Probe of a direct table: whether `key` is present, and its payload.
__device__ __forceinline__ bool direct_probe(const DirectView& v, int64_t key, uint32_t& val) {
  const uint64_t off = static_cast<uint64_t>(key - static_cast<int64_t>(v.kmin));
  if (off >= v.range) return false;
  const uint32_t i = static_cast<uint32_t>(off);
  if (!(v.mode & kDirectFull) && !((v.bits[i >> 5] >> (i & 31)) & 1u)) return false;
  const uint32_t width = v.mode >> 2;
  if (width == 1) val = static_cast<uint32_t>(static_cast<const uint8_t*>(v.vals)[i]) + v.pmin;
  else if (width == 2) val = static_cast<uint32_t>(static_cast<const uint16_t*>(v.vals)[i]) + v.pmin;
  else if (width == 4) val = static_cast<const uint32_t*>(v.vals)[i] + static_cast<uint32_t>(v.pmin);
  return true;
}

// Inserts n keys of column (data, idx, type); value of element i is
// val_col[i] widened to 32 bits when val_col is set, else its row id.
struct MapBuildParams {
  MapDesc map;
  const void* keys;
  const uint32_t* idx;
  int32_t type;
  int64_t n;
  const void* val_col;
  int32_t val_type;
  // Batched builds of direct tables with payloads (nwin > 0): the rows are
  // first grouped by window of kWinKeys keys, so that each window's bits and
  // payloads are set in LDS and written out whole (see launch_batch_build).
  uint64_t* wpairs;   // n (key, payload) pairs, window by window
  uint32_t* wcursor;  // nwin: rows per window (zero at the start), then its next free place
  uint32_t* wbegin;   // nwin + 1 offsets into wpairs
  uint32_t nwin;
};

constexpr uint64_t kBuildChunk = 8192;  // build rows per batch build item
constexpr uint32_t kWinBits = 14;
constexpr uint32_t kWinKeys = 1u << kWinBits;
constexpr uint32_t kMaxWins = 4096;  // windows of one dim (larger tables use slices)

void launch_map_init(const MapDesc& m, hipStream_t s);
// Three passes: key (and payload) ranges, the direct table if the range
// allows, the slot array unless the direct table holds every key once.
void launch_map_build(const MapBuildParams& p, hipStream_t s);

// Probe: emits (value, probe row id) for every match, with a wave-aggregated
// cursor in d_count (zeroed by launch_map_init's companion below).
struct MapProbeParams {
  MapDesc map;
  const void* keys;
  const uint32_t* idx;
  int32_t type;
  int64_t n;
  uint32_t* out_build;
  uint32_t* out_probe;
  int64_t cap;
  unsigned long long* d_count;
  BloomDesc bloom;  // words != NULL: probe keys absent from this filter skip the table
};

// Clears the filter (blocks * 32 bytes at words) and inserts the n keys of
// column (keys, idx, type).
struct BloomBuildParams {
  uint32_t* words;
  uint64_t bmask;
  const void* keys;
  const uint32_t* idx;
  int32_t type;
  int64_t n;
};
void launch_bloom_build(const BloomBuildParams& p, hipStream_t s);

void launch_map_probe(const MapProbeParams& p, int grid, int block, hipStream_t s);

// ------------------------------------------------------------- group-by

// The global group table may be replicated: workgroup w merges into replica
// w mod `replicas`, which divides the same-address atomic contention of few
// groups by the replica count; a merge pass folds the replicas into replica
// 0 before the finalize reads it.
struct GroupDesc {
  GroupKeyPack kp;
  AccPlan ap;
  uint64_t cap;      // slots of the open-addressing array (power of two)
  int32_t words;     // 64-bit words per slot
  int32_t replicas;  // >= 1
  uint64_t* slots;   // replicas * (cap + 1) * words words
  int32_t* overflow;
  unsigned long long* d_groups;  // output count (zeroed by init)
};

__device__ __forceinline__ GroupTable group_replica(const GroupDesc& g, uint32_t r) {
  return GroupTable{g.slots + static_cast<uint64_t>(r) * (g.cap + 1) * g.words, g.cap - 1, g.words,
                    g.overflow};
}

void launch_group_init(const GroupDesc& g, hipStream_t s);

struct GroupAggParams {
  GroupDesc g;
  const void* key_data[2];
  const uint32_t* key_idx[2];
  const void* val_data[kMaxAcc];
  const uint32_t* val_idx[kMaxAcc];
  int32_t val_type[kMaxAcc];
  int64_t n;
  int32_t lds_slots;  // 0: no LDS table
};

void launch_group_agg(const GroupAggParams& p, int grid, int block, hipStream_t s);

// Radix-partitioned aggregation for group tables far beyond the caches.
// Rows are split by the top pb = b1 + b2 bits of the key hash into 2^pb
// partitions in two scatter passes (2^b1 buckets, then 2^b2 partitions per
// bucket), so that each partition holds few enough distinct keys for an LDS
// table; the aggregation pass then folds each partition in LDS and merges the
// table into the global one. The global table indexes its slots by the top
// hash bits too, so partition q's merges stay within slot range q of the
// table. The first scatter keeps a small LDS table of its own: rows whose key
// it holds (the hot keys under skew) are aggregated there and never moved.
// A record is the packed key followed by the row's value columns (int64).
constexpr int kPartMaxBits = 14;     // at most 2^14 partitions
constexpr int kPartLevelBits = 7;    // at most 2^7 ways per scatter pass
constexpr int kPartThreads = 512;    // scatter workgroups
constexpr int kPartRows = 16;        // rows (records) per thread and scatter tile
constexpr int kPartTile = kPartThreads * kPartRows;
constexpr int kPartAggThreads = 1024;
constexpr int kPartPad = 16;         // words between claim cursors (one 128-byte line)
// The count and first scatter passes give workgroup w (of kPartGroups) the
// same fixed range of rows; (bucket b, workgroup w) is segment b * kPartGroups
// + w of the first record buffer, placed by a prefix sum over the counts, so
// the first scatter needs no global atomics.
constexpr int kPartGroups = 512;
constexpr uint64_t kPartSegs = static_cast<uint64_t>(kPartGroups) << kPartLevelBits;
// Control words: counts, prefix sums and claim cursors.
constexpr uint64_t kCtlHist2 = 0;                                   // 2^pb partition sizes
constexpr uint64_t kCtlZero = 1u << kPartMaxBits;                   // words zeroed per call
constexpr uint64_t kCtlSegCount = kCtlZero;                         // rows per segment
constexpr uint64_t kCtlSegStart = kCtlSegCount + kPartSegs;         // segment starts (+ total)
constexpr uint64_t kCtlSegFill = kCtlSegStart + kPartSegs + 256;    // records per segment
constexpr uint64_t kCtlTiles = kCtlSegFill + kPartSegs;             // second-scatter tile prefix
constexpr uint64_t kCtlStart2 = kCtlTiles + kPartSegs + 256;        // partition starts (+ total)
constexpr uint64_t kCtlPieces = kCtlStart2 + (1u << kPartMaxBits) + 256;  // piece prefix (+ total)
constexpr uint64_t kCtlCur2 = kCtlPieces + (1u << kPartMaxBits) + 256;    // padded cursors
constexpr uint64_t kCtlWords = kCtlCur2 + (1u << kPartMaxBits) * static_cast<uint64_t>(kPartPad);

struct PartParams {
  GroupDesc g;  // one replica
  const void* key_data[2];
  const uint32_t* key_idx[2];
  const void* col_data[kMaxAcc];  // value columns copied into the records
  const uint32_t* col_idx[kMaxAcc];
  int32_t col_type[kMaxAcc];
  int32_t ncols;
  int32_t src[kMaxAcc];  // accumulator a aggregates record word 1 + src[a]
  int32_t rw;            // record words: 1 + ncols
  int64_t n;
  int32_t b1, b2;
  int32_t pre_slots;  // LDS table of the first scatter (0: none)
  int32_t agg_slots;  // LDS table of the aggregation pass (power of two)
  uint32_t piece;     // records per aggregation work item
  uint64_t* rec_a;    // n * rw words: records grouped by bucket
  uint64_t* rec_b;    // n * rw words: records grouped by partition
  unsigned long long* ctl;  // kCtlWords control words
  // Map builds (map_key != 0): records are (key, row id or payload); the
  // partition is the top bits of the map's home hash (the 32-bit key hash for
  // int32 keys); sentinel keys go to the map's out-of-band list instead.
  int32_t map_key;  // 0: group-by; kI32 or kI64: the map's key type
  int32_t value_row;  // the record value is the row id (idx[r] or r)
  unsigned long long* oob_count;
  uint32_t* oob_vals;
  int32_t* dup;
};

constexpr uint64_t kCtlSpill = kCtlWords;  // map builds: records spilled past their range
constexpr uint64_t kCtlAll = kCtlWords + 32;

// Runs the counting, scatter and aggregation passes into p.g (initialised).
hipError_t launch_group_partitioned(const PartParams& p, hipStream_t s);

// Partitioned map build: the counting and scatter passes, then each range of
// 2^span_log2 slots built in LDS and written whole (`sub` ranges per
// partition), then the spilled keys by global CAS. Every slot of m is written.
hipError_t launch_map_partitioned(const PartParams& p, const MapDesc& m, int span_log2, int sub,
                                  hipStream_t s);

// Output agg a: op (rel_agg_op) and the accumulator it reads.
struct FinalizeParams {
  GroupDesc g;
  int32_t naggs;
  int32_t op[8];
  int32_t acc[8];  // accumulator index (SUM/MIN/MAX/AVG)
  void* out_keys[2];
  int32_t out_key_type[2];
  void* out_aggs[8];
  int64_t cap;
};

// Folds replicas 1.. of the global group table into replica 0.
void launch_group_merge(const GroupDesc& g, hipStream_t s);

void launch_group_finalize(const FinalizeParams& p, hipStream_t s);

// ------------------------------------------------------------- pipeline

struct PipeDim {
  MapDesc map;
  int32_t fk_col;
  int32_t in_lds;        // copy the slot array into LDS
  uint32_t lds_offset;   // byte offset of the copy in dynamic LDS
};

// Queued row fields: row id, the two foreign keys and the resume state of
// each dim's probe (0: not started; k: k buckets already scanned;
// kResolved | slot: found at that slot).
enum QueueField : int { kQRow = 0, kQFk0, kQFk1, kQSt0, kQSt1, kQueueFields };

// Spilled-row records of a batched plan (hash grouping, Section 4.2, for
// group counts beyond the LDS table): a row of the fused pass that finds no
// LDS slot is written out as a record of `words` 64-bit words (its packed
// group key, then the early value columns) instead of updating the global
// table with device-scope atomics. A scan turns the per-(partition, item)
// counts into offsets, a scatter groups the records by partition (the top
// bits of the key's LDS hash), and an aggregation pass folds each partition,
// in pieces, into an LDS table that then merges into the global table with
// one update per key. parts == 0: the plan's spilled rows use atomics.
struct RecDesc {
  uint64_t* recs;         // item j's records start at word j * item_tiles * kPipeTile * words
  uint64_t* parted;       // the records in partition order
  // Narrow records (narrow != 0, words == 2): the key's low 32 bits in their
  // own arrays (rkeys beside recs, pkeys beside parted; recs and parted then
  // hold the value word alone), 12 bytes a record; the packed key is the
  // 32 bits sign-extended (narrow 1: one int8 or int32 key) or zero-extended
  // (narrow 2: two keys of at most 32 bits together).
  uint32_t* rkeys;
  uint32_t* pkeys;
  uint32_t narrow;
  uint32_t* counts;       // [nitems][parts] records per (item, partition)
  uint32_t* item_n;       // records of each item
  uint32_t* part_begin;   // parts + 1 offsets into parted
  uint32_t* cursor;       // parts words, zero at the start: each partition's record total
                          // (the fused pass adds each item's), then its next free place
                          // in parted (set by the scan, taken by the scatter's atomics)
  uint32_t parts;         // a power of two, at most kMaxRecParts; 0 = off
  uint32_t agg_parts;     // partitions the aggregation pass folds one by one: runs of
                          // parts / agg_parts consecutive partitions (the top bits agree)
  uint32_t words;         // 64-bit words per record (2 or 3; 1 = COUNT only)
  uint32_t nitems;        // fused-pass items of the plan
  uint32_t item_tiles;    // fact tiles per item
  uint32_t lds_offset;    // fused pass: byte offset of the LDS histogram (parts + 1 words)
  uint32_t agg_slots;     // LDS table slots of the aggregation pass (a power of two)
};

constexpr uint32_t kMaxRecParts = 1024;
// At least this many partitions in the fused pass and the scatter, so that
// the lanes of a wave rarely count into the same LDS word.
constexpr uint32_t kMinRecParts = 16;
constexpr uint32_t kRecPiece = 1u << 17;  // records per aggregation work item
constexpr uint32_t kRecAggLds = 65536;     // bound on the aggregation pass's LDS table

struct PipelineParams {
  const void* fact[8];
  int32_t fact_type[8];
  int32_t fact_vec[8];
  int64_t n;
  int32_t nterms;
  int32_t term_col[4];
  int32_t term_op[4];
  int64_t term_lo[4], term_hi[4];
  int32_t ndims;
  PipeDim dim[2];
  // group key k: fact column (src 0) or dim payload (src 1 + d)
  int32_t key_src[2];
  int32_t key_col[2];
  GroupDesc g;
  int32_t acc_col[kMaxAcc];  // fact column of each accumulator
  int32_t early_col[2];       // value columns loaded with the keys (-1: none)
  int32_t acc_src[kMaxAcc];   // 0/1: value from early_col[k]; -1: loaded late
  int32_t lds_slots;          // LDS group table slots (0: none)
  int32_t spec;               // row spec of the fused kernels (0: generic)
  int64_t spec_lo;            // specialised kernels: the predicate term as the range
  uint64_t spec_span;         //   [spec_lo, spec_lo + spec_span) of the widened value
  const void* spec_key[2];    //   the fact columns of fact keys (no indirection in the loop)
  const int64_t* spec_val;    //   the value column
  int32_t directable;         // every dim reserved a direct table (or there are none)
  uint32_t lds_group_offset;  // byte offset of the LDS group table
  uint32_t lds_bytes;
  int64_t ntiles;
  // Per-wave row queues in LDS: field f of queued row i lives at
  // queue_offset + wave * queue_stride + field_offset[f] + i * (4 or 8).
  uint32_t queue_offset;
  uint32_t queue_stride;
  uint32_t field_offset[kQueueFields];
  int32_t field_wide[kQueueFields];   // 8-byte (1) or 4-byte (0) elements
  RecDesc rec;                        // batched plans only
};

constexpr int kPipeThreads = 512;
constexpr int kPipeTile = kPipeThreads * 4;  // rows per tile: four per thread
constexpr int kPipeQueue = 128;              // queued rows per wave (one batch + one push)
constexpr int kMaxPipeGrid = 2048;           // bound on the persistent grid

// Returns the first failing HIP status of the launch.
hipError_t launch_pipeline(const PipelineParams& p, int grid, hipStream_t s);

// --------------------------------------------------------------- batches
//
// A batch runs n plans of one shape (same dim count, dim key types and
// payload presence) with one launch per phase: fill, build, fused pass,
// duplicate-key pass, replica merge, finalize. Each phase walks a list of
// work items, each naming an instance and a half-open range of that phase's
// units (words, build rows, fact tiles, group slots). The fused pass is
// persistent and takes its items in order from a device counter; the other
// phases run one workgroup per item, handed out in order by the dispatcher.
// Either way a large instance is spread over the whole chip and many small
// ones share it.

// Units: tiles (fused and duplicate passes), rows (builds; aux = dim),
// slots (merge: replica slots 1.., finalize: replica 0).
struct BatchItem {
  uint32_t inst;
  uint32_t aux;
  uint64_t begin, end;
};

// Records [begin, end) of partition `part` of plan `inst`'s records.
struct RecPiece {
  uint32_t inst, part, begin, end;
};

enum FillKind : int32_t { kFillConst = 0, kFillPairs = 1, kFillGroup = 2 };

// Words [begin, end) of the region at p: the constant `pattern`, key/value
// pairs (kEmpty64, 0) of an int64 map, or the empty slots of instance
// `inst`'s group table (key kEmpty64, COUNT 0, accumulator identities).
struct FillItem {
  uint64_t* p;
  uint64_t begin, end;
  uint64_t pattern;
  int32_t kind;
  uint32_t inst;
};

// Device arrays (read-only during the batch) and item lists of one batch.
struct BatchParams {
  const PipelineParams* plans;   // n
  const MapBuildParams* builds;  // 2n: dim d of instance i at 2i + d
  const FinalizeParams* fins;    // n
  const FillItem* fill;
  const BatchItem* build_items;
  const BatchItem* tile_items;
  const BatchItem* merge_items;
  const BatchItem* fin_items;
  const BatchItem* slice_items;  // direct-table slices: begin = first bit, aux = dim
  const BatchItem* win_items;    // direct-table windows: begin = window, aux = dim
  uint32_t nfill, nbuild, ntile, nmerge, nfin, nslice, nwin;
  uint32_t slice_bits;           // bits of a direct-table slice (a power of two)
  uint32_t lds_bytes;        // dynamic LDS of the fused pass (same for every plan)
  uint32_t group_lds_bytes;  // LDS group table bytes of the largest plan
  unsigned long long* counter;  // fused-pass item counter, zero at the start
  // spilled-row records: every plan, every fused-pass item (all classes),
  // the aggregation pieces the scan lists, and the aggregation pass's LDS
  uint32_t nplans, ntile_all;
  uint32_t rec_plans;           // plans with records (0: the record passes are skipped)
  uint32_t agg_lds_bytes;
  uint32_t piece_cap;           // bound on the pieces the scan lists
  RecPiece* pieces;
  unsigned long long* npieces;  // written by the scan, zero at the start
  unsigned long long* agg_counter;  // zero at the start
};

// Reference to element i of a batch array: read through the constant address
// space, so that uniform reads become scalar loads hoisted out of the loops.
template <typename T>
__device__ __forceinline__ const T& batch_at(const T* base, uint64_t i) {
  typedef const __attribute__((address_space(4))) T ConstT;
  return *(const T*)((ConstT*)base + i);
}

void launch_batch_fill(const BatchParams& b, hipStream_t s);
void launch_batch_build(const BatchParams& b, hipStream_t s);
// Fused and duplicate-key passes; `shape` is any instance's plan (host copy),
// whose dims select the kernel variant (dims stay in HBM). grid <= 0 sizes
// the persistent grid by occupancy. Returns the first failing HIP status.
hipError_t launch_batch_pipeline(const BatchParams& b, const PipelineParams& shape, int grid,
                                 hipStream_t s);
// The record passes (scan, scatter, aggregation) of the plans with records.
void launch_batch_records(const BatchParams& b, hipStream_t s);
void launch_batch_merge(const BatchParams& b, hipStream_t s);
void launch_batch_finalize(const BatchParams& b, hipStream_t s);

// Set while a batch is being captured into a graph: profiling events are
// then not recorded.
extern thread_local bool g_capturing;

}  // namespace rel
