/* rel.h - C-ABI of the MI355X (gfx950) relational hot path:
 * filter -> hash join (build/probe) -> hash group-by aggregation.
 *
 * The operations follow the operator model of "Rethinking Analytical
 * Processing in the GPU Era" (arXiv 2508.04701):
 *   - operators are stateless calls; the executor owns all state
 *     (Section 3.2.2, push-based execution);
 *   - filter and join produce row ids rather than materialised columns
 *     (late materialisation, Section 3.2.2; row-id type, Section 3.2.3);
 *   - hash tables and other intermediates live in a processing region of
 *     device memory that the caller provides (Section 3.2.3, "Data
 *     Processing"); inputs stay resident in device memory (Section 3.2.3,
 *     "Data Caching"; hot runs, Section 4.1).
 *
 * Conventions shared by every call:
 *   Memory     All column data, row-id arrays, outputs, counts and workspaces
 *              are DEVICE pointers owned by the caller. Descriptor structs
 *              and the arrays of descriptors are HOST memory, read during
 *              the call only. The library never allocates device memory.
 *   Streams    `stream` is a hipStream_t passed as void* (NULL = the default
 *              stream). Calls only enqueue work: they return before the GPU
 *              finishes. Outputs and counts are valid once the stream has
 *              reached that point.
 *   Errors     Arguments are validated on the host before anything is
 *              enqueued; on failure nothing is launched and a status other
 *              than REL_OK is returned, with a message available from
 *              rel_last_error() in the calling thread. REL_EDEVICE reports a
 *              failed launch.
 *   Counts     Result sizes are written to a device int64 (`d_count`,
 *              `d_groups`) and are always the exact size, even when it
 *              exceeds `out_cap`; at most `out_cap` items are written.
 *   Rows       Row counts must be below 2^32 - 1. A row id is the original
 *              position of a row in its table (uint32).
 *   Workspace  `ws` must hold at least the bytes that the matching *_ws()
 *              function returns (REL_ENOMEM otherwise) and be 256-byte
 *              aligned. Calls that may overlap in time need distinct
 *              workspaces; the workspace is scratch and its contents are
 *              undefined after a call.
 *   Columns    Non-nullable fixed-width integers (int8, int32, int64).
 *              Decimals are int64 fixed-point values.
 */
#ifndef REL_H
#define REL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define REL_VERSION 1

typedef enum {
  REL_OK = 0,
  REL_EINVAL = 1,       /* malformed arguments */
  REL_ENOMEM = 2,       /* workspace smaller than required */
  REL_ECAPACITY = 3,    /* an output or table bound was exceeded (reported by the *_sync
                           forms and rel_filter_noalloc) */
  REL_EDEVICE = 4,      /* a HIP runtime call or kernel launch failed */
  REL_EUNSUPPORTED = 5  /* well-formed request outside what this build implements */
} rel_status;

typedef enum { REL_I8 = 1, REL_I32 = 2, REL_I64 = 3,
               REL_F64 = 4 /* binary64: only the order column of rel_topn (AVG outputs) */ } rel_dtype;

typedef uint32_t rel_rowid;

/* A logical column of `len` elements. Without `idx`, element i is data[i]
 * and carries row id i. With `idx` (device array of `len` row ids), element
 * i is data[idx[i]] and carries row id idx[i]: this is how a filter's or a
 * join's row-id output feeds the next operator without materialising
 * columns. */
typedef struct {
  const void* data;
  const rel_rowid* idx;
  int64_t len;
  int32_t type; /* rel_dtype */
  int32_t reserved;
} rel_column;

/* Comparison term; the value v is the element widened to int64 (signed).
 * REL_RANGE holds when lo <= v < hi; every other operator compares v with
 * lo (v < lo, v <= lo, v > lo, v >= lo, v == lo, v != lo). */
typedef enum { REL_LT = 0, REL_LE = 1, REL_GT = 2, REL_GE = 3, REL_EQ = 4, REL_NE = 5, REL_RANGE = 6 } rel_cmp;

typedef struct {
  int32_t col; /* index into the call's column array */
  int32_t op;  /* rel_cmp */
  int64_t lo;
  int64_t hi;
} rel_pred;

/* SUM wraps modulo 2^64; COUNT counts rows; MIN and MAX are signed; AVG is
 * the binary64 quotient (double)SUM / (double)COUNT rounded to nearest even
 * (an ungrouped AVG over no rows is the quiet NaN 0x7FF8000000000000).
 * SUM, COUNT, MIN and MAX are written as int64, AVG as double. */
typedef enum { REL_SUM = 0, REL_COUNT = 1, REL_MIN = 2, REL_MAX = 3, REL_AVG = 4 } rel_agg_op;

typedef struct {
  int32_t op;  /* rel_agg_op */
  int32_t col; /* value column index (ignored for REL_COUNT) */
} rel_agg;

/* Optional tuning; pass NULL (or zero fields) for the defaults. */
typedef struct {
  float load_factor; /* hash-table fill target in (0, 0.9]; 0 = default (0.5) */
  int32_t block;     /* threads per workgroup, a multiple of 64 up to 1024; 0 = default */
  int32_t grid;      /* workgroups of persistent kernels; 0 = default (from the CU count) */
  int32_t lds_slots; /* slots of the per-workgroup LDS group table; 0 = default, -1 = none
                        (partitioned rel_groupby_agg: the first scatter's table) */
  int32_t flags;     /* REL_TUNE_* bits; 0 = none */
  int32_t dim_lds_bytes; /* LDS bytes rel_pipeline may give to dim tables; 0 = default (32 KB),
                            -1 = none */
  int32_t chunk_tiles;   /* rel_pipeline_batch: fact tiles (2048 rows) per work item of the
                            fused pass; 0 = default (from the batch's total size, at most 8) */
  int32_t replicas;      /* copies of the global group table; workgroup w updates copy
                            w mod replicas (w mod 8 is its XCD) and a last pass folds them;
                            0 = default (64 when all groups fit the LDS tables, else 1) */
  int32_t fanout;        /* partitions of the radix-partitioned rel_groupby_agg and
                            rel_hash_join build, a power of two in [4, 16384]; 0 = default
                            (a group-by over at least 1M rows whose groups do not fit the
                            single pass's LDS table, with as many partitions as keep each
                            one's keys within an LDS table; a join whose slot array exceeds
                            64 MB, one partition per 128 KB range of slots); -1 = never.
                            rel_pipeline_batch: partitions of a plan's spilled-row records
                            (see there; -1 = no records) */
} rel_tuning;

/* rel_tuning.flags: keep dims of rel_pipeline in their hash tables even when
 * the build keys are dense (see rel_pipeline). */
#define REL_TUNE_NO_DIRECT 1
/* rel_tuning.flags: rel_hash_join also builds a Bloom filter over the build
 * keys (16 bits per key, in its workspace) and probes it before the hash
 * table, so probe keys without a partner skip the table walk (see
 * rel_bloom_build). */
#define REL_TUNE_BLOOM 2

#define REL_MAX_TERMS 4
#define REL_MAX_DIMS 2
#define REL_MAX_KEYS 2
#define REL_MAX_AGGS 8
#define REL_MAX_FACT_COLS 8

/* ----------------------------------------------------------------- basics */

/* Static text for a status code. */
const char* rel_status_str(rel_status s);

/* Message of the last failed call made by this thread ("" if none). */
const char* rel_last_error(void);

/* REL_VERSION of the built library. */
int rel_version(void);

/* --------------------------------------------------------------- filter */

/* Workspace bytes for rel_filter over n rows. */
size_t rel_filter_ws(int64_t n);

/* Selection (Section 4.2 names filters as the dominant cost of filter-heavy
 * queries; Section 3.2.2 lists predicate pushdown among the custom kernels):
 * writes the row ids of the elements of `cols` that satisfy every term of
 * the conjunction `preds`, in ascending element order.
 *   cols, ncols    1..REL_MAX_FACT_COLS columns of equal len; all share the
 *                  same idx pointer (or all have none).
 *   preds, npreds  1..REL_MAX_TERMS terms over those columns.
 *   out, out_cap   device row-id array; the first min(count, out_cap) ids.
 *   d_count        device int64: the number of passing elements.
 * Errors: REL_EINVAL for mismatched lengths or idx, bad term columns or
 * operators, NULL pointers; REL_ENOMEM for a short workspace. */
rel_status rel_filter(const rel_column* cols, int ncols, const rel_pred* preds, int npreds,
                      rel_rowid* out, int64_t out_cap, int64_t* d_count, void* ws,
                      size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory or size a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): rel_filter with the same arguments, semantics and output,
 * minus the workspace. The tile states live in a static device array that
 * the library holds per GPU (1 MiB, kept until the process ends); the first
 * call on a device looks up its address, later calls allocate nothing
 * (no hipMalloc, no hipFree, no allocating library routine).
 *   n (the columns' len) at most 2,146,959,360 rows.
 * Every call on a GPU shares that GPU's array, and each call clears the part
 * it uses first: calls that may overlap in time on one GPU (other streams,
 * other threads) race and must be serialised by the caller.
 * Errors: as rel_filter (never REL_ENOMEM); REL_ECAPACITY when n exceeds the
 * maximum above (nothing launched); REL_EDEVICE if the array's address
 * cannot be looked up. */
rel_status rel_filter_noalloc(const rel_column* cols, int ncols, const rel_pred* preds,
                              int npreds, rel_rowid* out, int64_t out_cap, int64_t* d_count,
                              void* stream);

/* --------------------------------------------------------- Bloom filters */

/* Bytes of a Bloom filter for n_keys keys at bits_per_key bits each (0: 16,
 * about 0.1% false positives; 4..64), rounded up to a power-of-two number of
 * 32-byte blocks (0 for invalid arguments). */
size_t rel_bloom_bytes(int64_t n_keys, int32_t bits_per_key);

/* Predicate transfer (Section 3.4 plans it among the engine's performance
 * optimizations): a Bloom filter over one table's join keys, built here, is
 * carried to the other table, where rel_bloom_filter drops the rows that
 * cannot find a partner before they reach a join.
 * Builds into `filter` (filter_bytes = 32 * 2^k bytes, 32-byte aligned,
 * device memory; its previous contents are cleared) the blocked Bloom filter
 * of `keys` (any integer type; values compare as int64, so int32 and int64
 * keys of equal value match). Each key sets one bit in each of the eight
 * 32-bit words of one 32-byte block chosen by its hash.
 * Errors: REL_EINVAL for a NULL or malformed column or filter. */
rel_status rel_bloom_build(const rel_column* keys, void* filter, size_t filter_bytes,
                           void* stream);

/* Semi-join reduction: writes the row ids (ascending, like rel_filter) of
 * the probe_keys elements whose value may be in the filter - every element
 * whose value was inserted (no false negatives) and a small share of the
 * others (false positives). Exactly the semi-join is then what a join with
 * the filtered rows returns. ws: rel_filter_ws(probe_keys->len) bytes; other
 * arguments as rel_filter.
 * Errors: REL_EINVAL (malformed column, filter, outputs), REL_ENOMEM. */
rel_status rel_bloom_filter(const rel_column* probe_keys, const void* filter, size_t filter_bytes,
                            rel_rowid* out, int64_t out_cap, int64_t* d_count, void* ws,
                            size_t ws_bytes, void* stream);

/* --------------------------------------------------- late materialisation */

/* Late materialisation (Section 3.2.2: operators pass row ids and a custom
 * kernel materialises columns at the end): out[c][i] = cols[c][ids[i]] for
 * i < n and each of the 1..8 columns, in the column's own type (out[c]:
 * device array of n elements). Columns take no idx. Every id must be below
 * its column's len (the outputs of rel_filter, rel_hash_join and rel_topn
 * are); other ids read outside the column.
 * Errors: REL_EINVAL (NULL arguments, bad column or count). */
rel_status rel_gather(const rel_column* cols, int ncols, const rel_rowid* ids, int64_t n,
                      void* const* out, void* stream);

/* Workspace bytes for rel_topn over n rows with limit N (0 for invalid
 * arguments). */
size_t rel_topn_ws(int64_t n, int64_t limit);

/* Order-by / top-N over a result table (Section 4.2 names it among
 * ClickBench's costs beside scans and aggregation): writes to out the
 * positions (row ids) of the first min(limit, n) of its n rows in the order
 * of `order` - ascending, or descending when desc != 0 - ties broken by the
 * key tuple ascending (signed, lexicographic) and then by the row position,
 * so the answer is unique; *d_count (device int64) = min(limit, n).
 *   order      device array of n values: REL_I64 (int64) or REL_F64
 *              (binary64, e.g. an AVG column; no NaN), 8-byte aligned.
 *   keys       0..2 key columns (len >= n, no idx): the tie-break.
 *   limit      0..1024.
 *   ws         rel_topn_ws(n, limit) bytes.
 * Feed the positions to rel_gather to materialise the rows.
 * Errors: REL_EINVAL, REL_ENOMEM, REL_EDEVICE (launch). */
rel_status rel_topn(const void* order, int32_t order_type, int32_t desc, const rel_column* keys,
                    int nkeys, int64_t n, int64_t limit, rel_rowid* out, int64_t* d_count,
                    void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ hash join */

/* Workspace bytes for rel_hash_join with n_build build rows (with a
 * partitioned build, see rel_tuning.fanout, two buffers of 16-byte records
 * per build row on top of the slot array). */
size_t rel_hash_join_ws(int32_t key_type, int64_t n_build, const rel_tuning* t);

/* Inner equi-join (the hash join of Sections 1 and 4.2): builds an
 * open-addressing hash table over build_keys in the workspace (large build
 * sides range by range in LDS, see rel_tuning.fanout), then probes it
 * with probe_keys and writes every matching pair (build row id, probe row
 * id). Duplicate keys on either side yield every pair. Pair order is
 * unspecified (compare after sorting by (probe, build)).
 *   build_keys, probe_keys  int32 or int64 columns of the same type.
 *   out_build, out_probe    device row-id arrays of out_cap entries.
 *   d_count                 device int64: the exact number of pairs.
 * Errors: REL_EINVAL for NULL or mismatched types; REL_ENOMEM for a short
 * workspace. */
rel_status rel_hash_join(const rel_column* build_keys, const rel_column* probe_keys,
                         rel_rowid* out_build, rel_rowid* out_probe, int64_t out_cap,
                         int64_t* d_count, const rel_tuning* t, void* ws, size_t ws_bytes,
                         void* stream);

/* ------------------------------------------------------------- group-by */

/* Workspace bytes for rel_groupby_agg over at most n_rows rows with at most
 * max_groups groups (0 for invalid arguments). With partitioning (see
 * rel_tuning.fanout) it includes two buffers of n_rows records, each the key
 * tuple and one int64 per distinct value column that an aggregate reads. */
size_t rel_groupby_ws(int nkeys, const int32_t* key_types, int naggs, const rel_agg* aggs,
                      int64_t n_rows, int64_t max_groups, const rel_tuning* t);

/* Hash group-by aggregation (Section 4.2: hash-based grouping, with memory
 * contention when there are few groups; many groups are radix-partitioned
 * first, see rel_tuning.fanout): one output row per distinct key
 * tuple of `keys` (0..REL_MAX_KEYS columns; with none, exactly one row, even
 * over no input rows), with the aggregates `aggs` over the value columns
 * `vals`. Row order is unspecified (compare after sorting by key tuple).
 *   keys, vals     columns of equal len (idx allowed). Key tuples must pack
 *                  into 64 bits (int8 = 8, int32 = 32, int64 = 64 bits).
 *   out_keys[k]    device array of out_cap elements of key k's own type.
 *   out_aggs[a]    device array of out_cap int64 (AVG: double).
 *   d_groups       device int64: the number of groups, or -1 when the input
 *                  holds more distinct groups than the table sized for
 *                  max_groups can take (outputs are then undefined).
 * Errors: REL_EINVAL, REL_ENOMEM, REL_EUNSUPPORTED (key tuple wider than
 * 64 bits). */
rel_status rel_groupby_agg(const rel_column* keys, int nkeys, const rel_column* vals, int nvals,
                           const rel_agg* aggs, int naggs, void* const* out_keys,
                           void* const* out_aggs, int64_t out_cap, int64_t* d_groups,
                           int64_t max_groups, const rel_tuning* t, void* ws, size_t ws_bytes,
                           void* stream);

/* A string column in the Arrow layout: string j is bytes[offsets[j] ..
 * offsets[j+1]) (n_strings + 1 ascending offsets). Without codes, row i is
 * string i (len == n_strings); with codes (device int32 array of len
 * entries, each in [0, n_strings)) the column is dictionary-encoded and row
 * i is string codes[i]. All arrays are device memory; the bytes are read in
 * aligned 4-byte words (a word holding a string byte is read whole). */
typedef struct {
  const int64_t* offsets;
  const uint8_t* bytes;
  const int32_t* codes;
  int64_t len;
  int64_t n_strings;
} rel_strings;

/* Workspace bytes for rel_groupby_str with at most max_groups groups over a
 * column whose dictionary holds n_dict strings (0 without codes; with codes,
 * n_dict = the column's n_strings); 0 for invalid arguments. */
size_t rel_groupby_str_ws(int64_t max_groups, int64_t n_dict, int naggs, const rel_agg* aggs);

/* Hash group-by on a string key (Section 4.2 reports the cost of string
 * group keys on ClickBench), optionally with an integer key beside it (a
 * two-column key): one output row per distinct (string, integer) pair - the
 * string's bytes decide, so equal strings under different dictionary codes
 * form one group - with the aggregates `aggs` over `vals` as in
 * rel_groupby_agg. Instead of the string, a group reports the smallest row
 * id holding it (out_rows; feed it to the codes or offsets to read the
 * string, or to rel_gather), and its integer key (out_ikey, ikey's type).
 * Row order is unspecified (compare after sorting by the key).
 *   ikey      NULL or an int8/int32/int64 column of key->len rows (no idx).
 *   vals      value columns of key->len rows (no idx).
 *   d_groups  device int64: the number of groups, or -1 when they exceed
 *             what a table sized for max_groups holds.
 * Equal rows of a wave combine their updates before one atomic per group
 * (wave-aggregated atomics).
 * Errors: REL_EINVAL, REL_ENOMEM. */
rel_status rel_groupby_str(const rel_strings* key, const rel_column* ikey, const rel_column* vals,
                           int nvals, const rel_agg* aggs, int naggs, rel_rowid* out_rows,
                           void* out_ikey, void* const* out_aggs, int64_t out_cap,
                           int64_t* d_groups, int64_t max_groups, void* ws, size_t ws_bytes,
                           void* stream);

/* ------------------------------------------------------------- pipeline */

/* One dimension join of the fused plan: fact column `fact_col` is a foreign
 * key into `key`; if `has_payload`, `payload` (int8 or int32, same len as
 * `key`) is a dim attribute that a group key may use. Dim columns take no
 * idx. */
typedef struct {
  int32_t fact_col;
  int32_t has_payload;
  rel_column key;
  rel_column payload;
} rel_dim;

typedef enum { REL_KEY_FACT = 0, REL_KEY_DIM = 1 } rel_key_src;

/* A group key: fact column `col` (REL_KEY_FACT) or the payload of dim `col`
 * (REL_KEY_DIM). */
typedef struct {
  int32_t src;
  int32_t col;
} rel_key_ref;

/* Fixed-shape plan: conjunctive filter on fact columns -> inner join with up
 * to two dims -> group-by. Fact columns are plain (no idx). */
typedef struct {
  const rel_column* fact;
  int32_t n_fact; /* 1..REL_MAX_FACT_COLS */
  const rel_pred* preds;
  int32_t n_preds; /* 0..REL_MAX_TERMS, over fact columns */
  const rel_dim* dims;
  int32_t n_dims; /* 0..REL_MAX_DIMS */
  const rel_key_ref* keys;
  int32_t n_keys; /* 0..REL_MAX_KEYS */
  const rel_agg* aggs;
  int32_t n_aggs; /* 1..REL_MAX_AGGS, over fact columns */
  int64_t max_groups;
  const rel_tuning* tuning; /* NULL = defaults */
} rel_pipeline_desc;

/* Group outputs: keys[k] has the type of its source column; aggs[a] is
 * int64 (AVG: double); cap entries each; d_groups as in rel_groupby_agg. */
typedef struct {
  void* keys[REL_MAX_KEYS];
  void* aggs[REL_MAX_AGGS];
  int64_t cap;
  int64_t* d_groups;
} rel_outputs;

/* Workspace bytes for rel_pipeline on plan d. */
size_t rel_pipeline_ws(const rel_pipeline_desc* d);

/* The whole plan on the GPU, from scan to result (Section 3.1): builds the
 * dim hash tables, then one fused pass over the fact table evaluates the
 * predicate, probes the dims and aggregates; a last pass writes the groups.
 * Per fact row passing the predicate, each combination of matching dim rows
 * contributes once (inner-join semantics; no match drops the row).
 * Errors: REL_EINVAL, REL_ENOMEM, REL_EUNSUPPORTED (key tuple wider than
 * 64 bits, int64 dim payloads). */
rel_status rel_pipeline(const rel_pipeline_desc* d, const rel_outputs* o, void* ws,
                        size_t ws_bytes, void* stream);

/* ----------------------------------------------------------- out of core */

/* Workspace bytes for rel_pipeline_stream on plan d with chunks of
 * chunk_rows fact rows (0 for invalid arguments): rel_pipeline_ws(d) plus two
 * staging slots of one chunk of every fact column. */
size_t rel_pipeline_stream_ws(const rel_pipeline_desc* d, int64_t chunk_rows);

/* Out-of-core execution (Section 3.4 plans it for data larger than device
 * memory): rel_pipeline over fact columns that stay in host memory. The fact
 * table goes through the device in chunks of chunk_rows rows: while the
 * fused pass runs over chunk k on `stream`, chunk k+1 is copied into the
 * other staging slot on a copy stream of the calling thread (created on
 * first use, default priority, kept until the process ends); every chunk
 * aggregates into the same group table, and the groups are written once at
 * the end. Results equal rel_pipeline on the whole table.
 *   d           as for rel_pipeline, except that the fact columns' data are
 *               HOST pointers, best pinned (hipHostMalloc) so that the
 *               copies run asynchronously at full speed; dims stay device
 *               memory. The host buffers must stay valid until `stream`
 *               has reached the end of the call.
 *   chunk_rows  a positive multiple of 2048.
 *   ws          rel_pipeline_stream_ws(d, chunk_rows) bytes.
 * Errors: as rel_pipeline; REL_EDEVICE if a copy or event call fails. */
rel_status rel_pipeline_stream(const rel_pipeline_desc* d, int64_t chunk_rows,
                               const rel_outputs* o, void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------- batches */

/* Workspace bytes for rel_pipeline_batch over the n plans d[0..n-1]
 * (0 if the plans are invalid or differ in shape). */
size_t rel_pipeline_batch_ws(const rel_pipeline_desc* d, int n);

/* Batch execution (Section 5 names it as future work for the many small
 * queries that leave a GPU underused): n independent plans, each with the
 * semantics of rel_pipeline and its own inputs and outputs o[i], run with
 * one launch per phase rather than n sequences of launches. Every phase
 * splits each plan into work items (build rows, runs of 2048-row fact tiles,
 * group slots); the fused pass is a persistent kernel whose workgroups take
 * the items of all plans in order from a device counter, so that one large
 * plan is spread over the chip and many small ones share it. Results are
 * identical to n rel_pipeline calls.
 * Spilled rows (hash grouping, Section 4.2): a grouped plan whose groups do
 * not fit the fused pass's LDS table at half load (or would need a table
 * over 64 KB), whose aggregates read at most two value columns and whose
 * fact table has at most 2^31 rows writes each row that finds no LDS slot
 * as a record of 12 to 24 bytes rather than updating the global table with
 * device-scope atomics; the records are grouped by partition of the key
 * hash and folded, partition by partition, in LDS, then merged into the
 * global table once per key. Such a plan runs its fused pass without an
 * LDS table (unless tuning.lds_slots sets one) and with one global table.
 * tuning.fanout: -1 keeps the atomics; 0 sizes the partitions for the
 * aggregation pass's LDS table (at most 1024 partitions: plans needing more
 * keep the atomics); a power of two sets the partition count (clamped to
 * 1024). Record regions take 2 x (rows x record bytes) of ws per plan, in
 * plan order while the batch's records fit 64 GiB; later plans keep the
 * atomics.
 *   d, n     1..65536 plans of one shape: the same number of dims, and for
 *            each dim the same key type and payload presence. Per-plan
 *            tuning (load factor, LDS group slots, replicas, fanout) is
 *            honoured; grid and chunk_tiles come from d[0].tuning. Dim
 *            tables are always read from HBM (no LDS copies, no compact
 *            sets).
 *   o        n outputs, as for rel_pipeline.
 *   ws       rel_pipeline_batch_ws(d, n) bytes.
 * The call builds the plans' kernel parameters and work lists on the host
 * and uploads them in one stream-ordered copy from a pinned staging buffer
 * that the library keeps per calling thread (host memory, allocated on
 * first use and grown as needed, never freed before the process ends).
 * Errors: as rel_pipeline, naming the failing plan; REL_EINVAL when plans
 * differ in shape. */
rel_status rel_pipeline_batch(const rel_pipeline_desc* d, int n, const rel_outputs* o, void* ws,
                              size_t ws_bytes, void* stream);

/* A batch captured once as a HIP graph (descriptor upload from pinned host
 * memory owned by the graph, then the batch's launches), for replay with one
 * hipGraphLaunch. Inputs, outputs and ws are bound at capture: they must
 * stay allocated, and their contents at each launch are the inputs. */
typedef struct rel_graph rel_graph;

/* Captures rel_pipeline_batch(d, n, o, ws, ws_bytes) into *out. Nothing is
 * executed. Errors: as rel_pipeline_batch; REL_EDEVICE if capture or
 * instantiation fails (nothing is then kept). */
rel_status rel_pipeline_batch_graph(const rel_pipeline_desc* d, int n, const rel_outputs* o,
                                    void* ws, size_t ws_bytes, rel_graph** out);

/* Enqueues one replay of g on `stream`. Replays that may overlap in time
 * race on the bound workspace and outputs. */
rel_status rel_graph_launch(rel_graph* g, void* stream);

/* Releases g (NULL is ignored); the caller makes sure no replay is still
 * running. */
void rel_graph_destroy(rel_graph* g);

/* Autotuner (batch execution, Section 5; the load factor, fan-out and block
 * shape of each batch instance per size bucket): for each sample plan, runs
 * every candidate tuning record as a one-plan rel_pipeline_batch on the
 * current device - the group-table load factor, the fan-out of an instance
 * over the persistent workgroups (chunk_tiles), the block shape (resident
 * workgroups per CU: grid, or the LDS group table's size, lds_slots) and the
 * global group-table copies (replicas) - checks that every candidate returns
 * the same groups (a difference is a race), and stores the fastest under the
 * key "<gfx arch>/pipeline_batch/f<F>-d<D>-g<G>" of a JSON object in the
 * file at cache_path (created if missing; other records are kept). F, D and
 * G are the even exponents at or below the ceiling log2 of the fact rows,
 * the largest dim and max_groups (buckets of 4x). Each record holds the
 * chosen fields ("tuning"), its time ("ms") and every candidate's time.
 * Samples of one bucket overwrite each other's record: pass one (a
 * representative plan, for instance the median instance) per bucket.
 * Unlike the operators, this offline call allocates and frees its own device
 * memory (workspace and outputs of the sample runs) and synchronises.
 * Errors: REL_EINVAL (invalid sample plan, unreadable or unwritable cache),
 * REL_ECAPACITY (a sample with more groups than its max_groups),
 * REL_EDEVICE (a failed run, or a candidate whose result differs). */
rel_status rel_autotune(const rel_pipeline_desc* samples, int n, const char* cache_path);

/* The record that rel_autotune stored for plan d's bucket on the current
 * device's architecture: *out receives its fields (others zero, i.e. the
 * defaults) and *found 1; with no record *found is 0 and *out all zero.
 * Only host work. Errors: REL_EINVAL (NULL arguments, unreadable cache,
 * unknown fields). */
rel_status rel_autotune_lookup(const char* cache_path, const rel_pipeline_desc* d,
                               rel_tuning* out, int* found);

/* -------------------------------------------------------------- serving */

/* A query server over resident tables (the pipeline tasks of Section 3.2.2
 * drawn from a global queue; hot data kept in device memory, Section 4.1):
 * queries are submitted as fused plans over device columns that stay
 * allocated, wait in a FIFO, and are admitted as lanes, query slots and
 * workspace bytes free up. Whenever a lane is free, a scheduler thread packs
 * the oldest waiting queries of one shape (as in rel_pipeline_batch) and one
 * max_groups class (up to 4096, up to 65536, more) into a batch, takes its
 * workspace from the arena (first fit) and launches it, so
 * that queries arriving while others run are batched and overlap them on the
 * device. A query completes once its batch has finished and its results are
 * in the host buffers given at submission; then its slot, lane and bytes are
 * released. Each query's results are those of rel_pipeline on its plan. */
typedef struct rel_server rel_server;

/* Runs batches for a server; NULL in the config selects the GPU executor
 * (rel_pipeline_batch on one HIP stream per lane, completion by event
 * polling, then copies of the result rows to the host buffers). A custom
 * executor lets the scheduler run anywhere (tests drive it with one that
 * computes on the host). All four are called from the scheduler thread,
 * batch_ws also from rel_server_submit.
 *   batch_ws  workspace bytes for plans d[0..n-1] (0: invalid plans).
 *   launch    starts the batch on `lane` (idle), with n plans, their device
 *             outputs o and host outputs host (entries with NULL d_groups
 *             take no copy); returns REL_OK or a failure of the batch.
 *   poll      1 once the lane's batch and its copies are done, 0 while they
 *             run, -status on failure.
 *   quiesce   after a failed launch or poll, before the batch's workspace
 *             goes back to the arena: returns once nothing the lane enqueued
 *             can still touch it (the GPU executor synchronises the lane's
 *             stream: a launch can fail after enqueueing some of its
 *             kernels). May be NULL. */
typedef struct {
  void* user;
  size_t (*batch_ws)(void* user, const rel_pipeline_desc* d, int n);
  rel_status (*launch)(void* user, int lane, const rel_pipeline_desc* d, int n,
                       const rel_outputs* o, const rel_outputs* host, void* ws, size_t ws_bytes);
  int (*poll)(void* user, int lane);
  void (*quiesce)(void* user, int lane);
} rel_executor;

typedef struct {
  void* arena;           /* device memory for batch workspaces, 256-byte aligned: the budget
                            for hash tables and per-batch state */
  size_t arena_bytes;
  int32_t max_slots;     /* queries in flight at once */
  int32_t max_batch;     /* queries per batch (1: one at a time) */
  int32_t lanes;         /* batches in flight at once, 1..64 */
  int32_t open_lane_at;  /* while a lane is busy, another starts a batch only when at least
                            this many queries wait (0 or 1: whenever one waits). A backlog
                            threshold keeps light load on one lane, whose next batch
                            gathers the waiting queries */
  const rel_executor* executor; /* NULL: the GPU executor on the current device */
} rel_server_config;

/* A completed query: status (REL_OK or the failure of its batch), the size
 * of its batch, and times on the rel_server_now_ns() clock. */
typedef struct {
  uint64_t ticket;
  int32_t status;
  int32_t batch_size;
  int64_t t_submit_ns;
  int64_t t_launch_ns;
  int64_t t_done_ns;
} rel_completion;

typedef struct {
  int64_t submitted, completed, failed, rejected, batches, batched_queries;
} rel_server_counts;

/* Starts a server (and its scheduler thread). The environment variable
 * REL_FAULT=launch:N makes the N-th batch launch fail with REL_EDEVICE
 * without running (failure handling tests): its queries fail, the server
 * goes on. Errors: REL_EINVAL (bad config), REL_EDEVICE (streams, events or
 * pinned memory of the GPU executor). */
rel_status rel_server_create(const rel_server_config* c, rel_server** out);

/* Queues plan d (copied; its columns stay caller-owned and allocated until
 * the query completes) with device outputs o and optional host outputs
 * `host` (pinned host memory, same layout; NULL: results stay on the
 * device). Returns the query's ticket. Errors: REL_EINVAL (invalid plan,
 * server stopping), REL_ENOMEM (the query alone needs more workspace than the
 * whole arena: rejected, others go on). */
rel_status rel_server_submit(rel_server* s, const rel_pipeline_desc* d, const rel_outputs* o,
                             const rel_outputs* host, uint64_t* ticket);

/* Moves up to max completions (in completion order) into out; returns the
 * count. */
int rel_server_poll(rel_server* s, rel_completion* out, int max);

/* Waits until every submitted query has completed; REL_ECAPACITY if
 * timeout_ms passes first. */
rel_status rel_server_drain(rel_server* s, int64_t timeout_ms);

/* Counters, the 50th and 99th percentile (nearest rank) of submit-to-done
 * latency over the successful queries so far (-1 if none), and their
 * throughput: the fact rows they scanned divided by the time from the first
 * one's submission to the last one's completion (0 if none). Any output
 * pointer may be NULL. */
rel_status rel_server_stats(rel_server* s, rel_server_counts* counts, int64_t* p50_ns,
                            int64_t* p99_ns, double* rows_per_s);

/* The server clock: a steady clock in nanoseconds. */
int64_t rel_server_now_ns(void);

/* Completes every queued query, stops the scheduler and frees the server. */
void rel_server_destroy(rel_server* s);

/* ---------------------------------------------------- synchronous forms */

/* Each *_sync call makes the asynchronous call of the same name, waits for
 * `stream`, and reads the exact result size (the value of d_count, d_groups
 * or o->d_groups) into the host int64 *count / *groups (may be NULL). It
 * returns REL_ECAPACITY when that size exceeds the output capacity (out_cap,
 * o->cap: the first out_cap items were written, the caller grows its output
 * and calls again) or, for group counts, is -1 (more distinct groups than
 * max_groups: outputs undefined); otherwise the status of the call, or
 * REL_EDEVICE if the copy or the wait fails. Nothing is read back when the
 * call itself fails. */
rel_status rel_filter_sync(const rel_column* cols, int ncols, const rel_pred* preds, int npreds,
                           rel_rowid* out, int64_t out_cap, int64_t* d_count, void* ws,
                           size_t ws_bytes, void* stream, int64_t* count);
rel_status rel_hash_join_sync(const rel_column* build_keys, const rel_column* probe_keys,
                              rel_rowid* out_build, rel_rowid* out_probe, int64_t out_cap,
                              int64_t* d_count, const rel_tuning* t, void* ws, size_t ws_bytes,
                              void* stream, int64_t* count);
rel_status rel_groupby_agg_sync(const rel_column* keys, int nkeys, const rel_column* vals,
                                int nvals, const rel_agg* aggs, int naggs, void* const* out_keys,
                                void* const* out_aggs, int64_t out_cap, int64_t* d_groups,
                                int64_t max_groups, const rel_tuning* t, void* ws,
                                size_t ws_bytes, void* stream, int64_t* groups);
rel_status rel_pipeline_sync(const rel_pipeline_desc* d, const rel_outputs* o, void* ws,
                             size_t ws_bytes, void* stream, int64_t* groups);

/* ---------------------------------------------------------- stream read */

/* The streaming-read ceiling that scan-bound operators are measured against
 * beside the HBM specification (the paper's measurements run on data resident
 * in device memory, Section 4.1 "hot runs"; Section 4.2 breaks query time
 * down by operator): reads each of the `bytes` bytes at `data` exactly once
 * with coalesced 16-byte non-temporal loads and writes to *d_xor the XOR of
 * all 64-bit little-endian words of the buffer (a last partial word
 * zero-padded), so that the reads cannot be elided and the result can be
 * checked on a host.
 *   data     device memory, 16-byte aligned (any size, 0 allowed).
 *   d_xor    device uint64, overwritten (stream-ordered).
 * Errors: REL_EINVAL for NULL or misaligned pointers or a negative size;
 * REL_EDEVICE for a failed launch. */
rel_status rel_stream_read(const void* data, int64_t bytes, uint64_t* d_xor, void* stream);

/* ------------------------------------------------------------- profiling */

/* Kernel classes timed by the per-kernel profiler (the per-operator time
 * breakdown of Section 4.2, "Performance Breakdown"). */
typedef enum {
  REL_K_FILL = 0,        /* workspace initialisation (tables, counters) */
  REL_K_FILTER = 1,      /* rel_filter's compaction kernel */
  REL_K_MAP_BUILD = 2,   /* hash-table build (join build side, dims) */
  REL_K_MAP_PROBE = 3,   /* join probe with pair output */
  REL_K_GROUP_AGG = 4,   /* rel_groupby_agg's aggregation kernel */
  REL_K_PIPELINE = 5,    /* rel_pipeline's fused filter-probe-aggregate kernel */
  REL_K_FINALIZE = 6,    /* group compaction into the outputs */
  REL_K_GROUP_PARTITION = 7, /* rel_groupby_agg's counting and scatter passes */
  REL_K_STREAM = 8,      /* rel_stream_read */
  REL_K_BLOOM = 9,       /* Bloom filter builds (rel_bloom_build, joins with REL_TUNE_BLOOM) */
  REL_K_GATHER = 10,     /* rel_gather */
  REL_K_TOPN = 11,       /* rel_topn */
  REL_K_COUNT = 12
} rel_kernel_class;

/* Static name of a kernel class. */
const char* rel_kernel_name(int k);

/* Turns per-kernel timing on (1) or off (0) for calls made afterwards from
 * any thread. While on, every kernel launch is bracketed by two HIP events
 * recorded on the caller's stream. */
void rel_profile_enable(int on);

/* Waits for the recorded events, then writes, for each kernel class k <
 * REL_K_COUNT (host arrays of REL_K_COUNT entries), the summed device time
 * in milliseconds and the number of launches since the last read, and
 * clears them. Returns REL_EDEVICE if an event query fails. */
rel_status rel_profile_read(double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* REL_H */
