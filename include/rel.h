/*
 * rel.h -- C ABI of librel, an MI355X (gfx950) library for the relational hot
 * path the paper profiles: a selection predicate, a primary-key/foreign-key
 * hash join and a hash group-by aggregation over columnar, device-resident
 * tables (the cuDF filter, join build/count/retrieve and shared-memory
 * group-by kernels of Section 7 and Table 9).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Columns are plain device arrays, one per column (the Arrow-compatible
 *   columnar layout of Section 2.3), non-nullable. Column pointers must be
 *   16-byte aligned (a fresh torch/hipMalloc allocation always is); a
 *   misaligned column is rejected with REL_INVALID_ARG.
 * - All column and output buffers are owned by the caller; librel never frees
 *   them. librel owns contexts, join tables, batches and planners and frees
 *   them in the matching *_destroy call. A context keeps its scratch device
 *   memory (hash tables, counters) between calls and frees it on destroy.
 * - Every call is stream-ordered on the context's HIP stream (borrowed, e.g.
 *   torch.cuda.current_stream().cuda_stream) and returns once the work is
 *   enqueued, unless it says it synchronises. Counts are written to device
 *   int64 words. Calls on one context must come from one host thread at a
 *   time, and work enqueued on one context must not overlap in time with
 *   other work that uses the same context's scratch memory.
 * - Errors: the return value. Argument errors are found on the host before
 *   any work is enqueued; out-parameters are written only on REL_OK.
 *   Conditions found on the device (a full table, a duplicate build key) set
 *   sticky bits in the context's device status word; rel_ctx_sync returns and
 *   clears them. A synchronising rel_filter_join_agg call and a batch report
 *   through status words of their own (cleared when they start), so they
 *   neither consume nor are charged with bits that earlier calls left.
 * - Integer sums and counts are 64-bit and wrap modulo 2^64, so results do not
 *   depend on the order in which atomic updates land.
 */
#ifndef REL_H_
#define REL_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rel_status {
  REL_OK = 0,
  REL_INVALID_ARG = 1,   /* null pointer, negative size, misaligned column, bad enum */
  REL_CAPACITY = 2,      /* an output buffer is smaller than a bound the host can prove */
  REL_DUPLICATE_KEY = 3, /* a build key occurs twice (reported by synchronising calls) */
  REL_HIP = 4,           /* HIP runtime error; rel_last_error has the message */
  REL_OOM = 5,           /* device allocation failed */
  REL_UNSUPPORTED = 6,   /* valid request this library does not implement */
  REL_OVERFLOW = 7       /* a table sized from a plan overflowed and no fallback was allowed */
} rel_status;

/* Device status bits (rel_ctx_sync). */
#define REL_DEV_OVERFLOW 0x1u  /* a hash table or output ran out of room; results incomplete */
#define REL_DEV_DUPKEY 0x2u    /* a join build met an equal key twice */
#define REL_DEV_BADARG 0x4u    /* a device-side argument check failed (e.g. negative payload) */

typedef struct rel_ctx rel_ctx;

/* Create a context on HIP device `device` whose work goes to `hip_stream`
 * (a hipStream_t, borrowed; NULL means the null stream). */
rel_status rel_ctx_create(int device, void* hip_stream, rel_ctx** out);
rel_status rel_ctx_destroy(rel_ctx* ctx);
/* Point the context at another borrowed stream. */
rel_status rel_ctx_set_stream(rel_ctx* ctx, void* hip_stream);
/* Synchronise the stream, then return and clear the device status bits
 * (status_bits nullable). */
rel_status rel_ctx_sync(rel_ctx* ctx, uint32_t* status_bits);
const char* rel_status_string(rel_status s);
/* Message of the last failing call on this context (empty if none). */
const char* rel_last_error(const rel_ctx* ctx);

/* Per-kernel timing (the measurement side of the paper's method: kernel time
 * is the unit of analysis, Section 3.2). When enabled, every kernel librel
 * launches on this context is bracketed by HIP events on the context's
 * stream. Enabling (or disabling) synchronises and clears past records. */
rel_status rel_ctx_enable_timing(rel_ctx* ctx, int enable);
/* Synchronise, resolve the recorded events and report up to `max` kernels:
 * names[i] (owned by the context, valid until timing is enabled again),
 * total_ms[i] summed over launches[i] launches. *count = kernels recorded. */
rel_status rel_ctx_kernel_times(rel_ctx* ctx, const char** names, double* total_ms, int64_t* launches, int max,
                                int* count);

/* ------------------------------------------------------------------------------------------------------------------
 * Selection (the filter step: cuDF's compute_column_kernel + DeviceScanKernel
 * pair of Table 9, whose interpreted expression evaluation Section 7 singles
 * out; here the comparison is compiled, not interpreted).
 */
typedef enum rel_cmp { REL_LT = 0, REL_LE = 1, REL_GT = 2, REL_GE = 3, REL_EQ = 4, REL_NE = 5 } rel_cmp;

/* out_idx[0..count) = the row ids i in [0, n) with col[i] <op> literal, in
 * ascending order (a stable selection vector); *d_out_count (device) = count.
 * col: int32[n]; out_idx: int32[out_cap], out_cap >= n (else REL_CAPACITY);
 * n < 2^31. */
rel_status rel_filter_compact(rel_ctx* ctx, const int32_t* col, int64_t n, rel_cmp op, int32_t literal,
                              int32_t* out_idx, int64_t out_cap, int64_t* d_out_count);

/* rel_filter_compact without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, result and errors as rel_filter_compact,
 * plus REL_UNSUPPORTED for n > 2^30 rows. Its scratch (the ticket and the
 * look-back tile states, at most 1 MiB) is a fixed device array that each GPU
 * holds until the process ends; its address is looked up by rel_ctx_create.
 * It enqueues two fill kernels and the compaction kernel on the context's
 * stream and calls no allocating routine. Every call on one GPU shares that
 * array: calls whose work overlaps in time on one GPU (two streams, two
 * contexts, two threads) race and give wrong results. */
rel_status rel_filter_compact_noalloc(rel_ctx* ctx, const int32_t* col, int64_t n, rel_cmp op, int32_t literal,
                                      int32_t* out_idx, int64_t out_cap, int64_t* d_out_count);

/* ------------------------------------------------------------------------------------------------------------------
 * General selection predicates (the compute-column step widened): a
 * conjunction of up to 8 terms over typed columns. Section 7 finds cuDF's
 * expression interpreter (compute_column_kernel) spending so many
 * instructions that a kernel with sequential accesses turns instruction-bound
 * on the high-bandwidth GPU. Here a predicate is either compiled, as a kernel
 * generated for it and built at run time with hipRTC (literals and column
 * types fixed in the code, each column read with 16-byte loads), or
 * interpreted by one fixed kernel that walks the term list for every row. Both
 * produce the stable selection vector of rel_filter_compact.
 */
typedef enum rel_dtype {
  REL_DT_I8 = 0, REL_DT_I16 = 1, REL_DT_I32 = 2, REL_DT_I64 = 3, REL_DT_F32 = 4, REL_DT_F64 = 5
} rel_dtype;
typedef enum rel_pred_op {
  REL_OP_LT = 0, REL_OP_LE = 1, REL_OP_GT = 2, REL_OP_GE = 3, REL_OP_EQ = 4, REL_OP_NE = 5,
  REL_OP_BETWEEN = 6, /* lo <= x <= hi */
  REL_OP_IN = 7       /* x equals one of the values */
} rel_pred_op;
typedef enum rel_pred_mode { REL_PRED_COMPILED = 0, REL_PRED_INTERPRETED = 1 } rel_pred_mode;
#define REL_PRED_MAX_TERMS 8
#define REL_PRED_MAX_VALUES 16

typedef struct rel_pred_term {
  int32_t column;   /* index into the columns array given to rel_pred_filter */
  int32_t dtype;    /* rel_dtype of that column */
  int32_t op;       /* rel_pred_op */
  int32_t n_values; /* 1 for the comparisons, 2 for BETWEEN (lo, hi), 1..16 for IN */
  int64_t ivalues[REL_PRED_MAX_VALUES]; /* literals for integer columns (the value is compared as int64) */
  double fvalues[REL_PRED_MAX_VALUES];  /* literals for f32/f64 columns (compared as double; NaN fails every op but NE) */
} rel_pred_term;

typedef struct rel_pred rel_pred;

/* Validate the terms and prepare the predicate: mode COMPILED generates and
 * compiles a kernel for it (a few hundred milliseconds; the device's own
 * architecture), INTERPRETED prepares the interpreter. The predicate is owned
 * by the caller through *out. Errors: REL_INVALID_ARG (no terms or more than
 * 8, bad column index, dtype, op or value count), REL_HIP (compilation or
 * module load failed; rel_last_error has the compiler log). */
rel_status rel_pred_create(rel_ctx* ctx, const rel_pred_term* terms, int32_t n_terms, int32_t mode, rel_pred** out);
/* Stable ascending indices of the rows i in [0, n) for which every term holds:
 * columns is a host array of n_columns device pointers (each 16-byte aligned,
 * at least n elements of its term's dtype; columns no term uses may be NULL).
 * *d_out_count (device) = number selected; out_cap >= n (else REL_CAPACITY). */
rel_status rel_pred_filter(rel_pred* pred, const void* const* columns, int32_t n_columns, int64_t n, int32_t* out_idx,
                           int64_t out_cap, int64_t* d_out_count);
rel_status rel_pred_destroy(rel_pred* pred);

/* ------------------------------------------------------------------------------------------------------------------
 * Hash join (cuDF's insert_if_n build and count/retrieve probe kernels of
 * Section 7). Open addressing with linear probing over a power-of-two table of
 * packed 64-bit slots {key, payload}.
 */
typedef enum rel_placement {
  REL_PLACE_AUTO = 0,        /* library decides from sizes */
  REL_PLACE_LDS = 1,         /* per-workgroup table in LDS (small tables only) */
  REL_PLACE_GLOBAL = 2,      /* one table in device memory updated with device-scope atomics */
  REL_PLACE_PARTITIONED = 3  /* radix-partitioned: per-partition tables in LDS */
} rel_placement;

typedef struct rel_table_opts {
  int64_t capacity_hint; /* slots or expected distinct keys; 0 = size from the input (plain sizing) */
  int32_t placement;     /* rel_placement */
  float max_load;        /* target load factor in (0, 0.9]; 0 = 0.5 */
} rel_table_opts;

typedef struct rel_join_table rel_join_table;

/* Build a join table over dim keys pk[0..m) with payload[j] (any int32) or,
 * when payload is NULL, the dim row id j. A repeated key sets REL_DEV_DUPKEY.
 * opts nullable (plain sizing: capacity = next power of two >= 2m). The table
 * is owned by the caller through *out and must outlive probes that use it. */
rel_status rel_join_build(rel_ctx* ctx, const int32_t* pk, const int32_t* payload, int64_t m,
                          const rel_table_opts* opts, rel_join_table** out);
rel_status rel_join_table_destroy(rel_join_table* table);

/* Probe: for each position k in [0, n) with row = sel ? sel[k] : k, if
 * fk[row] matches a build key, emit (row, payload). Pairs come out in no
 * particular order; *d_out_count (device) = number of pairs (<= n, since pk is
 * unique). out_cap >= n (else REL_CAPACITY). */
rel_status rel_join_probe(rel_ctx* ctx, const rel_join_table* table, const int32_t* fk, const int32_t* sel, int64_t n,
                          int32_t* out_fact_idx, int32_t* out_payload, int64_t out_cap, int64_t* d_out_count);

/* ------------------------------------------------------------------------------------------------------------------
 * Join-output materialisation: the gather out[i] = in[map[i]] that Section 7
 * finds behind the transform kernel, here with vectorised index loads and
 * output stores (the paper's advice for that kernel).
 */
typedef enum rel_side { REL_SIDE_FACT = 0, REL_SIDE_DIM = 1 } rel_side;

typedef struct rel_gather_col {
  const void* src;    /* device column of src_rows elements (aligned to elem_bytes) */
  void* dst;          /* device output of at least max_pairs elements, 16-byte aligned */
  int64_t src_rows;   /* rows of src; a row index outside [0, src_rows) is a device-side error */
  int32_t elem_bytes; /* 1, 2, 4 or 8 (any fixed-width type: the bytes are copied) */
  int32_t side;       /* rel_side: REL_SIDE_FACT indexes by fact_idx, REL_SIDE_DIM by dim_idx */
} rel_gather_col;

/* For i in [0, *d_n_pairs) (a device count, e.g. rel_join_probe's, at most
 * max_pairs) and each of the n_cols columns (1..8): dst[i] = src[fact_idx[i]]
 * (REL_SIDE_FACT) or src[dim_idx[i]] (REL_SIDE_DIM), where fact_idx / dim_idx
 * are a probe's out_fact_idx / out_payload (the dim row id when the table was
 * built without a payload). Index arrays: device, 16-byte aligned, needed only
 * for the sides some column uses. An index out of range of its column, or a
 * count above max_pairs, sets REL_DEV_BADARG (the element is written as 0, the
 * count is clamped). Host-side errors: REL_INVALID_ARG (null or misaligned
 * pointer, bad elem_bytes or side, n_cols outside 1..8), REL_UNSUPPORTED
 * (max_pairs >= 2^31). Stream-ordered, no synchronisation. */
rel_status rel_join_gather(rel_ctx* ctx, const int32_t* fact_idx, const int32_t* dim_idx, const int64_t* d_n_pairs,
                           int64_t max_pairs, const rel_gather_col* cols, int32_t n_cols);

/* ------------------------------------------------------------------------------------------------------------------
 * Group-by (cuDF's single_pass_shmem_aggs_kernel of Section 7: per-workgroup
 * aggregation in LDS, one device-memory update per group and workgroup).
 */
typedef struct rel_groups_out {
  int64_t* key;       /* device int64[cap] */
  int64_t* sum_price; /* device int64[cap] */
  int64_t* sum_qty;   /* device int64[cap] */
  int64_t* count;     /* device int64[cap] */
  int64_t cap;
  int64_t* d_n_groups; /* device int64: number of groups, written by every call that returns REL_OK (may exceed cap: then REL_DEV_OVERFLOW) */
} rel_groups_out;

/* Groups of the rows row = sel ? sel[k] : k, k in [0, n): key[row],
 * SUM(price[row]), SUM(qty[row]), COUNT(*). Output order unspecified. opts
 * nullable (plain sizing: capacity for min(n, 2^30) distinct keys). Every int64
 * key is allowed. */
rel_status rel_groupby_agg(rel_ctx* ctx, const int64_t* key, const int64_t* price, const int32_t* qty,
                           const int32_t* sel, int64_t n, const rel_table_opts* opts, rel_groups_out* out);

/* ------------------------------------------------------------------------------------------------------------------
 * The fused pipeline:
 *   SELECT g, SUM(price_cents), SUM(qty), COUNT(*) FROM fact JOIN dim ON fk = pk
 *   WHERE day < day_lt GROUP BY g
 * with g = (dim.prio, fact.flag) packed as prio * 256 + (uint8)flag, or
 * fact.fk, or dim.grp.
 */
typedef struct rel_fact {
  const int32_t* fk;
  const int64_t* price_cents;
  const int32_t* qty;
  const int32_t* day;
  const int8_t* flag; /* needed for REL_GROUP_PRIO_FLAG only */
  int64_t n;
} rel_fact;

typedef struct rel_dim {
  const int32_t* pk; /* unique */
  const int8_t* prio; /* needed for REL_GROUP_PRIO_FLAG only */
  const int32_t* grp; /* needed for REL_GROUP_DIM_GRP only */
  int64_t m;
} rel_dim;

typedef enum rel_group_by { REL_GROUP_PRIO_FLAG = 0, REL_GROUP_FK = 1, REL_GROUP_DIM_GRP = 2 } rel_group_by;

typedef struct rel_query {
  int32_t day_lt;   /* strict predicate day < day_lt */
  int32_t group_by; /* rel_group_by */
} rel_query;

/* Sizing and placement decided before the build (by the caller or by the
 * learned planner). Zero fields mean "plain sizing". */
typedef struct rel_plan {
  int64_t group_capacity;  /* expected distinct groups (0 = upper bound from the input) */
  int32_t group_placement; /* rel_placement */
  int32_t join_placement;  /* rel_placement */
  int32_t allow_fallback;  /* on overflow: 1 = rerun with plain sizing (synchronises), 0 = REL_OVERFLOW */
  int32_t reserved;
} rel_plan;

typedef struct rel_stats {
  int64_t rows_in;
  int64_t rows_passed;
  int64_t join_matches;
  int64_t groups;
  int64_t join_capacity;
  int64_t group_capacity;
  int32_t join_placement;
  int32_t group_placement;
  int32_t overflowed; /* the planned tables overflowed */
  int32_t fell_back;  /* the plain pipeline was rerun */
} rel_stats;

/* Run the fused pipeline. plan nullable (plain). stats nullable; when given,
 * the call synchronises and fills it. Returns REL_DUPLICATE_KEY / REL_OVERFLOW
 * only when it synchronises (stats given or fallback allowed); such a call
 * reads only the conditions its own kernels raised and leaves the sticky
 * status bits of earlier calls for rel_ctx_sync. A call that does not
 * synchronise leaves its conditions in the sticky bits. */
rel_status rel_filter_join_agg(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, const rel_query* q,
                               const rel_plan* plan, rel_groups_out* out, rel_stats* stats);

/* ------------------------------------------------------------------------------------------------------------------
 * Batched execution: many independent instances of the fused query in one
 * graph launch. Small kernels leave most of a large GPU idle (the paper's
 * undersaturation finding, Section 6.1, and its remedy of running work
 * concurrently); here every phase of every instance is a work item in one
 * persistent kernel per phase, and the phases are captured once in a HIP
 * graph, so a run is a single hipGraphLaunch.
 */
typedef struct rel_batch_item {
  rel_fact fact;
  rel_dim dim;
  rel_query q;
  rel_groups_out out;     /* device outputs of this instance */
  int64_t group_capacity; /* expected distinct groups (e.g. the NDV of dim.grp); 0 = upper bound min(n, m) */
} rel_batch_item;

/* One size bucket of the tuning table: instances with fact rows
 * n < 2^log2_rows_below use this configuration. Entries ascend; the last one
 * also takes every larger instance. */
typedef struct rel_batch_tuning {
  int32_t log2_rows_below;
  int32_t items_per_thread; /* fact rows per thread per step: 1, 2, 4 or 8 */
  int32_t block;            /* workgroup size: 64, 128, 256 or 512 */
  int32_t lds_groups_max;   /* LDS group table when the instance's group bound is at most this (<= 512); 0 = never */
  int32_t rows_per_item;    /* fact rows per work item (multiple of block * items_per_thread) */
  int32_t lds_join_max;     /* LDS join table (built per work item from the dim columns) when the instance's dim
                               has at most this many keys (<= 1024); 0 = never: the device-memory table */
} rel_batch_tuning;

typedef struct rel_batch rel_batch;

/* Plan, allocate and capture a batch of k instances (descriptors are copied;
 * the column and output buffers they point to must stay valid until
 * rel_batch_destroy). tuning nullable (library defaults), n_tuning entries. */
rel_status rel_batch_create(rel_ctx* ctx, const rel_batch_item* items, int32_t k, const rel_batch_tuning* tuning,
                            int32_t n_tuning, rel_batch** out);
/* Enqueue one run of every instance on the context's stream (one graph launch). */
rel_status rel_batch_run(rel_batch* b);
/* Synchronise and report on the last run: stats (nullable, k entries) with
 * rows passed / join matches / groups per instance; REL_OVERFLOW if any
 * instance's table overflowed, REL_DUPLICATE_KEY on a repeated pk (the batch's
 * own status word, cleared at the start of every run; the context's sticky
 * bits are not touched). */
rel_status rel_batch_sync(rel_batch* b, rel_stats* stats);
rel_status rel_batch_destroy(rel_batch* b);

/* ------------------------------------------------------------------------------------------------------------------
 * Learned planner. The paper's engine logs operator statistics (row counts,
 * selectivity, match ratios; Section 4.1) and cuDF sizes a join's output with
 * a separate counting kernel (Section 7). Here a small MLP predicts the join
 * output rows and the group count from a cheap sketch, so hash tables are
 * sized and placed before the build; an overflow reruns the plain pipeline,
 * so results never depend on the prediction.
 */
#define REL_SKETCH_FEATURES 40
#define REL_MLP_PARAMS 6914 /* 40x64 + 64 + 64x64 + 64 + 64x2 + 2 */

/* Sketch of a query's inputs: 64-register HyperLogLog of fact.fk (all rows)
 * and of dim.grp (when given), and statistics of k sampled fact rows and k
 * sampled dim rows, assembled into 40 features (in the fixed order the sketch
 * kernel writes them). d_fact_sample / d_dim_sample: device int64[k] row indices in
 * [0, n) / [0, m), drawn by the caller. Outputs (device): d_features float[40],
 * d_hll uint8[128] (fk registers, then grp registers). */
rel_status rel_sketch(rel_ctx* ctx, const rel_fact* fact, const rel_dim* dim, const rel_query* q,
                      const int64_t* d_fact_sample, const int64_t* d_dim_sample, int32_t k, float* d_features,
                      uint8_t* d_hll);

/* MLP 40 -> 64 -> 64 -> 2 with ReLU, FP32, parameters packed as
 * W1[40][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2] (input index
 * first, so a layer computes y[o] = b[o] + sum_i x[i] W[i][o]).
 * Forward: d_x float[B][40] -> d_y float[B][2]. */
rel_status rel_mlp_forward(rel_ctx* ctx, const float* d_params, const float* d_x, int32_t B, float* d_y);
/* Loss L = 1/(2B) sum (y - t)^2 and its gradient d_grad float[6914];
 * d_loss float[1] (nullable). Deterministic: no floating-point atomics. */
rel_status rel_mlp_backward(rel_ctx* ctx, const float* d_params, const float* d_x, const float* d_t, int32_t B,
                            float* d_grad, float* d_loss);
/* One Adam update (Kingma and Ba 2015) at step t >= 1 of params / first and
 * second moments (all device float[6914]). */
rel_status rel_mlp_adam_step(rel_ctx* ctx, float* d_params, float* d_m, float* d_v, const float* d_grad, int32_t t,
                             float lr, float beta1, float beta2, float eps);

typedef struct rel_planner rel_planner;

/* A planner from host arrays: params[6914], standardisation mean[40] /
 * scale[40] of the network's input, and the safety margin in log2 units added
 * to the predicted group count. The input is the sketch with its size-dependent
 * features taken relative to r, the log2 HyperLogLog estimate of the group key
 * (fk; dim.grp; for (prio, flag) the smaller of the fk estimate and
 * log2(1 + M)): features 0, 1, 12, 13, 16, 17 and 37 minus r, features 19..36
 * set to 0, then x' = (x - mean) / scale. The network's outputs are
 * log2(1 + join rows) - log2(1 + N) and log2(1 + groups) - r. */
rel_status rel_planner_create(rel_ctx* ctx, const float* params, const float* mean, const float* scale,
                              float margin_log2, rel_planner** out);
/* Sketch, predict and fill *plan (group capacity and placement, fallback
 * allowed). Group capacity = 2^(predicted log2 groups + margin), capped at the
 * plain bound; group placement LDS when that is at most 512 or a key is hot
 * (sampled max frequency >= 4/256), else device memory; join placement plain
 * (device memory) when a key is hot, the group key is a dim attribute and the
 * capacity is at most 2048, else left to the library. Synchronises once (a
 * few floats come back). pred (host, nullable) receives the predictions
 * log2(1 + join rows), log2(1 + groups). */
rel_status rel_planner_plan(rel_planner* p, const rel_fact* fact, const rel_dim* dim, const rel_query* q,
                            const int64_t* d_fact_sample, const int64_t* d_dim_sample, int32_t k, rel_plan* plan,
                            float* pred);
rel_status rel_planner_destroy(rel_planner* p);

/* ------------------------------------------------------------------------------------------------------------------
 * Bandwidth probe: the rate HBM gives this library's simplest access pattern
 * (16-byte loads and stores by consecutive lanes, eight per thread in
 * flight), the "achievable" bandwidth measured beside the vendor peak that the
 * rooflines use as their denominator (Section 3.1 and Table 2 take the
 * bandwidth of each GPU as the memory roofline).
 */
typedef enum rel_bw_mode { REL_BW_READ = 0, REL_BW_COPY = 1, REL_BW_WRITE = 2 } rel_bw_mode;

/* One streaming pass over `bytes` (a multiple of 16): READ reads src, COPY
 * copies src to dst, WRITE fills dst. src / dst are 16-byte aligned device
 * buffers (unused ones may be NULL); d_sink is one device uint64 that READ
 * may write so its loads are not optimised away. The grid is
 * blocks_per_cu (1..64) 256-thread workgroups per CU. Stream-ordered. */
rel_status rel_bw_probe(rel_ctx* ctx, int32_t mode, const void* src, void* dst, int64_t bytes, int32_t blocks_per_cu,
                        uint64_t* d_sink);

#ifdef __cplusplus
}
#endif

#endif /* REL_H_ */
