/*
 * hpa.h -- GPU PC-sample attribution on AMD Instinct MI355X (gfx950).
 *
 * Post-mortem core of GPU performance analysis as described in Zhou et al.,
 * "Measurement and Analysis of GPU-accelerated Applications with HPCToolkit"
 * (Parallel Computing 2021, arXiv 2109.06931):
 *
 *   1. map each sampled instruction address to its function, inlined code,
 *      loop and source line through an address-to-structure interval map
 *      (Section 5; Section 6.1 "Calling Context Expansion");
 *   2. aggregate samples by (calling context, PC, stall reason): a raw metric
 *      is the sum of the measured values (Section 4.2 sample record,
 *      Section 4.5 raw metrics);
 *   3. rebuild the approximate GPU calling context tree of each kernel
 *      invocation by splitting every GPU function's cost over its call sites
 *      in proportion to call-instruction samples, with recursion handled as
 *      strongly connected components (Section 6.3, steps 1-4);
 *   4. derive inclusive metrics and stall ratios such as the warp issue rate
 *      W = (S - S_stall) / S (Section 6.1 "Statistic Generation", Section 7.1).
 *
 * Conventions for every call
 * --------------------------
 *  - Every call returns hpa_status: HPA_OK (0) or a negative error code.  On
 *    error no output handle is created and out-parameters are left untouched;
 *    hpa_last_error() returns a message for the calling thread.
 *  - "host" pointers are CPU memory, borrowed for the duration of the call.
 *    "device" pointers are GPU memory on the context's device, borrowed until
 *    the given stream has executed the work the call enqueued.
 *  - All device work is enqueued on the stream passed in.  A call whose output
 *    size depends on the data synchronises that stream; each such call says
 *    how often.
 *  - Output handles own their device arrays (allocated through the context's
 *    allocator) and are immutable; *_view_get returns their device pointers.
 *    Release a handle with its *_free function; the handle must not be in use
 *    by queued work when it is freed.
 *  - A context (hpa_ctx) is used by one host thread at a time.  Handles may be
 *    read from several threads.
 *
 * Readings of points the paper leaves open (applied throughout):
 *  - a sample record without a weight counts once;
 *  - stall reason 0 means "not stalled", reasons 1..15 are stalls;
 *  - a PC outside every function is kept, under scope HPA_UNMAPPED, and
 *    attributed to an <unknown> node of the calling context tree;
 *  - overlapping functions: an address belongs to the containing function with
 *    the largest start, then the smallest end, then the smallest id;
 *  - inline and loop ranges form a laminar family, each inside the addresses
 *    of one function; equal ranges nest function > inline > loop, and among
 *    equal ranges of one kind the lower id is outer.
 */
#ifndef HPA_H
#define HPA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPA_OK = 0,
  HPA_E_INVAL = -1,       /* malformed argument or input value */
  HPA_E_UNSORTED = -2,    /* prebuilt intervals not in ascending order */
  HPA_E_OVERLAP = -3,     /* overlapping line ranges or prebuilt intervals */
  HPA_E_NOT_LAMINAR = -4, /* crossing inline/loop ranges, or one outside a function */
  HPA_E_NOMEM = -5,       /* the allocator returned NULL */
  HPA_E_BUDGET = -6,      /* calling context tree larger than the caller's node budget */
  HPA_E_DEVICE = -7,      /* a HIP runtime call failed */
  HPA_E_UNSUPPORTED = -8  /* valid input outside what the library as compiled handles (message says what) */
} hpa_status;

#define HPA_UNMAPPED 0xFFFFFFFFu           /* no scope / no interval / no parent */
#define HPA_NO_SITE 0xFFFFFFFFFFFFFFFFull  /* CCT node not entered through a call site */
#define HPA_N_STALL 16                     /* stall reasons 0..15 */

/* Thread-local message describing the last failure on this thread. */
const char* hpa_last_error(void);

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

/* Device-memory allocator.  alloc returns device memory usable on `stream`
 * (NULL on failure -> HPA_E_NOMEM); free releases it in stream order.  When
 * no allocator is given the library allocates with hipMallocAsync on the
 * device's default memory pool and keeps the blocks it releases (including
 * those of freed output handles) in a cache owned by the context, by size and
 * stream: a later allocation on the same stream reuses a cached block of at
 * most twice its size.  Cached blocks return to HIP when the context is
 * destroyed, or when an allocation would otherwise run out of memory. */
typedef struct {
  void* (*alloc)(size_t bytes, hipStream_t stream, void* user);
  void (*free)(void* ptr, hipStream_t stream, void* user);
  void* user;
} hpa_allocator;

typedef struct hpa_ctx hpa_ctx;

/* Create a context on HIP device `device`.  alloc may be NULL (default pool);
 * the struct is copied.  Errors: HPA_E_INVAL (bad device or out == NULL),
 * HPA_E_DEVICE. */
hpa_status hpa_ctx_create(int device, const hpa_allocator* alloc, hpa_ctx** out);
/* Destroy a context: waits for the device, then returns the cached blocks to
 * HIP.  Handles made with the context must be freed first. */
void hpa_ctx_destroy(hpa_ctx* ctx);

/* Stage timing, for profiling the library's own calls (not part of the
 * method).  When enabled, hpa_attribute records a hipEvent pair around each
 * of its stages on the call's stream and, after its final synchronisation,
 * adds the elapsed device time to the context's table, one row per stage
 * name: calls counted, and the items the stage read (samples or keys) and
 * wrote (keys).  hpa_ctx_set_timing(ctx, on) clears the table.  Names are
 * static strings owned by the library.  hpa_ctx_get_timing copies up to cap
 * rows into host memory `out` and sets *n_stages to the number of rows.
 * Errors: HPA_E_INVAL (NULL ctx or n_stages, or out NULL with cap > 0). */
typedef struct {
  const char* name;
  double ms;            /* summed device time over calls */
  uint64_t calls;
  uint64_t items_in;    /* summed over calls */
  uint64_t items_out;
} hpa_stage_time;
/* Number of times the library's calls on this context have waited for a
 * stream on the host (every synchronisation of every entry point is counted),
 * into *out (host).  A profiling aid: the difference around a call is the
 * number of times that call synchronised.  Errors: HPA_E_INVAL (NULL). */
hpa_status hpa_ctx_get_sync_count(const hpa_ctx* ctx, uint64_t* out);
hpa_status hpa_ctx_set_timing(hpa_ctx* ctx, int enable);
hpa_status hpa_ctx_get_timing(const hpa_ctx* ctx, hpa_stage_time* out, uint32_t cap, uint32_t* n_stages);

/* ------------------------------------------------------------------------ */
/* A1: structure map (Section 5; Section 6.1 calling-context expansion)      */
/* ------------------------------------------------------------------------ */

typedef enum { HPA_FUNC = 0, HPA_INLINE = 1, HPA_LOOP = 2 } hpa_scope_kind;

/* One address range [start, end) of a scope.  Functions are relocated to
 * unique addresses by the caller (Section 5); overlapping functions are split
 * by the library.  A scope id may repeat over several ranges (a loop spread
 * over several blocks); all ranges of one id share the kind and the parent. */
typedef struct {
  uint64_t start, end;
  uint32_t id;   /* scope id; the scope table is indexed by id */
  uint32_t kind; /* hpa_scope_kind */
} hpa_scope;

/* One source-line range [start, end).  Line ranges must not overlap; an
 * address inside a function but in no line range gets file 0, line 0. */
typedef struct {
  uint64_t start, end;
  uint32_t file, line;
} hpa_line_range;

/* Either scopes (+ optional lines), or prebuilt sorted disjoint intervals
 * (iv_start/iv_end, n_iv > 0; interval i is then labelled scope i with no
 * scope table).  All arrays are host memory. */
typedef struct {
  const hpa_scope* scopes;
  uint64_t n_scopes;
  const hpa_line_range* lines;
  uint64_t n_lines;
  const uint64_t* iv_start;
  const uint64_t* iv_end;
  uint64_t n_iv;
  int learned; /* 1: also train the learned interval index (HPA_LOOKUP_LEARNED) */
} hpa_structure_desc;

typedef struct hpa_structure_map hpa_structure_map;

/* Build the map: sorted, disjoint, maximally merged elementary intervals
 * [start, end) labelled (innermost scope, file, line), and the scope table
 * (parent, kind, owning function) indexed by scope id.  The host builds the
 * intervals and uploads them on `stream` (synchronised once at the end).
 * Errors: HPA_E_INVAL (start >= end, kind > 2, one id with two kinds),
 * HPA_E_OVERLAP (overlapping line ranges or prebuilt intervals),
 * HPA_E_UNSORTED (prebuilt intervals out of order), HPA_E_NOT_LAMINAR,
 * HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_build_structure_map(hpa_ctx* ctx, const hpa_structure_desc* desc, hipStream_t stream,
                                   hpa_structure_map** out);

/* Device arrays of a map (SoA; n_intervals and n_scope_ids entries). */
typedef struct {
  uint64_t n_intervals;
  uint32_t n_scope_ids;
  const uint64_t* start;
  const uint64_t* end;
  const uint32_t* scope;
  const uint32_t* file;
  const uint32_t* line;
  const uint32_t* parent; /* scope table: enclosing scope or HPA_UNMAPPED for functions */
  const uint8_t* kind;    /* hpa_scope_kind, 0xFF for unused ids */
  const uint32_t* func;   /* owning function scope id, HPA_UNMAPPED for unused ids */
} hpa_structure_map_view;

hpa_status hpa_structure_map_view_get(const hpa_structure_map* map, hpa_structure_map_view* out);
void hpa_structure_map_free(hpa_structure_map* map);

/* ------------------------------------------------------------------------ */
/* A3: address -> interval lookup (Section 6.1 calling-context expansion)    */
/* ------------------------------------------------------------------------ */

#define HPA_LOOKUP_PLAIN 0   /* binary search over interval starts */
#define HPA_LOOKUP_LEARNED 1 /* learned index + bounded search, verified (map built with learned=1) */

/* d_out[i] = the interval i with start[i] <= d_pc[i] < end[i], else
 * HPA_UNMAPPED.  d_pc (n x u64) and d_out (n x u32) are device memory.  Both
 * modes return identical results.  Asynchronous (no synchronisation).
 * Errors: HPA_E_INVAL (NULL pointers with n > 0, unknown mode),
 * HPA_E_UNSUPPORTED (learned mode on a map built without it). */
hpa_status hpa_lookup_intervals(hpa_ctx* ctx, const hpa_structure_map* map, const uint64_t* d_pc, uint64_t n,
                                uint32_t* d_out, int mode, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* A7: learned interval index (not in the paper; an index over the starts of  */
/* the same map whose answers are identical to the plain search)             */
/* ------------------------------------------------------------------------ */

/* Root network parameters, FP32, in this order: W1[64][2], b1[64],
 * W2[64][64], b2[64], w3[64], b3 (4417 floats).  Forward pass for input
 * (x0, x1): h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3;
 * leaf = clamp(floor(y * n_leaves), 0, n_leaves - 1). */
#define HPA_LEARNED_NPARAM 4417

typedef struct {
  uint32_t n_leaves;    /* 0: 4096 */
  uint32_t train_steps; /* Adam steps on the root (0: keep the initial, untrained root) */
  uint32_t batch;       /* rows per step (0: 8192) */
  uint32_t train_rows;  /* evenly spaced starts used as training rows (0: min(M, 2^20)) */
  float lr;             /* initial Adam step size, cosine-decayed (<= 0: 2e-3) */
  uint32_t window_cap;  /* largest window half-width a leaf keeps (0: 65536) */
  uint64_t seed;        /* initialisation seed (0: fixed default) */
} hpa_learned_opts;

typedef struct {
  uint32_t n_leaves, train_steps;
  double train_mse;      /* mean squared error of the root on its training rows (rank fraction) */
  double mean_window;    /* mean over the starts of their leaf's window (below + above + 1) */
  uint32_t max_window;   /* largest window of a leaf that some start is routed to */
  uint64_t uncovered;    /* starts (or start - 1 addresses) whose miss exceeded window_cap */
  const float* params;   /* device: the root's HPA_LEARNED_NPARAM parameters */
} hpa_learned_stats;

/* (Re)train the learned index of a map on its interval starts: the root
 * network by Adam on the device (forward/backward kernels of this library),
 * then one least-squares linear leaf per root output bucket and each leaf's
 * error window, evaluated with the lookup's own FP32 expression over every
 * start and every start - 1.  opts may be NULL (defaults).  Synchronises
 * `stream` twice.  hpa_build_structure_map with desc->learned = 1 calls this
 * with the defaults.  Errors: HPA_E_INVAL, HPA_E_UNSUPPORTED (fewer than two
 * intervals, or more than 2^32), HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_learned_train(hpa_ctx* ctx, hpa_structure_map* map, const hpa_learned_opts* opts, hipStream_t stream);

/* Summary of a map's learned index (params points to device memory owned by
 * the map).  Errors: HPA_E_INVAL, HPA_E_UNSUPPORTED (no learned index). */
hpa_status hpa_learned_stats_get(const hpa_structure_map* map, hpa_learned_stats* out);

/* HPA_LOOKUP_LEARNED that also adds, into device memory d_counts[2]
 * (u64, caller-initialised), the binary-search probes it made and the number
 * of queries that failed verification and took the plain search.
 * Asynchronous.  Errors as hpa_lookup_intervals. */
hpa_status hpa_lookup_learned_counted(hpa_ctx* ctx, const hpa_structure_map* map, const uint64_t* d_pc, uint64_t n,
                                      uint32_t* d_out, unsigned long long* d_counts, hipStream_t stream);

/* Gradient of the root's loss (1/n) sum_i (y(x_i) - t_i)^2 at parameters
 * d_params, by the training kernels: d_x is n x 2 FP32 inputs, d_t n FP32
 * targets (device); d_grad receives HPA_LEARNED_NPARAM gradients followed by
 * the summed squared error (device, HPA_LEARNED_NPARAM + 1 floats).  Sums are
 * FP32, per block of 128 rows, then over blocks in order.  Synchronises once.
 * Errors: HPA_E_INVAL (NULL, n == 0), HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_learned_grad(hpa_ctx* ctx, const float* d_params, const float* d_x, const float* d_t, uint64_t n,
                            float* d_grad, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* A2-A4: attribution (Section 4.2 sample record; Section 4.5 raw metrics)   */
/* ------------------------------------------------------------------------ */

/* PC samples, structure of arrays, device memory: pc[n] instruction address,
 * ctx[n] calling-context id (< n_ctx; the kernel invocation's placeholder),
 * stall[n] stall reason (< 16), weight[n] observation count or NULL (each
 * record then counts once). */
typedef struct {
  const uint64_t* pc;
  const uint32_t* ctx;
  const uint8_t* stall;
  const uint32_t* weight;
  uint64_t n;
  uint32_t n_ctx;
} hpa_samples;

typedef struct hpa_attribution hpa_attribution;

/* count[(ctx, pc, stall)] = sum of weights.  Output keys are unique and sorted
 * ascending by (ctx, pc, stall); scope is the innermost scope of pc (or
 * HPA_UNMAPPED); ctx_offsets (n_ctx + 1) is the CSR index of each context's
 * keys.  When the map's code fits a grid of at most 2^26 instruction
 * coordinates in at most 64 address windows (the map builds that grid itself)
 * and every sampled PC lies on it, the attribution runs device-driven and
 * synchronises `stream` once, to learn the number of keys; otherwise it
 * synchronises twice (once to size the work,
 * once to learn the number of keys).  Errors: HPA_E_INVAL (a stall >= 16 or ctx >= n_ctx,
 * NULL arrays), HPA_E_UNSUPPORTED (the PCs of one context span more than
 * 2^56 bytes after removing common trailing zero bits), HPA_E_NOMEM,
 * HPA_E_DEVICE. */
hpa_status hpa_attribute(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_samples* samples,
                         hipStream_t stream, hpa_attribution** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * attribution as hpa_attribute, with no hipMalloc, hipFree or other
 * allocating call.  Its working buffers live in one file-scope device array of
 * HPA_NOALLOC_SCRATCH_MIB MiB (one per GPU, held until the process ends); the
 * outputs are the caller's device arrays, each with room for samples->n keys
 * (ctx u32, pc u64, stall u8, count u64, scope u32) and ctx_offsets with
 * samples->n_ctx + 1 entries; *n_keys (host) receives the key count and
 * *scratch_used (host, may be NULL) the scratch bytes the call needed.  Calls
 * that overlap on one GPU share the array and race.  Synchronises `stream`
 * as hpa_attribute does.  Errors: HPA_E_INVAL (as hpa_attribute, or
 * samples->n over HPA_NOALLOC_MAX_SAMPLES, n_ctx over HPA_NOALLOC_MAX_CTX),
 * HPA_E_BUDGET (the scratch array is too small for this input),
 * HPA_E_UNSUPPORTED (a context with a caller allocator, or stage timing on),
 * HPA_E_DEVICE. */
#define HPA_NOALLOC_SCRATCH_MIB 128
#define HPA_NOALLOC_MAX_SAMPLES (1u << 20)
#define HPA_NOALLOC_MAX_CTX (1u << 16)
hpa_status hpa_attribute_noalloc(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_samples* samples,
                                 uint32_t* out_ctx, uint64_t* out_pc, uint8_t* out_stall, uint64_t* out_count,
                                 uint32_t* out_scope, uint64_t* out_ctx_offsets, uint64_t* n_keys,
                                 uint64_t* scratch_used, hipStream_t stream);

typedef struct {
  uint64_t n_keys;
  uint32_t n_ctx;
  const uint32_t* ctx;
  const uint64_t* pc;
  const uint8_t* stall;
  const uint64_t* count;
  const uint32_t* scope;
  const uint64_t* ctx_offsets;
} hpa_attribution_view;

hpa_status hpa_attribution_view_get(const hpa_attribution* a, hpa_attribution_view* out);
void hpa_attribution_free(hpa_attribution* a);

/* ------------------------------------------------------------------------ */
/* Batches of profiles (Section 6.1: profiles of threads and GPU streams are */
/* processed as concurrent tasks; Section 6.2: rounds under a memory cap)    */
/* ------------------------------------------------------------------------ */

typedef struct {
  const hpa_structure_map* map; /* the profile's structure map */
  uint64_t n_samples;           /* its records: the next n_samples of the batch arrays */
  uint32_t n_ctx;               /* its contexts; its records' ctx values are < n_ctx */
} hpa_profile_desc;

typedef struct {
  uint64_t max_round_samples; /* samples per round (0: 2^31); a larger profile forms a round of its own */
  int autotune;               /* 1: time the run-time parameters on a pilot (<= 2^26 samples of the first
                                 round) and keep the fastest in the context for later calls */
  uint32_t merge_rounds;      /* without autotune: rounds of unit-pair merges, 0..3 (default 2 when opts is NULL) */
  uint32_t scan_wg_per_cu;    /* without autotune: context-scan workgroups per compute unit (0: 4) */
} hpa_batch_opts;

typedef struct {
  uint32_t n_rounds, merge_rounds, scan_wg_per_cu, autotuned;
  uint64_t total_keys;
  double tune_ms; /* host time spent autotuning (0 when the context already had parameters) */
} hpa_batch_info;

typedef struct hpa_batch hpa_batch;

/* Attribute many profiles at once.  `samples` holds every profile's records
 * back to back in profile order (device SoA as for hpa_attribute; n is the
 * total, n_ctx is ignored).  Profiles are grouped into rounds; in a round the
 * contexts of all profiles are numbered globally and every stage of the
 * attribution runs once for the whole round (each unit of the sort holds
 * contexts of one profile and uses that profile's map).  When the profiles
 * share at most 64 maps, with at least two profiles per map on average, each
 * round holds profiles of one map (their records gathered into round buffers
 * when they are not adjacent) and runs the dense pipeline when the map has
 * dense coordinates; otherwise rounds are runs of consecutive profiles.  Each
 * profile's result equals hpa_attribute on its own records, byte for byte.
 * Synchronises `stream` a fixed number of times per round.  Errors: as
 * hpa_attribute (HPA_E_INVAL also when the profiles' counts do not add up to
 * samples->n or a record's ctx is not below its profile's n_ctx). */
hpa_status hpa_attribute_batched(hpa_ctx* ctx, uint32_t n_profiles, const hpa_profile_desc* profiles,
                                 const hpa_samples* samples, const hpa_batch_opts* opts, hipStream_t stream,
                                 hpa_batch** out);

/* One profile's result, as the view of its own attribution (device pointers
 * into the batch's arrays, ctx and ctx_offsets local to the profile). */
hpa_status hpa_batch_profile_view(const hpa_batch* b, uint32_t profile, hpa_attribution_view* out);
hpa_status hpa_batch_info_get(const hpa_batch* b, hpa_batch_info* out);
void hpa_batch_free(hpa_batch* b);

/* ------------------------------------------------------------------------ */
/* A5: GPU calling context tree (Section 6.3)                                */
/* ------------------------------------------------------------------------ */

/* Static call graph from function symbols and call instructions (Section
 * 6.3 step 1), host memory.  Node ids are function scope ids of the map and
 * n_funcs must equal its number of scope ids.  One entry per call
 * instruction: site_pc must lie in site_caller's addresses and be unique. */
typedef struct {
  uint32_t n_funcs;
  uint64_t n_sites;
  const uint64_t* site_pc;
  const uint32_t* site_caller;
  const uint32_t* site_callee;
} hpa_callgraph;

/* Host calling contexts, host memory: parent[c] (HPA_UNMAPPED for a root)
 * and kernel_entry[c], the GPU kernel function launched at placeholder c, or
 * -1.  A context with an entry uses the call graph restricted to what the
 * entry reaches; one without uses the whole graph with every function that
 * no other function calls as a root. */
typedef struct {
  uint32_t n;
  const uint32_t* parent;
  const int32_t* kernel_entry;
} hpa_context_table;

typedef struct hpa_callgraph_plan hpa_callgraph_plan;

/* Validate the call graph and context table against the map, find the SCCs
 * (Tarjan, Section 6.3 step 3; ids ranked by smallest member), build the
 * condensed graph and upload it.  Host work plus one synchronisation; reuse
 * the plan for every profile that shares the graph.  Errors: HPA_E_INVAL
 * (n_funcs mismatch, a caller/callee/entry that is not a function, duplicate
 * site_pc, a site outside its caller, a parent index out of range or a cycle
 * in the context table), HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_prepare_callgraph(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_callgraph* graph,
                                 const hpa_context_table* contexts, hipStream_t stream,
                                 hpa_callgraph_plan** out);
void hpa_callgraph_plan_free(hpa_callgraph_plan* plan);

typedef struct {
  int sample_based;        /* 1: edge weights are call-instruction samples, apply step 2 (required) */
  uint64_t max_cct_nodes;  /* 0: no limit; else HPA_E_BUDGET if the tree needs more nodes */
  uint64_t* required_nodes; /* host, may be NULL: receives the node count on HPA_OK and HPA_E_BUDGET */
} hpa_apportion_opts;

typedef struct hpa_gpu_cct hpa_gpu_cct;

/* Per context: self cost per function and stall; call-site weights (the call
 * instruction's samples); step 2 as the least fixpoint of its rule; SCC
 * condensation with the step-2 rule applied once more on the condensed graph;
 * unfolding from the roots into a tree whose nodes are call paths, children
 * ordered by call-site PC, with phi(path) the product of w(e) / W(callee)
 * along the path and exclusive cost phi * self (Section 6.3 step 4).  Paths
 * that reach no sample are pruned by an integer test.  Samples outside the
 * entry's reach form an <unreachable> node, unmapped PCs an <unknown> node.
 * Synchronises `stream` twice.  Errors: HPA_E_INVAL (attribution from another
 * map or context count), HPA_E_BUDGET, HPA_E_UNSUPPORTED (sample_based == 0),
 * HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_apportion_callpaths(hpa_ctx* ctx, const hpa_callgraph_plan* plan, const hpa_attribution* attr,
                                   const hpa_apportion_opts* opts, hipStream_t stream, hpa_gpu_cct** out);

/* Node kinds */
#define HPA_NODE_PATH 0
#define HPA_NODE_UNREACHABLE 1
#define HPA_NODE_UNKNOWN 2

/* Device arrays of a GPU CCT.  Nodes of context c are
 * [node_offsets[c], node_offsets[c+1]) in DFS preorder; parent is an index
 * local to the context (HPA_UNMAPPED for a child of the placeholder); node is
 * the condensed call-graph node (HPA_UNMAPPED for the special nodes); site is
 * the call-site PC of the edge into the node; excl holds 16 stall columns per
 * node.  w_offsets/w_site/w_val list, per context, the final positive weight
 * of every call edge between condensed nodes, by call-site PC. */
typedef struct {
  uint64_t n_nodes;
  uint32_t n_ctx;
  uint32_t n_funcs;
  const uint32_t* scc;
  const uint64_t* node_offsets;
  const uint32_t* parent;
  const uint32_t* node;
  const uint64_t* site;
  const uint8_t* kind;
  const double* phi;
  const double* excl;
  uint64_t n_weights;
  const uint64_t* w_offsets;
  const uint64_t* w_site;
  const uint64_t* w_val;
} hpa_gpu_cct_view;

hpa_status hpa_gpu_cct_view_get(const hpa_gpu_cct* t, hpa_gpu_cct_view* out);
void hpa_gpu_cct_free(hpa_gpu_cct* t);

/* ------------------------------------------------------------------------ */
/* A6: derived metrics (Section 6.1 statistic generation; Section 7.1)       */
/* ------------------------------------------------------------------------ */

typedef struct hpa_metrics hpa_metrics;

/* Inclusive values up three trees:
 *  - GPU CCT (FP64): incl(p,s) = excl(p,s) + children's incl in child order;
 *    S = sum over s, W = (S - S_stall) / S with S_stall over reasons 1..15
 *    (0 when S = 0);
 *  - host calling-context tree (integer): per context, the samples of its
 *    subtree per stall reason, and its W;
 *  - static scope tree per context (integer): for each scope on the ancestor
 *    chain of a sampled scope, the samples of the scope and everything nested
 *    in it; CSR by context, scopes ascending (HPA_UNMAPPED last).
 * Synchronises `stream` once.  Errors: HPA_E_INVAL (inputs from different
 * plans or attributions), HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_derive_metrics(hpa_ctx* ctx, const hpa_callgraph_plan* plan, const hpa_attribution* attr,
                              const hpa_gpu_cct* cct, hipStream_t stream, hpa_metrics** out);

typedef struct {
  uint64_t n_nodes;
  uint32_t n_ctx;
  const double* incl; /* n_nodes x 16 */
  const double* S;    /* n_nodes */
  const double* W;    /* n_nodes */
  const uint64_t* host_incl; /* n_ctx x 16 */
  const double* host_W;      /* n_ctx */
  uint64_t n_scope_rows;
  const uint64_t* sc_offsets; /* n_ctx + 1 */
  const uint32_t* sc_scope;
  const uint64_t* sc_val; /* n_scope_rows x 16 */
} hpa_metrics_view;

hpa_status hpa_metrics_view_get(const hpa_metrics* m, hpa_metrics_view* out);
void hpa_metrics_free(hpa_metrics* m);

/* ------------------------------------------------------------------------ */
/* Several profiles: unification, statistics, sparse layouts (Sections 4.5,  */
/* 6.1 and 6.2), and combination of runs (Section 4.7)                       */
/* ------------------------------------------------------------------------ */

typedef struct hpa_unified hpa_unified;

/* Unify the contexts of n_profiles attributions made on one map with one
 * context count: the unified contexts are the sorted union of their (ctx, pc)
 * pairs; metric m of a context is its sample count with stall reason m.
 * Builds, on the device:
 *  - CMS (context-major sparse): per unified context c, entries
 *    [cms_ctx_off[c], cms_ctx_off[c+1]) of (cms_pid, cms_val) ordered by
 *    metric then profile; its non-empty metrics are the pairs
 *    (cms_mid[j], cms_mstart[j]) for j in [cms_m_off[c], cms_m_off[c+1]);
 *  - PMS (profile-major sparse): per profile p, entries
 *    [pms_off[p], pms_off[p+1]) of (pms_mid, pms_val) ordered by context then
 *    metric, with (pms_ctx[h], pms_cstart[h]) for h in
 *    [pms_c_off[p], pms_c_off[p+1]) marking where each of its contexts starts;
 *  - statistics per CMS metric entry j (context cms_mctx[j], metric
 *    cms_mid[j]) over all profiles, an absent value counting as 0: sum, min,
 *    max (u64), mean = sum / P, population standard deviation and coefficient
 *    of variation std / mean (0 when the mean is 0) in FP64.
 * Synchronises `stream` (a fixed number of times, independent of P).
 * Errors: HPA_E_INVAL (no profiles, NULL, attributions of other maps,
 * context counts or contexts), HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_unify_profiles(hpa_ctx* ctx, uint32_t n_profiles, const hpa_attribution* const* profiles,
                              hipStream_t stream, hpa_unified** out);

typedef struct {
  uint32_t n_profiles;
  uint64_t n_contexts;         /* unified (ctx, pc) contexts */
  uint64_t n_nonzeros;         /* (profile, context, metric) entries */
  uint64_t n_metric_entries;   /* non-empty (context, metric) pairs */
  uint64_t n_profile_contexts; /* (profile, context) pairs */
  const uint32_t* ctx;
  const uint64_t* pc;
  const uint32_t* scope;
  const uint64_t *cms_ctx_off, *cms_m_off;
  const uint8_t* cms_mid;
  const uint64_t* cms_mstart;
  const uint32_t* cms_mctx;
  const uint32_t* cms_pid;
  const uint64_t* cms_val;
  const uint64_t *pms_off, *pms_c_off;
  const uint32_t* pms_ctx;
  const uint64_t* pms_cstart;
  const uint8_t* pms_mid;
  const uint64_t* pms_val;
  const uint64_t *st_sum, *st_min, *st_max;
  const double *st_mean, *st_std, *st_cov;
} hpa_unified_view;

hpa_status hpa_unified_view_get(const hpa_unified* u, hpa_unified_view* out);
void hpa_unified_free(hpa_unified* u);

#define HPA_SPARSE_CMS 0
#define HPA_SPARSE_PMS 1

/* Write one sparse layout to a file: eight u64 header words (magic
 * 0x45535241505350, format, contexts, profiles, metrics = 16, non-zeros,
 * metric entries (CMS) or profile contexts (PMS), section count), the
 * sections' u64 file offsets, then the sections, each at an 8-aligned offset
 * found by an exclusive scan of their sizes: ctx u32[C], pc u64[C], then for
 * CMS cms_ctx_off, cms_m_off, cms_mid, cms_mstart, cms_pid, cms_val and for
 * PMS pms_off, pms_c_off, pms_ctx, pms_cstart, pms_mid, pms_val.  Device
 * data reach the file through a host buffer of at most round_bytes
 * (0: 64 MiB), one round at a time.  Errors: HPA_E_INVAL (path, format),
 * HPA_E_DEVICE (I/O or copy failure). */
hpa_status hpa_unified_write(const hpa_unified* u, const char* path, int format, uint64_t round_bytes,
                             hipStream_t stream);

/* Combine runs: per (ctx, pc, stall) key, the sum of the runs' counts, as one
 * attribution (same layout as hpa_attribute's).  The runs must share a map
 * and a context count.  Synchronises `stream`.  Errors: as
 * hpa_unify_profiles, and as hpa_attribute. */
hpa_status hpa_combine_runs(hpa_ctx* ctx, uint32_t n_runs, const hpa_attribution* const* runs, hipStream_t stream,
                            hpa_attribution** out);

/* ------------------------------------------------------------------------ */
/* A9: serving ingest (Section 4.1: sample buffers delivered as they fill;   */
/* Section 4.5: the raw metric is a sum, so arrival order does not matter)   */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint32_t n_profiles;        /* independent profiles (streams), ids 0..n_profiles-1 */
  uint32_t n_ctx;             /* contexts per profile; a record's ctx must be < n_ctx (<= 2^28) */
  uint64_t table_slots;       /* per-profile key table capacity, rounded up to a power of two (0: 2^22) */
  uint64_t pc_slots;          /* distinct-PC table shared by all profiles (0: 2^20; <= 2^31) */
  uint64_t max_batch_bytes;   /* device staging per in-flight batch; also the largest buffer (0: 64 MiB) */
  uint32_t n_slots;           /* batches in flight at once, one HIP stream each (0: 4) */
  uint32_t max_batch_buffers; /* buffers coalesced into one launch (0: 512) */
  uint64_t hbm_budget;        /* device bytes the server may hold: state + staging (0: 200e9) */
} hpa_server_opts;

typedef struct {
  uint64_t buffers, samples, bytes, batches, errors;
  uint64_t max_inflight_bytes;
  double p50_us, p99_us, max_us, mean_us; /* submit -> attributed latency over completed buffers */
  double span_s;                          /* first submit to last completion */
} hpa_server_stats;

typedef struct hpa_server hpa_server;

/* Create a server over a structure map: per-profile device state (a key
 * table of (ctx, pc, stall) -> u64 count per profile, and one table of
 * distinct PCs) and n_slots staging areas, all allocated here; the state and
 * staging together must fit hbm_budget (else HPA_E_BUDGET).  A worker thread
 * owned by the server batches queued buffers into free slots and launches
 * their ingest on the slots' own streams, so batches overlap.  The map must
 * outlive the server.  Errors: HPA_E_INVAL, HPA_E_UNSUPPORTED, HPA_E_BUDGET,
 * HPA_E_NOMEM, HPA_E_DEVICE. */
hpa_status hpa_server_create(hpa_ctx* ctx, const hpa_structure_map* map, const hpa_server_opts* opts,
                             hpa_server** out);

/* Queue one sample buffer of `profile`: host memory holding, back to back,
 * pc u64[n], ctx u32[n], stall u8[n] (13 n bytes, 8-byte aligned; each
 * record counts once).  The buffer is read asynchronously and must stay
 * valid and unchanged until its ticket completes; pinned memory (hipHostMalloc)
 * gives the fastest copies.  Thread-safe.  Never blocks on the device.
 * Errors: HPA_E_INVAL, HPA_E_BUDGET (buffer larger than the batch staging),
 * HPA_E_DEVICE (the server stopped after a device error). */
hpa_status hpa_server_submit(hpa_server* srv, uint32_t profile, const void* buffer, uint64_t n_samples,
                             uint64_t* ticket);

/* Block until the ticket's buffer is folded into its profile's state;
 * *latency_us (may be NULL) receives submit -> completion time.  Returns the
 * batch's status: HPA_E_INVAL when a record of the batch had ctx >= n_ctx or
 * stall >= 16, HPA_E_BUDGET when a table ran out of slots (the profiles of
 * that batch then hold an undefined part of it). */
hpa_status hpa_server_wait(hpa_server* srv, uint64_t ticket, double* latency_us);

/* Block until every submitted buffer has completed. */
hpa_status hpa_server_drain(hpa_server* srv);

/* Counters and latency percentiles of completed buffers; reset != 0 clears them. */
hpa_status hpa_server_stats_get(hpa_server* srv, int reset, hpa_server_stats* out);

/* The profile's state as an attribution (same layout and guarantees as
 * hpa_attribute's output, built from the completed buffers): ingest pauses
 * while the table is read, then the table's entries go through the
 * attribution path on `stream`.  Call hpa_server_drain first to include
 * everything submitted.  Synchronises `stream`.  Errors: as hpa_attribute. */
hpa_status hpa_server_snapshot(hpa_server* srv, uint32_t profile, hipStream_t stream, hpa_attribution** out);

/* Stop the worker after the queued buffers are done and free the server. */
void hpa_server_destroy(hpa_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* HPA_H */
