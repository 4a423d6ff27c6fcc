/*
 * hgrd.h -- C ABI of the MI355X exact per-access-pair race query.
 *
 * The query (sections 2 and 6.1-6.4 of "Towards an Accurate GPU Data Race
 * Detector"; Table 2): for two accesses to the same array, at least one a
 * write, can two distinct threads of one launch reach the same address with
 * both guards true, in the same barrier interval when they share a block?
 * The paper encodes this as constraints and asks a SAT solver per access
 * pair (section 6.4).  This library decides it exactly by enumerating the
 * finite domains the host code fixes (launch extents, loop ranges and the
 * parameter tuples of section 6.3), on the GPU, and also returns exact
 * per-race-type counts and the lexicographically smallest witness.
 *
 * Conventions
 *   - All integers are little-endian host integers.  Every input array is
 *     owned by the caller, read-only to the library, and may be freed when
 *     the call returns.  Outputs are caller-owned.
 *   - Calls are synchronous on the stream given in the options (NULL: the
 *     null stream).  A context must not be used by two host threads at once.
 *   - A call returns RD_OK unless an argument is structurally unusable
 *     (RD_EINVAL: NULL pointer with a nonzero count, bad options), device
 *     memory runs out (RD_ENOMEM) or the device fails (RD_EDEVICE).  Errors
 *     that belong to one pair go to that pair's result (`status`), with
 *     verdict, counts and witness cleared; other pairs are unaffected.
 *   - EXACT mode is deterministic: every field is identical for any tiling,
 *     batching, tile order or graph replay.
 */
#ifndef HGRD_H
#define HGRD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes (pair statuses use the first five) ---------------- */
enum {
  RD_OK = 0,
  RD_EINVAL = -1,       /* malformed model, expression or pair */
  RD_EUNSUPPORTED = -2, /* outside the supported limits (below) */
  RD_ERANGE = -3,       /* an int64 operation overflowed, or a 32-bit
                           array's address left int32 */
  RD_EDIVZERO = -4,     /* division or remainder by zero */
  RD_ENOMEM = -5,
  RD_EDEVICE = -6,
  RD_ECAPACITY = -7     /* a caller buffer is too small */
};
/* When a pair has several errors the reported one is, strongest first:
 * EINVAL, EUNSUPPORTED, EDIVZERO, ERANGE. */

/* ---- expressions ----------------------------------------------------
 * Postfix integer bytecode.  Leaves: a constant (imm), kernel parameter
 * `arg`, threadIdx/blockIdx/blockDim/gridDim component `arg` (0=x, 1=y,
 * 2=z), or the value of model loop `arg`.  Operators follow C on int64:
 * '/' truncates toward zero, '%' takes the sign of the dividend, '>>' is
 * arithmetic, comparisons and logical operators give 0 or 1 and evaluate
 * both operands.  An operation that overflows int64, divides by zero, or
 * shifts by a count outside [0, 63] records an error and yields 0;
 * evaluation continues (so the set of errors is well defined).
 * Where each leaf may appear:
 *   launch extents          : CONST, PARAM
 *   loop init/bound/step    : + BDIM, GDIM
 *   bint, wint              : + LOOP (loops enclosing the access)
 *   addr, guard, acq, rel   : + TID, BID
 * Limits: at most 256 instructions and a stack depth of 16. */
enum {
  RD_OP_CONST = 1, RD_OP_PARAM = 2, RD_OP_TID = 3, RD_OP_BID = 4,
  RD_OP_BDIM = 5, RD_OP_GDIM = 6, RD_OP_LOOP = 7,
  RD_OP_ADD = 16, RD_OP_SUB, RD_OP_MUL, RD_OP_DIV, RD_OP_MOD, RD_OP_SHL,
  RD_OP_SHR, RD_OP_AND, RD_OP_OR, RD_OP_XOR, RD_OP_MIN, RD_OP_MAX,
  RD_OP_LT, RD_OP_LE, RD_OP_EQ, RD_OP_NE, RD_OP_GE, RD_OP_GT,
  RD_OP_LAND, RD_OP_LOR,
  RD_OP_NEG = 48, RD_OP_LNOT = 49
};

typedef struct {
  uint16_t op;   /* RD_OP_* */
  uint16_t arg;  /* parameter index, axis, or model loop index */
  uint32_t pad;
  int64_t imm;   /* RD_OP_CONST value */
} rd_insn;

typedef struct {
  uint32_t first; /* index into the model's instruction pool */
  uint32_t count; /* 0 = absent: guard true, bint/wint 0; addr required */
} rd_expr;

/* ---- kernel model ---------------------------------------------------- */
enum { RD_GLOBAL = 0, RD_SHARED = 1 };          /* array space (section 2) */
enum { RD_READ = 0, RD_WRITE = 1, RD_ATOMIC = 2 };
enum { RD_SCOPE_BLOCK = 0, RD_SCOPE_DEVICE = 1 }; /* atomic scope (app. A) */
enum { RD_CMP_LT = 0, RD_CMP_LE, RD_CMP_GT, RD_CMP_GE, RD_CMP_NE };
enum { RD_UPD_ADD = 0, RD_UPD_SUB, RD_UPD_MUL, RD_UPD_DIV, RD_UPD_SHL,
       RD_UPD_SHR };

/* Arrays with the same nonzero `alias` are views of one memory (two
 * pointers into one buffer; the paper is silent on aliasing): element k of
 * such an array is element base + k of the memory, so an access's effective
 * address is base + its address (an overflow is RD_ERANGE), and accesses
 * on two views may form a pair.  Views of one memory must share the space
 * (else the pair is RD_EINVAL); acquires and releases on two views of one
 * memory at one effective address are one lock.  alias = 0: a memory of
 * its own (base is ignored).  For a 32-bit array the effective address must
 * fit int32.  A vector access of w elements (e.g. float4 against float) is
 * modelled as an access inside an extra model loop j in [0, w) with address
 * a + j: its counts are then of element pairs. */
typedef struct {
  uint32_t space;     /* RD_GLOBAL or RD_SHARED (shared: one per block) */
  uint32_t addr_bits; /* 32: addresses must fit int32; 64 */
  uint32_t alias;     /* memory id shared by views (< 2^24), 0: none */
  uint32_t pad;
  int64_t base;       /* the view's first element in the memory */
} rd_array;

/* for (v = init; v <cmp> bound; v = v <upd> step); init, bound and step
 * are evaluated once per parameter tuple.  At most 65536 iterations. */
typedef struct {
  rd_expr init, bound, step;
  uint32_t cmp, upd;
} rd_loop;

/* An acquire (atomicCAS then fence) or a release (fence then atomicExch)
 * around an access (section 6.5, Figure 9; appendix A).  `addr` is the
 * address it operates on, an expression over the same leaves as the
 * access's address (count 0: none), in array `array` (any space; a 32-bit
 * array's addresses must fit int32 like data addresses).  `scope` is the
 * narrower of its atomic's and its fence's scopes (RD_SCOPE_*). */
typedef struct {
  rd_expr addr;
  uint32_t array, scope;
} rd_sync;

/* One static load, store or atomic (section 6.1, "Generating access
 * pairs").  `loops` lists the enclosing model loops, outermost first (at
 * most 4); the iteration index is row-major over them.  `bint` and `wint`
 * are barrier-interval ids in [0, 65536): two points of one block can race
 * only if their bint are equal (a block barrier between them otherwise,
 * section 6.1), and within one warp only if their wint are also equal.
 *
 * `acq` and `rel`: the acquire that dominates the access and the release
 * that post-dominates it, if any (section 6.5; the control-flow search for
 * them is the caller's).  At each point and for a required scope (device
 * for an inter-block conflict, block for intra-block and intra-warp ones;
 * appendix A, Figure 10) only operations at least that wide are seen, and
 * syn() is the lock when both are seen and hit one address of one array,
 * else the release of a write (producer), else the acquire of a read
 * (consumer), else none (Figure 9).  A conflicting point pair is no race
 * when both points have a syn() and the two hit the same address of the
 * same array (Table 2's last constraint, taken jointly with the others).
 * A lock or flag in a shared array is one per block, so it never orders
 * threads of two blocks.  Pairs with an acquire or release on either
 * access are joined by the HBM aggregation path whatever their size. */
typedef struct {
  uint32_t array, kind, scope, n_loops;
  uint32_t loops[4];
  rd_expr addr, guard, bint, wint;
  rd_sync acq, rel;
} rd_access;

typedef struct {
  const rd_insn* insns; uint32_t n_insns;
  const rd_array* arrays; uint32_t n_arrays;
  const rd_loop* loops; uint32_t n_loops;
  const rd_access* acc; uint32_t n_acc;
  uint32_t n_params;
} rd_kernel_model;

/* Launch geometry of a model (section 6.3 class 2): grid and block extents
 * as expressions (in the model's instruction pool) over parameters, and
 * the warp size of the analysed program (1..1024; 32 for CUDA).  A tuple
 * whose extents are not all >= 1 launches nothing.  Limits: a block of at
 * most 1024 threads, a grid of fewer than 2^26 blocks, fewer than 2^31
 * points (block x thread x iteration) per access and tuple. */
typedef struct {
  rd_expr grid[3], block[3];
  uint32_t warp_size;
  uint32_t pad;
} rd_launch_domain;

/* Host-fixed parameter tuples (section 6.3 classes 1-5): n_sets rows of
 * n_params values, row-major.  Each row is one launch; conflicts never
 * cross rows.  At most 4096 rows. */
typedef struct {
  uint32_t n_sets;
  uint32_t pad;
  const int64_t* values;
} rd_param_sets;

/* ---- host domain (section 4, classes 1-5; section 6.3, Figure 8) ------
 * What the host code of a program fixes about a launch, written as host
 * variables and conditions, expanded into the finite parameter tuples that
 * rd_check_pairs takes.  The five classes of host facts map as follows:
 *   class 1 (asserts)           : `asserts`, conditions that hold in every
 *                                 execution (assignments where one is 0 are
 *                                 dropped);
 *   class 2 (grid dimensions)   : `params` columns that the model's launch
 *                                 domain reads as parameters (e.g. a column
 *                                 hWidth / 16 used as gridDim.x);
 *   class 3 (shared variables)  : several `params` columns computed from one
 *                                 host variable keep their relation, since
 *                                 every tuple comes from one assignment;
 *   class 4 (host loop bounds)  : RD_HV_LOOP variables, one value per
 *                                 iteration of the host loop;
 *   class 5 (allocation sizes)  : `alloc_sizes`, sizes of allocations the
 *                                 host makes, positive in every execution
 *                                 (assignments where one is <= 0 are
 *                                 dropped).
 * Host variables are listed in program order.  Their expressions (and the
 * asserts, sizes and parameter columns) live in `insns` and may use only
 * RD_OP_CONST, RD_OP_PARAM k (the value of host variable k, k below the
 * variable's own index; any k below n_vars elsewhere) and the operators. */
enum {
  RD_HV_INPUT = 0, /* an input the program reads: takes each of
                      values[0 .. n_values) in turn (the caller's finite
                      stand-in for an unknown value) */
  RD_HV_EXPR = 1,  /* computed from earlier variables: `init` */
  RD_HV_LOOP = 2   /* the iterator of a host loop, for (v = init; v <cmp>
                      bound; v = v <upd> step), init/bound/step over earlier
                      variables, at most 65536 iterations (cmp and upd as
                      for rd_loop) */
};

typedef struct {
  uint32_t kind;            /* RD_HV_* */
  uint32_t cmp, upd;        /* RD_HV_LOOP */
  uint32_t n_values;        /* RD_HV_INPUT */
  const int64_t* values;    /* RD_HV_INPUT */
  rd_expr init, bound, step;
} rd_host_var;

typedef struct {
  const rd_insn* insns; uint32_t n_insns;
  const rd_host_var* vars; uint32_t n_vars;
  const rd_expr* asserts; uint32_t n_asserts;
  const rd_expr* alloc_sizes; uint32_t n_alloc;
  const rd_expr* params; uint32_t n_params;  /* one column per kernel
                                                parameter */
} rd_host_domain;

/* Enumerates every assignment of the host variables (inputs over their
 * values, loop iterators over their iterations, nested in program order,
 * the first variable outermost), keeps those whose asserts are all nonzero
 * and allocation sizes all positive, and evaluates the parameter columns
 * of each.  Equal tuples are kept once (the first), in enumeration order.
 * out->n_sets = the number of distinct tuples, out->values = buf (row-major,
 * n_params values per tuple).  Host-only; no device work.
 * Returns RD_OK; RD_ECAPACITY when n_sets x n_params exceeds cap_values
 * (out->n_sets still holds the count needed, buf holds the first tuples
 * that fit); RD_EINVAL for a NULL or malformed argument (a leaf other than
 * CONST or PARAM, a variable read before it is set, a bad kind, cmp or
 * upd); RD_EUNSUPPORTED for more than 65536 iterations of one host loop,
 * more than 2^24 assignments, or expressions over the limits of model
 * expressions; RD_EDIVZERO or RD_ERANGE when an expression divides by zero
 * or overflows in some assignment (the host program would fail there). */
int rd_expand_host_domain(const rd_host_domain* h, rd_param_sets* out,
                          int64_t* buf, uint64_t cap_values);

/* Race classes (Table 2). */
enum { RD_INTER = 1, RD_INTRA_BLOCK = 2, RD_INTRA_WARP = 4 };

/* An access pair: two accesses of one model on the same array, and the
 * classes the caller wants checked (RD_INTER | RD_INTRA_BLOCK | ...). */
/* ---- kernel body (section 6.1 "Avoiding race checks"; section 6.5) -----
 * A structured kernel body as a flat statement list, from which the
 * barrier-interval ids of every access and the acquire and release around
 * it are derived (rd_derive_body).  RD_ST_IF opens a two-way branch (its
 * condition is not modelled: the accesses' guards carry it), RD_ST_ELSE
 * switches to the other way, RD_ST_LOOP opens the body of model loop
 * `arg`, RD_ST_END closes the innermost open construct.  RD_ST_CAS and
 * RD_ST_EXCH are atomics on `addr` (an expression of the model's pool, over
 * the leaves of an access address, loops only those enclosing the
 * statement) in array `array` at `scope`; RD_ST_FENCE is a fence at
 * `scope`.  An acquire is a CAS followed by a fence, a release a fence
 * followed by an Exch (section 2). */
enum {
  RD_ST_ACCESS = 1,   /* arg: access index of the model (at most once) */
  RD_ST_BARRIER,      /* block barrier (syncthreads) */
  RD_ST_WARP_BARRIER, /* warp barrier (syncwarp) */
  RD_ST_IF, RD_ST_ELSE, RD_ST_END,
  RD_ST_LOOP,         /* arg: model loop index */
  RD_ST_CAS, RD_ST_EXCH, RD_ST_FENCE
};
typedef struct {
  uint32_t kind, arg, array, scope;
  rd_expr addr;
} rd_stmt;

/* Derives, for every access the body names, its enclosing loops, `bint`,
 * `wint`, `acq` and `rel` (the model's other accesses are copied as they
 * are) into acc_out[m->n_acc]; the new expressions follow a copy of the
 * model's instruction pool in insns_out (*n_insns_out entries), so a model
 * with insns = insns_out and acc = acc_out is the derived one.
 *   bint: the number of counted block barriers the thread has executed
 *   before the access (wint: warp barriers).  A barrier counts when it is
 *   outside every branch (a barrier is reached by all threads only in
 *   uniform code; one under a branch proves nothing, as it dominates no
 *   later access) and each enclosing loop is an ADD loop compared with LT
 *   or LE or a SUB loop compared with GT or GE (trip count and iteration
 *   index then have closed forms); two points of one block are separated
 *   by a barrier exactly when their counts differ.
 *   acq: the nearest fence that dominates the access, then the nearest CAS
 *   that dominates that fence (Figure 10's backward search); rel: the
 *   nearest fence that post-dominates the access, then the nearest Exch
 *   after it; each with the narrower of its two scopes.  A statement
 *   dominates (post-dominates) an access when it sits directly in a
 *   sequence that contains the access, before (after) it; a statement
 *   inside a branch or a loop body that does not contain the access does
 *   neither.  The nearest pair is taken whatever its scope.
 * Host only.  Returns RD_OK; RD_EINVAL for a malformed body (unbalanced or
 * misplaced IF/ELSE/END, a bad loop, access, array or scope, an access
 * named twice, a bad atomic address); RD_EUNSUPPORTED when an access sits
 * in more than 4 loops or a derived expression exceeds the expression
 * limits; RD_ECAPACITY when cap_insns is too small (*n_insns_out holds the
 * size needed). */
int rd_derive_body(const rd_kernel_model* m, const rd_stmt* body, uint32_t n_stmts,
                   rd_access* acc_out, rd_insn* insns_out, uint32_t cap_insns,
                   uint32_t* n_insns_out);

typedef struct {
  uint32_t model, a, b;
  uint32_t class_mask;
} rd_access_pair;

/* ---- options ---------------------------------------------------------- */
enum { RD_MODE_EXACT = 0, RD_MODE_VERDICT = 1 };
enum { RD_ORDER_LEX = 0, RD_ORDER_MLP = 1, RD_ORDER_INTERVAL = 2 };

/* The tile-scoring network of VERDICT mode: 32 tile features -> 64 -> 64 ->
 * 1 logit, ReLU, fp32.  Row-major, output-major weight matrices. */
typedef struct {
  float w1[64 * 32], b1[64];
  float w2[64 * 64], b2[64];
  float w3[64], b3;
} rd_mlp;

typedef struct {
  uint32_t mode;       /* RD_MODE_EXACT (default) or RD_MODE_VERDICT */
  uint32_t order;      /* VERDICT tile order: RD_ORDER_LEX (tile index),
                          RD_ORDER_MLP (network score) or RD_ORDER_INTERVAL
                          (tile index among the tiles whose two blocks'
                          address ranges meet; disjoint tiles last, as for
                          the network) */
  uint32_t prefilter;  /* 1: decide without enumeration (exact) the
                          (pair, tuple) units whose two accesses share no
                          address: their address ranges (bounds proven for
                          the term tables) do not meet, or their address
                          residues (every address = u + k G, G the gcd of
                          the table terms' known factors) admit no common
                          value, or (units of at least 2^18 points) the
                          unions of their per-block address intervals do
                          not meet; 0: off */
  uint32_t log_level;  /* 0 silent, 1 summary, 2 per-launch (stderr) */
  uint32_t lds_cap;    /* records per LDS join tile (1024, 1536 or 3072);
                          0 = the context's default (1024 until
                          rd_autotune picks one) */
  uint32_t tile_budget;/* VERDICT: tiles searched per (pair, tuple) before
                          the exact path; 0 = 256 */
  const rd_mlp* mlp;   /* weights for RD_ORDER_MLP (copied at prepare) */
  uint64_t max_device_bytes; /* HBM bucket bytes per partition wave;
                                0 = the context's default (3072 MiB until
                                rd_autotune picks one) */
  void* stream;        /* hipStream_t every launch goes to; NULL = a
                          stream the context owns */
} rd_options;

/* ---- results ----------------------------------------------------------
 * count_by_class: ordered point pairs (p from access a, q from access b)
 * of each class, summed over tuples (modulo 2^64); count = their sum;
 * verdict = count > 0; classes = bits of the nonzero classes.  Witness:
 * the smallest (set, b1, t1, i1, b2, t2, i2) in lexicographic order over
 * conflicting point pairs, with linear block, thread and iteration ids
 * (x fastest); witness_class is its class and w_addr its address.  The
 * witness fields are 0xFFFFFFFF (w_addr 0) when verdict is 0.
 * flags: bit 0 = trivially race-free (empty class mask, section 6.1);
 * bit 1 = VERDICT mode stopped at a conflicting tile (count is a lower
 * bound, witness valid but not necessarily the smallest).
 * evals: launch-box points of both accesses over all tuples (before
 * guards; a self-pair counts its box twice). */
typedef struct {
  uint64_t count, count_by_class[3];
  int32_t status;
  uint8_t verdict, classes, witness_class, flags;
  uint32_t w_set, w_b1, w_t1, w_i1, w_b2, w_t2, w_i2;
  uint32_t tiles;  /* VERDICT mode: rank + 1 of the tile that stopped the
                      search (tiles examined in order); 0 otherwise */
  int64_t w_addr;
  uint64_t evals;
} rd_pair_result;

typedef struct rd_context rd_context;

/* Creates a context on HIP device `hip_device`.  Returns RD_OK,
 * RD_EDEVICE or RD_ENOMEM.  *ctx is NULL on failure. */
int rd_context_create(rd_context** ctx, int hip_device);
void rd_context_destroy(rd_context* ctx);

/* Decides every pair (see the conventions above).  `launch` and `params`
 * are per model.  `opt` may be NULL.  `out` has n_pairs entries.
 * More than 4096 pairs (the environment variable HGRD_BATCH_PAIRS sets
 * the batch; 0 turns batching off) are decided in consecutive batches of
 * pairs, each its own plan: batch k + 1 is prepared on a host thread, on a
 * second context of the same device that ctx creates on first use and
 * keeps until rd_context_destroy, while batch k runs on ctx's stream, so
 * host lowering overlaps device work.  Not when opt->stream is set, nor
 * when that second context cannot be created (then one plan for all).  The results are those of one plan; rd_get_stats
 * then reports the sums over the batches (total_ms: the whole call). */
int rd_check_pairs(rd_context* ctx, const rd_kernel_model* models,
                   uint32_t n_models, const rd_access_pair* pairs,
                   uint32_t n_pairs, const rd_launch_domain* launch,
                   const rd_param_sets* params, const rd_options* opt,
                   rd_pair_result* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * query as rd_check_pairs, same arguments, same results, but every device
 * buffer it needs (descriptors, term tables, accumulators, HBM bucket
 * records, re-partition and fallback scratch, results) comes from one
 * fixed scratch area of RD_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating call, captures no graph and creates no event.
 * `ctx` must come from rd_context_create (which looks the area up on its
 * device).  Inputs stay caller-owned host memory, `out` caller-owned host
 * memory of n_pairs entries, as for rd_check_pairs.  Without an explicit
 * opt->max_device_bytes each partition wave takes an eighth of the area.
 * Returns the statuses of rd_check_pairs, and RD_ECAPACITY (with a message
 * on stderr naming the buffer that did not fit, `out` unspecified) when the
 * batch needs more than the area: split the batch or use rd_check_pairs.
 * The area keeps the last call's contents (every call clears what it
 * reads first).  Calls on one GPU share its area: within one process they
 * are serialised by a lock; work the caller overlaps with a call on the
 * same area from outside the library (e.g. a replayed graph of an earlier
 * call's kernels) races with it. */
#define RD_NOALLOC_SCRATCH_BYTES (128ull << 20)
int rd_check_pairs_noalloc(rd_context* ctx, const rd_kernel_model* models,
                           uint32_t n_models, const rd_access_pair* pairs,
                           uint32_t n_pairs, const rd_launch_domain* launch,
                           const rd_param_sets* params, const rd_options* opt,
                           rd_pair_result* out);

/* Two-step use of the same query: rd_prepare validates, lowers and plans
 * the batch and copies every descriptor to device memory; rd_execute runs
 * the kernels and returns the results, and may be called any number of
 * times on one plan (the results are identical each time).  The plan owns
 * its device memory until rd_plan_destroy.  rd_check_pairs is rd_prepare,
 * rd_execute and rd_plan_destroy in one call.  Statuses as for
 * rd_check_pairs.  A plan belongs to the context it was prepared on. */
typedef struct rd_plan rd_plan;
int rd_prepare(rd_context* ctx, const rd_kernel_model* models,
               uint32_t n_models, const rd_access_pair* pairs,
               uint32_t n_pairs, const rd_launch_domain* launch,
               const rd_param_sets* params, const rd_options* opt,
               rd_plan** plan);
int rd_execute(rd_context* ctx, rd_plan* plan, rd_pair_result* out);
void rd_plan_destroy(rd_plan* plan);

/* The first phase of rd_execute (accumulator set-up, the VERDICT tile
 * search, the LDS joins of small items and the HBM partition waves) has no
 * host round trip; the first rd_execute of a plan captures it in a HIP
 * graph and later calls replay that graph.  log_level 2 or the environment
 * variable HGRD_TIMING run it eagerly instead, with HIP events around the
 * partition kernels (rd_stats.scatter_ms and friends are only filled then
 * for the first phase).  Calls on one plan must not overlap. */

/* Batch autotuning: for the batch given (as rd_prepare), times rd_execute
 * for every LDS tile shape (1024, 1536, 3072 records) and partition-wave
 * size (768, 3072, 12288 MiB): one warm-up and `reps` timed runs each (1..16),
 * median wall time.  The fastest pair becomes the context's default for
 * plans whose options leave lds_cap and max_device_bytes at 0.  *best is a
 * copy of opt (or of zeroed options) with those two fields set; *best_ms
 * its median time (may be NULL).  Returns RD_EINVAL for a NULL ctx or
 * best, else the first non-OK status of rd_prepare or rd_execute. */
int rd_autotune(rd_context* ctx, const rd_kernel_model* models,
                uint32_t n_models, const rd_access_pair* pairs,
                uint32_t n_pairs, const rd_launch_domain* launch,
                const rd_param_sets* params, const rd_options* opt,
                uint32_t reps, rd_options* best, double* best_ms);

/* Timing and size figures of the last rd_execute (or rd_check_pairs). */
typedef struct {
  double total_ms;        /* host entry to results copied back */
  double device_ms;       /* first to last kernel, HIP events */
  double join_ms;         /* LDS join kernels (small items + buckets) */
  double scatter_ms;      /* generate-and-partition kernels */
  double witness_ms;      /* witness pass 2 */
  uint64_t evals;         /* sum of the pairs' evals */
  uint64_t records;       /* point bound of the HBM-partitioned items */
  uint64_t small_items, hbm_items, overflow_items, buckets;
  uint64_t join_launches; /* launches of the join kernels */
  double join_kernel_ms;  /* summed duration of those launches */
  double small_ms;        /* k_small_join */
  double bucket_ms;       /* k_bucket_join */
  double fallback_ms;     /* HBM aggregation of overflowed items */
  double retry_ms;        /* re-partitioning of overflowed items */
  uint64_t retry_items;   /* items re-partitioned with more buckets */
  double waves_ms;        /* all partition waves (scatter + bucket join) */
  double verdict_ms;      /* VERDICT mode: bounds, scores, order, tile search */
  uint64_t verdict_units; /* (query, tuple) units searched tile by tile */
  double split_ms;        /* items split by (address, block) */
  uint64_t split_items;
  uint64_t scatter_launches; /* table-path partition launches (k_scatter
                                with term tables), timed in scatter_tab_ms */
  uint64_t scatter_bytes;    /* record bytes all partition kernels wrote */
  uint64_t fallback_records; /* point bound of the fallback items */
  double scatter_tab_ms;     /* table-path partition kernels */
  uint64_t scatter_tab_bytes; /* record bytes they wrote */
  uint64_t prefiltered;      /* (pair, tuple) units the pre-filter decided */
  uint64_t join_tab_launches; /* table-path bucket join launches
                                 (k_bucket_join with term tables) */
  double join_tab_ms;        /* their summed duration */
  uint64_t join_tab_bytes;   /* record bytes they read */
  uint64_t presplit_items;   /* items sent to the (address, block) split
                                without a first partition pass */
  uint64_t filter_tab_launches; /* table-path address-filter launches
                                   (k_bucket_filter before the table-path
                                   join), timed in filter_tab_ms */
  double filter_tab_ms;      /* their summed duration */
  uint64_t filter_tab_bytes; /* record bytes they read */
  uint64_t units_apart;      /* HBM items the unit filter decided free of
                                conflicts: their two accesses share no
                                address (proven address ranges apart, or
                                residues that differ), or both compute their
                                address with one expression that sends
                                different threads to different addresses
                                (a mixed-radix dependence test on its affine
                                form), so nothing of them is partitioned or
                                joined;
                                small items are decided the same way inside
                                the LDS join (not counted).  The environment
                                variable HGRD_NO_UNIT_FILTER turns it off */
  uint64_t block_symmetric;  /* shared-array (pair, tuple) units joined on
                                block 0 only: neither access's address nor
                                guard depends on the block coordinates, so
                                every block holds the same conflicts and the
                                counts are block 0's times the blocks
                                (HGRD_NO_SYMMETRY at rd_prepare turns it off) */
  uint64_t fallback_groups;  /* records the fallback wrote: lanes of one
                                wavefront with equal (address, block,
                                iteration, warp, intervals) share one record
                                that carries its lane mask, so this is at most
                                the points of the fallback items */
  uint64_t sync_records;     /* point bound of the (pair, tuple) units with an
                                acquire or release, joined by the fallback
                                path with the synchronisation levels */
  uint64_t sync_decided;     /* such units decided conflict-free before any
                                join (the unit filter's tests at rd_prepare:
                                addresses apart, or one thread-injective
                                address expression) when every expression of
                                both accesses, acquire and release addresses
                                included, is proven error-free */
} rd_stats;

int rd_get_stats(const rd_context* ctx, rd_stats* out);

/* ---- learned tile order (VERDICT mode) -----------------------------------
 * A tile is block b1 of access a against block b2 of access b under one
 * tuple.  VERDICT mode searches the tiles of each eligible (pair, tuple) in
 * rounds of 1, 4, 16, ... tiles in LEX order (b1 * G + b2) or by descending
 * network score (ties by index), up to tile_budget tiles, and stops a pair at
 * its first conflicting tile: verdict 1, a valid (not necessarily smallest)
 * witness from that tile, counts = the conflicts inside that tile (flags bit
 * 1: count is a lower bound).  Pairs with no conflict in the searched tiles,
 * and pairs not eligible (shared arrays, more than 2^20 tiles, tiles larger
 * than one LDS join), get the EXACT result.  Statuses are the EXACT ones. */

/* Features (32 floats per tile) and labels (1: the tile holds a conflict,
 * 0: not, -1: the pair has an evaluation error) of every tile of every
 * eligible (pair, tuple), computed by the exact checker; `ids` gets (pair,
 * tuple, b1, b2) per row.  *n_rows is set to the number of rows; returns
 * RD_ECAPACITY (and writes nothing) when it exceeds max_rows. */
int rd_tile_data(rd_context* ctx, const rd_kernel_model* models,
                 uint32_t n_models, const rd_access_pair* pairs,
                 uint32_t n_pairs, const rd_launch_domain* launch,
                 const rd_param_sets* params, const rd_options* opt,
                 uint64_t max_rows, float* feats, float* labels, uint32_t* ids,
                 uint64_t* n_rows);

/* Network logits of n feature rows (n x 32, row-major). */
int rd_mlp_forward(rd_context* ctx, const rd_mlp* w, const float* x,
                   uint64_t n, float* logits, void* stream);

/* Mean binary cross-entropy on logits over n rows with labels y (0/1), and
 * its gradient with respect to every weight (same layout as rd_mlp). */
int rd_mlp_grad(rd_context* ctx, const rd_mlp* w, const float* x,
                const float* y, uint64_t n, rd_mlp* grad, float* loss,
                void* stream);

/* Trains w in place with Adam (learning rate lr, betas 0.9/0.999) on
 * minibatches of `batch` rows, `epochs` passes over a permutation drawn
 * from `seed`; epoch_loss[e] (optional) gets each epoch's mean loss. */
int rd_mlp_train(rd_context* ctx, rd_mlp* w, const float* x, const float* y,
                 uint64_t n, uint32_t epochs, uint32_t batch, float lr,
                 uint64_t seed, float* epoch_loss, void* stream);

/* Weights of the tile-scoring network on disk: a 32-byte header (the
 * bytes "HGRDMLP1", then uint32 version 1, uint32 weight count 6337,
 * uint32 feature version, uint32 reserved 0) followed by the weights as
 * little-endian float32 in the rd_mlp layout.  rd_mlp_save writes the file
 * (RD_EINVAL for NULL arguments or an unwritable path); rd_mlp_load reads
 * it into *w and sets *feature_version (may be NULL) -- RD_EINVAL for a
 * missing or short file, a wrong magic, version or count.  Host-only. */
int rd_mlp_save(const rd_mlp* w, uint32_t feature_version, const char* path);
int rd_mlp_load(rd_mlp* w, uint32_t* feature_version, const char* path);

const char* rd_strerror(int status);

/* Host-side self-checks of the library's integer helpers (no device work).
 * Returns 0 when they pass. */
int rd_selftest(void);

/* Host-only check of the exact pre-filters on one (pair, tuple) unit of
 * accesses access_a and access_b of `model` under tuple `set`: bit 0 of
 * *decided is set when the unit would be decided without enumeration by
 * rd_options.prefilter and by the unit filter of rd_execute (the two
 * accesses then share no address); bit 1 when the unit filter would
 * decide it because both accesses compute their address with one
 * expression that sends different threads to different addresses (a self
 * pair included).  Returns
 * RD_OK, 2 when an access has no instance for the tuple (errors, empty
 * launch), or RD_EINVAL for bad arguments.  Touches no device. */
int rd_prefilter_selftest(const rd_kernel_model* models, uint32_t n_models,
                          const rd_launch_domain* launch, const rd_param_sets* params,
                          uint32_t model, uint32_t access_a, uint32_t access_b,
                          uint32_t set, uint32_t* decided);

/* Host-side check of the term-table lowering of one access under one
 * parameter tuple (no device work): builds the tables as the device would,
 * then compares guard, address and interval ids at every point of the
 * launch box (or at max_points points spread over it when max_points is
 * nonzero and smaller) with the interpreter on the original expressions.
 * Returns 0 when they agree (*n_checked = points compared), 1 when the
 * access does not qualify for tables, 2 when it has an error or no points,
 * a negative value on a disagreement, RD_EINVAL on bad indices. */
int rd_table_selftest(const rd_kernel_model* models, uint32_t n_models,
                      const rd_launch_domain* launch, const rd_param_sets* params,
                      uint32_t model, uint32_t access, uint32_t set,
                      uint64_t max_points, uint64_t* n_checked);

#ifdef __cplusplus
}
#endif
#endif /* HGRD_H */
