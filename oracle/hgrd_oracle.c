/*
 * CPU oracle for the exact per-access-pair GPU race query.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  The GPU library never links
 * it, and it includes nothing from the GPU library: its structures, opcode
 * numbers and arithmetic are written here independently.
 *
 * What it computes (the paper's race definition and constraints):
 *   - a race is two accesses by different threads to the same address, at
 *     least one a write, not separated by synchronisation (section 2, "Data
 *     races on GPUs"; section 6.1, "Avoiding race checks");
 *   - race types (section 2 "Types of data races"; section 6.2; Table 2):
 *       inter-block  : addr equal, tb differ
 *       intra-block  : addr equal, tb equal, id differ, wp differ
 *       intra-warp   : addr equal, tb equal, id differ, wp equal
 *   - pairs that skip checks (section 6.1; appendix A.2): read/read and
 *     device-scoped atomic/atomic are trivially race-free; atomic/atomic with
 *     a block-scoped side only needs the inter-block check;
 *   - block and warp barriers between the accesses remove intra-block and
 *     intra-warp checks (section 6.1).  Here they are modelled per point by
 *     barrier-interval ids: two points of the same block race intra-block only
 *     in the same block-barrier interval, and intra-warp only when the
 *     warp-barrier intervals also match;
 *   - host-fixed values (sections 4 and 6.3, classes 1-5) arrive as finite
 *     parameter tuples; each tuple is one launch, so conflicts never cross
 *     tuples;
 *   - acquire-release synchronisation (section 6.5, Figure 9, Table 2's
 *     highlighted constraint; appendix A, Figure 10): an access may name
 *     the acquire and the release around it (address expression, array,
 *     scope).  At each point, for a required scope, syn() is the lock when
 *     acquire and release both reach that scope and hit the same address,
 *     else the release for a write (producer), else the acquire for a read
 *     (consumer), else none.  The required scope is device for an
 *     inter-block conflict and block for the other two.  A conflicting
 *     point pair is no race when both points have a syn() at the required
 *     scope and the two hit the same address of the same array (joint
 *     reading: the inequality is one more conjunct of the same constraint
 *     set).  A lock or flag in shared memory is one per block, so it never
 *     orders threads of two blocks.
 * The paper hands these constraints to a SAT solver (section 6.4).  Here the
 * domains are finite, so the oracle decides them by enumeration and also
 * reports exact per-class counts of ordered conflicting point pairs and the
 * lexicographically smallest conflicting (tuple, p, q).
 *
 * Two methods:
 *   method 0 (Oracle-A): the definition verbatim, a double loop over points.
 *   method 1 (Oracle-B): sort the points of both sides by
 *     (addr, block, bint, warp, wint, thread) and count pairs with equal key
 *     prefixes: the number of (p, q) with equal key K is the sum over key
 *     groups of n_i * n_j (an equi-join cardinality).  Class counts are
 *     differences of such sums.  Synchronised pairs are counted the same way
 *     over the points that have a syn() at the class's scope, with the
 *     synchronisation (array, address) added to each key, and subtracted.
 *     The witness is found in two passes: the smallest p with a partner,
 *     then the smallest partner q of that p.
 *
 * Integer semantics are C's on int64 (truncating '/', '%' with the sign of
 * the dividend, arithmetic '>>', comparisons giving 0/1).  An operation that
 * overflows, divides by zero or shifts by a count outside [0, 63] records an
 * error and yields 0; evaluation continues.  The guard is evaluated at every
 * point of the launch box; address and interval ids only where the guard is
 * nonzero.  Statuses, strongest first: EINVAL, EUNSUPPORTED, EDIVZERO,
 * ERANGE.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* ---- oracle-local encoding (the Python loader maps names to these) ---- */
enum {
  O_CONST = 1, O_PARAM, O_TID, O_BID, O_BDIM, O_GDIM, O_LOOP,
  O_ADD = 20, O_SUB, O_MUL, O_DIV, O_MOD, O_SHL, O_SHR, O_AND, O_OR, O_XOR,
  O_MIN, O_MAX, O_LT, O_LE, O_EQ, O_NE, O_GE, O_GT, O_LAND, O_LOR,
  O_NEG = 60, O_LNOT
};
enum { K_READ = 0, K_WRITE = 1, K_ATOMIC = 2 };
enum { SC_BLOCK = 0, SC_DEVICE = 1 };
enum { SP_GLOBAL = 0, SP_SHARED = 1 };
enum { C_INTER = 1, C_BLOCK = 2, C_WARP = 4 };
enum { ST_OK = 0, ST_INVAL = -1, ST_UNSUP = -2, ST_RANGE = -3, ST_DIVZERO = -4 };
enum { E_DIVZERO = 1, E_RANGE = 2, E_UNSUP = 4, E_INVAL = 8 };

#define MAX_TOKS 256
#define MAX_DEPTH 16
#define MAX_LOOPS 4
#define MAX_ITERS 65536
#define MAX_SETS 4096
#define MAX_BLOCK 1024
#define MAX_GRID (1LL << 26)
#define MAX_POINTS (1LL << 31)
#define INTERVAL_LIMIT 65536

typedef struct { int64_t op, arg; } OTok;
typedef struct { int32_t first, count; } OExpr;
/* alias != 0: a view of memory `alias` whose element 0 is the memory's
 * element `base` (views with one alias and space share their elements) */
typedef struct { int32_t space, addr_bits, alias, pad; int64_t base; } OArray;
typedef struct { OExpr init, bound, step; int32_t cmp, upd; } OLoop;
/* acquire or release: addr.count 0 = none */
typedef struct { OExpr addr; int32_t array, scope; } OSync;
typedef struct {
  int32_t array, kind, scope, n_loops;
  int32_t loops[8];
  OExpr addr, guard, bint, wint;
  OSync acq, rel;
} OAccess;
typedef struct {
  const OTok* toks; int32_t n_toks;
  const OArray* arrays; int32_t n_arrays;
  const OLoop* loops; int32_t n_loops;
  const OAccess* acc; int32_t n_acc;
  int32_t n_params;
  OExpr grid[3], block[3];
  int32_t warp;
  int32_t n_sets;
  const int64_t* sets; /* n_sets x n_params, row major */
} OModel;
typedef struct { int32_t model, a, b, mask; } OPair;
typedef struct {
  uint64_t count, by_class[3];
  int32_t status, verdict, classes, witness_class, flags, pad;
  int64_t w_set, w_b1, w_t1, w_i1, w_b2, w_t2, w_i2, w_addr;
  uint64_t evals;  /* box points of both sides over all tuples (self: twice) */
} OResult;

/* ------------------------------------------------------------------------ */
/* Checked int64 arithmetic.  On error: record the bit, return 0.            */

static int64_t op_bin(int op, int64_t a, int64_t b, int* err) {
  int64_t r;
  switch (op) {
    case O_ADD: if (__builtin_add_overflow(a, b, &r)) { *err |= E_RANGE; return 0; } return r;
    case O_SUB: if (__builtin_sub_overflow(a, b, &r)) { *err |= E_RANGE; return 0; } return r;
    case O_MUL: if (__builtin_mul_overflow(a, b, &r)) { *err |= E_RANGE; return 0; } return r;
    case O_DIV:
      if (b == 0) { *err |= E_DIVZERO; return 0; }
      if (a == INT64_MIN && b == -1) { *err |= E_RANGE; return 0; }
      return a / b;  /* C99: truncation toward zero */
    case O_MOD:
      if (b == 0) { *err |= E_DIVZERO; return 0; }
      if (a == INT64_MIN && b == -1) { *err |= E_RANGE; return 0; }
      return a % b;  /* C99: sign of the dividend */
    case O_SHL: {
      if (b < 0 || b > 63) { *err |= E_RANGE; return 0; }
      /* a << b is a * 2^b; it must be representable in int64 */
      __int128 w = (__int128)a * ((__int128)1 << b);
      if (w < (__int128)INT64_MIN || w > (__int128)INT64_MAX) { *err |= E_RANGE; return 0; }
      return (int64_t)w;
    }
    case O_SHR:
      if (b < 0 || b > 63) { *err |= E_RANGE; return 0; }
      /* arithmetic shift: floor(a / 2^b) */
      if (a >= 0) return a >> b;
      return -(int64_t)(((uint64_t)(-(a + 1))) >> b) - 1;
    case O_AND: return a & b;
    case O_OR: return a | b;
    case O_XOR: return a ^ b;
    case O_MIN: return a < b ? a : b;
    case O_MAX: return a > b ? a : b;
    case O_LT: return a < b;
    case O_LE: return a <= b;
    case O_EQ: return a == b;
    case O_NE: return a != b;
    case O_GE: return a >= b;
    case O_GT: return a > b;
    case O_LAND: return (a != 0) && (b != 0);
    case O_LOR: return (a != 0) || (b != 0);
  }
  *err |= E_INVAL;
  return 0;
}

static int is_binary(int64_t op) { return op >= O_ADD && op <= O_LOR; }
static int is_unary(int64_t op) { return op == O_NEG || op == O_LNOT; }
static int is_leaf(int64_t op) { return op >= O_CONST && op <= O_LOOP; }

/* Values a point expression can read. */
typedef struct {
  const int64_t* params;
  int64_t tid[3], bid[3], bdim[3], gdim[3];
  int64_t loopval[64]; /* indexed by model loop id */
} OEnv;

static int64_t eval(const OModel* m, OExpr e, const OEnv* env, int64_t dflt, int* err) {
  if (e.count == 0) return dflt;
  int64_t st[MAX_DEPTH];
  int sp = 0;
  for (int32_t k = 0; k < e.count; ++k) {
    const OTok* t = &m->toks[e.first + k];
    int64_t op = t->op, arg = t->arg;
    if (is_leaf(op)) {
      int64_t v = 0;
      switch (op) {
        case O_CONST: v = arg; break;
        case O_PARAM: v = env->params[arg]; break;
        case O_TID: v = env->tid[arg]; break;
        case O_BID: v = env->bid[arg]; break;
        case O_BDIM: v = env->bdim[arg]; break;
        case O_GDIM: v = env->gdim[arg]; break;
        case O_LOOP: v = env->loopval[arg]; break;
      }
      st[sp++] = v;
    } else if (is_unary(op)) {
      int64_t a = st[sp - 1];
      if (op == O_NEG) {
        if (a == INT64_MIN) { *err |= E_RANGE; st[sp - 1] = 0; }
        else st[sp - 1] = -a;
      } else {
        st[sp - 1] = (a == 0);
      }
    } else {
      int64_t b = st[--sp];
      int64_t a = st[sp - 1];
      st[sp - 1] = op_bin((int)op, a, b, err);
    }
  }
  return st[0];
}

/* Structural check of one expression.  ctx: 0 launch (const, param),
 * 1 loop bounds (+ bdim, gdim), 2 interval ids (+ loops of the access),
 * 3 address/guard (+ tid, bid).  Returns 0, E_INVAL or E_UNSUP. */
static int check_expr(const OModel* m, OExpr e, int ctx, const OAccess* a) {
  if (e.count == 0) return 0;
  if (e.first < 0 || e.count < 0 || (int64_t)e.first + e.count > m->n_toks) return E_INVAL;
  int depth = 0, maxd = 0;
  for (int32_t k = 0; k < e.count; ++k) {
    const OTok* t = &m->toks[e.first + k];
    if (is_leaf(t->op)) {
      switch (t->op) {
        case O_CONST: break;
        case O_PARAM: if (t->arg < 0 || t->arg >= m->n_params) return E_INVAL; break;
        case O_BDIM: case O_GDIM:
          if (ctx < 1 || t->arg < 0 || t->arg > 2) return E_INVAL;
          break;
        case O_TID: case O_BID:
          if (ctx < 3 || t->arg < 0 || t->arg > 2) return E_INVAL;
          break;
        case O_LOOP: {
          if (ctx < 2 || !a) return E_INVAL;
          int found = 0;
          for (int i = 0; i < a->n_loops; ++i) found |= (a->loops[i] == t->arg);
          if (!found) return E_INVAL;
          break;
        }
      }
      ++depth;
    } else if (is_unary(t->op)) {
      if (depth < 1) return E_INVAL;
    } else if (is_binary(t->op)) {
      if (depth < 2) return E_INVAL;
      --depth;
    } else {
      return E_INVAL;
    }
    if (depth > maxd) maxd = depth;
  }
  if (depth != 1) return E_INVAL;
  if (e.count > MAX_TOKS || maxd > MAX_DEPTH) return E_UNSUP;
  return 0;
}

static int check_access(const OModel* m, const OAccess* a) {
  int err = 0;
  if (a->array < 0 || a->array >= m->n_arrays) return E_INVAL;
  const OArray* arr = &m->arrays[a->array];
  if ((arr->space != SP_GLOBAL && arr->space != SP_SHARED) ||
      (arr->addr_bits != 32 && arr->addr_bits != 64) ||
      arr->alias < 0 || arr->alias >= (1 << 24)) return E_INVAL;
  if (a->kind < K_READ || a->kind > K_ATOMIC) return E_INVAL;
  if (a->scope != SC_BLOCK && a->scope != SC_DEVICE) return E_INVAL;
  if (a->n_loops < 0) return E_INVAL;
  /* the interface holds at most four enclosing loops; more is checked first */
  if (a->n_loops > MAX_LOOPS) return E_UNSUP;
  for (int i = 0; i < a->n_loops; ++i) {
    if (a->loops[i] < 0 || a->loops[i] >= m->n_loops || a->loops[i] >= 64) return E_INVAL;
    for (int j = 0; j < i; ++j) if (a->loops[j] == a->loops[i]) return E_INVAL;
  }
  if (a->addr.count == 0) return E_INVAL;
  const OSync* so[2] = {&a->acq, &a->rel};
  for (int k = 0; k < 2; ++k) {
    if (so[k]->addr.count == 0) continue;
    if (so[k]->array < 0 || so[k]->array >= m->n_arrays) return E_INVAL;
    if (so[k]->scope != SC_BLOCK && so[k]->scope != SC_DEVICE) return E_INVAL;
    err |= check_expr(m, so[k]->addr, 3, a);
  }
  err |= check_expr(m, a->addr, 3, a);
  err |= check_expr(m, a->guard, 3, a);
  err |= check_expr(m, a->bint, 2, a);
  err |= check_expr(m, a->wint, 2, a);
  for (int i = 0; i < a->n_loops; ++i) {
    const OLoop* l = &m->loops[a->loops[i]];
    if (l->init.count == 0 || l->bound.count == 0 || l->step.count == 0) return E_INVAL;
    if (l->cmp < 0 || l->cmp > 4 || l->upd < 0 || l->upd > 5) return E_INVAL;
    err |= check_expr(m, l->init, 1, a);
    err |= check_expr(m, l->bound, 1, a);
    err |= check_expr(m, l->step, 1, a);
  }
  if (err & E_INVAL) return E_INVAL;
  return err;
}

/* ------------------------------------------------------------------------ */
/* Enumerating the points of one access for one parameter tuple.            */

/* sa[k], sv[k]: memory and effective address of the point's syn() at
 * scope k (0 block, 1 device); sa[k] = -1: none. */
typedef struct {
  int64_t addr;
  uint32_t blin, tlin, ilin;
  uint16_t bint, wint;
  uint8_t side;
  int64_t sa[2];
  int64_t sv[2];
} OPoint;

typedef struct { OPoint* p; int64_t n, cap; } OPoints;

static void push_point(OPoints* v, OPoint pt) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 1024;
    v->p = (OPoint*)realloc(v->p, (size_t)v->cap * sizeof(OPoint));
  }
  v->p[v->n++] = pt;
}

/* Launch extents for one tuple.  Returns 0 if the domain is empty, 1 if not;
 * errors go to *err. */
static int launch_dims(const OModel* m, const int64_t* params, int64_t g[3], int64_t bd[3], int* err) {
  OEnv env;
  memset(&env, 0, sizeof env);
  env.params = params;
  int nonempty = 1;
  for (int d = 0; d < 3; ++d) {
    g[d] = eval(m, m->grid[d], &env, 1, err);
    bd[d] = eval(m, m->block[d], &env, 1, err);
    if (g[d] < 1 || bd[d] < 1) nonempty = 0;
  }
  if (!nonempty) return 0;
  int64_t nb = bd[0], ng = g[0];
  if (bd[0] > MAX_BLOCK || bd[1] > MAX_BLOCK || bd[2] > MAX_BLOCK) { *err |= E_UNSUP; return 0; }
  nb *= bd[1]; if (nb > MAX_BLOCK) { *err |= E_UNSUP; return 0; }
  nb *= bd[2]; if (nb > MAX_BLOCK) { *err |= E_UNSUP; return 0; }
  if (g[0] >= MAX_GRID || g[1] >= MAX_GRID || g[2] >= MAX_GRID) { *err |= E_UNSUP; return 0; }
  ng *= g[1]; if (ng >= MAX_GRID) { *err |= E_UNSUP; return 0; }
  ng *= g[2]; if (ng >= MAX_GRID) { *err |= E_UNSUP; return 0; }
  return 1;
}

static int cmp_holds(int cmp, int64_t v, int64_t bound) {
  switch (cmp) {
    case 0: return v < bound;
    case 1: return v <= bound;
    case 2: return v > bound;
    case 3: return v >= bound;
    default: return v != bound;
  }
}

static const int UPD_OP[6] = { O_ADD, O_SUB, O_MUL, O_DIV, O_SHL, O_SHR };

/* Value list of one loop for one tuple.  Returns the count (or -1 on error,
 * with the error recorded). */
static int64_t loop_values(const OModel* m, const OLoop* l, const int64_t* params,
                           const int64_t g[3], const int64_t bd[3], int64_t* out, int* err) {
  OEnv env;
  memset(&env, 0, sizeof env);
  env.params = params;
  for (int d = 0; d < 3; ++d) { env.gdim[d] = g[d]; env.bdim[d] = bd[d]; }
  int e = 0;
  int64_t v = eval(m, l->init, &env, 0, &e);
  int64_t bound = eval(m, l->bound, &env, 0, &e);
  int64_t step = eval(m, l->step, &env, 0, &e);
  if (e) { *err |= e; return -1; }
  int64_t n = 0;
  while (cmp_holds(l->cmp, v, bound)) {
    if (n == MAX_ITERS) { *err |= E_UNSUP; return -1; }
    out[n++] = v;
    int ue = 0;
    v = op_bin(UPD_OP[l->upd], v, step, &ue);
    if (ue) { *err |= ue; return -1; }
  }
  return n;
}

/* Memory identity of an array: its own, or the aliased memory of its views
 * (same alias id and space). */
static int64_t memory_id(const OModel* m, int32_t array) {
  const OArray* a = &m->arrays[array];
  if (!a->alias) return array;
  return ((int64_t)1 << 40) | ((int64_t)a->space << 32) | a->alias;
}

/* Effective address in the array's memory: base + address for a view. */
static int64_t effective(const OModel* m, int32_t array, int64_t addr, int* err) {
  const OArray* a = &m->arrays[array];
  if (!a->alias || !a->base) return addr;
  int64_t r;
  if (__builtin_add_overflow(addr, a->base, &r)) { *err |= E_RANGE; return 0; }
  return r;
}

/* syn() of Figures 9 and 10 at one point for required scope `scope`:
 * the acquire and release count only when their scope is at least as wide.
 * acqv, relv: their addresses at this point. */
static void syn_at(const OModel* m, const OAccess* a, int64_t acqv, int64_t relv,
                   int scope, int64_t* mem, int64_t* val) {
  int have_a = a->acq.addr.count && a->acq.scope >= scope;
  int have_r = a->rel.addr.count && a->rel.scope >= scope;
  int32_t arr = -1;
  *val = 0;
  if (have_a && have_r && memory_id(m, a->acq.array) == memory_id(m, a->rel.array) &&
      acqv == relv) {
    arr = a->acq.array;  /* lock: acquire and release on one address */
    *val = acqv;
  } else if (a->kind == K_WRITE && have_r) {
    arr = a->rel.array;  /* producer */
    *val = relv;
  } else if (a->kind == K_READ && have_a) {
    arr = a->acq.array;  /* consumer */
    *val = acqv;
  }
  /* shared memory is one per block: such a lock or flag never orders two
   * blocks, and device scope is only asked for inter-block conflicts */
  if (scope == SC_DEVICE && arr >= 0 && m->arrays[arr].space == SP_SHARED) arr = -1;
  *mem = arr >= 0 ? memory_id(m, arr) : -1;
}

/* All points of access a under tuple s, in lexicographic (blin, tlin, ilin)
 * order.  Returns the box size (points before guards) and appends the points
 * whose guard holds. */
static int64_t enumerate(const OModel* m, const OAccess* a, int32_t s, int side,
                         OPoints* out, int* err) {
  const int64_t* params = m->sets + (int64_t)s * m->n_params;
  int64_t g[3], bd[3];
  if (!launch_dims(m, params, g, bd, err)) return 0;
  /* loop value lists */
  int64_t* vals[MAX_LOOPS];
  int64_t nv[MAX_LOOPS];
  int64_t niota = 1;
  int ok = 1;
  for (int i = 0; i < a->n_loops; ++i) vals[i] = NULL;
  for (int i = 0; i < a->n_loops; ++i) {
    vals[i] = (int64_t*)malloc(sizeof(int64_t) * MAX_ITERS);
    nv[i] = loop_values(m, &m->loops[a->loops[i]], params, g, bd, vals[i], err);
    if (nv[i] < 0) { ok = 0; break; }
    niota *= nv[i];
    if (niota > MAX_ITERS) { *err |= E_UNSUP; ok = 0; break; }
  }
  int64_t nblk = g[0] * g[1] * g[2], nthr = bd[0] * bd[1] * bd[2];
  int64_t box = 0;
  if (ok) {
    box = nblk * nthr * niota;
    if (box >= MAX_POINTS) { *err |= E_UNSUP; ok = 0; box = 0; }
  }
  if (ok && niota > 0) {
    OEnv env;
    memset(&env, 0, sizeof env);
    env.params = params;
    for (int d = 0; d < 3; ++d) { env.gdim[d] = g[d]; env.bdim[d] = bd[d]; }
    int is32 = m->arrays[a->array].addr_bits == 32;
    for (int64_t bl = 0; bl < nblk; ++bl) {
      env.bid[0] = bl % g[0];
      env.bid[1] = (bl / g[0]) % g[1];
      env.bid[2] = bl / (g[0] * g[1]);
      for (int64_t tl = 0; tl < nthr; ++tl) {
        env.tid[0] = tl % bd[0];
        env.tid[1] = (tl / bd[0]) % bd[1];
        env.tid[2] = tl / (bd[0] * bd[1]);
        for (int64_t il = 0; il < niota; ++il) {
          /* row-major: the first (outermost) loop is most significant */
          int64_t rem = il;
          for (int i = a->n_loops - 1; i >= 0; --i) {
            env.loopval[a->loops[i]] = vals[i][rem % nv[i]];
            rem /= nv[i];
          }
          int64_t guard = eval(m, a->guard, &env, 1, err);
          if (guard == 0) continue;
          int e = 0;
          int64_t addr = effective(m, a->array, eval(m, a->addr, &env, 0, &e), &e);
          int64_t bi = eval(m, a->bint, &env, 0, &e);
          int64_t wi = eval(m, a->wint, &env, 0, &e);
          int64_t sval[2] = {0, 0};
          const OSync* so[2] = {&a->acq, &a->rel};
          for (int k = 0; k < 2; ++k) {
            if (so[k]->addr.count == 0) continue;
            sval[k] = effective(m, so[k]->array, eval(m, so[k]->addr, &env, 0, &e), &e);
            if (m->arrays[so[k]->array].addr_bits == 32 &&
                (sval[k] < INT32_MIN || sval[k] > INT32_MAX)) e |= E_RANGE;
          }
          if (is32 && (addr < INT32_MIN || addr > INT32_MAX)) e |= E_RANGE;
          if (bi < 0 || bi >= INTERVAL_LIMIT || wi < 0 || wi >= INTERVAL_LIMIT) e |= E_UNSUP;
          *err |= e;
          if (e) continue;
          OPoint pt;
          pt.addr = addr;
          pt.blin = (uint32_t)bl;
          pt.tlin = (uint32_t)tl;
          pt.ilin = (uint32_t)il;
          pt.bint = (uint16_t)bi;
          pt.wint = (uint16_t)wi;
          pt.side = (uint8_t)side;
          for (int k = 0; k < 2; ++k) syn_at(m, a, sval[0], sval[1], k, &pt.sa[k], &pt.sv[k]);
          push_point(out, pt);
        }
      }
    }
  }
  for (int i = 0; i < a->n_loops; ++i) free(vals[i]);
  return box;
}

/* ------------------------------------------------------------------------ */
/* Mask of classes to check (section 6.1; appendix A.2).                    */

static int class_mask(const OModel* m, const OAccess* x, const OAccess* y, int caller) {
  int mask = caller & 7;
  if (x->kind == K_READ && y->kind == K_READ) return 0;
  if (x->kind == K_ATOMIC && y->kind == K_ATOMIC) {
    if (x->scope == SC_DEVICE && y->scope == SC_DEVICE) return 0;
    mask &= C_INTER;
  }
  if (m->arrays[x->array].space == SP_SHARED) mask &= ~C_INTER;
  return mask;
}

/* Class of a conflicting point pair, or 0 if the pair does not conflict
 * (Table 2 plus the barrier-interval conditions). */
static int conflict_class(const OPoint* p, const OPoint* q, int64_t warp, int mask) {
  if (p->blin == q->blin && p->tlin == q->tlin) return 0;   /* same thread */
  if (p->addr != q->addr) return 0;
  int cls;
  if (p->blin != q->blin) cls = C_INTER;
  else if ((int64_t)p->tlin / warp == (int64_t)q->tlin / warp) cls = C_WARP;
  else cls = C_BLOCK;
  if (!(cls & mask)) return 0;
  if (cls == C_BLOCK && p->bint != q->bint) return 0;
  if (cls == C_WARP && (p->bint != q->bint || p->wint != q->wint)) return 0;
  /* Table 2: a race also needs addr(syn(Ai)) != addr(syn(Aj)); the scope
   * asked of syn() is device for inter-block, block otherwise (app. A) */
  int k = cls == C_INTER ? SC_DEVICE : SC_BLOCK;
  if (p->sa[k] >= 0 && p->sa[k] == q->sa[k] && p->sv[k] == q->sv[k]) return 0;
  return cls;
}

static int status_of(int err) {
  if (err & E_INVAL) return ST_INVAL;
  if (err & E_UNSUP) return ST_UNSUP;
  if (err & E_DIVZERO) return ST_DIVZERO;
  if (err & E_RANGE) return ST_RANGE;
  return ST_OK;
}

static void clear_result(OResult* r) {
  memset(r, 0, sizeof *r);
  r->w_set = r->w_b1 = r->w_t1 = r->w_i1 = r->w_b2 = r->w_t2 = r->w_i2 = -1;
}

static int class_index(int cls) { return cls == C_INTER ? 0 : cls == C_BLOCK ? 1 : 2; }

/* ------------------------------------------------------------------------ */
/* Oracle-A: the definition as a double loop.                               */

static void pair_a(const OModel* m, const OAccess* x, const OAccess* y, int self,
                   int mask, OResult* r, int* err) {
  int found = 0;
  for (int32_t s = 0; s < m->n_sets; ++s) {
    OPoints di = {0}, dj = {0};
    int64_t boxi = enumerate(m, x, s, 0, &di, err);
    int64_t boxj = boxi;
    if (!self) boxj = enumerate(m, y, s, 1, &dj, err);
    r->evals += (uint64_t)boxi + (uint64_t)boxj;
    const OPoints* pj = self ? &di : &dj;
    /* after an error only the remaining error bits matter: keep enumerating */
    if (!*err) {
      for (int64_t i = 0; i < di.n; ++i) {
        for (int64_t j = 0; j < pj->n; ++j) {
          int cls = conflict_class(&di.p[i], &pj->p[j], m->warp, mask);
          if (!cls) continue;
          r->by_class[class_index(cls)] += 1;
          if (!found) {  /* first in (s, p, q) lexicographic order */
            found = 1;
            r->w_set = s;
            r->w_b1 = di.p[i].blin; r->w_t1 = di.p[i].tlin; r->w_i1 = di.p[i].ilin;
            r->w_b2 = pj->p[j].blin; r->w_t2 = pj->p[j].tlin; r->w_i2 = pj->p[j].ilin;
            r->w_addr = di.p[i].addr;
            r->witness_class = cls;
          }
        }
      }
    }
    free(di.p);
    free(dj.p);
  }
}

/* ------------------------------------------------------------------------ */
/* Oracle-B: sort by (addr, block, bint, warp, wint, thread), count pairs    */
/* with equal key prefixes.                                                  */

static __thread int64_t t_warp; /* qsort has no context argument */

static int key_cmp_level(const OPoint* a, const OPoint* b, int64_t warp, int level) {
  if (a->addr != b->addr) return a->addr < b->addr ? -1 : 1;
  if (level == 0) return 0;
  if (a->blin != b->blin) return a->blin < b->blin ? -1 : 1;
  if (level == 1) return 0;
  if (a->bint != b->bint) return a->bint < b->bint ? -1 : 1;
  if (level == 2) return 0;
  int64_t wa = a->tlin / warp, wb = b->tlin / warp;
  if (wa != wb) return wa < wb ? -1 : 1;
  if (level == 3) return 0;
  if (a->wint != b->wint) return a->wint < b->wint ? -1 : 1;
  if (level == 4) return 0;
  if (a->tlin != b->tlin) return a->tlin < b->tlin ? -1 : 1;
  return 0;
}

static int full_cmp(const void* pa, const void* pb) {
  return key_cmp_level((const OPoint*)pa, (const OPoint*)pb, t_warp, 5);
}

/* order of point indices by (level key, syn() array and address at scope
 * t_scope), for the synchronised group sums */
static __thread const OPoint* t_pts;
static __thread int t_level, t_scope;

static int sync_cmp(const void* pa, const void* pb) {
  const OPoint* a = &t_pts[*(const int64_t*)pa];
  const OPoint* b = &t_pts[*(const int64_t*)pb];
  int c = key_cmp_level(a, b, t_warp, t_level);
  if (c) return c;
  if (a->sa[t_scope] != b->sa[t_scope]) return a->sa[t_scope] < b->sa[t_scope] ? -1 : 1;
  if (a->sv[t_scope] != b->sv[t_scope]) return a->sv[t_scope] < b->sv[t_scope] ? -1 : 1;
  return 0;
}

/* lexicographic point order (blin, tlin, ilin) */
static int point_less(const OPoint* a, const OPoint* b) {
  if (a->blin != b->blin) return a->blin < b->blin;
  if (a->tlin != b->tlin) return a->tlin < b->tlin;
  return a->ilin < b->ilin;
}

static void pair_b(const OModel* m, const OAccess* x, const OAccess* y, int self,
                   int mask, OResult* r, int* err) {
  int have_p = 0;
  int32_t ps = -1;
  OPoint pstar;
  memset(&pstar, 0, sizeof pstar);
  for (int32_t s = 0; s < m->n_sets; ++s) {
    OPoints d = {0};
    int64_t boxi = enumerate(m, x, s, 0, &d, err);
    int64_t boxj = self ? boxi : enumerate(m, y, s, 1, &d, err);
    r->evals += (uint64_t)boxi + (uint64_t)boxj;
    /* after an error only the remaining error bits matter: keep enumerating */
    if (*err) { free(d.p); continue; }
    t_warp = m->warp;
    qsort(d.p, (size_t)d.n, sizeof(OPoint), full_cmp);
    /* per level, group sums of n_i * n_j; side-j counts per record */
    int64_t n = d.n;
    uint64_t S[6] = {0, 0, 0, 0, 0, 0};
    uint64_t* partners = (uint64_t*)calloc((size_t)(n ? n : 1), sizeof(uint64_t));
    for (int level = 0; level < 6; ++level) {
      int64_t g0 = 0;
      while (g0 < n) {
        int64_t g1 = g0 + 1;
        while (g1 < n && key_cmp_level(&d.p[g0], &d.p[g1], m->warp, level) == 0) ++g1;
        uint64_t c0 = 0, c1 = 0;
        for (int64_t k = g0; k < g1; ++k) { if (d.p[k].side == 0) ++c0; else ++c1; }
        uint64_t nj = self ? c0 : c1;   /* partners on the j side */
        S[level] += c0 * nj;
        /* levels 0,2,4 add, 1,3,5 subtract; only classes in the mask */
        int cls = level < 2 ? C_INTER : level < 4 ? C_BLOCK : C_WARP;
        if (cls & mask) {
          for (int64_t k = g0; k < g1; ++k) {
            if (d.p[k].side != 0) continue;
            if (level % 2 == 0) partners[k] += nj; else partners[k] -= nj;
          }
        }
        g0 = g1;
      }
    }
    /* synchronised pairs: the same group sums over the points whose syn()
     * reaches the class's scope, with the synchronisation array and address
     * added to the key; they are subtracted from the counts and partners */
    uint64_t T[6] = {0, 0, 0, 0, 0, 0};
    int64_t* ix = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int level = 0; level < 6; ++level) {
      int cls = level < 2 ? C_INTER : level < 4 ? C_BLOCK : C_WARP;
      if (!(cls & mask)) continue;
      int k = cls == C_INTER ? SC_DEVICE : SC_BLOCK;
      int64_t ns = 0;
      for (int64_t i = 0; i < n; ++i) if (d.p[i].sa[k] >= 0) ix[ns++] = i;
      t_pts = d.p;
      t_level = level;
      t_scope = k;
      qsort(ix, (size_t)ns, sizeof(int64_t), sync_cmp);
      int64_t g0 = 0;
      while (g0 < ns) {
        int64_t g1 = g0 + 1;
        while (g1 < ns && sync_cmp(&ix[g0], &ix[g1]) == 0) ++g1;
        uint64_t c0 = 0, c1 = 0;
        for (int64_t x = g0; x < g1; ++x) { if (d.p[ix[x]].side == 0) ++c0; else ++c1; }
        uint64_t nj = self ? c0 : c1;
        T[level] += c0 * nj;
        for (int64_t x = g0; x < g1; ++x) {
          if (d.p[ix[x]].side != 0) continue;
          if (level % 2 == 0) partners[ix[x]] -= nj; else partners[ix[x]] += nj;
        }
        g0 = g1;
      }
    }
    free(ix);
    if (mask & C_INTER) r->by_class[0] += (S[0] - S[1]) - (T[0] - T[1]);
    if (mask & C_BLOCK) r->by_class[1] += (S[2] - S[3]) - (T[2] - T[3]);
    if (mask & C_WARP) r->by_class[2] += (S[4] - S[5]) - (T[4] - T[5]);
    /* witness pass 1: smallest p (in this tuple) with a partner */
    if (!have_p) {
      for (int64_t k = 0; k < n; ++k) {
        if (d.p[k].side != 0 || partners[k] == 0) continue;
        if (!have_p || point_less(&d.p[k], &pstar)) { pstar = d.p[k]; have_p = 1; ps = s; }
      }
      if (have_p) {
        /* witness pass 2: smallest q of this tuple that conflicts with p* */
        int haveq = 0;
        OPoint qstar;
        int qcls = 0;
        memset(&qstar, 0, sizeof qstar);
        for (int64_t k = 0; k < n; ++k) {
          if (!self && d.p[k].side != 1) continue;
          int cls = conflict_class(&pstar, &d.p[k], m->warp, mask);
          if (!cls) continue;
          if (!haveq || point_less(&d.p[k], &qstar)) { qstar = d.p[k]; haveq = 1; qcls = cls; }
        }
        r->w_set = ps;
        r->w_b1 = pstar.blin; r->w_t1 = pstar.tlin; r->w_i1 = pstar.ilin;
        r->w_b2 = qstar.blin; r->w_t2 = qstar.tlin; r->w_i2 = qstar.ilin;
        r->w_addr = pstar.addr;
        r->witness_class = qcls;
      }
    }
    free(partners);
    free(d.p);
  }
}

/* ------------------------------------------------------------------------ */

static void check_one(const OModel* models, int32_t n_models, const OPair* pr,
                      int method, OResult* r) {
  clear_result(r);
  if (pr->model < 0 || pr->model >= n_models) { r->status = ST_INVAL; return; }
  const OModel* m = &models[pr->model];
  if (pr->a < 0 || pr->a >= m->n_acc || pr->b < 0 || pr->b >= m->n_acc) { r->status = ST_INVAL; return; }
  const OAccess* x = &m->acc[pr->a];
  const OAccess* y = &m->acc[pr->b];
  int err = 0;
  err |= check_access(m, x);
  err |= check_access(m, y);
  if (!(err & E_INVAL)) {
    /* one memory: the same array or two views of one aliased memory */
    if (x->array != y->array && memory_id(m, x->array) != memory_id(m, y->array))
      err |= E_INVAL;
    if (m->warp < 1 || m->warp > 1024) err |= E_INVAL;
    if (m->n_sets < 0) err |= E_INVAL;
    for (int d = 0; d < 3; ++d) {
      err |= check_expr(m, m->grid[d], 0, NULL);
      err |= check_expr(m, m->block[d], 0, NULL);
    }
    if (m->n_sets > MAX_SETS) err |= E_UNSUP;
  }
  if (err) { r->status = status_of(err); return; }
  int mask = class_mask(m, x, y, pr->mask);
  if (mask == 0) { r->flags |= 1; return; }
  int self = (pr->a == pr->b);
  if (method == 0) pair_a(m, x, y, self, mask, r, &err);
  else pair_b(m, x, y, self, mask, r, &err);
  if (err) {
    uint64_t ev = r->evals;
    clear_result(r);
    r->status = status_of(err);
    r->evals = ev;
    return;
  }
  r->count = r->by_class[0] + r->by_class[1] + r->by_class[2];
  r->verdict = r->count != 0;
  r->classes = (r->by_class[0] ? C_INTER : 0) | (r->by_class[1] ? C_BLOCK : 0) |
               (r->by_class[2] ? C_WARP : 0);
  if (!r->verdict) {
    r->w_set = r->w_b1 = r->w_t1 = r->w_i1 = r->w_b2 = r->w_t2 = r->w_i2 = -1;
    r->w_addr = 0;
    r->witness_class = 0;
  }
}

typedef struct {
  const OModel* models; int32_t n_models;
  const OPair* pairs; int32_t n_pairs;
  int method;
  OResult* out;
  int64_t next;
  pthread_mutex_t mu;
} OJob;

static void* worker(void* arg) {
  OJob* j = (OJob*)arg;
  for (;;) {
    pthread_mutex_lock(&j->mu);
    int64_t k = j->next++;
    pthread_mutex_unlock(&j->mu);
    if (k >= j->n_pairs) break;
    check_one(j->models, j->n_models, &j->pairs[k], j->method, &j->out[k]);
  }
  return NULL;
}

/* Public entry: check n_pairs pairs with `method` (0 = A, 1 = B) on
 * n_threads host threads.  Returns the number of threads used. */
int oracle_check_pairs(const OModel* models, int32_t n_models, const OPair* pairs,
                       int32_t n_pairs, int32_t method, int32_t n_threads, OResult* out) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > n_pairs) n_threads = n_pairs > 0 ? n_pairs : 1;
  OJob job;
  job.models = models; job.n_models = n_models;
  job.pairs = pairs; job.n_pairs = n_pairs;
  job.method = method; job.out = out; job.next = 0;
  pthread_mutex_init(&job.mu, NULL);
  if (n_threads == 1) {
    worker(&job);
  } else {
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, worker, &job);
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th);
  }
  pthread_mutex_destroy(&job.mu);
  return n_threads;
}

/* Expression evaluation on its own, for the integer-semantics tests:
 * evaluates a parameter-only expression (ctx 0) of model m with tuple s.
 * Returns the value; *err_out gets the error bits. */
int64_t oracle_eval_uniform(const OModel* m, OExpr e, int32_t s, int32_t* err_out) {
  OEnv env;
  memset(&env, 0, sizeof env);
  env.params = m->sets + (int64_t)s * m->n_params;
  int err = 0;
  int64_t v = eval(m, e, &env, 0, &err);
  *err_out = err;
  return v;
}

/* Oracle conflict predicate on explicit point data, used to re-check
 * witnesses reported by other code paths. */
int oracle_conflict_class(int64_t addr_p, uint32_t b_p, uint32_t t_p, uint32_t bint_p, uint32_t wint_p,
                          int64_t addr_q, uint32_t b_q, uint32_t t_q, uint32_t bint_q, uint32_t wint_q,
                          int64_t warp, int32_t mask) {
  OPoint p, q;
  memset(&p, 0, sizeof p); memset(&q, 0, sizeof q);
  p.sa[0] = p.sa[1] = q.sa[0] = q.sa[1] = -1;  /* no synchronisation */
  p.addr = addr_p; p.blin = b_p; p.tlin = t_p; p.bint = (uint16_t)bint_p; p.wint = (uint16_t)wint_p;
  q.addr = addr_q; q.blin = b_q; q.tlin = t_q; q.bint = (uint16_t)bint_q; q.wint = (uint16_t)wint_q;
  return conflict_class(&p, &q, warp, mask);
}
