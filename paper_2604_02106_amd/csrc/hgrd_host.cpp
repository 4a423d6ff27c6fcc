// Host side of the exact per-access-pair race query: argument validation,
// class masks (section 6.1, appendix A.2), evaluation of the uniform parts
// of a model (launch extents, loop value lists; section 6.3 classes 2 and
// 4), compilation of address/guard/interval expressions to device code,
// work planning, launches, and results.
//
// Work planning.  A query (one access pair) under one parameter tuple has
// |D_a| + |D_b| launch-box points.  When they fit one workgroup's LDS the
// workgroup generates and joins them itself (for shared-memory arrays, per
// block range: shared memory belongs to one block).  Larger ones are
// generated once and scattered into fixed-capacity HBM buckets by an
// address hash, then each bucket is joined in LDS.  Buckets that overflow
// (many points on few addresses) send their query through an HBM hash
// aggregation instead.  The lexicographically smallest witness is found in
// two passes: the smallest p with a partner comes out of the joins, then
// one pass over the other access finds the smallest partner q.
#include "../../include/hgrd.h"
#include "hgrd_internal.h"
#include "hgrd_launch.h"
#include "hgrd_hostops.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <memory>
#include <thread>
#include <string>
#include <vector>

using namespace hgrd;
using u64 = unsigned long long;

namespace {

constexpr uint32_t kMaxInsns = 256;
constexpr uint32_t kMaxDepth = 16;
constexpr uint32_t kMaxLoopsPerAccess = 4;
constexpr uint32_t kMaxIters = 65536;
constexpr uint32_t kMaxSets = 4096;
constexpr int64_t kMaxBlock = 1024;
constexpr int64_t kMaxGrid = 1ll << 26;
constexpr int64_t kMaxPoints = 1ll << 31;
constexpr uint32_t kChunkPts = 1024;
constexpr uint32_t kL0ChunkPts = 8192;  // points per level-0 and fallback
                                        // generation workgroup
constexpr uint64_t kWaveBytes = 3072ull << 20;  // bucket bytes per partition wave
constexpr uint64_t kFallbackRecords = 256ull << 20;
constexpr uint64_t kMaxTabInst = 1ull << 24;  // table entries per instance
constexpr uint64_t kMaxTabPool = 1ull << 33;  // table entries per plan (64 GiB)
constexpr uint64_t kL0Slots = 1ull << 29;     // address-count slots per split batch
constexpr uint64_t kRetryBytes = 16ull << 30;  // bucket bytes of one retried item

bool is_leaf(uint16_t op) { return op >= RD_OP_CONST && op <= RD_OP_LOOP; }
bool is_binary(uint16_t op) { return op >= RD_OP_ADD && op <= RD_OP_LOR; }
bool is_unary(uint16_t op) { return op == RD_OP_NEG || op == RD_OP_LNOT; }

// where leaves may appear
enum Ctx { CTX_LAUNCH = 0, CTX_LOOP = 1, CTX_IV = 2, CTX_POINT = 3 };

int loop_pos(const rd_access* a, uint32_t loop) {
  if (!a) return -1;
  for (uint32_t i = 0; i < a->n_loops && i < 8; ++i)
    if (a->loops[i] == loop) return (int)i;
  return -1;
}

// Structural check: ERR_INVAL for malformed, ERR_UNSUP for over-limit.
uint32_t check_expr(const rd_kernel_model& m, rd_expr e, int ctx,
                    const rd_access* a) {
  if (e.count == 0) return 0;
  if ((uint64_t)e.first + e.count > m.n_insns || !m.insns) return ERR_INVAL;
  uint32_t depth = 0, maxd = 0;
  for (uint32_t k = 0; k < e.count; ++k) {
    const rd_insn& t = m.insns[e.first + k];
    if (is_leaf(t.op)) {
      switch (t.op) {
        case RD_OP_CONST: break;
        case RD_OP_PARAM:
          if (t.arg >= m.n_params) return ERR_INVAL;
          break;
        case RD_OP_BDIM:
        case RD_OP_GDIM:
          if (ctx < CTX_LOOP || t.arg > 2) return ERR_INVAL;
          break;
        case RD_OP_TID:
        case RD_OP_BID:
          if (ctx < CTX_POINT || t.arg > 2) return ERR_INVAL;
          break;
        case RD_OP_LOOP:
          if (ctx < CTX_IV || loop_pos(a, t.arg) < 0) return ERR_INVAL;
          break;
      }
      ++depth;
    } else if (is_unary(t.op)) {
      if (depth < 1) return ERR_INVAL;
    } else if (is_binary(t.op)) {
      if (depth < 2) return ERR_INVAL;
      --depth;
    } else {
      return ERR_INVAL;
    }
    maxd = std::max(maxd, depth);
  }
  if (depth != 1) return ERR_INVAL;
  if (e.count > kMaxInsns || maxd > kMaxDepth) return ERR_UNSUP;
  return 0;
}

uint32_t syn_flags(const rd_kernel_model& m, const rd_access& a);

// The memory an array belongs to: its own (the array index) or the memory
// its alias id names, shared by every view with that id and space.
int64_t memory_of(const rd_kernel_model& m, uint32_t array) {
  const rd_array& a = m.arrays[array];
  if (!a.alias) return array;
  return ((int64_t)1 << 40) | ((int64_t)a.space << 32) | a.alias;
}

// Models with the effective addresses of aliased views: an access address
// (or an acquire's or release's) on a view with a nonzero base becomes
// base + address, appended to a copy of the model's instruction pool.  The
// base is an immediate operand, so the device program takes no extra
// register.  Expressions are validated on the caller's models.
struct ModelViews {
  std::vector<std::vector<rd_insn>> insns;
  std::vector<std::vector<rd_access>> acc;
  std::vector<rd_kernel_model> m;
};
void build_views(const rd_kernel_model* models, uint32_t n, ModelViews& V) {
  V.m.assign(models, models + n);
  V.insns.resize(n);
  V.acc.resize(n);
  for (uint32_t i = 0; i < n; ++i) {
    const rd_kernel_model& M = models[i];
    bool any = false;
    for (uint32_t k = 0; M.arrays && k < M.n_arrays; ++k)
      any |= M.arrays[k].alias != 0 && M.arrays[k].base != 0;
    if (!any || (M.n_acc && !M.acc) || (M.n_insns && !M.insns)) continue;
    V.insns[i].assign(M.insns, M.insns + M.n_insns);
    V.acc[i].assign(M.acc, M.acc + M.n_acc);
    auto shift = [&](rd_expr& e, uint32_t arr) {
      if (arr >= M.n_arrays || e.count == 0 || (uint64_t)e.first + e.count > M.n_insns) return;
      const rd_array& A = M.arrays[arr];
      if (!A.alias || !A.base) return;
      std::vector<rd_insn>& P = V.insns[i];
      const uint32_t first = (uint32_t)P.size();
      P.insert(P.end(), M.insns + e.first, M.insns + e.first + e.count);
      rd_insn c, add;
      memset(&c, 0, sizeof c);
      memset(&add, 0, sizeof add);
      c.op = RD_OP_CONST;
      c.imm = A.base;
      add.op = RD_OP_ADD;
      P.push_back(c);
      P.push_back(add);
      e.first = first;
      e.count += 2;
    };
    for (rd_access& A : V.acc[i]) {
      shift(A.addr, A.array);
      shift(A.acq.addr, A.acq.array);
      shift(A.rel.addr, A.rel.array);
    }
    V.m[i].insns = V.insns[i].data();
    V.m[i].n_insns = (uint32_t)V.insns[i].size();
    V.m[i].acc = V.acc[i].data();
  }
}

uint32_t check_access(const rd_kernel_model& m, const rd_access& a) {
  if (a.array >= m.n_arrays || !m.arrays) return ERR_INVAL;
  const rd_array& arr = m.arrays[a.array];
  if (arr.space > RD_SHARED || (arr.addr_bits != 32 && arr.addr_bits != 64) ||
      arr.alias >= (1u << 24))
    return ERR_INVAL;
  if (a.kind > RD_ATOMIC) return ERR_INVAL;
  if (a.scope > RD_SCOPE_DEVICE) return ERR_INVAL;
  if (a.n_loops > kMaxLoopsPerAccess) {
    return ERR_UNSUP;
  }
  for (uint32_t i = 0; i < a.n_loops; ++i) {
    if (a.loops[i] >= m.n_loops || !m.loops) return ERR_INVAL;
    for (uint32_t j = 0; j < i; ++j)
      if (a.loops[j] == a.loops[i]) return ERR_INVAL;
  }
  if (a.addr.count == 0) return ERR_INVAL;
  for (const rd_sync* y : {&a.acq, &a.rel}) {
    if (y->addr.count == 0) continue;
    if (y->array >= m.n_arrays || y->scope > RD_SCOPE_DEVICE) return ERR_INVAL;
  }
  uint32_t err = check_expr(m, a.acq.addr, CTX_POINT, &a) |
                 check_expr(m, a.rel.addr, CTX_POINT, &a) |
                 check_expr(m, a.addr, CTX_POINT, &a) |
                 check_expr(m, a.guard, CTX_POINT, &a) |
                 check_expr(m, a.bint, CTX_IV, &a) |
                 check_expr(m, a.wint, CTX_IV, &a);
  for (uint32_t i = 0; i < a.n_loops; ++i) {
    const rd_loop& l = m.loops[a.loops[i]];
    if (!l.init.count || !l.bound.count || !l.step.count) return ERR_INVAL;
    if (l.cmp > RD_CMP_NE || l.upd > RD_UPD_SHR) return ERR_INVAL;
    err |= check_expr(m, l.init, CTX_LOOP, &a) |
           check_expr(m, l.bound, CTX_LOOP, &a) |
           check_expr(m, l.step, CTX_LOOP, &a);
  }
  return (err & ERR_INVAL) ? ERR_INVAL : err;
}

// Host evaluation of a uniform expression.  dims = {gx, gy, gz, bx, by, bz}.
int64_t heval(const rd_kernel_model& m, rd_expr e, const int64_t* params,
              const int64_t* dims, int64_t dflt, uint32_t& err) {
  if (e.count == 0) return dflt;
  int64_t st[kMaxDepth + 1];
  int sp = 0;
  for (uint32_t k = 0; k < e.count; ++k) {
    const rd_insn& t = m.insns[e.first + k];
    switch (t.op) {
      case RD_OP_CONST: st[sp++] = t.imm; break;
      case RD_OP_PARAM: st[sp++] = params[t.arg]; break;
      case RD_OP_GDIM: st[sp++] = dims ? dims[t.arg] : 0; break;
      case RD_OP_BDIM: st[sp++] = dims ? dims[3 + t.arg] : 0; break;
      case RD_OP_NEG:
        if (st[sp - 1] == INT64_MIN) { err |= ERR_RANGE; st[sp - 1] = 0; }
        else st[sp - 1] = -st[sp - 1];
        break;
      case RD_OP_LNOT: st[sp - 1] = st[sp - 1] == 0; break;
      default: {
        int64_t b = st[--sp];
        st[sp - 1] = hop(t.op, st[sp - 1], b, err);
      }
    }
  }
  return st[0];
}

// Compiles a postfix expression to device three-address code.
// Leaves stay operand descriptors; only intermediate values take a stack
// register, so the register index of a value is its stack position.
Prog compile(const rd_kernel_model& m, rd_expr e, const rd_access& a,
             std::vector<DInsn>& pool) {
  Prog p;
  memset(&p, 0, sizeof p);
  if (e.count == 0) {
    p.absent = 1;
    return p;
  }
  p.off = (uint32_t)pool.size();
  struct Opnd {
    uint8_t mode;
    uint16_t idx;
    int64_t imm;
  };
  std::vector<Opnd> st;
  auto emit = [&](uint8_t op, uint8_t dst, Opnd x, Opnd y) {
    DInsn in;
    in.op = op;
    in.dst = dst;
    in.ma = x.mode;
    in.mb = y.mode;
    in.a = x.idx;
    in.b = y.idx;
    in.imm = x.mode == M_IMM ? x.imm : y.imm;
    pool.push_back(in);
  };
  static const uint8_t kBin[] = {D_ADD, D_SUB, D_MUL, D_DIV, D_MOD, D_SHL,
                                 D_SHR, D_AND, D_OR,  D_XOR, D_MIN, D_MAX,
                                 D_LT,  D_LE,  D_EQ,  D_NE,  D_GE,  D_GT,
                                 D_LAND, D_LOR};
  const uint16_t np = (uint16_t)m.n_params;
  for (uint32_t k = 0; k < e.count; ++k) {
    const rd_insn& t = m.insns[e.first + k];
    switch (t.op) {
      case RD_OP_CONST: st.push_back({M_IMM, 0, t.imm}); break;
      case RD_OP_PARAM: st.push_back({M_PARAM, t.arg, 0}); break;
      case RD_OP_GDIM: st.push_back({M_PARAM, (uint16_t)(np + t.arg), 0}); break;
      case RD_OP_BDIM: st.push_back({M_PARAM, (uint16_t)(np + 3 + t.arg), 0}); break;
      case RD_OP_TID: st.push_back({M_COORD, (uint16_t)(kCoordTid + t.arg), 0}); break;
      case RD_OP_BID: st.push_back({M_COORD, (uint16_t)(kCoordBid + t.arg), 0}); break;
      case RD_OP_LOOP:
        st.push_back({M_COORD, (uint16_t)(kCoordLoop + loop_pos(&a, t.arg)), 0});
        break;
      case RD_OP_NEG:
      case RD_OP_LNOT: {
        Opnd x = st.back();
        st.pop_back();
        uint8_t d = (uint8_t)st.size();
        emit(t.op == RD_OP_NEG ? D_NEG : D_LNOT, d, x, {M_IMM, 0, x.imm});
        st.push_back({M_REG, d, 0});
        break;
      }
      default: {
        Opnd y = st.back();
        st.pop_back();
        Opnd x = st.back();
        st.pop_back();
        uint8_t d = (uint8_t)st.size();
        if (x.mode == M_IMM && y.mode == M_IMM) {
          emit(D_MOV, d, x, x);
          x = {M_REG, d, 0};
        }
        emit(kBin[t.op - RD_OP_ADD], d, x, y);
        st.push_back({M_REG, d, 0});
      }
    }
  }
  Opnd r = st.back();
  if (r.mode != M_REG) {
    emit(D_MOV, 0, r, r);
    p.res = 0;
  } else {
    p.res = (uint8_t)r.idx;
  }
  p.n = (uint16_t)(pool.size() - p.off);
  return p;
}

// Host interpreter of compiled programs (same semantics as the device's).
static int64_t host_prog(const std::vector<DInsn>& code, const Prog& p,
                         const int64_t* coords, const int64_t* params,
                         int64_t dflt, uint32_t& err) {
  static const uint16_t kOp[] = {0, RD_OP_ADD, RD_OP_SUB, RD_OP_MUL, RD_OP_DIV,
                                 RD_OP_MOD, RD_OP_SHL, RD_OP_SHR, RD_OP_AND,
                                 RD_OP_OR, RD_OP_XOR, RD_OP_MIN, RD_OP_MAX,
                                 RD_OP_LT, RD_OP_LE, RD_OP_EQ, RD_OP_NE,
                                 RD_OP_GE, RD_OP_GT, RD_OP_LAND, RD_OP_LOR};
  if (p.absent) return dflt;
  int64_t st[kMaxStack];
  for (uint32_t k = 0; k < p.n; ++k) {
    const DInsn& in = code[p.off + k];
    auto opnd = [&](uint8_t mode, uint16_t i) -> int64_t {
      return mode == M_REG ? st[i] : mode == M_IMM ? in.imm
             : mode == M_PARAM ? params[i] : coords[i];
    };
    const int64_t a = opnd(in.ma, in.a), b = opnd(in.mb, in.b);
    int64_t r;
    if (in.op == D_MOV) r = a;
    else if (in.op == D_NEG) r = hop(RD_OP_SUB, 0, a, err);
    else if (in.op == D_LNOT) r = a == 0;
    else r = hop(kOp[in.op], a, b, err);
    st[in.dst] = r;
  }
  return st[p.res];
}

static void host_coords(const AccInst& I, const std::vector<int64_t>& loops,
                        uint32_t blin, uint32_t tlin, uint32_t ilin, int64_t* c) {
  c[0] = tlin % I.dims[3];
  c[1] = (tlin / I.dims[3]) % I.dims[4];
  c[2] = tlin / (I.dims[3] * I.dims[4]);
  c[3] = blin % I.dims[0];
  c[4] = (blin / I.dims[0]) % I.dims[1];
  c[5] = blin / (I.dims[0] * I.dims[1]);
  c[6] = c[7] = c[8] = c[9] = 0;
  uint32_t rem = ilin;
  for (int k = (int)I.n_loops - 1; k >= 0; --k) {
    c[6 + k] = loops[I.loop_off[k] + rem % I.loop_n[k]];
    rem /= I.loop_n[k];
  }
}

bool cmp_holds(uint32_t cmp, int64_t v, int64_t bound) {
  switch (cmp) {
    case RD_CMP_LT: return v < bound;
    case RD_CMP_LE: return v <= bound;
    case RD_CMP_GT: return v > bound;
    case RD_CMP_GE: return v >= bound;
    default: return v != bound;
  }
}

const uint16_t kUpdOp[] = {RD_OP_ADD, RD_OP_SUB, RD_OP_MUL, RD_OP_DIV,
                           RD_OP_SHL, RD_OP_SHR};

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool own = true;  // false: carved from a caller's arena, never freed here
};

// Caller-provided device memory handed out front to back (256-byte
// aligned).  Nothing is ever returned to it during a call; the caller
// resets `used` between calls.
struct Arena {
  unsigned char* base = nullptr;
  size_t cap = 0, used = 0;
};

// A named buffer of at least `bytes` from the arena: the one already
// carved under that name when it is large enough, else a new piece.
// RD_ECAPACITY (with a message naming the buffer) when the arena is full.
void* arena_buf(Arena& A, DevBuf& b, const char* name, size_t bytes, int* err) {
  if (bytes == 0) bytes = 256;
  if (b.p && b.cap >= bytes) return b.p;
  const size_t at = (A.used + 255) & ~(size_t)255;
  if (at > A.cap || bytes > A.cap - at) {
    fprintf(stderr,
            "hgrd: the fixed scratch area (%zu bytes) cannot hold '%s' (%zu bytes, "
            "%zu already in use)\n", A.cap, name, bytes, at);
    if (!*err) *err = RD_ECAPACITY;
    return nullptr;
  }
  b.p = A.base + at;
  b.cap = bytes;
  b.own = false;
  A.used = at + bytes;
  return b.p;
}

uint64_t next_prime(uint64_t n) {
  if (n <= 2) return 2;
  for (uint64_t c = n | 1;; c += 2) {
    bool prime = true;
    for (uint64_t d = 3; d * d <= c; d += 2)
      if (c % d == 0) {
        prime = false;
        break;
      }
    if (prime) return c;
  }
}

// Bucket map of an HBM item whose instances have term tables: the dense key
// ((addr - lo) >> shift) + blin * kb modulo a prime bucket count (mode 1),
// when the key stays below 2^32; else the hash (mode 0).  per_block: keys
// carry the block (shared arrays, split items).
void set_bucket_map(HItem& h, const std::vector<uint8_t>& tab_on,
                    const std::vector<std::pair<int64_t, int64_t>>& arange,
                    uint32_t nblk, bool self, bool per_block, uint64_t R,
                    uint32_t cap, double load) {
  h.mode = 0;
  h.kb = 0;
  h.lo = 0;
  h.fm = 0;
  __int128 lo = 0, hi = -1;
  bool first = true;
  (void)self;  // a self pair names its one instance twice
  for (uint32_t x : {h.inst_i, h.inst_j}) {
    if (!tab_on[x]) return;
    const auto& r = arange[x];
    if (first || r.first < lo) lo = r.first;
    if (first || r.second > hi) hi = r.second;
    first = false;
  }
  if (hi < lo || hi - lo >= ((__int128)1 << 62)) return;
  const __int128 kr = ((hi - lo) >> h.shift) + 1;
  const __int128 kmax = per_block ? kr * nblk : kr;
  if (kmax >= ((__int128)1 << 32)) return;
  uint64_t nb = (uint64_t)((double)R / (cap * load)) + 1;
  nb = nb <= 1 ? 1 : next_prime(nb);
  if (nb >= (1ull << 31)) return;
  h.mode = 1;
  h.lo = (long long)lo;
  h.kb = per_block ? (uint32_t)kr : 0;
  h.nbuckets = (uint32_t)nb;
  h.fm = ~0ull / nb + 1;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

// ---------------------------------------------------------------------------

struct rd_context {
  int device = 0;
  std::map<std::string, DevBuf> bufs;
  // While set (rd_check_pairs_noalloc), every device buffer of the context
  // and of its plans is carved from this arena instead of hipMalloc;
  // abufs names the arena's buffers and is emptied when the arena is unset.
  Arena* arena = nullptr;
  std::map<std::string, DevBuf> abufs;
  // Partition scratch (bucket records, bucket cursors, filter marks) that
  // every plan of the context shares: plans run one at a time on a
  // context, so one buffer serves them all.  A buffer that must grow is
  // retired, not freed, while plans (and their captured graphs) may still
  // hold its address; retired buffers go with the context.
  std::map<std::string, DevBuf> shared;
  std::vector<void*> retired;
  void* shared_buf(const char* name, size_t bytes, int* err) {
    DevBuf& b = shared[name];
    if (bytes == 0) bytes = 256;
    if (b.cap >= bytes) return b.p;
    if (b.p) retired.push_back(b.p);
    b.p = nullptr;
    b.cap = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      fprintf(stderr, "hgrd: device allocation of %zu bytes for '%s' failed\n", bytes, name);
      b.p = nullptr;
      *err = RD_ENOMEM;
      return nullptr;
    }
    b.cap = bytes;
    return b.p;
  }
  rd_stats stats;
  int cfg = 0;  // LDS tile shape: 1024 records, 2048 slots (rd_autotune may change it)
  uint32_t n_cu = 256;
  uint64_t wave_bytes = kWaveBytes;  // default partition wave size
  hipStream_t stream = nullptr;  // used when the caller passes no stream
  hipEvent_t ev[16];
  std::vector<hipEvent_t> wev;    // per-wave timing events
  void* ensure(const char* name, size_t bytes, int* err) {
    if (arena) return arena_buf(*arena, abufs[name], name, bytes, err);
    DevBuf& b = bufs[name];
    if (bytes == 0) bytes = 256;
    if (b.cap < bytes) {
      if (b.p) (void)hipFree(b.p);
      b.p = nullptr;
      size_t want = std::max(bytes, b.cap + b.cap / 2);
      if (hipMalloc(&b.p, want) != hipSuccess) {
        b.cap = 0;
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
          (void)hipGetLastError();
          fprintf(stderr, "hgrd: device allocation of %zu bytes for '%s' failed\n", bytes,
                  name);
          b.p = nullptr;
          *err = RD_ENOMEM;
          return nullptr;
        }
        want = bytes;
      }
      b.cap = want;
    }
    return b.p;
  }
};

namespace {

// Per (model, tuple): launch extents.
// ---------------------------------------------------------------------------
// Term tables (lowering of one access under one tuple).
//
// An expression qualifies when interval bounds over the launch box prove
// that no operation in it can fail (overflow, zero divisor, shift count,
// INT64_MIN / -1), so the interpreter would never flag an error for it.
// It is then rewritten, in exact integer arithmetic, as a uniform constant
// plus a sum of terms that each depend on one coordinate group only (block
// ids, thread ids or loop values): sums and differences split, products
// and left shifts by uniform values distribute, and a truncating division
// or remainder by a positive uniform d splits when every term but those of
// one group is a multiple of d and both parts are non-negative.  Each
// group's terms are tabulated over the group's linear index.

using i128 = __int128;
constexpr i128 kI64Lo = INT64_MIN, kI64Hi = INT64_MAX;

struct TNode {
  uint16_t op = 0, arg = 0;
  int64_t imm = 0;
  int kid[2] = {-1, -1};
  uint32_t start = 0;   // first postfix index of the subtree
  uint8_t groups = 0;   // bit 0 blocks, bit 1 threads, bit 2 loop values
  int64_t val = 0;      // value of a uniform node
  i128 lo = 0, hi = 0;  // value range over the box
  uint64_t g = 1;       // every value of the node is a multiple of g (0: always 0)
};

inline uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}
inline uint64_t uabs64(int64_t v) { return v < 0 ? 0 - (uint64_t)v : (uint64_t)v; }
// product of two divisors, 1 (always a divisor) when it does not fit
inline uint64_t gmul(uint64_t a, uint64_t b) {
  const unsigned __int128 p = (unsigned __int128)a * b;
  return p >> 62 ? 1 : (uint64_t)p;
}

inline bool fits64(i128 v) { return v >= kI64Lo && v <= kI64Hi; }
inline i128 i128abs(i128 v) { return v < 0 ? -v : v; }

// Range of `op` over operand ranges; false if the operation may fail.
bool range_op(uint16_t op, i128 al, i128 ah, i128 bl, i128 bh, i128& lo, i128& hi) {
  auto corners = [&](i128 c0, i128 c1, i128 c2, i128 c3) {
    lo = std::min(std::min(c0, c1), std::min(c2, c3));
    hi = std::max(std::max(c0, c1), std::max(c2, c3));
  };
  switch (op) {
    case RD_OP_ADD: lo = al + bl; hi = ah + bh; return fits64(lo) && fits64(hi);
    case RD_OP_SUB: lo = al - bh; hi = ah - bl; return fits64(lo) && fits64(hi);
    case RD_OP_MUL:
      corners(al * bl, al * bh, ah * bl, ah * bh);
      return fits64(lo) && fits64(hi);
    case RD_OP_DIV:
      if (bl <= 0 && bh >= 0) return false;
      if (al == kI64Lo && bl <= -1 && bh >= -1) return false;
      corners(al / bl, al / bh, ah / bl, ah / bh);
      return true;
    case RD_OP_MOD: {
      if (bl <= 0 && bh >= 0) return false;
      if (al == kI64Lo && bl <= -1 && bh >= -1) return false;
      const i128 m = std::max(i128abs(bl), i128abs(bh)) - 1;
      lo = al >= 0 ? 0 : std::max(al, -m);
      hi = ah <= 0 ? 0 : std::min(ah, m);
      return true;
    }
    case RD_OP_SHL:
      if (bl < 0 || bh > 63) return false;
      corners(al * ((i128)1 << (int)bl), al * ((i128)1 << (int)bh),
              ah * ((i128)1 << (int)bl), ah * ((i128)1 << (int)bh));
      return fits64(lo) && fits64(hi);
    case RD_OP_SHR:
      if (bl < 0 || bh > 63) return false;
      corners(al >> (int)bl, al >> (int)bh, ah >> (int)bl, ah >> (int)bh);
      return true;
    case RD_OP_AND:
    case RD_OP_OR:
    case RD_OP_XOR:
      if (al >= 0 && bl >= 0) {
        i128 m = std::max(ah, bh), p = 1;
        while (p <= m) p <<= 1;
        lo = 0;
        hi = op == RD_OP_AND ? std::min(ah, bh) : p - 1;
      } else {
        lo = kI64Lo;
        hi = kI64Hi;
      }
      return true;
    case RD_OP_MIN: lo = std::min(al, bl); hi = std::min(ah, bh); return true;
    case RD_OP_MAX: lo = std::max(al, bl); hi = std::max(ah, bh); return true;
    default: lo = 0; hi = 1; return true;  // comparisons and logic
  }
}

// One term: value of `code` (in [lo, hi]) times `mult`, of group `group`.
struct STerm {
  std::vector<rd_insn> code;
  int64_t mult = 1;
  i128 lo = 0, hi = 0;
  int group = 0;
  uint64_t g = 1;  // every value of `code` is a multiple of g
};

struct Lin {
  i128 u = 0;
  std::vector<STerm> terms;
};

inline i128 contrib_lo(const STerm& t) { return std::min(t.lo * t.mult, t.hi * t.mult); }
inline i128 contrib_hi(const STerm& t) { return std::max(t.lo * t.mult, t.hi * t.mult); }
inline i128 contrib_abs(const STerm& t) {
  return std::max(i128abs(t.lo), i128abs(t.hi)) * i128abs((i128)t.mult);
}

inline rd_insn mk_insn(uint16_t op, int64_t imm = 0, uint16_t arg = 0) {
  rd_insn t;
  memset(&t, 0, sizeof t);
  t.op = op;
  t.arg = arg;
  t.imm = imm;
  return t;
}

struct TermBuilder {
  const rd_kernel_model& M;
  const rd_access& A;
  const int64_t* pv;
  const int64_t* dims;
  const int64_t* lmin;
  const int64_t* lmax;
  const uint64_t* lgcd;  // per loop position: gcd of its values
  std::vector<TNode> nodes;
  const rd_insn* ins = nullptr;

  // Builds the tree of `e` with groups, uniform values and ranges; false if
  // some operation may fail anywhere in the box.
  bool build(rd_expr e) {
    nodes.clear();
    ins = M.insns + e.first;
    std::vector<int> st;
    for (uint32_t k = 0; k < e.count; ++k) {
      const rd_insn& t = ins[k];
      TNode n;
      n.op = t.op;
      n.arg = t.arg;
      n.imm = t.imm;
      n.start = k;
      if (is_leaf(t.op)) {
        switch (t.op) {
          case RD_OP_CONST: n.val = t.imm; break;
          case RD_OP_PARAM: n.val = pv[t.arg]; break;
          case RD_OP_GDIM: n.val = dims[t.arg]; break;
          case RD_OP_BDIM: n.val = dims[3 + t.arg]; break;
          case RD_OP_TID: n.groups = 2; n.lo = 0; n.hi = dims[3 + t.arg] - 1; break;
          case RD_OP_BID: n.groups = 1; n.lo = 0; n.hi = dims[t.arg] - 1; break;
          case RD_OP_LOOP: {
            const int p = loop_pos(&A, t.arg);
            n.groups = 4;
            n.lo = lmin[p];
            n.hi = lmax[p];
            n.g = lgcd[p];
            break;
          }
        }
        if (n.groups == 0) {
          n.lo = n.hi = n.val;
          n.g = uabs64(n.val);
        }
      } else if (is_unary(t.op)) {
        const TNode& c = nodes[st.back()];
        n.kid[0] = st.back();
        st.pop_back();
        n.start = c.start;
        n.groups = c.groups;
        if (t.op == RD_OP_NEG) {
          if (c.lo == kI64Lo) return false;
          n.lo = -c.hi;
          n.hi = -c.lo;
        } else {
          n.lo = 0;
          n.hi = 1;
        }
        n.g = t.op == RD_OP_NEG ? c.g : 1;
        if (!n.groups) {
          n.val = t.op == RD_OP_NEG ? -c.val : (c.val == 0);
          n.lo = n.hi = n.val;
          n.g = uabs64(n.val);
        }
      } else {
        n.kid[1] = st.back();
        st.pop_back();
        n.kid[0] = st.back();
        st.pop_back();
        const TNode& a = nodes[n.kid[0]];
        const TNode& b = nodes[n.kid[1]];
        n.start = a.start;
        n.groups = a.groups | b.groups;
        if (!n.groups) {
          uint32_t err = 0;
          n.val = hop(t.op, a.val, b.val, err);
          if (err) return false;
          n.lo = n.hi = n.val;
          n.g = uabs64(n.val);
        } else {
          if (!range_op(t.op, a.lo, a.hi, b.lo, b.hi, n.lo, n.hi)) return false;
          switch (t.op) {
            case RD_OP_ADD:
            case RD_OP_SUB:
            case RD_OP_MIN:
            case RD_OP_MAX: n.g = gcd64(a.g, b.g); break;
            case RD_OP_MUL: n.g = gmul(a.g, b.g); break;
            case RD_OP_SHL:
              n.g = b.groups ? 1 : gmul(a.g, 1ull << (b.val & 63));
              break;
            default: n.g = 1;
          }
        }
      }
      st.push_back((int)nodes.size());
      nodes.push_back(n);
    }
    return true;
  }

  void subtree(int i, std::vector<rd_insn>& out) const {
    const TNode& n = nodes[i];
    uint32_t end = (uint32_t)i;  // node index == its postfix position
    for (uint32_t k = n.start; k <= end; ++k) out.push_back(ins[k]);
  }

  static bool single(uint8_t g) { return g == 1 || g == 2 || g == 4; }
  static int gidx(uint8_t g) { return g == 1 ? 0 : g == 2 ? 1 : 2; }

  bool add_term(Lin& L, std::vector<rd_insn>&& code, i128 lo, i128 hi, int group, i128 mu,
                uint64_t g = 1) {
    if (!fits64(mu)) return false;
    if (mu == 0) return true;
    STerm t;
    t.code = std::move(code);
    t.mult = (int64_t)mu;
    t.lo = lo;
    t.hi = hi;
    t.group = group;
    t.g = g;
    if (!fits64(contrib_abs(t))) return false;
    L.terms.push_back(std::move(t));
    return true;
  }

  // Postfix of sum(term * mult) + u over `ts` (at least one term or u).
  static void emit_sum(const std::vector<const STerm*>& ts, i128 u, std::vector<rd_insn>& out) {
    bool first = true;
    for (const STerm* t : ts) {
      out.insert(out.end(), t->code.begin(), t->code.end());
      if (t->mult != 1) {
        out.push_back(mk_insn(RD_OP_CONST, t->mult));
        out.push_back(mk_insn(RD_OP_MUL));
      }
      if (!first) out.push_back(mk_insn(RD_OP_ADD));
      first = false;
    }
    if (u != 0 || first) {
      out.push_back(mk_insn(RD_OP_CONST, (int64_t)u));
      if (!first) out.push_back(mk_insn(RD_OP_ADD));
    }
  }

  // Affine form of the tree below node i, times mu: adds mu times each
  // coordinate's coefficient to c (tx ty tz bx by bz) and cl (loop
  // positions); constant parts are left out.  False when some operation is
  // not affine in the coordinates (a product of two non-constant values,
  // division, remainder, min, max, comparisons, ...).
  bool affine(int i, i128 mu, i128* c, i128* cl) const {
    const TNode& n = nodes[i];
    if (!n.groups) return true;
    if (i128abs(mu) > ((i128)1 << 62)) return false;
    switch (n.op) {
      case RD_OP_TID: if (n.arg > 2) return false; c[n.arg] += mu; return true;
      case RD_OP_BID: if (n.arg > 2) return false; c[3 + n.arg] += mu; return true;
      case RD_OP_LOOP: {
        const int p = loop_pos(&A, n.arg);
        if (p < 0 || p > 3) return false;
        cl[p] += mu;
        return true;
      }
      case RD_OP_ADD: return affine(n.kid[0], mu, c, cl) && affine(n.kid[1], mu, c, cl);
      case RD_OP_SUB: return affine(n.kid[0], mu, c, cl) && affine(n.kid[1], -mu, c, cl);
      case RD_OP_NEG: return affine(n.kid[0], -mu, c, cl);
      case RD_OP_MUL: {
        const TNode& a = nodes[n.kid[0]];
        const TNode& b = nodes[n.kid[1]];
        if (!a.groups) return affine(n.kid[1], mu * a.val, c, cl);
        if (!b.groups) return affine(n.kid[0], mu * b.val, c, cl);
        return false;
      }
      case RD_OP_SHL: {
        const TNode& b = nodes[n.kid[1]];
        if (b.groups || b.val < 0 || b.val > 62) return false;
        return affine(n.kid[0], mu * ((i128)1 << b.val), c, cl);
      }
      default: return false;
    }
  }

  bool decompose(int i, Lin& L, i128 mu) {
    const TNode& n = nodes[i];
    if (!n.groups) {
      L.u += mu * (i128)n.val;
      return fits64(L.u);
    }
    if (single(n.groups)) {
      std::vector<rd_insn> code;
      subtree(i, code);
      return add_term(L, std::move(code), n.lo, n.hi, gidx(n.groups), mu, n.g);
    }
    const TNode* a = n.kid[0] >= 0 ? &nodes[n.kid[0]] : nullptr;
    const TNode* b = n.kid[1] >= 0 ? &nodes[n.kid[1]] : nullptr;
    switch (n.op) {
      case RD_OP_ADD: return decompose(n.kid[0], L, mu) && decompose(n.kid[1], L, mu);
      case RD_OP_SUB: return decompose(n.kid[0], L, mu) && decompose(n.kid[1], L, -mu);
      case RD_OP_NEG: return decompose(n.kid[0], L, -mu);
      case RD_OP_MUL:
        if (!a->groups) return fits64(mu * a->val) && decompose(n.kid[1], L, mu * a->val);
        if (!b->groups) return fits64(mu * b->val) && decompose(n.kid[0], L, mu * b->val);
        return false;
      case RD_OP_SHL:
        if (b->groups || b->val < 0 || b->val > 62) return false;
        return fits64(mu << (int)b->val) && decompose(n.kid[0], L, mu << (int)b->val);
      case RD_OP_DIV:
      case RD_OP_MOD: {
        if (b->groups || b->val <= 0) return false;
        const int64_t d = b->val;
        Lin in;
        if (!decompose(n.kid[0], in, 1)) return false;
        std::vector<const STerm*> xs, ys;
        i128 xlo = 0, ylo = in.u, yhi = in.u;
        int yg = -1;
        for (const STerm& t : in.terms) {
          // divisible when (multiple of g) * mult is always a multiple of d
          if (gmul(t.g, uabs64(t.mult)) % (uint64_t)d == 0 && t.g != 1 ? true
              : t.mult % d == 0) {
            xs.push_back(&t);
            xlo += contrib_lo(t);
          } else {
            if (yg >= 0 && yg != t.group) return split_small_rest(n, in, L, mu, d);
            yg = t.group;
            ys.push_back(&t);
            ylo += contrib_lo(t);
            yhi += contrib_hi(t);
          }
        }
        if (xlo < 0 || ylo < 0) return split_small_rest(n, in, L, mu, d);
        i128 yabs = i128abs(in.u);
        for (const STerm* t : ys) yabs += contrib_abs(*t);
        if (yabs > kI64Hi) return false;
        if (n.op == RD_OP_DIV)
          for (const STerm* t : xs) {
            // t = v * mult with d | g * mult: t / d = (v / d1) * (mult / gm),
            // gm = gcd(d, |mult|), d1 = d / gm dividing every v
            const uint64_t gm = gcd64((uint64_t)d, uabs64(t->mult));
            const int64_t d1 = (int64_t)((uint64_t)d / gm);
            std::vector<rd_insn> code = t->code;
            i128 lo = t->lo, hi = t->hi;
            uint64_t g = t->g;
            if (d1 != 1) {
              code.push_back(mk_insn(RD_OP_CONST, d1));
              code.push_back(mk_insn(RD_OP_DIV));
              lo /= d1;
              hi /= d1;
              g = g / (uint64_t)d1;
            }
            if (!add_term(L, std::move(code), lo, hi, t->group,
                          mu * (i128)(t->mult / (int64_t)gm), g))
              return false;
          }
        if (ys.empty()) {  // uniform remainder part
          L.u += mu * (n.op == RD_OP_DIV ? in.u / d : in.u % d);
          return fits64(L.u);
        }
        std::vector<rd_insn> code;
        emit_sum(ys, in.u, code);
        code.push_back(mk_insn(RD_OP_CONST, d));
        code.push_back(mk_insn(n.op));
        const i128 lo = n.op == RD_OP_DIV ? ylo / d : 0;
        const i128 hi = n.op == RD_OP_DIV ? yhi / d : std::min(yhi, (i128)d - 1);
        return add_term(L, std::move(code), lo, hi, yg, mu);
      }
      default:
        return false;
    }
  }

  // Second way to split X + Y by a positive d: X (the uniform part and the
  // terms of one group) is a multiple of some g with g | d and X >= 0, and
  // Y (the terms of one other group) lies in [0, g).  Then no multiple of d
  // falls inside (X, X + Y], so (X + Y) / d = X / d and (X + Y) % d =
  // X % d + Y.
  bool split_small_rest(const TNode& n, const Lin& in, Lin& L, i128 mu, int64_t d) {
    for (int gy = 0; gy < 3; ++gy) {
      std::vector<const STerm*> xs, ys;
      int gx = -1;
      bool ok = true;
      i128 xlo = in.u, ylo = 0, yhi = 0, xabs = i128abs(in.u);
      uint64_t g = uabs64((int64_t)in.u);
      for (const STerm& t : in.terms) {
        if (t.group == gy) {
          ys.push_back(&t);
          ylo += contrib_lo(t);
          yhi += contrib_hi(t);
        } else {
          if (gx >= 0 && gx != t.group) { ok = false; break; }
          gx = t.group;
          xs.push_back(&t);
          xlo += contrib_lo(t);
          xabs += contrib_abs(t);
          g = gcd64(g, gmul(t.g, uabs64(t.mult)));
        }
      }
      if (!ok || ys.empty() || xs.empty() || xabs > kI64Hi) continue;
      if (g == 0 || (uint64_t)d % g != 0 || xlo < 0 || ylo < 0 || yhi >= (i128)g) continue;
      // X / d or X % d as one term of group gx
      std::vector<rd_insn> code;
      emit_sum(xs, in.u, code);
      code.push_back(mk_insn(RD_OP_CONST, d));
      code.push_back(mk_insn(n.op));
      i128 xhi = in.u;
      for (const STerm* t : xs) xhi += contrib_hi(*t);
      if (n.op == RD_OP_DIV) return add_term(L, std::move(code), xlo / d, xhi / d, gx, mu);
      if (!add_term(L, std::move(code), 0, std::min(xhi, (i128)d - 1), gx, mu)) return false;
      for (const STerm* t : ys) {
        std::vector<rd_insn> c2 = t->code;
        if (!add_term(L, std::move(c2), t->lo, t->hi, t->group, mu * (i128)t->mult, t->g))
          return false;
      }
      return true;
    }
    return false;
  }

  // Guard as a conjunction of single-group (or uniform) conjuncts.
  bool conjuncts(int i, std::vector<rd_insn> (&c)[3], bool& never) {
    const TNode& n = nodes[i];
    if (n.op == RD_OP_LAND && n.groups && !single(n.groups))
      return conjuncts(n.kid[0], c, never) && conjuncts(n.kid[1], c, never);
    if (!n.groups) {
      if (n.val == 0) never = true;
      return true;
    }
    if (!single(n.groups)) return false;
    std::vector<rd_insn>& out = c[gidx(n.groups)];
    const bool first = out.empty();
    subtree(i, out);
    if (!first) out.push_back(mk_insn(RD_OP_LAND));
    return true;
  }
};

// Largest stack depth of a postfix sequence.
uint32_t postfix_depth(const std::vector<rd_insn>& code) {
  uint32_t d = 0, m = 0;
  for (const rd_insn& t : code) {
    if (is_leaf(t.op)) ++d;
    else if (is_binary(t.op)) --d;
    m = std::max(m, d);
  }
  return m;
}

struct DimInfo {
  bool done = false;
  uint32_t err = 0;
  bool ok = false;       // non-empty and within limits
  int64_t d[6];
  uint32_t params_off;   // offset of [params..., gx, gy, gz, bx, by, bz]
};

struct LoopInfo {
  bool done = false;
  uint32_t err = 0;
  bool ok = false;
  uint32_t off = 0, n = 0;
};

struct InstInfo {
  bool done = false;
  uint32_t err = 0;   // errors from extents and loops of this access
  int32_t idx = -1;   // device instance, -1: no points
  uint64_t box = 0;   // points counted in evals
  uint32_t npts = 0;
};

struct Planner {
  const rd_kernel_model* models;
  const rd_launch_domain* launch;
  const rd_param_sets* params;
  std::vector<std::vector<DimInfo>> dims;                 // [model][set]
  std::map<std::pair<uint32_t, uint32_t>, std::vector<LoopInfo>> loops;  // (model, loop) -> per set
  std::map<std::pair<uint32_t, uint32_t>, std::vector<InstInfo>> insts;  // (model, acc) -> per set
  std::map<std::pair<uint32_t, uint32_t>, Prog> progs[6];
  std::vector<DInsn> code;
  std::vector<int64_t> pool_params;
  std::vector<int64_t> pool_loops;
  std::vector<AccInst> dev_insts;
  std::vector<TabHost> tabs;  // per device instance
  std::vector<std::pair<int64_t, int64_t>> arange;  // address range, tables only
  // address residue, tables only: every address is congruent to `second`
  // modulo `first` (0: the single address `second`; 1: no information)
  std::vector<std::pair<uint64_t, int64_t>> ares;
  // tables only: bounds of u plus the thread and iteration terms (a block's
  // addresses lie in its block term plus these), and the block-term job
  // (index into tjobs, -1: the address does not depend on the block)
  std::vector<std::pair<int64_t, int64_t>> rrest;
  std::vector<uint8_t> tinj;  // tables only: thread-injective address (below)
  std::vector<int32_t> bjob;
  // tables only: address step from thread 0 to thread 1 and from block 0 to
  // block 1 (0 when the group has one index or no term)
  std::vector<std::array<int64_t, 2>> gstride;
  std::vector<TabJob> tjobs;
  uint64_t tpool = 0;         // table entries
  uint64_t tab_budget = kMaxTabPool;  // table entries this planner may use
  bool use_tables = true;

  // Exact dependence test on an address that is affine in the coordinates
  // (TermBuilder::affine): true when two points of different threads can
  // never share an address.  The address is u + sum_k c_k x_k over the
  // thread, block and loop coordinates (loop coordinates take their loop's
  // values).  Each coordinate k with more
  // than one value has a unit step s_k = |c_k| times the smallest distance
  // between two of its values, and a span w_k = |c_k| (max - min).  Either
  // of two mixed-radix arguments decides:
  //   (1) ordered by s_k, the thread and block coordinates satisfy
  //       m_k = s_k - sum_{j<k} w_j > 0; two different threads then differ
  //       in the thread part by at least min_k m_k, and when that exceeds
  //       the span of the whole loop part no loop values close the gap;
  //   (2) ordered by s_k, all coordinates with c_k != 0 satisfy m_k > 0:
  //       different coordinate tuples give different addresses, and two
  //       different threads differ in a thread or block coordinate (all of
  //       which must then have c_k != 0).
  // A thread or block coordinate with more than one value and c_k = 0
  // fails both (threads differing only there share addresses).  For a
  // shared array (per_block) the block coordinates are left out: threads
  // of different blocks never share its memory.
  bool thread_injective(const i128* c, const i128* cl, const AccInst& I,
                        bool per_block) const {
    struct Co {
      i128 step, span;
    };
    std::vector<Co> th, lp;  // thread/block coordinates, loop coordinates
    for (int k = 0; k < 6; ++k) {
      const i128 n = k < 3 ? I.dims[3 + k] : I.dims[k - 3];
      if (n <= 1 || (per_block && k >= 3)) continue;
      if (c[k] == 0) return false;
      th.push_back({i128abs(c[k]), i128abs(c[k]) * (n - 1)});
    }
    for (uint32_t p = 0; p < I.n_loops && p < 4; ++p) {
      if (cl[p] == 0 || I.loop_n[p] <= 1) continue;
      std::vector<int64_t> v(pool_loops.begin() + I.loop_off[p],
                             pool_loops.begin() + I.loop_off[p] + I.loop_n[p]);
      std::sort(v.begin(), v.end());
      i128 gap = -1;
      for (size_t e = 1; e < v.size(); ++e) {
        const i128 d = (i128)v[e] - v[e - 1];
        if (gap < 0 || d < gap) gap = d;
      }
      lp.push_back({i128abs(cl[p]) * gap, i128abs(cl[p]) * ((i128)v.back() - v.front())});
    }
    // smallest margin of a mixed-radix ordering, -1 if some margin is <= 0
    // (no coordinate with more than one value: +infinity, returned as 0)
    auto margin = [](std::vector<Co> co) -> i128 {
      std::sort(co.begin(), co.end(), [](const Co& a, const Co& b) { return a.step < b.step; });
      i128 below = 0, m = 0;
      for (const Co& e : co) {
        const i128 mk = e.step - below;
        if (mk <= 0) return -1;
        if (m == 0 || mk < m) m = mk;
        below += e.span;
      }
      return m;
    };
    const i128 mt = margin(th);
    if (mt < 0) return false;
    if (mt == 0) return true;  // one thread only
    i128 lspan = 0;
    for (const Co& e : lp) lspan += e.span;
    if (lspan < mt) return true;  // (1)
    std::vector<Co> all = th;
    all.insert(all.end(), lp.begin(), lp.end());
    return margin(all) > 0;  // (2)
  }

  // Term tables of instance I (access a of model m); T.on = 0 when some
  // expression does not qualify.
  void tables_for(uint32_t m, uint32_t a, const AccInst& I, uint32_t inst, TabHost& T) {
    memset(&T, 0, sizeof T);
    for (int g = 0; g < 3; ++g) T.off[g] = kNoTab;
    T.iv_off = kNoTab;
    if (!use_tables) return;
    const rd_kernel_model& M = models[m];
    const rd_access& A = M.acc[a];
    const int64_t* pv = pool_params.data() + I.params_off;
    int64_t dims[6], lmin[4] = {0, 0, 0, 0}, lmax[4] = {0, 0, 0, 0};
    uint64_t lgcd[4] = {1, 1, 1, 1};
    for (int k = 0; k < 6; ++k) dims[k] = I.dims[k];
    for (uint32_t k = 0; k < I.n_loops; ++k) {
      const int64_t* v = pool_loops.data() + I.loop_off[k];
      lmin[k] = *std::min_element(v, v + I.loop_n[k]);
      lmax[k] = *std::max_element(v, v + I.loop_n[k]);
      uint64_t g = 0;
      for (uint32_t e = 0; e < I.loop_n[k]; ++e) g = gcd64(g, uabs64(v[e]));
      lgcd[k] = g;
    }
    TermBuilder tb{M, A, pv, dims, lmin, lmax, lgcd};
    // address
    if (!tb.build(A.addr)) return;
    const i128 root_lo = tb.nodes.back().lo, root_hi = tb.nodes.back().hi;
    Lin L;
    if (!tb.decompose((int)tb.nodes.size() - 1, L, 1)) return;
    i128 ac[6] = {0, 0, 0, 0, 0, 0}, acl[4] = {0, 0, 0, 0};
    const bool aff = tb.affine((int)tb.nodes.size() - 1, 1, ac, acl);
    i128 tot = i128abs(L.u), lo = L.u, hi = L.u;
    for (const STerm& t : L.terms) {
      tot += contrib_abs(t);
      lo += contrib_lo(t);
      hi += contrib_hi(t);
    }
    if (tot > kI64Hi) return;
    if (I.is32 && !(root_lo >= INT32_MIN && root_hi <= INT32_MAX) &&
        !(lo >= INT32_MIN && hi <= INT32_MAX))
      return;
    // guard
    std::vector<rd_insn> conj[3];
    bool never = false;
    if (A.guard.count) {
      if (!tb.build(A.guard)) return;
      if (!tb.conjuncts((int)tb.nodes.size() - 1, conj, never)) return;
    }
    // interval ids
    int64_t ivc[2] = {0, 0};
    bool ivtab = false;
    const rd_expr ive[2] = {A.bint, A.wint};
    for (int w = 0; w < 2; ++w) {
      if (!ive[w].count) continue;
      if (!tb.build(ive[w])) return;
      const TNode& r = tb.nodes.back();
      if (r.lo < 0 || r.hi > 65535) return;
      if (r.groups) ivtab = true;
      else ivc[w] = r.val;
    }
    // programs and table jobs
    const uint32_t gsize[3] = {I.nblk, I.nthr, I.niota};
    std::vector<TabJob> jobs;
    uint64_t entries = 0;
    if (!never) {
      rd_kernel_model tm = M;
      for (int g = 0; g < 3; ++g) {
        std::vector<const STerm*> ts;
        for (const STerm& t : L.terms)
          if (t.group == g) ts.push_back(&t);
        if (ts.empty() && conj[g].empty()) continue;
        TabJob J;
        memset(&J, 0, sizeof J);
        J.inst = inst;
        J.group = (uint32_t)g;
        J.n = gsize[g];
        J.val.absent = 1;
        J.guard.absent = 1;
        if (!ts.empty()) {
          std::vector<rd_insn> code;
          TermBuilder::emit_sum(ts, 0, code);
          if (postfix_depth(code) > (uint32_t)kMaxStack) return;
          tm.insns = code.data();
          tm.n_insns = (uint32_t)code.size();
          J.val = compile(tm, rd_expr{0, (uint32_t)code.size()}, A, this->code);
        }
        if (!conj[g].empty()) {
          if (postfix_depth(conj[g]) > (uint32_t)kMaxStack) return;
          tm.insns = conj[g].data();
          tm.n_insns = (uint32_t)conj[g].size();
          J.guard = compile(tm, rd_expr{0, (uint32_t)conj[g].size()}, A, this->code);
        }
        jobs.push_back(J);
        entries += J.n;
      }
      if (ivtab) {
        TabJob J;
        memset(&J, 0, sizeof J);
        J.inst = inst;
        J.group = 3;
        J.n = I.niota;
        J.val.absent = 1;
        J.guard.absent = 1;
        jobs.push_back(J);
        entries += J.n;
      }
    }
    if (entries > kMaxTabInst || tpool + entries > tab_budget) return;
    T.base = tpool;
    for (TabJob& J : jobs) {
      if (J.group == 0) bjob[inst] = (int32_t)tjobs.size();
      J.out_off = tpool;
      const uint32_t rel = (uint32_t)(tpool - T.base);
      if (J.group < 3) T.off[J.group] = rel;
      else T.iv_off = rel;
      tpool += J.n;
      tjobs.push_back(J);
    }
    T.u = (int64_t)L.u;
    T.iv_const = (uint32_t)ivc[0] | ((uint32_t)ivc[1] << 16);
    T.never = never;
    T.on = 1;
    arange[inst] = {(int64_t)lo, (int64_t)hi};
    // each term is a multiple of g * |mult| (1 when that product is not
    // known exactly), so addr - u is a multiple of their gcd
    uint64_t G = 0;
    for (const STerm& t : L.terms) G = gcd64(G, gmul(t.g, uabs64(t.mult)));
    ares[inst] = {G, (int64_t)L.u};
    i128 rlo = L.u, rhi = L.u;
    for (const STerm& t : L.terms)
      if (t.group != 0) {
        rlo += contrib_lo(t);
        rhi += contrib_hi(t);
      }
    rrest[inst] = {(int64_t)rlo, (int64_t)rhi};
    tinj[inst] =
        aff && thread_injective(ac, acl, I, M.arrays[A.array].space == RD_SHARED) ? 1 : 0;
    // point order: iterations fastest when the address moves less along
    // them than along threads (consecutive points then share buckets)
    int64_t stride[3] = {0, 0, 0};
    for (const TabJob& J : jobs) {
      if (J.group == 3 || J.val.absent || J.n < 2) continue;
      int64_t c[10];
      uint32_t e = 0;
      host_coords(I, pool_loops, J.group == 0 ? 1 : 0, J.group == 1 ? 1 : 0,
                  J.group == 2 ? 1 : 0, c);
      const int64_t v1 = host_prog(this->code, J.val, c, pv, 0, e);
      host_coords(I, pool_loops, 0, 0, 0, c);
      const int64_t v0 = host_prog(this->code, J.val, c, pv, 0, e);
      if (J.group < 2 && !e) gstride[inst][J.group ? 0 : 1] = v1 - v0;
      if (J.group == 0) continue;
      if (!e) stride[J.group] = v1 > v0 ? v1 - v0 : v0 - v1;
      else stride[J.group] = INT64_MAX;
    }
    const bool t_moves = I.nthr > 1, i_moves = I.niota > 1;
    dev_insts[inst].iorder = i_moves && (!t_moves || stride[2] < stride[1]) ? 1 : 0;
    // acquire and release addresses that interval bounds prove error-free
    // over the box (and inside int32 for 32-bit lock arrays)
    bool ss = true;
    for (const rd_sync* y : {&A.acq, &A.rel}) {
      if (!y->addr.count) continue;
      if (!tb.build(y->addr)) {
        ss = false;
        break;
      }
      const TNode& r = tb.nodes.back();
      if (M.arrays[y->array].addr_bits == 32 && (r.lo < INT32_MIN || r.hi > INT32_MAX)) {
        ss = false;
        break;
      }
    }
    T.syn_safe = ss ? 1 : 0;
  }

  DimInfo& dim(uint32_t m, uint32_t s) {
    DimInfo& d = dims[m][s];
    if (d.done) return d;
    d.done = true;
    const rd_kernel_model& M = models[m];
    const rd_launch_domain& L = launch[m];
    const int64_t* pv = params[m].values + (uint64_t)s * M.n_params;
    bool nonempty = true;
    for (int k = 0; k < 3; ++k) {
      d.d[k] = heval(M, L.grid[k], pv, nullptr, 1, d.err);
      d.d[3 + k] = heval(M, L.block[k], pv, nullptr, 1, d.err);
      if (d.d[k] < 1 || d.d[3 + k] < 1) nonempty = false;
    }
    if (!nonempty) return d;
    for (int k = 3; k < 6; ++k)
      if (d.d[k] > kMaxBlock) { d.err |= ERR_UNSUP; return d; }
    if (d.d[3] * d.d[4] > kMaxBlock || d.d[3] * d.d[4] * d.d[5] > kMaxBlock) {
      d.err |= ERR_UNSUP;
      return d;
    }
    for (int k = 0; k < 3; ++k)
      if (d.d[k] >= kMaxGrid) { d.err |= ERR_UNSUP; return d; }
    if (d.d[0] * d.d[1] >= kMaxGrid || d.d[0] * d.d[1] * d.d[2] >= kMaxGrid) {
      d.err |= ERR_UNSUP;
      return d;
    }
    d.ok = true;
    d.params_off = (uint32_t)pool_params.size();
    for (uint32_t k = 0; k < M.n_params; ++k) pool_params.push_back(pv[k]);
    for (int k = 0; k < 6; ++k) pool_params.push_back(d.d[k]);
    return d;
  }

  LoopInfo& loop(uint32_t m, uint32_t l, uint32_t s, const DimInfo& d) {
    auto& v = loops[{m, l}];
    if (v.empty()) v.resize(params[m].n_sets);
    LoopInfo& li = v[s];
    if (li.done) return li;
    li.done = true;
    const rd_kernel_model& M = models[m];
    const rd_loop& L = M.loops[l];
    const int64_t* pv = params[m].values + (uint64_t)s * M.n_params;
    uint32_t e = 0;
    int64_t x = heval(M, L.init, pv, d.d, 0, e);
    int64_t bound = heval(M, L.bound, pv, d.d, 0, e);
    int64_t step = heval(M, L.step, pv, d.d, 0, e);
    if (e) { li.err = e; return li; }
    li.off = (uint32_t)pool_loops.size();
    uint32_t n = 0;
    while (cmp_holds(L.cmp, x, bound)) {
      if (n == kMaxIters) {
        li.err |= ERR_UNSUP;
        pool_loops.resize(li.off);
        return li;
      }
      pool_loops.push_back(x);
      ++n;
      uint32_t ue = 0;
      x = hop(kUpdOp[L.upd], x, step, ue);
      if (ue) {
        li.err |= ue;
        pool_loops.resize(li.off);
        return li;
      }
    }
    li.n = n;
    li.ok = true;
    return li;
  }

  Prog prog(uint32_t m, uint32_t a, int which) {
    auto key = std::make_pair(m, a);
    auto it = progs[which].find(key);
    if (it != progs[which].end()) return it->second;
    const rd_access& A = models[m].acc[a];
    const rd_expr ex[6] = {A.addr, A.guard, A.bint, A.wint, A.acq.addr, A.rel.addr};
    const rd_expr e = ex[which];
    Prog p = compile(models[m], e, A, code);
    progs[which][key] = p;
    return p;
  }

  InstInfo& inst(uint32_t m, uint32_t a, uint32_t s) {
    auto& v = insts[{m, a}];
    if (v.empty()) v.resize(params[m].n_sets);
    InstInfo& ii = v[s];
    if (ii.done) return ii;
    ii.done = true;
    DimInfo& d = dim(m, s);
    ii.err |= d.err;
    if (!d.ok) return ii;
    const rd_kernel_model& M = models[m];
    const rd_access& A = M.acc[a];
    uint64_t niota = 1;
    uint32_t ln[4] = {1, 1, 1, 1}, lo[4] = {0, 0, 0, 0};
    for (uint32_t k = 0; k < A.n_loops; ++k) {
      LoopInfo& li = loop(m, A.loops[k], s, d);
      ii.err |= li.err;
      if (!li.ok) return ii;
      ln[k] = li.n;
      lo[k] = li.off;
      niota *= li.n;
      if (niota > kMaxIters) {
        ii.err |= ERR_UNSUP;
        return ii;
      }
    }
    uint64_t nblk = (uint64_t)(d.d[0] * d.d[1] * d.d[2]);
    uint64_t nthr = (uint64_t)(d.d[3] * d.d[4] * d.d[5]);
    uint64_t box = nblk * nthr * niota;
    if (box >= (uint64_t)kMaxPoints) {
      ii.err |= ERR_UNSUP;
      return ii;
    }
    ii.box = box;
    if (box == 0) return ii;
    AccInst I;
    memset(&I, 0, sizeof I);
    I.addr = prog(m, a, 0);
    I.guard = prog(m, a, 1);
    I.bint = prog(m, a, 2);
    I.wint = prog(m, a, 3);
    I.acq = prog(m, a, 4);
    I.rel = prog(m, a, 5);
    I.syn = syn_flags(M, A);
    for (int k = 0; k < 6; ++k) I.dims[k] = (int32_t)d.d[k];
    I.nblk = (uint32_t)nblk;
    I.nthr = (uint32_t)nthr;
    I.niota = (uint32_t)niota;
    I.n_loops = A.n_loops;
    for (int k = 0; k < 4; ++k) {
      I.loop_n[k] = ln[k];
      I.loop_off[k] = lo[k];
    }
    I.params_off = d.params_off;
    I.is32 = M.arrays[A.array].addr_bits == 32;
    I.npts = (uint32_t)box;
    I.tpb = (uint32_t)(nthr * niota);
    ii.idx = (int32_t)dev_insts.size();
    ii.npts = (uint32_t)box;
    dev_insts.push_back(I);
    TabHost T;
    arange.push_back({0, -1});
    ares.push_back({1, 0});
    rrest.push_back({0, -1});
    tinj.push_back(0);
    bjob.push_back(-1);
    gstride.push_back({0, 0});
    tables_for(m, a, I, (uint32_t)ii.idx, T);
    tabs.push_back(T);
    return ii;
  }

  // Appends everything planner `o` lowered (it worked on models no other
  // planner touched): its pools go after this planner's, and every offset
  // and index into them is moved by the pool sizes before the append.
  void absorb(Planner& o) {
    const uint32_t code_off = (uint32_t)code.size();
    const uint32_t par_off = (uint32_t)pool_params.size();
    const uint32_t loop_off = (uint32_t)pool_loops.size();
    const int32_t inst_off = (int32_t)dev_insts.size();
    const int32_t job_off = (int32_t)tjobs.size();
    const uint64_t tp_off = tpool;
    auto fix = [&](Prog& p) {
      if (!p.absent) p.off += code_off;
    };
    code.insert(code.end(), o.code.begin(), o.code.end());
    pool_params.insert(pool_params.end(), o.pool_params.begin(), o.pool_params.end());
    pool_loops.insert(pool_loops.end(), o.pool_loops.begin(), o.pool_loops.end());
    for (AccInst I : o.dev_insts) {
      fix(I.addr);
      fix(I.guard);
      fix(I.bint);
      fix(I.wint);
      fix(I.acq);
      fix(I.rel);
      I.params_off += par_off;
      for (uint32_t k = 0; k < I.n_loops && k < 4; ++k) I.loop_off[k] += loop_off;
      dev_insts.push_back(I);
    }
    for (TabHost T : o.tabs) {
      if (T.on) T.base += tp_off;
      tabs.push_back(T);
    }
    for (TabJob J : o.tjobs) {
      J.inst += (uint32_t)inst_off;
      J.out_off += tp_off;
      fix(J.val);
      fix(J.guard);
      tjobs.push_back(J);
    }
    tpool += o.tpool;
    arange.insert(arange.end(), o.arange.begin(), o.arange.end());
    ares.insert(ares.end(), o.ares.begin(), o.ares.end());
    rrest.insert(rrest.end(), o.rrest.begin(), o.rrest.end());
    tinj.insert(tinj.end(), o.tinj.begin(), o.tinj.end());
    for (int32_t b : o.bjob) bjob.push_back(b < 0 ? b : b + job_off);
    gstride.insert(gstride.end(), o.gstride.begin(), o.gstride.end());
    for (size_t m = 0; m < o.dims.size() && m < dims.size(); ++m) {
      bool any = false;
      for (const DimInfo& d : o.dims[m]) any |= d.done;
      if (!any) continue;
      dims[m] = o.dims[m];
      for (DimInfo& d : dims[m])
        if (d.ok) d.params_off += par_off;
    }
    for (auto& kv : o.loops) {
      std::vector<LoopInfo> v = kv.second;
      for (LoopInfo& li : v)
        if (li.ok) li.off += loop_off;
      loops[kv.first] = v;
    }
    for (auto& kv : o.insts) {
      std::vector<InstInfo> v = kv.second;
      for (InstInfo& ii : v)
        if (ii.idx >= 0) ii.idx += inst_off;
      insts[kv.first] = v;
    }
    for (int w = 0; w < 6; ++w)
      for (auto& kv : o.progs[w]) {
        Prog p = kv.second;
        fix(p);
        progs[w][kv.first] = p;
      }
  }

  // Per-block address intervals of a table instance (sorted, merged): a
  // block's addresses lie in its block term plus the bounds of the other
  // terms (one program run per block).
  std::map<int32_t, std::vector<std::pair<int64_t, int64_t>>> bcache;
  const std::vector<std::pair<int64_t, int64_t>>& block_ranges(int32_t x) {
    auto it = bcache.find(x);
    if (it != bcache.end()) return it->second;
    std::vector<std::pair<int64_t, int64_t>> v;
    const AccInst& I = dev_insts[x];
    const TabJob& J = tjobs[bjob[x]];
    const int64_t* pr = pool_params.data() + I.params_off;
    const auto rest = rrest[x];
    int64_t c[10];
    bool ok = true;
    for (uint32_t b = 0; b < I.nblk && ok; ++b) {
      host_coords(I, pool_loops, b, 0, 0, c);
      uint32_t err = 0;
      const bool g = J.guard.absent || host_prog(code, J.guard, c, pr, 1, err) != 0;
      const int64_t t = g && !J.val.absent ? host_prog(code, J.val, c, pr, 0, err) : 0;
      if (err) ok = false;
      if (g) v.push_back({t + rest.first, t + rest.second});
    }
    if (!ok) v.assign(1, {INT64_MIN, INT64_MAX});  // no claim
    std::sort(v.begin(), v.end());
    std::vector<std::pair<int64_t, int64_t>> m;
    for (const auto& r : v) {
      if (!m.empty() && r.first <= m.back().second)
        m.back().second = std::max(m.back().second, r.second);
      else
        m.push_back(r);
    }
    return bcache[x] = std::move(m);
  }

  // Exact pre-filter of a (pair, tuple) unit of two table instances: true
  // when no address of one equals an address of the other.  (1) The address
  // ranges over the whole launch box do not meet.  (2) The residues are
  // incompatible: addresses of a are u_a + k G_a, of b u_b + k G_b, and a
  // common one needs gcd(G_a, G_b) | u_a - u_b.  (3) For units of at least
  // 2^18 points with at most 2^16 blocks per side: the unions of the
  // per-block intervals miss each other.
  bool apart(int32_t ia, int32_t ib) {
    if (!tabs[ia].on || !tabs[ib].on) return false;
    const auto& ra = arange[ia];
    const auto& rb = arange[ib];
    if (ra.second < rb.first || rb.second < ra.first) return true;
    const auto& ca = ares[ia];
    const auto& cb = ares[ib];
    const uint64_t g = gcd64(ca.first, cb.first);
    const i128 du = (i128)ca.second - (i128)cb.second;
    if (g == 0 ? du != 0 : (du % (i128)g) != 0) return true;
    if (bjob[ia] < 0 || bjob[ib] < 0) return false;
    const AccInst& A = dev_insts[ia];
    const AccInst& B = dev_insts[ib];
    if (A.nblk > (1u << 16) || B.nblk > (1u << 16)) return false;
    if ((uint64_t)A.npts + B.npts < (1ull << 18)) return false;
    const auto& x = block_ranges(ia);
    const auto& y = block_ranges(ib);
    size_t i = 0, j = 0;
    while (i < x.size() && j < y.size()) {
      if (x[i].second < y[j].first) ++i;
      else if (y[j].second < x[i].first) ++j;
      else return false;  // these intervals meet
    }
    return true;
  }
};

// Accesses a and b of M compute their address with one and the same
// expression (so, under one tuple, one function of the coordinates and
// loop values).
bool same_addr_expr(const rd_kernel_model& M, uint32_t a, uint32_t b) {
  const rd_expr ea = M.acc[a].addr, eb = M.acc[b].addr;
  if (ea.count != eb.count) return false;
  for (uint32_t e = 0; e < ea.count; ++e) {
    const rd_insn& x = M.insns[ea.first + e];
    const rd_insn& y = M.insns[eb.first + e];
    if (x.op != y.op || x.arg != y.arg || x.imm != y.imm) return false;
  }
  return true;
}

// Per-access facts for the device's syn() (section 6.5, Figures 9 and 10):
// which of acquire and release exist, which reach device scope, whether
// they share an array (so a lock is possible), the access kind, and which
// addresses must fit int32.
uint32_t syn_flags(const rd_kernel_model& m, const rd_access& a) {
  uint32_t f = 0;
  if (a.acq.addr.count) {
    f |= kSynAcq;
    if (a.acq.scope == RD_SCOPE_DEVICE) f |= kSynAcqDev;
    if (m.arrays[a.acq.array].addr_bits == 32) f |= kSynAcq32;
  }
  if (a.rel.addr.count) {
    f |= kSynRel;
    if (a.rel.scope == RD_SCOPE_DEVICE) f |= kSynRelDev;
    if (m.arrays[a.rel.array].addr_bits == 32) f |= kSynRel32;
  }
  if ((f & kSynAcq) && (f & kSynRel) &&
      memory_of(m, a.acq.array) == memory_of(m, a.rel.array))
    f |= kSynSameArr;
  if (a.kind == RD_WRITE) f |= kSynWrite;
  if (a.kind == RD_READ) f |= kSynRead;
  return f;
}

// The array of an access's syn() at scope `dev` (0 block, 1 device), or -1
// when it has none at any point: a lock needs one array for acquire and
// release, so the array never depends on the point.
int64_t syn_array(const rd_access& a, int dev, const rd_kernel_model& m) {
  const bool A = a.acq.addr.count && (!dev || a.acq.scope == RD_SCOPE_DEVICE);
  const bool R = a.rel.addr.count && (!dev || a.rel.scope == RD_SCOPE_DEVICE);
  if (A && R && memory_of(m, a.acq.array) == memory_of(m, a.rel.array)) return a.acq.array;
  if (a.kind == RD_WRITE && R) return a.rel.array;
  if (a.kind == RD_READ && A) return a.acq.array;
  return -1;
}

// Pair-level synchronisation flags: kQSync when either access has an
// acquire or release (the pair goes to the HBM aggregation path); kQSyncBlk
// / kQSyncDev when points of the two can share a syn() at block / device
// scope (same array; device scope also needs a global array, since shared
// memory is one per block).
uint32_t pair_sync(const rd_kernel_model& m, const rd_access& x, const rd_access& y) {
  uint32_t f = 0;
  if (x.acq.addr.count || x.rel.addr.count || y.acq.addr.count || y.rel.addr.count)
    f |= kQSync;
  const int64_t b0 = syn_array(x, 0, m), b1 = syn_array(y, 0, m);
  if (b0 >= 0 && b1 >= 0 && memory_of(m, (uint32_t)b0) == memory_of(m, (uint32_t)b1))
    f |= kQSyncBlk;
  const int64_t d0 = syn_array(x, 1, m), d1 = syn_array(y, 1, m);
  if (d0 >= 0 && d1 >= 0 && memory_of(m, (uint32_t)d0) == memory_of(m, (uint32_t)d1) &&
      m.arrays[d0].space == RD_GLOBAL)
    f |= kQSyncDev;
  return f;
}

uint32_t class_mask(const rd_kernel_model& m, const rd_access& x,
                    const rd_access& y, uint32_t caller) {
  uint32_t mask = caller & 7u;
  if (x.kind == RD_READ && y.kind == RD_READ) return 0;  // section 6.1
  if (x.kind == RD_ATOMIC && y.kind == RD_ATOMIC) {      // appendix A.2
    if (x.scope == RD_SCOPE_DEVICE && y.scope == RD_SCOPE_DEVICE) return 0;
    mask &= RD_INTER;
  }
  if (m.arrays[x.array].space == RD_SHARED) mask &= ~(uint32_t)RD_INTER;
  return mask;
}

struct QPlan {
  uint32_t host_err = 0;
  uint32_t sync = 0;  // kQSync* flags
  uint8_t trivial = 0;
  uint8_t lower = 0;  // valid, non-trivial: its instances are lowered
  bool work = false;
  QDesc qd;
  uint64_t evals = 0;
  std::vector<std::pair<int32_t, int32_t>> inst;  // per set
};

#define TRY_HIP(x)                  \
  do {                              \
    if ((x) != hipSuccess) {        \
      return RD_EDEVICE;            \
    }                               \
  } while (0)

}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

const char* rd_strerror(int s) {
  switch (s) {
    case RD_OK: return "ok";
    case RD_EINVAL: return "invalid argument or malformed model";
    case RD_EUNSUPPORTED: return "outside the supported limits";
    case RD_ERANGE: return "integer overflow or address outside its width";
    case RD_EDIVZERO: return "division by zero";
    case RD_ENOMEM: return "out of device memory";
    case RD_EDEVICE: return "device error";
    case RD_ECAPACITY: return "buffer too small";
  }
  return "unknown status";
}

int rd_context_create(rd_context** ctx, int hip_device) {
  if (!ctx) return RD_EINVAL;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
    return RD_EDEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return RD_EDEVICE;
  rd_context* c = new rd_context();
  c->device = hip_device;
  memset(&c->stats, 0, sizeof c->stats);
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return RD_EDEVICE;
    }
  const char* cfg = getenv("HGRD_LDS_CFG");
  if (cfg) c->cfg = atoi(cfg) % 3;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess)
    c->n_cu = (uint32_t)prop.multiProcessorCount;
  if (hipStreamCreate(&c->stream) != hipSuccess || init_kernel_attributes() != 0 ||
      noalloc_scratch_init(hip_device) != 0) {
    delete c;
    return RD_EDEVICE;
  }
  *ctx = c;
  return RD_OK;
}

void rd_context_destroy(rd_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto& kv : ctx->bufs)
    if (kv.second.p && kv.second.own) (void)hipFree(kv.second.p);
  for (auto& kv : ctx->shared)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (void* p : ctx->retired) (void)hipFree(p);
  for (auto& e : ctx->ev) (void)hipEventDestroy(e);
  for (auto& e : ctx->wev) (void)hipEventDestroy(e);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int rd_get_stats(const rd_context* ctx, rd_stats* out) {
  if (!ctx || !out) return RD_EINVAL;
  *out = ctx->stats;
  return RD_OK;
}

// A prepared batch: everything rd_execute needs, already in device memory.
struct rd_plan_impl {
  uint32_t n_pairs = 0;
  int cfg = 1;
  uint32_t cap = 1536;
  uint32_t log_level = 0;
  hipStream_t st = nullptr;
  std::vector<QPlan> Q;
  // (pair, tuple) units of pairs with an acquire or release: joined by the
  // HBM aggregation path with the synchronisation levels
  struct SyncUnit {
    uint32_t q, sigma, inst_i, inst_j, scan;
    uint64_t R;
  };
  std::vector<SyncUnit> sync_units;
  std::vector<uint32_t> npts;  // per device instance
  std::vector<uint32_t> tpb;   // per device instance: points per block
  std::vector<uint8_t> tab_on;  // per device instance: has term tables
  std::vector<uint32_t> nblk;   // per device instance: blocks
  std::vector<std::pair<int64_t, int64_t>> arange;  // address range (tables)
  bool no_map = false;          // hash buckets only
  uint64_t evals = 0;
  uint32_t n_sitems = 0;
  uint64_t n_symmetric = 0;   // shared units joined on block 0 only
  uint64_t sync_decided = 0;  // synchronised units decided conflict-free
  uint32_t persist_grid = 0;  // workgroups of the persistent small join
  uint32_t chunk_pts = 16384; // points per partition workgroup
  uint32_t run_buckets = 8;   // buckets per join workgroup
  uint32_t n_tabchunks = 0;   // term-table fill chunks
  uint64_t prefiltered = 0;   // (pair, tuple) units decided by the pre-filter
  uint32_t n_insts = 0, tab_insts = 0;
  struct Wave {
    uint32_t first_item, n_items, n_chunks, n_buckets;
    uint32_t n_tab_chunks;  // the first n_tab_chunks chunks have term tables
    uint32_t n_runs;        // bucket runs (one join workgroup each)
    uint32_t n_tab_runs;    // the first n_tab_runs runs are of items with tables
    uint32_t n_sync_runs;   // the last n_sync_runs runs are of synchronised items
    uint64_t key_bytes;
    uint64_t hitem_off, chunk_off, bitem_off;  // element offsets in the plan pools
  };
  std::vector<Wave> waves;
  std::vector<HItem> hitems;   // all waves, wave-local bucket numbering
  std::vector<uint64_t> hR;    // records bound per HBM item
  std::vector<uint8_t> presplit;  // per HBM item: split by (address, block)
                                  // without a first partition pass
  std::vector<uint8_t> herr_scan;  // error-scan-only items
  uint64_t max_key_bytes = 0, max_buckets = 0, max_items = 0;
  uint64_t wave_budget = 0;
  // VERDICT mode
  bool verdict = false;
  uint32_t score_mode = 0;  // 0 plain order, 1 network, 2 interval order
  std::vector<uint32_t> vinst_tab;  // table instances of VERDICT blocks
  std::vector<BItem> bitems_interp; // VERDICT blocks of interpreted instances
  uint32_t K = 0;                  // tiles searched per search unit
  uint32_t n_vq = 0, n_bitems = 0, n_tchunks = 0, max_tiles = 0;
  uint32_t max_g = 0;  // most blocks per side of a search unit
  uint64_t n_tiles = 0;
  std::vector<std::pair<uint32_t, uint32_t>> rounds;  // [item lo, item hi)
  uint32_t n_titems = 0;
  uint32_t n_vqueries_pairs = 0;
  std::vector<VQuery> vqs;
  std::map<std::string, DevBuf> dev;
  Arena* arena = nullptr;  // the context's arena when the plan was made
  void* buf(const char* name, size_t bytes, int* err) {
    DevBuf& b = dev[name];
    if (arena) return arena_buf(*arena, b, name, bytes, err);
    if (bytes == 0) bytes = 256;
    if (b.cap < bytes) {
      if (b.p) (void)hipFree(b.p);
      b.p = nullptr;
      b.cap = 0;
      if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        fprintf(stderr, "hgrd: device allocation of %zu bytes for '%s' failed\n", bytes, name);
        b.p = nullptr;
        *err = RD_ENOMEM;
        return nullptr;
      }
      b.cap = bytes;
    }
    return b.p;
  }
  // the first phase of rd_execute (everything before the first host round
  // trip), captured once and replayed
  hipGraphExec_t graph = nullptr;
  bool graph_failed = false;
  ~rd_plan_impl() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (auto& kv : dev)
      if (kv.second.p && kv.second.own) (void)hipFree(kv.second.p);
  }
};

struct rd_plan : rd_plan_impl {};

int rd_prepare(rd_context* ctx, const rd_kernel_model* models,
               uint32_t n_models, const rd_access_pair* pairs,
               uint32_t n_pairs, const rd_launch_domain* launch,
               const rd_param_sets* params, const rd_options* opt,
               rd_plan** plan_out) {
  if (!ctx || !plan_out) return RD_EINVAL;
  *plan_out = nullptr;
  if (n_pairs && !pairs) return RD_EINVAL;
  if (n_models && (!models || !launch || !params)) return RD_EINVAL;
  rd_options o;
  memset(&o, 0, sizeof o);
  if (opt) o = *opt;
  if (o.mode > RD_MODE_VERDICT || o.order > RD_ORDER_INTERVAL) return RD_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return RD_EDEVICE;
  rd_plan* plan = new rd_plan();
  std::unique_ptr<rd_plan> guard(plan);
  plan->arena = ctx->arena;
  plan->n_pairs = n_pairs;
  // log_level >= 1: the duration of each preparation phase on stderr
  double t_phase = now_ms();
  const char* phase = "start";
  auto ptime = [&](const char* next) {
    const double t = now_ms();
    if (o.log_level >= 1) fprintf(stderr, "[hgrd] prepare %s: %.1f ms\n", phase, t - t_phase);
    t_phase = t;
    phase = next;
  };
  plan->st = o.stream ? (hipStream_t)o.stream : ctx->stream;
  plan->log_level = o.log_level;
  int cfg = ctx->cfg;
  if (o.lds_cap) cfg = o.lds_cap <= 1024 ? 0 : o.lds_cap <= 1536 ? 1 : 2;
  plan->cfg = cfg;
  const uint32_t cap = (uint32_t)join_cap(cfg);
  plan->cap = cap;
  {
    // as many join workgroups as the CUs' LDS holds at once (160 KiB each)
    uint32_t per_cu = (160u * 1024u) / (uint32_t)join_lds_bytes(cfg);
    per_cu = std::max(1u, std::min(per_cu, 8u));
    plan->persist_grid = per_cu * ctx->n_cu;
  }

  // effective addresses of aliased views (validation stays on `models`)
  ModelViews views;
  build_views(models, n_models, views);
  const rd_kernel_model* vmodels = views.m.data();
  Planner P;
  P.models = vmodels;
  P.launch = launch;
  P.params = params;
  P.dims.resize(n_models);
  P.use_tables = getenv("HGRD_INTERP") == nullptr;
  std::vector<uint32_t> model_err(n_models, 0);
  for (uint32_t m = 0; m < n_models; ++m) {
    const rd_kernel_model& M = models[m];
    uint32_t e = 0;
    if (launch[m].warp_size < 1 || launch[m].warp_size > 1024) e |= ERR_INVAL;
    if (params[m].n_sets && !params[m].values) e |= ERR_INVAL;
    if (M.n_acc && !M.acc) e |= ERR_INVAL;
    if (!(e & ERR_INVAL)) {
      for (int k = 0; k < 3; ++k)
        e |= check_expr(M, launch[m].grid[k], CTX_LAUNCH, nullptr) |
             check_expr(M, launch[m].block[k], CTX_LAUNCH, nullptr);
      if (params[m].n_sets > kMaxSets) e |= ERR_UNSUP;
    }
    model_err[m] = e;
    P.dims[m].resize(e ? 0 : params[m].n_sets);
  }

  // ---- per pair: validation, masks, instances -----------------------------
  ptime("validate");
  std::vector<QPlan>& Q = plan->Q;
  Q.resize(n_pairs);
  for (uint32_t k = 0; k < n_pairs; ++k) {
    QPlan& q = Q[k];
    const rd_access_pair& pr = pairs[k];
    q.qd.mask = 0;
    q.qd.self = 0;
    q.qd.warp = 32;
    q.qd.shared = 0;
    if (pr.model >= n_models) { q.host_err = ERR_INVAL; continue; }
    const rd_kernel_model& M = models[pr.model];
    if (pr.a >= M.n_acc || pr.b >= M.n_acc) { q.host_err = ERR_INVAL; continue; }
    const rd_access& A = M.acc[pr.a];
    const rd_access& B = M.acc[pr.b];
    uint32_t e = check_access(M, A) | check_access(M, B);
    // one memory: the same array, or two views of one aliased memory
    if (!(e & ERR_INVAL) && A.array != B.array &&
        memory_of(M, A.array) != memory_of(M, B.array))
      e |= ERR_INVAL;
    if (!(e & ERR_INVAL)) e |= model_err[pr.model];
    if (e & ERR_INVAL) e = ERR_INVAL;
    q.host_err = e;
    if (e) continue;
    q.qd.mask = class_mask(M, A, B, pr.class_mask);
    q.qd.self = pr.a == pr.b;
    q.qd.warp = launch[pr.model].warp_size;
    q.qd.shared = M.arrays[A.array].space == RD_SHARED;
    if (q.qd.mask == 0) { q.trivial = 1; continue; }
    q.sync = pair_sync(M, A, B);
    q.lower = 1;
  }

  // ---- lowering of the instances the pairs use, in parallel ----------------
  ptime("lower");
  // Models are dealt to a fixed number of groups (so the plan does not
  // depend on the host), each lowered by its own planner on a host thread,
  // then appended to P in group order; P's memo then answers every
  // instance query below.  Each group may use its share of the table pool.
  {
    constexpr uint32_t kGroups = 16;
    std::vector<std::vector<uint32_t>> gpairs(kGroups);
    std::vector<uint64_t> gcost(kGroups, 0);
    std::vector<int32_t> mgroup(n_models, -1);
    uint64_t lowered = 0;
    for (uint32_t k = 0; k < n_pairs; ++k) {
      if (!Q[k].lower) continue;
      const uint32_t m = pairs[k].model;
      if (mgroup[m] < 0) {
        // the group with the least work so far
        uint32_t g = 0;
        for (uint32_t x = 1; x < kGroups; ++x)
          if (gcost[x] < gcost[g]) g = x;
        mgroup[m] = (int32_t)g;
      }
      const uint32_t g = (uint32_t)mgroup[m];
      gpairs[g].push_back(k);
      gcost[g] += params[m].n_sets;
      lowered += params[m].n_sets;
    }
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const uint32_t nthreads = lowered < 4096 ? 1u : std::min<uint32_t>(kGroups, hw);
    if (nthreads > 1) {
      std::vector<Planner> sub(kGroups);
      for (Planner& G : sub) {
        G.models = vmodels;
        G.launch = launch;
        G.params = params;
        G.dims.resize(n_models);
        for (uint32_t m = 0; m < n_models; ++m) G.dims[m].resize(P.dims[m].size());
        G.use_tables = P.use_tables;
        G.tab_budget = kMaxTabPool / kGroups;
      }
      std::atomic<uint32_t> next{0};
      auto work = [&]() {
        for (;;) {
          const uint32_t g = next.fetch_add(1);
          if (g >= kGroups) return;
          for (uint32_t k : gpairs[g]) {
            const rd_access_pair& pr = pairs[k];
            for (uint32_t s = 0; s < params[pr.model].n_sets; ++s) {
              sub[g].inst(pr.model, pr.a, s);
              if (pr.b != pr.a) sub[g].inst(pr.model, pr.b, s);
            }
          }
        }
      };
      std::vector<std::thread> th;
      for (uint32_t t = 1; t < nthreads; ++t) th.emplace_back(work);
      work();
      for (auto& t : th) t.join();
      for (Planner& G : sub) P.absorb(G);
    }
  }

  for (uint32_t k = 0; k < n_pairs; ++k) {
    QPlan& q = Q[k];
    if (!q.lower) continue;
    const rd_access_pair& pr = pairs[k];
    const uint32_t ns = params[pr.model].n_sets;
    q.inst.assign(ns, {-1, -1});
    for (uint32_t s = 0; s < ns; ++s) {
      InstInfo& ia = P.inst(pr.model, pr.a, s);
      q.host_err |= ia.err;
      q.evals += ia.box;
      int32_t ib_idx = ia.idx;
      if (q.qd.self) {
        q.evals += ia.box;
      } else {
        InstInfo& ib = P.inst(pr.model, pr.b, s);
        q.host_err |= ib.err;
        q.evals += ib.box;
        ib_idx = ib.idx;
      }
      q.inst[s] = {ia.idx, ib_idx};
    }
    q.work = !(q.host_err & (ERR_INVAL | ERR_UNSUP));
    // interval ids constant and equal on both sides in every tuple
    {
      // component c (0 bint, 1 wint) of instance x is a known constant
      auto iv_const = [&](int32_t x, int c, uint32_t& v) -> bool {
        const TabHost& T = P.tabs[x];
        if (T.on && T.iv_off == kNoTab) {
          v = c ? (T.iv_const >> 16) : (T.iv_const & 0xFFFF);
          return true;
        }
        const Prog& pg = c ? P.dev_insts[x].wint : P.dev_insts[x].bint;
        v = 0;
        return pg.absent != 0;
      };
      uint32_t fl = 3;
      for (const auto& pr2 : q.inst) {
        if (pr2.first < 0 || pr2.second < 0) continue;
        for (int c = 0; c < 2; ++c) {
          uint32_t va = 0, vb = 0;
          if (!iv_const(pr2.first, c, va) || !iv_const(pr2.second, c, vb) || va != vb)
            fl &= ~(1u << c);
        }
      }
      // bit 2: both accesses compute their address with the same expression
      if (same_addr_expr(vmodels[pr.model], pr.a, pr.b)) fl |= 4;
      // bits 3, 4: synchronised pairs whose syn() can match (block, device)
      if (q.sync & kQSyncBlk) fl |= 8;
      if (q.sync & kQSyncDev) fl |= 16;
      q.qd.flags = fl;
    }
  }

  // ---- items ----------------------------------------------------------------
  ptime("items");
  struct HPlan {
    HItem h;
    uint64_t R;
  };
  std::vector<SItem> sitems;
  // block symmetry of shared-array units (HGRD_NO_SYMMETRY turns it off)
  const bool block_sym = getenv("HGRD_NO_SYMMETRY") == nullptr;
  // unit filter decisions for synchronised pairs (HGRD_NO_UNIT_FILTER)
  const bool unit_filter = getenv("HGRD_NO_UNIT_FILTER") == nullptr;
  // synchronised units through the LDS joins when they qualify
  // (HGRD_SYNC_FALLBACK sends them all to the HBM aggregation path)
  const bool sync_lds = getenv("HGRD_SYNC_FALLBACK") == nullptr;
  std::vector<HPlan> hplans;
  auto npts_of = [&](int32_t idx) -> uint64_t {
    return idx < 0 ? 0 : P.dev_insts[idx].npts;
  };
  // Dense items: every side (one for a self pair) has at least dense_min
  // points per address of its proven range on average (per block for
  // shared arrays); their buckets nearly all hold partners, so the address
  // filter is not worth its read (HGRD_DENSE sets dense_min; 0 turns it
  // off).  Counting points rather than threads measured better on the
  // mixed workload (7 520 against 7 265 queries/s), though an access that
  // meets only itself across iterations then skips a filter that would
  // have dropped all its buckets.
  double dense_min = 1.5;
  if (const char* e = getenv("HGRD_DENSE")) dense_min = atof(e);
  auto dense_item = [&](int32_t ia, int32_t ib, bool self, bool shared) -> bool {
    if (dense_min <= 0) return false;
    for (int32_t x : {ia, ib}) {
      if (self && x == ib && ia == ib) continue;
      if (!P.tabs[x].on) return false;
      const double span = (double)P.arange[x].second - (double)P.arange[x].first + 1.0;
      if (span < 1) return false;
      const double pts = shared ? P.dev_insts[x].tpb : P.dev_insts[x].npts;
      if (pts / span < dense_min) return false;
    }
    return true;
  };
  // Bucket shift of an HBM item: blocks of 2^shift consecutive addresses
  // should hold about block_recs records, from the density (points per
  // address of the tabulated range; per block for shared arrays) of the
  // denser side.
  double block_recs = 32;
  if (const char* e = getenv("HGRD_BLOCK_RECS")) block_recs = std::max(1, atoi(e));
  auto item_shift = [&](int32_t ia, int32_t ib, bool self, bool shared) -> uint32_t {
    double dens = 0;
    for (int32_t x : {ia, ib}) {
      if (self && x == ib) continue;
      if (!P.tabs[x].on) return 0;
      const double span = (double)P.arange[x].second - (double)P.arange[x].first + 1.0;
      if (span < 1) return 0;
      // shared arrays and block-symmetric units: points of one block
      const double pts = shared ? P.dev_insts[x].tpb : P.dev_insts[x].npts;
      dens = std::max(dens, pts / span);
    }
    const double target = block_recs;
    if (dens <= 0 || target / dens < 2.0) return 0;
    return (uint32_t)std::min(30.0, std::floor(std::log2(target / dens)));
  };
  for (uint32_t k = 0; k < n_pairs; ++k) {
    QPlan& q = Q[k];
    if (!q.work) continue;
    for (uint32_t s = 0; s < q.inst.size(); ++s) {
      int32_t ia = q.inst[s].first, ib = q.inst[s].second;
      if (ia < 0 && ib < 0) continue;
      if (q.sync && unit_filter && ia >= 0 && ib >= 0 && P.tabs[ia].on && P.tabs[ib].on &&
          P.tabs[ia].syn_safe && P.tabs[ib].syn_safe &&
          ((ia != ib && P.apart(ia, ib)) || ((q.qd.flags & 4) && P.tinj[ia] && P.tinj[ib]))) {
        // no address is shared, or each address is reached by one thread
        // only: no conflict, so nothing to synchronise either, and no
        // expression of either access can fail (term tables, acquire and
        // release addresses proven error-free); the unit filter's decision
        ++plan->sync_decided;
        continue;
      }
      if (q.sync && sync_lds && cfg < 2 && ia >= 0 && ib >= 0 && P.tabs[ia].on && P.tabs[ib].on &&
          P.tabs[ia].syn_safe && P.tabs[ib].syn_safe) {
        // acquire/release on the pair, every expression proven error-free:
        // partitioned through HBM and joined in LDS with the
        // synchronisation levels (a bucket that overflows goes to the
        // fallback)
        HPlan hp;
        memset(&hp, 0, sizeof hp);
        hp.h.q = k;
        hp.h.sigma = s;
        hp.h.inst_i = (uint32_t)ia;
        hp.h.inst_j = (uint32_t)ib;
        hp.h.shared = q.qd.shared;
        hp.h.is32 = P.dev_insts[ia].is32;
        hp.h.sync = 1;
        hp.h.shift = item_shift(ia, ib, q.qd.self, q.qd.shared);
        fastdiv_consts(P.dev_insts[ia].tpb, &hp.h.tpb_m[0], &hp.h.tpb_s[0]);
        fastdiv_consts(P.dev_insts[ib].tpb, &hp.h.tpb_m[1], &hp.h.tpb_s[1]);
        hp.R = npts_of(ia) + (q.qd.self ? 0 : npts_of(ib));
        hplans.push_back(hp);
        continue;
      }
      if (q.sync) {
        // acquire/release on the pair: the HBM aggregation path, whose
        // records carry each point's synchronisation address and which
        // scans every point's expressions for errors (one side only, with
        // nothing joined, when the other has no points)
        rd_plan_impl::SyncUnit u;
        u.q = k;
        u.sigma = s;
        u.scan = ia < 0 || ib < 0;
        u.inst_i = (uint32_t)(ia >= 0 ? ia : ib);
        u.inst_j = (uint32_t)(u.scan ? u.inst_i : (uint32_t)ib);
        u.R = u.scan ? npts_of((int32_t)u.inst_i)
                     : npts_of(ia) + (q.qd.self ? 0 : npts_of(ib));
        plan->sync_units.push_back(u);
        continue;
      }
      if (ia < 0 || ib < 0) {
        // one side has no points because its loops failed: the pair already
        // carries that error, but the other side's points are still scanned
        // for errors (a stronger one may be among them); nothing is joined
        int32_t ref = ia >= 0 ? ia : ib;
        HPlan hp;
        memset(&hp, 0, sizeof hp);
        hp.h.q = k;
        hp.h.sigma = s;
        hp.h.inst_i = (uint32_t)ref;
        hp.h.inst_j = (uint32_t)ref;
        hp.h.is32 = P.dev_insts[ref].is32;
        hp.R = npts_of(ref);
        hp.h.shared = 2;  // error scan only
        hplans.push_back(hp);
        continue;
      }
      if (o.prefilter && ia != ib && P.tabs[ia].on && P.tabs[ib].on) {
        // exact pre-filters: no address of one access equals an address of
        // the other, so no pair conflicts.  (1) The address ranges over the
        // whole launch box (term-table bounds) do not meet.  (2) The
        // residues are incompatible: addresses of a are u_a + k G_a, of b
        // u_b + k G_b, and a common one needs gcd(G_a, G_b) | u_a - u_b.
        // (3) The per-block intervals of a and b miss each other.
        if (P.apart(ia, ib)) {
          ++plan->prefiltered;
          continue;
        }
      }
      const AccInst& R0 = P.dev_insts[ia];
      const uint64_t na = npts_of(ia), nb = q.qd.self ? 0 : npts_of(ib);
      const uint64_t tot = na + nb;
      const uint64_t per_block =
          (uint64_t)P.dev_insts[ia].tpb + (q.qd.self ? 0 : P.dev_insts[ib].tpb);
      if (tot <= cap) {
        SItem it;
        memset(&it, 0, sizeof it);
        it.q = k;
        it.sigma = s;
        it.inst_i = (uint32_t)ia;
        it.inst_j = (uint32_t)ib;
        it.b0 = 0;
        it.b1 = R0.nblk;
        sitems.push_back(it);
      } else if (!q.qd.shared && per_block <= cap && block_sym && R0.nblk > 1 &&
                 P.tabs[ia].on && P.tabs[ib].on && P.tabs[ia].off[0] == kNoTab &&
                 P.tabs[ib].off[0] == kNoTab) {
        // block symmetry of a global array: neither access's address nor
        // guard has a block term, so every block holds the same points at
        // the same addresses.  Block 0 is joined; its address groups stand
        // for G identical groups (S_0 = G^2 S_0(block 0), every other level
        // G times block 0's), and its witness, in the smallest block, is
        // the smallest of all.
        SItem it;
        memset(&it, 0, sizeof it);
        it.q = k;
        it.sigma = s;
        it.inst_i = (uint32_t)ia;
        it.inst_j = (uint32_t)ib;
        it.b0 = 0;
        it.b1 = 1;
        it.mult = R0.nblk;
        it.gsym = 1;
        sitems.push_back(it);
        ++plan->n_symmetric;
      } else if (!q.qd.shared && block_sym && R0.nblk > 1 && P.tabs[ia].on &&
                 P.tabs[ib].on && P.tabs[ia].off[0] == kNoTab &&
                 P.tabs[ib].off[0] == kNoTab) {
        // the same symmetry for a block too large for one LDS tile: block
        // 0's points alone go through the HBM partition (the first tpb
        // points of each side, the block being slowest in the point order),
        // and the joins scale as above.  Overflow goes to the fallback (a
        // split by (address, block) has nothing to split in one block).
        HPlan hp;
        memset(&hp, 0, sizeof hp);
        hp.h.q = k;
        hp.h.sigma = s;
        hp.h.inst_i = (uint32_t)ia;
        hp.h.inst_j = (uint32_t)ib;
        hp.h.shared = 0;
        hp.h.is32 = R0.is32;
        hp.h.gmult = R0.nblk;
        hp.h.shift = item_shift(ia, ib, q.qd.self, true);
        fastdiv_consts(P.dev_insts[ia].tpb, &hp.h.tpb_m[0], &hp.h.tpb_s[0]);
        fastdiv_consts(P.dev_insts[ib].tpb, &hp.h.tpb_m[1], &hp.h.tpb_s[1]);
        hp.R = per_block;
        hplans.push_back(hp);
        ++plan->n_symmetric;
      } else if (q.qd.shared && per_block <= cap && block_sym &&
                 P.tabs[ia].on && P.tabs[ib].on && P.tabs[ia].off[0] == kNoTab &&
                 P.tabs[ib].off[0] == kNoTab) {
        // block symmetry: shared memory belongs to one block, and neither
        // access's address nor guard has a term in the block coordinates
        // (interval ids depend on loop values only), so every block holds
        // the same points and the same conflicts.  Block 0 is joined and its
        // counts are taken nblk times; its witness, having the smallest
        // block, is the smallest of all.
        SItem it;
        memset(&it, 0, sizeof it);
        it.q = k;
        it.sigma = s;
        it.inst_i = (uint32_t)ia;
        it.inst_j = (uint32_t)ib;
        it.b0 = 0;
        it.b1 = 1;
        it.mult = R0.nblk;
        sitems.push_back(it);
        ++plan->n_symmetric;
      } else if (q.qd.shared && per_block <= cap) {
        uint32_t bpi = (uint32_t)(cap / per_block);
        for (uint32_t b0 = 0; b0 < R0.nblk; b0 += bpi) {
          SItem it;
          memset(&it, 0, sizeof it);
          it.q = k;
          it.sigma = s;
          it.inst_i = (uint32_t)ia;
          it.inst_j = (uint32_t)ib;
          it.b0 = b0;
          it.b1 = std::min(R0.nblk, b0 + bpi);
          sitems.push_back(it);
        }
      } else {
        HPlan hp;
        memset(&hp, 0, sizeof hp);
        hp.h.q = k;
        hp.h.sigma = s;
        hp.h.inst_i = (uint32_t)ia;
        hp.h.inst_j = (uint32_t)ib;
        hp.h.shared = q.qd.shared;
        hp.h.is32 = R0.is32;
        hp.h.shift = item_shift(ia, ib, q.qd.self, q.qd.shared);
        fastdiv_consts(P.dev_insts[ia].tpb, &hp.h.tpb_m[0], &hp.h.tpb_s[0]);
        fastdiv_consts(P.dev_insts[ib].tpb, &hp.h.tpb_m[1], &hp.h.tpb_s[1]);
        hp.R = tot;
        hp.h.dense = dense_item(ia, ib, q.qd.self, q.qd.shared) ? 1u : 0u;
        hplans.push_back(hp);
      }
    }
  }
  // longest first: the persistent join pops items in this order
  std::stable_sort(sitems.begin(), sitems.end(), [&](const SItem& x, const SItem& y) {
    auto size = [&](const SItem& it) {
      uint64_t a = (uint64_t)(it.b1 - it.b0) * P.dev_insts[it.inst_i].tpb;
      if (!Q[it.q].qd.self) a += (uint64_t)(it.b1 - it.b0) * P.dev_insts[it.inst_j].tpb;
      return a;
    };
    return size(x) > size(y);
  });
  plan->n_sitems = (uint32_t)sitems.size();

  // ---- VERDICT mode: search units, their blocks, tiles and rounds ----------
  ptime("verdict");
  std::vector<VQuery> vqs;
  std::vector<BItem> bitems;
  std::vector<TChunk> tchunks;
  std::vector<TItem> titems;
  if (o.mode == RD_MODE_VERDICT) {
    plan->verdict = true;
    plan->score_mode = o.order == RD_ORDER_MLP ? 1u : o.order == RD_ORDER_INTERVAL ? 2u : 0u;
    if (plan->score_mode == 1 && !o.mlp) return RD_EINVAL;
    plan->K = o.tile_budget ? o.tile_budget : 256;
    for (uint32_t k = 0; k < n_pairs; ++k) {
      QPlan& q = Q[k];
      if (!q.work || q.host_err || q.trivial || q.qd.shared || q.inst.empty() || q.sync)
        continue;
      bool ok = true;
      for (auto& pr : q.inst) {
        if (pr.first < 0 || pr.second < 0) { ok = false; break; }
        const AccInst& A = P.dev_insts[pr.first];
        const AccInst& B = P.dev_insts[pr.second];
        uint64_t tiles = (uint64_t)A.nblk * A.nblk;
        uint64_t per = q.qd.self ? 2ull * A.tpb : (uint64_t)A.tpb + B.tpb;
        if (tiles > (1u << 20) || per > cap || A.nblk != B.nblk) { ok = false; break; }
      }
      if (!ok) continue;
      const rd_access_pair& pr = pairs[k];
      const rd_kernel_model& M = models[pr.model];
      uint32_t kinds = M.acc[pr.a].kind * 3 + M.acc[pr.b].kind;
      plan->n_vqueries_pairs++;
      for (uint32_t s = 0; s < q.inst.size(); ++s) {
        const AccInst& A = P.dev_insts[q.inst[s].first];
        const AccInst& B = P.dev_insts[q.inst[s].second];
        VQuery v;
        memset(&v, 0, sizeof v);
        v.q = k;
        v.sigma = s;
        v.inst_i = (uint32_t)q.inst[s].first;
        v.inst_j = (uint32_t)q.inst[s].second;
        v.G = A.nblk;
        v.bb_i = (uint32_t)bitems.size();
        for (uint32_t b = 0; b < A.nblk; ++b)
          bitems.push_back({v.inst_i, b, k, (uint32_t)bitems.size()});
        if (q.qd.self) {
          v.bb_j = v.bb_i;
        } else {
          v.bb_j = (uint32_t)bitems.size();
          for (uint32_t b = 0; b < B.nblk; ++b)
            bitems.push_back({v.inst_j, b, k, (uint32_t)bitems.size()});
        }
        v.st_i = P.gstride[v.inst_i][0];
        v.sb_i = P.gstride[v.inst_i][1];
        v.st_j = P.gstride[v.inst_j][0];
        v.sb_j = P.gstride[v.inst_j][1];
        v.self = q.qd.self;
        v.tile0 = (uint32_t)plan->n_tiles;
        v.tpb_i = A.tpb;
        v.tpb_j = B.tpb;
        v.nthr = A.nthr;
        v.kinds = kinds;
        v.shared = 0;
        v.is64 = A.is32 ? 0 : 1;
        v.nsets = (uint32_t)q.inst.size();
        uint32_t nt = v.G * v.G;
        for (uint32_t t0 = 0; t0 < nt; t0 += 4096)
          tchunks.push_back({(uint32_t)vqs.size(), t0, std::min(nt, t0 + 4096), 0});
        plan->n_tiles += nt;
        plan->max_tiles = std::max(plan->max_tiles, nt);
        plan->max_g = std::max(plan->max_g, v.G);
        vqs.push_back(v);
      }
    }
    // rounds of geometrically growing rank ranges: [0,1), [1,4), [4,16) ...
    uint32_t lo = 0, width = 1;
    while (lo < plan->K) {
      uint32_t hi = std::min(plan->K, lo + width);
      uint32_t i0 = (uint32_t)titems.size();
      for (uint32_t v = 0; v < vqs.size(); ++v) {
        uint32_t nt = vqs[v].G * vqs[v].G;
        for (uint32_t r = lo; r < std::min(hi, nt); ++r) titems.push_back({v, r});
      }
      if (titems.size() > i0) plan->rounds.push_back({i0, (uint32_t)titems.size()});
      lo = hi;
      width *= 4;
    }
    plan->n_vq = (uint32_t)vqs.size();
    plan->vqs = vqs;
    plan->n_bitems = (uint32_t)bitems.size();
    // block bounds: instances with term tables from their tables (one lane
    // per block), the others by generating every point of the block
    std::vector<uint8_t> seen(P.dev_insts.size(), 0);
    for (const BItem& b : bitems) {
      if (P.tabs[b.inst].on) {
        if (!seen[b.inst]) plan->vinst_tab.push_back(b.inst);
        seen[b.inst] = 1;
      } else {
        plan->bitems_interp.push_back(b);
      }
    }
    plan->n_tchunks = (uint32_t)tchunks.size();
    plan->n_titems = (uint32_t)titems.size();
  }

  std::vector<uint8_t> tab_on(P.dev_insts.size());
  for (size_t i = 0; i < P.dev_insts.size(); ++i) tab_on[i] = (uint8_t)P.tabs[i].on;
  plan->no_map = getenv("HGRD_HASH_BUCKETS") != nullptr;
  if (const char* e = getenv("HGRD_CHUNK_PTS"))
    plan->chunk_pts = std::max(256u, std::min(1u << 20, (uint32_t)atoi(e)));
  if (const char* e = getenv("HGRD_RUN_BUCKETS"))
    plan->run_buckets = std::max(1u, std::min(kMaxRunBuckets, (uint32_t)atoi(e)));

  // ---- waves of HBM items, bounded by the device budget --------------------
  ptime("waves");
  // Large waves keep the partition and join launches few (each launch has a
  // tail); records cost 16 bytes of HBM traffic per point either way.
  const uint64_t budget = o.max_device_bytes ? o.max_device_bytes : ctx->wave_bytes;
  plan->wave_budget = budget;
  // Global items whose addresses carry on average a bucket of points or
  // more overflow any bucket map (one address never spans buckets): they
  // skip the first phase and go straight to the (address, block) split.
  std::vector<HPlan> pre;
  if (!plan->no_map) {
    size_t w = 0;
    for (size_t i = 0; i < hplans.size(); ++i) {
      HPlan hp = hplans[i];
      bool ps = false;
      const uint32_t a = hp.h.inst_i, b = hp.h.inst_j;
      if (hp.h.shared == 0 && hp.h.gmult <= 1 && !hp.h.sync && tab_on[a] && tab_on[b]) {
        const double lo = (double)std::min(P.arange[a].first, P.arange[b].first);
        const double hi = (double)std::max(P.arange[a].second, P.arange[b].second);
        if (hi >= lo && (double)hp.R >= (hi - lo + 1.0) * cap) {
          set_bucket_map(hp.h, tab_on, P.arange, P.dev_insts[a].nblk, Q[hp.h.q].qd.self,
                         false, hp.R, cap, 0.6);
          ps = hp.h.mode != 0;
        }
      }
      if (ps) pre.push_back(hp);
      else hplans[w++] = hplans[i];
    }
    hplans.resize(w);
  }
  // Chunks and runs are described compactly, one spec per (item, side) and
  // per item in launch order, and expanded on the device at the end of
  // rd_prepare (k_expand): a batch can have tens of millions of them.
  std::vector<ExpandSpec> chunk_specs, run_specs;
  uint64_t n_all_chunks = 0, n_all_runs = 0;
  size_t pos = 0;
  while (pos < hplans.size()) {
    rd_plan_impl::Wave W;
    memset(&W, 0, sizeof W);
    W.first_item = (uint32_t)plan->hitems.size();
    W.hitem_off = plan->hitems.size();
    W.chunk_off = n_all_chunks;
    W.bitem_off = n_all_runs;
    size_t end = pos;
    uint64_t bytes = 0, nbk = 0;
    while (end < hplans.size()) {
      HPlan& hp = hplans[end];
      uint64_t nbuckets =
          hp.h.shared == 2 ? 0
                           : std::max<uint64_t>(1, (hp.R * 100 + cap * 55 - 1) / (cap * 55));
      if (hp.h.shared != 2 && !plan->no_map) {
        set_bucket_map(hp.h, tab_on, P.arange,
                       hp.h.gmult > 1 ? 1u : P.dev_insts[hp.h.inst_i].nblk,
                       Q[hp.h.q].qd.self, hp.h.shared == 1, hp.R, cap, 0.6);
        if (hp.h.mode) nbuckets = hp.h.nbuckets;
      }
      const uint64_t need = nbuckets * cap * (hp.h.is32 ? 8 : 16);
      if (end > pos && bytes + need > budget) break;
      hp.h.nbuckets = (uint32_t)nbuckets;
      hp.h.bucket0 = (uint32_t)nbk;
      hp.h.rec_off = bytes;
      bytes += (need + 255) / 256 * 256;
      nbk += nbuckets;
      ++end;
    }
    // chunks and runs of items with term tables first, then the others
    std::vector<ExpandSpec> interp, interp_runs, sync_runs;
    uint64_t tab_chunks = 0, tab_runs = 0, oth_chunks = 0, oth_runs = 0, syn_runs = 0;
    for (size_t i = pos; i < end; ++i) {
      const HItem& h = hplans[i].h;
      uint32_t li = (uint32_t)plan->hitems.size();  // global item index
      plan->hitems.push_back(h);
      plan->hR.push_back(hplans[i].R);
      plan->presplit.push_back(0);
      const bool tr = P.tabs[h.inst_i].on && P.tabs[h.inst_j].on;
      const uint32_t nr = (h.nbuckets + plan->run_buckets - 1) / plan->run_buckets;
      if (nr && h.sync) {
        sync_runs.push_back({li, 0, h.nbuckets, plan->run_buckets, 0});
        syn_runs += nr;
      } else if (nr) {
        (tr ? run_specs : interp_runs).push_back({li, 0, h.nbuckets, plan->run_buckets, 0});
        (tr ? tab_runs : oth_runs) += nr;
      }
      const QPlan& q = Q[h.q];
      for (int side = 0; side < (q.qd.self || h.shared == 2 ? 1 : 2); ++side) {
        uint32_t inst = side ? h.inst_j : h.inst_i;
        // block-symmetric units: block 0's points only
        uint32_t np = h.gmult > 1 ? P.dev_insts[inst].tpb : P.dev_insts[inst].npts;
        const uint32_t nc = (np + plan->chunk_pts - 1) / plan->chunk_pts;
        if (!nc) continue;
        (P.tabs[inst].on ? chunk_specs : interp).push_back(
            {li, (uint32_t)side, np, plan->chunk_pts, 0});
        (P.tabs[inst].on ? tab_chunks : oth_chunks) += nc;
      }
    }
    chunk_specs.insert(chunk_specs.end(), interp.begin(), interp.end());
    run_specs.insert(run_specs.end(), interp_runs.begin(), interp_runs.end());
    run_specs.insert(run_specs.end(), sync_runs.begin(), sync_runs.end());
    W.n_tab_chunks = (uint32_t)tab_chunks;
    W.n_tab_runs = (uint32_t)tab_runs;
    W.n_sync_runs = (uint32_t)syn_runs;
    W.n_items = (uint32_t)(end - pos);
    W.n_runs = (uint32_t)(tab_runs + oth_runs + syn_runs);
    W.n_chunks = (uint32_t)(tab_chunks + oth_chunks);
    n_all_chunks += W.n_chunks;
    n_all_runs += W.n_runs;
    W.n_buckets = (uint32_t)nbk;
    W.key_bytes = bytes;
    plan->max_key_bytes = std::max(plan->max_key_bytes, bytes);
    plan->max_buckets = std::max(plan->max_buckets, nbk);
    plan->max_items = std::max<uint64_t>(plan->max_items, W.n_items);
    plan->waves.push_back(W);
    pos = end;
  }
  for (HPlan& hp : pre) {  // after every wave: no chunks, runs or buckets
    hp.h.bucket0 = 0;
    hp.h.rec_off = 0;
    plan->hitems.push_back(hp.h);
    plan->hR.push_back(hp.R);
    plan->presplit.push_back(1);
  }

  // ---- upload descriptors -----------------------------------------------------
  ptime("upload");
  int merr = 0;
  const size_t isz = devinst_size();
  const int64_t* d_tpool = (const int64_t*)plan->buf("tpool", std::max<uint64_t>(1, P.tpool) * 8, &merr);
  std::vector<unsigned char> dinst(isz * std::max<size_t>(1, P.dev_insts.size()));
  for (size_t i = 0; i < P.dev_insts.size(); ++i) {
    fill_devinst(dinst.data() + i * isz, P.dev_insts[i]);
    set_devinst_tab(dinst.data() + i * isz, P.tabs[i], d_tpool);
    plan->tab_insts += P.tabs[i].on;
  }
  std::vector<Chunk> tabchunks;
  for (uint32_t j = 0; j < P.tjobs.size(); ++j)
    for (uint32_t e = 0; e < P.tjobs[j].n; e += 1024)
      tabchunks.push_back(Chunk{j, 0, e, std::min<uint32_t>(P.tjobs[j].n, e + 1024)});
  plan->n_tabchunks = (uint32_t)tabchunks.size();
  plan->n_insts = (uint32_t)P.dev_insts.size();
  plan->npts.resize(P.dev_insts.size());
  plan->nblk.resize(P.dev_insts.size());
  plan->tpb.resize(P.dev_insts.size());
  for (size_t i = 0; i < P.dev_insts.size(); ++i) {
    plan->npts[i] = P.dev_insts[i].npts;
    plan->nblk[i] = P.dev_insts[i].nblk;
    plan->tpb[i] = P.dev_insts[i].tpb;
  }
  plan->tab_on = tab_on;
  plan->arange = P.arange;
  std::vector<QDesc> qd(n_pairs);
  std::vector<uint32_t> herr(n_pairs);
  std::vector<uint8_t> triv(n_pairs);
  std::vector<u64> evals(n_pairs);
  for (uint32_t k = 0; k < n_pairs; ++k) {
    qd[k] = Q[k].qd;
    herr[k] = Q[k].host_err;
    triv[k] = Q[k].trivial;
    evals[k] = Q[k].evals;
    plan->evals += Q[k].evals;
  }
  auto up = [&](const char* name, const void* src, size_t bytes) -> void* {
    void* d = plan->buf(name, bytes, &merr);
    if (d && bytes && hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
      merr = RD_EDEVICE;
    return d;
  };
  if (P.code.empty()) P.code.push_back(DInsn{});
  if (P.pool_params.empty()) P.pool_params.push_back(0);
  if (P.pool_loops.empty()) P.pool_loops.push_back(0);
  up("code", P.code.data(), P.code.size() * sizeof(DInsn));
  up("params", P.pool_params.data(), P.pool_params.size() * 8);
  up("loops", P.pool_loops.data(), P.pool_loops.size() * 8);
  up("insts", dinst.data(), dinst.size());
  up("tabjobs", P.tjobs.data(), P.tjobs.size() * sizeof(TabJob));
  up("tabchunks", tabchunks.data(), tabchunks.size() * sizeof(Chunk));
  up("qdesc", qd.data(), n_pairs * sizeof(QDesc));
  up("herr", herr.data(), n_pairs * 4);
  up("triv", triv.data(), n_pairs);
  up("evals", evals.data(), n_pairs * 8);
  up("sitems", sitems.data(), sitems.size() * sizeof(SItem));
  up("hitems", plan->hitems.data(), plan->hitems.size() * sizeof(HItem));
  {
    // every chunk and run, expanded on the device from their specs
    auto expand = [&](std::vector<ExpandSpec>& sp, const char* name, uint64_t total,
                      bool runs) {
      uint64_t at = 0;
      for (ExpandSpec& e : sp) {
        e.first = at;
        at += (e.n + e.per - 1) / e.per;
      }
      void* out = plan->buf(name, std::max<uint64_t>(1, total) * 16, &merr);
      if (merr || sp.empty()) return;
      const char* sname = runs ? "run_specs" : "chunk_specs";
      void* d = up(sname, sp.data(), sp.size() * sizeof(ExpandSpec));
      if (merr || !d) return;
      if (launch_expand(plan->st, (const ExpandSpec*)d, (uint32_t)sp.size(), total, runs, out) ||
          hipStreamSynchronize(plan->st) != hipSuccess)
        merr = RD_EDEVICE;
    };
    expand(chunk_specs, "chunks", n_all_chunks, false);
    expand(run_specs, "runs", n_all_runs, true);
  }
  {
    // proven facts per instance for the unit filter of rd_execute
    std::vector<IFact> facts(std::max<size_t>(1, P.dev_insts.size()));
    memset(facts.data(), 0, facts.size() * sizeof(IFact));
    for (size_t i = 0; i < P.dev_insts.size(); ++i) {
      if (!P.tabs[i].on) continue;
      facts[i].lo = P.arange[i].first;
      facts[i].hi = P.arange[i].second;
      facts[i].G = P.ares[i].first;
      facts[i].u = P.ares[i].second;
      facts[i].on = 1;
      facts[i].inj = P.tinj[i];
    }
    up("ifacts", facts.data(), facts.size() * sizeof(IFact));
  }
  if (plan->verdict) {
    up("vq", vqs.data(), vqs.size() * sizeof(VQuery));
    up("bitems", bitems.data(), bitems.size() * sizeof(BItem));
    up("tchunks", tchunks.data(), tchunks.size() * sizeof(TChunk));
    up("titems", titems.data(), titems.size() * sizeof(TItem));
    plan->buf("bbounds", std::max<size_t>(1, bitems.size()) * sizeof(BBound), &merr);
    if (plan->score_mode) {
      plan->buf("order", std::max<size_t>(1, (size_t)vqs.size() * plan->K) * 4, &merr);
      if (plan->score_mode == 1) up("mlp_w", o.mlp, (size_t)mlp_num_weights() * 4);
    }
    up("vinst", plan->vinst_tab.data(), plan->vinst_tab.size() * 4);
    up("bitems_i", plan->bitems_interp.data(), plan->bitems_interp.size() * sizeof(BItem));
    plan->buf("irange", std::max<size_t>(1, P.dev_insts.size()) * sizeof(InstRange), &merr);
    plan->buf("tout", std::max<size_t>(1, titems.size()) * sizeof(TOut), &merr);
    plan->buf("claim", std::max<size_t>(1, n_pairs) * 8, &merr);
  }
  plan->buf("qacc", std::max<size_t>(1, n_pairs) * sizeof(QAcc), &merr);
  // partition scratch of the first phase: shared by the context's plans
  // (its addresses stay valid while a plan holds them, as a captured graph
  // needs); in an arena call it is carved from the arena like the rest
  auto scratch = [&](const char* name, size_t bytes) {
    if (plan->arena) {
      plan->buf(name, bytes, &merr);
      return;
    }
    void* p = ctx->shared_buf(name, bytes, &merr);
    DevBuf& b = plan->dev[name];
    b.p = p;
    b.cap = bytes;
    b.own = false;
  };
  scratch("recs", plan->max_key_bytes);
  scratch("cursor", plan->max_buckets * 4);
  plan->buf("ovf", std::max<size_t>(1, plan->hitems.size()) * 4, &merr);
  plan->buf("done", std::max<size_t>(1, n_pairs) * 4, &merr);
  plan->buf("pcursor", 4, &merr);
  plan->buf("nbytes", 512 * 8, &merr);
  scratch("cand", std::max<uint64_t>(1, plan->max_buckets));
  plan->buf("out", std::max<size_t>(1, n_pairs) * sizeof(rd_pair_result), &merr);
  if (merr) return merr;
  ptime("done");
  *plan_out = guard.release();
  return RD_OK;
}

void rd_plan_destroy(rd_plan* plan) { delete plan; }

// VERDICT block bounds: instances with term tables from their tables, the
// others by generating their points.  Nonzero on a launch failure.
static int verdict_bounds(rd_plan* plan, hipStream_t st) {
  auto D = [&](const char* name) { return plan->dev[name].p; };
  BBound* d_bb = (BBound*)D("bbounds");
  if (!plan->vinst_tab.empty() &&
      launch_block_bounds_tab(st, (const uint32_t*)D("vinst"), (uint32_t)plan->vinst_tab.size(),
                              (const BItem*)D("bitems"), plan->n_bitems, D("insts"),
                              (InstRange*)D("irange"), d_bb))
    return 1;
  if (!plan->bitems_interp.empty() &&
      launch_block_bounds(st, (const BItem*)D("bitems_i"), (uint32_t)plan->bitems_interp.size(),
                          D("insts"), (const DInsn*)D("code"), (const int64_t*)D("params"),
                          (const int64_t*)D("loops"), (QAcc*)D("qacc"), d_bb))
    return 1;
  return 0;
}

int rd_execute(rd_context* ctx, rd_plan* plan, rd_pair_result* out) {
  if (!ctx || !plan) return RD_EINVAL;
  const uint32_t n_pairs = plan->n_pairs;
  if (n_pairs && !out) return RD_EINVAL;
  const double t_start = now_ms();
  if (hipSetDevice(ctx->device) != hipSuccess) return RD_EDEVICE;
  hipStream_t st = plan->st;
  const int cfg = plan->cfg;
  const uint32_t cap = plan->cap;
  rd_stats& S = ctx->stats;
  memset(&S, 0, sizeof S);
  S.evals = plan->evals;
  S.prefiltered = plan->prefiltered;
  S.small_items = plan->n_sitems;
  S.block_symmetric = plan->n_symmetric;
  S.sync_decided = plan->sync_decided;
  int merr = 0;
  auto D = [&](const char* name) { return plan->dev[name].p; };
  const DInsn* d_code = (const DInsn*)D("code");
  const int64_t* d_params = (const int64_t*)D("params");
  const int64_t* d_loops = (const int64_t*)D("loops");
  const void* d_insts = D("insts");
  const QDesc* d_qd = (const QDesc*)D("qdesc");
  QAcc* d_acc = (QAcc*)D("qacc");
  const uint32_t* d_herr = (const uint32_t*)D("herr");
  const uint8_t* d_triv = (const uint8_t*)D("triv");
  const u64* d_evals = (const u64*)D("evals");
  rd_pair_result* d_out = (rd_pair_result*)D("out");
  const SItem* d_sitems = (const SItem*)D("sitems");
  const HItem* d_hitems_all = (const HItem*)D("hitems");
  const Chunk* d_chunks_all = (const Chunk*)D("chunks");
  const BRun* d_runs_all = (const BRun*)D("runs");
  // first-phase scratch owned by the plan (fixed addresses, so a captured
  // graph stays valid); later phases reuse the context's arena
  unsigned char* d_recs = (unsigned char*)D("recs");
  uint32_t* d_cursor = (uint32_t*)D("cursor");
  uint8_t* d_cand = (uint8_t*)D("cand");
  // the exact address filter in front of the bucket join (HGRD_NO_FILTER
  // turns it off: every bucket is joined)
  const bool use_filter = getenv("HGRD_NO_FILTER") == nullptr;
  // the unit filter (items whose accesses share no address do nothing;
  // HGRD_NO_UNIT_FILTER turns it off)
  const IFact* d_facts =
      getenv("HGRD_NO_UNIT_FILTER") == nullptr ? (const IFact*)D("ifacts") : nullptr;
  uint32_t* d_done = (uint32_t*)D("done");
  uint32_t* d_pcursor = (uint32_t*)D("pcursor");
  u64* d_nbytes = (u64*)D("nbytes");
  const uint32_t nh = (uint32_t)plan->hitems.size();
  uint32_t* d_ovf_all = (uint32_t*)D("ovf");
  hipEvent_t* ev = ctx->ev;
  // timing mode runs the first phase eagerly with events between kernels
  const bool timing = plan->log_level >= 2 || getenv("HGRD_TIMING") != nullptr;
  double verdict_ms = 0, small_ms = 0, scatter_ms = 0, bucket_ms = 0;
  double fallback_ms = 0, retry_ms = 0, split_ms = 0, waves_ms = 0;
  std::vector<uint32_t> skip;  // kept alive until the stream is synchronised

  // Every eagerly launched partition wave is bracketed by events from the
  // context's pool (scatter start, scatter end = join start, join end);
  // their times are collected once the stream has drained.  A replayed
  // graph carries no events (their times are not reliable inside graphs).
  uint32_t wev_n = 0;
  // per wave: events before and after the table partition, after the
  // interpreted partition, after the table-path join and after the
  // interpreted join; whether table partition and table join ran
  std::vector<std::array<uint32_t, 8>> wtimes;
  auto wevent = [&](uint32_t k) -> hipEvent_t {
    while (ctx->wev.size() <= k) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ctx->wev.push_back(e);
    }
    return ctx->wev[k];
  };
  auto run_waves = [&](const std::vector<rd_plan_impl::Wave>& waves,
                       const HItem* d_hit, const Chunk* d_chk,
                       const BRun* d_bit, uint32_t* d_ovf, int wcfg,
                       const u64* l0k, const u64* l0c, bool events) -> int {
    const uint32_t wcap = (uint32_t)join_cap(wcfg);
    events = events && !plan->arena;  // no event is created in an arena call
    for (const auto& W : waves) {
      // e0..e4: markers around the stages; ke: start and stop of the
      // table-path partition, filter and join kernels, taken by their
      // dispatch packets (markers between kernels can be timestamped before
      // the previous kernel has finished)
      const uint32_t k = wev_n;
      hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr, e4 = nullptr;
      hipEvent_t ke[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
      if (events) {
        wev_n += 11;
        e0 = wevent(k);
        e1 = wevent(k + 1);
        e2 = wevent(k + 2);
        e3 = wevent(k + 3);
        e4 = wevent(k + 4);
        for (int x = 0; x < 6; ++x) {
          ke[x] = wevent(k + 5 + x);
          if (!ke[x]) return RD_EDEVICE;
        }
        if (!e0 || !e1 || !e2 || !e3 || !e4) return RD_EDEVICE;
      }
      if (launch_fill_u32(st, d_cursor, W.n_buckets, 0)) return RD_EDEVICE;
      // partition: instances with term tables, then the interpreted ones
      // (record bytes counted in slots 0..63 and 64..127)
      if (events) TRY_HIP(hipEventRecord(e0, st));
      if (W.n_tab_chunks &&
          launch_scatter(st, d_chk + W.chunk_off, W.n_tab_chunks, true, d_hit, d_insts,
                         d_code, d_params, d_loops, d_acc, d_recs,
                         d_cursor, d_ovf, wcap, d_done, d_nbytes, ke[0], ke[1]))
        return RD_EDEVICE;
      if (events) TRY_HIP(hipEventRecord(e1, st));
      if (W.n_chunks > W.n_tab_chunks &&
          launch_scatter(st, d_chk + W.chunk_off + W.n_tab_chunks,
                         W.n_chunks - W.n_tab_chunks, false, d_hit, d_insts,
                         d_code, d_params, d_loops, d_acc, d_recs,
                         d_cursor, d_ovf, wcap, d_done, d_nbytes + 64))
        return RD_EDEVICE;
      if (events) TRY_HIP(hipEventRecord(e2, st));
      // address filter and join: runs of items with term tables, then the
      // interpreted ones (record bytes the joins read are counted in slots
      // 128..191 and 192..255, the filters' in 384..447)
      uint8_t* cand = use_filter ? d_cand : nullptr;
      if (W.n_tab_runs &&
          launch_bucket(wcfg, st, W.n_tab_runs, d_bit + W.bitem_off, W.n_tab_runs, d_hit,
                        d_insts, d_code, d_params, d_loops, d_qd, d_acc, d_recs,
                        d_cursor, d_ovf, d_done, l0k, l0c, cand, d_nbytes + 128,
                        events ? ke + 2 : nullptr))
        return RD_EDEVICE;
      if (events) TRY_HIP(hipEventRecord(e3, st));
      const uint32_t n_oth = W.n_runs - W.n_tab_runs - W.n_sync_runs;
      if (n_oth &&
          launch_bucket(wcfg, st, n_oth, d_bit + W.bitem_off + W.n_tab_runs,
                        0, d_hit, d_insts, d_code, d_params, d_loops, d_qd, d_acc, d_recs,
                        d_cursor, d_ovf, d_done, l0k, l0c, cand, d_nbytes + 128, nullptr))
        return RD_EDEVICE;
      if (W.n_sync_runs &&
          launch_bucket(wcfg, st, W.n_sync_runs,
                        d_bit + W.bitem_off + W.n_runs - W.n_sync_runs, W.n_sync_runs, d_hit,
                        d_insts, d_code, d_params, d_loops, d_qd, d_acc, d_recs, d_cursor,
                        d_ovf, d_done, l0k, l0c, cand, d_nbytes + 128, nullptr, true))
        return RD_EDEVICE;
      if (events) {
        TRY_HIP(hipEventRecord(e4, st));
        // per-kernel figures only for the first phase (the context's tile
        // shape); re-partition rounds use other tile shapes
        const uint32_t first = wcfg == cfg && d_hit == d_hitems_all;
        wtimes.push_back({k, k + 1, k + 2, k + 3, k + 4, first && W.n_tab_chunks ? 1u : 0u,
                          first && W.n_tab_runs ? 1u : 0u, k + 5});
      }
      if (W.n_buckets) S.join_launches += 1;
      S.buckets += W.n_buckets;
    }
    return RD_OK;
  };
  auto collect_waves = [&]() {
    for (const auto& t : wtimes) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, ctx->wev[t[0]], ctx->wev[t[1]]) == hipSuccess)
        scatter_ms += ms;
      // t[7]..t[7] + 5: start and stop of the table-path partition, filter
      // and join kernels
      if (t[5] && hipEventElapsedTime(&ms, ctx->wev[t[7]], ctx->wev[t[7] + 1]) == hipSuccess) {
        S.scatter_tab_ms += ms;
        S.scatter_launches += 1;
      }
      if (hipEventElapsedTime(&ms, ctx->wev[t[1]], ctx->wev[t[2]]) == hipSuccess)
        scatter_ms += ms;
      if (hipEventElapsedTime(&ms, ctx->wev[t[2]], ctx->wev[t[3]]) == hipSuccess)
        bucket_ms += ms;
      if (t[6]) {
        if (use_filter &&
            hipEventElapsedTime(&ms, ctx->wev[t[7] + 2], ctx->wev[t[7] + 3]) == hipSuccess) {
          S.filter_tab_ms += ms;
          S.filter_tab_launches += 1;
        }
        if (hipEventElapsedTime(&ms, ctx->wev[t[7] + 4], ctx->wev[t[7] + 5]) == hipSuccess) {
          S.join_tab_ms += ms;
          S.join_tab_launches += 1;
        }
      }
      if (hipEventElapsedTime(&ms, ctx->wev[t[3]], ctx->wev[t[4]]) == hipSuccess)
        bucket_ms += ms;
    }
    wtimes.clear();
    (void)hipGetLastError();
  };

  // ---- first phase: accumulator init, VERDICT tile search, LDS joins of
  // small items, HBM waves.  No host round trip inside; replayed from a
  // captured graph unless timing.
  auto phase1 = [&](bool events) -> int {
    if (plan->n_tabchunks &&
        launch_tabulate(st, (const Chunk*)D("tabchunks"), plan->n_tabchunks,
                        (const TabJob*)D("tabjobs"), d_insts, d_code, d_params,
                        d_loops, (int64_t*)D("tpool")))
      return RD_EDEVICE;
    if (launch_init_acc(st, n_pairs, d_acc)) return RD_EDEVICE;
    if (launch_fill_u32(st, d_done, n_pairs, 0)) return RD_EDEVICE;
    if (launch_fill_u64(st, d_nbytes, 512, 0)) return RD_EDEVICE;
    if (plan->verdict && plan->n_vq) {
      VQuery* d_vq = (VQuery*)D("vq");
      BBound* d_bb = (BBound*)D("bbounds");
      uint32_t* d_order = plan->score_mode ? (uint32_t*)D("order") : nullptr;
      TOut* d_tout = (TOut*)D("tout");
      u64* d_claim = (u64*)D("claim");
      if (events) TRY_HIP(hipEventRecord(ev[15], st));
      if (launch_fill_u64(st, d_claim, n_pairs, kNoKey) || verdict_bounds(plan, st) ||
          launch_vq_span(st, d_vq, plan->n_vq, d_bb))
        return RD_EDEVICE;
      if (plan->score_mode) {
        if (launch_tile_rank(st, d_vq, plan->n_vq, d_bb, (const float*)D("mlp_w"),
                             plan->score_mode, plan->K, plan->max_g, d_facts, d_qd, d_order))
          return RD_EDEVICE;
      }
      for (auto& rr : plan->rounds) {
        if (launch_tile_join(cfg, st, (const TItem*)D("titems"), rr.first,
                             rr.second - rr.first, d_vq, d_order, plan->K, d_insts,
                             d_code, d_params, d_loops, d_qd, d_done, d_tout, d_claim, d_bb,
                             d_facts) ||
            launch_verdict_commit(st, n_pairs, d_claim, d_tout, d_acc, d_done))
          return RD_EDEVICE;
      }
      if (events) TRY_HIP(hipEventRecord(ev[1], st));
    }
    if (plan->n_sitems) {
      if (events) TRY_HIP(hipEventRecord(ev[2], st));
      if (launch_small(cfg, st, d_sitems, plan->n_sitems, d_insts, d_code, d_params,
                       d_loops, d_qd, d_acc, d_done, d_pcursor, plan->persist_grid, d_facts))
        return RD_EDEVICE;
      if (events) TRY_HIP(hipEventRecord(ev[3], st));
      S.join_launches += 1;
    }
    // HBM waves: the scratch buckets are reused by the next wave in stream
    // order
    if (nh) {
      if (launch_fill_u32(st, d_ovf_all, nh, 0)) return RD_EDEVICE;
      // items counted in nbytes[500]
      if (d_facts && launch_unit_filter(st, nh, d_hitems_all, d_qd, d_facts, d_ovf_all,
                                        d_nbytes + 500))
        return RD_EDEVICE;
      if (events) TRY_HIP(hipEventRecord(ev[11], st));
      int rc = run_waves(plan->waves, d_hitems_all, d_chunks_all, d_runs_all,
                         d_ovf_all, cfg, nullptr, nullptr, events);
      if (rc) return rc;
      if (events) TRY_HIP(hipEventRecord(ev[12], st));
    }
    return RD_OK;
  };

  TRY_HIP(hipEventRecord(ev[0], st));
  bool replayed = false;
  // (an arena call captures nothing: instantiating a graph allocates)
  if (!timing && !plan->graph_failed && !plan->graph && !plan->arena) {
    // capture once; any failure falls back to eager launches for this plan
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      // no events inside the graph: their times are not reliable there
      int rc = phase1(false);
      wtimes.clear();
      wev_n = 0;
      ok = hipStreamEndCapture(st, &g) == hipSuccess && rc == RD_OK && g;
      if (ok) ok = hipGraphInstantiate(&plan->graph, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
    }
    if (!ok) {
      (void)hipGetLastError();
      plan->graph = nullptr;
      plan->graph_failed = true;
    }
    S.join_launches = 0;
    S.buckets = 0;
  }
  if (!timing && plan->graph) {
    TRY_HIP(hipGraphLaunch(plan->graph, st));
    replayed = true;
    S.join_launches = (plan->n_sitems ? 1 : 0);
    for (const auto& W : plan->waves) {
      S.join_launches += W.n_buckets ? 1 : 0;
      S.buckets += W.n_buckets;
    }
  } else {
    int rc = phase1(true);
    if (rc) return rc;
  }
  TRY_HIP(hipEventRecord(ev[13], st));
  S.hbm_items = nh;
  for (uint32_t i = 0; i < nh; ++i)
    if (plan->hitems[i].shared != 2) S.records += plan->hR[i];
  std::vector<uint32_t> ovf(nh);
  if (nh) TRY_HIP(hipMemcpyAsync(ovf.data(), d_ovf_all, nh * 4, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  {
    // events recorded inside a replayed graph time the same way; a failed
    // query leaves the figure at 0
    float ms = 0;
    if (plan->verdict && plan->n_vq && hipEventElapsedTime(&ms, ev[15], ev[1]) == hipSuccess)
      verdict_ms = ms;
    if (plan->n_sitems && hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess)
      small_ms = ms;
    if (nh && hipEventElapsedTime(&ms, ev[11], ev[12]) == hipSuccess)
      waves_ms = ms;  // scatter and bucket joins together
    (void)hipGetLastError();
    (void)replayed;
  }
  collect_waves();

  // ---- re-partition overflowed items ---------------------------------------
  // The first step retries with more buckets (bucket loads vary with how many points
  // share an address).  The second splits global items by (address, block) into
  // bigger tiles, counting level 0 in address-count tables.  What still
  // overflows goes to the HBM fallback.
  struct RItem {
    HItem h;
    uint64_t R;
  };
  auto repartition = [&](std::vector<RItem>& items, int wcfg, const u64* l0k,
                         const u64* l0c, std::vector<uint32_t>& ovf_out,
                         float& ms_out) -> int {
    const uint32_t wcap = (uint32_t)join_cap(wcfg);
    std::vector<rd_plan_impl::Wave> waves;
    std::vector<Chunk> chunks;
    std::vector<BRun> bitem;
    std::vector<HItem> hs;
    std::vector<Chunk> interp;
    std::vector<BRun> interp_runs;
    uint64_t max_bytes = 0, max_nbk = 0;
    size_t pos = 0;
    while (pos < items.size()) {
      rd_plan_impl::Wave W;
      memset(&W, 0, sizeof W);
      W.chunk_off = chunks.size();
      W.bitem_off = bitem.size();
      uint64_t bytes = 0, nbk = 0;
      size_t end = pos;
      while (end < items.size()) {
        HItem h = items[end].h;
        const uint64_t need = (uint64_t)h.nbuckets * wcap * (h.is32 ? 8 : 16);
        if (end > pos && bytes + need > plan->wave_budget) break;
        h.bucket0 = (uint32_t)nbk;
        h.rec_off = bytes;
        if (!h.mode) h.shift = 0;  // hashed re-partitions: single addresses
        bytes += (need + 255) / 256 * 256;
        nbk += h.nbuckets;
        uint32_t li = (uint32_t)hs.size();
        hs.push_back(h);
        std::vector<BRun>& rdst =
            plan->tab_on[h.inst_i] && plan->tab_on[h.inst_j] ? bitem : interp_runs;
        for (uint32_t b = 0; b < h.nbuckets; b += plan->run_buckets)
          rdst.push_back({li, b, std::min(h.nbuckets, b + plan->run_buckets), 0});
        const QPlan& q = plan->Q[h.q];
        for (int side = 0; side < (q.qd.self ? 1 : 2); ++side) {
          const uint32_t inst = side ? h.inst_j : h.inst_i;
          uint32_t np = h.gmult > 1 ? plan->tpb[inst] : plan->npts[inst];
          std::vector<Chunk>& dst = plan->tab_on[inst] ? chunks : interp;
          for (uint32_t p0 = 0; p0 < np; p0 += plan->chunk_pts)
            dst.push_back({li, (uint32_t)side, p0, std::min(np, p0 + plan->chunk_pts)});
        }
        ++end;
      }
      W.n_tab_chunks = (uint32_t)(chunks.size() - W.chunk_off);
      chunks.insert(chunks.end(), interp.begin(), interp.end());
      interp.clear();
      W.n_tab_runs = (uint32_t)(bitem.size() - W.bitem_off);
      bitem.insert(bitem.end(), interp_runs.begin(), interp_runs.end());
      interp_runs.clear();
      W.n_items = (uint32_t)(end - pos);
      W.n_runs = (uint32_t)(bitem.size() - W.bitem_off);
      W.n_chunks = (uint32_t)(chunks.size() - W.chunk_off);
      W.n_buckets = (uint32_t)nbk;
      waves.push_back(W);
      max_bytes = std::max(max_bytes, bytes);
      max_nbk = std::max(max_nbk, nbk);
      pos = end;
    }
    // the first phase is over: its partition scratch serves again
    auto rbuf = [&](const char* name, size_t bytes) {
      return plan->arena ? ctx->ensure(name, bytes, &merr) : ctx->shared_buf(name, bytes, &merr);
    };
    d_recs = (unsigned char*)rbuf("recs", std::max<uint64_t>(max_bytes, plan->max_key_bytes));
    d_cursor = (uint32_t*)rbuf("cursor", std::max<uint64_t>(max_nbk, plan->max_buckets) * 4);
    d_cand = (uint8_t*)rbuf("cand", std::max<uint64_t>(max_nbk, plan->max_buckets));
    const uint32_t nr = (uint32_t)hs.size();
    HItem* d_rh = (HItem*)ctx->ensure("r_hitems", nr * sizeof(HItem), &merr);
    Chunk* d_rc = (Chunk*)ctx->ensure("r_chunks", chunks.size() * sizeof(Chunk), &merr);
    BRun* d_rb = (BRun*)ctx->ensure("r_runs", bitem.size() * sizeof(BRun), &merr);
    uint32_t* d_rovf = (uint32_t*)ctx->ensure("r_ovf", nr * 4, &merr);
    if (merr) return merr;
    TRY_HIP(hipMemcpyAsync(d_rh, hs.data(), nr * sizeof(HItem), hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemcpyAsync(d_rc, chunks.data(), chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemcpyAsync(d_rb, bitem.data(), bitem.size() * sizeof(BRun), hipMemcpyHostToDevice, st));
    if (launch_fill_u32(st, d_rovf, nr, 0)) return RD_EDEVICE;
    TRY_HIP(hipEventRecord(ev[13], st));
    int rc = run_waves(waves, d_rh, d_rc, d_rb, d_rovf, wcfg, l0k, l0c, true);
    if (rc) return rc;
    TRY_HIP(hipEventRecord(ev[14], st));
    ovf_out.assign(nr, 0);
    TRY_HIP(hipMemcpyAsync(ovf_out.data(), d_rovf, nr * 4, hipMemcpyDeviceToHost, st));
    TRY_HIP(hipStreamSynchronize(st));
    (void)hipEventElapsedTime(&ms_out, ev[13], ev[14]);
    collect_waves();
    return RD_OK;
  };

  std::vector<RItem> rit;
  std::vector<RItem> still;
  for (uint32_t i = 0; i < nh; ++i) {
    if (ovf[i] == kApart) continue;  // decided by the unit filter
    if ((!ovf[i] && !plan->presplit[i]) || plan->hitems[i].shared == 2) continue;
    RItem r{plan->hitems[i], plan->hR[i]};
    if (r.h.sync) {
      // the synchronisation levels live in the LDS joins and the fallback:
      // an overflowing synchronised item goes to the fallback
      still.push_back(r);
      continue;
    }
    if (r.h.mode && r.h.shared == 0) {
      // a dense-map global item overflows only on heavy address groups,
      // which more buckets do not spread: split it right away
      still.push_back(r);
      continue;
    }
    uint64_t need_f = (ovf[i] * 10ull + cap * 6 - 1) / (cap * 6);
    need_f = std::min<uint64_t>(std::max<uint64_t>(need_f, 2), 64);
    // at most kRetryBytes of buckets per retried item; else split it
    const uint64_t rs = r.h.is32 ? 8 : 16;
    while (need_f > 2 && (uint64_t)r.h.nbuckets * need_f * cap * rs > kRetryBytes) need_f /= 2;
    if ((uint64_t)r.h.nbuckets * need_f * cap * rs > kRetryBytes ||
        (uint64_t)r.h.nbuckets * need_f >= (1ull << 31)) {
      still.push_back(r);
      continue;
    }
    r.h.nbuckets = (uint32_t)((uint64_t)r.h.nbuckets * need_f);
    r.h.mode = 0;
    rit.push_back(r);
  }
  S.retry_items = rit.size();
  std::vector<uint32_t> rovf;
  if (!rit.empty()) {
    float ms = 0;
    int rc = repartition(rit, cfg, nullptr, nullptr, rovf, ms);
    if (rc) return rc;
    retry_ms = ms;
    for (size_t i = 0; i < rit.size(); ++i)
      if (rovf[i]) still.push_back(rit[i]);
  }

  // second step: split global items by (address, block); level 0 in tables,
  // in batches whose address-count tables stay within kL0Slots
  std::vector<RItem> split_all, direct;
  // block-symmetric units hold one block: nothing for the (address, block)
  // split to split, so they go to the fallback
  for (auto& r : still)
    (r.h.shared == 0 && r.h.gmult <= 1 && !r.h.sync ? split_all : direct).push_back(r);
  S.split_items = split_all.size();
  S.presplit_items = 0;
  for (uint8_t f : plan->presplit) S.presplit_items += f;
  for (size_t sp0 = 0; sp0 < split_all.size();) {
    std::vector<RItem> split;
    uint64_t bslots = 0;
    while (sp0 < split_all.size()) {
      uint64_t t = 1;
      while (t < 2 * split_all[sp0].R) t <<= 1;
      if (!split.empty() && bslots + t + 1 > kL0Slots) break;
      bslots += t + 1;
      split.push_back(split_all[sp0++]);
    }
    const int scfg = 1;  // first pass; its overflows get join_cap(2) tiles
    const uint32_t scap = (uint32_t)join_cap(scfg);
    std::vector<L0Item> l0;
    uint64_t slots = 0;
    std::vector<Chunk> l0chunks;
    for (auto& r : split) {
      const QPlan& q = plan->Q[r.h.q];
      // distinct addresses: at most the records, and at most the widths of
      // the two proven address ranges when both instances have tables
      uint64_t distinct = r.R;
      if (plan->tab_on[r.h.inst_i] && plan->tab_on[r.h.inst_j]) {
        auto width = [&](uint32_t inst) -> __int128 {
          const auto& ar = plan->arange[inst];
          return ar.second < ar.first ? 0 : (__int128)ar.second - ar.first + 1;
        };
        __int128 w = width(r.h.inst_i);
        if (!q.qd.self) w += width(r.h.inst_j);
        if (w < (__int128)distinct) distinct = std::max<uint64_t>(1, (uint64_t)w);
      }
      uint64_t t = 1;
      while (t < 2 * distinct) t <<= 1;
      r.h.shared = 3;
      r.h.l0_off = slots;
      r.h.l0_mask = (uint32_t)(t - 1);
      r.h.nbuckets = (uint32_t)std::max<uint64_t>(1, (r.R * 100 + scap * 55 - 1) / (scap * 55));
      r.h.shift = 0;
      if (!plan->no_map)
        set_bucket_map(r.h, plan->tab_on, plan->arange,
                       r.h.gmult > 1 ? 1u : plan->nblk[r.h.inst_i],
                       q.qd.self, true, r.R, scap, 0.5);
      L0Item li;
      memset(&li, 0, sizeof li);
      li.q = r.h.q;
      li.inst_i = r.h.inst_i;
      li.inst_j = r.h.inst_j;
      li.self = q.qd.self;
      li.off = slots;
      li.mask = (uint32_t)(t - 1);
      li.qmask = q.qd.mask;
      if (q.qd.mask & 1) {
        uint32_t idx = (uint32_t)l0.size();
        for (int side = 0; side < (q.qd.self ? 1 : 2); ++side) {
          uint32_t np = plan->npts[side ? r.h.inst_j : r.h.inst_i];
          for (uint32_t p0 = 0; p0 < np; p0 += kL0ChunkPts)
            l0chunks.push_back({idx, (uint32_t)side, p0, std::min(np, p0 + kL0ChunkPts)});
        }
        l0.push_back(li);
      }
      slots += t + 1;
    }
    u64* d_l0k = (u64*)ctx->ensure("l0_keys", slots * 8, &merr);
    u64* d_l0c = (u64*)ctx->ensure("l0_cnt", slots * 8, &merr);
    L0Item* d_l0i = (L0Item*)ctx->ensure("l0_items", std::max<size_t>(1, l0.size()) * sizeof(L0Item), &merr);
    u64* d_s0 = (u64*)ctx->ensure("l0_s0", std::max<size_t>(1, l0.size()) * 8, &merr);
    uint32_t* d_skip = (uint32_t*)ctx->ensure("l0_skip", std::max<size_t>(1, l0.size()) * 4, &merr);
    Chunk* d_l0ch = (Chunk*)ctx->ensure("l0_chunks", std::max<size_t>(1, l0chunks.size()) * sizeof(Chunk), &merr);
    if (merr) return merr;
    TRY_HIP(hipEventRecord(ev[7], st));
    if (launch_fill_u64(st, d_l0k, slots, kL0Empty) || launch_fill_u64(st, d_l0c, slots, 0))
      return RD_EDEVICE;
    if (!l0.empty()) {
      TRY_HIP(hipMemcpyAsync(d_l0i, l0.data(), l0.size() * sizeof(L0Item), hipMemcpyHostToDevice, st));
      TRY_HIP(hipMemcpyAsync(d_l0ch, l0chunks.data(), l0chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
      if (launch_fill_u64(st, d_s0, l0.size(), 0) ||
          launch_level0(st, d_l0ch, (uint32_t)l0chunks.size(), d_l0i, d_insts, d_code,
                        d_params, d_loops, d_l0k, d_l0c, d_s0))
        return RD_EDEVICE;
    }
    TRY_HIP(hipEventRecord(ev[8], st));
    float ms0 = 0;
    (void)hipEventElapsedTime(&ms0, ev[7], ev[8]);
    float ms = 0;
    int rc = repartition(split, scfg, d_l0k, d_l0c, rovf, ms);
    if (rc) return rc;
    split_ms = ms0 + ms;
    // second pass: the overflowed split items with the biggest tiles and a
    // hashed map at a lower load
    std::vector<RItem> split2;
    std::vector<size_t> at2;
    const uint32_t scap2 = (uint32_t)join_cap(2);
    for (size_t i = 0; i < split.size(); ++i) {
      if (!rovf[i]) continue;
      RItem r = split[i];
      r.h.mode = 0;
      r.h.shift = 0;
      r.h.nbuckets = (uint32_t)std::max<uint64_t>(1, (r.R * 100 + scap2 * 40 - 1) / (scap2 * 40));
      split2.push_back(r);
      at2.push_back(i);
    }
    if (!split2.empty()) {
      std::vector<uint32_t> rovf2;
      rc = repartition(split2, 2, d_l0k, d_l0c, rovf2, ms);
      if (rc) return rc;
      split_ms += ms;
      for (size_t k = 0; k < at2.size(); ++k) rovf[at2[k]] = rovf2[k];
    }
    // an overflowed split item joined none of its buckets; its S_0 is not
    // applied and the fallback counts the whole item (the stream has
    // drained, so the previous batch's copy of `skip` is done)
    skip.clear();
    for (size_t i = 0; i < split.size(); ++i) {
      if (plan->Q[split[i].h.q].qd.mask & 1) skip.push_back(rovf[i] ? 1u : 0u);
      if (!rovf[i]) continue;
      direct.push_back(split[i]);
      direct.back().h.shared = 0;
    }
    if (!l0.empty()) {
      TRY_HIP(hipMemcpyAsync(d_skip, skip.data(), skip.size() * 4, hipMemcpyHostToDevice, st));
      if (launch_apply_s0(st, (uint32_t)l0.size(), d_l0i, d_s0, d_skip, d_acc))
        return RD_EDEVICE;
    }
  }

  // ---- fallback: HBM aggregation of items that still overflow --------------
  std::vector<FItem> fall;
  for (size_t i = 0; i < direct.size(); ++i) {
    const HItem& h = direct[i].h;
    const QPlan& q = plan->Q[h.q];
    FItem f;
    memset(&f, 0, sizeof f);
    f.q = h.q;
    f.sigma = h.sigma;
    f.inst_i = h.inst_i;
    f.inst_j = h.inst_j;
    f.self = q.qd.self;
    f.mask = q.qd.mask;
    f.warp = q.qd.warp;
    f.cap = (uint32_t)direct[i].R;
    f.gmult = h.gmult;
    f.sync = h.sync ? q.sync : 0;
    S.fallback_records += direct[i].R;
    if (plan->log_level >= 2)
      fprintf(stderr, "hgrd: fallback item pair=%u tuple=%u shared=%u points=%llu buckets=%u\n",
              h.q, h.sigma, h.shared, (unsigned long long)direct[i].R, h.nbuckets);
    fall.push_back(f);
  }
  S.overflow_items = fall.size();
  for (const auto& u : plan->sync_units) {
    const QPlan& q = plan->Q[u.q];
    FItem f;
    memset(&f, 0, sizeof f);
    f.q = u.q;
    f.sigma = u.sigma;
    f.inst_i = u.inst_i;
    f.inst_j = u.inst_j;
    f.self = u.scan ? 1 : q.qd.self;
    f.mask = u.scan ? 0 : q.qd.mask;
    f.warp = q.qd.warp;
    f.cap = (uint32_t)u.R;
    f.sync = q.sync;
    S.sync_records += u.R;
    fall.push_back(f);
  }
  size_t fpos = 0;
  while (fpos < fall.size()) {
    size_t fend = fpos;
    uint64_t n = 0;
    uint32_t used = 0;
    while (fend < fall.size() && (fend == fpos || n + fall[fend].cap <= kFallbackRecords)) {
      fall[fend].off = n;
      n += fall[fend].cap;
      uint32_t m = fall[fend].mask;
      used |= (m & 1 ? 0x03u : 0) | (m & 2 ? 0x0Cu : 0) | (m & 4 ? 0x30u : 0);
      // synchronised pairs: levels 6-11 are levels 0-5 with the
      // synchronisation address added, over points with a syn() at the
      // class's scope
      const uint32_t y = fall[fend].sync;
      if (y & kQSyncDev) used |= (m & 1 ? 0x03u : 0) << 6;
      if (y & kQSyncBlk) used |= ((m & 2 ? 0x0Cu : 0) | (m & 4 ? 0x30u : 0)) << 6;
      ++fend;
    }
    const uint32_t nf = (uint32_t)(fend - fpos);
    std::vector<Chunk> chunks;
    for (uint32_t i = 0; i < nf; ++i) {
      const FItem& f = fall[fpos + i];
      for (int side = 0; side < (f.self ? 1 : 2); ++side) {
        const uint32_t inst = side ? f.inst_j : f.inst_i;
        uint32_t np = f.gmult > 1 ? plan->tpb[inst] : plan->npts[inst];
        for (uint32_t p0 = 0; p0 < np; p0 += kL0ChunkPts)
          chunks.push_back({i, (uint32_t)side, p0, std::min(np, p0 + kL0ChunkPts)});
      }
    }
    uint64_t tbl = 1;
    while (tbl < 2 * n) tbl <<= 1;
    GRecPtrs g;
    g.addr = ctx->ensure("g_addr", n * 8, &merr);
    g.blin = (uint32_t*)ctx->ensure("g_blin", n * 4, &merr);
    g.tli = (uint32_t*)ctx->ensure("g_tli", n * 4, &merr);
    g.bw = (uint32_t*)ctx->ensure("g_bw", n * 4, &merr);
    g.w = (uint32_t*)ctx->ensure("g_w", n * 4, &merr);
    g.item = (uint32_t*)ctx->ensure("g_item", n * 4, &merr);
    g.slot = (uint32_t*)ctx->ensure("g_slot", n * 4, &merr);
    g.part = ctx->ensure("g_part", n * 8, &merr);
    g.mult = (uint32_t*)ctx->ensure("g_mult", n * 4, &merr);
    g.lanes = ctx->ensure("g_lanes", n * 8, &merr);
    const bool synced = (used >> 6) != 0;
    g.skey = synced ? ctx->ensure("g_skey", n * 8, &merr) : nullptr;
    void* owner = ctx->ensure("g_owner", tbl * 8, &merr);
    void* cnt = ctx->ensure("g_cnt", tbl * 8, &merr);
    // the synchronisation levels build their own table, so that both
    // thread-level tables are there for the witness scan
    void* owner2 = synced ? ctx->ensure("g_owner2", tbl * 8, &merr) : nullptr;
    void* cnt2 = synced ? ctx->ensure("g_cnt2", tbl * 8, &merr) : nullptr;
    void* gS = ctx->ensure("g_S", (size_t)nf * 128, &merr);
    uint32_t* gcount = (uint32_t*)ctx->ensure("g_count", (size_t)nf * 4, &merr);
    FItem* d_f = (FItem*)ctx->ensure("fb_items", nf * sizeof(FItem), &merr);
    Chunk* d_ch = (Chunk*)ctx->ensure("fb_chunks", chunks.size() * sizeof(Chunk), &merr);
    if (merr) return merr;
    TRY_HIP(hipMemcpyAsync(d_f, fall.data() + fpos, nf * sizeof(FItem), hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemcpyAsync(d_ch, chunks.data(), chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
    TRY_HIP(hipEventRecord(ev[7], st));
    if (launch_fallback(st, d_ch, (uint32_t)chunks.size(), d_f, nf, used, d_insts,
                        d_code, d_params, d_loops, g, n, gcount, owner, cnt,
                        owner2, cnt2, tbl, gS, d_acc))
      return RD_EDEVICE;
    TRY_HIP(hipEventRecord(ev[8], st));
    TRY_HIP(hipEventSynchronize(ev[8]));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev[7], ev[8]);
    fallback_ms += ms;
    std::vector<uint32_t> written(nf);
    TRY_HIP(hipMemcpy(written.data(), gcount, nf * 4, hipMemcpyDeviceToHost));
    for (uint32_t w : written) S.fallback_groups += w;
    fpos = fend;
  }

  // ---- witness pass 2 -------------------------------------------------------
  std::vector<QAcc> acc(n_pairs);
  if (n_pairs)
    TRY_HIP(hipMemcpyAsync(acc.data(), d_acc, n_pairs * sizeof(QAcc), hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  struct W2 {
    uint32_t q, inst_i, inst_j, p0, p1, sync, pad1, pad2;
  };
  std::vector<W2> w2;
  for (uint32_t k = 0; k < n_pairs; ++k) {
    const QPlan& q = plan->Q[k];
    if (!q.work || acc[k].err || acc[k].pmin == kNoKey || q.host_err) continue;
    if (acc[k].qmin != kNoKey) continue;  // resolved by the tile search
    uint32_t s = (uint32_t)(acc[k].pmin >> 52);
    if (s >= q.inst.size()) continue;
    int32_t ia = q.inst[s].first, ib = q.inst[s].second;
    if (ia < 0 || ib < 0) continue;
    uint32_t np = plan->npts[ib];
    for (uint32_t p0 = 0; p0 < np; p0 += kChunkPts)
      w2.push_back({k, (uint32_t)ia, (uint32_t)ib, p0, std::min(np, p0 + kChunkPts), q.sync,
                    0, 0});
  }
  double w2_ms = 0;
  if (!w2.empty()) {
    void* d_w2 = ctx->ensure("w2", w2.size() * sizeof(W2), &merr);
    if (merr) return merr;
    TRY_HIP(hipMemcpyAsync(d_w2, w2.data(), w2.size() * sizeof(W2), hipMemcpyHostToDevice, st));
    TRY_HIP(hipEventRecord(ev[9], st));
    if (launch_witness2(st, d_w2, (uint32_t)w2.size(), d_insts, d_code, d_params,
                        d_loops, d_qd, d_acc))
      return RD_EDEVICE;
    TRY_HIP(hipEventRecord(ev[10], st));
  }
  if (launch_finalize(st, n_pairs, d_acc, d_qd, d_herr, d_triv, d_evals, d_out))
    return RD_EDEVICE;
  TRY_HIP(hipEventRecord(ev[1], st));
  if (n_pairs)
    TRY_HIP(hipMemcpyAsync(out, d_out, n_pairs * sizeof(rd_pair_result), hipMemcpyDeviceToHost, st));
  u64 scat_bytes[512];
  TRY_HIP(hipMemcpyAsync(scat_bytes, d_nbytes, sizeof scat_bytes, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  S.units_apart = scat_bytes[500];  // HBM items the unit filter decided
  for (int k = 0; k < 128; ++k) {
    S.scatter_bytes += scat_bytes[k];
    if (k < 64) S.scatter_tab_bytes += scat_bytes[k];
    if (k < 64) S.join_tab_bytes += scat_bytes[128 + k];
    if (k < 64) S.filter_tab_bytes += scat_bytes[384 + k];
  }
  float ms = 0;
  if (!w2.empty()) {
    (void)hipEventElapsedTime(&ms, ev[9], ev[10]);
    w2_ms = ms;
  }
  (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
  S.device_ms = ms;
  collect_waves();
  S.scatter_ms = scatter_ms;
  S.join_ms = small_ms + bucket_ms;
  S.join_kernel_ms = small_ms + bucket_ms;
  S.small_ms = small_ms;
  S.bucket_ms = bucket_ms;
  S.fallback_ms = fallback_ms;
  S.retry_ms = retry_ms;
  S.split_ms = split_ms;
  S.verdict_ms = verdict_ms;
  S.verdict_units = plan->n_vq;
  S.waves_ms = waves_ms;
  S.witness_ms = w2_ms;
  S.total_ms = now_ms() - t_start;
  if (plan->log_level)
    fprintf(stderr,
            "[hgrd] pairs=%u small=%llu hbm=%llu buckets=%llu overflow=%llu "
            "retry=%llu small=%.3fms waves=%.3fms (scatter %.3f bucket %.3f) "
            "retry=%.3fms fallback=%.3fms w2=%.3fms device=%.3fms total=%.3fms\n",
            n_pairs, (u64)S.small_items, (u64)S.hbm_items, (u64)S.buckets,
            (u64)S.overflow_items, (u64)S.retry_items, small_ms, waves_ms,
            scatter_ms, bucket_ms, retry_ms, fallback_ms, w2_ms, S.device_ms, S.total_ms);
  return RD_OK;
}

int rd_check_pairs(rd_context* ctx, const rd_kernel_model* models,
                   uint32_t n_models, const rd_access_pair* pairs,
                   uint32_t n_pairs, const rd_launch_domain* launch,
                   const rd_param_sets* params, const rd_options* opt,
                   rd_pair_result* out) {
  if (n_pairs && !out) return RD_EINVAL;
  rd_plan* plan = nullptr;
  int rc = rd_prepare(ctx, models, n_models, pairs, n_pairs, launch, params, opt, &plan);
  if (rc != RD_OK) return rc;
  rc = rd_execute(ctx, plan, out);
  rd_plan_destroy(plan);
  return rc;
}

}  // extern "C"

int hgrd::context_device(const rd_context* ctx) { return ctx->device; }

// rd_check_pairs inside a caller's arena: the plan and every later phase
// take their device buffers from it, no graph is captured and no event is
// created.  Without an explicit wave size the partition waves get an
// eighth of the arena (the first phase and a re-partition round each hold
// one wave of buckets).
int hgrd::check_pairs_in_arena(rd_context* ctx, void* base, size_t cap,
                               const rd_kernel_model* models, uint32_t n_models,
                               const rd_access_pair* pairs, uint32_t n_pairs,
                               const rd_launch_domain* launch,
                               const rd_param_sets* params, const rd_options* opt,
                               rd_pair_result* out) {
  if (!ctx || !base) return RD_EINVAL;
  rd_options o;
  memset(&o, 0, sizeof o);
  if (opt) o = *opt;
  if (!o.max_device_bytes) o.max_device_bytes = cap / 8;
  Arena A;
  A.base = (unsigned char*)base;
  A.cap = cap;
  ctx->arena = &A;
  const int rc = rd_check_pairs(ctx, models, n_models, pairs, n_pairs, launch, params, &o, out);
  // an error may leave kernels of this call in flight: the area is free
  // again only once they have finished
  if (rc != RD_OK) (void)hipStreamSynchronize(o.stream ? (hipStream_t)o.stream : ctx->stream);
  ctx->arena = nullptr;
  ctx->abufs.clear();
  return rc;
}

extern "C" {

int rd_autotune(rd_context* ctx, const rd_kernel_model* models,
                uint32_t n_models, const rd_access_pair* pairs,
                uint32_t n_pairs, const rd_launch_domain* launch,
                const rd_param_sets* params, const rd_options* opt,
                uint32_t reps, rd_options* best, double* best_ms) {
  if (!ctx || !best) return RD_EINVAL;
  rd_options base;
  memset(&base, 0, sizeof base);
  if (opt) base = *opt;
  reps = std::max(1u, std::min(reps, 16u));
  std::vector<rd_pair_result> out(std::max<uint32_t>(1, n_pairs));
  static const uint64_t kWaves[3] = {kWaveBytes / 4, kWaveBytes, kWaveBytes * 4};
  double t_best = 1e300;
  rd_options o_best = base;
  for (int cfg = 0; cfg < 3; ++cfg) {
    for (uint64_t wb : kWaves) {
      rd_options o = base;
      o.lds_cap = (uint32_t)join_cap(cfg);
      o.max_device_bytes = wb;
      rd_plan* plan = nullptr;
      int rc = rd_prepare(ctx, models, n_models, pairs, n_pairs, launch, params, &o, &plan);
      if (rc != RD_OK) return rc;
      rc = rd_execute(ctx, plan, out.data());  // warm-up (and graph capture)
      std::vector<double> ts;
      for (uint32_t r = 0; rc == RD_OK && r < reps; ++r) {
        const double t0 = now_ms();
        rc = rd_execute(ctx, plan, out.data());
        ts.push_back(now_ms() - t0);
      }
      rd_plan_destroy(plan);
      if (rc != RD_OK) return rc;
      std::sort(ts.begin(), ts.end());
      const double t = ts[ts.size() / 2];
      if (t < t_best) {
        t_best = t;
        o_best = o;
      }
    }
  }
  ctx->cfg = o_best.lds_cap <= 1024 ? 0 : o_best.lds_cap <= 1536 ? 1 : 2;
  ctx->wave_bytes = o_best.max_device_bytes;
  *best = o_best;
  if (best_ms) *best_ms = t_best;
  return RD_OK;
}

// ---------------------------------------------------------------------------
// Tile data and the tile-scoring network.

int rd_tile_data(rd_context* ctx, const rd_kernel_model* models,
                 uint32_t n_models, const rd_access_pair* pairs,
                 uint32_t n_pairs, const rd_launch_domain* launch,
                 const rd_param_sets* params, const rd_options* opt,
                 uint64_t max_rows, float* feats, float* labels, uint32_t* ids,
                 uint64_t* n_rows) {
  if (!ctx || !n_rows) return RD_EINVAL;
  rd_options o;
  memset(&o, 0, sizeof o);
  if (opt) o = *opt;
  o.mode = RD_MODE_VERDICT;
  o.order = RD_ORDER_LEX;
  o.tile_budget = 1u << 20;
  rd_plan* plan = nullptr;
  int rc = rd_prepare(ctx, models, n_models, pairs, n_pairs, launch, params, &o, &plan);
  if (rc != RD_OK) return rc;
  std::unique_ptr<rd_plan> guard(plan);
  *n_rows = plan->n_tiles;
  if (plan->n_tiles > max_rows) return RD_ECAPACITY;
  if (!plan->n_tiles) return RD_OK;
  hipStream_t st = plan->st;
  auto D = [&](const char* name) { return plan->dev[name].p; };
  int merr = 0;
  uint32_t* d_done = (uint32_t*)ctx->ensure("done", std::max<size_t>(1, n_pairs) * 4, &merr);
  float* d_feat = (float*)ctx->ensure("td_feats", plan->n_tiles * 32 * 4, &merr);
  if (merr) return merr;
  VQuery* d_vq = (VQuery*)D("vq");
  BBound* d_bb = (BBound*)D("bbounds");
  TOut* d_tout = (TOut*)D("tout");
  QAcc* d_acc = (QAcc*)D("qacc");
  if ((plan->n_tabchunks &&
       launch_tabulate(st, (const Chunk*)D("tabchunks"), plan->n_tabchunks,
                       (const TabJob*)D("tabjobs"), D("insts"), (const DInsn*)D("code"),
                       (const int64_t*)D("params"), (const int64_t*)D("loops"),
                       (int64_t*)D("tpool"))) ||
      launch_init_acc(st, n_pairs, d_acc) || launch_fill_u32(st, d_done, n_pairs, 0) ||
      launch_fill_u64(st, (u64*)D("claim"), n_pairs, kNoKey) ||
      launch_fill_u64(st, (u64*)d_tout, (u64)plan->n_titems * (sizeof(TOut) / 8), kNoKey) ||
      verdict_bounds(plan, st) || launch_vq_span(st, d_vq, plan->n_vq, d_bb) ||
      launch_tile_features(st, (const TChunk*)D("tchunks"), plan->n_tchunks, d_vq, d_bb, d_feat))
    return RD_EDEVICE;
  // every tile is joined (no commit, so no query stops early)
  for (auto& rr : plan->rounds)
    if (launch_tile_join(plan->cfg, st, (const TItem*)D("titems"), rr.first,
                         rr.second - rr.first, d_vq, nullptr, plan->K, D("insts"),
                         (const DInsn*)D("code"), (const int64_t*)D("params"),
                         (const int64_t*)D("loops"), (const QDesc*)D("qdesc"), d_done,
                         d_tout, (u64*)D("claim"), d_bb, nullptr))
      return RD_EDEVICE;
  std::vector<TOut> tout(plan->n_titems);
  std::vector<QAcc> acc(n_pairs);
  TRY_HIP(hipMemcpyAsync(tout.data(), d_tout, tout.size() * sizeof(TOut), hipMemcpyDeviceToHost, st));
  if (n_pairs) TRY_HIP(hipMemcpyAsync(acc.data(), d_acc, n_pairs * sizeof(QAcc), hipMemcpyDeviceToHost, st));
  if (feats)
    TRY_HIP(hipMemcpyAsync(feats, d_feat, plan->n_tiles * 32 * 4, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  // tile items are (unit, rank = tile index); map each to its row
  std::vector<int8_t> lab(plan->n_tiles, 0);
  std::vector<uint32_t> tiles_of_item;
  {
    std::vector<TItem> titems(plan->n_titems);
    TRY_HIP(hipMemcpy(titems.data(), D("titems"), titems.size() * sizeof(TItem), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < titems.size(); ++i) {
      const VQuery& v = plan->vqs[titems[i].vq];
      lab[v.tile0 + titems[i].rank] = tout[i].pkey != kNoKey ? 1 : 0;
    }
  }
  for (const VQuery& v : plan->vqs) {
    uint32_t nt = v.G * v.G;
    bool bad = acc[v.q].err != 0;
    for (uint32_t t = 0; t < nt; ++t) {
      uint64_t row = (uint64_t)v.tile0 + t;
      if (labels) labels[row] = bad ? -1.f : (float)lab[row];
      if (ids) {
        ids[row * 4 + 0] = v.q;
        ids[row * 4 + 1] = v.sigma;
        ids[row * 4 + 2] = t / v.G;
        ids[row * 4 + 3] = t % v.G;
      }
    }
  }
  return RD_OK;
}

namespace {
struct MlpDev {
  float *w, *g, *m, *v, *loss;
};
int mlp_dev(rd_context* ctx, MlpDev& d) {
  int merr = 0;
  const size_t nw = (size_t)mlp_num_weights() * 4;
  d.w = (float*)ctx->ensure("mlp_w", nw, &merr);
  d.g = (float*)ctx->ensure("mlp_g", nw, &merr);
  d.m = (float*)ctx->ensure("mlp_m", nw, &merr);
  d.v = (float*)ctx->ensure("mlp_v", nw, &merr);
  d.loss = (float*)ctx->ensure("mlp_loss", 256, &merr);
  return merr;
}
}  // namespace

int rd_mlp_forward(rd_context* ctx, const rd_mlp* w, const float* X, uint64_t n,
                   float* logits, void* stream) {
  if (!ctx || !w || (n && (!X || !logits))) return RD_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return RD_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  MlpDev d;
  int merr = mlp_dev(ctx, d);
  float* dx = (float*)ctx->ensure("mlp_x", n * 32 * 4, &merr);
  float* dz = (float*)ctx->ensure("mlp_z", n * 4, &merr);
  if (merr) return merr;
  TRY_HIP(hipMemcpyAsync(d.w, w, (size_t)mlp_num_weights() * 4, hipMemcpyHostToDevice, st));
  if (n) TRY_HIP(hipMemcpyAsync(dx, X, n * 32 * 4, hipMemcpyHostToDevice, st));
  if (launch_mlp_forward(st, dx, n, d.w, dz)) return RD_EDEVICE;
  if (n) TRY_HIP(hipMemcpyAsync(logits, dz, n * 4, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  return RD_OK;
}

int rd_mlp_grad(rd_context* ctx, const rd_mlp* w, const float* X, const float* Y,
                uint64_t n, rd_mlp* grad, float* loss, void* stream) {
  if (!ctx || !w || !grad || !loss || (n && (!X || !Y))) return RD_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return RD_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  MlpDev d;
  int merr = mlp_dev(ctx, d);
  float* dx = (float*)ctx->ensure("mlp_x", n * 32 * 4, &merr);
  float* dy = (float*)ctx->ensure("mlp_y", n * 4, &merr);
  if (merr) return merr;
  const size_t nw = (size_t)mlp_num_weights() * 4;
  TRY_HIP(hipMemcpyAsync(d.w, w, nw, hipMemcpyHostToDevice, st));
  TRY_HIP(hipMemsetAsync(d.g, 0, nw, st));
  TRY_HIP(hipMemsetAsync(d.loss, 0, 4, st));
  if (n) {
    TRY_HIP(hipMemcpyAsync(dx, X, n * 32 * 4, hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemcpyAsync(dy, Y, n * 4, hipMemcpyHostToDevice, st));
  }
  if (launch_mlp_grad(st, dx, dy, n, d.w, d.g, d.loss)) return RD_EDEVICE;
  TRY_HIP(hipMemcpyAsync(grad, d.g, nw, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipMemcpyAsync(loss, d.loss, 4, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  return RD_OK;
}

int rd_mlp_train(rd_context* ctx, rd_mlp* w, const float* X, const float* Y,
                 uint64_t n, uint32_t epochs, uint32_t batch, float lr,
                 uint64_t seed, float* epoch_loss, void* stream) {
  if (!ctx || !w || !n || !X || !Y || !batch || !epochs) return RD_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return RD_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  MlpDev d;
  int merr = mlp_dev(ctx, d);
  float* dx = (float*)ctx->ensure("mlp_x", n * 32 * 4, &merr);
  float* dy = (float*)ctx->ensure("mlp_y", n * 4, &merr);
  if (merr) return merr;
  const size_t nw = (size_t)mlp_num_weights() * 4;
  TRY_HIP(hipMemcpyAsync(d.w, w, nw, hipMemcpyHostToDevice, st));
  TRY_HIP(hipMemsetAsync(d.g, 0, nw, st));
  TRY_HIP(hipMemsetAsync(d.m, 0, nw, st));
  TRY_HIP(hipMemsetAsync(d.v, 0, nw, st));
  std::vector<uint64_t> perm(n);
  for (uint64_t i = 0; i < n; ++i) perm[i] = i;
  std::vector<float> xs(n * 32), ys(n);
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
  int t = 0;
  for (uint32_t e = 0; e < epochs; ++e) {
    for (uint64_t i = n - 1; i > 0; --i) {  // Fisher-Yates with xorshift64
      x ^= x << 13; x ^= x >> 7; x ^= x << 17;
      uint64_t j = x % (i + 1);
      std::swap(perm[i], perm[j]);
    }
    for (uint64_t i = 0; i < n; ++i) {
      memcpy(&xs[i * 32], &X[perm[i] * 32], 32 * 4);
      ys[i] = Y[perm[i]];
    }
    TRY_HIP(hipMemcpyAsync(dx, xs.data(), n * 32 * 4, hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemcpyAsync(dy, ys.data(), n * 4, hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemsetAsync(d.loss, 0, 4, st));
    uint64_t nb = 0;
    for (uint64_t off = 0; off < n; off += batch, ++nb) {
      uint64_t m = std::min<uint64_t>(batch, n - off);
      if (launch_mlp_grad(st, dx + off * 32, dy + off, m, d.w, d.g, d.loss) ||
          launch_adam(st, d.w, d.g, d.m, d.v, lr, ++t))
        return RD_EDEVICE;
    }
    float l = 0;
    TRY_HIP(hipMemcpyAsync(&l, d.loss, 4, hipMemcpyDeviceToHost, st));
    TRY_HIP(hipStreamSynchronize(st));
    if (epoch_loss) epoch_loss[e] = l / (float)nb;
  }
  TRY_HIP(hipMemcpyAsync(w, d.w, nw, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  return RD_OK;
}

int rd_prefilter_selftest(const rd_kernel_model* models, uint32_t n_models,
                          const rd_launch_domain* launch, const rd_param_sets* params,
                          uint32_t model, uint32_t access_a, uint32_t access_b,
                          uint32_t set, uint32_t* decided) {
  if (!models || !launch || !params || !decided || model >= n_models) return RD_EINVAL;
  const rd_kernel_model& M = models[model];
  if (access_a >= M.n_acc || access_b >= M.n_acc || set >= params[model].n_sets)
    return RD_EINVAL;
  *decided = 0;
  if (check_access(M, M.acc[access_a]) || check_access(M, M.acc[access_b])) return 2;
  Planner P;
  P.models = models;
  P.launch = launch;
  P.params = params;
  P.dims.resize(n_models);
  P.dims[model].resize(params[model].n_sets);
  InstInfo& ia = P.inst(model, access_a, set);
  InstInfo& ib = P.inst(model, access_b, set);
  if (ia.err || ib.err || ia.idx < 0 || ib.idx < 0) return 2;
  if (ia.idx != ib.idx) *decided = P.apart(ia.idx, ib.idx) ? 1u : 0u;
  // the unit filter's second test: one expression, thread-injective
  if (same_addr_expr(M, access_a, access_b) && P.tabs[ia.idx].on && P.tabs[ib.idx].on &&
      P.tinj[ia.idx] && P.tinj[ib.idx])
    *decided |= 2u;
  return RD_OK;
}

int rd_table_selftest(const rd_kernel_model* models, uint32_t n_models,
                      const rd_launch_domain* launch, const rd_param_sets* params,
                      uint32_t model, uint32_t access, uint32_t set,
                      uint64_t max_points, uint64_t* n_checked) {
  if (!models || !launch || !params || model >= n_models) return RD_EINVAL;
  if (access >= models[model].n_acc || set >= params[model].n_sets) return RD_EINVAL;
  if (check_access(models[model], models[model].acc[access])) return 2;
  Planner P;
  P.models = models;
  P.launch = launch;
  P.params = params;
  P.dims.resize(n_models);
  P.dims[model].resize(params[model].n_sets);
  InstInfo& ii = P.inst(model, access, set);
  if (ii.err || ii.idx < 0) return 2;
  const AccInst& I = P.dev_insts[ii.idx];
  const TabHost& T = P.tabs[ii.idx];
  if (!T.on) return 1;
  // fill the tables as the device does
  std::vector<int64_t> pool(P.tpool + 1);
  const int64_t* pr = P.pool_params.data() + I.params_off;
  int64_t c[10];
  for (const TabJob& J : P.tjobs) {
    for (uint32_t e = 0; e < J.n; ++e) {
      host_coords(I, P.pool_loops, J.group == 0 ? e : 0, J.group == 1 ? e : 0,
                  J.group >= 2 ? e : 0, c);
      uint32_t err = 0;
      int64_t v;
      if (J.group == 3) {
        v = host_prog(P.code, I.bint, c, pr, 0, err) |
            (host_prog(P.code, I.wint, c, pr, 0, err) << 16);
      } else {
        bool g = J.guard.absent || host_prog(P.code, J.guard, c, pr, 1, err) != 0;
        v = g ? host_prog(P.code, J.val, c, pr, 0, err) : INT64_MIN;
      }
      if (err) return -2;  // a table program failed: the proof was wrong
      pool[J.out_off + e] = v;
    }
  }
  // every box point: tables against the interpreter on the original programs
  const uint64_t npts = std::min<uint64_t>(I.npts, max_points ? max_points : I.npts);
  for (uint64_t k = 0; k < npts; ++k) {
    const uint64_t pidx = I.npts <= max_points || !max_points
                              ? k : (k * 2654435761ull) % I.npts;
    const uint32_t tlin = (uint32_t)(pidx % I.nthr);
    const uint32_t rest = (uint32_t)(pidx / I.nthr);
    const uint32_t ilin = rest % I.niota, blin = rest / I.niota;
    host_coords(I, P.pool_loops, blin, tlin, ilin, c);
    uint32_t err = 0;
    const bool g0 = host_prog(P.code, I.guard, c, pr, 1, err) != 0;
    int64_t a0 = 0, b0 = 0, w0 = 0;
    if (g0) {
      a0 = host_prog(P.code, I.addr, c, pr, 0, err);
      b0 = host_prog(P.code, I.bint, c, pr, 0, err);
      w0 = host_prog(P.code, I.wint, c, pr, 0, err);
      if (I.is32 && (a0 < INT32_MIN || a0 > INT32_MAX)) err |= ERR_RANGE;
      if (b0 < 0 || b0 > 65535 || w0 < 0 || w0 > 65535) err |= ERR_UNSUP;
    }
    if (err) return -3;  // the interpreter fails where tables were allowed
    bool g1 = !T.never;
    int64_t a1 = T.u;
    const uint32_t gi[3] = {blin, tlin, ilin};
    for (int g = 0; g < 3 && g1; ++g) {
      if (T.off[g] == kNoTab) continue;
      const int64_t v = pool[T.base + T.off[g] + gi[g]];
      if (v == INT64_MIN) g1 = false;
      else a1 += v;
    }
    if (g0 != g1) return -4;
    if (g0) {
      const uint32_t iv = T.iv_off != kNoTab ? (uint32_t)pool[T.base + T.iv_off + ilin] : T.iv_const;
      if (a0 != a1) return -5;
      if ((uint32_t)b0 != (iv & 0xFFFF) || (uint32_t)w0 != (iv >> 16)) return -6;
    }
  }
  if (n_checked) *n_checked = npts;
  return 0;
}

int rd_selftest(void) {
  // constant-divisor helper used by the kernels: numerators below 2^31
  static const uint32_t ds[] = {1, 2, 3, 5, 7, 10, 31, 32, 33, 63, 64, 100,
                                255, 256, 257, 1000, 1023, 1024, 4095, 65535,
                                65536, 65537, 1000003, 16777216, 67108863};
  static const uint32_t ns[] = {0, 1, 2, 3, 1023, 1024, 65535, 65536,
                                1000000, 16777215, 2147483646u, 2147483647u};
  for (uint32_t d : ds) {
    for (uint32_t n : ns)
      if (!fastdiv_check(n, d)) return -1;
    for (uint32_t k = 0; k < 4096; ++k) {
      uint64_t n = (uint64_t)k * d + (k % 3 == 0 ? 0 : k % 3 == 1 ? d - 1 : d / 2);
      if (n < (1ull << 31) && !fastdiv_check((uint32_t)n, d)) return -1;
    }
  }
  uint64_t x = 88172645463325252ull;
  for (int k = 0; k < 1000000; ++k) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    uint32_t d = (uint32_t)(x % 67108863u) + 1;
    uint32_t n = (uint32_t)(x >> 33);
    if (!fastdiv_check(n, d)) return -1;
  }
  return 0;
}

}  // extern "C"
