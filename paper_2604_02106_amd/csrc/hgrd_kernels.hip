// gfx950 kernels of the exact per-access-pair race query.
//
// The query (section 6.2 and Table 2 of the paper): two points p (access a)
// and q (access b) of one launch conflict when they come from different
// threads, reach the same address, and fall in a class the pair is checked
// for -- inter-block (different blocks), intra-block (same block, different
// warps, same block-barrier interval) or intra-warp (same warp, same block-
// and warp-barrier intervals).  The paper asks a SAT solver whether such a
// pair exists (section 6.4); here every point of the finite launch domain is
// generated and the conflicts are counted exactly.
//
// Counting.  Sort keys are (addr, blin, bint, warp, wint, tlin).  For a key
// prefix of length L+1 let S_L be the number of (p, q) pairs whose prefixes
// are equal: the sum over prefix groups of n_a * n_b.  Then
//   inter       = S_0 - S_1
//   intra-block = S_2 - S_3
//   intra-warp  = S_4 - S_5
// (each difference removes the pairs that agree on one more key field).
// S_L is computed without sorting, by aggregating records into an LDS hash
// table keyed by the prefix: a record that joins a group adds the opposite
// side's count seen at that moment, so every (p, q) is counted once.
//
// Layout.  Lanes of a wavefront take consecutive thread ids of one (set,
// block, iteration), so one wavefront always evaluates one access instance:
// the expression code, loop tables and launch extents are uniform and live
// in scalar registers.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "hgrd_internal.h"
#include "hgrd_launch.h"
#include <string.h>

namespace hgrd {

using u64 = unsigned long long;

// ---------------------------------------------------------------------------
// Division by a uniform 32-bit divisor for numerators below 2^31, by a
// multiply-high and a shift (Granlund and Montgomery, "Division by invariant
// integers using multiplication", PLDI 1994, section 4).
struct FastDiv {
  uint32_t d, m, s, pad;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  f.s = l;
  // m = floor(2^32 * (2^l - d) / d) + 1
  f.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
  f.pad = 0;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  uint32_t t = __umulhi(f.m, n);
  return (t + n) >> f.s;
}

// ---------------------------------------------------------------------------
// Checked int64 arithmetic: on error set a bit and yield 0 (C semantics
// otherwise: truncating '/', '%' with the dividend's sign, arithmetic '>>').
__device__ __forceinline__ int64_t alu(uint8_t op, int64_t a, int64_t b,
                                       uint32_t& err) {
  int64_t r;
  switch (op) {
    case D_MOV: return a;
    case D_ADD:
      if (__builtin_add_overflow(a, b, &r)) { err |= ERR_RANGE; return 0; }
      return r;
    case D_SUB:
      if (__builtin_sub_overflow(a, b, &r)) { err |= ERR_RANGE; return 0; }
      return r;
    case D_MUL:
      if (__builtin_mul_overflow(a, b, &r)) { err |= ERR_RANGE; return 0; }
      return r;
    case D_DIV:
      if (b == 0) { err |= ERR_DIVZERO; return 0; }
      if (a == INT64_MIN && b == -1) { err |= ERR_RANGE; return 0; }
      return a / b;
    case D_MOD:
      if (b == 0) { err |= ERR_DIVZERO; return 0; }
      if (a == INT64_MIN && b == -1) { err |= ERR_RANGE; return 0; }
      return a % b;
    case D_SHL: {
      if (b < 0 || b > 63) { err |= ERR_RANGE; return 0; }
      int64_t s = (int64_t)((uint64_t)a << b);
      if ((s >> b) != a) { err |= ERR_RANGE; return 0; }
      return s;
    }
    case D_SHR:
      if (b < 0 || b > 63) { err |= ERR_RANGE; return 0; }
      return a >> b;
    case D_AND: return a & b;
    case D_OR: return a | b;
    case D_XOR: return a ^ b;
    case D_MIN: return a < b ? a : b;
    case D_MAX: return a > b ? a : b;
    case D_LT: return a < b;
    case D_LE: return a <= b;
    case D_EQ: return a == b;
    case D_NE: return a != b;
    case D_GE: return a >= b;
    case D_GT: return a > b;
    case D_LAND: return (a != 0) & (b != 0);
    case D_LOR: return (a != 0) | (b != 0);
    case D_NEG:
      if (a == INT64_MIN) { err |= ERR_RANGE; return 0; }
      return -a;
    case D_LNOT: return a == 0;
  }
  return 0;
}

// Point coordinates live in named fields (read through a uniform switch);
// only the stack slots form an indexed array, which keeps it in VGPRs.
struct Regs {
  int64_t c0, c1, c2, c3, c4, c5, c6, c7, c8, c9;
};
typedef int64_t Stack[kMaxStack];

__device__ __forceinline__ int64_t coord(const Regs& R, uint32_t i) {
  switch (i) {
    case 0: return R.c0;
    case 1: return R.c1;
    case 2: return R.c2;
    case 3: return R.c3;
    case 4: return R.c4;
    case 5: return R.c5;
    case 6: return R.c6;
    case 7: return R.c7;
    case 8: return R.c8;
    default: return R.c9;
  }
}

struct DevInst {
  AccInst a;
  FastDiv f_nthr, f_niota, f_gx, f_gxy, f_bx, f_bxy;
  FastDiv f_loop[4];
};

// Runs one compiled expression.  `code`, `p`, `params` and `dims` are
// uniform across the wavefront.
__device__ __forceinline__ int64_t run_prog(const DInsn* __restrict__ code,
                                            const Prog p, const Regs& R,
                                            const int64_t* __restrict__ params,
                                            int64_t dflt, uint32_t& err) {
  if (p.absent) return dflt;
  Stack st;
  for (uint32_t k = 0; k < p.n; ++k) {
    const DInsn in = code[p.off + k];
    int64_t a, b;
    // launch extents follow the parameters of the tuple in the pool
    if (in.ma == M_REG) a = st[in.a];
    else if (in.ma == M_IMM) a = in.imm;
    else if (in.ma == M_PARAM) a = params[in.a];
    else a = coord(R, in.a);
    if (in.mb == M_REG) b = st[in.b];
    else if (in.mb == M_IMM) b = in.imm;
    else if (in.mb == M_PARAM) b = params[in.b];
    else b = coord(R, in.b);
    st[in.dst] = alu(in.op, a, b, err);
  }
  return st[p.res];
}

// Point coordinates of point index `pidx` = (blin * niota + ilin) * nthr + tlin.
struct PointIds {
  uint32_t blin, tlin, ilin;
};

__device__ __forceinline__ PointIds decode(const DevInst& I, uint32_t pidx) {
  PointIds o;
  uint32_t rest = fdiv(pidx, I.f_nthr);
  o.tlin = pidx - rest * I.a.nthr;
  o.blin = fdiv(rest, I.f_niota);
  o.ilin = rest - o.blin * I.a.niota;
  return o;
}

__device__ __forceinline__ void set_coords(const DevInst& I, const PointIds& p,
                                           const int64_t* __restrict__ loopvals,
                                           Regs& R) {
  uint32_t t1 = fdiv(p.tlin, I.f_bx);
  R.c0 = p.tlin - t1 * (uint32_t)I.a.dims[3];
  uint32_t t2 = fdiv(p.tlin, I.f_bxy);
  R.c1 = t1 - t2 * (uint32_t)I.a.dims[4];
  R.c2 = t2;
  uint32_t b1 = fdiv(p.blin, I.f_gx);
  R.c3 = p.blin - b1 * (uint32_t)I.a.dims[0];
  uint32_t b2 = fdiv(p.blin, I.f_gxy);
  R.c4 = b1 - b2 * (uint32_t)I.a.dims[1];
  R.c5 = b2;
  R.c6 = R.c7 = R.c8 = R.c9 = 0;
  uint32_t rem = p.ilin;
  const uint32_t nl = I.a.n_loops;
  if (nl > 3) {
    uint32_t q = fdiv(rem, I.f_loop[3]);
    R.c9 = loopvals[I.a.loop_off[3] + (rem - q * I.a.loop_n[3])];
    rem = q;
  }
  if (nl > 2) {
    uint32_t q = fdiv(rem, I.f_loop[2]);
    R.c8 = loopvals[I.a.loop_off[2] + (rem - q * I.a.loop_n[2])];
    rem = q;
  }
  if (nl > 1) {
    uint32_t q = fdiv(rem, I.f_loop[1]);
    R.c7 = loopvals[I.a.loop_off[1] + (rem - q * I.a.loop_n[1])];
    rem = q;
  }
  if (nl > 0) {
    uint32_t q = fdiv(rem, I.f_loop[0]);
    R.c6 = loopvals[I.a.loop_off[0] + (rem - q * I.a.loop_n[0])];
  }
}

struct Point {
  int64_t addr;
  uint32_t bint, wint;
};

// Evaluates guard, then (if it holds) address and interval ids, recording
// errors exactly as the C-level semantics say.  Returns the guard.
__device__ __forceinline__ bool eval_point(const DevInst& I,
                                           const DInsn* __restrict__ code,
                                           const int64_t* __restrict__ params,
                                           Regs& R, Point& pt, uint32_t& err) {
  const int64_t* pr = params + I.a.params_off;
  int64_t g = run_prog(code, I.a.guard, R, pr, 1, err);
  if (g == 0) return false;
  uint32_t e = 0;
  pt.addr = run_prog(code, I.a.addr, R, pr, 0, e);
  int64_t bi = run_prog(code, I.a.bint, R, pr, 0, e);
  int64_t wi = run_prog(code, I.a.wint, R, pr, 0, e);
  if (I.a.is32 && (pt.addr < INT32_MIN || pt.addr > INT32_MAX)) e |= ERR_RANGE;
  if (bi < 0 || bi > 65535 || wi < 0 || wi > 65535) e |= ERR_UNSUP;
  err |= e;
  pt.bint = (uint32_t)bi & 0xFFFF;
  pt.wint = (uint32_t)wi & 0xFFFF;
  return e == 0;
}

__device__ __forceinline__ void load_inst(DevInst& D,
                                          const DevInst* __restrict__ insts,
                                          uint32_t k) {
  k = __builtin_amdgcn_readfirstlane(k);
  D = insts[k];
}

// ---------------------------------------------------------------------------
// Reductions.

__device__ __forceinline__ u64 wave_sum(u64 v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ u64 wave_min(u64 v) {
  for (int o = 32; o > 0; o >>= 1) {
    u64 w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// LDS join of up to CAP records (both sides of one query under one tuple).

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kInactive = 1u << 14;  // in tli
constexpr uint32_t kSide = 1u << 15;      // in tli

template <int CAP, int TBL>
struct JoinLds {
  u64 addr[CAP];
  uint32_t blin[CAP];
  uint32_t tli[CAP];  // ilin << 16 | side << 15 | inactive << 14 | tlin
  uint32_t bw[CAP];   // bint << 16 | wint
  uint16_t w[CAP];    // warp of the analysed program
  uint16_t slot[CAP];
  int32_t part[CAP];
  uint32_t owner[TBL];
  uint32_t cnt[TBL];
  u64 red[8];
  uint32_t n;
  uint32_t err;
};

__device__ __forceinline__ uint32_t level_hash(int L, u64 addr, uint32_t blin,
                                               uint32_t bw, uint32_t w,
                                               uint32_t t) {
  u64 h = addr * 0x9E3779B97F4A7C15ull;
  if (L >= 1) h ^= (u64)(blin + 1) * 0xC2B2AE3D27D4EB4Full;
  if (L >= 2) h ^= (u64)((bw >> 16) + 1) * 0x165667B19E3779F9ull;
  if (L >= 3) h ^= (u64)(w + 1) * 0x27D4EB2F165667C5ull;
  if (L >= 4) h ^= (u64)((bw & 0xFFFF) + 1) * 0x94D049BB133111EBull;
  if (L >= 5) h ^= (u64)(t + 1) * 0xBF58476D1CE4E5B9ull;
  h ^= h >> 31;
  h *= 0x9E3779B97F4A7C15ull;
  h ^= h >> 29;
  return (uint32_t)(h >> 32);
}

template <int CAP, int TBL>
__device__ __forceinline__ bool level_eq(const JoinLds<CAP, TBL>& S, int L,
                                         uint32_t x, uint32_t y) {
  if (S.addr[x] != S.addr[y]) return false;
  if (L >= 1 && S.blin[x] != S.blin[y]) return false;
  if (L >= 2 && (S.bw[x] >> 16) != (S.bw[y] >> 16)) return false;
  if (L >= 3 && S.w[x] != S.w[y]) return false;
  if (L >= 4 && (S.bw[x] & 0xFFFF) != (S.bw[y] & 0xFFFF)) return false;
  if (L >= 5 && (S.tli[x] & 0x3FF) != (S.tli[y] & 0x3FF)) return false;
  return true;
}

// Joins the S.n records in LDS; adds class counts and the witness candidate
// to the query accumulators.  All threads of the block must call it.
template <int CAP, int TBL>
__device__ void lds_join(JoinLds<CAP, TBL>& S, const QDesc& qd, uint32_t sigma,
                         QAcc* __restrict__ acc) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t n = S.n;
  const uint32_t mask = qd.mask;
  const bool self = qd.self != 0;
  uint32_t used = 0;
  if (mask & 1) used |= 0x03;
  if (mask & 2) used |= 0x0C;
  if (mask & 4) used |= 0x30;
  if (used == 0 || n == 0) return;
  const int f = __ffs(used) - 1;
  u64 Sl[6] = {0, 0, 0, 0, 0, 0};
  for (uint32_t r = tid; r < n; r += nt) S.part[r] = 0;
  bool any = true;
  for (int L = f; L < 6; ++L) {
    if (!((used >> L) & 1)) continue;
    for (uint32_t k = tid; k < TBL; k += nt) {
      S.owner[k] = kEmpty;
      S.cnt[k] = 0;
    }
    __syncthreads();
    u64 s = 0;
    for (uint32_t r = tid; r < n; r += nt) {
      uint32_t tl = S.tli[r];
      if (tl & kInactive) continue;
      uint32_t h = level_hash(L, S.addr[r], S.blin[r], S.bw[r], S.w[r],
                              tl & 0x3FF) & (TBL - 1);
      for (;;) {
        uint32_t o = atomicCAS(&S.owner[h], kEmpty, r);
        if (o == kEmpty || level_eq(S, L, o, r)) break;
        h = (h + 1) & (TBL - 1);
      }
      uint32_t side = (tl & kSide) ? 1u : 0u;
      uint32_t old = atomicAdd(&S.cnt[h], (self || !side) ? 1u : 0x10000u);
      if (self) s += 2ull * (old & 0xFFFF) + 1;
      else s += side ? (old & 0xFFFF) : (old >> 16);
      S.slot[r] = (uint16_t)h;
    }
    __syncthreads();
    const int sign = (L & 1) ? -1 : 1;
    const uint32_t cls = L < 2 ? 1u : (L < 4 ? 2u : 4u);
    bool any_local = false;
    for (uint32_t r = tid; r < n; r += nt) {
      uint32_t tl = S.tli[r];
      if (tl & kInactive) continue;
      uint32_t c = S.cnt[S.slot[r]];
      if (L == f) {
        bool cand = self ? ((c & 0xFFFF) >= 2) : ((c & 0xFFFF) && (c >> 16));
        if (!cand) {
          S.tli[r] = tl | kInactive;
          if (self) s -= 1;  // a lone record pairs only with itself
          continue;
        }
        any_local = true;
      }
      if (!self && (tl & kSide)) continue;
      if (cls & mask) {
        int32_t nj = (int32_t)(self ? (c & 0xFFFF) : (c >> 16));
        S.part[r] += sign * nj;
      }
    }
    Sl[L] = s;
    if (L == f) {
      any = __syncthreads_or(any_local);
      if (!any) break;
    } else {
      __syncthreads();
    }
  }
  if (!any) return;
  // class counts: reduce S_L over the block
  u64 c0 = (mask & 1) ? Sl[0] - Sl[1] : 0;
  u64 c1 = (mask & 2) ? Sl[2] - Sl[3] : 0;
  u64 c2 = (mask & 4) ? Sl[4] - Sl[5] : 0;
  u64 best = kNoKey;
  for (uint32_t r = tid; r < n; r += nt) {
    uint32_t tl = S.tli[r];
    if ((tl & kInactive) || (!self && (tl & kSide))) continue;
    if (S.part[r] > 0) {
      u64 k = pkey(sigma, S.blin[r], tl & 0x3FF, tl >> 16);
      best = k < best ? k : best;
    }
  }
  if (tid < 4) S.red[tid] = tid == 3 ? kNoKey : 0;
  __syncthreads();
  c0 = wave_sum(c0);
  c1 = wave_sum(c1);
  c2 = wave_sum(c2);
  best = wave_min(best);
  if ((tid & 63) == 0) {
    if (c0) atomicAdd(&S.red[0], c0);
    if (c1) atomicAdd(&S.red[1], c1);
    if (c2) atomicAdd(&S.red[2], c2);
    if (best != kNoKey) atomicMin(&S.red[3], best);
  }
  __syncthreads();
  if (tid == 0) {
    if (S.red[0]) atomicAdd(&acc->cnt[0], S.red[0]);
    if (S.red[1]) atomicAdd(&acc->cnt[1], S.red[1]);
    if (S.red[2]) atomicAdd(&acc->cnt[2], S.red[2]);
    if (S.red[3] != kNoKey) atomicMin(&acc->pmin, S.red[3]);
  }
}

// Appends a record to the LDS arrays (wavefront-aggregated slot claim).
template <int CAP, int TBL>
__device__ __forceinline__ void lds_append(JoinLds<CAP, TBL>& S, bool valid,
                                           const Point& pt, const PointIds& id,
                                           uint32_t side, uint32_t warp_w) {
  u64 bal = __ballot(valid);
  if (bal == 0) return;
  uint32_t lane = threadIdx.x & 63;
  uint32_t leader = __ffsll((long long)bal) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(&S.n, (uint32_t)__popcll(bal));
  base = __shfl(base, leader, 64);
  if (valid) {
    uint32_t r = base + __popcll(bal & ((1ull << lane) - 1));
    if (r >= CAP) {  // the planner never lets this happen; never write past
      atomicOr(&S.err, ERR_INTERNAL);
      return;
    }
    S.addr[r] = (u64)pt.addr;
    S.blin[r] = id.blin;
    S.tli[r] = (id.ilin << 16) | (side << 15) | id.tlin;
    S.bw[r] = (pt.bint << 16) | pt.wint;
    S.w[r] = (uint16_t)warp_w;
  }
}

// ---------------------------------------------------------------------------
// Kernel: generate both sides of a small item straight into LDS and join.

template <int CAP, int TBL>
__global__ void __launch_bounds__(256)
k_small_join(const SItem* __restrict__ items, const DevInst* __restrict__ insts,
             const DInsn* __restrict__ code, const int64_t* __restrict__ params,
             const int64_t* __restrict__ loopvals, const QDesc* __restrict__ qd,
             QAcc* __restrict__ acc) {
  extern __shared__ __align__(16) unsigned char smem[];
  JoinLds<CAP, TBL>& S = *reinterpret_cast<JoinLds<CAP, TBL>*>(smem);
  const SItem it = items[blockIdx.x];
  const QDesc q = qd[it.q];
  if (threadIdx.x == 0) {
    S.n = 0;
    S.err = 0;
  }
  __syncthreads();
  uint32_t err = 0;
  const int nside = q.self ? 1 : 2;
  for (int side = 0; side < nside; ++side) {
    DevInst I;
    load_inst(I, insts, side ? it.inst_j : it.inst_i);
    const uint32_t p0 = it.b0 * I.a.tpb, p1 = it.b1 * I.a.tpb;
    for (uint32_t base = p0; base < p1; base += blockDim.x) {
      uint32_t pidx = base + threadIdx.x;
      bool valid = false;
      Point pt;
      PointIds id;
      if (pidx < p1) {
        id = decode(I, pidx);
        Regs R;
        set_coords(I, id, loopvals, R);
        valid = eval_point(I, code, params, R, pt, err);
      }
      uint32_t w = valid ? id.tlin / q.warp : 0;
      lds_append(S, valid, pt, id, (uint32_t)side, w);
    }
  }
  err = wave_or(err);
  if ((threadIdx.x & 63) == 0 && err) atomicOr(&S.err, err);
  __syncthreads();
  if (S.err) {
    if (threadIdx.x == 0) atomicOr(&acc[it.q].err, S.err);
    return;
  }
  lds_join(S, q, it.sigma, &acc[it.q]);
}

// ---------------------------------------------------------------------------
// Kernel: generate points and scatter (key, point id) records into
// fixed-capacity HBM buckets chosen by a hash of the address (and of the
// block for shared arrays, whose memory is per block).

__device__ __forceinline__ u64 mix64(u64 x) {
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDull;
  x ^= x >> 33;
  x *= 0xC4CEB9FE1A85EC53ull;
  x ^= x >> 33;
  return x;
}

__global__ void __launch_bounds__(256)
k_scatter(const Chunk* __restrict__ chunks, const HItem* __restrict__ hitems,
          const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
          const int64_t* __restrict__ params,
          const int64_t* __restrict__ loopvals, QAcc* __restrict__ acc,
          unsigned char* __restrict__ keys, uint32_t* __restrict__ pids,
          uint32_t* __restrict__ cursor, uint32_t* __restrict__ ovf,
          uint32_t capb) {
  const Chunk ch = chunks[blockIdx.x];
  const HItem h = hitems[ch.item];
  DevInst I;
  load_inst(I, insts, ch.side ? h.inst_j : h.inst_i);
  uint32_t err = 0;
  bool over = false;
  for (uint32_t base = ch.p0; base < ch.p1; base += blockDim.x) {
    uint32_t pidx = base + threadIdx.x;
    if (pidx >= ch.p1) break;
    PointIds id = decode(I, pidx);
    Regs R;
    set_coords(I, id, loopvals, R);
    Point pt;
    if (!eval_point(I, code, params, R, pt, err)) continue;
    if (h.nbuckets == 0) continue;  // error scan only
    u64 hk = (u64)pt.addr;
    if (h.shared) hk ^= (u64)(id.blin + 1) * 0x9E3779B97F4A7C15ull;
    uint32_t b = (uint32_t)__umul64hi(mix64(hk), (u64)h.nbuckets);
    uint32_t g = h.bucket0 + b;
    uint32_t pos = atomicAdd(&cursor[g], 1u);
    if (pos < capb) {
      u64 slot = (u64)b * capb + pos;
      if (h.is32)
        reinterpret_cast<int32_t*>(keys + h.key_off)[slot] = (int32_t)pt.addr;
      else
        reinterpret_cast<int64_t*>(keys + h.key_off)[slot] = pt.addr;
      pids[h.pid_off + slot] = (ch.side << 31) | pidx;
    } else {
      over = true;
      atomicMax(&ovf[ch.item], pos + 1);  // largest bucket load seen
    }
  }
  err = wave_or(err);
  if ((threadIdx.x & 63) == 0 && err) atomicOr(&acc[h.q].err, err);
  (void)over;
}

// ---------------------------------------------------------------------------
// Kernel: one workgroup per HBM bucket; load its records into LDS and join.

template <int CAP, int TBL>
__global__ void __launch_bounds__(256)
k_bucket_join(const uint32_t* __restrict__ bucket_item,
              const HItem* __restrict__ hitems,
              const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
              const int64_t* __restrict__ params,
              const int64_t* __restrict__ loopvals,
              const QDesc* __restrict__ qd, QAcc* __restrict__ acc,
              const unsigned char* __restrict__ keys,
              const uint32_t* __restrict__ pids,
              const uint32_t* __restrict__ cursor,
              const uint32_t* __restrict__ ovf, uint32_t bucket_base) {
  extern __shared__ __align__(16) unsigned char smem[];
  JoinLds<CAP, TBL>& S = *reinterpret_cast<JoinLds<CAP, TBL>*>(smem);
  const uint32_t g = bucket_base + blockIdx.x;
  const uint32_t hi = bucket_item[g];
  const HItem h = hitems[hi];
  if (ovf[hi]) return;
  uint32_t n = cursor[g];
  if (n == 0) return;
  if (n > CAP) n = CAP;  // cannot happen without the overflow flag
  const QDesc q = qd[h.q];
  const uint32_t b = g - h.bucket0;
  const u64 slot0 = (u64)b * CAP;
  uint32_t err = 0;
  for (int side = 0; side < 2; ++side) {
    DevInst I;
    load_inst(I, insts, side ? h.inst_j : h.inst_i);
    const bool need_iv = !(I.a.bint.absent && I.a.wint.absent);
    for (uint32_t r = threadIdx.x; r < n; r += blockDim.x) {
      uint32_t pid = pids[h.pid_off + slot0 + r];
      if ((pid >> 31) != (uint32_t)side) continue;
      PointIds id = decode(I, pid & 0x7FFFFFFFu);
      int64_t a;
      if (h.is32)
        a = reinterpret_cast<const int32_t*>(keys + h.key_off)[slot0 + r];
      else
        a = reinterpret_cast<const int64_t*>(keys + h.key_off)[slot0 + r];
      uint32_t bi = 0, wi = 0;
      if (need_iv) {
        Regs R;
        set_coords(I, id, loopvals, R);
        const int64_t* pr = params + I.a.params_off;
        uint32_t e = 0;
        bi = (uint32_t)run_prog(code, I.a.bint, R, pr, 0, e) & 0xFFFF;
        wi = (uint32_t)run_prog(code, I.a.wint, R, pr, 0, e) & 0xFFFF;
      }
      S.addr[r] = (u64)a;
      S.blin[r] = id.blin;
      S.tli[r] = (id.ilin << 16) | ((uint32_t)side << 15) | id.tlin;
      S.bw[r] = (bi << 16) | wi;
      S.w[r] = (uint16_t)(id.tlin / q.warp);
    }
  }
  (void)err;
  if (threadIdx.x == 0) S.n = n;
  __syncthreads();
  lds_join(S, q, h.sigma, &acc[h.q]);
}

// ---------------------------------------------------------------------------
// Fallback for items that still overflow after a retry with more buckets
// (a single address, or a single (address, block), carries more points than
// one LDS tile holds).  Records of all such items go to one flat HBM array;
// every prefix level is aggregated in an HBM hash table keyed by (item,
// level key).  Each workgroup first merges its tile of records in an LDS
// table, so a hot key costs one global atomic per workgroup, not per point.

struct GRec {
  u64* addr;
  uint32_t* blin;
  uint32_t* tli;
  uint32_t* bw;
  uint32_t* w;
  uint32_t* item;  // fallback item index, 0xFFFFFFFF: empty slot
  uint32_t* slot;
  long long* part;
};

__global__ void __launch_bounds__(256)
k_gen_linear(const Chunk* __restrict__ chunks, const FItem* __restrict__ fitems,
             const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
             const int64_t* __restrict__ params,
             const int64_t* __restrict__ loopvals, GRec rec,
             uint32_t* __restrict__ count) {
  const Chunk ch = chunks[blockIdx.x];
  const FItem f = fitems[ch.item];
  DevInst I;
  load_inst(I, insts, ch.side ? f.inst_j : f.inst_i);
  uint32_t err = 0;
  for (uint32_t base = ch.p0; base < ch.p1; base += blockDim.x) {
    uint32_t pidx = base + threadIdx.x;
    bool valid = false;
    Point pt;
    PointIds id;
    if (pidx < ch.p1) {
      id = decode(I, pidx);
      Regs R;
      set_coords(I, id, loopvals, R);
      valid = eval_point(I, code, params, R, pt, err);
    }
    u64 bal = __ballot(valid);
    if (bal == 0) continue;
    uint32_t lane = threadIdx.x & 63;
    uint32_t leader = __ffsll((long long)bal) - 1;
    uint32_t b0 = 0;
    if (lane == leader) b0 = atomicAdd(&count[ch.item], (uint32_t)__popcll(bal));
    b0 = __shfl(b0, leader, 64);
    if (valid) {
      uint32_t k = b0 + __popcll(bal & ((1ull << lane) - 1));
      if (k < f.cap) {
        u64 r = f.off + k;
        rec.addr[r] = (u64)pt.addr;
        rec.blin[r] = id.blin;
        rec.tli[r] = (id.ilin << 16) | (ch.side << 15) | id.tlin;
        rec.bw[r] = (pt.bint << 16) | pt.wint;
        rec.w[r] = id.tlin / f.warp;
        rec.item[r] = ch.item;
        rec.part[r] = 0;
      }
    }
  }
}

__device__ __forceinline__ bool g_level_eq(const GRec& g, int L, u64 x, u64 y) {
  if (g.item[x] != g.item[y]) return false;
  if (g.addr[x] != g.addr[y]) return false;
  if (L >= 1 && g.blin[x] != g.blin[y]) return false;
  if (L >= 2 && (g.bw[x] >> 16) != (g.bw[y] >> 16)) return false;
  if (L >= 3 && g.w[x] != g.w[y]) return false;
  if (L >= 4 && (g.bw[x] & 0xFFFF) != (g.bw[y] & 0xFFFF)) return false;
  if (L >= 5 && (g.tli[x] & 0x3FF) != (g.tli[y] & 0x3FF)) return false;
  return true;
}

__device__ __forceinline__ uint32_t g_hash(const GRec& g, int L, u64 r) {
  return level_hash(L, g.addr[r] ^ ((u64)g.item[r] * 0x2545F4914F6CDD1Dull),
                    g.blin[r], g.bw[r], g.w[r], g.tli[r] & 0x3FF);
}

__device__ __forceinline__ bool uses_level(uint32_t mask, int L) {
  return (mask >> (L >> 1)) & 1;
}

constexpr int kGTile = 1024;  // records per workgroup step
constexpr int kGLocal = 2048; // LDS table slots

// Inserts every record at level L.  S[item * 8 + L] += pair contributions.
__global__ void __launch_bounds__(256)
k_ginsert(GRec g, u64 n, int L, const FItem* __restrict__ fitems,
          uint32_t* __restrict__ owner, u64* __restrict__ cnt, u64 tbl_mask,
          u64* __restrict__ S) {
  __shared__ uint32_t lown[kGLocal];
  __shared__ uint32_t lcnt[kGLocal];
  __shared__ uint32_t lgs[kGLocal];
  const uint32_t tid = threadIdx.x;
  for (u64 t0 = (u64)blockIdx.x * kGTile; t0 < n; t0 += (u64)gridDim.x * kGTile) {
    for (uint32_t k = tid; k < kGLocal; k += blockDim.x) {
      lown[k] = kEmpty;
      lcnt[k] = 0;
    }
    __syncthreads();
    uint16_t ls[kGTile / 256];
#pragma unroll
    for (int j = 0; j < kGTile / 256; ++j) {
      ls[j] = 0xFFFF;
      u64 r = t0 + j * 256 + tid;
      if (r >= n) continue;
      uint32_t it = g.item[r];
      if (it == kEmpty) continue;
      const FItem f = fitems[it];
      if (!uses_level(f.mask, L)) continue;
      uint32_t h = g_hash(g, L, r) & (kGLocal - 1);
      const uint32_t lr = (uint32_t)(r - t0);
      for (;;) {
        uint32_t o = atomicCAS(&lown[h], kEmpty, lr);
        if (o == kEmpty || g_level_eq(g, L, t0 + o, r)) break;
        h = (h + 1) & (kGLocal - 1);
      }
      uint32_t side = (g.tli[r] >> 15) & 1;
      atomicAdd(&lcnt[h], (f.self || !side) ? 1u : 0x10000u);
      ls[j] = (uint16_t)h;
    }
    __syncthreads();
    // merge each local group into the global table
    for (uint32_t k = tid; k < kGLocal; k += blockDim.x) {
      uint32_t lr = lown[k];
      if (lr == kEmpty) continue;
      u64 r = t0 + lr;
      const uint32_t it = g.item[r];
      const FItem f = fitems[it];
      u64 h = g_hash(g, L, r) & tbl_mask;
      for (;;) {
        uint32_t o = atomicCAS(&owner[h], kEmpty, (uint32_t)r);
        if (o == kEmpty || g_level_eq(g, L, o, r)) break;
        h = (h + 1) & tbl_mask;
      }
      uint32_t c = lcnt[k];
      u64 li = c & 0xFFFF, lj = c >> 16;
      u64 old = atomicAdd(&cnt[h], f.self ? li : (li | (lj << 32)));
      u64 contrib;
      if (f.self) contrib = 2 * old * li + li * li;  // (old + k)^2 - old^2
      else contrib = li * (old >> 32) + lj * (old & 0xFFFFFFFFull) + li * lj;
      if (contrib) atomicAdd(&S[(u64)it * 8 + L], contrib);
      lgs[k] = (uint32_t)h;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kGTile / 256; ++j) {
      u64 r = t0 + j * 256 + tid;
      if (ls[j] != 0xFFFF) g.slot[r] = lgs[ls[j]];
    }
    __syncthreads();
  }
}

// Adds +-(partners at level L) to every record of side a (self: all).
__global__ void __launch_bounds__(256)
k_gpartner(GRec g, u64 n, int L, const FItem* __restrict__ fitems,
           const u64* __restrict__ cnt) {
  const long long sign = (L & 1) ? -1 : 1;
  for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (u64)gridDim.x * blockDim.x) {
    uint32_t it = g.item[r];
    if (it == kEmpty) continue;
    const FItem f = fitems[it];
    if (!uses_level(f.mask, L)) continue;
    uint32_t side = (g.tli[r] >> 15) & 1;
    if (!f.self && side) continue;
    u64 c = cnt[g.slot[r]];
    long long nj = f.self ? (long long)c : (long long)(c >> 32);
    g.part[r] += sign * nj;
  }
}

// Witness candidates of the fallback records.
__global__ void __launch_bounds__(256)
k_gfinish(GRec g, u64 n, const FItem* __restrict__ fitems,
          QAcc* __restrict__ acc) {
  for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (u64)gridDim.x * blockDim.x) {
    uint32_t it = g.item[r];
    if (it == kEmpty) continue;
    const FItem f = fitems[it];
    uint32_t tl = g.tli[r];
    if (!f.self && (tl & kSide)) continue;
    if (g.part[r] > 0) {
      u64 k = pkey(f.sigma, g.blin[r], tl & 0x3FF, tl >> 16);
      if (k < acc[f.q].pmin) atomicMin(&acc[f.q].pmin, k);
    }
  }
}

// Class counts of each fallback item from its level sums.
__global__ void k_gcounts(uint32_t nitems, const FItem* __restrict__ fitems,
                          const u64* __restrict__ S, QAcc* __restrict__ acc) {
  uint32_t it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitems) return;
  const FItem f = fitems[it];
  const u64* s = S + (u64)it * 8;
  if (f.mask & 1) atomicAdd(&acc[f.q].cnt[0], s[0] - s[1]);
  if (f.mask & 2) atomicAdd(&acc[f.q].cnt[1], s[2] - s[3]);
  if (f.mask & 4) atomicAdd(&acc[f.q].cnt[2], s[4] - s[5]);
}

__global__ void k_fill_u64(u64* __restrict__ p, u64 n, u64 v) {
  for (u64 k = (u64)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (u64)gridDim.x * blockDim.x)
    p[k] = v;
}

// ---------------------------------------------------------------------------
// Witness pass 2: with p* fixed, the smallest q of access b (same tuple)
// that conflicts with it.

struct W2Item {
  uint32_t q, inst_i, inst_j, p0, p1, pad0, pad1, pad2;
};

__global__ void __launch_bounds__(256)
k_witness2(const W2Item* __restrict__ items, const DevInst* __restrict__ insts,
           const DInsn* __restrict__ code, const int64_t* __restrict__ params,
           const int64_t* __restrict__ loopvals, const QDesc* __restrict__ qd,
           QAcc* __restrict__ acc) {
  const W2Item it = items[blockIdx.x];
  const QDesc q = qd[it.q];
  const u64 pk = acc[it.q].pmin;
  const uint32_t ps = (uint32_t)(pk >> 52);
  const uint32_t pb = (uint32_t)(pk >> 26) & ((1u << 26) - 1);
  const uint32_t pt_ = (uint32_t)(pk >> 16) & 0x3FF;
  const uint32_t pi = (uint32_t)pk & 0xFFFF;
  // p*: every lane evaluates the same point
  Point P;
  uint32_t e = 0;
  {
    DevInst I;
    load_inst(I, insts, it.inst_i);
    PointIds id;
    id.blin = pb;
    id.tlin = pt_;
    id.ilin = pi;
    Regs R;
    set_coords(I, id, loopvals, R);
    eval_point(I, code, params, R, P, e);
  }
  const uint32_t pw = pt_ / q.warp;
  if (it.p0 == 0 && threadIdx.x == 0) acc[it.q].waddr = P.addr;
  DevInst J;
  load_inst(J, insts, it.inst_j);
  u64 best = kNoKey;
  uint32_t err = 0;
  for (uint32_t base = it.p0; base < it.p1; base += blockDim.x) {
    uint32_t pidx = base + threadIdx.x;
    if (pidx >= it.p1) break;
    PointIds id = decode(J, pidx);
    Regs R;
    set_coords(J, id, loopvals, R);
    Point Q;
    if (!eval_point(J, code, params, R, Q, err)) continue;
    if (Q.addr != P.addr) continue;
    if (id.blin == pb && id.tlin == pt_) continue;
    uint32_t cls;
    if (id.blin != pb) cls = 1;
    else if (id.tlin / q.warp == pw) cls = 4;
    else cls = 2;
    if (!(cls & q.mask)) continue;
    if (cls != 1 && Q.bint != P.bint) continue;
    if (cls == 4 && Q.wint != P.wint) continue;
    u64 k = pkey(ps, id.blin, id.tlin, id.ilin);
    best = k < best ? k : best;
  }
  best = wave_min(best);
  if ((threadIdx.x & 63) == 0 && best != kNoKey) atomicMin(&acc[it.q].qmin, best);
}



// ---------------------------------------------------------------------------
// Small fills (used instead of memset nodes so that a captured graph
// replays correctly).

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += gridDim.x * blockDim.x)
    p[k] = v;
}

__global__ void k_init_acc(QAcc* __restrict__ acc, uint32_t n) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += gridDim.x * blockDim.x) {
    QAcc a;
    a.cnt[0] = a.cnt[1] = a.cnt[2] = 0;
    a.pmin = kNoKey;
    a.qmin = kNoKey;
    a.err = 0;
    a.qclass = 0;
    a.waddr = 0;
    acc[k] = a;
  }
}

// ---------------------------------------------------------------------------
// Results: status by precedence, counts, verdict and the decoded witness.

__global__ void __launch_bounds__(256)
k_finalize(uint32_t n, const QAcc* __restrict__ acc,
           const QDesc* __restrict__ qd, const uint32_t* __restrict__ host_err,
           const uint8_t* __restrict__ trivial,
           const unsigned long long* __restrict__ evals,
           rd_pair_result* __restrict__ out) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  rd_pair_result r;
  memset(&r, 0, sizeof r);
  r.w_set = r.w_b1 = r.w_t1 = r.w_i1 = r.w_b2 = r.w_t2 = r.w_i2 = 0xFFFFFFFFu;
  r.evals = evals[k];
  const QAcc a = acc[k];
  uint32_t e = host_err[k] | a.err;
  if (e & ERR_INTERNAL) r.status = RD_EDEVICE;
  else if (e & ERR_INVAL) r.status = RD_EINVAL;
  else if (e & ERR_UNSUP) r.status = RD_EUNSUPPORTED;
  else if (e & ERR_DIVZERO) r.status = RD_EDIVZERO;
  else if (e & ERR_RANGE) r.status = RD_ERANGE;
  if (r.status == 0 && trivial[k]) r.flags = 1;
  if (r.status == 0 && !trivial[k]) {
    r.count_by_class[0] = a.cnt[0];
    r.count_by_class[1] = a.cnt[1];
    r.count_by_class[2] = a.cnt[2];
    r.count = a.cnt[0] + a.cnt[1] + a.cnt[2];
    r.verdict = r.count != 0;
    r.classes = (a.cnt[0] ? 1 : 0) | (a.cnt[1] ? 2 : 0) | (a.cnt[2] ? 4 : 0);
    if (r.verdict && a.pmin != kNoKey && a.qmin != kNoKey) {
      const uint32_t m26 = (1u << 26) - 1;
      r.w_set = (uint32_t)(a.pmin >> 52);
      r.w_b1 = (uint32_t)(a.pmin >> 26) & m26;
      r.w_t1 = (uint32_t)(a.pmin >> 16) & 0x3FF;
      r.w_i1 = (uint32_t)a.pmin & 0xFFFF;
      r.w_b2 = (uint32_t)(a.qmin >> 26) & m26;
      r.w_t2 = (uint32_t)(a.qmin >> 16) & 0x3FF;
      r.w_i2 = (uint32_t)a.qmin & 0xFFFF;
      r.w_addr = a.waddr;
      if (r.w_b1 != r.w_b2) r.witness_class = 1;
      else if (r.w_t1 / qd[k].warp == r.w_t2 / qd[k].warp) r.witness_class = 4;
      else r.witness_class = 2;
    }
  }
  out[k] = r;
}

// ---------------------------------------------------------------------------
// Launch wrappers (host side).

#define HGRD_CHECK(x)                     \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return (int)e_; \
  } while (0)

template <int CAP, int TBL>
static int launch_small_t(hipStream_t st, const SItem* items, uint32_t n,
                          const DevInst* insts, const DInsn* code,
                          const int64_t* params, const int64_t* loopvals,
                          const QDesc* qd, QAcc* acc) {
  size_t lds = sizeof(JoinLds<CAP, TBL>);
  static bool attr = false;
  if (!attr) {
    HGRD_CHECK(hipFuncSetAttribute((const void*)k_small_join<CAP, TBL>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
    attr = true;
  }
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL((k_small_join<CAP, TBL>), dim3(m), dim3(256), lds, st,
                       items + off, insts, code, params, loopvals, qd, acc);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

template <int CAP, int TBL>
static int launch_bucket_t(hipStream_t st, uint32_t nb, uint32_t base,
                           const uint32_t* bucket_item, const HItem* hitems,
                           const DevInst* insts, const DInsn* code,
                           const int64_t* params, const int64_t* loopvals,
                           const QDesc* qd, QAcc* acc,
                           const unsigned char* keys, const uint32_t* pids,
                           const uint32_t* cursor, const uint32_t* ovf) {
  size_t lds = sizeof(JoinLds<CAP, TBL>);
  static bool attr = false;
  if (!attr) {
    HGRD_CHECK(hipFuncSetAttribute((const void*)k_bucket_join<CAP, TBL>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((k_bucket_join<CAP, TBL>), dim3(nb), dim3(256), lds, st,
                     bucket_item, hitems, insts, code, params, loopvals, qd,
                     acc, keys, pids, cursor, ovf, base);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

}  // namespace hgrd

// ---- entry points used by the host driver ---------------------------------
namespace hgrd {

size_t devinst_size() { return sizeof(DevInst); }

void fill_devinst(void* dst, const AccInst& a) {
  DevInst d;
  memset(&d, 0, sizeof d);
  d.a = a;
  d.f_nthr = make_fastdiv(a.nthr ? a.nthr : 1);
  d.f_niota = make_fastdiv(a.niota ? a.niota : 1);
  d.f_gx = make_fastdiv(a.dims[0] > 0 ? a.dims[0] : 1);
  d.f_gxy = make_fastdiv(a.dims[0] > 0 && a.dims[1] > 0 ? a.dims[0] * a.dims[1] : 1);
  d.f_bx = make_fastdiv(a.dims[3] > 0 ? a.dims[3] : 1);
  d.f_bxy = make_fastdiv(a.dims[3] > 0 && a.dims[4] > 0 ? a.dims[3] * a.dims[4] : 1);
  for (int k = 0; k < 4; ++k) d.f_loop[k] = make_fastdiv(a.loop_n[k] ? a.loop_n[k] : 1);
  memcpy(dst, &d, sizeof d);
}

// Host check of the division helper (exported for the CPU tests).
int fastdiv_check(uint32_t n, uint32_t d) {
  FastDiv f = make_fastdiv(d);
  uint32_t t = (uint32_t)(((u64)f.m * n) >> 32);
  uint32_t q = (t + n) >> f.s;
  return q == n / d;
}

int join_lds_bytes(int cfg) {
  switch (cfg) {
    case 0: return (int)sizeof(JoinLds<1024, 2048>);
    case 1: return (int)sizeof(JoinLds<1536, 4096>);
    default: return (int)sizeof(JoinLds<3072, 8192>);
  }
}

int join_cap(int cfg) { return cfg == 0 ? 1024 : cfg == 1 ? 1536 : 3072; }

int launch_small(int cfg, hipStream_t st, const SItem* items, uint32_t n,
                 const void* insts, const DInsn* code, const int64_t* params,
                 const int64_t* loopvals, const QDesc* qd, QAcc* acc) {
  const DevInst* I = (const DevInst*)insts;
  switch (cfg) {
    case 0: return launch_small_t<1024, 2048>(st, items, n, I, code, params, loopvals, qd, acc);
    case 1: return launch_small_t<1536, 4096>(st, items, n, I, code, params, loopvals, qd, acc);
    default: return launch_small_t<3072, 8192>(st, items, n, I, code, params, loopvals, qd, acc);
  }
}

int launch_scatter(hipStream_t st, const Chunk* chunks, uint32_t n,
                   const HItem* hitems, const void* insts, const DInsn* code,
                   const int64_t* params, const int64_t* loopvals, QAcc* acc,
                   unsigned char* keys, uint32_t* pids, uint32_t* cursor,
                   uint32_t* ovf, uint32_t capb) {
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL(k_scatter, dim3(m), dim3(256), 0, st, chunks + off,
                       hitems, (const DevInst*)insts, code, params, loopvals,
                       acc, keys, pids, cursor, ovf, capb);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_bucket(int cfg, hipStream_t st, uint32_t nb, uint32_t base,
                  const uint32_t* bucket_item, const HItem* hitems,
                  const void* insts, const DInsn* code, const int64_t* params,
                  const int64_t* loopvals, const QDesc* qd, QAcc* acc,
                  const unsigned char* keys, const uint32_t* pids,
                  const uint32_t* cursor, const uint32_t* ovf) {
  const DevInst* I = (const DevInst*)insts;
  switch (cfg) {
    case 0: return launch_bucket_t<1024, 2048>(st, nb, base, bucket_item, hitems, I, code, params, loopvals, qd, acc, keys, pids, cursor, ovf);
    case 1: return launch_bucket_t<1536, 4096>(st, nb, base, bucket_item, hitems, I, code, params, loopvals, qd, acc, keys, pids, cursor, ovf);
    default: return launch_bucket_t<3072, 8192>(st, nb, base, bucket_item, hitems, I, code, params, loopvals, qd, acc, keys, pids, cursor, ovf);
  }
}

static uint32_t grid_for(u64 n, uint32_t per) {
  u64 g = (n + per - 1) / per;
  if (g > 8192) g = 8192;
  if (g == 0) g = 1;
  return (uint32_t)g;
}

int launch_fallback(hipStream_t st, const Chunk* chunks, uint32_t nchunks,
                    const FItem* fitems, uint32_t nitems, uint32_t used_levels,
                    const void* insts, const DInsn* code, const int64_t* params,
                    const int64_t* loopvals, GRecPtrs gp, u64 n,
                    uint32_t* count, uint32_t* owner, void* cnt, u64 tbl,
                    void* S, QAcc* acc) {
  GRec g{(u64*)gp.addr, gp.blin, gp.tli, gp.bw, gp.w, gp.item, gp.slot,
         (long long*)gp.part};
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, st,
                     gp.item, (uint32_t)n, kEmpty);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, count, nitems, 0u);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((u64)nitems * 8, 256)), dim3(256),
                     0, st, (u64*)S, (u64)nitems * 8, 0ull);
  for (uint32_t off = 0; off < nchunks; off += 1u << 20) {
    uint32_t m = nchunks - off < (1u << 20) ? nchunks - off : (1u << 20);
    hipLaunchKernelGGL(k_gen_linear, dim3(m), dim3(256), 0, st, chunks + off,
                       fitems, (const DevInst*)insts, code, params, loopvals, g,
                       count);
  }
  HGRD_CHECK(hipGetLastError());
  for (int L = 0; L < 6; ++L) {
    if (!((used_levels >> L) & 1)) continue;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(tbl, 256)), dim3(256), 0, st,
                       owner, (uint32_t)tbl, kEmpty);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(tbl, 256)), dim3(256), 0, st,
                       (u64*)cnt, tbl, 0ull);
    hipLaunchKernelGGL(k_ginsert, dim3(grid_for(n, kGTile)), dim3(256), 0, st, g,
                       n, L, fitems, owner, (u64*)cnt, tbl - 1, (u64*)S);
    hipLaunchKernelGGL(k_gpartner, dim3(grid_for(n, 256)), dim3(256), 0, st, g,
                       n, L, fitems, (const u64*)cnt);
    HGRD_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_gfinish, dim3(grid_for(n, 256)), dim3(256), 0, st, g, n,
                     fitems, acc);
  hipLaunchKernelGGL(k_gcounts, dim3((nitems + 255) / 256), dim3(256), 0, st,
                     nitems, fitems, (const u64*)S, acc);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_witness2(hipStream_t st, const void* items, uint32_t n,
                    const void* insts, const DInsn* code, const int64_t* params,
                    const int64_t* loopvals, const QDesc* qd, QAcc* acc) {
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL(k_witness2, dim3(m), dim3(256), 0, st,
                       (const W2Item*)items + off, (const DevInst*)insts, code,
                       params, loopvals, qd, acc);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

size_t w2item_size() { return sizeof(W2Item); }

int launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t n, uint32_t v) {
  if (n == 0) return 0;
  uint32_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, st, p, n, v);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_init_acc(hipStream_t st, uint32_t n, QAcc* acc) {
  if (n == 0) return 0;
  uint32_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_init_acc, dim3(g), dim3(256), 0, st, acc, n);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_finalize(hipStream_t st, uint32_t n, const QAcc* acc,
                    const QDesc* qd, const uint32_t* host_err,
                    const uint8_t* trivial, const unsigned long long* evals,
                    rd_pair_result* out) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, st, n,
                     acc, qd, host_err, trivial, evals, out);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

}  // namespace hgrd
