// Device building blocks shared by the gfx950 kernel files: expression
// interpreter, point decoding and evaluation, reductions, and the LDS
// prefix-group join.  See hgrd_kernels.hip for the method.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include "hgrd_internal.h"

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
      // both operands in int32: the product fits int64 (one 32x32 multiply)
      if ((uint64_t)a + 0x80000000ull < 0x100000000ull &&
          (uint64_t)b + 0x80000000ull < 0x100000000ull)
        return (int64_t)(int32_t)a * (int64_t)(int32_t)b;
      if (__builtin_mul_overflow(a, b, &r)) { err |= ERR_RANGE; return 0; }
      return r;
    case D_DIV:
      if (b == 0) { err |= ERR_DIVZERO; return 0; }
      // both operands in [0, 2^31): a 32-bit unsigned division
      if (((uint64_t)(a | b) >> 31) == 0) return (int64_t)((uint32_t)a / (uint32_t)b);
      if (a == INT64_MIN && b == -1) { err |= ERR_RANGE; return 0; }
      return a / b;
    case D_MOD:
      if (b == 0) { err |= ERR_DIVZERO; return 0; }
      if (((uint64_t)(a | b) >> 31) == 0) return (int64_t)((uint32_t)a % (uint32_t)b);
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
  // term tables (tab != 0), see TabHost
  const int64_t* tpool;
  int64_t tu;
  uint32_t toff[3];
  uint32_t iv_off, iv_const, tnever, tab, tpad;
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

// Point coordinates of point index `pidx`: (blin * niota + ilin) * nthr +
// tlin, or (blin * nthr + tlin) * niota + ilin when iterations go fastest
// (the block is always slowest, so block b owns [b * tpb, (b + 1) * tpb)).
struct PointIds {
  uint32_t blin, tlin, ilin;
};

__device__ __forceinline__ PointIds decode(const DevInst& I, uint32_t pidx) {
  PointIds o;
  if (I.a.iorder) {
    uint32_t rest = fdiv(pidx, I.f_niota);
    o.ilin = pidx - rest * I.a.niota;
    o.blin = fdiv(rest, I.f_nthr);
    o.tlin = rest - o.blin * I.a.nthr;
  } else {
    uint32_t rest = fdiv(pidx, I.f_nthr);
    o.tlin = pidx - rest * I.a.nthr;
    o.blin = fdiv(rest, I.f_niota);
    o.ilin = rest - o.blin * I.a.niota;
  }
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

// Table lookups only (the instance has term tables).
__device__ __forceinline__ bool point_tab(const DevInst& I, const PointIds& id,
                                          Point& pt) {
  // all lookups issued before any is tested: one memory round trip
  const int64_t v0 = I.toff[0] != kNoTab ? I.tpool[I.toff[0] + id.blin] : 0;
  const int64_t v1 = I.toff[1] != kNoTab ? I.tpool[I.toff[1] + id.tlin] : 0;
  const int64_t v2 = I.toff[2] != kNoTab ? I.tpool[I.toff[2] + id.ilin] : 0;
  const uint32_t iv =
      I.iv_off != kNoTab ? (uint32_t)I.tpool[I.iv_off + id.ilin] : I.iv_const;
  if (I.tnever || v0 == INT64_MIN || v1 == INT64_MIN || v2 == INT64_MIN) return false;
  pt.addr = I.tu + v0 + v1 + v2;
  pt.bint = iv & 0xFFFF;
  pt.wint = iv >> 16;
  return true;
}

// Guard, address and interval ids of one point: table lookups when the
// instance has term tables, else the interpreter.
__device__ __forceinline__ bool point_eval(const DevInst& I, const PointIds& id,
                                           const DInsn* __restrict__ code,
                                           const int64_t* __restrict__ params,
                                           const int64_t* __restrict__ loopvals,
                                           Point& pt, uint32_t& err) {
  if (I.tab) return point_tab(I, id, pt);
  Regs R;
  set_coords(I, id, loopvals, R);
  return eval_point(I, code, params, R, pt, err);
}

// syn() of an access at one point (section 6.5, Figures 9 and 10): bit 0
// of the result when the access has one at block scope, bit 1 at device
// scope (only operations at least that wide are seen); `val` gets its
// address.  Where both bits are set the address is the same: the operations
// seen at device scope are among those seen at block scope, and a lock's
// acquire and release hit one address.  The array never depends on the
// point (a lock needs acquire and release in one array), so the pair's
// flags say whether two syn() can match at all.
__device__ __forceinline__ uint32_t point_syn(const DevInst& I, const PointIds& id,
                                              const DInsn* __restrict__ code,
                                              const int64_t* __restrict__ params,
                                              const int64_t* __restrict__ loopvals,
                                              int64_t& val, uint32_t& err) {
  const uint32_t f = I.a.syn;
  val = 0;
  if (!(f & (kSynAcq | kSynRel))) return 0;
  Regs R;
  set_coords(I, id, loopvals, R);
  const int64_t* pr = params + I.a.params_off;
  uint32_t e = 0;
  const int64_t va = (f & kSynAcq) ? run_prog(code, I.a.acq, R, pr, 0, e) : 0;
  const int64_t vr = (f & kSynRel) ? run_prog(code, I.a.rel, R, pr, 0, e) : 0;
  if ((f & kSynAcq32) && (va < INT32_MIN || va > INT32_MAX)) e |= ERR_RANGE;
  if ((f & kSynRel32) && (vr < INT32_MIN || vr > INT32_MAX)) e |= ERR_RANGE;
  err |= e;
  uint32_t bits = 0;
  for (int s = 0; s < 2; ++s) {
    const bool A = (f & kSynAcq) && (s == 0 || (f & kSynAcqDev));
    const bool Rl = (f & kSynRel) && (s == 0 || (f & kSynRelDev));
    if (A && Rl && (f & kSynSameArr) && va == vr) {
      bits |= 1u << s;  // lock
      val = va;
    } else if ((f & kSynWrite) && Rl) {
      bits |= 1u << s;  // producer
      val = vr;
    } else if ((f & kSynRead) && A) {
      bits |= 1u << s;  // consumer
      val = va;
    }
  }
  return bits;
}

// Interval ids of a point already known to be present.
__device__ __forceinline__ void point_iv(const DevInst& I, const PointIds& id,
                                         const DInsn* __restrict__ code,
                                         const int64_t* __restrict__ params,
                                         const int64_t* __restrict__ loopvals,
                                         uint32_t& bi, uint32_t& wi) {
  if (I.tab) {
    const uint32_t iv =
        I.iv_off != kNoTab ? (uint32_t)I.tpool[I.iv_off + id.ilin] : I.iv_const;
    bi = iv & 0xFFFF;
    wi = iv >> 16;
    return;
  }
  if (I.a.bint.absent && I.a.wint.absent) {
    bi = wi = 0;
    return;
  }
  Regs R;
  set_coords(I, id, loopvals, R);
  const int64_t* pr = params + I.a.params_off;
  uint32_t e = 0;
  bi = (uint32_t)run_prog(code, I.a.bint, R, pr, 0, e) & 0xFFFF;
  wi = (uint32_t)run_prog(code, I.a.wint, R, pr, 0, e) & 0xFFFF;
}

__device__ __forceinline__ void load_inst(DevInst& D,
                                          const DevInst* __restrict__ insts,
                                          uint32_t k) {
  k = __builtin_amdgcn_readfirstlane(k);
  D = insts[k];
}

// ---------------------------------------------------------------------------
// Exact unit test: two access instances of one tuple share no address when
// their proven address ranges do not meet, or when their residues differ:
// addresses of a are u_a + k G_a, of b u_b + k G_b, and a common one needs
// gcd(G_a, G_b) | u_a - u_b.  False whenever nothing is known.

__device__ __forceinline__ u64 gcd_u64(u64 a, u64 b) {
  while (b) {
    const u64 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// x mod g in [0, g) for any int64 x and g > 0 (no signed overflow).
__device__ __forceinline__ u64 mod_u64(long long x, u64 g) {
  if (x >= 0) return (u64)x % g;
  const u64 m = (u64)(-(x + 1));  // x = -(m + 1)
  return g - 1 - m % g;
}

__device__ __forceinline__ bool facts_apart(const IFact& a, const IFact& b) {
  if (!a.on || !b.on) return false;
  if (a.hi < b.lo || b.hi < a.lo) return true;
  const u64 g = gcd_u64(a.G, b.G);
  if (g == 0) return a.u != b.u;
  return mod_u64(a.u, g) != mod_u64(b.u, g);
}

// A (pair, tuple) unit holds no conflict when its two accesses share no
// address (two different instances, facts_apart), or when both compute
// their address with one expression (QDesc flag bit 2; a self pair always
// does) that sends different threads to different addresses: a common
// address then belongs to one thread only.
__device__ __forceinline__ bool unit_free(const IFact& a, const IFact& b, uint32_t qflags,
                                          bool distinct) {
  if ((qflags & 4) && a.on && b.on && a.inj && b.inj) return true;
  return distinct && facts_apart(a, b);
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
// in tli of synchronised joins: the point has a syn() at block / device scope
constexpr uint32_t kSynBlkBit = 1u << 10, kSynDevBit = 1u << 11;
constexpr uint32_t kMultiThread = 1u << 31;  // in a group's count

template <int CAP, int TBL>
struct JoinLds {
  u64 addr[CAP];
  uint32_t blin[CAP];
  uint32_t tli[CAP];  // ilin << 16 | side << 15 | inactive << 14 | tlin
  uint32_t bw[CAP];   // bint << 16 | wint
  uint16_t w[CAP];    // warp of the analysed program
  uint32_t key[CAP];  // a record's group key at the level being joined
  int32_t part[CAP];
  uint32_t owner[TBL];
  uint32_t cnt[TBL];
  u64 red[8];
  uint32_t n;
  uint32_t err;
  uint32_t vote[3];          // block-wide votes (see block_vote)
  uint32_t bn[kMaxRunBuckets];  // record counts of the buckets to join
  uint32_t bl[kMaxRunBuckets];  // their offsets in the run
  uint32_t nbl;                 // how many
};

// Block-wide OR with one barrier (the library's __syncthreads_or costs
// three): waves holding a true lane store `tag` into an LDS word, then all
// compare it after the barrier.  The caller keeps every earlier vote on
// the same word behind a barrier and never repeats a tag while the word
// still holds it.
__device__ __forceinline__ bool block_vote(bool v, uint32_t* word, uint32_t tag) {
  if (__ballot(v) != 0 && (threadIdx.x & 63) == 0) *word = tag;
  __syncthreads();
  return *reinterpret_cast<volatile uint32_t*>(word) == tag;
}

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

// Joins the S.n records in LDS.  Leaves the class counts in S.red[0..2] and
// the smallest p key with a partner in S.red[3] (kNoKey: none); the caller
// sets S.red to (0, 0, 0, kNoKey) and synchronises before the call.  All NT
// threads of the block must call it; it ends with a barrier.
//
// Level L groups refine level L - 1 groups, so after the first level a
// record's group at L is (its group at the previous level, the one field
// that L adds): the previous group's table slot and that field make a
// 32-bit key (the block, 32 bits itself, is compared beside the key),
// written during the previous level's count pass.  An insert reads its
// slot, then claims it with one compare-and-swap or compares the owner's
// key and adds its count; the first level compares the fields themselves.
//
// l0ext: the records hold whole (address, block) groups but not whole
// address groups; level 0 (S_0, the address-only sums) is counted elsewhere
// and the caller has put each side-a record's level-0 partner count in
// S.part.  Then S.red[0] gets -S_1 (inter = S_0 - S_1 modulo 2^64) and no
// record is filtered out.
//
// gmult = G > 1: the records are block 0 of a global array's G blocks that
// hold the same points up to the block (no block term in either access):
// an address group of block 0 stands for G such groups, so S_0 is G times
// block 0's (S.red[0] = G S_0 - S_1; the caller multiplies every count by G
// again, giving G^2 S_0 - G S_1), and a record's address-level partners
// include the other blocks' copies.  Partner counts only decide "any
// partner": the address level adds 2 nj instead of G nj (the inter share
// (G - 1) nj and nj have the same sign), and no record is filtered out
// (a record alone in block 0 still pairs with its copies).
__device__ __forceinline__ uint32_t key_slot(uint32_t k, uint32_t b, uint32_t tbl) {
  uint32_t x = k * 0x9E3779B1u ^ b * 0x85EBCA77u;
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  return x & (tbl - 1);
}

// SYN (pairs with acquire/release, section 6.5): skey[r] holds record r's
// synchronisation address and tli bits 10/11 whether it has a syn() at
// block / device scope.  After each conflict level L the same groups are
// split by the synchronisation address over the active records with a
// syn() at the level's scope (device for the inter-block levels, block for
// the others), when the pair's flags (QDesc bits 3/4) say two of them can
// match: those sums T_L are the synchronised pairs, subtracted from the
// class counts (inter = S_0 - S_1 - (T_0 - T_1), ...) and, with the
// opposite sign, from the partner counts.  The key of a record at T_L is
// its S_L slot and its synchronisation address.
template <uint32_t NT, int CAP, int TBL, bool SYN = false>
__device__ void lds_join(JoinLds<CAP, TBL>& S, const QDesc& qd, uint32_t sigma,
                         bool l0ext = false, uint32_t gmult = 1,
                         const u64* __restrict__ skey = nullptr) {
  constexpr int RPT = (CAP + NT - 1) / NT;
  const uint32_t tid = threadIdx.x;
  const uint32_t n = S.n;
  const uint32_t mask = qd.mask;
  const bool self = qd.self != 0;
  uint32_t used = 0;
  if (mask & 1) used |= l0ext ? 0x02 : 0x03;
  if (mask & 2) used |= 0x0C;
  if (mask & 4) used |= 0x30;
  if (used == 0 || n == 0) return;
  // filter level (none: 99)
  const int f = l0ext || (gmult > 1 && (used & 1)) ? 99 : __ffs(used) - 1;
  // a level whose groups equal the previous level's (constant, equal
  // interval ids) is not recomputed: its sums and counts are the previous
  // level's
  const bool same2 = (qd.flags & 1) && ((used >> 1) & 1) && ((used >> 2) & 1);
  const bool same4 = (qd.flags & 2) && ((used >> 3) & 1) && ((used >> 4) & 1);
  u64 Sl[6] = {0, 0, 0, 0, 0, 0};
  // The table holds one 64-bit word per slot: side-a (self: every) count in
  // bits 0-15, side-b count in 16-31, owner record in 32-43, generation in
  // 44-47, the two-thread mark in bit 48.  Every level (and synchronisation
  // pass) joins with a generation of its own, so a word of an older one is
  // an empty slot: the table is cleared once per call, not per level, and a
  // level's keys are written during the previous level's count pass.
  static_assert(CAP <= 4096, "owner field");
  using JL = JoinLds<CAP, TBL>;
  static_assert(offsetof(JL, owner) % 8 == 0 && offsetof(JL, cnt) == offsetof(JL, owner) + 4 * TBL,
                "owner and cnt form TBL aligned 64-bit words");
  u64* slot = reinterpret_cast<u64*>(S.owner);  // owner and cnt: TBL words
  uint32_t gen = 0;
  // per record of this thread: tli (kInactive also past the end) and the
  // table slot of its group at the last computed level
  uint32_t tl[RPT], gid[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const uint32_t r = tid + (uint32_t)j * NT;
    tl[j] = r < n ? S.tli[r] : kInactive;
    gid[j] = 0;
    if (!l0ext && r < n) S.part[r] = 0;
  }
  for (uint32_t k = tid; k < TBL; k += NT) slot[k] = 0;
  if (tid == 0) S.vote[2] = 0;  // the filter level's vote (after a barrier)
  // levels computed (not skipped as equal to the previous one) and whose
  // key is the previous computed level's slot and the one field they add
  // (a skipped level between adds a field that is one constant for every
  // record)
  bool comp[6], incl[6];
  {
    int P = -1;
    for (int L = 0; L < 6; ++L) {
      comp[L] = ((used >> L) & 1) && !((L == 2 && same2) || (L == 4 && same4));
      incl[L] = comp[L] && P >= 0 &&
                (L == P + 1 || (L == 3 && P == 1 && same2) || (L == 5 && P == 3 && same4));
      if (comp[L]) P = L;
    }
  }
  // one record's field at level L (the part its key adds to the previous
  // level's slot)
  auto field = [&](int L, uint32_t r, uint32_t t) -> uint32_t {
    if (L == 2) return S.bw[r] >> 16;
    if (L == 3) return S.w[r];
    if (L == 4) return S.bw[r] & 0xFFFF;
    if (L == 5) return t & 0x3FF;
    return 0;  // L == 1: the block is compared beside the key
  };
  // inserts record r with key test eq(owner) from slot h on; returns the
  // group's slot (the first record of a group claims an empty slot with its
  // count, the others add theirs)
  auto insert = [&](uint32_t h, uint32_t r, u64 add, auto&& eq) -> uint32_t {
    const u64 mine = ((u64)gen << 44) | ((u64)r << 32) | add;
    u64 o = slot[h];
    for (;;) {
      if (((uint32_t)(o >> 44) & 0xF) != gen) {
        const u64 prev = atomicCAS(&slot[h], o, mine);
        if (prev == o) return h;
        o = prev;  // claimed meanwhile (a claim is final within a level)
        continue;
      }
      if (eq((uint32_t)(o >> 32) & 0xFFF)) {
        atomicAdd(&slot[h], add);
        return h;
      }
      h = (h + 1) & (TBL - 1);
      o = slot[h];
    }
  };
  __syncthreads();
  u64 Tl[6] = {0, 0, 0, 0, 0, 0};
  // synchronised pairs of level L (SYN): groups (S_L slot, sync address);
  // a record's S_L slot is its key >> 16 (written in that level's count
  // pass)
  auto tpass = [&](int L) {
    const uint32_t cls = L < 2 ? 1u : (L < 4 ? 2u : 4u);
    const uint32_t need = L < 2 ? (qd.flags & 16u) : (qd.flags & 8u);
    const uint32_t bit = L < 2 ? kSynDevBit : kSynBlkBit;
    if (!(cls & mask) || !need) return;
    ++gen;
    uint32_t tg[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const uint32_t r = tid + (uint32_t)j * NT;
      tg[j] = kEmpty;
      if ((tl[j] & kInactive) || !(tl[j] & bit)) continue;
      const u64 v = skey[r];
      const uint32_t g = gid[j];
      tg[j] = insert(key_slot(g, (uint32_t)v ^ (uint32_t)(v >> 32), TBL), r,
                     (self || !(tl[j] & kSide)) ? 1ull : 0x10000ull,
                     [&](uint32_t o) { return (S.key[o] >> 16) == g && skey[o] == v; });
    }
    __syncthreads();
    const int sign = (L & 1) ? -1 : 1;
    u64 t = 0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const uint32_t r = tid + (uint32_t)j * NT;
      if (tg[j] == kEmpty) continue;
      const uint32_t c = (uint32_t)slot[tg[j]];
      if (!self && (tl[j] & kSide)) continue;
      const uint32_t nj = self ? (c & 0xFFFF) : (c >> 16);
      t += nj;
      S.part[r] -= sign * (int32_t)nj;
    }
    Tl[L] = t;
    __syncthreads();
  };
  bool any = true;
  for (int L = 0; L < 6; ++L) {
    if (!((used >> L) & 1)) continue;
    if (!comp[L]) {
      Sl[L] = Sl[L - 1];
      // the level's groups are the previous level's: its slots stand
      if (SYN) tpass(L);
      continue;
    }
    const bool twin = (L == 1 && same2) || (L == 3 && same4);
    const bool inc = incl[L];
    ++gen;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const uint32_t r = tid + (uint32_t)j * NT;
      if (tl[j] & kInactive) continue;
      const u64 add = (self || !(tl[j] & kSide)) ? 1ull : 0x10000ull;
      if (inc) {
        const uint32_t kr = S.key[r];
        const uint32_t kb = L == 1 ? S.blin[r] : 0u;
        gid[j] = insert(key_slot(kr, kb, TBL), r, add, [&](uint32_t o) {
          return S.key[o] == kr && (L != 1 || S.blin[o] == kb);
        });
      } else {
        gid[j] = insert(level_hash(L, S.addr[r], S.blin[r], S.bw[r], S.w[r], tl[j] & 0x3FF) &
                            (TBL - 1),
                        r, add, [&](uint32_t o) { return level_eq(S, L, o, r); });
      }
    }
    __syncthreads();
    if (L == f) {
      // groups holding records of two different threads are marked (bit 48
      // of the word); the others pair only a thread with itself, which is no
      // conflict at any level
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const uint32_t r = tid + (uint32_t)j * NT;
        if (tl[j] & kInactive) continue;
        const uint32_t o = (uint32_t)(slot[gid[j]] >> 32) & 0xFFF;
        if (o != r && (S.blin[o] != S.blin[r] || ((S.tli[o] ^ tl[j]) & 0x3FF)))
          atomicOr(&slot[gid[j]], 1ull << 48);
      }
      __syncthreads();
    }
    // the next computed level, whose keys this count pass writes
    int nx = L + 1;
    while (nx < 6 && !comp[nx]) ++nx;
    const bool nx_inc = nx < 6 && incl[nx];
    const int sign = (L & 1) ? -1 : 1;
    const uint32_t cls = L < 2 ? 1u : (L < 4 ? 2u : 4u);
    bool any_local = false;
    u64 s = 0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const uint32_t r = tid + (uint32_t)j * NT;
      if (tl[j] & kInactive) continue;
      const u64 cw = slot[gid[j]];
      const uint32_t c = (uint32_t)cw;
      const bool sb = (tl[j] & kSide) != 0;
      // ordered pairs of the group: a self pair counts every record with
      // each of its group (itself included), a pair of two accesses each
      // side-a record with the group's side-b records
      if (self) s += c & 0xFFFF;
      else if (!sb) s += c >> 16;
      if (L == f) {
        // a record can conflict only in a group with records of the other
        // side (self pair: two records) and of two different threads; the
        // others' pairs (none, or only a thread with itself) count zero in
        // every class, so their share of S_f goes and they leave
        const bool cand = ((cw >> 48) & 1) &&
                          (self ? ((c & 0xFFFF) >= 2) : ((c & 0xFFFF) && (c >> 16)));
        if (!cand) {
          tl[j] |= kInactive;
          S.tli[r] = tl[j];
          if (self) s -= c & 0xFFFF;
          else if (!sb) s -= c >> 16;
          continue;
        }
        any_local = true;
      }
      // key of the next level (and S_L slot of the synchronisation pass)
      S.key[r] = (gid[j] << 16) | (nx_inc ? field(nx, r, tl[j]) : 0u);
      if (!self && sb) continue;
      const int32_t nj = (int32_t)(self ? (c & 0xFFFF) : (c >> 16));
      if (cls & mask) S.part[r] += sign * nj * (L == 0 && gmult > 1 ? 2 : 1);
      if (twin && ((cls << 1) & mask)) S.part[r] -= sign * nj;  // level L + 1
    }
    Sl[L] = L == 0 ? s * gmult : s;
    if (L == f) {
      any = block_vote(any_local, &S.vote[2], 1u);
      if (!any) break;
    } else {
      __syncthreads();
    }
    if (SYN) tpass(L);
  }
  if (!any) return;
  // class counts: reduce S_L over the block (minus synchronised pairs)
  u64 c0 = (mask & 1) ? (Sl[0] - Sl[1]) - (Tl[0] - Tl[1]) : 0;  // l0ext: Sl[0] = 0, so -S_1
  u64 c1 = (mask & 2) ? (Sl[2] - Sl[3]) - (Tl[2] - Tl[3]) : 0;
  u64 c2 = (mask & 4) ? (Sl[4] - Sl[5]) - (Tl[4] - Tl[5]) : 0;
  u64 best = kNoKey;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const uint32_t r = tid + (uint32_t)j * NT;
    if ((tl[j] & kInactive) || (!self && (tl[j] & kSide))) continue;
    if (S.part[r] > 0) {
      u64 k = pkey(sigma, S.blin[r], tl[j] & 0x3FF, tl[j] >> 16);
      best = k < best ? k : best;
    }
  }
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
}

// Address-level pre-filter by signatures: a conflict needs equal addresses
// whatever the classes, so a record whose address no record of the other
// side (for a self pair: no other record) holds can take no part in the
// join.  Each side sets two bits per record, chosen by two hashes of the
// address, in a bitmap of 32 * TBL bits (S.owner for side a, S.cnt for
// side b; for a self pair S.owner marks addresses seen once and S.cnt
// seen twice).  A record stays active when the other bitmap has both its
// bits: no record with a partner is ever dropped, and the few kept by
// colliding hashes are dropped exactly at the join's first level.
template <int TBL>
__device__ __forceinline__ void sig_index(u64 a, uint32_t salt, uint32_t& i1,
                                          uint32_t& i2) {
  constexpr uint32_t lgb = 5 + (TBL >= 8192 ? 13 : TBL >= 4096 ? 12 : 11);
  static_assert(TBL == 2048 || TBL == 4096 || TBL == 8192, "signature bitmap size");
  const uint32_t x = (uint32_t)a ^ ((uint32_t)(a >> 32) * 0x85EBCA6Bu) ^
                     (salt * 0x27D4EB2Fu);
  i1 = (x * 0x9E3779B1u) >> (32 - lgb);
  i2 = ((x ^ (x >> 15)) * 0xC2B2AE35u) >> (32 - lgb);
}

template <uint32_t NT, int CAP, int TBL>
__device__ __forceinline__ void sig_clear(JoinLds<CAP, TBL>& S) {
  uint4* o = reinterpret_cast<uint4*>(S.owner);
  uint4* c = reinterpret_cast<uint4*>(S.cnt);
#pragma unroll
  for (uint32_t k = threadIdx.x; k < TBL / 4; k += NT) {
    o[k] = make_uint4(0, 0, 0, 0);
    c[k] = make_uint4(0, 0, 0, 0);
  }
}

template <int CAP, int TBL>
__device__ __forceinline__ void sig_insert(JoinLds<CAP, TBL>& S, uint32_t i1,
                                           uint32_t i2, bool side, bool self) {
  const uint32_t m1 = 1u << (i1 & 31), m2 = 1u << (i2 & 31);
  if (self) {
    if (atomicOr(&S.owner[i1 >> 5], m1) & m1) atomicOr(&S.cnt[i1 >> 5], m1);
    if (atomicOr(&S.owner[i2 >> 5], m2) & m2) atomicOr(&S.cnt[i2 >> 5], m2);
  } else {
    uint32_t* t = side ? S.cnt : S.owner;
    atomicOr(&t[i1 >> 5], m1);
    atomicOr(&t[i2 >> 5], m2);
  }
}

template <int CAP, int TBL>
__device__ __forceinline__ bool sig_test(const JoinLds<CAP, TBL>& S, uint32_t i1,
                                         uint32_t i2, bool side, bool self) {
  const uint32_t* t = (self || !side) ? S.cnt : S.owner;
  return ((t[i1 >> 5] >> (i1 & 31)) & (t[i2 >> 5] >> (i2 & 31)) & 1u) != 0;
}

// Adds a join's results (S.red) to a query's accumulators (thread 0), the
// counts taken `mult` times (modulo 2^64, as the sum of mult copies).
template <int CAP, int TBL>
__device__ __forceinline__ void commit_join(const JoinLds<CAP, TBL>& S,
                                            QAcc* __restrict__ acc, u64 mult = 1) {
  if (threadIdx.x == 0) {
    if (S.red[0]) atomicAdd(&acc->cnt[0], S.red[0] * mult);
    if (S.red[1]) atomicAdd(&acc->cnt[1], S.red[1] * mult);
    if (S.red[2]) atomicAdd(&acc->cnt[2], S.red[2] * mult);
    if (S.red[3] != kNoKey) atomicMin(&acc->pmin, S.red[3]);
  }
}

template <int CAP, int TBL>
__device__ __forceinline__ void init_red(JoinLds<CAP, TBL>& S) {
  if (threadIdx.x < 8) S.red[threadIdx.x] = (threadIdx.x == 3 || threadIdx.x == 4) ? kNoKey : 0;
  if (threadIdx.x < 3) S.vote[threadIdx.x] = 0;
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
  base = (uint32_t)__builtin_amdgcn_readlane((int)base, (int)leader);
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

}  // namespace hgrd
