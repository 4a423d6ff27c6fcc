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
#include <hip/hip_ext.h>
#include <stdint.h>
#include "hgrd_internal.h"
#include "hgrd_launch.h"
#include "hgrd_device.h"
#include <string.h>

namespace hgrd {

using u64 = unsigned long long;

// ---------------------------------------------------------------------------
// Small items: generate both sides straight into LDS and join.

template <int CAP, int TBL>
__device__ __forceinline__ void small_item(JoinLds<CAP, TBL>& S, const SItem& it,
                                           const DevInst* __restrict__ insts,
                                           const DInsn* __restrict__ code,
                                           const int64_t* __restrict__ params,
                                           const int64_t* __restrict__ loopvals,
                                           const QDesc* __restrict__ qd,
                                           QAcc* __restrict__ acc,
                                           const uint32_t* __restrict__ done,
                                           const IFact* __restrict__ facts) {
  if (done[it.q]) return;
  const QDesc q = qd[it.q];
  // a unit proven free of conflicts: nothing to join
  if (facts && unit_free(facts[it.inst_i], facts[it.inst_j], q.flags,
                         !q.self && it.inst_i != it.inst_j))
    return;
  if (threadIdx.x == 0) {
    S.n = 0;
    S.err = 0;
  }
  init_red(S);
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
        valid = point_eval(I, id, code, params, loopvals, pt, err);
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
  lds_join<256>(S, q, it.sigma, false, it.gsym && it.mult > 1 ? it.mult : 1u);
  commit_join(S, &acc[it.q], it.mult > 1 ? (u64)it.mult : 1ull);
}

// One workgroup per item.
template <int CAP, int TBL>
__global__ void __launch_bounds__(256)
k_small_join(const SItem* __restrict__ items, const DevInst* __restrict__ insts,
             const DInsn* __restrict__ code, const int64_t* __restrict__ params,
             const int64_t* __restrict__ loopvals, const QDesc* __restrict__ qd,
             QAcc* __restrict__ acc, const uint32_t* __restrict__ done,
             const IFact* __restrict__ facts) {
  extern __shared__ __align__(16) unsigned char smem[];
  JoinLds<CAP, TBL>& S = *reinterpret_cast<JoinLds<CAP, TBL>*>(smem);
  small_item(S, items[blockIdx.x], insts, code, params, loopvals, qd, acc, done, facts);
}

// Persistent form: a grid sized to the machine pops items (largest first,
// as the host orders them) from a work counter until none is left, a few
// at a time (one counter round trip per kSmallPop items).
constexpr uint32_t kSmallPop = 4;
template <int CAP, int TBL>
__global__ void __launch_bounds__(256)
k_small_persist(const SItem* __restrict__ items, uint32_t n,
                uint32_t* __restrict__ cursor, const DevInst* __restrict__ insts,
                const DInsn* __restrict__ code, const int64_t* __restrict__ params,
                const int64_t* __restrict__ loopvals, const QDesc* __restrict__ qd,
                QAcc* __restrict__ acc, const uint32_t* __restrict__ done,
                const IFact* __restrict__ facts) {
  extern __shared__ __align__(16) unsigned char smem[];
  JoinLds<CAP, TBL>& S = *reinterpret_cast<JoinLds<CAP, TBL>*>(smem);
  __shared__ uint32_t cur;
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(cursor, kSmallPop);
    __syncthreads();
    const uint32_t k0 = cur;
    __syncthreads();
    if (k0 >= n) break;
    const uint32_t k1 = min(n, k0 + kSmallPop);
    for (uint32_t k = k0; k < k1; ++k) {
      small_item(S, items[k], insts, code, params, loopvals, qd, acc, done, facts);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Kernel: fill term tables.  One workgroup per chunk of one table; every
// entry evaluates the group's programs at that group index (the other
// coordinates are zero and unused).  The host proved these programs free of
// errors over the whole box.
__global__ void __launch_bounds__(256)
k_tabulate(const Chunk* __restrict__ chunks, const TabJob* __restrict__ jobs,
           const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
           const int64_t* __restrict__ params,
           const int64_t* __restrict__ loopvals, int64_t* __restrict__ pool) {
  const Chunk ch = chunks[blockIdx.x];
  const TabJob J = jobs[ch.item];
  DevInst I;
  load_inst(I, insts, J.inst);
  const int64_t* pr = params + I.a.params_off;
  for (uint32_t e = ch.p0 + threadIdx.x; e < ch.p1; e += blockDim.x) {
    PointIds id;
    id.blin = J.group == 0 ? e : 0;
    id.tlin = J.group == 1 ? e : 0;
    id.ilin = J.group >= 2 ? e : 0;
    Regs R;
    set_coords(I, id, loopvals, R);
    uint32_t err = 0;
    int64_t v;
    if (J.group == 3) {
      const int64_t b = run_prog(code, I.a.bint, R, pr, 0, err);
      const int64_t w = run_prog(code, I.a.wint, R, pr, 0, err);
      v = b | (w << 16);
    } else {
      const bool g = J.guard.absent || run_prog(code, J.guard, R, pr, 1, err) != 0;
      v = g ? run_prog(code, J.val, R, pr, 0, err) : INT64_MIN;
    }
    pool[J.out_off + e] = v;
  }
}

// ---------------------------------------------------------------------------
// Kernel: generate points and scatter (key, point id) records into
// fixed-capacity HBM buckets chosen by a hash of the address (and of the
// block for shared arrays, whose memory is per block).

// 64-bit finalizer of MurmurHash3 (Austin Appleby's public-domain fmix64:
// xor-shift 33, multiply, xor-shift 33, multiply, xor-shift 33).
__device__ __forceinline__ u64 mix64(u64 x) {
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDull;
  x ^= x >> 33;
  x *= 0xC4CEB9FE1A85EC53ull;
  x ^= x >> 33;
  return x;
}

// Bucket of a record.  mode 1: the dense key modulo the prime bucket count
// (Lemire's 32-bit fastmod: one 64-bit multiply and a multiply-high);
// mode 0: a hash of (address >> shift), and of the block for shared arrays
// and split items.
__device__ __forceinline__ uint32_t bucket_of(const HItem& h, int64_t addr,
                                              uint32_t blin) {
  if (h.mode) {
    const uint32_t k = (uint32_t)((u64)(addr - h.lo) >> h.shift) + blin * h.kb;
    return (uint32_t)__umul64hi(h.fm * (u64)k, (u64)h.nbuckets);
  }
  u64 hk = (u64)(addr >> h.shift);
  if (h.shared == 1 || h.shared == 3) hk ^= (u64)(blin + 1) * 0x9E3779B97F4A7C15ull;
  return (uint32_t)__umul64hi(mix64(hk), (u64)h.nbuckets);
}

// One workgroup takes one chunk of one side: it generates the points,
// merges the chunk's records per bucket in LDS (open addressing on the
// bucket id; a run of lanes holding one bucket claims the slot and its
// ranks with one LDS atomic), reserves each bucket's run with one global
// atomic (all of a tile's reservations in flight at once), then writes the
// runs.  Points follow
// address order closely (see iorder) and buckets keep blocks of 2^shift
// addresses together, so a chunk touches few buckets and its writes are
// runs of whole lines.  TAB: every instance of the launch has term tables
// (no interpreter code, fewer registers, more waves in flight).
constexpr uint32_t kScatterThreads = 512;  // partition workgroup size
constexpr uint32_t kScatterPts = 2048;     // points per LDS tile
constexpr uint32_t kScatterSlots = 4096;
constexpr uint32_t kByteSlots = 64;     // spread of the record-byte counters
template <bool TAB>
__global__ void __launch_bounds__(kScatterThreads)
k_scatter(const Chunk* __restrict__ chunks, const HItem* __restrict__ hitems,
          const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
          const int64_t* __restrict__ params,
          const int64_t* __restrict__ loopvals, QAcc* __restrict__ acc,
          unsigned char* __restrict__ recs, uint32_t* __restrict__ cursor,
          uint32_t* __restrict__ ovf, uint32_t capb, const uint32_t* __restrict__ done,
          u64* __restrict__ nbytes) {
  __shared__ uint32_t skey[kScatterSlots];  // bucket + 1, 0 = empty
  __shared__ uint32_t scnt[kScatterSlots];  // count, then the run's base
  __shared__ uint16_t used[kScatterPts];    // slots taken in this tile
  __shared__ uint32_t nused;
  __shared__ u64 sbytes;
  const Chunk ch = chunks[blockIdx.x];
  const HItem h = hitems[ch.item];
  if (done[h.q] || ovf[ch.item] == kApart) return;
  DevInst I;
  load_inst(I, insts, ch.side ? h.inst_j : h.inst_i);
  uint32_t err = 0;
  const bool store = h.nbuckets != 0;  // 0: error scan only
  const uint32_t rs = h.is32 ? 8 : 16;
  constexpr int kPer = kScatterPts / kScatterThreads;
  for (uint32_t k = threadIdx.x; k < kScatterSlots; k += kScatterThreads) {
    skey[k] = 0;
    scnt[k] = 0;
  }
  if (threadIdx.x == 0) {
    nused = 0;
    sbytes = 0;
  }
  for (uint32_t t0 = ch.p0; t0 < ch.p1; t0 += kScatterPts) {
    __syncthreads();
    int64_t ad[kPer];
    uint32_t pv[kPer], sl[kPer], rk[kPer], bk[kPer];
    if constexpr (TAB) {
      // every table lookup of the tile's points in flight before any is
      // used: one memory round trip per tile instead of one per point
      int64_t v0[kPer], v1[kPer], v2[kPer];
      uint32_t bl[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const uint32_t pidx = t0 + (uint32_t)j * kScatterThreads + threadIdx.x;
        const PointIds id = decode(I, pidx < ch.p1 ? pidx : ch.p0);
        bl[j] = id.blin;
        v0[j] = I.toff[0] != kNoTab ? I.tpool[I.toff[0] + id.blin] : 0;
        v1[j] = I.toff[1] != kNoTab ? I.tpool[I.toff[1] + id.tlin] : 0;
        v2[j] = I.toff[2] != kNoTab ? I.tpool[I.toff[2] + id.ilin] : 0;
      }
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const uint32_t pidx = t0 + (uint32_t)j * kScatterThreads + threadIdx.x;
        sl[j] = kScatterSlots;
        bk[j] = 0xFFFFFFFFu;
        const bool ok = store && pidx < ch.p1 && !I.tnever && v0[j] != INT64_MIN &&
                        v1[j] != INT64_MIN && v2[j] != INT64_MIN;
        ad[j] = I.tu + v0[j] + v1[j] + v2[j];
        pv[j] = (ch.side << 31) | pidx;
        if (ok) bk[j] = bucket_of(h, ad[j], bl[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        sl[j] = kScatterSlots;
        bk[j] = 0xFFFFFFFFu;  // no record
        const uint32_t pidx = t0 + (uint32_t)j * kScatterThreads + threadIdx.x;
        if (pidx >= ch.p1) continue;
        const PointIds id = decode(I, pidx);
        Point pt;
        const bool ok = point_eval(I, id, code, params, loopvals, pt, err);
        if (!ok || !store) continue;
        ad[j] = pt.addr;
        pv[j] = (ch.side << 31) | pidx;
        bk[j] = bucket_of(h, pt.addr, id.blin);
      }
    }
    // claim LDS slots and ranks by runs: the lanes of a wave that hold one
    // bucket in a row (consecutive points of a dense-map item) form a run;
    // the run's first lane claims the slot and the run's length at once,
    // the others take slot and base from it and add their offset in the run
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint32_t b = bk[j];
      const bool v = b != 0xFFFFFFFFu;
      const uint32_t bp = __shfl_up(b, 1, 64);
      const bool head = v && (lane == 0 || bp != b);
      const u64 H = __ballot(head);
      const u64 V = __ballot(v);
      if (!V) continue;
      uint32_t s = 0, base = 0;
      if (head) {
        const u64 above = lane == 63 ? 0ull : (~0ull << (lane + 1));
        const u64 stop = (H | ~V) & above;
        const uint32_t end = stop ? (uint32_t)__ffsll((long long)stop) - 1 : 64u;
        s = (b * 0x9E3779B1u) >> 20;  // 12 bits: kScatterSlots
        for (;;) {
          const uint32_t k = atomicCAS(&skey[s], 0u, b + 1);
          if (k == 0) used[atomicAdd(&nused, 1u)] = (uint16_t)s;
          if (k == 0 || k == b + 1) break;
          s = (s + 1) & (kScatterSlots - 1);
        }
        base = atomicAdd(&scnt[s], end - lane);
      }
      const u64 upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
      const uint32_t hl = 63u - (uint32_t)__clzll((long long)(H & upto));
      const uint32_t hs = (uint32_t)__shfl((int)s, (int)hl, 64);
      const uint32_t hb = (uint32_t)__shfl((int)base, (int)hl, 64);
      if (v) {
        sl[j] = hs;
        rk[j] = hb + lane - hl;
      }
    }
    __syncthreads();
    // one reservation per bucket present in the tile; scnt becomes the base
    const uint32_t nu = nused;
    u64 written = 0;
    for (uint32_t u = threadIdx.x; u < nu; u += kScatterThreads) {
      const uint32_t k = used[u];
      const uint32_t n = scnt[k];
      const uint32_t base = atomicAdd(&cursor[h.bucket0 + skey[k] - 1], n);
      if (base + n > capb) atomicMax(&ovf[ch.item], base + n);  // largest load
      const uint32_t kept = base >= capb ? 0 : (base + n > capb ? capb - base : n);
      written += (u64)kept * rs;
      scnt[k] = base;
    }
    written = wave_sum(written);
    if ((threadIdx.x & 63) == 0 && written) atomicAdd(&sbytes, written);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      if (sl[j] == kScatterSlots) continue;
      const uint32_t pos = scnt[sl[j]] + rk[j];
      if (pos >= capb) continue;
      const u64 slot = (u64)(skey[sl[j]] - 1) * capb + pos;
      if (h.is32) {
        reinterpret_cast<u64*>(recs + h.rec_off)[slot] =
            (u64)(uint32_t)(int32_t)ad[j] | ((u64)pv[j] << 32);
      } else {
        reinterpret_cast<ulonglong2*>(recs + h.rec_off)[slot] =
            make_ulonglong2((u64)ad[j], (u64)pv[j]);
      }
    }
    __syncthreads();
    // clear the slots this tile used
    for (uint32_t u = threadIdx.x; u < nu; u += kScatterThreads) {
      skey[used[u]] = 0;
      scnt[used[u]] = 0;
    }
    if (threadIdx.x == 0) nused = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0 && sbytes) atomicAdd(&nbytes[blockIdx.x & (kByteSlots - 1)], sbytes);
  if (!TAB) {
    err = wave_or(err);
    if ((threadIdx.x & 63) == 0 && err) atomicOr(&acc[h.q].err, err);
  }
}

// ---------------------------------------------------------------------------
// Address-count tables (level 0 of split items): open addressing on the
// 64-bit address with INT64_MIN as the empty marker; that address itself
// has a slot of its own after the table.

__device__ __forceinline__ u64 l0_hash(long long a) {
  return mix64((u64)a * 0x9E3779B97F4A7C15ull);
}

__device__ __forceinline__ u64 l0_lookup(const u64* __restrict__ keys,
                                         const u64* __restrict__ cnt, u64 off,
                                         uint32_t mask, long long a, bool self) {
  u64 slot;
  if ((u64)a == kL0Empty) {
    slot = off + mask + 1;
  } else {
    u64 h = l0_hash(a) & mask;
    for (;;) {
      u64 k = keys[off + h];
      if (k == (u64)a) break;
      if (k == kL0Empty) return 0;
      h = (h + 1) & mask;
    }
    slot = off + h;
  }
  u64 c = cnt[slot];
  return self ? c : (c >> 32);
}

// Level 0 of split items: every point is counted into its item's
// address-count table.  Each workgroup first merges 1024 points at a time
// in LDS by address, so a hot address costs one global atomic per
// workgroup step.  Each item's S_0 is summed in s0[item].
__global__ void __launch_bounds__(256)
k_level0(const Chunk* __restrict__ chunks, const L0Item* __restrict__ items,
         const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
         const int64_t* __restrict__ params,
         const int64_t* __restrict__ loopvals, u64* __restrict__ keys,
         u64* __restrict__ cnt, u64* __restrict__ s0) {
  constexpr int kT = 2048;
  __shared__ u64 lkey[kT + 1];
  __shared__ uint32_t lcnt[kT + 1];
  __shared__ u64 lsum;
  const Chunk ch = chunks[blockIdx.x];
  const L0Item it = items[ch.item];
  DevInst I;
  load_inst(I, insts, ch.side ? it.inst_j : it.inst_i);
  const uint32_t inc = (it.self || !ch.side) ? 1u : 0x10000u;
  if (threadIdx.x == 0) lsum = 0;
  u64 s = 0;
  uint32_t err = 0;
  for (uint32_t t0 = ch.p0; t0 < ch.p1; t0 += 1024) {
    for (uint32_t k = threadIdx.x; k <= kT; k += blockDim.x) {
      lkey[k] = kL0Empty;
      lcnt[k] = 0;
    }
    __syncthreads();
    for (uint32_t j = 0; j < 4; ++j) {
      uint32_t pidx = t0 + j * 256 + threadIdx.x;
      if (pidx >= ch.p1) break;
      PointIds id = decode(I, pidx);
      Point pt;
      if (!point_eval(I, id, code, params, loopvals, pt, err)) continue;
      uint32_t h;
      if ((u64)pt.addr == kL0Empty) {
        h = kT;
      } else {
        h = (uint32_t)l0_hash(pt.addr) & (kT - 1);
        for (;;) {
          u64 k = atomicCAS(&lkey[h], kL0Empty, (u64)pt.addr);
          if (k == kL0Empty || k == (u64)pt.addr) break;
          h = (h + 1) & (kT - 1);
        }
      }
      atomicAdd(&lcnt[h], inc);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k <= kT; k += blockDim.x) {
      const uint32_t c = lcnt[k];
      if (!c) continue;
      const u64 a = lkey[k];
      u64 slot;
      if (k == kT) {
        slot = it.off + it.mask + 1;
      } else {
        u64 h = l0_hash((long long)a) & it.mask;
        for (;;) {
          u64 kk = atomicCAS(&keys[it.off + h], kL0Empty, a);
          if (kk == kL0Empty || kk == a) break;
          h = (h + 1) & it.mask;
        }
        slot = it.off + h;
      }
      const u64 ni = c & 0xFFFF, nj = c >> 16;
      const u64 old = atomicAdd(&cnt[slot], it.self ? ni : (ni | (nj << 32)));
      if (it.self) s += 2 * old * ni + ni * ni;
      else s += ni * (old >> 32) + nj * (old & 0xFFFFFFFFull) + ni * nj;
    }
    __syncthreads();
  }
  (void)err;  // the first partition pass has recorded evaluation errors
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(&lsum, s);
  __syncthreads();
  if (threadIdx.x == 0 && lsum) atomicAdd(&s0[ch.item], lsum);
}

// Adds each split item's S_0 to its inter-block count, unless the item's
// split pass overflowed (its whole count is then redone by the fallback).
__global__ void k_apply_s0(uint32_t n, const L0Item* __restrict__ items,
                           const u64* __restrict__ s0,
                           const uint32_t* __restrict__ skip,
                           QAcc* __restrict__ acc) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || skip[k] || !(items[k].qmask & 1) || !s0[k]) return;
  atomicAdd(&acc[items[k].q].cnt[0], s0[k]);
}

// Unit filter of the HBM items: an item proven free of conflicts
// (unit_free) is marked kApart in ovf, so that its partition, address
// filter and join do nothing and no later phase takes it up.  Error-scan
// items and items without facts stay.  The marked items are counted in
// *napart.
__global__ void k_unit_filter(uint32_t n, const HItem* __restrict__ hitems,
                              const QDesc* __restrict__ qd,
                              const IFact* __restrict__ facts,
                              uint32_t* __restrict__ ovf, u64* __restrict__ napart) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  bool apart = false;
  if (k < n) {
    const HItem h = hitems[k];
    const QDesc q = qd[h.q];
    apart = h.shared != 2 && unit_free(facts[h.inst_i], facts[h.inst_j], q.flags,
                                       !q.self && h.inst_i != h.inst_j);
    if (apart) ovf[k] = kApart;
  }
  const u64 c = (u64)__popcll(__ballot(apart));
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(napart, c);
}

// ---------------------------------------------------------------------------
// Kernel: exact filter of HBM buckets, one workgroup per run of buckets of
// one item, all its threads on one bucket at a time.
//
// A conflict needs two records of one bucket with equal addresses (and
// equal blocks for shared arrays, whose memory is per block) that belong to
// two different threads, one record from each access (for a self pair: any
// two records).  The workgroup keeps an LDS open-addressing table of 2 CAP
// 64-bit slots, a slot holding key << 32 | owner: key is the address itself
// for a 32-bit global array, otherwise a 32-bit hash of the address (and
// the block); owner is 1 + the thread id (block * threads per block +
// thread) of the first side-a record that brought the key, or kMulti once
// records of two different threads brought it.  Side-a records (every
// record of a self pair) are inserted; a self-pair record that finds its
// key there from another thread has a partner.  Side-b records then look
// their key up and have a partner when it is there from another thread.
// The bucket goes on to the join only if some record has a partner.  Keys
// that only hash alike can keep a bucket but never drop one, so skipping a
// bucket without partners is exact.  When thread ids of the launch do not
// fit 32 bits, owners are kMulti from the start (an address test alone).
// Items split by (address, block) (their level 0 is counted elsewhere)
// always go on.

constexpr uint32_t kFilterThreads = 256;
constexpr uint32_t kMulti = 0xFFFFFFFFu;

template <int CAP>
struct FilterLds {
  u64 slot[2 * CAP];
  uint32_t vote[2];
};

// What a record needs from its side's instance: points per block, the
// point order inside a block and the thread / iteration extents.
struct SideGeo {
  uint32_t tpb, iorder, nthr, niota;
  FastDiv f_tpb, f_nthr, f_niota;
};

__device__ __forceinline__ SideGeo side_geo(const DevInst* __restrict__ insts, uint32_t k) {
  k = __builtin_amdgcn_readfirstlane(k);
  const DevInst& I = insts[k];
  SideGeo g;
  g.tpb = I.a.tpb;
  g.iorder = I.a.iorder;
  g.nthr = I.a.nthr;
  g.niota = I.a.niota;
  g.f_nthr = I.f_nthr;
  g.f_niota = I.f_niota;
  g.f_tpb = make_fastdiv(g.tpb);
  return g;
}

// Block and thread of point index p (the block is the slowest coordinate).
__device__ __forceinline__ void block_thread(const SideGeo& g, uint32_t p, uint32_t& b,
                                             uint32_t& t) {
  b = fdiv(p, g.f_tpb);
  const uint32_t in = p - b * g.tpb;
  if (g.iorder) t = fdiv(in, g.f_niota);
  else t = in - fdiv(in, g.f_nthr) * g.nthr;
}

// What the table-path join needs to decode a record of one side: the point
// order and extents, and where the side's packed interval ids are.
struct SideDec {
  FastDiv f_nthr, f_niota;
  uint32_t nthr, niota, iorder, iv_off, iv_const;
  const int64_t* tpool;
};

__device__ __forceinline__ SideDec side_dec(const DevInst* __restrict__ insts, uint32_t k) {
  k = __builtin_amdgcn_readfirstlane(k);
  const DevInst& I = insts[k];
  SideDec d;
  d.f_nthr = I.f_nthr;
  d.f_niota = I.f_niota;
  d.nthr = I.a.nthr;
  d.niota = I.a.niota;
  d.iorder = I.a.iorder;
  d.iv_off = I.iv_off;
  d.iv_const = I.iv_const;
  d.tpool = I.tpool;
  return d;
}

// decode() with the side chosen per lane: point pidx of side `side`.
__device__ __forceinline__ PointIds decode_side(const SideDec& d0, const SideDec& d1,
                                                uint32_t side, uint32_t pidx) {
  const FastDiv fn = side ? d1.f_nthr : d0.f_nthr;
  const FastDiv fi = side ? d1.f_niota : d0.f_niota;
  const uint32_t nthr = side ? d1.nthr : d0.nthr;
  const uint32_t niota = side ? d1.niota : d0.niota;
  PointIds o;
  if (side ? d1.iorder : d0.iorder) {
    const uint32_t rest = fdiv(pidx, fi);
    o.ilin = pidx - rest * niota;
    o.blin = fdiv(rest, fn);
    o.tlin = rest - o.blin * nthr;
  } else {
    const uint32_t rest = fdiv(pidx, fn);
    o.tlin = pidx - rest * nthr;
    o.blin = fdiv(rest, fi);
    o.ilin = rest - o.blin * niota;
  }
  return o;
}

__device__ __forceinline__ uint32_t filter_key(u64 a, uint32_t b, bool exact32) {
  if (exact32) return (uint32_t)a;
  uint32_t x = (uint32_t)a * 0x9E3779B1u ^ (uint32_t)(a >> 32) * 0x85EBCA77u ^
               b * 0xC2B2AE3Du;
  x ^= x >> 15;
  x *= 0x2C1B3C6Du;
  x ^= x >> 12;
  return x;
}

__device__ __forceinline__ uint32_t filter_slot(uint32_t key, uint32_t mask) {
  uint32_t x = key * 0x9E3779B1u;
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  return x & mask;
}

template <int CAP>
__global__ void __launch_bounds__(kFilterThreads)
k_bucket_filter(const BRun* __restrict__ runs, const HItem* __restrict__ hitems,
                const QDesc* __restrict__ qd, const DevInst* __restrict__ insts,
                const unsigned char* __restrict__ recs,
                const uint32_t* __restrict__ cursor, const uint32_t* __restrict__ ovf,
                const uint32_t* __restrict__ done, uint8_t* __restrict__ cand,
                u64* __restrict__ nbytes) {
  constexpr int RPT = CAP / kFilterThreads;
  constexpr uint32_t mask = 2 * CAP - 1;
  static_assert(CAP % kFilterThreads == 0, "filter records per thread");
  static_assert((2 * CAP * 8) % (16 * kFilterThreads) == 0, "filter table clear");
  extern __shared__ __align__(16) unsigned char smem[];
  FilterLds<CAP>& T = *reinterpret_cast<FilterLds<CAP>*>(smem);
  const BRun R = runs[blockIdx.x];
  const HItem h = hitems[R.item];
  if (ovf[R.item] || done[h.q]) return;  // the join skips these runs too
  // level 0 counted per address, block 0 of identical blocks with the
  // inter-block class (a record pairs with its copies in other blocks), or
  // a dense item (its buckets nearly all pass): always joined
  if (h.shared == 3 || h.dense || (h.gmult > 1 && (qd[h.q].mask & 1))) {
    for (uint32_t b = R.b0 + threadIdx.x; b < R.b1; b += kFilterThreads)
      cand[h.bucket0 + b] = 1;
    return;
  }
  const bool self = qd[h.q].self != 0;
  const bool shared = h.shared == 1;
  const bool is32 = h.is32 != 0;
  const bool exact32 = is32 && !shared;  // the key is the address itself
  const SideGeo ga = side_geo(insts, h.inst_i);
  const SideGeo gb = self ? ga : side_geo(insts, h.inst_j);
  // thread ids below kMulti - 1 (same launch on both sides)
  const uint32_t nblk = insts[__builtin_amdgcn_readfirstlane(h.inst_i)].a.nblk;
  const bool tid_ok = (u64)nblk * ga.nthr < (u64)kMulti - 1;
  const u64* r8 = reinterpret_cast<const u64*>(recs + h.rec_off);
  const ulonglong2* r16 = reinterpret_cast<const ulonglong2*>(recs + h.rec_off);
  u64 ad[RPT];
  uint32_t pid[RPT];
  auto fetch = [&](uint32_t b, uint32_t n) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const uint32_t r = (uint32_t)j * kFilterThreads + threadIdx.x;
      ad[j] = 0;
      pid[j] = 0;
      if (r < n) {
        if (is32) {
          const u64 v = r8[(u64)b * CAP + r];
          ad[j] = (u64)(int64_t)(int32_t)(uint32_t)v;
          pid[j] = (uint32_t)(v >> 32);
        } else {
          const ulonglong2 v = r16[(u64)b * CAP + r];
          ad[j] = v.x;
          pid[j] = (uint32_t)v.y;
        }
      }
    }
  };
  if (threadIdx.x < 2) T.vote[threadIdx.x] = 0;  // ordered by the first barrier
  u64 nread = 0;  // record bytes read (every thread counts; thread 0 adds)
  uint32_t n = R.b0 < R.b1 ? min(cursor[h.bucket0 + R.b0], (uint32_t)CAP) : 0;
  if (R.b0 < R.b1) fetch(R.b0, n);
  for (uint32_t b = R.b0; b < R.b1; ++b) {
    const uint32_t gbk = h.bucket0 + b;
    nread += (u64)n * (is32 ? 8u : 16u);
    // keys and owners of this bucket's records
    uint32_t key[RPT], own[RPT];
    bool sb[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      sb[j] = (pid[j] >> 31) != 0;
      const SideGeo& g = sb[j] ? gb : ga;
      uint32_t bl, tl;
      block_thread(g, pid[j] & 0x7FFFFFFFu, bl, tl);
      key[j] = filter_key(ad[j], shared ? bl : 0u, exact32);
      own[j] = tid_ok ? bl * ga.nthr + tl + 1 : kMulti;
    }
    const uint32_t nb = n;
    // the next bucket's records load while this one is filtered
    if (b + 1 < R.b1) {
      n = min(cursor[gbk + 1], (uint32_t)CAP);
      fetch(b + 1, n);
    }
    // clear the table (the previous bucket's lookups ended at its vote)
    uint4* t4 = reinterpret_cast<uint4*>(T.slot);
#pragma unroll
    for (uint32_t k = 0; k < (2 * CAP * 8) / (16 * kFilterThreads); ++k)
      t4[k * kFilterThreads + threadIdx.x] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    bool found = false;
    // side a (every record of a self pair) inserts
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const uint32_t r = (uint32_t)j * kFilterThreads + threadIdx.x;
      if (r >= nb || (!self && sb[j])) continue;
      const u64 v = ((u64)key[j] << 32) | own[j];
      uint32_t sl = filter_slot(key[j], mask);
      for (;;) {
        u64 o = atomicCAS(&T.slot[sl], 0ull, v);
        if (o == 0) break;
        if ((uint32_t)(o >> 32) == key[j]) {
          uint32_t ow = (uint32_t)o;
          if (ow != own[j] || ow == kMulti) {
            found |= self;
            // two threads of side a hold the key (monotone: the owner only
            // ever becomes kMulti, so a failed swap means it already is)
            if (!self && ow != kMulti)
              (void)atomicCAS(&T.slot[sl], o, ((u64)key[j] << 32) | kMulti);
          }
          break;
        }
        sl = (sl + 1) & mask;
      }
    }
    __syncthreads();
    // side b looks up
    if (!self) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const uint32_t r = (uint32_t)j * kFilterThreads + threadIdx.x;
        if (r >= nb || !sb[j]) continue;
        uint32_t sl = filter_slot(key[j], mask);
        for (;;) {
          const u64 o = T.slot[sl];
          if (o == 0) break;
          if ((uint32_t)(o >> 32) == key[j]) {
            const uint32_t ow = (uint32_t)o;
            found |= ow != own[j] || ow == kMulti;
            break;
          }
          sl = (sl + 1) & mask;
        }
      }
    }
    // tag b + 1 on the word of b's parity (its previous vote, bucket b - 2,
    // was read before this bucket's first barrier)
    const bool any = block_vote(found, &T.vote[b & 1], b + 1);
    if (threadIdx.x == 0) cand[gbk] = any ? 1 : 0;
  }
  if (threadIdx.x == 0 && nread) atomicAdd(&nbytes[blockIdx.x & (kByteSlots - 1)], nread);
}

// ---------------------------------------------------------------------------
// Kernel: join the records of HBM buckets in LDS.

constexpr uint32_t kJoinThreads = 512;  // bucket-join workgroup size

// Workgroups of the bucket join that the LDS of one CU holds (160 KiB; the
// synchronised join also holds a synchronisation address per record): the
// register budget of the table-path joins is set so that as many fit by
// registers too (the interpreter path keeps its registers: no spills).
template <int CAP, int TBL, bool SYN = false>
constexpr uint32_t join_waves_per_simd() {
  return 2u * (uint32_t)(163840 / (sizeof(JoinLds<CAP, TBL>) + (SYN ? CAP * sizeof(u64) : 0)));
}

// One workgroup joins a run of buckets of one item.  The item's header,
// query and bucket counts are loaded once per run; the next bucket's
// records are loaded into registers while the current one is joined; an
// address pre-filter by signatures drops buckets (and records) that cannot
// pair before any point id is decoded; the counts are committed once per
// run.  TAB: both instances of every item of the launch have term tables
// (interval ids by lookup, no interpreter code).
template <int CAP, int TBL, bool TAB, bool SYN = false>
__global__ void __launch_bounds__(kJoinThreads)
__attribute__((amdgpu_waves_per_eu(TAB ? join_waves_per_simd<CAP, TBL, SYN>() : 1u)))
k_bucket_join(const BRun* __restrict__ runs, const HItem* __restrict__ hitems,
              const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
              const int64_t* __restrict__ params,
              const int64_t* __restrict__ loopvals,
              const QDesc* __restrict__ qd, QAcc* __restrict__ acc,
              const unsigned char* __restrict__ recs,
              const uint32_t* __restrict__ cursor,
              const uint32_t* __restrict__ ovf,
              const uint32_t* __restrict__ done, const u64* __restrict__ l0keys,
              const u64* __restrict__ l0cnt, const uint8_t* __restrict__ cand,
              u64* __restrict__ nbytes) {
  extern __shared__ __align__(16) unsigned char smem[];
  JoinLds<CAP, TBL>& S = *reinterpret_cast<JoinLds<CAP, TBL>*>(smem);
  // SYN: the records' synchronisation addresses after the join's LDS
  u64* skey = SYN ? reinterpret_cast<u64*>(smem + sizeof(JoinLds<CAP, TBL>)) : nullptr;
  const BRun R = runs[blockIdx.x];
  const HItem h = hitems[R.item];
  if (ovf[R.item] || done[h.q]) return;
  const QDesc q = qd[h.q];
  init_red(S);
  const bool l0ext = h.shared == 3;
  // the signature pre-filter only when no exact bucket filter ran before
  // (a bucket it passed holds records with partners, and the join's first
  // level drops the others exactly)
  const uint32_t gmult = h.gmult > 1 ? h.gmult : 1u;
  const bool sig = cand == nullptr && !(gmult > 1 && (q.mask & 1));
  const bool is32 = h.is32 != 0;
  constexpr int RPT = (CAP + kJoinThreads - 1) / kJoinThreads;
  u64 rx[RPT], ry[RPT];
  const u64* r8 = reinterpret_cast<const u64*>(recs + h.rec_off);
  const ulonglong2* r16 = reinterpret_cast<const ulonglong2*>(recs + h.rec_off);
#define HGRD_FETCH(B, N)                                            \
  {                                                                 \
    const u64 slot0 = (u64)(B) * CAP;                               \
    _Pragma("unroll") for (int j = 0; j < RPT; ++j) {               \
      const uint32_t r = threadIdx.x + (uint32_t)j * kJoinThreads;  \
      rx[j] = 0;                                                    \
      ry[j] = 0;                                                    \
      if (r < (N)) {                                                \
        if (is32) {                                                 \
          rx[j] = r8[slot0 + r];                                    \
        } else {                                                    \
          const ulonglong2 v = r16[slot0 + r];                      \
          rx[j] = v.x;                                              \
          ry[j] = v.y;                                              \
        }                                                           \
      }                                                             \
    }                                                               \
  }
  // the run's buckets that the address filter passed (all of them without
  // a filter), compacted by one wavefront, with their record counts
  if (threadIdx.x < 64) {
    const uint32_t k = threadIdx.x;
    const bool c = k < R.b1 - R.b0 && (!cand || cand[h.bucket0 + R.b0 + k]);
    const u64 bal = __ballot(c);
    if (c) {
      const uint32_t pos = (uint32_t)__popcll(bal & ((1ull << k) - 1));
      S.bl[pos] = k;
      S.bn[pos] = min(cursor[h.bucket0 + R.b0 + k], (uint32_t)CAP);
    }
    if (k == 0) S.nbl = (uint32_t)__popcll(bal);
  }
  __syncthreads();  // S.red, S.vote, S.bl, S.bn ready
  const uint32_t nbl = S.nbl;
  if (nbl == 0) return;
  uint32_t n = S.bn[0];
  u64 nread = 0;  // record bytes read (thread 0)
  HGRD_FETCH(R.b0 + S.bl[0], n)
  const bool self = q.self != 0;
  // table path without synchronisation: both sides' decoding constants
  // once per run, both sides decoded in one pass
  SideDec d0, d1;
  if (TAB && !SYN) {
    d0 = side_dec(insts, h.inst_i);
    d1 = side_dec(insts, h.inst_j);
  }
  for (uint32_t kb = 0; kb < nbl; ++kb) {
    const uint32_t b = R.b0 + S.bl[kb];
    bool go = n != 0;
    nread += (u64)n * (is32 ? 8u : 16u);
    uint32_t i1[RPT], i2[RPT];
    bool sd[RPT];
    if (!l0ext) {
      // address and point id only (the point id waits in S.blin until the
      // records that may share an address with the other side are known);
      // the signature bitmap is cleared for this bucket
      if (sig) sig_clear<kJoinThreads>(S);
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const uint32_t r = threadIdx.x + (uint32_t)j * kJoinThreads;
        const uint32_t pid = is32 ? (uint32_t)(rx[j] >> 32) : (uint32_t)ry[j];
        const u64 a = is32 ? (u64)(int64_t)(int32_t)(uint32_t)rx[j] : rx[j];
        sd[j] = (pid >> 31) != 0;
        // shared arrays: memory is per block, so the block joins the address
        uint32_t salt = 0;
        if (h.shared == 1) {
          const uint32_t p = pid & 0x7FFFFFFFu;
          const uint32_t m = sd[j] ? h.tpb_m[1] : h.tpb_m[0];
          const uint32_t sh = sd[j] ? h.tpb_s[1] : h.tpb_s[0];
          salt = ((__umulhi(m, p) + p) >> sh) + 1;
        }
        if (sig) sig_index<TBL>(a, salt, i1[j], i2[j]);
        if (r >= n) continue;
        S.addr[r] = a;
        S.blin[r] = pid;
        if (!sig) S.tli[r] = sd[j] ? kSide : 0u;  // every record active
      }
    }
    // the next bucket's records load while this one is joined
    const bool more = kb + 1 < nbl;
    const uint32_t n1 = more ? S.bn[kb + 1] : 0;
    const uint32_t b1n = more ? R.b0 + S.bl[kb + 1] : 0;
    if (!l0ext) {
      if (more) HGRD_FETCH(b1n, n1)
    }
    if (!l0ext && sig) {
      __syncthreads();
      if (go) {
#pragma unroll
        for (int j = 0; j < RPT; ++j)
          if (threadIdx.x + (uint32_t)j * kJoinThreads < n) sig_insert(S, i1[j], i2[j], sd[j], self);
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const uint32_t r = threadIdx.x + (uint32_t)j * kJoinThreads;
          if (r >= n) continue;
          const bool cand = sig_test(S, i1[j], i2[j], sd[j], self);
          any |= cand;
          S.tli[r] = (sd[j] ? kSide : 0u) | (cand ? 0u : kInactive);
        }
        // tag kb + 1 on the word of kb's parity: the same word's previous
        // vote (bucket kb - 2) was read before this bucket's first barrier
        go = block_vote(any, &S.vote[kb & 1], kb + 1);
      }
    }
    const uint32_t wsh = (q.warp & (q.warp - 1)) == 0 ? (uint32_t)__ffs((int)q.warp) - 1 : 32u;
    if (go && TAB && !SYN) {
      // full records of the candidates: ids by the side's constants, the
      // interval ids by one lookup in the side's table (one round trip for
      // both sides)
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const uint32_t r = threadIdx.x + (uint32_t)j * kJoinThreads;
        if (r >= n) continue;
        uint32_t pid;
        int64_t a;
        if (l0ext) {
          pid = is32 ? (uint32_t)(rx[j] >> 32) : (uint32_t)ry[j];
          a = is32 ? (int64_t)(int32_t)(uint32_t)rx[j] : (int64_t)rx[j];
        } else {
          if (S.tli[r] & kInactive) continue;
          pid = S.blin[r];
          a = (int64_t)S.addr[r];
        }
        const uint32_t side = pid >> 31;
        const PointIds id = decode_side(d0, d1, side, pid & 0x7FFFFFFFu);
        const uint32_t ivo = side ? d1.iv_off : d0.iv_off;
        const int64_t* tp = side ? d1.tpool : d0.tpool;
        const uint32_t iv = ivo != kNoTab ? (uint32_t)tp[ivo + id.ilin]
                                          : (side ? d1.iv_const : d0.iv_const);
        S.addr[r] = (u64)a;
        S.blin[r] = id.blin;
        S.tli[r] = (id.ilin << 16) | (side << 15) | id.tlin;
        S.bw[r] = ((iv & 0xFFFF) << 16) | (iv >> 16);
        S.w[r] = (uint16_t)(wsh < 32 ? id.tlin >> wsh : id.tlin / q.warp);
        if (l0ext) {
          // level-0 partners of a side-a record: the other side's count
          // at its address in the item's address-count table
          int32_t nj = 0;
          if ((q.mask & 1) && (q.self || !side))
            nj = (int32_t)l0_lookup(l0keys, l0cnt, h.l0_off, h.l0_mask, (long long)a,
                                    q.self != 0);
          S.part[r] = nj;
        }
      }
    } else if (go) {
      // full records of the candidates, one side at a time (the instance
      // stays uniform: scalar loads, no divergent interpreter)
      for (uint32_t side = 0; side < 2; ++side) {
        DevInst I;
        load_inst(I, insts, side ? h.inst_j : h.inst_i);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const uint32_t r = threadIdx.x + (uint32_t)j * kJoinThreads;
          if (r >= n) continue;
          uint32_t pid;
          int64_t a;
          if (l0ext) {
            pid = is32 ? (uint32_t)(rx[j] >> 32) : (uint32_t)ry[j];
            a = is32 ? (int64_t)(int32_t)(uint32_t)rx[j] : (int64_t)rx[j];
          } else {
            if (S.tli[r] & kInactive) continue;
            pid = S.blin[r];
            a = (int64_t)S.addr[r];
          }
          if ((pid >> 31) != side) continue;
          const PointIds id = decode(I, pid & 0x7FFFFFFFu);
          uint32_t bi, wi;
          if (TAB) {
            const uint32_t iv = I.iv_off != kNoTab ? (uint32_t)I.tpool[I.iv_off + id.ilin]
                                                   : I.iv_const;
            bi = iv & 0xFFFF;
            wi = iv >> 16;
          } else {
            point_iv(I, id, code, params, loopvals, bi, wi);
          }
          S.addr[r] = (u64)a;
          S.blin[r] = id.blin;
          S.tli[r] = (id.ilin << 16) | (side << 15) | id.tlin;
          if (SYN) {
            // syn() of the point (its addresses are proven error-free)
            int64_t v;
            uint32_t e2 = 0;
            const uint32_t b = point_syn(I, id, code, params, loopvals, v, e2);
            skey[r] = (u64)v;
            S.tli[r] |= b << 10;
          }
          S.bw[r] = (bi << 16) | wi;
          S.w[r] = (uint16_t)(wsh < 32 ? id.tlin >> wsh : id.tlin / q.warp);
          if (l0ext) {
            // level-0 partners of a side-a record: the other side's count
            // at its address in the item's address-count table
            int32_t nj = 0;
            if ((q.mask & 1) && (q.self || !side))
              nj = (int32_t)l0_lookup(l0keys, l0cnt, h.l0_off, h.l0_mask, (long long)a,
                                      q.self != 0);
            S.part[r] = nj;
          }
        }
      }
    }
    if (l0ext && more) HGRD_FETCH(b1n, n1)
#undef HGRD_FETCH
    if (threadIdx.x == 0) S.n = n;
    __syncthreads();
    if (go) lds_join<kJoinThreads, CAP, TBL, SYN>(S, q, h.sigma, l0ext, gmult, skey);
    __syncthreads();
    n = n1;
  }
  commit_join(S, &acc[h.q], gmult);
  if (threadIdx.x == 0 && nread) atomicAdd(&nbytes[blockIdx.x & 63], nread);
}

// ---------------------------------------------------------------------------
// Fallback for items that still overflow after a retry with more buckets
// (a single address, or a single (address, block), carries more points than
// one LDS tile holds).  Records of all such items go to one flat HBM array;
// every prefix level is aggregated in an HBM hash table keyed by (item,
// level key).  Each workgroup first merges its tile of records in an LDS
// table, so a hot key costs one global atomic per workgroup, not per point.
//
// Records are compressed within a wavefront: the lanes of one wavefront
// hold consecutive points, and when those are consecutive threads of one
// block and iteration (the instance's thread-fastest point order), lanes
// with equal addresses in one warp of the analysed program are matched
// (one ballot per distinct key) and written as one record: the first
// lane's point, the number of points (mult) and the lanes' mask relative to
// the first lane (thread tlin + k for bit k).  All points of a record share
// every key field up to the warp and the warp-barrier interval (one block,
// one iteration, so the same interval ids; one warp), so levels 0-4 count
// it with weight mult; the thread level (5) takes its lanes one by one.  A
// hot address (every thread on one element, as in a final reduction step)
// then costs one record per warp and wavefront instead of one per point.

struct GRec {
  u64* addr;
  uint32_t* blin;
  uint32_t* tli;   // ilin << 16 | side << 15 | tlin of the first lane
  uint32_t* bw;
  uint32_t* w;
  uint32_t* item;  // fallback item index, 0xFFFFFFFF: empty slot
  uint32_t* slot;
  long long* part;
  uint32_t* mult;  // points in the record
  u64* lanes;      // bit k: thread tlin + k
  u64* skey;       // synchronisation address (pairs with acquire/release);
                   // tli bit 10: a syn() at block scope, bit 11: at device
};

__global__ void __launch_bounds__(256)
k_gen_linear(const Chunk* __restrict__ chunks, const FItem* __restrict__ fitems,
             const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
             const int64_t* __restrict__ params,
             const int64_t* __restrict__ loopvals, GRec rec,
             uint32_t* __restrict__ count, QAcc* __restrict__ acc) {
  const Chunk ch = chunks[blockIdx.x];
  const FItem f = fitems[ch.item];
  DevInst I;
  load_inst(I, insts, ch.side ? f.inst_j : f.inst_i);
  const bool match = I.a.iorder == 0;  // lanes are consecutive threads of a row
  const bool syn = (I.a.syn & (kSynAcq | kSynRel)) != 0;
  const uint32_t lane = threadIdx.x & 63;
  uint32_t err = 0;
  for (uint32_t base = ch.p0; base < ch.p1; base += blockDim.x) {
    uint32_t pidx = base + threadIdx.x;
    bool valid = false;
    Point pt{0, 0, 0};
    PointIds id{0, 0, 0};
    int64_t sv = 0;
    uint32_t sb = 0;
    if (pidx < ch.p1) {
      id = decode(I, pidx);
      valid = point_eval(I, id, code, params, loopvals, pt, err);
      if (valid && syn) sb = point_syn(I, id, code, params, loopvals, sv, err);
    }
    const uint32_t wp = valid ? id.tlin / f.warp : 0;
    // match: a lane leads the group of pending lanes equal to it in
    // (address, block, iteration, warp, intervals); with threads fastest in
    // the point order, lane l + k of such a group is thread tlin + k
    bool pending = valid, lead = false;
    u64 mine_mask = 0;
    for (;;) {
      const u64 P = __ballot(pending);
      if (!P) break;
      const int l = __ffsll((long long)P) - 1;
      const u64 a = (u64)__shfl((long long)pt.addr, l, 64);
      const uint32_t b = (uint32_t)__shfl((int)id.blin, l, 64);
      const uint32_t il = (uint32_t)__shfl((int)id.ilin, l, 64);
      const uint32_t ww = (uint32_t)__shfl((int)wp, l, 64);
      const uint32_t iv = (uint32_t)__shfl((int)((pt.bint << 16) | pt.wint), l, 64);
      const int64_t v = (int64_t)__shfl((long long)sv, l, 64);
      const uint32_t vb = (uint32_t)__shfl((int)sb, l, 64);
      const bool mine =
          pending && (match ? ((u64)pt.addr == a && id.blin == b && id.ilin == il &&
                               wp == ww && ((pt.bint << 16) | pt.wint) == iv &&
                               sv == v && sb == vb)
                            : lane == (uint32_t)l);
      const u64 M = __ballot(mine);
      if (lane == (uint32_t)l) {
        lead = true;
        mine_mask = M >> l;
      }
      if (mine) pending = false;
    }
    const u64 Lb = __ballot(lead);
    if (Lb == 0) continue;
    const uint32_t leader = __ffsll((long long)Lb) - 1;
    uint32_t b0 = 0;
    if (lane == leader) b0 = atomicAdd(&count[ch.item], (uint32_t)__popcll(Lb));
    b0 = (uint32_t)__builtin_amdgcn_readlane((int)b0, (int)leader);
    if (lead) {
      uint32_t k = b0 + __popcll(Lb & ((1ull << lane) - 1));
      if (k < f.cap) {
        u64 r = f.off + k;
        rec.addr[r] = (u64)pt.addr;
        rec.blin[r] = id.blin;
        rec.tli[r] = (id.ilin << 16) | (ch.side << 15) | (sb << 10) | id.tlin;
        if (rec.skey) rec.skey[r] = (u64)sv;
        rec.bw[r] = (pt.bint << 16) | pt.wint;
        rec.w[r] = wp;
        rec.item[r] = ch.item;
        rec.part[r] = 0;
        rec.mult[r] = (uint32_t)__popcll(mine_mask);
        rec.lanes[r] = mine_mask;
      }
    }
  }
  // evaluation errors (items of synchronised pairs come here unscanned)
  for (int o = 32; o; o >>= 1) err |= (uint32_t)__shfl_xor((int)err, o, 64);
  if (lane == 0 && err) atomicOr(&acc[f.q].err, err);
}

// Levels 0-5 group records by (address, block, bint, warp, wint, thread)
// prefixes.  Levels 6-11 are the same groups with the synchronisation
// address added, over the records whose points have a syn() at the class's
// scope (device for levels 6 and 7, the inter-block class; block for 8-11):
// their pairs are the synchronised ones, subtracted from the conflicts.
// Key equality of (record x, lane kx) and (record y, lane ky) at level L
// (lanes matter at the thread level only).
__device__ __forceinline__ bool g_level_eq(const GRec& g, int L, u64 x, uint32_t kx, u64 y,
                                           uint32_t ky) {
  if (g.item[x] != g.item[y]) return false;
  if (g.addr[x] != g.addr[y]) return false;
  if (L >= 6) {
    if (g.skey[x] != g.skey[y]) return false;
    L -= 6;
  }
  if (L >= 1 && g.blin[x] != g.blin[y]) return false;
  if (L >= 2 && (g.bw[x] >> 16) != (g.bw[y] >> 16)) return false;
  if (L >= 3 && g.w[x] != g.w[y]) return false;
  if (L >= 4 && (g.bw[x] & 0xFFFF) != (g.bw[y] & 0xFFFF)) return false;
  if (L >= 5 && (g.tli[x] & 0x3FF) + kx != (g.tli[y] & 0x3FF) + ky) return false;
  return true;
}
__device__ __forceinline__ uint32_t g_hash(const GRec& g, int L, u64 r, uint32_t k) {
  u64 a = g.addr[r] ^ ((u64)g.item[r] * 0x2545F4914F6CDD1Dull);
  if (L >= 6) {
    a ^= g.skey[r] * 0xD6E8FEB86659FD93ull;
    L -= 6;
  }
  return level_hash(L, a, g.blin[r], g.bw[r], g.w[r], (g.tli[r] & 0x3FF) + k);
}

// Level L counts for item f: its class is in the mask and, for a
// synchronisation level, the pair's points can share a syn() at that scope.
__device__ __forceinline__ bool level_on(const FItem& f, int L) {
  const int b = L >= 6 ? L - 6 : L;
  if (!((f.mask >> (b >> 1)) & 1)) return false;
  return L < 6 || (f.sync & (b < 2 ? kQSyncDev : kQSyncBlk)) != 0;
}

// Record r takes part in level L (synchronisation levels: its points have
// a syn() at the level's scope).
__device__ __forceinline__ bool rec_on(const GRec& g, u64 r, int L) {
  return L < 6 || ((g.tli[r] >> (L < 8 ? 11 : 10)) & 1) != 0;
}

constexpr int kGTile = 1024;  // records per workgroup step
constexpr int kGLocal = 2048; // LDS table slots

// Inserts every record at level L.  S[item * 8 + L] += pair contributions.
__global__ void __launch_bounds__(256)
k_ginsert(GRec g, u64 n, int L, const FItem* __restrict__ fitems,
          u64* __restrict__ owner, u64* __restrict__ cnt, u64 tbl_mask,
          u64* __restrict__ S) {
  __shared__ uint32_t lown[kGLocal];
  __shared__ uint32_t lca[kGLocal];  // side-a (self: all) points of the local group
  __shared__ uint32_t lcb[kGLocal];  // side-b points
  __shared__ uint32_t lgs[kGLocal];
  // level sums of the items of this workgroup's records, merged in LDS so a
  // big item does not serialise on one global counter
  constexpr int kSlots = 16;
  __shared__ uint32_t sitem[kSlots];
  __shared__ u64 ssum[kSlots];
  const uint32_t tid = threadIdx.x;
  if (tid < kSlots) {
    sitem[tid] = kEmpty;
    ssum[tid] = 0;
  }
  // adds a group's points (li on side a, lj on side b) to the global table
  // and the level sum of item it
  auto add_global = [&](u64 r, uint32_t k, uint32_t it, bool self, u64 li, u64 lj) -> u64 {
    u64 h = g_hash(g, L, r, k) & tbl_mask;
    const u64 me = (r << 6) | k;
    for (;;) {
      const u64 o = atomicCAS(&owner[h], ~0ull, me);
      if (o == ~0ull || g_level_eq(g, L, o >> 6, (uint32_t)(o & 63), r, k)) break;
      h = (h + 1) & tbl_mask;
    }
    const u64 old = atomicAdd(&cnt[h], self ? li : (li | (lj << 32)));
    u64 contrib;
    if (self) contrib = 2 * old * li + li * li;  // (old + k)^2 - old^2
    else contrib = li * (old >> 32) + lj * (old & 0xFFFFFFFFull) + li * lj;
    if (contrib) {
      const uint32_t sl = it % kSlots;
      uint32_t prev = atomicCAS(&sitem[sl], kEmpty, it);
      if (prev == kEmpty || prev == it) atomicAdd(&ssum[sl], contrib);
      else atomicAdd(&S[(u64)it * 16 + L], contrib);
    }
    return h;
  };
  __syncthreads();
  for (u64 t0 = (u64)blockIdx.x * kGTile; t0 < n; t0 += (u64)gridDim.x * kGTile) {
    if (L == 5 || L == 11) {
      // thread level: every lane of a record is its own key; thread groups
      // are small, so lanes go straight to the global table
#pragma unroll
      for (int j = 0; j < kGTile / 256; ++j) {
        const u64 r = t0 + j * 256 + tid;
        if (r >= n) continue;
        const uint32_t it = g.item[r];
        if (it == kEmpty) continue;
        const FItem f = fitems[it];
        if (!level_on(f, L) || !rec_on(g, r, L)) continue;
        const bool sb = ((g.tli[r] >> 15) & 1) != 0;
        for (u64 m = g.lanes[r]; m; m &= m - 1) {
          const uint32_t k = (uint32_t)__ffsll((long long)m) - 1;
          add_global(r, k, it, f.self, (f.self || !sb) ? 1 : 0, (f.self || !sb) ? 0 : 1);
        }
      }
      continue;
    }
    for (uint32_t k = tid; k < kGLocal; k += blockDim.x) {
      lown[k] = kEmpty;
      lca[k] = 0;
      lcb[k] = 0;
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
      if (!level_on(f, L) || !rec_on(g, r, L)) continue;
      uint32_t h = g_hash(g, L, r, 0) & (kGLocal - 1);
      const uint32_t lr = (uint32_t)(r - t0);
      for (;;) {
        uint32_t o = atomicCAS(&lown[h], kEmpty, lr);
        if (o == kEmpty || g_level_eq(g, L, t0 + o, 0, r, 0)) break;
        h = (h + 1) & (kGLocal - 1);
      }
      uint32_t side = (g.tli[r] >> 15) & 1;
      // a record weighs its points (levels 0-4 hold all of its lanes)
      atomicAdd((f.self || !side) ? &lca[h] : &lcb[h], g.mult[r]);
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
      lgs[k] = (uint32_t)add_global(r, 0, it, f.self, lca[k], lcb[k]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kGTile / 256; ++j) {
      u64 r = t0 + j * 256 + tid;
      if (ls[j] != 0xFFFF) g.slot[r] = lgs[ls[j]];
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid < kSlots && sitem[tid] != kEmpty && ssum[tid])
    atomicAdd(&S[(u64)sitem[tid] * 16 + L], ssum[tid]);
}

// Adds +-(partners at level L, not a thread level) to every record of side
// a (self: all): the group at such a level holds all of a record's lanes,
// so the figure is the same for each of them.  Synchronisation levels
// count with the opposite sign.
__global__ void __launch_bounds__(256)
k_gpartner(GRec g, u64 n, int L, const FItem* __restrict__ fitems,
           const u64* __restrict__ cnt) {
  long long sign = (L & 1) ? -1 : 1;
  if (L >= 6) sign = -sign;  // (L - 6) & 1 == L & 1
  for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (u64)gridDim.x * blockDim.x) {
    uint32_t it = g.item[r];
    if (it == kEmpty) continue;
    const FItem f = fitems[it];
    if (!level_on(f, L) || !rec_on(g, r, L)) continue;
    uint32_t side = (g.tli[r] >> 15) & 1;
    if (!f.self && side) continue;
    u64 c = cnt[g.slot[r]];
    long long nj = f.self ? (long long)c : (long long)(c >> 32);
    // block 0 of identical blocks: the address level also counts the other
    // blocks' copies (only the sign of a partner count matters: 2 nj)
    if (L == 0 && f.gmult > 1) nj *= 2;
    g.part[r] += sign * nj;
  }
}

// Other-side points in the thread-level group of (record r, lane k) at
// level L (5 or 11), from that level's table (built last for its half).
__device__ __forceinline__ long long g_thread_count(const GRec& g, int L, u64 r, uint32_t k,
                                                    bool self, const u64* __restrict__ owner,
                                                    const u64* __restrict__ cnt, u64 tbl_mask) {
  u64 h = g_hash(g, L, r, k) & tbl_mask;
  for (;;) {
    const u64 o = owner[h];
    if (o == ~0ull) return 0;  // (never: every lane was inserted)
    if (g_level_eq(g, L, o >> 6, (uint32_t)(o & 63), r, k)) {
      const u64 c = cnt[h];
      return self ? (long long)c : (long long)(c >> 32);
    }
    h = (h + 1) & tbl_mask;
  }
}

// Witness candidates of the fallback records: the first lane of a record
// whose partner count is positive.  With a thread level in an item's
// classes, each lane subtracts its own thread group's other-side count
// (level 5, table A) and adds back its synchronised share (level 11,
// table B); both tables were the last built in their halves.
__global__ void __launch_bounds__(256)
k_gfinish(GRec g, u64 n, const FItem* __restrict__ fitems, const u64* __restrict__ owner,
          const u64* __restrict__ cnt, const u64* __restrict__ owner2,
          const u64* __restrict__ cnt2, u64 tbl_mask, uint32_t used,
          QAcc* __restrict__ acc) {
  for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (u64)gridDim.x * blockDim.x) {
    uint32_t it = g.item[r];
    if (it == kEmpty) continue;
    const FItem f = fitems[it];
    uint32_t tl = g.tli[r];
    if (!f.self && (tl & kSide)) continue;
    const bool l5 = ((used >> 5) & 1) && level_on(f, 5);
    const bool l11 = ((used >> 11) & 1) && level_on(f, 11) && rec_on(g, r, 11);
    for (u64 m = g.lanes[r]; m; m &= m - 1) {
      const uint32_t k = (uint32_t)__ffsll((long long)m) - 1;
      long long part = g.part[r];
      if (l5) part -= g_thread_count(g, 5, r, k, f.self, owner, cnt, tbl_mask);
      if (l11) part += g_thread_count(g, 11, r, k, f.self, owner2, cnt2, tbl_mask);
      if (part > 0) {
        u64 key = pkey(f.sigma, g.blin[r], (tl & 0x3FF) + k, tl >> 16);
        if (key < acc[f.q].pmin) atomicMin(&acc[f.q].pmin, key);
        break;  // later lanes have larger keys
      }
    }
  }
}

// Class counts of each fallback item from its level sums.
__global__ void k_gcounts(uint32_t nitems, const FItem* __restrict__ fitems,
                          const u64* __restrict__ S, QAcc* __restrict__ acc) {
  uint32_t it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitems) return;
  const FItem f = fitems[it];
  const u64* s = S + (u64)it * 16;
  // conflicts minus synchronised pairs (levels 6-11 are zero without them);
  // block 0 of G identical blocks: G^2 S_0 - G S_1, the others G times
  const u64 G = f.gmult > 1 ? f.gmult : 1;
  if (f.mask & 1) atomicAdd(&acc[f.q].cnt[0], G * (G * s[0] - s[1]) - (s[6] - s[7]));
  if (f.mask & 2) atomicAdd(&acc[f.q].cnt[1], G * (s[2] - s[3]) - (s[8] - s[9]));
  if (f.mask & 4) atomicAdd(&acc[f.q].cnt[2], G * (s[4] - s[5]) - (s[10] - s[11]));
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
  uint32_t q, inst_i, inst_j, p0, p1, sync, pad1, pad2;  // sync: kQSync* flags
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
  // synchronisation: p*'s syn() (bits: block, device scope) and address
  const bool sy = (it.sync & (kQSyncBlk | kQSyncDev)) != 0;
  int64_t pv = 0;
  uint32_t pbits = 0;
  {
    DevInst I;
    load_inst(I, insts, it.inst_i);
    PointIds id;
    id.blin = pb;
    id.tlin = pt_;
    id.ilin = pi;
    point_eval(I, id, code, params, loopvals, P, e);
    if (sy) pbits = point_syn(I, id, code, params, loopvals, pv, e);
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
    Point Q;
    if (!point_eval(J, id, code, params, loopvals, Q, err)) continue;
    if (Q.addr != P.addr) continue;
    if (id.blin == pb && id.tlin == pt_) continue;
    uint32_t cls;
    if (id.blin != pb) cls = 1;
    else if (id.tlin / q.warp == pw) cls = 4;
    else cls = 2;
    if (!(cls & q.mask)) continue;
    if (cls != 1 && Q.bint != P.bint) continue;
    if (cls == 4 && Q.wint != P.wint) continue;
    if (sy) {
      // no race when both syn() at the class's scope hit one address
      const uint32_t need = cls == 1 ? 2u : 1u;
      if (it.sync & (cls == 1 ? kQSyncDev : kQSyncBlk)) {
        int64_t qv;
        const uint32_t qbits = point_syn(J, id, code, params, loopvals, qv, err);
        if ((pbits & need) && (qbits & need) && pv == qv) continue;
      }
    }
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
    r.flags = (uint8_t)(a.qclass & 2);
    r.tiles = a.qclass >> 8;
  }
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
                          const QDesc* qd, QAcc* acc, const uint32_t* done,
                          uint32_t* cursor, uint32_t persist_grid, const IFact* facts) {
  size_t lds = sizeof(JoinLds<CAP, TBL>);
  if (cursor) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, cursor, 1u, 0u);
    hipLaunchKernelGGL((k_small_persist<CAP, TBL>), dim3(persist_grid), dim3(256),
                       lds, st, items, n, cursor, insts, code, params, loopvals,
                       qd, acc, done, facts);
    HGRD_CHECK(hipGetLastError());
    return 0;
  }
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL((k_small_join<CAP, TBL>), dim3(m), dim3(256), lds, st,
                       items + off, insts, code, params, loopvals, qd, acc, done, facts);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

template <int CAP, int TBL>
static int set_lds_attrs() {
  const int lds = (int)sizeof(JoinLds<CAP, TBL>);
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_small_join<CAP, TBL>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_small_persist<CAP, TBL>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_bucket_join<CAP, TBL, true>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_bucket_join<CAP, TBL, false>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  // the synchronised join also holds a synchronisation address per record
  // (the largest tile shape has no room for it: its items use the fallback)
  if (lds + CAP * (int)sizeof(u64) <= 160 * 1024)
    HGRD_CHECK(hipFuncSetAttribute((const void*)k_bucket_join<CAP, TBL, true, true>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   lds + CAP * (int)sizeof(u64)));
  HGRD_CHECK(hipFuncSetAttribute(
      (const void*)k_bucket_filter<CAP>, hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)sizeof(FilterLds<CAP>)));
  return 0;
}

template <int CAP, int TBL>
static int launch_bucket_t(hipStream_t st, uint32_t nruns, const BRun* runs,
                           uint32_t n_tab, const HItem* hitems, const DevInst* insts,
                           const DInsn* code, const int64_t* params,
                           const int64_t* loopvals, const QDesc* qd, QAcc* acc,
                           const unsigned char* recs, const uint32_t* cursor,
                           const uint32_t* ovf, const uint32_t* done,
                           const u64* l0keys, const u64* l0cnt, uint8_t* cand,
                           u64* nbytes, const hipEvent_t* kev, bool syn = false) {
  // syn: every run is of a synchronised item with term tables (joined with
  // the synchronisation levels, no per-kernel events).
  // Otherwise runs [0, n_tab) are of items whose instances have term tables; record
  // bytes read by the join are counted in nbytes[0..63] and nbytes[64..127],
  // by the address filter (when cand is given) in nbytes[256..319].  The
  // filter runs over every run first; `mid` (optional) is recorded between
  // filter and join.
  size_t lds = sizeof(JoinLds<CAP, TBL>);
  // kev (optional): start and stop events of the filter, then of the join
  // of the first n_tab runs, taken by the dispatch packets themselves
  const hipEvent_t f0 = kev ? kev[0] : nullptr, f1 = kev ? kev[1] : nullptr;
  const hipEvent_t j0 = kev ? kev[2] : nullptr, j1 = kev ? kev[3] : nullptr;
  if (cand) {
    const size_t flds = sizeof(FilterLds<CAP>);
    for (uint32_t off = 0; off < nruns; off += 1u << 20) {
      uint32_t m = nruns - off < (1u << 20) ? nruns - off : (1u << 20);
      const hipEvent_t a = off == 0 ? f0 : nullptr;
      const hipEvent_t b = off + m == nruns ? f1 : nullptr;
      if (a || b)
        hipExtLaunchKernelGGL(k_bucket_filter<CAP>, dim3(m), dim3(kFilterThreads), flds, st, a,
                              b, 0, runs + off, hitems, qd, insts, recs, cursor, ovf, done,
                              cand, nbytes + 256);
      else
        hipLaunchKernelGGL(k_bucket_filter<CAP>, dim3(m), dim3(kFilterThreads), flds,
                           st, runs + off, hitems, qd, insts, recs, cursor, ovf, done, cand,
                           nbytes + 256);
      HGRD_CHECK(hipGetLastError());
    }
  }
  if (syn) {
    if (lds + CAP * sizeof(u64) > 160 * 1024) return 1;  // never planned so
    for (uint32_t off = 0; off < nruns; off += 1u << 20) {
      uint32_t m = nruns - off < (1u << 20) ? nruns - off : (1u << 20);
      hipLaunchKernelGGL((k_bucket_join<CAP, TBL, true, true>), dim3(m), dim3(kJoinThreads),
                         lds + CAP * sizeof(u64), st, runs + off, hitems, insts, code, params,
                         loopvals, qd, acc, recs, cursor, ovf, done, l0keys, l0cnt, cand,
                         nbytes + 64);
      HGRD_CHECK(hipGetLastError());
    }
    return 0;
  }
  for (uint32_t off = 0; off < nruns; off += 1u << 20) {
    uint32_t m = nruns - off < (1u << 20) ? nruns - off : (1u << 20);
    uint32_t mt = off >= n_tab ? 0 : (n_tab - off < m ? n_tab - off : m);
    if (mt) {
      const hipEvent_t a = off == 0 ? j0 : nullptr;
      const hipEvent_t b = off + mt == n_tab ? j1 : nullptr;
      if (a || b)
        hipExtLaunchKernelGGL((k_bucket_join<CAP, TBL, true>), dim3(mt), dim3(kJoinThreads), lds,
                              st, a, b, 0, runs + off, hitems, insts, code, params, loopvals, qd,
                              acc, recs, cursor, ovf, done, l0keys, l0cnt, (const uint8_t*)cand,
                              nbytes);
      else
        hipLaunchKernelGGL((k_bucket_join<CAP, TBL, true>), dim3(mt), dim3(kJoinThreads), lds,
                           st, runs + off, hitems, insts, code, params, loopvals, qd, acc,
                           recs, cursor, ovf, done, l0keys, l0cnt, cand, nbytes);
    }
    if (m > mt)
      hipLaunchKernelGGL((k_bucket_join<CAP, TBL, false>), dim3(m - mt), dim3(kJoinThreads),
                         lds, st, runs + off + mt, hitems, insts, code, params, loopvals,
                         qd, acc, recs, cursor, ovf, done, l0keys, l0cnt, cand, nbytes + 64);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

}  // namespace hgrd

// ---- entry points used by the host driver ---------------------------------
namespace hgrd {

size_t devinst_size() { return sizeof(DevInst); }

void set_devinst_tab(void* dst, const TabHost& t, const int64_t* pool) {
  DevInst d;
  memcpy(&d, dst, sizeof d);
  d.tpool = pool + t.base;
  d.tu = t.u;
  for (int g = 0; g < 3; ++g) d.toff[g] = t.off[g];
  d.iv_off = t.iv_off;
  d.iv_const = t.iv_const;
  d.tnever = t.never;
  d.tab = t.on;
  memcpy(dst, &d, sizeof d);
}

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
void fastdiv_consts(uint32_t d, uint32_t* m, uint32_t* s) {
  const FastDiv f = make_fastdiv(d);
  *m = f.m;
  *s = f.s;
}

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
                 const int64_t* loopvals, const QDesc* qd, QAcc* acc,
                 const uint32_t* done, uint32_t* cursor, uint32_t persist_grid,
                 const IFact* facts) {
  const DevInst* I = (const DevInst*)insts;
  switch (cfg) {
    case 0: return launch_small_t<1024, 2048>(st, items, n, I, code, params, loopvals, qd, acc, done, cursor, persist_grid, facts);
    case 1: return launch_small_t<1536, 4096>(st, items, n, I, code, params, loopvals, qd, acc, done, cursor, persist_grid, facts);
    default: return launch_small_t<3072, 8192>(st, items, n, I, code, params, loopvals, qd, acc, done, cursor, persist_grid, facts);
  }
}

// Raises the LDS limit of every join kernel (once per device, before any
// launch or graph capture).
int init_kernel_attributes() {
  if (set_lds_attrs<1024, 2048>() || set_lds_attrs<1536, 4096>() ||
      set_lds_attrs<3072, 8192>())
    return -1;
  return init_verdict_attributes();
}

int launch_tabulate(hipStream_t st, const Chunk* chunks, uint32_t n,
                    const TabJob* jobs, const void* insts, const DInsn* code,
                    const int64_t* params, const int64_t* loopvals, int64_t* pool) {
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL(k_tabulate, dim3(m), dim3(256), 0, st, chunks + off, jobs,
                       (const DevInst*)insts, code, params, loopvals, pool);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

// One thread per output entry: the spec holding it by binary search over
// the specs' first entries, then its slice.
__global__ void k_expand(const ExpandSpec* __restrict__ specs, uint32_t n, u64 total,
                         bool runs, uint4* __restrict__ out) {
  for (u64 e = (u64)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (u64)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = n - 1;  // the last spec whose first entry is <= e
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (specs[mid].first <= e) lo = mid;
      else hi = mid - 1;
    }
    const ExpandSpec sp = specs[lo];
    const uint32_t a = (uint32_t)(e - sp.first) * sp.per;
    const uint32_t b = min(sp.n, a + sp.per);
    out[e] = runs ? make_uint4(sp.item, a, b, 0u) : make_uint4(sp.item, sp.side, a, b);
  }
}

int launch_expand(hipStream_t st, const ExpandSpec* specs, uint32_t n, u64 total, bool runs,
                  void* out) {
  if (n == 0 || total == 0) return 0;
  const u64 blocks = (total + 255) / 256;
  hipLaunchKernelGGL(k_expand, dim3((uint32_t)(blocks < 65536 ? blocks : 65536)), dim3(256), 0,
                     st, specs, n, total, runs, (uint4*)out);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_unit_filter(hipStream_t st, uint32_t n, const HItem* hitems, const QDesc* qd,
                       const IFact* facts, uint32_t* ovf, unsigned long long* napart) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_unit_filter, dim3((n + 255) / 256), dim3(256), 0, st, n, hitems, qd,
                     facts, ovf, napart);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_scatter(hipStream_t st, const Chunk* chunks, uint32_t n, bool tab,
                   const HItem* hitems, const void* insts, const DInsn* code,
                   const int64_t* params, const int64_t* loopvals, QAcc* acc,
                   unsigned char* recs, uint32_t* cursor,
                   uint32_t* ovf, uint32_t capb, const uint32_t* done,
                   unsigned long long* nbytes, hipEvent_t t0, hipEvent_t t1) {
  // tab: every chunk's instance has term tables; t0, t1 (optional): start
  // and stop events taken by the dispatch packets themselves
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    const hipEvent_t a = off == 0 ? t0 : nullptr;
    const hipEvent_t b = off + m == n ? t1 : nullptr;
    if (tab && (a || b))
      hipExtLaunchKernelGGL(k_scatter<true>, dim3(m), dim3(kScatterThreads), 0, st, a, b, 0,
                            chunks + off, hitems, (const DevInst*)insts, code, params,
                            loopvals, acc, recs, cursor, ovf, capb, done, nbytes);
    else if (tab)
      hipLaunchKernelGGL(k_scatter<true>, dim3(m), dim3(kScatterThreads), 0, st, chunks + off,
                         hitems, (const DevInst*)insts, code, params, loopvals,
                         acc, recs, cursor, ovf, capb, done, nbytes);
    else
      hipLaunchKernelGGL(k_scatter<false>, dim3(m), dim3(kScatterThreads), 0, st, chunks + off,
                         hitems, (const DevInst*)insts, code, params, loopvals,
                         acc, recs, cursor, ovf, capb, done, nbytes);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_bucket(int cfg, hipStream_t st, uint32_t nruns, const BRun* runs,
                  uint32_t n_tab, const HItem* hitems, const void* insts,
                  const DInsn* code, const int64_t* params, const int64_t* loopvals,
                  const QDesc* qd, QAcc* acc, const unsigned char* recs,
                  const uint32_t* cursor, const uint32_t* ovf, const uint32_t* done,
                  const u64* l0keys, const u64* l0cnt, uint8_t* cand, u64* nbytes,
                  const hipEvent_t* kev, bool syn) {
  const DevInst* I = (const DevInst*)insts;
  switch (cfg) {
    case 0: return launch_bucket_t<1024, 2048>(st, nruns, runs, n_tab, hitems, I, code, params, loopvals, qd, acc, recs, cursor, ovf, done, l0keys, l0cnt, cand, nbytes, kev, syn);
    case 1: return launch_bucket_t<1536, 4096>(st, nruns, runs, n_tab, hitems, I, code, params, loopvals, qd, acc, recs, cursor, ovf, done, l0keys, l0cnt, cand, nbytes, kev, syn);
    default: return launch_bucket_t<3072, 8192>(st, nruns, runs, n_tab, hitems, I, code, params, loopvals, qd, acc, recs, cursor, ovf, done, l0keys, l0cnt, cand, nbytes, kev, syn);
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
                    uint32_t* count, void* owner, void* cnt, void* owner2, void* cnt2,
                    u64 tbl, void* S, QAcc* acc) {
  GRec g{(u64*)gp.addr, gp.blin, gp.tli, gp.bw, gp.w, gp.item, gp.slot,
         (long long*)gp.part, gp.mult, (u64*)gp.lanes, (u64*)gp.skey};
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, st,
                     gp.item, (uint32_t)n, kEmpty);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, count, nitems, 0u);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((u64)nitems * 16, 256)), dim3(256),
                     0, st, (u64*)S, (u64)nitems * 16, 0ull);
  for (uint32_t off = 0; off < nchunks; off += 1u << 20) {
    uint32_t m = nchunks - off < (1u << 20) ? nchunks - off : (1u << 20);
    hipLaunchKernelGGL(k_gen_linear, dim3(m), dim3(256), 0, st, chunks + off,
                       fitems, (const DevInst*)insts, code, params, loopvals, g,
                       count, acc);
  }
  HGRD_CHECK(hipGetLastError());
  for (int L = 0; L < 12; ++L) {
    if (!((used_levels >> L) & 1)) continue;
    // levels 0-5 use table A, the synchronisation levels table B
    u64* ow = (u64*)(L < 6 ? owner : owner2);
    u64* ct = (u64*)(L < 6 ? cnt : cnt2);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(tbl, 256)), dim3(256), 0, st, ow, tbl,
                       ~0ull);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(tbl, 256)), dim3(256), 0, st, ct, tbl,
                       0ull);
    hipLaunchKernelGGL(k_ginsert, dim3(grid_for(n, kGTile)), dim3(256), 0, st, g,
                       n, L, fitems, ow, ct, tbl - 1, (u64*)S);
    // the thread levels are applied per lane by the finish kernel
    if (L != 5 && L != 11)
      hipLaunchKernelGGL(k_gpartner, dim3(grid_for(n, 256)), dim3(256), 0, st, g,
                         n, L, fitems, (const u64*)ct);
    HGRD_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_gfinish, dim3(grid_for(n, 256)), dim3(256), 0, st, g, n,
                     fitems, (const u64*)owner, (const u64*)cnt, (const u64*)owner2,
                     (const u64*)cnt2, tbl - 1, used_levels, acc);
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

int launch_level0(hipStream_t st, const Chunk* chunks, uint32_t n,
                  const L0Item* items, const void* insts, const DInsn* code,
                  const int64_t* params, const int64_t* loopvals, u64* keys,
                  u64* cnt, u64* s0) {
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL(k_level0, dim3(m), dim3(256), 0, st, chunks + off, items,
                       (const DevInst*)insts, code, params, loopvals, keys, cnt,
                       s0);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_apply_s0(hipStream_t st, uint32_t n, const L0Item* items,
                    const u64* s0, const uint32_t* skip, QAcc* acc) {
  if (!n) return 0;
  hipLaunchKernelGGL(k_apply_s0, dim3((n + 255) / 256), dim3(256), 0, st, n,
                     items, s0, skip, acc);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_fill_u64(hipStream_t st, u64* p, u64 n, u64 v) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

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
