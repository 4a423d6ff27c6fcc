// Internal layouts shared by the host driver (hgrd_host.cpp) and the gfx950
// kernels (hgrd_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace hgrd {

// ---------------------------------------------------------------------------
// Device expression code.  The host compiles each postfix expression into
// three-address code over a register file of kMaxStack int64 slots (small
// enough to stay in VGPRs); every lane of a wavefront runs the same
// instruction stream (one access instance per wavefront), so dispatch is a
// uniform branch and register indices are uniform.  Operands are a stack
// register, an immediate, a parameter of the tuple (launch extents follow
// the parameters in the pool) or a point coordinate.
constexpr int kCoordTid = 0;   // tx, ty, tz
constexpr int kCoordBid = 3;   // bx, by, bz
constexpr int kCoordLoop = 6;  // loop values, position 0..3 in the access
constexpr int kNumCoords = 10;
constexpr int kMaxStack = 16;

enum DOp : uint8_t {
  D_MOV = 0, D_ADD, D_SUB, D_MUL, D_DIV, D_MOD, D_SHL, D_SHR, D_AND, D_OR,
  D_XOR, D_MIN, D_MAX, D_LT, D_LE, D_EQ, D_NE, D_GE, D_GT, D_LAND, D_LOR,
  D_NEG, D_LNOT
};
enum DMode : uint8_t { M_REG = 0, M_IMM = 1, M_PARAM = 2, M_COORD = 3 };

struct DInsn {
  uint8_t op, dst, ma, mb;  // opcode, destination register, operand modes
  uint16_t a, b;            // register / parameter / coordinate index
  int64_t imm;              // immediate operand (mode M_IMM)
};
static_assert(sizeof(DInsn) == 16, "DInsn layout");

// A compiled expression: `n` instructions at `off`; the value ends in
// register `res`.  absent != 0: no expression (the default value).
struct Prog {
  uint32_t off;
  uint16_t n;
  uint8_t res;
  uint8_t absent;
};

// Error bits (same meaning on host and device).
constexpr uint32_t ERR_DIVZERO = 1, ERR_RANGE = 2, ERR_UNSUP = 4, ERR_INVAL = 8;
// a tile received more records than planned (a library bug, never an input
// property); reported as RD_EDEVICE for the pair
constexpr uint32_t ERR_INTERNAL = 16;

// AccInst::syn flags: the access's acquire and release (section 6.5).
constexpr uint32_t kSynAcq = 1, kSynRel = 2, kSynAcqDev = 4, kSynRelDev = 8,
                   kSynSameArr = 16, kSynWrite = 32, kSynRead = 64,
                   kSynAcq32 = 128, kSynRel32 = 256;
// Pair synchronisation flags (FItem::sync, witness pass 2): an acquire or
// release on either access; points can share a syn() at block / device
// scope.
constexpr uint32_t kQSync = 1, kQSyncBlk = 2, kQSyncDev = 4;

// One access under one parameter tuple.
struct alignas(16) AccInst {
  Prog addr, guard, bint, wint;  // 32 B
  Prog acq, rel;                 // acquire / release addresses (absent: none)
  int32_t dims[6];               // gx gy gz bx by bz
  uint32_t nblk, nthr, niota;    // |grid|, |block|, |iterations|
  uint32_t n_loops;
  uint32_t loop_n[4];            // iteration counts per enclosing loop
  uint32_t loop_off[4];          // offsets into the loop-value pool
  uint32_t params_off;           // offset into the parameter pool
  uint32_t is32;                 // 32-bit array
  uint32_t npts;                 // nblk * nthr * niota (< 2^31)
  uint32_t tpb;                  // nthr * niota (points per block)
  uint32_t iorder;               // point order inside a block: 0 thread
                                 // fastest, 1 iteration fastest
  uint32_t syn;                  // kSyn* flags
};
static_assert(sizeof(AccInst) == 144, "AccInst layout");

// Term tables of one instance.  When an expression is proven free of
// errors over the whole launch box it is split into a uniform part and one
// term per coordinate group (blocks, threads, loop iterations), each
// tabulated over its group's linear index:
//   addr = u + T_B[blin] + T_T[tlin] + T_L[ilin]
// A table entry of INT64_MIN marks a group index at which a conjunct of
// the guard is false.  iv: (bint | wint << 16) per iteration, or constant.
constexpr uint32_t kNoTab = 0xFFFFFFFFu;
struct TabHost {
  int64_t u;
  unsigned long long base;  // first pool entry of this instance's tables
  uint32_t off[3];    // entry offsets from base per group, kNoTab = none
  uint32_t iv_off;    // kNoTab: iv_const for every iteration
  uint32_t iv_const;
  uint32_t never;     // a uniform guard conjunct is false
  uint32_t on;        // tables in use for this instance
  uint32_t syn_safe;  // acquire/release addresses proven error-free
};

// One table to fill: entries [0, n) of group `group` (0 blocks, 1 threads,
// 2 iterations, 3 packed interval ids over iterations) of instance `inst`.
struct TabJob {
  uint32_t inst, group, n, pad;
  unsigned long long out_off;  // first pool entry written
  Prog val, guard;  // value and guard-conjunct programs of the group
};
static_assert(sizeof(TabJob) == 40, "TabJob layout");

// Per-query description and accumulators.
struct QDesc {
  uint32_t mask;     // classes to check (bit 0 inter, 1 block, 2 warp)
  uint32_t self;     // access a == access b
  uint32_t warp;     // warp size of the analysed program
  uint32_t shared;   // shared-memory array
  uint32_t flags;    // bit 0: both accesses have one and the same block-
                     // barrier interval id in every tuple (the block level
                     // groups equal the (address, block) groups); bit 1: the
                     // same for the warp-barrier id; bit 2: both accesses
                     // compute their address with one expression; bits 3, 4:
                     // syn() of the two accesses can match at block / device
                     // scope (acquire/release, section 6.5)
};

struct QAcc {
  unsigned long long cnt[3];  // ordered pair counts per class
  unsigned long long pmin;    // smallest p key with a partner
  unsigned long long qmin;    // smallest q key for pmin (pass 2)
  unsigned int err;           // error bits seen on the device
  unsigned int qclass;        // class of the witness (pass 2)
  long long waddr;            // address of the witness
};

// A point key for the lexicographic witness order:
// set (12 bits) | blin (26) | tlin (10) | ilin (16).
__host__ __device__ inline unsigned long long pkey(uint32_t s, uint32_t b,
                                                   uint32_t t, uint32_t i) {
  return ((unsigned long long)s << 52) | ((unsigned long long)b << 26) |
         ((unsigned long long)t << 16) | (unsigned long long)i;
}
constexpr unsigned long long kNoKey = ~0ull;

// Facts about one access instance that its lowering proved (instances
// with term tables only): every address lies in [lo, hi] and is congruent
// to u modulo G (G = 0: every address equals u); inj: two points of
// different threads never share an address.  on = 0: nothing known.
struct IFact {
  long long lo, hi;
  unsigned long long G;
  long long u;
  uint32_t on, inj, pad[2];
};
static_assert(sizeof(IFact) == 48, "IFact layout");
// ovf mark of an HBM item whose two accesses share no address (decided by
// the unit filter at the start of an execute): nothing to partition.
constexpr uint32_t kApart = 0xFFFFFFFFu;

// Work item joined in one workgroup's LDS: both sides of query q under
// tuple `sigma`, blocks [b0, b1).
struct SItem {
  uint32_t q, sigma, inst_i, inst_j;
  uint32_t b0, b1;
  uint32_t mult;  // 0 or 1: as joined; k > 1: block 0 of k identical blocks
                  //   (its counts are taken k times)
  uint32_t gsym;  // 1: a global array's k identical blocks; the address-only
                  //   level also pairs block 0 with the other k - 1 blocks
};

// Work item partitioned through HBM.
struct HItem {
  uint32_t q, sigma, inst_i, inst_j;
  uint32_t nbuckets;      // number of buckets
  uint32_t bucket0;       // first global bucket index
  uint32_t shared;        // hash (addr, blin) instead of addr
  uint32_t is32;          // 32-bit keys
  unsigned long long rec_off;  // byte offset of bucket 0's records
  uint32_t tpb_m[2];           // points per block of side a, b as fast-division
                               // multipliers (block of a point = pidx / tpb)
  unsigned long long l0_off;   // mode 3: the item's address-count table
  uint32_t l0_mask;            //   (slots l0_off .. l0_off + l0_mask + 1)
  uint32_t shift;              // buckets see address >> shift (blocks of
                               // 2^shift consecutive addresses stay together)
  // Bucket map.  mode 0: a hash of the key.  mode 1: the key
  //   k = ((addr - lo) >> shift) + blin * kb   (below 2^32 by construction)
  // modulo nbuckets (a prime), so a dense key range fills the buckets
  // evenly whatever the group sizes; fm = floor(2^64 / nbuckets) + 1.
  uint32_t mode, kb;
  long long lo;
  unsigned long long fm;
  uint32_t tpb_s[2];           // and shifts
  // gmult = G > 1: block 0 of a global array's G identical blocks (no block
  // term in either access); only block 0's points are generated, the
  // address-only level stands for G groups and every count is taken G times
  uint32_t gmult;
  uint32_t sync;  // 1: a pair with acquire/release (joined with the
                  //   synchronisation levels; never split, overflow to the
                  //   fallback)
  uint32_t dense; // 1: both accesses put several points on an address on
                  //   average: the address filter would pass nearly every
                  //   bucket, so it passes them all without reading them
  uint32_t pad_;
};
static_assert(sizeof(HItem) == 112, "HItem layout");
// A run of buckets [b0, b1) of one HBM item, joined by one workgroup.
constexpr uint32_t kMaxRunBuckets = 64;  // buckets per join workgroup at most
struct BRun {
  uint32_t item, b0, b1, pad;
};

// Records: int32 keys as one u64 (address | point id << 32), int64 keys as
// 16 bytes (address, point id); point id = side << 31 | point index.
// HItem.shared: 0 global (hash of the address), 1 shared array (hash of
// address and block), 2 error scan only (never joined), 3 global item split
// by (address, block) with its level 0 counted in an address-count table.

// An item whose level 0 is counted in an address-count table: slots
// [off, off + mask + 1) hold (address, n_a | n_b << 32), slot off + mask + 1
// the address INT64_MIN (the empty-slot marker).
struct L0Item {
  uint32_t q, inst_i, inst_j, self;
  unsigned long long off;
  uint32_t mask, qmask;
};
constexpr unsigned long long kL0Empty = 0x8000000000000000ull;

// A query/tuple aggregated in HBM (fallback for heavy keys): its records
// occupy [off, off + cap) of the flat record arrays.
struct FItem {
  uint32_t q, sigma, inst_i, inst_j;
  uint32_t self, mask, warp, cap;
  unsigned long long off;
  uint32_t sync;   // kQSync* flags of the pair
  uint32_t gmult;  // as HItem::gmult
};

// A slice of one side's points, generated and scattered by one workgroup.
struct Chunk {
  uint32_t item, side;
  uint32_t p0, p1;  // point index range
};

// Compact description of consecutive chunks or bucket runs: [0, n) (points
// of one side, or buckets of one item) cut into pieces of `per`, which
// become entries first, first + 1, ... of the Chunk (item, side, p0, p1)
// or BRun (item, b0, b1) array.
struct ExpandSpec {
  uint32_t item, side, n, per;
  unsigned long long first;
};
static_assert(sizeof(ExpandSpec) == 24, "ExpandSpec layout");

// ---- VERDICT mode (learned tile order) --------------------------------------

// Block-bounds work item: block `block` of access instance `inst` (query q);
// its bounds go to BBound `out`.
struct BItem {
  uint32_t inst, block, q, out;
};
// Address bounds of the thread and iteration term tables of an instance:
// smallest and largest valid entry and the number of valid entries (an
// absent table counts as one entry of value 0 per thread or iteration).
struct InstRange {
  long long tmin, tmax, imin, imax;
  uint32_t tcnt, icnt;
};
// Smallest and largest address of a block's guarded points, and their number.
struct BBound {
  long long mn, mx;
  uint32_t cnt, pad;
};
// One search unit: a query under one tuple, with G blocks per side; its
// tiles are (b1, b2) in [0, G)^2, tile index b1 * G + b2.
struct VQuery {
  uint32_t q, sigma, inst_i, inst_j;
  uint32_t G, bb_i, bb_j, self;   // bb_*: first BBound of each side
  uint32_t tile0, tpb_i, tpb_j, nthr;
  uint32_t kinds, shared, is64, nsets;
  long long amin, amax;           // address span over both sides
  long long st_i, sb_i, st_j, sb_j;  // address step per thread and per
                                     // block of each side (0: unknown)
};
// Tiles [t0, t1) of search unit vq (scores / features).
struct TChunk {
  uint32_t vq, t0, t1, pad;
};
// One tile to search: the rank-th tile of search unit vq in its order.
struct TItem {
  uint32_t vq, rank;
};
// Result of a conflicting tile.
struct TOut {
  unsigned long long cnt[3];
  unsigned long long pkey, qkey;
  long long addr;
};

}  // namespace hgrd
