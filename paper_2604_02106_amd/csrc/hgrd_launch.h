// Launch wrappers exported by hgrd_kernels.hip to the host driver.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime.h>
#include "hgrd_internal.h"
#include "../../include/hgrd.h"

namespace hgrd {

struct GRecPtrs {
  void* addr;
  uint32_t* blin;
  uint32_t* tli;
  uint32_t* bw;
  uint32_t* w;
  uint32_t* item;
  uint32_t* slot;
  void* part;
};

size_t devinst_size();
void fill_devinst(void* dst, const AccInst& a);
int fastdiv_check(uint32_t n, uint32_t d);
int join_lds_bytes(int cfg);
int join_cap(int cfg);
size_t w2item_size();

int launch_small(int cfg, hipStream_t st, const SItem* items, uint32_t n,
                 const void* insts, const DInsn* code, const int64_t* params,
                 const int64_t* loopvals, const QDesc* qd, QAcc* acc);
int launch_scatter(hipStream_t st, const Chunk* chunks, uint32_t n,
                   const HItem* hitems, const void* insts, const DInsn* code,
                   const int64_t* params, const int64_t* loopvals, QAcc* acc,
                   unsigned char* keys, uint32_t* pids, uint32_t* cursor,
                   uint32_t* ovf, uint32_t capb);
int launch_bucket(int cfg, hipStream_t st, uint32_t nb, uint32_t base,
                  const uint32_t* bucket_item, const HItem* hitems,
                  const void* insts, const DInsn* code, const int64_t* params,
                  const int64_t* loopvals, const QDesc* qd, QAcc* acc,
                  const unsigned char* keys, const uint32_t* pids,
                  const uint32_t* cursor, const uint32_t* ovf);
int launch_fallback(hipStream_t st, const Chunk* chunks, uint32_t nchunks,
                    const FItem* fitems, uint32_t nitems, uint32_t used_levels,
                    const void* insts, const DInsn* code, const int64_t* params,
                    const int64_t* loopvals, GRecPtrs gp, unsigned long long n,
                    uint32_t* count, uint32_t* owner, void* cnt,
                    unsigned long long tbl, void* S, QAcc* acc);
int launch_witness2(hipStream_t st, const void* items, uint32_t n,
                    const void* insts, const DInsn* code, const int64_t* params,
                    const int64_t* loopvals, const QDesc* qd, QAcc* acc);
int launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t n, uint32_t v);
int launch_init_acc(hipStream_t st, uint32_t n, QAcc* acc);
int launch_finalize(hipStream_t st, uint32_t n, const QAcc* acc,
                    const QDesc* qd, const uint32_t* host_err,
                    const uint8_t* trivial, const unsigned long long* evals,
                    rd_pair_result* out);

}  // namespace hgrd
