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
  uint32_t* mult;  // points per record
  void* lanes;     // u64 per record: bit k = thread tlin + k of the record
  void* skey;      // i64 per record: synchronisation address (or null)
};

size_t devinst_size();
void fill_devinst(void* dst, const AccInst& a);
void set_devinst_tab(void* dst, const TabHost& t, const int64_t* pool);
int launch_tabulate(hipStream_t st, const Chunk* chunks, uint32_t n,
                    const TabJob* jobs, const void* insts, const DInsn* code,
                    const int64_t* params, const int64_t* loopvals, int64_t* pool);
int fastdiv_check(uint32_t n, uint32_t d);
void fastdiv_consts(uint32_t d, uint32_t* m, uint32_t* s);
int join_lds_bytes(int cfg);
int join_cap(int cfg);
size_t w2item_size();

int launch_small(int cfg, hipStream_t st, const SItem* items, uint32_t n,
                 const void* insts, const DInsn* code, const int64_t* params,
                 const int64_t* loopvals, const QDesc* qd, QAcc* acc,
                 const uint32_t* done, uint32_t* cursor, uint32_t persist_grid,
                 const IFact* facts);
// Writes every Chunk (runs = false) or BRun (runs = true) the specs
// describe (`total` in all, 16 bytes each) to `out`.
int launch_expand(hipStream_t st, const ExpandSpec* specs, uint32_t n, unsigned long long total,
                  bool runs, void* out);
int launch_unit_filter(hipStream_t st, uint32_t n, const HItem* hitems, const QDesc* qd,
                       const IFact* facts, uint32_t* ovf, unsigned long long* napart);
int init_kernel_attributes();
int init_verdict_attributes();
int launch_scatter(hipStream_t st, const Chunk* chunks, uint32_t n, bool tab,
                   const HItem* hitems, const void* insts, const DInsn* code,
                   const int64_t* params, const int64_t* loopvals, QAcc* acc,
                   unsigned char* recs, uint32_t* cursor,
                   uint32_t* ovf, uint32_t capb, const uint32_t* done,
                   unsigned long long* nbytes, hipEvent_t t0 = nullptr,
                   hipEvent_t t1 = nullptr);
int launch_bucket(int cfg, hipStream_t st, uint32_t nruns, const BRun* runs,
                  uint32_t n_tab, const HItem* hitems, const void* insts,
                  const DInsn* code, const int64_t* params, const int64_t* loopvals,
                  const QDesc* qd, QAcc* acc, const unsigned char* recs,
                  const uint32_t* cursor, const uint32_t* ovf, const uint32_t* done,
                  const unsigned long long* l0keys, const unsigned long long* l0cnt,
                  uint8_t* cand, unsigned long long* nbytes, const hipEvent_t* kev,
                  bool syn = false);
int launch_level0(hipStream_t st, const Chunk* chunks, uint32_t n,
                  const L0Item* items, const void* insts, const DInsn* code,
                  const int64_t* params, const int64_t* loopvals,
                  unsigned long long* keys, unsigned long long* cnt,
                  unsigned long long* s0);
int launch_apply_s0(hipStream_t st, uint32_t n, const L0Item* items,
                    const unsigned long long* s0, const uint32_t* skip,
                    QAcc* acc);
int launch_fallback(hipStream_t st, const Chunk* chunks, uint32_t nchunks,
                    const FItem* fitems, uint32_t nitems, uint32_t used_levels,
                    const void* insts, const DInsn* code, const int64_t* params,
                    const int64_t* loopvals, GRecPtrs gp, unsigned long long n,
                    uint32_t* count, void* owner, void* cnt, void* owner2,
                    void* cnt2,
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

int launch_fill_u64(hipStream_t st, unsigned long long* p, unsigned long long n,
                    unsigned long long v);

// VERDICT mode and the tile-scoring network (hgrd_verdict.hip)
int launch_block_bounds(hipStream_t st, const BItem* items, uint32_t n,
                        const void* insts, const DInsn* code,
                        const int64_t* params, const int64_t* loopvals,
                        QAcc* acc, BBound* out);
int launch_block_bounds_tab(hipStream_t st, const uint32_t* ilist, uint32_t ni,
                            const BItem* items, uint32_t n, const void* insts,
                            InstRange* ir, BBound* out);
int launch_vq_span(hipStream_t st, VQuery* vq, uint32_t n, const BBound* bb);
int launch_tile_scores(hipStream_t st, const TChunk* chunks, uint32_t n,
                       const VQuery* vq, const BBound* bb, const float* w,
                       uint32_t mode, float* scores);
int launch_tile_features(hipStream_t st, const TChunk* chunks, uint32_t n,
                         const VQuery* vq, const BBound* bb, float* feats);
// Tile order of every search unit (mode 1 network, 2 interval order):
// candidates are the tiles whose blocks' address ranges meet; K slots per
// unit in order[] (kNoTile when fewer).  max_g: the largest G of the units.
int launch_tile_rank(hipStream_t st, const VQuery* vq, uint32_t nvq, const BBound* bb,
                     const float* w, uint32_t mode, uint32_t K, uint32_t max_g,
                     const IFact* facts, const QDesc* qd, uint32_t* order);
int launch_topk(hipStream_t st, const VQuery* vq, uint32_t nvq,
                const float* scores, uint32_t K, uint32_t max_tiles,
                uint32_t* order);
int launch_tile_join(int cfg, hipStream_t st, const TItem* items, uint32_t item0,
                     uint32_t n, const VQuery* vq, const uint32_t* order,
                     uint32_t K, const void* insts, const DInsn* code,
                     const int64_t* params, const int64_t* loopvals,
                     const QDesc* qd, uint32_t* done, TOut* tout,
                     unsigned long long* claim, const BBound* bb,
                     const IFact* facts);
int launch_verdict_commit(hipStream_t st, uint32_t n,
                          const unsigned long long* claim, const TOut* tout,
                          QAcc* acc, uint32_t* done);
int launch_mlp_forward(hipStream_t st, const float* X, unsigned long long n,
                       const float* w, float* out);
int launch_mlp_grad(hipStream_t st, const float* X, const float* Y,
                    unsigned long long n, const float* w, float* grad,
                    float* loss);
int launch_adam(hipStream_t st, float* w, float* g, float* m, float* v,
                float lr, int t);
int mlp_num_weights();

// The fixed scratch area of rd_check_pairs_noalloc (hgrd_noalloc.cpp):
// looks up its device address on `device` (the current device) once and
// keeps it; nonzero when the lookup fails.
int noalloc_scratch_init(int device);
// The HIP device a context was created on.
int context_device(const rd_context* ctx);
// rd_check_pairs with every device buffer carved from [base, base + cap)
// (hgrd_host.cpp); RD_ECAPACITY when the batch needs more.
int check_pairs_in_arena(rd_context* ctx, void* base, size_t cap,
                         const rd_kernel_model* models, uint32_t n_models,
                         const rd_access_pair* pairs, uint32_t n_pairs,
                         const rd_launch_domain* launch, const rd_param_sets* params,
                         const rd_options* opt, rd_pair_result* out);

}  // namespace hgrd
