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
#include "hgrd_lower.h"


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
  rd_context_destroy(ctx->aux);
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
  // Dense items first: nearly all their buckets go on to the join, so the
  // heavy join work fills the first waves' launches instead of thinning out
  // over every wave (measured: join time per step 336 against 340 ms).
  std::stable_sort(hplans.begin(), hplans.end(),
                   [](const HPlan& x, const HPlan& y) { return x.h.dense > y.h.dense; });
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
  // copies on the plan's stream, finished before the source may go (the
  // null stream would also wait for other contexts' work on the device)
  auto up = [&](const char* name, const void* src, size_t bytes) -> void* {
    void* d = plan->buf(name, bytes, &merr);
    if (d && bytes &&
        (hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, plan->st) != hipSuccess ||
         hipStreamSynchronize(plan->st) != hipSuccess))
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
    TRY_HIP(hipMemcpyAsync(written.data(), gcount, nf * 4, hipMemcpyDeviceToHost, st));
    TRY_HIP(hipStreamSynchronize(st));
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

// More pairs than one batch: consecutive batches of pairs, each prepared
// and executed as a plan of its own (a pair's result does not depend on
// the other pairs of its plan).  Batch k + 1 is prepared on a host thread,
// on a second context of the same device that ctx keeps, while batch k
// executes: the host lowering and the descriptor uploads of one batch
// overlap the device work of the other, and each context serves one
// thread at a time.  The stats are the sums over the batches, total_ms
// the whole call.
int rd_check_pairs(rd_context* ctx, const rd_kernel_model* models,
                   uint32_t n_models, const rd_access_pair* pairs,
                   uint32_t n_pairs, const rd_launch_domain* launch,
                   const rd_param_sets* params, const rd_options* opt,
                   rd_pair_result* out) {
  if (!ctx) return RD_EINVAL;
  if (n_pairs && !out) return RD_EINVAL;
  uint64_t B = kBatchPairs;
  if (const char* e = getenv("HGRD_BATCH_PAIRS")) B = strtoull(e, nullptr, 10);
  // (a second context that cannot be created leaves one plan for all)
  if (B && n_pairs > B && !ctx->arena && !(opt && opt->stream) && pairs && !ctx->aux &&
      rd_context_create(&ctx->aux, ctx->device) != RD_OK)
    ctx->aux = nullptr;
  if (B == 0 || n_pairs <= B || ctx->arena || (opt && opt->stream) || !pairs || !ctx->aux) {
    rd_plan* plan = nullptr;
    int rc = rd_prepare(ctx, models, n_models, pairs, n_pairs, launch, params, opt, &plan);
    if (rc != RD_OK) return rc;
    rc = rd_execute(ctx, plan, out);
    rd_plan_destroy(plan);
    return rc;
  }
  const double t0 = now_ms();
  ctx->aux->cfg = ctx->cfg;
  ctx->aux->wave_bytes = ctx->wave_bytes;
  rd_context* C[2] = {ctx, ctx->aux};
  rd_stats total;
  memset(&total, 0, sizeof total);
  const uint32_t nb = (uint32_t)((n_pairs + B - 1) / B);
  auto count = [&](uint32_t k) { return (uint32_t)std::min<uint64_t>(B, n_pairs - k * B); };
  rd_plan* cur = nullptr;
  int rc = rd_prepare(C[0], models, n_models, pairs, count(0), launch, params, opt, &cur);
  for (uint32_t k = 0; rc == RD_OK && k < nb; ++k) {
    rd_plan* next = nullptr;
    int rc_next = RD_OK;
    auto prep_next = [&, k] {
      rc_next = rd_prepare(C[(k + 1) & 1], models, n_models, pairs + (k + 1) * B, count(k + 1),
                           launch, params, opt, &next);
    };
    std::thread th;
    if (k + 1 < nb) {
      try {
        th = std::thread(prep_next);
      } catch (...) {
        // no host thread: the next batch is prepared after this one runs
      }
    }
    rc = rd_execute(C[k & 1], cur, out + k * B);
    add_stats(total, C[k & 1]->stats);
    rd_plan_destroy(cur);
    if (th.joinable()) th.join();
    else if (k + 1 < nb && rc == RD_OK) prep_next();
    if (rc == RD_OK) rc = rc_next;
    cur = next;
  }
  if (cur) rd_plan_destroy(cur);
  total.total_ms = now_ms() - t0;
  ctx->stats = total;
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
