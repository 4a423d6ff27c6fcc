// Host entry points around the race query: rd_autotune (tile shape and
// wave size of a context), rd_tile_data (tile features and labels for the
// scorer), the scorer's forward, gradient and training calls, and the
// host self-tests of term tables, pre-filters and division constants.
#include "hgrd_lower.h"


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
