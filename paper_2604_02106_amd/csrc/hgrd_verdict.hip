// VERDICT mode with a learned block-pair tile order, and the kernels that
// train the tile-scoring network.
//
// A tile is one block b1 of access a against one block b2 of access b under
// one parameter tuple; every conflict of a query lies in exactly one tile.
// VERDICT mode searches tiles in the order of a score and stops a query at
// its first conflicting tile; a query with no conflict among its searched
// tiles goes through the exact path (race freedom needs every point).  The
// score is either the tile index (LEX) or the output of a small network over
// 32 tile features (MLP), trained on tile labels the exact checker produces.
// Nothing here changes EXACT results.
//
// Network: 32 -> 64 -> 64 -> 1, ReLU, fp32, binary cross-entropy on logits.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include "hgrd_device.h"
#include "hgrd_launch.h"

namespace hgrd {

using u64 = unsigned long long;

// ---------------------------------------------------------------------------
// Per-block address bounds of one access instance: min, max and the number
// of points whose guard holds.  Also records evaluation errors, so VERDICT
// mode reports the same statuses as EXACT.

__global__ void __launch_bounds__(256)
k_block_bounds(const BItem* __restrict__ items, const DevInst* __restrict__ insts,
               const DInsn* __restrict__ code, const int64_t* __restrict__ params,
               const int64_t* __restrict__ loopvals, QAcc* __restrict__ acc,
               BBound* __restrict__ out) {
  const BItem it = items[blockIdx.x];
  DevInst I;
  load_inst(I, insts, it.inst);
  __shared__ long long smn[4], smx[4];
  __shared__ uint32_t scnt[4], serr[4];
  long long mn = INT64_MAX, mx = INT64_MIN;
  uint32_t cnt = 0, err = 0;
  const uint32_t p0 = it.block * I.a.tpb, p1 = p0 + I.a.tpb;
  for (uint32_t base = p0; base < p1; base += blockDim.x) {
    uint32_t pidx = base + threadIdx.x;
    if (pidx >= p1) break;
    PointIds id = decode(I, pidx);
    Point pt;
    if (!point_eval(I, id, code, params, loopvals, pt, err)) continue;
    mn = pt.addr < mn ? pt.addr : mn;
    mx = pt.addr > mx ? pt.addr : mx;
    ++cnt;
  }
  for (int o = 32; o > 0; o >>= 1) {
    long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
    cnt += __shfl_xor(cnt, o, 64);
    err |= __shfl_xor(err, o, 64);
  }
  const uint32_t w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smn[w] = mn;
    smx[w] = mx;
    scnt[w] = cnt;
    serr[w] = err;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t k = 1; k < (blockDim.x >> 6); ++k) {
      mn = smn[k] < mn ? smn[k] : mn;
      mx = smx[k] > mx ? smx[k] : mx;
      cnt += scnt[k];
      err |= serr[k];
    }
    BBound b;
    b.mn = mn;
    b.mx = mx;
    b.cnt = cnt;
    b.pad = 0;
    out[it.out] = b;
    if (err) atomicOr(&acc[it.q].err, err);
  }
}

// Bounds of the thread and iteration term tables of one instance (one
// workgroup per instance).
__global__ void __launch_bounds__(256)
k_inst_ranges(const uint32_t* __restrict__ list, const DevInst* __restrict__ insts,
              InstRange* __restrict__ out) {
  const uint32_t x = list[blockIdx.x];
  DevInst I;
  load_inst(I, insts, x);
  __shared__ long long smn[4], smx[4];
  __shared__ uint32_t scnt[4];
  InstRange r;
  for (int g = 1; g <= 2; ++g) {
    const uint32_t n = g == 1 ? I.a.nthr : I.a.niota;
    long long mn = INT64_MAX, mx = INT64_MIN;
    uint32_t cnt = 0;
    if (I.toff[g] == kNoTab) {
      mn = mx = 0;
      cnt = threadIdx.x == 0 ? n : 0;
    } else {
      for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) {
        const long long v = I.tpool[I.toff[g] + e];
        if (v == INT64_MIN) continue;  // a guard conjunct of this group fails
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
        ++cnt;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
      cnt += __shfl_xor(cnt, o, 64);
    }
    const uint32_t w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      smn[w] = mn;
      smx[w] = mx;
      scnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (uint32_t k = 1; k < (blockDim.x >> 6); ++k) {
        mn = smn[k] < mn ? smn[k] : mn;
        mx = smx[k] > mx ? smx[k] : mx;
        cnt += scnt[k];
      }
      if (g == 1) { r.tmin = mn; r.tmax = mx; r.tcnt = cnt; }
      else { r.imin = mn; r.imax = mx; r.icnt = cnt; }
    }
  }
  if (threadIdx.x == 0) out[x] = r;
}

// Block bounds of instances with term tables, one lane per block: the
// address is u + T_B[b] + T_T[t] + T_L[i] over the valid entries of each
// table, so a block's smallest (largest) address is its block term plus the
// smallest (largest) thread and iteration terms, and its point count the
// product of the valid entries (no point of a table instance can fail, so
// there is no error to record).  Items of interpreted instances are left
// to k_block_bounds.
__global__ void __launch_bounds__(256)
k_block_bounds_tab(const BItem* __restrict__ items, uint32_t n,
                   const DevInst* __restrict__ insts, const InstRange* __restrict__ ir,
                   BBound* __restrict__ out) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const BItem it = items[k];
  const DevInst& I = insts[it.inst];
  if (!I.tab) return;
  const InstRange r = ir[it.inst];
  BBound b;
  b.mn = 0;
  b.mx = 0;
  b.cnt = 0;
  b.pad = 0;
  const long long vb = I.toff[0] != kNoTab ? I.tpool[I.toff[0] + it.block] : 0;
  if (!I.tnever && vb != INT64_MIN && r.tcnt && r.icnt) {
    b.mn = I.tu + vb + r.tmin + r.imin;
    b.mx = I.tu + vb + r.tmax + r.imax;
    b.cnt = r.tcnt * r.icnt;
  } else {
    b.mn = INT64_MAX;
    b.mx = INT64_MIN;
  }
  out[it.out] = b;
}

// Span of a search unit: the smallest and largest address over both sides.
__global__ void __launch_bounds__(256)
k_vq_span(VQuery* __restrict__ vq, uint32_t n, const BBound* __restrict__ bb) {
  uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  VQuery v = vq[k];
  long long mn = INT64_MAX, mx = INT64_MIN;
  for (uint32_t b = 0; b < v.G; ++b) {
    const BBound x = bb[v.bb_i + b], y = bb[v.bb_j + b];
    if (x.cnt) { mn = x.mn < mn ? x.mn : mn; mx = x.mx > mx ? x.mx : mx; }
    if (y.cnt) { mn = y.mn < mn ? y.mn : mn; mx = y.mx > mx ? y.mx : mx; }
  }
  if (mn > mx) { mn = 0; mx = 0; }
  vq[k].amin = mn;
  vq[k].amax = mx;
}

// ---------------------------------------------------------------------------
// 32 tile features (all in [-1, 1] or small positive values).

__device__ __forceinline__ float flog2p(double x) { return (float)(log2(1.0 + x) / 64.0); }
// sign(x) log2(1 + |x|) / 32
__device__ __forceinline__ float slog(long long x) {
  const double a = x < 0 ? -(double)x : (double)x;
  const float m = (float)(log2(1.0 + a) / 32.0);
  return x < 0 ? -m : m;
}

__device__ void tile_features(const VQuery& v, uint32_t b1, uint32_t b2,
                              const BBound& x, const BBound& y, float* f) {
  const double span = (double)v.amax - (double)v.amin + 1.0;
  const double G = (double)v.G;
  const bool ex = x.cnt > 0, ey = y.cnt > 0;
  double lo = ex && ey ? fmax((double)x.mn, (double)y.mn) : 0;
  double hi = ex && ey ? fmin((double)x.mx, (double)y.mx) : -1;
  double ov = ex && ey && hi >= lo ? hi - lo + 1 : 0;
  double gap = ex && ey && hi < lo ? lo - hi : 0;
  double ext1 = ex ? (double)x.mx - (double)x.mn + 1 : 0;
  double ext2 = ey ? (double)y.mx - (double)y.mn + 1 : 0;
  double c1 = ex ? 0.5 * ((double)x.mn + (double)x.mx) : 0;
  double c2 = ey ? 0.5 * ((double)y.mn + (double)y.mx) : 0;
  f[0] = (float)(b1 / G);
  f[1] = (float)(b2 / G);
  f[2] = (float)(fabs((double)b1 - (double)b2) / G);
  f[3] = b1 == b2 ? 1.f : 0.f;
  f[4] = (float)(ov / span);
  f[5] = (float)(gap / span);
  f[6] = (float)(fabs(c1 - c2) / span);
  f[7] = ov > 0 ? 1.f : 0.f;
  f[8] = flog2p(ov);
  f[9] = flog2p(gap);
  f[10] = (float)(ext1 / span);
  f[11] = (float)(ext2 / span);
  f[12] = (float)x.cnt / (float)v.tpb_i;
  f[13] = (float)y.cnt / (float)v.tpb_j;
  f[14] = (!ex || !ey) ? 1.f : 0.f;
  f[15] = (float)(log2(G) / 26.0);
  f[16] = (float)(log2((double)v.nthr) / 10.0);
  f[17] = (float)(log2((double)v.tpb_i / v.nthr + 1.0) / 16.0);
  f[18] = v.self ? 1.f : 0.f;
  f[19] = (float)v.kinds / 8.f;
  // address steps per thread and per block of each side (sign and log)
  f[20] = slog(v.st_i);
  f[21] = slog(v.st_j);
  f[22] = ex && ey ? (float)(((double)x.mn - (double)y.mn) / span) : 0.f;
  f[23] = ex && ey ? (float)(((double)x.mx - (double)y.mx) / span) : 0.f;
  f[24] = ext1 > 0 ? (float)(x.cnt / ext1) : 0.f;
  f[25] = ext2 > 0 ? (float)(y.cnt / ext2) : 0.f;
  f[26] = slog(v.sb_i);
  f[27] = ext1 > 0 ? (float)(ov / ext1) : 0.f;
  f[28] = ext2 > 0 ? (float)(ov / ext2) : 0.f;
  f[29] = ex && ey ? (x.mn < y.mn ? -1.f : (x.mn > y.mn ? 1.f : 0.f)) : 0.f;
  f[30] = slog(v.sb_j);
  f[31] = (v.st_i == v.st_j && v.sb_i == v.sb_j) ? 1.f : 0.f;
}

// ---------------------------------------------------------------------------
// Network evaluation.  Weights (6337 floats) are staged in LDS per
// workgroup; each lane scores one sample.

constexpr int kIn = 32, kHid = 64;
constexpr int kW1 = 0, kB1 = kW1 + kHid * kIn, kW2 = kB1 + kHid,
              kB2 = kW2 + kHid * kHid, kW3 = kB2 + kHid, kB3 = kW3 + kHid,
              kNW = kB3 + 1;

__device__ __forceinline__ float mlp_logit(const float* __restrict__ W,
                                           const float* x) {
  float h1[kHid];
#pragma unroll 4
  for (int o = 0; o < kHid; ++o) {
    float a = W[kB1 + o];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a = fmaf(W[kW1 + o * kIn + i], x[i], a);
    h1[o] = a > 0.f ? a : 0.f;
  }
  float z = W[kB3];
  for (int o = 0; o < kHid; ++o) {
    float a = W[kB2 + o];
#pragma unroll
    for (int i = 0; i < kHid; ++i) a = fmaf(W[kW2 + o * kHid + i], h1[i], a);
    z = fmaf(W[kW3 + o], a > 0.f ? a : 0.f, z);
  }
  return z;
}

__device__ __forceinline__ void stage_weights(float* sw, const float* __restrict__ w) {
  for (int k = threadIdx.x; k < kNW; k += blockDim.x) sw[k] = w[k];
  __syncthreads();
}

// Scores of every tile of every search unit.  mode 1 (network): the
// network's logit; mode 2 (interval order): minus the tile index; in both,
// tiles whose blocks' address ranges are disjoint (no conflict possible)
// score -inf, last in order.  mode 0 (plain order): minus the index.
__global__ void __launch_bounds__(256)
k_tile_scores(const TChunk* __restrict__ chunks, const VQuery* __restrict__ vq,
              const BBound* __restrict__ bb, const float* __restrict__ w,
              uint32_t mode, float* __restrict__ scores) {
  __shared__ float sw[kNW];
  if (mode == 1) stage_weights(sw, w);
  const TChunk ch = chunks[blockIdx.x];
  const VQuery v = vq[ch.vq];
  for (uint32_t t = ch.t0 + threadIdx.x; t < ch.t1; t += blockDim.x) {
    float s = -(float)t;
    if (mode != 0) {
      uint32_t b1 = t / v.G, b2 = t - b1 * v.G;
      const BBound x = bb[v.bb_i + b1], y = bb[v.bb_j + b2];
      if (!x.cnt || !y.cnt || x.mx < y.mn || y.mx < x.mn) {
        s = -INFINITY;
      } else if (mode == 1) {
        float f[kIn];
        tile_features(v, b1, b2, x, y, f);
        s = mlp_logit(sw, f);
      }
    }
    scores[v.tile0 + t] = s;
  }
}

// Features of every tile (for training and tests).
__global__ void __launch_bounds__(256)
k_tile_features(const TChunk* __restrict__ chunks, const VQuery* __restrict__ vq,
                const BBound* __restrict__ bb, float* __restrict__ feats) {
  const TChunk ch = chunks[blockIdx.x];
  const VQuery v = vq[ch.vq];
  for (uint32_t t = ch.t0 + threadIdx.x; t < ch.t1; t += blockDim.x) {
    uint32_t b1 = t / v.G, b2 = t - b1 * v.G;
    float f[kIn];
    tile_features(v, b1, b2, bb[v.bb_i + b1], bb[v.bb_j + b2], f);
    float* o = feats + (u64)(v.tile0 + t) * kIn;
#pragma unroll
    for (int i = 0; i < kIn; ++i) o[i] = f[i];
  }
}

// Logits of n feature rows.
__global__ void __launch_bounds__(256)
k_mlp_forward(const float* __restrict__ X, u64 n, const float* __restrict__ w,
              float* __restrict__ out) {
  __shared__ float sw[kNW];
  stage_weights(sw, w);
  for (u64 k = (u64)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (u64)gridDim.x * blockDim.x) {
    float x[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) x[i] = X[k * kIn + i];
    out[k] = mlp_logit(sw, x);
  }
}

// Loss and gradient of the mean binary cross-entropy over n rows.  Each lane
// runs forward and backward for one row; gradients are summed in LDS, then
// added to `grad` (kNW floats) once per workgroup.  `scale` = 1/n.
__global__ void __launch_bounds__(256)
k_mlp_grad(const float* __restrict__ X, const float* __restrict__ Y, u64 n,
           const float* __restrict__ w, float scale, float* __restrict__ grad,
           float* __restrict__ loss) {
  __shared__ float sw[kNW];
  __shared__ float sg[kNW];
  for (int k = threadIdx.x; k < kNW; k += blockDim.x) sg[k] = 0.f;
  stage_weights(sw, w);
  float lsum = 0.f;
  for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (u64)gridDim.x * blockDim.x) {
    float x[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) x[i] = X[r * kIn + i];
    float h1[kHid], a2[kHid];
    for (int o = 0; o < kHid; ++o) {
      float a = sw[kB1 + o];
#pragma unroll
      for (int i = 0; i < kIn; ++i) a = fmaf(sw[kW1 + o * kIn + i], x[i], a);
      h1[o] = a > 0.f ? a : 0.f;
    }
    float z = sw[kB3];
    for (int o = 0; o < kHid; ++o) {
      float a = sw[kB2 + o];
#pragma unroll
      for (int i = 0; i < kHid; ++i) a = fmaf(sw[kW2 + o * kHid + i], h1[i], a);
      a2[o] = a;
      z = fmaf(sw[kW3 + o], a > 0.f ? a : 0.f, z);
    }
    const float y = Y[r];
    // loss = max(z,0) - z y + log(1 + exp(-|z|)); dL/dz = sigmoid(z) - y
    lsum += fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)));
    const float dz = (1.f / (1.f + expf(-z)) - y) * scale;
    atomicAdd(&sg[kB3], dz);
    float dh1[kHid];
#pragma unroll
    for (int i = 0; i < kHid; ++i) dh1[i] = 0.f;
    for (int o = 0; o < kHid; ++o) {
      const float h2 = a2[o] > 0.f ? a2[o] : 0.f;
      atomicAdd(&sg[kW3 + o], dz * h2);
      if (a2[o] <= 0.f) continue;
      const float da2 = dz * sw[kW3 + o];
      atomicAdd(&sg[kB2 + o], da2);
      for (int i = 0; i < kHid; ++i) {
        if (h1[i] != 0.f) atomicAdd(&sg[kW2 + o * kHid + i], da2 * h1[i]);
        dh1[i] = fmaf(da2, sw[kW2 + o * kHid + i], dh1[i]);
      }
    }
    for (int o = 0; o < kHid; ++o) {
      if (h1[o] <= 0.f) continue;
      const float da1 = dh1[o];
      atomicAdd(&sg[kB1 + o], da1);
      for (int i = 0; i < kIn; ++i)
        if (x[i] != 0.f) atomicAdd(&sg[kW1 + o * kIn + i], da1 * x[i]);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kNW; k += blockDim.x)
    if (sg[k] != 0.f) atomicAdd(&grad[k], sg[k]);
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, lsum * scale);
}

// Adam update of the weights with the accumulated gradient; clears it.
__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ w, float* __restrict__ g, float* __restrict__ m,
       float* __restrict__ v, float lr, float b1, float b2, float eps,
       float c1, float c2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNW) return;
  float gk = g[k];
  float mk = b1 * m[k] + (1.f - b1) * gk;
  float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  g[k] = 0.f;
}

// ---------------------------------------------------------------------------
// Search order: the `K` best tiles of each search unit by (score desc,
// index asc).  The tiles with a finite score (ranges that meet) are
// gathered in LDS, sorted by a bitonic network, and the first K written;
// the rest of the K ranks take the -inf tiles in index order.  More finite
// tiles than the LDS holds: K rounds of a workgroup arg-max, each below
// the previous pick in that order.
constexpr uint32_t kTopCap = 4096;

__device__ __forceinline__ bool tile_before(float sa, uint32_t ia, float sb, uint32_t ib) {
  return sa > sb || (sa == sb && ia < ib);
}

__global__ void __launch_bounds__(256)
k_topk(const VQuery* __restrict__ vq, const float* __restrict__ scores,
       uint32_t K, uint32_t* __restrict__ order) {
  __shared__ float ks[kTopCap];
  __shared__ uint32_t ki[kTopCap];
  __shared__ uint32_t cnt, base;
  __shared__ float bs[4];
  __shared__ uint32_t bi[4];
  const VQuery v = vq[blockIdx.x];
  const uint32_t nt = v.G * v.G;
  const uint32_t kk = K < nt ? K : nt;
  const float* sc = scores + v.tile0;
  uint32_t* out = order + (u64)blockIdx.x * K;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) {
    const float s = sc[t];
    if (s == -INFINITY) continue;
    const uint32_t p = atomicAdd(&cnt, 1u);
    if (p < kTopCap) {
      ks[p] = s;
      ki[p] = t;
    }
  }
  __syncthreads();
  const uint32_t c = cnt;
  uint32_t nfin;
  if (c <= kTopCap) {
    uint32_t P = 1;
    while (P < c) P <<= 1;
    for (uint32_t k = c + threadIdx.x; k < P; k += blockDim.x) {
      ks[k] = -INFINITY;
      ki[k] = 0xFFFFFFFFu;
    }
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
        for (uint32_t k = threadIdx.x; k < P; k += blockDim.x) {
          const uint32_t j = k ^ stride;
          if (j <= k) continue;
          const bool up = (k & size) == 0;  // this run is sorted "before first"
          const bool jb = tile_before(ks[j], ki[j], ks[k], ki[k]);
          if (jb == up) {
            const float ts = ks[k];
            const uint32_t ti = ki[k];
            ks[k] = ks[j];
            ki[k] = ki[j];
            ks[j] = ts;
            ki[j] = ti;
          }
        }
        __syncthreads();
      }
    }
    nfin = c < kk ? c : kk;
    for (uint32_t r = threadIdx.x; r < nfin; r += blockDim.x) out[r] = ki[r];
  } else {
    // K rounds of arg-max below the previous pick
    float ps = INFINITY;
    uint32_t pi = 0;
    bool first = true;
    nfin = 0;
    for (uint32_t r = 0; r < kk; ++r) {
      float best = -INFINITY;
      uint32_t bidx = 0xFFFFFFFFu;
      for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) {
        const float s = sc[t];
        if (s == -INFINITY) continue;
        if (!first && !tile_before(ps, pi, s, t)) continue;
        if (bidx == 0xFFFFFFFFu || tile_before(s, t, best, bidx)) { best = s; bidx = t; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const float s2 = __shfl_xor(best, o, 64);
        const uint32_t i2 = __shfl_xor(bidx, o, 64);
        if (i2 != 0xFFFFFFFFu && (bidx == 0xFFFFFFFFu || tile_before(s2, i2, best, bidx))) {
          best = s2;
          bidx = i2;
        }
      }
      const uint32_t w = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) { bs[w] = best; bi[w] = bidx; }
      __syncthreads();
      if (threadIdx.x == 0) {
        for (uint32_t k = 1; k < (blockDim.x >> 6); ++k)
          if (bi[k] != 0xFFFFFFFFu && (bidx == 0xFFFFFFFFu || tile_before(bs[k], bi[k], best, bidx))) {
            best = bs[k];
            bidx = bi[k];
          }
        bs[0] = best;
        bi[0] = bidx;
        if (bidx != 0xFFFFFFFFu) out[r] = bidx;
      }
      __syncthreads();
      if (bi[0] == 0xFFFFFFFFu) break;
      ps = bs[0];
      pi = bi[0];
      first = false;
      nfin = r + 1;
      __syncthreads();
    }
  }
  // the remaining ranks: -inf tiles in index order
  if (threadIdx.x == 0) base = nfin;
  __syncthreads();
  for (uint32_t t0 = 0; t0 < nt; t0 += blockDim.x) {
    if (base >= kk) break;
    const uint32_t t = t0 + threadIdx.x;
    const bool inf = t < nt && sc[t] == -INFINITY;
    // rank of this tile among the -inf tiles of the chunk
    const u64 bal = __ballot(inf);
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) bi[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < w; ++k) before += bi[k];
    const uint32_t pos = base + before + (uint32_t)__popcll(bal & ((1ull << lane) - 1));
    if (inf && pos < kk) out[pos] = t;
    __syncthreads();
    if (threadIdx.x == 0) base += bi[0] + bi[1] + bi[2] + bi[3];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Tile order of one search unit per workgroup (network or interval order):
// the blocks' address bounds of both sides are staged in LDS, every tile
// whose two blocks' address ranges meet becomes a candidate (the others
// hold no conflict and are never searched), the candidates are scored in a
// compacted list (every lane busy: mode 1 runs the network on each, mode 2
// keeps index order) and sorted by (score descending, index); the first K
// go to order[], the rest of the K slots get kNoTile.  A unit the unit
// filter proves free of conflicts gets no tile at all.  At most kTopCap
// candidates per unit (the first ones in index order).
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

__global__ void __launch_bounds__(256)
k_tile_rank(const VQuery* __restrict__ vq, const BBound* __restrict__ bb,
            const float* __restrict__ w, uint32_t mode, uint32_t K,
            const IFact* __restrict__ facts, const QDesc* __restrict__ qd,
            uint32_t* __restrict__ order) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float cs[kTopCap];
  __shared__ uint32_t ci[kTopCap];
  __shared__ uint32_t ncand;
  const VQuery v = vq[blockIdx.x];
  const uint32_t G = v.G;
  uint32_t* out = order + (u64)blockIdx.x * K;
  const QDesc q = qd[v.q];
  if (facts && unit_free(facts[v.inst_i], facts[v.inst_j], q.flags,
                         !q.self && v.inst_i != v.inst_j)) {
    for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) out[r] = kNoTile;
    return;
  }
  // LDS: [weights (mode 1)] bounds of side a, then of side b
  float* sw = reinterpret_cast<float*>(smem);
  BBound* ba = reinterpret_cast<BBound*>(smem + (mode == 1 ? ((kNW * 4 + 15) & ~15) : 0));
  BBound* bbb = ba + G;
  if (mode == 1)
    for (int k = threadIdx.x; k < kNW; k += blockDim.x) sw[k] = w[k];
  for (uint32_t b = threadIdx.x; b < G; b += blockDim.x) {
    ba[b] = bb[v.bb_i + b];
    bbb[b] = bb[v.bb_j + b];
  }
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  // candidates, rows in index order
  for (uint32_t b1 = 0; b1 < G; ++b1) {
    const BBound x = ba[b1];
    if (!x.cnt) continue;
    for (uint32_t b2 = threadIdx.x; b2 < G; b2 += blockDim.x) {
      const BBound y = bbb[b2];
      if (!y.cnt || x.mx < y.mn || y.mx < x.mn) continue;
      const uint32_t p = atomicAdd(&ncand, 1u);
      if (p < kTopCap) ci[p] = b1 * G + b2;
    }
  }
  __syncthreads();
  const uint32_t n = ncand < kTopCap ? ncand : kTopCap;
  for (uint32_t c = threadIdx.x; c < n; c += blockDim.x) {
    float sc = 0.f;  // interval order: by index alone
    if (mode == 1) {
      const uint32_t t = ci[c];
      const uint32_t b1 = t / G, b2 = t - b1 * G;
      float f[kIn];
      tile_features(v, b1, b2, ba[b1], bbb[b2], f);
      sc = mlp_logit(sw, f);
    }
    cs[c] = sc;
  }
  uint32_t P = 1;
  while (P < n) P <<= 1;
  for (uint32_t k = n + threadIdx.x; k < P; k += blockDim.x) {
    cs[k] = -INFINITY;
    ci[k] = kNoTile;
  }
  __syncthreads();
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t k = threadIdx.x; k < P; k += blockDim.x) {
        const uint32_t j = k ^ stride;
        if (j <= k) continue;
        const bool up = (k & size) == 0;
        const bool jb = tile_before(cs[j], ci[j], cs[k], ci[k]);
        if (jb == up) {
          const float ts = cs[k];
          const uint32_t ti = ci[k];
          cs[k] = cs[j];
          ci[k] = ci[j];
          cs[j] = ts;
          ci[j] = ti;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t r = threadIdx.x; r < K; r += blockDim.x) out[r] = r < n ? ci[r] : kNoTile;
}

// ---------------------------------------------------------------------------
// Tile search: join block b1 of access a with block b2 of access b in LDS.
// A query already resolved skips its tiles.  A conflicting tile records its
// counts and a witness pair from inside the tile, and claims the query by
// the smallest (round rank, tile item).

template <int CAP, int TBL>
__global__ void __launch_bounds__(256)
k_tile_join(const TItem* __restrict__ items, const VQuery* __restrict__ vq,
            const uint32_t* __restrict__ order, uint32_t K,
            const DevInst* __restrict__ insts, const DInsn* __restrict__ code,
            const int64_t* __restrict__ params,
            const int64_t* __restrict__ loopvals, const QDesc* __restrict__ qd,
            uint32_t* __restrict__ done, TOut* __restrict__ tout,
            u64* __restrict__ claim, uint32_t item0, const BBound* __restrict__ bb,
            const IFact* __restrict__ facts) {
  extern __shared__ __align__(16) unsigned char smem[];
  JoinLds<CAP, TBL>& S = *reinterpret_cast<JoinLds<CAP, TBL>*>(smem);
  __shared__ uint32_t pidx_star;
  const uint32_t gi = item0 + blockIdx.x;
  const TItem it = items[gi];
  const VQuery v = vq[it.vq];
  if (done[v.q]) return;
  const QDesc q = qd[v.q];
  const uint32_t tile = order ? order[(u64)it.vq * K + it.rank] : it.rank;
  if (tile == kNoTile) return;  // fewer candidate tiles than ranks
  // plain order: a unit proven free of conflicts searches nothing
  if (!order && facts && unit_free(facts[v.inst_i], facts[v.inst_j], q.flags,
                                   !q.self && v.inst_i != v.inst_j))
    return;
  const uint32_t b1 = tile / v.G, b2 = tile - (tile / v.G) * v.G;
  {
    // a tile whose blocks' address ranges are disjoint holds no conflict
    const BBound x = bb[v.bb_i + b1], y = bb[v.bb_j + b2];
    if (!x.cnt || !y.cnt || x.mx < y.mn || y.mx < x.mn) return;
  }
  if (threadIdx.x == 0) {
    S.n = 0;
    S.err = 0;
    pidx_star = 0xFFFFFFFFu;
  }
  init_red(S);
  __syncthreads();
  uint32_t err = 0;
  const int nside = q.self ? 1 : 2;
  for (int side = 0; side < 2; ++side) {
    // a self-pair's tile holds block b1 and block b2 of the same access,
    // both as side 0 (the join counts ordered pairs among them)
    DevInst I;
    load_inst(I, insts, (side && !q.self) ? v.inst_j : v.inst_i);
    const uint32_t blk = side ? b2 : b1;
    if (side == 1 && q.self && b1 == b2) break;
    const uint32_t p0 = blk * I.a.tpb, p1 = p0 + I.a.tpb;
    const uint32_t sd = q.self ? 0u : (uint32_t)side;
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
      lds_append(S, valid, pt, id, sd, w);
    }
    (void)nside;
  }
  __syncthreads();
  if (S.err) return;  // errors are reported by the bounds pass
  lds_join<256>(S, q, v.sigma);
  const u64 pk = S.red[3];
  if (pk == kNoKey) return;
  // p*: the record with key pk on side 0; then the smallest partner q
  const uint32_t n = S.n;
  for (uint32_t r = threadIdx.x; r < n; r += blockDim.x) {
    uint32_t tl = S.tli[r];
    if (tl & kSide) continue;
    if (pkey(v.sigma, S.blin[r], tl & 0x3FF, tl >> 16) == pk) pidx_star = r;
  }
  __syncthreads();
  const uint32_t ps = pidx_star;
  u64 best = kNoKey;
  uint32_t bcls = 0;
  for (uint32_t r = threadIdx.x; r < n; r += blockDim.x) {
    uint32_t tl = S.tli[r];
    if (!q.self && !(tl & kSide)) continue;
    if (S.addr[r] != S.addr[ps]) continue;
    if (S.blin[r] == S.blin[ps] && (tl & 0x3FF) == (S.tli[ps] & 0x3FF)) continue;
    uint32_t cls;
    if (S.blin[r] != S.blin[ps]) cls = 1;
    else if (S.w[r] == S.w[ps]) cls = 4;
    else cls = 2;
    if (!(cls & q.mask)) continue;
    if (cls != 1 && (S.bw[r] >> 16) != (S.bw[ps] >> 16)) continue;
    if (cls == 4 && (S.bw[r] & 0xFFFF) != (S.bw[ps] & 0xFFFF)) continue;
    u64 k = pkey(v.sigma, S.blin[r], tl & 0x3FF, tl >> 16);
    if (k < best) { best = k; bcls = cls; }
  }
  best = wave_min(best);
  __shared__ u64 sbest;
  if (threadIdx.x == 0) sbest = kNoKey;
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && best != kNoKey) atomicMin(&sbest, best);
  __syncthreads();
  if (threadIdx.x == 0 && sbest != kNoKey) {
    TOut o;
    o.cnt[0] = S.red[0];
    o.cnt[1] = S.red[1];
    o.cnt[2] = S.red[2];
    o.pkey = pk;
    o.qkey = sbest;
    o.addr = (long long)S.addr[ps];
    tout[gi] = o;
    atomicMin(&claim[v.q], ((u64)it.rank << 32) | gi);
    (void)bcls;
  }
}

// Moves each claimed query's tile result into its accumulators and marks it
// resolved (count is a lower bound in VERDICT mode).
__global__ void k_verdict_commit(uint32_t n, const u64* __restrict__ claim,
                                 const TOut* __restrict__ tout,
                                 QAcc* __restrict__ acc, uint32_t* __restrict__ done) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n || claim[q] == kNoKey || done[q]) return;
  const TOut o = tout[(uint32_t)claim[q]];
  acc[q].cnt[0] = o.cnt[0];
  acc[q].cnt[1] = o.cnt[1];
  acc[q].cnt[2] = o.cnt[2];
  acc[q].pmin = o.pkey;
  acc[q].qmin = o.qkey;
  acc[q].waddr = o.addr;
  // result flag 2: count is a lower bound; bits 8..: tiles examined
  acc[q].qclass = 2u | ((uint32_t)((claim[q] >> 32) + 1) << 8);
  done[q] = 1;
}

// ---------------------------------------------------------------------------
// Launch wrappers.

#define HGRD_CHECK(x)                     \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return (int)e_; \
  } while (0)

int launch_block_bounds_tab(hipStream_t st, const uint32_t* ilist, uint32_t ni,
                            const BItem* items, uint32_t n, const void* insts,
                            InstRange* ir, BBound* out) {
  for (uint32_t off = 0; off < ni; off += 1u << 20) {
    uint32_t m = ni - off < (1u << 20) ? ni - off : (1u << 20);
    hipLaunchKernelGGL(k_inst_ranges, dim3(m), dim3(256), 0, st, ilist + off,
                       (const DevInst*)insts, ir);
    HGRD_CHECK(hipGetLastError());
  }
  if (n) {
    hipLaunchKernelGGL(k_block_bounds_tab, dim3((n + 255) / 256), dim3(256), 0, st, items,
                       n, (const DevInst*)insts, ir, out);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_block_bounds(hipStream_t st, const BItem* items, uint32_t n,
                        const void* insts, const DInsn* code,
                        const int64_t* params, const int64_t* loopvals,
                        QAcc* acc, BBound* out) {
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL(k_block_bounds, dim3(m), dim3(256), 0, st, items + off,
                       (const DevInst*)insts, code, params, loopvals, acc, out);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_vq_span(hipStream_t st, VQuery* vq, uint32_t n, const BBound* bb) {
  if (!n) return 0;
  hipLaunchKernelGGL(k_vq_span, dim3((n + 255) / 256), dim3(256), 0, st, vq, n, bb);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_tile_scores(hipStream_t st, const TChunk* chunks, uint32_t n,
                       const VQuery* vq, const BBound* bb, const float* w,
                       uint32_t mode, float* scores) {
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL(k_tile_scores, dim3(m), dim3(256), 0, st, chunks + off,
                       vq, bb, w, mode, scores);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_tile_features(hipStream_t st, const TChunk* chunks, uint32_t n,
                         const VQuery* vq, const BBound* bb, float* feats) {
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL(k_tile_features, dim3(m), dim3(256), 0, st, chunks + off,
                       vq, bb, feats);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_tile_rank(hipStream_t st, const VQuery* vq, uint32_t nvq, const BBound* bb,
                     const float* w, uint32_t mode, uint32_t K, uint32_t max_g,
                     const IFact* facts, const QDesc* qd, uint32_t* order) {
  if (!nvq) return 0;
  const size_t lds = (mode == 1 ? ((kNW * 4 + 15) & ~(size_t)15) : 0) +
                     2 * (size_t)max_g * sizeof(BBound);
  hipLaunchKernelGGL(k_tile_rank, dim3(nvq), dim3(256), lds, st, vq, bb, w, mode, K, facts,
                     qd, order);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_topk(hipStream_t st, const VQuery* vq, uint32_t nvq,
                const float* scores, uint32_t K, uint32_t max_tiles,
                uint32_t* order) {
  if (!nvq) return 0;
  (void)max_tiles;
  hipLaunchKernelGGL(k_topk, dim3(nvq), dim3(256), 0, st, vq, scores, K, order);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

template <int CAP, int TBL>
static int launch_tile_join_t(hipStream_t st, const TItem* items, uint32_t item0,
                              uint32_t n, const VQuery* vq, const uint32_t* order,
                              uint32_t K, const void* insts, const DInsn* code,
                              const int64_t* params, const int64_t* loopvals,
                              const QDesc* qd, uint32_t* done, TOut* tout,
                              u64* claim, const BBound* bb, const IFact* facts) {
  size_t lds = sizeof(JoinLds<CAP, TBL>);
  for (uint32_t off = 0; off < n; off += 1u << 20) {
    uint32_t m = n - off < (1u << 20) ? n - off : (1u << 20);
    hipLaunchKernelGGL((k_tile_join<CAP, TBL>), dim3(m), dim3(256), lds, st,
                       items, vq, order, K, (const DevInst*)insts, code, params,
                       loopvals, qd, done, tout, claim, item0 + off, bb, facts);
    HGRD_CHECK(hipGetLastError());
  }
  return 0;
}

int launch_tile_join(int cfg, hipStream_t st, const TItem* items, uint32_t item0,
                     uint32_t n, const VQuery* vq, const uint32_t* order,
                     uint32_t K, const void* insts, const DInsn* code,
                     const int64_t* params, const int64_t* loopvals,
                     const QDesc* qd, uint32_t* done, TOut* tout,
                     unsigned long long* claim, const BBound* bb, const IFact* facts) {
  switch (cfg) {
    case 0: return launch_tile_join_t<1024, 2048>(st, items, item0, n, vq, order, K, insts, code, params, loopvals, qd, done, tout, claim, bb, facts);
    case 1: return launch_tile_join_t<1536, 4096>(st, items, item0, n, vq, order, K, insts, code, params, loopvals, qd, done, tout, claim, bb, facts);
    default: return launch_tile_join_t<3072, 8192>(st, items, item0, n, vq, order, K, insts, code, params, loopvals, qd, done, tout, claim, bb, facts);
  }
}

int launch_verdict_commit(hipStream_t st, uint32_t n, const unsigned long long* claim,
                          const TOut* tout, QAcc* acc, uint32_t* done) {
  if (!n) return 0;
  hipLaunchKernelGGL(k_verdict_commit, dim3((n + 255) / 256), dim3(256), 0, st,
                     n, claim, tout, acc, done);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

static uint32_t grid_rows(u64 n) {
  u64 g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  return g ? (uint32_t)g : 1;
}

int launch_mlp_forward(hipStream_t st, const float* X, u64 n, const float* w,
                       float* out) {
  if (!n) return 0;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid_rows(n)), dim3(256), 0, st, X, n, w, out);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_mlp_grad(hipStream_t st, const float* X, const float* Y, u64 n,
                    const float* w, float* grad, float* loss) {
  if (!n) return 0;
  hipLaunchKernelGGL(k_mlp_grad, dim3(grid_rows(n)), dim3(256), 0, st, X, Y, n,
                     w, 1.0f / (float)n, grad, loss);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int launch_adam(hipStream_t st, float* w, float* g, float* m, float* v, float lr,
                int t) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((kNW + 255) / 256), dim3(256), 0, st, w, g, m,
                     v, lr, b1, b2, eps, c1, c2);
  HGRD_CHECK(hipGetLastError());
  return 0;
}

int mlp_num_weights() { return kNW; }

int init_verdict_attributes() {
  // tile ranking: weights and the bounds of both sides of up to 1024 blocks
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_tile_rank,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(((kNW * 4 + 15) & ~15) + 2 * 1024 * sizeof(BBound))));
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_tile_join<1024, 2048>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sizeof(JoinLds<1024, 2048>)));
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_tile_join<1536, 4096>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sizeof(JoinLds<1536, 4096>)));
  HGRD_CHECK(hipFuncSetAttribute((const void*)k_tile_join<3072, 8192>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sizeof(JoinLds<3072, 8192>)));
  return 0;
}

}  // namespace hgrd
