// Host domain expansion (section 4, classes 1-5; section 6.3, Figure 8):
// the facts a program's host code fixes about a kernel launch -- asserts,
// grid dimensions computed on the host, kernel parameters derived from one
// host variable, host loop iterators passed as parameters, allocation sizes
// that are parameters too -- turned into the finite parameter tuples the
// race query takes.  The paper builds an expression tree per kernel
// parameter and hands the relations to a solver as constraints over
// unknown inputs; here the unknown inputs take caller-given finite value
// lists, so the same relations become a plain enumeration: every
// assignment of the host variables in program order, filtered by the
// asserts (class 1) and by positive allocation sizes (class 5), each
// yielding one tuple of kernel parameters.  Parameters computed from one
// host variable (class 3) keep their relation because they come from one
// assignment; loop iterators (class 4) take exactly their iterations;
// launch extents (class 2) are parameter columns that the model's launch
// domain reads.  Host-only code.  Also the tile-scoring network's weight
// file (save / load).
#include "../../include/hgrd.h"
#include "hgrd_hostops.h"

#include <cstdio>
#include <cstring>
#include <unordered_set>
#include <string>
#include <vector>

using namespace hgrd;

namespace {

constexpr uint32_t kMaxHostInsns = 256;    // per expression, as for models
constexpr uint32_t kMaxHostDepth = 16;
constexpr uint64_t kMaxHostIters = 65536;  // iterations of one host loop
constexpr uint64_t kMaxAssignments = 1ull << 24;

// Structural check of one expression: leaves CONST and PARAM k (k < nvars)
// only, a well-formed postfix sequence within the limits.  Returns RD_OK,
// RD_EINVAL or RD_EUNSUPPORTED.
int check_host_expr(const rd_host_domain& h, rd_expr e, uint32_t nvars, bool required) {
  if (e.count == 0) return required ? RD_EINVAL : RD_OK;
  if (!h.insns || (uint64_t)e.first + e.count > h.n_insns) return RD_EINVAL;
  if (e.count > kMaxHostInsns) return RD_EUNSUPPORTED;
  uint32_t depth = 0, maxd = 0;
  for (uint32_t k = 0; k < e.count; ++k) {
    const rd_insn& t = h.insns[e.first + k];
    if (t.op == RD_OP_CONST || t.op == RD_OP_PARAM) {
      if (t.op == RD_OP_PARAM && t.arg >= nvars) return RD_EINVAL;
      ++depth;
    } else if (t.op == RD_OP_NEG || t.op == RD_OP_LNOT) {
      if (depth < 1) return RD_EINVAL;
    } else if (t.op >= RD_OP_ADD && t.op <= RD_OP_LOR) {
      if (depth < 2) return RD_EINVAL;
      --depth;
    } else {
      return RD_EINVAL;  // thread, block, launch or loop leaves: not host values
    }
    maxd = depth > maxd ? depth : maxd;
  }
  if (depth != 1) return RD_EINVAL;
  return maxd > kMaxHostDepth ? RD_EUNSUPPORTED : RD_OK;
}

int64_t host_eval(const rd_host_domain& h, rd_expr e, const int64_t* vars, uint32_t& err) {
  int64_t st[kMaxHostDepth + 1];
  uint32_t sp = 0;
  for (uint32_t k = 0; k < e.count; ++k) {
    const rd_insn& t = h.insns[e.first + k];
    switch (t.op) {
      case RD_OP_CONST: st[sp++] = t.imm; break;
      case RD_OP_PARAM: st[sp++] = vars[t.arg]; break;
      case RD_OP_NEG:
        if (st[sp - 1] == INT64_MIN) { err |= ERR_RANGE; st[sp - 1] = 0; }
        else st[sp - 1] = -st[sp - 1];
        break;
      case RD_OP_LNOT: st[sp - 1] = st[sp - 1] == 0; break;
      default: {
        const int64_t b = st[--sp];
        st[sp - 1] = hop(t.op, st[sp - 1], b, err);
      }
    }
  }
  return st[0];
}

bool host_cmp(uint32_t cmp, int64_t v, int64_t bound) {
  switch (cmp) {
    case RD_CMP_LT: return v < bound;
    case RD_CMP_LE: return v <= bound;
    case RD_CMP_GT: return v > bound;
    case RD_CMP_GE: return v >= bound;
    default: return v != bound;
  }
}

uint16_t upd_op(uint32_t upd) {
  static const uint16_t kOps[] = {RD_OP_ADD, RD_OP_SUB, RD_OP_MUL,
                                  RD_OP_DIV, RD_OP_SHL, RD_OP_SHR};
  return kOps[upd];
}

struct TupleHash {
  size_t operator()(const std::vector<int64_t>& v) const {
    uint64_t x = 0x9E3779B97F4A7C15ull;
    for (int64_t a : v) {
      x ^= (uint64_t)a + 0x9E3779B97F4A7C15ull + (x << 6) + (x >> 2);
      x *= 0xBF58476D1CE4E5B9ull;
    }
    return (size_t)x;
  }
};

struct Expander {
  const rd_host_domain& h;
  std::vector<int64_t> vals;
  uint32_t err = 0;
  bool too_many = false;
  uint64_t assignments = 0;
  std::unordered_set<std::vector<int64_t>, TupleHash> seen;
  std::vector<int64_t> rows;  // distinct tuples, enumeration order

  explicit Expander(const rd_host_domain& hd) : h(hd), vals(hd.n_vars, 0) {}

  void leaf() {
    if (++assignments > kMaxAssignments) {
      too_many = true;
      return;
    }
    uint32_t e = 0;
    for (uint32_t k = 0; k < h.n_asserts; ++k)
      if (host_eval(h, h.asserts[k], vals.data(), e) == 0 && !e) return;
    for (uint32_t k = 0; k < h.n_alloc; ++k)
      if (host_eval(h, h.alloc_sizes[k], vals.data(), e) <= 0 && !e) return;
    std::vector<int64_t> row(h.n_params);
    for (uint32_t k = 0; k < h.n_params; ++k) row[k] = host_eval(h, h.params[k], vals.data(), e);
    err |= e;
    if (e) return;
    if (seen.insert(row).second) rows.insert(rows.end(), row.begin(), row.end());
  }

  void walk(uint32_t v) {
    if (too_many) return;
    if (v == h.n_vars) {
      leaf();
      return;
    }
    const rd_host_var& x = h.vars[v];
    if (x.kind == RD_HV_INPUT) {
      for (uint32_t k = 0; k < x.n_values && !too_many; ++k) {
        vals[v] = x.values[k];
        walk(v + 1);
      }
    } else if (x.kind == RD_HV_EXPR) {
      uint32_t e = 0;
      vals[v] = host_eval(h, x.init, vals.data(), e);
      err |= e;
      if (!e) walk(v + 1);
    } else {
      uint32_t e = 0;
      int64_t it = host_eval(h, x.init, vals.data(), e);
      const int64_t bound = host_eval(h, x.bound, vals.data(), e);
      const int64_t step = host_eval(h, x.step, vals.data(), e);
      err |= e;
      if (e) return;
      uint64_t n = 0;
      while (host_cmp(x.cmp, it, bound) && !too_many) {
        if (++n > kMaxHostIters) {
          too_many = true;
          return;
        }
        vals[v] = it;
        walk(v + 1);
        uint32_t ue = 0;
        it = hop(upd_op(x.upd), it, step, ue);
        if (ue) {  // the host program's update overflows or divides by zero
          err |= ue;
          return;
        }
      }
    }
  }
};

}  // namespace

extern "C" {

int rd_expand_host_domain(const rd_host_domain* h, rd_param_sets* out, int64_t* buf,
                          uint64_t cap_values) {
  if (!h || !out) return RD_EINVAL;
  out->n_sets = 0;
  out->values = buf;
  if ((h->n_vars && !h->vars) || (h->n_asserts && !h->asserts) ||
      (h->n_alloc && !h->alloc_sizes) || (h->n_params && !h->params) ||
      (cap_values && !buf))
    return RD_EINVAL;
  int worst = RD_OK;
  auto note = [&](int s) {
    if (s == RD_EINVAL || (s == RD_EUNSUPPORTED && worst != RD_EINVAL)) worst = s;
  };
  for (uint32_t v = 0; v < h->n_vars; ++v) {
    const rd_host_var& x = h->vars[v];
    if (x.kind == RD_HV_INPUT) {
      if (x.n_values && !x.values) note(RD_EINVAL);
    } else if (x.kind == RD_HV_EXPR) {
      note(check_host_expr(*h, x.init, v, true));
    } else if (x.kind == RD_HV_LOOP) {
      if (x.cmp > RD_CMP_NE || x.upd > RD_UPD_SHR) note(RD_EINVAL);
      note(check_host_expr(*h, x.init, v, true));
      note(check_host_expr(*h, x.bound, v, true));
      note(check_host_expr(*h, x.step, v, true));
    } else {
      note(RD_EINVAL);
    }
  }
  for (uint32_t k = 0; k < h->n_asserts; ++k) note(check_host_expr(*h, h->asserts[k], h->n_vars, true));
  for (uint32_t k = 0; k < h->n_alloc; ++k) note(check_host_expr(*h, h->alloc_sizes[k], h->n_vars, true));
  for (uint32_t k = 0; k < h->n_params; ++k) note(check_host_expr(*h, h->params[k], h->n_vars, true));
  if (worst != RD_OK) return worst;

  Expander X(*h);
  X.walk(0);
  if (X.too_many) return RD_EUNSUPPORTED;
  if (X.err & ERR_DIVZERO) return RD_EDIVZERO;
  if (X.err) return RD_ERANGE;
  const uint64_t n = h->n_params ? X.rows.size() / h->n_params : (X.seen.empty() ? 0 : 1);
  out->n_sets = (uint32_t)n;
  const uint64_t fit = std::min<uint64_t>(X.rows.size(), cap_values - cap_values % (h->n_params ? h->n_params : 1));
  if (fit) memcpy(buf, X.rows.data(), fit * sizeof(int64_t));
  return X.rows.size() > cap_values ? RD_ECAPACITY : RD_OK;
}

// ---- tile-scoring network weights on disk --------------------------------

static const char kMlpMagic[8] = {'H', 'G', 'R', 'D', 'M', 'L', 'P', '1'};
static constexpr uint32_t kMlpFloats = sizeof(rd_mlp) / sizeof(float);
static_assert(kMlpFloats == 6337, "rd_mlp layout");

int rd_mlp_save(const rd_mlp* w, uint32_t feature_version, const char* path) {
  if (!w || !path) return RD_EINVAL;
  FILE* f = fopen(path, "wb");
  if (!f) return RD_EINVAL;
  const uint32_t hdr[4] = {1u, kMlpFloats, feature_version, 0u};
  bool ok = fwrite(kMlpMagic, 1, 8, f) == 8 && fwrite(hdr, 4, 4, f) == 4;
  // 8 + 16 bytes so far; pad the header to 32 bytes
  const uint32_t pad[2] = {0u, 0u};
  ok = ok && fwrite(pad, 4, 2, f) == 2;
  ok = ok && fwrite(w, sizeof(float), kMlpFloats, f) == kMlpFloats;
  ok = (fclose(f) == 0) && ok;
  return ok ? RD_OK : RD_EINVAL;
}

int rd_mlp_load(rd_mlp* w, uint32_t* feature_version, const char* path) {
  if (!w || !path) return RD_EINVAL;
  FILE* f = fopen(path, "rb");
  if (!f) return RD_EINVAL;
  char magic[8];
  uint32_t hdr[6];
  rd_mlp tmp;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMlpMagic, 8) == 0 &&
            fread(hdr, 4, 6, f) == 6 && hdr[0] == 1u && hdr[1] == kMlpFloats &&
            fread(&tmp, sizeof(float), kMlpFloats, f) == kMlpFloats;
  fclose(f);
  if (!ok) return RD_EINVAL;
  *w = tmp;
  if (feature_version) *feature_version = hdr[2];
  return RD_OK;
}

}  // extern "C"
