// Kernel-body front end (section 6.1 "Avoiding race checks"; section 6.5,
// Figures 9 and 10): from a structured kernel body -- accesses, block and
// warp barriers, two-way branches, model loops, and the atomics and fences
// that make up acquires and releases -- derive what the race query takes
// per access: its enclosing loops, its barrier-interval ids and the
// acquire and release around it.
//
// The paper asks, per access pair, whether a barrier post-dominates the
// first access and dominates the second (then the pair skips the
// intra-block checks).  Here the query works per point, so the barrier
// structure becomes a count: bint of a point is the number of block
// barriers its thread has executed before it, and two points of one block
// share a barrier interval exactly when their counts are equal.  In
// uniform code (no enclosing branch) the count has a closed form over the
// loop values: for every sequence on the access's path (the body, and each
// enclosing loop's body), the barriers of that sequence's other statements
// run once per completed iteration of the loops around the sequence, and
// those of the statements before the access's own run once more:
//
//   bint = sum over sequences c on the path of  I_c * W_c + P_c
//
// with I_c the number of completed iterations of c (linearised over the
// enclosing loops: ((idx_1 T_2 + idx_2) T_3 + ...) + idx_k), W_c the
// barriers one run of c executes outside the access's own statement (a
// barrier inside nested loops counts their trip counts), and P_c those
// before it.  Host only.
#include "../../include/hgrd.h"

#include <cstring>
#include <vector>

namespace {

constexpr uint32_t kMaxInsns = 256;  // the model expression limits
constexpr uint32_t kMaxDepth = 16;
constexpr uint32_t kMaxLoops = 4;

using Code = std::vector<rd_insn>;

rd_insn leaf(uint16_t op, uint16_t arg, int64_t imm = 0) {
  rd_insn t;
  memset(&t, 0, sizeof t);
  t.op = op;
  t.arg = arg;
  t.imm = imm;
  return t;
}
Code cst(int64_t v) { return Code{leaf(RD_OP_CONST, 0, v)}; }
bool is_const(const Code& c, int64_t v) {
  return c.size() == 1 && c[0].op == RD_OP_CONST && c[0].imm == v;
}
Code bin(uint16_t op, const Code& a, const Code& b) {
  Code r = a;
  r.insert(r.end(), b.begin(), b.end());
  r.push_back(leaf(op, 0));
  return r;
}
// a + b and a * b with the obvious constant cases folded
Code add(const Code& a, const Code& b) {
  if (is_const(a, 0)) return b;
  if (is_const(b, 0)) return a;
  return bin(RD_OP_ADD, a, b);
}
Code mul(const Code& a, const Code& b) {
  if (is_const(a, 0) || is_const(b, 0)) return cst(0);
  if (is_const(a, 1)) return b;
  if (is_const(b, 1)) return a;
  return bin(RD_OP_MUL, a, b);
}

// Stack depth of a postfix sequence (well-formed by construction).
uint32_t depth_of(const Code& c) {
  uint32_t d = 0, m = 0;
  for (const rd_insn& t : c) {
    if (t.op >= RD_OP_CONST && t.op <= RD_OP_LOOP) ++d;
    else if (t.op >= RD_OP_ADD && t.op <= RD_OP_LOR) --d;
    m = d > m ? d : m;
  }
  return m;
}

struct Node {
  uint32_t kind = 0, stmt = 0;  // RD_ST_*; index in the body
  // child sequences: loop body and the root in seq[0]; a branch's two ways
  // in seq[0] and seq[1]
  std::vector<uint32_t> seq[2];
  bool in_else = false;  // parsing: an IF past its ELSE
};

// One step of an access's path: sequence (node, way) and the position of
// the access's statement in it.
struct Step {
  uint32_t node, way, pos;
};

struct Deriver {
  const rd_kernel_model& M;
  const rd_stmt* body;
  std::vector<Node> nodes;  // nodes[0]: the root sequence
  std::vector<int32_t> where;  // access -> node (-1: not in the body)

  Deriver(const rd_kernel_model& m, const rd_stmt* b) : M(m), body(b) {}

  // Copy of a model expression.
  Code expr(rd_expr e) const {
    return Code(M.insns + e.first, M.insns + e.first + e.count);
  }

  // A loop whose trip count and iteration index have closed forms.
  bool simple_loop(uint32_t l) const {
    const rd_loop& L = M.loops[l];
    return (L.upd == RD_UPD_ADD && (L.cmp == RD_CMP_LT || L.cmp == RD_CMP_LE)) ||
           (L.upd == RD_UPD_SUB && (L.cmp == RD_CMP_GT || L.cmp == RD_CMP_GE));
  }
  // Completed iterations before the current one: (v - init) / step for an
  // ADD loop, (init - v) / step for a SUB loop.
  Code index(uint32_t l) const {
    const rd_loop& L = M.loops[l];
    const Code v{leaf(RD_OP_LOOP, (uint16_t)l)};
    const Code d = L.upd == RD_UPD_ADD ? bin(RD_OP_SUB, v, expr(L.init))
                                       : bin(RD_OP_SUB, expr(L.init), v);
    return bin(RD_OP_DIV, d, expr(L.step));
  }
  // Iterations of one run: max(0, (span + step - 1) / step) for LT / GT,
  // max(0, (span + step) / step) for LE / GE, span = bound - init (ADD) or
  // init - bound (SUB).
  Code trips(uint32_t l) const {
    const rd_loop& L = M.loops[l];
    const Code span = L.upd == RD_UPD_ADD ? bin(RD_OP_SUB, expr(L.bound), expr(L.init))
                                          : bin(RD_OP_SUB, expr(L.init), expr(L.bound));
    const bool strict = L.cmp == RD_CMP_LT || L.cmp == RD_CMP_GT;
    Code num = bin(RD_OP_ADD, span, expr(L.step));
    if (strict) num = bin(RD_OP_SUB, num, cst(1));
    return bin(RD_OP_MAX, cst(0), bin(RD_OP_DIV, num, expr(L.step)));
  }

  // Barriers of kind `bk` one run of statement node n executes (counted
  // ones only: none under a branch, none in a loop without closed forms).
  Code run_count(uint32_t n, uint32_t bk) const {
    const Node& N = nodes[n];
    if (N.kind == bk) return cst(1);
    if (N.kind == RD_ST_IF) return cst(0);
    if (N.kind != RD_ST_LOOP) return cst(0);
    const uint32_t l = body[N.stmt].arg;
    if (!simple_loop(l)) return cst(0);
    const Code inner = seq_count(n, 0, 0, (uint32_t)N.seq[0].size(), bk);
    return is_const(inner, 0) ? inner : mul(trips(l), inner);
  }
  Code seq_count(uint32_t n, uint32_t way, uint32_t from, uint32_t to, uint32_t bk) const {
    Code s = cst(0);
    for (uint32_t k = from; k < to; ++k) s = add(s, run_count(nodes[n].seq[way][k], bk));
    return s;
  }

  // bint (bk = RD_ST_BARRIER) or wint (RD_ST_WARP_BARRIER) of the access
  // whose path is `path`.
  Code interval(const std::vector<Step>& path, uint32_t bk) const {
    Code total = cst(0);
    Code lin = cst(0);  // completed iterations of the current sequence
    bool ok = true;     // every loop so far has closed forms, no branch
    for (const Step& s : path) {
      const Node& N = nodes[s.node];
      if (N.kind == RD_ST_IF) ok = false;  // barriers under a branch: none
      if (N.kind == RD_ST_LOOP) {
        const uint32_t l = body[N.stmt].arg;
        if (!simple_loop(l)) ok = false;
        if (ok) lin = add(mul(lin, trips(l)), index(l));
      }
      if (!ok) break;
      const uint32_t len = (uint32_t)N.seq[s.way].size();
      const Code before = seq_count(s.node, s.way, 0, s.pos, bk);
      const Code after = seq_count(s.node, s.way, s.pos + 1, len, bk);
      const Code w = add(before, after);
      total = add(total, add(mul(lin, w), before));
    }
    return total;
  }

  // Statements that dominate (before) or post-dominate (after) the access,
  // nearest first: those directly in a sequence of its path.
  std::vector<uint32_t> around(const std::vector<Step>& path, bool after) const {
    std::vector<uint32_t> out;
    if (!after) {
      for (size_t i = path.size(); i-- > 0;) {
        const Step& s = path[i];
        const std::vector<uint32_t>& q = nodes[s.node].seq[s.way];
        for (uint32_t k = s.pos; k-- > 0;) out.push_back(q[k]);
      }
    } else {
      for (size_t i = path.size(); i-- > 0;) {
        const Step& s = path[i];
        const std::vector<uint32_t>& q = nodes[s.node].seq[s.way];
        for (uint32_t k = s.pos + 1; k < q.size(); ++k) out.push_back(q[k]);
      }
    }
    return out;
  }

  // The acquire (CAS then fence, searched backwards: fence first) or the
  // release (fence then Exch, searched forwards).  Returns the atomic's
  // statement and the narrower scope, or -1.
  int32_t sync_op(const std::vector<Step>& path, bool release, uint32_t& scope) const {
    const std::vector<uint32_t> ops = around(path, release);
    int32_t fence = -1;
    for (uint32_t n : ops) {
      const rd_stmt& t = body[nodes[n].stmt];
      if (fence < 0) {
        if (t.kind == RD_ST_FENCE) fence = (int32_t)n;
        continue;
      }
      if (t.kind == (release ? (uint32_t)RD_ST_EXCH : (uint32_t)RD_ST_CAS)) {
        const uint32_t fs = body[nodes[fence].stmt].scope;
        scope = t.scope < fs ? t.scope : fs;
        return (int32_t)n;
      }
    }
    return -1;
  }
};

// Structural check of an atomic's address: a well-formed postfix sequence
// over the leaves of an access address, loop leaves only of `loops`.
bool check_addr(const rd_kernel_model& M, rd_expr e, const std::vector<uint32_t>& loops) {
  if (e.count == 0 || !M.insns || (uint64_t)e.first + e.count > M.n_insns) return false;
  uint32_t d = 0;
  for (uint32_t k = 0; k < e.count; ++k) {
    const rd_insn& t = M.insns[e.first + k];
    if (t.op >= RD_OP_CONST && t.op <= RD_OP_LOOP) {
      if (t.op == RD_OP_PARAM && t.arg >= M.n_params) return false;
      if ((t.op == RD_OP_TID || t.op == RD_OP_BID || t.op == RD_OP_BDIM ||
           t.op == RD_OP_GDIM) && t.arg > 2)
        return false;
      if (t.op == RD_OP_LOOP) {
        bool found = false;
        for (uint32_t l : loops) found |= l == t.arg;
        if (!found) return false;
      }
      ++d;
    } else if (t.op == RD_OP_NEG || t.op == RD_OP_LNOT) {
      if (d < 1) return false;
    } else if (t.op >= RD_OP_ADD && t.op <= RD_OP_LOR) {
      if (d < 2) return false;
      --d;
    } else {
      return false;
    }
  }
  return d == 1;
}

}  // namespace

extern "C" int rd_derive_body(const rd_kernel_model* m, const rd_stmt* body, uint32_t n_stmts,
                              rd_access* acc_out, rd_insn* insns_out, uint32_t cap_insns,
                              uint32_t* n_insns_out) {
  if (!m || !acc_out || !n_insns_out || (n_stmts && !body)) return RD_EINVAL;
  if ((m->n_acc && !m->acc) || (m->n_insns && !m->insns) || (m->n_loops && !m->loops))
    return RD_EINVAL;
  const rd_kernel_model& M = *m;
  Deriver D(M, body);
  D.nodes.emplace_back();  // the root
  D.where.assign(M.n_acc, -1);
  // parse into a tree; open: the stack of open constructs (root at 0)
  std::vector<uint32_t> open{0};
  std::vector<uint32_t> open_loops;  // model loops of the open LOOPs
  auto cur_seq = [&]() -> std::vector<uint32_t>& {
    Node& N = D.nodes[open.back()];
    return N.seq[N.in_else ? 1 : 0];
  };
  for (uint32_t k = 0; k < n_stmts; ++k) {
    const rd_stmt& t = body[k];
    if (t.kind == RD_ST_END) {
      if (open.size() < 2) return RD_EINVAL;
      if (D.nodes[open.back()].kind == RD_ST_LOOP) open_loops.pop_back();
      open.pop_back();
      continue;
    }
    if (t.kind == RD_ST_ELSE) {
      Node& N = D.nodes[open.back()];
      if (open.size() < 2 || N.kind != RD_ST_IF || N.in_else) return RD_EINVAL;
      N.in_else = true;
      continue;
    }
    if (t.kind < RD_ST_ACCESS || t.kind > RD_ST_FENCE) return RD_EINVAL;
    if (t.kind == RD_ST_ACCESS && (t.arg >= M.n_acc || D.where[t.arg] >= 0)) return RD_EINVAL;
    if (t.kind == RD_ST_LOOP) {
      if (t.arg >= M.n_loops) return RD_EINVAL;
      for (uint32_t l : open_loops)
        if (l == t.arg) return RD_EINVAL;
    }
    if (t.kind == RD_ST_CAS || t.kind == RD_ST_EXCH || t.kind == RD_ST_FENCE) {
      if (t.scope > RD_SCOPE_DEVICE) return RD_EINVAL;
      if (t.kind != RD_ST_FENCE &&
          (t.array >= M.n_arrays || !M.arrays || !check_addr(M, t.addr, open_loops)))
        return RD_EINVAL;
    }
    const uint32_t n = (uint32_t)D.nodes.size();
    cur_seq().push_back(n);
    D.nodes.emplace_back();
    D.nodes[n].kind = t.kind;
    D.nodes[n].stmt = k;
    if (t.kind == RD_ST_ACCESS) D.where[t.arg] = (int32_t)n;
    if (t.kind == RD_ST_IF || t.kind == RD_ST_LOOP) {
      open.push_back(n);
      if (t.kind == RD_ST_LOOP) open_loops.push_back(t.arg);
    }
  }
  if (open.size() != 1) return RD_EINVAL;
  // paths of the accesses: parent links
  std::vector<int32_t> parent(D.nodes.size(), -1), pway(D.nodes.size(), 0),
      ppos(D.nodes.size(), 0);
  for (uint32_t n = 0; n < D.nodes.size(); ++n)
    for (uint32_t w = 0; w < 2; ++w)
      for (uint32_t k = 0; k < D.nodes[n].seq[w].size(); ++k) {
        const uint32_t c = D.nodes[n].seq[w][k];
        parent[c] = (int32_t)n;
        pway[c] = (int32_t)w;
        ppos[c] = (int32_t)k;
      }
  std::vector<rd_insn> pool(M.insns, M.insns + M.n_insns);
  int status = RD_OK;
  for (uint32_t a = 0; a < M.n_acc; ++a) {
    rd_access A = M.acc[a];
    if (D.where[a] >= 0) {
      std::vector<Step> path;
      for (int32_t n = D.where[a]; parent[n] >= 0; n = parent[n])
        path.insert(path.begin(), Step{(uint32_t)parent[n], (uint32_t)pway[n], (uint32_t)ppos[n]});
      std::vector<uint32_t> loops;
      for (const Step& s : path)
        if (D.nodes[s.node].kind == RD_ST_LOOP) loops.push_back(body[D.nodes[s.node].stmt].arg);
      if (loops.size() > kMaxLoops) {
        status = RD_EUNSUPPORTED;
        continue;
      }
      A.n_loops = (uint32_t)loops.size();
      for (uint32_t k = 0; k < kMaxLoops; ++k) A.loops[k] = k < loops.size() ? loops[k] : 0;
      rd_expr* iv[2] = {&A.bint, &A.wint};
      const uint32_t kinds[2] = {RD_ST_BARRIER, RD_ST_WARP_BARRIER};
      for (int w = 0; w < 2; ++w) {
        const Code c = D.interval(path, kinds[w]);
        if (is_const(c, 0)) {
          iv[w]->first = 0;
          iv[w]->count = 0;  // absent: 0
          continue;
        }
        if (c.size() > kMaxInsns || depth_of(c) > kMaxDepth) {
          status = RD_EUNSUPPORTED;
          continue;
        }
        iv[w]->first = (uint32_t)pool.size();
        iv[w]->count = (uint32_t)c.size();
        pool.insert(pool.end(), c.begin(), c.end());
      }
      rd_sync* so[2] = {&A.acq, &A.rel};
      for (int r = 0; r < 2; ++r) {
        uint32_t scope = 0;
        const int32_t n = D.sync_op(path, r == 1, scope);
        memset(so[r], 0, sizeof(rd_sync));
        if (n < 0) continue;
        const rd_stmt& t = body[D.nodes[n].stmt];
        so[r]->addr = t.addr;  // already in the model's pool
        so[r]->array = t.array;
        so[r]->scope = scope;
      }
    }
    acc_out[a] = A;
  }
  *n_insns_out = (uint32_t)pool.size();
  if (status != RD_OK) return status;
  if (pool.size() > cap_insns || (!insns_out && !pool.empty())) return RD_ECAPACITY;
  if (!pool.empty()) memcpy(insns_out, pool.data(), pool.size() * sizeof(rd_insn));
  return RD_OK;
}
