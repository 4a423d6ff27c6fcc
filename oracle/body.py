"""CPU oracle for the kernel-body front end (section 6.1 "Avoiding race
checks"; section 6.5, Figures 9 and 10).

TEST INFRASTRUCTURE.  Only the test suite loads this file; the GPU library
never calls it, and it shares no code with the library's derivation.

Two things are computed from a structured kernel body (statements
("access", k), ("barrier",), ("warp_barrier",), ("if",), ("else",),
("end",), ("loop", k), ("cas", array, addr, scope), ("exch", array, addr,
scope), ("fence", scope)):

* barrier counts, by running the body: for one parameter tuple every loop
  takes its value list, both ways of every branch are walked (a branch's
  condition is not modelled; the accesses' guards carry it), and each
  access occurrence records how many block and warp barriers its thread
  has executed before it.  A barrier counts only outside every branch and
  inside loops whose trip count and iteration index have closed forms (an
  ADD loop compared with lt or le, a SUB loop compared with gt or ge);

* the acquire and release of every access, from an explicit control-flow
  graph: dominator and post-dominator sets by the iterative data-flow
  equations, then Figure 10's search along the dominator chain (nearest
  first) for a fence and, beyond it, a CAS (acquire), and along the
  post-dominator chain for a fence and, beyond it, an Exch (release).
"""
import oracle

_SCOPE_RANK = {"block": 0, "device": 1}


def _seq(node):
    """The sequence new statements go to (a branch's way by its flag)."""
    return node[2] if node[3] else node[1]


def _tree(body):
    root = ["root", []]
    stack = [root]
    for st in body:
        kind = st[0]
        top = stack[-1]
        cur = top[1] if top[0] != "if" else _seq(top)
        if kind == "if":
            node = ["if", [], [], False]
            cur.append(node)
            stack.append(node)
        elif kind == "loop":
            node = ["loop", [], st[1]]
            cur.append(node)
            stack.append(node)
        elif kind == "else":
            assert top[0] == "if" and not top[3]
            top[3] = True
        elif kind == "end":
            stack.pop()
        else:
            cur.append(("stmt",) + tuple(st))
    assert len(stack) == 1
    return root[1]


def _loop_values(model, k, params):
    """The value list of model loop k for one tuple (C semantics)."""
    L = model.loops[k]
    v, e1 = oracle.eval_uniform(L.init, params)
    b, e2 = oracle.eval_uniform(L.bound, params)
    s, e3 = oracle.eval_uniform(L.step, params)
    assert not (e1 or e2 or e3)
    cmp = {"lt": lambda x: x < b, "le": lambda x: x <= b, "gt": lambda x: x > b,
           "ge": lambda x: x >= b, "ne": lambda x: x != b}[L.cmp]
    out = []
    while cmp(v):
        out.append(v)
        assert len(out) <= 65536
        if L.upd == "add":
            v = v + s
        elif L.upd == "sub":
            v = v - s
        elif L.upd == "mul":
            v = v * s
        elif L.upd == "div":
            q = abs(v) // abs(s)
            v = -q if (v < 0) != (s < 0) else q
        elif L.upd == "shl":
            v = v << s
        else:
            v = v >> s
    return out


def _closed_form(model, k):
    L = model.loops[k]
    return (L.upd == "add" and L.cmp in ("lt", "le")) or \
        (L.upd == "sub" and L.cmp in ("gt", "ge"))


def barrier_counts(model, body, params):
    """{access: {loop-value tuple: (block barriers, warp barriers)}} for one
    tuple, by running the body."""
    tree = _tree(body)
    out = {}
    cnt = [0, 0]

    def run(items, counted, vals):
        for it in items:
            if it[0] == "stmt":
                kind = it[1]
                if kind == "access":
                    out.setdefault(it[2], {})[tuple(vals)] = (cnt[0], cnt[1])
                elif kind == "barrier" and counted:
                    cnt[0] += 1
                elif kind == "warp_barrier" and counted:
                    cnt[1] += 1
            elif it[0] == "if":
                run(it[1], False, vals)
                run(it[2], False, vals)
            else:
                k = it[2]
                ok = counted and _closed_form(model, k)
                for v in _loop_values(model, k, params):
                    run(it[1], ok, vals + [v])

    run(tree, True, [])
    return out


def _cfg(body):
    """Control-flow graph: node ids, successor lists, node -> statement."""
    tree = _tree(body)
    succ = {"entry": [], "exit": []}
    stmt = {}
    counter = [0]

    def new(label):
        counter[0] += 1
        n = (label, counter[0])
        succ[n] = []
        return n

    def emit(items, preds):
        for it in items:
            if it[0] == "stmt":
                n = new("s")
                stmt[n] = it[1:]
                for p in preds:
                    succ[p].append(n)
                preds = [n]
            elif it[0] == "if":
                b = new("branch")
                for p in preds:
                    succ[p].append(b)
                t = emit(it[1], [b])
                e = emit(it[2], [b])
                j = new("join")
                for p in t + e:
                    succ[p].append(j)
                preds = [j]
            else:
                h = new("header")
                for p in preds:
                    succ[p].append(h)
                out = emit(it[1], [h])
                for p in out:
                    succ[p].append(h)  # back edge
                preds = [h]            # the loop leaves from its header
        return preds

    last = emit(tree, ["entry"])
    for p in last:
        succ[p].append("exit")
    return succ, stmt


def _dominators(succ, start):
    nodes = list(succ)
    pred = {n: [] for n in nodes}
    for n, ss in succ.items():
        for s in ss:
            pred[s].append(n)
    dom = {n: set(nodes) for n in nodes}
    dom[start] = {start}
    changed = True
    while changed:
        changed = False
        for n in nodes:
            if n == start:
                continue
            ps = [dom[p] for p in pred[n]]
            new = set.intersection(*ps) if ps else set()
            new = new | {n}
            if new != dom[n]:
                dom[n] = new
                changed = True
    return dom


def sync_ops(body):
    """{access: (acq, rel)}: each a (array, addr expression, scope) or None,
    by Figure 10's search on the dominator / post-dominator chains."""
    succ, stmt = _cfg(body)
    dom = _dominators(succ, "entry")
    rev = {n: [] for n in succ}
    for n, ss in succ.items():
        for s in ss:
            rev[s].append(n)
    pdom = _dominators(rev, "exit")
    out = {}
    for n, st in stmt.items():
        if st[0] != "access":
            continue
        res = []
        for d, atomic in ((dom, "cas"), (pdom, "exch")):
            # the chain of (post-)dominators, nearest first: a nearer one is
            # itself dominated by every farther one, so its set is larger
            chain = sorted((x for x in d[n] if x != n and x in stmt),
                           key=lambda x: -len(d[x]))
            found, fence = None, None
            for x in chain:
                s = stmt[x]
                if fence is None:
                    if s[0] == "fence":
                        fence = s
                    continue
                if s[0] == atomic:
                    scope = min(_SCOPE_RANK[s[3]], _SCOPE_RANK[fence[1]])
                    found = (s[1], s[2], ["block", "device"][scope])
                    break
            res.append(found)
        out[st[1]] = tuple(res)
    return out
