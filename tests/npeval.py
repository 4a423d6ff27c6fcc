"""A small vectorised point enumerator for tests (numpy, int64).

Used only to cross-check the oracle through routes other than its own code:
the equi-join identity via numpy.unique, and re-checking witnesses.  It
follows C integer rules for the operators and does not detect overflow, so
callers keep values small.
"""
import numpy as np

_CMP = {"lt": np.less, "le": np.less_equal, "gt": np.greater,
        "ge": np.greater_equal, "ne": np.not_equal}


def _cdiv(a, b):
    q = np.abs(a) // np.abs(b)
    return np.where((a < 0) ^ (b < 0), -q, q)


def ev(expr, env, shape, default):
    if expr is None:
        return np.full(shape, default, dtype=np.int64)
    st = []
    for t in expr.code:
        op = t[0]
        if op == "const":
            st.append(np.full(shape, t[1], dtype=np.int64))
        elif op in ("param", "tid", "bid", "bdim", "gdim", "loop"):
            st.append(np.broadcast_to(np.asarray(env[(op, t[1])], dtype=np.int64), shape).copy())
        elif op == "neg":
            st[-1] = -st[-1]
        elif op == "lnot":
            st[-1] = (st[-1] == 0).astype(np.int64)
        else:
            b = st.pop()
            a = st.pop()
            if op == "add": r = a + b
            elif op == "sub": r = a - b
            elif op == "mul": r = a * b
            elif op == "div": r = _cdiv(a, b)
            elif op == "mod": r = a - b * _cdiv(a, b)
            elif op == "shl": r = a * (np.int64(2) ** b)
            elif op == "shr": r = np.right_shift(a, b)
            elif op == "and": r = a & b
            elif op == "or": r = a | b
            elif op == "xor": r = a ^ b
            elif op == "min": r = np.minimum(a, b)
            elif op == "max": r = np.maximum(a, b)
            elif op == "lt": r = (a < b).astype(np.int64)
            elif op == "le": r = (a <= b).astype(np.int64)
            elif op == "eq": r = (a == b).astype(np.int64)
            elif op == "ne": r = (a != b).astype(np.int64)
            elif op == "ge": r = (a >= b).astype(np.int64)
            elif op == "gt": r = (a > b).astype(np.int64)
            elif op == "land": r = ((a != 0) & (b != 0)).astype(np.int64)
            elif op == "lor": r = ((a != 0) | (b != 0)).astype(np.int64)
            else: raise ValueError(op)
            st.append(r)
    assert len(st) == 1
    return st[0]


def _scalar(expr, params, dims=None):
    env = {("param", k): v for k, v in enumerate(params)}
    if dims:
        g, b = dims
        for d in range(3):
            env[("gdim", d)] = g[d]
            env[("bdim", d)] = b[d]
    return int(ev(expr, env, (), 0))


def loop_values(loop, params, dims):
    v = _scalar(loop.init, params, dims)
    bound = _scalar(loop.bound, params, dims)
    step = _scalar(loop.step, params, dims)
    out = []
    while _CMP[loop.cmp](v, bound):
        out.append(v)
        if loop.upd == "add": v += step
        elif loop.upd == "sub": v -= step
        elif loop.upd == "mul": v *= step
        elif loop.upd == "shl": v *= 2 ** step
        elif loop.upd == "shr": v >>= step
        else: v = int(_cdiv(np.int64(v), np.int64(step)))
        assert len(out) <= 65536
    return out


def points(model, acc_index, s):
    """Arrays (addr, blin, tlin, ilin, bint, wint) of guarded points of one
    access under tuple s, or None if the launch box is empty."""
    params = model.param_sets[s]
    g = [_scalar(x, params) for x in model.launch.grid]
    b = [_scalar(x, params) for x in model.launch.block]
    if min(g) < 1 or min(b) < 1:
        return None
    a = model.accesses[acc_index]
    lv = [loop_values(model.loops[k], params, (g, b)) for k in a.loops]
    niota = int(np.prod([len(v) for v in lv])) if lv else 1
    nb, nt = g[0] * g[1] * g[2], b[0] * b[1] * b[2]
    bl, tl, il = np.meshgrid(np.arange(nb), np.arange(nt), np.arange(niota), indexing="ij")
    bl, tl, il = bl.ravel(), tl.ravel(), il.ravel()
    env = {("param", k): v for k, v in enumerate(params)}
    for d in range(3):
        env[("gdim", d)] = g[d]
        env[("bdim", d)] = b[d]
    env[("bid", 0)] = bl % g[0]
    env[("bid", 1)] = (bl // g[0]) % g[1]
    env[("bid", 2)] = bl // (g[0] * g[1])
    env[("tid", 0)] = tl % b[0]
    env[("tid", 1)] = (tl // b[0]) % b[1]
    env[("tid", 2)] = tl // (b[0] * b[1])
    rem = il.copy()
    for pos in range(len(a.loops) - 1, -1, -1):
        vals = np.asarray(lv[pos], dtype=np.int64)
        env[("loop", a.loops[pos])] = vals[rem % len(vals)] if len(vals) else rem
        rem = rem // max(1, len(vals))
    shape = bl.shape
    guard = ev(a.guard, env, shape, 1) != 0
    addr = ev(a.addr, env, shape, 0)
    bi = ev(a.bint, env, shape, 0)
    wi = ev(a.wint, env, shape, 0)
    sel = guard
    return addr[sel], bl[sel], tl[sel], il[sel], bi[sel], wi[sel]
