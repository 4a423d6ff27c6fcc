"""CPU oracle for the exact per-access-pair race query (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library: ``hgrd_oracle.c`` has its own
structures, opcode numbers and checked int64 evaluator, and this loader has
its own marshalling.  The only thing both sides take from elsewhere is the
seeded input description in ``workloads``.

Two methods (see the header of hgrd_oracle.c):
  method="A"  the definition written out: a double loop over point pairs;
  method="B"  sort + prefix-group counting, pinned to method A by tests.
"""
import ctypes as C
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgrd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# oracle-local opcode numbering (mirrors the enum in hgrd_oracle.c only)
_OPC = {"const": 1, "param": 2, "tid": 3, "bid": 4, "bdim": 5, "gdim": 6,
        "loop": 7, "add": 20, "sub": 21, "mul": 22, "div": 23, "mod": 24,
        "shl": 25, "shr": 26, "and": 27, "or": 28, "xor": 29, "min": 30,
        "max": 31, "lt": 32, "le": 33, "eq": 34, "ne": 35, "ge": 36, "gt": 37,
        "land": 38, "lor": 39, "neg": 60, "lnot": 61}
_KIND = {"read": 0, "write": 1, "atomic": 2}
_SCOPE = {"block": 0, "device": 1}
_SPACE = {"global": 0, "shared": 1}
_CMP = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "ne": 4}
_UPD = {"add": 0, "sub": 1, "mul": 2, "div": 3, "shl": 4, "shr": 5}

STATUS = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "ERANGE",
          -4: "EDIVZERO"}


class OTok(C.Structure):
    _fields_ = [("op", C.c_int64), ("arg", C.c_int64)]


class OExpr(C.Structure):
    _fields_ = [("first", C.c_int32), ("count", C.c_int32)]


class OArray(C.Structure):
    _fields_ = [("space", C.c_int32), ("addr_bits", C.c_int32), ("alias", C.c_int32),
                ("pad", C.c_int32), ("base", C.c_int64)]


class OLoop(C.Structure):
    _fields_ = [("init", OExpr), ("bound", OExpr), ("step", OExpr),
                ("cmp", C.c_int32), ("upd", C.c_int32)]


class OSync(C.Structure):
    _fields_ = [("addr", OExpr), ("array", C.c_int32), ("scope", C.c_int32)]


class OAccess(C.Structure):
    _fields_ = [("array", C.c_int32), ("kind", C.c_int32), ("scope", C.c_int32),
                ("n_loops", C.c_int32), ("loops", C.c_int32 * 8),
                ("addr", OExpr), ("guard", OExpr), ("bint", OExpr),
                ("wint", OExpr), ("acq", OSync), ("rel", OSync)]


class OModel(C.Structure):
    _fields_ = [("toks", C.POINTER(OTok)), ("n_toks", C.c_int32),
                ("arrays", C.POINTER(OArray)), ("n_arrays", C.c_int32),
                ("loops", C.POINTER(OLoop)), ("n_loops", C.c_int32),
                ("acc", C.POINTER(OAccess)), ("n_acc", C.c_int32),
                ("n_params", C.c_int32),
                ("grid", OExpr * 3), ("block", OExpr * 3),
                ("warp", C.c_int32), ("n_sets", C.c_int32),
                ("sets", C.POINTER(C.c_int64))]


class OPair(C.Structure):
    _fields_ = [("model", C.c_int32), ("a", C.c_int32), ("b", C.c_int32),
                ("mask", C.c_int32)]


class OResult(C.Structure):
    _fields_ = [("count", C.c_uint64), ("by_class", C.c_uint64 * 3),
                ("status", C.c_int32), ("verdict", C.c_int32),
                ("classes", C.c_int32), ("witness_class", C.c_int32),
                ("flags", C.c_int32), ("pad", C.c_int32),
                ("w_set", C.c_int64), ("w_b1", C.c_int64), ("w_t1", C.c_int64),
                ("w_i1", C.c_int64), ("w_b2", C.c_int64), ("w_t2", C.c_int64),
                ("w_i2", C.c_int64), ("w_addr", C.c_int64),
                ("evals", C.c_uint64)]


def build(force=False):
    """Compile hgrd_oracle.c with gcc into oracle/liboracle.so."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lpthread"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.oracle_check_pairs.restype = C.c_int
        _lib.oracle_check_pairs.argtypes = [
            C.POINTER(OModel), C.c_int32, C.POINTER(OPair), C.c_int32,
            C.c_int32, C.c_int32, C.POINTER(OResult)]
        _lib.oracle_eval_uniform.restype = C.c_int64
        _lib.oracle_eval_uniform.argtypes = [C.POINTER(OModel), OExpr, C.c_int32,
                                             C.POINTER(C.c_int32)]
        _lib.oracle_conflict_class.restype = C.c_int
        _lib.oracle_conflict_class.argtypes = [
            C.c_int64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
            C.c_int64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
            C.c_int64, C.c_int32]
    return _lib


class _Packed:
    """ctypes image of one model; keeps every buffer alive."""

    def __init__(self, model):
        toks = []

        def put(e):
            if e is None:
                return OExpr(0, 0)
            first = len(toks)
            for t in e.code:
                op = _OPC.get(t[0], 0)  # unknown names become invalid opcode 0
                arg = int(t[1]) if len(t) > 1 else 0
                toks.append((op, arg))
            return OExpr(first, len(e.code))

        self.arrays = (OArray * max(1, len(model.arrays)))(
            *[OArray(_SPACE[a.space], a.addr_bits, getattr(a, "alias", 0), 0,
                     getattr(a, "base", 0)) for a in model.arrays])
        loops = []
        for l in model.loops:
            loops.append(OLoop(put(l.init), put(l.bound), put(l.step),
                               _CMP[l.cmp], _UPD[l.upd]))
        self.loops = (OLoop * max(1, len(loops)))(*loops)
        accs = []
        for a in model.accesses:
            oa = OAccess()
            oa.array, oa.kind, oa.scope = a.array, _KIND[a.kind], _SCOPE[a.scope]
            oa.n_loops = len(a.loops)
            for i, k in enumerate(a.loops[:8]):
                oa.loops[i] = k
            oa.addr, oa.guard = put(a.addr), put(a.guard)
            oa.bint, oa.wint = put(a.bint), put(a.wint)
            for k in ("acq", "rel"):
                sy = getattr(a, k, None)
                if sy is not None:
                    setattr(oa, k, OSync(put(sy.addr), sy.array, _SCOPE[sy.scope]))
            accs.append(oa)
        self.acc = (OAccess * max(1, len(accs)))(*accs)
        grid = [put(x) for x in model.launch.grid]
        block = [put(x) for x in model.launch.block]
        self.toks = (OTok * max(1, len(toks)))(*[OTok(o, a) for o, a in toks])
        flat = [v for row in model.param_sets for v in row]
        self.sets = (C.c_int64 * max(1, len(flat)))(*flat)
        m = OModel()
        m.toks, m.n_toks = self.toks, len(toks)
        m.arrays, m.n_arrays = self.arrays, len(model.arrays)
        m.loops, m.n_loops = self.loops, len(loops)
        m.acc, m.n_acc = self.acc, len(accs)
        m.n_params = model.n_params
        for d in range(3):
            m.grid[d] = grid[d]
            m.block[d] = block[d]
        m.warp = model.launch.warp
        m.n_sets = len(model.param_sets)
        m.sets = self.sets
        self.m = m


def _result_dict(r):
    return {"status": r.status, "verdict": r.verdict, "count": r.count,
            "by_class": [r.by_class[0], r.by_class[1], r.by_class[2]],
            "classes": r.classes, "witness_class": r.witness_class,
            "flags": r.flags,
            "witness": (r.w_set, r.w_b1, r.w_t1, r.w_i1, r.w_b2, r.w_t2, r.w_i2),
            "w_addr": r.w_addr, "evals": r.evals}


def check_pairs(workload, method="B", threads=None):
    """Run the oracle on every pair of ``workload``.

    Returns (list of result dicts, number of host threads used).
    """
    L = lib()
    packed = [_Packed(m) for m in workload.models]
    models = (OModel * max(1, len(packed)))(*[p.m for p in packed])
    pairs = (OPair * max(1, len(workload.pairs)))(
        *[OPair(m, a, b, k) for (m, a, b, k) in workload.pairs])
    out = (OResult * max(1, len(workload.pairs)))()
    if threads is None:
        threads = os.cpu_count() or 1
    used = L.oracle_check_pairs(models, len(packed), pairs, len(workload.pairs),
                                0 if method == "A" else 1, int(threads), out)
    return [_result_dict(out[k]) for k in range(len(workload.pairs))], used


def eval_uniform(expr, params):
    """Evaluate a parameter-only expression with the oracle's int64 rules.

    Returns (value, error bits) with bits 1 = divide by zero, 2 = out of
    range, 8 = malformed.
    """
    from workloads import Model, Launch, Array, Access
    m = Model(len(params), [Array()], [Access(0, "read", 0)], Launch(),
              [list(params)])
    p = _Packed(m)
    first = p.m.n_toks
    # append the expression to the token pool
    toks = [(_OPC.get(t[0], 0), int(t[1]) if len(t) > 1 else 0) for t in expr.code]
    allt = [(p.toks[i].op, p.toks[i].arg) for i in range(p.m.n_toks)] + toks
    p.toks = (OTok * max(1, len(allt)))(*[OTok(o, a) for o, a in allt])
    p.m.toks, p.m.n_toks = p.toks, len(allt)
    err = C.c_int32(0)
    v = lib().oracle_eval_uniform(C.byref(p.m), OExpr(first, len(toks)), 0,
                                  C.byref(err))
    return v, err.value


def conflict_class(p, q, warp, mask):
    """Oracle conflict predicate on explicit points.

    p, q: (addr, blin, tlin, bint, wint).  Returns the class bit or 0.
    """
    return lib().oracle_conflict_class(p[0], p[1], p[2], p[3], p[4],
                                       q[0], q[1], q[2], q[3], q[4],
                                       warp, mask)
