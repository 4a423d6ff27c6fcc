"""Kernel-model and workload containers (plain data, no evaluation).

A kernel model describes one analysed GPU kernel as the race query sees it:

* arrays, each in global or shared memory (shared memory belongs to one
  thread block, section 2 "Data races on GPUs");
* loops with uniform bounds (init, comparison, bound, update, step);
* accesses (section 6.1 "Generating access pairs"): a load, store or atomic on
  one array, inside a set of loops, with an address expression, a guard (the
  branch condition under which the access executes), and two barrier-interval
  ids, ``bint`` (block barriers) and ``wint`` (warp barriers), that stand for
  the dominance checks of section 6.1;
* optionally, the acquire and release that guard an access (section 6.5,
  Figure 9; appendix A): the address expression of each, the array holding
  the lock or flag, and its scope;
* launch geometry (grid and block extents as expressions over parameters,
  section 6.3 class 2) and the warp size;
* host-fixed parameter tuples: each tuple is one launch, and its values are
  joint (section 6.3 class 3), already filtered by host asserts (class 1),
  loop bounds (class 4) and allocation-size positivity (class 5).

A workload is a list of models plus a list of access pairs
(model, access a, access b, caller class mask).
"""
import json

from .expr import E, lift

READ, WRITE, ATOMIC = "read", "write", "atomic"
SCOPE_BLOCK, SCOPE_DEVICE = "block", "device"
GLOBAL, SHARED = "global", "shared"
INTER, INTRA_BLOCK, INTRA_WARP = 1, 2, 4
ALL_CLASSES = 7

KINDS = (READ, WRITE, ATOMIC)
SCOPES = (SCOPE_BLOCK, SCOPE_DEVICE)
SPACES = (GLOBAL, SHARED)
CMPS = ("lt", "le", "gt", "ge", "ne")
UPDS = ("add", "sub", "mul", "div", "shl", "shr")


def _opt(e):
    return None if e is None else lift(e)


class Array:
    """An array; arrays with the same nonzero ``alias`` are views of one
    memory, element k of the view being element base + k of the memory."""

    def __init__(self, space=GLOBAL, addr_bits=64, alias=0, base=0):
        assert space in SPACES and addr_bits in (32, 64)
        self.space, self.addr_bits = space, addr_bits
        self.alias, self.base = int(alias), int(base)

    def to_json(self):
        j = {"space": self.space, "addr_bits": self.addr_bits}
        if self.alias:
            j["alias"], j["base"] = self.alias, self.base
        return j


class Loop:
    """for (v = init; v <cmp> bound; v = v <upd> step)."""

    def __init__(self, init, cmp, bound, upd="add", step=1):
        assert cmp in CMPS and upd in UPDS
        self.init, self.cmp, self.bound = lift(init), cmp, lift(bound)
        self.upd, self.step = upd, lift(step)

    def to_json(self):
        return {"init": self.init.to_json(), "cmp": self.cmp,
                "bound": self.bound.to_json(), "upd": self.upd,
                "step": self.step.to_json()}


class Sync:
    """An acquire (atomicCAS then fence) or release (fence then atomicExch)
    around an access: the address it synchronises on, in array ``array``,
    and its scope, the narrower of its atomic's and its fence's."""

    def __init__(self, array, addr, scope=SCOPE_DEVICE):
        assert scope in SCOPES
        self.array, self.addr, self.scope = int(array), lift(addr), scope

    def to_json(self):
        return {"array": self.array, "addr": self.addr.to_json(),
                "scope": self.scope}

    @staticmethod
    def from_json(j):
        return None if j is None else Sync(j["array"], E.from_json(j["addr"]),
                                           j["scope"])


class Access:
    def __init__(self, array, kind, addr, guard=None, loops=(), bint=None,
                 wint=None, scope=SCOPE_DEVICE, name="", acq=None, rel=None):
        assert kind in KINDS and scope in SCOPES
        self.array, self.kind, self.scope = int(array), kind, scope
        self.addr, self.guard = lift(addr), _opt(guard)
        self.loops = [int(k) for k in loops]
        self.bint, self.wint = _opt(bint), _opt(wint)
        self.name = name
        self.acq, self.rel = acq, rel

    def to_json(self):
        j = {"array": self.array, "kind": self.kind, "scope": self.scope,
             "loops": self.loops, "addr": self.addr.to_json()}
        for k in ("guard", "bint", "wint"):
            v = getattr(self, k)
            j[k] = None if v is None else v.to_json()
        if self.name:
            j["name"] = self.name
        for k in ("acq", "rel"):
            v = getattr(self, k)
            if v is not None:
                j[k] = v.to_json()
        return j


class Launch:
    def __init__(self, grid=(1, 1, 1), block=(1, 1, 1), warp=32):
        g = list(grid) + [1] * (3 - len(grid))
        b = list(block) + [1] * (3 - len(block))
        self.grid = [lift(x) for x in g]
        self.block = [lift(x) for x in b]
        self.warp = int(warp)

    def to_json(self):
        return {"grid": [x.to_json() for x in self.grid],
                "block": [x.to_json() for x in self.block], "warp": self.warp}


class Model:
    def __init__(self, n_params, arrays, accesses, launch, param_sets,
                 loops=(), name=""):
        self.n_params = int(n_params)
        self.arrays = list(arrays)
        self.loops = list(loops)
        self.accesses = list(accesses)
        self.launch = launch
        self.param_sets = [[int(v) for v in row] for row in param_sets]
        self.name = name
        for row in self.param_sets:
            assert len(row) == self.n_params, (name, row)

    def to_json(self):
        return {"name": self.name, "n_params": self.n_params,
                "arrays": [a.to_json() for a in self.arrays],
                "loops": [l.to_json() for l in self.loops],
                "accesses": [a.to_json() for a in self.accesses],
                "launch": self.launch.to_json(),
                "param_sets": self.param_sets}

    @staticmethod
    def from_json(j):
        arrays = [Array(a["space"], a["addr_bits"], a.get("alias", 0), a.get("base", 0))
                  for a in j["arrays"]]
        loops = [Loop(E.from_json(l["init"]), l["cmp"], E.from_json(l["bound"]),
                      l["upd"], E.from_json(l["step"])) for l in j["loops"]]
        accs = []
        for a in j["accesses"]:
            op = lambda k: None if a.get(k) is None else E.from_json(a[k])
            accs.append(Access(a["array"], a["kind"], E.from_json(a["addr"]),
                               op("guard"), a["loops"], op("bint"), op("wint"),
                               a["scope"], a.get("name", ""),
                               Sync.from_json(a.get("acq")),
                               Sync.from_json(a.get("rel"))))
        la = j["launch"]
        launch = Launch([E.from_json(x) for x in la["grid"]],
                        [E.from_json(x) for x in la["block"]], la["warp"])
        return Model(j["n_params"], arrays, accs, launch, j["param_sets"],
                     loops, j.get("name", ""))


class Workload:
    """Models plus access pairs (model index, access a, access b, mask)."""

    def __init__(self, models, pairs, name="", meta=None):
        self.models = list(models)
        self.pairs = [(int(m), int(a), int(b), int(k)) for (m, a, b, k) in pairs]
        self.name = name
        self.meta = dict(meta or {})

    def to_json(self):
        return {"name": self.name, "meta": self.meta,
                "models": [m.to_json() for m in self.models],
                "pairs": [list(p) for p in self.pairs]}

    def dumps(self):
        return json.dumps(self.to_json(), sort_keys=True)

    @staticmethod
    def from_json(j):
        return Workload([Model.from_json(m) for m in j["models"]],
                        [tuple(p) for p in j["pairs"]], j.get("name", ""),
                        j.get("meta", {}))

    def subset(self, idx):
        """A workload with only the pairs in ``idx`` (models kept)."""
        return Workload(self.models, [self.pairs[i] for i in idx],
                        self.name + "[subset]", self.meta)

    def compact(self, idx):
        """A workload with only the pairs in ``idx`` and the models they
        use, renumbered in order of first use (the same queries)."""
        remap, models, pairs = {}, [], []
        for i in idx:
            m, a, b, k = self.pairs[i]
            if m not in remap:
                remap[m] = len(models)
                models.append(self.models[m])
            pairs.append((remap[m], a, b, k))
        meta = dict(self.meta)
        if "evals" in meta:
            meta["evals"] = [meta["evals"][i] for i in idx]
        return Workload(models, pairs, self.name + "[compact]", meta)
