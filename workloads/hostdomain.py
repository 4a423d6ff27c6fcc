"""Host-domain containers (plain data, no evaluation): what a program's host
code fixes about a kernel launch, in the five classes of section 4 (asserts,
grid dimensions, parameters derived from one host variable, host loop
iterators, allocation sizes).  The library's rd_expand_host_domain turns one
into the parameter tuples of a kernel model.

Expressions are the same ``E`` trees as kernel models; ``param(k)`` reads
host variable k.
"""
from .expr import lift

INPUT, EXPR, LOOP = "input", "expr", "loop"


class HostVar:
    """One host variable, in program order.

    * ``HostVar.input(values)``: an input the program reads; it takes each
      of the finite stand-in values in turn.
    * ``HostVar.expr(e)``: computed from earlier variables.
    * ``HostVar.loop(init, cmp, bound, upd, step)``: the iterator of a host
      loop ``for (v = init; v <cmp> bound; v = v <upd> step)``.
    """

    def __init__(self, kind, values=(), init=None, cmp="lt", bound=None,
                 upd="add", step=None):
        self.kind, self.values = kind, [int(v) for v in values]
        self.init = None if init is None else lift(init)
        self.cmp, self.upd = cmp, upd
        self.bound = None if bound is None else lift(bound)
        self.step = None if step is None else lift(step)

    @staticmethod
    def input(values):
        return HostVar(INPUT, values=values)

    @staticmethod
    def expr(e):
        return HostVar(EXPR, init=e)

    @staticmethod
    def loop(init, cmp, bound, upd="add", step=1):
        return HostVar(LOOP, init=init, cmp=cmp, bound=bound, upd=upd, step=step)


class HostDomain:
    """Host variables, asserts (class 1), allocation sizes (class 5) and one
    expression per kernel parameter (classes 2 and 3)."""

    def __init__(self, variables, params, asserts=(), alloc_sizes=(), name=""):
        self.vars = list(variables)
        self.params = [lift(e) for e in params]
        self.asserts = [lift(e) for e in asserts]
        self.alloc_sizes = [lift(e) for e in alloc_sizes]
        self.name = name
