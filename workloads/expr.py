"""A tiny builder for postfix integer expressions.

An expression is a list of tokens in postfix order.  Leaves are constants,
kernel parameters, thread/block coordinates, launch dimensions and loop
variables; inner nodes are C integer operators.  The operators and their
meaning follow the address/guard arithmetic that the paper's constraint
generator reads from kernel code (section 6.2, Table 2) and the host-side
expression trees (section 6.3, Figure 8a): constants, unknown inputs and
binary operations.

Tokens are tuples: ("const", v), ("param", k), ("tid", d), ("bid", d),
("bdim", d), ("gdim", d), ("loop", k), and (op,) for the operators in OPS.
Nothing here evaluates an expression.
"""

BINARY = ("add", "sub", "mul", "div", "mod", "shl", "shr", "and", "or", "xor",
          "min", "max", "lt", "le", "eq", "ne", "ge", "gt", "land", "lor")
UNARY = ("neg", "lnot")
LEAVES = ("const", "param", "tid", "bid", "bdim", "gdim", "loop")
OPS = LEAVES + BINARY + UNARY


class E:
    """A postfix expression; Python operators build larger expressions."""

    __slots__ = ("code",)

    def __init__(self, code):
        self.code = list(code)

    # arithmetic -----------------------------------------------------------
    def __add__(self, o):
        return _bin("add", self, o)

    def __radd__(self, o):
        return _bin("add", o, self)

    def __sub__(self, o):
        return _bin("sub", self, o)

    def __rsub__(self, o):
        return _bin("sub", o, self)

    def __mul__(self, o):
        return _bin("mul", self, o)

    def __rmul__(self, o):
        return _bin("mul", o, self)

    def __floordiv__(self, o):  # C truncating division, not Python floor
        return _bin("div", self, o)

    def __mod__(self, o):  # C remainder (sign of the dividend)
        return _bin("mod", self, o)

    def __lshift__(self, o):
        return _bin("shl", self, o)

    def __rshift__(self, o):
        return _bin("shr", self, o)

    def __and__(self, o):
        return _bin("and", self, o)

    def __or__(self, o):
        return _bin("or", self, o)

    def __xor__(self, o):
        return _bin("xor", self, o)

    def __neg__(self):
        return E(self.code + [("neg",)])

    def __repr__(self):
        return "E(%r)" % (self.code,)

    def to_json(self):
        return [list(t) for t in self.code]

    @staticmethod
    def from_json(j):
        return E([tuple(t) for t in j])


def lift(x):
    if isinstance(x, E):
        return x
    if isinstance(x, bool):
        x = int(x)
    if isinstance(x, int):
        return E([("const", int(x))])
    raise TypeError("cannot make an expression from %r" % (x,))


def _bin(op, a, b):
    return E(lift(a).code + lift(b).code + [(op,)])


def c(v):
    return lift(int(v))


def param(k):
    return E([("param", int(k))])


def tid(d=0):
    return E([("tid", int(d))])


def bid(d=0):
    return E([("bid", int(d))])


def bdim(d=0):
    return E([("bdim", int(d))])


def gdim(d=0):
    return E([("gdim", int(d))])


def loop(k):
    return E([("loop", int(k))])


def div(a, b):
    return _bin("div", a, b)


def mod(a, b):
    return _bin("mod", a, b)


def shl(a, b):
    return _bin("shl", a, b)


def shr(a, b):
    return _bin("shr", a, b)


def band(a, b):
    return _bin("and", a, b)


def bor(a, b):
    return _bin("or", a, b)


def bxor(a, b):
    return _bin("xor", a, b)


def emin(a, b):
    return _bin("min", a, b)


def emax(a, b):
    return _bin("max", a, b)


def lt(a, b):
    return _bin("lt", a, b)


def le(a, b):
    return _bin("le", a, b)


def eq(a, b):
    return _bin("eq", a, b)


def ne(a, b):
    return _bin("ne", a, b)


def ge(a, b):
    return _bin("ge", a, b)


def gt(a, b):
    return _bin("gt", a, b)


def land(a, b):
    return _bin("land", a, b)


def lor(a, b):
    return _bin("lor", a, b)


def lnot(a):
    return E(lift(a).code + [("lnot",)])


def neg(a):
    return E(lift(a).code + [("neg",)])
