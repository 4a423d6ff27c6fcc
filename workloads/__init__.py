"""Seeded synthetic inputs for the exact per-access-pair race query.

This package builds kernel models (accesses with address, guard and
barrier-interval expressions, loops, launch geometry and host-fixed parameter
tuples) and access-pair lists.  It holds no part of the race query itself: it
never evaluates an expression, enumerates a thread or compares addresses.  Both
the CPU oracle and the GPU library consume its output, each through its own
marshalling code.
"""
from .expr import (E, c, param, tid, bid, bdim, gdim, loop, div, mod, shl, shr,
                   band, bor, bxor, emin, emax, lt, le, eq, ne, ge, gt, land,
                   lor, lnot, neg, OPS)
from .model import (Model, Workload, Access, Sync, Loop, Array, Launch, READ, WRITE,
                    ATOMIC, SCOPE_BLOCK, SCOPE_DEVICE, GLOBAL, SHARED, INTER,
                    INTRA_BLOCK, INTRA_WARP, ALL_CLASSES)
from .hostdomain import HostDomain, HostVar
