"""Hand-built kernel models with verdicts known without running the query.

Two groups:

* closed-form families F1-F4 (tests derive their expected counts, class
  counts and witnesses by hand, independently of any checker):
    F1  neighbour writes A[g] and A[g+1]      (global)
    F2  tree reduction with a missing barrier (shared)
    F3  stride-aliasing modulo index A[tid % W]
    F4  guard-disjoint halves A[tid % H]
* the paper's worked examples K1-K5, written from its printed snippets
  (section 4, Figures 1-5), with the launch geometry the paper leaves out
  chosen here and stated in each docstring.
"""
from .expr import bid, bdim, gdim, tid, param, loop, c, eq, gt, lt, land, shr
from .model import (Access, Array, Launch, Loop, Model, Workload, GLOBAL,
                    SHARED, READ, WRITE, ALL_CLASSES)


# ---------------------------------------------------------------------------
# closed-form families

def f1_neighbour(G=4, B=64, warp=32):
    """W A[g] vs W A[g+1], g = blockIdx.x * blockDim.x + threadIdx.x.

    Accesses: 0 = A[g], 1 = A[g+1].  One tuple, no parameters.
    """
    g = bid(0) * bdim(0) + tid(0)
    m = Model(0, [Array(GLOBAL, 32)],
              [Access(0, WRITE, g, name="A[g]"),
               Access(0, WRITE, g + 1, name="A[g+1]")],
              Launch((G, 1, 1), (B, 1, 1), warp), [[]], name="F1")
    return m


def f2_tree_reduction(B=64, warp=32, barrier=False):
    """Shared-memory tree reduction in one block of B = 2^L threads.

    for k in [0, L): s = B >> (k + 1); if (tid < s) sd[tid] += sd[tid + s]
    Accesses: 0 = write sd[tid], 1 = read sd[tid + s], 2 = read sd[tid].
    Without a barrier in the loop body every iteration is in one barrier
    interval (bint = 0); with it, iteration k is interval k (bint = k).
    """
    L = B.bit_length() - 1
    assert 1 << L == B
    s = shr(bdim(0), loop(0) + 1)
    guard = lt(tid(0), s)
    bi = loop(0) if barrier else None
    m = Model(0, [Array(SHARED, 32)],
              [Access(0, WRITE, tid(0), guard, [0], bint=bi, name="W sd[tid]"),
               Access(0, READ, tid(0) + s, guard, [0], bint=bi,
                      name="R sd[tid+s]"),
               Access(0, READ, tid(0), guard, [0], bint=bi, name="R sd[tid]")],
              Launch((1, 1, 1), (B, 1, 1), warp), [[]],
              loops=[Loop(0, "lt", L, "add", 1)], name="F2")
    return m


def f3_stride_mod(B=64, Ws=(16,), warp=32, space=GLOBAL):
    """Self-pair W A[tid % W], one block, W a parameter (one tuple per W)."""
    m = Model(1, [Array(space, 32)],
              [Access(0, WRITE, tid(0) % param(0), name="A[tid%W]")],
              Launch((1, 1, 1), (B, 1, 1), warp), [[w] for w in Ws], name="F3")
    return m


def f4_guard_halves(B=64, extra=0, guarded=True, warp=32):
    """Self-pair W A[tid % H], H = B/2, guard tid < H + extra (or none)."""
    H = B // 2
    guard = lt(tid(0), H + extra) if guarded else None
    m = Model(0, [Array(GLOBAL, 32)],
              [Access(0, WRITE, tid(0) % H, guard, name="A[tid%H]")],
              Launch((1, 1, 1), (B, 1, 1), warp), [[]], name="F4")
    return m


# ---------------------------------------------------------------------------
# the paper's worked examples (section 4, Figures 1-5)

def k1_copy_upp_low(sets):
    """Figure 1: copyUppLowKernel, A[j*cols + i] = A[i*cols + j] under
    (j > i && j < rows), i = bid.x*bdim.x + tid.x, j = bid.y*bdim.y + tid.y.

    Parameters (rows, cols).  Geometry chosen here: 16x16 blocks and a grid of
    ceil(cols/16) x ceil(rows/16) blocks.  Accesses: 0 = read A[i*cols+j],
    1 = write A[j*cols+i].
    """
    rows, cols = param(0), param(1)
    i = bid(0) * bdim(0) + tid(0)
    j = bid(1) * bdim(1) + tid(1)
    guard = land(gt(j, i), lt(j, rows))
    return Model(2, [Array(GLOBAL, 32)],
                 [Access(0, READ, i * cols + j, guard, name="R A[i*cols+j]"),
                  Access(0, WRITE, j * cols + i, guard, name="W A[j*cols+i]")],
                 Launch(((cols + 15) // 16, (rows + 15) // 16, 1), (16, 16, 1)),
                 sets, name="K1")


def k2_reduce_final(sets, threads=256):
    """Figure 2: reduceFinal, if (threadIdx.x == 0) res[0] = ...

    Parameter (gridDim.x).  The host launches it with one block; other values
    stand for a host-agnostic analysis.  Access 0 = write res[0].
    """
    return Model(1, [Array(GLOBAL, 32)],
                 [Access(0, WRITE, c(0), eq(tid(0), 0), name="W res[0]")],
                 Launch((param(0), 1, 1), (threads, 1, 1)), sets, name="K2")


def k3_tone_mapping(sets):
    """Figure 3: toneMapping, output[width*channels*y + x*channels] = val.

    Parameters (width, gridDim.x, gridDim.y).  The host derives gridDim.x =
    hWidth/16 and width = hWidth from one variable (class 3); the 16x16
    block is implied by the /16.  channels = 4.  Access 0 = the write.
    """
    width = param(0)
    x = bid(0) * bdim(0) + tid(0)
    y = bid(1) * bdim(1) + tid(1)
    return Model(3, [Array(GLOBAL, 32)],
                 [Access(0, WRITE, width * 4 * y + x * 4, name="W output")],
                 Launch((param(1), param(2), 1), (16, 16, 1)), sets, name="K3")


def k4_lud_internal(sets, bs=16):
    """Figure 4: ludInternal, m[(rid + ty)*dim + cid + tx] = sum with
    rid = offset + (bid.y + 1)*BS, cid = offset + (bid.x + 1)*BS.

    Parameters (dim, offset).  Geometry assumed (not printed): BS = 16,
    16x16 blocks, a square grid of (dim - offset)/BS - 1 blocks per side, so
    that cid + tx < dim whenever offset >= 0.  Access 0 = the write.
    """
    dim, off = param(0), param(1)
    rid = off + (bid(1) + 1) * bs
    cid = off + (bid(0) + 1) * bs
    g = (dim - off) // bs - 1
    return Model(2, [Array(GLOBAL, 32)],
                 [Access(0, WRITE, (rid + tid(1)) * dim + cid + tid(0),
                         name="W m[...]")],
                 Launch((g, g, 1), (bs, bs, 1)), sets, name="K4")


def k5_shift(sets, width=64, rows=64):
    """Figure 5: shift, matrix[yid*(rowSize/4) + xid] = tex[...].

    Parameter (rowSize), the pitch in bytes returned by the pitched
    allocation.  Geometry chosen here: 16x16 blocks covering width x rows
    elements.  Access 0 = the write.
    """
    rs = param(0)
    xid = bid(0) * bdim(0) + tid(0)
    yid = bid(1) * bdim(1) + tid(1)
    return Model(1, [Array(GLOBAL, 32)],
                 [Access(0, WRITE, yid * (rs // 4) + xid, name="W matrix")],
                 Launch((width // 16, rows // 16, 1), (16, 16, 1)), sets,
                 name="K5")


def single(model, a, b, mask=ALL_CLASSES):
    """A one-pair workload."""
    return Workload([model], [(0, a, b, mask)], name=model.name)


# ---------------------------------------------------------------------------
# Host code of Figures 1-5 as host domains (section 4, classes 1-5).  Each
# returns the domain; unknown inputs take the finite stand-in values given.
# The parameter columns are those of the kernel model of the same figure.

def k1_host(rows=(16, 32, 48), cols=(1, 16, 32, 48)):
    """Figure 1 host code: rows and cols are inputs, the host asserts
    rows == cols (class 1), and passes (rows, cols)."""
    from .hostdomain import HostDomain, HostVar
    return HostDomain([HostVar.input(rows), HostVar.input(cols)],
                      params=[param(0), param(1)],
                      asserts=[eq(param(0), param(1))], name="K1 host")


def k2_host():
    """Figure 2 host code: reduceFinal is launched with a grid of one block
    (class 2); the model's one parameter is that grid extent."""
    from .hostdomain import HostDomain
    return HostDomain([], params=[c(1)], name="K2 host")


def k3_host(h_width=(16, 32, 48), h_height=(32,)):
    """Figure 3 host code: hWidth and hHeight are inputs; the grid is
    (hWidth / 16, hHeight / 16) and the kernel's width parameter is hWidth
    itself (class 3: both from one host variable).  Columns (width,
    gridDim.x, gridDim.y)."""
    from .hostdomain import HostDomain, HostVar
    hw, hh = param(0), param(1)
    return HostDomain([HostVar.input(h_width), HostVar.input(h_height)],
                      params=[hw, hw // 16, hh // 16], name="K3 host")


def k4_host(h_matrix_dim=(64,), step=16):
    """Figure 4 host code: hMatrixDim is an input and the kernel's offset is
    the iterator of for (hOffset = 0; hOffset < hMatrixDim; hOffset +=
    step) (class 4; the printed loop elides its update, the block size is
    used here).  Columns (dim, offset)."""
    from .hostdomain import HostDomain, HostVar
    return HostDomain([HostVar.input(h_matrix_dim),
                       HostVar.loop(0, "lt", param(0), "add", step)],
                      params=[param(0), param(1)], name="K4 host")


def k5_host(pitches=(0, 256, 512)):
    """Figure 5 host code: hRowSize is the pitch a pitched allocation
    returns (stand-in values) and sizes that allocation, so it is positive
    in every execution (class 5).  Column (rowSize)."""
    from .hostdomain import HostDomain, HostVar
    return HostDomain([HostVar.input(pitches)], params=[param(0)],
                      alloc_sizes=[param(0)], name="K5 host")
