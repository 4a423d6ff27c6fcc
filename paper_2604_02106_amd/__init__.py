"""MI355X exact per-access-pair race query: Python binding.

A thin ctypes layer over ``libhgrd.so`` (declared in ``include/hgrd.h``).  It
only marshals a ``workloads.Workload`` into the C structures and passes the
current torch stream; every step of the query runs in the library's gfx950
kernels.  There is no CPU fallback: without the built library or a GPU the
calls raise.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgrd.so")

RD_OK, RD_EINVAL, RD_EUNSUPPORTED, RD_ERANGE, RD_EDIVZERO = 0, -1, -2, -3, -4
RD_ENOMEM, RD_EDEVICE, RD_ECAPACITY = -5, -6, -7
MODE_EXACT, MODE_VERDICT = 0, 1
ORDER_LEX, ORDER_MLP, ORDER_INTERVAL = 0, 1, 2

# opcode numbers of include/hgrd.h
_OP = {"const": 1, "param": 2, "tid": 3, "bid": 4, "bdim": 5, "gdim": 6,
       "loop": 7, "add": 16, "sub": 17, "mul": 18, "div": 19, "mod": 20,
       "shl": 21, "shr": 22, "and": 23, "or": 24, "xor": 25, "min": 26,
       "max": 27, "lt": 28, "le": 29, "eq": 30, "ne": 31, "ge": 32, "gt": 33,
       "land": 34, "lor": 35, "neg": 48, "lnot": 49}
_KIND = {"read": 0, "write": 1, "atomic": 2}
_SCOPE = {"block": 0, "device": 1}
_SPACE = {"global": 0, "shared": 1}
_CMP = {"lt": 0, "le": 1, "gt": 2, "ge": 3, "ne": 4}
_UPD = {"add": 0, "sub": 1, "mul": 2, "div": 3, "shl": 4, "shr": 5}


class rd_insn(C.Structure):
    _fields_ = [("op", C.c_uint16), ("arg", C.c_uint16), ("pad", C.c_uint32),
                ("imm", C.c_int64)]


class rd_expr(C.Structure):
    _fields_ = [("first", C.c_uint32), ("count", C.c_uint32)]


class rd_array(C.Structure):
    _fields_ = [("space", C.c_uint32), ("addr_bits", C.c_uint32), ("alias", C.c_uint32),
                ("pad", C.c_uint32), ("base", C.c_int64)]


class rd_loop(C.Structure):
    _fields_ = [("init", rd_expr), ("bound", rd_expr), ("step", rd_expr),
                ("cmp", C.c_uint32), ("upd", C.c_uint32)]


class rd_sync(C.Structure):
    _fields_ = [("addr", rd_expr), ("array", C.c_uint32), ("scope", C.c_uint32)]


class rd_access(C.Structure):
    _fields_ = [("array", C.c_uint32), ("kind", C.c_uint32),
                ("scope", C.c_uint32), ("n_loops", C.c_uint32),
                ("loops", C.c_uint32 * 4), ("addr", rd_expr),
                ("guard", rd_expr), ("bint", rd_expr), ("wint", rd_expr),
                ("acq", rd_sync), ("rel", rd_sync)]


class rd_kernel_model(C.Structure):
    _fields_ = [("insns", C.POINTER(rd_insn)), ("n_insns", C.c_uint32),
                ("arrays", C.POINTER(rd_array)), ("n_arrays", C.c_uint32),
                ("loops", C.POINTER(rd_loop)), ("n_loops", C.c_uint32),
                ("acc", C.POINTER(rd_access)), ("n_acc", C.c_uint32),
                ("n_params", C.c_uint32)]


class rd_launch_domain(C.Structure):
    _fields_ = [("grid", rd_expr * 3), ("block", rd_expr * 3),
                ("warp_size", C.c_uint32), ("pad", C.c_uint32)]


class rd_param_sets(C.Structure):
    _fields_ = [("n_sets", C.c_uint32), ("pad", C.c_uint32),
                ("values", C.POINTER(C.c_int64))]


class rd_stmt(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("arg", C.c_uint32), ("array", C.c_uint32),
                ("scope", C.c_uint32), ("addr", rd_expr)]


class rd_access_pair(C.Structure):
    _fields_ = [("model", C.c_uint32), ("a", C.c_uint32), ("b", C.c_uint32),
                ("class_mask", C.c_uint32)]


class rd_host_var(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("cmp", C.c_uint32), ("upd", C.c_uint32),
                ("n_values", C.c_uint32), ("values", C.POINTER(C.c_int64)),
                ("init", rd_expr), ("bound", rd_expr), ("step", rd_expr)]


class rd_host_domain(C.Structure):
    _fields_ = [("insns", C.POINTER(rd_insn)), ("n_insns", C.c_uint32),
                ("vars", C.POINTER(rd_host_var)), ("n_vars", C.c_uint32),
                ("asserts", C.POINTER(rd_expr)), ("n_asserts", C.c_uint32),
                ("alloc_sizes", C.POINTER(rd_expr)), ("n_alloc", C.c_uint32),
                ("params", C.POINTER(rd_expr)), ("n_params", C.c_uint32)]


N_MLP = 6337  # 32*64 + 64 + 64*64 + 64 + 64 + 1
rd_mlp = C.c_float * N_MLP  # w1, b1, w2, b2, w3, b3 (include/hgrd.h)


class rd_options(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("order", C.c_uint32),
                ("prefilter", C.c_uint32), ("log_level", C.c_uint32),
                ("lds_cap", C.c_uint32), ("tile_budget", C.c_uint32),
                ("mlp", C.c_void_p),
                ("max_device_bytes", C.c_uint64), ("stream", C.c_void_p)]


class rd_pair_result(C.Structure):
    _fields_ = [("count", C.c_uint64), ("count_by_class", C.c_uint64 * 3),
                ("status", C.c_int32), ("verdict", C.c_uint8),
                ("classes", C.c_uint8), ("witness_class", C.c_uint8),
                ("flags", C.c_uint8), ("w_set", C.c_uint32),
                ("w_b1", C.c_uint32), ("w_t1", C.c_uint32),
                ("w_i1", C.c_uint32), ("w_b2", C.c_uint32),
                ("w_t2", C.c_uint32), ("w_i2", C.c_uint32),
                ("tiles", C.c_uint32),
                ("w_addr", C.c_int64), ("evals", C.c_uint64)]


class rd_stats(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("device_ms", C.c_double),
                ("join_ms", C.c_double), ("scatter_ms", C.c_double),
                ("witness_ms", C.c_double), ("evals", C.c_uint64),
                ("records", C.c_uint64), ("small_items", C.c_uint64),
                ("hbm_items", C.c_uint64), ("overflow_items", C.c_uint64),
                ("buckets", C.c_uint64), ("join_launches", C.c_uint64),
                ("join_kernel_ms", C.c_double), ("small_ms", C.c_double),
                ("bucket_ms", C.c_double), ("fallback_ms", C.c_double),
                ("retry_ms", C.c_double), ("retry_items", C.c_uint64),
                ("waves_ms", C.c_double), ("verdict_ms", C.c_double),
                ("verdict_units", C.c_uint64), ("split_ms", C.c_double),
                ("split_items", C.c_uint64), ("scatter_launches", C.c_uint64),
                ("scatter_bytes", C.c_uint64), ("fallback_records", C.c_uint64),
                ("scatter_tab_ms", C.c_double), ("scatter_tab_bytes", C.c_uint64),
                ("prefiltered", C.c_uint64), ("join_tab_launches", C.c_uint64),
                ("join_tab_ms", C.c_double), ("join_tab_bytes", C.c_uint64),
                ("presplit_items", C.c_uint64),
                ("filter_tab_launches", C.c_uint64), ("filter_tab_ms", C.c_double),
                ("filter_tab_bytes", C.c_uint64),
                ("units_apart", C.c_uint64),
                ("block_symmetric", C.c_uint64),
                ("fallback_groups", C.c_uint64),
                ("sync_records", C.c_uint64),
                ("sync_decided", C.c_uint64)]


assert C.sizeof(rd_pair_result) == 88

EXPORTS = ("rd_context_create", "rd_context_destroy", "rd_check_pairs",
           "rd_prepare", "rd_execute", "rd_plan_destroy", "rd_get_stats",
           "rd_strerror", "rd_selftest", "rd_tile_data", "rd_mlp_forward",
           "rd_mlp_grad", "rd_mlp_train", "rd_autotune", "rd_table_selftest",
           "rd_prefilter_selftest", "rd_expand_host_domain", "rd_mlp_save",
           "rd_mlp_load", "rd_derive_body")

_lib = None


def lib():
    """Loads libhgrd.so (built by ``paper_2604_02106_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhgrd.so is not built: run "
                               "python -m paper_2604_02106_amd.build")
        L = C.CDLL(LIB_PATH)
        L.rd_context_create.restype = C.c_int
        L.rd_context_create.argtypes = [C.POINTER(C.c_void_p), C.c_int]
        L.rd_context_destroy.restype = None
        L.rd_context_destroy.argtypes = [C.c_void_p]
        L.rd_check_pairs.restype = C.c_int
        L.rd_check_pairs.argtypes = [
            C.c_void_p, C.POINTER(rd_kernel_model), C.c_uint32,
            C.POINTER(rd_access_pair), C.c_uint32, C.POINTER(rd_launch_domain),
            C.POINTER(rd_param_sets), C.POINTER(rd_options),
            C.POINTER(rd_pair_result)]
        L.rd_check_pairs_noalloc.restype = C.c_int
        L.rd_check_pairs_noalloc.argtypes = L.rd_check_pairs.argtypes
        L.rd_prepare.restype = C.c_int
        L.rd_prepare.argtypes = [
            C.c_void_p, C.POINTER(rd_kernel_model), C.c_uint32,
            C.POINTER(rd_access_pair), C.c_uint32, C.POINTER(rd_launch_domain),
            C.POINTER(rd_param_sets), C.POINTER(rd_options),
            C.POINTER(C.c_void_p)]
        L.rd_autotune.restype = C.c_int
        L.rd_autotune.argtypes = [
            C.c_void_p, C.POINTER(rd_kernel_model), C.c_uint32,
            C.POINTER(rd_access_pair), C.c_uint32, C.POINTER(rd_launch_domain),
            C.POINTER(rd_param_sets), C.POINTER(rd_options), C.c_uint32,
            C.POINTER(rd_options), C.POINTER(C.c_double)]
        L.rd_execute.restype = C.c_int
        L.rd_execute.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(rd_pair_result)]
        L.rd_plan_destroy.restype = None
        L.rd_plan_destroy.argtypes = [C.c_void_p]
        L.rd_tile_data.restype = C.c_int
        L.rd_tile_data.argtypes = [
            C.c_void_p, C.POINTER(rd_kernel_model), C.c_uint32,
            C.POINTER(rd_access_pair), C.c_uint32, C.POINTER(rd_launch_domain),
            C.POINTER(rd_param_sets), C.POINTER(rd_options), C.c_uint64,
            C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]
        L.rd_mlp_forward.restype = C.c_int
        L.rd_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_uint64, C.c_void_p, C.c_void_p]
        L.rd_mlp_grad.restype = C.c_int
        L.rd_mlp_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.rd_mlp_train.restype = C.c_int
        L.rd_mlp_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_uint64, C.c_uint32, C.c_uint32, C.c_float,
                                   C.c_uint64, C.c_void_p, C.c_void_p]
        L.rd_prefilter_selftest.restype = C.c_int
        L.rd_prefilter_selftest.argtypes = [
            C.POINTER(rd_kernel_model), C.c_uint32, C.POINTER(rd_launch_domain),
            C.POINTER(rd_param_sets), C.c_uint32, C.c_uint32, C.c_uint32,
            C.c_uint32, C.POINTER(C.c_uint32)]
        L.rd_table_selftest.restype = C.c_int
        L.rd_table_selftest.argtypes = [
            C.POINTER(rd_kernel_model), C.c_uint32, C.POINTER(rd_launch_domain),
            C.POINTER(rd_param_sets), C.c_uint32, C.c_uint32, C.c_uint32,
            C.c_uint64, C.POINTER(C.c_uint64)]
        L.rd_derive_body.restype = C.c_int
        L.rd_derive_body.argtypes = [C.POINTER(rd_kernel_model), C.POINTER(rd_stmt),
                                     C.c_uint32, C.POINTER(rd_access),
                                     C.POINTER(rd_insn), C.c_uint32,
                                     C.POINTER(C.c_uint32)]
        L.rd_expand_host_domain.restype = C.c_int
        L.rd_expand_host_domain.argtypes = [C.POINTER(rd_host_domain),
                                            C.POINTER(rd_param_sets),
                                            C.POINTER(C.c_int64), C.c_uint64]
        L.rd_mlp_save.restype = C.c_int
        L.rd_mlp_save.argtypes = [C.c_void_p, C.c_uint32, C.c_char_p]
        L.rd_mlp_load.restype = C.c_int
        L.rd_mlp_load.argtypes = [C.c_void_p, C.POINTER(C.c_uint32), C.c_char_p]
        L.rd_selftest.restype = C.c_int
        L.rd_selftest.argtypes = []
        L.rd_get_stats.restype = C.c_int
        L.rd_get_stats.argtypes = [C.c_void_p, C.POINTER(rd_stats)]
        L.rd_strerror.restype = C.c_char_p
        L.rd_strerror.argtypes = [C.c_int]
        _lib = L
    return _lib


def rd_strerror(status):
    return lib().rd_strerror(int(status)).decode()


class Context:
    """An rd_context on one HIP device."""

    def __init__(self, device=0):
        self.h = C.c_void_p()
        st = lib().rd_context_create(C.byref(self.h), int(device))
        if st != RD_OK:
            raise RuntimeError("rd_context_create failed: %s" % rd_strerror(st))

    def close(self):
        if self.h:
            lib().rd_context_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        s = rd_stats()
        lib().rd_get_stats(self.h, C.byref(s))
        return {k: getattr(s, k) for k, _ in rd_stats._fields_}


class Packed:
    """C image of a workload's models, launch domains and parameter tuples.
    ``extra`` (optional): model index -> list of expressions put into that
    model's instruction pool after its own; their rd_expr in self.extra."""

    def __init__(self, workload, extra=None):
        n = len(workload.models)
        self.keep = []
        self.extra = {}
        self.models = (rd_kernel_model * max(1, n))()
        self.launch = (rd_launch_domain * max(1, n))()
        self.params = (rd_param_sets * max(1, n))()
        for mi, m in enumerate(workload.models):
            insns = []

            def put(e):
                if e is None:
                    return rd_expr(0, 0)
                first = len(insns)
                for t in e.code:
                    op = _OP.get(t[0], 0)
                    if t[0] == "const":
                        insns.append((op, 0, int(t[1])))
                    else:
                        insns.append((op, int(t[1]) if len(t) > 1 else 0, 0))
                return rd_expr(first, len(e.code))

            arrays = (rd_array * max(1, len(m.arrays)))(
                *[rd_array(_SPACE[a.space], a.addr_bits, getattr(a, "alias", 0), 0,
                           getattr(a, "base", 0)) for a in m.arrays])
            loops = (rd_loop * max(1, len(m.loops)))()
            for k, l in enumerate(m.loops):
                loops[k] = rd_loop(put(l.init), put(l.bound), put(l.step),
                                   _CMP[l.cmp], _UPD[l.upd])
            accs = (rd_access * max(1, len(m.accesses)))()
            for k, a in enumerate(m.accesses):
                x = accs[k]
                x.array, x.kind, x.scope = a.array, _KIND[a.kind], _SCOPE[a.scope]
                x.n_loops = len(a.loops)
                for i, lk in enumerate(a.loops[:4]):
                    x.loops[i] = lk
                x.addr, x.guard = put(a.addr), put(a.guard)
                x.bint, x.wint = put(a.bint), put(a.wint)
                for name in ("acq", "rel"):
                    sy = getattr(a, name, None)
                    if sy is not None:
                        setattr(x, name, rd_sync(put(sy.addr), sy.array,
                                                 _SCOPE[sy.scope]))
            if extra and mi in extra:
                self.extra[mi] = [put(e) for e in extra[mi]]
            ld = self.launch[mi]
            for d in range(3):
                ld.grid[d] = put(m.launch.grid[d])
                ld.block[d] = put(m.launch.block[d])
            ld.warp_size = m.launch.warp
            ins = (rd_insn * max(1, len(insns)))(
                *[rd_insn(o, a & 0xFFFF, 0, v) for (o, a, v) in insns])
            flat = [v for row in m.param_sets for v in row]
            vals = (C.c_int64 * max(1, len(flat)))(*flat)
            self.params[mi] = rd_param_sets(len(m.param_sets), 0, vals)
            md = self.models[mi]
            md.insns, md.n_insns = ins, len(insns)
            md.arrays, md.n_arrays = arrays, len(m.arrays)
            md.loops, md.n_loops = loops, len(m.loops)
            md.acc, md.n_acc = accs, len(m.accesses)
            md.n_params = m.n_params
            self.keep += [ins, arrays, loops, accs, vals]
        self.n_models = n

    @classmethod
    def concat(cls, packs):
        """One image of several images' models, in order: model k of
        packs[j] becomes model sum(len(packs[:j])) + k (the parts keep
        owning the arrays the models point to; the result keeps them)."""
        self = cls.__new__(cls)
        n = sum(p.n_models for p in packs)
        self.keep = list(packs)
        self.extra = {}
        self.models = (rd_kernel_model * max(1, n))()
        self.launch = (rd_launch_domain * max(1, n))()
        self.params = (rd_param_sets * max(1, n))()
        k = 0
        for p in packs:
            for i in range(p.n_models):
                self.models[k] = p.models[i]
                self.launch[k] = p.launch[i]
                self.params[k] = p.params[i]
                k += 1
        self.n_models = n
        return self


def _stream_handle(stream):
    if stream is not None:
        return int(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def _as_f32(a, n=None):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def _options(mode, order, lds_cap, max_device_bytes, log_level, stream,
             mlp=None, tile_budget=0, prefilter=0):
    o = rd_options(mode, order, prefilter, log_level, lds_cap, tile_budget, None,
                   max_device_bytes, _stream_handle(stream))
    keep = None
    if mlp is not None:
        keep = _as_f32(mlp, N_MLP)
        o.mlp = keep.ctypes.data
    return o, keep


def _pairs(workload):
    n = len(workload.pairs)
    return (rd_access_pair * max(1, n))(
        *[rd_access_pair(m, a, b, k) for (m, a, b, k) in workload.pairs])


class Plan:
    """rd_prepare'd batch: descriptors resident in device memory."""

    def __init__(self, ctx, workload, mode=MODE_EXACT, order=ORDER_LEX,
                 lds_cap=0, max_device_bytes=0, log_level=0, stream=None,
                 mlp=None, tile_budget=0, prefilter=0):
        self.ctx = ctx
        self.n = len(workload.pairs)
        pk = Packed(workload)
        self.packed = pk
        pairs = _pairs(workload)
        opt, keep = _options(mode, order, lds_cap, max_device_bytes, log_level,
                             stream, mlp, tile_budget, prefilter)
        self.h = C.c_void_p()
        st = lib().rd_prepare(ctx.h, pk.models, pk.n_models, pairs, self.n,
                              pk.launch, pk.params, C.byref(opt), C.byref(self.h))
        if st != RD_OK:
            raise RuntimeError("rd_prepare failed: %s" % rd_strerror(st))
        self.out = (rd_pair_result * max(1, self.n))()

    def execute(self, raw=False):
        st = lib().rd_execute(self.ctx.h, self.h, self.out)
        if st != RD_OK:
            raise RuntimeError("rd_execute failed: %s" % rd_strerror(st))
        if raw:
            return self.out
        return [result_dict(self.out[k]) for k in range(self.n)]

    def tiles(self):
        """Per pair: tiles examined before VERDICT mode stopped (0: not
        stopped by the tile search)."""
        return [self.out[k].tiles for k in range(self.n)]

    def close(self):
        if self.h:
            lib().rd_plan_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rd_check_pairs(ctx, workload, mode=MODE_EXACT, order=ORDER_LEX,
                   lds_cap=0, max_device_bytes=0, log_level=0, stream=None,
                   packed=None, mlp=None, tile_budget=0, prefilter=0):
    """Decides every pair of ``workload`` on the GPU.

    Returns a list of result dicts (same fields as rd_pair_result).
    """
    pk = packed or Packed(workload)
    n = len(workload.pairs)
    pairs = _pairs(workload)
    out = (rd_pair_result * max(1, n))()
    opt, keep = _options(mode, order, lds_cap, max_device_bytes, log_level,
                         stream, mlp, tile_budget, prefilter)
    st = lib().rd_check_pairs(ctx.h, pk.models, pk.n_models, pairs, n,
                              pk.launch, pk.params, C.byref(opt), out)
    if st != RD_OK:
        raise RuntimeError("rd_check_pairs failed: %s" % rd_strerror(st))
    return [result_dict(out[k]) for k in range(n)]


def rd_check_pairs_noalloc(ctx, workload, mode=MODE_EXACT, order=ORDER_LEX,
                           lds_cap=0, max_device_bytes=0, log_level=0, stream=None,
                           packed=None, mlp=None, tile_budget=0, prefilter=0):
    """rd_check_pairs inside the library's fixed scratch area (no device
    allocation).  Returns (status, results): status is RD_OK or the
    library's error (RD_ECAPACITY when the batch does not fit the area);
    results is None unless the status is RD_OK."""
    pk = packed or Packed(workload)
    n = len(workload.pairs)
    pairs = _pairs(workload)
    out = (rd_pair_result * max(1, n))()
    opt, keep = _options(mode, order, lds_cap, max_device_bytes, log_level,
                         stream, mlp, tile_budget, prefilter)
    st = lib().rd_check_pairs_noalloc(ctx.h, pk.models, pk.n_models, pairs, n,
                                      pk.launch, pk.params, C.byref(opt), out)
    if st != RD_OK:
        return st, None
    return st, [result_dict(out[k]) for k in range(n)]


def rd_autotune(ctx, workload, reps=3, mode=MODE_EXACT, order=ORDER_LEX,
                stream=None, mlp=None, tile_budget=0):
    """Times the batch for every tile shape and wave size and makes the
    fastest the context's default.  Returns (lds_cap, max_device_bytes,
    median ms)."""
    pk = Packed(workload)
    pairs = _pairs(workload)
    opt, keep = _options(mode, order, 0, 0, 0, stream, mlp, tile_budget)
    best = rd_options()
    ms = C.c_double()
    st = lib().rd_autotune(ctx.h, pk.models, pk.n_models, pairs, len(workload.pairs),
                           pk.launch, pk.params, C.byref(opt), reps,
                           C.byref(best), C.byref(ms))
    if st != RD_OK:
        raise RuntimeError("rd_autotune failed: %s" % rd_strerror(st))
    return best.lds_cap, best.max_device_bytes, ms.value


def prefilter_selftest(workload, model, access_a, access_b, tuple_index, packed=None):
    """rd_prefilter_selftest: (status, decided).  Host only."""
    pk = packed or Packed(workload)
    d = C.c_uint32()
    st = lib().rd_prefilter_selftest(pk.models, pk.n_models, pk.launch, pk.params,
                                     model, access_a, access_b, tuple_index, C.byref(d))
    return st, d.value


def table_selftest(workload, model, access, tuple_index, max_points=0, packed=None):
    """rd_table_selftest: (status, points compared).  Host only."""
    pk = packed or Packed(workload)
    n = C.c_uint64()
    st = lib().rd_table_selftest(pk.models, pk.n_models, pk.launch, pk.params,
                                 model, access, tuple_index, max_points, C.byref(n))
    return st, n.value


def result_dict(r):
    none = 0xFFFFFFFF
    w = (r.w_set, r.w_b1, r.w_t1, r.w_i1, r.w_b2, r.w_t2, r.w_i2)
    w = tuple(-1 if x == none else x for x in w)
    return {"status": r.status, "verdict": r.verdict, "count": r.count,
            "by_class": [r.count_by_class[0], r.count_by_class[1],
                         r.count_by_class[2]],
            "classes": r.classes, "witness_class": r.witness_class,
            "flags": r.flags, "witness": w, "w_addr": r.w_addr,
            "evals": r.evals}



_default_ctx = None


def check_pairs(workload, **kw):
    """rd_check_pairs on a process-wide context for device 0."""
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return rd_check_pairs(_default_ctx, workload, **kw)


def default_context():
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return _default_ctx


def rd_tile_data(ctx, workload, max_rows=None, stream=None):
    """Features (n x 32 float32), labels (n, 1/0/-1) and ids (n x 4: pair,
    tuple, b1, b2) of every tile of every eligible (pair, tuple)."""
    import numpy as np
    pk = Packed(workload)
    pairs = _pairs(workload)
    opt, _ = _options(MODE_VERDICT, ORDER_LEX, 0, 0, 0, stream)
    n = C.c_uint64(0)
    st = lib().rd_tile_data(ctx.h, pk.models, pk.n_models, pairs,
                            len(workload.pairs), pk.launch, pk.params,
                            C.byref(opt), 0, None, None, None, C.byref(n))
    if st not in (RD_OK, RD_ECAPACITY):
        raise RuntimeError("rd_tile_data failed: %s" % rd_strerror(st))
    rows = n.value
    if max_rows is not None and rows > max_rows:
        raise RuntimeError("%d tile rows exceed %d" % (rows, max_rows))
    X = np.zeros((rows, 32), dtype=np.float32)
    Y = np.zeros(rows, dtype=np.float32)
    ids = np.zeros((rows, 4), dtype=np.uint32)
    st = lib().rd_tile_data(ctx.h, pk.models, pk.n_models, pairs,
                            len(workload.pairs), pk.launch, pk.params,
                            C.byref(opt), rows, X.ctypes.data, Y.ctypes.data,
                            ids.ctypes.data, C.byref(n))
    if st != RD_OK:
        raise RuntimeError("rd_tile_data failed: %s" % rd_strerror(st))
    return X, Y, ids


def rd_mlp_forward(ctx, w, X, stream=None):
    import numpy as np
    w = _as_f32(w, N_MLP)
    X = _as_f32(X)
    n = X.shape[0]
    out = np.zeros(n, dtype=np.float32)
    st = lib().rd_mlp_forward(ctx.h, w.ctypes.data, X.ctypes.data, n,
                              out.ctypes.data, _stream_handle(stream))
    if st != RD_OK:
        raise RuntimeError("rd_mlp_forward failed: %s" % rd_strerror(st))
    return out


def rd_mlp_grad(ctx, w, X, Y, stream=None):
    import numpy as np
    w = _as_f32(w, N_MLP)
    X, Y = _as_f32(X), _as_f32(Y)
    g = np.zeros(N_MLP, dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    st = lib().rd_mlp_grad(ctx.h, w.ctypes.data, X.ctypes.data, Y.ctypes.data,
                           X.shape[0], g.ctypes.data, loss.ctypes.data,
                           _stream_handle(stream))
    if st != RD_OK:
        raise RuntimeError("rd_mlp_grad failed: %s" % rd_strerror(st))
    return g, float(loss[0])


def rd_mlp_train(ctx, w, X, Y, epochs=10, batch=4096, lr=1e-3, seed=0,
                 stream=None):
    """Returns (trained weights, per-epoch mean loss)."""
    import numpy as np
    w = _as_f32(w, N_MLP).copy()
    X, Y = _as_f32(X), _as_f32(Y)
    losses = np.zeros(epochs, dtype=np.float32)
    st = lib().rd_mlp_train(ctx.h, w.ctypes.data, X.ctypes.data, Y.ctypes.data,
                            X.shape[0], epochs, batch, lr, seed,
                            losses.ctypes.data, _stream_handle(stream))
    if st != RD_OK:
        raise RuntimeError("rd_mlp_train failed: %s" % rd_strerror(st))
    return w, losses


_HV_KIND = {"input": 0, "expr": 1, "loop": 2}


def expand_host_domain(domain, cap_values=1 << 20):
    """rd_expand_host_domain on a ``workloads.HostDomain``: the list of
    parameter tuples (lists of ints).  Host only.  Raises on a non-OK
    status (the status is in the message)."""
    insns = []

    def put(e):
        if e is None:
            return rd_expr(0, 0)
        first = len(insns)
        for t in e.code:
            op = _OP.get(t[0], 0)
            if t[0] == "const":
                insns.append((op, 0, int(t[1])))
            else:
                insns.append((op, int(t[1]) if len(t) > 1 else 0, 0))
        return rd_expr(first, len(e.code))

    keep = []
    hv = (rd_host_var * max(1, len(domain.vars)))()
    for k, v in enumerate(domain.vars):
        x = hv[k]
        x.kind = _HV_KIND[v.kind]
        x.cmp, x.upd = _CMP.get(v.cmp, 0), _UPD.get(v.upd, 0)
        vals = (C.c_int64 * max(1, len(v.values)))(*v.values)
        keep.append(vals)
        x.n_values, x.values = len(v.values), vals
        x.init, x.bound, x.step = put(v.init), put(v.bound), put(v.step)

    def exprs(lst):
        arr = (rd_expr * max(1, len(lst)))(*[put(e) for e in lst])
        keep.append(arr)
        return arr, len(lst)

    h = rd_host_domain()
    h.vars, h.n_vars = hv, len(domain.vars)
    h.asserts, h.n_asserts = exprs(domain.asserts)
    h.alloc_sizes, h.n_alloc = exprs(domain.alloc_sizes)
    h.params, h.n_params = exprs(domain.params)
    ins = (rd_insn * max(1, len(insns)))(
        *[rd_insn(o, a & 0xFFFF, 0, v) for (o, a, v) in insns])
    h.insns, h.n_insns = ins, len(insns)
    out = rd_param_sets()
    buf = (C.c_int64 * max(1, cap_values))()
    st = lib().rd_expand_host_domain(C.byref(h), C.byref(out), buf, cap_values)
    if st != RD_OK:
        raise RuntimeError("rd_expand_host_domain failed: %s (%d)" % (rd_strerror(st), st))
    n = len(domain.params)
    return [[buf[r * n + k] for k in range(n)] for r in range(out.n_sets)]


_ST = {"access": 1, "barrier": 2, "warp_barrier": 3, "if": 4, "else": 5, "end": 6,
       "loop": 7, "cas": 8, "exch": 9, "fence": 10}
_OP_NAME = {v: k for k, v in _OP.items()}
_KIND_NAME = {v: k for k, v in _KIND.items()}
_SCOPE_NAME = {v: k for k, v in _SCOPE.items()}


def derive_body(model, body, cap_insns=1 << 16):
    """rd_derive_body on a ``workloads.Model`` and a kernel body given as a
    list of statements: ("access", k), ("barrier",), ("warp_barrier",),
    ("if",), ("else",), ("end",), ("loop", k), ("cas", array, addr, scope),
    ("exch", array, addr, scope), ("fence", scope).  Returns the derived
    model (a new ``workloads.Model``).  Host only.  Raises on a non-OK
    status (the status is in the message)."""
    from workloads import E, Model, Access, Sync, Workload
    exprs = [st[2] for st in body if st[0] in ("cas", "exch")]
    pk = Packed(Workload([model], []), extra={0: exprs})
    stm = (rd_stmt * max(1, len(body)))()
    ex = iter(pk.extra.get(0, []))
    for k, st in enumerate(body):
        x = stm[k]
        x.kind = _ST[st[0]]
        if st[0] in ("access", "loop"):
            x.arg = int(st[1])
        elif st[0] in ("cas", "exch"):
            x.array, x.scope, x.addr = int(st[1]), _SCOPE[st[3]], next(ex)
        elif st[0] == "fence":
            x.scope = _SCOPE[st[1]]
    n_acc = len(model.accesses)
    acc = (rd_access * max(1, n_acc))()
    pool = (rd_insn * max(1, cap_insns))()
    n = C.c_uint32(0)
    st = lib().rd_derive_body(C.byref(pk.models[0]), stm, len(body), acc, pool,
                              cap_insns, C.byref(n))
    if st != RD_OK:
        raise RuntimeError("rd_derive_body failed: %s (%d)" % (rd_strerror(st), st))

    def expr_of(e):
        if e.count == 0:
            return None
        code = []
        for i in range(e.first, e.first + e.count):
            t = pool[i]
            name = _OP_NAME[t.op]
            if name == "const":
                code.append(("const", int(t.imm)))
            elif t.op < 16:
                code.append((name, int(t.arg)))
            else:
                code.append((name,))
        return E(code)

    accs = []
    for k, a in enumerate(model.accesses):
        x = acc[k]
        syn = []
        for y in (x.acq, x.rel):
            syn.append(None if y.addr.count == 0 else
                       Sync(y.array, expr_of(y.addr), _SCOPE_NAME[y.scope]))
        accs.append(Access(x.array, _KIND_NAME[x.kind], expr_of(x.addr), expr_of(x.guard),
                           [int(x.loops[i]) for i in range(x.n_loops)], expr_of(x.bint),
                           expr_of(x.wint), _SCOPE_NAME[x.scope], a.name, syn[0], syn[1]))
    return Model(model.n_params, model.arrays, accs, model.launch, model.param_sets,
                 loops=model.loops, name=model.name)


def mlp_save(w, path, feature_version):
    """rd_mlp_save: writes the network's weights (N_MLP float32) to path."""
    w = _as_f32(w, N_MLP)
    st = lib().rd_mlp_save(w.ctypes.data, int(feature_version), os.fsencode(path))
    if st != RD_OK:
        raise RuntimeError("rd_mlp_save failed: %s" % rd_strerror(st))


def mlp_load(path):
    """rd_mlp_load: (weights as float32 array, feature version)."""
    import numpy as np
    w = np.zeros(N_MLP, dtype=np.float32)
    fv = C.c_uint32()
    st = lib().rd_mlp_load(w.ctypes.data, C.byref(fv), os.fsencode(path))
    if st != RD_OK:
        raise RuntimeError("rd_mlp_load failed on %s: %s" % (path, rd_strerror(st)))
    return w, fv.value
