"""ctypes binding of libcoot's C ABI (include/coot.h): argument marshalling only.

Every function here has the name of the C entry point it wraps and raises
CootError (with the library's message) on a non-zero status.  The library is
loaded from this package directory; if it is missing, importing fails loudly —
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoot.so")

# enums (coot.h)
COOT_OK, COOT_EINVAL, COOT_ESHAPE, COOT_ETYPE, COOT_EALIAS, COOT_ECOMPILE, COOT_EHIP, COOT_ENOMEM, \
    COOT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8
COOT_U32, COOT_S32, COOT_F32, COOT_F64, COOT_F16, COOT_BF16 = 0, 1, 2, 3, 4, 5
COOT_MAT, COOT_COL, COOT_ROW, COOT_BCAST = 0, 1, 2, 3
OPCODES = {"load": 0, "scalar": 1, "add": 2, "sub": 3, "schur": 4, "div": 5, "neg": 6, "abs": 7,
           "exp": 8, "log": 9, "sqrt": 10, "square": 11, "trans": 12}
COOT_RED_ACCU, COOT_RED_SUM, COOT_RED_DOT, COOT_RED_NORM = 0, 1, 2, 3
COOT_RED_MIN, COOT_RED_MAX, COOT_RED_MEAN, COOT_RED_NORM1, COOT_RED_NORMINF = 4, 5, 6, 7, 8
COOT_RED_MEAN_DIM, COOT_RED_VAR, COOT_RED_VAR_DIM = 9, 10, 11
COOT_CF_UNFUSED = 0x1
COOT_RF_PLAIN = 0x1
COOT_RF_VAR_N = 0x2
COOT_PF_COMPILE_ONLY = 0x100
DTYPE_CODE = {"u32": COOT_U32, "s32": COOT_S32, "f32": COOT_F32, "f64": COOT_F64, "f16": COOT_F16,
              "bf16": COOT_BF16}
N_FEATURES = 23  # cost-model feature vector length
STATUS_NAME = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ETYPE", -4: "EALIAS", -5: "ECOMPILE", -6: "EHIP",
               -7: "ENOMEM", -8: "EUNSUPPORTED"}


class coot_op(C.Structure):
    _fields_ = [("code", C.c_int32), ("arg", C.c_uint32)]


class coot_slot_type(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("kind", C.c_int32)]


class coot_operand(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n_rows", C.c_int64), ("n_cols", C.c_int64), ("ld", C.c_int64),
                ("dtype", C.c_int32), ("kind", C.c_int32)]


class coot_launch_cfg(C.Structure):
    _fields_ = [("vec", C.c_uint16), ("ept", C.c_uint16), ("waves", C.c_uint16), ("grid_mult", C.c_uint16),
                ("tile_r", C.c_uint16), ("tile_c", C.c_uint16)]


def cfg_tuple(c: coot_launch_cfg) -> tuple:
    """(vec, ept, waves, grid_mult, tile_r, tile_c) of a launch configuration."""
    return (c.vec, c.ept, c.waves, c.grid_mult, c.tile_r, c.tile_c)


class CootError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAME.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libcoot.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    return C.CDLL(LIB_PATH)


lib = _load()

_P = C.c_void_p
_sig = {
    "coot_init": (C.c_int, [C.c_int]),
    "coot_set_allocator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "coot_expr_compile": (C.c_int, [C.POINTER(coot_op), C.c_uint32, C.POINTER(coot_slot_type), C.c_uint32,
                                    C.c_uint32, C.c_uint32, C.POINTER(_P)]),
    "coot_expr_prepare": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_uint32, C.POINTER(coot_launch_cfg)]),
    "coot_expr_out_shape": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "coot_expr_eval": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_double), C.POINTER(coot_operand),
                                 C.POINTER(coot_launch_cfg), _P]),
    "coot_reduce": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_double), C.c_int32, C.c_int32,
                              C.c_uint32, C.POINTER(coot_operand), C.POINTER(coot_launch_cfg), _P]),
    "coot_reduce_noalloc": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_double), C.c_int32, C.c_int32,
                                      C.c_uint32, C.POINTER(coot_operand), C.POINTER(coot_launch_cfg), _P]),
    "coot_flush_caches": (C.c_int, [_P]),
    "coot_expr_eval_reduce": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_double), C.POINTER(coot_operand),
                                        _P, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int32,
                                        C.POINTER(coot_operand), C.POINTER(coot_launch_cfg), _P]),
    "coot_expr_release": (None, [_P]),
    "coot_expr_kernel_name": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(coot_launch_cfg), C.c_char_p,
                                        C.c_size_t]),
    "coot_cache_info": (C.c_int, [C.POINTER(C.c_int64)]),
    "coot_cache_trim": (C.c_int, [C.POINTER(C.c_int64)]),
    "coot_stats": (None, [C.POINTER(C.c_double)]),
    "coot_last_error": (C.c_char_p, []),
    "coot_debug_codegen": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_uint32, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_int32, C.c_int32, C.c_char_p, C.c_size_t,
                                     C.POINTER(C.c_size_t)]),
    "coot_batch_create": (C.c_int, [C.c_uint32, C.POINTER(_P), C.POINTER(C.POINTER(coot_operand)),
                                    C.POINTER(C.POINTER(C.c_double)), C.POINTER(coot_operand),
                                    C.POINTER(coot_launch_cfg), _P, C.POINTER(_P)]),
    "coot_batch_launch": (C.c_int, [_P, _P]),
    "coot_batch_launch_each": (C.c_int, [_P, _P]),
    "coot_batch_tune": (C.c_int, [_P, _P, C.POINTER(coot_launch_cfg), C.POINTER(C.c_float)]),
    "coot_batch_info": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "coot_batch_release": (None, [_P]),
    "coot_tune_space": (C.c_uint32, [C.c_int32, C.POINTER(coot_launch_cfg), C.c_uint32]),
    "coot_tune_prepare": (C.c_int, [_P, C.POINTER(coot_operand), C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "coot_tune_runnable": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(coot_operand), C.c_int32, C.c_int32,
                                     C.POINTER(coot_launch_cfg), C.c_uint32, C.POINTER(C.c_int32)]),
    "coot_tune_table": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_double), C.POINTER(coot_operand),
                                  C.c_int32, C.c_int32, C.POINTER(coot_launch_cfg), C.c_uint32, C.c_uint32, C.c_int32,
                                  C.POINTER(C.c_float), _P]),
    "coot_tune_launch": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_double), C.POINTER(coot_operand),
                                   C.c_int32, C.c_int32, C.POINTER(coot_launch_cfg), _P]),
    "coot_mlp_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_float), C.POINTER(_P)]),
    "coot_mlp_num_params": (C.c_uint32, [_P]),
    "coot_mlp_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "coot_mlp_get_grads": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "coot_mlp_forward": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "coot_mlp_backward": (C.c_int, [_P, _P, _P, _P, C.c_int32, C.c_float, _P, _P]),
    "coot_mlp_adam_step": (C.c_int, [_P, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32, _P]),
    "coot_mlp_train": (C.c_int, [_P, _P, _P, _P, C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_int32,
                                 C.c_uint32, C.c_float, C.POINTER(C.c_float), _P]),
    "coot_mlp_release": (None, [_P]),
    "coot_costmodel_features": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int32, C.POINTER(coot_launch_cfg),
                                          C.c_uint32, C.POINTER(C.c_float)]),
    "coot_costmodel_train": (C.c_int, [C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int32,
                                       C.POINTER(C.c_float), C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_uint32, C.c_float, C.POINTER(C.c_float), _P, C.POINTER(_P)]),
    "coot_costmodel_predict": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int32, C.POINTER(coot_launch_cfg),
                                         C.c_uint32, C.POINTER(C.c_float), C.POINTER(C.c_uint32), _P]),
    "coot_costmodel_save": (C.c_int, [_P, C.c_char_p]),
    "coot_costmodel_load": (C.c_int, [C.c_char_p, C.POINTER(_P)]),
    "coot_costmodel_release": (None, [_P]),
    "coot_tune": (C.c_int, [_P, C.POINTER(coot_operand), C.POINTER(C.c_double), C.POINTER(coot_operand), C.c_int32,
                            C.c_int32, C.c_int32, _P, C.POINTER(coot_launch_cfg), C.POINTER(C.c_float), _P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def _check(status):
    if status != COOT_OK:
        raise CootError(status, lib.coot_last_error().decode(errors="replace"))


def _arr(ctype, items):
    items = list(items)
    a = (ctype * max(1, len(items)))()
    for i, it in enumerate(items):
        a[i] = it
    return a


def _cfg(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, coot_launch_cfg):
        return C.byref(cfg)
    return C.byref(coot_launch_cfg(*cfg))   # (vec, ept, waves, grid_mult[, tile_r, tile_c])


# ---- entry points -----------------------------------------------------------------

def coot_init(device: int = 0) -> None:
    _check(lib.coot_init(device))


def coot_expr_compile(postfix, slot_types, n_scalars: int, flags: int = 0) -> int:
    """postfix: [(name, arg?), ...]; slot_types: [(dtype_code, kind_code), ...]. Returns a handle."""
    ops = _arr(coot_op, [coot_op(OPCODES[it[0]], it[1] if len(it) > 1 else 0) for it in postfix])
    slots = _arr(coot_slot_type, [coot_slot_type(d, k) for d, k in slot_types])
    h = _P()
    _check(lib.coot_expr_compile(ops, len(postfix), slots, len(slot_types), n_scalars, flags, C.byref(h)))
    return h.value


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_allocator_refs = []  # keeps the installed callbacks alive


def coot_set_allocator(alloc=None, dealloc=None) -> None:
    """alloc(bytes, stream) -> int device pointer, dealloc(ptr, stream); None, None for hipMalloc."""
    if (alloc is None) != (dealloc is None):
        raise ValueError("give both functions or neither")
    if alloc is None:
        _check(lib.coot_set_allocator(None, None, None))
        _allocator_refs.clear()
        return
    fa = ALLOC_FN(lambda n, s, ctx: alloc(n, s or 0))
    fd = FREE_FN(lambda p, s, ctx: dealloc(p, s or 0))
    _check(lib.coot_set_allocator(C.cast(fa, C.c_void_p), C.cast(fd, C.c_void_p), None))
    _allocator_refs[:] = [fa, fd]


def coot_expr_prepare(h: int, mode: int = -1, dim: int = -1, rflags: int = 0, cfg=None) -> None:
    _check(lib.coot_expr_prepare(h, mode, dim, rflags, _cfg(cfg)))


def coot_expr_out_shape(h: int, operands) -> tuple:
    ops = _arr(coot_operand, operands)
    r, c = C.c_int64(), C.c_int64()
    _check(lib.coot_expr_out_shape(h, ops, C.byref(r), C.byref(c)))
    return r.value, c.value


def coot_expr_eval(h: int, operands, scalars, out: coot_operand, cfg=None, stream: int = 0) -> None:
    ops = _arr(coot_operand, operands)
    sc = _arr(C.c_double, scalars)
    _check(lib.coot_expr_eval(h, ops, sc, C.byref(out), _cfg(cfg), stream))


def coot_expr_eval_reduce(h: int, operands, scalars, out: coot_operand, r: int, r_src, r_scalars, kind: int,
                          r_out: coot_operand, cfg=None, stream: int = 0) -> None:
    _check(lib.coot_expr_eval_reduce(h, _arr(coot_operand, operands), _arr(C.c_double, scalars), C.byref(out), r,
                                     _arr(C.c_int32, r_src), _arr(C.c_double, r_scalars), kind, C.byref(r_out),
                                     _cfg(cfg), stream))


def coot_reduce(h: int, operands, scalars, kind: int, dim: int, flags: int, out: coot_operand, cfg=None,
                stream: int = 0) -> None:
    ops = _arr(coot_operand, operands)
    sc = _arr(C.c_double, scalars)
    _check(lib.coot_reduce(h, ops, sc, kind, dim, flags, C.byref(out), _cfg(cfg), stream))


def coot_reduce_noalloc(h: int, operands, scalars, kind: int, dim: int, flags: int, out: coot_operand, cfg=None,
                        stream: int = 0) -> None:
    ops = _arr(coot_operand, operands)
    sc = _arr(C.c_double, scalars)
    _check(lib.coot_reduce_noalloc(h, ops, sc, kind, dim, flags, C.byref(out), _cfg(cfg), stream))


def coot_flush_caches(stream: int = 0) -> None:
    _check(lib.coot_flush_caches(stream))


def coot_expr_release(h: int) -> None:
    lib.coot_expr_release(h)


def coot_expr_kernel_name(h: int, mode: int = -1, dim: int = -1, cfg=None) -> str:
    buf = C.create_string_buffer(256)
    _check(lib.coot_expr_kernel_name(h, mode, dim, _cfg(cfg), buf, 256))
    return buf.value.decode()


def coot_cache_info() -> dict:
    a = (C.c_int64 * 4)()
    _check(lib.coot_cache_info(a))
    return {"modules": a[0], "cap": a[1], "evictions": a[2], "awaiting_unload": a[3]}


def coot_cache_trim() -> int:
    n = C.c_int64()
    _check(lib.coot_cache_trim(C.byref(n)))
    return n.value


def coot_stats() -> dict:
    a = (C.c_double * 5)()
    lib.coot_stats(a)
    return {"compiles": a[0], "mem_hits": a[1], "disk_hits": a[2], "launches": a[3], "compile_ms": a[4]}


def coot_last_error() -> str:
    return lib.coot_last_error().decode(errors="replace")


def coot_debug_codegen(h: int, mode: int, dim: int, rflags: int, fam: int, vec: int, ept: int, tile,
                       compile: bool):
    buf = C.create_string_buffer(1 << 18)
    n = C.c_size_t()
    tr, tc = (tile, tile) if isinstance(tile, int) else tile     # an edge, or (tile_r, tile_c)
    _check(lib.coot_debug_codegen(h, mode, dim, rflags, fam, vec, ept, tr, tc, int(compile), buf, 1 << 18,
                                  C.byref(n)))
    return buf.value.decode(), n.value


# ---- batches ---------------------------------------------------------------------------

def coot_batch_create(handles, operand_lists, scalar_lists, outs, cfg=None, stream: int = 0) -> int:
    n = len(handles)
    hs = (_P * max(1, n))(*handles)
    op_arrays = [_arr(coot_operand, ops) for ops in operand_lists]
    sc_arrays = [_arr(C.c_double, sc) for sc in scalar_lists]
    opp = (C.POINTER(coot_operand) * max(1, n))(*[C.cast(a, C.POINTER(coot_operand)) for a in op_arrays])
    scp = (C.POINTER(C.c_double) * max(1, n))(*[C.cast(a, C.POINTER(C.c_double)) for a in sc_arrays])
    outa = _arr(coot_operand, outs)
    b = _P()
    _check(lib.coot_batch_create(n, hs, opp, scp, outa, _cfg(cfg), stream, C.byref(b)))
    return b.value


def coot_batch_launch(b: int, stream: int = 0) -> None:
    _check(lib.coot_batch_launch(b, stream))


def coot_batch_launch_each(b: int, stream: int = 0) -> None:
    _check(lib.coot_batch_launch_each(b, stream))


def coot_batch_tune(b: int, stream: int = 0):
    best = coot_launch_cfg()
    us = C.c_float()
    _check(lib.coot_batch_tune(b, stream, C.byref(best), C.byref(us)))
    return (best.vec, best.ept, best.waves, best.grid_mult), us.value


def coot_batch_info(b: int) -> dict:
    a = (C.c_int64 * 15)()
    _check(lib.coot_batch_info(b, a))
    return {"n_exprs": a[0], "n_tiles": a[1], "bytes": a[2], "tile": a[3], "grid": a[4], "vec4_exprs": a[5],
            "flat_exprs": a[6], "lds_stack": a[7], "lds_staged": a[8], "tile_2d": a[9], "grid_2d": a[10],
            "flat_tiles": a[11], "concurrent": a[12], "g": a[13], "g_2d": a[14]}


def coot_batch_release(b: int) -> None:
    lib.coot_batch_release(b)


# ---- autotuning ---------------------------------------------------------------------------

def coot_tune_space(family: int) -> list:
    n = lib.coot_tune_space(family, None, 0)
    a = (coot_launch_cfg * n)()
    lib.coot_tune_space(family, a, n)
    return [cfg_tuple(c) for c in a]


def _cfgs(cfgs):
    return _arr(coot_launch_cfg, [coot_launch_cfg(*c) for c in cfgs])


def coot_tune_prepare(h: int, operands, mode: int = -1, dim: int = -1) -> int:
    fam = C.c_int32()
    _check(lib.coot_tune_prepare(h, _arr(coot_operand, operands), mode, dim, C.byref(fam)))
    return fam.value


def coot_tune_runnable(h: int, operands, out, mode: int, cfgs, dim: int = -1) -> list:
    ok = (C.c_int32 * max(1, len(cfgs)))()
    _check(lib.coot_tune_runnable(h, _arr(coot_operand, operands), C.byref(out) if out is not None else None, mode,
                                  dim, _cfgs(cfgs), len(cfgs), ok))
    return [bool(ok[i]) for i in range(len(cfgs))]


def coot_tune_table(h: int, operands, scalars, out: coot_operand, mode: int, cfgs, reps: int = 5, flush: bool = True,
                    stream: int = 0, dim: int = -1) -> list:
    t = (C.c_float * max(1, len(cfgs)))()
    _check(lib.coot_tune_table(h, _arr(coot_operand, operands), _arr(C.c_double, scalars), C.byref(out), mode, dim,
                               _cfgs(cfgs), len(cfgs), reps, int(flush), t, stream))
    return [t[i] for i in range(len(cfgs))]


def coot_tune_launch(h: int, operands, scalars, out: coot_operand, mode: int, cfg, stream: int = 0,
                     dim: int = -1) -> None:
    _check(lib.coot_tune_launch(h, _arr(coot_operand, operands), _arr(C.c_double, scalars), C.byref(out), mode, dim,
                                C.byref(coot_launch_cfg(*cfg)), stream))


def coot_tune(h: int, operands, scalars, out: coot_operand, mode: int, policy: int, cm: int = 0, stream: int = 0,
              dim: int = -1):
    best = coot_launch_cfg()
    us = C.c_float()
    _check(lib.coot_tune(h, _arr(coot_operand, operands), _arr(C.c_double, scalars), C.byref(out), mode, dim,
                         policy, cm or None, C.byref(best), C.byref(us), stream))
    return cfg_tuple(best), us.value


# ---- MLP and cost model -------------------------------------------------------------------

def _fptr(a):
    """numpy float32 array -> ctypes float pointer (the array must stay alive)."""
    import numpy as np
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_float))


def coot_mlp_create(n_in: int, h1: int, h2: int, params) -> int:
    m = _P()
    _check(lib.coot_mlp_create(n_in, h1, h2, _fptr(params), C.byref(m)))
    return m.value


def coot_mlp_num_params(m: int) -> int:
    return lib.coot_mlp_num_params(m)


def coot_mlp_get_params(m: int):
    import numpy as np
    out = np.empty(coot_mlp_num_params(m), np.float32)
    _check(lib.coot_mlp_get_params(m, _fptr(out)))
    return out


def coot_mlp_get_grads(m: int):
    import numpy as np
    out = np.empty(coot_mlp_num_params(m), np.float32)
    _check(lib.coot_mlp_get_grads(m, _fptr(out)))
    return out


def coot_mlp_forward(m: int, X_dev: int, B: int, out_dev: int, stream: int = 0) -> None:
    _check(lib.coot_mlp_forward(m, X_dev, B, out_dev, stream))


def coot_mlp_backward(m: int, X_dev: int, y_dev: int, mask_dev: int, B: int, inv_count: float, loss_dev: int = 0,
                      stream: int = 0) -> None:
    _check(lib.coot_mlp_backward(m, X_dev, y_dev, mask_dev, B, inv_count, loss_dev or None, stream))


def coot_mlp_adam_step(m: int, lr: float, beta1: float, beta2: float, eps: float, t: int, stream: int = 0) -> None:
    _check(lib.coot_mlp_adam_step(m, lr, beta1, beta2, eps, t, stream))


def coot_mlp_train(m: int, X_dev: int, y_dev: int, mask_dev: int, mask_host, N: int, batch: int, epochs: int,
                   seed: int, lr: float, stream: int = 0):
    import numpy as np
    losses = np.zeros(max(1, epochs), np.float32)
    _check(lib.coot_mlp_train(m, X_dev, y_dev, mask_dev, _fptr(mask_host), N, batch, epochs, seed, lr,
                              _fptr(losses), stream))
    return losses[:epochs]


def coot_mlp_release(m: int) -> None:
    lib.coot_mlp_release(m)


def coot_costmodel_features(h: int, n_rows: int, n_cols: int, red: int, cfgs):
    import numpy as np
    out = np.zeros((len(cfgs), N_FEATURES), np.float32)
    _check(lib.coot_costmodel_features(h, n_rows, n_cols, red, _cfgs(cfgs), len(cfgs), _fptr(out)))
    return out


def coot_costmodel_train(feats, target, mask, init_params, h1: int, h2: int, epochs: int, batch: int, seed: int,
                         lr: float, stream: int = 0, n_models: int = 1):
    """init_params: n_models parameter vectors, concatenated (or a (n_models, P) array)."""
    import numpy as np
    feats = np.ascontiguousarray(feats, np.float32)
    target = np.ascontiguousarray(target, np.float32)
    mask = np.ascontiguousarray(mask, np.float32)
    init_params = np.ascontiguousarray(np.ravel(init_params), np.float32)
    n_par = h1 * N_FEATURES + h1 + h2 * h1 + h2 + h2 + 1
    if init_params.size != n_models * n_par:
        raise ValueError(f"init_params must hold {n_models} x {n_par} values")
    losses = np.zeros(max(1, epochs), np.float32)
    cm = _P()
    _check(lib.coot_costmodel_train(_fptr(feats), _fptr(target), _fptr(mask), len(target), _fptr(init_params),
                                    n_models, h1, h2, epochs, batch, seed, lr, _fptr(losses), stream, C.byref(cm)))
    return cm.value, losses[:epochs]


def coot_costmodel_predict(cm: int, h: int, n_rows: int, n_cols: int, red: int, cfgs, stream: int = 0):
    import numpy as np
    pred = np.zeros(len(cfgs), np.float32)
    best = C.c_uint32()
    _check(lib.coot_costmodel_predict(cm, h, n_rows, n_cols, red, _cfgs(cfgs), len(cfgs), _fptr(pred),
                                      C.byref(best), stream))
    return int(best.value), pred


def coot_costmodel_save(cm: int, path: str) -> None:
    _check(lib.coot_costmodel_save(cm, path.encode()))


def coot_costmodel_load(path: str) -> int:
    cm = _P()
    _check(lib.coot_costmodel_load(path.encode(), C.byref(cm)))
    return cm.value


def coot_costmodel_release(cm: int) -> None:
    lib.coot_costmodel_release(cm)
