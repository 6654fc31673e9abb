"""Armadillo-flavoured lazy expressions on top of libcoot (expression capture).

Section 3 of the paper: functions and operators return expression objects, not
matrices; nothing is computed until the whole expression is assigned (delayed
evaluation).  Here operator overloads build a small tree; `eval` (assignment),
`+=`, and the closing reductions flatten it to the postfix list of the C ABI and
issue ONE fused library call.

Storage: a column-major n_rows x n_cols matrix lives in a torch tensor on the
HIP device whose memory holds the columns one after another (the tensor is kept
as the logical (n_rows, n_cols) view with strides (1, n_rows)).  PyTorch is used
for device memory and the current stream only; every element of every result is
computed by libcoot's kernels.
"""
from __future__ import annotations

import builtins

import numpy as np
import torch

from . import _coot as cc

_TORCH = {"f32": torch.float32, "f64": torch.float64, "u32": torch.int32, "s32": torch.int32,
          "f16": torch.float16, "bf16": torch.bfloat16}
# host arrays of each element type (bfloat16 values travel as float32 arrays)
_NP = {"f32": np.float32, "f64": np.float64, "u32": np.uint32, "s32": np.int32, "f16": np.float16,
       "bf16": np.float32}
_KIND = {"mat": cc.COOT_MAT, "col": cc.COOT_COL, "row": cc.COOT_ROW, "bcast": cc.COOT_BCAST}


class Expr:
    """A lazy expression node."""

    # element-wise binary (eGlue)
    def __add__(self, o):
        return _bin("add", self, o)

    def __radd__(self, o):
        return _bin("add", o, self)

    def __sub__(self, o):
        return _bin("sub", self, o)

    def __rsub__(self, o):
        return _bin("sub", o, self)

    def __mod__(self, o):                     # Schur product, as in Armadillo
        return _bin("schur", self, o)

    def __truediv__(self, o):
        return _bin("div", self, o)

    def __rtruediv__(self, o):
        return _bin("div", o, self)

    def __mul__(self, o):
        if isinstance(o, Expr):
            raise NotImplementedError("matrix product is outside the fused element-wise path; use % for Schur")
        return _bin("schur", self, o)

    def __rmul__(self, o):
        if isinstance(o, Expr):
            raise NotImplementedError("matrix product is outside the fused element-wise path")
        return _bin("schur", o, self)

    def __neg__(self):
        return Node("neg", [self])

    def t(self):
        return trans(self)


class Node(Expr):
    __slots__ = ("op", "kids")

    def __init__(self, op, kids):
        self.op = op
        self.kids = kids


class Scalar(Expr):
    __slots__ = ("value",)

    def __init__(self, value):
        self.value = float(value)


def _lift(x):
    if isinstance(x, Expr):
        return x
    if isinstance(x, (int, float, np.integer, np.floating)):
        return Scalar(x)
    raise TypeError(f"cannot use {type(x).__name__} in an expression")


def _bin(op, a, b):
    return Node(op, [_lift(a), _lift(b)])


class Mat(Expr):
    """Device matrix (Mat<eT>), column vector (Col<eT>) or row vector (Row<eT>)."""

    def __init__(self, tensor: torch.Tensor, dtype: str, kind: str = "mat"):
        if tensor.dim() != 2:
            raise ValueError("a Mat wraps the 2-D logical view of its storage")
        r, c = (int(v) for v in tensor.shape)
        s0, s1 = tensor.stride()
        # a stride along a dimension of extent 1 (or of an empty matrix) carries no meaning
        if r > 1 and c > 0 and s0 != 1:
            raise ValueError("storage must be column-major (row stride 1)")
        if kind == "bcast":
            if c > 1 and s1 != 0:
                raise ValueError("a broadcast operand repeats one column (column stride 0)")
        elif c > 1 and r > 0 and s1 < r:
            raise ValueError("storage must be column-major (column stride >= n_rows)")
        self.tensor = tensor
        self.dtype = dtype
        self.kind = kind
        self.n_rows, self.n_cols = r, c
        self.ld = 0 if kind == "bcast" else (int(s1) if (c > 1 and r > 0) else builtins.max(1, r))

    # ---- construction ---------------------------------------------------------------
    @staticmethod
    def empty(n_rows, n_cols, dtype="f32", kind="mat", device="cuda"):
        store = torch.empty((n_cols, n_rows), dtype=_TORCH[dtype], device=device)
        return Mat(store.t(), dtype, kind)

    @staticmethod
    def from_numpy(a: np.ndarray, dtype: str | None = None, kind: str | None = None, device="cuda"):
        a = np.asarray(a)
        if a.ndim == 1:
            a = a.reshape(-1, 1)
            kind = kind or "col"
        dtype = dtype or {np.dtype(np.float32): "f32", np.dtype(np.float64): "f64",
                          np.dtype(np.uint32): "u32", np.dtype(np.int32): "s32",
                          np.dtype(np.float16): "f16"}[a.dtype]
        a = a.astype(_NP[dtype], copy=False)
        if dtype == "u32":
            a = a.view(np.int32)
        cm = np.ascontiguousarray(a.T)                 # columns one after another
        store = torch.from_numpy(cm)
        if dtype == "bf16":
            store = store.to(torch.bfloat16)           # exact for values that are bfloat16 values
        store = store.to(device)
        return Mat(store.t(), dtype, kind or "mat")

    def numpy(self) -> np.ndarray:
        t = self.tensor.detach()
        if self.dtype == "bf16":
            t = t.float()                              # exact: every bfloat16 value is a binary32 value
        a = t.cpu().numpy()
        if self.dtype == "u32":
            a = a.view(np.uint32)
        return np.asarray(a)

    def operand(self) -> cc.coot_operand:
        return cc.coot_operand(self.tensor.data_ptr(), self.n_rows, self.n_cols, self.ld,
                               cc.DTYPE_CODE[self.dtype], _KIND[self.kind])

    def diag(self):
        """The main diagonal as a 1 x min(n_rows, n_cols) Row view whose elements lie ld + 1
        apart (trans() of it is the column Armadillo's diag() returns); it can be read in
        expressions and updated in place (d = Z.diag(); d += 100)."""
        n = builtins.min(self.n_rows, self.n_cols)
        view = torch.as_strided(self.tensor, (1, n), (1, self.ld + 1), self.tensor.storage_offset())
        return Mat(view, self.dtype, "row")

    # ---- submatrix views (Armadillo's submat / rows / cols / row / col) ----------------
    def submat(self, r0: int, c0: int, r1: int, c1: int):
        """Rows r0..r1 and columns c0..c1 (inclusive) as a view sharing this matrix's
        storage: same leading dimension, base address moved to element (r0, c0).  Views
        can be read in expressions and updated in place (s = X.submat(...); s += Y)."""
        if self.kind == "bcast":
            raise ValueError("a broadcast operand has no submatrix views")
        if not (0 <= r0 <= r1 < self.n_rows and 0 <= c0 <= c1 < self.n_cols):
            raise IndexError("submatrix bounds outside the matrix")
        view = self.tensor[r0:r1 + 1, c0:c1 + 1]
        kind = "row" if r0 == r1 and self.n_rows > 1 else ("col" if c0 == c1 and self.n_cols > 1 else self.kind)
        return Mat(view, self.dtype, kind)

    def rows(self, r0: int, r1: int):
        return self.submat(r0, 0, r1, self.n_cols - 1)

    def cols(self, c0: int, c1: int):
        return self.submat(0, c0, self.n_rows - 1, c1)

    def row(self, i: int):
        """Row i as a 1 x n_cols view whose elements lie ld apart."""
        return self.submat(i, 0, i, self.n_cols - 1)

    def col(self, j: int):
        return self.submat(0, j, self.n_rows - 1, j)

    def each_col(self):
        """Armadillo's each_col(): X.each_col() + v adds the column vector v to every column."""
        return _Each(self, bcast_col)

    def each_row(self):
        """Armadillo's each_row(): X.each_row() % w multiplies every row by the row vector w."""
        return _Each(self, bcast_row)

    def __iadd__(self, other):                       # B += 3*A : axpy, evaluated in place
        eval(self + other, out=self)
        return self

    def __isub__(self, other):
        eval(self - other, out=self)
        return self


# ---- broadcasting (each_col / each_row) ------------------------------------------------
def bcast_col(v: Mat, n_cols: int) -> Mat:
    """The n_rows x 1 column v repeated across n_cols columns: a broadcast operand (column
    stride 0), read in place of a materialised copy."""
    if v.n_cols != 1 or (v.n_rows > 1 and v.tensor.stride(0) != 1):
        raise ValueError("bcast_col needs a contiguous column vector")
    return Mat(v.tensor.expand(v.n_rows, n_cols), v.dtype, "bcast")


def bcast_row(w: Mat, n_rows: int) -> Expr:
    """The 1 x n_cols row w repeated down n_rows rows: trans() of the broadcast of w's
    elements taken as a column."""
    if w.n_rows != 1 or (w.n_cols > 1 and w.tensor.stride(1) != 1):
        raise ValueError("bcast_row needs a row vector with contiguous elements")
    return trans(bcast_col(Mat(w.tensor.t(), w.dtype, "col"), n_rows))


def _leaf_trans(e, flip=False):
    """The same expression with every trans() moved down onto the leaves (element-wise
    operators commute with transposition)."""
    if isinstance(e, Scalar):
        return e
    if isinstance(e, Mat):
        return trans(e) if flip else e
    if e.op == "trans":
        return _leaf_trans(_lift(e.kids[0]), not flip)
    return Node(e.op, [_leaf_trans(_lift(k), flip) for k in e.kids])


def _bcast_cols(e, n_cols: int):
    """An expression over column vectors, repeated across n_cols columns: broadcasting
    commutes with element-wise operators, so it is pushed down to the leaves (as trans()
    is), and every leaf becomes a broadcast operand."""
    def rec(x):
        if isinstance(x, Scalar):
            return x
        if isinstance(x, Mat):
            return bcast_col(x, n_cols)
        if x.op == "trans":           # a row vector read as a column
            k = x.kids[0]
            if isinstance(k, Mat) and k.n_rows == 1 and (k.n_cols <= 1 or k.tensor.stride(1) == 1):
                return bcast_col(Mat(k.tensor.t(), k.dtype, "col"), n_cols)
            raise ValueError("broadcasting needs column vectors (or rows with contiguous elements)")
        return Node(x.op, [rec(_lift(k)) for k in x.kids])
    return rec(_leaf_trans(_lift(e)))


def _bcast_rows(e, n_rows: int):
    """An expression over row vectors repeated down n_rows rows: the trans() of the
    column broadcast of its transpose."""
    if isinstance(e, Scalar):
        return e
    return trans(_bcast_cols(trans(e), n_rows))


class _Each:
    """X.each_col() / X.each_row(): binary operators with a vector (or an expression of
    vectors) broadcast over X."""

    def __init__(self, m: Mat, how):
        self.m, self.how = m, how

    def _b(self, v):
        v = _lift(v)
        if self.how is bcast_col:
            return _bcast_cols(v, self.m.n_cols)
        return _bcast_rows(v, self.m.n_rows)

    def __add__(self, v):
        return self.m + self._b(v)

    def __sub__(self, v):
        return self.m - self._b(v)

    def __mod__(self, v):
        return self.m % self._b(v)

    def __truediv__(self, v):
        return self.m / self._b(v)

    def __iadd__(self, v):
        eval(self.m + self._b(v), out=self.m)
        return self

    def __isub__(self, v):
        eval(self.m - self._b(v), out=self.m)
        return self


# ---- element-wise functions (eOp) and transpose (Op<op_trans>) -----------------------
def trans(x):
    return Node("trans", [_lift(x)])


def exp(x):
    return Node("exp", [_lift(x)])


def log(x):
    return Node("log", [_lift(x)])


def sqrt(x):
    return Node("sqrt", [_lift(x)])


def square(x):
    return Node("square", [_lift(x)])


def abs(x):  # noqa: A001 — the Armadillo name
    return Node("abs", [_lift(x)])


# ---- flattening -----------------------------------------------------------------------
class Flat:
    __slots__ = ("postfix", "mats", "scalars", "dtype")

    def __init__(self, postfix, mats, scalars, dtype):
        self.postfix = postfix
        self.mats = mats
        self.scalars = scalars
        self.dtype = dtype


def flatten(e: Expr) -> Flat:
    postfix, mats, scalars = [], [], []
    ids = {}
    stack = [(e, False)]
    while stack:
        node, done = stack.pop()
        if isinstance(node, Mat):
            k = ids.get(id(node))
            if k is None:
                k = ids[id(node)] = len(mats)
                mats.append(node)
            postfix.append(("load", k))
        elif isinstance(node, Scalar):
            postfix.append(("scalar", len(scalars)))
            scalars.append(node.value)
        elif done:
            postfix.append((node.op,))
        else:
            stack.append((node, True))
            for kid in reversed(node.kids):
                stack.append((kid, False))
    dts = {m.dtype for m in mats}
    if len(dts) > 1:
        raise cc.CootError(cc.COOT_ETYPE, "operands of one expression must share an element type")
    return Flat(postfix, mats, scalars, dts.pop() if dts else "f32")


_handles: dict = {}


def compiled(flat: Flat, flags: int = 0) -> int:
    """Library handle for the flattened expression (compiled once per signature and flags)."""
    slots = tuple((cc.DTYPE_CODE[m.dtype], _KIND[m.kind]) for m in flat.mats)
    key = (tuple(flat.postfix), slots, len(flat.scalars), flags)
    h = _handles.get(key)
    if h is None:
        h = cc.coot_expr_compile(flat.postfix, slots, len(flat.scalars), flags)
        _handles[key] = h
    return h


def _prepare_worker(job):
    """Spawned process: compile one expression's element-wise module into the on-disk
    code-object cache (no device use)."""
    postfix, slots, n_sc = job
    from paper_2508_11385_amd import _coot as c2
    h = c2.coot_expr_compile(postfix, list(slots), n_sc)
    c2.coot_expr_prepare(h, -1, rflags=c2.COOT_PF_COMPILE_ONLY)
    c2.coot_expr_release(h)
    return True


def precompile(exprs, workers: int = 12) -> list:
    """Compile the element-wise kernels of many expressions ahead of time; returns their
    flattened forms.  hipRTC compilations do not overlap across threads of one process, so
    they run in `workers` spawned processes (no device use in them) that fill the on-disk
    code-object cache (COOT_CACHE_DIR chooses it); this process then loads every module
    from there."""
    import multiprocessing as mp
    import os
    flats = [flatten(_lift(e)) for e in exprs]
    jobs = {}
    for f in flats:
        slots = tuple((cc.DTYPE_CODE[m.dtype], _KIND[m.kind]) for m in f.mats)
        jobs[(tuple(f.postfix), slots, len(f.scalars))] = None
    if workers > 1 and len(jobs) > 1 and not os.environ.get("COOT_NO_DISK_CACHE"):
        with mp.get_context("spawn").Pool(builtins.min(workers, len(jobs))) as pool:
            list(pool.imap_unordered(_prepare_worker, list(jobs), chunksize=4))
    for f in flats:
        cc.coot_expr_prepare(compiled(f), -1)
    return flats


def use_torch_allocator(enable: bool = True) -> None:
    """Take the library's workspaces and comparator temporaries from PyTorch's caching
    allocator (stream-ordered), or give them back to hipMalloc."""
    if not enable:
        cc.coot_set_allocator(None, None)
        return
    dev = torch.cuda.current_device()

    def alloc(n, stream):
        return int(torch.cuda.caching_allocator_alloc(int(n), device=dev, stream=int(stream)))

    def dealloc(p, stream):
        torch.cuda.caching_allocator_delete(int(p))

    cc.coot_set_allocator(alloc, dealloc)


if hasattr(torch._C, "_cuda_getCurrentRawStream"):
    def _stream() -> int:
        # the current stream's handle without building a Stream object (a microsecond per call)
        return torch._C._cuda_getCurrentRawStream(torch._C._cuda_getDevice())
else:
    def _stream() -> int:
        return torch.cuda.current_stream().cuda_stream


class _Bound:
    """What a call on one expression object needs, built once: the flattened form, the
    library handle, the ctypes operand and scalar arrays, the result's dimensions and,
    when the caller gives it, the output operand.  Expression trees are immutable (their
    Mats keep their storage), so a repeated call on the same object does no tree walk."""
    __slots__ = ("flat", "h", "ops", "sc", "shape", "out", "out_op", "cfg")

    def __init__(self, e, flags, cfg):
        self.flat = flatten(e)
        self.h = compiled(self.flat, flags)
        self.ops = cc._arr(cc.coot_operand, [m.operand() for m in self.flat.mats])
        self.sc = cc._arr(cc.C.c_double, self.flat.scalars)
        self.shape = None
        self.out = None
        self.out_op = None
        self.cfg = cc._cfg(cfg)


def _bound(e, flags, cfg, out, tag):
    """The cached call state of expression object e for (tag, flags, cfg, out)."""
    try:
        cache = e.__dict__.setdefault("_calls", {})
    except AttributeError:                      # e.g. a Scalar (no instance dict)
        cache = {}
    key = (tag, flags, None if cfg is None else tuple(cfg), id(out) if out is not None else None)
    b = cache.get(key)
    if b is None or (out is not None and b.out is not out):
        if len(cache) >= 8:                     # bounded: an entry holds its output alive
            cache.clear()
        b = _Bound(e, flags, cfg)
        if out is not None:
            b.out = out
            b.out_op = out.operand()
        cache[key] = b
    return b


def _fresh_out(b, r, c):
    kind = "col" if c == 1 and r != 1 else ("row" if r == 1 and c != 1 else "mat")
    return Mat.empty(r, c, b.flat.dtype, kind, device=b.flat.mats[0].tensor.device)


def eval(e: Expr, out: Mat | None = None, cfg=None, unfused: bool = False) -> Mat:  # noqa: A001
    """Assignment: evaluate the whole expression in one fused pass (or the unfused comparator)."""
    if isinstance(e, (int, float)):
        raise TypeError("nothing to evaluate")
    e = _lift(e)
    b = _bound(e, cc.COOT_CF_UNFUSED if unfused else 0, cfg, out, "eval")
    if out is None:
        if b.shape is None:
            b.shape = cc.coot_expr_out_shape(b.h, b.ops)
        res = _fresh_out(b, *b.shape)
        res_op = res.operand()
    else:
        res, res_op = b.out, b.out_op
    st = cc.lib.coot_expr_eval(b.h, b.ops, b.sc, cc.C.byref(res_op), b.cfg, _stream())
    if st != cc.COOT_OK:
        cc._check(st)
    return res


_RED_KIND = {"accu": cc.COOT_RED_ACCU, "dot": cc.COOT_RED_DOT, "min": cc.COOT_RED_MIN, "max": cc.COOT_RED_MAX,
             "mean": cc.COOT_RED_MEAN, "norm1": cc.COOT_RED_NORM1, "norm_inf": cc.COOT_RED_NORMINF}


class _Pair:
    """Cached call state of a statement pair (see eval_reduce)."""
    __slots__ = ("r", "out", "res", "he", "hr", "ops", "sc", "out_op", "src", "rsc", "res_op", "cfg")


def eval_reduce(e: Expr, out: Mat, r: Expr, kind: str = "accu", cfg=None, res: Mat | None = None) -> Mat:
    """Two statements in one pass: out = e, then the reduction `kind` of r, which may read
    e's operands and `out` (the value just computed): y = 2.5*x + y; d = accu(x % y) becomes
    eval_reduce(2.5 * x + y, y, x % y).  Returns the 1x1 result (written into res when
    given).  A repeated call on the same expression objects reuses their flattened forms."""
    e, r = _lift(e), _lift(r)
    cache = e.__dict__.setdefault("_calls", {})
    key = ("pair", id(r), kind, None if cfg is None else tuple(cfg), id(out), id(res) if res is not None else None)
    p = cache.get(key)
    if p is None or p.r is not r or p.out is not out or (res is not None and p.res is not res):
        fe, fr = flatten(e), flatten(r)

        def same(a: Mat, b: Mat):
            return (a.tensor.data_ptr() == b.tensor.data_ptr() and a.n_rows == b.n_rows and a.n_cols == b.n_cols
                    and a.ld == b.ld)

        src = []
        for m in fr.mats:
            if same(m, out):
                src.append(-1)
            else:
                k = next((i for i, a in enumerate(fe.mats) if same(m, a)), None)
                if k is None:
                    raise ValueError("the reduced statement may read only the operands of the first one and its "
                                     "result")
                src.append(k)
        if len(cache) >= 8:
            cache.clear()
        p = _Pair()
        p.r, p.out = r, out                     # (not e: e holds this cache; no reference cycle)
        p.he, p.hr = compiled(fe), compiled(fr)
        p.ops = cc._arr(cc.coot_operand, [m.operand() for m in fe.mats])
        p.sc = cc._arr(cc.C.c_double, fe.scalars)
        p.out_op = out.operand()
        p.src = cc._arr(cc.C.c_int32, src)
        p.rsc = cc._arr(cc.C.c_double, fr.scalars)
        p.res = res
        p.res_op = res.operand() if res is not None else None
        p.cfg = cc._cfg(cfg)
        cache[key] = p
    if res is None:
        dst = Mat.empty(1, 1, out.dtype, device=out.tensor.device)
        dst_op = dst.operand()
    else:
        dst, dst_op = p.res, p.res_op
    st = cc.lib.coot_expr_eval_reduce(p.he, p.ops, p.sc, cc.C.byref(p.out_op), p.hr, p.src, p.rsc, _RED_KIND[kind],
                                      cc.C.byref(dst_op), p.cfg, _stream())
    if st != cc.COOT_OK:
        cc._check(st)
    return dst


def _reduce(e, kind, dim, plain, out_shape, cfg, unfused, flags=0, out=None):
    e = _lift(e)
    b = _bound(e, cc.COOT_CF_UNFUSED if unfused else 0, cfg, out, "reduce")
    if out is None:
        if b.shape is None:
            b.shape = cc.coot_expr_out_shape(b.h, b.ops)
        orr, oc = out_shape(*b.shape)
        okind = "mat" if orr == oc == 1 else ("row" if orr == 1 else "col")
        res = Mat.empty(orr, oc, b.flat.dtype, okind, device=b.flat.mats[0].tensor.device)
        res_op = res.operand()
    else:
        res, res_op = b.out, b.out_op
    st = cc.lib.coot_reduce(b.h, b.ops, b.sc, kind, dim, (cc.COOT_RF_PLAIN if plain else 0) | flags,
                            cc.C.byref(res_op), b.cfg, _stream())
    if st != cc.COOT_OK:
        cc._check(st)
    return res


def _along(dim):
    if dim not in (0, 1):
        raise ValueError("dim must be 0 or 1")
    return (lambda r, c: (1, c)) if dim == 0 else (lambda r, c: (r, 1))


def accu(e, plain=False, cfg=None, unfused=False, out=None) -> Mat:
    """Sum of all elements, as a 1x1 device Mat (Fig. 1: sum(A) of a vector); out: a 1x1
    Mat to write instead of a new one (every reduction takes it)."""
    return _reduce(e, cc.COOT_RED_ACCU, -1, plain, lambda r, c: (1, 1), cfg, unfused, out=out)


def sum(e, dim=None, plain=False, cfg=None, unfused=False, out=None) -> Mat:  # noqa: A001
    """sum(X, 0): per column (1 x n_cols); sum(X, 1): per row (n_rows x 1).
    Without dim: a vector gives its total, a matrix sums per column (Armadillo's convention)."""
    if dim is None:
        flat = flatten(_lift(e))
        r, c = cc.coot_expr_out_shape(compiled(flat), [m.operand() for m in flat.mats])
        if r == 1 or c == 1:
            return accu(e, plain, cfg, unfused, out)
        dim = 0
    shape = (lambda r, c: (1, c)) if dim == 0 else (lambda r, c: (r, 1))
    return _reduce(e, cc.COOT_RED_SUM, dim, plain, shape, cfg, unfused, out=out)


def dot(a, b, plain=False, cfg=None, unfused=False, out=None) -> Mat:
    return _reduce(_bin("schur", a, b), cc.COOT_RED_DOT, -1, plain, lambda r, c: (1, 1), cfg, unfused, out=out)


def norm(e, plain=False, cfg=None, unfused=False, out=None) -> Mat:
    """2-norm of a vector / Frobenius norm of a matrix expression."""
    return _reduce(e, cc.COOT_RED_NORM, -1, plain, lambda r, c: (1, 1), cfg, unfused, out=out)


def min(e, cfg=None, unfused=False, out=None) -> Mat:  # noqa: A001 — the Armadillo name
    """Smallest element, as a 1x1 device Mat (NaN if any element is NaN)."""
    return _reduce(e, cc.COOT_RED_MIN, -1, False, lambda r, c: (1, 1), cfg, unfused, out=out)


def max(e, cfg=None, unfused=False, out=None) -> Mat:  # noqa: A001
    """Largest element, as a 1x1 device Mat (NaN if any element is NaN)."""
    return _reduce(e, cc.COOT_RED_MAX, -1, False, lambda r, c: (1, 1), cfg, unfused, out=out)


def mean(e, dim=None, plain=False, cfg=None, unfused=False, out=None) -> Mat:
    """Mean of all elements (compensated sum / count, rounded once), or with dim along a
    dimension as Armadillo's mean(X, dim): dim 0 per column (1 x n_cols), dim 1 per row
    (n_rows x 1)."""
    if dim is None:
        return _reduce(e, cc.COOT_RED_MEAN, -1, plain, lambda r, c: (1, 1), cfg, unfused, out=out)
    return _reduce(e, cc.COOT_RED_MEAN_DIM, dim, plain, _along(dim), cfg, unfused, out=out)


def var(e, norm_type=0, dim=None, plain=False, cfg=None, unfused=False, out=None) -> Mat:
    """Variance as Armadillo's var(X, norm_type, dim): normalised by N - 1 (norm_type 0)
    or N (norm_type 1); without dim over all elements, with dim 0 per column, dim 1 per
    row.  One pass over the expression: compensated moments about a value of the data,
    combined in binary64."""
    if norm_type not in (0, 1):
        raise ValueError("norm_type must be 0 or 1")
    flags = cc.COOT_RF_VAR_N if norm_type == 1 else 0
    if dim is None:
        return _reduce(e, cc.COOT_RED_VAR, -1, plain, lambda r, c: (1, 1), cfg, unfused, flags, out)
    return _reduce(e, cc.COOT_RED_VAR_DIM, dim, plain, _along(dim), cfg, unfused, flags, out)


def norm1(e, plain=False, cfg=None, unfused=False, out=None) -> Mat:
    """Sum of |x| over the elements (the 1-norm of the elements taken as a vector)."""
    return _reduce(e, cc.COOT_RED_NORM1, -1, plain, lambda r, c: (1, 1), cfg, unfused, out=out)


def norm_inf(e, cfg=None, unfused=False, out=None) -> Mat:
    """Largest |x| over the elements (the infinity norm of the elements as a vector)."""
    return _reduce(e, cc.COOT_RED_NORMINF, -1, False, lambda r, c: (1, 1), cfg, unfused, out=out)


def init(device: int = 0) -> None:
    cc.coot_init(device)


class Batch:
    """Many small independent expressions evaluated by one persistent, graph-captured launch.

    items: list of (expression, out Mat or None).  Outputs are allocated when None.
    The operands' and outputs' storage must stay alive while the batch exists.
    """

    def __init__(self, items, cfg=None):
        handles, ops, scs, outs = [], [], [], []
        self.outs = []
        self._keep = []
        for e, out in items:
            flat = flatten(_lift(e))
            h = compiled(flat)
            o = [m.operand() for m in flat.mats]
            if out is None:
                r, c = cc.coot_expr_out_shape(h, o)
                out = Mat.empty(r, c, flat.dtype, device=flat.mats[0].tensor.device)
            handles.append(h)
            ops.append(o)
            scs.append(flat.scalars)
            outs.append(out.operand())
            self.outs.append(out)
            self._keep.append(flat.mats)
        self.handle = cc.coot_batch_create(handles, ops, scs, outs, cfg, _stream())

    def launch(self):
        cc.coot_batch_launch(self.handle, _stream())

    def launch_each(self):
        cc.coot_batch_launch_each(self.handle, _stream())

    def tune(self):
        return cc.coot_batch_tune(self.handle, _stream())

    def info(self):
        return cc.coot_batch_info(self.handle)

    def __del__(self):
        try:
            cc.coot_batch_release(self.handle)
        except Exception:
            pass
