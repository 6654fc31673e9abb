"""Seeded synthetic inputs for the fused-expression path.

This module is shared by the CPU oracle, the tests and the benchmark.  It draws
random numbers and builds workload descriptions (operand arrays, postfix
expression lists, random expression trees); it performs none of the method's
arithmetic.  Every array it returns is a *logical* matrix of shape
(n_rows, n_cols); storing it column-major on the device is the caller's job.

Postfix vocabulary (the wire format both sides read):
    ("load", k)    push operand slot k
    ("scalar", k)  push scalar slot k (broadcast)
    ("add",) ("sub",) ("schur",) ("div",)          binary, element-wise
    ("neg",) ("abs",) ("exp",) ("log",) ("sqrt",) ("square",)   unary
    ("trans",)     transpose of the value on top of the stack

The workloads follow the paper's evaluation protocol (synthetic uniform data,
Section 5) and the expression types of Section 3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = (2508, 11385)

DTYPES = ("u32", "s32", "f32", "f64", "f16", "bf16")
# numpy container of each element type (bfloat16 values are held in float32 arrays)
NP_DTYPE = {"u32": np.uint32, "s32": np.int32, "f32": np.float32, "f64": np.float64, "f16": np.float16,
            "bf16": np.float32}


def _to_dtype(x: np.ndarray, dtype: str) -> np.ndarray:
    """binary64 draws as the element type: a numpy cast, and for bf16 the binary32 cast
    with its low 16 bits cleared (a bfloat16 value, truncated toward zero)."""
    if dtype != "bf16":
        return x.astype(NP_DTYPE[dtype])
    b = x.astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    return b.view(np.float32)

BINARY = ("add", "sub", "schur", "div")
UNARY = ("neg", "abs", "exp", "log", "sqrt", "square")
INT_LEGAL = ("load", "scalar", "add", "sub", "schur", "neg", "abs", "square", "trans")


def rng_for(*key: int) -> np.random.Generator:
    """Generator seeded from SeedSequence([2508, 11385, *key])."""
    return np.random.default_rng(np.random.SeedSequence(list(SEED_ROOT) + [int(k) for k in key]))


def uniform(rng: np.random.Generator, shape, dtype: str, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform[lo, hi) drawn in binary64, then converted to dtype (float types only)."""
    x = rng.uniform(lo, hi, size=shape)
    return _to_dtype(x, dtype)


def uniform_int(rng: np.random.Generator, shape, dtype: str, lo: int, hi: int) -> np.ndarray:
    """Integers uniform in [lo, hi) as dtype."""
    x = rng.integers(lo, hi, size=shape, dtype=np.int64)
    if dtype == "u32":
        return (x & 0xFFFFFFFF).astype(np.uint32)
    return x.astype(np.int64).astype(np.int32)


def lognormal_signed(rng: np.random.Generator, n: int, sigma: float = 4.0, dtype: str = "f32",
                     chunk: int = 1 << 24) -> np.ndarray:
    """exp(N(0, sigma)) with a random sign of probability 1/2, drawn in binary64, rounded to dtype."""
    out = np.empty(n, dtype=NP_DTYPE[dtype])
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        mag = rng.lognormal(0.0, sigma, size=m)
        sign = rng.integers(0, 2, size=m, dtype=np.int8)
        mag[sign == 1] *= -1.0
        out[s:s + m] = _to_dtype(mag, dtype)
    return out


# ---------------------------------------------------------------------------
# The four fixed workloads
# ---------------------------------------------------------------------------

def axpy_inputs(n: int = 1_000_000, dtype: str = "f32"):
    """Column vectors x, y ~ U[-1,1] for y <- 2.5*x + y followed by accu(x % y)."""
    g = rng_for(0)
    x = uniform(g, (n, 1), dtype)
    y = uniform(g, (n, 1), dtype)
    return x, y


def matrix_inputs(n: int = 4096, dtype: str = "f32", n_rows: int | None = None, n_cols: int | None = None):
    """A, B, C (n_rows x n_cols) and D (n_cols x n_rows) ~ U[-1,1] for the 2-D expressions.

    D is the operand read through trans(), so its stored shape is the transpose.
    """
    r = n if n_rows is None else n_rows
    c = n if n_cols is None else n_cols
    g = rng_for(1, 0 if dtype == "f32" else 1)
    A = uniform(g, (r, c), dtype)
    B = uniform(g, (r, c), dtype)
    C = uniform(g, (r, c), dtype)
    D = uniform(g, (c, r), dtype)
    return A, B, C, D


def int_inputs(n: int = 8192, which: str = "u32", n_rows: int | None = None, n_cols: int | None = None):
    """Integer matrices: u32 A, B, C uniform in [0, 2^16); s32 A, B either over all of int32
    ('s32_full') or over [0, 2^16) ('s32_small')."""
    r = n if n_rows is None else n_rows
    c = n if n_cols is None else n_cols
    if which == "u32":
        g = rng_for(2, 0)
        return tuple(uniform_int(g, (r, c), "u32", 0, 1 << 16) for _ in range(3))
    if which == "s32_full":
        g = rng_for(2, 1)
        return tuple(uniform_int(g, (r, c), "s32", -(1 << 31), 1 << 31) for _ in range(2))
    if which == "s32_small":
        g = rng_for(2, 2)
        return tuple(uniform_int(g, (r, c), "s32", 0, 1 << 16) for _ in range(2))
    raise ValueError(which)


def hard_reduction_inputs(n: int = 1 << 28, dtype: str = "f32"):
    """lognormal(0,4) magnitudes with random signs, as a column vector of n values."""
    g = rng_for(2, 3)
    return lognormal_signed(g, n, 4.0, dtype).reshape(n, 1)


# ---------------------------------------------------------------------------
# Random expression trees (batched workload and tuner training set)
# ---------------------------------------------------------------------------

@dataclass
class TreeSpec:
    """A random expression: postfix list, operand shapes, scalar values, dtype, output shape."""
    postfix: list
    slot_shapes: list
    scalars: list
    dtype: str
    out_shape: tuple
    depth: int
    meta: dict = field(default_factory=dict)


class _Node:
    __slots__ = ("op", "kids", "orient", "slot", "scalar")

    def __init__(self, op, kids=(), orient=0):
        self.op = op
        self.kids = list(kids)
        self.orient = orient
        self.slot = None
        self.scalar = None


def _gen(rng, depth, orient, is_int, force):
    """Subtree whose longest root-to-leaf path has exactly `depth` op levels when `force`
    is set, and at most `depth` otherwise."""
    if depth == 0:
        return _Node("leaf", orient=orient)
    if not force and rng.random() < 0.3:
        return _gen(rng, int(rng.integers(0, depth)), orient, is_int, False)
    u = rng.random()
    if u < 0.6:
        ops = ("add", "sub", "schur") if is_int else BINARY
        op = ops[int(rng.integers(0, len(ops)))]
        if op == "div" and depth < 3:
            op = "schur"
        first = int(rng.integers(0, 2))
        budget = [depth - 1, depth - 3 if op == "div" else depth - 1]
        kids = [_gen(rng, budget[s], orient, is_int, force and s == first) for s in range(2)]
        if op == "div":
            # a / (1 + abs(b)) keeps every value finite
            one = _Node("scalar_const", orient=orient)
            one.scalar = 1.0
            kids[1] = _Node("add", [one, _Node("abs", [kids[1]], orient)], orient)
        return _Node(op, kids, orient)
    if u < 0.9:
        if is_int:
            choice = ("neg", "abs", "square", "sscale", "sshift")
        else:
            choice = ("neg", "abs", "expneg", "sqrtabs", "sscale", "sshift")
        kind = choice[int(rng.integers(0, len(choice)))]
        if (kind == "expneg" and depth < 3) or (kind == "sqrtabs" and depth < 2):
            kind = "abs"
        cost = {"expneg": 3, "sqrtabs": 2}.get(kind, 1)
        kid = _gen(rng, depth - cost, orient, is_int, force)
        if kind in ("neg", "abs", "square"):
            return _Node(kind, [kid], orient)
        if kind == "expneg":
            return _Node("exp", [_Node("neg", [_Node("abs", [kid], orient)], orient)], orient)
        if kind == "sqrtabs":
            return _Node("sqrt", [_Node("abs", [kid], orient)], orient)
        s = _Node("scalar_rand", orient=orient)
        return _Node("schur" if kind == "sscale" else "add", [s, kid], orient)
    kid = _gen(rng, depth - 1, 1 - orient, is_int, force)
    return _Node("trans", [kid], orient)


def _depth(node):
    if node.op in ("leaf", "scalar_const", "scalar_rand"):
        return 0
    return 1 + max(_depth(k) for k in node.kids)


def random_tree(rng: np.random.Generator, depth: int, n_operands: int, n_rows: int, n_cols: int,
                dtype: str = "f32") -> TreeSpec:
    """Random element-wise expression tree with `depth` op levels on its longest path.

    Leaves reference operand slots; a slot keeps one orientation, so a slot read under an
    odd number of trans() is stored transposed.  Every slot is used at least once.
    Divisions are emitted as a / (1 + abs(b)) and exp as exp(-abs(a)).
    """
    is_int = dtype in ("u32", "s32")
    square = n_rows == n_cols
    root = _gen(rng, depth, 0, is_int, True)
    leaves = []

    def walk(nd):
        if nd.op == "leaf":
            leaves.append(nd)
        for k in nd.kids:
            walk(k)

    walk(root)
    k = max(1, min(n_operands, len(leaves)))
    order = list(rng.permutation(len(leaves)))
    # first uses: make sure each orientation that occurs gets a slot of its own
    slot_orient = []
    first = []
    if not square:
        for o in (0, 1):
            for idx in order:
                if leaves[idx].orient == o:
                    first.append(idx)
                    break
    for idx in order:
        if len(first) >= k:
            break
        if idx not in first:
            first.append(idx)
    for s, idx in enumerate(first):
        leaves[idx].slot = s
        slot_orient.append(leaves[idx].orient)
    for idx in order:
        lf = leaves[idx]
        if lf.slot is not None:
            continue
        cands = [s for s, o in enumerate(slot_orient) if square or o == lf.orient]
        lf.slot = cands[int(rng.integers(0, len(cands)))]
    slot_shapes = [(n_rows, n_cols) if (o == 0 or square) else (n_cols, n_rows) for o in slot_orient]

    postfix = []
    scalars = []

    def emit(nd):
        if nd.op == "leaf":
            postfix.append(("load", nd.slot))
            return
        if nd.op == "scalar_const":
            postfix.append(("scalar", len(scalars)))
            scalars.append(float(nd.scalar))
            return
        if nd.op == "scalar_rand":
            postfix.append(("scalar", len(scalars)))
            if is_int:
                scalars.append(float(int(rng.integers(1, 6))))
            else:
                scalars.append(float(np.round(rng.uniform(0.5, 2.0), 2)))
            return
        for kd in nd.kids:
            emit(kd)
        postfix.append((nd.op,))

    emit(root)
    return TreeSpec(postfix=postfix, slot_shapes=slot_shapes, scalars=scalars, dtype=dtype,
                    out_shape=(n_rows, n_cols), depth=_depth(root),
                    meta={"n_operands": len(slot_orient)})


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    """round(exp(U[ln lo, ln hi]))."""
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_workload(n_exprs: int = 10_000, seed: int = 3, dtype: str = "f32",
                   dim_lo: int = 8, dim_hi: int = 512, depth_lo: int = 1, depth_hi: int = 6,
                   ops_lo: int = 2, ops_hi: int = 5):
    """Independent random expressions with rows, cols log-uniform in [dim_lo, dim_hi]."""
    g = rng_for(seed)
    specs = []
    for _ in range(n_exprs):
        r = log_uniform_int(g, dim_lo, dim_hi)
        c = log_uniform_int(g, dim_lo, dim_hi)
        d = int(g.integers(depth_lo, depth_hi + 1))
        k = int(g.integers(ops_lo, ops_hi + 1))
        specs.append(random_tree(g, d, k, r, c, dtype))
    return specs


def operands_for(spec: TreeSpec, rng: np.random.Generator) -> list:
    """Operand arrays for a tree: U[-1,1] for floats, [0, 2^16) for integers."""
    out = []
    for shp in spec.slot_shapes:
        if spec.dtype in ("f32", "f64", "f16", "bf16"):
            out.append(uniform(rng, shp, spec.dtype))
        else:
            out.append(uniform_int(rng, shp, spec.dtype, 0, 1 << 16))
    return out
