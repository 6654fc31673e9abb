"""Cost-model feature vector (test infrastructure only).

Reading chosen for the learned tuner (the paper has none):
an expression signature on a shape, plus one launch configuration, becomes

    [ n_ops, n_operands, onehot(dtype: u32 s32 f32 f64),
      log2(1 + n_rows), log2(1 + n_cols), n_trans,
      onehot(reduction: none all dim0 dim1),
      log2(vec), log2(ept), log2(waves), log2(grid_mult),
      log2(1 + elements), tiled, log2(workgroups), log2(1 + elements per thread),
      log2(tile_r), log2(tile_c) ]                                  (23 values)

n_ops counts the operator entries of the postfix list (not load / scalar pushes),
n_operands the distinct operand slots, n_trans the trans() entries.  The next four
describe the launch the configuration implies for contiguous operands on 256 CUs:
the tiled family (some leaf read transposed, i.e. under an odd number of trans(),
or a dimension sum) runs 256 threads per tile_r x tile_c tile (64 x 64 when the
configuration names none) and min(tiles, grid_mult * 256) workgroups; the flat
family runs 64 * waves threads per workgroup, each taking ept groups of vec
elements, and min(ceil(ceil(elements / vec) / (threads * ept)), grid_mult * 256)
workgroups (at least 1).  The last two are the tile's edges for the tiled family
and 0 for the flat one (the tile shape is part of the tiled family's configuration
space).  A configuration is (vec, ept, waves, grid_mult[, tile_r, tile_c]).
"""
from __future__ import annotations

import math

import numpy as np

DTYPE_ORDER = ("u32", "s32", "f32", "f64")
RED_ORDER = ("none", "all", "dim0", "dim1")
N_FEATURES = 23
CUS = 256


def expr_features(postfix, dtype: str, n_rows: int, n_cols: int, red: str = "none") -> list:
    n_ops = sum(1 for it in postfix if it[0] not in ("load", "scalar"))
    n_operands = len({it[1] for it in postfix if it[0] == "load"})
    n_trans = sum(1 for it in postfix if it[0] == "trans")
    f = [float(n_ops), float(n_operands)]
    f += [1.0 if dtype == d else 0.0 for d in DTYPE_ORDER]
    f += [math.log2(1 + n_rows), math.log2(1 + n_cols), float(n_trans)]
    f += [1.0 if red == r else 0.0 for r in RED_ORDER]
    return f


def cfg_features(vec: int, ept: int, waves: int, grid_mult: int) -> list:
    return [math.log2(vec), math.log2(ept), math.log2(waves), math.log2(grid_mult)]


def has_transposed_leaf(postfix) -> bool:
    """Whether some load sits under an odd number of trans() (walk the postfix tree)."""
    st = []
    for it in postfix:
        if it[0] in ("load", "scalar"):
            st.append([(it[0] == "load", 0)])
        elif it[0] in ("add", "sub", "schur", "div"):
            b, a = st.pop(), st.pop()
            st.append(a + b)
        elif it[0] == "trans":
            st.append([(is_load, p ^ 1) for is_load, p in st.pop()])
        else:
            pass  # unary ops keep their operand's leaves
    return any(is_load and p == 1 for is_load, p in st[-1])


def launch_features(postfix, n_rows, n_cols, red, cfg) -> list:
    vec, ept, waves, grid_mult = cfg[:4]
    tile_r, tile_c = (cfg[4], cfg[5]) if len(cfg) > 4 and cfg[4] else (64, 64)
    n = n_rows * n_cols
    tiled = has_transposed_leaf(postfix) or red in ("dim0", "dim1")
    cap = grid_mult * CUS
    if tiled:
        grid = min(math.ceil(n_rows / tile_r) * math.ceil(n_cols / tile_c), cap)
        threads = 256
    else:
        threads = 64 * waves
        grid = min(math.ceil(max(1, math.ceil(n / vec)) / (threads * ept)), cap)
    grid = max(1, grid)
    tile = [math.log2(tile_r), math.log2(tile_c)] if tiled else [0.0, 0.0]
    return [math.log2(1 + n), 1.0 if tiled else 0.0, math.log2(grid), math.log2(1 + n / (grid * threads))] + tile


def features(postfix, dtype, n_rows, n_cols, red, cfg) -> np.ndarray:
    vec, ept, waves, grid_mult = cfg[:4]
    return np.asarray(expr_features(postfix, dtype, n_rows, n_cols, red) + cfg_features(vec, ept, waves, grid_mult)
                      + launch_features(postfix, n_rows, n_cols, red, cfg), dtype=np.float64)
