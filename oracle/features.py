"""Cost-model feature vector (test infrastructure only).

Reading chosen for the learned tuner (the paper has none; listed in the design doc):
an expression signature on a shape, plus one launch configuration, becomes

    [ n_ops, n_operands, onehot(dtype: u32 s32 f32 f64),
      log2(1 + n_rows), log2(1 + n_cols), n_trans,
      onehot(reduction: none all dim0 dim1),
      log2(vec), log2(ept), log2(waves), log2(grid_mult) ]          (17 values)

n_ops counts the operator entries of the postfix list (not load / scalar pushes),
n_operands the distinct operand slots, n_trans the trans() entries.
"""
from __future__ import annotations

import math

import numpy as np

DTYPE_ORDER = ("u32", "s32", "f32", "f64")
RED_ORDER = ("none", "all", "dim0", "dim1")
N_FEATURES = 17


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


def features(postfix, dtype, n_rows, n_cols, red, cfg) -> np.ndarray:
    vec, ept, waves, grid_mult = cfg
    return np.asarray(expr_features(postfix, dtype, n_rows, n_cols, red) + cfg_features(vec, ept, waves, grid_mult),
                      dtype=np.float64)
