"""coot-mi355x: fused dense-expression evaluation on MI355X (gfx950).

`_coot` is the ctypes binding of libcoot's C ABI (include/coot.h); `frontend`
holds the Armadillo-flavoured lazy expressions (Mat, trans, exp, accu, sum, dot,
norm, min, max, mean, var, norm1, norm_inf, eval).  Importing this package loads libcoot.so and fails if it is not
built — there is no CPU fallback.
"""
from . import _coot  # noqa: F401
from .frontend import (Batch, Expr, Mat, Node, Scalar, abs, accu, bcast_col, bcast_row, dot, eval,  # noqa: F401
                       eval_reduce, exp,
                       flatten, init, log, max, mean, min, norm, norm1, norm_inf, precompile, sqrt, square, sum, var,
                       trans, use_torch_allocator)
