"""CPU oracle for the fused-expression path — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its Python binding) never
imports, calls or links anything here, and this package imports nothing from the
product.  Inputs come from the separate `synth` generators.

What it computes (plain definitions, no fusion, no blocking):

* `elementwise.evaluate` — an Armadillo-style expression given as a postfix list
  (the Op / eOp / eGlue node kinds of Section 3, evaluated on assignment as the
  delayed-evaluation paragraph of Section 3 describes) computed one operator at a
  time into a full temporary.  Floating types (f32, f64 and the 16-bit storage
  types f16, bf16): each operator's exact result rounded once to the element
  type.  u32 / s32: exact integer arithmetic reduced mod 2^32.
* `reduce` — accu / sum along a dimension / dot / norm (Fig. 1 and Section 5,
  task 1) as exact sums of the element values (Fractions), rounded once for
  reporting; integer sums mod 2^32.
* `mlp` — the binary64 reference of the learned launch-configuration cost model:
  a 3-Linear-layer ReLU network, masked mean-squared error and Adam.
* `features` — the feature vector the cost model reads.

Parity status of each function is listed in its docstring; every function here is
pinned by the `-m "not gpu"` tests under tests/ (closed forms, brute force with
exact rationals, finite differences).
"""
from . import elementwise, reduce, mlp, features  # noqa: F401
