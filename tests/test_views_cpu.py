"""Host logic of the views (no GPU): submatrix, row / column, diagonal and broadcast
views keep the parent's storage and carry the right shape, leading dimension and
kind into the operand description the boundary receives."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def coot():
    import paper_2508_11385_amd as coot
    return coot


def test_submatrix_views_share_storage(coot):
    a = np.arange(150 * 97, dtype=np.float32).reshape(97, 150).T      # 150 x 97, column-major values
    P = coot.Mat.from_numpy(a, device="cpu")
    assert (P.n_rows, P.n_cols, P.ld) == (150, 97, 150)
    s = P.submat(5, 7, 65, 51)
    assert (s.n_rows, s.n_cols, s.ld, s.kind) == (61, 45, 150, "mat")
    assert s.tensor.data_ptr() == P.tensor.data_ptr() + (5 + 7 * 150) * 4
    assert np.array_equal(s.numpy(), a[5:66, 7:52])
    r = P.row(149)
    assert (r.n_rows, r.n_cols, r.ld, r.kind) == (1, 97, 150, "row")
    assert np.array_equal(r.numpy().ravel(), a[149])
    c = P.col(3)
    assert (c.n_rows, c.n_cols, c.kind) == (150, 1, "col")
    assert (P.rows(10, 12).n_rows, P.cols(90, 96).n_cols) == (3, 7)
    op = s.operand()
    assert (op.n_rows, op.n_cols, op.ld) == (61, 45, 150)
    for bad in ((0, 0, 150, 3), (3, 0, 2, 5), (0, -1, 4, 4), (0, 0, 4, 97)):
        with pytest.raises(IndexError):
            P.submat(*bad)


def test_diagonal_and_broadcast_views(coot):
    X = coot.Mat.from_numpy(np.arange(7 * 3, dtype=np.float32).reshape(3, 7).T, device="cpu")   # 7 x 3
    d = X.diag()
    assert (d.n_rows, d.n_cols, d.ld, d.kind) == (1, 3, 8, "row")
    assert np.array_equal(d.numpy().ravel(), np.diag(X.numpy()))
    v = coot.Mat.from_numpy(np.ones((7, 1), np.float32), kind="col", device="cpu")
    b = coot.bcast_col(v, 5)
    assert (b.n_rows, b.n_cols, b.ld, b.kind) == (7, 5, 0, "bcast")
    with pytest.raises(ValueError):
        b.submat(0, 0, 1, 1)
    with pytest.raises(ValueError):
        coot.var(X, norm_type=2)
