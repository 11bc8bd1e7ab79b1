"""Host tests of the SILU_REORDER relabeling (silu_reorder_rcm: reverse
Cuthill-McKee on the strong couplings).  No GPU: the entry point works on host
arrays."""
import numpy as np
import pytest

from paper_2111_09512_amd import workloads as W


@pytest.fixture(scope="module")
def B():
    from paper_2111_09512_amd import binding

    return binding


def _is_perm(order, n):
    return order.shape == (n,) and np.array_equal(np.sort(order), np.arange(n))


def _path(n, perm=None):
    """Tridiagonal (2, -1) matrix, optionally with its rows and columns relabeled."""
    d = np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    if perm is not None:
        d = d[np.ix_(perm, perm)]
    return W.CSR.from_dense(d)


def test_path_graph_in_natural_order(B):
    """A path from its end (the least-degree row 0): BFS visits 0, 1, ..., n-1
    and the reversal gives n-1, ..., 0."""
    n = 9
    np.testing.assert_array_equal(B.reorder_rcm(_path(n)), np.arange(n)[::-1])


def test_relabeled_path_is_recovered(B):
    """Whatever the labels, consecutive positions of the result are path
    neighbours: every coupling spans one position."""
    n = 200
    perm = np.random.default_rng(3).permutation(n)
    A = _path(n, perm)
    order = B.reorder_rcm(A)
    assert _is_perm(order, n)
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    off = rows != A.col
    assert np.abs(pos[rows[off]] - pos[A.col[off]]).max() == 1


def test_weak_long_range_couplings_are_ignored(B):
    """The permuted 7-point operator with random long-range couplings of weight
    <= 1e-2: the grid couplings (weight 1) end up within a few planes of N^2
    positions, the random ones do not steer the order."""
    N = 12
    A = W.permuted_longrange7(N, seed=1)
    order = B.reorder_rcm(A)
    assert _is_perm(order, A.n)
    pos = np.empty(A.n, np.int64)
    pos[order] = np.arange(A.n)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    strong = (rows != A.col) & (np.abs(A.val) >= 0.5)
    span = np.abs(pos[rows[strong]] - pos[A.col[strong]])
    before = np.abs(rows[strong] - A.col[strong])
    assert np.percentile(span, 99) <= 3 * N * N  # level sets of a 3-D grid hold ~N^2 rows
    assert np.median(span) <= N * N and np.median(span) < np.median(before) / 3
    # with every coupling counted as strong (theta = 0) the long-range ones
    # join the graph and spread the grid couplings out
    order0 = B.reorder_rcm(A, theta=0.0)
    pos0 = np.empty(A.n, np.int64)
    pos0[order0] = np.arange(A.n)
    span0 = np.abs(pos0[rows[strong]] - pos0[A.col[strong]])
    assert np.percentile(span0, 99) > np.percentile(span, 99)


@pytest.mark.parametrize("make", [lambda: W.poisson7(6), lambda: W.aniso27(5), lambda: W.random_mmatrix(150, 0.04, seed=2),
                                  lambda: W.CSR.from_dense(np.diag(np.arange(1.0, 8.0)))],
                         ids=["poisson6", "aniso5", "mmatrix150", "diagonal7"])
def test_always_a_permutation_and_deterministic(B, make):
    A = make()
    o1, o2 = B.reorder_rcm(A), B.reorder_rcm(A)
    assert _is_perm(o1, A.n)
    np.testing.assert_array_equal(o1, o2)


def test_errors(B):
    A = _path(5)
    with pytest.raises(B.SiluError) as e:
        B.reorder_rcm(A, theta=-1.0)
    assert e.value.status == -1
    bad = W.CSR(A.n, A.row_ptr.copy(), A.col.copy(), A.val.copy())
    bad.col[2] = 7  # outside 0..n-1
    with pytest.raises(B.SiluError) as e:
        B.reorder_rcm(bad)
    assert e.value.status == -3
