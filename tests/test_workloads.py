"""The paper's test tensors (Sec. 7) as built by the input generators: the
properties the paper states for them, checked on seeded instances."""
import numpy as np

import workloads as W


def test_tensor3_density_bound_and_distinct_coordinates():
    """Tensor 3: a term of eq. (tsr_sparse) is nonzero with probability p^4, so the
    expected density is at most R_true^3 p^4 (the realised density of one seed
    is within 30 % of it); coordinates are distinct and values nonzero."""
    s, R, alpha, p = 400, 5, 1.2, 0.05
    idx, val = W.paper_tensor3(s, R, alpha, p, seed=3)
    Rt = W.true_rank(R, alpha)
    assert idx.shape[0] / s ** 3 <= 1.3 * Rt ** 3 * p ** 4
    assert idx.shape[0] > 0.3 * Rt ** 3 * p ** 4 * s ** 3
    lin = np.ravel_multi_index(idx.T.astype(np.int64), (s, s, s))
    assert np.unique(lin).size == lin.size
    assert np.all(val != 0.0)


def test_tensor3_equals_dense_definition_small():
    """The sparse construction equals C x_1 B1 x_2 B2 x_3 B3 formed densely from
    the same masked Gaussian draws (same generator calls, p large)."""
    s, R, alpha, p, seed = 12, 3, 1.0, 0.6, 4
    idx, val = W.paper_tensor3(s, R, alpha, p, seed)
    rs = np.random.default_rng(seed)
    keep = lambda shape: np.where(rs.random(shape) < p, rs.standard_normal(shape), 0.0)
    core = keep((3, 3, 3))
    fac = [keep((s, 3)) for _ in range(3)]
    X = np.einsum("xyz,ix,jy,kz->ijk", core, *fac)
    Y = np.zeros((s, s, s))
    Y[tuple(idx.T)] = val
    np.testing.assert_allclose(Y, X, atol=1e-12)


def test_tensor2_power_law_spikes():
    """Tensor 2 adds n = 5 unit rank-1 terms of size C ||T|| / i^(1+eta); random
    unit directions in 200 dimensions are nearly orthogonal, so the added norm^2
    is sum lambda_i^2 within a few per cent."""
    s, R, alpha = 200, 5, 1.6
    X1 = W.paper_tensor1(s, R, alpha, seed=2)
    X2 = W.paper_tensor2(s, R, alpha, seed=2)
    lam = 3.0 * np.linalg.norm(X1) / np.arange(1, 6) ** 1.5
    np.testing.assert_allclose(np.linalg.norm(X2 - X1) ** 2, np.sum(lam ** 2), rtol=0.03)


def test_tensor4_coherent_entries():
    """Tensor 4 adds n = 10 entries at distinct random positions with values
    N(||T|| / sqrt(n), 1): E ||N|| / ||T|| = 1."""
    s, R, alpha = 100, 5, 1.6
    X1 = W.paper_tensor1(s, R, alpha, seed=5)
    X4 = W.paper_tensor4_dense(s, R, alpha, seed=5)
    D = X4 - X1
    nz = np.flatnonzero(D)
    assert nz.size == 10
    np.testing.assert_allclose(np.linalg.norm(D) / np.linalg.norm(X1), 1.0, rtol=0.01)
    idx, val = W.paper_tensor3(300, 5, 1.2, 0.05, seed=1)
    idx4, val4 = W.paper_tensor4_sparse(300, 5, 1.2, 0.05, seed=1)
    assert idx.shape[0] <= idx4.shape[0] <= idx.shape[0] + 10
    np.testing.assert_allclose(np.linalg.norm(val4) ** 2,
                               np.linalg.norm(val) ** 2 * 2, rtol=0.05)


def test_sparse2000det_first_sweep_sketches_full_rank(monkeypatch):
    """The deterministic-selection workload keeps m = 24 R^2 rows so that the
    selected sketch Z of every subproblem spans all r = 100 directions (its Gram
    is then invertible, as RSVD-LRLS requires); checked in the oracle over the
    first sweep from the range-finder start."""
    from oracle import sketch as osk, solve as osv, tucker as otk
    w = W.sparse2000det()
    assert w.m == 24 * w.ranks[0] ** 2
    To = osk.Tensor(w.dims, w.idx, w.val.astype(np.float64))
    ranks = []
    orig = osv.rsvd_lrls

    def spy(Z, Y, R, Om):
        ranks.append(np.linalg.matrix_rank(Z))
        return orig(Z, Y, R, Om)

    monkeypatch.setattr(osv, "rsvd_lrls", spy)
    otk.sketch_tucker_als(To, w.ranks, w.m, 1, seed=0, sketch_kind="lev_det", solve_kind="rsvd",
                          record_fit=False)
    assert ranks == [100, 100, 100]
