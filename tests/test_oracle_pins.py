"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a published
generator vector, a hand-worked example, a brute-force evaluation of a
definition with explicit matrices, a closed form, an exact identity of the
paper (Kronecker leverage lemma, orthogonal residual split of the
rank-constrained theorem), a statistical law with a stated bound, or the
unsketched HOOI of Alg. 1.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import adjoint, cp, rng, sketch, solve, tucker
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# generator
# ----------------------------------------------------------------------------
def test_splitmix64_published_vectors():
    # SplitMix64 outputs from state 0 and from state 1234567 (the reference
    # test vectors of the published generator).
    got0 = [int(v) for v in rng.draw(rng.stream_key(0), [0, 1, 2])]
    assert got0 == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got1 = [int(v) for v in rng.draw(rng.stream_key(1234567), range(5))]
    assert got1 == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                    4593380528125082431, 16408922859458223821]


def test_bucket_sign_uniform_statistics():
    m, n = 97, 200_000
    x = rng.draw(rng.stream_key(7, rng.P_TS, 0, 1), np.arange(n))
    b = rng.bucket(x, m).astype(np.int64)
    assert b.min() >= 0 and b.max() < m
    cnt = np.bincount(b, minlength=m)
    chi2 = float(np.sum((cnt - n / m) ** 2 / (n / m)))
    # chi^2 with 96 dof: mean 96, sd ~13.9; 6 sd bound
    assert chi2 < 96 + 6 * 13.9
    s = rng.sign(x)
    assert abs(s.mean()) < 6 / np.sqrt(n)
    u = rng.uniform(x)
    assert 0 <= u.min() and u.max() < 1 and abs(u.mean() - 0.5) < 6 * np.sqrt(1 / 12 / n)


def test_gauss_moments():
    g = rng.gauss(rng.stream_key(3, rng.P_RRF_G, 1), np.arange(200_000))
    assert abs(g.mean()) < 6 / np.sqrt(2e5)
    assert abs(g.var() - 1) < 6 * np.sqrt(2 / 2e5)


# ----------------------------------------------------------------------------
# TensorSketch (Sec. 3.1)
# ----------------------------------------------------------------------------
def _golden_tables(d):
    return {int(k): (np.array(d["h"][k], dtype=np.int64), np.array(d["sigma"][k], float))
            for k in d["h"]}


def test_golden_worked_example():
    d = json.load(open(os.path.join(GOLDEN, "ts_worked_example.json")))
    dims, m, n = tuple(d["dims"]), d["m"], d["n"]
    X = np.zeros(dims)
    for i in itertools.product(*map(range, dims)):
        X[i] = 1 + 6 * i[0] + 2 * i[1] + i[2]
    T = sketch.Tensor.from_dense(X)
    tabs = _golden_tables(d)
    Y = sketch.ts_rhs(T, m, tabs, n)
    np.testing.assert_array_equal(Y, np.array(d["Y"]))
    A1, A2 = np.array(d["A1"]), np.array(d["A2"])
    np.testing.assert_array_equal(sketch.countsketch(A1, *tabs[1], m)[:, 0], d["CS1"])
    np.testing.assert_array_equal(sketch.countsketch(A2, *tabs[2], m)[:, 0], d["CS2"])
    Z = sketch.ts_lhs([None, A1, A2], tabs, m, n)
    np.testing.assert_allclose(Z[:, 0], d["Z"], atol=1e-15)
    A, W, _ = solve.rc_solve(Z, Y, 1)
    np.testing.assert_allclose(A[:, 0], d["A0"], rtol=1e-14)
    np.testing.assert_allclose(W[0, 0], d["W"], rtol=1e-14)


def _explicit_ts_matrix(dims, tables, m, n):
    """S^(n) as an explicit m x K matrix built entry by entry from the definition
    (Omega(H(i), i) = 1, D(i, i) = S(i)) over the row-major other-mode index."""
    ks = [k for k in range(len(dims)) if k != n]
    K = int(np.prod([dims[k] for k in ks]))
    S = np.zeros((m, K))
    for col, multi in enumerate(itertools.product(*[range(dims[k]) for k in ks])):
        H, sg = 0, 1.0
        for k, i in zip(ks, multi):
            H += int(tables[k][0][i])
            sg *= tables[k][1][i]
        S[H % m, col] = sg
    return S


@pytest.mark.parametrize("dims,m,n", [((3, 4, 5), 7, 0), ((4, 3, 5), 6, 1),
                                      ((2, 3, 2, 3), 5, 3), ((5, 6), 4, 1)])
def test_ts_rhs_equals_explicit_matrix(dims, m, n):
    rs = np.random.default_rng(1)
    X = rs.standard_normal(dims)
    T = sketch.Tensor.from_dense(X)
    tabs = sketch.ts_tables(dims, m, 11, n)
    S = _explicit_ts_matrix(dims, tabs, m, n)
    Y_bf = S @ tucker.unfold(X, n).T
    np.testing.assert_allclose(sketch.ts_rhs(T, m, tabs, n), Y_bf, atol=1e-13)
    # COO with duplicates: the sketch is linear, duplicates add
    idx = np.concatenate([T.idx, T.idx[:5]])
    val = np.concatenate([T.val, -2 * T.val[:5]])
    X2 = X.copy()
    for e in range(5):
        X2[tuple(T.idx[e])] -= 2 * T.val[e]
    Y2 = sketch.ts_rhs(sketch.Tensor(dims, idx, val), m, tabs, n)
    np.testing.assert_allclose(Y2, S @ tucker.unfold(X2, n).T, atol=1e-13)


@pytest.mark.parametrize("dims,ranks,m,n", [((4, 5, 6), (2, 3, 2), 8, 0),
                                            ((4, 5, 6), (2, 3, 2), 9, 2),
                                            ((3, 4, 3, 4), (2, 2, 3, 2), 10, 1)])
def test_ts_lhs_three_routes(dims, ranks, m, n):
    """S P by (a) explicit S times the explicit Kronecker chain, (b) the oracle's
    direct circular convolution, (c) NumPy's FFT of the CountSketches."""
    rs = np.random.default_rng(2)
    facs = [rs.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    tabs = sketch.ts_tables(dims, m, 5, n)
    ks = [k for k in range(len(dims)) if k != n]
    Z_explicit = _explicit_ts_matrix(dims, tabs, m, n) @ tucker.kron_chain([facs[k] for k in ks])
    Z_conv = sketch.ts_lhs(facs, tabs, m, n)
    spec = np.ones((m, 1), dtype=complex)
    for k in ks:
        F = np.fft.fft(sketch.countsketch(facs[k], *tabs[k], m), axis=0)
        spec = (spec[:, :, None] * F[:, None, :]).reshape(m, -1)
    Z_fft = np.fft.ifft(spec, axis=0).real
    np.testing.assert_allclose(Z_conv, Z_explicit, atol=1e-12)
    np.testing.assert_allclose(Z_fft, Z_explicit, atol=1e-12)


def test_ts_norm_unbiased_and_variance_bound():
    """E ||S x||^2 = ||x||^2 for TensorSketch; Var <= (2 + 3^{N'}) / m ||x||^4
    (approximate matrix product lemma with P = B = x), checked over 4000 seeds."""
    dims, m = (6, 7), 16
    rs = np.random.default_rng(3)
    x = rs.standard_normal(dims)
    T = sketch.Tensor.from_dense(x[None])                 # order 3, mode 0 of size 1
    nx2 = float(np.sum(x * x))
    vals = []
    for seed in range(4000):
        tabs = sketch.ts_tables((1,) + dims, m, seed, 0)
        y = sketch.ts_rhs(T, m, tabs, 0)
        vals.append(float(np.sum(y * y)))
    vals = np.array(vals)
    var_bound = (2 + 3 ** 2) / m * nx2 ** 2
    assert abs(vals.mean() - nx2) < 5 * np.sqrt(var_bound / len(vals))
    assert vals.var() <= var_bound * 1.2


# ----------------------------------------------------------------------------
# Leverage scores (Sec. 3.2)
# ----------------------------------------------------------------------------
def test_leverage_kronecker_lemma():
    rs = np.random.default_rng(4)
    facs = [np.linalg.qr(rs.standard_normal((s, r)))[0] for s, r in ((5, 2), (4, 3), (6, 2))]
    P = tucker.kron_chain(facs)
    Q, _ = np.linalg.qr(P)
    lev_P = np.sum(Q * Q, axis=1)
    prod = np.ones(1)
    for F in facs:
        prod = np.multiply.outer(prod, sketch.leverage_scores(F)).reshape(-1)
    np.testing.assert_allclose(lev_P, prod, atol=1e-14)
    for F in facs:
        assert abs(sketch.leverage_scores(F).sum() - F.shape[1]) < 1e-13


def test_leverage_sampling_law_and_unbiasedness():
    rs = np.random.default_rng(5)
    facs = [np.linalg.qr(rs.standard_normal((s, 2)))[0] for s in (7, 5, 6)]
    m, n = 20000, 0
    idx, w = sketch.leverage_sample(facs, m, 9, 0, n)
    for t, k in enumerate((1, 2)):
        p = sketch.leverage_scores(facs[k]) / facs[k].shape[1]
        cnt = np.bincount(idx[:, t], minlength=p.size)
        chi2 = np.sum((cnt - m * p) ** 2 / (m * p))
        assert chi2 < (p.size - 1) + 6 * np.sqrt(2 * (p.size - 1))
    # weights: D(j, j) = 1/sqrt(m p_i), p_i = prod_k l_{i_k} / R_k
    p_row = np.ones(m)
    for t, k in enumerate((1, 2)):
        p_row *= sketch.leverage_scores(facs[k])[idx[:, t]] / facs[k].shape[1]
    np.testing.assert_allclose(w, 1 / np.sqrt(m * p_row), rtol=1e-12)
    # E ||S x||^2 = sum_i p_i * m * x_i^2 / (m p_i) = ||x||^2 exactly (enumeration)
    x = rs.standard_normal(7 * 5 * 6).reshape(7, 5, 6)
    pk = [sketch.leverage_scores(F) / F.shape[1] for F in facs]
    expect = 0.0
    for i in itertools.product(range(5), range(6)):
        pi = pk[1][i[0]] * pk[2][i[1]]
        expect += pi * m * np.sum(x[:, i[0], i[1]] ** 2) / (m * pi)
    assert abs(expect - np.sum(x * x)) < 1e-9 * np.sum(x * x)


def test_leverage_rows_match_explicit_kronecker():
    rs = np.random.default_rng(6)
    facs = [np.linalg.qr(rs.standard_normal((s, r)))[0] for s, r in ((5, 2), (4, 3), (6, 2))]
    idx, w = sketch.leverage_sample(facs, 50, 1, 0, 1)
    P = tucker.kron_chain([facs[0], facs[2]])
    rows = idx[:, 0] * 6 + idx[:, 1]
    np.testing.assert_allclose(sketch.leverage_lhs(facs, idx, w, 1), w[:, None] * P[rows], atol=1e-15)
    X = rs.standard_normal((5, 4, 6))
    Y = sketch.leverage_rhs_dense(X, idx, w, 1)
    np.testing.assert_allclose(Y, w[:, None] * tucker.unfold(X, 1).T[rows], atol=1e-15)
    Ys = sketch.leverage_rhs_sparse(sketch.Tensor.from_dense(X), idx, w, 1)
    np.testing.assert_allclose(Ys, Y, atol=1e-14)


def test_leverage_select_hand_worked_ties():
    """Deterministic selection with ties, worked by hand.  Mode-0 scores
    (1, 4, 4) from rows (1), (2), (2); mode-2 scores (9, 1) from rows (3), (1).
    Row scores: (0,0) 9, (0,1) 1, (1,0) 36, (1,1) 4, (2,0) 36, (2,1) 4.  Per-mode
    ranks (score descending, index ascending): mode 0 -> (2, 0, 1), mode 2 ->
    (0, 1).  Order: 36 (1,0) before (2,0) by rank; 9 (0,0); 4 (1,1) before
    (2,1); 1 (0,1)."""
    facs = [np.array([[1.0], [2.0], [2.0]]), np.eye(4, 2), np.array([[3.0], [1.0]])]
    idx, w = sketch.leverage_select(facs, 5, 1)
    assert idx.tolist() == [[1, 0], [2, 0], [0, 0], [1, 1], [2, 1]]
    assert np.all(w == 1.0)
    Z = sketch.leverage_lhs(facs, idx, w, 1)
    np.testing.assert_array_equal(Z[:, 0], [6.0, 6.0, 3.0, 2.0, 2.0])
    # ties where rank order and index order disagree: scores (1, 4) and (4, 1);
    # pi(0,0) = pi(1,1) = 4 with rank tuples (1, 0) and (0, 1): (1,1) comes first
    facs = [np.array([[1.0], [2.0]]), np.eye(3, 1), np.array([[2.0], [1.0]])]
    idx, _ = sketch.leverage_select(facs, 4, 1)
    assert idx.tolist() == [[1, 0], [1, 1], [0, 0], [0, 1]]


def test_leverage_select_is_top_rows_of_explicit_kronecker():
    """The kept rows are the m rows of largest squared norm of the explicit
    Kronecker product P = A^(0) (x) A^(2) (its leverage scores, orthonormal
    columns), in decreasing order; the fixture has a clear gap at m."""
    rs = np.random.default_rng(12)
    facs = [np.linalg.qr(rs.standard_normal((s, r)))[0] for s, r in ((9, 2), (5, 3), (8, 3))]
    P = tucker.kron_chain([facs[0], facs[2]])
    lev = np.sum(P * P, axis=1)
    m = 17
    top = np.argsort(-lev, kind="stable")
    assert lev[top[m - 1]] - lev[top[m]] > 1e-9
    idx, _ = sketch.leverage_select(facs, m, 1)
    rows = idx[:, 0] * 8 + idx[:, 1]
    assert sorted(rows.tolist()) == sorted(top[:m].tolist())
    assert np.all(np.diff(lev[rows]) <= 1e-15)
    np.testing.assert_allclose(lev.sum(), 2 * 3, rtol=1e-13)   # sum of scores = prod R_k


def test_leverage_select_rank_dominance_bound():
    """A kept row's per-mode ranks satisfy prod_k (rank_k + 1) <= m: the rows
    that dominate it in every mode all come first (pi is monotone in every
    factor; equal pi is ordered by the ranks).  The library enumerates exactly
    these candidates, so the bound is checked here, on ties too."""
    rs = np.random.default_rng(3)
    for dims, n, m in (((30, 20, 25), 0, 60), ((12, 9, 10, 8), 2, 150)):
        facs = [np.linalg.qr(rs.standard_normal((s, 3)))[0] for s in dims]
        facs[(n + 1) % len(dims)][3] = facs[(n + 1) % len(dims)][4]    # a tie
        idx, _ = sketch.leverage_select(facs, m, n)
        ks = [k for k in range(len(dims)) if k != n]
        ranks = [sketch.score_ranks(sketch.leverage_scores(facs[k])) for k in ks]
        bound = np.ones(m, dtype=np.int64)
        for t in range(len(ks)):
            bound *= ranks[t][idx[:, t]] + 1
        assert bound.max() <= m


def test_leverage_select_all_rows_reproduces_identity_sketch():
    """Keeping every row (m = prod_{k != n} s_k) with weight 1 permutes the
    rows of the full subproblem, so the driver reproduces the unsketched one."""
    X = workloads.tucker_dense((9, 9, 9), (3, 2, 3), noise=0.2, seed=5)
    T = sketch.Tensor.from_dense(X)
    init = tucker.hosvd(X, (3, 2, 3))
    a = tucker.sketch_tucker_als(T, (3, 2, 3), m=81, sweeps=2, init="user", init_factors=init,
                                 sketch_kind="lev_det")
    b = tucker.sketch_tucker_als(T, (3, 2, 3), m=0, sweeps=2, init="user", init_factors=init,
                                 identity_sketch=True)
    np.testing.assert_allclose(a["fits"], b["fits"], atol=1e-12)
    for Fa, Fb in zip(a["factors"], b["factors"]):
        np.testing.assert_allclose(Fa, Fb, atol=1e-10)


# ----------------------------------------------------------------------------
# Rank-constrained solve (Sec. 4)
# ----------------------------------------------------------------------------
def test_solve_orthonormal_Z_is_eckart_young():
    """Z with orthonormal columns: the best rank-R approximation of Z^+ Y is the
    rank-R minimiser of ||Z X - Y|| and the residual splits orthogonally,
    ||Z X_r - Y||^2 = ||B_perp||^2 + ||X_r - X_opt||^2."""
    rs = np.random.default_rng(7)
    Z = np.linalg.qr(rs.standard_normal((60, 12)))[0]
    Y = rs.standard_normal((60, 15))
    R = 3
    A, W, X = solve.rc_solve(Z, Y, R)
    Xr = W @ A.T
    U, S, Vt = np.linalg.svd(Z.T @ Y)
    Xr_ey = (U[:, :R] * S[:R]) @ Vt[:R]
    np.testing.assert_allclose(Xr, Xr_ey, atol=1e-12)
    Bperp = Z @ (Z.T @ Y) - Y
    lhs = np.sum((Z @ Xr - Y) ** 2)
    rhs = np.sum(Bperp ** 2) + np.sum((Xr - Z.T @ Y) ** 2)
    assert abs(lhs - rhs) < 1e-10 * lhs
    # no other rank-R matrix does better (random rank-R perturbations)
    for _ in range(20):
        D = 1e-3 * rs.standard_normal((12, R)) @ rs.standard_normal((R, 15))
        U2, S2, V2 = np.linalg.svd(Xr + D)
        Xc = (U2[:, :R] * S2[:R]) @ V2[:R]
        assert np.sum((Z @ Xc - Y) ** 2) >= lhs - 1e-12
    np.testing.assert_allclose(A.T @ A, np.eye(R), atol=1e-13)


def test_solve_general_Z_matches_qr_route():
    rs = np.random.default_rng(8)
    Z = rs.standard_normal((80, 10)) @ np.diag(np.logspace(0, 1, 10))
    Y = rs.standard_normal((80, 30))
    A, W, X = solve.rc_solve(Z, Y, 4)
    Q, Rz = np.linalg.qr(Z)
    X_qr = np.linalg.solve(Rz, Q.T @ Y)
    np.testing.assert_allclose(X, X_qr, atol=1e-11)
    _, _, Vt = np.linalg.svd(X_qr)
    V = Vt[:4].T
    # same subspace and, after the sign rule, the same columns
    np.testing.assert_allclose(A @ A.T, V @ V.T, atol=1e-11)
    Vf, _ = solve.sign_fix(V)
    np.testing.assert_allclose(A, Vf, atol=1e-11)
    np.testing.assert_allclose(W, X_qr @ Vf, atol=1e-10)


def test_sign_fix_rule():
    A = np.array([[0.1, -0.5], [-0.9, 0.5], [0.2, 0.1]])
    F, s = solve.sign_fix(A)
    np.testing.assert_array_equal(s, [-1.0, -1.0])   # tie in column 1 -> first index
    np.testing.assert_array_equal(F, -A)


def test_rsvd_lrls_exact_when_rank_fits():
    """Alg. 5 with a test matrix of >= rank(X_opt) columns reproduces the exact
    truncated solve (the randomized range is the whole range)."""
    rs = np.random.default_rng(9)
    Z = rs.standard_normal((50, 6))
    Y = Z @ rs.standard_normal((6, 3)) @ rs.standard_normal((3, 20)) + 1e-3 * rs.standard_normal((50, 20))
    A, W, _ = solve.rc_solve(Z, Y, 2)
    Om = rs.standard_normal((20, 6))
    A2, W2 = solve.rsvd_lrls(Z, Y, 2, Om)
    np.testing.assert_allclose(A2, A, atol=1e-10)
    np.testing.assert_allclose(W2, W, atol=1e-10)


# ----------------------------------------------------------------------------
# Drivers
# ----------------------------------------------------------------------------
def test_identity_sketch_reproduces_hooi():
    """With S = I every subproblem is the HOOI update (Alg. 1), so from the same
    initial factors the two drivers produce the same factors and fits."""
    X = workloads.tucker_dense((12, 10, 11), (3, 4, 3), noise=0.3, seed=3)
    T = sketch.Tensor.from_dense(X)
    init = tucker.hosvd(X, (3, 4, 3))
    a = tucker.sketch_tucker_als(T, (3, 4, 3), m=0, sweeps=3, init="user",
                                 init_factors=init, identity_sketch=True)
    b = tucker.hooi(X, (3, 4, 3), 3, init_factors=init)
    for Fa, Fb in zip(a["factors"], b["factors"]):
        np.testing.assert_allclose(Fa, Fb, atol=1e-10)
    np.testing.assert_allclose(a["fits"], b["fits"], atol=1e-12)
    np.testing.assert_allclose(a["core"], b["core"], atol=1e-10)


@pytest.mark.parametrize("kind", ["ts", "lev"])
def test_exact_tucker_rank_recovered(kind):
    """Noise-free tensor of Tucker rank R with RRF init: one sweep reaches a
    relative residual at rounding level (the sketched problem is consistent)."""
    X = workloads.tucker_dense((20, 18, 16), (3, 3, 3), noise=0.0, seed=4)
    T = sketch.Tensor.from_dense(X)
    out = tucker.sketch_tucker_als(T, (3, 3, 3), m=8 * 9, sweeps=1, seed=2, sketch_kind=kind)
    assert out["fits"][-1] < 1e-12


def test_exact_rank_sparse_coo_fit_formula():
    X = workloads.tucker_dense((9, 8, 7), (2, 2, 2), noise=0.0, seed=5)
    Td = sketch.Tensor.from_dense(X)
    Ts = sketch.Tensor(X.shape, Td.idx, Td.val)                  # same data, COO path
    out = tucker.sketch_tucker_als(Ts, (2, 2, 2), m=40, sweeps=2, seed=1)
    assert out["fits"][-1] < 1e-6          # sparse formula: sqrt of a cancelling sum
    dense = tucker.relative_residual(Td, out["core"], out["factors"])
    assert dense < 1e-12


def test_rrf_recovers_exact_column_space():
    """Thm. (good low-rank subspace) with zero tail: for T_(n) of exact rank R
    the range finder returns a basis of its column space."""
    X = workloads.tucker_dense((15, 30, 14), (4, 5, 3), noise=0.0, seed=6)
    T = sketch.Tensor.from_dense(X)
    for n, R in ((1, 5), (2, 3)):
        A = tucker.init_rrf(T, n, R, k1=2 * R, k2=R * R + 2 * R, seed=3)
        U = np.linalg.svd(tucker.unfold(X, n), full_matrices=False)[0][:, :R]
        cosines = np.linalg.svd(A.T @ U, compute_uv=False)
        assert np.all(np.abs(1 - cosines) < 1e-12)


def test_sketched_fit_close_to_hooi():
    """Fit of sketched Tucker-ALS is at least HOOI's and close to it (Sec. 4
    theorems; Sec. 7 reports < 8.5% relative fitness gap at K = 16)."""
    w = workloads.dense40()
    T = sketch.Tensor.from_dense(w.dense)
    out = tucker.sketch_tucker_als(T, w.ranks, 16 * 25, 5, seed=0)
    h = tucker.hooi(w.dense, w.ranks, 5)
    assert out["fits"][-1] >= h["fits"][-1] - 1e-12
    assert (1 - out["fits"][-1]) > 0.915 * (1 - h["fits"][-1])


# ----------------------------------------------------------------------------
# CP on the core (Alg. 2, Alg. 6)
# ----------------------------------------------------------------------------
def test_cp_als_exact_cp_tensor():
    rs = np.random.default_rng(10)
    facs = [rs.standard_normal((s, 3)) for s in (8, 7, 6)]
    X = cp.cp_reconstruct(facs)
    init = [F + 0.05 * rs.standard_normal(F.shape) for F in facs]
    A = cp.cp_als(X, init, 60)
    assert cp.cp_relative_residual(sketch.Tensor.from_dense(X), A) < 1e-8


def test_mttkrp_matches_elementwise_definition():
    rs = np.random.default_rng(11)
    X = rs.standard_normal((4, 3, 5))
    F = [rs.standard_normal((s, 2)) for s in (4, 3, 5)]
    M = cp.mttkrp(X, F, 1)
    ref = np.zeros((3, 2))
    for i, j, k in itertools.product(range(4), range(3), range(5)):
        ref[j] += X[i, j, k] * F[0][i] * F[2][k]
    np.testing.assert_allclose(M, ref, atol=1e-13)


def test_cp_via_tucker_exact_cp_tensor():
    """An exact CP-rank-R tensor has Tucker rank <= R; Alg. 6 then recovers a CP
    model with residual at rounding level (Sec. 6.2)."""
    rs = np.random.default_rng(12)
    facs = [rs.standard_normal((s, 3)) for s in (14, 13, 12)]
    X = cp.cp_reconstruct(facs)
    out = cp.cp_sketch_tucker(sketch.Tensor.from_dense(X), 3, (3, 3, 3), m=90,
                              tucker_sweeps=2, cp_sweeps=200, seed=0, sketch_kind="ts")
    assert out["fit"] < 1e-6


# ----------------------------------------------------------------------------
# Adjoint of the sketched residual
# ----------------------------------------------------------------------------
def _adjoint_case(seed=13, dims=(6, 5, 7), ranks=(2, 3, 2), m=11, n=0):
    rs = np.random.default_rng(seed)
    facs = [rs.standard_normal((s, r)) for s, r in zip(dims, ranks)]
    core = rs.standard_normal(ranks)
    tabs = sketch.ts_tables(dims, m, 4, n)
    X = rs.standard_normal(dims)
    Y = sketch.ts_rhs(sketch.Tensor.from_dense(X), m, tabs, n)
    return facs, core, tabs, Y, m, n, X


def test_adjoint_matches_finite_differences():
    """L is quadratic in every single entry, so the central difference with
    h = 1e-3 is exact up to rounding."""
    facs, core, tabs, Y, m, n, _ = _adjoint_case()
    L, grads, gC = adjoint.residual_and_grads(facs, core, tabs, Y, m, n)
    h = 1e-3
    rs = np.random.default_rng(0)
    for k in range(3):
        for _ in range(6):
            i, c = rs.integers(facs[k].shape[0]), rs.integers(facs[k].shape[1])
            fp = [F.copy() for F in facs]; fm = [F.copy() for F in facs]
            fp[k][i, c] += h; fm[k][i, c] -= h
            fd = (adjoint.residual(fp, core, tabs, Y, m, n) -
                  adjoint.residual(fm, core, tabs, Y, m, n)) / (2 * h)
            assert abs(fd - grads[k][i, c]) <= 1e-8 * max(1.0, abs(fd))
    for _ in range(8):
        j = tuple(rs.integers(r) for r in core.shape)
        cp_, cm_ = core.copy(), core.copy()
        cp_[j] += h; cm_[j] -= h
        fd = (adjoint.residual(facs, cp_, tabs, Y, m, n) -
              adjoint.residual(facs, cm_, tabs, Y, m, n)) / (2 * h)
        assert abs(fd - gC[j]) <= 1e-8 * max(1.0, abs(fd))


def test_adjoint_matches_explicit_matrix_gradient():
    """Same gradients from explicit S (m x K) and explicit Kronecker P: the
    residual is ||S P W A^T - S T_(n)^T||^2 = ||S (P W A^T - T_(n)^T)||^2."""
    facs, core, tabs, Y, m, n, X = _adjoint_case(dims=(5, 4, 3), ranks=(2, 2, 2), m=7, n=1)
    S = _explicit_ts_matrix(X.shape, tabs, m, n)
    P = tucker.kron_chain([facs[0], facs[2]])
    W = tucker.core_to_W(core, n)
    A = facs[n]
    E = S @ (P @ W @ A.T - tucker.unfold(X, n).T)
    L, grads, gC = adjoint.residual_and_grads(facs, core, tabs, Y, m, n)
    assert abs(L - np.sum(E * E)) < 1e-10 * L
    gP = 2 * S.T @ E @ A @ W.T                                   # dL/dP
    # P = A0 (x) A2 : dL/dA0[i, a] = sum_{j, b} gP[i*4 + j, a*2 + b] A2[j, b]
    gP4 = gP.reshape(5, 3, 2, 2)
    g0 = np.einsum("ijab,jb->ia", gP4, facs[2])
    g2 = np.einsum("ijab,ia->jb", gP4, facs[0])
    np.testing.assert_allclose(grads[0], g0, atol=1e-10)
    np.testing.assert_allclose(grads[2], g2, atol=1e-10)
    np.testing.assert_allclose(grads[1], 2 * E.T @ S @ P @ W, atol=1e-10)


def test_rsvd_driver_equals_exact_when_test_matrix_spans():
    """RSVD-LRLS (Alg. 5) with as many Gaussian columns as Z has (k = r): C = X Omega
    spans the whole row space of X = Z^+ Y almost surely, so Q Q^T X = X and the
    randomized solve returns the exact truncated SVD; the sweeps then coincide with
    the exact solve.  With few columns on a noisy tensor they must differ."""
    X = workloads.tucker_dense((12, 11, 10), (3, 3, 3), noise=0.05, seed=8)
    T = sketch.Tensor.from_dense(X)
    ranks, m = (3, 3, 3), 60
    ex = tucker.sketch_tucker_als(T, ranks, m, 3, seed=4)
    rs = tucker.sketch_tucker_als(T, ranks, m, 3, seed=4, solve_kind="rsvd", rsvd_p=100)
    np.testing.assert_allclose(rs["fits"], ex["fits"], rtol=0, atol=1e-12)
    lo = tucker.sketch_tucker_als(T, ranks, m, 3, seed=4, solve_kind="rsvd", rsvd_p=0)
    assert abs(lo["fits"][-1] - ex["fits"][-1]) > 1e-9


def test_rsvd_omega_stream():
    """The test matrix is the (seed, RSVD, sweep, n) Gaussian stream, row-major."""
    Om = tucker.rsvd_omega(7, 2, 1, 5, 3)
    key = rng.stream_key(7, rng.P_RSVD, 2, 1)
    np.testing.assert_array_equal(Om.reshape(-1), rng.gauss(key, np.arange(15)))
    assert tucker.rsvd_width(10, 100) == 20 and tucker.rsvd_width(5, 9) == 9


def test_driver_resumes_at_a_sweep():
    """Two sweeps in one run equal one sweep followed by a run resumed at sweep 1
    from its factors (the per-sweep streams are keyed by the absolute sweep)."""
    X = workloads.tucker_dense((14, 13, 12), (3, 3, 3), 0.05, seed=4)
    T = sketch.Tensor.from_dense(X)
    for kind, solve_kind in (("ts", "rsvd"), ("lev", "exact")):
        full = tucker.sketch_tucker_als(T, (3, 3, 3), 60, 2, seed=5, sketch_kind=kind,
                                        solve_kind=solve_kind)
        one = tucker.sketch_tucker_als(T, (3, 3, 3), 60, 1, seed=5, sketch_kind=kind,
                                       solve_kind=solve_kind)
        rest = tucker.sketch_tucker_als(T, (3, 3, 3), 60, 1, seed=5, sketch_kind=kind,
                                        solve_kind=solve_kind, init="user",
                                        init_factors=one["factors"], first_sweep=1)
        assert full["fits"][1] == rest["fits"][0]
        for a, b in zip(full["factors"], rest["factors"]):
            assert np.array_equal(a, b)


# ----------------------------------------------------------------------------
# HOSVD, random initialisation, COO semantics, CP fit on COO tensors
# ----------------------------------------------------------------------------
def _exact_tucker(dims, ranks, seed):
    """C x_1 Q1 ... x_N QN with orthonormal Q_n and a core whose mode-n
    unfoldings have well separated singular values (a diagonal-dominant core)."""
    rs = np.random.default_rng(seed)
    Qs = [np.linalg.qr(rs.standard_normal((s, R)))[0] for s, R in zip(dims, ranks)]
    C = 0.05 * rs.standard_normal(ranks)
    for t in range(min(ranks)):
        C[(t,) * len(ranks)] = 10.0 * 0.5 ** t     # singular values 10, 5, 2.5, ...
    X = C
    for k, Q in enumerate(Qs):
        X = np.moveaxis(np.tensordot(Q, X, axes=(1, k)), 0, k)
    return X, Qs


def test_hosvd_left_singular_vectors_of_unfoldings():
    """HOSVD (Sec. 2.2, the initialisation of Alg. 1 and of the CP step of Alg. 6):
    A^(n) spans the column space of X_(n) and its columns are the left singular
    vectors in order of decreasing singular value.  Checked through the
    eigen-decomposition of X_(n) X_(n)^T (a different LAPACK route), and on an
    exact Tucker tensor whose factors are known."""
    dims, ranks = (9, 7, 5), (3, 3, 2)
    X, Qs = _exact_tucker(dims, ranks, 11)
    A = tucker.hosvd(X, ranks)
    for n in range(3):
        assert A[n].shape == (dims[n], ranks[n])               # left, not right, vectors
        np.testing.assert_allclose(A[n].T @ A[n], np.eye(ranks[n]), atol=1e-13)
        # exact column space of the known factor
        cos = np.linalg.svd(A[n].T @ Qs[n], compute_uv=False)
        np.testing.assert_allclose(cos, 1.0, atol=1e-12)
        # eigenvectors of X_(n) X_(n)^T, descending, sign rule applied by hand
        M = tucker.unfold(X, n)
        lam, V = np.linalg.eigh(M @ M.T)
        V = V[:, ::-1][:, :ranks[n]]
        for c in range(ranks[n]):
            p = int(np.argmax(np.abs(V[:, c])))
            V[:, c] *= np.sign(V[p, c])
        np.testing.assert_allclose(A[n], V, atol=1e-10)
        # column c carries the c-th largest singular value
        norms = np.linalg.norm(M.T @ A[n], axis=0)
        np.testing.assert_allclose(norms, np.sqrt(lam[::-1][:ranks[n]]), rtol=1e-12)
        assert np.all(np.diff(norms) < 0)


def test_hosvd_catches_transposed_or_unsorted_variants():
    """A right-singular-vector or unsorted variant of the HOSVD fails the checks
    above (the test would catch the plausible mistakes)."""
    dims, ranks = (9, 7, 5), (3, 3, 2)
    X, Qs = _exact_tucker(dims, ranks, 12)
    M = tucker.unfold(X, 0)
    _, _, Vt = np.linalg.svd(M, full_matrices=False)
    assert Vt[:3].T.shape != (dims[0], ranks[0])               # right vectors: wrong shape
    U = np.linalg.svd(M, full_matrices=False)[0][:, :3]
    norms = np.linalg.norm(M.T @ U[:, ::-1], axis=0)
    assert not np.all(np.diff(norms) < 0)                      # reversed order detected


def test_init_random_orthonormal_signed_gaussian_span():
    """Random initialisation (Gaussian then QR, reading of the paper's random
    start): orthonormal columns, the sign rule, and the column space of the
    (seed, INIT, n) Gaussian draw."""
    s, R, n, seed = 23, 4, 2, 9
    A = tucker.init_random(s, R, n, seed)
    np.testing.assert_allclose(A.T @ A, np.eye(R), atol=1e-14)
    for c in range(R):
        p = int(np.argmax(np.abs(A[:, c])))
        assert A[p, c] > 0
        assert np.all(np.abs(A[:, c]) <= A[p, c])
    G = rng.gauss(rng.stream_key(seed, rng.P_INIT, n), np.arange(s * R)).reshape(s, R)
    np.testing.assert_allclose(A @ (A.T @ G), G, atol=1e-12)   # same column space
    # Gram-Schmidt order: the first column is the normalised first Gaussian column
    g0 = G[:, 0] / np.linalg.norm(G[:, 0])
    assert abs(abs(A[:, 0] @ g0) - 1.0) < 1e-14
    # different n or seed: a different draw
    assert not np.allclose(A, tucker.init_random(s, R, n + 1, seed))


def test_coalesced_sums_duplicates_hand_worked():
    """COO semantics (duplicates add): a hand-worked example."""
    idx = np.array([[1, 0, 2], [0, 1, 1], [1, 0, 2], [2, 2, 0], [0, 1, 1], [1, 0, 2]])
    val = np.array([1.0, 2.0, 10.0, -3.0, 0.5, 100.0])
    T = sketch.Tensor((3, 3, 3), idx, val)
    c = T.coalesced()
    got = {tuple(int(x) for x in i): v for i, v in zip(c.idx, c.val)}
    assert got == {(0, 1, 1): 2.5, (1, 0, 2): 111.0, (2, 2, 0): -3.0}
    assert T.norm2() == 2.5 ** 2 + 111.0 ** 2 + 9.0
    D = T.to_dense()
    assert D[1, 0, 2] == 111.0 and D[0, 1, 1] == 2.5 and np.count_nonzero(D) == 3


def test_cp_relative_residual_coo_equals_dense():
    """CP fit (Sec. 7): the COO formula ||T||^2 - 2<T, T~> + ||T~||^2 equals the
    dense definition on a tensor stored with duplicate coordinates."""
    rs = np.random.default_rng(13)
    dims, R = (6, 5, 4), 3
    idx = np.stack([rs.integers(0, d, 80) for d in dims], axis=1)
    idx = np.concatenate([idx, idx[:25]])                      # 25 duplicates
    val = rs.standard_normal(idx.shape[0])
    Tcoo = sketch.Tensor(dims, idx, val)
    D = np.zeros(dims)
    for i, v in zip(idx, val):                                 # plain loop, duplicates add
        D[tuple(i)] += v
    Td = sketch.Tensor.from_dense(D)
    facs = [rs.standard_normal((d, R)) for d in dims]
    want = np.linalg.norm(D - cp.cp_reconstruct(facs)) / np.linalg.norm(D)
    assert abs(cp.cp_relative_residual(Tcoo, facs) - want) < 1e-12
    assert abs(cp.cp_relative_residual(Td, facs) - want) < 1e-12
    # the exact CP tensor stored as COO with split duplicates has residual 0
    Dx = cp.cp_reconstruct(facs)
    full = np.stack(np.unravel_index(np.arange(Dx.size), dims), axis=1)
    halves = sketch.Tensor(dims, np.concatenate([full, full]),
                           np.concatenate([0.25 * Dx.reshape(-1), 0.75 * Dx.reshape(-1)]))
    assert cp.cp_relative_residual(halves, facs) < 1e-7
