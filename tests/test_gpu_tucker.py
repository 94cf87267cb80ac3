"""End-to-end GPU parity of Sketch-Tucker-ALS (Alg. 4) and CP-Sketch-Tucker
(Alg. 6) against the FP64 oracle on the same seeded inputs.

Tolerances on the relative residual after every sweep: 1e-10 for the FP64
path, 1e-5 for FP32 operands; BF16 operands are reported against FP32 with a
proposed 1e-3 bound.  Factors are compared after the sign rule when the
spectral gap allows (it does for these inputs)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import cp as ocp, sketch as osk, tucker as otk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tsk():
    import paper_2104_01101_amd as t
    t.lib()
    return t


def _dense(tsk, X):
    return tsk.Tensor.dense(torch.from_numpy(np.ascontiguousarray(X)).to(DEV))


def _coo(tsk, dims, idx, val):
    return tsk.Tensor.coo(torch.from_numpy(idx).to(DEV), torch.from_numpy(val).to(DEV), dims)


def test_dense40_fp64_parity(tsk):
    """Small dense case: 40^3 FP64, Tucker rank 5 + 1% noise, TensorSketch m = 200,
    RRF init, 5 sweeps."""
    w = workloads.dense40()
    T = _dense(tsk, w.dense)
    core, factors, fits = tsk.tucker_sketch_als(T, w.ranks, w.m, w.sweeps, prec="f64", seed=0)
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(w.dense), w.ranks, w.m, w.sweeps, seed=0)
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=1e-10)
    for F, Fo in zip(factors, ref["factors"]):
        np.testing.assert_allclose(F.cpu().numpy(), Fo, atol=1e-8)
    np.testing.assert_allclose(core.cpu().numpy(), ref["core"], atol=1e-8 * np.abs(ref["core"]).max())


def test_dense40_deterministic(tsk):
    w = workloads.dense40()
    T = _dense(tsk, w.dense)
    a = tsk.tucker_sketch_als(T, w.ranks, w.m, 3, prec="f64", seed=4)
    b = tsk.tucker_sketch_als(T, w.ranks, w.m, 3, prec="f64", seed=4)
    assert torch.equal(a[0], b[0]) and all(torch.equal(x, y) for x, y in zip(a[1], b[1]))
    assert a[2] == b[2]


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-10)])
def test_sparse_small_parity(tsk, prec, tol):
    """Sparse workload family at reduced size: sparse 300^3, 50k distinct uniform
    coordinates, Tucker signal + N(0,1), TensorSketch m = 16 R^2."""
    dims, R = (300, 300, 300), 6
    idx, val = workloads.sparse_tucker(dims, 50_000, (R, R, R), seed=1)
    val = val.astype(np.float32 if prec == "f32" else np.float64)
    T = _coo(tsk, dims, idx, val)
    m = 16 * R * R
    _, factors, fits = tsk.tucker_sketch_als(T, (R, R, R), m, 4, prec=prec, seed=1)
    ref = otk.sketch_tucker_als(osk.Tensor(dims, idx, val.astype(np.float64)), (R, R, R), m, 4, seed=1)
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=tol)


def test_exact_low_rank_recovered(tsk):
    X = workloads.tucker_dense((30, 28, 26), (4, 4, 4), noise=0.0, seed=3)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        _, _, fits = tsk.tucker_sketch_als(_dense(tsk, X), (4, 4, 4), 8 * 16, 1, prec=prec)
        assert fits[-1] < tol


def test_random_init_parity(tsk):
    w = workloads.dense40()
    _, _, fits = tsk.tucker_sketch_als(_dense(tsk, w.dense), w.ranks, w.m, 3, init="random",
                                      prec="f64", seed=2)
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(w.dense), w.ranks, w.m, 3, seed=2,
                                init="random")
    np.testing.assert_allclose(fits, ref["fits"], atol=1e-10)


def test_leverage_dense_order4_fp64(tsk):
    """Order-4 dense family at reduced size: dense 24^4, rank 3, leverage m = 4000
    scaled to 400 rows."""
    X = workloads.tucker_dense((24, 24, 24, 24), (3, 3, 3, 3), noise=0.01, seed=2)
    ranks, m = (3, 3, 3, 3), 400
    _, factors, fits = tsk.tucker_sketch_als(_dense(tsk, X), ranks, m, 3, sketch="lev",
                                             prec="f64", seed=6)
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(X), ranks, m, 3, seed=6, sketch_kind="lev")
    np.testing.assert_allclose(fits, ref["fits"], atol=1e-10)


def test_leverage_bf16_vs_f32(tsk):
    X = workloads.tucker_dense((40, 40, 40, 40), (4, 4, 4, 4), noise=0.01, seed=7,
                               dtype=np.float32)
    ranks, m = (4, 4, 4, 4), 4 * 64
    T = _dense(tsk, X)
    _, _, f32 = tsk.tucker_sketch_als(T, ranks, m, 3, sketch="lev", prec="f32", seed=1)
    _, _, bf = tsk.tucker_sketch_als(T, ranks, m, 3, sketch="lev", prec="bf16", seed=1)
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(X.astype(np.float64)), ranks, m, 3, seed=1,
                                sketch_kind="lev")
    print("lev fits f32", f32, "bf16", bf, "oracle", ref["fits"])
    assert abs(f32[-1] - ref["fits"][-1]) < 1e-3
    assert abs(bf[-1] - f32[-1]) < 1e-3


def test_cp_via_tucker_fp64(tsk):
    """Collinear CP family at reduced size: dense 40^3, CP rank 4 with
    collinearity 0.9 + 1% noise; Tucker rank 6 by leverage sampling; CP-ALS on the
    core."""
    X, _ = workloads.cp_collinear((40, 40, 40), 4, 0.9, 0.01, seed=3, dtype=np.float64)
    T = _dense(tsk, X)
    facs, fit = tsk.cp_via_tucker(T, 4, (6, 6, 6), m=16 * 36, tucker_sweeps=3, cp_sweeps=25,
                                  sketch="lev", prec="f64", seed=2)
    ref = ocp.cp_sketch_tucker(osk.Tensor.from_dense(X), 4, (6, 6, 6), 16 * 36, 3, 25, seed=2,
                               sketch_kind="lev")
    assert abs(fit - ref["fit"]) < 1e-8
    for F, Fo in zip(facs, ref["factors"]):
        np.testing.assert_allclose(F.cpu().numpy(), Fo, atol=1e-6 * np.abs(Fo).max())


@pytest.mark.parametrize("prec,solve,tol", [("f64", "exact", 1e-10), ("f32", "exact", 1e-5),
                                             ("f64", "rsvd", 1e-10)])
def test_sparse_leverage_parity(tsk, prec, solve, tol):
    """Leverage-score sampling of a COO tensor through the per-mode fibre indices:
    80 x 70 x 60 with 100k distinct uniform coordinates (30 % of the entries),
    Tucker (5, 4, 3) signal + N(0, 0.1^2), m = 400 samples per subproblem, RRF
    init, 4 sweeps, against the oracle's sampled fibres of the coalesced tensor."""
    dims, ranks, m = (80, 70, 60), (5, 4, 3), 400
    idx, val = workloads.sparse_tucker(dims, 100_000, ranks, seed=4, noise_std=0.1)
    val = val.astype(np.float32 if prec == "f32" else np.float64)
    T = _coo(tsk, dims, idx, val)
    _, factors, fits = tsk.tucker_sketch_als(T, ranks, m, 4, sketch="lev", prec=prec, seed=3,
                                             solve=solve)
    ref = otk.sketch_tucker_als(osk.Tensor(dims, idx, val.astype(np.float64)), ranks, m, 4,
                                seed=3, sketch_kind="lev", solve_kind=solve)
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=tol)
    if prec == "f64":
        for F, Fo in zip(factors, ref["factors"]):
            np.testing.assert_allclose(F.cpu().numpy(), Fo, atol=1e-8)


def test_lev_det_order4_dense_parity(tsk):
    """Deterministic selection with three other modes (candidate tuples of three
    levels): dense 16 x 14 x 12 x 10, Tucker (3,3,2,2) + 5 % noise, m = 8 r_max.
    At m = 4 r_max the kept rows of the last mode leave Z numerically singular
    (condition 6e15), and both sides then solve an ill-posed problem; at 8 r_max
    the condition number of every sketch stays below 2.3."""
    ranks = (3, 3, 2, 2)
    X = workloads.tucker_dense((16, 14, 12, 10), ranks, 0.05, seed=6)
    m = 8 * 18
    _, factors, fits = tsk.tucker_sketch_als(_dense(tsk, X), ranks, m, 3, sketch="lev_det",
                                             prec="f64", seed=2)
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(X), ranks, m, 3, seed=2,
                                sketch_kind="lev_det")
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=1e-10)


def test_sparse_leverage_order4_fp32(tsk):
    """Leverage sampling of an order-4 COO tensor (fibre keys over three other
    modes): 30 x 25 x 20 x 15 with 40k entries, FP32 operands."""
    dims, ranks = (30, 25, 20, 15), (3, 3, 2, 2)
    idx, val = workloads.sparse_tucker(dims, 40_000, ranks, seed=7, noise_std=0.1)
    T = _coo(tsk, dims, idx, val)
    m = 16 * 18
    _, _, fits = tsk.tucker_sketch_als(T, ranks, m, 3, sketch="lev", prec="f32", seed=4)
    ref = otk.sketch_tucker_als(osk.Tensor(dims, idx, val.astype(np.float64)), ranks, m, 3,
                                seed=4, sketch_kind="lev")
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=1e-5)


def test_sparse_leverage_dense_equivalent(tsk):
    """The same small tensor stored densely and as COO (every entry, shuffled)
    gives the same leverage run: the fibre index changes the access, not the sketch.
    Random init (independent of T) keeps the range finder's layout-dependent
    summation order out of the comparison, so the factors agree bit for bit."""
    X = workloads.tucker_dense((24, 22, 20), (3, 3, 3), 0.05, seed=8)
    dims = X.shape
    To = osk.Tensor.from_dense(X)
    perm = np.random.default_rng(0).permutation(To.val.size)
    idx, val = To.idx[perm].astype(np.int32), To.val[perm].copy()
    a = tsk.tucker_sketch_als(_dense(tsk, X), (3, 3, 3), 200, 3, sketch="lev", init="random",
                              prec="f64", seed=9)
    b = tsk.tucker_sketch_als(_coo(tsk, dims, idx, val), (3, 3, 3), 200, 3, sketch="lev",
                              init="random", prec="f64", seed=9)
    for F, G in zip(a[1], b[1]):
        assert torch.equal(F, G)
    np.testing.assert_allclose(a[2], b[2], rtol=0, atol=1e-13)


@pytest.mark.parametrize("sparse,solve", [(False, "exact"), (True, "exact"), (True, "rsvd")])
def test_lev_det_parity(tsk, sparse, solve):
    """Deterministic leverage selection (the m rows of largest Kronecker score,
    weights 1) in the driver, FP64, against the oracle's brute-force selection:
    dense 30 x 28 x 26 (Tucker (3,3,3) + 5 % noise) or the 80 x 70 x 60 COO tensor
    with 100k entries; m = 16 R^2 rows per subproblem, RRF init, 3 sweeps."""
    if sparse:
        dims, ranks = (80, 70, 60), (5, 4, 3)
        idx, val = workloads.sparse_tucker(dims, 100_000, ranks, seed=4, noise_std=0.1)
        val = val.astype(np.float64)
        T, To = _coo(tsk, dims, idx, val), osk.Tensor(dims, idx, val)
    else:
        ranks = (3, 3, 3)
        X = workloads.tucker_dense((30, 28, 26), ranks, 0.05, seed=2)
        T, To = _dense(tsk, X), osk.Tensor.from_dense(X)
    m = 16 * max(ranks) ** 2
    _, factors, fits = tsk.tucker_sketch_als(T, ranks, m, 3, sketch="lev_det", prec="f64",
                                             seed=5, solve=solve)
    ref = otk.sketch_tucker_als(To, ranks, m, 3, seed=5, sketch_kind="lev_det",
                                solve_kind=solve)
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=1e-10)
    for F, Fo in zip(factors, ref["factors"]):
        np.testing.assert_allclose(F.cpu().numpy(), Fo, atol=1e-8)


# -------------------------------------------- RSVD-LRLS subproblem solver ----
def test_dense40_rsvd_fp64_parity(tsk):
    """The small dense case with the paper's subproblem solver (Alg. 4 calls RSVD-LRLS,
    Alg. 5): same Gaussian test matrices on both sides, relative residuals after
    every sweep within 1e-10, factors within 1e-8."""
    w = workloads.dense40()
    T = _dense(tsk, w.dense)
    core, factors, fits = tsk.tucker_sketch_als(T, w.ranks, w.m, w.sweeps, prec="f64", seed=0,
                                                solve="rsvd")
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(w.dense), w.ranks, w.m, w.sweeps, seed=0,
                                solve_kind="rsvd")
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=1e-10)
    for F, Fo in zip(factors, ref["factors"]):
        np.testing.assert_allclose(F.cpu().numpy(), Fo, atol=1e-8)


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-10)])
def test_sparse_small_rsvd_parity(tsk, prec, tol):
    dims, R = (300, 300, 300), 6
    idx, val = workloads.sparse_tucker(dims, 50_000, (R, R, R), seed=1)
    val = val.astype(np.float32 if prec == "f32" else np.float64)
    T = _coo(tsk, dims, idx, val)
    m = 16 * R * R
    _, _, fits = tsk.tucker_sketch_als(T, (R, R, R), m, 4, prec=prec, seed=1, solve="rsvd")
    ref = otk.sketch_tucker_als(osk.Tensor(dims, idx, val.astype(np.float64)), (R, R, R), m, 4,
                                seed=1, solve_kind="rsvd")
    np.testing.assert_allclose(fits, ref["fits"], rtol=0, atol=tol)


def test_rsvd_exact_low_rank_recovered(tsk):
    X = workloads.tucker_dense((30, 28, 26), (4, 4, 4), noise=0.0, seed=3)
    _, _, fits = tsk.tucker_sketch_als(_dense(tsk, X), (4, 4, 4), 8 * 16, 1, prec="f64",
                                       solve="rsvd")
    assert fits[-1] < 1e-12


@pytest.mark.parametrize("kind,solve", [("ts", "rsvd"), ("lev", "exact")])
def test_resume_at_a_sweep_bitwise(tsk, kind, solve):
    """first_sweep (checkpoint / resume of the sweep loop of Alg. 4): two sweeps in
    one call equal one sweep followed by a call resumed at sweep 1 from its
    factors, bit for bit (the per-sweep streams are keyed by the absolute sweep),
    and the resumed call matches the oracle resumed the same way."""
    X = workloads.tucker_dense((14, 13, 12), (3, 3, 3), 0.05, seed=4)
    T = _dense(tsk, X)
    kw = dict(sketch=kind, prec="f64", seed=5, solve=solve)
    full = tsk.tucker_sketch_als(T, (3, 3, 3), 60, 2, **kw)
    one = tsk.tucker_sketch_als(T, (3, 3, 3), 60, 1, **kw)
    init = [F.clone() for F in one[1]]
    rest = tsk.tucker_sketch_als(T, (3, 3, 3), 60, 1, init="user", init_factors=init,
                                 first_sweep=1, **kw)
    assert rest[2][0] == full[2][1]
    assert all(torch.equal(a, b) for a, b in zip(full[1], rest[1]))
    assert torch.equal(full[0], rest[0])
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(X), (3, 3, 3), 60, 2, seed=5,
                                sketch_kind=kind, solve_kind=solve)
    np.testing.assert_allclose(rest[2], ref["fits"][1:], rtol=0, atol=1e-10)


def test_tolerance_stops_and_final_fit(tsk):
    """tol: the loop stops after the first sweep whose residual moved by less than
    tol (the oracle's residual sequence says where); FINAL_FIT evaluates only the
    last sweep and equals the per-sweep record there."""
    w = workloads.dense40()
    T = _dense(tsk, w.dense)
    ref = otk.sketch_tucker_als(osk.Tensor.from_dense(w.dense), w.ranks, w.m, 8, seed=0)
    d = np.abs(np.diff(ref["fits"]))
    tol = 1e-12                          # d = 2.3e-7, 4.2e-11, 2.8e-15, ...: stop after sweep 4
    expect = 1 + next(i for i in range(1, len(ref["fits"])) if d[i - 1] < tol)
    assert expect == 4 and d[1] > 10 * tol and d[2] < tol / 100
    plan = tsk.TuckerPlan(T, w.ranks, w.m, 8, prec="f64", seed=0, tol=tol)
    _, _, fits = plan.run()
    assert plan.sweeps_done == expect and len(fits) == expect
    np.testing.assert_allclose(fits, ref["fits"][:expect], rtol=0, atol=1e-10)
    _, _, every = tsk.tucker_sketch_als(T, w.ranks, w.m, 4, prec="f64", seed=0)
    _, _, last = tsk.tucker_sketch_als(T, w.ranks, w.m, 4, prec="f64", seed=0,
                                       record_fit="final")
    assert all(np.isnan(last[:3])) and last[3] == every[3]
