"""GPU parity of each step of the hot path against the FP64 oracle, through the
C ABI.  Integer outputs (hash maps, signs, sampled indices) must be bit-exact;
FP64 outputs that are sums in a fixed order must match to the stated rounding
bound; FP32/BF16 outputs within their precision's bound."""
import json
import os

import numpy as np
import pytest
import torch

import workloads
from oracle import sketch as osk, solve as osv, tucker as otk, adjoint as oadj

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def tsk():
    import paper_2104_01101_amd as t
    t.lib()  # fail loudly if the library is missing
    return t


def _gpu_tensor(tsk, dims, idx=None, val=None, dense=None):
    if dense is not None:
        return tsk.Tensor.dense(torch.from_numpy(np.ascontiguousarray(dense)).to(DEV))
    return tsk.Tensor.coo(torch.from_numpy(idx).to(DEV), torch.from_numpy(val).to(DEV), dims)


def _maps(dims, n, m, seed):
    """The oracle's TensorSketch maps of subproblem n ({k: (h, sigma)}), and the
    same maps as device tensors (int32 h, int8 sigma) handed to the library."""
    tabs = osk.ts_tables(dims, m, seed, n)
    h = [None if k == n else torch.from_numpy(tabs[k][0].astype(np.int32)).to(DEV)
         for k in range(len(dims))]
    s = [None if k == n else torch.from_numpy(tabs[k][1].astype(np.int8)).to(DEV)
         for k in range(len(dims))]
    return tabs, h, s


# ---------------------------------------------------------------- a1 ----
@pytest.mark.parametrize("dims,m,n,seed", [((40, 40, 40), 200, 0, 0), ((2000, 37, 5), 1600, 1, 3),
                                           ((7, 9, 11, 13), 2048, 3, 11), ((10000, 3), 2048, 0, 0)])
def test_hash_tables_bit_exact(tsk, dims, m, n, seed):
    h, s = tsk.hash_tables(dims, n, m, seed, DEV)
    ref = osk.ts_tables(dims, m, seed, n)
    for k, (hr, sr) in ref.items():
        assert np.array_equal(h[k].cpu().numpy().astype(np.int64), hr)
        assert np.array_equal(s[k].cpu().numpy().astype(np.float64), sr)


# ---------------------------------------------------------------- a2 ----
def test_sketch_rhs_golden(tsk):
    d = json.load(open(os.path.join(GOLDEN, "ts_worked_example.json")))
    dims, m, n = tuple(d["dims"]), d["m"], d["n"]
    X = np.fromfunction(lambda a, b, c: 1 + 6 * a + 2 * b + c, dims)
    T = _gpu_tensor(tsk, dims, dense=X)
    h = [None] + [torch.tensor(d["h"][str(k)], dtype=torch.int32, device=DEV) for k in (1, 2)]
    s = [None] + [torch.tensor(d["sigma"][str(k)], dtype=torch.int8, device=DEV) for k in (1, 2)]
    Y = tsk.sketch_rhs_ts(T, n, m, h, s)
    assert np.array_equal(Y.cpu().numpy(), np.array(d["Y"]))


@pytest.mark.parametrize("dims,nnz,m,n", [((40, 40, 40), 0, 200, 0),          # dense
                                          ((300, 200, 100), 50_000, 1600, 1),
                                          ((30, 20, 10, 7), 9_000, 97, 2),    # ragged, prime m
                                          ((5000, 6, 4), 20_000, 64, 0),      # wide rows: tiles split columns
                                          ((50, 50, 50), 1, 16, 2)])
def test_sketch_rhs_fp64_bitwise(tsk, dims, nnz, m, n):
    """FP64 cells are the in-order sum of their entries, exactly as the oracle's
    sequential bincount: bitwise equal."""
    rs = np.random.default_rng(nnz + m)
    if nnz == 0:
        X = rs.standard_normal(dims)
        T = _gpu_tensor(tsk, dims, dense=X)
        To = osk.Tensor.from_dense(X)
    else:
        idx = np.stack([rs.integers(0, d, nnz) for d in dims], 1).astype(np.int32)
        idx[nnz // 2:nnz // 2 + min(100, nnz // 4)] = idx[:min(100, nnz // 4)]  # duplicates
        val = rs.standard_normal(nnz)
        T = _gpu_tensor(tsk, dims, idx, val)
        To = osk.Tensor(dims, idx, val)
    tabs, h, s = _maps(dims, n, m, 5)
    Y = tsk.sketch_rhs_ts(T, n, m, h, s).cpu().numpy()
    Yo = osk.ts_rhs(To, m, tabs, n)
    assert np.array_equal(Y, Yo)


def test_sketch_rhs_fp32_bound_and_determinism(tsk):
    dims, nnz, m, n = (2000, 2000, 2000), 200_000, 1600, 2
    w = workloads.sparse_tucker(dims, nnz, (10, 10, 10), seed=2)
    idx, val = w
    T = _gpu_tensor(tsk, dims, idx, val)
    tabs, h, s = _maps(dims, n, m, 0)
    Y1 = tsk.sketch_rhs_ts(T, n, m, h, s)
    Y2 = tsk.sketch_rhs_ts(T, n, m, h, s)
    assert torch.equal(Y1, Y2)
    To = osk.Tensor(dims, idx, val.astype(np.float64))
    Yo = osk.ts_rhs(To, m, tabs, n)
    H, S = osk.ts_hash_sign(tabs, To.idx, m)
    key = H * dims[n] + To.idx[:, n]
    absum = np.bincount(key, weights=np.abs(To.val), minlength=m * dims[n]).reshape(m, -1)
    cnt = np.bincount(key, minlength=m * dims[n]).reshape(m, -1)
    bound = (cnt + 2) * 2.0 ** -24 * absum
    assert np.all(np.abs(Y1.cpu().numpy().astype(np.float64) - Yo) <= bound + 1e-30)


def test_sketch_rhs_empty_tensor(tsk):
    dims = (10, 20, 30)
    T = tsk.Tensor.coo([torch.zeros(0, dtype=torch.int32, device=DEV)] * 3,
                       torch.zeros(0, dtype=torch.float32, device=DEV), dims)
    h, s = tsk.hash_tables(dims, 1, 50, 0, DEV)
    Y = tsk.sketch_rhs_ts(T, 1, 50, h, s)
    assert Y.shape == (50, 20) and torch.count_nonzero(Y) == 0


# ------------------------------------------------------------- a3, a4 ----
@pytest.mark.parametrize("dims,ranks,m,n", [((40, 40, 40), (5, 5, 5), 200, 0),
                                            ((2000, 300, 200), (10, 10, 10), 1600, 1),
                                            ((500, 400, 300), (16, 16, 16), 2048, 2),
                                            ((30, 20, 10, 12), (3, 4, 2, 5), 77, 3),
                                            ((9, 8, 7), (2, 3, 3), 7, 0),
                                            ((9, 8, 7), (2, 1, 1), 1, 0)])
def test_sketch_lhs_matches_convolution(tsk, dims, ranks, m, n):
    rs = np.random.default_rng(m)
    facs = [np.linalg.qr(rs.standard_normal((d, r)))[0] for d, r in zip(dims, ranks)]
    fg = [torch.from_numpy(F).to(DEV) for F in facs]
    tabs, h, s = _maps(dims, n, m, 1)
    Zo = osk.ts_lhs(facs, tabs, m, n)
    scale = np.abs(Zo).max() + 1e-300
    Z = tsk.sketch_lhs_ts(dims, ranks, n, m, h, s, fg, "f64").cpu().numpy()
    assert np.abs(Z - Zo).max() <= 1e-13 * scale * np.log2(m + 1)
    Z32 = tsk.sketch_lhs_ts(dims, ranks, n, m, h, s, fg, "f32").cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Z32 - Zo) <= 2.0 ** -24 * np.abs(Zo) + 1e-13 * scale * np.log2(m + 1))
    Zb = tsk.sketch_lhs_ts(dims, ranks, n, m, h, s, fg, "bf16").float().cpu().numpy()
    assert np.all(np.abs(Zb - Zo) <= 2.0 ** -8 * np.abs(Zo) + 1e-7 * scale)


# ---------------------------------------------------------------- a6, a7 ----
@pytest.mark.parametrize("m,r,s,R", [(200, 25, 40, 5), (1600, 100, 2000, 10), (400, 30, 20, 4),
                                     (333, 64, 65, 7), (4000, 100, 200, 10), (90, 90, 1, 1),
                                     (700, 121, 150, 6), (800, 128, 150, 8)])
def test_rc_solve_fp64(tsk, m, r, s, R):
    rs = np.random.default_rng(r * s)
    Z = rs.standard_normal((m, r)) / np.sqrt(m)
    Y = Z @ rs.standard_normal((r, R)) @ rs.standard_normal((R, s)) + 0.1 * rs.standard_normal((m, s))
    A, W = tsk.rc_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R)
    Ao, Wo, Xo = osv.rc_solve(Z, Y, R)
    A, W = A.cpu().numpy(), W.cpu().numpy()
    np.testing.assert_allclose(A, Ao, atol=1e-10 * max(1, np.abs(Ao).max()))
    np.testing.assert_allclose(W, Wo, atol=1e-10 * max(1, np.abs(Wo).max()))
    np.testing.assert_allclose(A.T @ A, np.eye(R), atol=1e-13)


@pytest.mark.parametrize("prec,tol", [("f32", 1e-4), ("bf16", 3e-2)])
def test_rc_solve_low_precision(tsk, prec, tol):
    m, r, s, R = 1600, 100, 300, 10
    rs = np.random.default_rng(3)
    Z = rs.standard_normal((m, r)) / np.sqrt(m)
    Y = Z @ (10 * rs.standard_normal((r, R))) @ rs.standard_normal((R, s)) + 0.1 * rs.standard_normal((m, s))
    dt = {"f32": torch.float32, "bf16": torch.bfloat16}[prec]
    Zc, Yc = torch.from_numpy(Z).to(dt), torch.from_numpy(Y).to(dt)  # rounded on the host
    A, W = tsk.rc_solve(Zc.to(DEV), Yc.to(DEV), R, prec)
    # oracle on the rounded operands: the only difference left is the accumulation
    Ao, Wo, _ = osv.rc_solve(Zc.double().numpy(), Yc.double().numpy(), R)
    A = A.cpu().numpy()
    assert np.abs(A @ A.T - Ao @ Ao.T).max() < tol


# ---------------------------------------------------------------- a9 ----
def test_rrf_init_matches_oracle(tsk):
    w = workloads.dense40()
    T = _gpu_tensor(tsk, w.dims, dense=w.dense)
    To = osk.Tensor.from_dense(w.dense)
    for n in (1, 2):
        A = tsk.rrf_init(T, n, 5, 15, 40, 0).cpu().numpy()
        Ao = otk.init_rrf(To, n, 5, 15, 40, 0)
        np.testing.assert_allclose(A, Ao, atol=1e-10)


def test_rrf_init_sparse_fp32(tsk):
    dims = (300, 250, 200)
    idx, val = workloads.sparse_tucker(dims, 40_000, (6, 6, 6), seed=4)
    T = _gpu_tensor(tsk, dims, idx, val)
    To = osk.Tensor(dims, idx, val.astype(np.float64))
    A = tsk.rrf_init(T, 1, 6, 30, 66, 9).cpu().numpy()
    Ao = otk.init_rrf(To, 1, 6, 30, 66, 9)
    assert np.abs(A @ A.T - Ao @ Ao.T).max() < 1e-4


# ---------------------------------------------------------------- a5 ----
@pytest.mark.parametrize("dims,ranks,m,n", [((200, 200, 200, 200), (10, 10, 10, 10), 4000, 1),
                                            ((500, 500, 500), (30, 30, 30), 14400, 0),
                                            ((40, 40, 40), (5, 5, 5), 200, 2),
                                            # cdfs beyond the LDS staging budget
                                            ((9000, 3000, 50), (4, 4, 4), 300, 2)])
def test_leverage_sample_bit_exact(tsk, dims, ranks, m, n):
    rs = np.random.default_rng(sum(dims))
    facs = [np.linalg.qr(rs.standard_normal((d, r)))[0] for d, r in zip(dims, ranks)]
    fg = [torch.from_numpy(F).to(DEV) for F in facs]
    idx, w = tsk.leverage_sample(dims, ranks, n, m, 3, 2, fg)
    io, wo = osk.leverage_sample(facs, m, 3, 2, n)
    assert np.array_equal(idx.cpu().numpy().astype(np.int64), io)
    np.testing.assert_allclose(w.cpu().numpy(), wo, rtol=1e-15)


def test_leverage_rows_match(tsk):
    dims, ranks, m, n = (30, 25, 20, 15), (3, 4, 2, 3), 500, 2
    rs = np.random.default_rng(1)
    X = rs.standard_normal(dims)
    facs = [np.linalg.qr(rs.standard_normal((d, r)))[0] for d, r in zip(dims, ranks)]
    fg = [torch.from_numpy(F).to(DEV) for F in facs]
    io, wo = osk.leverage_sample(facs, m, 1, 0, n)  # oracle samples, handed to the library
    idx = torch.from_numpy(io.astype(np.int32)).to(DEV)
    w = torch.from_numpy(wo).to(DEV)
    T = _gpu_tensor(tsk, dims, dense=X)
    Z, Y = tsk.sketch_lev(T, ranks, n, m, idx, w, fg, "f64")
    np.testing.assert_array_equal(Z.cpu().numpy(), osk.leverage_lhs(facs, io, wo, n))
    np.testing.assert_allclose(Y.cpu().numpy(), osk.leverage_rhs_dense(X, io, wo, n), rtol=1e-15)


# ------------------------------------- deterministic leverage selection ----
@pytest.mark.parametrize("dims,ranks,m,n,tie", [
    ((40, 30, 20), (4, 3, 2), 200, 0, False),
    ((60, 50, 40, 30), (3, 3, 3, 3), 500, 1, False),     # order 4: three levels of candidates
    ((500, 500, 500), (30, 30, 30), 14400, 0, False),    # CP-size sketch
    ((2000, 2000, 2000), (10, 10, 10), 1600, 2, False),  # full size, 4e6 rows
    ((30, 25, 20), (3, 3, 3), 150, 1, True),             # equal scores in two modes
    ((6, 5, 4), (2, 2, 2), 20, 0, False),                # every row kept
])
def test_leverage_select_bit_exact(tsk, dims, ranks, m, n, tie):
    rs = np.random.default_rng(sum(dims) + m)
    facs = [np.linalg.qr(rs.standard_normal((d, r)))[0] for d, r in zip(dims, ranks)]
    if tie:
        for k in range(len(dims)):
            if k != n:
                facs[k][1] = facs[k][0]
                facs[k][5] = -facs[k][2]
    fg = [torch.from_numpy(F).to(DEV) for F in facs]
    idx = tsk.leverage_select(dims, ranks, n, m, fg)
    io, _ = osk.leverage_select(facs, m, n)
    assert np.array_equal(idx.cpu().numpy().astype(np.int64), io)


# ------------------------------------------------- sparse fibres (f2) ----
def _coo_with_duplicates(dims, nnz, dup, rs, dtype):
    """nnz distinct uniform coordinates, `dup` of them stored again with fresh
    values, all shuffled (COO: duplicates add)."""
    idx, _ = workloads.distinct_coords(
        dims, nnz, lambda r, c: np.stack([r.integers(0, d, c) for d in dims], 1), rs)
    if dup and nnz:
        idx = np.concatenate([idx, idx[rs.integers(0, nnz, dup)]])
    val = rs.standard_normal(idx.shape[0])
    perm = rs.permutation(idx.shape[0])
    return idx[perm].astype(np.int32), val[perm].astype(dtype)


def _fibre_samples(dims, n, idx, m, rs):
    """m sampled other-mode coordinates: half taken from stored entries (non-empty
    fibres, duplicates included), half uniform; positive weights."""
    others = [k for k in range(len(dims)) if k != n]
    uni = np.stack([rs.integers(0, dims[k], m) for k in others], 1)
    if idx.shape[0]:
        hit = idx[rs.integers(0, idx.shape[0], m)][:, others]
        uni[: m // 2] = hit[: m // 2]
    return uni.astype(np.int32), rs.uniform(0.5, 2.0, m)


def _check_fibres(tsk, dims, idx, val, n, samples, w):
    T = _gpu_tensor(tsk, dims, idx, val)
    fx = tsk.fiber_index(T, n)
    ig, wg = torch.from_numpy(samples).to(DEV), torch.from_numpy(w).to(DEV)
    Yo = osk.leverage_rhs_sparse(osk.Tensor(dims, idx, val), samples.astype(np.int64), w, n)
    Y64 = tsk.sketch_lev_coo(T, fx, samples.shape[0], ig, wg, "f64").cpu().numpy()
    np.testing.assert_array_equal(Y64, Yo)
    Y32 = tsk.sketch_lev_coo(T, fx, samples.shape[0], ig, wg, "f32").cpu().numpy()
    np.testing.assert_array_equal(Y32, Yo.astype(np.float32))
    Ybf = tsk.sketch_lev_coo(T, fx, samples.shape[0], ig, wg, "bf16").cpu()
    assert torch.equal(Ybf, torch.from_numpy(Yo).float().bfloat16())
    return Yo


@pytest.mark.parametrize("dims,nnz,dup,n,m,dtype", [
    ((30, 25, 20), 3000, 500, 1, 700, np.float64),       # several search rounds
    ((300, 300, 300), 200_000, 20_000, 0, 2000, np.float32),
    ((5000, 9, 7), 40_000, 1000, 0, 300, np.float64),    # s_n > 4096: two LDS chunks
    ((12, 10, 8, 6), 4000, 300, 2, 500, np.float32),     # order 4
    ((7, 6, 5), 40, 10, 2, 64, np.float64),              # fewer entries than one probe round
    ((20, 20, 20), 0, 0, 1, 50, np.float64),             # empty tensor
    ((4096, 6, 5), 20_000, 500, 0, 100, np.float32),     # s_n = one LDS chunk exactly
    ((5, 4097, 6), 20_000, 500, 1, 100, np.float64),     # one column past the chunk
])
def test_fibre_gather_bit_exact(tsk, dims, nnz, dup, n, m, dtype):
    rs = np.random.default_rng(nnz + n)
    idx, val = _coo_with_duplicates(dims, nnz, dup, rs, dtype)
    samples, w = _fibre_samples(dims, n, idx, m, rs)
    Yo = _check_fibres(tsk, dims, idx, val, n, samples, w)
    if nnz:
        assert np.count_nonzero(Yo) > 0


def test_fibre_gather_every_mode_and_sampler(tsk):
    """All modes of one tensor, samples from the library's leverage sampler."""
    dims, ranks = (40, 30, 20), (4, 3, 2)
    rs = np.random.default_rng(11)
    idx, val = _coo_with_duplicates(dims, 8000, 800, rs, np.float32)
    facs = [np.linalg.qr(rs.standard_normal((d, r)))[0] for d, r in zip(dims, ranks)]
    fg = [torch.from_numpy(F).to(DEV) for F in facs]
    for n in range(3):
        ig, wg = tsk.leverage_sample(dims, ranks, n, 600, 5, 1, fg)
        _check_fibres(tsk, dims, idx, val, n, ig.cpu().numpy(), wg.cpu().numpy())


def test_sketch_lev_coo_rejects_dense_route(tsk):
    dims = (10, 9, 8)
    rs = np.random.default_rng(2)
    idx, val = _coo_with_duplicates(dims, 100, 0, rs, np.float64)
    T = _gpu_tensor(tsk, dims, idx, val)
    ig = torch.zeros((4, 2), dtype=torch.int32, device=DEV)
    wg = torch.ones(4, dtype=torch.float64, device=DEV)
    fg = [torch.eye(d, 2, dtype=torch.float64, device=DEV) for d in dims]
    with pytest.raises(RuntimeError, match="tsk_sketch_lev_coo"):
        tsk.sketch_lev(T, (2, 2, 2), 0, 4, ig, wg, fg, "f64")


# ---------------------------------------------------------------- a11 ----
@pytest.mark.parametrize("sparse", [False, True])
def test_fit_matches_oracle(tsk, sparse):
    dims, ranks = (30, 25, 20), (4, 3, 5)
    rs = np.random.default_rng(2)
    facs = [np.linalg.qr(rs.standard_normal((d, r)))[0] for d, r in zip(dims, ranks)]
    core = rs.standard_normal(ranks)
    X = otk.reconstruct(core, facs) + 0.1 * rs.standard_normal(dims)
    if sparse:
        To = osk.Tensor.from_dense(X)
        To = osk.Tensor(dims, To.idx[::3], To.val[::3])
        T = _gpu_tensor(tsk, dims, To.idx.astype(np.int32), To.val)
    else:
        To = osk.Tensor.from_dense(X)
        T = _gpu_tensor(tsk, dims, dense=X)
    f = tsk.fit(T, torch.from_numpy(core).to(DEV), [torch.from_numpy(F).to(DEV) for F in facs])
    assert abs(f - otk.relative_residual(To, core, facs)) < 1e-12


def _distinct_coo(dims, nnz, rs, last_probs=None):
    """nnz distinct coordinates in random order; the last mode's index drawn
    from last_probs when given (skewed run lengths), else uniformly."""
    idx = np.zeros((0, 3), dtype=np.int64)
    while idx.shape[0] < nnz:
        c = 2 * nnz
        last = (rs.choice(dims[2], c, p=last_probs) if last_probs is not None
                else rs.integers(0, dims[2], c))
        new = np.stack([rs.integers(0, dims[0], c), rs.integers(0, dims[1], c), last], 1)
        idx = np.concatenate([idx, new])
        lin = np.ravel_multi_index(idx.T, dims)
        _, first = np.unique(lin, return_index=True)
        idx = idx[np.sort(first)]
    return idx[rs.permutation(idx.shape[0])[:nnz]].astype(np.int32)


@pytest.mark.parametrize("case", ["zipf_last", "one_last_index", "uniform_f32", "below_cutoff"])
def test_fit_rank16_grouped_by_last_index(tsk, case):
    """Rank-16 order-3 COO residuals from 2^16 entries on group the entries by
    their last index (a stable sort) and take <T, T~> as u0^T W_k u1 with
    W_k = C x_3 A^(3)(k, :); compared with the oracle's definition (Sec. 7) on
    skewed runs (a Zipf last index: runs of 3 to 14439 of the 100003
    entries), a single last index (one run over every wave), FP32 values, and
    one entry below the cutoff (the per-entry R^3 kernel)."""
    rs = np.random.default_rng({"zipf_last": 31, "one_last_index": 32, "uniform_f32": 33,
                                "below_cutoff": 34}[case])
    R = 16
    if case == "zipf_last":
        dims, nnz = (300, 200, 1000), 100_003
        p = 1.0 / np.arange(1, dims[2] + 1) ** 1.1
        idx = _distinct_coo(dims, nnz, rs, p / p.sum())
    elif case == "one_last_index":
        dims, nnz = (400, 300, 20), 70_001
        idx = _distinct_coo(dims, nnz, rs, np.eye(dims[2])[5])
    else:
        dims = (200, 150, 3000)
        nnz = 65_536 if case == "uniform_f32" else 65_535
        idx = _distinct_coo(dims, nnz, rs)
    facs = [rs.standard_normal((d, R)) for d in dims]  # not orthonormal
    core = rs.standard_normal((R, R, R))
    model = otk.values_at(core, facs, idx)
    val = model + 0.3 * model.std() * rs.standard_normal(nnz)
    if case == "uniform_f32":
        val = val.astype(np.float32)
    T = _gpu_tensor(tsk, dims, idx, val)
    f = tsk.fit(T, torch.from_numpy(core).to(DEV), [torch.from_numpy(F).to(DEV) for F in facs])
    v64 = val.astype(np.float64)
    want = otk.relative_residual(osk.Tensor(dims, idx, v64), core, facs)
    # the tolerance resolves a relative error of 1e-6 in <T, T~>:
    # d(res)/res = -d<T, T~> / (res^2 ||T||^2)
    assert np.dot(v64, model) / (want ** 2 * np.dot(v64, v64)) > 1e-4
    assert abs(f - want) < 1e-10 * want


# ---------------------------------------------------------------- a12 ----
def test_adjoint_matches_oracle_and_fd(tsk):
    dims, ranks, m, n = (60, 50, 40), (3, 4, 2), 64, 1
    rs = np.random.default_rng(5)
    facs = [rs.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    core = rs.standard_normal(ranks)
    X = rs.standard_normal(dims)
    tabs, h, s = _maps(dims, n, m, 2)
    Yo = osk.ts_rhs(osk.Tensor.from_dense(X), m, tabs, n)
    fg = [torch.from_numpy(F).to(DEV) for F in facs]
    cg = torch.from_numpy(core).to(DEV)
    Yg = torch.from_numpy(Yo).to(DEV)
    L = tsk.sketched_residual(dims, ranks, n, m, h, s, fg, cg, Yg).item()
    Lo, go, gCo = oadj.residual_and_grads(facs, core, tabs, Yo, m, n)
    assert abs(L - Lo) <= 1e-11 * Lo
    grads, gC = tsk.sketched_residual_grads(dims, ranks, n, m, h, s, fg, cg, Yg)
    for k in range(3):
        np.testing.assert_allclose(grads[k].cpu().numpy(), go[k], atol=1e-9 * np.abs(go[k]).max())
    np.testing.assert_allclose(gC.cpu().numpy(), gCo, atol=1e-9 * np.abs(gCo).max())
    # autograd.Function + central differences on the GPU forward (L quadratic per entry)
    fa = [F.clone().requires_grad_(True) for F in fg]
    ca = cg.clone().requires_grad_(True)
    out = tsk.SketchedResidual.apply((dims, ranks, n, m, h, s, Yg), ca, *fa)
    out.backward()
    hstep = 1e-3
    for k in range(3):
        for _ in range(4):
            i, c = rs.integers(dims[k]), rs.integers(ranks[k])
            fp = [F.clone() for F in fg]; fm = [F.clone() for F in fg]
            fp[k][i, c] += hstep; fm[k][i, c] -= hstep
            fd = (tsk.sketched_residual(dims, ranks, n, m, h, s, fp, cg, Yg).item() -
                  tsk.sketched_residual(dims, ranks, n, m, h, s, fm, cg, Yg).item()) / (2 * hstep)
            g = fa[k].grad[i, c].item()
            assert abs(fd - g) <= 1e-7 * max(1.0, abs(fd))


# ------------------------------------------------------------ RSVD-LRLS ----
@pytest.mark.parametrize("m,r,s,R,k", [(300, 100, 400, 10, 20), (80, 25, 40, 5, 15),
                                       (400, 144, 150, 12, 22), (150, 36, 50, 12, 20),
                                       (200, 40, 60, 26, 30), (500, 120, 90, 7, 13),
                                       (400, 128, 200, 10, 24), (60, 17, 30, 3, 8),
                                       (50, 9, 20, 1, 1), (250, 64, 100, 16, 16)])
def test_rsvd_solve_fp64_vs_oracle(tsk, m, r, s, R, k):
    """RSVD-LRLS (Alg. 5) with the same Gaussian test matrix: FP64 library vs
    the oracle.  r = 144 exercises the Cholesky branch of the Gram solve,
    k = 30 the unfused chain and the order-32 eigensolver with R = 26 vectors,
    r = 120 a large register SPD inverse; r = 128 with k = 24 is the largest
    fused shape, r = 17 with k = 8 a ragged one at the smallest column block,
    R = k = 1 the degenerate sketch of one column, R = k = 16 all vectors kept."""
    rs = np.random.default_rng(m + r)
    Z = rs.standard_normal((m, r))
    Y = rs.standard_normal((m, s))
    Om = rs.standard_normal((s, k))
    A, W = tsk.rsvd_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R,
                          torch.from_numpy(Om).to(DEV))
    Ao, Wo = osv.rsvd_lrls(Z, Y, R, Om)
    np.testing.assert_allclose(A.cpu().numpy(), Ao, atol=1e-9)
    np.testing.assert_allclose(W.cpu().numpy(), Wo, atol=1e-9 * np.abs(Wo).max())


def test_rsvd_solve_rank_deficient(tsk):
    """Z^+ Y of rank 3 < k: the test matrix product C is rank deficient; the
    Householder QR still returns an orthonormal Q and the leading 3 triplets are
    exact."""
    rs = np.random.default_rng(5)
    m, r, s, R, k = 200, 36, 60, 3, 13
    Z = rs.standard_normal((m, r))
    X = rs.standard_normal((r, R)) @ rs.standard_normal((R, s))
    Y = Z @ X
    Om = rs.standard_normal((s, k))
    A, W = tsk.rsvd_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R,
                          torch.from_numpy(Om).to(DEV))
    np.testing.assert_allclose(W.cpu().numpy() @ A.cpu().numpy().T, X, atol=1e-9 * np.abs(X).max())


@pytest.mark.parametrize("solver", ["rsvd", "exact"])
def test_solve_zero_rhs_is_a_breakdown(tsk, solver):
    """An all-zero right-hand side: every singular value of the subproblem is
    zero, so A = D^T U Sigma^{-1} is undefined; both solvers report a numerical
    breakdown rather than non-finite factors."""
    from paper_2104_01101_amd import _lib as L
    rs = np.random.default_rng(11)
    m, r, s, R, k = 200, 36, 60, 3, 13
    Z = torch.from_numpy(rs.standard_normal((m, r))).to(DEV)
    Y = torch.zeros((m, s), dtype=torch.float64, device=DEV)
    with pytest.raises(L.TskError) as e:
        if solver == "rsvd":
            tsk.rsvd_solve(Z, Y, R, torch.from_numpy(rs.standard_normal((s, k))).to(DEV))
        else:
            tsk.rc_solve(Z, Y, R)
    assert e.value.status == L.ENUMERIC


@pytest.mark.parametrize("init", ["random", "rrf"])
@pytest.mark.parametrize("solve", ["rsvd", "exact"])
def test_zero_tensor_is_a_breakdown(tsk, solve, init):
    """Sketch-Tucker-ALS on an all-zero tensor: from a random start the first
    subproblem has a zero right-hand side; from the range-finder start the
    range finder's B = W G is zero already.  Either way the call reports a
    breakdown."""
    from paper_2104_01101_amd import _lib as L
    T = tsk.Tensor.dense(torch.zeros((30, 30, 30), dtype=torch.float64, device=DEV))
    with pytest.raises(L.TskError) as e:
        tsk.tucker_sketch_als(T, (4, 4, 4), 200, 2, init=init, prec="f64", solve=solve)
    assert e.value.status == L.ENUMERIC
    assert ("initialisation" if init == "rrf" else "rank below R") in str(e.value), e.value


def test_rsvd_solve_fp32_operands(tsk):
    rs = np.random.default_rng(9)
    m, r, s, R, k = 1600, 100, 2000, 10, 20
    Z = rs.standard_normal((m, r)).astype(np.float32)
    Y = rs.standard_normal((m, s)).astype(np.float32)
    Om = rs.standard_normal((s, k))
    A, W = tsk.rsvd_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R,
                          torch.from_numpy(Om).to(DEV))
    Ao, Wo = osv.rsvd_lrls(Z.astype(np.float64), Y.astype(np.float64), R, Om)
    # compare the rank-R solutions (subspace and scale), FP32 operand rounding
    Xg = W.cpu().numpy() @ A.cpu().numpy().T
    Xo = Wo @ Ao.T
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) < 1e-4


# ------------------------------------------------- large Grams (r > 142) ----
@pytest.mark.parametrize("m,r,s,R,k", [(2048, 256, 1500, 16, 26), (4000, 1000, 200, 10, 20),
                                       (14400, 900, 500, 30, 40), (1300, 300, 700, 8, 40),
                                       (700, 143, 90, 5, 12), (2048, 256, 10000, 16, 26)])
def test_rsvd_solve_large_r_fp64(tsk, m, r, s, R, k):
    """RSVD-LRLS at the Gram orders of the 10000^3 (r = 256), 200^4 (r = 1000)
    and 500^3 (r = 900) workloads: the Gram is inverted by block sweeps (32
    pivots per block; r = 300 and 143 leave a ragged last block) and the
    products with Y follow the O(m s k) order; s = 10^4 (the 10000^3 shape)
    takes D D^T over K = s by split partial tiles.  FP64 library vs the oracle
    with the same test matrix."""
    rs = np.random.default_rng(m + r + 7)
    Z = rs.standard_normal((m, r))
    Y = Z @ rs.standard_normal((r, R)) @ rs.standard_normal((R, s)) + 0.1 * rs.standard_normal((m, s))
    Om = rs.standard_normal((s, k))
    A, W = tsk.rsvd_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R,
                          torch.from_numpy(Om).to(DEV))
    Ao, Wo = osv.rsvd_lrls(Z, Y, R, Om)
    np.testing.assert_allclose(A.cpu().numpy(), Ao, atol=1e-9)
    np.testing.assert_allclose(W.cpu().numpy(), Wo, atol=1e-9 * np.abs(Wo).max())


@pytest.mark.parametrize("noise", [1e-2, 1e-6, 1e-9])
def test_rsvd_solve_range_basis_conditioning(tsk, noise):
    """The thin QR of C = B Z^T Y Omega at r = 256, k = 26 with Y of rank R = 16
    plus noise: C has R large and k - R small singular values, so kappa(C)
    grows as the noise shrinks.  Noise 1e-2 (kappa(C) 5.2e4, first-factor
    diagonal ratio 1.4e4) keeps two plain Cholesky QR passes; at 1e-6 and 1e-9
    the first unshifted Cholesky factorisation breaks down (the Gram of C is
    not numerically positive definite) and the kernel restarts with the three
    shifted passes.  FP64 against the oracle: the rank-R solution W A^T within
    1e-9 relative."""
    rs = np.random.default_rng(31)
    m, r, s, R, k = 2048, 256, 1500, 16, 26
    Z = rs.standard_normal((m, r))
    Y = Z @ rs.standard_normal((r, R)) @ rs.standard_normal((R, s)) + noise * rs.standard_normal((m, s))
    Om = rs.standard_normal((s, k))
    A, W = tsk.rsvd_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R,
                          torch.from_numpy(Om).to(DEV))
    Ao, Wo = osv.rsvd_lrls(Z, Y, R, Om)
    Xg = W.cpu().numpy() @ A.cpu().numpy().T
    Xo = Wo @ Ao.T
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) < 1e-9
    np.testing.assert_allclose(A.cpu().numpy().T @ A.cpu().numpy(), np.eye(R), atol=1e-10)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("m,r,s,R,k", [(2048, 256, 1500, 16, 26), (14400, 900, 500, 30, 40),
                                       (1000, 102, 301, 6, 20), (1000, 200, 4004, 8, 17),
                                       (1500, 160, 2000, 4, 12), (777, 130, 1501, 5, 30)])
def test_rsvd_solve_large_r_low_precision(tsk, prec, m, r, s, R, k):
    """RSVD-LRLS with FP32 or BF16 operands at the shapes of the 10000^3 and
    500^3 jobs (the vectorised FP32 / BF16 matrix-core products: r = 900 has
    rows of 900 elements, 8-byte but not 16-byte aligned; r = 102 and s = 301
    leave ragged tiles).  With FP32 operands, rows of Y of a multiple of 4
    elements and k <= 32, the products with Y take the skinny streaming
    kernel: m = 1000 and s = 4004 leave ragged 64-row tiles and contraction
    ranges, k = 17 one column in the second 16-column tile, k = 12 none;
    s = 1501 (rows not a multiple of 4) takes the tiled kernel instead.  The
    operands are rounded on the host and the oracle
    runs on the rounded values in FP64.  In the O(m s k) order the library
    also rounds the test matrix Omega and the product Z P to the operand type
    before the products with Y: the rank-R solution X = W A^T is within 1e-5
    of the oracle's with FP32 operands (accumulation and that rounding) and
    within 1e-3 with BF16 (unit roundoff 2^-8 on Omega and Z P)."""
    rs = np.random.default_rng(m + r + 11)
    Z = rs.standard_normal((m, r))
    Y = Z @ rs.standard_normal((r, R)) @ rs.standard_normal((R, s)) + 0.1 * rs.standard_normal((m, s))
    Om = rs.standard_normal((s, k))
    dt = {"f32": torch.float32, "bf16": torch.bfloat16}[prec]
    Zc, Yc = torch.from_numpy(Z).to(dt), torch.from_numpy(Y).to(dt)  # rounded on the host
    A, W = tsk.rsvd_solve(Zc.to(DEV), Yc.to(DEV), R, torch.from_numpy(Om).to(DEV), prec=prec)
    Ao, Wo = osv.rsvd_lrls(Zc.double().numpy(), Yc.double().numpy(), R, Om)
    Xg = W.cpu().numpy() @ A.cpu().numpy().T
    Xo = Wo @ Ao.T
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) < (1e-5 if prec == "f32" else 1e-3)


@pytest.mark.parametrize("m,r,s,R", [(2048, 256, 1500, 16), (4000, 1000, 200, 10),
                                     (1300, 300, 700, 8)])
def test_rc_solve_large_r_fp64(tsk, m, r, s, R):
    """The exact solve with the blocked inverse of the Gram (r > 142)."""
    rs = np.random.default_rng(m * 3 + r)
    Z = rs.standard_normal((m, r)) / np.sqrt(m)
    Y = Z @ rs.standard_normal((r, R)) @ rs.standard_normal((R, s)) + 0.1 * rs.standard_normal((m, s))
    A, W = tsk.rc_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R)
    Ao, Wo, _ = osv.rc_solve(Z, Y, R)
    A, W = A.cpu().numpy(), W.cpu().numpy()
    np.testing.assert_allclose(A, Ao, atol=1e-9 * max(1, np.abs(Ao).max()))
    np.testing.assert_allclose(W, Wo, atol=1e-9 * max(1, np.abs(Wo).max()))


@pytest.mark.parametrize("solver", ["rsvd", "exact"])
@pytest.mark.parametrize("r,zero", [(200, 150), (400, 0), (400, 399)])
def test_blocked_inverse_singular_gram(tsk, solver, r, zero):
    """A zero column of Z makes the Gram singular: its Schur pivot is exactly 0
    in every block position (first, inner, last index), and both solvers report
    a breakdown from the blocked inverse."""
    from paper_2104_01101_amd import _lib as L
    rs = np.random.default_rng(r + zero)
    m, s, R, k = 3 * r, 80, 4, 12
    Z = rs.standard_normal((m, r))
    Z[:, zero] = 0.0
    Y = torch.from_numpy(rs.standard_normal((m, s))).to(DEV)
    Zg = torch.from_numpy(Z).to(DEV)
    with pytest.raises(L.TskError) as e:
        if solver == "rsvd":
            tsk.rsvd_solve(Zg, Y, R, torch.from_numpy(rs.standard_normal((s, k))).to(DEV))
        else:
            tsk.rc_solve(Zg, Y, R)
    assert e.value.status == L.ENUMERIC


@pytest.mark.parametrize("m,r,s,R,k", [(800, 200, 120, 4, 30), (900, 260, 150, 2, 50)])
def test_rsvd_solve_rank_deficient_large(tsk, m, r, s, R, k):
    """Z^+ Y of rank R < k at Gram orders beyond the register kernels: the
    sketched range C = B Z^T Y Omega has rank R, the shifted Cholesky QR breaks
    down in its second pass and the Householder fallback runs; the rank-R
    solution is still exact."""
    rs = np.random.default_rng(m + s)
    Z = rs.standard_normal((m, r))
    X = rs.standard_normal((r, R)) @ rs.standard_normal((R, s))
    Y = Z @ X
    Om = rs.standard_normal((s, k))
    A, W = tsk.rsvd_solve(torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), R,
                          torch.from_numpy(Om).to(DEV))
    np.testing.assert_allclose(W.cpu().numpy() @ A.cpu().numpy().T, X, atol=1e-9 * np.abs(X).max())
