"""Seeded synthetic tensors shaped like the paper's workloads.

This module only builds inputs.  It holds none of the method's arithmetic (no
hashing, sketching, solving or fitting); both the HIP library's tests/benchmark
and the FP64 oracle take their tensors from here.  Random numbers come from
NumPy's PCG64 (np.random.default_rng), unrelated to the method's own
counter-based streams.

Families (Sec. 7 of the paper builds all its tensors synthetically):
* tucker_dense   T = C x_1 B1 x_2 B2 ... + noise  (Tensor 1, eq. tsr_dense), with
                 Gaussian core and either Gaussian or QR-orthonormalised factors
* sparse_tucker  distinct uniform coordinates, value = Tucker signal at the
                 coordinate + N(0,1)
* sparse_zipf    distinct coordinates with Zipf-distributed indices per mode,
                 lognormal values
* cp_collinear   sum of rank-1 terms with unit-norm factor columns of pairwise
                 cosine c, + noise (the CP experiments of Sec. 7)
* paper_tensor1..4  the four test tensors of Sec. 7 as the paper defines them
                 (Gaussian Tucker; + power-law rank-1 spikes; sparse Tucker with
                 entries kept with probability p; + a few coherent large entries)
* the named configurations c1..c5 (full size or scaled down)
"""
import numpy as np


class Workload(dict):
    """dims, dense (ndarray | None), idx (nnz x N int32 | None), val (nnz), and
    the method parameters of the configuration."""
    __getattr__ = dict.__getitem__


def _orth(G):
    Q, _ = np.linalg.qr(G)
    return Q


def _tucker_values(core, factors, idx, chunk=1 << 15):
    out = np.empty(idx.shape[0])
    for lo in range(0, idx.shape[0], chunk):
        sl = slice(lo, lo + chunk)
        X = np.tensordot(factors[0][idx[sl, 0]], core, axes=(1, 0))
        for k in range(1, len(factors)):
            X = np.einsum("er,er...->e...", factors[k][idx[sl, k]], X)
        out[sl] = X
    return out


def _dense_from_tucker(core, factors):
    X = core
    for k, B in enumerate(factors):
        X = np.moveaxis(np.tensordot(B, X, axes=(1, k)), 0, k)
    return X


def tucker_dense(dims, ranks, noise=0.01, seed=0, orthonormal=True, dtype=np.float64):
    rs = np.random.default_rng(seed)
    core = rs.standard_normal(ranks)
    fac = [rs.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    if orthonormal:
        fac = [_orth(B) for B in fac]
    X = _dense_from_tucker(core, fac)
    if noise > 0:
        E = rs.standard_normal(dims)
        X = X + noise * np.linalg.norm(X) / np.linalg.norm(E) * E
    return X.astype(dtype)


def distinct_coords(dims, nnz, sampler, rs):
    """Draw coordinates with `sampler(rs, count) -> (count, N)` until nnz distinct
    ones exist; keep the first nnz distinct in draw order, then shuffle."""
    dims = np.asarray(dims, dtype=np.int64)
    kept = np.empty((0, len(dims)), dtype=np.int64)
    seen = np.empty(0, dtype=np.int64)
    draws = 0
    while kept.shape[0] < nnz:
        need = nnz - kept.shape[0]
        c = sampler(rs, int(need * 1.3) + 1024)
        draws += c.shape[0]
        lin = np.ravel_multi_index(c.T, dims)
        allc = np.concatenate([seen, lin])
        _, first = np.unique(allc, return_index=True)
        first = np.sort(first)
        new = first[first >= seen.size] - seen.size
        kept = np.concatenate([kept, c[new][:need]])
        seen = np.ravel_multi_index(kept.T, dims)
    perm = rs.permutation(nnz)
    return kept[perm], draws


def sparse_tucker(dims, nnz, ranks, seed=0, noise_std=1.0, dtype=np.float32):
    rs = np.random.default_rng(seed)
    idx, _ = distinct_coords(
        dims, nnz, lambda r, c: np.stack([r.integers(0, d, c) for d in dims], 1), rs)
    core = rs.standard_normal(ranks)
    fac = [rs.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    val = _tucker_values(core, fac, idx) + noise_std * rs.standard_normal(nnz)
    return idx.astype(np.int32), val.astype(dtype)


def zipf_sampler(dims, a):
    cdfs = []
    for d in dims:
        p = np.arange(1, d + 1, dtype=np.float64) ** (-a)
        c = np.cumsum(p)
        cdfs.append(c / c[-1])

    def sample(rs, count):
        cols = [np.minimum(np.searchsorted(c, rs.random(count), side="right"), len(c) - 1)
                for c in cdfs]
        return np.stack(cols, 1).astype(np.int64)
    return sample


def sparse_zipf(dims, nnz, a=1.1, seed=0, dtype=np.float32):
    rs = np.random.default_rng(seed)
    idx, draws = distinct_coords(dims, nnz, zipf_sampler(dims, a), rs)
    val = rs.lognormal(0.0, 1.0, nnz)
    return idx.astype(np.int32), val.astype(dtype), draws


def cp_collinear(dims, rank, collinearity=0.9, noise=0.01, seed=0, dtype=np.float32):
    """A^(k) = Q_k L^T with L L^T = (1-c) I + c 11^T, Q_k = qr(N(0,1)^{s x R}):
    unit-norm columns with pairwise cosine c."""
    rs = np.random.default_rng(seed)
    Mc = (1 - collinearity) * np.eye(rank) + collinearity * np.ones((rank, rank))
    L = np.linalg.cholesky(Mc)
    fac = [_orth(rs.standard_normal((d, rank))) @ L.T for d in dims]
    X = np.zeros(dims)
    for r in range(rank):
        t = fac[0][:, r]
        for F in fac[1:]:
            t = np.multiply.outer(t, F[:, r])
        X += t
    if noise > 0:
        E = rs.standard_normal(dims)
        X = X + noise * np.linalg.norm(X) / np.linalg.norm(E) * E
    return X.astype(dtype), fac


# ----------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------
# ----------------------------------------------------------------------------
# The four test tensors of Sec. 7 (order 3, s x s x s, R_true = round(alpha R))
# ----------------------------------------------------------------------------
def true_rank(R, alpha):
    return int(round(alpha * R))


def paper_tensor1(s, R, alpha, seed=0):
    """Tensor 1 (eq. tsr_dense): T = C x_1 B1 x_2 B2 x_3 B3 with every entry of the
    core (R_true^3) and of the factors (s x R_true) i.i.d. N(0, 1).  Dense FP64."""
    rs = np.random.default_rng(seed)
    Rt = true_rank(R, alpha)
    core = rs.standard_normal((Rt, Rt, Rt))
    fac = [rs.standard_normal((s, Rt)) for _ in range(3)]
    return _dense_from_tucker(core, fac)


def paper_tensor2(s, R, alpha, seed=0, n=5, C=3.0, eta=0.5):
    """Tensor 2: Tensor 1 + sum_{i=1..n} lambda_i a1_i o a2_i o a3_i with unit-norm
    Gaussian directions and power-law magnitudes lambda_i = C ||T||_F / i^(1+eta)
    (n = 5, C = 3, eta = 0.5 as in the experiments).  Dense FP64."""
    X = paper_tensor1(s, R, alpha, seed)
    rs = np.random.default_rng(seed + 7919)
    nrm = np.linalg.norm(X)
    for i in range(1, n + 1):
        a = [v / np.linalg.norm(v) for v in (rs.standard_normal(s) for _ in range(3))]
        X = X + (C * nrm / i ** (1.0 + eta)) * np.einsum("i,j,k->ijk", *a)
    return X


def paper_tensor3(s, R, alpha, p, seed=0):
    """Tensor 3 (eq. tsr_sparse): Tensor 1 with every core and factor entry kept
    with probability p (N(0,1)) and zero otherwise, so a term of the sum is
    nonzero with probability p^4 and the expected density is at most
    R_true^3 p^4.  Built from the nonzero core entries: each adds the outer
    product of its three factor columns' supports; coinciding coordinates are
    summed.  Returns (idx int32 nnz x 3, val float64), coordinates distinct."""
    rs = np.random.default_rng(seed)
    Rt = true_rank(R, alpha)
    keep = lambda shape: np.where(rs.random(shape) < p, rs.standard_normal(shape), 0.0)
    core = keep((Rt, Rt, Rt))
    fac = [keep((s, Rt)) for _ in range(3)]
    keys, vals = [], []
    for x, y, z in zip(*np.nonzero(core)):
        cols = [np.nonzero(fac[0][:, x])[0], np.nonzero(fac[1][:, y])[0],
                np.nonzero(fac[2][:, z])[0]]
        if min(c.size for c in cols) == 0:
            continue
        v = core[x, y, z] * np.einsum("i,j,k->ijk", fac[0][cols[0], x], fac[1][cols[1], y],
                                      fac[2][cols[2], z])
        ii, jj, kk = np.meshgrid(*cols, indexing="ij")
        keys.append(((ii * s + jj) * s + kk).reshape(-1))
        vals.append(v.reshape(-1))
    if not keys:
        return np.zeros((0, 3), np.int32), np.zeros(0)
    key = np.concatenate(keys)
    u, inv = np.unique(key, return_inverse=True)
    val = np.bincount(inv, weights=np.concatenate(vals), minlength=u.size)
    nz = val != 0.0
    idx = np.stack(np.unravel_index(u[nz], (s, s, s)), 1).astype(np.int32)
    perm = rs.permutation(idx.shape[0])
    return idx[perm], val[nz][perm]


def coherent_spikes(dims, norm, seed=0, n=10):
    """The N of Tensor 4: n distinct random positions, values i.i.d.
    N(norm / sqrt(n), 1) (so E ||N||_F / norm = 1 with norm = ||T||_F)."""
    rs = np.random.default_rng(seed + 104729)
    lin = rs.choice(int(np.prod(dims)), size=n, replace=False)
    idx = np.stack(np.unravel_index(lin, dims), 1).astype(np.int32)
    return idx, rs.normal(norm / np.sqrt(n), 1.0, n)


def paper_tensor4_dense(s, R, alpha, seed=0, n=10):
    """Tensor 4 on Tensor 1: a dense FP64 s^3 tensor plus n coherent entries."""
    X = paper_tensor1(s, R, alpha, seed)
    idx, val = coherent_spikes(X.shape, np.linalg.norm(X), seed, n)
    X[tuple(idx.T)] += val
    return X


def paper_tensor4_sparse(s, R, alpha, p, seed=0, n=10):
    """Tensor 4 on Tensor 3: COO (distinct coordinates) plus n coherent entries
    (a spike on a stored coordinate is added to its value)."""
    idx, val = paper_tensor3(s, R, alpha, p, seed)
    sidx, sval = coherent_spikes((s, s, s), np.linalg.norm(val), seed, n)
    key = np.concatenate([np.ravel_multi_index(idx.T.astype(np.int64), (s, s, s)),
                          np.ravel_multi_index(sidx.T.astype(np.int64), (s, s, s))])
    u, inv = np.unique(key, return_inverse=True)
    v = np.bincount(inv, weights=np.concatenate([val, sval]), minlength=u.size)
    out = np.stack(np.unravel_index(u, (s, s, s)), 1).astype(np.int32)
    perm = np.random.default_rng(seed + 1).permutation(u.size)
    return out[perm], v[perm]


def dense40(seed=0, s=40, R=5, K=8):
    """Dense 3-way s^3 FP64, Tucker rank (R,R,R) with Gaussian core and QR
    factors, 1% noise; TensorSketch m = K R^2, RRF init, 5 sweeps, FP64."""
    X = tucker_dense((s, s, s), (R, R, R), 0.01, seed, True, np.float64)
    return Workload(name="dense40", dims=X.shape, dense=X, idx=None, val=None,
                    ranks=(R, R, R), m=K * R * R, sweeps=5, sketch="ts",
                    prec="f64", init="rrf")


def sparse2000(seed=0, s=2000, nnz=1_000_000, R=10, K=16, sweeps=10):
    """Sparse 3-way s^3 FP32 with nnz distinct uniform coordinates, value =
    Gaussian Tucker rank-(R,R,R) signal + N(0,1); TensorSketch m = K R^2."""
    idx, val = sparse_tucker((s, s, s), nnz, (R, R, R), seed)
    return Workload(name="sparse2000", dims=(s, s, s), dense=None, idx=idx, val=val,
                    ranks=(R, R, R), m=K * R * R, sweeps=sweeps, sketch="ts",
                    prec="f32", init="rrf")


def sparse2000lev(seed=0, s=2000, nnz=1_000_000, R=10, K=16, sweeps=10):
    """The sparse2000 tensor under leverage-score sampling (m = K R^2 sampled
    fibres per subproblem, redrawn every subproblem) instead of TensorSketch."""
    w = sparse2000(seed, s, nnz, R, K, sweeps)
    w["name"], w["sketch"] = "sparse2000lev", "lev"
    return w


def sparse2000det(seed=0, s=2000, nnz=1_000_000, R=10, K=24, sweeps=10):
    """The sparse2000 tensor under deterministic leverage selection (the m = K R^2
    rows of largest Kronecker leverage score per subproblem, weights 1).  K = 24:
    at K = 16 the rows selected from the range-finder start span only 97 of the
    100 directions in the second subproblem (a singular sketched Gram), while at
    K = 24 every selection of the 10 sweeps has full rank (smallest Gram
    eigenvalue 8e-4)."""
    w = sparse2000(seed, s, nnz, R, K, sweeps)
    w["name"], w["sketch"] = "sparse2000det", "lev_det"
    return w


def dense4d200(seed=0, s=200, R=10, m=4000, sweeps=5, prec="f32"):
    """Dense 4-way s^4 FP32 Tucker rank-(R,..,R) signal + 1% noise; leverage-score
    sampling with m rows per subproblem."""
    X = tucker_dense((s,) * 4, (R,) * 4, 0.01, seed, True, np.float32)
    return Workload(name="dense4d200", dims=X.shape, dense=X, idx=None, val=None,
                    ranks=(R,) * 4, m=m, sweeps=sweeps, sketch="lev", prec=prec,
                    init="rrf")


def zipf10k(seed=0, s=10_000, nnz=10_000_000, R=16, K=8):
    """Sparse 3-way s^3 FP32, nnz distinct coordinates with Zipf(1.1) indices,
    lognormal(0,1) values; Tucker rank (R,R,R), TensorSketch m = K R^2."""
    idx, val, draws = sparse_zipf((s, s, s), nnz, 1.1, seed)
    return Workload(name="zipf10k", dims=(s, s, s), dense=None, idx=idx, val=val,
                    ranks=(R, R, R), m=K * R * R, sweeps=5, sketch="ts",
                    prec="f32", init="rrf", draws=draws)


def cp500(seed=0, s=500, cp_rank=20, R=30, K=16, prec="bf16"):
    """Dense 3-way s^3 FP32 CP rank-20 signal (pairwise collinearity 0.9) + 1%
    noise; sketched Tucker (leverage, m = K R^2) to rank (R,R,R), then CP-ALS of
    rank cp_rank on the core (5 Tucker + 25 CP sweeps)."""
    X, fac = cp_collinear((s, s, s), cp_rank, 0.9, 0.01, seed, np.float32)
    return Workload(name="cp500", dims=X.shape, dense=X, idx=None, val=None,
                    ranks=(R, R, R), m=K * R * R, sweeps=5, sketch="lev",
                    prec=prec, init="rrf", cp_rank=cp_rank, cp_sweeps=25)
