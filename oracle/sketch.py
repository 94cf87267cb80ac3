"""Sketching operators of sketched Tucker-ALS (oracle side; test infrastructure only).

Everything is FP64 NumPy, written from the paper's definitions:

* CountSketch S = Omega D                       -- Definition (CountSketch), Sec. 3.1
* TensorSketch hash H = sum_k H_k mod m, sign S = prod_k S_k
                                                -- Definition (TensorSketch), eq. (h_ts), (s_ts)
* S P for a Kronecker chain P via the spectra of S^(k) A^(k)
                                                -- Sec. 3.1, the FFT identity below the definition
  The oracle evaluates that identity as what it is, a length-m circular
  convolution, computed directly (no FFT), so the FFT route of the library is
  checked against a different computation.
* leverage scores and Kronecker-factored sampling
                                                -- Definition (leverage scores), Definition
                                                   (importance sampling), Lemma (Kronecker leverage)
* deterministic leverage selection (the m rows of largest score, no rescaling)
                                                -- Sec. 3.2, the deterministic alternative to
                                                   importance sampling
* composite sketch S = T G of the range finder  -- Definition (composite sketch), Sec. 5

Index conventions.  Tensors are row-major (last index fastest).  For mode n the
"other-mode multi-index" (i_k)_{k != n} is linearised row-major in increasing k,
which is also the row order of the Kronecker chain A^(k1) (x) A^(k2) (x) ... and
the column order rho = (rho_k)_{k != n} of Z = S P.  The paper's definition
writes the linear index first-index-fastest; the hash values depend only on the
multi-index, so the choice changes nothing but the order of rows and columns.
"""
import numpy as np

from . import rng


# ----------------------------------------------------------------------------
# tensors
# ----------------------------------------------------------------------------
class Tensor:
    """Order-N tensor as coordinates + values (a dense array is given all its
    entries as coordinates, in row-major order)."""

    def __init__(self, dims, idx, val):
        self.dims = tuple(int(d) for d in dims)
        self.idx = np.asarray(idx, dtype=np.int64).reshape(-1, len(self.dims))
        self.val = np.asarray(val, dtype=np.float64).reshape(-1)

    @classmethod
    def from_dense(cls, X):
        X = np.asarray(X, dtype=np.float64)
        idx = np.stack(np.unravel_index(np.arange(X.size), X.shape), axis=1)
        t = cls(X.shape, idx, X.reshape(-1))
        t.dense = X
        return t

    @property
    def order(self):
        return len(self.dims)

    def coalesced(self):
        """Sum duplicate coordinates (COO semantics: duplicates add)."""
        lin = np.ravel_multi_index(self.idx.T, self.dims)
        u, inv = np.unique(lin, return_inverse=True)
        v = np.bincount(inv, weights=self.val, minlength=u.size)
        idx = np.stack(np.unravel_index(u, self.dims), axis=1)
        return Tensor(self.dims, idx, v)

    def to_dense(self):
        if getattr(self, "dense", None) is not None:
            return self.dense
        X = np.zeros(self.dims)
        np.add.at(X, tuple(self.idx.T), self.val)
        return X

    def norm2(self):
        c = self.coalesced()
        return float(np.dot(c.val, c.val))


def other_modes(N, n):
    return [k for k in range(N) if k != n]


def other_linear_index(dims, idx, n):
    """Row-major linear index of (i_k)_{k != n}."""
    lin = np.zeros(idx.shape[0], dtype=np.int64)
    for k in other_modes(len(dims), n):
        lin = lin * dims[k] + idx[:, k]
    return lin


# ----------------------------------------------------------------------------
# TensorSketch (Sec. 3.1)
# ----------------------------------------------------------------------------
def ts_tables(dims, m, seed, n):
    """Hash and sign maps H_k : [s_k] -> [m], S_k : [s_k] -> {+1,-1} of the
    order-(N-1) TensorSketch used by subproblem n, for every k != n.
    Returns {k: (h int64[s_k], sigma float64[s_k])}."""
    out = {}
    for k in other_modes(len(dims), n):
        x = rng.draw(rng.stream_key(seed, rng.P_TS, n, k), np.arange(dims[k]))
        out[k] = (rng.bucket(x, m).astype(np.int64), rng.sign(x))
    return out


def ts_hash_sign(tables, idx, m):
    """H(i) = (sum_k H_k(i_k)) mod m and S(i) = prod_k S_k(i_k), eq. (h_ts)/(s_ts)
    (0-based form of the paper's 1-based formula)."""
    H = np.zeros(idx.shape[0], dtype=np.int64)
    S = np.ones(idx.shape[0])
    for k, (h, sg) in tables.items():
        H = H + h[idx[:, k]]
        S = S * sg[idx[:, k]]
    return H % m, S


def ts_rhs(T, m, tables, n):
    """Y = S^(n) T_(n)^T in R^{m x s_n}: every entry v at coordinate i adds
    S(i_{-n}) v to Y[H(i_{-n}), i_n].  Accumulated with bincount (FP64, in input
    order) -- Alg. 4 sketch of the right-hand side."""
    s_n = T.dims[n]
    H, S = ts_hash_sign(tables, T.idx, m)
    key = H * s_n + T.idx[:, n]
    return np.bincount(key, weights=S * T.val, minlength=m * s_n).reshape(m, s_n)


def countsketch(A, h, sigma, m):
    """S^(k) A^(k) for CountSketch S^(k) = Omega D: row i of A, signed by sigma(i),
    is added to row h(i)."""
    A = np.asarray(A, dtype=np.float64)
    out = np.zeros((m, A.shape[1]))
    for c in range(A.shape[1]):
        out[:, c] = np.bincount(h, weights=sigma * A[:, c], minlength=m)
    return out


def circulant(b):
    """C with C[j, t] = b[(j - t) mod m], so C @ a is the circular convolution."""
    m = b.shape[0]
    return b[(np.arange(m)[:, None] - np.arange(m)[None, :]) % m]


def ts_lhs(factors, tables, m, n):
    """Z = S^(n) P^(n), P^(n) = kron_{k != n} A^(k), as the column-wise circular
    convolution of the CountSketches S^(k) A^(k)  (Sec. 3.1: the FFT identity is
    the convolution theorem applied to this product).  Column rho is row-major
    over (rho_k)_{k != n}.  Direct O(m^2) convolution, no FFT."""
    Z = np.zeros((m, 1))
    Z[0, 0] = 1.0                          # unit impulse: identity of convolution
    for k in sorted(tables):
        h, sg = tables[k]
        CS = countsketch(factors[k], h, sg, m)
        blocks = [circulant(CS[:, c]) @ Z for c in range(CS.shape[1])]
        Z = np.stack(blocks, axis=2).reshape(m, -1)      # [:, rho_prev, c] row-major
    return Z


# ----------------------------------------------------------------------------
# Leverage-score sampling (Sec. 3.2)
# ----------------------------------------------------------------------------
def leverage_scores(A):
    """l_i = ||A(i,:)||^2 for A with orthonormal columns (Def. leverage scores,
    Q = A).  Summed sequentially over columns, each square rounded before the
    add, so that the sampled indices are a deterministic function of A."""
    A = np.asarray(A, dtype=np.float64)
    ell = np.zeros(A.shape[0])
    for c in range(A.shape[1]):
        sq = A[:, c] * A[:, c]
        ell = ell + sq
    return ell


def leverage_sample(factors, m, seed, sweep, n):
    """Per-mode independent leverage sampling of the rows of kron_{k != n} A^(k)
    (Lemma on Kronecker leverage scores: p_i = prod_k p^(k)_{i_k}).

    For sample j and mode k, u = uniform(seed, LEV, sweep, n, k; j) and i_k is the
    first t with cdf_k[t] > u * cdf_k[-1] (cdf a sequential FP64 prefix sum of
    the scores).  p^(k) = l^(k) / sum(l^(k)); the row weight is
    w_j = 1 / sqrt(m * prod_k p^(k)_{i_k})  (Def. importance sampling, D(j,j)).
    Returns (idx int64[m, N-1] in increasing k, w float64[m])."""
    N = len(factors)
    ks = other_modes(N, n)
    idx = np.zeros((m, len(ks)), dtype=np.int64)
    prob = np.ones(m)
    j = np.arange(m)
    for t, k in enumerate(ks):
        ell = leverage_scores(factors[k])
        cdf = np.cumsum(ell)
        total = cdf[-1]
        u = rng.uniform(rng.draw(rng.stream_key(seed, rng.P_LEV, sweep, n, k), j))
        pos = np.searchsorted(cdf, u * total, side="right")
        pos = np.minimum(pos, ell.shape[0] - 1)
        idx[:, t] = pos
        prob = prob * (ell[pos] / total)
    w = 1.0 / np.sqrt(m * prob)
    return idx, w


def score_ranks(ell):
    """Position of every row in the order (score descending, index ascending)."""
    order = np.argsort(-np.asarray(ell), kind="stable")
    rank = np.empty(order.size, dtype=np.int64)
    rank[order] = np.arange(order.size)
    return rank


def leverage_select(factors, m, n):
    """Deterministic leverage sampling (Sec. 3.2: instead of drawing rows with
    probability proportional to their leverage scores, keep the rows with the
    largest scores).  The rows of kron_{k != n} A^(k) are the multi-indices
    (i_k)_{k != n}; by the Lemma on Kronecker leverage scores the score of a row
    is pi = prod_k l^(k)_{i_k} (multiplied in increasing k).  The m rows of
    largest pi are kept, in decreasing pi; rows of equal pi are ordered by their
    per-mode ranks (score_ranks), compared lexicographically in increasing k.
    No rescaling: every weight is 1.  Evaluated by brute force over all rows.
    Returns (idx int64[m, N-1] in increasing k, w float64[m] = 1)."""
    N = len(factors)
    ks = other_modes(N, n)
    ells = [leverage_scores(factors[k]) for k in ks]
    total = int(np.prod([e.size for e in ells]))
    if m > total:
        raise ValueError("more rows requested than the Kronecker chain has")
    grids = np.meshgrid(*[np.arange(e.size) for e in ells], indexing="ij")
    flat = [g.reshape(-1) for g in grids]
    pi = ells[0][flat[0]]
    for t in range(1, len(ells)):
        pi = pi * ells[t][flat[t]]
    ranks = [score_ranks(e)[f] for e, f in zip(ells, flat)]
    order = np.lexsort(ranks[::-1] + [-pi])[:m]
    idx = np.stack([f[order] for f in flat], 1).astype(np.int64)
    return idx, np.ones(m)


def leverage_lhs(factors, idx, w, n):
    """Z[j, :] = w_j * kron_{k != n} A^(k)(i_k, :)."""
    ks = other_modes(len(factors), n)
    Z = np.ones((idx.shape[0], 1))
    for t, k in enumerate(ks):
        rows = np.asarray(factors[k], dtype=np.float64)[idx[:, t]]
        Z = (Z[:, :, None] * rows[:, None, :]).reshape(idx.shape[0], -1)
    return Z * w[:, None]


def leverage_rhs_dense(X, idx, w, n):
    """Y[j, :] = w_j * T(i_1, .., i_{n-1}, :, i_{n+1}, ..) (the sampled mode-n fibers)."""
    X = np.asarray(X, dtype=np.float64)
    ks = other_modes(X.ndim, n)
    sel = [None] * X.ndim
    for t, k in enumerate(ks):
        sel[k] = idx[:, t]
    sel[n] = slice(None)
    # advanced indices separated by a slice: result is (m, s_n) when n is not
    # between them; build explicitly to keep the layout obvious
    Y = np.empty((idx.shape[0], X.shape[n]))
    for i in range(X.shape[n]):
        sel_i = list(sel)
        sel_i[n] = np.full(idx.shape[0], i)
        Y[:, i] = X[tuple(sel_i)]
    return Y * w[:, None]


def leverage_rhs_sparse(T, idx, w, n):
    """Sampled mode-n fibers of a COO tensor (duplicates summed)."""
    Tc = T.coalesced()
    ks = other_modes(T.order, n)
    key_T = other_linear_index(T.dims, Tc.idx, n)
    key_S = np.zeros(idx.shape[0], dtype=np.int64)
    for t, k in enumerate(ks):
        key_S = key_S * T.dims[k] + idx[:, t]
    s_n = T.dims[n]
    Y = np.zeros((idx.shape[0], s_n))
    order = np.argsort(key_T, kind="stable")
    ks_sorted = key_T[order]
    lo = np.searchsorted(ks_sorted, key_S, side="left")
    hi = np.searchsorted(ks_sorted, key_S, side="right")
    for j in range(idx.shape[0]):
        e = order[lo[j]:hi[j]]
        np.add.at(Y[j], Tc.idx[e, n], Tc.val[e])
    return Y * w[:, None]


# ----------------------------------------------------------------------------
# Composite sketch of the randomized range finder (Sec. 5)
# ----------------------------------------------------------------------------
def rrf_countsketch(T, n, k2, seed):
    """W = T_(n) Omega_cs^T: the CountSketch (hash g : [K] -> [k2], sign tau) of
    the K = prod_{k != n} s_k columns of the mode-n unfolding, g and tau drawn
    from the stream (seed, RRF, n) at the column's row-major linear index."""
    j = other_linear_index(T.dims, T.idx, n)
    x = rng.draw(rng.stream_key(seed, rng.P_RRF, n), j)
    g = rng.bucket(x, k2).astype(np.int64)
    tau = rng.sign(x)
    s_n = T.dims[n]
    return np.bincount(T.idx[:, n] * k2 + g, weights=tau * T.val,
                       minlength=s_n * k2).reshape(s_n, k2)


def rrf_gaussian(n, k1, k2, seed):
    """G in R^{k2 x k1} with i.i.d. N(0, 1/k1) entries (Def. composite sketch)."""
    c = np.arange(k2 * k1)
    return rng.gauss(rng.stream_key(seed, rng.P_RRF_G, n), c).reshape(k2, k1) / np.sqrt(k1)
