"""Tucker drivers (oracle side; test infrastructure only).

* Init-RRF (Alg. 3) with the composite sketch (Def. composite, Sec. 5)
* Sketch-Tucker-ALS (Alg. 4): C <- 0; RRF init of A^(2..N); I_max sweeps of the
  N sketched rank-constrained subproblems.  TensorSketch hashes are drawn once
  and the sketched right-hand sides are formed once ("preparation", Sec. 6.1);
  leverage samples are redrawn for every subproblem.
* HOOI (Alg. 1) with HOSVD initialisation -- the unsketched reference.
* relative residual ||T - T~||_F / ||T||_F  (= 1 - fitness, Sec. 7).
"""
import numpy as np

from . import rng, sketch, solve


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------
def unfold(X, n):
    """T_(n): rows i_n, columns the other modes row-major in increasing k."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def core_to_W(C, n):
    """W = C_(n)^T : rows (rho_k)_{k != n} row-major, columns rho_n."""
    return unfold(C, n).T


def W_to_core(W, ranks, n):
    other = [ranks[k] for k in range(len(ranks)) if k != n]
    return np.moveaxis(W.T.reshape([ranks[n]] + other), 0, n)


def kron_chain(mats):
    P = np.ones((1, 1))
    for M in mats:
        P = np.kron(P, M)
    return P


def reconstruct(C, factors):
    X = np.asarray(C, dtype=np.float64)
    for k, A in enumerate(factors):
        X = np.moveaxis(np.tensordot(A, X, axes=(1, k)), 0, k)
    return X


def values_at(C, factors, idx, chunk=1 << 16):
    """T~(i) = sum_rho C(rho) prod_k A^(k)(i_k, rho_k) at the given coordinates."""
    C = np.asarray(C, dtype=np.float64)
    out = np.empty(idx.shape[0])
    for lo in range(0, idx.shape[0], chunk):
        sl = slice(lo, lo + chunk)
        X = np.tensordot(factors[0][idx[sl, 0]], C, axes=(1, 0))   # (e, R2..RN)
        for k in range(1, len(factors)):
            X = np.einsum("er,er...->e...", factors[k][idx[sl, k]], X)
        out[sl] = X
    return out


def relative_residual(T, C, factors):
    """||T - T~||_F / ||T||_F with T~ = C x_1 A^(1) ... x_N A^(N)."""
    if getattr(T, "dense", None) is not None:
        D = T.dense - reconstruct(C, factors)
        return float(np.linalg.norm(D) / np.linalg.norm(T.dense))
    Tc = T.coalesced()
    nT2 = float(np.dot(Tc.val, Tc.val))
    inner = float(np.dot(Tc.val, values_at(C, factors, Tc.idx)))
    G = np.asarray(C, dtype=np.float64)
    for k, A in enumerate(factors):                      # ||T~||^2 = <C x_k A^T A, C>
        G = np.moveaxis(np.tensordot(A.T @ A, G, axes=(1, k)), 0, k)
    nR2 = float(np.sum(G * C))
    return float(np.sqrt(max(nT2 - 2.0 * inner + nR2, 0.0)) / np.sqrt(nT2))


# ----------------------------------------------------------------------------
# initialisations
# ----------------------------------------------------------------------------
def init_rrf(T, n, R, k1, k2, seed):
    """Init-RRF (Alg. 3) of mode n: the leading R left singular vectors
    (sign-fixed) of T_(n) sketched from the right by the composite sketch of
    Sec. 5 (a CountSketch to k2 columns followed by a k2 x k1 Gaussian map)."""
    Wcs = sketch.rrf_countsketch(T, n, k2, seed)
    G = sketch.rrf_gaussian(n, k1, k2, seed)
    B = Wcs @ G
    U, _, _ = np.linalg.svd(B, full_matrices=False)
    A, _ = solve.sign_fix(U[:, :R])
    return A


def init_random(s, R, n, seed):
    """Gaussian s x R matrix (stream (seed, INIT, n)), orthonormalised by QR and
    sign-fixed."""
    G = rng.gauss(rng.stream_key(seed, rng.P_INIT, n), np.arange(s * R)).reshape(s, R)
    Q, _ = np.linalg.qr(G)
    A, _ = solve.sign_fix(Q)
    return A


def hosvd(X, ranks):
    """HOSVD: A^(n) = leading R_n left singular vectors of X_(n) (sign-fixed)."""
    out = []
    for n, R in enumerate(ranks):
        U, _, _ = np.linalg.svd(unfold(X, n), full_matrices=False)
        out.append(solve.sign_fix(U[:, :R])[0])
    return out


def default_rrf_sizes(m, ranks, n):
    """k1 = ceil(sqrt(K) R), k2 = R^2 + k1 with K = m / prod_{k != n} R_k: the
    experiments' range-finder size sqrt(K) R (Sec. 7) and the composite-sketch
    orders k1 = O(R/eps), k2 = O(R^2 + R/eps) with unit constants."""
    r = int(np.prod([ranks[k] for k in range(len(ranks)) if k != n]))
    K = m / r
    R = ranks[n]
    k1 = int(np.ceil(np.sqrt(K) * R - 1e-9))
    return k1, R * R + k1


# ----------------------------------------------------------------------------
# Sketch-Tucker-ALS (Alg. 4)
# ----------------------------------------------------------------------------
def rsvd_width(R, r, p=10):
    """Columns of the Gaussian test matrix of RSVD-LRLS: O(R) read as R + p
    (oversampling p = 10), at most r (the rank of Z^+ Y is at most r)."""
    return min(R + p, r)


def rsvd_omega(seed, sweep, n, s, k):
    """Gaussian test matrix of subproblem (sweep, n): s x k, row-major draws of
    the stream (seed, RSVD, sweep, n)."""
    return rng.gauss(rng.stream_key(seed, rng.P_RSVD, sweep, n), np.arange(s * k)).reshape(s, k)


def sketch_tucker_als(T, ranks, m, sweeps, seed=0, sketch_kind="ts", init="rrf",
                      rrf_k1=0, rrf_k2=0, init_factors=None, record_fit=True,
                      identity_sketch=False, solve_kind="exact", rsvd_p=10, first_sweep=0):
    """Sketched Tucker-ALS, Alg. 4.

    T        oracle.sketch.Tensor (COO or dense)
    ranks    Tucker ranks (R_1..R_N)
    m        sketch size (rows of every sketched subproblem)
    sketch_kind  "ts" (TensorSketch), "lev" (leverage-score sampling) or
             "lev_det" (deterministic leverage selection, weights 1)
    init     "rrf" (Alg. 3 for n = 2..N), "random" or "user" (init_factors)
    identity_sketch  replace S^(n) by the identity (then each subproblem is
             exactly the HOOI update) -- used to pin the driver to Alg. 1.
    solve_kind  "exact" (truncated SVD of Z^+ Y) or "rsvd" (RSVD-LRLS, Alg. 5,
             the subproblem solver Alg. 4 calls, with a fresh Gaussian test
             matrix of rsvd_width(R, r, rsvd_p) columns per subproblem)
    first_sweep  index of the first sweep in the per-sweep random streams
             (leverage samples, RSVD test matrices), so that a run can resume
             at that sweep from given factors (init="user")

    Returns dict(core, factors, fits, samples)."""
    N = T.order
    dims = T.dims
    factors = [None] * N
    # Alg. 4 initialises modes 2..N (zero-based 1..N-1) before the first sweep
    if init == "user":
        factors = [np.array(A, dtype=np.float64) for A in init_factors]
    else:
        for n in range(1, N):
            if init == "rrf":
                k1, k2 = default_rrf_sizes(m, ranks, n)
                k1 = rrf_k1 or k1
                k2 = rrf_k2 or k2
                factors[n] = init_rrf(T, n, ranks[n], k1, k2, seed)
            else:
                factors[n] = init_random(dims[n], ranks[n], n, seed)
    core = np.zeros(ranks)

    Xd = T.to_dense() if (identity_sketch or sketch_kind in ("lev", "lev_det")) and \
        getattr(T, "dense", None) is not None else None
    # TensorSketch: S^(n) drawn once and Y^(n) formed once (preparation cost)
    tables, Ys = {}, {}
    if sketch_kind == "ts" and not identity_sketch:
        for n in range(N):
            tables[n] = sketch.ts_tables(dims, m, seed, n)
            Ys[n] = sketch.ts_rhs(T, m, tables[n], n)
    fits, samples = [], []
    for sweep in range(first_sweep, first_sweep + sweeps):
        for n in range(N):
            if identity_sketch:
                P = kron_chain([factors[k] for k in range(N) if k != n])
                Z, Y = P, unfold(T.to_dense(), n).T
            elif sketch_kind == "ts":
                Z = sketch.ts_lhs(factors, tables[n], m, n)
                Y = Ys[n]
            else:
                if sketch_kind == "lev_det":
                    idx, w = sketch.leverage_select(factors, m, n)
                else:
                    idx, w = sketch.leverage_sample(factors, m, seed, sweep, n)
                samples.append((sweep, n, idx, w))
                Z = sketch.leverage_lhs(factors, idx, w, n)
                Y = sketch.leverage_rhs_dense(Xd, idx, w, n) if Xd is not None \
                    else sketch.leverage_rhs_sparse(T, idx, w, n)
            if solve_kind == "rsvd":
                r = Z.shape[1]
                Om = rsvd_omega(seed, sweep, n, dims[n], rsvd_width(ranks[n], r, rsvd_p))
                A, W = solve.rsvd_lrls(Z, Y, ranks[n], Om)
            else:
                A, W, _ = solve.rc_solve(Z, Y, ranks[n])
            factors[n] = A
            core = W_to_core(W, ranks, n)
        if record_fit:
            fits.append(relative_residual(T, core, factors))
    return dict(core=core, factors=factors, fits=fits, samples=samples)


# ----------------------------------------------------------------------------
# HOOI (Alg. 1)
# ----------------------------------------------------------------------------
def hooi(X, ranks, sweeps, init_factors=None):
    """Tucker-ALS / HOOI, Alg. 1: Y^(n) = T x_{k != n} A^(k)T (eq. Yn),
    A^(n) <- leading R_n left singular vectors of Y^(n)_(n) (sign-fixed);
    C <- Y^(N) x_N A^(N)T after each sweep."""
    X = np.asarray(X, dtype=np.float64)
    N = X.ndim
    factors = [np.array(A) for A in init_factors] if init_factors is not None \
        else hosvd(X, ranks)
    fits = []
    for _ in range(sweeps):
        for n in range(N):
            Yn = X
            for k in range(N):
                if k != n:
                    Yn = np.moveaxis(np.tensordot(factors[k].T, Yn, axes=(1, k)), 0, k)
            U, _, _ = np.linalg.svd(unfold(Yn, n), full_matrices=False)
            factors[n] = solve.sign_fix(U[:, :ranks[n]])[0]
        C = np.moveaxis(np.tensordot(factors[N - 1].T, Yn, axes=(1, N - 1)), 0, N - 1)
        fits.append(float(np.linalg.norm(X - reconstruct(C, factors)) / np.linalg.norm(X)))
    return dict(core=C, factors=factors, fits=fits)
