"""CP decomposition on the Tucker core (oracle side; test infrastructure only).

* CP-ALS (Alg. 2): each subproblem (eq. subproblem) solved through the normal
  equations  A^(n) = MTTKRP(X, n) * pinv(hadamard_{k != n} A^(k)T A^(k))
  (Sec. 2.3); no column normalisation, no weights (the CP model of Sec. 2.3
  has none).
* CP-Sketch-Tucker (Alg. 6): sketched Tucker-ALS, CP-ALS on the core with the
  HOSVD of the core as initialisation (Sec. 7, CP experiments), and the
  products B^(n) A^(n).
"""
import numpy as np

from . import solve, tucker


def khatri_rao(mats):
    """Column-wise Kronecker product, rows row-major (last factor fastest)."""
    R = mats[0].shape[1]
    out = np.ones((1, R))
    for M in mats:
        out = (out[:, None, :] * M[None, :, :]).reshape(-1, R)
    return out


def mttkrp(X, factors, n):
    """X_(n) (khatri-rao_{k != n} A^(k)) -- the MTTKRP of Sec. 2.3."""
    others = [factors[k] for k in range(X.ndim) if k != n]
    return tucker.unfold(X, n) @ khatri_rao(others)


def cp_als(X, init_factors, sweeps):
    """Alg. 2 from the given initial factors."""
    X = np.asarray(X, dtype=np.float64)
    A = [np.array(F, dtype=np.float64) for F in init_factors]
    N = X.ndim
    for _ in range(sweeps):
        for n in range(N):
            G = np.ones((A[0].shape[1], A[0].shape[1]))
            for k in range(N):
                if k != n:
                    G = G * (A[k].T @ A[k])
            A[n] = mttkrp(X, A, n) @ np.linalg.pinv(G)
    return A


def cp_reconstruct(factors):
    R = factors[0].shape[1]
    X = 0
    for r in range(R):
        t = factors[0][:, r]
        for F in factors[1:]:
            t = np.multiply.outer(t, F[:, r])
        X = X + t
    return X


def cp_relative_residual(T, factors):
    """||T - sum_r a_r o b_r o ...||_F / ||T||_F."""
    if getattr(T, "dense", None) is not None:
        return float(np.linalg.norm(T.dense - cp_reconstruct(factors)) / np.linalg.norm(T.dense))
    Tc = T.coalesced()
    nT2 = float(np.dot(Tc.val, Tc.val))
    vals = np.ones((Tc.idx.shape[0], factors[0].shape[1]))
    for k, F in enumerate(factors):
        vals = vals * F[Tc.idx[:, k]]
    inner = float(np.dot(Tc.val, vals.sum(axis=1)))
    G = np.ones((factors[0].shape[1],) * 2)
    for F in factors:
        G = G * (F.T @ F)
    return float(np.sqrt(max(nT2 - 2 * inner + G.sum(), 0.0)) / np.sqrt(nT2))


def cp_sketch_tucker(T, cp_rank, tucker_ranks, m, tucker_sweeps, cp_sweeps, seed=0,
                     sketch_kind="lev", init="rrf", solve_kind="exact"):
    """Alg. 6: Tucker compression by Alg. 4 (subproblem solver solve_kind),
    CP-ALS on the core (HOSVD init), return the factors B^(n) A^(n) and the CP
    relative residual."""
    tk = tucker.sketch_tucker_als(T, tucker_ranks, m, tucker_sweeps, seed=seed,
                                  sketch_kind=sketch_kind, init=init, record_fit=False,
                                  solve_kind=solve_kind)
    C, B = tk["core"], tk["factors"]
    init_cp = tucker.hosvd(C, [cp_rank] * C.ndim)
    A = cp_als(C, init_cp, cp_sweeps)
    out = [B[n] @ A[n] for n in range(C.ndim)]
    return dict(factors=out, tucker=tk, core_factors=A, init=init_cp,
                fit=cp_relative_residual(T, out))
