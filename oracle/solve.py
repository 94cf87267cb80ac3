"""Rank-constrained sketched least squares (oracle side; test infrastructure only).

The mode-n subproblem of Tucker-ALS is  min_B 1/2 ||P B - T_(n)^T||  s.t.
rank(B) <= R (eq. tucker_ls); A^(n) are the right singular vectors of the
optimal B and C_(n)^T = B A^(n).  Sketched, it becomes min ||Z X - Y|| with
Z = S P, Y = S T_(n)^T.  Following the theorems of Sec. 4 (TensorSketch and
leverage-score rank-constrained LS), the sketched rank-constrained solution is
the best rank-R approximation of the sketched unconstrained solution
X_opt = Z^+ Y -- not the reduced-rank-regression minimiser of ||Z X - Y||.
"""
import numpy as np


def sign_fix(A):
    """Make the entry of largest magnitude of every column positive (first
    index on ties).  Returns (A_fixed, signs)."""
    A = np.array(A, dtype=np.float64, copy=True)
    if A.size == 0:
        return A, np.ones(A.shape[1])
    piv = np.argmax(np.abs(A), axis=0)
    s = np.where(A[piv, np.arange(A.shape[1])] < 0, -1.0, 1.0)
    return A * s[None, :], s


def rc_solve(Z, Y, R):
    """Exact sketched rank-constrained solve.

    X_opt = argmin_X ||Z X - Y||_F  (= Z^+ Y for full column rank Z),
    X_opt = U Sigma V^T,  A = V[:, :R] (sign-fixed),  W = X_opt A = C_(n)^T.
    Returns (A  s x R, W  r x R, X_opt  r x s)."""
    Z = np.asarray(Z, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    X = np.linalg.lstsq(Z, Y, rcond=None)[0]
    _, _, Vt = np.linalg.svd(X, full_matrices=False)
    A, _ = sign_fix(Vt[:R].T)
    W = X @ A
    return A, W, X


def rsvd_lrls(Z, Y, R, Omega):
    """RSVD-LRLS (Alg. 5): the randomized SVD, with the given Gaussian test
    matrix Omega (s x k, k = R + p), of the least-squares solution X = Z^+ Y.

    The range of X is captured by an orthonormal basis Q of X Omega; the SVD of
    the small k x s matrix Q^T X gives the approximate leading singular triplets
    of X: X ~ (Q U) Sigma V^T.  A^(n) = V_R (sign rule) and C_(n)^T = Q U_R Sigma_R.

    Returns (A = V[:, :R] sign-fixed, W = Q U_R Sigma_R with matching signs)."""
    Z = np.asarray(Z, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    X = np.linalg.lstsq(Z, Y, rcond=None)[0]                   # Z^+ Y, r x s
    Q = np.linalg.qr(X @ Omega)[0]                             # basis of range(X Omega)
    U, S, Vt = np.linalg.svd(Q.T @ X, full_matrices=False)
    A, sgn = sign_fix(Vt[:R].T)
    W = (Q @ U[:, :R]) * (S[:R] * sgn)[None, :]
    return A, W
