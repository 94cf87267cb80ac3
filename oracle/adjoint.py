"""Sketched mode-n residual and its gradients (oracle side; test infrastructure only).

L_n = || Z W A^T - Y ||_F^2 with Z = S^(n) P^(n) (TensorSketch of the Kronecker
chain of the other factors, Sec. 3.1), W = C_(n)^T, A = A^(n) and
Y = S^(n) T_(n)^T -- the sketched objective of the mode-n subproblem of Alg. 4
(twice the 1/2-scaled objective of eq. tucker_ls after sketching).

With E = Z W A^T - Y:
    dL/dA       = 2 E^T (Z W)
    dL/dW       = 2 Z^T (E A)             (reshaped to the core)
    dL/dZ       = 2 (E A) W^T
    dL/dCS_k[:, c] = sum_{rho : rho_k = c} Circ(Q_rho)^T dL/dZ[:, rho]
                 where Z[:, rho] = Circ(Q_rho) CS_k[:, c] and Q_rho is the circular
                 convolution of the other CountSketches CS_l[:, rho_l], l != n, k
    dL/dA^(k)[i, :] = sigma_k(i) dL/dCS_k[h_k(i), :]
"""
import numpy as np

from . import sketch, tucker


def _conv_columns(CS_list, m):
    """Columns rho (row-major over the list) of the circular convolution chain."""
    Z = np.zeros((m, 1))
    Z[0, 0] = 1.0
    for CS in CS_list:
        Z = np.stack([sketch.circulant(CS[:, c]) @ Z for c in range(CS.shape[1])],
                     axis=2).reshape(m, -1)
    return Z


def residual_and_grads(factors, core, tables, Y, m, n):
    N = len(factors)
    ks = sorted(tables)
    CS = {k: sketch.countsketch(factors[k], tables[k][0], tables[k][1], m) for k in ks}
    Z = _conv_columns([CS[k] for k in ks], m)
    W = tucker.core_to_W(np.asarray(core, dtype=np.float64), n)
    A = np.asarray(factors[n], dtype=np.float64)
    ZW = Z @ W
    E = ZW @ A.T - Y
    L = float(np.sum(E * E))
    EA = E @ A
    gA = 2.0 * E.T @ ZW
    gW = 2.0 * Z.T @ EA
    gZ = 2.0 * EA @ W.T
    ranks = [F.shape[1] for F in factors]
    grads = [None] * N
    grads[n] = gA
    shape = [ranks[k] for k in ks]
    for t, k in enumerate(ks):
        gCS = np.zeros_like(CS[k])
        for rho in np.ndindex(*shape):
            others = [CS[l][:, rho[u]:rho[u] + 1] for u, l in enumerate(ks) if l != k]
            q = _conv_columns(others, m)[:, 0]
            col = int(np.ravel_multi_index(rho, shape))
            gCS[:, rho[t]] += sketch.circulant(q).T @ gZ[:, col]
        h, sg = tables[k]
        grads[k] = sg[:, None] * gCS[h]
    gC = tucker.W_to_core(gW, ranks, n)
    return L, grads, gC


def residual(factors, core, tables, Y, m, n):
    ks = sorted(tables)
    CS = [sketch.countsketch(factors[k], tables[k][0], tables[k][1], m) for k in ks]
    Z = _conv_columns(CS, m)
    W = tucker.core_to_W(np.asarray(core, dtype=np.float64), n)
    E = Z @ W @ np.asarray(factors[n]).T - Y
    return float(np.sum(E * E))
