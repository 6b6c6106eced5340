"""Tucker completion: model values, loss and gradient (oracle; test infrastructure only).

Not in the paper: the differentiation form applies the Tucker model of
Section 2.2 (T ~ G x_1 F_1 ... x_N F_N) to a list of observed coordinates.
For observation e with coordinates (l_1..l_N) the model value is

    m_e = sum_c G[c_1..c_N] prod_n F_n[l_n, c_n],

the loss is L = sum_e (m_e - v_e)^2, and with r_e = m_e - v_e the gradient is

    dL/dG[c]        = 2 sum_e r_e prod_n F_n[l_n(e), c_n]
    dL/dF_n[i, c_n] = 2 sum_{e : l_n(e) = i} r_e * (G x_{j != n} F_j[l_j(e), :])[c_n].

The second line is the Kronecker reformulation (eq. 1) run with values 2 r_e
and the result multiplied by G_(n)^T.  All FP64.
"""
from __future__ import annotations

import numpy as np


def _kron_all(factors, idx, e, skip=None):
    kr = np.ones((len(e), 1))
    for j, f in enumerate(factors):
        if j == skip:
            continue
        rows = np.asarray(f, np.float64)[np.asarray(idx[j])[e]]
        kr = (rows[:, :, None] * kr[:, None, :]).reshape(len(e), -1)
    return kr


def model_values(G, factors, idx, chunk=1 << 14):
    G = np.asarray(G, np.float64)
    g = G.ravel(order="F")
    n_obs = np.asarray(idx[0]).shape[0]
    out = np.empty(n_obs)
    for a in range(0, n_obs, chunk):
        e = np.arange(a, min(a + chunk, n_obs))
        out[e] = _kron_all(factors, idx, e) @ g
    return out


def loss(G, factors, idx, vals):
    r = model_values(G, factors, idx) - np.asarray(vals, np.float64)
    return float(r @ r)


def gradient(G, factors, idx, vals=None, g=None, chunk=1 << 14):
    """(dG, [dF_n]) of L = sum (m_e - v_e)^2, or of sum_e g_e m_e when the
    upstream gradient g is given instead of vals."""
    G = np.asarray(G, np.float64)
    K = G.shape
    N = len(factors)
    if g is None:
        g = 2.0 * (model_values(G, factors, idx) - np.asarray(vals, np.float64))
    g = np.asarray(g, np.float64)
    n_obs = g.shape[0]
    dG = np.zeros(int(np.prod(K)))
    dF = [np.zeros_like(np.asarray(f, np.float64)) for f in factors]
    for a in range(0, n_obs, chunk):
        e = np.arange(a, min(a + chunk, n_obs))
        dG += g[e] @ _kron_all(factors, idx, e)
        for n in range(N):
            # G_(n): K_n x prod_{j != n} K_j with the first remaining mode fastest
            Gn = np.moveaxis(G, n, 0).reshape(K[n], -1, order="F")
            contrib = (g[e, None] * _kron_all(factors, idx, e, skip=n)) @ Gn.T   # (e, K_n)
            np.add.at(dF[n], np.asarray(idx[n])[e], contrib)
    return dG.reshape(K, order="F"), dF
