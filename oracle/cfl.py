"""Stability limit of the explicit leapfrog (Sec. 3.1, eqs. full_d_dfl and
full_d_dal).

Source-free, the scheme is  E^{n+1} = E^n - dt^2 M K E^n + ...  with
K = C^T [*mu^-1] C on free edges, so a mode of M K with eigenvalue lam is
stable iff dt^2 lam <= 4: dt_max = 2 / sqrt(lam_max(M K)).  lam_max is found
by power iteration with a Rayleigh quotient (the paper gives only absolute
time steps; the limit itself is the standard leapfrog bound).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def curl_curl(topo, H):
    """K = C^T diag(H) C restricted to free edges (N1 x N1, zero elsewhere)."""
    F = sp.diags(topo.edge_free.astype(float))
    K = topo.C.T @ sp.diags(H) @ topo.C
    return (F @ K @ F).tocsr()


def cfl_dt(topo, H, M, iters=400, seed=0):
    K = curl_curl(topo, H)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(topo.n1) * topo.edge_free
    lam = 0.0
    for _ in range(iters):
        y = M @ (K @ x)
        lam = float(x @ y / (x @ x))
        x = y / np.linalg.norm(y)
    y = M @ (K @ x)
    lam = float(np.linalg.norm(y) / np.linalg.norm(x))
    return 2.0 / np.sqrt(lam), lam
