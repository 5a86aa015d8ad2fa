"""The paper's predictive load balancing in its continuous form (test
infrastructure only).

Sec. 5: with g_l^p the level-l workload of processor p, w_l^p the part of it
already done and s_l the number of level-l steps left in the coarse step, the
predicted remaining work on levels 0..l is
    eta_l^p = sum_{l' <= l} (s_l' g_l'^p - w_l'^p),
and level l is distributed as
    g_l^p = gbar_l - (eta_{l-1}^p - etabar_{l-1}) / s_l,
so that eta_l^p is the same for every p.  Bars are means over processors.
"""

import numpy as np


def eta(s, g, w):
    """eta_l^p for every level: s[l], g[l][p], w[l][p] -> array (L, P)."""
    g = np.asarray(g, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    terms = np.asarray(s, dtype=np.float64)[:, None] * g - w
    return np.cumsum(terms, axis=0)


def distribute(gbar, s_l, eta_prev):
    """g_l^p for one level, given eta_{l-1}^p (zeros for the first level)."""
    eta_prev = np.asarray(eta_prev, dtype=np.float64)
    return gbar - (eta_prev - eta_prev.mean()) / s_l


def successive(s, gbar, w, nproc):
    """Distribute levels 0..L-1 in order; returns g (L, P)."""
    L = len(s)
    g = np.zeros((L, nproc))
    w = np.asarray(w, dtype=np.float64)
    prev = np.zeros(nproc)
    for l in range(L):
        # the completed part enters eta with a minus sign, as in the paper
        g[l] = distribute(gbar[l], s[l], prev)
        prev = prev + s[l] * g[l] - w[l]
    return g


def window_targets(eta_cycles, gbar):
    """The one-window form used with launch cycles as processors (one step
    per window, s = 1): share of each cycle."""
    return distribute(gbar, 1.0, eta_cycles)
