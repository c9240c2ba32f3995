"""Activation-time map of a space-time solution (oracle).

The paper studies how the conductivity perturbation changes the activation
map (abstract, Sec. 1) without a formula for it.  Reading used here: the
activation time of a node is the first time the potential reaches the
threshold (0.5, midway between rest 0 and peak 1), located by linear
interpolation in time between the two backward-Euler time levels that bracket
the first up-crossing.  A node already at or above threshold at t = 0 has
activation time 0; a node that never reaches it is censored at T.

Test infrastructure only (see the package docstring).
"""

import numpy as np


def activation_map(u0, U, dt, threshold=0.5):
    """Return (t_act (n,), n_censored) for initial state u0 (n,) and U (m, n).

    Plain per-node scan in time order.
    """
    m, n = U.shape
    T = m * dt
    t_act = np.empty(n)
    censored = 0
    for i in range(n):
        if u0[i] >= threshold:
            t_act[i] = 0.0
            continue
        prev = u0[i]
        for k in range(m):
            cur = U[k, i]
            if cur >= threshold:
                t_act[i] = k * dt + dt * (threshold - prev) / (cur - prev)
                break
            prev = cur
        else:
            t_act[i] = T
            censored += 1
    return t_act, censored
