"""Float64 reference of the planner-side IG terms (Sec. IV) -- TEST INFRASTRUCTURE ONLY.

  G(x)  Eq. 3: inverse distance weighting of the perspectives' IG, summed over
        the N_B most recent information distributions (IDs) with weight
        1/(N_B - u) for ID u (u = 0 the oldest, u = N_B - 1 the newest);
        the distance power is p (p = 2 in the experiments).
  O(x)  orientation factor: cosine of the angle between the camera's viewing
        axis and the direction to the PoI, 0 when the PoI is outside the
        field of view (or behind the camera).
  c_I   sum over the horizon states of w_I / (O G + eps), eps = 1e-7.

Readings (the paper is silent): a query that coincides exactly with one or
more perspectives of an ID takes their mean IG for that ID (the limit of the
weighting); the field-of-view test is |x_c / z_c| <= tan(FoV_h/2) and
|y_c / z_c| <= tan(FoV_v/2) with z_c > 0 in camera coordinates.
"""

from __future__ import annotations

import numpy as np


def idw_one(query, pos, ig, p=2.0):
    """Eq. 3's inner ratio for one ID: sum g d^-p / sum d^-p."""
    q = np.asarray(query, dtype=np.float64)
    P = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    g = np.asarray(ig, dtype=np.float64)
    d = P - q
    same = np.all(d == 0.0, axis=1)
    if np.any(same):
        return float(np.mean(g[same]))
    r = np.sqrt(np.sum(d * d, axis=1))
    w = r ** (-p)
    return float(np.sum(g * w) / np.sum(w))


def interpolate(query, id_pos, id_ig, p=2.0):
    """G(x): id_pos [N_B, N_P, 3], id_ig [N_B, N_P], oldest first."""
    nb = id_pos.shape[0]
    return sum(idw_one(query, id_pos[u], id_ig[u], p) / (nb - u) for u in range(nb))


def orientation_factor(pose, poi, tan_h, tan_v):
    R = np.asarray(pose, dtype=np.float64)[:9].reshape(3, 3)
    t = np.asarray(pose, dtype=np.float64)[9:12]
    v = np.asarray(poi, dtype=np.float64) - t
    c = R.T @ v
    n = np.linalg.norm(v)
    if c[2] <= 0.0 or n == 0.0:
        return 0.0
    if abs(c[0] / c[2]) > tan_h or abs(c[1] / c[2]) > tan_v:
        return 0.0
    return float(c[2] / n)


def horizon_cost(poses, poi, tan_h, tan_v, id_pos, id_ig, p=2.0, w_i=1.0, eps=1e-7):
    """(G [K], O [K], c_I) for one horizon of K camera poses [K, 12]."""
    G = np.array([interpolate(q[9:12], id_pos, id_ig, p) for q in poses])
    O = np.array([orientation_factor(q, poi, tan_h, tan_v) for q in poses])
    return G, O, float(np.sum(w_i / (O * G + eps)))
