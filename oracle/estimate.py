"""CPU oracle of the pose estimate (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never routes through it.

The paper takes as the pose estimate the weighted average of the particles, or
the particle of highest weight (§III), and computes the weighted sum of the
poses as a second GPU reduction (§V).  It does not say how rotations are
averaged.  Reading taken here, written out as its plain definition in float64:

  position  t* = sum_n w_n t_n / sum_n w_n
  rotation  R* = argmax over R in SO(3) of trace(R^T S),  S = sum_n w_n R_n,
            i.e. the rotation nearest to S in the Frobenius norm (the weighted
            chordal L2 mean).  Computed from the singular value decomposition
            S = U diag(s) V^T as R* = U diag(1, 1, det(U V^T)) V^T.
  best      the smallest index among the largest weights, and its pose.
  sum_n w_n = 0 is read as equal weights.

The particle matrices are taken as given (float32 values widened to float64),
orthonormal or not.
"""

from __future__ import annotations

import numpy as np


def weighted_sums(w: np.ndarray, poses: np.ndarray):
    """(sum w, S [3, 3], sum w t [3]) in float64, with the equal-weight reading."""
    w = np.asarray(w, np.float64)
    P = np.asarray(poses, np.float32).astype(np.float64)
    ws = float(w.sum())
    if not ws > 0.0:
        w = np.ones_like(w)
        ws = float(w.shape[0])
    S = (P[0:9] * w).sum(axis=1).reshape(3, 3)
    T = (P[9:12] * w).sum(axis=1)
    return ws, S, T


def nearest_rotation(S: np.ndarray) -> np.ndarray:
    """The rotation R maximising trace(R^T S) (the special orthogonal polar factor)."""
    U, _, Vt = np.linalg.svd(S)
    d = 1.0 if np.linalg.det(U @ Vt) >= 0.0 else -1.0
    return U @ np.diag([1.0, 1.0, d]) @ Vt


def best_particle(w: np.ndarray) -> int:
    """Smallest index of the largest weight; -1 if no weight exceeds -inf."""
    w = np.asarray(w, np.float64)
    ok = w > -np.inf            # NaN compares false
    if not ok.any():
        return -1
    m = w[ok].max()
    return int(np.flatnonzero(w == m)[0])


def pose_estimate(w: np.ndarray, poses: np.ndarray):
    """(mean float64 [12] in the particle layout r00..r22 tx ty tz, best index,
    best pose float32 [12] or None)."""
    ws, S, T = weighted_sums(w, poses)
    R = nearest_rotation(S)
    mean = np.concatenate([R.reshape(9), T / ws])
    b = best_particle(w)
    bp = np.asarray(poses, np.float32)[:, b].copy() if b >= 0 else None
    return mean, b, bp
