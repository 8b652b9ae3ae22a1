"""Line-of-sight geometry (oracle side).

* The object direction xhat = (x - o)/|x - o| from the observer o (Sec. II.B).
* (e_theta, e_phi) are the first two columns of the standard rotation S(xhat)
  that takes the 3-axis into xhat (App. E, eq. def_standard_rotation).  At
  the poles (sin theta = 0) phi is taken as 0; every estimator output is
  invariant under the choice because gamma e*_ij is basis independent.
* e_ij = e+_i e+_j with e+ = (e_theta + i e_phi)/sqrt(2) (Sec. II.B, eqs.
  def_of_eij_+2, def_polarization_vector); the estimators use its conjugate
  e*_ij.
"""
from __future__ import annotations

import numpy as np


def standard_rotation(xhat: np.ndarray) -> np.ndarray:
    """S(xhat) for each row of xhat: columns (e_theta, e_phi, xhat)."""
    ct = np.clip(xhat[:, 2], -1.0, 1.0)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    rho = np.hypot(xhat[:, 0], xhat[:, 1])
    safe = np.where(rho > 0, rho, 1.0)
    cp = np.where(rho > 0, xhat[:, 0] / safe, 1.0)
    sp = np.where(rho > 0, xhat[:, 1] / safe, 0.0)
    S = np.empty((xhat.shape[0], 3, 3))
    S[:, :, 0] = np.stack([ct * cp, ct * sp, -st], axis=1)
    S[:, :, 1] = np.stack([-sp, cp, np.zeros_like(cp)], axis=1)
    S[:, :, 2] = np.stack([st * cp, st * sp, ct], axis=1)
    return S


def los(pos: np.ndarray, observer) -> np.ndarray:
    r = pos - np.asarray(observer, dtype=np.float64)[None, :]
    return r / np.linalg.norm(r, axis=1)[:, None]


def basis(pos: np.ndarray, observer):
    """(xhat, e_theta, e_phi) per object."""
    xh = los(pos, observer)
    S = standard_rotation(xh)
    return xh, S[:, :, 0], S[:, :, 1]


def e_tensor(e_theta: np.ndarray, e_phi: np.ndarray) -> np.ndarray:
    """e_ij = e+_i e+_j, shape (n, 3, 3) complex."""
    ep = (e_theta + 1j * e_phi) / np.sqrt(2.0)
    return ep[:, :, None] * ep[:, None, :]
