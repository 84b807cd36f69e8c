"""Slice potentials: Fourier coefficients of sums of Gaussian wells.

The local potential is taken as z-independent inside each thin slice
(Sec. II.A, the slicing along the transport direction).  Here the slice
potential is the z-average of a sum of 3D Gaussian wells

    V(r) = - sum_w D_w exp(-|r - c_w|^2 / (2 sigma_w^2)),

periodic in the transverse plane and truncated to the junction slab
(V = 0 in both leads).  Its transverse Fourier coefficients, with the
convention V(r_perp) = sum_Q V(Q) exp(i Q . r_perp), follow in closed form
from the 2D Gaussian transform (transverse periodic images by Poisson
summation) and the erf integral of the Gaussian over the slice:

    V^p(Q) = -(1/A) sum_w D_w 2 pi sigma_w^2 exp(-sigma_w^2 |Q|^2 / 2)
             exp(-i Q . c_w,perp) zeta_w^p,
    zeta_w^p = sigma_w sqrt(pi/2) / dz_p
               [erf((z_p - c_wz)/(sqrt2 sigma_w)) - erf((z_{p-1} - c_wz)/(sqrt2 sigma_w))].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erf


@dataclass
class Wells:
    """Gaussian wells: centres (W, 3) bohr, depths (W,) Ry (positive = attractive), widths (W,) bohr."""

    centres: np.ndarray
    depth: np.ndarray
    sigma: np.ndarray

    def __post_init__(self):
        self.centres = np.atleast_2d(np.asarray(self.centres, dtype=np.float64))
        w = self.centres.shape[0]
        self.depth = np.broadcast_to(np.asarray(self.depth, dtype=np.float64), (w,)).copy()
        self.sigma = np.broadcast_to(np.asarray(self.sigma, dtype=np.float64), (w,)).copy()


def slice_edges(dz) -> np.ndarray:
    """z_0 = 0, z_p = z_{p-1} + dz_p (reference planes at the right end of each slice)."""
    dz = np.asarray(dz, dtype=np.float64)
    return np.concatenate([[0.0], np.cumsum(dz)])


def vq_gaussian_wells(cell, q_miller, wells: Wells, dz, vconst=0.0) -> np.ndarray:
    """V^p(Q) for every slice p and difference vector Q: (n_slices, n_q) complex128.

    ``vconst`` (scalar or (n_slices,)) adds a z-dependent constant V_c(p) at Q = 0.
    """
    b = cell.bvec
    qv = np.asarray(q_miller, dtype=np.float64) @ b            # (n_q, 2)
    q2 = np.sum(qv * qv, axis=1)
    z = slice_edges(dz)
    dz = np.asarray(dz, dtype=np.float64)
    out = np.zeros((dz.size, qv.shape[0]), dtype=np.complex128)
    for c, d, s in zip(wells.centres, wells.depth, wells.sigma):
        e = erf((z - c[2]) / (np.sqrt(2.0) * s))
        zeta = s * np.sqrt(np.pi / 2.0) * (e[1:] - e[:-1]) / dz          # (n_slices,)
        form = -(d / cell.area) * 2.0 * np.pi * s * s * np.exp(-0.5 * s * s * q2) \
            * np.exp(-1j * (qv @ c[:2]))                                  # (n_q,)
        out += zeta[:, None] * form[None, :]
    q0 = np.where((np.asarray(q_miller) == 0).all(axis=1))[0]
    if q0.size:
        out[:, q0[0]] += np.broadcast_to(np.asarray(vconst, dtype=np.float64), (dz.size,))
    return out
