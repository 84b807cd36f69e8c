"""Transverse lattice, plane-wave basis selection and difference-vector map.

The transverse (x, y) plane is periodic with lattice vectors a1, a2; wave
functions are expanded in plane waves exp(i (k_par + G) . r_perp) with
G = m1 b1 + m2 b2 (Sec. II.A, the two-dimensional plane-wave basis of N_2D
reciprocal vectors G_perp).  The basis keeps the N vectors of lowest
|k_par + G|^2; ties at a partly filled shell are broken by (m1, m2) so the
choice is deterministic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Cell:
    """2D Bravais cell.  a1, a2 in bohr (2-vectors)."""

    a1: tuple
    a2: tuple

    @property
    def avec(self) -> np.ndarray:
        return np.array([self.a1, self.a2], dtype=np.float64)

    @property
    def area(self) -> float:
        a = self.avec
        return float(abs(a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]))

    @property
    def bvec(self) -> np.ndarray:
        """Reciprocal vectors b1, b2 (rows) with a_i . b_j = 2 pi delta_ij."""
        return 2.0 * np.pi * np.linalg.inv(self.avec).T


def plane_wave_basis(cell: Cell, kpar, n: int) -> np.ndarray:
    """Miller indices (n, 2) int32 of the n lowest |k_par + G|^2.

    Sort key: (|k_par+G|^2 rounded to 1e-9, m1, m2).  The enumeration box is
    checked to contain every vector up to the cut-off shell.
    """
    kpar = np.asarray(kpar, dtype=np.float64)
    b = cell.bvec
    # radius that holds ~n reciprocal points, with a margin
    rad = np.sqrt(4.0 * np.pi * n / cell.area) * 1.5 + np.linalg.norm(kpar) + 2 * np.linalg.norm(b, axis=1).max()
    a = cell.avec
    mmax = [int(np.ceil(rad * np.linalg.norm(a[i]) / (2 * np.pi))) + 2 for i in range(2)]
    m1, m2 = np.meshgrid(np.arange(-mmax[0], mmax[0] + 1), np.arange(-mmax[1], mmax[1] + 1), indexing="ij")
    m1 = m1.ravel()
    m2 = m2.ravel()
    g = m1[:, None] * b[0] + m2[:, None] * b[1]
    q = np.sum((kpar + g) ** 2, axis=1)
    order = np.lexsort((m2, m1, np.round(q, 9)))
    if n > order.size:
        raise ValueError("basis enumeration box too small")
    keep = order[:n]
    qcut = q[keep[-1]]
    edge = (np.abs(m1) == mmax[0]) | (np.abs(m2) == mmax[1])
    if np.any(q[edge] <= qcut + 1e-9):
        raise ValueError("basis enumeration box does not contain the cut-off shell")
    return np.stack([m1[keep], m2[keep]], axis=1).astype(np.int32)


def difference_set(miller: np.ndarray):
    """Distinct differences G_i - G_j of the basis.

    Returns (q_miller (n_q, 2) int32, q_of_ij (n, n) int32) with
    q_miller[q_of_ij[i, j]] = miller[i] - miller[j].
    """
    miller = np.asarray(miller, dtype=np.int64)
    d = miller[:, None, :] - miller[None, :, :]
    flat = d.reshape(-1, 2)
    uniq, inv = np.unique(flat, axis=0, return_inverse=True)
    return uniq.astype(np.int32), inv.reshape(miller.shape[0], miller.shape[0]).astype(np.int32)
