"""The synthetic junction workloads.

They stand in for the paper's graphene side-contact junctions (Sec. II.B and
Fig. 1 geometry; self-consistent DFT potentials are not available), with the
shapes, sizes and sampling of that problem:

* ``config1``  square cell a = 5 bohr, 4 seeded Gaussian wells, N_G = 37,
  24 slices of 0.25 bohr, 8 energies at k_par = 0 (the small case).
* ``config2``  hexagonal 2x2 graphene-like supercell, two sheets normal to z
  6.3 bohr apart in AA or AB registry, N_G = 300, 160 slices of 0.1 bohr,
  64 energies x 16 k_par.
* ``config3``  rectangular 4.65 x 40 bohr cell holding two graphene-like
  sheets normal to y whose edges overlap 15 bohr along the transport
  direction z, vacuum gap {5.0, 6.3, 7.5} bohr, N_G = 1200, 400 slices of
  0.05 bohr, 32 energies x 8 k_par (k_x only).
* ``config4_instances``  512 uneven (N_G, slice count, E, k_par) instances
  drawn from the config-2 geometry.
* ``config5``  config 3 at gap 6.3 bohr, k_par = 0, 16 energies.

Free-electron leads (V = 0) on both sides throughout.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lattice import Cell, plane_wave_basis, difference_set
from .potential import Wells, vq_gaussian_wells

# carbon-carbon distance of the graphene-like sheets and their zigzag period
_A_GR = 4.65
_D_CC = _A_GR / np.sqrt(3.0)


@dataclass
class Junction:
    name: str
    cell: Cell
    wells: Wells
    dz: np.ndarray
    energies: np.ndarray
    kpars: np.ndarray
    n_g: int
    meta: dict = field(default_factory=dict)

    @property
    def n_slices(self) -> int:
        return int(np.asarray(self.dz).size)

    @property
    def length(self) -> float:
        return float(np.sum(self.dz))


def junction_inputs(j: Junction, kpar, n_g: int | None = None, vconst=0.0) -> dict:
    """Arrays both the oracle and the library consume for one k_par."""
    n_g = j.n_g if n_g is None else n_g
    kpar = np.asarray(kpar, dtype=np.float64)
    miller = plane_wave_basis(j.cell, kpar, n_g)
    q_miller, q_of_ij = difference_set(miller)
    vq = vq_gaussian_wells(j.cell, q_miller, j.wells, j.dz, vconst=vconst)
    return dict(miller=miller, q_miller=q_miller, q_of_ij=q_of_ij, vq=vq,
                dz=np.asarray(j.dz, dtype=np.float64).copy(), bvec=j.cell.bvec,
                kpar=kpar, area=j.cell.area)


def config1(seed: int = 1) -> Junction:
    rng = np.random.default_rng(seed)
    a, zlen = 5.0, 6.0
    centres = rng.uniform(size=(4, 3)) * np.array([a, a, zlen])
    depth = rng.uniform(0.5, 1.0, size=4)
    return Junction("config1", Cell((a, 0.0), (0.0, a)), Wells(centres, depth, 0.8),
                    np.full(24, 0.25), np.linspace(0.1, 1.0, 8), np.zeros((1, 2)), 37,
                    dict(seed=seed))


def _hex_sheet(shift=(0.0, 0.0)):
    p1 = np.array([_A_GR, 0.0])
    p2 = np.array([_A_GR / 2, _A_GR * np.sqrt(3.0) / 2])
    out = []
    for i in range(2):
        for j in range(2):
            for basis in (np.zeros(2), (p1 + p2) / 3.0):
                out.append(i * p1 + j * p2 + basis + np.asarray(shift))
    return np.array(out)


def config2(registry: str = "AA", n_g: int = 300, n_slices: int = 160) -> Junction:
    big = 2 * _A_GR
    cell = Cell((big, 0.0), (big / 2, big * np.sqrt(3.0) / 2))
    zlen = 16.0
    z_bot, z_top = zlen / 2 - 3.15, zlen / 2 + 3.15
    p1 = np.array([_A_GR, 0.0])
    p2 = np.array([_A_GR / 2, _A_GR * np.sqrt(3.0) / 2])
    bot = _hex_sheet()
    top = _hex_sheet((p1 + p2) / 3.0 if registry == "AB" else (0.0, 0.0))
    centres = np.concatenate([np.c_[bot, np.full(8, z_bot)], np.c_[top, np.full(8, z_top)]])
    b = cell.bvec
    f = np.array([-3, -1, 1, 3]) / 16.0
    kpars = np.array([f1 * b[0] + f2 * b[1] for f1 in f for f2 in f])
    return Junction(f"config2-{registry}", cell, Wells(centres, 1.2, 0.6),
                    np.full(n_slices, zlen / n_slices), np.linspace(0.1, 1.0, 64), kpars, n_g,
                    dict(registry=registry))


def _zigzag_sheet(y, zlo, zhi, zshift=0.0):
    """Graphene-like sheet in the (x, z) plane: zigzag rows along x (period 4.65 bohr)."""
    pts = []
    for n in range(-4, 40):
        for dzr in (0.0, _D_CC):
            z = 1.5 * _D_CC * n + dzr + zshift
            if zlo - 1e-9 <= z <= zhi + 1e-9:
                pts.append(((n % 2) * _A_GR / 2, y, z))
    return np.array(pts)


def config3(gap: float = 6.3, registry: str = "AA", n_g: int = 1200, n_slices: int = 400,
            n_e: int = 32) -> Junction:
    lx, ly, zlen = _A_GR, 40.0, 20.0
    cell = Cell((lx, 0.0), (0.0, ly))
    bot = _zigzag_sheet(ly / 2 - gap / 2, 0.0, 17.5)
    top = _zigzag_sheet(ly / 2 + gap / 2, 2.5, zlen, zshift=_D_CC if registry == "AB" else 0.0)
    centres = np.concatenate([bot, top])
    b1 = cell.bvec[0]
    f = np.array([-7, -5, -3, -1, 1, 3, 5, 7]) / 32.0
    kpars = np.array([fi * b1 for fi in f])
    return Junction(f"config3-gap{gap}-{registry}", cell, Wells(centres, 1.2, 0.6),
                    np.full(n_slices, zlen / n_slices), np.linspace(0.1, 1.0, n_e), kpars, n_g,
                    dict(gap=gap, registry=registry))


def config3_electrode(side: str = "bottom", gap: float = 6.3, registry: str = "AA", n_g: int = 1200,
                      n_slices: int = 160) -> Junction:
    """One z-period (3 d_cc = 8.05 bohr) of a config-3 sheet continued along z: the periodic
    electrode cell of the bottom sheet (``side="bottom"``, y = 20 - gap/2) or of the top one
    (y = 20 + gap/2, shifted by d_cc along z for the AB registry), with the wells of the
    neighbouring periods included so the potential is periodic.  Same transverse cell and
    basis size as config 3."""
    lx, ly = _A_GR, 40.0
    period = 3.0 * _D_CC
    cell = Cell((lx, 0.0), (0.0, ly))
    y = ly / 2 - gap / 2 if side == "bottom" else ly / 2 + gap / 2
    zs = _D_CC if (side == "top" and registry == "AB") else 0.0
    centres = _zigzag_sheet(y, -period - 1e-9, 2.0 * period, zshift=zs - 6 * period)
    return Junction(f"config3-electrode-{side}-gap{gap}-{registry}", cell, Wells(centres, 1.2, 0.6),
                    np.full(n_slices, period / n_slices), np.linspace(0.1, 1.0, 32), np.zeros((1, 2)), n_g,
                    dict(gap=gap, registry=registry, side=side, period=period))


def config4_instances(n: int = 512, seed: int = 4):
    """Uneven instances from the config-2 geometry: list of dicts (junction, E, k_par index)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        n_g = int(rng.choice([200, 450, 800, 1200]))
        ns = int(rng.integers(100, 401))
        reg = "AA" if rng.integers(0, 2) == 0 else "AB"
        j = config2(reg, n_g=n_g, n_slices=ns)
        out.append(dict(junction=j, energy=float(rng.uniform(0.1, 1.0)),
                        k_index=int(rng.integers(0, 16))))
    return out


def config5() -> Junction:
    j = config3(6.3, "AA", n_e=16)
    j.kpars = np.zeros((1, 2))
    j.name = "config5"
    return j


CONFIGS = {"config1": config1, "config2": config2, "config3": config3, "config5": config5}
