"""Plain container for one steady-state solve request (raw inputs only)."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CELL_TYPES = ("tri3", "quad4", "tet4", "hex8")
BC_KINDS = ("thermalizing", "specular", "diffuse", "partial")


@dataclass
class Boundary:
    tag: int
    kind: str            # one of BC_KINDS
    T_wall: float = 0.0  # K, used by thermalizing walls
    specularity: float = 0.0  # p in [0,1], used by partial walls


@dataclass
class Problem:
    name: str
    dim: int
    xyz: np.ndarray          # (n_nodes, dim) float64, metres
    cell_type: str           # one of CELL_TYPES
    cells: np.ndarray        # (n_cells, nv) int64
    bfaces: np.ndarray       # (n_bf, nfv) int64
    bface_tag: np.ndarray    # (n_bf,) int32
    boundaries: list         # list[Boundary]
    C: np.ndarray            # (B,) J m^-3 K^-1
    v: np.ndarray            # (B,) m/s
    tau: np.ndarray          # (B,) s
    s: np.ndarray            # (D, 3) unit directions
    w: np.ndarray            # (D,) weights > 0
    Q: np.ndarray            # (n_cells,) W m^-3
    T_ref: float = 300.0
    scheme: str = "synthetic"     # sequential | synthetic | synthetic_literal
    precision: str = "mixed"      # fp64 | mixed
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return int(self.cells.shape[0])

    @property
    def n_bands(self):
        return int(self.C.shape[0])

    @property
    def n_dirs(self):
        return int(self.w.shape[0])

    @property
    def updates_per_sweep(self):
        return self.n_cells * self.n_bands * self.n_dirs
