"""Workload definitions (sizes of the synthetic stand-ins for the paper's workloads).

Rock-salt (001) slabs with a = 5.64 A and +-0.7 e stand in for NaCl; synthetic
chain / planar polyaromatic / size-series molecules stand in for PTCDA and
xylitol.  Grid spacing 0.1 A as in the paper's CPU tests; z origin 1 A above the
top atomic plane.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import synth


@dataclass(frozen=True)
class GridCfg:
    n_cells: int
    n_planes: int
    nx: int
    ny: int
    nz: int
    z0: float = 1.0            # above the top plane (z_top = 0)
    dz: float = 0.1
    alpha: float = synth.ALPHA
    rcut: float = 17.0
    vacancy: tuple = ()        # (i, j, plane) sites removed from the slab

    def substrate(self):
        return synth.rocksalt_slab(self.n_cells, self.n_planes, vacancy=list(self.vacancy))


# 2x2 conventional cells, 3 atomic planes (48 atoms), 112 x 112 x 150 nodes
GRID_SMALL = GridCfg(2, 3, 112, 112, 150)
# 8x8 conventional cells, 12 atomic planes (3072 atoms), 452 x 452 x 200 nodes
GRID_LARGE = GridCfg(8, 12, 452, 452, 200)
# a neutral point defect in a large supercell (the paper's dragging-over-a-defect case):
# 20x20 conventional cells, 3 planes, one adjacent cation-anion pair removed from the top
# plane at the cell centre (4798 atoms); 1128 x 1128 x 80 nodes (112.8 x 112.8 x 7.9 A,
# 1.69 GB in FP32), and the same supercell without the defect
GRID_DEFECT = GridCfg(20, 3, 1128, 1128, 80, vacancy=((20, 20, 0), (21, 20, 0)))
GRID_DEFECT_PRISTINE = GridCfg(20, 3, 1128, 1128, 80)


@dataclass(frozen=True)
class Workload:
    name: str
    grid: GridCfg
    molecules: str            # synth.molecule_types key
    n_rep: int
    mode: str                 # "fire" | "nve"
    n_steps: int
    storage: str = "f32"


C1_CHAIN_FIRE = Workload("chain24-fire-256", GRID_SMALL, "chain24", 256, "fire", 1000)
C2_PAH_NVE = Workload("pah38-nve-16384", GRID_SMALL, "pah38", 16384, "nve", 5000)
C3_SIZES_FIRE = Workload("sizes-fire-4096", GRID_SMALL, "sizes", 4096, "fire", 1000)
C5_PAH_FIRE_LARGE = Workload("pah38-fire-65536-large", GRID_LARGE, "pah38", 65536, "fire", 2000)
