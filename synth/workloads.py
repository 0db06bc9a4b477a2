"""Named synthetic workloads (system + model + evaluation settings).

    water192      64-molecule periodic water box, 192 atoms, r_c = 5 A, no skin,
                  T = 2, the plain water model (K=8, 2x64 SiLU, weights N(0, 1/fan_in),
                  zero biases); small parity case.
    cu100800      FCC Cu-like crystal, a = 3.61 A, 30x30x28 cells = 100,800 atoms,
                  sigma = 0.1 A, r_c = 6 A with a 1 A skin, T = 3, Cu model
                  (K=12, 3x128 SiLU); the throughput workload.
    water1207296  water box of 402,432 molecules on a 48x64x131 site grid at the
                  reference spacing (1,207,296 atoms), r_c = 5 A, 1 A skin, split
                  2x2x2 into subdomains; water model with T_max = 6 for T sweeps.
"""
from __future__ import annotations

from . import models, systems

WATER_SPACING = systems.WATER_BOX_L / 4


def _water192(seed=0):
    return dict(system=systems.water_box(seed=seed), model=models.water_model_plain(T_max=2, seed=seed),
                T=2, skin=0.0, decomp=(1, 1, 1))


def _cu100800(seed=0):
    return dict(system=systems.fcc_crystal((30, 30, 28), seed=seed),
                model=models.cu_model(T_max=3, seed=seed), T=3, skin=1.0, decomp=(1, 1, 1))


def _water1207296(seed=0):
    return dict(system=systems.water_box(grid=(48, 64, 131), spacing=WATER_SPACING, seed=seed),
                model=models.water_model(T_max=6, seed=seed), T=3, skin=1.0, decomp=(2, 2, 2))


WORKLOADS = {"water192": _water192, "cu100800": _cu100800, "water1207296": _water1207296}


def workload(name: str, seed: int = 0) -> dict:
    return WORKLOADS[name](seed)
