"""The five benchmark workloads (seeded, synthetic).

C1  rotated surface-code Z-memory d=3, 3 rounds, p=1e-3, 16,384 shots
C2  rotated surface-code Z-memory d=11, 11 rounds, p=1e-3, 2^24 shots (pure frame)
C3  near-Clifford n=20, 400 layers, 24 pi/8 rotations, 60 measurements, p=5e-4, peak width 8, 2^20 shots
C4  128 near-Clifford programs, n = 12..40, peak widths 1..12, shots log-uniform 2^10..2^18
C5  near-Clifford n=48, 400 layers, 80 rotations, 200 measurements, p=5e-4, peak width 14 (and a
    variant peaking at 16), 2^16 shots
POST  coherent-noise surface code d=5, 5 rounds, exp(-i 0.1 Z / 2) on every data qubit each round,
    p=1e-3, peak width 12, every detector postselected (aggregate counts), 2^18 shots

Sampling seeds are 0x5EED0000 + config number.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass
from functools import lru_cache
from typing import List, Tuple

from . import near_clifford as nc
from .circuit import Circuit
from .distill import distill_15to1
from .surface import rotated_memory_z

_SEEDS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "seeds.json")


@lru_cache(maxsize=1)
def _seeds():
    with open(_SEEDS) as f:
        return json.load(f)


@dataclass
class Workload:
    name: str
    circuit: Circuit
    shots: int
    seed: int


def c1() -> Workload:
    return Workload("surface_d3_r3_p1e-3", rotated_memory_z(3, 3, 1e-3), 16384, 0x5EED0001)


def c2(shots: int = 1 << 24) -> Workload:
    return Workload("surface_d11_r11_p1e-3", rotated_memory_z(11, 11, 1e-3), shots, 0x5EED0002)


def c3(shots: int = 1 << 20) -> Workload:
    return Workload("near_clifford_n20_k8", nc.c3(_seeds()["c3"]), shots, 0x5EED0003)


def c4() -> List[Workload]:
    out = []
    for i, s in enumerate(_seeds()["c4"]):
        n, k, shots = nc.c4_params(i)
        out.append(Workload(f"batch_{i}_n{n}_k{k}", nc.c4_program(i, s), shots, 0x5EED0004 + (i << 32)))
    return out


def c5(k: int = 14, shots: int = 1 << 16) -> Workload:
    key = "c5_k14" if k == 14 else "c5_k16"
    return Workload(f"near_clifford_n48_k{k}", nc.c5(_seeds()[key], k), shots, 0x5EED0005)


def postselect() -> Workload:
    return Workload("coherent_surface_d5_r5_theta0.1_postselect", rotated_memory_z(5, 5, 1e-3, coherent=0.1),
                    1 << 18, 0x5EED0006)


def distill() -> Workload:
    return Workload("distill_15to1_p1e-3_postselect", distill_15to1(1e-3), 1 << 22, 0x5EED0007)


def small_surface() -> Tuple[Circuit, int]:
    return rotated_memory_z(3, 3, 1e-3), 0x5EED0001
