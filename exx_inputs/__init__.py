"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds no exchange arithmetic; see ``generator`` for the grid convention.
"""
from .generator import (FREE, PERIODIC, SURFACE, WIRE, OrbitalRecipe, System, draw_system, loewdin,
                        make_system)
from .workloads import BATCH, SINGLE, batch_recipes, pair_count, recipe, scaled, system

__all__ = [
    "FREE", "PERIODIC", "SURFACE", "WIRE", "OrbitalRecipe", "System", "draw_system", "loewdin", "make_system",
    "BATCH", "SINGLE", "batch_recipes", "pair_count", "recipe", "scaled", "system",
]
