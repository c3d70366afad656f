"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds no exchange arithmetic; see ``generator`` for the grid convention.
"""
from .generator import (FREE, PERIODIC, SURFACE, WIRE, OrbitalRecipe, System, draw_system, loewdin,
                        make_system)
from .workloads import (BATCH, BATCH_SMALL, SINGLE, batch_recipes, pair_count, recipe, scaled,
                        small_batch_recipes, system)

__all__ = [
    "FREE", "PERIODIC", "SURFACE", "WIRE", "OrbitalRecipe", "System", "draw_system", "loewdin", "make_system",
    "BATCH", "BATCH_SMALL", "SINGLE", "batch_recipes", "pair_count", "recipe", "scaled",
    "small_batch_recipes", "system",
]
