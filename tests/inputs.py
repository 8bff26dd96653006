"""Seeded synthetic inputs for the larger workloads, shared by the GPU tests
and the oracle side of those tests.

Holds none of the method's arithmetic: every draw comes from numpy's own
Philox bit generator (Philox4x64-10, `numpy.random.Philox(key=...)`), never
from the assembly's Philox4x32-10 stream, and the arrays are handed to both
sides unchanged.  The paper's own workloads are exhaustive enumerations of
genotype spaces (§4: S_{1,8}, S_{2,8}, the three-tile space); these are the
random streams and samples that stand in for its larger spaces.

  mixed_stream   genotypes of 1, 2 or 3 tiles (uniform), colours iid uniform
                 over c = 8, grid 16 or 32 (uniform), default rng_id;
                 Philox key 7.
  three_tile     t = 3 genotypes: a contiguous lexicographic slice starting
                 at a drawn offset, and a uniform sample of the 8^12 space;
                 Philox key 11.
  population     a uniform random GA population of t-tile genotypes;
                 Philox key 5.
"""
import numpy as np

C = 8
BITS = 3


def _gen(key: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=key))


def mixed_stream(n: int, key: int = 7):
    """(genomes uint64, t uint8, grid uint8) of n items."""
    g = _gen(key)
    t = g.integers(1, 4, size=n, dtype=np.uint8)
    grid = np.where(g.integers(0, 2, size=n, dtype=np.uint8) == 0, 16, 32).astype(np.uint8)
    raw = g.integers(0, (1 << 64) - 1, size=n, dtype=np.uint64, endpoint=True)
    genomes = raw >> (np.uint64(64) - np.uint64(4 * BITS) * t.astype(np.uint64))
    return genomes, t, grid


def three_tile_slice_start(n: int, key: int = 11) -> int:
    """First genotype of a contiguous n-genotype slice of the 8^12 space."""
    space = C ** 12
    return int(_gen(key).integers(0, space - n, endpoint=True))


def three_tile_sample(n: int, key: int = 11):
    """n genotypes drawn uniformly (with replacement) from the 8^12 space."""
    g = np.random.Generator(np.random.Philox(key=key).jumped())   # apart from the slice's
    return g.integers(0, C ** 12, size=n, dtype=np.uint64)


def population(n: int, t: int, key: int = 5):
    """A uniform random population of n t-tile genotypes."""
    return _gen(key).integers(0, 1 << (4 * BITS * t), size=n, dtype=np.uint64)
