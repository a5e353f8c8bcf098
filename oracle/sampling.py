"""Row sampling for the random-sampling convergence criterion (oracle).

The paper names a random-sampling convergence criterion (acronym list) but
never defines it.  Reading: the residual is evaluated on S distinct rows drawn
uniformly without replacement.  The draw uses

  * SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
    generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the output
    z is mixed by  z = (z ^ z>>30) * 0xBF58476D1CE4E5B9,
                   z = (z ^ z>>27) * 0x94D049BB133111EB,  z ^ z>>31;
  * Floyd's algorithm (Bentley & Floyd, CACM 30(9), 1987) for S distinct
    integers in [0, N): for j = N-S .. N-1 draw t uniform in [0, j]; insert t,
    or j if t is already present;
  * a uniform integer in [0, j] as the high 64 bits of z * (j + 1).

The generator is seeded with seed + check_index (the number of criterion
evaluations made before for that right-hand side); the result is sorted.
"""
from __future__ import annotations

MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)


def sample_rows(n: int, s: int, seed: int) -> list[int]:
    """S distinct sorted row indices in [0, n) (Floyd's algorithm over SplitMix64)."""
    if s >= n:
        return list(range(n))
    rng = SplitMix64(seed)
    chosen: set[int] = set()
    for j in range(n - s, n):
        t = (rng.next() * (j + 1)) >> 64
        chosen.add(j if t in chosen else t)
    return sorted(chosen)
