"""Accuracy-driven Ewald / PME parameters (test infrastructure only).

The paper picks the number of reciprocal vectors of the regular Ewald sum and
the PME grid from a target Ewald accuracy delta "with the same tuning
heuristics as OpenMM" (Sections "Regular Ewald Summation", "Particle Mesh
Ewald Summation" and "Ewald Summation"; its runs use delta = 5e-4 and
rc = 10 A). The paper does not print the heuristics; they are the ones
OpenMM's documentation states:

* splitting parameter:  alpha = sqrt(-ln(2 delta)) / rc, i.e. exp(-(alpha rc)^2)
  equals 2 delta;
* direct Ewald: the estimated error with |n_d| <= k along an edge L is
  0.05 sqrt(L alpha) k exp(-(pi k / (L alpha))^2); kmax is the smallest k past
  the maximum of this estimate (k >= ceil(L alpha / (pi sqrt 2)), k >= 1)
  whose estimate is <= delta;
* PME: K = ceil(2 alpha L / (3 delta^(1/5))) points per edge, raised to at
  least 2p and to the next size whose prime factors are 2, 3 and 5 (the FFT
  sizes the library accepts).

Written as plain Python loops over the formulas above.
"""
import math

__all__ = ["alpha_for", "ewald_error", "ewald_kmax", "pme_grid_min", "next_smooth", "pme_grid", "choose"]


def alpha_for(delta: float, rc: float) -> float:
    """Splitting parameter whose real-space tail factor exp(-(alpha rc)^2) is 2 delta."""
    return math.sqrt(-math.log(2.0 * delta)) / rc


def ewald_error(L: float, alpha: float, k: int) -> float:
    """OpenMM's estimate of the direct-Ewald error with |n| <= k along an edge L."""
    t = math.pi * k / (L * alpha)
    return 0.05 * math.sqrt(L * alpha) * k * math.exp(-t * t)


def ewald_kmax(L: float, alpha: float, delta: float, limit: int = 10_000) -> int:
    k = max(1, math.ceil(L * alpha / (math.pi * math.sqrt(2.0))))
    while ewald_error(L, alpha, k) > delta and k < limit:
        k += 1
    return k


def pme_grid_min(L: float, alpha: float, delta: float) -> int:
    return math.ceil(2.0 * alpha * L / (3.0 * delta ** 0.2))


def next_smooth(k: int) -> int:
    """Smallest m >= k whose only prime factors are 2, 3 and 5."""
    m = max(1, k)
    while True:
        r = m
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 1


def pme_grid(L: float, alpha: float, delta: float, order: int) -> int:
    return next_smooth(max(pme_grid_min(L, alpha, delta), 2 * order))


def choose(box, n, rc, delta, order, method, pme_min_atoms):
    """Parameters as a dict: alpha, grid (3), kmax (3), method ("pme"/"ewald").
    method "auto" takes Ewald below pme_min_atoms atoms if its kmax is <= 64."""
    box = [float(x) for x in (box if hasattr(box, "__len__") else (box, box, box))]
    a = alpha_for(delta, rc)
    grid = [pme_grid(L, a, delta, order) for L in box]
    kmax = [ewald_kmax(L, a, delta) for L in box]
    if method == "auto":
        method = "ewald" if (n < pme_min_atoms and max(kmax) <= 64) else "pme"
    return {"alpha": a, "grid": grid, "kmax": kmax, "method": method}
