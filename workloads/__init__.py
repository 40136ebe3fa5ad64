"""Seeded synthetic lattice-sum problems.

This module only describes inputs: kernels, grids, lattice blocks, defect lists and
sample points, drawn from seeded generators.  It contains none of the arithmetic of
the summation method itself (no quadrature, no collocation, no snapping, no sums),
so that both the CPU oracle and the GPU library can consume the same inputs without
sharing any of the computation.

Conventions (shared by every consumer):

* grid: ``N[l]`` odd cell counts per axis and one mesh size ``h``; cell ``i`` of axis
  ``l`` is centred at ``(i - (N[l]-1)/2) * h``, so the box is ``[-B_l - h/2, B_l + h/2]``
  with ``B_l = (N[l]-1) h / 2``.
* a lattice block is ``L[3]`` sites per axis with spacing ``b[3]`` whose geometric
  centre is ``center[3]``; site ``k`` of axis ``l`` sits at
  ``(k - (L[l]-1)/2) * b[l] + center[l]``.
* every site of a block carries the block's ``charge`` (1 by default; a block of charge
  -1 laid over another block is a tensor sub-lattice of vacancies).
* a defect is ``(block, site[3], dZ)``: the charge of that site changes by ``dZ``
  (``dZ = -1`` is a vacancy, ``dZ = Z - 1`` an impurity of charge ``Z`` substituting
  the unit charge).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

SEED_BASE = 1411_1994

NEWTON, YUKAWA, SLATER = 0, 1, 2
KERNEL_NAMES = {NEWTON: "newton", YUKAWA: "yukawa", SLATER: "slater"}
FP64, FP32, BF16X3 = 0, 1, 2


@dataclass
class Block:
    L: Tuple[int, int, int]
    b: Tuple[float, float, float]
    center: Tuple[float, float, float]
    charge: float = 1.0         # charge of every site (-1: a sub-lattice of vacancies)
    coords: Optional[Tuple] = None   # optional explicit site coordinates per axis (None: b, center)


@dataclass
class Defect:
    block: int
    site: Tuple[int, int, int]
    dZ: float


@dataclass
class Problem:
    name: str
    kind: int
    param: float
    M: int
    N: Tuple[int, int, int]
    h: float
    blocks: List[Block]
    defects: List[Defect] = field(default_factory=list)
    eps: float = 0.0            # <= 0: canonical output, no rank reduction
    precision: int = FP64
    h_u: float = 0.0            # 0: library/oracle default
    s: float = 0.0              # 0: library/oracle default
    tile_lo: Tuple[int, int, int] = (0, 0, 0)
    tile_T: Tuple[int, int, int] = (0, 0, 0)
    exact_sites: bool = False   # True: sites at exact positions (no snapping to cell centres)
    method: int = 0             # 1: Tucker-reference summation (eps > 0, no defects)
    als_sweeps: int = 0         # ALS sweeps after the RHOSVD (eps > 0)

    @property
    def n_sites(self) -> int:
        return int(sum(np.prod(b.L) for b in self.blocks))


def cubic_block(L: int, b: float = 1.0, center=(0.0, 0.0, 0.0)) -> Block:
    return Block((L, L, L), (b, b, b), tuple(float(c) for c in center))


def grid_for_halfwidth(B: float, N: int) -> float:
    """Mesh size of an odd N-cell grid whose outermost cell centres sit at +-B."""
    return 2.0 * B / (N - 1)


def draw_defects(rng: np.random.Generator, blocks: List[Block], n_vac: int, n_imp: int,
                 z_lo: float = 0.5, z_hi: float = 2.0) -> List[Defect]:
    """Distinct sites drawn uniformly without replacement over all blocks; the first
    ``n_vac`` become vacancies, the next ``n_imp`` impurities with Z ~ U[z_lo, z_hi]."""
    sizes = [int(np.prod(b.L)) for b in blocks]
    total = int(sum(sizes))
    n = n_vac + n_imp
    if n > total:
        raise ValueError("more defects than sites")
    flat = rng.choice(total, size=n, replace=False)
    zs = rng.uniform(z_lo, z_hi, size=n_imp)
    out = []
    starts = np.cumsum([0] + sizes)
    for idx, f in enumerate(flat):
        bi = int(np.searchsorted(starts, f, side="right") - 1)
        loc = int(f - starts[bi])
        L = blocks[bi].L
        # site index ordering: axis 0 slowest
        s0 = loc // (L[1] * L[2])
        s1 = (loc // L[2]) % L[1]
        s2 = loc % L[2]
        dZ = -1.0 if idx < n_vac else float(zs[idx - n_vac] - 1.0)
        out.append(Defect(bi, (int(s0), int(s1), int(s2)), dZ))
    return out


def config(c: int) -> Problem:
    """The five named workloads (1-based index)."""
    rng = np.random.default_rng(SEED_BASE + c)
    if c == 1:
        # Newton, 4x4x4 unit lattice, box half-width 6, N = 129, M = 32
        N = 129
        return Problem("cfg1-newton-L4-N129", NEWTON, 0.0, 32, (N, N, N),
                       grid_for_halfwidth(6.0, N), [cubic_block(4)])
    if c == 2:
        # Newton, 64^3 lattice, half-width L/2 + 8, N = 4097, M = 40
        N, L = 4097, 64
        return Problem("cfg2-newton-L64-N4097", NEWTON, 0.0, 40, (N, N, N),
                       grid_for_halfwidth(L / 2 + 8, N), [cubic_block(L)])
    if c == 3:
        # Newton, 48^3 lattice, N = 2049, 300 vacancies + 100 impurities, eps = 1e-6, FP32 contractions
        N, L = 2049, 48
        blocks = [cubic_block(L)]
        defects = draw_defects(rng, blocks, 300, 100)
        return Problem("cfg3-newton-L48-N2049-def400", NEWTON, 0.0, 40, (N, N, N),
                       grid_for_halfwidth(L / 2 + 8, N), blocks, defects, eps=1e-6,
                       precision=FP32)
    if c == 4:
        # Yukawa kappa = 0.5 on a step-shaped union of three blocks, 500 vacancies, eps = 1e-5,
        # 512^3 reconstruction tile centred in the box.
        N = 2049
        # global site indices: A=[0,40)x[0,40)x[0,20), B=[0,40)x[0,20)x[20,40), C=[0,20)x[0,20)x[40,60);
        # the union's bounding box [0,40)x[0,40)x[0,60) is centred at the origin.
        blocks = [Block((40, 40, 20), (1.0, 1.0, 1.0), (0.0, 0.0, -20.0)),
                  Block((40, 20, 20), (1.0, 1.0, 1.0), (0.0, -10.0, 0.0)),
                  Block((20, 20, 20), (1.0, 1.0, 1.0), (-10.0, -10.0, 20.0))]
        defects = draw_defects(rng, blocks, 500, 0)
        lo = (N - 1) // 2 - 256
        return Problem("cfg4-yukawa-step-N2049-vac500", YUKAWA, 0.5, 40, (N, N, N),
                       grid_for_halfwidth(60 / 2 + 8, N), blocks, defects, eps=1e-5,
                       precision=FP32, tile_lo=(lo, lo, lo), tile_T=(512, 512, 512))
    raise ValueError(f"unknown config {c}")


def sample_points(c: int, n: int, B: Tuple[float, float, float]) -> np.ndarray:
    """n seeded points uniform in the box [-B, B] (per axis), shape (n, 3), float64."""
    rng = np.random.default_rng(SEED_BASE + 100 + c)
    lo = -np.asarray(B, dtype=np.float64)
    return rng.uniform(lo, -lo, size=(n, 3))


def half_widths(p: Problem) -> Tuple[float, float, float]:
    return tuple((n - 1) * p.h / 2 for n in p.N)


def subgrid(N: int, m: int = 32) -> np.ndarray:
    """m evenly spread cell indices of an N-cell axis (m=32, N=4097 gives 64 + 128 j)."""
    step = (N - 1) // m
    return step // 2 + step * np.arange(m)


# ----------------------------------------------------------------------------------------
# served mixed workload
# ----------------------------------------------------------------------------------------

SERVE_N = (257, 513, 1025, 2049, 4097)


def served_request(rng: np.random.Generator, idx: int, L_range=(8, 96), n_choices=SERVE_N,
                   max_defects: int = 500) -> Problem:
    """One request of the served mixed workload: rectangular L per axis, N for the longest
    axis, kernel uniform over the three, 0..max_defects vacancies/impurities (p = 1/2 each),
    eps in {1e-4, 1e-6}."""
    L = tuple(int(x) for x in rng.integers(L_range[0], L_range[1] + 1, size=3))
    Bs = [l / 2 + 8 for l in L]
    Nmax = int(rng.choice(n_choices))
    h = 2.0 * max(Bs) / (Nmax - 1)
    N = tuple(Nmax if B == max(Bs) else min(Nmax, int(2 * np.ceil(B / h) + 1)) for B in Bs)
    kind = int(rng.integers(0, 3))
    param = {NEWTON: 0.0, YUKAWA: 0.5, SLATER: 1.0}[kind]
    blocks = [Block(L, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))]
    nd = int(rng.integers(0, max_defects + 1))
    nd = min(nd, int(np.prod(L)))
    kinds = rng.random(nd) < 0.5
    n_vac = int(kinds.sum())
    defects = draw_defects(rng, blocks, n_vac, nd - n_vac)
    eps = float(rng.choice([1e-4, 1e-6]))
    # mixed precision where its arithmetic error (a few 1e-7 relative) is far below eps
    prec = FP32 if eps >= 1e-4 else FP64
    return Problem(f"serve-{idx}", kind, param, 40, N, h, blocks, defects, eps=eps, precision=prec)


def served_stream(n: int, rate_per_s: float, seed_offset: int = 5, **kw):
    """(arrival_time_s, Problem) pairs with Poisson arrivals at ``rate_per_s``."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps)
    return [(float(t[i]), served_request(rng, i, **kw)) for i in range(n)]


def served_mix_stream(count: int, n_total: int = 10_000):
    """The first ``count`` requests of the served mixed workload of ``n_total`` requests with
    Poisson arrivals: (gap at unit rate, Problem) pairs.  All ``n_total`` gaps are drawn first,
    then the requests in order, so a prefix is the same for any ``count``; arrival times at rate
    lam are the cumulative gaps divided by lam."""
    if count > n_total:
        raise ValueError("count exceeds the stream")
    rng = np.random.default_rng(SEED_BASE + 5)
    gaps = rng.exponential(1.0, size=n_total)
    return [(float(gaps[i]), served_request(rng, i)) for i in range(count)]
