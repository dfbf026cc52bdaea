"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds problem definitions and schedules only: boxes, shift vectors
(drawn with numpy's seeded generator), chain counts and temperature schedules.
It contains none of the annealing arithmetic and imports neither the GPU
library nor the oracle.

Workloads (the paper's test functions at the sizes used here):
  schwefel_n4_fp64       normalized Schwefel (Sec. 4.1, eq. (6)), n=4, box [-500,500]^4,
                         256 chains, FP64, T0=10, alpha=0.99, 200 levels x 50 steps, seed 0
  schwefel_n100_fp32     normalized Schwefel, n=100, box [-500,500]^100, 65536 chains, FP32,
                         T0=10, alpha=0.995, 500 levels x 100 steps, seed 1
  rastrigin_n512_fp32    Rastrigin (Appendix, Test 13), n=512, box [-5.12,5.12]^512,
                         shift uniform in the inner 80% of the box, 131072 chains, FP32,
                         1000 levels x 64 steps
  ackley_n1024_fp32      Ackley (Appendix, Test 1), n=1024, box [-32.768,32.768]^1024, shift as
                         above, 131072 chains, FP32, 1000 levels x 64 steps
  griewank_n100_fp32     Griewank (Appendix, Test 8), n=100, box [-600,600]^100, 65536 chains,
                         FP32, T0=10, alpha=0.97, 200 levels x 100 steps, seed 5 (full
                         re-evaluation of f at every move)
Every move uses the radius rule with radius 0.1 (u - l) unless stated.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SCHWEFEL, RASTRIGIN, ACKLEY = 0, 1, 2
# Non-separable families (Appendix: Test 8 Griewank, Test 10 Levy-Montalvo,
# Test 14 generalized Rosenbrock): every move re-evaluates the whole cost.
GRIEWANK, LEVY_MONTALVO, ROSENBROCK = 3, 4, 5
# Centre families (Appendix: Test 18 Shekel, m = 5, 7, 10, n = 4; Test 19
# modified Shekel foxholes and Test 11 modified Langerman, n <= 10).
SHEKEL5, SHEKEL7, SHEKEL10, FOXHOLES, LANGERMAN = 6, 7, 8, 9, 10
FP32, FP64 = 0, 1

# Half-width of each family's canonical box [-h, h]^n: the paper's boxes for
# Rastrigin (Test 13), Griewank (Test 8), Levy-Montalvo (Test 10) and
# Rosenbrock (Test 14); Schwefel and Ackley at the widths used by the
# annealing workloads here (500 and 32.768).
HALF_BOX = {SCHWEFEL: 500.0, RASTRIGIN: 5.12, ACKLEY: 32.768, GRIEWANK: 600.0, LEVY_MONTALVO: 10.0,
            ROSENBROCK: 2.048}
# The centre families' boxes as the paper gives them: [0, 10] (Shekel,
# Langerman) and [-5, 15] (foxholes) in every coordinate.
CENTRE_BOX = {SHEKEL5: (0.0, 10.0), SHEKEL7: (0.0, 10.0), SHEKEL10: (0.0, 10.0), FOXHOLES: (-5.0, 15.0),
              LANGERMAN: (0.0, 10.0)}

# Closed-form minimum of the normalized Schwefel function (Sec. 4.1): the
# paper prints x_i* = 420.968746 and f* = -418.982887 (tests/golden/paper_values.txt);
# the digits below solve d/dx [x sin(sqrt x)] = 0 in FP64 (a root finder on the
# derivative; the oracle tests pin both against the printed values).
SCHWEFEL_X_STAR = 420.968746359982
SCHWEFEL_F_STAR = -418.9828872724337


@dataclass
class Workload:
    name: str
    func: int
    n: int
    lower: np.ndarray
    upper: np.ndarray
    shift: Optional[np.ndarray]
    chains: int
    levels: int
    steps: int
    T0: float
    alpha: float
    seed: int
    precision: int
    radius_frac: float = 0.1
    f_star: Optional[float] = None
    x_star: Optional[np.ndarray] = None
    notes: dict = field(default_factory=dict)

    @property
    def moves(self) -> int:
        return self.chains * self.levels * self.steps

    def with_(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def _box(n, half):
    return np.full(n, -half), np.full(n, half)


def inner_shift(lower, upper, rng):
    """Shift vector uniform in the inner 80% of the box."""
    w = upper - lower
    return rng.uniform(lower + 0.1 * w, upper - 0.1 * w)


def schwefel_n4_fp64() -> Workload:
    lo, hi = _box(4, 500.0)
    return Workload("schwefel_n4_fp64", SCHWEFEL, 4, lo, hi, None, chains=256, levels=200, steps=50, T0=10.0,
                    alpha=0.99, seed=0, precision=FP64, f_star=SCHWEFEL_F_STAR,
                    x_star=np.full(4, SCHWEFEL_X_STAR))


def schwefel_n100_fp32() -> Workload:
    lo, hi = _box(100, 500.0)
    return Workload("schwefel_n100_fp32", SCHWEFEL, 100, lo, hi, None, chains=65536, levels=500, steps=100,
                    T0=10.0, alpha=0.995, seed=1, precision=FP32, f_star=SCHWEFEL_F_STAR,
                    x_star=np.full(100, SCHWEFEL_X_STAR))


def rastrigin_n512_fp32(shift_seed: int = 512) -> Workload:
    lo, hi = _box(512, 5.12)
    s = inner_shift(lo, hi, np.random.default_rng(shift_seed))
    return Workload("rastrigin_n512_fp32", RASTRIGIN, 512, lo, hi, s, chains=131072, levels=1000, steps=64,
                    T0=10.0, alpha=0.99, seed=2, precision=FP32, f_star=0.0, x_star=s.copy())


def ackley_n1024_fp32(shift_seed: int = 1024) -> Workload:
    lo, hi = _box(1024, 32.768)
    s = inner_shift(lo, hi, np.random.default_rng(shift_seed))
    return Workload("ackley_n1024_fp32", ACKLEY, 1024, lo, hi, s, chains=131072, levels=1000, steps=64,
                    T0=10.0, alpha=0.99, seed=3, precision=FP32, f_star=0.0, x_star=s.copy())


def griewank_n100_fp32() -> Workload:
    """Griewank (Appendix, Test 8) at the paper's smallest size n = 100 (F8_a),
    box [-600, 600]^100, unshifted (minimum 0 at the origin); non-separable,
    so every move re-evaluates f in full."""
    lo, hi = _box(100, 600.0)
    return Workload("griewank_n100_fp32", GRIEWANK, 100, lo, hi, None, chains=65536, levels=200, steps=100,
                    T0=10.0, alpha=0.97, seed=5, precision=FP32, f_star=0.0, x_star=np.zeros(100))


def shekel10_n4_fp32() -> Workload:
    """Shekel with m = 10 (Appendix, Test 18; F18_c), box [0, 10]^4; f* and
    x* as printed there."""
    lo, hi = np.zeros(4), np.full(4, 10.0)
    return Workload("shekel10_n4_fp32", SHEKEL10, 4, lo, hi, None, chains=65536, levels=200, steps=100, T0=1.0,
                    alpha=0.97, seed=6, precision=FP32, f_star=-10.5364, x_star=np.full(4, 4.0))


def foxholes_n5_fp32() -> Workload:
    """Modified Shekel foxholes at n = 5 (Appendix, Test 19; F19_b), box
    [-5, 15]^5; f* and x* as printed there."""
    lo, hi = np.full(5, -5.0), np.full(5, 15.0)
    return Workload("foxholes_n5_fp32", FOXHOLES, 5, lo, hi, None, chains=65536, levels=200, steps=100, T0=1.0,
                    alpha=0.97, seed=7, precision=FP32, f_star=-10.4056,
                    x_star=np.array([8.025, 9.152, 5.114, 7.621, 4.564]))


def random_problem(func: int, n: int, seed: int, shifted: bool = True) -> Workload:
    """A small random problem of one of the families, for parity tests:
    canonical box, optional inner shift, random FP32 schedule."""
    if func in CENTRE_BOX:
        lo, hi = np.full(n, CENTRE_BOX[func][0]), np.full(n, CENTRE_BOX[func][1])
    else:
        lo, hi = _box(n, HALF_BOX[func])
    rng = np.random.default_rng(seed)
    s = inner_shift(lo, hi, rng) if shifted else None
    return Workload(f"random_f{func}_n{n}_s{seed}", func, n, lo, hi, s, chains=256, levels=8, steps=32, T0=10.0,
                    alpha=0.95, seed=seed, precision=FP32)


def uneven_box(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Per-coordinate boxes of different widths and centres."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-100.0, 100.0, n)
    w = rng.uniform(1.0, 400.0, n)
    return c - w / 2, c + w / 2


def batch_problems(nprob: int = 1024, seed: int = 4, nmin: int = 2, nmax: int = 256):
    """Batched workload: nprob problems, function uniform over the three
    families, n uniform in {nmin..nmax}, per-problem shift uniform in the inner
    80% of the canonical box (Schwefel: the box translated by the shift, so its
    minimiser stays inside).  Returns [(func, lower, upper, shift)]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nprob):
        func = int(rng.integers(0, 3))
        n = int(rng.integers(nmin, nmax + 1))
        lo, hi = _box(n, HALF_BOX[func])
        s = inner_shift(lo, hi, rng)
        if func == SCHWEFEL:
            lo, hi = lo + s, hi + s
        out.append((func, lo, hi, s))
    return out


ALL = {
    "schwefel_n4_fp64": schwefel_n4_fp64,
    "schwefel_n100_fp32": schwefel_n100_fp32,
    "rastrigin_n512_fp32": rastrigin_n512_fp32,
    "ackley_n1024_fp32": ackley_n1024_fp32,
    "griewank_n100_fp32": griewank_n100_fp32,
}
