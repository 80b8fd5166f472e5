"""Seeded synthetic RPCA instances shared by the FP64 oracle and the GPU path.

This module only draws random inputs. It holds none of the method's arithmetic:
it builds M = L* + S* from planted factors and a planted sparse matrix, the way
the paper's experiments do (Section 4.1, "Problem Generation"), and it draws
the initial factor U^(0) that Algorithm 1 leaves to the implementer.

Every array that either side consumes is rounded to FP32 once, here, and then
handed out as float64 arrays whose values are exactly representable in FP32.
The oracle computes in FP64 on those values; the GPU path uploads the same
values as FP32, so the two start from bit-identical inputs.

Recipes (all seeded; independent streams for factors, support, values and U^(0)):

* planted low-rank part: L* = U* V*^T with i.i.d. N(0,1) factors (Section 4.1),
  or, for the geometric-spectrum workload, L* = Q_U diag(sigma) Q_V^T with
  orthonormal Q from the QR factorisation of Gaussian matrices;
* planted sparse part: an exact count round(s*m*n) of positions drawn without
  replacement (Section 4.1 draws "smn random nonzero entries"), or an
  independent Bernoulli(s) mask for instances too large to permute;
* corruption values: uniform on [-a, a] ("uniform") or a uniform magnitude on
  [lo, hi] with a fair random sign ("signed");
* client widths: equal blocks, or log-uniform widths in [lo, hi] rounded to
  integers (the uneven-client workload);
* instances too large for dense FP64 work arrays are built one client block at
  a time (Bernoulli support, per-block streams) and kept as FP32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Instance",
    "planted_instance",
    "equal_widths",
    "loguniform_widths",
    "gaussian_init",
    "splitmix64_outputs",
    "splitmix_gaussian_init",
    "recipe",
    "RECIPES",
    "controller_family",
]

# Stream identifiers for numpy SeedSequence spawning; fixed so that a change to
# one recipe field never shifts the random numbers drawn for another.
_STREAM_FACTORS = 1
_STREAM_SUPPORT = 2
_STREAM_VALUES = 3
_STREAM_SIGNS = 4
_STREAM_INIT = 5
_STREAM_WIDTHS = 6


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def _f32(x: np.ndarray) -> np.ndarray:
    """Round to FP32 once and return float64 holding exactly those values."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@dataclasses.dataclass
class Instance:
    """One synthetic RPCA problem, M = L* + S*, split column-wise over clients.

    M is (m, n) float64 with FP32-representable values; the block of client i
    is M[:, offsets[i]:offsets[i+1]] (Section 2.1: each client holds a
    contiguous set of columns). Ustar @ Vstar.T is the planted low-rank part
    before the FP32 rounding of M.
    """

    M: np.ndarray
    widths: List[int]
    Ustar: np.ndarray
    Vstar: np.ndarray
    Sstar: np.ndarray
    seed: int
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.M.shape[0])

    @property
    def n(self) -> int:
        return int(self.M.shape[1])

    @property
    def E(self) -> int:
        return len(self.widths)

    @property
    def offsets(self) -> List[int]:
        off = [0]
        for w in self.widths:
            off.append(off[-1] + int(w))
        return off

    def blocks(self) -> List[np.ndarray]:
        off = self.offsets
        return [self.M[:, off[i]:off[i + 1]] for i in range(self.E)]

    @property
    def Lstar(self) -> np.ndarray:
        return self.Ustar @ self.Vstar.T


def equal_widths(n: int, E: int) -> List[int]:
    """E contiguous blocks whose widths differ by at most one column."""
    base, extra = divmod(int(n), int(E))
    return [base + (1 if i < extra else 0) for i in range(E)]


def loguniform_widths(E: int, lo: int, hi: int, seed: int) -> List[int]:
    """E widths round(exp(U[ln lo, ln hi])), clipped to [lo, hi]."""
    rng = _rng(seed, _STREAM_WIDTHS)
    w = np.exp(rng.uniform(math.log(lo), math.log(hi), size=E))
    return [int(min(max(int(round(x)), lo), hi)) for x in w]


def gaussian_init(m: int, r: int, seed: int) -> np.ndarray:
    """U^(0) with i.i.d. N(0,1) entries, FP32-rounded (Algorithm 1 leaves the
    distribution open; a Gaussian start avoids the stationary point U = 0)."""
    return _f32(_rng(seed, _STREAM_INIT).standard_normal((m, r)))


_GOLDEN64 = 0x9E3779B97F4A7C15
_MASK64 = (1 << 64) - 1


def splitmix64_outputs(seed: int, first: int, count: int) -> np.ndarray:
    """Outputs first .. first + count - 1 of SplitMix64 (Steele, Lea and Flood,
    2014) seeded with `seed`: output j mixes the state seed + (j + 1) times
    the golden-ratio increment (mod 2^64). uint64 array."""
    with np.errstate(over="ignore"):
        j = np.arange(first, first + count, dtype=np.uint64)
        z = np.uint64(int(seed) & _MASK64) + (j + np.uint64(1)) * np.uint64(_GOLDEN64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix_gaussian_init(m: int, r: int, seed: int) -> np.ndarray:
    """The U^(0) that the library draws on the device when given no start:
    entry (i, c) is the Box-Muller normal sqrt(-2 ln(1 - u1)) cos(2 pi u2) of
    the SplitMix64 outputs 2k and 2k + 1, k = c m + i, with u = (x >> 11)
    2^-53, formed in FP64 and rounded to FP32. (m, r) float64 array."""
    x = splitmix64_outputs(seed, 0, 2 * m * r)
    u = (x >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u1, u2 = u[0::2], u[1::2]
    z = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)
    return _f32(z.reshape(r, m).T)


def _planted_factors(m: int, n: int, rstar: int, seed: int, spectrum: str, sigma_hi: float,
                     sigma_lo: float):
    """Planted factors with L* = U* V*^T: i.i.d. N(0,1) ("gaussian"), or
    Q_U diag(sigma) Q_V^T split as (Q_U sqrt(sigma), Q_V sqrt(sigma)) with Q from
    the QR factorisation of Gaussian matrices and sigma geometric from
    sigma_hi down to sigma_lo ("geometric")."""
    frng = _rng(seed, _STREAM_FACTORS)
    if spectrum == "gaussian":
        return frng.standard_normal((m, rstar)), frng.standard_normal((n, rstar))
    if spectrum == "geometric":
        qu, _ = np.linalg.qr(frng.standard_normal((m, rstar)))
        qv, _ = np.linalg.qr(frng.standard_normal((n, rstar)))
        if rstar > 1:
            k = np.arange(rstar, dtype=np.float64)
            sig = sigma_hi * (sigma_lo / sigma_hi) ** (k / (rstar - 1))
        else:
            sig = np.array([sigma_hi])
        return qu * np.sqrt(sig)[None, :], qv * np.sqrt(sig)[None, :]
    raise ValueError(f"unknown spectrum {spectrum!r}")


def planted_instance(
    m: int,
    widths: Sequence[int],
    rstar: int,
    s: float,
    values: str = "signed",
    lo: float = 5.0,
    hi: float = 20.0,
    seed: int = 0,
    spectrum: str = "gaussian",
    sigma_hi: float = 100.0,
    sigma_lo: float = 1.0,
    support: str = "exact",
    name: str = "",
) -> Instance:
    """Draw M = L* + S* with a planted rank-rstar part and a fraction s of
    corrupted entries.

    values="uniform": corruption ~ U[-hi, hi]; values="signed": magnitude
    ~ U[lo, hi] with a fair random sign. spectrum="gaussian": L* = U* V*^T with
    N(0,1) factors; spectrum="geometric": singular values geometric from
    sigma_hi down to sigma_lo on orthonormal random singular vectors.
    """
    widths = [int(w) for w in widths]
    n = int(sum(widths))
    Ustar, Vstar = _planted_factors(m, n, rstar, seed, spectrum, sigma_hi, sigma_lo)

    total = m * n
    srng = _rng(seed, _STREAM_SUPPORT)
    if support == "exact":
        count = int(round(s * total))
        flat = srng.choice(total, size=count, replace=False)
    elif support == "bernoulli":
        flat = np.flatnonzero(srng.random(total) < s)
        count = flat.size
    else:
        raise ValueError(f"unknown support {support!r}")
    vrng = _rng(seed, _STREAM_VALUES)
    if values == "uniform":
        vals = vrng.uniform(-hi, hi, size=count)
    elif values == "signed":
        mag = vrng.uniform(lo, hi, size=count)
        sign = np.where(_rng(seed, _STREAM_SIGNS).random(count) < 0.5, -1.0, 1.0)
        vals = sign * mag
    else:
        raise ValueError(f"unknown values {values!r}")
    Sstar = np.zeros(total, dtype=np.float64)
    Sstar[flat] = vals
    # Column-major flattening: flat index = row + m * col, matching the
    # column-major device layout (the choice does not affect the law).
    Sstar = Sstar.reshape(n, m).T.copy()
    M = _f32(Ustar @ Vstar.T + Sstar)
    return Instance(M=M, widths=widths, Ustar=Ustar, Vstar=Vstar, Sstar=Sstar,
                    seed=int(seed), name=name)


def planted_instance_large(
    m: int,
    widths: Sequence[int],
    rstar: int,
    s: float,
    values: str = "signed",
    lo: float = 1.0,
    hi: float = 50.0,
    seed: int = 0,
    name: str = "",
    spectrum: str = "gaussian",
    sigma_hi: float = 100.0,
    sigma_lo: float = 1.0,
) -> Instance:
    """The laws of planted_instance (Gaussian or geometric-spectrum factors,
    Bernoulli(s) support) for instances too large for dense FP64 work arrays:
    M is built one client block at a time, each block drawing its support and
    values from streams of its own, and is kept as FP32, column-major (M.T is
    C-contiguous). S* is not kept (Sstar is None)."""
    widths = [int(w) for w in widths]
    n = int(sum(widths))
    Ustar, Vstar = _planted_factors(m, n, rstar, seed, spectrum, sigma_hi, sigma_lo)
    Mt = np.empty((n, m), dtype=np.float32)
    off = 0
    for i, w in enumerate(widths):
        Lt = Vstar[off:off + w] @ Ustar.T                     # (w, m): client block, transposed
        srng = np.random.default_rng(np.random.SeedSequence([int(seed), _STREAM_SUPPORT, i]))
        mask = srng.random((w, m)) < s
        count = int(mask.sum())
        vrng = np.random.default_rng(np.random.SeedSequence([int(seed), _STREAM_VALUES, i]))
        if values == "uniform":
            vals = vrng.uniform(-hi, hi, size=count)
        elif values == "signed":
            mag = vrng.uniform(lo, hi, size=count)
            sg = np.random.default_rng(np.random.SeedSequence([int(seed), _STREAM_SIGNS, i]))
            vals = np.where(sg.random(count) < 0.5, -1.0, 1.0) * mag
        else:
            raise ValueError(f"unknown values {values!r}")
        Lt[mask] += vals
        Mt[off:off + w] = Lt
        off += w
    return Instance(M=Mt.T, widths=widths, Ustar=Ustar, Vstar=Vstar, Sstar=None,
                    seed=int(seed), name=name)


# Named workloads. Each entry gives the instance recipe and the solver
# parameters the workload is quoted with (lambda = 1/sqrt(n), rho = 0.1).
RECIPES = {
    # m = n = 500, rank 5, 5% of entries corrupted uniformly in [-10, 10],
    # five clients of 100 columns, r = 5, 100 rounds.
    "plain_500x500_r5": dict(m=500, n=500, E=5, rstar=5, s=0.05, values="uniform",
                             lo=0.0, hi=10.0, r=5, rho=0.1, T=100),
    # m = 4000, n = 8000, rank 20, 10% corrupted with magnitude U[5, 20],
    # sixteen clients of 500 columns, r = 20, 200 rounds.
    "plain_4000x8000_r20": dict(m=4000, n=8000, E=16, rstar=20, s=0.10, values="signed",
                                lo=5.0, hi=20.0, r=20, rho=0.1, T=200),
    # A 2000 x 2000 single-client instance with the large workload's recipe
    # (rank 64, geometric spectrum 100 -> 1, 5% corrupted, magnitude U[1, 100]).
    "geom_2000x2000_r64": dict(m=2000, n=2000, E=1, rstar=64, s=0.05, values="signed",
                               lo=1.0, hi=100.0, r=64, rho=0.1, T=100,
                               spectrum="geometric"),
    # m = 10000, 64 clients with widths log-uniform in [64, 4096] (seeded),
    # rank 32, 5% of entries corrupted (Bernoulli) with magnitude U[1, 50],
    # r = 32. About 62,000 columns: M is 2.5 GB in FP32, built blockwise.
    "uneven_10000_r32": dict(m=10000, E=64, widths=("loguniform", 64, 4096), rstar=32,
                             s=0.05, values="signed", lo=1.0, hi=50.0, r=32, rho=0.1,
                             T=200, large=True),
    # m = 20000, n = 100000, fifty clients of 2000 columns, rank 64 with a
    # geometric spectrum 100 -> 1, 5% of entries corrupted (Bernoulli) with
    # magnitude U[1, 100], r = 64. M is 8 GB in FP32, built blockwise.
    "geom_20000x100000_r64": dict(m=20000, n=100000, E=50, rstar=64, s=0.05,
                                  values="signed", lo=1.0, hi=100.0, r=64, rho=0.1, T=100,
                                  spectrum="geometric", large=True),
    # m = 8000, n = 32000, 32 clients of 1000 columns, rank 40, 15% of entries
    # corrupted (Bernoulli) with magnitude U[5, 20], r = 40: the learned
    # controller's evaluation instance. Relative error 1e-4 against L* is
    # reachable here. M is 1 GB in FP32, built blockwise.
    "plain_8000x32000_r40": dict(m=8000, n=32000, E=32, rstar=40, s=0.15, values="signed",
                                 lo=5.0, hi=20.0, r=40, rho=0.1, T=200, large=True,
                                 recovery=True),
}


def controller_family(seed: int, n: int = 2000):
    """A training instance for the learned controller, drawn from the
    evaluation workload's family: m = n, clients of 250 columns (at least
    one), rank uniform in {5..50} (capped at n / 4), corruption fraction
    uniform in [0.01, 0.2] with magnitude U[5, 20] and a random sign. Returns
    (instance, rank)."""
    rng = _rng(seed, _STREAM_WIDTHS + 1)
    r = int(min(rng.integers(5, 51), max(1, n // 4)))
    s = float(rng.uniform(0.01, 0.20))
    return planted_instance(n, equal_widths(n, max(1, n // 250)), r, s, values="signed", lo=5.0,
                            hi=20.0, seed=seed), r


def recipe(name: str, seed: int = 0, E: Optional[int] = None) -> Instance:
    """Instantiate a named workload (see RECIPES)."""
    cfg = dict(RECIPES[name])
    E = int(E if E is not None else cfg["E"])
    if cfg.get("large"):
        if "widths" in cfg:
            kind, wlo, whi = cfg["widths"]
            widths = loguniform_widths(E, wlo, whi, seed)
        else:
            widths = equal_widths(cfg["n"], E)
        return planted_instance_large(cfg["m"], widths, cfg["rstar"], cfg["s"],
                                      values=cfg["values"], lo=cfg["lo"], hi=cfg["hi"],
                                      seed=seed, name=name,
                                      spectrum=cfg.get("spectrum", "gaussian"))
    widths = equal_widths(cfg["n"], E)
    return planted_instance(cfg["m"], widths, cfg["rstar"], cfg["s"], values=cfg["values"],
                            lo=cfg["lo"], hi=cfg["hi"], seed=seed,
                            spectrum=cfg.get("spectrum", "gaussian"), name=name)
