"""Synthetic molecules, geometries and force labels (input generation only).

The paper trains on MD17/MD22 trajectories (section "Experimental results"),
which are not available here.  These seeded stand-ins reproduce their structure:
one molecule of M atoms per system, N thermally displaced copies of an
equilibrium geometry, and force labels of shape (N, M, 3) flattened in the
(geometry, atom, xyz) order the paper uses when it reshapes an n-vector into
(n_train, d, 3) (appendix "Technical details", atomic contribution).

Recipe:
  * equilibrium geometry: a random tree; atom p bonds to a uniformly chosen
    earlier atom at a distance drawn from U[1.0, 1.5] Angstrom in a uniformly
    random direction; a placement is redrawn while any non-bonded distance is
    below 1.0 Angstrom;
  * geometries: N independent copies with i.i.d. N(0, sd^2) displacements of
    every coordinate (sd = 0.05 or 0.08 Angstrom); the equilibrium geometry
    itself is not included;
  * force field: a Morse term on every atom pair, D ~ U[0.5, 2.0],
    a ~ U[1.0, 2.5] 1/Angstrom, r0 = equilibrium pair distance; optionally a
    Coulomb-like q_p q_q / r term with q ~ U[-0.3, 0.3];
  * forces: F = -dE/dR, evaluated analytically (central pair forces, so every
    geometry has zero net force and zero net torque).

Random numbers come from numpy's PCG64 generator seeded per purpose.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Config:
    name: str
    M: int
    N: int
    sd: float
    coulomb: bool
    k: int
    lam: float
    strategy: str
    sigma: float = 10.0
    mol_seed: int = 0
    disp_seed: int = 0
    ff_seed: int = 0
    sel_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def D(self) -> int:
        return self.M * (self.M - 1) // 2

    @property
    def n(self) -> int:
        return 3 * self.M * self.N


def _cfg(c: int, **kw) -> Config:
    return Config(mol_seed=1000 * c, disp_seed=1000 * c + 1, ff_seed=1000 * c + 2,
                  sel_seed=1000 * c + 3, **kw)


# The five workloads, keyed by atoms and geometries: the small plain-FP64 case
# (uniform selection), the mixed-precision cases (pivoted Cholesky, leverage),
# the learned-selection case and the large single-GPU case.  lambda is 1e-9
# where the workload does not state it.  Seeds derive from the workload index.
CONFIGS = {
    "m9_n200": _cfg(1, name="m9_n200", M=9, N=200, sd=0.05, coulomb=False, k=100, lam=1e-8,
               strategy="uniform"),
    "m21_n2000": _cfg(2, name="m21_n2000", M=21, N=2000, sd=0.08, coulomb=True, k=2000, lam=1e-9,
               strategy="pivchol"),
    "m42_n5000": _cfg(3, name="m42_n5000", M=42, N=5000, sd=0.08, coulomb=True, k=5000, lam=1e-9,
               strategy="leverage"),
    "m21_n10000": _cfg(4, name="m21_n10000", M=21, N=10000, sd=0.08, coulomb=True, k=4000, lam=1e-9,
               strategy="learned",
               extra={"train_systems": 20, "train_N": 2000, "train_disp_seed0": 4100,
                      "test_disp_seed": 4200}),
    "m60_n20000": _cfg(5, name="m60_n20000", M=60, N=20000, sd=0.08, coulomb=True, k=8000, lam=1e-9,
               strategy="learned"),
}


@dataclass
class System:
    R: np.ndarray        # (N, M, 3) float64 geometries
    F: np.ndarray        # (N, M, 3) float64 force labels
    R0: np.ndarray       # (M, 3) equilibrium geometry
    E: np.ndarray        # (N,) energies

    @property
    def N(self) -> int:
        return self.R.shape[0]

    @property
    def M(self) -> int:
        return self.R.shape[1]

    def flat_forces(self) -> np.ndarray:
        return self.F.reshape(-1)


def equilibrium_geometry(M: int, seed: int, bond=(1.0, 1.5), min_nonbonded=1.0,
                         max_tries=10000) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    R = np.zeros((M, 3))
    parent = np.full(M, -1)
    for p in range(1, M):
        for _ in range(max_tries):
            par = int(rng.integers(0, p))
            length = rng.uniform(bond[0], bond[1])
            direction = rng.normal(size=3)
            direction /= np.linalg.norm(direction)
            cand = R[par] + length * direction
            dist = np.linalg.norm(R[:p] - cand, axis=1)
            dist[par] = np.inf
            if p == 1 or dist.min() >= min_nonbonded:
                R[p] = cand
                parent[p] = par
                break
        else:
            raise RuntimeError("could not place atom %d" % p)
    return R


def displaced_geometries(R0: np.ndarray, N: int, sd: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return R0[None, :, :] + sd * rng.normal(size=(N,) + R0.shape)


def draw_force_field(R0: np.ndarray, seed: int, coulomb: bool) -> dict:
    M = R0.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    iu = np.triu_indices(M, 1)
    npair = len(iu[0])
    De = rng.uniform(0.5, 2.0, size=npair)
    a = rng.uniform(1.0, 2.5, size=npair)
    r0 = np.linalg.norm(R0[iu[0]] - R0[iu[1]], axis=1)
    q = rng.uniform(-0.3, 0.3, size=M) if coulomb else np.zeros(M)
    return {"i": iu[0], "j": iu[1], "De": De, "a": a, "r0": r0, "q": q,
            "coulomb": bool(coulomb)}


def energy_and_forces(R: np.ndarray, ff: dict, chunk: int = 1024):
    """Energies (N,) and forces (N, M, 3) of the pair potential, F = -dE/dR."""
    N, M, _ = R.shape
    i, j = ff["i"], ff["j"]
    qq = ff["q"][i] * ff["q"][j]
    E = np.empty(N)
    F = np.empty_like(R)
    for s in range(0, N, chunk):
        Rc = R[s:s + chunk]
        diff = Rc[:, i, :] - Rc[:, j, :]                     # (c, P, 3)
        r = np.sqrt((diff ** 2).sum(-1))                      # (c, P)
        ex = np.exp(-ff["a"] * (r - ff["r0"]))
        E[s:s + chunk] = (ff["De"] * (1.0 - ex) ** 2).sum(-1) + (qq / r).sum(-1)
        dEdr = 2.0 * ff["De"] * ff["a"] * ex * (1.0 - ex) - qq / r ** 2
        fpair = (dEdr / r)[..., None] * diff                  # dE/dR_i for pair
        Fc = np.zeros_like(Rc)
        for ax in range(3):
            np.add.at(Fc[:, :, ax].T, i, -fpair[:, :, ax].T)
            np.add.at(Fc[:, :, ax].T, j, fpair[:, :, ax].T)
        F[s:s + chunk] = Fc
    return E, F


def make_system(M: int, N: int, sd: float, coulomb: bool, mol_seed: int,
                disp_seed: int, ff_seed: int) -> System:
    R0 = equilibrium_geometry(M, mol_seed)
    R = displaced_geometries(R0, N, sd, disp_seed)
    ff = draw_force_field(R0, ff_seed, coulomb)
    E, F = energy_and_forces(R, ff)
    return System(R=R, F=F, R0=R0, E=E)


def mixture_system(M: int, N: int, sds, fractions, coulomb: bool, mol_seed: int, disp_seed: int,
                   ff_seed: int) -> System:
    """N geometries of one molecule displaced at several scales: a fraction
    fractions[q] of them with standard deviation sds[q] (the first scale
    takes the rounding remainder), in a seeded random order."""
    R0 = equilibrium_geometry(M, mol_seed)
    counts = [int(round(f * N)) for f in fractions]
    counts[0] += N - sum(counts)
    R = np.concatenate([displaced_geometries(R0, c, sd, disp_seed * 16 + q)
                        for q, (sd, c) in enumerate(zip(sds, counts))])
    R = R[np.random.Generator(np.random.PCG64(disp_seed)).permutation(N)]
    ff = draw_force_field(R0, ff_seed, coulomb)
    E, F = energy_and_forces(R, ff)
    return System(R=R, F=F, R0=R0, E=E)


def config_system(cfg: Config, N: int | None = None, disp_seed: int | None = None) -> System:
    return make_system(cfg.M, cfg.N if N is None else N, cfg.sd, cfg.coulomb,
                       cfg.mol_seed, cfg.disp_seed if disp_seed is None else disp_seed,
                       cfg.ff_seed)


def random_vectors(n: int, seed: int, count: int | None = None) -> np.ndarray:
    """Standard-normal test vectors (n,) or (count, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=n if count is None else (count, n))


def random_weights(n: int, seed: int, low: float = 0.01, high: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(low, high, size=n)
