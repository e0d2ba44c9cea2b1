"""Synthetic crystals standing in for the paper's silicon supercells and materials.

The paper benchmarks Si supercells built from the 8-atom conventional diamond
cell (Section 5.2, Table 5) and three materials (Table 3) whose structures and
SG15 pseudopotentials are not available here.  The inputs below have the same
shapes (diamond-site atoms, Gamma point, norm-conserving-style local potential
plus Kleinman-Bylander projectors, a plane-wave sphere set by a kinetic-energy
cutoff, Section 3.1 and the FFT discussion in Section 4.1) and are fully
determined by seeds.

Conventions (Hartree atomic units, cubic cell of side L, b = 2 pi / L):
  * plane waves: G = b m for integer Miller indices m with |m|^2 <= M2;
    the density sphere (|m|^2 <= 4 M2) is the support of every potential,
    which makes potentials band-limited on an alias-free grid
    (4 max|m_i| + 1 <= N).
  * wave functions: psi(r) = Omega^{-1/2} sum_G c(G) exp(i G.r).
  * real-space grid points r = (i0, i1, i2) L / N, arrays in C order
    (i0 slowest); grid index i <-> Miller component m = i (i < N/2) or i - N.
  * local potential: v_a(r) = -V0 exp(-|r - R_a|^2 / (2 sigma^2)) per atom.
  * projectors: beta_{a,p}(G) = Omega^{-1/2} f_p(G) exp(-i G.R_a) with an
    L2-normalised Gaussian s channel and three p channels.
  * Delta V_j: white noise drawn from numpy's default_rng([seed_dv, j]),
    Gaussian low-pass filtered in G space (width q_f), G = 0 removed,
    truncated to the density sphere, normalised to (Omega/N^3) sum dV^2 = 1.
"""
from __future__ import annotations

import dataclasses
from functools import lru_cache

import numpy as np

A_SI = 10.26  # bohr, conventional diamond cell edge used by the paper's Si supercells

_DIAMOND_FRAC = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    lattice: str          # "diamond" (n x n x n replica of the 8-atom cell) or "sc" (simple cubic)
    reps: int             # replicas per axis
    L: float              # cubic cell edge, bohr
    N: int                # FFT grid points per axis
    M2: int               # wave-function sphere: |m|^2 <= M2
    channels: int         # KB channels per atom: 1 (s) or 4 (s, px, py, pz)
    nv: int               # valence bands
    npert: int            # perturbations Delta V_j
    seed_kb: int          # seed of the KB coefficients D_p
    seed_dv: int = 1      # seed of the perturbations
    V0: float = 2.0       # Ha, depth of the Gaussian local potential
    sigma: float = 0.8    # bohr, Gaussian width of the local potential
    r_beta: float = 0.8   # bohr, Gaussian radius of the projectors
    q_f: float = 1.0      # bohr^-1, low-pass width of Delta V
    tol: float = 1e-10    # relative residual the workload is quoted at
    precision: str = "fp64"

    @property
    def natoms(self) -> int:
        return (8 if self.lattice == "diamond" else 1) * self.reps ** 3

    @property
    def nproj(self) -> int:
        return self.natoms * self.channels

    @property
    def omega(self) -> float:
        return self.L ** 3

    @property
    def b(self) -> float:
        return 2.0 * np.pi / self.L

    @property
    def ecut(self) -> float:
        return 0.5 * self.b ** 2 * self.M2

    @property
    def nsolves(self) -> int:
        return self.npert * self.nv


# Seeds for the KB coefficients were picked so that a clear gap sits above the
# last valence band; tests/golden/gap_table.txt records the gaps the oracle finds.
CONFIGS = {
    # tiny crystal: 8 atoms, 24^3 grid, Ecut 5 Ha -> M2 = 26, 587 plane waves
    "cfg1": Config("cfg1", "diamond", 1, A_SI, 24, 26, 1, 8, 16, seed_kb=0, tol=1e-10),
    # 64-atom supercell, 72^3 grid, 22,575 plane waves, 128 bands, 256 perturbations
    "cfg2": Config("cfg2", "diamond", 2, 2 * A_SI, 72, 306, 4, 128, 256, seed_kb=9, tol=1e-10),
    # mixed precision on the tiny crystal
    "cfg3": Config("cfg3", "diamond", 1, A_SI, 24, 26, 1, 8, 16, seed_kb=0, tol=1e-8,
                   precision="mixed"),
    # served systems of uneven size
    "cfg4a": Config("cfg4a", "sc", 3, 13.68, 48, 132, 4, 54, 32, seed_kb=1, tol=1e-8,
                    precision="mixed"),
    "cfg4b": Config("cfg4b", "diamond", 2, 2 * A_SI, 72, 306, 4, 128, 32, seed_kb=9, tol=1e-8,
                    precision="mixed"),
    "cfg4c": Config("cfg4c", "diamond", 3, 3 * A_SI, 96, 552, 4, 432, 32, seed_kb=0, tol=1e-8,
                    precision="mixed"),
    # large single-GPU share
    "cfg5": Config("cfg5", "diamond", 4, 4 * A_SI, 144, 1260, 4, 1024, 64, seed_kb=0, tol=1e-8,
                   precision="mixed"),
}


def get_config(name: str, **overrides) -> Config:
    cfg = CONFIGS[name]
    return dataclasses.replace(cfg, **overrides) if overrides else cfg


def atom_positions(cfg: Config) -> np.ndarray:
    """Cartesian atom positions [natoms, 3] in bohr."""
    if cfg.lattice == "diamond":
        base = _DIAMOND_FRAC
    elif cfg.lattice == "sc":
        base = np.zeros((1, 3))
    else:
        raise ValueError(cfg.lattice)
    n = cfg.reps
    shifts = np.array([(i, j, k) for i in range(n) for j in range(n) for k in range(n)], float)
    frac = (base[None, :, :] + shifts[:, None, :]).reshape(-1, 3) / n
    return frac * cfg.L


@lru_cache(maxsize=16)
def _sphere_cached(M2: int) -> np.ndarray:
    r = int(np.floor(np.sqrt(M2)))
    ax = np.arange(-r, r + 1)
    m = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    m2 = (m * m).sum(1)
    m = m[m2 <= M2]
    m2 = m2[m2 <= M2]
    # caller order: by shell |m|^2, then lexicographic in (m0, m1, m2)
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], m2))
    out = m[order].astype(np.int32)
    out.setflags(write=False)
    return out


def miller_sphere(M2: int) -> np.ndarray:
    """Miller indices [npw, 3] (int32) of {m : |m|^2 <= M2}, ordered by shell."""
    return _sphere_cached(int(M2)).copy()


def grid_gvectors(cfg: Config):
    """Integer Miller components of the FFT grid along one axis, and b."""
    N = cfg.N
    return np.fft.fftfreq(N, 1.0 / N).astype(np.int64), cfg.b


def _density_grid_G(cfg: Config):
    f, b = grid_gvectors(cfg)
    m0, m1, m2 = np.meshgrid(f, f, f, indexing="ij")
    msq = m0 * m0 + m1 * m1 + m2 * m2
    G = b * np.stack([m0, m1, m2], -1)
    return G, msq


def vloc_r(cfg: Config) -> np.ndarray:
    """Local potential V(r) on the N^3 grid (real, C order), band-limited to the
    density sphere.  V(G) = (1/Omega) sum_a vhat(|G|) exp(-i G.R_a) with
    vhat(q) = -V0 (2 pi sigma^2)^{3/2} exp(-q^2 sigma^2 / 2)."""
    G, msq = _density_grid_G(cfg)
    g2 = (G * G).sum(-1)
    vhat = -cfg.V0 * (2.0 * np.pi * cfg.sigma ** 2) ** 1.5 * np.exp(-0.5 * g2 * cfg.sigma ** 2)
    R = atom_positions(cfg)
    sf = np.zeros(msq.shape, complex)
    for Ra in R:
        sf += np.exp(-1j * (G @ Ra))
    VG = vhat * sf / cfg.omega
    VG[msq > 4 * cfg.M2] = 0.0
    N = cfg.N
    v = np.fft.ifftn(VG) * N ** 3
    return np.ascontiguousarray(v.real)


def beta_projectors(cfg: Config, miller: np.ndarray) -> np.ndarray:
    """KB projectors [nproj, npw] complex128 in the order of ``miller``.
    Projector index = atom * channels + channel (s, then px, py, pz)."""
    G = cfg.b * miller.astype(np.float64)
    g2 = (G * G).sum(1)
    rb = cfg.r_beta
    fs = (4.0 * np.pi * rb * rb) ** 0.75 * np.exp(-0.5 * g2 * rb * rb)
    radial = [fs]
    if cfg.channels == 4:
        for a in range(3):
            radial.append(-1j * np.sqrt(2.0) * rb * G[:, a] * fs)
    elif cfg.channels != 1:
        raise ValueError("channels must be 1 or 4")
    R = atom_positions(cfg)
    out = np.empty((cfg.natoms * cfg.channels, len(miller)), complex)
    inv = 1.0 / np.sqrt(cfg.omega)
    for ia, Ra in enumerate(R):
        phase = np.exp(-1j * (G @ Ra)) * inv
        for c in range(cfg.channels):
            out[ia * cfg.channels + c] = radial[c] * phase
    return out


def dij(cfg: Config) -> np.ndarray:
    """KB coefficients [nproj] (Ha): one value per angular channel (s, and p shared by
    px, py, pz) drawn uniformly in [-1, 1] from ``seed_kb`` and shared by all atoms
    (one species)."""
    nd = 1 if cfg.channels == 1 else 2
    d = np.random.default_rng(cfg.seed_kb).uniform(-1.0, 1.0, nd)
    if cfg.channels == 4:
        d = np.array([d[0], d[1], d[1], d[1]])  # the three p components share one value
    return np.tile(d, cfg.natoms)


def dv_r(cfg: Config, j: int) -> np.ndarray:
    """Perturbation Delta V_j(r) on the grid (real, C order)."""
    N = cfg.N
    w = np.random.default_rng([cfg.seed_dv, j]).standard_normal((N, N, N))
    W = np.fft.fftn(w)
    G, msq = _density_grid_G(cfg)
    g2 = (G * G).sum(-1)
    W *= np.exp(-g2 / (2.0 * cfg.q_f ** 2))
    W[0, 0, 0] = 0.0
    W[msq > 4 * cfg.M2] = 0.0
    dv = np.fft.ifftn(W).real
    dv /= np.sqrt(cfg.omega / N ** 3 * (dv * dv).sum())
    return np.ascontiguousarray(dv)


def dv_block(cfg: Config, js) -> np.ndarray:
    """Stack of perturbations [len(js), N, N, N]."""
    return np.stack([dv_r(cfg, int(j)) for j in js])
