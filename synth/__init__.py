"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Holds only input generation: rigid 3-site SPC/E water boxes placed by random
sequential addition, their force-field parameters (charges, Lennard-Jones
C6/C12 per type pair, masses, intramolecular exclusions) and ballistic
free-flight trajectories.  No pair-interaction, clustering or pair-list
arithmetic lives here.

Water model (Berendsen et al. 1987, SPC/E; the paper's drift study uses it):
O-H 0.1 nm, H-O-H 109.47 deg, q_O = -0.8476 e, q_H = +0.4238 e, LJ on O only
(sigma 0.3166 nm, epsilon 0.650 kJ/mol).  Units: nm, ps, kJ/mol, e, u.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "water_gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")

# physical constants and SPC/E parameters
KB = 0.0083144626          # kJ mol^-1 K^-1
AVOGADRO = 602.214076      # converts u/nm^3 to g/cm^3: rho[g/cm3] = m[u]/V[nm3]/602.214
MASS_O = 15.9994
MASS_H = 1.008
Q_O = -0.8476
Q_H = 0.4238
SIGMA_O = 0.3166
EPS_O = 0.650
WATER_MASS = MASS_O + 2 * MASS_H
D_OO_MIN = 0.25            # nm, hard-core O-O distance for placement
D_ANY_MIN = 0.15           # nm, hard-core intermolecular atom-pair distance


def build(force: bool = False) -> str:
    """Compile the generator with gcc into synth/libsynth.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.synth_water_rsa.restype = ctypes.c_int
        lib.synth_water_rsa.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_uint64,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double)]
        _lib_handle = lib
    return _lib_handle


def lj_table_spce() -> np.ndarray:
    """(2, 2, 2) float64 table: [ti, tj] -> (C6, C12); type 0 = O, type 1 = H.

    C6 = 4 eps sigma^6, C12 = 4 eps sigma^12 for O-O; geometric combination
    makes every pair involving H zero.
    """
    c6 = 4.0 * EPS_O * SIGMA_O ** 6
    c12 = 4.0 * EPS_O * SIGMA_O ** 12
    t = np.zeros((2, 2, 2))
    t[0, 0] = (c6, c12)
    return t


@dataclass
class WaterBox:
    xyz: np.ndarray        # (n, 3) float32, atoms O,H,H per molecule
    q: np.ndarray          # (n,) float32
    type: np.ndarray       # (n,) int32  (0 = O, 1 = H)
    mass: np.ndarray       # (n,) float64
    excl_off: np.ndarray   # (n+1,) int32  CSR of intramolecular exclusions (symmetric, no self)
    excl_idx: np.ndarray   # int32
    box: np.ndarray        # (3,) float64 box edges (nm); float32(box) is the box the kernels use
    n_mol: int
    seed: int
    fallbacks: int

    @property
    def n(self) -> int:
        return self.xyz.shape[0]

    def xyzq(self, xyz=None) -> np.ndarray:
        """(n, 4) float32 packed x, y, z, q."""
        x = self.xyz if xyz is None else xyz
        out = np.empty((self.n, 4), np.float32)
        out[:, :3] = x
        out[:, 3] = self.q
        return out


def box_edge_for(n_mol: int, density_g_cm3: float = 1.0) -> float:
    """Cubic box edge (nm) holding n_mol waters at the given mass density."""
    return (n_mol * WATER_MASS / (AVOGADRO * density_g_cm3)) ** (1.0 / 3.0)


def water_box(n_mol: int, L, seed: int = 1306, max_tries: int = 1000) -> WaterBox:
    """Random sequential addition of n_mol rigid SPC/E waters in a periodic box of edge(s) L (nm)."""
    Ls = np.array([L, L, L] if np.isscalar(L) else L, dtype=np.float64)
    buf = np.empty(9 * n_mol, np.float64)
    fb = _lib().synth_water_rsa(int(n_mol), Ls.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.c_uint64(seed), D_OO_MIN, D_ANY_MIN, int(max_tries),
                                buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if fb < 0:
        raise RuntimeError("water generator failed (code %d)" % fb)
    n = 3 * n_mol
    xyz = buf.reshape(n, 3).astype(np.float32)
    q = np.tile(np.array([Q_O, Q_H, Q_H], np.float32), n_mol)
    typ = np.tile(np.array([0, 1, 1], np.int32), n_mol)
    mass = np.tile(np.array([MASS_O, MASS_H, MASS_H]), n_mol)
    # each atom excludes the two other atoms of its molecule
    base = np.repeat(np.arange(n_mol, dtype=np.int64) * 3, 3)
    k = np.tile(np.arange(3), n_mol)
    partners = np.stack([base + (k + 1) % 3, base + (k + 2) % 3], axis=1)
    partners.sort(axis=1)
    excl_idx = partners.reshape(-1).astype(np.int32)
    excl_off = (np.arange(n + 1, dtype=np.int64) * 2).astype(np.int32)
    return WaterBox(xyz, q, typ, mass, excl_off, excl_idx, Ls, n_mol, seed, fb)


def velocities(mass: np.ndarray, T: float, seed: int) -> np.ndarray:
    """Maxwell-Boltzmann velocities, per component N(0, kB T / m), float64 (n, 3)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x7E1]))
    return rng.standard_normal((mass.shape[0], 3)) * np.sqrt(KB * T / mass)[:, None]


def free_flight(xyz: np.ndarray, v: np.ndarray, dt: float, steps: int):
    """Ballistic positions x_k = x_0 + v k dt for k = 0..steps-1, float32, unwrapped."""
    x0 = xyz.astype(np.float64)
    return [(x0 + v * (k * dt)).astype(np.float32) for k in range(steps)]


def gaussian_displacement(mass: np.ndarray, T: float, t: float, seed: int) -> np.ndarray:
    """Free-particle displacement after time t: per component N(0, kB T t^2 / m), float64 (n, 3)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xD15]))
    return rng.standard_normal((mass.shape[0], 3)) * np.sqrt(KB * T * t * t / mass)[:, None]


# ----------------------------------------------------------------------------
# named workloads (sizes and parameters of the paper-scale water boxes)
# ----------------------------------------------------------------------------
COULOMB_F = 138.935458     # 1/(4 pi eps0) in kJ mol^-1 nm e^-2


@dataclass
class Workload:
    name: str
    n_mol: int
    L: float
    rc: float
    rlist: float
    beta: float
    m: int
    n: int
    nstlist: int = 10
    dt: float = 0.002
    T: float = 300.0


TINY = Workload("water-3k-4x4", 1000, 3.104, 0.9, 0.9, 3.47, 4, 4)
PRODUCTION = Workload("water-96k-8x8", 32000, 9.86, 1.0, 1.1, 3.12, 8, 8)
PRECISION = Workload("water-3M-8x8", 1000000, 31.1, 1.0, 1.1, 3.12, 8, 8)


def batched_sizes(n_rep: int = 256, lo_atoms: int = 1500, hi_atoms: int = 24000, seed: int = 1306):
    """Log-uniform replica sizes in waters: round(exp(U(ln lo/3, ln hi/3)))."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xBA7]))
    u = rng.uniform(math.log(lo_atoms / 3), math.log(hi_atoms / 3), n_rep)
    return np.rint(np.exp(u)).astype(np.int64)
