"""Seeded synthetic inputs for the form-factor engine and its oracle.

This module is shared by the FP64 oracle, the HIP library's tests and the
benchmark.  It holds no arithmetic of the method itself: it only draws
geometries, Gaussian shells (exponents and contraction coefficients),
transition density matrices and q-grids.  Normalisation, overlap integrals
and Fourier transforms live on each side separately.

The paper's own inputs (a 100-molecule cc-pVDZ test set with PySCF TD-DFT
transition matrices; Sec. 5.1 and Table I) are not available, so seeded
stand-ins of the same shape are drawn here:

* heavy atoms carry a double-zeta-like Cartesian shell set (3 s + 2 p + 1 d,
  or 3 s + 2 p without d for the tiny case), hydrogens 2 s (+ 1 p);
* 3 primitives per shell, exponents log-uniform in [0.1, 100] bohr^-2 sorted
  descending, contraction coefficients U(0.1, 1);
* T^s = C_occ X^s C_vir^T with C a Euclidean-orthonormal matrix (QR of a
  Gaussian matrix) and X^s i.i.d. normal with unit Frobenius norm, the
  Casida X-only form of the transition density matrix (Sec. 2.2);
* q_i = linspace(-q_max, +q_max, N) on each axis, in atomic units.

All lengths are in bohr, exponents in bohr^-2, momenta in a.u.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

ANGSTROM_TO_BOHR = 1.0 / 0.529177210903

# Cartesian component order per shell; the library ABI and the oracle both use it.
CART_ORDER = {
    0: [(0, 0, 0)],
    1: [(1, 0, 0), (0, 1, 0), (0, 0, 1)],
    2: [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)],
}


def n_cart(l: int) -> int:
    """Number of Cartesian components of a shell of angular momentum l."""
    return (l + 1) * (l + 2) // 2


@dataclasses.dataclass
class Molecule:
    """Geometry plus a contracted Cartesian Gaussian basis (flat arrays)."""
    Z: np.ndarray            # [n_atoms] int
    xyz: np.ndarray          # [n_atoms, 3] float64, bohr
    shell_atom: np.ndarray   # [n_shells] int32
    shell_l: np.ndarray      # [n_shells] int32
    shell_nprim: np.ndarray  # [n_shells] int32
    exps: np.ndarray         # [sum nprim] float64, bohr^-2
    coefs: np.ndarray        # [sum nprim] float64

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(n_cart(int(l)) for l in self.shell_l))

    def translated(self, d: Sequence[float]) -> "Molecule":
        return dataclasses.replace(self, xyz=self.xyz + np.asarray(d, dtype=np.float64)[None, :])


@dataclasses.dataclass
class Grid:
    n: tuple            # (nx, ny, nz)
    qmin: tuple         # 3 floats, a.u.
    qmax: tuple

    def axis(self, a: int) -> np.ndarray:
        return np.linspace(self.qmin[a], self.qmax[a], self.n[a])

    def points(self) -> np.ndarray:
        """All grid points, [nx*ny*nz, 3], z fastest (row-major [ix][iy][iz])."""
        gx, gy, gz = np.meshgrid(self.axis(0), self.axis(1), self.axis(2), indexing="ij")
        return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)

    @property
    def n_points(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


@dataclasses.dataclass
class Workload:
    name: str
    mol: Molecule
    T: np.ndarray        # [n_states, nbf, nbf] float64
    grid: Grid
    seed: int


# ---------------------------------------------------------------- geometry

def _uniform_box(rng, n, edge_bohr, min_sep_bohr, max_tries=100000):
    pts: List[np.ndarray] = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place atoms with the requested separation")
        p = (rng.random(3) - 0.5) * edge_bohr
        if all(np.linalg.norm(p - q) >= min_sep_bohr for q in pts):
            pts.append(p)
    return np.array(pts)


def _place_hydrogens_random(rng, heavy, n_h, bond, min_sep, max_tries=100000):
    """Each H sits `bond` from a distinct randomly chosen heavy atom."""
    hosts = rng.choice(len(heavy), size=n_h, replace=False)
    out = []
    for h in hosts:
        for _ in range(max_tries):
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            p = heavy[h] + bond * v
            others = [heavy[i] for i in range(len(heavy)) if i != h] + out
            if all(np.linalg.norm(p - q) >= min_sep for q in others):
                out.append(p)
                break
        else:
            raise RuntimeError("could not place hydrogen")
    return np.array(out).reshape(-1, 3)


def _two_fused_hexagons(rng, bond_A=1.40):
    """Naphthalene-like skeleton: 10 ring atoms, the 2 fusion atoms at index 0 and 5."""
    b = bond_A * ANGSTROM_TO_BOHR
    # fused bond along y through the origin; ring centres at x = +-b*sqrt(3)/2
    cx = b * np.sqrt(3.0) / 2.0
    ring = []
    for sign in (+1.0, -1.0):
        c = np.array([sign * cx, 0.0, 0.0])
        for k in range(6):
            ang = np.pi / 6.0 + k * np.pi / 3.0
            ring.append(c + b * np.array([np.cos(ang), np.sin(ang), 0.0]))
    ring = np.array(ring)
    # merge duplicated fusion atoms (x ~ 0)
    uniq: List[np.ndarray] = []
    for p in ring:
        if not any(np.linalg.norm(p - q) < 1e-6 for q in uniq):
            uniq.append(p)
    atoms = np.array(uniq)
    assert atoms.shape[0] == 10
    fusion = [i for i in range(10) if abs(atoms[i, 0]) < 1e-6]
    jitter = np.concatenate([rng.normal(0.0, 0.05, size=(10, 2)),
                             rng.normal(0.0, 0.02, size=(10, 1))], axis=1) * ANGSTROM_TO_BOHR
    return atoms + jitter, fusion


def _place_hydrogens_planar(heavy, fusion, bond):
    centre = heavy.mean(axis=0)
    out = []
    for i in range(heavy.shape[0]):
        if i in fusion:
            continue
        # radially outward from the centre of the ring the atom belongs to
        ring_centre = np.array([np.sign(heavy[i, 0]) * np.abs(heavy[:, 0]).max() / 2.0, 0.0, 0.0])
        v = heavy[i] - ring_centre
        v[2] = 0.0
        v /= np.linalg.norm(v)
        out.append(heavy[i] + bond * v)
    del centre
    return np.array(out)


# ------------------------------------------------------------------- basis

def _shells_for(rng, Z_list, with_d_heavy=True, h_p=True, nprim=3):
    shell_atom, shell_l, shell_nprim, exps, coefs = [], [], [], [], []
    for ia, Z in enumerate(Z_list):
        if Z == 1:
            ls = [0, 0] + ([1] if h_p else [])
        else:
            ls = [0, 0, 0, 1, 1] + ([2] if with_d_heavy else [])
        for l in ls:
            e = np.exp(rng.uniform(np.log(0.1), np.log(100.0), size=nprim))
            e = np.sort(e)[::-1]
            c = rng.uniform(0.1, 1.0, size=nprim)
            shell_atom.append(ia)
            shell_l.append(l)
            shell_nprim.append(nprim)
            exps.extend(e.tolist())
            coefs.extend(c.tolist())
    return (np.array(shell_atom, np.int32), np.array(shell_l, np.int32),
            np.array(shell_nprim, np.int32), np.array(exps), np.array(coefs))


def make_molecule(rng, n_heavy, n_h, layout="box", box_A=4.0, with_d=True, h_p=True):
    """Draw a molecule. layout = 'box' (uniform 3D) or 'naphthalene' (two fused rings)."""
    min_sep = 1.2 * ANGSTROM_TO_BOHR
    bond_h = 1.09 * ANGSTROM_TO_BOHR
    if layout == "naphthalene":
        assert n_heavy == 10 and n_h == 8
        heavy, fusion = _two_fused_hexagons(rng)
        hyd = _place_hydrogens_planar(heavy, fusion, bond_h)
    else:
        heavy = _uniform_box(rng, n_heavy, box_A * ANGSTROM_TO_BOHR, min_sep)
        hyd = _place_hydrogens_random(rng, heavy, n_h, bond_h, 0.9 * ANGSTROM_TO_BOHR)
    Zh = rng.choice([6, 7, 8], size=n_heavy)
    Z = np.concatenate([Zh, np.ones(n_h, dtype=Zh.dtype)]).astype(np.int64)
    xyz = np.concatenate([heavy, hyd], axis=0).astype(np.float64)
    sa, sl, sn, ex, co = _shells_for(rng, Z.tolist(), with_d_heavy=with_d, h_p=h_p)
    return Molecule(Z=Z, xyz=xyz, shell_atom=sa, shell_l=sl, shell_nprim=sn, exps=ex, coefs=co)


# ------------------------------------------------------------- transitions

def make_transitions(rng, nbf: int, n_occ: int, n_states: int,
                     C: Optional[np.ndarray] = None) -> np.ndarray:
    """T^s = C_occ X^s C_vir^T, X^s ~ N(0,1) with ||X^s||_F = 1.

    C defaults to a Euclidean-orthonormal matrix (QR of a Gaussian matrix,
    column signs fixed so that diag(R) > 0).  A caller may pass any other
    coefficient matrix (e.g. S^{-1/2} Q for S-orthonormal orbitals).
    """
    if C is None:
        G = rng.normal(size=(nbf, nbf))
        Q, R = np.linalg.qr(G)
        C = Q * np.sign(np.diag(R))[None, :]
    n_vir = nbf - n_occ
    T = np.empty((n_states, nbf, nbf))
    for s in range(n_states):
        X = rng.normal(size=(n_occ, n_vir))
        X /= np.linalg.norm(X)
        T[s] = C[:, :n_occ] @ X @ C[:, n_occ:].T
    return T


def n_occupied(Z: np.ndarray) -> int:
    return int(np.sum(Z)) // 2


# ----------------------------------------------------------------- configs

CONFIG_NAMES = {
    0: "tiny: 4 heavy + 4 H, 3s2p/2s basis (44 bf), 1 transition, 32^3 grid |q_i|<=5",
    1: "naphthalene-like: 10 heavy + 8 H, 3s2p1d/2s1p basis (190 bf), 12 transitions, 64^3 grid |q_i|<=6",
    2: "naphthalene-like: 10 heavy + 8 H, 190 bf, 12 transitions, 128^3 grid |q_i|<=6",
    3: "random 3D: 30 heavy + 24 H in a 12 A box, 570 bf, 24 transitions, 96^3 grid |q_i|<=8",
}


def make_config(cfg: int, seed: Optional[int] = None) -> Workload:
    """The fixed synthetic workloads (sizes of the paper's Cartesian benchmark class)."""
    if cfg == 2:
        base = make_config(1, seed)
        g = Grid(n=(128, 128, 128), qmin=(-6.0,) * 3, qmax=(6.0,) * 3)
        return Workload(name=CONFIG_NAMES[2], mol=base.mol, T=base.T, grid=g, seed=base.seed)
    if seed is None:
        seed = 1000 + cfg
    rng = np.random.Generator(np.random.PCG64(seed))
    if cfg == 0:
        mol = make_molecule(rng, 4, 4, layout="box", box_A=4.0, with_d=False, h_p=False)
        n_states, grid = 1, Grid(n=(32, 32, 32), qmin=(-5.0,) * 3, qmax=(5.0,) * 3)
    elif cfg == 1:
        mol = make_molecule(rng, 10, 8, layout="naphthalene")
        n_states, grid = 12, Grid(n=(64, 64, 64), qmin=(-6.0,) * 3, qmax=(6.0,) * 3)
    elif cfg == 3:
        mol = make_molecule(rng, 30, 24, layout="box", box_A=12.0)
        n_states, grid = 24, Grid(n=(96, 96, 96), qmin=(-8.0,) * 3, qmax=(8.0,) * 3)
    else:
        raise ValueError(f"unknown config {cfg}")
    T = make_transitions(rng, mol.nbf, n_occupied(mol.Z), n_states)
    return Workload(name=CONFIG_NAMES[cfg], mol=mol, T=T, grid=grid, seed=seed)


def make_serving_request(rng) -> Workload:
    """One request of the serving mix: 2-30 heavy atoms, round(0.8 n) H, 1-24 states, N^3 with N in [32, 96]."""
    n_heavy = int(rng.integers(2, 31))
    n_h = int(round(0.8 * n_heavy))
    n_h = min(n_h, n_heavy)
    box = 12.0 * (n_heavy / 30.0) ** (1.0 / 3.0)
    mol = make_molecule(rng, n_heavy, n_h, layout="box", box_A=max(box, 2.5))
    n_states = int(rng.integers(1, 25))
    N = int(rng.integers(32, 97))
    qmax = float(rng.uniform(5.0, 8.0))
    T = make_transitions(rng, mol.nbf, n_occupied(mol.Z), n_states)
    g = Grid(n=(N, N, N), qmin=(-qmax,) * 3, qmax=(qmax,) * 3)
    return Workload(name=f"serve: {n_heavy} heavy, {n_states} states, {N}^3", mol=mol, T=T, grid=g, seed=-1)


def sample_grid_indices(grid: Grid, n: int, seed: int) -> np.ndarray:
    """A seeded sample of flat grid indices, always including the 8 corners."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tot = grid.n_points
    idx = set(rng.choice(tot, size=min(n, tot), replace=False).tolist())
    nx, ny, nz = grid.n
    for ix in (0, nx - 1):
        for iy in (0, ny - 1):
            for iz in (0, nz - 1):
                idx.add((ix * ny + iy) * nz + iz)
    return np.array(sorted(idx), dtype=np.int64)


# ------------------------------------------------------------- FFT method boxes

def fft_box(mol: Molecule, n, margin_bohr: float = 5.0, scale: float = 2.0):
    """Real-space box of the FFT method (paper Sec. 3, Fig. of the box scale):
    the atoms' bounding box with `margin_bohr` on every side, enlarged
    `scale` times about its centre, sampled at n points per axis.
    Returns (n, xmin, L) as tuples."""
    lo = mol.xyz.min(axis=0) - margin_bohr
    hi = mol.xyz.max(axis=0) + margin_bohr
    centre = 0.5 * (lo + hi)
    L = scale * (hi - lo)
    xmin = centre - 0.5 * L
    return tuple(int(x) for x in n), tuple(float(x) for x in xmin), tuple(float(x) for x in L)
