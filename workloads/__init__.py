"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only draws numbers: geometries, shell lists with raw (unnormalised)
exponents and contraction coefficients, densities and primitive-quartet sets.
It holds none of the method's arithmetic (no normalisation, no integrals), so
both sides of every parity test can take their inputs from here without
sharing any computation.

The molecules and cc-pVXZ basis sets used in the paper's evaluation are not
available; these molecule-shaped inputs stand in for them.  Shell compositions
3s2p1d / 4s3p2d1f / 5s4p3d2f1g mirror the l_max = 2 / 3 / 4 levels of the
correlation-consistent basis families (Sec. V-C).

Units: coordinates are returned in bohr (drawn in angstrom, converted with
the CODATA 2018 Bohr radius); exponents are in bohr^-2.
"""
from __future__ import annotations

import dataclasses

import numpy as np

BOHR_ANGSTROM = 0.529177210903          # CODATA 2018 Bohr radius in angstrom
ANGSTROM_TO_BOHR = 1.0 / BOHR_ANGSTROM


def nsph(l: int) -> int:
    """Pure-spherical functions per shell (p kept as x, y, z)."""
    return 2 * l + 1


@dataclasses.dataclass
class Basis:
    """A flat shell list: shell s has angular momentum l[s], nprim[s] primitives
    (exponents/coefficients at exps[off[s]:off[s]+nprim[s]]) and centre
    centers[s] in bohr.  Coefficients are raw draws, not normalised."""
    l: np.ndarray          # int32 [nshell]
    nprim: np.ndarray      # int32 [nshell]
    centers: np.ndarray    # float64 [nshell, 3] (bohr)
    exps: np.ndarray       # float64 [sum nprim] (bohr^-2)
    coefs: np.ndarray      # float64 [sum nprim] (raw)
    atom: np.ndarray       # int32 [nshell] owning atom
    atoms: np.ndarray      # float64 [natom, 3] (bohr)

    @property
    def nshell(self) -> int:
        return int(self.l.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(nsph(int(x)) for x in self.l))

    def prim_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.nprim)]).astype(np.int64)

    def shell_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([nsph(int(x)) for x in self.l])]).astype(np.int64)

    def subset(self, shells) -> "Basis":
        """The basis restricted to the listed shells (in that order)."""
        shells = np.asarray(shells, dtype=np.int64)
        off = self.prim_offsets()
        idx = np.concatenate([np.arange(off[s], off[s + 1]) for s in shells]) if len(shells) else np.zeros(0, np.int64)
        return Basis(self.l[shells].copy(), self.nprim[shells].copy(), self.centers[shells].copy(),
                     self.exps[idx].copy(), self.coefs[idx].copy(), self.atom[shells].copy(), self.atoms.copy())


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def build_basis(atoms_bohr: np.ndarray, template, rng, exp_range, coef_range=(0.1, 1.0)) -> Basis:
    """Place `template` shells on every atom.  template: list of (l, nprim) where
    nprim is an int or a (lo, hi) inclusive range drawn per shell.  Draw order:
    atom-major, then shell, then nprim, exponents (sorted descending), coefficients."""
    ls, nps, cens, exps, coefs, own = [], [], [], [], [], []
    for a, pos in enumerate(atoms_bohr):
        for (l, np_spec) in template:
            if isinstance(np_spec, tuple):
                k = int(rng.integers(np_spec[0], np_spec[1] + 1))
            else:
                k = int(np_spec)
            e = np.sort(_log_uniform(rng, exp_range[0], exp_range[1], k))[::-1]
            c = rng.uniform(coef_range[0], coef_range[1], size=k)
            ls.append(l); nps.append(k); cens.append(pos); exps.append(e); coefs.append(c); own.append(a)
    return Basis(np.array(ls, np.int32), np.array(nps, np.int32), np.array(cens, np.float64).reshape(-1, 3),
                 np.concatenate(exps).astype(np.float64), np.concatenate(coefs).astype(np.float64),
                 np.array(own, np.int32), np.asarray(atoms_bohr, np.float64).reshape(-1, 3))


def grow_molecule(rng, natom: int, bond=(1.0, 1.6), min_dist=0.9) -> np.ndarray:
    """Random near-molecular geometry in angstrom: each new atom sits at a bond
    length U[bond] in a uniformly random direction from a random existing atom;
    a placement closer than min_dist to any atom is redrawn."""
    pos = [np.zeros(3)]
    while len(pos) < natom:
        host = pos[int(rng.integers(0, len(pos)))]
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        cand = host + rng.uniform(bond[0], bond[1]) * v
        if min(np.linalg.norm(cand - p) for p in pos) >= min_dist:
            pos.append(cand)
    return np.array(pos)


def psd_density(n: int, seed: int) -> np.ndarray:
    """Symmetric positive semi-definite density D = A A^T / n, A ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, n))
    d = a @ a.T / max(n, 1)
    return 0.5 * (d + d.T)


# ---------------------------------------------------------------------------
# The workloads.
# ---------------------------------------------------------------------------

def tiny_system(seed: int = 1001):
    """4 atoms uniform in a 4 A cube; per atom s(3 prims), s(1), p(1); exponents
    log-uniform [0.1, 50]; coefficients U[0.1, 1].  Unscreened.  N = 20
    (12 shells, 78 shell pairs, 3081 unique shell quartets)."""
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(0.0, 4.0, size=(4, 3)) * ANGSTROM_TO_BOHR
    basis = build_basis(atoms, [(0, 3), (0, 1), (1, 1)], rng, (0.1, 50.0))
    D = psd_density(basis.nbf, seed + 1000)
    return basis, D


def molecule_3s2p1d(seed: int = 1002, natom: int = 30):
    """30-atom random near-molecular geometry (bonds U[1.0, 1.6] A, minimum
    spacing 0.9 A); per atom s, s, s, p, p, d each with U{1..6} primitives;
    exponents log-uniform [0.05, 5e3]; coefficients U[0.1, 1]; spherical d.
    N = 420, 180 shells.  Screened at tau = 1e-12."""
    rng = np.random.default_rng(seed)
    atoms = grow_molecule(rng, natom) * ANGSTROM_TO_BOHR
    tmpl = [(0, (1, 6)), (0, (1, 6)), (0, (1, 6)), (1, (1, 6)), (1, (1, 6)), (2, (1, 6))]
    basis = build_basis(atoms, tmpl, rng, (0.05, 5.0e3))
    D = psd_density(basis.nbf, seed + 1000)
    return basis, D


def prim_quartets(l: int, n: int, seed: int = 1003, box: float = 6.0, exp_range=(0.1, 100.0)):
    """n independent primitive quartets of class (ll|ll): four centres uniform
    in a `box` A cube (returned in bohr, [n, 4, 3]) and four exponents
    log-uniform in exp_range ([n, 4]).  The coefficient is 1 on normalised
    primitives.  Each class draws from its own stream (seed + 10 l)."""
    rng = np.random.default_rng(seed + 10 * l)
    centers = rng.uniform(0.0, box, size=(n, 4, 3)) * ANGSTROM_TO_BOHR
    exps = _log_uniform(rng, exp_range[0], exp_range[1], 4 * n).reshape(n, 4)
    return centers, exps


def random_small_basis(seed: int, natom: int = 3, lmax: int = 2, maxprim: int = 3,
                       box: float = 3.0, exp_range=(0.2, 20.0)) -> Basis:
    """Small random basis for property tests: natom atoms in a `box` A cube,
    one shell of each l <= lmax per atom with U{1..maxprim} primitives."""
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(0.0, box, size=(natom, 3)) * ANGSTROM_TO_BOHR
    tmpl = [(l, (1, maxprim)) for l in range(lmax + 1)]
    return build_basis(atoms, tmpl, rng, exp_range)


CONFIGS = {
    "tiny": dict(builder=tiny_system, tau=0.0),
    "mol30_3s2p1d": dict(builder=molecule_3s2p1d, tau=1.0e-12),
}


def batch_systems(seed: int = 1004, n: int = 64, natom=(5, 60), lmax: int = 3, nprim=(1, 8), with_density=True):
    """n molecules of U{natom} atoms each, grown like molecule_3s2p1d, with
    the shell set of the given l_max per atom (l_max 3: 4s3p2d1f) and U{nprim}
    primitives per shell; exponents log-uniform [0.05, 5e3].  Returns a list
    of (basis, density), each density from its own stream (None without
    with_density)."""
    rng = np.random.default_rng(seed)
    shells = {2: [0, 0, 0, 1, 1, 2], 3: [0, 0, 0, 0, 1, 1, 1, 2, 2, 3],
              4: [0] * 5 + [1] * 4 + [2] * 3 + [3] * 2 + [4]}[lmax]
    out = []
    for k in range(n):
        na = int(rng.integers(natom[0], natom[1] + 1))
        atoms = grow_molecule(rng, na) * ANGSTROM_TO_BOHR
        basis = build_basis(atoms, [(l, nprim) for l in shells], rng, (0.05, 5.0e3))
        out.append((basis, psd_density(basis.nbf, seed + 1000 + k) if with_density else None))
    return out
