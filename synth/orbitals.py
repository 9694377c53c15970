"""Synthetic Kohn-Sham-like complex orbitals on a periodic real-space grid.

Stand-ins for the paper's liquid-water and SiO2 systems (the paper's own
structures and orbitals are not published).  Recipe per orbital:

* random complex plane-wave coefficients c_G ~ CN(0, 1) for every reciprocal
  vector G = 2*pi*m/L with |G|^2/2 <= Ecut and m inside the FFT box
  [-n/2, n/2-1]^3;
* u(r) = inverse FFT of the coefficient box;
* an atom envelope E(r) = sum_a exp(-|r - R_a|^2_mic / (2 sigma^2)) with
  minimum-image distances, sigma = 0.6 Angstrom;
* a Bloch phase exp(i k.r) with k = 2*pi/L * k_frac;
* phi = E * u * exp(i k.r), then the set is orthonormalised on the grid by a
  Householder QR, so that Phi^H Phi = I (no volume element).

Grid point p = (i*n + j)*n + k sits at (i, j, k) * h with h = L/n.  Orbitals
are returned r-major: a C-contiguous complex128 array of shape (N_r, N_e).

Every random draw comes from numpy's PCG64 seeded with 1000*cfg + purpose:
1 atoms, 2 coefficients, 3 K-means seeds, 4 loss field, 5 probe entries.
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177
SIGMA_ANGSTROM = 0.6
MIN_SEPARATION_ANGSTROM = 0.9


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cfg: int            # seed base: seeds are 1000*cfg + purpose
    n: int              # grid points per edge (cubic grid, N_r = n^3)
    box_angstrom: float
    n_phi: int
    n_psi: int
    aliased: bool       # Psi is Phi (same array)
    n_mu: int
    kmeans_iters: int
    k_frac: tuple
    natoms: int = 0
    sio2: bool = False
    ecut_ha: float = 30.0
    rblock: int = 0     # 0: one r-block

    @property
    def n_r(self) -> int:
        return self.n ** 3


WORKLOADS = {
    # 8-water-like box: 24 atoms in a 6.2 A cube on a 24^3 grid.
    "water8": Workload("water8", 1, 24, 6.2, 32, 32, True, 256, 30, (0.25, 0.0, 0.0), natoms=24),
    # 64-water-like box: 192 atoms in a 12.4 A cube on a 64^3 grid.
    "water64": Workload("water64", 2, 64, 12.4, 256, 256, True, 2048, 50, (0.25, 0.25, 0.0), natoms=192),
    # SiO2-like crystal: 24 Si + 48 O in a 10 A cube on a 72^3 grid, Psi adds virtuals.
    "sio2": Workload("sio2", 3, 72, 10.0, 192, 384, False, 3072, 50, (0.25, 0.25, 0.0), sio2=True),
    # adjoint workload: water64 shape with a loss field g.
    "water64_adj": Workload("water64_adj", 4, 64, 12.4, 256, 256, True, 2048, 50, (0.25, 0.25, 0.0), natoms=192),
    # 512-water-like box: 1536 atoms in a 24.8 A cube on a 128^3 grid.
    "water512": Workload("water512", 5, 128, 24.8, 1024, 1024, True, 8192, 50, (0.25, 0.25, 0.0),
                         natoms=1536, rblock=65536),
}


def _rng(cfg: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * cfg + purpose))


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def atom_positions(wl: Workload) -> np.ndarray:
    """Atom centres in Bohr, shape (natoms, 3)."""
    rng = _rng(wl.cfg, 1)
    L = wl.box_angstrom * BOHR_PER_ANGSTROM
    if wl.sio2:
        # 24 Si on a 2x3x4 lattice of the cube, O at the midpoints of each Si's
        # +x and +y periodic neighbour bonds; every coordinate jittered by
        # +-0.1 A.
        dims = (2, 3, 4)
        si = []
        for a in range(dims[0]):
            for b in range(dims[1]):
                for c in range(dims[2]):
                    si.append(((a + 0.5) / dims[0], (b + 0.5) / dims[1], (c + 0.5) / dims[2]))
        si = np.array(si) * L
        ox = []
        for s in si:
            for ax in (0, 1):
                step = np.zeros(3)
                step[ax] = L / dims[ax]
                ox.append(np.mod(s + 0.5 * step, L))
        pos = np.concatenate([si, np.array(ox)], axis=0)
        jitter = rng.uniform(-0.1, 0.1, size=pos.shape) * BOHR_PER_ANGSTROM
        return np.mod(pos + jitter, L)
    dmin = MIN_SEPARATION_ANGSTROM * BOHR_PER_ANGSTROM
    pos = np.empty((0, 3))
    while pos.shape[0] < wl.natoms:
        cand = rng.uniform(0.0, L, size=3)
        if pos.shape[0]:
            d = _min_image(pos - cand, L)
            if np.min(np.einsum("ij,ij->i", d, d)) < dmin * dmin:
                continue
        pos = np.vstack([pos, cand])
    return pos


def envelope(wl: Workload, atoms: np.ndarray) -> np.ndarray:
    """E(r) on the grid, flattened r-major, float64 (N_r,)."""
    n = wl.n
    L = wl.box_angstrom * BOHR_PER_ANGSTROM
    h = L / n
    sig = SIGMA_ANGSTROM * BOHR_PER_ANGSTROM
    ax = np.arange(n) * h
    env = np.zeros((n, n, n))
    for R in atoms:
        # separable Gaussian: exp(-(dx^2+dy^2+dz^2)/2s^2) = gx*gy*gz
        g = [np.exp(-_min_image(ax - R[a], L) ** 2 / (2 * sig * sig)) for a in range(3)]
        env += g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
    return env.reshape(-1)


def _sphere_mask(wl: Workload) -> np.ndarray:
    n = wl.n
    L = wl.box_angstrom * BOHR_PER_ANGSTROM
    m = np.fft.fftfreq(n, d=1.0 / n)  # integers in FFT order, [-n/2, n/2-1]
    G = 2 * np.pi * m / L
    g2 = G[:, None, None] ** 2 + G[None, :, None] ** 2 + G[None, None, :] ** 2
    return 0.5 * g2 <= wl.ecut_ha


def make_orbitals(wl: Workload, n_orb: int | None = None) -> np.ndarray:
    """Orthonormal complex orbitals, complex128 (N_r, n_orb), r-major.

    For a non-aliased workload the n_psi orbitals are generated and
    orthonormalised jointly; Phi is their first n_phi columns.
    """
    if n_orb is None:
        n_orb = wl.n_psi if not wl.aliased else wl.n_phi
    n = wl.n
    L = wl.box_angstrom * BOHR_PER_ANGSTROM
    h = L / n
    atoms = atom_positions(wl)
    env = envelope(wl, atoms)
    mask = _sphere_mask(wl)
    npw = int(mask.sum())
    rng = _rng(wl.cfg, 2)
    idx = np.arange(n) * h
    k = 2 * np.pi / L * np.asarray(wl.k_frac, dtype=np.float64)
    phase = np.exp(1j * (k[0] * idx[:, None, None] + k[1] * idx[None, :, None] + k[2] * idx[None, None, :]))
    mod = (env.reshape(n, n, n) * phase).reshape(-1)
    out = np.empty((wl.n_r, n_orb), dtype=np.complex128)
    box = np.zeros((n, n, n), dtype=np.complex128)
    for j in range(n_orb):
        c = (rng.standard_normal(npw) + 1j * rng.standard_normal(npw)) * np.sqrt(0.5)
        box[...] = 0
        box[mask] = c
        u = np.fft.ifftn(box) * (n ** 3)
        out[:, j] = u.reshape(-1) * mod
    q, _ = np.linalg.qr(out, mode="reduced")
    return np.ascontiguousarray(q)


def random_orthonormal(n_r: int, n_orb: int, seed: int, real: bool = False) -> np.ndarray:
    """Plain random orthonormal columns (tiny test inputs), complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((n_r, n_orb))
    if not real:
        x = x + 1j * rng.standard_normal((n_r, n_orb))
    q, _ = np.linalg.qr(x, mode="reduced")
    return np.ascontiguousarray(q.astype(np.complex128))


def init_centroids(prob: np.ndarray, n: int, n_mu: int, seed: int) -> np.ndarray:
    """K-means seeds: n_mu distinct grid points drawn without replacement with
    probability proportional to the nonnegative field `prob` (uniform if
    None).  Returned in grid units, float64 (n_mu, 3), as (i, j, k)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_r = n ** 3
    if prob is None:
        p = None
    else:
        p = np.asarray(prob, dtype=np.float64)
        p = p / p.sum()
    pts = rng.choice(n_r, size=n_mu, replace=False, p=p)
    i, rem = np.divmod(pts, n * n)
    j, k = np.divmod(rem, n)
    return np.stack([i, j, k], axis=1).astype(np.float64)


def loss_field(n_r: int, seed: int) -> np.ndarray:
    """g(r) ~ U[0.5, 1.5], float64 (N_r,)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.5, 1.5, size=n_r)


_CACHE_DIR = os.environ.get("ISDF_SYNTH_CACHE", "/tmp/isdf_synth_cache")


def make_workload(name: str, cache: bool = True) -> dict:
    """Everything a run of workload `name` needs: orbitals, seeds, g field.

    Returns dict(wl, phi, psi, c0, g, env).  For an aliased workload psi is
    phi (the same array object).  Results are cached as .npy under
    $ISDF_SYNTH_CACHE (default /tmp/isdf_synth_cache).
    """
    wl = WORKLOADS[name]
    path = os.path.join(_CACHE_DIR, f"{name}.npz")
    orb = env = None
    if cache and os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            orb, env = z["orb"], z["env"]
    if orb is None:
        orb = make_orbitals(wl)
        env = envelope(wl, atom_positions(wl))
        if cache:
            os.makedirs(_CACHE_DIR, exist_ok=True)
            tmp = path + ".tmp.npz"
            np.savez(tmp, orb=orb, env=env)
            os.replace(tmp, path)
    if wl.aliased:
        phi = psi = orb
    else:
        psi = orb
        phi = orb[:, : wl.n_phi]  # strided view: leading dimension n_psi
    c0 = init_centroids(env * env, wl.n, wl.n_mu, 1000 * wl.cfg + 3)
    g = loss_field(wl.n_r, 1000 * wl.cfg + 4)
    return dict(wl=wl, phi=phi, psi=psi, c0=c0, g=g, env=env)
