"""Checks of the seeded input generators (no ISDF arithmetic here)."""
import dataclasses

import numpy as np

import synth
from synth import orbitals as so


def test_plane_wave_counts_match_the_recipe():
    """Plane waves inside the 30 Ha sphere and the FFT box."""
    counts = {name: int(so._sphere_mask(so.WORKLOADS[name]).sum()) for name in ("water8", "water64", "sio2")}
    assert counts == {"water8": 11018, "water64": 100929, "sio2": 52923}


def _small_large(n_orb=12):
    return dataclasses.replace(so.WORKLOADS["water8"], n_phi=n_orb, n_psi=n_orb, large=True)


def test_large_generator_small_box():
    """The threaded generator of the 512-water box, run on an 8-water-sized
    box: orthonormal columns, independent of the thread count."""
    wl = _small_large()
    x = so.make_orbitals_large(wl, threads=4)
    assert x.shape == (wl.n_r, 12) and x.dtype == np.complex128
    assert np.max(np.abs(x.conj().T @ x - np.eye(12))) <= 1e-12
    y = so.make_orbitals_large(wl, threads=1)
    assert np.array_equal(x, y)


def test_large_generator_orbitals_are_band_limited():
    """Every column lies in span{E(r) e^{ik.r} e^{iG.r}: G in the sphere}:
    dividing by the envelope and the Bloch phase leaves a field whose
    spectrum vanishes outside the sphere (up to rounding)."""
    wl = _small_large(3)
    phi = so.make_orbitals_large(wl, threads=2)
    env = so.envelope(wl, so.atom_positions(wl))
    n = wl.n
    L = wl.box_angstrom * so.BOHR_PER_ANGSTROM
    ax = np.arange(n) * L / n
    k = 2 * np.pi / L * np.asarray(wl.k_frac)
    ph = np.exp(1j * (k[0] * ax[:, None, None] + k[1] * ax[None, :, None] + k[2] * ax[None, None, :]))
    mask = so._sphere_mask(wl)
    for j in range(3):
        u = phi[:, j].reshape(n, n, n) / (env.reshape(n, n, n) * ph)
        spec = np.fft.fftn(u)
        assert np.linalg.norm(spec[~mask]) <= 1e-8 * np.linalg.norm(spec[mask])
