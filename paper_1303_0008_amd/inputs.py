"""Seeded synthetic density fields for the Vainshtein multigrid solver.

This module only *generates inputs*: it holds none of the solver's
arithmetic (no stencil, no nonlinear root, no multigrid).  Both the CPU
oracle's tests and the GPU path draw their inputs from here, so the two
sides see byte-identical fields.  Its cloud-in-cell deposit builds the
Zel'dovich density the way the workload recipe states; the mass assignment
the library offers (and the oracle's, pinned by moment and lattice tests of
its own) is a separate implementation.

Layout of every 3D field: a C-contiguous numpy array of shape
``(n2, n1, n0)`` -- z slowest, x fastest -- i.e. cell ``(i, j, k)`` sits at
flat index ``(k*n1 + j)*n0 + i`` and has its centre at ``((i+.5)h, (j+.5)h,
(k+.5)h)`` in a unit box.

The paper's workloads (N-body snapshots started from MPGRAFIC initial
conditions, Sec. V) are not available; the recipes below stand in for them
with the shapes and statistics of the benchmark configurations:

* ``tophat``      -- mean-subtracted spherical top-hat (the spherical
                     overdensity test of Sec. IV.C).
* ``lognormal``   -- exp of a Gaussian random field with power-law spectrum,
                     normalised to mean density 1 (so ``delta >= -1``).
* ``zeldovich_cic`` -- particles on a lattice displaced by a Zel'dovich field
                     and deposited with cloud-in-cell weights.
* ``patch_set``   -- many cubic refinement patches of uneven sizes, each with
                     its own lognormal field.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

BASE_SEED = 20130008


def _shape(n):
    if np.isscalar(n):
        n = (int(n),) * 3
    n0, n1, n2 = (int(v) for v in n)
    return n0, n1, n2


def sha256(a: np.ndarray) -> str:
    """Hex digest of the raw bytes of a contiguous float64 array."""
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def cell_centres(n):
    """Per-axis cell-centre coordinates (x, y, z) of a unit box with ``n`` cells."""
    n0, n1, n2 = _shape(n)
    return ((np.arange(n0) + 0.5) / n0, (np.arange(n1) + 0.5) / n1, (np.arange(n2) + 0.5) / n2)


def tophat(n, radius=0.1, amplitude=50.0, centre=(0.5, 0.5, 0.5)):
    """Top-hat sphere: ``amplitude`` strictly inside ``radius`` of ``centre``, 0 outside,
    then the mean is subtracted so that the periodic field has zero mean."""
    x, y, z = cell_centres(n)
    r2 = ((z[:, None, None] - centre[2]) ** 2 + (y[None, :, None] - centre[1]) ** 2
          + (x[None, None, :] - centre[0]) ** 2)
    d = np.where(r2 < radius * radius, amplitude, 0.0)
    return np.ascontiguousarray(d - d.mean())


def tophat_region(shape, h, corner, domain_n, radius=0.1, amplitude=50.0, centre=(0.5, 0.5, 0.5)):
    """The top-hat of ``tophat(domain_n, ...)`` sampled at the cell centres of a
    region of ``shape`` = (n0, n1, n2) cells of size ``h`` whose cell (0,0,0)
    corner sits at ``corner`` (box units; taken modulo 1), minus the same mean
    as the domain field, shaped (n2, n1, n0)."""
    n0, n1, n2 = shape
    dom = np.where(_tophat_r2(cell_centres(domain_n), centre) < radius * radius, amplitude, 0.0)
    axes = [np.mod(corner[a] + (np.arange(n) + 0.5) * h, 1.0) for a, n in enumerate((n0, n1, n2))]
    d = np.where(_tophat_r2(axes, centre) < radius * radius, amplitude, 0.0)
    return np.ascontiguousarray(d - dom.mean())


def _tophat_r2(axes, centre):
    x, y, z = axes
    return ((z[:, None, None] - centre[2]) ** 2 + (y[None, :, None] - centre[1]) ** 2
            + (x[None, None, :] - centre[0]) ** 2)


def gaussian_field(n, spectral_index, seed, std=1.0, kmax_cells=None):
    """Gaussian random field with power spectrum P(k) proportional to k**spectral_index.

    White noise (PCG64 ``standard_normal`` in C order) is Fourier transformed,
    multiplied by |k|**(spectral_index/2) with k = 2*pi*(integer frequency) and
    the k = 0 mode removed, optionally truncated at |m| > kmax_cells (integer
    frequency units), transformed back and rescaled to standard deviation ``std``.
    """
    n0, n1, n2 = _shape(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((n2, n1, n0))
    wk = np.fft.rfftn(white)
    mz = np.fft.fftfreq(n2) * n2
    my = np.fft.fftfreq(n1) * n1
    mx = np.fft.rfftfreq(n0) * n0
    m2 = mz[:, None, None] ** 2 + my[None, :, None] ** 2 + mx[None, None, :] ** 2
    kmag = 2.0 * np.pi * np.sqrt(m2)
    with np.errstate(divide="ignore"):
        amp = np.where(m2 > 0, kmag ** (0.5 * spectral_index), 0.0)
    if kmax_cells is not None:
        amp = np.where(m2 <= kmax_cells * kmax_cells, amp, 0.0)
    g = np.fft.irfftn(wk * amp, s=(n2, n1, n0), axes=(0, 1, 2))
    s = g.std()
    if s > 0:
        g *= std / s
    return np.ascontiguousarray(g)


def lognormal(n, seed, sigma=1.0, spectral_index=-2.0):
    """Lognormal density contrast: g Gaussian (P ~ k**index, std sigma),
    rho = exp(g) normalised to unit mean, delta = rho - 1 (exact zero mean, delta >= -1)."""
    g = gaussian_field(n, spectral_index, seed, std=sigma)
    rho = np.exp(g - g.max())          # shift avoids overflow; normalisation removes it
    rho /= rho.mean()
    d = rho - 1.0
    d -= d.mean()                        # remove the last ulp-level offset
    return np.ascontiguousarray(d)


def _displacement(n, seed, spectral_index, kcut_cells):
    """Zel'dovich displacement Psi with div(Psi) = -delta_lin for a unit-std
    linear field delta_lin with P ~ k**index, truncated at |m| <= kcut_cells."""
    n0, n1, n2 = _shape(n)
    dl = gaussian_field(n, spectral_index, seed, std=1.0, kmax_cells=kcut_cells)
    dk = np.fft.rfftn(dl)
    kz = 2 * np.pi * np.fft.fftfreq(n2) * n2
    ky = 2 * np.pi * np.fft.fftfreq(n1) * n1
    kx = 2 * np.pi * np.fft.rfftfreq(n0) * n0
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    out = []
    for kc in (kx[None, None, :], ky[None, :, None], kz[:, None, None]):
        out.append(np.fft.irfftn(1j * kc * dk * inv, s=(n2, n1, n0), axes=(0, 1, 2)))
    return out  # (Psi_x, Psi_y, Psi_z), each (n2, n1, n0)


def cic_deposit(n, px, py, pz):
    """Cloud-in-cell density rho/rho_mean of unit-mass particles at positions in [0,1)."""
    n0, n1, n2 = _shape(n)
    npart = px.size
    acc = np.zeros(n0 * n1 * n2)
    parts = []
    for p, nd in ((px, n0), (py, n1), (pz, n2)):
        u = p * nd - 0.5
        i0 = np.floor(u)
        t = u - i0
        i0 = i0.astype(np.int64) % nd
        parts.append((i0, (i0 + 1) % nd, 1.0 - t, t))
    (x0, x1, wx0, wx1), (y0, y1, wy0, wy1), (z0, z1, wz0, wz1) = parts
    for zi, wz in ((z0, wz0), (z1, wz1)):
        for yi, wy in ((y0, wy0), (y1, wy1)):
            base = (zi * n1 + yi) * n0
            wzy = wz * wy
            for xi, wx in ((x0, wx0), (x1, wx1)):
                acc += np.bincount(base + xi, weights=wzy * wx, minlength=acc.size)
    rho = acc.reshape(n2, n1, n0) * (n0 * n1 * n2 / npart)
    return rho


def _zeldovich_positions(n, seed, spectral_index, kcut_frac_nyquist):
    n0, n1, n2 = _shape(n)
    kcut_cells = kcut_frac_nyquist * 0.5 * min(n0, n1, n2)   # |k| <= f*pi*N  <=>  |m| <= f*N/2
    psi = _displacement((n0, n1, n2), seed, spectral_index, kcut_cells)
    x, y, z = cell_centres((n0, n1, n2))
    q = np.meshgrid(z, y, x, indexing="ij")[::-1]            # (qx, qy, qz)
    return q, psi


def _deposit_displaced(n, q, psi, amplitude):
    p = [np.mod(qc + amplitude * pc, 1.0).ravel() for qc, pc in zip(q, psi)]
    rho = cic_deposit(n, p[0], p[1], p[2])
    d = rho - 1.0
    d -= d.mean()
    return np.ascontiguousarray(d)


def zeldovich_cic(n, seed, amplitude, spectral_index=-1.5, kcut_frac_nyquist=0.25):
    """Density contrast of n^3 lattice particles displaced by amplitude*Psi (Zel'dovich),
    deposited with CIC.  The linear spectrum is P ~ k**index up to
    kcut_frac_nyquist * k_Nyquist (k_Nyquist = pi*n) and zero above."""
    q, psi = _zeldovich_positions(n, seed, spectral_index, kcut_frac_nyquist)
    return _deposit_displaced(n, q, psi, amplitude)


def zeldovich_particles(n, seed, amplitude, spectral_index=-1.5, kcut_frac_nyquist=0.25):
    """Positions (N x 3 array, columns x, y, z, in [0, 1)) of the n^3 lattice
    particles of zeldovich_cic after the same Zel'dovich displacement."""
    q, psi = _zeldovich_positions(n, seed, spectral_index, kcut_frac_nyquist)
    return np.ascontiguousarray(np.stack([np.mod(qc + amplitude * pc, 1.0).ravel() for qc, pc in zip(q, psi)],
                                         axis=1))


def scan_zeldovich_amplitude(n, seed, amplitudes, spectral_index=-1.5, kcut_frac_nyquist=0.25):
    """max(delta) for each displacement amplitude (the displacement field is built once).

    max(delta) is not monotone in the amplitude: once streams cross, Zel'dovich
    particles keep moving through the caustics and the peak density falls again.
    """
    q, psi = _zeldovich_positions(n, seed, spectral_index, kcut_frac_nyquist)
    return [float(_deposit_displaced(n, q, psi, a).max()) for a in amplitudes]


# Frozen displacement amplitude, in units of the unit-std linear field's displacement.
# A scan at 256^3 (seed BASE_SEED+3, amplitudes 0.8..2.0 step 0.1) gives the largest
# peak density at 1.2: max(delta) = 143.5, std(delta) = 1.79.  The recipe's caustics
# cap max(delta) near 1.4e2 at this resolution, so 1e3 is not reachable; 1.2 is the
# amplitude closest to it.
ZELDOVICH_AMPLITUDE = 1.2


@dataclasses.dataclass
class Patch:
    n: int                      # cells per side
    origin: tuple               # integer cell offset of cell (0,0,0) on the 1/h lattice
    delta: np.ndarray           # (n, n, n) density contrast


def patch_set(count=96, sides=(16, 24, 32, 48, 64), seed=BASE_SEED + 4, lattice=512,
              sigma=1.5, spectral_index=-2.0):
    """Refinement patches: ``count`` cubes with side drawn uniformly from ``sides``,
    origins uniform on the ``lattice`` (cells of size 1/lattice, periodic box), and
    per patch a lognormal field generated on the patch's own periodic n^3 grid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = rng.choice(np.asarray(sides), size=count)
    origin = rng.integers(0, lattice, size=(count, 3))
    out = []
    for p in range(count):
        n = int(side[p])
        d = lognormal(n, seed * 1000 + p, sigma=sigma, spectral_index=spectral_index)
        out.append(Patch(n=n, origin=tuple(int(v) for v in origin[p]), delta=d))
    return out


def uniform_guess(n, seed, half_width=0.05):
    """Initial guess uniform in [-half_width, half_width] (uniform-density test, Sec. IV.A)."""
    n0, n1, n2 = _shape(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.uniform(-half_width, half_width, size=(n2, n1, n0)))


# ---------------------------------------------------------------------------
# Benchmark / parity workloads (sizes and statistics of the five configurations)
# ---------------------------------------------------------------------------
WORKLOADS = {
    "tophat32": dict(n=32, alpha=0.05, kappa=1.5, tol=1e-10),
    "lognormal128": dict(n=128, alpha=0.1, kappa=1.5, tol=1e-8),
    "zeldovich256": dict(n=256, alpha=0.2, kappa=1.5, tol=1e-8),
    "patches96": dict(n=None, alpha=0.1, kappa=1.5, tol=1e-8),
    "lognormal512a": dict(n=512, alpha=0.2, kappa=1.5, tol=1e-8),
    "lognormal512b": dict(n=512, alpha=-0.2, kappa=1.5, tol=1e-8),
}


def workload_delta(name, n=None):
    """Density contrast of a named workload (optionally at a different size ``n``)."""
    if name == "tophat32":
        return tophat(n or 32)
    if name == "lognormal128":
        return lognormal(n or 128, BASE_SEED + 2, sigma=1.0)
    if name == "zeldovich256":
        return zeldovich_cic(n or 256, BASE_SEED + 3, ZELDOVICH_AMPLITUDE)
    if name in ("lognormal512a", "lognormal512b"):
        return lognormal(n or 512, BASE_SEED + 5, sigma=1.5)
    raise KeyError(name)
