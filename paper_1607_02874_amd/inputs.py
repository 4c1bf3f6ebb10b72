"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only generates data: voxel maps (0 = fluid, 1 = inert solid,
2 = catalytic solid) and workload parameters.  It holds none of the lattice
Boltzmann arithmetic, so the HIP library and the FP64 oracle can both be fed
from it without sharing any of the method.

Geometry recipe (stand-in for the paper's nanoporous gold sample, which is
2-D disk carving at porosity 0.70, "Experimental details and Nanoporous
Catalyst reconstruction"): a periodic Gaussian random field with Gaussian
covariance exp(-r^2 / (2 ell^2)) is level-cut so that exactly
round((1 - phi) * n_block) voxels of the porous block are solid.  The solid
phase is bicontinuous for phi in [0.5, 0.75].  Every porous-solid voxel is
catalytic: in the paper each solid node in contact with gas acts as a
catalytic node (Appendix, sputtering boundary condition).
"""

from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

FLUID, INERT, CATALYTIC = 0, 1, 2


def grf_solid_mask(shape, phi, ell, seed):
    """Boolean solid mask of a periodic Gaussian random field level cut.

    shape is (nz, ny, nx).  White noise N(0, 1) is drawn from
    ``numpy.random.default_rng(seed)`` in C order, filtered in Fourier space
    by the amplitude exp(-k^2 ell^2 / 4) (covariance exp(-r^2 / 2 ell^2)),
    and the round((1 - phi) * n) largest values become solid; ties are
    broken by flat index, so the porosity is exact.
    """
    nz, ny, nx = shape
    n = nz * ny * nx
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    kz = 2.0 * np.pi * np.fft.fftfreq(nz)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    kx = 2.0 * np.pi * np.fft.rfftfreq(nx)
    spec = np.fft.rfftn(noise)
    del noise
    filt = np.exp(-(kz[:, None, None] ** 2) * ell * ell / 4.0)
    spec *= filt
    spec *= np.exp(-(ky[None, :, None] ** 2) * ell * ell / 4.0)
    spec *= np.exp(-(kx[None, None, :] ** 2) * ell * ell / 4.0)
    field = np.fft.irfftn(spec, s=shape, axes=(0, 1, 2)).ravel()
    del spec
    n_solid = int(round((1.0 - phi) * n))
    solid = np.zeros(n, dtype=bool)
    if n_solid > 0:
        # stable sort on the negated field: largest first, ties by flat index
        order = np.argsort(-field, kind="stable")
        solid[order[:n_solid]] = True
    return solid.reshape(shape)


def porous_slab(nx, ny, nz, phi, ell, seed, x_lo=4, x_hi=None, solid_flag=CATALYTIC):
    """Voxel map (nz, ny, nx) uint8 with a GRF porous block in x in [x_lo, x_hi).

    The planes outside the block are empty gas buffers; y and z are periodic.
    """
    if x_hi is None:
        x_hi = nx - 4
    vox = np.zeros((nz, ny, nx), dtype=np.uint8)
    block = grf_solid_mask((nz, ny, x_hi - x_lo), phi, ell, seed)
    vox[:, :, x_lo:x_hi][block] = solid_flag
    return vox


def disk_ingot(w, h=200, length=250, width=500, phi=0.70, diameter=3.0, seed=0, tol=0.005):
    """The paper's 2-D reactor ("Experimental details and Nanoporous Catalyst
    reconstruction"; Table 1): a (1, width, length) voxel map, flow along x,
    with a rectangular catalytic ingot w along the flow and h across it,
    centred in the domain, made porous by carving disks of the given
    diameter (30 nm = 3 lattice units) around uniformly random centres inside
    the rectangle until its porosity reaches phi within tol.  One inert wall
    row at y = 0 bounds the tube (y is periodic, so it bounds both sides).
    """
    rng = np.random.default_rng(seed)
    vox = np.zeros((1, width, length), dtype=np.uint8)
    x0, y0 = (length - w) // 2, (width - h) // 2
    block = np.ones((h, w), dtype=bool)  # True = solid
    yy, xx = np.mgrid[0:h, 0:w]
    r2 = (diameter / 2.0) ** 2
    n = h * w
    while 1.0 - block.sum() / n < phi - tol:
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        # pixel centres at (i + 1/2, j + 1/2)
        block[(yy + 0.5 - cy) ** 2 + (xx + 0.5 - cx) ** 2 <= r2] = False
    vox[0, y0:y0 + h, x0:x0 + w][block] = CATALYTIC
    vox[0, 0, :] = INERT
    return vox


def crop(vox, nx, ny, nz, outlet_planes=4):
    """Crop voxels [0:nz, 0:ny, 0:nx] and force the last outlet planes to gas."""
    c = np.ascontiguousarray(vox[:nz, :ny, :nx]).copy()
    if outlet_planes:
        c[:, :, nx - outlet_planes:] = FLUID
    return c


def channel(n_fluid, nx=1, nz=1):
    """Plane channel: gas rows y = 0..n-1, one inert wall row at y = n.

    With y periodic the single wall row bounds both sides, so the walls sit
    halfway at y = -1/2 and y = n - 1/2.
    """
    vox = np.zeros((nz, n_fluid + 1, nx), dtype=np.uint8)
    vox[:, n_fluid, :] = INERT
    return vox


def reactive_slab(n_fluid, ny=1, nz=1):
    """1-D reactive slab: gas x = 0..n-1 and a catalytic plane at x = n."""
    vox = np.zeros((nz, ny, n_fluid + 1), dtype=np.uint8)
    vox[:, :, n_fluid] = CATALYTIC
    return vox


def porosity(vox):
    return float(np.count_nonzero(vox == FLUID)) / vox.size


def sha256(vox):
    return hashlib.sha256(np.ascontiguousarray(vox).tobytes()).hexdigest()


def body_force(ell, tau_gas):
    """Body-force density on the gas along x for a GRF sample.

    Chosen so the mean pore velocity is of order 1e-2 (Mach about 0.02) at
    porosity 0.65: F_x = 2e-4 * (4 / ell)^2 * (nu / 0.1), nu = (tau - 1/2) / 3
    (permeability grows as ell^2, the velocity as F / nu).
    """
    nu = (tau_gas - 0.5) / 3.0
    return (2e-4 * (4.0 / ell) ** 2 * (nu / 0.1), 0.0, 0.0)


@dataclasses.dataclass
class Workload:
    """One synthetic workload: geometry recipe plus physical parameters."""

    name: str
    nx: int
    ny: int
    nz: int
    phi: float
    ell: float
    seed: int
    tau: tuple
    da: float
    steps: int
    x_lo: int = 4
    x_hi: int | None = None
    c_inlet: float = 1.0
    p_stick: float = 0.95

    def voxels(self):
        return porous_slab(self.nx, self.ny, self.nz, self.phi, self.ell, self.seed,
                           self.x_lo, self.x_hi)

    def force(self):
        return body_force(self.ell, self.tau[0])

    @property
    def pore_size(self):
        return float(self.ell)


# The five workloads: the small plain case, the 256^3 single sample, the 512^3
# precision study, the 64-sample batch and the 1024x512x512 thin membrane.
PLAIN_32 = Workload("porous32_plain", 32, 32, 32, 0.65, 4.0, 1000, (0.8, 0.7), 1.0, 200)
SINGLE_256 = Workload("porous256_single", 256, 256, 256, 0.60, 8.0, 1001, (0.8, 0.7), 1.0, 2000)
PRECISION_512 = Workload("porous512_precision", 512, 512, 512, 0.70, 12.0, 1002, (0.8, 0.7), 1.0, 1000)
MEMBRANE_1024 = Workload("membrane1024x512x512", 1024, 512, 512, 0.65, 10.0, 1004, (0.8, 0.7), 10.0,
                         5000, x_lo=384, x_hi=640)


def batch_samples(n=64, seed=2000):
    """The mixed-size batch: cubes of side U{48..128}, phi U[0.5, 0.75],
    tau U[0.55, 1.2] (equal for both lattices), Da log-uniform in [0.01, 100],
    correlation length 6."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n):
        side = int(rng.integers(48, 129))
        phi = float(rng.uniform(0.5, 0.75))
        tau = float(rng.uniform(0.55, 1.2))
        da = float(10.0 ** rng.uniform(-2.0, 2.0))
        out.append(Workload(f"batch{s}", side, side, side, phi, 6.0, seed + s, (tau, tau), da, 1000))
    return out


def random_density_perturbation(shape, amp, seed):
    """Seeded i.i.d. uniform numbers in [-amp, amp] (for perturbed initial states)."""
    return np.random.default_rng(seed).uniform(-amp, amp, size=shape)

