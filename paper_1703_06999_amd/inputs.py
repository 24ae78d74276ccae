"""Seeded synthetic inputs: grids and cells, densities with analytic gradients, and kernel tables.

This module is shared by the CPU oracle and the GPU path.  It holds none of the method's
arithmetic: it only draws random numbers, places density blobs on a periodic grid and tabulates
a kernel on a k-grid.  Everything here is plain numpy / torch in float64.

Units are Hartree atomic units (bohr, electrons/bohr^3).  Cells are given as a 3x3 matrix whose
rows are the lattice vectors a1, a2, a3; arrays are row-major [N1][N2][N3] with the third axis
contiguous, the layout of the paper's Sec. 3 (the data is distributed over the first, least
contiguous axis).

Workloads (shapes and density models follow the paper's benchmark systems, which are not
available: a molecular pair in a small box, Slater-type blob "molecules" in vacuum, and a
metal-core/ligand-shell nanoparticle in a large cell, Sec. 4-5):

* ``two_gaussians_32``  - 32^3 grid, 8 Angstrom cube, two Gaussians + 1e-6 floor.
* ``slater_128``        - 128^3 grid, 20 Angstrom cube, 200 Slater blobs in the central 60%.
* ``slater_192``        - 192^3 grid, 28 Angstrom cube, 600 Slater blobs.
* ``serving``           - grid N in {48, 64, 96, 128, 160}, cell N*0.15625 Angstrom, 50-400 blobs.
* ``nanoparticle_512``  - 512^3 grid, 48 Angstrom cube, 576 core + 9120 shell blobs.
* ``nanoparticle_slab`` - any grid at the nanoparticle's spacing, its blob model scaled to the cell.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BOHR_IN_ANGSTROM = 0.529177210903  # CODATA 2018
ANGSTROM = 1.0 / BOHR_IN_ANGSTROM  # bohr per Angstrom

# Relative cut-off of a Slater blob exp(-2 zeta d): beyond exp(-2 zeta d) < 1e-20 it contributes
# exactly zero, so far-vacuum points carry n = 0.
SLATER_CUTOFF_EXPONENT = 20.0 * math.log(10.0)

SEED_BASE = 17030699


def cubic_cell(length_bohr: float) -> np.ndarray:
    return np.eye(3) * float(length_bohr)


# ----------------------------------------------------------------------------------------------
# kernel table (q-mesh + phi_ab(k) on a uniform k-grid)
# ----------------------------------------------------------------------------------------------

@dataclass
class KernelTable:
    """Radial kernels phi_ab(k) tabulated at k_j = j*kmax/(nk-1), j = 0..nk-1, on a q-mesh.

    ``table`` has shape [nk][M][M] (float64, symmetric in the last two axes); ``qmesh`` has M
    increasing values ending at the saturation value q_cut (5 bohr^-1 in the paper's appendix).
    """

    qmesh: np.ndarray
    kmax: float
    table: np.ndarray
    name: str = "synthetic-gaussian"

    @property
    def nq(self) -> int:
        return int(self.qmesh.shape[0])

    @property
    def nk(self) -> int:
        return int(self.table.shape[0])

    def save(self, path: str) -> None:
        """Binary file read by the C library: magic 'VDWK', u32 version=1, u32 M, u32 nk,
        f64 kmax, f64 qmesh[M], f64 table[nk][M][M] (little endian)."""
        with open(path, "wb") as f:
            f.write(b"VDWK")
            np.array([1, self.nq, self.nk], dtype="<u4").tofile(f)
            np.array([self.kmax], dtype="<f8").tofile(f)
            np.ascontiguousarray(self.qmesh, dtype="<f8").tofile(f)
            np.ascontiguousarray(self.table, dtype="<f8").tofile(f)

    @staticmethod
    def load(path: str) -> "KernelTable":
        with open(path, "rb") as f:
            if f.read(4) != b"VDWK":
                raise ValueError("not a kernel table file")
            version, m, nk = np.fromfile(f, dtype="<u4", count=3)
            if version != 1:
                raise ValueError(f"unsupported kernel table version {version}")
            kmax = float(np.fromfile(f, dtype="<f8", count=1)[0])
            q = np.fromfile(f, dtype="<f8", count=int(m))
            t = np.fromfile(f, dtype="<f8", count=int(nk) * int(m) * int(m)).reshape(nk, m, m)
        return KernelTable(q, kmax, t, name="file")


def log_qmesh(m: int = 20, qmin: float = 1e-5, qcut: float = 5.0, lam: float = 1.2) -> np.ndarray:
    """M mesh points from qmin to qcut with geometrically growing spacing (ratio ``lam``).

    The paper uses Quantum ESPRESSO's 20 points ending at 5 a.u. (Sec. 2 and the appendix); their
    values are not printed, so this log-like mesh stands in for them.
    """
    a = np.arange(m, dtype=np.float64)
    return qmin + (qcut - qmin) * (lam ** a - 1.0) / (lam ** (m - 1) - 1.0)


def synthetic_kernel_table(qmesh: np.ndarray | None = None, nk: int = 1024, kmax: float = 40.0,
                           amplitude: float = 0.05, kappa0: float = 0.5) -> KernelTable:
    """A smooth symmetric stand-in for the vdW-DF radial kernels phi_ab(k).

    phi_ab(k) = -A (pi/kappa_ab^2)^{3/2} exp(-k^2 / (4 kappa_ab^2)),
    kappa_ab^2 = (q_a^2 + q_b^2)/2 + kappa0^2,
    i.e. the Fourier transform of an attractive Gaussian -A exp(-kappa^2 r^2) whose range shrinks
    as the two mesh values q_a, q_b grow.  It is an input of the method (the paper takes its table
    from Quantum ESPRESSO), not part of it: every parity statement holds for any symmetric table.
    """
    q = log_qmesh() if qmesh is None else np.asarray(qmesh, dtype=np.float64)
    k = np.arange(nk, dtype=np.float64) * (kmax / (nk - 1))
    kap2 = 0.5 * (q[:, None] ** 2 + q[None, :] ** 2) + kappa0 ** 2
    pref = -amplitude * (math.pi / kap2) ** 1.5
    tab = pref[None, :, :] * np.exp(-(k[:, None, None] ** 2) / (4.0 * kap2[None, :, :]))
    tab = 0.5 * (tab + np.transpose(tab, (0, 2, 1)))
    return KernelTable(q, float(kmax), np.ascontiguousarray(tab))


# ----------------------------------------------------------------------------------------------
# densities
# ----------------------------------------------------------------------------------------------

def _torch():
    import torch  # imported lazily: the oracle-only tests need numpy alone
    return torch


def gaussian_pair_density(grid, length_bohr: float, centres_bohr, width_bohr: float,
                          peak: float, floor: float):
    """n = floor + sum_i peak * exp(-|r - R_i|^2 / (2 s^2)), summed over the 27 nearest images;
    returns (n, grad) as float64 numpy arrays, grad of shape [3][N1][N2][N3]."""
    n1, n2, n3 = grid
    h = np.array([length_bohr / n1, length_bohr / n2, length_bohr / n3])
    xs = [np.arange(g) * hh for g, hh in zip(grid, h)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    n = np.full(grid, float(floor))
    grad = np.zeros((3,) + tuple(grid))
    for c in centres_bohr:
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                for sz in (-1, 0, 1):
                    dx = X - (c[0] + sx * length_bohr)
                    dy = Y - (c[1] + sy * length_bohr)
                    dz = Z - (c[2] + sz * length_bohr)
                    g = peak * np.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * width_bohr ** 2))
                    n += g
                    grad[0] -= g * dx / width_bohr ** 2
                    grad[1] -= g * dy / width_bohr ** 2
                    grad[2] -= g * dz / width_bohr ** 2
    return n, grad


def _axis_lengths(length_bohr):
    """(L1, L2, L3) of a rectangular cell from one length (cube) or three."""
    if np.ndim(length_bohr) == 0:
        return (float(length_bohr),) * 3
    return tuple(float(x) for x in length_bohr)


def slater_blob_density(grid, length_bohr, centres_bohr: np.ndarray, zetas: np.ndarray,
                        device: str = "cpu", progress=None):
    """n = sum_i (zeta_i^3/pi) exp(-2 zeta_i d_i) on a periodic rectangular cell (``length_bohr``:
    one edge length for a cube, or three), d_i the minimum-image distance; each blob is cut off
    where exp(-2 zeta d) < 1e-20.  Returns torch float64 tensors (n [N1,N2,N3], grad [3,N1,N2,N3])
    on ``device``.  Each blob is added on its own sub-box of the grid, in blob order, so the bytes
    are reproducible for a given device.  ``progress``, if given, is called as
    progress(done, total) after every 1000 blobs."""
    torch = _torch()
    n1, n2, n3 = (int(g) for g in grid)
    dims = (n1, n2, n3)
    Ls = _axis_lengths(length_bohr)
    h = [Lx / g for Lx, g in zip(Ls, dims)]
    dev = torch.device(device)
    n = torch.zeros(dims, dtype=torch.float64, device=dev)
    grad = torch.zeros((3,) + dims, dtype=torch.float64, device=dev)
    total = len(zetas)
    for done, (c, z) in enumerate(zip(np.asarray(centres_bohr, dtype=np.float64), np.asarray(zetas, dtype=np.float64))):
        if progress is not None and done and done % 1000 == 0:
            progress(done, total)
        dcut = SLATER_CUTOFF_EXPONENT / (2.0 * z)
        idx, dist = [], []
        for ax in range(3):
            g, L = dims[ax], Ls[ax]
            lo = math.floor((c[ax] - dcut) / h[ax])
            hi = math.ceil((c[ax] + dcut) / h[ax])
            if hi - lo + 1 >= g:
                # the whole axis: every grid point once, distance to the nearest image
                j = torch.arange(g, dtype=torch.float64, device=dev)
                d = j * h[ax] - c[ax]
                d = d - L * torch.round(d / L)
                ii = torch.arange(g, device=dev)
            else:
                j = torch.arange(lo, hi + 1, dtype=torch.float64, device=dev)
                d = j * h[ax] - c[ax]
                ii = torch.remainder(torch.arange(lo, hi + 1, device=dev), g)
            idx.append(ii)
            dist.append(d)
        dx = dist[0][:, None, None]
        dy = dist[1][None, :, None]
        dz = dist[2][None, None, :]
        r = torch.sqrt(dx * dx + dy * dy + dz * dz)
        val = (z ** 3 / math.pi) * torch.exp(-2.0 * z * r)
        val = torch.where(2.0 * z * r > SLATER_CUTOFF_EXPONENT, torch.zeros_like(val), val)
        # gradient of exp(-2 z r): -2 z val (r_vec / r), zero at r = 0
        safe_r = torch.where(r > 0, r, torch.ones_like(r))
        coef = torch.where(r > 0, -2.0 * z * val / safe_r, torch.zeros_like(val))
        ix = idx[0][:, None, None]
        iy = idx[1][None, :, None]
        iz = idx[2][None, None, :]
        n[ix, iy, iz] += val
        grad[0][ix, iy, iz] += coef * dx
        grad[1][ix, iy, iz] += coef * dy
        grad[2][ix, iy, iz] += coef * dz
    return n, grad


def slater_blob_density_dense(grid, length_bohr: float, centres_bohr: np.ndarray, zetas: np.ndarray,
                              device: str = "cpu", chunk: int = 8):
    """The same density model as `slater_blob_density` (minimum image, cut at
    exp(-2 zeta d) < 1e-20), evaluated on the whole grid for `chunk` blobs at a time: faster for
    small cells where each blob's cut-off sphere covers most of the cell.  The summation order
    differs, so its bytes differ from the sub-box version at the rounding level."""
    torch = _torch()
    dims = tuple(int(g) for g in grid)
    L = float(length_bohr)
    dev = torch.device(device)
    ax = [torch.arange(g, dtype=torch.float64, device=dev) * (L / g) for g in dims]
    c = torch.as_tensor(np.asarray(centres_bohr, dtype=np.float64), device=dev)
    z = torch.as_tensor(np.asarray(zetas, dtype=np.float64), device=dev)
    n = torch.zeros(dims, dtype=torch.float64, device=dev)
    grad = torch.zeros((3,) + dims, dtype=torch.float64, device=dev)
    for s0 in range(0, c.shape[0], chunk):
        cc, zz = c[s0:s0 + chunk], z[s0:s0 + chunk]
        d = []
        for i in range(3):
            di = ax[i][None, :] - cc[:, i:i + 1]
            d.append(di - L * torch.round(di / L))
        dx = d[0][:, :, None, None]
        dy = d[1][:, None, :, None]
        dz = d[2][:, None, None, :]
        r = torch.sqrt(dx * dx + dy * dy + dz * dz)
        zb = zz[:, None, None, None]
        val = (zb ** 3 / math.pi) * torch.exp(-2.0 * zb * r)
        val = torch.where(2.0 * zb * r > SLATER_CUTOFF_EXPONENT, torch.zeros_like(val), val)
        safe_r = torch.where(r > 0, r, torch.ones_like(r))
        coef = torch.where(r > 0, -2.0 * zb * val / safe_r, torch.zeros_like(val))
        n += val.sum(0)
        grad[0] += (coef * dx).sum(0)
        grad[1] += (coef * dy).sum(0)
        grad[2] += (coef * dz).sum(0)
    return n, grad


def _blobs_uniform_cube(rng, count, lo, hi, zmin, zmax):
    centres = rng.uniform(lo, hi, size=(count, 3))
    zetas = rng.uniform(zmin, zmax, size=count)
    return centres, zetas


def _blobs_nanoparticle(rng, length_bohr):
    """576 'metal' blobs uniform in a ball of radius 8 Angstrom (zeta in [1.9, 2.1]) and 9120
    'ligand' blobs uniform in volume over the shell 8-20 Angstrom (zeta in [0.9, 1.1]), centred in
    the cell: four replicas of a 2424-atom ligand-protected nanoparticle (Sec. 5)."""
    def ball(count, r0, r1):
        v = rng.normal(size=(count, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        u = rng.uniform(size=count)
        r = (r0 ** 3 + u * (r1 ** 3 - r0 ** 3)) ** (1.0 / 3.0)
        return v * r[:, None]
    core = ball(576, 0.0, 8.0 * ANGSTROM)
    shell = ball(9120, 8.0 * ANGSTROM, 20.0 * ANGSTROM)
    centres = np.concatenate([core, shell]) + 0.5 * length_bohr
    zetas = np.concatenate([rng.uniform(1.9, 2.1, 576), rng.uniform(0.9, 1.1, 9120)])
    return centres, zetas


# grid spacing of the nanoparticle workload: 48 Angstrom over 512 points
NANO_SPACING = 48.0 * ANGSTROM / 512


def _blobs_nanoparticle_scaled(rng, lengths_bohr):
    """The nanoparticle's core + shell blob model squeezed into a rectangular cell: positions drawn
    as in `_blobs_nanoparticle` (ball of 8 Angstrom, shell 8-20 Angstrom), each axis scaled by
    L_axis / 48 Angstrom about the cell centre, and the blob counts scaled by the cell's volume
    relative to the 48 Angstrom cube (at least one of each kind)."""
    L0 = 48.0 * ANGSTROM
    s = np.asarray(lengths_bohr, dtype=np.float64) / L0
    frac = float(np.prod(s))
    ncore, nshell = max(1, round(576 * frac)), max(1, round(9120 * frac))

    def ball(count, r0, r1):
        v = rng.normal(size=(count, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        u = rng.uniform(size=count)
        r = (r0 ** 3 + u * (r1 ** 3 - r0 ** 3)) ** (1.0 / 3.0)
        return v * r[:, None]
    core = ball(ncore, 0.0, 8.0 * ANGSTROM)
    shell = ball(nshell, 8.0 * ANGSTROM, 20.0 * ANGSTROM)
    centres = np.concatenate([core, shell]) * s[None, :] + 0.5 * np.asarray(lengths_bohr)[None, :]
    zetas = np.concatenate([rng.uniform(1.9, 2.1, ncore), rng.uniform(0.9, 1.1, nshell)])
    return centres, zetas


@dataclass
class Workload:
    name: str
    grid: tuple
    cell: np.ndarray
    centres: np.ndarray | None = None
    zetas: np.ndarray | None = None

    @property
    def npoints(self) -> int:
        return int(np.prod(self.grid))

    def density(self, device: str = "cpu", progress=None):
        """(n, grad) as torch float64 tensors on ``device`` (``progress``: see slater_blob_density)."""
        torch = _torch()
        L = float(self.cell[0, 0])
        if self.name.startswith("nanoparticle_slab"):
            return slater_blob_density(self.grid, np.diag(self.cell), self.centres, self.zetas, device=device,
                                       progress=progress)
        if self.name.startswith("serving_"):
            return slater_blob_density_dense(self.grid, L, self.centres, self.zetas, device=device)
        if self.name == "two_gaussians_32":
            cA = np.array([4.0 - 1.75, 4.0, 4.0]) * ANGSTROM
            cB = np.array([4.0 + 1.75, 4.0, 4.0]) * ANGSTROM
            n, g = gaussian_pair_density(self.grid, L, [cA, cB], 0.8 * ANGSTROM, 0.3, 1e-6)
            return (torch.from_numpy(n).to(device), torch.from_numpy(g).to(device))
        return slater_blob_density(self.grid, L, self.centres, self.zetas, device=device, progress=progress)


def workload(name: str, grid_n: int | None = None, seed_offset: int = 0, grid=None) -> Workload:
    """The named synthetic workloads; RNG numpy.random.default_rng(17030699 + index).

    ``nanoparticle_slab`` takes ``grid`` (N1, N2, N3): a rectangular cell at the nanoparticle's
    grid spacing (48 Angstrom / 512), N_i points along axis i, holding the nanoparticle's
    core + shell blob model scaled to the cell (`_blobs_nanoparticle_scaled`).  (64, 512, 512) is
    one GPU's x-slab of the 512^3 grid split eight ways, (512, 64, 64) a pencil along x: between
    them they exercise every 512-point axis of the full-size workload at sizes the oracle finishes."""
    if name == "two_gaussians_32":
        return Workload(name, (32, 32, 32), cubic_cell(8.0 * ANGSTROM))
    if name == "slater_128":
        L = 20.0 * ANGSTROM
        rng = np.random.default_rng(SEED_BASE + 1 + seed_offset)
        c, z = _blobs_uniform_cube(rng, 200, 0.2 * L, 0.8 * L, 0.8, 2.0)
        return Workload(name, (128, 128, 128), cubic_cell(L), c, z)
    if name == "slater_192":
        L = 28.0 * ANGSTROM
        rng = np.random.default_rng(SEED_BASE + 2 + seed_offset)
        c, z = _blobs_uniform_cube(rng, 600, 0.2 * L, 0.8 * L, 0.8, 2.0)
        return Workload(name, (192, 192, 192), cubic_cell(L), c, z)
    if name == "serving":
        rng = np.random.default_rng(SEED_BASE + 3 + seed_offset)
        g = int(grid_n) if grid_n is not None else int(rng.choice([48, 64, 96, 128, 160]))
        L = g * 0.15625 * ANGSTROM
        count = int(rng.integers(50, 401))
        c, z = _blobs_uniform_cube(rng, count, 0.2 * L, 0.8 * L, 0.8, 2.0)
        return Workload(f"serving_{g}", (g, g, g), cubic_cell(L), c, z)
    if name == "nanoparticle_512":
        L = 48.0 * ANGSTROM
        rng = np.random.default_rng(SEED_BASE + 4 + seed_offset)
        c, z = _blobs_nanoparticle(rng, L)
        return Workload(name, (512, 512, 512), cubic_cell(L), c, z)
    if name == "nanoparticle_slab":
        dims = tuple(int(g) for g in grid)
        lengths = [NANO_SPACING * g for g in dims]
        rng = np.random.default_rng(SEED_BASE + 5 + seed_offset)
        c, z = _blobs_nanoparticle_scaled(rng, lengths)
        return Workload(f"nanoparticle_slab_{dims[0]}x{dims[1]}x{dims[2]}", dims, np.diag(lengths), c, z)
    raise KeyError(name)


def small_slater(grid, length_bohr: float, count: int, seed: int, floor: float = 0.0,
                 device: str = "cpu"):
    """A small random Slater-blob density on any (possibly ragged) grid in a cubic cell, for
    parity tests: returns torch float64 (n, grad)."""
    torch = _torch()
    rng = np.random.default_rng(SEED_BASE + 100 + seed)
    c, z = _blobs_uniform_cube(rng, count, 0.2 * length_bohr, 0.8 * length_bohr, 0.8, 2.0)
    n, g = slater_blob_density(grid, length_bohr, c, z, device=device)
    if floor:
        n = n + floor
    return n, g


def random_positive_field(grid, seed: int, lo: float = 0.05, hi: float = 1.0):
    """A rough random positive density (float64 numpy) for tiny-grid checks."""
    rng = np.random.default_rng(SEED_BASE + 200 + seed)
    return rng.uniform(lo, hi, size=tuple(grid))


def hello_world_inputs():
    """The paper's minimal example (Sec. 6): a 1x2x2 grid in a diag(1,2,2) bohr cell with
    rho = 1,2,3,4 and sigma = 0.5,1.5,2.5,3.5, vdW-DF1."""
    n = np.array([1.0, 2.0, 3.0, 4.0]).reshape(1, 2, 2)
    sigma = np.array([0.5, 1.5, 2.5, 3.5]).reshape(1, 2, 2)
    cell = np.diag([1.0, 2.0, 2.0])
    return (1, 2, 2), cell, n, sigma
