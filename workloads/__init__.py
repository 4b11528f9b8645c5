"""Seeded synthetic inputs for ML(n)BiCGStab solves.

This module builds matrices, right-hand sides and shadow blocks only.  It holds
none of the solver's arithmetic, so both the CPU oracle and the GPU path (and
their tests and benchmarks) may draw inputs from it.

The paper's own test matrices (a Matrix Market plasma matrix, a complex quantum
chemistry matrix and a reservoir model; Section 5) are not available, so the
generators below stand in for them with discretised PDE operators of the same
character: real nonsymmetric (convection-diffusion), complex non-Hermitian
(shifted Helmholtz with convection) and a 3x3-block reservoir-shaped system.

Every draw comes from ``numpy.random.Generator(PCG64(SeedSequence([11063678,
config, stream])))`` so that a (config, stream) pair always yields the same
array on any machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.ndimage
import scipy.sparse as sp

PAPER_SEED = 11063678


def rng(config: int, stream: int) -> np.random.Generator:
    """The generator for one (config, stream) pair."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([PAPER_SEED, int(config), int(stream)])))


# ---------------------------------------------------------------------------
# Convection-diffusion on the unit square / cube
# ---------------------------------------------------------------------------
#
# -nu * Laplace(u) + v . grad(u) on m interior points per dimension,
# h = 1/(m+1), lexicographic order (x fastest), homogeneous Dirichlet
# boundary (neighbours outside the domain are dropped).  The operator is
# multiplied by h^2.  Per dimension d with local velocity v_d the row gets
#   diagonal        += 2 nu + h |v_d|
#   upwind  neighbour (index - sign(v_d)) : -nu - h |v_d|
#   downwind neighbour                   : -nu
# which is a nonsymmetric, weakly row-diagonally-dominant M-matrix.
# Cell Peclet number Pe = |v|_2 h / (2 nu), so |v| = 2 Pe nu / h.


def _stencil_csr(shape, vel, nu=1.0, shift=0.0, dtype=np.float64):
    """Assemble the h^2-scaled upwind convection-diffusion operator.

    ``shape`` is (m,) * d, ``vel`` a list of d arrays (one per dimension, each
    of ``shape``) holding v_d at every grid point.  ``shift`` is added to the
    diagonal (it may be complex).
    """
    d = len(shape)
    m = shape[0]
    h = 1.0 / (m + 1)
    npts = int(np.prod(shape))
    idx = np.arange(npts, dtype=np.int64).reshape(shape[::-1])  # axis 0 = slowest
    diag = np.full(npts, shift, dtype=dtype)
    rows, cols, vals = [], [], []
    for dim in range(d):
        # dimension 0 is x (fastest) -> numpy axis d-1
        axis = d - 1 - dim
        v = np.asarray(vel[dim], dtype=np.float64).reshape(shape[::-1])
        av = np.abs(v)
        diag += (2.0 * nu + h * av).ravel()
        for step in (-1, +1):
            # neighbour at index + step along this axis
            src = [slice(None)] * d
            dst = [slice(None)] * d
            if step < 0:
                src[axis] = slice(1, None)
                dst[axis] = slice(None, -1)
            else:
                src[axis] = slice(None, -1)
                dst[axis] = slice(1, None)
            r = idx[tuple(src)].ravel()
            c = idx[tuple(dst)].ravel()
            vloc = v[tuple(src)].ravel()
            # upwind neighbour is index - sign(v): step == -sign(v)
            upwind = (np.sign(vloc) == -step) & (vloc != 0)
            val = np.where(upwind, -nu - h * np.abs(vloc), -nu)
            rows.append(r)
            cols.append(c)
            vals.append(val.astype(dtype))
    rows.append(np.arange(npts, dtype=np.int64))
    cols.append(np.arange(npts, dtype=np.int64))
    vals.append(diag)
    A = sp.csr_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
        shape=(npts, npts),
        dtype=dtype,
    )
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def convdiff_2d(m: int, pe: float, direction=(1.0, 0.5), nu: float = 1.0):
    """2D upwind convection-diffusion, constant velocity along ``direction``."""
    h = 1.0 / (m + 1)
    dvec = np.asarray(direction, dtype=np.float64)
    dvec = dvec / np.linalg.norm(dvec)
    speed = 2.0 * pe * nu / h
    vel = [np.full((m, m), speed * dvec[0]), np.full((m, m), speed * dvec[1])]
    return _stencil_csr((m, m), vel, nu=nu)


def smooth_direction_field(m: int, gen: np.random.Generator, sigma: float = 8.0, d: int = 3):
    """Unit-length velocity directions: Gaussian-filtered white noise per component."""
    comps = []
    for _ in range(d):
        z = gen.standard_normal((m,) * d)
        comps.append(scipy.ndimage.gaussian_filter(z, sigma=sigma, mode="reflect"))
    norm = np.sqrt(sum(c * c for c in comps))
    norm = np.where(norm == 0, 1.0, norm)
    # numpy axis order is (z, y, x); return per-dimension (x, y, z) components
    return [comps[d - 1 - k] / norm for k in range(d)]


def convdiff_3d(m: int, pe: float, gen: np.random.Generator | None = None, sigma: float = 8.0,
                nu: float = 1.0, direction=None, shift=0.0, dtype=np.float64):
    """3D upwind convection-diffusion with a smooth seeded direction field of uniform speed.

    With ``direction`` given, the velocity is constant along it instead.
    """
    h = 1.0 / (m + 1)
    speed = 2.0 * pe * nu / h
    if direction is not None:
        dvec = np.asarray(direction, dtype=np.float64)
        dvec = dvec / np.linalg.norm(dvec)
        vel = [np.full((m, m, m), speed * dvec[k]) for k in range(3)]
    else:
        dirs = smooth_direction_field(m, gen, sigma=sigma, d=3)
        vel = [speed * c for c in dirs]
    return _stencil_csr((m, m, m), vel, nu=nu, shift=shift, dtype=dtype)


def helmholtz_3d(m: int, pe: float, k: float, gen: np.random.Generator, sigma: float = 8.0,
                 velocity: str = "constant"):
    """Complex shifted Laplacian with upwind convection, h^2-scaled.

    A = L + C - (k h)^2 (1 - 0.5 i) I : complex non-Hermitian.  The convection
    has uniform speed along a seeded direction (velocity="smooth": a smooth
    seeded direction field).
    """
    h = 1.0 / (m + 1)
    shift = -((k * h) ** 2) * (1.0 - 0.5j)
    if velocity == "smooth":
        return convdiff_3d(m, pe, gen=gen, sigma=sigma, shift=shift, dtype=np.complex128)
    return convdiff_3d(m, pe, direction=gen.standard_normal(3), shift=shift, dtype=np.complex128)


# ---------------------------------------------------------------------------
# Reservoir-shaped 3x3 block system (BSR, 7-point block stencil)
# ---------------------------------------------------------------------------


def reservoir_bsr3(nx: int, ny: int, nz: int, gen: np.random.Generator, ln_sigma: float = 2.0,
                   corr: float = 8.0, accum: float = 1e-2):
    """Block-diagonally-dominant nonsymmetric 3x3-block system on an nx*ny*nz grid.

    ln K = ln_sigma * Z with Z white noise Gaussian-filtered (std corr/sqrt(2)
    cells) and normalised to unit variance.  Face transmissibility T_ab is the
    harmonic mean of K.  Off-diagonal block A_ab = -T_ab (C + theta_ab U) with
    C = I + 0.2 E_C, U = 0.5 |E_U| (E seeded 3x3 normals) and theta_ab = 1 if
    b is upwind of a under a smooth seeded potential with a linear x trend.
    Diagonal block A_aa = sum_b T_ab (C + theta_ab U) + D_a with
    D_a = (accum mean_b T_ab + 1e-3) I (an accumulation term).  Cells ordered x fastest.
    """
    shape = (nz, ny, nx)
    z = gen.standard_normal(shape)
    z = scipy.ndimage.gaussian_filter(z, sigma=corr / math.sqrt(2.0), mode="reflect")
    z = (z - z.mean()) / (z.std() if z.std() > 0 else 1.0)
    K = np.exp(ln_sigma * z)
    pot = gen.standard_normal(shape)
    pot = scipy.ndimage.gaussian_filter(pot, sigma=corr, mode="reflect")
    pot = pot / (pot.std() if pot.std() > 0 else 1.0)
    xs = np.arange(nx, dtype=np.float64)[None, None, :]
    pot = pot + 4.0 * xs / max(nx - 1, 1)
    C = np.eye(3) + 0.2 * gen.standard_normal((3, 3))
    U = 0.5 * np.abs(gen.standard_normal((3, 3)))

    ncell = nx * ny * nz
    cid = np.arange(ncell, dtype=np.int64).reshape(shape)
    brow, bcol, bval = [], [], []
    diag = np.zeros((ncell, 3, 3))
    tsum = np.zeros(ncell)
    tcount = np.zeros(ncell)
    for axis in range(3):
        for step in (-1, +1):
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if step < 0:
                src[axis] = slice(1, None)
                dst[axis] = slice(None, -1)
            else:
                src[axis] = slice(None, -1)
                dst[axis] = slice(1, None)
            a = cid[tuple(src)].ravel()
            b = cid[tuple(dst)].ravel()
            Ka = K[tuple(src)].ravel()
            Kb = K[tuple(dst)].ravel()
            T = 2.0 * Ka * Kb / (Ka + Kb)
            theta = (pot[tuple(dst)].ravel() > pot[tuple(src)].ravel()).astype(np.float64)
            blk = T[:, None, None] * (C[None] + theta[:, None, None] * U[None])
            brow.append(a)
            bcol.append(b)
            bval.append(-blk)
            np.add.at(diag, a, blk)
            np.add.at(tsum, a, T)
            np.add.at(tcount, a, 1.0)
    dshift = accum * tsum / np.maximum(tcount, 1.0) + 1e-3
    diag += dshift[:, None, None] * np.eye(3)[None]
    brow.append(np.arange(ncell, dtype=np.int64))
    bcol.append(np.arange(ncell, dtype=np.int64))
    bval.append(diag)
    brow = np.concatenate(brow)
    bcol = np.concatenate(bcol)
    bval = np.concatenate(bval)
    order = np.lexsort((bcol, brow))
    brow, bcol, bval = brow[order], bcol[order], bval[order]
    indptr = np.zeros(ncell + 1, dtype=np.int64)
    np.add.at(indptr, brow + 1, 1)
    indptr = np.cumsum(indptr)
    A = sp.bsr_matrix((np.ascontiguousarray(bval), bcol.astype(np.int32), indptr.astype(np.int32)),
                      shape=(3 * ncell, 3 * ncell), blocksize=(3, 3))
    return A


# ---------------------------------------------------------------------------
# Solve configurations
# ---------------------------------------------------------------------------


@dataclass
class Problem:
    name: str
    A: object            # scipy csr_matrix or bsr_matrix (blocksize 3)
    b: np.ndarray
    Q: np.ndarray        # N x n, column-major (Fortran order)
    x0: np.ndarray
    n: int
    tol: float
    maxit: int
    kappa: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.A.shape[0]


def _gauss(gen, shape, complex_=False):
    if complex_:
        return gen.standard_normal(shape) + 1j * gen.standard_normal(shape)
    return gen.standard_normal(shape)


def _qblock(gen, N, n, complex_=False):
    return np.asfortranarray(_gauss(gen, (N, n), complex_))


def config1(n: int = 4, m: int = 32):
    """2D convection-diffusion 32x32, Pe 5, velocity along (1, 0.5); b = A 1 + N(0, 1e-3)."""
    A = convdiff_2d(m, pe=5.0, direction=(1.0, 0.5))
    N = A.shape[0]
    g = rng(1, 1)
    b = A @ np.ones(N) + 1e-3 * g.standard_normal(N)
    Q = _qblock(rng(1, 2), N, n)
    return Problem(f"convdiff2d_m{m}_pe5_n{n}", A, b, Q, np.zeros(N), n, 1e-10, 2000,
                   meta=dict(dims=2, m=m, pe=5.0))


def config2(n: int = 4, m: int = 128, maxit: int = 20000, velocity: str = "constant"):
    """3D convection-diffusion m^3, Pe 20, uniform speed along a seeded direction; b, Q ~ N(0, 1).

    velocity="smooth" uses a smooth seeded direction field instead (Gaussian-filtered
    noise, sigma 8 cells, normalised): on it the unpreconditioned method stalls with
    residual excursions of ~4.5e3 ||b|| and a true residual near 1e-5 (the oracle
    too), so the default is a constant seeded direction.
    """
    if velocity == "smooth":
        A = convdiff_3d(m, pe=20.0, gen=rng(2, 0))
    else:
        A = convdiff_3d(m, pe=20.0, direction=rng(2, 0).standard_normal(3))
    N = A.shape[0]
    b = rng(2, 1).standard_normal(N)
    Q = _qblock(rng(2, 2), N, n)
    return Problem(f"convdiff3d_m{m}_pe20_n{n}", A, b, Q, np.zeros(N), n, 1e-10, maxit,
                   meta=dict(dims=3, m=m, pe=20.0))


def config3(n: int = 8, grid=(60, 220, 85), maxit: int = 20000, accum: float = 1e-2):
    """Reservoir-shaped 3x3-block system on a nx*ny*nz grid (BSR3)."""
    nx, ny, nz = grid
    A = reservoir_bsr3(nx, ny, nz, rng(3, 0), accum=accum)
    N = A.shape[0]
    b = rng(3, 1).standard_normal(N)
    Q = _qblock(rng(3, 2), N, n)
    return Problem(f"reservoir_bsr3_{nx}x{ny}x{nz}_n{n}", A, b, Q, np.zeros(N), n, 1e-10, maxit,
                   meta=dict(grid=grid))


def config5(n: int = 16, m: int = 96, k: float = 10.0, maxit: int = 20000):
    """Complex shifted 3D Laplacian + convection m^3, shift -(kh)^2 (1 - 0.5i), Pe 10."""
    A = helmholtz_3d(m, pe=10.0, k=k, gen=rng(5, 0))
    N = A.shape[0]
    b = _gauss(rng(5, 1), N, complex_=True)
    Q = _qblock(rng(5, 2), N, n, complex_=True)
    return Problem(f"helmholtz3d_m{m}_k{k:g}_pe10_n{n}", A, b, Q, np.zeros(N, dtype=np.complex128), n,
                   1e-10, maxit, meta=dict(dims=3, m=m, pe=10.0, k=k))


# ---------------------------------------------------------------------------
# Serving trace: Poisson arrivals of uneven solves
# ---------------------------------------------------------------------------


@dataclass
class Request:
    rid: int
    arrival_s: float
    dims: int
    m: int
    pe: float
    n: int
    seed_stream: int

    @property
    def N(self):
        return self.m ** self.dims


def serving_trace(count: int = 2000, rate_per_s: float = 200.0, n_min: float = 1e3, n_max: float = 5e5,
                  pe_range=(0.5, 50.0), n_choices=(2, 4, 8), config: int = 4):
    """Poisson arrivals (exponential gaps of mean 1/rate) of 2D/3D convection-diffusion solves."""
    g = rng(config, 0)
    gaps = g.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(count):
        dims = int(g.integers(2, 4))
        ntarget = math.exp(g.uniform(math.log(n_min), math.log(n_max)))
        m = max(2, int(round(ntarget ** (1.0 / dims))))
        pe = float(g.uniform(*pe_range))
        n = int(g.choice(n_choices))
        reqs.append(Request(i, float(t[i]), dims, m, pe, n, 1000 + i))
    return reqs


def serving_problem(req: Request, config: int = 4, tol: float = 1e-10, maxit: int = 20000):
    """The linear system of one serving request (constant random unit direction)."""
    g = rng(config, req.seed_stream)
    direction = g.standard_normal(req.dims)
    if req.dims == 2:
        A = convdiff_2d(req.m, pe=req.pe, direction=direction)
    else:
        A = convdiff_3d(req.m, pe=req.pe, direction=direction)
    N = A.shape[0]
    b = g.standard_normal(N)
    Q = _qblock(g, N, req.n)
    return Problem(f"serve{req.rid}_d{req.dims}_m{req.m}_n{req.n}", A, b, Q, np.zeros(N), req.n, tol, maxit,
                   meta=dict(dims=req.dims, m=req.m, pe=req.pe, rid=req.rid))
