"""Fluid side of the coupling in the drag-dominated limit of model A (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy/scipy, written
from section 2.2 of arXiv:2211.06142: eq 6 is the locally averaged momentum and
continuity balance of the fluid, whose particle-fluid force is the negative of
the cell drag source of eq 7.  In a packed bed the unsteady, advective and
viscous terms of eq 6 are small against the pressure gradient and the drag, so
the momentum balance reduces to  n grad(p) = -beta (u - v_s)  with beta the
cell's drag coefficient (cell drag force per volume and per unit slip); with the
bed at rest relative to the fluid (v_s = 0), continuity div(n u) = 0 becomes the
pressure equation  div(K grad p) = 0,  K = n^2 / beta, for the dynamic pressure.

Discretisation: cell-centred finite volumes on the coupling grid; the flux
through the face between cells a and b is T (p_a - p_b) with
T = (face area / centre distance) * 2 K_a K_b / (K_a + K_b) (harmonic mean; 0
next to a solid cell or the grid's outer boundary).  Cell kinds: 0 unknown
pressure, 1 fixed pressure, 2 solid (no flow).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

KIND_OPEN, KIND_PRESSURE, KIND_SOLID = 0, 1, 2


def cell_coefficient(n, fdrag_cell, u_interstitial, mu_f, h):
    """K = n^2 / (beta + beta_open) per cell.  beta = |eq 7 drag source| /
    |interstitial velocity| (the drag law linearised at the current slip);
    beta_open = 12 mu_f / h_min^2, the resistance of viscous flow between
    plates one cell apart, keeps particle-free cells finite."""
    n = np.asarray(n, float)
    fm = np.linalg.norm(np.asarray(fdrag_cell, float).reshape(-1, 3), axis=1)
    um = np.linalg.norm(np.asarray(u_interstitial, float).reshape(-1, 3), axis=1)
    beta = np.where(um > 0.0, fm / np.where(um > 0.0, um, 1.0), 0.0)
    beta_open = 12.0 * mu_f / min(h) ** 2
    return n * n / (beta + beta_open)


def assemble(grid, K, kind, p_fixed):
    """the linear system A p = b over the open cells; returns (A, b, open index)"""
    lo, hi, nn = grid
    nx, ny, nz = (int(q) for q in nn)
    h = [(hi[c] - lo[c]) / nn[c] for c in range(3)]
    geo = [h[1] * h[2] / h[0], h[0] * h[2] / h[1], h[0] * h[1] / h[2]]
    ncell = nx * ny * nz
    kind = np.asarray(kind)
    open_idx = np.flatnonzero(kind == KIND_OPEN)
    pos = -np.ones(ncell, int)
    pos[open_idx] = np.arange(open_idx.size)
    rows, cols, vals = [], [], []
    b = np.zeros(open_idx.size)
    diag = np.zeros(open_idx.size)
    for q, c in enumerate(open_idx):
        ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
        for axis, (dx, dy, dz) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            for sgn in (-1, 1):
                jx, jy, jz = ix + sgn * dx, iy + sgn * dy, iz + sgn * dz
                if not (0 <= jx < nx and 0 <= jy < ny and 0 <= jz < nz):
                    continue
                j = (jz * ny + jy) * nx + jx
                if kind[j] == KIND_SOLID:
                    continue
                T = geo[axis] * 2.0 * K[c] * K[j] / (K[c] + K[j])
                diag[q] += T
                if kind[j] == KIND_PRESSURE:
                    b[q] += T * p_fixed[j]
                else:
                    rows.append(q)
                    cols.append(pos[j])
                    vals.append(-T)
    A = sp.csr_matrix((np.concatenate([diag, vals]),
                       (np.concatenate([np.arange(open_idx.size), rows]),
                        np.concatenate([np.arange(open_idx.size), cols]))), shape=(open_idx.size,) * 2)
    return A, b, open_idx


def solve(grid, K, kind, p_fixed):
    """pressure of every cell (fixed cells keep theirs, solid cells 0)"""
    A, b, open_idx = assemble(grid, K, kind, p_fixed)
    p = np.where(np.asarray(kind) == KIND_PRESSURE, p_fixed, 0.0).astype(float)
    if open_idx.size:
        p[open_idx] = spla.spsolve(A.tocsc(), b)
    return p


def face_flux(grid, K, kind, p):
    """superficial flux (m/s) through every face between two non-solid cells,
    as a dict (cell a, cell b) -> flux from a to b"""
    lo, hi, nn = grid
    nx, ny, nz = (int(q) for q in nn)
    h = [(hi[c] - lo[c]) / nn[c] for c in range(3)]
    out = {}
    for c in range(nx * ny * nz):
        if kind[c] == KIND_SOLID:
            continue
        ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
        for axis, (dx, dy, dz) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            jx, jy, jz = ix + dx, iy + dy, iz + dz
            if not (jx < nx and jy < ny and jz < nz):
                continue
            j = (jz * ny + jy) * nx + jx
            if kind[j] == KIND_SOLID:
                continue
            Kf = 2.0 * K[c] * K[j] / (K[c] + K[j])
            out[(c, j)] = -Kf * (p[j] - p[c]) / h[axis]
    return out


def cell_fields(grid, K, kind, p):
    """cell-centred superficial velocity (mean of the two face fluxes of each
    axis; a missing face counts as no flow) and pressure gradient (mean of the
    available one-sided differences); zero in solid cells"""
    lo, hi, nn = grid
    nx, ny, nz = (int(q) for q in nn)
    h = [(hi[c] - lo[c]) / nn[c] for c in range(3)]
    ncell = nx * ny * nz
    U = np.zeros((ncell, 3))
    G = np.zeros((ncell, 3))
    for c in range(ncell):
        if kind[c] == KIND_SOLID:
            continue
        ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
        for axis, (dx, dy, dz) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            flux, grads = [], []
            for sgn in (-1, 1):
                jx, jy, jz = ix + sgn * dx, iy + sgn * dy, iz + sgn * dz
                if not (0 <= jx < nx and 0 <= jy < ny and 0 <= jz < nz):
                    flux.append(0.0)
                    continue
                j = (jz * ny + jy) * nx + jx
                if kind[j] == KIND_SOLID:
                    flux.append(0.0)
                    continue
                g = sgn * (p[j] - p[c]) / h[axis]
                Kf = 2.0 * K[c] * K[j] / (K[c] + K[j])
                flux.append(-Kf * g)
                grads.append(g)
            U[c, axis] = 0.5 * (flux[0] + flux[1])
            G[c, axis] = sum(grads) / len(grads) if grads else 0.0
    return U, G
