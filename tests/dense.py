"""Test helpers that build dense matrices by explicit loops over cells.

Written independently of the oracle's stencil helpers so that an indexing
mistake in either shows up as a mismatch."""
import numpy as np

# neighbour offsets (di, dj, dk) in the block-row direction order
# 0 self, -x, +x, -y, +y, -z, +z
OFFSETS = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def dense_from_blocks(J):
    """Dense point-block matrix of J[7, b, b, nz, ny, nx]: unknown (cell, r)
    at row cell*b + r, cell = i + nx*(j + ny*k)."""
    _, b, _, nz, ny, nx = J.shape
    n = nx * ny * nz
    M = np.zeros((n * b, n * b))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                row = i + nx * (j + ny * k)
                for d, (di, dj, dk) in enumerate(OFFSETS):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                        assert np.all(J[d, :, :, k, j, i] == 0.0)
                        continue
                    col = ii + nx * (jj + ny * kk)
                    M[row * b:(row + 1) * b, col * b:(col + 1) * b] = J[d, :, :, k, j, i]
    return M


def dense_from_stencil(A):
    """Dense matrix of a scalar 7-point stencil A[7, nz, ny, nx]."""
    return dense_from_blocks(A[:, None, None])


def to_pointblock(v):
    """(b, nz, ny, nx) -> flat vector ordered cell*b + r."""
    b = v.shape[0]
    return np.moveaxis(v.reshape(b, -1), 0, 1).ravel()


def from_pointblock(f, shape):
    b = shape[0]
    return np.moveaxis(f.reshape(-1, b), 1, 0).reshape(shape)
