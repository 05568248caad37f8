"""Dense real-space operators on tiny grids (brute force, no FFT).

The rotated scheme is read as the 8-corner finite-difference gradient
(Sec. 3.2; the reading of the discretisation taken here): nodal displacements u live at voxel corners, node
(i0, i1, i2) at the lower corner of voxel (i0, i1, i2); the gradient at a
voxel centre along axis a is the mean over the four corner edges parallel
to a of the edge difference divided by h_a.  The compatible fields are the
range of this gradient, and the orthogonal projector onto that range is
    G_dense = D (D^T D)^+ D^T,
which is what the Fourier projector of ``spectral.project`` must equal.
Vector ordering: a tensor field A (3, 3, N0, N1, N2) is A.ravel(); a
displacement field u (3, N0, N1, N2) is u.ravel().
"""
from __future__ import annotations

import itertools

import numpy as np


def corner_gradient_matrix(shape, spacing):
    """D (9N x 3N): u -> voxel-centred gradient F_ij = du_i/dx_j."""
    n0, n1, n2 = shape
    N = n0 * n1 * n2

    def node(i, j, k):
        return ((i % n0) * n1 + (j % n1)) * n2 + (k % n2)

    D = np.zeros((9 * N, 3 * N))
    for i, j, k in itertools.product(range(n0), range(n1), range(n2)):
        v = (i * n1 + j) * n2 + k
        for a in range(3):
            for corner in itertools.product((0, 1), repeat=3):
                off = list(corner)
                sign = 1.0 if off[a] == 1 else -1.0
                nd = node(i + off[0], j + off[1], k + off[2])
                w = sign / (4.0 * spacing[a])
                for comp in range(3):
                    D[(3 * comp + a) * N + v, comp * N + nd] += w
    return D


def projector_dense(shape, spacing, rcond=1e-10):
    D = corner_gradient_matrix(shape, spacing)
    return D @ np.linalg.pinv(D.T @ D, rcond=rcond) @ D.T


def tangent_blockdiag(K):
    """K (9, 9, N0, N1, N2) as a (9N x 9N) matrix acting on A.ravel()."""
    N = int(np.prod(K.shape[2:]))
    Kf = K.reshape(9, 9, N)
    M = np.zeros((9 * N, 9 * N))
    idx = np.arange(N)
    for a in range(9):
        for b in range(9):
            M[a * N + idx, b * N + idx] = Kf[a, b]
    return M
