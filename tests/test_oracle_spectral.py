"""Pins of oracle/spectral.py: projector against the dense real-space
projector (brute force, no FFT), symbol identities, stencils."""
import numpy as np
import pytest

from oracle import dense, spectral

GRIDS = [((4, 4, 4), (0.25, 0.25, 0.25)), ((4, 6, 8), (0.3, 0.2, 0.1)), ((6, 4, 4), (1.0, 1.0, 0.5))]


@pytest.mark.parametrize("shape,spacing", GRIDS)
def test_projector_equals_dense_real_space_projector(shape, spacing):
    """G applied to every unit field equals D (D^T D)^+ D^T (includes the
    null set where two or more q_j = pi)."""
    N = int(np.prod(shape))
    Gd = dense.projector_dense(shape, spacing)
    cols = np.zeros((9 * N, 9 * N))
    for k in range(9 * N):
        e = np.zeros(9 * N)
        e[k] = 1.0
        cols[:, k] = spectral.project(e.reshape((3, 3) + shape), spacing).ravel()
    assert np.max(np.abs(cols - Gd)) <= 1e-13 * max(1.0, np.max(np.abs(Gd)))


@pytest.mark.parametrize("shape,spacing", GRIDS)
def test_projector_idempotent_symmetric(shape, spacing):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((3, 3) + shape)
    B = rng.standard_normal((3, 3) + shape)
    GA = spectral.project(A, spacing)
    assert np.allclose(spectral.project(GA, spacing), GA, atol=1e-13)
    lhs = np.sum(GA * B)
    rhs = np.sum(A * spectral.project(B, spacing))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # zero mean
    assert np.max(np.abs(GA.reshape(9, -1).mean(axis=1))) < 1e-14


@pytest.mark.parametrize("shape,spacing", GRIDS)
def test_projector_keeps_gradients(shape, spacing):
    """G(D u) = D u for random nodal u, and D^T (I - G) xi = 0."""
    rng = np.random.default_rng(2)
    D = dense.corner_gradient_matrix(shape, spacing)
    u = rng.standard_normal(3 * int(np.prod(shape)))
    Du = (D @ u).reshape((3, 3) + shape)
    assert np.allclose(spectral.project(Du, spacing), Du, atol=1e-12 * np.abs(Du).max())
    xi = rng.standard_normal((3, 3) + shape)
    res = D.T @ (xi - spectral.project(xi, spacing)).ravel()
    assert np.max(np.abs(res)) < 1e-11 * np.max(np.abs(D.T @ xi.ravel()))


@pytest.mark.parametrize("shape,spacing", [((4, 6, 4), (0.5, 0.25, 1.0)), ((3, 4, 5), (1.0, 1.0, 1.0))])
def test_projector_range_is_gradient_range(shape, spacing):
    """range(G) = range(D): G is the orthogonal projector onto the corner-
    stencil gradients, G = D (D^T D)^+ D^T.  So every compatible field (each
    CG residual, direction and solution of the mechanics) is D of a
    3-component potential, which is what the GPU CG stores."""
    n9 = 9 * int(np.prod(shape))
    G = np.stack([spectral.project(e.reshape((3, 3) + shape), spacing).ravel() for e in np.eye(n9)], axis=1)
    D = dense.corner_gradient_matrix(shape, spacing)
    PD = D @ np.linalg.pinv(D)
    assert np.max(np.abs(G - PD)) < 1e-10
    assert np.linalg.matrix_rank(D) == round(np.trace(G))


def test_rotated_vector_matches_complex_symbol():
    """k_j = i r_j exp(i sum q / 2) with r real, and k equals the symbol of
    the dense 8-corner stencil applied to plane waves."""
    shape, spacing = (6, 4, 8), (0.5, 0.25, 0.125)
    r = spectral.rotated_vector(shape, spacing)
    k = spectral.rotated_symbol(shape, spacing)
    m = [np.arange(n) for n in shape]
    m[2] = np.arange(shape[2] // 2 + 1)
    q = np.meshgrid(*[2 * np.pi * mm / n for mm, n in zip(m, shape)], indexing="ij")
    phase = np.exp(0.5j * (q[0] + q[1] + q[2]))
    assert np.max(np.abs(k - 1j * r * phase)) < 1e-12 * np.abs(k).max()
    # stencil: gradient of a random u computed densely vs through the symbol
    rng = np.random.default_rng(3)
    u = rng.standard_normal((3,) + shape)
    D = dense.corner_gradient_matrix(shape, spacing)
    Du = (D @ u.ravel()).reshape((3, 3) + shape)
    uh = spectral.rfft3(u)
    via = np.stack([np.stack([spectral.irfft3(k[j] * uh[i], shape) for j in range(3)]) for i in range(3)])
    assert np.max(np.abs(via - Du)) < 1e-12 * np.abs(Du).max()


def test_null_set_exact_zero():
    """r = 0 exactly where two or more q_j = pi; nonzero where exactly one."""
    shape, spacing = (4, 6, 8), (1.0, 1.0, 1.0)
    r = spectral.rotated_vector(shape, spacing)
    assert np.all(r[:, 2, 3, :] == 0.0)
    assert np.all(r[:, 2, :, 4] == 0.0)
    assert np.all(r[:, :, 3, 4] == 0.0)
    assert np.sum(r[:, 2, 1, 1] ** 2) > 0.0
    assert r[0, 0, 0, 0] == 0.0 and r[1, 0, 0, 0] == 0.0 and r[2, 0, 0, 0] == 0.0


def test_laplacian_and_difference_symbols_vs_stencils():
    shape, spacing = (6, 8, 4), (0.5, 0.2, 0.3)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(shape)
    lam = spectral.laplacian_symbol(shape, spacing)
    Lv = spectral.irfft3(lam * spectral.rfft3(v), shape)
    st = np.zeros(shape)
    for ax in range(3):
        st += (2 * v - np.roll(v, 1, ax) - np.roll(v, -1, ax)) / spacing[ax] ** 2
    assert np.max(np.abs(Lv - st)) < 1e-12 * np.abs(st).max()
    xi = spectral.forward_difference_symbol(shape, spacing)
    for ax in range(3):
        fd = (np.roll(v, -1, ax) - v) / spacing[ax]
        via = spectral.irfft3(xi[ax] * spectral.rfft3(v), shape)
        assert np.max(np.abs(via - fd)) < 1e-12 * np.abs(fd).max()
