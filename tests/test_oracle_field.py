"""Pins of the oracle's field solve (Sec. 3.5: tridiagonal Poisson system of eq.
poisson_normalized, solved by the Thomas algorithm; E = -dPhi/dx on the nodes)."""
import numpy as np
import pytest


def dense_bounded(n, rho, phi_left):
    """The same finite-difference system assembled densely and solved by LAPACK."""
    m = n - 1
    A = np.zeros((m, m))
    for i in range(m):
        A[i, i] = -2.0
        if i > 0:
            A[i, i - 1] = 1.0
        if i < m - 1:
            A[i, i + 1] = 1.0
    b = -np.asarray(rho[1:n], dtype=float).copy()
    b[0] -= phi_left
    phi = np.zeros(n + 1)
    phi[0] = phi_left
    phi[1:n] = np.linalg.solve(A, b)
    return phi


@pytest.mark.parametrize("n", [2, 3, 7, 16, 64])
def test_thomas_equals_dense_solve(oracle_mod, n):
    rng = np.random.default_rng(n)
    rho = rng.normal(size=n + 1) * 10
    vl = float(rng.normal() * 100)
    phi, ef = oracle_mod.solve(False, n, rho, vl)
    ref = dense_bounded(n, rho, vl)
    assert np.allclose(phi, ref, rtol=1e-12, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("n", [8, 128, 4096])
def test_uniform_charge_parabola(oracle_mod, n):
    """rho = rho0 between grounded plates: Phi_j = rho0 j (N - j) / 2 (exact for the
    three-point Laplacian); E_j = rho0 (j - N/2) inside; Gauss's law over the half cells
    at the electrodes with half-cell node charge rho0/2 gives the continuum wall field
    -/+ rho0 N / 2.  Thomas elimination loses accuracy like N^2 eps (the condition number of
    the Laplacian), hence the tolerance."""
    rho0 = 3.25
    rho = np.full(n + 1, rho0)
    rho[0] = rho[-1] = rho0 / 2
    phi, ef = oracle_mod.solve(False, n, rho, 0.0)
    j = np.arange(n + 1)
    exact = rho0 * j * (n - j) / 2.0
    tol = 1e-17 * n * n
    assert np.max(np.abs(phi - exact)) <= tol * exact.max() + 1e-12
    assert np.max(np.abs(ef[1:-1] - rho0 * (j[1:-1] - n / 2.0))) <= tol * rho0 * n + 1e-12
    assert ef[0] == pytest.approx(-rho0 * n / 2, rel=1e-10)
    assert ef[-1] == pytest.approx(rho0 * n / 2, rel=1e-10)


def test_vacuum_gap_linear_potential(oracle_mod):
    """No charge: the potential falls linearly from the driven to the grounded plate."""
    n, v = 100, 37.5
    phi, ef = oracle_mod.solve(False, n, np.zeros(n + 1), v)
    j = np.arange(n + 1)
    assert np.allclose(phi, v * (1 - j / n), rtol=1e-12, atol=1e-12)
    assert np.allclose(ef, v / n, rtol=1e-10)


@pytest.mark.parametrize("n,m", [(16, 1), (128, 3), (512, 40)])
def test_periodic_discrete_eigenmode(oracle_mod, n, m):
    """rho_j = cos(k j), k = 2 pi m / N, is an eigenvector of the periodic three-point
    Laplacian with eigenvalue -4 sin^2(k/2); with Phi_0 pinned to 0 the solution is
    (cos(k j) - 1) / (4 sin^2(k/2)), and E_j = sin(k) sin(k j) / (4 sin^2(k/2))."""
    k = 2 * np.pi * m / n
    j = np.arange(n)
    rho = np.cos(k * j)
    phi, ef = oracle_mod.solve(True, n, rho, 0.0)
    lam = 4 * np.sin(k / 2) ** 2
    assert np.allclose(phi, (np.cos(k * j) - 1) / lam, atol=1e-10 / lam)
    assert np.allclose(ef, np.sin(k) * np.sin(k * j) / lam, atol=1e-10 / lam)


def test_periodic_full_system_and_mean_removal(oracle_mod):
    """The pinned Dirichlet solve of the mean-free charge satisfies the periodic equation at
    every node, node 0 included; a uniform background does not change the field; sum E = 0."""
    n = 96
    rng = np.random.default_rng(3)
    rho = rng.normal(size=n) * 5
    phi, ef = oracle_mod.solve(True, n, rho, 0.0)
    rho_free = rho - rho.mean()
    lap = np.roll(phi, 1) - 2 * phi + np.roll(phi, -1)
    assert np.allclose(lap, -rho_free, atol=1e-9)
    assert abs(ef.sum()) < 1e-9
    phi2, ef2 = oracle_mod.solve(True, n, rho + 17.0, 0.0)
    assert np.allclose(ef2, ef, atol=1e-9)
