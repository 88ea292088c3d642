"""Pins for the oracle's BiCGSTAB solve (right preconditioning, affine warm start).

* the solve agrees with a dense LU solve on tiny grids;
* preconditioned, unpreconditioned and warm-started solves reach the same
  solution (the preconditioner changes the iteration, not the solution);
* a warm start at the exact solution needs no iteration;
* a zero base field reproduces the null-initialised solve exactly;
* the adjoint solve agrees with a dense LU solve of A^H.
"""

import numpy as np
import pytest

from oracle import psfd_ref as R
from psfd_synth import base_config, eps_absorber_default, rect_layout, random_field


def _problem(pol=0, n=4, nabs=4, seed=3):
    rng = np.random.default_rng(seed)
    cfg = base_config(n, n, nabs, 7.5, theta_deg=6.0, phi_deg=15.0, pol=pol)
    a = rect_layout(n, n, rng, wmin=1, wmax=2)
    return R.Problem(cfg, R.eps_from_fill(cfg, R.smooth_layout(cfg, a), eps_absorber_default()))


@pytest.fixture(scope="module")
def dense_te():
    P = _problem(0)
    A = R.dense_by_columns(P)
    b = R.rhs(P)
    return P, A, b, np.linalg.solve(A, b.ravel()).reshape(P.g.shape)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("pc", [0, 1])
def test_bicgstab_matches_lu(dense_te, pc):
    P, A, b, E_lu = dense_te
    E, info = R.solve(P, tol=1e-13, precond=pc)
    assert info["status"] == "converged"
    assert _rel(E, E_lu) <= 1e-10


def test_warm_start_reaches_same_solution(dense_te, rng):
    P, A, b, E_lu = dense_te
    x0 = E_lu + 0.05 * np.abs(E_lu).max() * random_field(E_lu.shape, rng)
    E, info = R.solve(P, x0=x0, tol=1e-13, precond=1)
    assert _rel(E, E_lu) <= 1e-10


def test_exact_warm_start_needs_no_iteration(dense_te):
    P, A, b, E_lu = dense_te
    E, info = R.solve(P, x0=E_lu, tol=1e-10, precond=1)
    assert info["iters"] == 0 and info["status"] == "converged"


def test_zero_base_field_equals_null_start(dense_te):
    P, A, b, E_lu = dense_te
    h1, h2 = [], []
    E1, i1 = R.solve(P, tol=1e-8, precond=1, history=h1)
    E2, i2 = R.solve(P, x0=np.zeros_like(E1), tol=1e-8, precond=1, history=h2)
    assert i1["iters"] == i2["iters"] and h1 == h2
    assert np.array_equal(E1, E2)


def test_adjoint_solve_matches_lu(dense_te, rng):
    P, A, b, E_lu = dense_te
    g = random_field(P.g.shape, rng)
    lam, info = R.solve(P, b=g, tol=1e-13, precond=1, adjoint=True)
    ref = np.linalg.solve(A.conj().T, g.ravel()).reshape(P.g.shape)
    assert _rel(lam, ref) <= 1e-10


def test_tm_solve_matches_lu():
    P = _problem(1, seed=5)
    A = R.dense_by_columns(P)
    b = R.rhs(P)
    E_lu = np.linalg.solve(A, b.ravel()).reshape(P.g.shape)
    E, info = R.solve(P, tol=1e-13, precond=1)
    assert _rel(E, E_lu) <= 1e-10


def test_preconditioner_reduces_iterations():
    """Qualitative claim of the paper (Fig. 5 discussion): spectral damping
    cuts the iteration count several-fold against the null preconditioner."""
    rng = np.random.default_rng(3)
    cfg = base_config(16, 16, 8, 15.0, theta_deg=6.0)
    a = rect_layout(16, 16, rng, wmin=2, wmax=6)
    P = R.Problem(cfg, R.eps_from_fill(cfg, R.smooth_layout(cfg, a), eps_absorber_default()))
    _, i0 = R.solve(P, tol=1e-4, precond=0)
    _, i1 = R.solve(P, tol=1e-4, precond=1)
    assert i0["status"] == i1["status"] == "converged"
    assert i1["iters"] * 3 < i0["iters"]
