"""Pins for the oracle's MLEM (Shepp and Vardi 1982, on the matched
projector pair): equal to MLEM written with an explicit system matrix
(assembled column by column from the oracle's forward projector); the
sensitivity-weighted total of each iterate equals the total of the data
(the expectation step preserves counts); the Poisson log-likelihood rises
every iteration on consistent data and the iterates approach the true
volume."""
import numpy as np

import synth

G = synth.Geom(nx=5, ny=4, nz=3, nu=9, nv=6, sod=30.0, sdd=60.0, du=1.5, dv=1.5)
ANG = synth.angles(7, start=0.3)
FLOOR = 1e-3


def system_matrix(orc):
    n = G.nz * G.ny * G.nx
    cols = []
    for m in range(n):
        x = np.zeros(n)
        x[m] = 1.0
        cols.append(orc.forward_project(G, ANG, x.reshape(G.nz, G.ny, G.nx)).reshape(-1))
    return np.stack(cols, 1)


def matrix_mlem(A, p, x, n_iter):
    s = A.sum(0)
    C = 1.0 / np.maximum(s, FLOOR * s.max())
    for _ in range(n_iter):
        ax = A @ x
        den = np.maximum(ax, FLOOR * ax.max())
        x = x * C * (A.T @ np.where(den > 0, p / np.where(den > 0, den, 1.0), 0.0))
    return x


def test_mlem_equals_matrix_mlem(orc):
    A = system_matrix(orc)
    p = np.random.default_rng(5).uniform(0, 3, A.shape[0])
    x0 = np.random.default_rng(6).uniform(0.5, 1.5, A.shape[1])
    want = matrix_mlem(A, p, x0, 6)
    got = orc.mlem(G, ANG, p.reshape(len(ANG), G.nv, G.nu), 6, x0=x0.reshape(G.nz, G.ny, G.nx))
    assert np.abs(got.reshape(-1) - want).max() <= 1e-12 * np.abs(want).max()
    # default start: ones
    assert np.allclose(orc.mlem(G, ANG, p.reshape(len(ANG), G.nv, G.nu), 2).reshape(-1),
                       matrix_mlem(A, p, np.ones(A.shape[1]), 2), rtol=1e-12, atol=0)


def test_mlem_preserves_counts(orc):
    """sum_j s_j x_j' = sum_i p_i (A x)_i / den_i: with C = 1 / s, the
    update redistributes each ray's data over the voxels it crosses."""
    A = system_matrix(orc)
    s = A.sum(0)
    assert s.min() > FLOOR * s.max()        # the column floor does not bind here
    rng = np.random.default_rng(7)
    p = A @ rng.uniform(0.5, 1.5, A.shape[1])
    x = rng.uniform(0.5, 1.5, A.shape[1])
    for _ in range(5):
        ax = A @ x
        den = np.maximum(ax, FLOOR * ax.max())
        want = float(np.sum(np.where(den > 0, p * ax / np.where(den > 0, den, 1.0), 0.0)))
        x = orc.mlem(G, ANG, p.reshape(len(ANG), G.nv, G.nu), 1,
                     x0=x.reshape(G.nz, G.ny, G.nx)).reshape(-1)
        assert abs(float(s @ x) - want) <= 1e-12 * want


def test_mlem_likelihood_rises_on_consistent_data(orc):
    A = system_matrix(orc)
    rng = np.random.default_rng(8)
    xt = rng.uniform(0.5, 1.5, A.shape[1])
    p = A @ xt
    seen = A.sum(1) > 0
    x = np.ones(A.shape[1])
    prev = -np.inf
    for _ in range(60):
        x = orc.mlem(G, ANG, p.reshape(len(ANG), G.nv, G.nu), 1,
                     x0=x.reshape(G.nz, G.ny, G.nx)).reshape(-1)
        assert x.min() >= 0.0
        ax = A @ x
        ll = float(np.sum(p[seen] * np.log(ax[seen]) - ax[seen]))
        assert ll >= prev - 1e-12 * abs(ll)
        prev = ll
    err = np.linalg.norm(x - xt) / np.linalg.norm(xt)
    assert err < 0.2, err
    assert np.linalg.norm(A @ x - p) < 2e-2 * np.linalg.norm(p)
