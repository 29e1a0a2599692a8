"""Pins for the oracle's SIRT: equal to SIRT written with an explicit system
matrix (assembled column by column from the oracle's forward projector),
and on consistent data the weighted residual decreases every iteration and
the iterates approach the true volume."""
import numpy as np

import synth

G = synth.Geom(nx=5, ny=4, nz=3, nu=9, nv=6, sod=30.0, sdd=60.0, du=1.5, dv=1.5)
ANG = synth.angles(7, start=0.3)


def system_matrix(orc):
    n = G.nz * G.ny * G.nx
    cols = []
    for m in range(n):
        x = np.zeros(n)
        x[m] = 1.0
        cols.append(orc.forward_project(G, ANG, x.reshape(G.nz, G.ny, G.nx)).reshape(-1))
    return np.stack(cols, 1)


def test_sirt_equals_matrix_sirt(orc):
    A = system_matrix(orc)
    rs, cs = A.sum(1), A.sum(0)
    R = 1.0 / np.maximum(rs, 1e-3 * rs.max())
    C = 1.0 / np.maximum(cs, 1e-3 * cs.max())
    rng = np.random.default_rng(5)
    p = rng.uniform(0, 3, A.shape[0])
    x = np.zeros(A.shape[1])
    for _ in range(6):
        x = x + 0.8 * C * (A.T @ (R * (p - A @ x)))
    got = orc.sirt(G, ANG, p.reshape(len(ANG), G.nv, G.nu), 6, lam=0.8)
    assert np.abs(got.reshape(-1) - x).max() <= 1e-12 * np.abs(x).max()
    Rw, Cw = orc.sirt_weights(G, ANG)
    assert np.allclose(Rw.reshape(-1), R, rtol=1e-12, atol=0)
    assert np.allclose(Cw.reshape(-1), C, rtol=1e-12, atol=0)


def test_sirt_converges_on_consistent_data(orc):
    A = system_matrix(orc)
    rng = np.random.default_rng(6)
    xt = rng.uniform(0.5, 1.5, A.shape[1])
    p = (A @ xt).reshape(len(ANG), G.nv, G.nu)
    R, _ = orc.sirt_weights(G, ANG)
    prev = np.inf
    x = None
    for k in range(1, 40):
        x = orc.sirt(G, ANG, p, 1, x0=x)
        r = p - orc.forward_project(G, ANG, x)
        wres = float(np.sum(R * r * r))
        assert wres <= prev * (1 + 1e-12)
        prev = wres
    err = np.linalg.norm(x.reshape(-1) - xt) / np.linalg.norm(xt)
    assert err < 0.2, err
    # the weighted residual has dropped by orders of magnitude
    r0 = float(np.sum(R * p * p))
    assert prev < 1e-3 * r0
