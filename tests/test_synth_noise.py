"""CPU checks of the seeded noise generator the slab workload uses (and the
oracle side of its parity test recomputes): SplitMix64 bits equal the
oracle's own implementation (itself pinned to known answers), the
Box-Muller output is standard normal, and the keying by (view, row, column)
is the documented pixel counter."""
import numpy as np
from scipy import stats

import oracle
import synth

G = synth.Geom(nx=8, ny=8, nz=8, nu=300, nv=200, sod=100.0, sdd=200.0)


def test_bits_match_oracle_splitmix64():
    c = np.array([0, 1, 2, 3, 2 ** 33 + 5, 2 ** 40 - 1], dtype=np.uint64)
    got = synth._splitmix64(987654321, c)
    assert [int(x) for x in got] == [oracle.splitmix64(987654321, int(x)) for x in c]


def test_box_muller_from_documented_draws():
    # pixel (view 3, row 17, column 41): counter m = (3 Nv + 17) Nu + 41
    m = (3 * G.nv + 17) * G.nu + 41
    x1, x2 = oracle.splitmix64(55, 2 * m), oracle.splitmix64(55, 2 * m + 1)
    u1 = ((x1 >> 11) + 1) * 2.0 ** -53
    u2 = (x2 >> 11) * 2.0 ** -53
    want = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    assert synth.normal_draws(55, G, 3, 17, 41) == want


def test_standard_normal_distribution():
    x = synth.normal_draws(2024, G, np.arange(8)[:, None, None], np.arange(200)[None, :, None],
                           np.arange(300)[None, None, :]).ravel()
    assert x.size == 480000
    # mean and variance within 5 standard errors; KS against the normal CDF
    assert abs(x.mean()) < 5 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # neighbouring pixels are uncorrelated
    assert abs(np.corrcoef(x[:-1], x[1:])[0, 1]) < 5 / np.sqrt(x.size)


def test_keys_select_independent_streams():
    a = synth.normal_draws(7, G, 0, 0, np.arange(1000))
    b = synth.normal_draws(8, G, 0, 0, np.arange(1000))
    c = synth.normal_draws(7, G, 1, 0, np.arange(1000))
    assert not np.allclose(a, b) and not np.allclose(a, c)
    # the same pixel from a broadcast grid and from a scalar key agree
    grid = synth.normal_draws(7, G, np.arange(3)[:, None], 5, np.arange(4)[None, :])
    assert grid[2, 3] == synth.normal_draws(7, G, 2, 5, 3)
