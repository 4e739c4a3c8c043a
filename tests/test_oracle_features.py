"""Pins of the oracle's predictor features (oracle/features.py): closed forms
on diagonal matrices, a symmetry that fixes mu_0, brute-force Gershgorin
discs and histogram counts."""
import numpy as np
import scipy.sparse as sp

from oracle import features as of
from oracle.csr import Csr


def diag_csr(d):
    n = d.size
    return Csr(n, np.arange(n + 1), np.arange(n), d.astype(np.float64))


def test_diagonal_matrix_closed_forms():
    rng = np.random.default_rng(0)
    d = rng.uniform(-1.3, 0.4, 37)
    Hp = diag_csr(d)
    f, (lo, hi), (hd, hr) = of.features(Hp, Hp.with_values(None), 4, 0.3, 2.0, 11.0, 0.01)
    assert lo == d.min() and hi == d.max()
    c, w = 0.5 * (lo + hi), 0.5 * (hi - lo)
    x = (d - c) / w
    # Tr T_k(x) = sum_i cos(k arccos x_i)
    for k in range(1, 9):
        assert abs(f[8 + k] - np.cos(k * np.arccos(np.clip(x, -1, 1))).sum() / d.size) < 1e-13
    # no off-diagonal entries: every radius in the first bin
    assert hr[0] == d.size and hr[1:].sum() == 0
    # diagonal histogram against numpy's (last bin closed, as the clamp makes it)
    ref, _ = np.histogram(x, bins=np.linspace(-1.0, 1.0, 25))
    assert np.array_equal(hd, ref)
    assert f[0] == c and f[1] == w and f[6] == 11.0 / 37
    assert f[61] == x.min() and f[62] == x.max()


def test_symmetric_spectrum_at_half_filling_puts_mu0_at_the_centre():
    # erfc occupation: f(c + y) = 1 - f(c - y); a spectrum symmetric about c
    # with N_e = n / 2 has N(c) = n / 2 for every degree
    d = np.array([-1.0, -0.7, -0.2, 0.2, 0.7, 1.0]) * 0.8 - 0.3
    f, (lo, hi), _ = of.features(diag_csr(d), diag_csr(d).with_values(None), 4, 0.3, 2.0, 3.0, 0.01)
    assert abs(f[63]) < 1e-8


def test_gershgorin_and_radii_brute_force():
    rng = np.random.default_rng(1)
    n = 23
    A = sp.random(n, n, density=0.2, random_state=2).toarray()
    A = A + A.T + np.diag(rng.uniform(-1, 1, n))
    Hp = Csr.from_scipy(sp.csr_matrix(A))
    f, (lo, hi), (hd, hr) = of.features(Hp, Hp.with_values(None), 4, 0.3, 2.0, 10.0, 0.02)
    R = np.array([sum(abs(A[i, j]) for j in range(n) if j != i) for i in range(n)])
    dd = np.diag(A)
    assert abs(lo - min(dd - R)) < 1e-15 and abs(hi - max(dd + R)) < 1e-15
    w = 0.5 * (hi - lo)
    counts = np.zeros(16, dtype=int)
    for r in R / w:
        counts[min(15, int(np.floor(r * 16)))] += 1
    assert np.array_equal(hr, counts)
    assert abs(f[59] - (R / w).mean()) < 1e-15 and abs(f[60] - (R / w).max()) < 1e-15
