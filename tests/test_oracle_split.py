"""Pins of the oracle's split (shifted) three-point kernel, Sec. III.A.2.

The paper defines the split kernel as 2^-d times the product over axes of
phi(x - s/2) + phi(x + s/2). What the mathematics then fixes, checked here
without reusing the oracle's own formulas:
  * s = 0 gives back the three-point kernel;
  * each shifted copy sums to one and has zero first moment, so their mean
    does too, at every position (brute force over a wide node range);
  * the support is |d| < 3/2 + s/2, inside the four-node layout for s <= h;
  * the blob volume uses the position average of sum phi^2, checked against
    a brute-force average over 200000 positions, and its cross term is an
    autocorrelation A with A(0) = 1/2 and integral of A = 1;
  * the interpolation of a field linear near the blob is exact, and J S 1
    equals the position-dependent sum of squares (product over axes).
"""
import numpy as np
import pytest

from oracle import icm


def P(**kw):
    return icm.Params(**kw)


def brute_split(r, sigma):
    """The paper's one-axis factor written out: (phi(r - s/2) + phi(r + s/2)) / 2."""
    return 0.5 * (icm.phi3(np.asarray(r) - sigma / 2.0) + icm.phi3(np.asarray(r) + sigma / 2.0))


def test_zero_shift_is_the_three_point_kernel():
    r = np.linspace(-2.5, 2.5, 1001)
    assert np.array_equal(icm.split_phi3(r, 0.0), icm.phi3(r))
    p = P(kernel=3, kernel_shift=0.0)
    assert p.blob_volume == P(kernel=3).blob_volume


@pytest.mark.parametrize("sigma", [0.1, 0.37, 0.5, 0.83, 1.0])
def test_unity_and_first_moment_at_every_position(sigma):
    x = np.random.default_rng(1).uniform(0.0, 1.0, 4000)
    k = np.arange(-6, 7)
    d = x[:, None] - k[None, :]
    w = icm.split_phi3(d, sigma)
    assert np.max(np.abs(w.sum(axis=1) - 1.0)) < 1e-14
    assert np.max(np.abs((w * d).sum(axis=1))) < 1e-14
    assert np.min(w) >= 0.0
    # the same weights as the paper's factor written out
    assert np.max(np.abs(w - brute_split(d, sigma))) == 0.0


@pytest.mark.parametrize("sigma", [0.2, 0.6, 1.0])
def test_support_fits_the_four_node_layout(sigma):
    r = np.linspace(-3.0, 3.0, 6001)
    w = icm.split_phi3(r, sigma)
    assert np.all(w[np.abs(r) >= 1.5 + sigma / 2.0] == 0.0)
    assert np.all(w[np.abs(r) < 1.5 + sigma / 2.0 - 1e-9] > 0.0)
    # the oracle's four nodes floor(x) + {-1, 0, 1, 2} carry all the weight
    x = np.random.default_rng(2).uniform(-7.0, 7.0, 500)
    nodes, d = icm.stencil_nodes(4, x)
    assert np.max(np.abs(icm.split_phi3(d, sigma).sum(axis=1) - 1.0)) < 1e-14


@pytest.mark.parametrize("sigma", [0.3, 0.75, 1.0])
def test_split_derivative_matches_finite_difference(sigma):
    r = np.linspace(-2.1, 2.1, 413) + 1e-3
    eps = 1e-6
    fd = (icm.split_phi3(r + eps, sigma) - icm.split_phi3(r - eps, sigma)) / (2 * eps)
    assert np.max(np.abs(fd - icm.dsplit_phi3(r, sigma))) < 1e-6


def test_autocorrelation_closed_values():
    """A(0) = integral of phi3^2 = 1/2 (the constant sum of squares averaged
    over a cell); A vanishes beyond lag 3; the integral of A over all lags is
    (integral of phi3)^2 = 1."""
    from scipy.integrate import quad
    assert icm.phi3_autocorrelation(0.0) == pytest.approx(0.5, abs=1e-13)
    assert icm.phi3_autocorrelation(3.0) == 0.0
    total = quad(icm.phi3_autocorrelation, -3.0, 3.0, points=[-2, -1, 0, 1, 2], limit=200)[0]
    assert total == pytest.approx(1.0, abs=1e-10)


@pytest.mark.parametrize("sigma", [0.25, 0.5, 1.0])
def test_blob_volume_is_the_position_average(sigma):
    """dV = h^3 / <sum phi^2>^3 with the average over the position in a cell,
    taken here by brute force (midpoint rule, 200000 positions)."""
    m = 200000
    x = (np.arange(m) + 0.5) / m
    k = np.arange(-6, 7)
    w = brute_split(x[:, None] - k[None, :], sigma)
    avg = np.mean(np.sum(w * w, axis=1))
    p = P(kernel=3, kernel_shift=sigma, h=0.8, rho=1.3)
    assert p.blob_volume == pytest.approx(0.8 ** 3 / avg ** 3, rel=1e-9)
    assert p.m_f == pytest.approx(1.3 * p.blob_volume, rel=1e-15)
    # larger shifts spread the blob over more fluid
    assert p.blob_volume > P(kernel=3, h=0.8).blob_volume


def test_interp_of_a_locally_linear_field_is_exact():
    """Unity and zero first moment make J reproduce a linear field at the
    blob; the field is linear over the blob's stencil (periodic wrap far)."""
    n = (16, 16, 16)
    p = P(n=n, kernel=3, kernel_shift=0.7)
    nx, ny, nz = n
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    v = np.zeros((3, nz, ny, nx))
    g = np.array([[0.3, -1.1, 0.45], [0.9, 0.2, -0.6], [-0.25, 0.7, 1.3]])
    c = np.array([1.0, -2.0, 0.5])
    offs = {0: (0.0, 0.5, 0.5), 1: (0.5, 0.0, 0.5), 2: (0.5, 0.5, 0.0)}
    for a in range(3):
        ox, oy, oz = offs[a]
        v[a] = c[a] + g[a, 0] * (ii + ox) + g[a, 1] * (jj + oy) + g[a, 2] * (kk + oz)
    q = np.array([[7.3, 8.85, 6.02], [8.5, 7.0, 9.49]])
    u = icm.interp(p, v, q)
    expect = c[None, :] + q @ g.T
    assert np.max(np.abs(u - expect)) < 1e-12


def test_JS1_is_the_position_dependent_sum_of_squares():
    """J S applied to a unit force is, per component, the product over the
    three axes of sum phi_s^2 at that component's offsets, over dV_f."""
    p = P(n=(12, 12, 12), kernel=3, kernel_shift=0.6, h=1.1)
    q = np.array([[5.17, 4.42, 6.93]])
    k = np.arange(-20, 21)
    for a in range(3):
        F = np.zeros((1, 3))
        F[0, a] = 1.0
        got = icm.interp(p, icm.spread(p, F, q), q)[0, a]
        prod = 1.0
        for b in range(3):
            o = 0.0 if b == a else 0.5
            x = q[0, b] / p.h - o
            prod *= float(np.sum(brute_split(x - k, 0.6) ** 2))
        assert got == pytest.approx(prod / p.cell_volume, rel=1e-13)


def test_split_kernel_rejected_with_four_point_or_large_shift():
    for kw in (dict(kernel=4, kernel_shift=0.5), dict(kernel=3, kernel_shift=1.5),
               dict(kernel=3, kernel_shift=-0.1)):
        with pytest.raises(ValueError):
            icm.interp(P(n=(8, 8, 8), **kw), np.zeros((3, 8, 8, 8)), np.array([[1.0, 2.0, 3.0]]))
