"""The library's host-side tridiagonal eigenvalue routine (bri_ritz_values),
called through the C ABI on the CPU: bisection against numpy's dense
eigenvalues, and the spurious-copy filter on a Lanczos run without
re-orthogonalisation done here in numpy on a matrix with a known spectrum."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def api():
    from paper_1012_3615_amd import api as a
    return a


def test_bisection_matches_dense(api):
    rng = np.random.default_rng(9001)
    for k in (1, 2, 7, 60, 200):
        a = rng.standard_normal(k)
        b = rng.standard_normal(k)
        t = np.diag(a) + np.diag(b[1:], 1) + np.diag(b[1:], -1)
        got = api.bri_ritz_values(a, b, filter=False)
        assert np.abs(got - np.linalg.eigvalsh(t)).max() < 1e-13 * max(1.0, np.abs(a).max() + 2 * np.abs(b).max())


def test_spurious_filter_on_lanczos_without_reorthogonalisation(api):
    """A diagonal matrix with 40 well-separated eigenvalues, 150 Lanczos steps
    without re-orthogonalisation: the raw Ritz values contain repeated copies
    of converged eigenvalues; the filtered ones are the distinct eigenvalues."""
    rng = np.random.default_rng(9002)
    lam = np.sort(rng.uniform(0.1, 10.0, 40))
    lam = np.concatenate([lam, [0.05, 12.0]])
    n = len(lam)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    k = 150
    al, be = np.zeros(k), np.zeros(k)
    be[0] = 1.0
    vp = np.zeros(n)
    for j in range(k):
        w = lam * v
        al[j] = v @ w
        w = w - al[j] * v - (be[j] * vp if j else 0)
        if j + 1 < k:
            be[j + 1] = np.linalg.norm(w)
            vp, v = v, w / be[j + 1]
    raw = api.bri_ritz_values(al, be, filter=False)
    good = api.bri_ritz_values(al, be, filter=True)
    assert len(raw) == k and len(good) < k
    assert abs(good[0] - lam.min()) < 1e-10 and abs(good[-1] - lam.max()) < 1e-10
    # every exact eigenvalue is represented, and every kept value is close to one
    for x in lam:
        assert np.abs(good - x).min() < 1e-8
    for g in good:
        assert np.abs(lam - g).min() < 1e-6


def test_sign_error_bound_and_degree(api):
    """The library's error bound of the x^-1/2 interpolant equals a direct
    evaluation with numpy's Chebyshev interpolation at the same nodes, and
    sign_degree returns the smallest degree meeting a target."""
    lo, hi = 0.02, 2.5
    for deg in (5, 40, 120):
        c = np.polynomial.chebyshev.chebinterpolate(
            lambda t: 1.0 / np.sqrt(0.5 * (hi - lo) * t + 0.5 * (hi + lo)), deg)
        xs = np.linspace(lo, hi, 20001)
        p = np.polynomial.chebyshev.chebval((2 * xs - hi - lo) / (hi - lo), c)
        want = np.max(np.abs(1 - np.sqrt(xs) * p))
        # agreement up to the rounding of evaluating a degree-120 polynomial (~1e-13)
        assert abs(api.bri_sign_approx_error(lo, hi, deg) - want) <= 1e-6 * want + 1e-12
    d = api.sign_degree(lo, hi, 1e-10)
    assert api.bri_sign_approx_error(lo, hi, d) < 1e-10 <= api.bri_sign_approx_error(lo, hi, d - 1)
