"""Pins of the CCD oracle (supplement Section 3) against mathematics it must
satisfy: the coplanarity cubic equals the determinant at every t, the
relative-displacement bound is no larger than the standard one and
independent of the frame, it bounds the relative motion of every pair of
points of the primitives, and the safe step never passes a root of the
cubic and stops within the bisection's resolution of the first one."""
import numpy as np
import pytest

from oracle import ccd


def test_cubic_coefficients_hand_case():
    # unit tetrahedron whose apex moves down at unit speed: volume 1 - t
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    p = np.zeros((4, 3))
    p[3, 2] = -1.0
    np.testing.assert_allclose(ccd.cubic_coefficients(x, p), [1.0, -1.0, 0.0, 0.0], atol=1e-13)
    # all three edges shrinking: (1 - t)^3
    p = -x.copy()
    np.testing.assert_allclose(ccd.cubic_coefficients(x, p), [1.0, -3.0, 3.0, -1.0], atol=1e-12)


def test_cubic_matches_determinant_at_every_t():
    rng = np.random.default_rng(0)
    for _ in range(50):
        x, p = rng.standard_normal((2, 4, 3))
        coef = ccd.cubic_coefficients(x, p)
        for t in rng.uniform(-2, 2, 5):
            assert ccd._f(coef, t) == pytest.approx(ccd.volume(x + t * p), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("kind", [ccd.PT, ccd.EE])
def test_relative_bound_tighter_and_frame_invariant(kind):
    rng = np.random.default_rng(1)
    for _ in range(200):
        p = rng.standard_normal((4, 3))
        lt, lo = ccd.l_tight(p, kind), ccd.l_original(p, kind)
        assert lt <= lo * (1 + 1e-15)
        vc = 5.0 * rng.standard_normal(3)
        assert ccd.l_tight(p + vc, kind) == pytest.approx(lt, rel=1e-12)
    # a common motion costs the standard bound but not the relative one
    p = np.tile([3.0, 0.0, 0.0], (4, 1))
    assert ccd.l_tight(p, kind) == 0.0 and ccd.l_original(p, kind) == pytest.approx(6.0)


@pytest.mark.parametrize("kind", [ccd.PT, ccd.EE])
def test_relative_bound_covers_every_point_pair(kind):
    """Brute force over barycentric points of both primitives."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        p = rng.standard_normal((4, 3))
        lt = ccd.l_tight(p, kind)
        worst = 0.0
        for _ in range(400):
            if kind == ccd.PT:
                w = rng.dirichlet(np.ones(3))
                dp = p[0] - w @ p[1:]
            else:
                s, t = rng.uniform(0, 1, 2)
                dp = (1 - s) * p[0] + s * p[1] - (1 - t) * p[2] - t * p[3]
            worst = max(worst, np.linalg.norm(dp))
        assert worst <= lt * (1 + 1e-12)
        assert worst >= 0.5 * lt      # the vertex pairs themselves are among the samples' limits


def _first_root(coef, lo):
    """Smallest real root of the cubic in [lo, 1], by numpy.roots."""
    d, c, b, a = coef
    r = np.roots([a, b, c, d]) if a != 0 else (np.roots([b, c, d]) if b != 0 else
                                                (np.array([-d / c]) if c != 0 else np.array([])))
    r = np.real(r[np.abs(np.imag(r)) <= 1e-12 * np.maximum(1.0, np.abs(np.real(r)))])
    r = r[(r >= lo) & (r <= 1.0)]
    return r.min() if r.size else None


def test_cubic_safe_never_passes_a_root_and_is_tight():
    rng = np.random.default_rng(3)
    n_root = 0
    for k in range(3000):
        coef = rng.standard_normal(4) * rng.choice([1e-3, 1.0, 1e3], 4)
        if k % 3 == 0:          # cubics with a root planted in (0, 1)
            r0 = rng.uniform(0.05, 0.95)
            a, b = rng.standard_normal(2)
            # (t - r0)(a t^2 + b t + c2) with c2 > b^2 / (4a) when a > 0 keeps one real root
            c2 = b * b / (4 * abs(a)) + rng.uniform(0.1, 1.0)
            c2 = c2 if a > 0 else -c2
            coef = np.array([-r0 * c2, c2 - r0 * b, b - r0 * a, a])
        al = rng.choice([0.0, rng.uniform(0, 0.5)])
        alpha = ccd.cubic_safe(coef, al)
        x0 = max(0.0, al)
        assert x0 <= alpha <= 1.0
        r = _first_root(coef, x0)
        if r is None:
            assert alpha == 1.0
            continue
        n_root += 1
        assert alpha <= r + 1e-12
        # f keeps its sign on [x0, alpha]
        ts = np.linspace(x0, alpha, 64)
        f = ccd._f(coef, ts)
        f0 = ccd._f(coef, x0)
        if f0 != 0.0:
            assert np.all(np.sign(f[f != 0]) == np.sign(f0))
    assert n_root > 500


def test_cubic_safe_linear_and_special_cases():
    # linear f = 1 - 2t: root at 0.5, bisection stops within 2^-16 below it
    a = ccd.cubic_safe([1.0, -2.0, 0.0, 0.0], 0.0)
    assert 0.5 - 2.0 ** -16 <= a <= 0.5
    # no root in [0, 1]
    assert ccd.cubic_safe([1.0, 1.0, 1.0, 1.0], 0.0) == 1.0
    # lower bound past 1
    assert ccd.cubic_safe([1.0, -2.0, 0.0, 0.0], 1.5) == 1.0
    # start exactly on a root
    assert ccd.cubic_safe([0.0, 1.0, 0.0, 0.0], 0.0) == 0.0
    # lower bound beyond the root is trusted (the root is taken as a non-contact)
    assert ccd.cubic_safe([1.0, -2.0, 0.0, 0.0], 0.75) == 1.0


@pytest.mark.parametrize("kind", [ccd.PT, ccd.EE])
def test_pair_step_frame_invariant_and_safe(kind):
    rng = np.random.default_rng(4)
    for _ in range(200):
        x = rng.standard_normal((4, 3))
        p = rng.standard_normal((4, 3))
        a1 = ccd.pair_step(x, p, kind, 0.0)
        vc = 3.0 * rng.standard_normal(3)
        a2 = ccd.pair_step(x, p + vc, kind, 0.0)
        assert a2 == pytest.approx(a1, abs=1e-9)
        coef = ccd.cubic_coefficients(x, p)
        r = _first_root(coef, 0.0)
        assert (r is None and a1 == 1.0) or a1 <= r + 1e-12


def test_tight_lower_bound_normal_approach():
    """A point falling straight onto a triangle, the triangle moving away
    more slowly: the time of contact t_c is exactly dist / l_tight, where
    rounding can leave f past its root.  The step comes before the contact
    (the point stays above the plane), no earlier than the lower bound
    0.9 t_c, and within the bisection's 2^-16 of t_c when that is finer."""
    for gap, vt in ((1e-9, 0.3), (1e-3, 0.0), (0.25, 0.5), (3e-7, 0.9)):
        x4 = np.array([[0.1, 0.2, gap], [-1.0, -1.0, 0.0], [1.0, -1.0, 0.0], [0.0, 1.0, 0.0]])
        p4 = np.array([[0.0, 0.0, -1.0]] + [[0.0, 0.0, -vt]] * 3)
        t_c = gap / (1.0 - vt)
        step = ccd.pair_step(x4, p4, ccd.PT, gap)
        if t_c >= 1.0:
            assert step == 1.0
            continue
        assert 0.9 * t_c * (1.0 - 1e-12) <= step < t_c
        assert t_c - step <= max(0.1 * t_c, 2.0 ** -16) * (1.0 + 1e-9)
        z = x4[0, 2] + step * p4[0, 2] - step * p4[1, 2]
        assert z > 0.0
