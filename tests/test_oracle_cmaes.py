"""Pins of the oracle's CMA-ES (the reference-parameter search of Sec. II C) on problems
whose behaviour is known: convergence on a shifted sphere and on a rotated ill-conditioned
ellipsoid (which needs a working covariance update), invariance under order-preserving
transformations of the fitness (selection by rank only), growth of the step size on a
linear function (cumulative step-size adaptation), and the box (no candidate outside it
is ever the best)."""
import numpy as np

from oracle import cmaes


def _normals(seed, gens, lam, n):
    return np.random.default_rng(seed).standard_normal((gens, lam, n))


def _run(f, x0, sigma0, lam, normals):
    es = cmaes.CMAES(x0, sigma0, lam)
    for z in normals:
        x = es.ask(z)
        es.tell(f(x))
    return es


def test_converges_on_shifted_sphere():
    n = 13
    xs = np.linspace(0.2, 0.8, n)
    es = _run(lambda x: -np.sum((x - xs) ** 2, axis=1), np.full(n, 0.5), 0.3, 16, _normals(1, 400, 16, n))
    assert np.max(np.abs(es.m - xs)) < 1e-8
    assert es.sigma < 1e-7


def test_converges_on_rotated_ill_conditioned_ellipsoid():
    """Condition number 1e4 in a random rotation: without covariance learning the step
    size could not shrink past the long axis in this budget."""
    n = 8
    rng = np.random.default_rng(2)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    h = q @ np.diag(np.logspace(0, 4, n)) @ q.T
    xs = rng.uniform(-1, 1, n)
    f = lambda x: -np.einsum("ki,ij,kj->k", x - xs, h, x - xs)  # noqa: E731
    es = _run(f, np.zeros(n), 0.5, 12, _normals(3, 900, 12, n))
    assert np.max(np.abs(es.m - xs)) < 1e-6
    ev = np.linalg.eigvalsh(es.C)
    assert ev.max() / ev.min() > 1e3   # the covariance has learned the conditioning


def test_selection_uses_ranks_only():
    n = 13
    z = _normals(4, 60, 10, n)
    f = lambda x: -np.sum(np.abs(x - 0.3) ** 1.5, axis=1)  # noqa: E731
    a = _run(f, np.full(n, 0.5), 0.2, 10, z)
    b = _run(lambda x: np.exp(f(x)) * 3.0 - 7.0, np.full(n, 0.5), 0.2, 10, z)
    assert np.array_equal(a.m, b.m) and a.sigma == b.sigma and np.array_equal(a.C, b.C)


def test_step_size_grows_on_a_linear_function():
    n = 13
    es = _run(lambda x: x[:, 0], np.zeros(n), 1e-3, 10, _normals(5, 60, 10, n))
    assert es.sigma > 100 * 1e-3
    assert es.m[0] > 10 * 1e-3


def test_box_search_stays_inside_and_reaches_the_bound():
    n = 13
    lo, hi = np.zeros(n), np.ones(n)
    z = _normals(6, 150, 12, n)
    best_x, best_f, traces = cmaes.search(lambda th: th[:, 0] - np.sum((th[:, 1:] - 0.5) ** 2, axis=1), lo, hi,
                                          np.full(n, 0.5), 0.2, 12, z[None])
    trace = traces[0]
    assert np.all((best_x >= 0) & (best_x <= 1))
    assert best_x[0] > 0.99 and best_f > 0.98
    assert np.all(np.diff(trace[:, 0]) >= 0)          # the best-so-far never decreases


def test_large_population_learns_faster_with_the_rank_mu_update():
    """Condition 1e6, lambda = 64: the rank-mu update lets the covariance learn from the whole
    selected population each generation (fewer than 200 generations to 1e-6; with the rank-one
    update alone over 400)."""
    n = 8
    rng = np.random.default_rng(2)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    h = q @ np.diag(np.logspace(0, 6, n)) @ q.T
    xs = rng.uniform(-1, 1, n)
    es = cmaes.CMAES(np.zeros(n), 0.5, 64)
    z = _normals(3, 200, 64, n)
    for g in range(200):
        x = es.ask(z[g])
        es.tell(-np.einsum("ki,ij,kj->k", x - xs, h, x - xs))
    assert np.max(np.abs(es.m - xs)) < 1e-6


def test_step_size_path_is_independent_of_the_covariance():
    """Under random selection (fitness independent of x) the step-size path is built from
    A^{-1} <y>_w, which is N(0, I)-like whatever C is, so sigma only wanders; with a very
    elongated C it would otherwise grow without bound."""
    n = 13
    for trial in range(3):
        es = cmaes.CMAES(np.zeros(n), 1.0, 12)
        es.C = np.diag([1e4] + [1.0] * (n - 1))
        rng = np.random.default_rng(10 + trial)
        for _ in range(100):
            es.ask(rng.standard_normal((12, n)))
            es.tell(rng.standard_normal(12))
        assert abs(np.log(es.sigma)) < 5.0


def test_recombination_weights_give_mu_eff_near_a_quarter_of_lambda():
    """The default log-decreasing weights make mu_eff about lambda/4 (equal weights would
    make it lambda/2)."""
    for lam in (8, 16, 32, 64, 128, 1024):
        es = cmaes.CMAES(np.zeros(13), 1.0, lam)
        assert 0.2 < es.mueff / lam < 0.35


def test_multistart_keeps_the_best_mode_and_its_runs_do_not_interact():
    """Two separated maxima, the higher at b: a run started at each converges to its own, the
    multistart returns b's (found by the first run, so keeping the last run's best fails), and
    each run's trace is the one it has when run alone."""
    n = 4
    lo, hi = np.zeros(n), np.ones(n)
    a, b = np.full(n, 0.25), np.full(n, 0.75)

    def f(th):
        return np.exp(-np.sum((th - a) ** 2, axis=1) / 0.005) + 2.0 * np.exp(-np.sum((th - b) ** 2, axis=1) / 0.005)

    starts = np.array([b - 0.02, a + 0.02])
    z = np.stack([_normals(11, 120, 10, n), _normals(12, 120, 10, n)])
    best_x, best_f, traces = cmaes.search(f, lo, hi, starts, 0.05, 10, z)
    assert abs(best_f - 2.0) < 1e-9 and np.max(np.abs(best_x - b)) < 1e-4
    assert abs(traces[1][-1, 0] - 1.0) < 1e-9 and np.max(np.abs(traces[1][-1, 2:] - a)) < 1e-4
    for r in range(2):
        _, _, alone = cmaes.search(f, lo, hi, starts[r], 0.05, 10, z[r:r + 1])
        np.testing.assert_array_equal(traces[r], alone[0])
