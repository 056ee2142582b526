"""Host tests of the library's L-BFGS (pbs_lbfgs_minimize, no GPU needed):
known minima of a convex quadratic and of the Rosenbrock function, the stop
reasons, and error propagation from a failing objective."""

import numpy as np
import pytest

from paper_2606_28952_amd import api


def _lib_or_skip():
    from paper_2606_28952_amd import _abi

    try:
        _abi.lib()
    except (RuntimeError, OSError) as exc:
        pytest.skip(f"library not loadable: {exc}")


def test_quadratic_minimum():
    _lib_or_skip()
    rng = np.random.default_rng(0)
    a = rng.normal(size=(20, 20))
    A = a @ a.T + 0.5 * np.eye(20)
    b = rng.normal(size=20)
    x, f, it, ev, why = api.lbfgs_minimize(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(20),
                                           g_tol=1e-10, f_tol=0.0)
    xs = np.linalg.solve(A, b)
    assert why == "gradient"
    assert np.abs(x - xs).max() < 1e-8
    assert abs(f - (-0.5 * b @ xs)) < 1e-12
    assert it <= 130  # scipy L-BFGS-B (10 pairs) needs 86 iterations here


def test_rosenbrock_minimum():
    _lib_or_skip()

    def fg(x):
        f = np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)
        g = np.zeros_like(x)
        g[:-1] = -400.0 * x[:-1] * (x[1:] - x[:-1] ** 2) - 2 * (1 - x[:-1])
        g[1:] += 200.0 * (x[1:] - x[:-1] ** 2)
        return f, g

    x, f, it, ev, why = api.lbfgs_minimize(fg, np.full(6, -1.2), max_iter=1000, g_tol=1e-8, f_tol=0.0)
    assert why == "gradient"
    assert np.abs(x - 1.0).max() < 1e-6
    assert ev >= it


def test_iteration_limit_and_decrease_stop():
    _lib_or_skip()
    A = np.diag(np.linspace(1, 100, 30))
    fg = lambda x: (0.5 * x @ A @ x, A @ x)
    _, _, it, _, why = api.lbfgs_minimize(fg, np.ones(30), max_iter=3, g_tol=0.0, f_tol=0.0)
    assert (it, why) == (3, "iterations")
    _, _, _, _, why = api.lbfgs_minimize(fg, np.ones(30), max_iter=500, g_tol=0.0, f_tol=1e-3)
    assert why == "decrease"
    _, _, it, ev, why = api.lbfgs_minimize(fg, np.zeros(30), g_tol=1e-12)
    assert (it, ev, why) == (0, 1, "gradient")


def test_objective_failure_propagates():
    _lib_or_skip()

    def bad(x):
        raise FloatingPointError("boom")

    with pytest.raises(FloatingPointError):
        api.lbfgs_minimize(bad, np.ones(3))
