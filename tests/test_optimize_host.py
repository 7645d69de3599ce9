"""Host-side statistics of the optimisation CLI (no GPU): the plateau summary
of the last two windows of iteration energies."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1807_10633_amd.optimize import paper_schedule, plateau  # noqa: E402


def test_plateau_of_a_flat_series_is_within_its_error_bars():
    rng = np.random.default_rng(3)
    e = list(-5.0 + 0.02 * rng.normal(size=400))
    p = plateau(e, 200)
    assert abs(p["difference_in_sigma"]) < 4.0
    # block means of independent noise: stderr near 0.02 / sqrt(200)
    assert 0.5 * 0.02 / np.sqrt(200) < p["last"]["stderr"] < 2.0 * 0.02 / np.sqrt(200)


def test_plateau_sees_a_drift():
    e = list(np.linspace(0.0, -1.0, 400) + 1e-3 * np.random.default_rng(4).normal(size=400))
    p = plateau(e, 200)
    assert p["difference"] == pytest.approx(-0.5, abs=0.01)
    assert p["difference_in_sigma"] < -10.0


def test_paper_schedule():
    # section "Performance of the optimizer": 0.001 for five iterations, then 0.01
    assert [paper_schedule(i) for i in range(7)] == [0.001] * 5 + [0.01] * 2
