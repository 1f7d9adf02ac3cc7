"""The paper's own training instances (Sec. 4.1 Poisson, Sec. 4.2 Burgers
after its change of variable): shapes, point placement and targets."""
import numpy as np

from paper_2409_14248_amd import workloads as WL


def test_poisson_paper_instance():
    pr = WL.make_problem(WL.WORKLOADS["poisson_paper"])
    assert pr.net.widths == (2, 2, 1) and pr.net.G == 5 and pr.net.n_basis == 8
    assert pr.n_int == 960 and pr.n_bc == 120
    assert np.all(np.abs(pr.x_int) <= 1.0)
    # 30 evenly spaced points on each of the four edges, target 0
    on_edge = np.isclose(np.abs(pr.x_bc), 1.0).any(axis=1)
    assert on_edge.all() and np.all(pr.g_bc == 0.0)


def test_burgers_paper_instance():
    pr = WL.make_problem(WL.WORKLOADS["burgers_paper"])
    assert pr.net.widths == (2, 3, 3, 3, 1) and pr.net.G == 7
    assert (pr.net.lo, pr.net.hi) == (0.0, 2.5)
    assert pr.pde.adv == 0.25 and np.isclose(pr.pde.nu, 0.001 / 16)
    assert pr.n_int == 10000 and pr.n_bc == 300
    assert np.all((pr.x_int >= 0.0) & (pr.x_int <= 2.5))
    ic, w0, w1 = pr.x_bc[:100], pr.x_bc[100:200], pr.x_bc[200:]
    assert np.all(ic[:, 1] == 0.0) and np.all(w0[:, 0] == 0.0) and np.all(w1[:, 0] == 2.5)
    np.testing.assert_allclose(pr.g_bc[:100], 1.0 / np.cosh(4.0 * ic[:, 0] - 5.0))
    assert np.all(pr.g_bc[100:] == 0.0)
    # the initial profile peaks at x = 1.25 (the original x = 0)
    assert abs(ic[np.argmax(pr.g_bc[:100]), 0] - 1.25) < 0.02
