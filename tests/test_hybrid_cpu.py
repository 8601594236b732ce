"""Host logic of the hybrid driver: step accounting against the paper's printed
step reductions, the paper's table arithmetic, and the prediction guard."""
import pytest

from paper_2604_27158_amd import hybrid as H


@pytest.mark.parametrize("k,printed", [(1, 50), (2, 34), (3, 25)])
def test_step_reduction_reproduces_paper(k, printed):
    """1:k hybrids (one FNO step of dT, k*dT of LBM): eps_N = 1/(1+k); the paper
    prints 50 / 34 / 25 % (33.3 rounded up in print)."""
    e = 100 * H.step_reduction(1, 223, k * 223)
    assert abs(e - printed) <= 1.0


def test_flagship_cycle_accounting():
    """K = 5 FNO calls of dt = 100, then 200 lattice steps, 20 cycles: 100 FNO calls
    and 4000 lattice steps cover a 14 000-step horizon."""
    k, dt, n, cycles = 5, 100, 200, 20
    assert cycles * (k * dt + n) == 14000
    assert cycles * k == 100 and cycles * n == 4000
    assert abs(H.step_reduction(k, dt, n) - 5 / 7) < 1e-15


@pytest.mark.parametrize("lbm,fno,printed", [(49, 33, 32.7), (20, 6, 70.0), (40, 23, 42.5),
                                             (105, 96, 8.57), (28, 14, 50.0), (74, 53, 28.4),
                                             (42, 26, 38.1), (70, 48, 31.4)])
def test_convergence_speedups_reproduce_paper_table(lbm, fno, printed):
    """Speed-up = (N_LBM - N_FNO) / N_LBM recomputed from the paper's convergence
    table columns (the v row at 1e-4, 63 -> 53 printed as 11.7 %, is inconsistent
    with the formula and left out)."""
    assert abs(100 * H.convergence_speedup(lbm, fno) - printed) < 0.06


def test_error_and_runtime_reduction_formulas():
    assert H.error_reduction(2.0, 0.5) == 0.75
    assert abs(H.runtime_reduction(10.0, 8.82) - 0.118) < 1e-12


def test_guard_rejects_and_accepts():
    g = H.Guard(max_speed=0.3, mass_rel_tol=0.05)
    ok = {"nonfinite": 0, "max_speed": 0.1, "mass": 100.0}
    assert g.accept(ok, 100.0)[0]
    assert not g.accept(dict(ok, nonfinite=3), 100.0)[0]
    assert not g.accept(dict(ok, max_speed=0.5), 100.0)[0]
    assert not g.accept(dict(ok, mass=110.0), 100.0)[0]
    assert g.accept(dict(ok, mass=104.0), 100.0)[0]
