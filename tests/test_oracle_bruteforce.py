"""Brute-force pin of the FP64 lattice oracle: the D2Q9 BGK step of the paper's
Sec. 2.1 (moments Eqs. 4-5 with the half-force velocity, equilibrium Eq. 1,
collision Eq. 2 read as f* = f - (f - f_eq)/tau, plus the Guo source; streaming
Eq. 3 with halfway bounce-back; Zou-He columns) written out here a second time in
exact rational arithmetic (fractions.Fraction) and in 50-digit decimal arithmetic,
on 8x8 lattices with obstacles, a body force, walls and open columns.

The exact form is written independently of the oracle: dictionary-of-nodes state,
push-form streaming (every post-collision value is sent along its link, or back
into the node on a blocked link), and each formula typed from its textbook
definition.  All inputs are dyadic rationals, so the oracle sees them exactly; the
oracle's FP64 result must then agree to 1e-13 after 3 exact steps, and after 100
steps at 50 digits."""
import decimal
from fractions import Fraction

import numpy as np
import pytest

from oracle import lbm
from paper_2604_27158_amd import workloads as W

# D2Q9 (the velocity order of the library and the oracle; textbook weights)
C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
OPP = [C.index((-a, -b)) for a, b in C]


def weights(num):
    return [num(4) / num(9)] + [num(1) / num(9)] * 4 + [num(1) / num(36)] * 4


def equilibrium(num, w, rho, ux, uy):
    """Eq. 1: f_eq_q = w_q rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u)."""
    usq = ux * ux + uy * uy
    out = []
    for q, (cx, cy) in enumerate(C):
        cu = cx * ux + cy * uy
        out.append(w[q] * rho * (num(1) + 3 * cu + num(9) / num(2) * cu * cu - num(3) / num(2) * usq))
    return out


def zou_he(num, f, x, nx, u_in, rho_out):
    """Zou & He (1997) closures on a boundary column node: velocity (u_in, 0) at
    x = 0 (unknown f1, f5, f8), density rho_out at x = nx - 1 (unknown f3, f6, f7)."""
    f = list(f)
    if x == 0:
        rho = (f[0] + f[2] + f[4] + 2 * (f[3] + f[6] + f[7])) / (num(1) - u_in)
        f[1] = f[3] + num(2) / num(3) * rho * u_in
        f[5] = f[7] - (f[2] - f[4]) / 2 + num(1) / num(6) * rho * u_in
        f[8] = f[6] + (f[2] - f[4]) / 2 + num(1) / num(6) * rho * u_in
    elif x == nx - 1:
        ux = -num(1) + (f[0] + f[2] + f[4] + 2 * (f[1] + f[5] + f[8])) / rho_out
        f[3] = f[1] - num(2) / num(3) * rho_out * ux
        f[6] = f[8] - (f[2] - f[4]) / 2 - num(1) / num(6) * rho_out * ux
        f[7] = f[5] + (f[2] - f[4]) / 2 - num(1) / num(6) * rho_out * ux
    return f


class Exact:
    """Lattice state f(n) (pre-collision, after streaming and closures) on the fluid
    nodes, in the number type `num` (Fraction or Decimal)."""

    def __init__(self, num, lat, mask, rho0, ux0, uy0, g=(0, 0)):
        self.num, self.lat, self.mask = num, lat, mask
        self.nx, self.ny = lat.nx, lat.ny
        self.w = weights(num)
        self.tau = num(lat.tau_exact)
        self.gx, self.gy = num(g[0]), num(g[1])
        self.u_in, self.rho_out = num(lat.u_in_exact), num(1)
        self.fluid = [(i, j) for j in range(self.ny) for i in range(self.nx) if mask[j, i] == 0]
        self.f = {}
        for (i, j) in self.fluid:
            feq = equilibrium(num, self.w, num(rho0[j][i]), num(ux0[j][i]), num(uy0[j][i]))
            self.f[(i, j)] = self.close(feq, i)

    def close(self, f, i):
        if self.lat.bc_x == W.BC_ZOUHE and i in (0, self.nx - 1):
            return zou_he(self.num, f, i, self.nx, self.u_in, self.rho_out)
        return f

    def target(self, i, j, q):
        """Node that the link (i, j) + c_q reaches, or None when it is blocked (a wall,
        an open boundary or a solid node)."""
        ti, tj = i + C[q][0], j + C[q][1]
        if not 0 <= ti < self.nx:
            if self.lat.bc_x != W.BC_PERIODIC:
                return None
            ti %= self.nx
        if not 0 <= tj < self.ny:
            if self.lat.bc_y != W.BC_PERIODIC:
                return None
            tj %= self.ny
        return None if self.mask[tj, ti] else (ti, tj)

    def step(self):
        num, w, tau = self.num, self.w, self.tau
        post = {}
        for node, f in self.f.items():
            rho = sum(f)
            jx = sum(C[q][0] * f[q] for q in range(9))
            jy = sum(C[q][1] * f[q] for q in range(9))
            ux = (jx + rho * self.gx / 2) / rho          # Guo's half-force velocity
            uy = (jy + rho * self.gy / 2) / rho
            feq = equilibrium(num, w, rho, ux, uy)
            out = []
            for q, (cx, cy) in enumerate(C):
                cu = cx * ux + cy * uy
                # Guo, Zheng & Shi (2002): (1 - 1/(2 tau)) w [3 (c - u) + 9 (c.u) c] . (rho g)
                src = (1 - 1 / (2 * tau)) * w[q] * rho * (
                    3 * ((cx - ux) * self.gx + (cy - uy) * self.gy) + 9 * cu * (cx * self.gx + cy * self.gy))
                out.append(f[q] - (f[q] - feq[q]) / tau + src)
            post[node] = out
        new = {node: [None] * 9 for node in self.f}
        for (i, j), out in post.items():
            for q in range(9):
                t = self.target(i, j, q)
                if t is None:
                    slot, d = (i, j), OPP[q]            # halfway bounce-back
                else:
                    slot, d = t, q
                assert new[slot][d] is None
                new[slot][d] = out[q]
        for (i, j), f in new.items():
            assert all(v is not None for v in f)
            new[(i, j)] = self.close(f, i)
        self.f = new

    def array(self):
        out = np.zeros((9, self.ny, self.nx))
        for (i, j), f in self.f.items():
            out[:, j, i] = [float(v) for v in f]
        return out


def dyadic_fields(seed, nx, ny, amp_rho_bits, amp_u_bits, u0=0.0):
    """Random fields whose values are k / 2^24 (exact in FP64 and as fractions)."""
    rng = np.random.default_rng(seed)
    den = 1 << 24
    r = rng.integers(-(1 << amp_rho_bits), 1 << amp_rho_bits, size=(ny, nx))
    a = rng.integers(-(1 << amp_u_bits), 1 << amp_u_bits, size=(ny, nx))
    b = rng.integers(-(1 << amp_u_bits), 1 << amp_u_bits, size=(ny, nx))
    rho = [[Fraction(den + int(r[j, i]), den) for i in range(nx)] for j in range(ny)]
    ux = [[Fraction(int(a[j, i]), den) + Fraction(u0) for i in range(nx)] for j in range(ny)]
    uy = [[Fraction(int(b[j, i]), den) for i in range(nx)] for j in range(ny)]
    return rho, ux, uy


class Case:
    """An 8x8 configuration with dyadic parameters."""

    def __init__(self, bc_x, bc_y, tau, g, u_in, solid):
        self.nx = self.ny = 8
        self.bc_x, self.bc_y = bc_x, bc_y
        self.tau_exact, self.u_in_exact, self.g = Fraction(tau), Fraction(u_in), (Fraction(g[0]), Fraction(g[1]))
        self.mask = np.zeros((8, 8), np.uint8)
        for (i, j) in solid:
            self.mask[j, i] = 1
        self.lat = W.Lattice(nx=8, ny=8, tau=float(tau), gx=float(g[0]), gy=float(g[1]), bc_x=bc_x,
                             bc_y=bc_y, u_in=float(u_in), rho_out=1.0)
        self.lat.tau_exact, self.lat.u_in_exact = self.tau_exact, self.u_in_exact


CASES = {
    # periodic x, walls in y, an obstacle (a plus sign and a lone cell), a body force
    "walls+force+obstacles": Case(W.BC_PERIODIC, W.BC_WALL, Fraction(3, 4), (2.0 ** -13, -(2.0 ** -15)), 0,
                                  [(3, 4), (2, 4), (4, 4), (3, 3), (3, 5), (6, 1)]),
    # walls on all four sides, a diagonal obstacle pair (corner links only), force
    "closed box+force": Case(W.BC_WALL, W.BC_WALL, Fraction(5, 8), (-(2.0 ** -14), 2.0 ** -13), 0,
                             [(4, 4), (5, 5), (1, 6)]),
    # Zou-He inlet/outlet in x, periodic in y, obstacles, no force
    "zou-he+obstacles": Case(W.BC_ZOUHE, W.BC_PERIODIC, Fraction(7, 8), (0, 0), Fraction(1, 32),
                             [(3, 3), (4, 3), (3, 4), (5, 6)]),
}


def oracle_after(case, rho0, ux0, uy0, n):
    f64 = lambda a: np.array([[float(v) for v in row] for row in a])
    s = lbm.Sim(case.lat, case.mask).init(f64(rho0), f64(ux0), f64(uy0))
    s.run(n)
    return s.f * (case.mask == 0)[None]     # the oracle keeps the rest weights on solids


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_equals_exact_rational_three_steps(name):
    case = CASES[name]
    u0 = float(case.u_in_exact)
    rho0, ux0, uy0 = dyadic_fields(len(name), 8, 8, 16, 17, u0)
    ex = Exact(Fraction, case.lat, case.mask, rho0, ux0, uy0, case.g)
    f_or = oracle_after(case, rho0, ux0, uy0, 0)
    d0 = np.max(np.abs(f_or - ex.array()))
    for _ in range(3):
        ex.step()
    f_ex = ex.array()
    f_or = oracle_after(case, rho0, ux0, uy0, 3)
    d = np.max(np.abs(f_or - f_ex))
    print(f"{name}: max |oracle - exact| init {d0:.2e}, after 3 steps {d:.2e}")
    assert d0 <= 1e-15 and d <= 1e-13


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_equals_fifty_digit_run_over_100_steps(name):
    case = CASES[name]
    decimal.getcontext().prec = 50

    def num(v):
        if isinstance(v, Fraction):
            return decimal.Decimal(v.numerator) / decimal.Decimal(v.denominator)
        return decimal.Decimal(v)

    u0 = float(case.u_in_exact)
    rho0, ux0, uy0 = dyadic_fields(len(name) + 1, 8, 8, 16, 17, u0)
    ex = Exact(num, case.lat, case.mask, rho0, ux0, uy0, case.g)
    for _ in range(100):
        ex.step()
    f_ex = ex.array()
    f_or = oracle_after(case, rho0, ux0, uy0, 100)
    d = np.max(np.abs(f_or - f_ex))
    # the run is not trivial: the state moved far beyond the bar
    moved = np.max(np.abs(f_ex - oracle_after(case, rho0, ux0, uy0, 0)))
    print(f"{name}: max |oracle - 50-digit| after 100 steps {d:.2e} (state moved {moved:.2e})")
    assert d <= 1e-13 and moved > 1e-6
