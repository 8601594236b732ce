"""Pins of the FP64 lattice Boltzmann oracle against facts fixed by the mathematics
(closed forms, invariants, a textbook eigenvalue, integer counts) -- never against
a retyped copy of its own formulas."""
import math

import numpy as np
import pytest

from oracle import lbm
from paper_2604_27158_amd import workloads as W


CX, CY, OPP, WQ = lbm.lattice()


# ------------------------------------------------------------- lattice / f_eq

def test_lattice_isotropy():
    """D2Q9 weights: zeroth, second and fourth moments of an isotropic lattice
    with c_s^2 = 1/3 (Eq. 1's c_s; Kruger et al. 2017, Table 3.2)."""
    c = np.stack([CX, CY], 1).astype(float)
    assert abs(WQ.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("q,qa,qb->ab", WQ, c, c), np.eye(2) / 3, atol=1e-15)
    d = np.eye(2)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("q,qa,qb,qc,qd->abcd", WQ, c, c, c, c), iso4, atol=1e-15)
    for q in range(9):
        assert CX[OPP[q]] == -CX[q] and CY[OPP[q]] == -CY[q]


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.03, 0.05, -0.02), (0.97, -0.1, 0.07)])
def test_feq_moments(rho, ux, uy):
    """Eq. 1's equilibrium carries mass rho, momentum rho u and momentum flux
    rho (c_s^2 I + u u) exactly (Eqs. 4-5 applied to f_eq)."""
    f = lbm.feq(rho, ux, uy)
    c = np.stack([CX, CY], 1).astype(float)
    u = np.array([ux, uy])
    assert abs(f.sum() - rho) < 1e-14
    assert np.allclose(c.T @ f, rho * u, atol=1e-15)
    assert np.allclose(np.einsum("q,qa,qb->ab", f, c, c), rho * (np.eye(2) / 3 + np.outer(u, u)),
                       atol=1e-15)


# ------------------------------------------------------------------- masks

def test_raster_gauss_circle_counts():
    """Integer disc x^2 + y^2 <= r^2: the Gauss circle counts N(r) = 1, 5, 13, 29,
    49, 81 for r = 0..5 (OEIS A000328)."""
    counts = [1, 5, 13, 29, 49, 81]
    for r, n in enumerate(counts):
        m = lbm.raster(32, 32, np.array([W.circle(16, 16, r)]), False, False)
        assert int(m.sum()) == n


def test_raster_hand_pattern():
    """r = 2 disc drawn by hand (tests/golden/disc_r2.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "disc_r2.txt")
    rows = [ln.strip() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    ref = np.array([[1 if ch == "#" else 0 for ch in row] for row in rows], dtype=np.uint8)
    m = lbm.raster(7, 7, np.array([W.circle(3, 3, 2)]), False, False)
    assert np.array_equal(m, ref)


def test_raster_periodic_wrap_and_clip():
    """A disc centred on column 0 wraps to the last columns when x is periodic and
    is clipped when it is not; same count either way inside the domain."""
    sh = np.array([W.circle(0, 10, 3)])
    mw = lbm.raster(20, 20, sh, True, False)
    mc = lbm.raster(20, 20, sh, False, False)
    assert int(mw.sum()) == 29
    assert int(mc.sum()) == 29 - int(mw[:, 17:].sum())
    assert np.array_equal(mw[:, :4], mc[:, :4])
    assert mw[10, 17] == 1 and mw[10, 16] == 0


def test_raster_quadratic_form_matches_circle():
    """Ellipse path with a = b = 8 (2^24 / 64 exact) equals the integer disc of r = 8;
    an axis-aligned ellipse a=8, b=4 has the hand-countable extent."""
    e = W.ellipse(20, 20, 8.0, 8.0, 0.0)
    m1 = lbm.raster(40, 40, np.array([e]), False, False)
    m2 = lbm.raster(40, 40, np.array([W.circle(20, 20, 8)]), False, False)
    assert np.array_equal(m1, m2)
    e2 = W.ellipse(20, 20, 8.0, 4.0, 0.0)
    m3 = lbm.raster(40, 40, np.array([e2]), False, False)
    assert m3[20, 12] == 1 and m3[20, 11] == 0 and m3[16, 20] == 1 and m3[15, 20] == 0
    # rotation by pi/2 swaps the axes
    e3 = W.ellipse(20, 20, 8.0, 4.0, math.pi / 2)
    m4 = lbm.raster(40, 40, np.array([e3]), False, False)
    assert np.array_equal(m4, m3.T)


# ---------------------------------------------------------------- physics

def poiseuille_exact(N, tau, g):
    """Steady Poiseuille profile of D2Q9 BGK + Guo forcing with halfway bounce-back
    walls at y = -1/2 and y = N - 1/2: u_j = g/(2 nu) (j+1/2)(N-1/2-j) + g(48 nu^2 - 1)/(8 nu),
    nu = (tau - 1/2)/3 (the discrete scheme's exact solution; its slip term vanishes
    at (tau - 1/2)^2 = 3/16, He, Zou, Luo & Dembo 1997)."""
    nu = (tau - 0.5) / 3.0
    j = np.arange(N)
    return g / (2 * nu) * (j + 0.5) * (N - 0.5 - j) + g * (48 * nu * nu - 1) / (8 * nu)


@pytest.mark.parametrize("tau", [0.6, 0.8, 0.5 + math.sqrt(3) / 4, 1.2])
def test_poiseuille_exact_discrete(tau):
    N, g = 16, 1e-6
    lat = W.Lattice(nx=2, ny=N, tau=tau, gx=g, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL)
    mask = np.zeros((N, 2), np.uint8)
    ue = poiseuille_exact(N, tau, g)
    s = lbm.Sim(lat, mask).init(ux=np.repeat(ue[:, None], 2, 1))
    nu = (tau - 0.5) / 3
    steps = int(40.0 * N * N / (math.pi ** 2 * nu)) + 2000
    s.run(steps)
    rho, ux, uy = s.macros()
    assert np.max(np.abs(ux[:, 0] - ue)) / ue.max() < 1e-9
    assert np.max(np.abs(uy)) < 1e-10 * ue.max()
    assert np.max(np.abs(rho - rho.mean())) < 1e-12


@pytest.mark.parametrize("tau", [0.56, 0.8, 1.3])
def test_shear_wave_decay_rate_is_linear_operator_eigenvalue(tau):
    """A small shear wave u_x = U sin(k y) decays, after the non-hydrodynamic modes
    have died out, by the shear eigenvalue of the linearised one-step operator
    diag(exp(-i k.c_q)) [I - (I - E)/tau], E_qp = w_q (1 + 3 c_q.c_p) (Lallemand &
    Luo 2000), computed here with numpy.linalg.eigvals."""
    ny, U = 32, 1e-6
    k = 2 * math.pi / ny
    lat = W.periodic_box(2, ny, tau)
    y = np.arange(ny)
    ux0 = np.repeat((U * np.sin(k * y))[:, None], 2, 1)
    s = lbm.Sim(lat, np.zeros((ny, 2), np.uint8)).init(ux=ux0)
    s.run(400)

    def amp():
        return 2.0 / ny * np.sum(s.macros()[1][:, 0] * np.sin(k * y))
    a0 = amp(); s.run(1); a1 = amp()
    c = np.stack([CX, CY], 1).astype(float)
    E = WQ[:, None] * (1.0 + 3.0 * c @ c.T)
    L = np.diag(np.exp(-1j * k * CY)) @ (np.eye(9) - (np.eye(9) - E) / tau)
    ev = np.linalg.eigvals(L)
    nu = (tau - 0.5) / 3
    lam = ev[np.argmin(np.abs(ev - (1 - nu * k * k)))]
    assert abs(lam.imag) < 1e-12
    assert abs(a1 / a0 - lam.real) < 1e-9


def test_taylor_green_second_order():
    """Taylor-Green vortex (exact Navier-Stokes solution): the velocity error at a
    fixed diffusive time falls by ~4 per doubling of N (second order)."""
    errs = []
    tau = 0.8
    nu = (tau - 0.5) / 3
    for N in (16, 32, 64):
        k = 2 * math.pi / N
        U = 0.64 / N
        y, x = np.mgrid[0:N, 0:N].astype(float)
        ux = -U * np.cos(k * x) * np.sin(k * y)
        uy = U * np.sin(k * x) * np.cos(k * y)
        rho = 1.0 - 3.0 * U * U / 4.0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
        steps = int(round(0.5 / (nu * k * k)))
        s = lbm.Sim(W.periodic_box(N, N, tau), np.zeros((N, N), np.uint8)).init(rho, ux, uy)
        s.run(steps)
        _, u1, v1 = s.macros()
        d = math.exp(-2 * nu * k * k * steps)
        e = math.sqrt(np.sum((u1 - ux * d) ** 2 + (v1 - uy * d) ** 2) / np.sum((ux * d) ** 2 + (uy * d) ** 2))
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.3 < r2 < 4.8, errs


def test_conservation_periodic_with_obstacles_and_force():
    """Periodic box: mass is conserved with obstacles; without obstacles the
    momentum sum(c f) grows by exactly (total mass) * g per step (Guo forcing)."""
    nx, ny = 24, 20
    rho0, ux0, uy0 = W.random_macro_fields(3, nx, ny)
    g = (2e-5, -1e-5)
    lat = W.periodic_box(nx, ny, 0.7, gx=g[0], gy=g[1], shapes=[W.circle(8, 9, 3), W.circle(18, 2, 2)])
    s = lbm.Sim(lat).init(rho0, ux0, uy0)
    m0 = s.f[:, s.mask == 0].sum()
    s.run(100)
    assert abs(s.f[:, s.mask == 0].sum() - m0) < 1e-12 * m0

    lat2 = W.periodic_box(nx, ny, 0.7, gx=g[0], gy=g[1])
    s2 = lbm.Sim(lat2).init(rho0, ux0, uy0)
    M = s2.f.sum()
    j0 = np.array([(CX[:, None, None] * s2.f).sum(), (CY[:, None, None] * s2.f).sum()])
    s2.run(50)
    j1 = np.array([(CX[:, None, None] * s2.f).sum(), (CY[:, None, None] * s2.f).sum()])
    assert np.allclose(j1 - j0, 50 * M * np.array(g), rtol=1e-10, atol=1e-14)


def test_uniform_flow_is_fixed_point():
    nx, ny = 10, 12
    lat = W.periodic_box(nx, ny, 0.9)
    s = lbm.Sim(lat, np.zeros((ny, nx), np.uint8)).init(ux=np.full((ny, nx), 0.07), uy=np.full((ny, nx), -0.03))
    f0 = s.f.copy()
    s.run(50)
    assert np.max(np.abs(s.f - f0)) < 1e-15


def test_zouhe_prescriptions_and_plug_flow_fixed_point():
    """Zou-He closures reproduce the prescribed inlet velocity and outlet density
    at the boundary nodes, and the uniform plug flow (1, (u_in, 0)) is an exact
    fixed point of a Zou-He channel periodic in y."""
    nx, ny, u_in = 16, 12, 0.05
    lat = W.Lattice(nx=nx, ny=ny, tau=0.7, bc_x=W.BC_ZOUHE, bc_y=W.BC_PERIODIC, u_in=u_in, rho_out=1.0)
    mask = np.zeros((ny, nx), np.uint8)
    rho0, ux0, uy0 = W.random_macro_fields(5, nx, ny)
    s = lbm.Sim(lat, mask).init(rho0, ux0 + u_in, uy0)
    s.run(7)
    rho, ux, uy = s.macros()
    assert np.max(np.abs(ux[:, 0] - u_in)) < 1e-15 and np.max(np.abs(uy[:, 0])) < 1e-15
    assert np.max(np.abs(rho[:, -1] - 1.0)) < 1e-15 and np.max(np.abs(uy[:, -1])) < 1e-15
    s2 = lbm.Sim(lat, mask).init(ux=np.full((ny, nx), u_in))
    f0 = s2.f.copy()
    s2.run(40)
    assert np.max(np.abs(s2.f - f0)) < 1e-15


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC, W.BC_WALL), (W.BC_PERIODIC, W.BC_PERIODIC), (W.BC_WALL, W.BC_WALL)])
def test_streaming_is_a_permutation_of_fluid_slots(bc):
    """Streaming with halfway bounce-back moves every fluid population to exactly one
    fluid slot (built as an explicit 0/1 matrix from unit vectors on 8x8)."""
    nx = ny = 8
    lat = W.Lattice(nx=nx, ny=ny, tau=1.0, bc_x=bc[0], bc_y=bc[1],
                    shapes=[W.circle(3, 4, 1)], wrap_x=bc[0] == 0, wrap_y=bc[1] == 0)
    mask = lbm.raster(nx, ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
    fluid = np.repeat((mask == 0)[None], 9, 0).ravel()
    idx = np.flatnonzero(fluid)
    M = np.zeros((idx.size, idx.size))
    for col, k in enumerate(idx):
        e = np.zeros(9 * nx * ny); e[k] = 1.0
        out = lbm.stream(lat, mask, e.reshape(9, ny, nx)).ravel()
        M[:, col] = out[idx]
    assert set(np.unique(M)) <= {0.0, 1.0}
    assert np.all(M.sum(0) == 1) and np.all(M.sum(1) == 1)


def test_sums_are_correctly_rounded():
    """Fluid-node FP64 sums agree with math.fsum (correctly rounded)."""
    rng = np.random.default_rng(0)
    nx, ny = 33, 17
    mask = (rng.random((ny, nx)) < 0.2).astype(np.uint8)
    rho = 1.0 + 1e-3 * rng.standard_normal((ny, nx))
    rp = rho + 1e-7 * rng.standard_normal((ny, nx))
    ux = 1e-2 * rng.standard_normal((ny, nx)); uy = 1e-2 * rng.standard_normal((ny, nx))
    r, m, jx, jy = lbm.sums(mask, rho, rp, ux, uy)
    fl = mask == 0
    mm = math.fsum(rho[fl])
    assert abs(m - mm) <= 2e-16 * mm
    assert abs(r - math.fsum(np.abs(rho - rp)[fl]) / mm) <= 1e-15 * r
    assert abs(jx - math.fsum((rho * ux)[fl])) <= 1e-15 * math.fsum(np.abs(rho * ux)[fl])


# ----------------------------------------------------------------- adjoint

def test_adjoint_matches_central_finite_differences():
    """Gradient of L = MSE(macros after n steps, target) w.r.t. the initial fields,
    by the step adjoint, equals FP64 central finite differences (h = 1e-6) along
    random directions on a 32x32 lattice with obstacles, walls and a body force."""
    nx = ny = 32
    lat = W.Lattice(nx=nx, ny=ny, tau=0.75, gx=3e-6, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                    shapes=[W.circle(10, 12, 4), W.circle(24, 25, 3)], wrap_x=True, wrap_y=False)
    mask = lbm.raster(nx, ny, lat.shapes_array(), True, False)
    rho0, ux0, uy0 = W.random_macro_fields(11, nx, ny)
    tgt = W.random_macro_fields(12, nx, ny)
    n = 30
    g = lbm.rollout_grad(lat, mask, rho0, ux0, uy0, n, tgt)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(3):
        d = [rng.standard_normal((ny, nx)) * (mask == 0) for _ in range(3)]
        lp = lbm.rollout_loss(lat, mask, rho0 + h * d[0], ux0 + h * d[1], uy0 + h * d[2], n, tgt)
        lm = lbm.rollout_loss(lat, mask, rho0 - h * d[0], ux0 - h * d[1], uy0 - h * d[2], n, tgt)
        fd = (lp - lm) / (2 * h)
        an = sum(float(np.sum(a * b)) for a, b in zip(g, d))
        assert abs(fd - an) <= 1e-7 * abs(an), (fd, an)


def test_adjoint_transpose_identity():
    """<J v, w> = <v, J^T w> for one step, with J v from central differences of the
    oracle's forward step (exact for the linear streaming part, O(h^2) for the rational collision map)."""
    nx, ny = 12, 10
    lat = W.Lattice(nx=nx, ny=ny, tau=0.9, gx=1e-5, gy=2e-6, bc_x=W.BC_WALL, bc_y=W.BC_PERIODIC,
                    shapes=[W.circle(6, 5, 2)], wrap_x=False, wrap_y=True)
    mask = lbm.raster(nx, ny, lat.shapes_array(), False, True)
    rng = np.random.default_rng(2)
    s = lbm.Sim(lat, mask).init(*W.random_macro_fields(4, nx, ny))
    f = s.f.copy()
    fl = np.repeat((mask == 0)[None], 9, 0)
    v = rng.standard_normal(f.shape) * fl
    w = rng.standard_normal(f.shape) * fl

    def step(ff):
        return lbm.stream(lat, mask, lbm.collide(lat, mask, ff))
    h = 1e-6
    Jv = (step(f + h * v) - step(f - h * v)) / (2 * h)
    JTw = lbm.adjoint_step(lat, mask, f, w)
    a, b = float(np.sum(Jv * w * fl)), float(np.sum(v * JTw))
    assert abs(a - b) <= 1e-8 * abs(b)


def zouhe_lattice(nx=24, ny=12):
    return W.Lattice(nx=nx, ny=ny, tau=0.7, bc_x=W.BC_ZOUHE, bc_y=W.BC_PERIODIC, u_in=0.03,
                     rho_out=1.01, shapes=[W.circle(nx // 2, ny // 2, 3)], wrap_x=False, wrap_y=True)


def test_adjoint_with_zouhe_columns_matches_central_finite_differences():
    """Through the Zou-He inlet and outlet closures (and the closures applied to the
    initial equilibrium): adjoint gradient of the rollout loss vs FP64 central
    differences along random directions, 24x12 lattice with an obstacle, 25 steps."""
    lat = zouhe_lattice()
    mask = lbm.raster(lat.nx, lat.ny, lat.shapes_array(), False, True)
    rho0, ux0, uy0 = W.random_macro_fields(21, lat.nx, lat.ny, amp_rho=0.02, amp_u=0.03)
    tgt = W.random_macro_fields(22, lat.nx, lat.ny)
    n = 25
    g = lbm.rollout_grad(lat, mask, rho0, ux0, uy0, n, tgt)
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(3):
        d = [rng.standard_normal((lat.ny, lat.nx)) * (mask == 0) for _ in range(3)]
        lp = lbm.rollout_loss(lat, mask, rho0 + h * d[0], ux0 + h * d[1], uy0 + h * d[2], n, tgt)
        lm = lbm.rollout_loss(lat, mask, rho0 - h * d[0], ux0 - h * d[1], uy0 - h * d[2], n, tgt)
        fd = (lp - lm) / (2 * h)
        an = sum(float(np.sum(a * b)) for a, b in zip(g, d))
        assert abs(fd - an) <= 1e-7 * abs(an), (fd, an)


def test_zouhe_closure_adjoint_transpose_identity():
    """<J v, w> = <v, J^T w> for one step whose streaming includes the Zou-He closures,
    and for the closures alone (affine, so central differences are exact up to rounding)."""
    lat = zouhe_lattice(14, 10)
    mask = lbm.raster(lat.nx, lat.ny, lat.shapes_array(), False, True)
    rng = np.random.default_rng(6)
    s = lbm.Sim(lat, mask).init(*W.random_macro_fields(7, lat.nx, lat.ny, amp_u=0.03))
    f = s.f.copy()
    fl = np.repeat((mask == 0)[None], 9, 0)
    v = rng.standard_normal(f.shape) * fl
    w = rng.standard_normal(f.shape) * fl

    def step(ff):
        return lbm.stream(lat, mask, lbm.collide(lat, mask, ff))
    h = 1e-6
    Jv = (step(f + h * v) - step(f - h * v)) / (2 * h)
    JTw = lbm.adjoint_step(lat, mask, f, w)
    a, b = float(np.sum(Jv * w * fl)), float(np.sum(v * JTw))
    assert abs(a - b) <= 1e-8 * abs(b)
    # the closures alone: Z applied to post-streaming values is stream() of the
    # collided state, so perturb the collided state and compare with bc_vjp
    fs = lbm.collide(lat, mask, f)
    Zv = (lbm.stream(lat, mask, fs + h * v) - lbm.stream(lat, mask, fs - h * v)) / (2 * h)
    wz = lbm.bc_vjp(lat, mask, w)
    periodic = W.Lattice(nx=lat.nx, ny=lat.ny, tau=lat.tau, bc_x=W.BC_WALL, bc_y=W.BC_PERIODIC,
                         shapes=lat.shapes, wrap_x=False, wrap_y=True)
    # stream with walls in x and Zou-He columns differ only by the closures, whose
    # unknown slots the wall bounce-back fills: <Z P v, w> = <P v, Z^T w>
    Pv = (lbm.stream(periodic, mask, fs + h * v) - lbm.stream(periodic, mask, fs - h * v)) / (2 * h)
    a2, b2 = float(np.sum(Zv * w * fl)), float(np.sum(Pv * wz * fl))
    assert abs(a2 - b2) <= 1e-8 * abs(b2)


# ------------------------------------------------- non-equilibrium initialisation

def test_neq_init_moments_are_the_viscous_stress():
    """f(0) - f_eq has zero mass and momentum at every node, and its second moment is
    the Chapman-Enskog viscous stress -rho c_s^2 tau (grad u + grad u^T), with the
    gradient taken here by numpy central differences on a periodic box."""
    nx, ny, tau = 20, 16, 0.9
    lat = W.Lattice(nx=nx, ny=ny, tau=tau, bc_x=W.BC_PERIODIC, bc_y=W.BC_PERIODIC, shapes=[],
                    wrap_x=True, wrap_y=True)
    mask = np.zeros((ny, nx), np.uint8)
    rho, ux, uy = W.random_macro_fields(31, nx, ny, amp_u=0.05)
    f_eq = lbm.Sim(lat, mask).init(rho, ux, uy).f
    f = lbm.Sim(lat, mask).init(rho, ux, uy, neq=True).f
    d = f - f_eq
    cx, cy, _, _ = lbm.lattice()
    assert np.abs(d.sum(axis=0)).max() < 1e-15
    assert np.abs(np.tensordot(cx, d, 1)).max() < 1e-15 and np.abs(np.tensordot(cy, d, 1)).max() < 1e-15
    ddx = lambda a: 0.5 * (np.roll(a, -1, 1) - np.roll(a, 1, 1))
    ddy = lambda a: 0.5 * (np.roll(a, -1, 0) - np.roll(a, 1, 0))
    k = -rho * tau / 3.0
    pxx = np.tensordot(cx * cx, d, 1)
    pxy = np.tensordot(cx * cy, d, 1)
    pyy = np.tensordot(cy * cy, d, 1)
    assert np.allclose(pxx, k * 2 * ddx(ux), rtol=0, atol=1e-15)
    assert np.allclose(pyy, k * 2 * ddy(uy), rtol=0, atol=1e-15)
    assert np.allclose(pxy, k * (ddy(ux) + ddx(uy)), rtol=0, atol=1e-15)


def test_neq_init_removes_the_shear_wave_start_transient():
    """A decaying shear wave u_x = A sin(k y) started from f_eq alone carries a start
    transient (the missing viscous stress) that leaves a lasting amplitude error; with
    the non-equilibrium part the lattice follows A exp(-nu k^2 t) sin(k y) far closer."""
    nx, ny, tau, A = 8, 64, 0.8, 1e-3
    nu, kk = (tau - 0.5) / 3.0, 2 * np.pi / ny
    lat = W.Lattice(nx=nx, ny=ny, tau=tau, bc_x=W.BC_PERIODIC, bc_y=W.BC_PERIODIC, shapes=[],
                    wrap_x=True, wrap_y=True)
    mask = np.zeros((ny, nx), np.uint8)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    exact = lambda t: A * np.exp(-nu * kk * kk * t) * np.sin(kk * y)
    err = {}
    for neq in (False, True):
        s = lbm.Sim(lat, mask).init(np.ones((ny, nx)), exact(0), np.zeros((ny, nx)), neq=neq).run(5)
        err[neq] = np.abs(s.macros()[1] - exact(5)).max() / A
    assert err[False] > 3e-4 and err[True] < 1e-5, err


# ------------------------------------------------------------ TRT collision

@pytest.mark.parametrize("tau", [0.56, 0.8, 1.3])
def test_trt_magic_three_sixteenths_gives_exact_parabolic_poiseuille(tau):
    """With the magic parameter 3/16 the TRT scheme with halfway bounce-back carries
    the parabolic Poiseuille profile u(y) = g/(2 nu) (y + 1/2)(N - 1/2 - y), walls
    exactly halfway, at every tau (Ginzburg & d'Humieres); BGK does so only at one tau."""
    N, g = 16, 1e-6
    lat = W.Lattice(nx=2, ny=N, tau=tau, gx=g, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL, trt_lambda=3.0 / 16)
    mask = np.zeros((N, 2), np.uint8)
    nu = (tau - 0.5) / 3
    y = np.arange(N)
    ue = g / (2 * nu) * (y + 0.5) * (N - 0.5 - y)
    s = lbm.Sim(lat, mask).init(ux=np.repeat(ue[:, None], 2, 1))
    s.run(int(40.0 * N * N / (math.pi ** 2 * nu)) + 2000)
    rho, ux, uy = s.macros()
    assert np.max(np.abs(ux[:, 0] - ue)) / ue.max() < 1e-9
    assert np.max(np.abs(uy)) < 1e-10 * ue.max()


def test_trt_with_equal_relaxation_times_is_bgk():
    """lambda = (tau - 1/2)^2 makes tau- = tau+: the TRT step is the BGK step."""
    lat = W.Lattice(nx=30, ny=22, tau=0.83, gx=2e-5, gy=-1e-5, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                    shapes=[W.circle(12, 10, 4)], wrap_x=True, wrap_y=False)
    mask = lbm.raster(lat.nx, lat.ny, lat.shapes_array(), True, False)
    f0 = lbm.Sim(lat, mask).init(*W.random_macro_fields(41, lat.nx, lat.ny, amp_u=0.05)).f
    trt = W.Lattice(**{**lat.__dict__, "trt_lambda": (lat.tau - 0.5) ** 2})
    a = lbm.collide(lat, mask, f0)
    b = lbm.collide(trt, mask, f0)
    assert np.max(np.abs(a - b)) < 1e-15


@pytest.mark.parametrize("tau,lam", [(0.52, 0.25), (0.8, 3.0 / 16), (1.2, 0.1)])
def test_trt_shear_wave_decay_is_linear_operator_eigenvalue(tau, lam):
    """A small shear wave decays by the shear eigenvalue of the linearised TRT step
    diag(exp(-i k.c_q)) [I - (P+/tau+ + P-/tau-)(I - E)], with P+- the projectors onto
    the parts even and odd under c -> -c (numpy.linalg.eigvals)."""
    ny, U = 32, 1e-6
    k = 2 * math.pi / ny
    lat = W.Lattice(nx=2, ny=ny, tau=tau, trt_lambda=lam)
    y = np.arange(ny)
    s = lbm.Sim(lat, np.zeros((ny, 2), np.uint8)).init(ux=np.repeat((U * np.sin(k * y))[:, None], 2, 1))
    s.run(400)

    def amp():
        return 2.0 / ny * np.sum(s.macros()[1][:, 0] * np.sin(k * y))
    a0 = amp(); s.run(1); a1 = amp()
    c = np.stack([CX, CY], 1).astype(float)
    opp = np.array([np.where((c == -c[q]).all(1))[0][0] for q in range(9)])
    Pp = 0.5 * (np.eye(9) + np.eye(9)[opp])
    Pm = 0.5 * (np.eye(9) - np.eye(9)[opp])
    tau_m = 0.5 + lam / (tau - 0.5)
    E = WQ[:, None] * (1.0 + 3.0 * c @ c.T)
    L = np.diag(np.exp(-1j * k * CY)) @ (np.eye(9) - (Pp / tau + Pm / tau_m) @ (np.eye(9) - E))
    ev = np.linalg.eigvals(L)
    nu = (tau - 0.5) / 3
    mu = ev[np.argmin(np.abs(ev - (1 - nu * k * k)))]
    assert abs(mu.imag) < 1e-12
    assert abs(a1 / a0 - mu.real) < 1e-9


# ------------------------------------------------------------- TRT adjoint

def test_trt_adjoint_transpose_identity():
    """<J v, w> = <v, J^T w> for one TRT step (lambda = 1/4, tau = 0.9, so tau- = 0.875
    differs from tau) with a body force, walls and an obstacle: J v from central
    differences of the oracle's forward TRT step."""
    import dataclasses
    nx, ny = 12, 10
    lat = W.Lattice(nx=nx, ny=ny, tau=0.9, gx=1e-5, gy=2e-6, bc_x=W.BC_WALL, bc_y=W.BC_PERIODIC,
                    shapes=[W.circle(6, 5, 2)], wrap_x=False, wrap_y=True)
    lat = dataclasses.replace(lat, trt_lambda=0.25)
    mask = lbm.raster(nx, ny, lat.shapes_array(), False, True)
    rng = np.random.default_rng(7)
    s = lbm.Sim(lat, mask).init(*W.random_macro_fields(4, nx, ny))
    f = s.f.copy()
    fl = np.repeat((mask == 0)[None], 9, 0)
    v = rng.standard_normal(f.shape) * fl
    w = rng.standard_normal(f.shape) * fl

    def step(ff):
        return lbm.stream(lat, mask, lbm.collide(lat, mask, ff))
    h = 1e-6
    Jv = (step(f + h * v) - step(f - h * v)) / (2 * h)
    JTw = lbm.adjoint_step(lat, mask, f, w)
    a, b = float(np.sum(Jv * w * fl)), float(np.sum(v * JTw))
    assert abs(a - b) <= 1e-8 * abs(b)
    # the BGK adjoint of the same state is a different map (the pin would catch a
    # TRT adjoint that ignored lambda)
    bgk = lbm.adjoint_step(dataclasses.replace(lat, trt_lambda=0.0), mask, f, w)
    assert abs(float(np.sum(v * bgk)) - b) > 1e-6 * abs(b)


@pytest.mark.parametrize("lam", [0.25, 3.0 / 16])
def test_trt_adjoint_rollout_matches_central_finite_differences(lam):
    """TRT rollout gradient through Zou-He columns (24x12 lattice with an obstacle, 25
    steps) and on a forced walled channel (32x16, 20 steps) vs FP64 central
    differences along random directions."""
    import dataclasses
    lats = [zouhe_lattice(),
            W.Lattice(nx=32, ny=16, tau=0.75, gx=3e-6, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                      shapes=[W.circle(10, 8, 3)], wrap_x=True, wrap_y=False)]
    for lat, n, seed in zip(lats, (25, 20), (31, 41)):
        lat = dataclasses.replace(lat, trt_lambda=lam)
        mask = lbm.raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
        rho0, ux0, uy0 = W.random_macro_fields(seed, lat.nx, lat.ny, amp_rho=0.02, amp_u=0.03)
        tgt = W.random_macro_fields(seed + 1, lat.nx, lat.ny)
        g = lbm.rollout_grad(lat, mask, rho0, ux0, uy0, n, tgt)
        rng = np.random.default_rng(seed)
        h = 1e-6
        for _ in range(2):
            d = [rng.standard_normal((lat.ny, lat.nx)) * (mask == 0) for _ in range(3)]
            lp = lbm.rollout_loss(lat, mask, rho0 + h * d[0], ux0 + h * d[1], uy0 + h * d[2], n, tgt)
            lm = lbm.rollout_loss(lat, mask, rho0 - h * d[0], ux0 - h * d[1], uy0 - h * d[2], n, tgt)
            fd = (lp - lm) / (2 * h)
            an = sum(float(np.sum(a * b)) for a, b in zip(g, d))
            assert abs(fd - an) <= 1e-7 * abs(an), (lat.name, fd, an)


def test_trt_adjoint_with_equal_times_is_the_bgk_adjoint():
    """lambda = (tau - 1/2)^2 gives tau- = tau: the TRT adjoint is then the BGK adjoint
    (to rounding)."""
    import dataclasses
    nx, ny = 16, 12
    lat = W.Lattice(nx=nx, ny=ny, tau=0.8, gx=2e-6, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                    shapes=[W.circle(8, 6, 2)], wrap_x=True, wrap_y=False)
    mask = lbm.raster(nx, ny, lat.shapes_array(), True, False)
    s = lbm.Sim(lat, mask).init(*W.random_macro_fields(9, nx, ny))
    w = np.random.default_rng(3).standard_normal(s.f.shape) * np.repeat((mask == 0)[None], 9, 0)
    a = lbm.adjoint_step(lat, mask, s.f, w)
    b = lbm.adjoint_step(dataclasses.replace(lat, trt_lambda=0.3 ** 2), mask, s.f, w)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))


# ------------------------------------------------ mass-conserving re-initialisation

def test_mass_conserving_init_shifts_density_uniformly():
    """init(..., mass=M) on walls and a periodic axis: the state's fluid mass is M
    (f_eq sums to rho), the density differs from the handed-over one by a single
    constant on every fluid node, the velocity is unchanged, and the lattice keeps M
    over 50 forced steps (mass conservation of the BGK step with the Guo source)."""
    nx, ny = 24, 14
    lat = W.Lattice(nx=nx, ny=ny, tau=0.8, gx=2e-6, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                    shapes=[W.circle(8, 7, 3)], wrap_x=True, wrap_y=False)
    mask = lbm.raster(nx, ny, lat.shapes_array(), True, False)
    fl = mask == 0
    rho, ux, uy = W.random_macro_fields(5, nx, ny, amp_rho=0.01, amp_u=0.02)
    target = math.fsum(rho[fl].tolist()) * (1.0 + 3e-3)
    s = lbm.Sim(lat, mask).init(rho, ux, uy, mass=target)
    assert abs(s.mass() - target) <= 1e-13 * target
    r, u, v = s.macros()
    d = (r - rho)[fl]
    assert abs(d.mean() - 3e-3 * math.fsum(rho[fl].tolist()) / fl.sum()) <= 1e-12
    assert np.max(np.abs(d - d.mean())) <= 1e-13
    # the velocity is unchanged (the moments add half the force, g/2, to the handed-over u)
    assert np.max(np.abs(u - ux - 0.5 * lat.gx)[fl]) <= 1e-13 and np.max(np.abs(v - uy)[fl]) <= 1e-13
    plain = lbm.Sim(lat, mask).init(rho, ux, uy)
    assert abs(plain.mass() - math.fsum(rho[fl].tolist())) <= 1e-13 * target
    s.run(50)
    assert abs(s.mass() - target) <= 1e-12 * target
