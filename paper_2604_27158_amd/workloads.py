"""Seeded synthetic inputs for the hybrid FNO-LBM hot path.

This module produces *inputs only*: obstacle descriptors, lattice sizes, relaxation
times and random fields.  It contains none of the method's arithmetic (no
rasterisation, no equilibrium, no collision), so both the GPU path and the CPU
oracle can consume what it produces without sharing any computation.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), one stream per seed; floats take the
top 53 bits of a draw.

Obstacle descriptor (int64 x 7): ``(cx, cy, A, B, C, F, R)``.  A lattice cell
``(i, j)`` belongs to the obstacle iff, with ``dx, dy`` the (optionally periodic)
offsets of the cell from ``(cx, cy)`` and ``|dx|, |dy| <= R``::

    A*dx*dx + B*dx*dy + C*dy*dy <= F

A circle of integer radius r is ``(cx, cy, 1, 0, 1, r*r, r)``; an ellipse is its
quadratic form scaled by 2**24 and rounded to integers here, so the obstacle test
itself is exact integer arithmetic on both sides.  Obstacles model the porous
media of the paper's steady experiment (Sec. 3.1.1, Eq. 8: random circles, porosity
phi = fluid area / total area) and the bluff bodies of the batched unsteady flows.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

MASK64 = (1 << 64) - 1

# Boundary-condition codes shared by the C ABI (include/lbmfno.h) and the oracle.
BC_PERIODIC = 0
BC_WALL = 1      # halfway bounce-back wall half a cell outside the first/last row
BC_ZOUHE = 2     # x only: Zou-He velocity inlet at x=0, pressure outlet at x=nx-1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + self.next_u64() % (hi - lo + 1)

    def normal_array(self, n: int) -> np.ndarray:
        """n standard normals by Box-Muller on the stream's uniforms."""
        m = (n + 1) // 2
        u1 = np.array([self.uniform() for _ in range(m)])
        u2 = np.array([self.uniform() for _ in range(m)])
        u1 = np.maximum(u1, 1e-300)
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
        return z[:n]


def circle(cx: int, cy: int, r: int) -> Tuple[int, ...]:
    return (int(cx), int(cy), 1, 0, 1, int(r) * int(r), int(r))


ELLIPSE_SCALE = 1 << 24


def ellipse(cx: int, cy: int, a: float, b: float, theta: float) -> Tuple[int, ...]:
    """Integer quadratic-form descriptor of an ellipse with semi-axes a, b (cells)
    rotated by theta, centred on cell (cx, cy)."""
    c, s = math.cos(theta), math.sin(theta)
    ia2, ib2 = 1.0 / (a * a), 1.0 / (b * b)
    A = round(ELLIPSE_SCALE * (c * c * ia2 + s * s * ib2))
    B = round(ELLIPSE_SCALE * 2.0 * s * c * (ia2 - ib2))
    C = round(ELLIPSE_SCALE * (s * s * ia2 + c * c * ib2))
    R = int(math.ceil(max(a, b))) + 1
    return (int(cx), int(cy), int(A), int(B), int(C), ELLIPSE_SCALE, R)


@dataclass
class Lattice:
    """One lattice workload: size, physics parameters and obstacle list."""
    nx: int
    ny: int
    tau: float
    gx: float = 0.0
    gy: float = 0.0
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    u_in: float = 0.0
    rho_out: float = 1.0
    shapes: List[Tuple[int, ...]] = field(default_factory=list)
    wrap_x: bool = True     # obstacles wrap around periodic x
    wrap_y: bool = True
    seed: int = 0
    name: str = ""
    trt_lambda: float = 0.0   # > 0: two-relaxation-time collision with this magic parameter

    def shapes_array(self) -> np.ndarray:
        if not self.shapes:
            return np.zeros((0, 7), dtype=np.int64)
        return np.ascontiguousarray(np.array(self.shapes, dtype=np.int64).reshape(-1, 7))


def channel_walls_circles(seed: int, nx: int = 128, ny: int = 64, n_circles: int = 10,
                          rmin: int = 4, rmax: int = 8, tau: float = 0.8,
                          g: float = 1e-6) -> Lattice:
    """Body-force-driven channel: periodic in x, bounce-back walls in y, overlapping
    random circles of radius rmin..rmax clipped at the walls."""
    rng = SplitMix64(seed)
    shapes = []
    for _ in range(n_circles):
        r = rng.randint(rmin, rmax)
        cx = rng.randint(r, nx - 1 - r)
        cy = rng.randint(0, ny - 1)
        shapes.append(circle(cx, cy, r))
    return Lattice(nx=nx, ny=ny, tau=tau, gx=g, gy=0.0, bc_x=BC_PERIODIC, bc_y=BC_WALL,
                   shapes=shapes, wrap_x=True, wrap_y=False, seed=seed,
                   name=f"channel{nx}x{ny}-circles{n_circles}-s{seed}")


def porous_circles(seed: int, nx: int = 1024, ny: int = 512, rmin: int = 8, rmax: int = 20,
                   phi_lo: float = 0.6, phi_hi: float = 0.8, gap: int = 2, keepout: int = 40,
                   tau: float = 0.6, u_in: float = 0.02, rho_out: float = 1.0,
                   max_attempts: int = 60000) -> Lattice:
    """Porous medium: non-overlapping circles (centre distance >= r1 + r2 + gap,
    periodic in y) added at random until the estimated porosity reaches a target
    drawn from U(phi_lo, phi_hi); `keepout` columns at inlet and outlet stay free.
    Zou-He velocity inlet / pressure outlet in x, periodic in y.  The inlet speed
    0.02 keeps the density rise needed to push the flow through 1024 columns of
    this medium near 10 %; at 0.05 it exceeds 40 % and the BGK run diverges."""
    rng = SplitMix64(seed)
    phi_target = rng.uniform(phi_lo, phi_hi)
    area = float(nx * ny)
    solid_est = 0.0
    cxs = np.zeros(0, dtype=np.int64)
    cys = np.zeros(0, dtype=np.int64)
    rs = np.zeros(0, dtype=np.int64)
    attempts = 0
    while 1.0 - solid_est / area > phi_target and attempts < max_attempts:
        attempts += 1
        r = rng.randint(rmin, rmax)
        cx = rng.randint(keepout + r, nx - 1 - keepout - r)
        cy = rng.randint(0, ny - 1)
        if rs.size:
            dx = cxs - cx
            dy = np.abs(cys - cy)
            dy = np.minimum(dy, ny - dy)
            need = rs + r + gap
            if np.any(dx * dx + dy * dy < need * need):
                continue
        cxs = np.append(cxs, cx)
        cys = np.append(cys, cy)
        rs = np.append(rs, r)
        solid_est += math.pi * r * r
    shapes = [circle(int(a), int(b), int(c)) for a, b, c in zip(cxs, cys, rs)]
    return Lattice(nx=nx, ny=ny, tau=tau, bc_x=BC_ZOUHE, bc_y=BC_PERIODIC, u_in=u_in,
                   rho_out=rho_out, shapes=shapes, wrap_x=False, wrap_y=True, seed=seed,
                   name=f"porous{nx}x{ny}-phi{phi_target:.3f}-s{seed}")


BATCH_SIZES = ((256, 128), (384, 192), (512, 256))


def ellipse_flow(seed: int, size=None, re_lo: float = 100.0, re_hi: float = 200.0,
                 u_in: float = 0.1, nmin: int = 1, nmax: int = 5, gap: int = 8,
                 max_attempts: int = 200, block_frac: float = 0.5, re_length: float = 0.25) -> Lattice:
    """Flow past 1-5 random ellipses: lattice size drawn from BATCH_SIZES unless given,
    semi-axes a ~ U(ny/16, ny/8), b = a*U(0.3, 1), angle U(0, pi); Reynolds number
    Re ~ U(re_lo, re_hi) on D = re_length*ny sets nu = u_in*D/Re and tau = 3*nu + 1/2.
    Zou-He inlet/outlet in x, periodic in y; ellipses stay clear of the first and
    last ny/8 + 2 columns, their bounding circles keep `gap` cells apart (periodic
    in y), and ellipses whose x-extents overlap block at most `block_frac` of the
    channel height, which keeps the jets between them below the lattice sound speed.
    The flows start from the plug flow (rho = 1, u = (u_in, 0)); see plug_flow()."""
    rng = SplitMix64(seed)
    if size is None:
        nx, ny = BATCH_SIZES[rng.randint(0, len(BATCH_SIZES) - 1)]
    else:
        nx, ny = size
    re = rng.uniform(re_lo, re_hi)
    nu = u_in * (re_length * ny) / re
    tau = 3.0 * nu + 0.5
    n = rng.randint(nmin, nmax)
    keep = ny // 8 + 2
    shapes, placed = [], []
    attempts = 0
    while len(shapes) < n and attempts < max_attempts:
        attempts += 1
        a = rng.uniform(ny / 16.0, ny / 8.0)
        b = a * rng.uniform(0.3, 1.0)
        th = rng.uniform(0.0, math.pi)
        R = int(math.ceil(a)) + 1
        cx = rng.randint(keep + R, nx - 1 - keep - R)
        cy = rng.randint(0, ny - 1)
        ok = True
        blocked = 2 * R
        for (px, py, pr) in placed:
            dy = abs(cy - py)
            dy = min(dy, ny - dy)
            if (cx - px) ** 2 + dy * dy < (R + pr + gap) ** 2:
                ok = False
                break
            if abs(cx - px) <= R + pr:
                blocked += 2 * pr
        if not ok or blocked > int(block_frac * ny):
            continue
        placed.append((cx, cy, R))
        shapes.append(ellipse(cx, cy, a, b, th))
    return Lattice(nx=nx, ny=ny, tau=tau, bc_x=BC_ZOUHE, bc_y=BC_PERIODIC, u_in=u_in,
                   rho_out=1.0, shapes=shapes, wrap_x=False, wrap_y=True, seed=seed,
                   name=f"ellipses{nx}x{ny}-n{len(shapes)}-Re{re:.0f}-s{seed}")


def batch_flow(seed: int, size=None) -> Lattice:
    """The batched-trajectory workload: flows past 1-5 ellipses at Re ~ U(100, 200),
    with the Reynolds number on the channel half-height (D = ny/2) and u_in = 0.08,
    tau in [0.58, 0.80].  On D = ny/4 (ellipse_flow's default) the 256 x 128 lattices
    resolve the Re > 150 wakes with a cell Reynolds number u/nu = 4 Re/ny of 5-6 and a
    fifth of the BGK runs lose stability within 20 000 steps; on ny/2 none do."""
    return ellipse_flow(seed, size=size, u_in=0.08, re_length=0.5)


def plug_flow(lat: "Lattice"):
    """Initial fields (rho, ux, uy) = (1, u_in, 0), float64 [ny][nx]."""
    shp = (lat.ny, lat.nx)
    return np.ones(shp), np.full(shp, float(lat.u_in)), np.zeros(shp)


def periodic_box(nx: int, ny: int, tau: float, gx: float = 0.0, gy: float = 0.0,
                 shapes=None, seed: int = 0) -> Lattice:
    return Lattice(nx=nx, ny=ny, tau=tau, gx=gx, gy=gy, bc_x=BC_PERIODIC, bc_y=BC_PERIODIC,
                   shapes=list(shapes or []), wrap_x=True, wrap_y=True, seed=seed,
                   name=f"box{nx}x{ny}")


# Double shear layer (the paper's unsteady case, Sec. 3.2.1, Eqs. 9-10): a periodic
# unit square at n x n, U = 1 m/s, nu = 0.001 m^2/s, outputs every 223 lattice steps
# over a 3 s horizon of 30 outputs.  Lattice units: dt = 3 s / (30 * 223),
# dx = 1/n, so u_lat = U dt / dx and nu_lat = nu dt / dx^2.
SHEAR_DT_OUT = 223
SHEAR_OUTPUTS = 30


def shear_units(n: int = 128):
    """(u_lat, tau) of the double shear layer at n x n."""
    dt = 3.0 / (SHEAR_OUTPUTS * SHEAR_DT_OUT)
    dx = 1.0 / n
    u_lat = 1.0 * dt / dx
    nu_lat = 0.001 * dt / (dx * dx)
    return u_lat, 0.5 + 3.0 * nu_lat


def double_shear_layer(seed: int, n: int = 128, re_lo: float = 8.0, re_hi: float = 50.0):
    """(Lattice, rho, ux, uy) of one double-shear-layer trajectory.  u = U tanh(A1 (y1 - y))
    for y >= 1/2 and U tanh(A2 (y - y2)) below, v = 0.1 U sin(2 pi (x + 1/4)), rho = 1,
    node (i, j) at (x, y) = (i/n, j/n).  Randomised: the layer centres y1 ~ U(0.7, 0.8),
    y2 ~ U(0.2, 0.3), and each layer's Reynolds number on its thickness 1/A,
    Re = U / (A nu) ~ U(8, 50), so A = U / (Re nu)."""
    rng = SplitMix64(seed)
    y1, y2 = rng.uniform(0.7, 0.8), rng.uniform(0.2, 0.3)
    re1, re2 = rng.uniform(re_lo, re_hi), rng.uniform(re_lo, re_hi)
    a1, a2 = 1.0 / (re1 * 0.001), 1.0 / (re2 * 0.001)
    u_lat, tau = shear_units(n)
    y, x = np.mgrid[0:n, 0:n].astype(np.float64) / n
    ux = np.where(y >= 0.5, np.tanh(a1 * (y1 - y)), np.tanh(a2 * (y - y2))) * u_lat
    uy = 0.1 * u_lat * np.sin(2.0 * np.pi * (x + 0.25))
    rho = np.ones((n, n))
    lat = periodic_box(n, n, tau, seed=seed)
    lat.name = f"shear{n}-Re{re1:.0f}-{re2:.0f}-s{seed}"
    return lat, rho, ux, uy


def random_macro_fields(seed: int, nx: int, ny: int, amp_rho: float = 1e-2,
                        amp_u: float = 2e-2, modes: int = 3):
    """Smooth random (rho, ux, uy) fields: rho = 1 + small band-limited perturbation,
    velocity a few low Fourier modes; float64 arrays of shape [ny][nx]."""
    rng = SplitMix64(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    out = []
    for amp in (amp_rho, amp_u, amp_u):
        fld = np.zeros((ny, nx))
        for _ in range(modes):
            kx = rng.randint(0, 3)
            ky = rng.randint(0, 3)
            ph = rng.uniform(0.0, 2 * math.pi)
            a = rng.uniform(-1.0, 1.0)
            fld += a * np.cos(2 * math.pi * (kx * x / nx + ky * y / ny) + ph)
        out.append(amp * fld / modes)
    out[0] = out[0] + 1.0
    return out[0], out[1], out[2]


def random_array(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """Standard-normal array (float64) times `scale`, from the seeded stream."""
    rng = np.random.Generator(np.random.Philox(key=seed & MASK64))
    return scale * rng.standard_normal(size=shape)


@dataclass
class FnoSpec:
    """Structure of an FNO (Sec. 2.2, Eq. 6): input channels, latent width, number of
    Fourier layers, kept modes per dimension (m1 two-sided along H, m2 one-sided along
    W), decoder depth and width, output channels, padding, coordinate channels and
    activations."""
    cin: int = 4
    width: int = 32
    layers: int = 4
    m1: int = 12
    m2: int = 12
    dec_layers: int = 1
    dec_size: int = 32
    cout: int = 3
    padding: int = 0
    coords: bool = True
    act: str = "gelu"        # inside the lift and the Fourier layers
    dec_act: str = "silu"    # inside the decoder


def fno_random_params(seed: int, layout, width: int) -> np.ndarray:
    """Packed float64 parameter vector with a fan-in scaled random initialisation.
    `layout` is a list of (name, shape) in packing order (names ending in ".b" are
    biases, names containing ".r_" are spectral weights)."""
    rng = np.random.Generator(np.random.Philox(key=(seed * 7919 + 17) & MASK64))
    parts = []
    for name, shp in layout:
        if name.endswith(".b"):
            parts.append(0.1 * rng.standard_normal(size=shp).ravel())
        elif ".r_" in name:
            scale = 1.0 / (width * width)
            parts.append(scale * rng.uniform(-1.0, 1.0, size=shp).ravel() * 4.0)
        else:
            fan_in = shp[1]
            parts.append(rng.standard_normal(size=shp).ravel() / math.sqrt(fan_in))
    return np.concatenate(parts)
