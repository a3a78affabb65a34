"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws numbers and evaluates initial-condition formulas. It
holds none of the method's arithmetic (no fluxes, limiters, ghost filling,
refinement criteria or time stepping). Every workload is an analytic initial
condition in the style of the paper's tests (Sec. 4), so no dataset is used.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw n of seed s is mix(s + (n + 1) * 0x9E3779B97F4A7C15).
Uniform doubles in [-1, 1) are (x >> 11) * 2^-53 * 2 - 1.

Fields are returned as conserved variables (rho, m_x, m_y[, m_z], E) with
E = p / (gamma - 1) + rho |v|^2 / 2, the equation of state of the Euler
system (Sec. 3.5); that is the definition of the problem input, not a step of
the scheme.
"""
from __future__ import annotations

import math
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Draws start .. start+n-1 of the SplitMix64 stream of `seed` (uint64)."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed) + ctr * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [-1, 1) from the SplitMix64 stream."""
    x = splitmix64(seed, n, start)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def uniform01(seed: int, n: int, start: int = 0) -> np.ndarray:
    x = splitmix64(seed, n, start)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def conserved_from_primitive(rho, vel, p, gamma, xp=np):
    """Stack (rho, rho*v_d..., E) for the given primitive fields (xp: numpy
    or torch, for inputs that live on the host or on the device)."""
    if xp is np:
        rho = np.asarray(rho, dtype=np.float64)
        vel = [np.asarray(v, dtype=np.float64) for v in vel]
        p = np.asarray(p, dtype=np.float64)
    mom = [rho * v for v in vel]
    ke = 0.5 * sum(m * v for m, v in zip(mom, vel))
    E = p / (gamma - 1.0) + ke
    one = xp.ones_like(E)
    return xp.stack([rho * one] + [m * one for m in mom] + [E])


# --------------------------------------------------------------------------
# Workload descriptions.  A workload is a dict with the mesh shape and a
# field function; a field function takes cell-centre coordinate arrays
# (x, y[, z]) and returns conserved variables stacked on axis 0.
# --------------------------------------------------------------------------

def periodic_2d_wave():
    """2D smoke workload: 4x4 trees of 8x8 cells on the unit square,
    rho = 1 + 0.2 sin(2 pi x) sin(2 pi y), v = (1, 0.5), p = 1, gamma 1.4."""
    gamma = 1.4

    def field(x, y):
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
        one = np.ones_like(rho)
        return conserved_from_primitive(rho, [one, 0.5 * one], one, gamma)

    return dict(name="wave2d_32x32_b8", ndim=2, trees=(4, 4, 1), N=8, g=2,
                tree_size=0.25, level=0, gamma=gamma, cfl=0.5, field=field,
                steps=20)


def smoothed_noise_grid(n: int, seed: int) -> np.ndarray:
    """Periodic n^3 noise in [-1,1) (i fastest), smoothed by a separable
    3-point box filter [1,1,1]/3 along x, then y, then z."""
    u = uniform_pm1(seed, n * n * n).reshape(n, n, n)  # [k][j][i]
    for ax in (2, 1, 0):
        u = (np.roll(u, 1, axis=ax) + u + np.roll(u, -1, axis=ax)) / 3.0
    return u


def uniform_noise_shear(block: int = 16, n: int = 256, seed: int = 0):
    """3D uniform workload: n^3 cells in blocks of block^3 on the periodic unit
    cube; rho = 1 + 0.1 u (u = smoothed seeded noise), v = (0.2 sin 2 pi y, 0, 0),
    p = 2.5, gamma 1.4."""
    gamma = 1.4
    nt = n // block

    def grid_field():
        u = smoothed_noise_grid(n, seed)
        rho = 1.0 + 0.1 * u
        y = (np.arange(n) + 0.5) / n
        vx = np.broadcast_to(0.2 * np.sin(2 * np.pi * y)[None, :, None], rho.shape)
        zero = np.zeros_like(rho)
        return conserved_from_primitive(rho, [vx, zero, zero], 2.5 * np.ones_like(rho), gamma)

    return dict(name=f"noise_shear_{n}^3_b{block}", ndim=3, trees=(nt, nt, nt), N=block,
                g=2, tree_size=1.0 / nt, level=0, gamma=gamma, cfl=0.5,
                grid_field=grid_field, steps=50)


def rayleigh_taylor(block: int = 16, n: int = 256, ndim: int = 3, p_top: float = 1.0):
    """Rayleigh-Taylor workload of Sec. 4.2 on n^ndim cells in blocks of
    block^ndim: heavy fluid (rho 1.0) above the interface z = h(x, y) =
    0.8 + 0.05 sin(2 pi x) sin(2 pi y) (2D: y = 0.8 + 0.05 sin(2 pi x)), light
    fluid (rho 0.1) below, at rest, gamma 5/3, gravity -1 along the last axis,
    periodic along the other axes and closed by reflecting walls along the
    last one (bc_type: normal momentum Dirichlet 0, the rest Neumann 0),
    pressure in hydrostatic balance with p = p_top at the top:
    p = p_top + rho_h (1 - z) above h, p_top + rho_h (1 - h) + rho_l (h - z)
    below.  (The paper does not give p_top; 1.0 is this workload's choice.)
    The state is evaluated at cell centres."""
    gamma = 5.0 / 3.0
    nt = n // block
    rho_h, rho_l, h0, delta, k = 1.0, 0.1, 0.8, 0.05, 2 * math.pi

    def field(x, y, z=None):
        if ndim == 3:
            h, zz = h0 + delta * np.sin(k * x) * np.sin(k * y), z
        else:
            h, zz = h0 + delta * np.sin(k * x), y
        above = zz >= h
        rho = np.where(above, rho_h, rho_l)
        p = np.where(above, p_top + rho_h * (1.0 - zz), p_top + rho_h * (1.0 - h) + rho_l * (h - zz))
        zero = np.zeros_like(rho)
        return conserved_from_primitive(rho, [zero] * ndim, p, gamma)

    def grid_field():
        c = (np.arange(n) + 0.5) / n
        if ndim == 3:
            z, y, x = np.meshgrid(c, c, c, indexing="ij")
            return field(x, y, z)
        y, x = np.meshgrid(c, c, indexing="ij")
        return field(x, y)

    grav = (0.0, 0.0, -1.0) if ndim == 3 else (0.0, -1.0, 0.0)
    bc_type = np.ones((6, 5), np.int32)
    bc_type[2 * (ndim - 1), ndim] = bc_type[2 * (ndim - 1) + 1, ndim] = 0  # m_z (2D: m_y) Dirichlet 0
    periodic = tuple(d != ndim - 1 for d in range(3))
    return dict(name=f"rayleigh_taylor_{n}^{ndim}_b{block}", ndim=ndim, trees=(nt,) * ndim + (1,) * (3 - ndim),
                N=block, g=2, tree_size=1.0 / nt, level=0, gamma=gamma, cfl=0.5, field=field,
                grid_field=grid_field, limiter="vanleer", flux="rusanov", gravity=grav, steps=50,
                periodic=periodic, bc_type=bc_type, bc_value=np.zeros((6, 5)))


def blast_field(gamma=1.4, p_in=100.0, p_out=1e-3, r0=0.05, centre=(0.5, 0.5, 0.5)):
    def field(x, y, z, xp=np):
        r = xp.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
        rho = xp.ones_like(r)
        p = xp.where(r < r0, xp.full_like(r, p_in), xp.full_like(r, p_out))
        zero = xp.zeros_like(r)
        return conserved_from_primitive(rho, [zero, zero, zero], p, gamma, xp=xp)
    return field


def box_intersects_ball(lo, hi, centre, radius):
    """True where the axis-aligned box [lo, hi) meets the open ball."""
    d2 = 0.0
    for a in range(3):
        c = centre[a]
        q = np.clip(c, lo[a], hi[a])
        d2 = d2 + (q - c) ** 2
    return d2 < radius * radius


def two_level_blast(base_trees: int = 16, block: int = 8):
    """3D static two-level workload: base level of base_trees^3 blocks of
    block^3 cells; base blocks whose box meets the ball |x - 1/2| < 1/4 are
    refined once (2:1 balance applies); blast p = 100 in r < 0.05, else 1e-3."""
    gamma = 1.4
    ts = 1.0 / base_trees

    def refine_flags(tree_xyz):
        """+1 for base blocks (level 0, one per tree) meeting the ball."""
        t = np.asarray(tree_xyz, dtype=np.float64)
        lo = [t[:, a] * ts for a in range(3)]
        hi = [(t[:, a] + 1) * ts for a in range(3)]
        return np.where(box_intersects_ball(lo, hi, (0.5, 0.5, 0.5), 0.25), 1, 0).astype(np.int8)

    return dict(name=f"blast_two_level_{base_trees * block}^3_b{block}", ndim=3,
                trees=(base_trees,) * 3, N=block, g=2, tree_size=ts, level=0,
                gamma=gamma, cfl=0.5, field=blast_field(gamma), refine_flags=refine_flags,
                steps=100)


def batch_problem(p: int):
    """Problem p of the 64-problem batch (seed 1000 + p): block size drawn from
    {8, 16, 32}, block count log-uniform on [8, 4096], a periodic brick of
    trees near that count, smooth seeded rho and p in [0.5, 2], v = 0."""
    seed = 1000 + p
    d = uniform01(seed, 32)
    N = (8, 16, 32)[min(int(d[0] * 3), 2)]
    B = math.exp(math.log(8.0) + d[1] * (math.log(4096.0) - math.log(8.0)))
    nz = max(1, int(round(B ** (1.0 / 3.0))))
    ny = max(1, int(round(math.sqrt(B / nz))))
    nx = max(1, int(round(B / (nz * ny))))
    nmax = max(nx, ny, nz)
    ts = 1.0 / nmax
    L = (nx * ts, ny * ts, nz * ts)
    gamma = 1.4

    def modes(off):
        ks, amps, phis = [], [], []
        for m in range(4):
            base = off + 5 * m
            k = [int(min(4, math.floor(d[base + a] * 5))) - 2 for a in range(3)]
            ks.append(k)
            amps.append(0.5 + 0.5 * d[base + 3])
            phis.append(2 * math.pi * d[base + 4])
        return ks, amps, phis

    extra = uniform01(seed, 64, start=32)
    d = np.concatenate([d, extra])
    mr = modes(2)
    mp = modes(22)

    def smooth(x, y, z, mo, xp):
        ks, amps, phis = mo
        s = xp.zeros_like(x)
        for k, a, ph in zip(ks, amps, phis):
            s = s + a * xp.sin(2 * np.pi * (k[0] * x / L[0] + k[1] * y / L[1] + k[2] * z / L[2]) + ph)
        return s

    def field(x, y, z, xp=np):
        """xp = numpy (host) or torch (device tensors)."""
        sr = smooth(x, y, z, mr, xp)
        sp = smooth(x, y, z, mp, xp)
        mr_ = float(xp.max(xp.abs(sr)))
        mp_ = float(xp.max(xp.abs(sp)))
        rho = 1.25 + 0.75 * (sr / mr_ if mr_ > 0 else 0.0 * sr)
        pr = 1.25 + 0.75 * (sp / mp_ if mp_ > 0 else 0.0 * sp)
        zero = xp.zeros_like(x)
        return conserved_from_primitive(rho, [zero, zero, zero], pr, gamma, xp)

    return dict(name=f"batch_p{p}", ndim=3, trees=(nx, ny, nz), N=N, g=2, tree_size=ts,
                level=0, gamma=gamma, cfl=0.5, field=field, steps=20)


def mirrored_sod(nx_cells: int, block: int = 16, ndim: int = 2):
    """Periodic mirrored Sod tube along x: (rho, v, p) = (1, 0, 1) for
    x in [0.25, 0.75), (0.125, 0, 0.1) elsewhere; gamma 1.4.  The y (and z)
    extent is one tree so that every row is the same 1D problem."""
    gamma = 1.4
    nt = nx_cells // block

    def field(x, y, z=None):
        inside = (x >= 0.25) & (x < 0.75)
        rho = np.where(inside, 1.0, 0.125)
        p = np.where(inside, 1.0, 0.1)
        zero = np.zeros_like(rho)
        vel = [zero] * ndim
        return conserved_from_primitive(rho, vel, p, gamma)

    return dict(name=f"sod_{nx_cells}", ndim=ndim, trees=(nt, 1, 1), N=block, g=2,
                tree_size=1.0 / nt, level=0, gamma=gamma, cfl=0.5, field=field)


def adaptive_blast(centre=(0.5, 0.5, 0.5), p_in=100.0, trees=4, block=16, max_level=3, steps=400,
                   regrid_every=10, r0=0.05):
    """3D adaptive blast: trees^3 periodic trees of block^3 cells, levels
    0..max_level, blast p = p_in inside r < r0 around centre, p = 1e-3
    outside, rho = 1, v = 0.  Initial refinement is geometric: blocks that
    meet the ball of radius 2 r0 are refined, max_level times (the density
    criterion sees nothing in a uniform density).  The run regrids every
    regrid_every steps."""
    gamma = 1.4
    ts = 1.0 / trees

    def init_flags(level, G):
        size = ts / (2.0 ** np.asarray(level, dtype=np.float64))
        G = np.asarray(G, dtype=np.float64)
        lo = [G[:, a] * size for a in range(3)]
        hi = [(G[:, a] + 1) * size for a in range(3)]
        return np.where(box_intersects_ball(lo, hi, centre, 2 * r0), 1, 0).astype(np.int8)

    return dict(name=f"adaptive_blast_{trees * block}^3_L{max_level}_b{block}", ndim=3, trees=(trees,) * 3,
                N=block, g=2, tree_size=ts, level=0, max_level=max_level, gamma=gamma, cfl=0.5,
                field=blast_field(gamma, p_in, 1e-3, r0, centre), init_flags=init_flags, steps=steps,
                regrid_every=regrid_every, centre=tuple(centre), p_in=p_in)


def blast_training_runs(n_centres=4, seed=500):
    """(centre, p_in) of the indicator's training runs: centres drawn
    uniformly within +-0.05 of the domain centre, p_in in {30, 300} (the
    evaluation run uses the domain centre and p_in = 100)."""
    u = uniform_pm1(seed, 3 * n_centres).reshape(n_centres, 3) * 0.05
    return [(tuple(0.5 + u[c]), p) for p in (30.0, 300.0) for c in range(n_centres)]


# --------------------------------------------------------------------------
# Scalar advection (Sec. 3.4, Sec. 4.1): one variable rho, uniform velocity.
# Field functions return rho stacked as a single variable on axis 0.
# --------------------------------------------------------------------------

def advection_sphere_field(ndim, R=0.1, delta=0.05, centre=(0.5, 0.5, 0.5)):
    """The smoothed sphere of eq. advection-sphere-sol: rho = 1 for
    d < R - delta, 1 - 3 q^2 + 2 q^3 with q = 1 + (d - R) / delta for
    R - delta <= d < R, and 0 for d >= R, d the distance from the centre."""
    def field(*x, xp=np):
        d2 = sum((x[a] - centre[a]) ** 2 for a in range(ndim))
        d = xp.sqrt(d2)
        q = 1.0 + (d - R) / delta
        shell = 1.0 - 3.0 * q * q + 2.0 * q * q * q
        rho = xp.where(d < R - delta, xp.ones_like(d), xp.where(d < R, shell, xp.zeros_like(d)))
        return xp.stack([rho])
    return field


def advection_gauss_field(ndim, R=0.1, centre=(0.5, 0.5, 0.5)):
    """The Gaussian of eq. advection-sphere-gauss: rho = exp(-d^2 / R^2)."""
    def field(*x, xp=np):
        d2 = sum((x[a] - centre[a]) ** 2 for a in range(ndim))
        return xp.stack([xp.exp(-d2 / (R * R))])
    return field


def advection(ndim=3, block=16, n=256, init="sphere", limiter="vanleer", g=None, velocity=None, cfl=0.5):
    """Uniform scalar-advection workload of Sec. 4.1 / Sec. 5.2 (table of
    results on uniform grids): n^ndim cells in blocks of block^ndim on the
    periodic unit square or cube, v = (1, 1[, 1]), the smoothed sphere of
    radius 0.1 (init "sphere") or the Gaussian (init "gauss") at the centre."""
    nt = n // block
    vel = tuple(velocity) if velocity is not None else (1.0,) * ndim
    f = advection_sphere_field(ndim) if init == "sphere" else advection_gauss_field(ndim)
    return dict(name=f"advection_{init}_{n}^{ndim}_b{block}", ndim=ndim, trees=(nt,) * ndim + (1,) * (3 - ndim),
                N=block, g=(3 if limiter == "weno5" else 2) if g is None else g, tree_size=1.0 / nt, level=0,
                gamma=1.4, cfl=cfl, field=f, limiter=limiter, flux="rusanov", physics="advection",
                velocity=vel + (0.0,) * (3 - len(vel)), steps=50)


def advection_flux_fix(ndim=2, block=16, base_trees=4, levels=2, limiter="vanleer"):
    """The flux-fixing test of Sec. 4.1.1: the smoothed sphere on a statically
    refined periodic unit square or cube, v = (1, 1[, 1]), advanced to t = 1
    so that it crosses every refinement boundary and returns to its start.
    refine_rounds[r](level, G) gives the flags of round r: blocks of the
    current finest level that meet the ball of radius R + 0.1 around the
    centre are refined, `levels` times (2:1 balance applies)."""
    ts = 1.0 / base_trees
    centre = (0.5, 0.5, 0.5)

    def flags_at(level, G):
        size = ts / (2.0 ** np.asarray(level, dtype=np.float64))
        G = np.asarray(G, dtype=np.float64)
        lo = [G[:, a] * size if a < ndim else np.zeros(len(size)) for a in range(3)]
        hi = [(G[:, a] + 1) * size if a < ndim else np.ones(len(size)) for a in range(3)]
        c = centre if ndim == 3 else (0.5, 0.5, 0.5)
        hit = box_intersects_ball(lo, hi, c, 0.2)
        return np.where(hit, 1, 0).astype(np.int8)

    w = advection(ndim, block, base_trees * block, init="sphere", limiter=limiter)
    w.update(name=f"advection_flux_fix_{ndim}d_b{block}_L{levels}", max_level=levels, refine_rounds=levels,
             refine_flags_at=flags_at, t_end=1.0)
    return w
