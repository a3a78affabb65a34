"""Pins of the oracle's Runge-Kutta schemes beyond Heun: the SSP schemes with
three and four stages (Sec. 3.1: built from sub-steps of eq. feuler) and
classical RK4 (eq. rk4), CPU only."""
import math

import numpy as np
import pytest

import synth
from oracle import OracleMesh

RK = ["ssprk3", "ssprk43", "rk4"]


def two_level(ndim=3, integrator="heun", **kw):
    m = OracleMesh(ndim, (4, 4, 4), 8, 2, 0.25, integrator=integrator, **kw)
    cent = [(np.array([G[d] for _, G in m.forest.leaves]) + 0.5) / 4 for d in range(ndim)]
    m.regrid(np.where(sum((c - 0.5) ** 2 for c in cent) < 0.09, 1, 0).astype(np.int8), 0, 1)
    assert set(m.level.tolist()) == {0, 1}
    return m


def smooth_state(m, seed=3):
    xc = m.forest.cell_centres(m.N, m.tree_size)
    k = np.random.default_rng(seed).random(6)
    x, y = xc[:, 0], xc[:, 1]
    z = xc[:, 2] if m.ndim == 3 else 0 * x
    rho = 1 + 0.3 * np.sin(2 * np.pi * (x + k[0])) * np.cos(2 * np.pi * (y + k[1])) + 0.1 * np.sin(2 * np.pi * z)
    vel = [0.4 * np.cos(2 * np.pi * (y + k[2])), 0.3 * np.sin(2 * np.pi * (x + k[3]))]
    if m.ndim == 3:
        vel.append(0.2 * np.sin(2 * np.pi * (z + k[4])))
    U = synth.conserved_from_primitive(rho, vel, 1 + 0.2 * np.cos(2 * np.pi * (x + z + k[5])), 1.4)
    m.interior()[...] = np.moveaxis(U, 0, 1)


def forward_euler(m, u, c, dt):
    """u + c dt L(u) with its ghost fill and flux fix, from the Heun scheme's
    first stage (pinned elsewhere): the building block of every sub-step."""
    out = m.alloc()
    m.ghost_fill(u)
    m.stage(u, None, out, 1, c * dt)
    m.flux_fix(u, out, c * dt)
    return out


@pytest.mark.parametrize("integrator", RK)
@pytest.mark.parametrize("ndim", [2, 3])
def test_step_is_the_shu_osher_composition(ndim, integrator):
    """One step equals the scheme written with forward-Euler steps E(u, c dt)
    = u + c dt L(u) (Shu-Osher form for the SSP schemes):
      SSP-RK3:    u1 = E(u, dt); u2 = 3/4 u + 1/4 E(u1, dt); u' = 1/3 u + 2/3 E(u2, dt)
      SSP-RK(4,3): u1 = E(u, dt/2); u2 = E(u1, dt/2); u3 = 2/3 u + 1/3 E(u2, dt/2);
                   u' = E(u3, dt/2)
      RK4:        k_i = L(u_i) with u_1 = u, u_2 = u + dt/2 k_1, u_3 = u + dt/2 k_2,
                  u_4 = u + dt k_3; u' = u + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4)
    on a two-level mesh (ghost rounds and flux fixing in every sub-step)."""
    m = two_level(ndim, integrator)
    smooth_state(m)
    u = m.u.copy()
    dt = m.dt(u)
    if integrator == "ssprk3":
        u1 = forward_euler(m, u, 1.0, dt)
        u2 = 0.75 * u + 0.25 * forward_euler(m, u1, 1.0, dt)
        want = u / 3.0 + 2.0 / 3.0 * forward_euler(m, u2, 1.0, dt)
    elif integrator == "ssprk43":
        u1 = forward_euler(m, u, 0.5, dt)
        u2 = forward_euler(m, u1, 0.5, dt)
        u3 = 2.0 / 3.0 * u + u2 / 3.0 + (forward_euler(m, u2, 0.5, dt) - u2) / 3.0
        want = forward_euler(m, u3, 0.5, dt)
    else:
        k = []  # dt k_i as forward-Euler increments
        ui = u
        for c in (0.5, 0.5, 1.0, None):
            inc = forward_euler(m, ui, 1.0, dt) - ui
            k.append(inc)
            if c is not None:
                ui = u + c * inc
        want = u + (k[0] + 2 * k[1] + 2 * k[2] + k[3]) / 6.0
    m.step(1)
    got, ref = m.interior(), m.interior(want)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("integrator", RK)
def test_gravity_closed_form(integrator):
    """A uniform state under gravity follows m = m0 + rho g t,
    E = E0 + g.m0 t + rho |g|^2 t^2 / 2, which every scheme of order >= 2
    reproduces step by step."""
    g = (0.3, -0.5, -1.0)
    m = two_level(3, integrator, gravity=g, gamma=5.0 / 3.0)
    rho, v, p = 1.3, np.array([0.4, -0.2, 0.1]), 2.0
    m0 = rho * v
    E0 = p / (2.0 / 3.0) + 0.5 * rho * v @ v
    m.interior()[...] = np.array([rho, *m0, E0]).reshape(1, 5, 1, 1, 1)
    m.step(5)
    t, gv = m.t, np.array(g)
    want = [rho, *(m0 + rho * gv * t), E0 + gv @ m0 * t + 0.5 * rho * (gv @ gv) * t * t]
    for k, e in enumerate(want):
        assert np.allclose(m.interior()[:, k], e, rtol=1e-14, atol=1e-14), k


@pytest.mark.parametrize("integrator", RK)
def test_two_level_conservation(integrator):
    """Flux fixing after every sub-step keeps the totals to rounding."""
    m = two_level(3, integrator)
    smooth_state(m)
    t0 = m.totals()
    vol = np.array([(m.tree_size / (m.N << l)) ** 3 for l in m.level])
    scale = np.abs(m.interior()).reshape(m.nb, m.nvar, -1).sum(-1).T @ vol
    m.step(3)
    assert np.all(np.abs(m.totals() - t0) <= 1e-13 * scale)


def _wave(integrator, cfl, t_end=0.2, limiter="vanleer"):
    g = 3 if limiter == "weno5" else 2
    m = OracleMesh(2, (4, 1, 1), 8, g, 0.25, gamma=1.4, cfl=cfl, limiter=limiter, integrator=integrator)

    def field(x, y):
        one = np.ones_like(x)
        return synth.conserved_from_primitive(1 + 0.2 * np.sin(2 * np.pi * x), [one, 0 * one], one, 1.4)

    m.set_interior_from_field(field)
    while m.t < t_end - 1e-15:
        dt = m.dt()
        if m.t + dt > t_end:
            m.cfl = m._c.cfl = cfl * (t_end - m.t) / dt
        m.step(1)
    return m.interior()[:, 0].copy()


def test_time_error_below_heun():
    """On one mesh with the van Leer limiter the time-stepping error (against
    the same scheme at CFL 0.02) of the third- and fourth-order schemes at
    CFL 0.4 is at least 10x below Heun's; Heun and the two SSP schemes fall
    under CFL halving at order >= 1.9.  Classical RK4 is not held to an order
    here: van Leer's limiter is only piecewise smooth in the data, and its
    switches cap RK4's observed order near 1.7 (its order is pinned on the
    smooth WENO5 operator below)."""
    errs = {}
    for integ in ["heun"] + RK:
        ref = _wave(integ, 0.02)
        errs[integ] = [float(np.mean(np.abs(_wave(integ, c) - ref))) for c in (0.4, 0.2)]
    for integ in RK:
        assert errs[integ][0] * 10 <= errs["heun"][0], errs
    for integ in ("heun", "ssprk3", "ssprk43"):
        assert math.log2(errs[integ][0] / errs[integ][1]) >= 1.9, (integ, errs)


def test_time_order_on_a_smooth_operator():
    """With WENO5 reconstruction the semi-discrete operator L is smooth in
    the data (its nonlinear weights are differentiable), so on a fixed mesh
    each integrator shows its classical order in time (Sec. 3.1: Heun 2,
    SSP-RK3 and SSP-RK(4,3) 3, RK4 4): the error against the same scheme at
    CFL 0.02 falls by 2^order per halving of CFL 0.4 -> 0.2 -> 0.1.  A wrong
    weight in any sub-step table drops the order to at most 1 or 2."""
    want = {"heun": 1.9, "ssprk3": 2.9, "ssprk43": 2.9, "rk4": 3.8}
    for integ, lo in want.items():
        ref = _wave(integ, 0.02, limiter="weno5")
        e = [float(np.mean(np.abs(_wave(integ, c, limiter="weno5") - ref))) for c in (0.4, 0.2, 0.1)]
        orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        assert all(lo <= o <= lo + 0.4 for o in orders), (integ, e, orders)
