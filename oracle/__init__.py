"""Plain FP64 CPU oracle of the foap4 block-AMR Euler step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and
by the benchmark's CPU-baseline leg, never by the HIP library or its Python
binding.  It shares no code with paper_2605_07612_amd/.

Topology (leaf order, neighbour search, ghost pattern, balance, regrid map)
lives in oracle/mesh.py; the cell and face arithmetic lives in
oracle/foap4_oracle.c, which this module builds with gcc on first use and
calls through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .mesh import Forest

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "foap4_oracle.c")
_LIB = os.path.join(_HERE, "libfoap4_oracle.so")
# a separately built copy (e.g. with host sanitizers) may be named here
_LIB_OVERRIDE = os.environ.get("FOAP4_ORACLE_LIB")


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, FP64, no FMA contraction, OpenMP over
    independent blocks and records)."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        _lib.om_ghost_fill.argtypes = [P, P]
        _lib.om_ghost_round.argtypes = [P, P, ctypes.c_int]
        _lib.om_stage.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_double]
        _lib.om_flux_fix.argtypes = [P, P, P, ctypes.c_double]
        _lib.om_dt.argtypes = [P, P]
        _lib.om_dt.restype = ctypes.c_double
        _lib.om_step.argtypes = [P, P, P]
        _lib.om_step.restype = ctypes.c_double
        _lib.om_run.argtypes = [P, P, P, ctypes.c_int32, P]
        _lib.om_run.restype = ctypes.c_int32
        _lib.om_totals.argtypes = [P, P, P]
        _lib.om_count_unphysical.argtypes = [P, P]
        _lib.om_count_unphysical.restype = ctypes.c_int64
        _lib.om_lohner_flags.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, P]
        _lib.om_remap.argtypes = [P, P, P, P, P, P, P]
        _lib.om_block_raw_features.argtypes = [P, P, P]
        _lib.om_limiter.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        _lib.om_limiter.restype = ctypes.c_double
        _lib.om_riemann_flux.argtypes = [P, P, P, ctypes.c_int32, P]
        _lib.om_weno5.argtypes = [P]
        _lib.om_weno5.restype = ctypes.c_double
    return _lib


class _MeshC(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("N", ctypes.c_int32), ("g", ctypes.c_int32),
                ("nvar", ctypes.c_int32), ("nb", ctypes.c_int64), ("level", ctypes.c_void_p),
                ("dx0", ctypes.c_double), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("srl", ctypes.c_void_p), ("srl_off", ctypes.c_void_p),
                ("f2c", ctypes.c_void_p), ("f2c_off", ctypes.c_void_p),
                ("c2f", ctypes.c_void_p), ("c2f_off", ctypes.c_void_p),
                ("bc", ctypes.c_void_p), ("bc_off", ctypes.c_void_p),
                ("bc_type", (ctypes.c_int32 * 5) * 6), ("bc_val", (ctypes.c_double * 5) * 6),
                ("bc_data", ctypes.c_void_p),
                ("limiter", ctypes.c_int32), ("flux", ctypes.c_int32), ("grav", ctypes.c_double * 3),
                ("rk", ctypes.c_int32), ("phys", ctypes.c_int32), ("vel", ctypes.c_double * 3)]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# Lohner criterion constants of the paper's AMR runs (Sec. 5.4)
LOHNER = dict(c_ref=5e-2, c_deref=6.25e-3, eps=1e-2, eps_abs=1e-10)

# scheme options of Sec. 3.2: reconstruction limiter and numerical flux
LIMITERS = {"minmod": 0, "vanleer": 1, "weno5": 2}
FLUXES = {"rusanov": 0, "hll": 1}
# time integrators of Sec. 3.1
INTEGRATORS = {"heun": 0, "ssprk3": 1, "ssprk43": 2, "rk4": 3}
# systems: the Euler equations (Sec. 3.5) and scalar advection (Sec. 3.4)
PHYSICS = {"euler": 0, "advection": 1}


def limiter(kind, a, b):
    """Limited slope of a cell from its backward and forward differences."""
    return lib().om_limiter(LIMITERS[kind], float(a), float(b))


def weno5(v):
    """WENO5 value at the right face of the middle of five values."""
    a = np.ascontiguousarray(v, dtype=np.float64)
    return lib().om_weno5(_ptr(a))


def riemann_flux(wl, wr, ax=0, flux="rusanov", gamma=1.4, ndim=3):
    """Numerical flux between primitive states (rho, vx, vy, vz, p) along ax,
    in conservative variable order (rho, m_x .. m_ndim, E)."""
    c = _MeshC()
    c.ndim, c.nvar, c.gamma, c.flux = ndim, ndim + 2, float(gamma), FLUXES[flux]
    a = np.ascontiguousarray(wl, dtype=np.float64)
    b = np.ascontiguousarray(wr, dtype=np.float64)
    F = np.zeros(5)
    lib().om_riemann_flux(ctypes.byref(c), _ptr(a), _ptr(b), ax, _ptr(F))
    return F[:ndim + 2]


class OracleMesh:
    """A forest plus its FP64 state arrays [nb][nvar][P^ndim], P = N + 2g."""

    def __init__(self, ndim, trees, N, g=2, tree_size=1.0, level=0, gamma=1.4, cfl=0.5,
                 periodic=(True, True, True), origin=(0.0, 0.0, 0.0), limiter="minmod",
                 flux="rusanov", gravity=(0.0, 0.0, 0.0), bc_type=None, bc_value=None, integrator="heun",
                 physics="euler", velocity=(0.0, 0.0, 0.0)):
        """bc_type / bc_value: [2 ndim faces -x, +x, -y, +y, -z, +z][nvar]
        Dirichlet (0) or Neumann (1) conditions and their values (Sec. 2.4),
        used on the faces of non-periodic axes.  physics "advection": the
        scalar advection problem of Sec. 3.4 (one variable rho, uniform
        velocity `velocity`, not all zero); gamma and gravity are then unused."""
        if N % 2 or N < 2 * g or g < 2:
            raise ValueError("need even N >= 2g and g >= 2")
        if limiter == "weno5" and g < 3:
            raise ValueError("WENO5 needs g >= 3")
        self.physics = PHYSICS[physics]
        self.velocity = tuple(float(x) for x in velocity) + (0.0,) * (3 - len(velocity))
        if self.physics == 1 and not any(self.velocity[:ndim]):
            raise ValueError("scalar advection needs a non-zero velocity")
        self.ndim, self.N, self.g = ndim, N, g
        self.nvar = 1 if self.physics == 1 else 2 + ndim
        self.tree_size, self.gamma, self.cfl = float(tree_size), float(gamma), float(cfl)
        self.origin = origin
        self.limiter, self.flux = LIMITERS[limiter], FLUXES[flux]
        self.rk = INTEGRATORS[integrator]
        self.gravity = tuple(float(x) for x in gravity) + (0.0,) * (3 - len(gravity))
        self.bc_data = None
        self.bc_callback = None
        self.bc_type = np.zeros((6, 5), np.int32)
        self.bc_value = np.zeros((6, 5))
        if bc_type is not None:
            t = np.asarray(bc_type, np.int32)
            self.bc_type[: t.shape[0], : t.shape[1]] = t
        if bc_value is not None:
            v = np.asarray(bc_value, np.float64)
            self.bc_value[: v.shape[0], : v.shape[1]] = v
        self.forest = Forest(ndim, trees, periodic, level)
        self._refresh()
        self.u = self.alloc()
        self.t = 0.0

    # --------------------------------------------------------------- helpers
    @property
    def P(self):
        return self.N + 2 * self.g

    @property
    def nb(self):
        return self.forest.nb

    def alloc(self):
        return np.zeros((self.nb, self.nvar) + (self.P,) * self.ndim)

    def _refresh(self):
        self.pat = self.forest.pattern()
        self.level = self.forest.levels()
        self._c = _MeshC()
        c = self._c
        c.ndim, c.N, c.g, c.nvar, c.nb = self.ndim, self.N, self.g, self.nvar, self.nb
        c.level = _ptr(self.level)
        c.dx0 = self.tree_size / self.N
        c.gamma, c.cfl = self.gamma, self.cfl
        c.limiter, c.flux, c.rk = self.limiter, self.flux, self.rk
        c.grav[:] = list(self.gravity)
        c.phys = self.physics
        c.vel[:] = list(self.velocity)
        c.bc_data = _ptr(self.bc_data) if self.bc_data is not None else None
        for f in range(6):
            c.bc_type[f][:] = [int(x) for x in self.bc_type[f]]
            c.bc_val[f][:] = [float(x) for x in self.bc_value[f]]
        keep = []
        for name in ("srl", "srl_off", "f2c", "f2c_off", "c2f", "c2f_off", "bc", "bc_off"):
            arr = np.ascontiguousarray(self.pat[name], dtype=np.int32)
            if arr.size == 0:
                arr = np.zeros(1, np.int32)
            keep.append(arr)
            setattr(c, name, _ptr(arr))
        self._keep = keep

    def cref(self):
        return ctypes.byref(self._c)

    def set_bc_data(self, data, callback=None):
        """Spatially varying boundary values (eq. bc-data): [n boundary
        records][nvar][N^(ndim-1)] in the order of pat['bc'], face cells
        with the lower tangential axis fastest; None: the uniform values.
        callback(mesh) -> data is called after every regrid that changes the
        mesh (Sec. 2.4); without one the data is dropped then."""
        self.bc_callback = callback
        if data is None:
            self.bc_data = None
        else:
            nbf = int(self.pat["bc_off"][-1])
            self.bc_data = np.ascontiguousarray(data, dtype=np.float64).reshape(nbf, self.nvar, -1)
            assert self.bc_data.shape[2] == self.N ** (self.ndim - 1)
        self._c.bc_data = _ptr(self.bc_data) if self.bc_data is not None else None

    def interior(self, u=None):
        u = self.u if u is None else u
        g, N = self.g, self.N
        sl = (slice(None), slice(None)) + (slice(g, g + N),) * self.ndim
        return u[sl]

    def set_interior_from_field(self, field):
        """Evaluate field(x, y[, z]) at the cell centres and store it."""
        xc = self.forest.cell_centres(self.N, self.tree_size, self.origin)
        vals = field(*[xc[:, d] for d in range(self.ndim)])  # [nvar][nb][N..]
        self.interior()[...] = np.moveaxis(vals, 0, 1)

    def set_interior_from_grid(self, grid):
        """grid: [nvar][nz][ny][nx] (or [nvar][ny][nx]) on the uniform level of the mesh."""
        N = self.N
        for n, (l, G) in enumerate(self.forest.leaves):
            if self.ndim == 3:
                self.u[n][:, self.g:self.g + N, self.g:self.g + N, self.g:self.g + N] = \
                    grid[:, G[2] * N:(G[2] + 1) * N, G[1] * N:(G[1] + 1) * N, G[0] * N:(G[0] + 1) * N]
            else:
                self.u[n][:, self.g:self.g + N, self.g:self.g + N] = \
                    grid[:, G[1] * N:(G[1] + 1) * N, G[0] * N:(G[0] + 1) * N]

    # -------------------------------------------------------------- numerics
    def ghost_fill(self, u=None):
        u = self.u if u is None else u
        lib().om_ghost_fill(self.cref(), _ptr(u))
        return u

    def ghost_round(self, rnd, u=None):
        """Round 1 (SRL, F2C) or round 2 (C2F) of the ghost fill alone."""
        u = self.u if u is None else u
        lib().om_ghost_round(self.cref(), _ptr(u), rnd)
        return u

    def dt(self, u=None):
        return lib().om_dt(self.cref(), _ptr(self.u if u is None else u))

    def stage(self, ud, up, uo, stage, dt):
        lib().om_stage(self.cref(), _ptr(ud), _ptr(up) if up is not None else None, _ptr(uo),
                       stage, dt)

    def flux_fix(self, ud, uo, dt_s):
        lib().om_flux_fix(self.cref(), _ptr(ud), _ptr(uo), dt_s)

    def step(self, n=1):
        """n Heun steps; returns the list of dts."""
        u1 = self.alloc()
        dts = np.zeros(max(n, 1))
        bad = lib().om_run(self.cref(), _ptr(self.u), _ptr(u1), n, _ptr(dts))
        if bad:
            raise FloatingPointError(f"oracle: unphysical state after step {bad}")
        self.t += float(np.sum(dts[:n]))
        return dts[:n]

    def totals(self, u=None):
        out = np.zeros(self.nvar)
        lib().om_totals(self.cref(), _ptr(self.u if u is None else u), _ptr(out))
        return out

    def count_unphysical(self, u=None):
        return lib().om_count_unphysical(self.cref(), _ptr(self.u if u is None else u))

    def lohner_flags(self, u=None, **kw):
        c = dict(LOHNER)
        c.update(kw)
        flags = np.zeros(self.nb, np.int8)
        lib().om_lohner_flags(self.cref(), _ptr(self.u if u is None else u), c["c_ref"],
                              c["c_deref"], c["eps"], c["eps_abs"], _ptr(flags))
        return flags

    def raw_features(self, u=None):
        """[nb][2]: max |grad rho|/rho and max |grad p|/p per block (face ghosts needed)."""
        if self.physics != 0:
            raise ValueError("the indicator features are defined for the Euler system")
        r = np.zeros((self.nb, 2))
        lib().om_block_raw_features(self.cref(), _ptr(self.u if u is None else u), _ptr(r))
        return r

    def regrid(self, flags, lmin, lmax):
        """Adapt the mesh and remap the state (old ghosts are filled first).
        Returns the (op, src, arg) map, or None when the mesh is unchanged."""
        self.ghost_fill()
        old_c, old_keep, old_level, old_u = self._c, self._keep, self.level, self.u
        res = self.forest.regrid(flags, lmin, lmax)
        if res is None:
            return None
        op, src, arg = res
        self.bc_data = None
        self._refresh()
        if self.bc_callback is not None:
            self.set_bc_data(self.bc_callback(self), self.bc_callback)
        self.u = self.alloc()
        lib().om_remap(ctypes.byref(old_c), _ptr(old_u), self.cref(), _ptr(self.u),
                       _ptr(op), _ptr(src), _ptr(arg))
        del old_keep, old_level
        return res


def rel_l1(a, b, vol=None):
    """sum |a - b| dV / sum |b| dV over all variables together (a, b: [nb][nvar][...])."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    w = 1.0 if vol is None else vol.reshape((-1,) + (1,) * (a.ndim - 1))
    return float(np.sum(np.abs(a - b) * w) / np.sum(np.abs(b) * w))
