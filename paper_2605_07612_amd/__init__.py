"""Python binding of libfoap4.so, the MI355X (gfx950) foap4 hot path.

Argument marshalling only: every operation runs in the library's HIP
kernels.  PyTorch provides the device memory of the two state buffers and
the stream.  The binding refuses to run without the built library (there is
no CPU fallback).  The C ABI is documented in include/foap4.h.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfoap4.so")

F32, F64 = 0, 1
IND_LOHNER, IND_MLP = 0, 1
_STATUS = {0: "OK", -1: "E_INVALID", -2: "E_CAPACITY", -3: "E_HIP", -4: "E_ORDER", -5: "E_UNPHYSICAL"}


class Foap4Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n_trees", ctypes.c_int32 * 3), ("periodic", ctypes.c_int32 * 3),
                ("origin", ctypes.c_double * 3), ("tree_size", ctypes.c_double), ("block_n", ctypes.c_int32),
                ("n_ghost", ctypes.c_int32), ("init_level", ctypes.c_int32), ("min_level", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("max_blocks", ctypes.c_int64), ("prec", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("limiter", ctypes.c_int32),
                ("flux", ctypes.c_int32), ("gravity", ctypes.c_double * 3),
                ("bc_type", (ctypes.c_int32 * 5) * 6), ("bc_value", (ctypes.c_double * 5) * 6),
                ("integrator", ctypes.c_int32), ("physics", ctypes.c_int32), ("velocity", ctypes.c_double * 3)]

# stage scheme options (include/foap4.h: foap4_limiter, foap4_flux)
LIMITERS = {"minmod": 0, "vanleer": 1, "weno5": 2}
FLUXES = {"rusanov": 0, "hll": 1}
BC_DIRICHLET, BC_NEUMANN = 0, 1
INTEGRATORS = {"heun": 0, "ssprk3": 1, "ssprk43": 2, "rk4": 3}
# systems (include/foap4.h: foap4_physics)
PHYSICS = {"euler": 0, "advection": 1}


def wall_bc(ndim):
    """(bc_type, bc_value) [6][5] of reflecting walls on every face: the
    normal momentum Dirichlet 0, every other variable Neumann 0."""
    t = np.full((6, 5), BC_NEUMANN, np.int32)
    for f in range(2 * ndim):
        t[f, 1 + f // 2] = BC_DIRICHLET
    return t, np.zeros((6, 5))


_lib = None
P = ctypes.c_void_p
_BC_CB = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
I32, I64, DBL = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

EXPORTS = {
    # name: (restype, argtypes)
    "foap4_mesh_create": (I32, [ctypes.POINTER(MeshDesc), P, P, ctypes.c_size_t, P, ctypes.POINTER(P)]),
    "foap4_mesh_destroy": (I32, [P]),
    "foap4_set_bc_data": (I32, [P, P, I64, P, P]),
    "foap4_mesh_set_extra_state": (I32, [P, I32, P, ctypes.c_size_t]),
    "foap4_mesh_info": (I32, [P, P, P, P]),
    "foap4_mesh_export": (I32, [P, P, P, P]),
    "foap4_ghost_pattern_build": (I32, [P]),
    "foap4_ghost_pattern_counts": (I32, [P, P]),
    "foap4_ghost_pattern_export": (I32, [P, P, P, P, P]),
    "foap4_ghost_fill": (I32, [P, I32]),
    "foap4_compute_dt": (I32, [P]),
    "foap4_step": (I32, [P, I32, P, P]),
    "foap4_time": (I32, [P, P, P]),
    "foap4_conserved_totals": (I32, [P, P]),
    "foap4_conserved_totals_noalloc": (I32, [P, P]),
    "foap4_refine_flags": (I32, [P, I32, P]),
    "foap4_regrid": (I32, [P, P, P]),
    "foap4_batch_create": (I32, [P, I32, ctypes.POINTER(P)]),
    "foap4_batch_destroy": (I32, [P]),
    "foap4_batch_set_config": (I32, [P, I32, I32, I32, I32, I32]),
    "foap4_batch_autotune": (I32, [P, ctypes.c_char_p, P]),
    "foap4_batch_step": (I32, [P, I32]),
    "foap4_batch_phase_times": (I32, [P, I32, P]),
    "foap4_block_features": (I32, [P, P, P]),
    "foap4_mesh_set_indicator": (I32, [P, I32, P]),
    "foap4_mesh_capture_features": (I32, [P, I32]),
    "foap4_captured_features": (I32, [P, P, P]),
    "foap4_indicator_fallbacks": (I32, [P, P]),
    "foap4_mlp_create": (I32, [P, ctypes.POINTER(P)]),
    "foap4_mlp_destroy": (I32, [P]),
    "foap4_mlp_set_params": (I32, [P, P, I64]),
    "foap4_mlp_get_params": (I32, [P, P, I64]),
    "foap4_mlp_set_threshold": (I32, [P, ctypes.c_float]),
    "foap4_mlp_forward": (I32, [P, P, I64, P]),
    "foap4_mlp_loss_grad": (I32, [P, P, P, I64, P, P, P]),
    "foap4_mlp_train": (I32, [P, P, P, I64, P, I32, ctypes.c_float, P]),
    "foap4_last_error": (ctypes.c_char_p, [P]),
}

MLP_NIN, MLP_NHID, MLP_NOUT, MLP_NPARAM = 16, 64, 3, 5443


def lib():
    """Load libfoap4.so (built by __graft_entry__.build()); fails loudly if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _check(st, handle=None):
    if st != 0:
        msg = lib().foap4_last_error(handle)
        raise Foap4Error(st, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


class Mesh:
    """A mesh, its two caller-owned state buffers (torch tensors on the GPU)
    and the library handle."""

    def __init__(self, ndim, trees, N, g=2, tree_size=1.0, level=0, min_level=0, max_level=None,
                 max_blocks=None, prec=F64, gamma=1.4, cfl=0.5, origin=(0.0, 0.0, 0.0), device="cuda",
                 stream=None, limiter="minmod", flux="rusanov", gravity=(0.0, 0.0, 0.0),
                 periodic=(True, True, True), bc_type=None, bc_value=None, integrator="heun",
                 physics="euler", velocity=(0.0, 0.0, 0.0)):
        torch = _torch()
        self.ndim, self.N, self.g = ndim, N, g
        self.physics = physics
        self.nvar = 1 if physics == "advection" else ndim + 2
        self.P = N + 2 * g
        self.prec = prec
        self.dtype = torch.float64 if prec == F64 else torch.float32
        nt = list(trees[:ndim]) + [1] * (3 - ndim)
        base = int(np.prod(nt[:ndim]))
        if max_level is None:
            max_level = level
        if max_blocks is None:
            max_blocks = base * (1 << (ndim * max_level))
        self.max_blocks = int(max_blocks)
        d = MeshDesc()
        d.ndim = ndim
        d.n_trees[:] = nt
        d.periodic[:] = [1 if p else 0 for p in periodic[:3]]
        bt = np.zeros((6, 5), np.int32) if bc_type is None else np.asarray(bc_type, np.int32)
        bv = np.zeros((6, 5)) if bc_value is None else np.asarray(bc_value, np.float64)
        for f in range(bt.shape[0]):
            for v in range(bt.shape[1]):
                d.bc_type[f][v] = int(bt[f, v])
        for f in range(bv.shape[0]):
            for v in range(bv.shape[1]):
                d.bc_value[f][v] = float(bv[f, v])
        d.origin[:] = list(origin)
        d.tree_size = tree_size
        d.block_n = N
        d.n_ghost = g
        d.init_level = level
        d.min_level = min_level
        d.max_level = max_level
        d.max_blocks = self.max_blocks
        d.prec = prec
        d.gamma = gamma
        d.cfl = cfl
        d.integrator = INTEGRATORS[integrator]
        d.limiter = LIMITERS[limiter]
        d.flux = FLUXES[flux]
        d.gravity[:] = [float(x) for x in gravity] + [0.0] * (3 - len(gravity))
        d.physics = PHYSICS[physics]
        d.velocity[:] = [float(x) for x in velocity] + [0.0] * (3 - len(velocity))
        self.desc = d
        shape = (self.max_blocks, self.nvar, self.P ** ndim)  # row part, then x ghosts (include/foap4.h)
        self.state = [torch.zeros(shape, dtype=self.dtype, device=device),
                      torch.zeros(shape, dtype=self.dtype, device=device)]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = self.state[0].numel() * self.state[0].element_size()
        h = ctypes.c_void_p()
        st = lib().foap4_mesh_create(ctypes.byref(d), P(self.state[0].data_ptr()), P(self.state[1].data_ptr()),
                                     nbytes, P(self.stream.cuda_stream), ctypes.byref(h))
        _check(st)
        self.h = h
        # the extra states of the longer integrators (SSP: one, RK4: two)
        for idx in range(2, 2 + {"heun": 0, "rk4": 2}.get(integrator, 1)):
            self.state.append(torch.zeros(shape, dtype=self.dtype, device=device))
            _check(lib().foap4_mesh_set_extra_state(self.h, idx, P(self.state[idx].data_ptr()), nbytes), self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().foap4_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- queries
    def info(self):
        nb, rev, cur = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib().foap4_mesh_info(self.h, ctypes.byref(nb), ctypes.byref(rev), ctypes.byref(cur)), self.h)
        return nb.value, rev.value, cur.value

    @property
    def nb(self):
        return self.info()[0]

    @property
    def cur(self):
        return self.info()[2]

    def export(self):
        nb = self.nb
        lev = np.zeros(nb, np.int32)
        tree = np.zeros(nb, np.int32)
        anc = np.zeros((nb, 3), np.int32)
        _check(lib().foap4_mesh_export(self.h, _ptr(lev), _ptr(tree), _ptr(anc)), self.h)
        return lev, tree, anc

    def pattern_counts(self):
        c = np.zeros(24, np.int32)
        _check(lib().foap4_ghost_pattern_counts(self.h, _ptr(c)), self.h)
        return c.reshape(4, 6)

    def pattern_export(self):
        c = self.pattern_counts()
        n = c.sum(axis=1)
        srl = np.zeros((n[0], 2), np.int32)
        f2c = np.zeros((n[1], 4), np.int32)
        c2f = np.zeros((n[2], 3), np.int32)
        bc = np.zeros((n[3],), np.int32)
        _check(lib().foap4_ghost_pattern_export(self.h, _ptr(srl), _ptr(f2c), _ptr(c2f), _ptr(bc)), self.h)
        nf = 2 * self.ndim
        offs = [np.concatenate([[0], np.cumsum(c[t, :nf])]).astype(np.int32) for t in range(4)]
        return dict(srl=srl, srl_off=offs[0], f2c=f2c, f2c_off=offs[1], c2f=c2f, c2f_off=offs[2], bc=bc,
                    bc_off=offs[3])

    # ---------------------------------------------------------- operations
    def pattern_build(self):
        _check(lib().foap4_ghost_pattern_build(self.h), self.h)

    def ghost_fill(self, state=None):
        _check(lib().foap4_ghost_fill(self.h, self.cur if state is None else state), self.h)

    def compute_dt(self):
        _check(lib().foap4_compute_dt(self.h), self.h)

    def step(self, n=1, sync=False):
        if sync:
            t, dt = ctypes.c_double(), ctypes.c_double()
            _check(lib().foap4_step(self.h, n, ctypes.byref(t), ctypes.byref(dt)), self.h)
            return t.value, dt.value
        _check(lib().foap4_step(self.h, n, None, None), self.h)
        return None

    def time(self):
        t, dt = ctypes.c_double(), ctypes.c_double()
        _check(lib().foap4_time(self.h, ctypes.byref(t), ctypes.byref(dt)), self.h)
        return t.value, dt.value

    def totals(self):
        out = np.zeros(self.nvar)
        _check(lib().foap4_conserved_totals(self.h, _ptr(out)), self.h)
        return out

    def totals_noalloc(self, out):
        """Conserved totals into the caller's device tensor `out` (FP64, at
        least nvar values) without any allocation; enqueue only."""
        torch = _torch()
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < self.nvar or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of at least nvar values")
        _check(lib().foap4_conserved_totals_noalloc(self.h, P(out.data_ptr())), self.h)
        return out

    def refine_flags(self, indicator=IND_LOHNER):
        f = np.zeros(self.nb, np.int8)
        _check(lib().foap4_refine_flags(self.h, indicator, _ptr(f)), self.h)
        return f

    def block_features(self, raw=False):
        """Per-block features [nb][16] (FP32, device); with raw=True also the
        FP64 raw maxima [nb][2]."""
        torch = _torch()
        nb = self.nb
        feat = torch.empty((max(nb, 1), 16), dtype=torch.float32, device=self.state[0].device)
        r = torch.empty((max(nb, 1), 2), dtype=torch.float64, device=self.state[0].device) if raw else None
        _check(lib().foap4_block_features(self.h, P(feat.data_ptr()), P(r.data_ptr()) if raw else None), self.h)
        return (feat[:nb], r[:nb]) if raw else feat[:nb]

    def capture_features(self, on=True):
        """Let every later step() capture the features of the state at the
        start of its last step, inside that step's first stage."""
        _check(lib().foap4_mesh_capture_features(self.h, 1 if on else 0), self.h)

    def captured_features(self, raw=False):
        """Features [nb][16] (and raw [nb][2]) captured by the last step()."""
        torch = _torch()
        nb = self.nb
        feat = torch.empty((max(nb, 1), 16), dtype=torch.float32, device=self.state[0].device)
        r = torch.empty((max(nb, 1), 2), dtype=torch.float64, device=self.state[0].device) if raw else None
        _check(lib().foap4_captured_features(self.h, P(feat.data_ptr()), P(r.data_ptr()) if raw else None), self.h)
        return (feat[:nb], r[:nb]) if raw else feat[:nb]

    def set_bc_data(self, data, callback=None):
        """Spatially varying boundary values (eq. bc-data; include/foap4.h):
        data is an FP64 device tensor [n_bc][nvar][N^(ndim-1)] in the order of
        pattern_export()["bc"] (face cells with the lower tangential axis
        fastest), or None for the uniform values.  callback(mesh) -> tensor or
        None is called after every regrid that changes the mesh, to give the
        values for the new boundary records."""
        self._bc_py = callback
        self._bc_cb = None
        if callback is not None:
            def trampoline(_h, _user):
                self._apply_bc(self._bc_py(self))
            self._bc_cb = _BC_CB(trampoline)
        self._apply_bc(data)

    def _apply_bc(self, data):
        torch = _torch()
        if data is not None:
            data = data.to(device=self.state[0].device, dtype=torch.float64).contiguous()
        self._bc_data = data  # kept alive while the library may read it
        ptr = P(data.data_ptr()) if data is not None else None
        n = data.numel() if data is not None else 0
        cb = ctypes.cast(self._bc_cb, P) if self._bc_cb is not None else None
        _check(lib().foap4_set_bc_data(self.h, ptr, n, cb, None), self.h)

    def set_indicator(self, indicator, mlp=None):
        """Indicator used by regrid() without flags; mlp is kept referenced."""
        _check(lib().foap4_mesh_set_indicator(self.h, indicator, mlp.h if mlp is not None else None), self.h)
        self._mlp = mlp

    def fallbacks(self):
        n = ctypes.c_int64()
        _check(lib().foap4_indicator_fallbacks(self.h, ctypes.byref(n)), self.h)
        return n.value

    def regrid(self, flags=None):
        ch = ctypes.c_int32()
        fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.int8)
        _check(lib().foap4_regrid(self.h, _ptr(fl), ctypes.byref(ch)), self.h)
        return bool(ch.value)

    # ------------------------------------------------------------- states
    def current(self, state=None):
        """A copy of the leaf blocks' state as padded cubes [nb][nvar][P]^ndim
        (index order k, j, i; cell (i, j, k) at (k+g, j+g, i+g))."""
        from . import layout
        u = self.state[self.cur if state is None else state][: self.nb]
        return layout.to_padded(u, self.N, self.g, self.ndim)

    def interior(self, state=None):
        """Writable view [nb][nvar][N]^ndim (k, j, i) of the interior cells."""
        from . import layout
        u = self.state[self.cur if state is None else state][: self.nb]
        g, N = self.g, self.N
        rows = layout.rows_view(u, N, g, self.ndim)
        sl = (slice(None), slice(None)) + (slice(g, g + N),) * (self.ndim - 1) + (slice(None),)
        return rows[sl]


class Batch:
    """Several meshes of one precision advanced by one persistent launch per
    stage, with steps replayed from a HIP graph."""

    def __init__(self, meshes):
        self.meshes = list(meshes)
        arr = (ctypes.c_void_p * len(self.meshes))(*[m.h.value for m in self.meshes])
        h = ctypes.c_void_p()
        _check(lib().foap4_batch_create(arr, len(self.meshes), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().foap4_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_config(self, kslabs=1, wg_per_cu=0, xcd_order=1, gather_halos=1, wg_stage2=None):
        """wg_per_cu: workgroups per CU of stage 1, and of stage 2 unless
        wg_stage2 is given."""
        w2 = wg_per_cu if wg_stage2 is None else wg_stage2
        _check(lib().foap4_batch_set_config(self.h, kslabs, wg_per_cu, w2, xcd_order, gather_halos))

    def autotune(self, cache_path=None):
        """Returns the chosen (kslabs, wg_stage1, wg_stage2, xcd_order)."""
        cfg = np.zeros(4, np.int32)
        cp = cache_path.encode() if cache_path else None
        _check(lib().foap4_batch_autotune(self.h, cp, _ptr(cfg)))
        return tuple(int(x) for x in cfg)

    def step(self, n=1):
        _check(lib().foap4_batch_step(self.h, n))

    PHASES = ("ghost_r1", "ghost_r2", "stage", "fluxfix", "finalize", "step", "stage1", "stage2")

    def phase_times(self, n=3):
        """Average ms per launch/step of each phase (advances the meshes n steps)."""
        out = np.zeros(8)
        _check(lib().foap4_batch_phase_times(self.h, n, _ptr(out)))
        return dict(zip(self.PHASES, out.tolist()))


class Mlp:
    """The learned refinement indicator's network: FP32 master weights and
    training state in device memory, BF16 matrix-core kernels."""

    def __init__(self, weights=None, stream=None):
        torch = _torch()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().foap4_mlp_create(P(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        if weights is not None:
            self.set_params(weights)

    def close(self):
        if getattr(self, "h", None):
            lib().foap4_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib().foap4_mlp_set_params(self.h, _ptr(w), w.size))

    def get_params(self):
        w = np.zeros(MLP_NPARAM, np.float32)
        _check(lib().foap4_mlp_get_params(self.h, _ptr(w), w.size))
        return w

    def set_threshold(self, thr):
        _check(lib().foap4_mlp_set_threshold(self.h, float(thr)))

    @staticmethod
    def _rows(x):
        torch = _torch()
        if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != 16 or not x.is_cuda:
            raise ValueError("features must be a float32 CUDA tensor [n][16]")
        return x.contiguous()

    @staticmethod
    def _labels(y, n):
        torch = _torch()
        if y.dtype != torch.int8 or y.numel() != n or not y.is_cuda:
            raise ValueError("labels must be an int8 CUDA tensor of n entries")
        return y.contiguous()

    def forward(self, x):
        """Logits [n][3] of feature rows x [n][16] (device tensors)."""
        torch = _torch()
        x = self._rows(x)
        out = torch.empty((max(x.shape[0], 1), 3), dtype=torch.float32, device=x.device)
        _check(lib().foap4_mlp_forward(self.h, P(x.data_ptr()), x.shape[0], P(out.data_ptr())))
        return out[: x.shape[0]]

    def loss_grad(self, x, y, class_w=(1.0, 1.0, 1.0)):
        """(loss, gradient[NPARAM]) of the class-weighted cross-entropy."""
        x = self._rows(x)
        y = self._labels(y, x.shape[0])
        cw = np.ascontiguousarray(class_w, dtype=np.float32)
        loss = ctypes.c_double()
        g = np.zeros(MLP_NPARAM, np.float32)
        _check(lib().foap4_mlp_loss_grad(self.h, P(x.data_ptr()), P(y.data_ptr()), x.shape[0], _ptr(cw),
                                         ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def train(self, x, y, iters, lr=1e-3, class_w=(1.0, 1.0, 1.0)):
        """iters full-batch Adam steps; returns the loss before each step."""
        x = self._rows(x)
        y = self._labels(y, x.shape[0])
        cw = np.ascontiguousarray(class_w, dtype=np.float32)
        losses = np.zeros(max(iters, 1))
        _check(lib().foap4_mlp_train(self.h, P(x.data_ptr()), P(y.data_ptr()), x.shape[0], _ptr(cw), iters,
                                     float(lr), _ptr(losses)))
        return losses[:iters]
