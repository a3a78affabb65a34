"""GPU parity of physical boundaries (Sec. 2.4, Dirichlet and Neumann per face
direction and variable) against the FP64 oracle, through the C ABI: ghost
patterns and ghost values bit for bit, the paper's linear-solution test with
the solution on the boundary, states after steps within 1e-12 (FP64) and
2e-5 (FP32) relative L1, regrid bit for bit, batched equal to plain."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_helpers import build_pair, face_ghost_mask, gpu_mesh, gpu_state, interior, oracle_mesh, check_state

pytestmark = pytest.mark.gpu

TOL = {0: 2e-5, 1: 1e-12}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def f4():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_07612_amd as f4
    f4.lib()
    return f4


def wall_bc(ndim):
    t = np.ones((6, 5), np.int32)
    for f in range(2 * ndim):
        t[f, 1 + f // 2] = 0
    return t, np.zeros((6, 5))


def closed_box_blast(ndim=3, periodic=(False, False, False), base_trees=4, block=8):
    """The two-level blast (off centre, so no symmetry hides an index error)
    in a box with reflecting walls on its bounded axes."""
    w = synth.two_level_blast(base_trees=base_trees, block=block) if ndim == 3 else two_level_2d()
    if ndim == 3:
        w["field"] = synth.blast_field(p_in=10.0, p_out=0.1, r0=0.15, centre=(0.4, 0.55, 0.47))
    t, v = wall_bc(ndim)
    w.update(periodic=tuple(periodic), bc_type=t, bc_value=v)
    w["name"] = f'box{ndim}d_{"".join("p" if p else "w" for p in periodic[:ndim])}_b{w["N"]}'
    return w


def two_level_2d():
    gamma = 1.4

    def field(x, y):
        r = np.sqrt((x - 0.42) ** 2 + (y - 0.55) ** 2)
        rho = 1.0 + 0 * r
        p = np.where(r < 0.12, 10.0, 0.1)
        return synth.conserved_from_primitive(rho, [0 * r, 0 * r], p, gamma)

    def refine_flags(G):
        G = np.asarray(G)
        return np.all((G[:, :2] >= 3) & (G[:, :2] <= 4), axis=1).astype(np.int8)

    return dict(name="blast2d", ndim=2, trees=(8, 8, 1), N=8, g=2, tree_size=1.0 / 8, level=0, gamma=gamma,
                cfl=0.5, field=field, refine_flags=refine_flags)


def wind_tunnel_2d():
    """2D channel along x (periodic in y): Dirichlet inflow (rho 1, u 0.8,
    v 0, p 1) at -x, Neumann 0 outflow at +x, the 2D blast inside."""
    w = two_level_2d()
    gamma = w["gamma"]
    t = np.zeros((6, 5), np.int32)
    v = np.zeros((6, 5))
    E = 1.0 / (gamma - 1) + 0.5 * 0.8 ** 2
    v[0, :4] = [1.0, 0.8, 0.0, E]
    t[1, :4] = 1
    w.update(periodic=(False, True, True), bc_type=t, bc_value=v, name="wind_tunnel_2d")
    return w


def random_bc(ndim, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, (6, 5)).astype(np.int32), rng.uniform(-0.5, 0.5, (6, 5))


def run_pair(w, prec, steps):
    gm, om = build_pair(w, prec)
    gm.step(steps)
    t_gpu, _ = gm.time()
    om.step(steps)
    lev = gm.export()[0]
    a = interior(gpu_state(gm), w["g"], w["N"], w["ndim"])
    err, err_elem = check_state(a, om.interior(), lev, w["ndim"], w["tree_size"], w["N"], prec)
    say(w["name"], "prec", prec, "steps", steps, "rel L1", err, "t", t_gpu, om.t)
    return gm, om, err, t_gpu


# ------------------------------------------------------------------ pattern

@pytest.mark.parametrize("ndim,periodic", [(3, (False, True, True)), (3, (True, False, False)), (3, (False,) * 3),
                                           (2, (False, True, True)), (2, (False, False, True))])
def test_pattern_bit_exact(f4, ndim, periodic):
    """Leaf table and all four record kinds (boundary faces included) equal
    the oracle's on two-level meshes with bounded axes."""
    w = closed_box_blast(ndim, periodic)
    gm, om = build_pair(w, 1)
    pg, po = gm.pattern_export(), om.pat
    for key in ("srl", "srl_off", "f2c", "f2c_off", "c2f", "c2f_off", "bc", "bc_off"):
        assert np.array_equal(np.asarray(pg[key]).reshape(-1), np.asarray(po[key]).reshape(-1)), key
    nbc = int(po["bc_off"][-1])
    say(w["name"], "boundary faces", nbc)
    assert nbc > 0


# --------------------------------------------------------------- ghost fill

@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_ghost_fill_bit_exact(f4, ndim, prec):
    """Random Dirichlet / Neumann types and values per face and variable on
    a two-level mesh bounded in every direction: the GPU's face ghosts equal
    the oracle's bit for bit (FP32: the oracle on the same FP32 values, each
    round's FP64 result rounded once)."""
    w = closed_box_blast(ndim)
    w["bc_type"], w["bc_value"] = random_bc(ndim, 7 + ndim)
    gm, om = build_pair(w, prec)
    om.u[...] = 0.0
    om.interior()[...] = interior(gpu_state(gm), w["g"], w["N"], ndim)
    gm.ghost_fill()
    om.ghost_round(1)
    if prec == 0:
        om.u[...] = om.u.astype(np.float32)
    om.ghost_round(2)
    mask = face_ghost_mask(ndim, w["N"], w["g"])
    G = gpu_state(gm)[:, :, mask]
    O = om.u[:, :, mask]
    if prec == 0:
        O = O.astype(np.float32).astype(np.float64)
    assert np.array_equal(G, O)


@pytest.mark.parametrize("ndim,g", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_linear_solution_exact(f4, ndim, g):
    """Sec. 4.3 with the solution on the boundary: u_v = A_v + B_v (x + 2y +
    3z) on the non-periodic unit square/cube, Neumann values = its outward
    normal derivatives, refined twice towards a corner (the GPU's remap
    prolongs the data); every face ghost the GPU fills is exact to 1e-15 of
    the magnitude."""
    from paper_2605_07612_amd import layout
    A = (0.0, 1.0, -1.0, 2.0, 5.0)
    B = (1.0, -2.0, 0.5, 3.0, 0.0)
    coef = (1.0, 2.0, 3.0)
    nv = ndim + 2
    t = np.ones((6, 5), np.int32)
    val = np.zeros((6, 5))
    for f in range(2 * ndim):
        for v in range(nv):
            val[f, v] = (1.0 if f % 2 else -1.0) * B[v] * coef[f // 2]
    N = 8
    m = f4.Mesh(ndim, (2, 2, 2), N, g, 0.5, level=0, max_level=3, max_blocks=2 ** ndim * 8 ** ndim,
                prec=f4.F64, periodic=(False,) * 3, bc_type=t, bc_value=val)

    def field(*x):
        phi = sum(coef[d] * x[d] for d in range(ndim))
        return np.stack([A[v] + B[v] * phi for v in range(nv)])

    layout.set_from_field(m, field)
    for lev in range(2):
        _, G = layout.global_coords(m)
        lv = m.export()[0]
        corner = np.all(G[:, :ndim] == 0, axis=1) & (lv == lev)
        m.regrid(corner.astype(np.int8))
    m.ghost_fill()
    u = gpu_state(m)
    lev, Gc = layout.global_coords(m)
    P = N + 2 * g
    idx = np.arange(-g, N + g) + 0.5
    mask = face_ghost_mask(ndim, N, g)
    checked = 0
    for n in range(m.nb):
        dx = 0.5 / (N << int(lev[n]))
        cent = []
        for d in range(ndim):
            shape = [1] * ndim
            shape[ndim - 1 - d] = P
            cent.append(np.broadcast_to(((Gc[n, d] * N + idx) * dx).reshape(shape), (P,) * ndim))
        phi = sum(coef[d] * cent[d] for d in range(ndim))
        for v in range(nv):
            want = (A[v] + B[v] * phi)[mask]
            got = u[n, v][mask]  # gpu_state gives padded cubes
            assert np.all(np.abs(got - want) <= 1e-15 * max(1.0, abs(A[v]) + 6 * abs(B[v]))), (n, v)
            checked += got.size
    say("linear ghosts checked", checked, "levels", sorted(set(lev.tolist())))
    assert sorted(set(lev.tolist())) == [0, 1, 2]


# --------------------------------------------------------------- the step

@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
@pytest.mark.parametrize("case", ["box3d", "box3d_half", "box2d", "wind_tunnel_2d", "rt3d", "rt2d", "box3d_s7"])
def test_step_parity(f4, case, prec):
    """Walls on two-level meshes (flux fixing next to walls), a Dirichlet
    inflow with a Neumann outflow, and the Rayleigh-Taylor workload of Sec.
    4.2 with its z walls, against the oracle."""
    steps = 10
    if case == "box3d":
        w = closed_box_blast(3)
    elif case == "box3d_half":
        w = closed_box_blast(3, (True, False, True))
    elif case == "box2d":
        w, steps = closed_box_blast(2), 20
    elif case == "wind_tunnel_2d":
        w, steps = wind_tunnel_2d(), 20
    elif case == "rt3d":
        w = synth.rayleigh_taylor(block=16, n=64)
    elif case == "rt2d":
        w, steps = synth.rayleigh_taylor(block=16, n=128, ndim=2), 30
    else:
        w = closed_box_blast(3)
        w.update(limiter="vanleer", flux="hll", gravity=(0.0, 0.0, -1.0), name="box3d_vanleer_hll_gravity")
    gm, om, err, t = run_pair(w, prec, steps)
    assert err <= TOL[prec]
    assert abs(t - om.t) <= (1e-13 if prec == 1 else 1e-5) * om.t


@pytest.mark.parametrize("prec", [0, 1], ids=["f32", "f64"])
def test_closed_box_conserves_mass_and_energy(f4, prec):
    w = closed_box_blast(3)
    gm, _ = build_pair(w, prec)
    t0 = gm.totals()
    gm.step(20)
    t1 = gm.totals()
    rel = np.abs(t1 - t0) / (np.abs(t0) + 1.0)
    say("box drift", rel)
    assert rel[0] <= (1e-13 if prec == 1 else 1e-6) and rel[-1] <= (1e-13 if prec == 1 else 1e-6)


def test_regrid_bit_exact(f4):
    """Lohner flags (boundary ghosts as neighbours) and the regrid of a
    bounded mesh (balance without wrap-around) equal the oracle's."""
    from paper_2605_07612_amd import layout
    w = closed_box_blast(3, (False, True, False))
    gm = gpu_mesh(w, 1, max_level=2, max_blocks=4 ** 3 * 64)
    om = oracle_mesh(w)
    lev, G = layout.global_coords(gm)
    f0 = w["refine_flags"](G)
    gm.regrid(f0)
    om.regrid(f0, 0, 2)
    layout.set_from_field(gm, w["field"])
    om.set_interior_from_field(w["field"])
    gm.step(4)
    om.u[...] = 0.0
    om.interior()[...] = interior(gpu_state(gm), 2, w["N"], 3)
    om.ghost_fill()
    flags = gm.refine_flags()
    assert np.array_equal(flags, om.lohner_flags())
    say("flags", np.bincount(flags + 1, minlength=3))
    changed = gm.regrid(flags)
    res = om.regrid(flags, 0, 2)
    assert changed == (res is not None) and changed
    a, b = gm.export(), om.forest.export()
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert np.array_equal(interior(gpu_state(gm), 2, w["N"], 3), om.interior())


@pytest.mark.parametrize("prec", [0, 1], ids=["f32", "f64"])
def test_batch_equals_plain(f4, prec):
    """A closed box and the Rayleigh-Taylor workload (bounded along z) in one
    batch, gathered halos (boundary faces read the block's own ghosts): equal
    to the plain steps bit for bit."""
    rt = synth.rayleigh_taylor(block=16, n=64)
    box = closed_box_blast(3)
    box.update(limiter=rt["limiter"], flux=rt["flux"], gravity=(0.2, 0.0, -1.0))
    ws = [box, rt]
    plain, batched = [], []
    for w in ws:
        plain.append(build_pair(w, prec)[0])
        batched.append(build_pair(w, prec)[0])
    for m in plain:
        m.step(5)
    b = f4.Batch(batched)
    b.set_config(kslabs=2, wg_per_cu=2, xcd_order=1)
    b.step(5)
    for w, p, q in zip(ws, plain, batched):
        A = interior(gpu_state(p), w["g"], w["N"], w["ndim"])
        B = interior(gpu_state(q), w["g"], w["N"], w["ndim"])
        assert np.array_equal(A, B), w["name"]
        assert p.time() == q.time()
    b.close()


# -------------------------------------------------- spatially varying values

def face_values(mesh, fn, nvar):
    """bc_data (eq. bc-data) of a GPU mesh: fn(v, x) at the centre of every
    face cell of every boundary record, from the mesh's own pattern export
    and leaf coordinates."""
    import torch
    from paper_2605_07612_amd import layout
    pat = mesh.pattern_export()
    lev, G = layout.global_coords(mesh)
    N, nd = mesh.N, mesh.ndim
    n2 = N if nd == 3 else 1
    p1, p2 = np.meshgrid(np.arange(N), np.arange(n2), indexing="xy")
    p1, p2 = p1.ravel(), p2.ravel()
    out = np.zeros((len(pat["bc"]), nvar, N * n2))
    for f in range(2 * nd):
        ax, side = f // 2, f % 2
        t = [d for d in range(nd) if d != ax]
        for r in range(pat["bc_off"][f], pat["bc_off"][f + 1]):
            b = int(pat["bc"][r])
            dx = mesh.desc.tree_size / (N << int(lev[b]))
            x = [None] * nd
            x[ax] = np.full(N * n2, (G[b, ax] * N + (N if side else 0)) * dx)
            x[t[0]] = (G[b, t[0]] * N + p1 + 0.5) * dx
            if nd == 3:
                x[t[1]] = (G[b, t[1]] * N + p2 + 0.5) * dx
            for v in range(nvar):
                out[r, v] = fn(v, x)
    return torch.tensor(out, device="cuda")


@pytest.mark.parametrize("ndim", [2, 3])
def test_bc_data_linear_exact_through_regrids(f4, ndim):
    """The paper's form of the Sec. 4.3 test on the GPU: Dirichlet values of
    the linear solution at every boundary face cell through the spatially
    varying array, renewed by the mesh-change callback at each regrid (the
    uniform values are 1e9, so any cell that missed the array shows)."""
    from paper_2605_07612_amd import layout
    A = (0.0, 1.0, -1.0, 2.0, 5.0)
    B = (1.0, -2.0, 0.5, 3.0, 0.0)
    coef = (1.0, 2.0, 3.0)
    nv = ndim + 2
    fn = lambda v, x: A[v] + B[v] * sum(coef[d] * x[d] for d in range(ndim))
    N, g = 8, 2
    m = f4.Mesh(ndim, (2, 2, 2), N, g, 0.5, level=0, max_level=3, max_blocks=2 ** ndim * 8 ** ndim, prec=f4.F64,
                periodic=(False,) * 3, bc_type=np.zeros((6, 5), np.int32), bc_value=np.full((6, 5), 1e9))
    calls = []

    def renew(mesh):
        calls.append(mesh.nb)
        return face_values(mesh, fn, nv)

    m.set_bc_data(face_values(m, fn, nv), callback=renew)
    layout.set_from_field(m, lambda *x: np.stack([fn(v, list(x)) for v in range(nv)]))
    for lev in range(2):
        _, G = layout.global_coords(m)
        lv = m.export()[0]
        m.regrid((np.all(G[:, :ndim] == 0, axis=1) & (lv == lev)).astype(np.int8))
    assert len(calls) == 2
    m.ghost_fill()
    u = gpu_state(m)
    lev, Gc = layout.global_coords(m)
    P = N + 2 * g
    idx = np.arange(-g, N + g) + 0.5
    mask = face_ghost_mask(ndim, N, g)
    for n in range(m.nb):
        dx = 0.5 / (N << int(lev[n]))
        cent = []
        for d in range(ndim):
            shape = [1] * ndim
            shape[ndim - 1 - d] = P
            cent.append(np.broadcast_to(((Gc[n, d] * N + idx) * dx).reshape(shape), (P,) * ndim))
        for v in range(nv):
            want = fn(v, cent)[mask]
            assert np.all(np.abs(u[n, v][mask] - want) <= 1e-15 * max(1.0, abs(A[v]) + 6 * abs(B[v]))), (n, v)


@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
def test_bc_data_step_parity_and_batch(f4, prec):
    """A bounded two-level blast with spatially varying Dirichlet (density,
    energy) and Neumann (momenta) values: the plain step against the oracle
    given the same array, and a batch that picks up the array set after the
    batch was created, bit for bit equal to the plain step."""
    import torch
    w = closed_box_blast(3)
    t = np.ones((6, 5), np.int32)
    t[:, 0] = t[:, 4] = 0
    val = np.zeros((6, 5))
    val[:, 0], val[:, 4] = 1.0, 0.25  # uniform values: the blast's ambient state
    w["bc_type"], w["bc_value"] = t, val

    def fn(v, x):
        s = np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]) + 0.5 * np.sin(2 * np.pi * x[2])
        return (1.0 + 0.2 * s) if v == 0 else (0.3 + 0.05 * s) if v == 4 else 0.1 * s

    gm, om = build_pair(w, prec)
    gm.set_bc_data(face_values(gm, fn, 5))
    om.set_bc_data(face_values(gm, fn, 5).cpu().numpy())
    gm2 = build_pair(w, prec)[0]
    b = f4.Batch([gm2])
    b.step(1)  # the batch's descriptors without the array
    gm2.set_bc_data(face_values(gm2, fn, 5))
    gm.step(1)
    steps = 8
    om.step(steps + 1)
    gm.step(steps)
    b.step(steps)
    lev = gm.export()[0]
    a = interior(gpu_state(gm), 2, w["N"], 3)
    err, err_elem = check_state(a, om.interior(), lev, 3, w["tree_size"], w["N"], prec)
    say("bc_data parity", prec, err)
    assert err <= TOL[prec]
    # the batch took its first step with the uniform values, so compare it
    # with a plain mesh that did the same
    gm3 = build_pair(w, prec)[0]
    gm3.step(1)
    gm3.set_bc_data(face_values(gm3, fn, 5))
    gm3.step(steps)
    assert np.array_equal(interior(gpu_state(gm2), 2, w["N"], 3), interior(gpu_state(gm3), 2, w["N"], 3))
    b.close()


def test_bc_data_size_is_checked(f4):
    import torch
    w = closed_box_blast(3)
    gm, _ = build_pair(w, 0)
    nbc = len(gm.pattern_export()["bc"])
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        gm.set_bc_data(torch.zeros((nbc, 5, 63), dtype=torch.float64, device="cuda"))
    gm.set_bc_data(None)
    gm.step(1)
