"""Degenerate cases and error paths of the HIP path (GPU), through the C ABI.

* A uniform state is a fixed point of the scheme: every face flux is the
  same, limited prolongation (zero slopes) and restriction of equal values
  return those values, and the flux fix adds zero (Sec. 2.5-2.7).  On the
  GPU it must stay bitwise uniform under the plain and the batched step,
  on single-level and two-level meshes, FP32 and FP64, 2D and 3D.
* A regrid that would exceed max_blocks fails with FOAP4_E_CAPACITY and
  leaves the mesh (leaf table, ghost pattern and state) unchanged.
* A state with a negative density is reported as FOAP4_E_UNPHYSICAL.
* A step count of zero changes nothing; a batch of meshes of different
  precisions is refused.
* The autotuner leaves the meshes as it found them and caches its choice.
* Creating and destroying meshes, batches and networks returns all device
  memory the library allocated."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_helpers import gpu_state, interior

pytestmark = pytest.mark.gpu


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


def uniform_field(ndim, rho=1.3, vel=(0.4, -0.2, 0.1), p=0.7, gamma=1.4):
    def field(*x):
        one = np.ones_like(x[0])
        return synth.conserved_from_primitive(rho * one, [v * one for v in vel[:ndim]], p * one, gamma)
    return field


def make_mesh(f4, ndim, N, prec, two_level, trees=4):
    """Periodic brick of trees^ndim base blocks; with two_level the central
    2^ndim base blocks are refined once (2:1 balance is then automatic)."""
    from paper_2605_07612_amd import layout
    nt = (trees,) * ndim
    ml = 1 if two_level else 0
    m = f4.Mesh(ndim, nt, N, 2, 1.0 / trees, level=0, max_level=ml,
                max_blocks=(trees ** ndim) * (1 << (ndim * ml)), prec=prec)
    if two_level:
        _, G = layout.global_coords(m)
        mid = trees // 2
        flags = np.all((G[:, :ndim] == mid - 1) | (G[:, :ndim] == mid), axis=1).astype(np.int8)
        assert m.regrid(flags)
        assert sorted(set(m.export()[0].tolist())) == [0, 1]
    return m


@pytest.mark.parametrize("two_level", [False, True], ids=["one_level", "two_level"])
@pytest.mark.parametrize("prec", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_state_is_a_fixed_point(f4, ndim, prec, two_level):
    from paper_2605_07612_amd import layout
    N, g = 8, 2
    say("uniform", ndim, prec, two_level)
    m_plain = make_mesh(f4, ndim, N, prec, two_level)
    m_batch = make_mesh(f4, ndim, N, prec, two_level)
    for m in (m_plain, m_batch):
        layout.set_from_field(m, uniform_field(ndim))
    ref = interior(gpu_state(m_plain), g, N, ndim)
    first = ref[:1, :, ...]
    assert np.array_equal(ref, np.broadcast_to(first, ref.shape))
    m_plain.step(6)
    b = f4.Batch([m_batch])
    b.set_config(kslabs=1, wg_per_cu=2, xcd_order=1)
    b.step(6)
    for name, m in (("plain", m_plain), ("batch", m_batch)):
        u = interior(gpu_state(m), g, N, ndim)
        say(name, "max |u - u0|", float(np.max(np.abs(u - ref))))
        assert np.array_equal(u, ref), name
    (t_p, dt_p), (t_b, dt_b) = m_plain.time(), m_batch.time()
    assert t_p > 0 and t_p == t_b and dt_p == dt_b
    b.close()


def test_regrid_capacity_error_leaves_mesh_unchanged(f4):
    from paper_2605_07612_amd import layout
    w = synth.two_level_blast(base_trees=2, block=8)
    m = f4.Mesh(3, w["trees"], 8, 2, w["tree_size"], level=0, max_level=2, max_blocks=16, prec=f4.F64)
    layout.set_from_field(m, w["field"])
    before = m.export()
    pat = m.pattern_export()
    state = m.current().cpu().numpy().copy()
    nb_rev = m.info()[:2]
    with pytest.raises(f4.Foap4Error, match="E_CAPACITY") as e:
        m.regrid(np.ones(m.nb, np.int8))  # 8 -> 64 blocks > 16
    assert e.value.status == -2
    assert m.info()[:2] == nb_rev
    after = m.export()
    assert all(np.array_equal(a, c) for a, c in zip(before, after))
    pat2 = m.pattern_export()
    assert all(np.array_equal(pat[k], pat2[k]) for k in pat)
    assert np.array_equal(m.current().cpu().numpy(), state)
    t, dt = m.step(1, sync=True)  # the mesh still steps
    assert t > 0 and dt > 0


def test_zero_steps_change_nothing(f4):
    from paper_2605_07612_amd import layout
    w = synth.two_level_blast(base_trees=2, block=8)
    m = f4.Mesh(3, w["trees"], 8, 2, w["tree_size"], prec=f4.F32)
    layout.set_from_field(m, w["field"])
    s0 = m.current().cpu().numpy().copy()
    cur = m.cur
    t, _ = m.step(0, sync=True)
    assert t == 0.0 and m.cur == cur
    assert np.array_equal(m.current().cpu().numpy(), s0)


@pytest.mark.parametrize("prec", [0, 1], ids=["f32", "f64"])
def test_negative_density_is_reported(f4, prec):
    from paper_2605_07612_amd import layout
    w = synth.two_level_blast(base_trees=2, block=8)
    m = f4.Mesh(3, w["trees"], 8, 2, w["tree_size"], prec=prec)
    layout.set_from_field(m, w["field"])
    m.interior()[3, 0, 2, 3, 4] = -1.0
    say("negative density", prec)
    with pytest.raises(f4.Foap4Error, match="E_UNPHYSICAL"):
        m.step(1, sync=True)


def test_batch_refuses_mixed_precision(f4):
    a = f4.Mesh(3, (2, 2, 2), 8, 2, 0.5, prec=f4.F32)
    b = f4.Mesh(3, (2, 2, 2), 8, 2, 0.5, prec=f4.F64)
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        f4.Batch([a, b])


def test_autotune_restores_state_and_caches(f4, tmp_path):
    """The autotuner times candidate configurations on the batch itself; the
    meshes' states and times are restored bit for bit afterwards, the chosen
    per-stage grids are valid, and a second call reads them from the cache."""
    from paper_2605_07612_amd import layout
    ws = [synth.two_level_blast(base_trees=4, block=8), synth.two_level_blast(base_trees=2, block=16)]
    ms = []
    for w in ws:
        m = f4.Mesh(3, w["trees"], w["N"], 2, w["tree_size"], prec=f4.F32)
        layout.set_from_field(m, w["field"])
        m.step(1, sync=True)
        ms.append(m)
    before = [(m.current().cpu().numpy().copy(), m.time()) for m in ms]
    b = f4.Batch(ms)
    cache = str(tmp_path / "tune.json")
    cfg = b.autotune(cache)
    say("autotune", cfg)
    ks, w1, w2, x = cfg
    assert ks in (1, 2) and x in (0, 1, 2) and w1 in (0, 1, 2, 3, 4, 6, 8) and w2 in (0, 1, 2, 3, 4, 6, 8)
    for (s0, t0), m in zip(before, ms):
        assert np.array_equal(m.current().cpu().numpy(), s0)
        assert m.time() == t0
    assert b.autotune(cache) == cfg
    assert '"' in open(cache).read()


def test_autotune_on_fresh_meshes_then_steps_equal_plain(f4, tmp_path):
    """Autotuning meshes that have not taken a step yet (their first dt not
    computed) and then stepping the batch gives exactly the plain form's
    steps: states and times bit for bit (a regression test: the tuner once
    restored a zero dt behind a mesh that counted its dt as computed, so the
    first step after tuning advanced by nothing)."""
    from paper_2605_07612_amd import layout
    w = synth.rayleigh_taylor(block=16, n=32)

    def make():
        m = f4.Mesh(3, w["trees"], w["N"], w["g"], w["tree_size"], prec=f4.F64, gamma=w["gamma"], cfl=w["cfl"],
                    limiter=w["limiter"], flux=w["flux"], gravity=w["gravity"], periodic=w["periodic"],
                    bc_type=w["bc_type"], bc_value=w["bc_value"])
        layout.set_from_grid(m, w["grid_field"]())
        return m

    plain, tuned = make(), make()
    b = f4.Batch([tuned])
    cfg = b.autotune(str(tmp_path / "tune.json"))
    say("autotune on fresh meshes", cfg)
    b.step(3)
    plain.step(3)
    assert tuned.time() == plain.time()
    assert np.array_equal(interior(gpu_state(tuned), 2, 16, 3), interior(gpu_state(plain), 2, 16, 3))
    b.close()
    plain.close()
    tuned.close()


def test_no_device_memory_leak(f4):
    """Meshes, batches and networks created and destroyed in a loop (with
    regrids, captured features and training in between) give back the
    device memory the library allocates."""
    import gc
    import torch
    from paper_2605_07612_amd import layout

    def cycle():
        w = synth.two_level_blast(base_trees=4, block=8)
        m = f4.Mesh(3, w["trees"], 8, 2, w["tree_size"], level=0, max_level=2, max_blocks=4 ** 3 * 64, prec=f4.F32)
        layout.set_from_field(m, w["field"])
        m.capture_features(True)
        m.step(2, sync=True)
        m.regrid(m.refine_flags())
        net = f4.Mlp(weights=0.1 * np.random.default_rng(0).standard_normal(f4.MLP_NPARAM).astype(np.float32))
        x = m.block_features()
        net.train(x, torch.zeros(m.nb, dtype=torch.int8, device=x.device), 2)
        m.set_indicator(f4.IND_MLP, net)
        m.step(1, sync=True)
        m.regrid()
        b = f4.Batch([m])
        b.step(2)
        m.time()
        b.close()
        net.close()
        m.close()

    cycle()  # first use: library-wide allocations, caches
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(20):
        cycle()
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free1 = torch.cuda.mem_get_info()[0]
    say("device memory free before / after 20 cycles (MB)", free0 / 2 ** 20, free1 / 2 ** 20)
    assert free0 - free1 < 64 * 2 ** 20


@pytest.mark.parametrize("kw", [dict(kslabs=3), dict(wg_per_cu=65), dict(wg_per_cu=-1), dict(wg_stage2=65),
                                dict(xcd_order=3), dict(gather_halos=2)])
def test_batch_config_rejects_bad_arguments(f4, kw):
    """Batch configuration outside the documented ranges is refused with
    FOAP4_E_INVALID and the batch keeps its previous configuration."""
    m = f4.Mesh(3, (2, 2, 2), 8, 2, 0.5, prec=f4.F32)
    from paper_2605_07612_amd import layout
    layout.set_from_field(m, synth.two_level_blast(base_trees=2, block=8)["field"])
    b = f4.Batch([m])
    b.set_config(kslabs=2, wg_per_cu=2, xcd_order=1)
    args = dict(kslabs=2, wg_per_cu=2, xcd_order=1)
    args.update(kw)
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        b.set_config(**args)
    b.step(1)
    assert m.time()[0] > 0
