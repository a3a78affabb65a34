"""The allocation-free conserved totals (foap4_conserved_totals_noalloc),
through the C ABI on the GPU.

It runs the kernels of foap4_conserved_totals with a fixed device array as
scratch, so its totals must equal that entry point's bit for bit.  Two calls
in a row, the second on a smaller mesh, check that the shared array's
leftover contents from the first call do not leak into the second; a mesh
past the array's size is refused before anything is enqueued, and the mesh
still works afterwards."""
import sys

import numpy as np
import pytest

import synth

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


def wave_field(ndim, seed):
    """Smooth periodic density and pressure with seeded phases, v = (0.3, -0.2, 0.1)."""
    ph = synth.uniform01(seed, 4) * 2 * np.pi

    def field(*x):
        s = np.sin(2 * np.pi * x[0] + ph[0]) * np.cos(2 * np.pi * x[1] + ph[1])
        if ndim == 3:
            s = s * np.cos(2 * np.pi * x[2] + ph[2])
        one = np.ones_like(x[0])
        vel = [0.3 * one, -0.2 * one, 0.1 * one][:ndim]
        return synth.conserved_from_primitive(1.0 + 0.3 * s, vel, 1.0 + 0.2 * s, 1.4)
    return field


def wave_mesh(f4, ndim, trees, N, prec, seed):
    """Periodic brick on the unit square / cube with the wave field."""
    from paper_2605_07612_amd import layout
    m = f4.Mesh(ndim, trees, N, 2, 1.0 / max(trees[:ndim]), prec=prec)
    layout.set_from_field(m, wave_field(ndim, seed))
    return m


def noalloc_totals(f4, m):
    import torch
    out = torch.full((m.nvar + 3,), float("nan"), dtype=torch.float64, device=m.state[0].device)
    m.totals_noalloc(out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(np.isnan(o[m.nvar:])), "wrote past nvar values"
    return o[: m.nvar]


def test_noalloc_totals_equal_the_allocating_entry_point(f4):
    # first call: the larger mesh (3-D, 512 blocks of 8^3, FP32)
    say("noalloc: 3-D 8^3 x 512 blocks FP32")
    big = wave_mesh(f4, 3, (8, 8, 8), 8, f4.F32, seed=7)
    a = noalloc_totals(f4, big)
    b = big.totals()
    assert np.array_equal(a, b), (a, b)
    big.step(2)
    a = noalloc_totals(f4, big)
    b = big.totals()
    assert np.array_equal(a, b), (a, b)
    # second call right after it: a smaller mesh (2-D, 16 blocks of 16^2, FP64)
    say("noalloc: 2-D 16^2 x 16 blocks FP64")
    small = wave_mesh(f4, 2, (4, 4), 16, f4.F64, seed=8)
    a = noalloc_totals(f4, small)
    b = small.totals()
    assert np.array_equal(a, b), (a, b)
    small.step(3)
    a = noalloc_totals(f4, small)
    b = small.totals()
    assert np.array_equal(a, b), (a, b)
    # the totals are the plain FP64 sums of the state (a property, any size)
    u = small.interior().double().cpu().numpy()
    vol = (1.0 / 4 / 16) ** 2
    ref = u.sum(axis=tuple(i for i in range(u.ndim) if i != 1)) * vol
    assert np.allclose(a, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    big.close()
    small.close()


def test_noalloc_totals_refuse_a_mesh_past_the_scratch(f4):
    # 2-D, nvar 4: 129 x 128 trees at level 1 = 66048 blocks need 264192
    # partial sums > 262144
    say("noalloc: 2-D 8^2 x 66048 blocks FP32 (refused)")
    m = f4.Mesh(2, (129, 128), 8, 2, 1.0 / 129, level=1, prec=f4.F32)
    import torch
    out = torch.zeros(m.nvar, dtype=torch.float64, device=m.state[0].device)
    with pytest.raises(f4.Foap4Error) as e:
        m.totals_noalloc(out)
    assert e.value.status == -2
    assert "scratch" in str(e.value)
    assert torch.all(out == 0)
    m.close()
    # a mesh at the limit is accepted (65536 blocks x 4 = 262144)
    say("noalloc: 2-D 8^2 x 65536 blocks FP32 (at the limit)")
    m = f4.Mesh(2, (128, 128), 8, 2, 1.0 / 128, level=1, prec=f4.F32)
    from paper_2605_07612_amd import layout
    layout.set_from_field(m, wave_field(2, 11))
    a = noalloc_totals(f4, m)
    assert np.array_equal(a, m.totals())
    m.close()
