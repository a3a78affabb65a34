"""The state layout helpers (host side): to_padded / from_padded are inverse
bijections, and every cell lands at the offset the C ABI documents
(include/foap4.h): row * N + i for interior x, else P^(d-1) N + row 2g + c."""
import numpy as np
import pytest

from paper_2605_07612_amd import layout


def documented_offset(i, j, k, N, g, ndim):
    P = N + 2 * g
    row = (k + g) * P + (j + g) if ndim == 3 else (j + g)
    if 0 <= i < N:
        return row * N + i
    c = i + g if i < 0 else i - N + g
    return P ** (ndim - 1) * N + row * 2 * g + c


@pytest.mark.parametrize("ndim,N,g", [(2, 8, 2), (3, 8, 2), (3, 16, 2), (3, 8, 3), (2, 16, 4)])
def test_padded_round_trip_and_offsets(ndim, N, g):
    P = N + 2 * g
    rng = np.random.default_rng(7)
    cube = rng.standard_normal((3, ndim + 2) + (P,) * ndim)
    flat = layout.from_padded(cube, N, g, ndim)
    assert flat.shape == (3, ndim + 2, P ** ndim)
    assert np.array_equal(layout.to_padded(flat, N, g, ndim), cube)
    # every padded position maps to its documented offset, and the map is onto
    seen = np.zeros(P ** ndim, bool)
    ks = range(-g, N + g) if ndim == 3 else [0]
    for k in ks:
        for j in range(-g, N + g):
            for i in range(-g, N + g):
                o = documented_offset(i, j, k, N, g, ndim)
                idx = (k + g, j + g, i + g) if ndim == 3 else (j + g, i + g)
                assert flat[1, 2, o] == cube[(1, 2) + idx]
                seen[o] = True
    assert seen.all()


def test_interior_planes_are_contiguous():
    """The interior of plane k of one variable is N^2 consecutive values."""
    N, g, ndim = 16, 2, 3
    offs = [documented_offset(i, j, 5, N, g, ndim) for j in range(N) for i in range(N)]
    assert offs == list(range(offs[0], offs[0] + N * N))
    assert (offs[0] * 4) % 128 == 0  # FP32: starts on a 128-byte line


def test_torch_views_write_through():
    torch = pytest.importorskip("torch")
    N, g, ndim = 8, 2, 3
    P = N + 2 * g
    u = torch.zeros((2, 5, P ** ndim), dtype=torch.float64)
    rows = layout.rows_view(u, N, g, ndim)
    rows[1, 3, 4, 5, 6] = 2.5  # k = 2, j = 3, i = 6
    assert u[1, 3, documented_offset(6, 3, 2, N, g, ndim)] == 2.5
    xg = layout.xghost_view(u, N, g, ndim)
    xg[0, 1, 2, 3, 0] = -1.0  # k = 0, j = 1, i = -2
    assert u[0, 1, documented_offset(-2, 1, 0, N, g, ndim)] == -1.0
