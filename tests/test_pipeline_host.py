"""Window arithmetic of the streaming pipeline (include/tomo_pipeline.h), through the C ABI on
the host: the kept interiors tile the volume exactly once, every solve window has the plan's
slice count, lies inside the volume and contains its interior with up to `halo` slices of
context on each side (the full halo wherever the volume has it)."""
import pytest


def _tomo():
    from paper_2603_28756_amd import tomo
    import os
    if not os.path.exists(tomo.LIB_PATH):
        pytest.skip("libtomo.so not built (run __graft_entry__.build())")
    return tomo


@pytest.mark.parametrize("n_total,nz,halo", [(10, 4, 0), (11, 4, 0), (4, 4, 0), (12, 6, 1), (13, 6, 2),
                                             (100, 16, 3), (17, 17, 8), (64, 8, 2)])
def test_windows_tile_the_volume(n_total, nz, halo):
    tomo = _tomo()
    C = nz - 2 * halo
    first, k0, k1, W = tomo.pipeline_window(n_total, nz, halo, 0)
    assert W == -(-n_total // C)
    covered = []
    for k in range(W):
        f, a, b, w = tomo.pipeline_window(n_total, nz, halo, k)
        assert w == W
        assert a == k * C and b == min(a + C, n_total)
        assert 0 <= f and f + nz <= n_total          # inside the volume, nz slices
        assert f <= a and b <= f + nz               # contains its interior
        assert a - f >= min(halo, a)                # full context below where it exists
        assert f + nz - b >= min(halo, n_total - b)  # and above
        covered.extend(range(a, b))
    assert covered == list(range(n_total))


@pytest.mark.parametrize("n_total,nz,halo,k", [(3, 4, 0, 0), (10, 4, 2, 0), (10, 4, -1, 0), (10, 4, 0, 3),
                                               (10, 4, 0, -1)])
def test_invalid_windows_are_rejected(n_total, nz, halo, k):
    tomo = _tomo()
    with pytest.raises(tomo.TomoError) as e:
        tomo.pipeline_window(n_total, nz, halo, k)
    assert e.value.status == tomo.TOMO_ERR_INVALID_ARG
