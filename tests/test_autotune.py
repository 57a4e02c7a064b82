"""Host logic of the tile-shape tuner (no GPU): candidate tilings are ones
the library accepts, balanced batch tilings cut every instance into tiles of
about the same size, and table lookups scale to untuned sizes."""
import pytest

from paper_0807_4471_amd import autotune


@pytest.mark.parametrize("n", [64, 100, 128, 250, 512, 1000, 4096])
@pytest.mark.parametrize("batch", [False, True])
def test_candidates_are_valid(n, batch):
    for c in autotune.candidates(n, n, batch):
        W, H, waves, stacked, th = c[:5]
        wt = c[5] if len(c) > 5 else 0
        assert th in (0, 1) and wt in (0, 1) and (stacked or not wt) and not (batch and wt)
        if stacked:
            assert waves in ((4,) if batch else (4, 8)) and H == waves and W <= 60
        else:
            assert waves in ((4,) if batch else (1, 2, 4))
            assert W <= 64 * waves - 4 and min(4, n) <= H <= max(n, 4)
        assert min(32, n) <= W <= n


@pytest.mark.parametrize("per_wg", [1, 3, 6])
def test_balanced_tilings(per_wg):
    shapes = [(128, 128), (192, 192), (256, 256), (384, 384), (512, 512), (64, 40)]
    cap = 768
    tl = autotune.balanced_tilings(shapes, cap, per_wg)
    target = sum(a * b for a, b in shapes) / (cap * per_wg)
    tiles = 0
    for (nx, ny), (W, H, waves, stacked, th) in zip(shapes, tl):
        assert waves == 4 and stacked == 0 and th == 0
        assert W <= 252 and -(-nx // W) == -(-nx // 252)
        assert min(4, ny) <= H <= ny
        if min(4, ny) < H < ny:       # not clamped: tile size near the target
            assert abs(W * H - target) <= W / 2 + 1
        tiles += -(-nx // W) * -(-ny // H)
    assert tiles >= 1


def test_tiling_for_scales_from_nearest_entry():
    table = {"f32/periodic/1024x1024": {"tiling": [205, 21, 4, 0, 0]},
             "f32/periodic/256x256": {"tiling": [52, 4, 4, 1, 0]}}
    assert autotune.tiling_for(1024, 1024, "f32", "periodic", table=table) == (205, 21, 4, 0, 0)
    W, H, waves, stacked, th = autotune.tiling_for(2048, 2048, "f32", "periodic", table=table)
    assert (waves, stacked) == (4, 0) and W <= 252 and H == 42
    assert autotune.tiling_for(300, 300, "f32", "periodic", table=table)[3] == 1
    assert autotune.tiling_for(300, 300, "f64", "periodic", table=table) is None
