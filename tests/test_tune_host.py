"""Host logic of the autotuner (no device): candidate lists and the sample shape."""
from paper_2208_06194_amd import tune


def test_default_candidates():
    c = tune.default_candidates(1000)
    assert all(b <= 1000 for b, _, _ in c)
    assert (512, "tiled", 16) in c and (512, "tiled", 32) not in c
    assert (256, "block_column", 32) in c and (1024, "block_column", 16) not in c
    assert {v for _, v, _ in c} == {"block_column", "tiled"}


def test_sample_shape_is_a_tile_multiple_with_the_aspect_ratio():
    cands = [(128, "block_column", 16), (256, "block_column", 16), (1024, "tiled", 16)]
    ms, ns = tune.sample_shape(131072, 65536, cands)
    assert ns == 16 * 1024 and ms == 2 * ns
    assert ms % 1024 == 0 and ns % 1024 == 0
    # a matrix smaller than the sample is taken whole (rounded to the tile multiples)
    ms, ns = tune.sample_shape(4096, 2048, cands)
    assert (ms, ns) == (4096, 2048)
    assert tune.dense_equiv_flops(4, 2) == 2.0 * 4 * 4 - 2.0 / 3.0 * 8
