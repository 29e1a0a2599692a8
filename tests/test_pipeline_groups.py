"""CPU checks of the slab pipeline's launch grouping: contiguous chunks are
gathered into back-projection launches of at most `batch` views, and
chunks that do not continue each other start a new launch."""
import pytest

from paper_1909_02724_amd.pipeline import launch_groups


def test_contiguous_chunks_gathered():
    g = launch_groups(list(range(0, 4096, 16)), 16, 32, 4096)
    assert len(g) == 128 and all(len(x) == 2 for x in g)
    assert g[0] == [(0, 16), (16, 16)] and g[-1] == [(4064, 16), (4080, 16)]


def test_ragged_tail_and_gaps():
    assert launch_groups([0, 16, 32], 16, 32, 40) == [[(0, 16), (16, 16)], [(32, 8)]]
    assert launch_groups([0, 1024, 2048], 16, 32, 4096) == [[(0, 16)], [(1024, 16)], [(2048, 16)]]
    assert launch_groups([0, 16, 32], 16, 16, 48) == [[(0, 16)], [(16, 16)], [(32, 16)]]


def test_batch_not_multiple_of_chunk():
    # 16-view chunks in launches of at most 40 views: two chunks per launch
    assert launch_groups([0, 16, 32, 48], 16, 40, 64) == [[(0, 16), (16, 16)], [(32, 16), (48, 16)]]


def test_chunk_outside_scan_rejected():
    with pytest.raises(ValueError):
        launch_groups([0, 64], 16, 32, 64)
