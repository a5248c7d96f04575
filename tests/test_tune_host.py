"""Host logic of the batched-launch autotuner (no GPU)."""
from paper_2004_09211_amd import tune


def test_chunk_rows_uniform_and_balanced():
    assert tune.chunk_rows_for(256, 256, 1024, 256, False) == 1
    assert tune.chunk_rows_for(32, 32, 1024, 256, False) == 8
    assert tune.chunk_rows_for(32, 32, 1024, 4096, False) == 32  # clamped to the image
    assert tune.chunk_rows_for(64, 64, 4000, 1024, True) == 4     # 1024 * 1024/4000 px
    assert tune.chunk_rows_for(64, 64, 500, 256, True) == 8       # 256 * 1024/500 px
    assert tune.chunk_rows_for(256, 256, 4000, 64, True) == 1     # never below one row


def test_candidate_set():
    c = tune.candidates(256)
    assert {x["item_px"] for x in c} == set(tune.PIXEL_TARGETS)
    assert any(x["balanced"] for x in c) and any(not x["balanced"] for x in c)
    assert {x["blocks"] for x in c} >= {0, 512, 2048}
