"""The measurement hook for memory ceilings (gsk_stream_mix_ms) on the GPU."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0812_2769_amd import gsk
    return gsk


def test_stream_mix_times_every_supported_mix(G):
    n = 1 << 22
    for reads, writes in ((1, 0), (1, 1), (6, 2), (9, 1), (11, 2)):
        r = G.stream_mix(reads, writes, n, reps=3)
        assert r["best_ms"] > 0.0 and r["bytes"] == 8 * (reads + writes) * n
        assert 50.0 < r["GBs"] < 20000.0, r
    # a ragged n (a partial tile and rounded workgroup count)
    assert G.stream_mix(11, 2, 1000003, reps=2)["best_ms"] > 0.0


def test_stream_mix_rejects_other_mixes(G):
    with pytest.raises(G.GskError):
        G.stream_mix(2, 2, 1 << 20)
    with pytest.raises(G.GskError):
        G.stream_mix(11, 2, 0)
