"""The library's event profiler (needs a GPU): per-launch records of the
filter's SpMM passes, and pausing without losing or waiting for records."""
import pytest

from paper_2502_17632_amd import workload as W

pytestmark = pytest.mark.gpu

EQ4 = ([4.0] * 4, [1, 2, 4, 8], [0.25] * 4)


def test_profiler_records_pauses_and_resumes():
    import torch
    import paper_2502_17632_amd as gift
    nl = W.tiny()
    g = gift.build_graph(nl.num_cells, nl.net_ptr, nl.pin_cell, sigmas=[4.0])
    x = torch.tensor(W.make_signal(nl), dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    gift.profile_enable(True)
    try:
        gift.filter_placement(g, *EQ4, x, out=y)  # 8 passes: 7, then the final one
        gift.profile_pause(True)
        gift.filter_placement(g, *EQ4, x, out=y)  # not recorded
        gift.profile_pause(False)
        gift.filter_placement(g, *EQ4, x, out=y)
        torch.cuda.synchronize()
        sp = gift.profile_collect("spmm")
        fin = gift.profile_collect("spmm_final")
        assert sp["launches"] == 14 and fin["launches"] == 2, (sp, fin)
        assert sp["total_ms"] > 0.0 and sp["max_ms"] <= sp["total_ms"]
        assert sp["bytes"] > 0.0
        # collecting cleared the records
        assert gift.profile_collect("spmm")["launches"] == 0
        # paused on its own: nothing is recorded until resumed
        gift.profile_pause(True)
        gift.filter_placement(g, *EQ4, x, out=y)
        torch.cuda.synchronize()
        assert gift.profile_collect("spmm")["launches"] == 0
    finally:
        gift.profile_enable(False)
    # profiling off: nothing is recorded
    gift.filter_placement(g, *EQ4, x, out=y)
    torch.cuda.synchronize()
    assert gift.profile_collect("spmm")["launches"] == 0
    g.close()
