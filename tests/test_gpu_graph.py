"""HIP graph replay of the fused step loop.

A graph recorded from lb_step(n) must advance the lattice exactly like n eager
steps, replay after replay, with the program's own eager work and
synchronisations between the replays.
"""

import pytest

from helpers import gpu_available
from paper_1703_00186_amd import workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1703_00186_amd.lb import LB


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_graph_replay_matches_eager(precision):
    lx, ly = 96, 130
    f = workload.rt_fields(lx, ly, seed=11)[:4]
    eager = LB(lx, ly, *f, precision=precision)
    graphed = LB(lx, ly, *f, precision=precision)
    g = graphed.capture(4)  # advances graphed by 2 warm-up steps
    eager.step(2)
    for _ in range(5):
        g.replay()
        eager.step(4)
        torch.cuda.synchronize()
        _ = graphed.moments()  # eager work on the same lattice between replays
        torch.cuda.synchronize()
        assert torch.equal(graphed.get_state(), eager.get_state())
