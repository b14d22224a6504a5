"""The HIP-graph-captured step equals the eager step, replay after replay."""
import numpy as np
import pytest

from paper_2410_09146_amd import inputs as I
from parity_util import say

pytestmark = pytest.mark.gpu


def test_graph_replays_equal_eager():
    import torch
    from paper_2410_09146_amd import grmhd as G
    prob = I.torus(n=(32, 32, 16))
    eager = G.Pack(prob)
    graph = G.Pack(prob)
    for p in (eager, graph):
        p.init()
        p.reductions(sync=False)
    for r in range(3):
        eager.step_c(None, cfl=prob.cfl)
        graph.step_graph(1)
        # eager work and a synchronisation between replays
        a, b = eager.download("P"), graph.download("P")
        ra, rb = eager.reductions(), graph.reductions()
        say("replay", r, "max |dP|", np.abs(a - b).max(), "dt", ra["dt"], rb["dt"])
        assert np.array_equal(a, b)
        assert np.array_equal(eager.download("Bf"), graph.download("Bf"))
        assert ra["dt"] == rb["dt"]
