"""The coupled substep captured in a HIP graph gives the eager result on every
replay, with eager work and synchronisations between replays, with the
phases on one stream and with the wind branch on a second stream."""
import pytest
import torch

from paper_2603_09668_amd import scenes
from paper_2603_09668_amd.sim import CoupledSim

from gpu_util import rel, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("concurrent", [False, True])
def test_graph_replays_match_eager(concurrent):
    """Serial graph and the graph with the wind and particle branches on two
    streams."""
    sc = scenes.flag_and_leaves_scene(seed=4, n=20_000, res=32, n_clusters=4, lbm_dims=(32, 16, 16))
    eager = CoupledSim(sc)
    graphed = CoupledSim(sc)
    graphed.capture(2, concurrent=concurrent)
    for r in range(4):
        say(f"graph replay {r} concurrent={concurrent}")
        eager.step()
        eager.step()
        graphed.replay()
        torch.cuda.synchronize()
        assert int(graphed.t_a.item()) == int(eager.t_a.item()) == 2 * (r + 1)
        for name in ("x", "v", "C", "F"):
            # each sim stores its particles in its own cell-tile order
            a = graphed.in_scene_order(getattr(graphed.p, name))
            b = eager.in_scene_order(getattr(eager.p, name))
            den = b.abs().max().item()
            if den > 0:
                assert rel(a.cpu(), b.cpu()) < 1e-5, (r, name)
            else:
                assert a.abs().max().item() == 0
        assert rel(graphed.fa.cpu(), eager.fa.cpu()) < 1e-5
        assert torch.equal(graphed.solid, eager.solid)
        assert graphed.status() == 0 and eager.status() == 0
