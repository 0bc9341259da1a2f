"""The applies launch nothing but kernels on the caller's stream (no
allocation, no synchronisation, no memset), so they can be captured in a HIP
graph: D, D^dag and the fused 12-RHS apply captured once, replayed several
times with eager work and synchronisations in between, every replay equal
to the eager result bit for bit."""
import pytest

import synth
from tests.helpers import dev, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,nrhs", [((8, 8, 8, 8), 1), ((32, 16, 2, 4), 1), ((16, 6, 4, 4), 12)])
def test_graph_replays_match_eager(dims, nrhs):
    import torch
    import paper_1012_3615_amd as bri
    u = synth.gauge_links(dims, 0.3, 8601)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F32, 80)
    x = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 8602, nrhs=nrhs)), bri.F32)
    x2 = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 8603, nrhs=nrhs)), bri.F32)
    y, z = torch.empty_like(x), torch.empty_like(x)
    log(f"graph capture {dims} nrhs={nrhs}")
    ref_y = bri.bri_apply(dims, W, x, 0.1)
    ref_z = bri.bri_apply_dag(dims, W, ref_y, 0.1)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bri.bri_apply(dims, W, x, 0.1, out=y)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bri.bri_apply(dims, W, x, 0.1, out=y)
        bri.bri_apply_dag(dims, W, y, 0.1, out=z)
    for rep in range(3):
        y.zero_()
        z.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref_y) and torch.equal(z, ref_z), rep
        # eager work on other buffers between replays
        other = bri.bri_apply(dims, W, x2, 0.3)
        torch.cuda.synchronize()
        assert torch.isfinite(other).all()
