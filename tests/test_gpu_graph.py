"""Library calls recorded into a HIP graph and replayed: every replay must give the
eager result, with other eager work and synchronisations between replays."""
import numpy as np
import pytest

from paper_2305_14306_amd import synth

pytestmark = pytest.mark.gpu


def test_graph_replays_chain_and_batch(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_14306_amd import hav
    s = torch.cuda.Stream()
    x = synth.lidar_scan()
    xd = torch.from_numpy(x).cuda()
    Ms = [16384, 4096, 1024, 256]
    chain_s = hav.Sampler()
    out = torch.empty(sum(Ms), dtype=torch.int32, device="cuda")
    clouds, bMs = synth.batch_lidar_clouds(n_clouds=5, n_min=3000, n_max=30000)
    offs = np.concatenate([[0], np.cumsum([c.shape[0] for c in clouds])])
    xb = torch.from_numpy(np.concatenate(clouds)).cuda()
    batch_s = hav.Sampler()
    outb = torch.empty(sum(bMs), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    def calls():
        chain_s.chain(xd, Ms, out=out, stream=s)
        batch_s.sample_batch(xb, offs, bMs, out=outb, stream=s)

    calls()  # eager: initialises the workspaces
    s.synchronize()
    eager, eagerb = out.clone(), outb.clone()
    st, want, _ = orc.chain(x, Ms)
    assert st == 0 and np.array_equal(eager.cpu().numpy(), np.concatenate(want))
    g = hav.Graph.capture(s, calls)
    other = hav.Sampler()
    y = torch.from_numpy(synth.random_cloud(20000, 3)).cuda()
    for rep in range(4):
        out.fill_(-1)
        outb.fill_(-1)
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        assert torch.equal(out, eager), rep
        assert torch.equal(outb, eagerb), rep
        other.sample(y, 5000)  # eager work between replays
        torch.cuda.synchronize()
    g.close()
