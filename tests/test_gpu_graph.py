"""GPU: the entry points can be captured in a HIP graph.

Every call only enqueues kernels on the caller's stream (no allocation, no
memset node, no host synchronisation), so a caller may capture it, here
with torch.cuda.CUDAGraph.  A batched null-model call and a plain kNN + RDF
call are captured once and replayed three times, with other eager library
work and synchronisations between the replays; the outputs are poisoned
before each replay, and every replay must equal the eager results bit for
bit.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

AL, SC, SI, ANY = 0, 1, 2, 255


def test_batched_and_plain_calls_replay_from_a_graph(synth):
    import torch

    import paper_2004_05188_amd as aptstat

    assert torch.cuda.is_available()
    print("case graph capture: clustered needle 40 x 12 -> 8 nm, batched 6 pairs x 8 seeds, knn_rdf Sc->any",
          flush=True)
    xyz, lab, d = synth.clustered_needle(40.0, 12.0, 8.0, noise=0.2, seed=5).generate()
    dev = torch.device("cuda:0")
    cloud = aptstat.Cloud(torch.from_numpy(xyz).to(dev), torch.from_numpy(lab).to(dev),
                          torch.from_numpy(d).to(dev))
    pairs = [(a, b, 1.0) for a, b in [(AL, SC), (AL, SI), (SC, AL), (SC, SI), (SI, AL), (SI, SC)]]
    seeds = list(range(101, 109))
    ws_b, ws_p = aptstat.Workspace(), aptstat.Workspace()
    cap = int(aptstat.count_targets(cloud, SC, 1.0, ws=ws_p).item())

    # eager results (also sizes both workspaces before the capture)
    rh0, kh0, st0 = aptstat.rdf_batched(cloud, pairs, seeds, kb_nbins=500, ws=ws_b)
    r0 = aptstat.knn_rdf(cloud, SC, ANY, 1.0, 10, capacity=cap, kb_nbins=500, ws=ws_p)
    torch.cuda.synchronize()
    want = [t.clone() for t in (rh0, kh0, st0, r0.rdf_hist, r0.knn_hist, r0.dist, r0.nbr_id, r0.target_id,
                                r0.n_targets, r0.status)]
    assert int(st0.item()) == 0 and int(r0.status.item()) == 0

    # static outputs the graph writes
    rh, kh, st = torch.empty_like(rh0), torch.empty_like(kh0), torch.empty_like(st0)
    outs = tuple(torch.empty_like(t) for t in (r0.target_id, r0.dist, r0.nbr_id, r0.knn_hist, r0.n_targets,
                                                r0.status, r0.rdf_hist))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # warm-up on the capture stream, as torch recommends
        aptstat.rdf_batched(cloud, pairs, seeds, kb_nbins=500, ws=ws_b, out=(rh, kh, st))
        aptstat.knn_rdf(cloud, SC, ANY, 1.0, 10, capacity=cap, kb_nbins=500, ws=ws_p, outputs=outs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        aptstat.rdf_batched(cloud, pairs, seeds, kb_nbins=500, ws=ws_b, out=(rh, kh, st))
        aptstat.knn_rdf(cloud, SC, ANY, 1.0, 10, capacity=cap, kb_nbins=500, ws=ws_p, outputs=outs)
    torch.cuda.synchronize()

    other = aptstat.Workspace()
    for rep in range(3):
        for t in (rh, kh, st) + outs:
            t.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [rh, kh, st, outs[6], outs[3], outs[1], outs[2], outs[0], outs[4], outs[5]]
        for w, x in zip(want, got):
            assert torch.equal(w, x), f"replay {rep} differs from the eager call"
        # eager library work between replays, on its own workspace
        aptstat.rdf(cloud, SI, AL, 1.0, 2.0, 200, ws=other)
        torch.cuda.synchronize()
    print(f"graph replays equal the eager results; rdf total {int(np.asarray(want[3].cpu()).sum())}",
          flush=True)
