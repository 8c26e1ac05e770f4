"""GPU: the autotuner only changes speed.

It times a small grid of tunings on a seeded clustered needle and keeps the
fastest; the kNN rows and histograms computed under the chosen tuning must
equal those under the defaults bit for bit, and the choice must come from the
grid.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

AL, SC, SI, ANY = 0, 1, 2, 255


def _rows(aptstat, torch, cloud, ws, A, B):
    r = aptstat.knn_rdf(cloud, A, B, 1.0, 10, r_max=2.0, n_bins=200, kb_rmax=5.0, kb_nbins=500, ws=ws)
    torch.cuda.synchronize()
    assert int(r.status.item()) == 0
    t = int(r.n_targets.item())
    return (r.target_id[:t].cpu().numpy(), r.nbr_id[:t].cpu().numpy(), r.dist[:t].cpu().numpy(),
            r.rdf_hist.cpu().numpy(), r.knn_hist.cpu().numpy())


def test_autotune_keeps_results(synth):
    import torch

    import paper_2004_05188_amd as aptstat
    from paper_2004_05188_amd.autotune import autotune

    assert torch.cuda.is_available()
    spec = synth.clustered_needle(60.0, 12.0, 8.0, seed=7)
    xyz, lab, d = spec.generate()
    dev = torch.device("cuda:0")
    cloud = aptstat.Cloud(torch.from_numpy(xyz).to(dev), torch.from_numpy(lab).to(dev),
                          torch.from_numpy(d).to(dev))
    ws = aptstat.Workspace()
    queries = [(SC, ANY), (AL, SC)]
    aptstat.set_tuning()
    try:
        ref = [_rows(aptstat, torch, cloud, ws, A, B) for A, B in queries]
        grid = {"tile_policy": (1, 2), "cell_occ": (2.0, 4.0), "h_min_frac": (0.5,)}
        res = autotune(cloud, queries, d_srf=1.0, k=10, r_max=2.0, n_bins=200, grid=grid, reps=2, ws=ws)
        best = res["best"]
        assert best["tile_policy"] in (1, 2) and best["cell_occ"] in (2.0, 4.0)
        # tile_policy 2 ignores cell_occ: three distinct settings
        assert len(res["ms"]) == 3 and all(v > 0 for v in res["ms"].values())
        assert aptstat.get_tuning()["tile_policy"] == best["tile_policy"]
        for (A, B), want in zip(queries, ref):
            got = _rows(aptstat, torch, cloud, ws, A, B)
            for g, w in zip(got, want):
                assert np.array_equal(g, w)
    finally:
        aptstat.set_tuning()
