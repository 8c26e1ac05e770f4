"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Histograms, kNN identities and target rows must be bit-exact; kNN distances
agree within 1e-6 relative (they are the FP32 square roots of identical FP32
squared distances).  Inputs are seeded synthetic clouds from aptsynth plus
hand-made edge cases.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

AL, SC, SI, ANY = 0, 1, 2, 255


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_2004_05188_amd as aptstat

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    aptstat.lib()
    return aptstat, torch, aptstat.Workspace()


def _to_dev(torch, xyz, lab, d):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).to(dev),
            torch.from_numpy(np.ascontiguousarray(lab, np.uint8)).to(dev),
            None if d is None else torch.from_numpy(np.ascontiguousarray(d, np.float32)).to(dev))


def run_gpu(gpu, xyz, lab, d, A, B, d_srf, k=10, r_max=2.0, n_bins=200, r_knn_max=math.inf,
            kb_rmax=5.0, kb_nbins=5000, capacity=None, want_rdf=True, k_on=True):
    aptstat, torch, ws = gpu
    cloud = aptstat.Cloud(*_to_dev(torch, xyz, lab, d))
    out = {}
    if k_on:
        r = aptstat.knn_rdf(cloud, A, B, d_srf, k, r_max=r_max, n_bins=n_bins, r_knn_max=r_knn_max,
                            capacity=capacity, kb_rmax=kb_rmax, kb_nbins=kb_nbins, want_rdf=want_rdf, ws=ws)
        torch.cuda.synchronize()
        nt = int(r.n_targets.item())
        cap = r.target_id.shape[0] if capacity is None else capacity
        t = min(nt, cap)
        out.update(n_targets=nt, tid=r.target_id[:t].cpu().numpy(), dist=r.dist[:t].cpu().numpy(),
                   nid=r.nbr_id[:t].cpu().numpy(), khist=r.knn_hist.cpu().numpy().astype(np.uint64),
                   status=int(r.status.item()))
        if want_rdf:
            out["rdf"] = r.rdf_hist.cpu().numpy().astype(np.uint64)
    else:
        status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        h = aptstat.rdf(cloud, A, B, d_srf, r_max, n_bins, ws=ws, status=status)
        torch.cuda.synchronize()
        out.update(rdf=h.cpu().numpy().astype(np.uint64), status=int(status.item()))
    return out


def check_against_oracle(orc, g, xyz, lab, d, A, B, d_srf, k=10, r_max=2.0, n_bins=200,
                         r_knn_max=math.inf, kb_rmax=5.0, kb_nbins=5000, want_rdf=True, k_on=True):
    if want_rdf:
        ref = orc.rdf(xyz, lab, d, A, B, d_srf, r_max, n_bins)
        assert np.array_equal(g["rdf"], ref), f"RDF differs in {np.count_nonzero(g['rdf'] != ref)} bins"
    if k_on:
        tid, dist, nid, kh = orc.knn(xyz, lab, d, A, B, d_srf, k, r_knn_max, kb_rmax, kb_nbins)
        assert g["n_targets"] == len(tid)
        assert np.array_equal(g["tid"], tid[: len(g["tid"])])
        assert np.array_equal(g["nid"], nid[: len(g["nid"])]), "kNN identities differ"
        gd, od = g["dist"], dist[: len(g["dist"])]
        assert np.array_equal(np.isinf(gd), np.isinf(od))
        fin = np.isfinite(od)
        assert np.all(np.abs(gd[fin] - od[fin]) <= 1e-6 * np.abs(od[fin])), "kNN distances differ"
        assert np.array_equal(g["khist"], kh), "k-th distance histogram differs"


# ---------------------------------------------------------------------------
# synthetic workloads
# ---------------------------------------------------------------------------

def test_box240k_sc_sc_knn10_rdf(gpu, orc, synth):
    _say("case box240k Sc->Sc k=10 rdf 2nm/200")
    xyz, lab, _ = synth.box240k().generate()
    g = run_gpu(gpu, xyz, lab, None, SC, SC, 0.0)
    assert g["status"] == 0
    check_against_oracle(orc, g, xyz, lab, None, SC, SC, 0.0)


@pytest.fixture(scope="module")
def small_needle(synth):
    spec = synth.clustered_needle(40.0, 12.0, 8.0, noise=0.2, seed=5)
    return spec.generate()


@pytest.mark.parametrize("A,B,k,d_srf,r_knn_max", [
    (SC, SC, 10, 1.0, math.inf), (SC, AL, 10, 1.0, math.inf), (SI, SC, 10, 1.0, math.inf),
    (AL, SC, 10, 1.0, math.inf), (SC, ANY, 1, 2.0, math.inf), (ANY, SI, 3, 0.5, math.inf),
    (SC, SI, 37, 1.0, math.inf), (SC, SC, 10, 1.0, 1.3), (SI, AL, 64, 0.0, math.inf),
    (SC, ANY, 100, 1.0, math.inf), (SI, SC, 100, 1.0, math.inf),
])
def test_needle_queries(gpu, orc, small_needle, A, B, k, d_srf, r_knn_max):
    _say(f"case needle A={A} B={B} k={k} d_srf={d_srf} rknn={r_knn_max}")
    xyz, lab, d = small_needle
    g = run_gpu(gpu, xyz, lab, d, A, B, d_srf, k=k, r_knn_max=r_knn_max)
    check_against_oracle(orc, g, xyz, lab, d, A, B, d_srf, k=k, r_knn_max=r_knn_max)


def test_rdf_only_and_knn_only_entry_points(gpu, orc, small_needle):
    _say("case needle apt_rdf and apt_knn alone")
    xyz, lab, d = small_needle
    g = run_gpu(gpu, xyz, lab, d, SC, AL, 1.0, k_on=False)
    check_against_oracle(orc, g, xyz, lab, d, SC, AL, 1.0, k_on=False)
    g = run_gpu(gpu, xyz, lab, d, SC, SC, 1.0, want_rdf=False)
    check_against_oracle(orc, g, xyz, lab, d, SC, SC, 1.0, want_rdf=False)


def test_large_bin_count_uses_global_histogram(gpu, orc, small_needle):
    _say("case needle rdf 5000 bins")
    xyz, lab, d = small_needle
    g = run_gpu(gpu, xyz, lab, d, SC, ANY, 1.0, k_on=False, r_max=2.5, n_bins=5000)
    check_against_oracle(orc, g, xyz, lab, d, SC, ANY, 1.0, r_max=2.5, n_bins=5000, k_on=False)


def test_candidate_count_bounds(gpu, orc, small_needle):
    """The diagnostic candidate count lies between the in-range pair count
    (every pair the RDF counts must be visited) and targets x neighbours and
    repeats exactly; no eligible target gives zero."""
    _say("case needle candidate counts")
    aptstat, torch, ws = gpu
    xyz, lab, d = small_needle
    cloud = aptstat.Cloud(*_to_dev(torch, xyz, lab, d))
    for A, B in ((SC, ANY), (SC, SC), (AL, SI)):
        n_t = len(orc.knn(xyz, lab, d, A, B, 1.0, 1, math.inf, 5.0, 10)[0])
        n_b = int(np.count_nonzero(lab == B)) if B != ANY else len(lab)
        for r_max, k in ((2.0, 0), (1.0, 0), (1.0, 10)):
            hits = int(orc.rdf(xyz, lab, d, A, B, 1.0, r_max, 200).sum())
            c = int(aptstat.count_candidates(cloud, A, B, 1.0, r_max, 200, k=k, ws=ws).item())
            assert hits <= c <= n_t * n_b, (A, B, r_max, k, hits, c, n_t * n_b)
            assert int(aptstat.count_candidates(cloud, A, B, 1.0, r_max, 200, k=k, ws=ws).item()) == c
    assert int(aptstat.count_candidates(cloud, SC, ANY, 1e6, ws=ws).item()) == 0


def test_deterministic_repeat(gpu, small_needle):
    _say("case needle repeat determinism")
    xyz, lab, d = small_needle
    a = run_gpu(gpu, xyz, lab, d, SC, ANY, 1.0)
    b = run_gpu(gpu, xyz, lab, d, SC, ANY, 1.0)
    for key in ("rdf", "tid", "nid", "dist", "khist"):
        assert np.array_equal(a[key], b[key])


# ---------------------------------------------------------------------------
# hand-made edge cases
# ---------------------------------------------------------------------------

def test_pairs_on_and_near_bin_edges(gpu, orc):
    _say("case bin edges")
    base = np.array([10.0, 10.0, 10.0])
    offs = [0.5, 1.0, 1.5, 0.25, 2.0, 0.5 + 1e-6, 0.5 - 1e-6, 1.0 + 3e-7, 1.0 - 3e-7, 2.0 - 1e-6,
            2.0 + 1e-6, 1.03, 0.01, 0.0, 1.9999999]
    pts = [base]
    for m, o in enumerate(offs):
        u = np.array([math.cos(0.3 * m), math.sin(0.3 * m), 0.0])
        pts.append(base + o * u)
    xyz = np.array(pts, np.float32)
    lab = np.full(len(xyz), SC, np.uint8)
    for A, B in ((SC, SC), (SC, ANY)):
        g = run_gpu(gpu, xyz, lab, None, A, B, 0.0, k=5)
        check_against_oracle(orc, g, xyz, lab, None, A, B, 0.0, k=5)


def test_coincident_ions_and_self_exclusion(gpu, orc):
    _say("case coincident")
    xyz = np.array([[1, 1, 1], [1, 1, 1], [1, 1, 1], [1.5, 1, 1], [3, 3, 3]], np.float32)
    lab = np.array([SC, SC, AL, AL, SC], np.uint8)
    for A, B in ((SC, ANY), (SC, SC), (ANY, ANY), (AL, SC)):
        g = run_gpu(gpu, xyz, lab, None, A, B, 0.0, k=3, r_max=1.0, n_bins=10)
        check_against_oracle(orc, g, xyz, lab, None, A, B, 0.0, k=3, r_max=1.0, n_bins=10)


def test_fewer_than_k_empty_species_and_no_targets(gpu, orc, synth):
    _say("case fewer than k / empty species")
    s = synth.Specimen(shape="box", L=(6.0, 6.0, 6.0), n=500, seed=13, p_m_sc=0.2)
    xyz, lab, d = s.generate()
    lab = lab.copy()
    lab[np.flatnonzero(lab == AL)[:3]] = SI                      # three Si only
    for A, B, k in ((SC, SI, 5), (SC, 77, 4), (77, SC, 4), (SI, SI, 5)):
        g = run_gpu(gpu, xyz, lab, d, A, B, 0.0, k=k)
        check_against_oracle(orc, g, xyz, lab, d, A, B, 0.0, k=k)


def test_surface_filter_inclusive_and_nan(gpu, orc, synth):
    _say("case d_bnd filter")
    s = synth.Specimen(shape="box", L=(8.0, 8.0, 8.0), n=3000, seed=17, p_m_sc=0.3)
    xyz, lab, d = s.generate()
    d = d.copy()
    d[::7] = 1.25                    # exactly d_srf: eligible
    d[3::11] = np.nan                # never eligible
    g = run_gpu(gpu, xyz, lab, d, SC, ANY, 1.25)
    check_against_oracle(orc, g, xyz, lab, d, SC, ANY, 1.25)


def test_nonfinite_positions_flagged(gpu, orc, synth):
    _say("case NaN/inf positions")
    s = synth.Specimen(shape="box", L=(8.0, 8.0, 8.0), n=3000, seed=19, p_m_sc=0.3)
    xyz, lab, d = s.generate()
    xyz = xyz.copy()
    xyz[5, 0] = np.nan
    xyz[np.flatnonzero(lab == SC)[3], 2] = np.inf
    g = run_gpu(gpu, xyz, lab, None, SC, ANY, 0.0, k=4)
    assert g["status"] & 1
    check_against_oracle(orc, g, xyz, lab, None, SC, ANY, 0.0, k=4)


def test_capacity_smaller_than_targets(gpu, orc, synth):
    _say("case capacity")
    s = synth.Specimen(shape="box", L=(8.0, 8.0, 8.0), n=3000, seed=23, p_m_sc=0.3)
    xyz, lab, d = s.generate()
    g = run_gpu(gpu, xyz, lab, None, SC, SC, 0.0, k=4, capacity=50)
    assert g["status"] & 2
    assert len(g["tid"]) == 50
    check_against_oracle(orc, g, xyz, lab, None, SC, SC, 0.0, k=4)


def test_empty_and_single_ion_clouds(gpu, orc):
    _say("case n=0 and n=1")
    for n in (0, 1):
        xyz = np.zeros((n, 3), np.float32) + 3.0
        lab = np.full(n, SC, np.uint8)
        g = run_gpu(gpu, xyz, lab, None, SC, SC, 0.0, k=2, capacity=max(n, 1))
        assert g["n_targets"] == n
        assert g["rdf"].sum() == 0
        if n:
            assert np.all(g["nid"] == -1)


def test_fcc_lattice_ties_and_near_edge_shell(gpu, orc):
    _say("case fcc lattice")
    a, M = 0.404, 12
    r = np.arange(2 * M)
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    keep = (I + J + K) % 2 == 0
    xyz = (np.stack([I[keep], J[keep], K[keep]], 1) * (a / 2)).astype(np.float32)
    rng = np.random.default_rng(3)
    xyz = xyz[rng.permutation(len(xyz))]
    hi = (2 * M - 1) * a / 2
    d = np.minimum(xyz, hi - xyz).min(1).astype(np.float32)
    lab = np.zeros(len(xyz), np.uint8)
    g = run_gpu(gpu, xyz, lab, d, AL, AL, 2.01, k=14)
    check_against_oracle(orc, g, xyz, lab, d, AL, AL, 2.01, k=14)


def test_exact_lattice_index_tiebreak(gpu, orc):
    _say("case simple cubic ties")
    gl = np.arange(9, dtype=np.float32) * 0.5
    X, Y, Z = np.meshgrid(gl, gl, gl, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    xyz = xyz[np.random.default_rng(4).permutation(len(xyz))]
    lab = np.zeros(len(xyz), np.uint8)
    g = run_gpu(gpu, xyz, lab, None, AL, AL, 0.0, k=9, r_max=1.5, n_bins=6)
    check_against_oracle(orc, g, xyz, lab, None, AL, AL, 0.0, k=9, r_max=1.5, n_bins=6)


def test_flat_cloud_and_far_outlier(gpu, orc, synth):
    _say("case flat cloud with outlier")
    s = synth.Specimen(shape="box", L=(30.0, 30.0, 0.001), n=5000, seed=29, p_m_sc=0.2)
    xyz, lab, d = s.generate()
    xyz = xyz.copy()
    xyz[0] = (1e4, -1e4, 5e3)
    g = run_gpu(gpu, xyz, lab, None, SC, ANY, 0.0, k=6)
    check_against_oracle(orc, g, xyz, lab, None, SC, ANY, 0.0, k=6)


# ---------------------------------------------------------------------------
# full-size needle: 7 696 902 ions, the three queries of the workload
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def needle7m(synth):
    return synth.frustum7m().generate()


@pytest.mark.parametrize("A,B", [(SC, SC), (SC, AL), (SI, SC)])
def test_frustum7m_queries(gpu, orc, needle7m, A, B):
    _say(f"case frustum7m A={A} B={B} k=10 d_srf=1")
    xyz, lab, d = needle7m
    g = run_gpu(gpu, xyz, lab, d, A, B, 1.0, k=10)
    assert g["status"] == 0
    check_against_oracle(orc, g, xyz, lab, d, A, B, 1.0, k=10)


@pytest.mark.parametrize("A,B", [(SC, SC), (SC, AL), (SI, SC)])
def test_frustum7m_rdf_only(gpu, orc, needle7m, A, B):
    """apt_rdf alone (no kNN: its rows are walked in raster order)."""
    _say(f"case frustum7m rdf-only A={A} B={B} d_srf=1")
    xyz, lab, d = needle7m
    g = run_gpu(gpu, xyz, lab, d, A, B, 1.0, k_on=False)
    assert g["status"] == 0
    check_against_oracle(orc, g, xyz, lab, d, A, B, 1.0, k_on=False)


# ---------------------------------------------------------------------------
# label permutation (null model)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,seed", [(0, 1), (1, 5), (31, 7), (1000, 11), (2049, 3), (240_000, 2**64 - 1),
                                    (7_696_902, 123457), (16_777_216, 8), (17_000_000, 99)])
def test_permute_labels_bit_exact(gpu, orc, synth, n, seed):
    _say(f"case permute n={n} seed={seed}")
    aptstat, torch, ws = gpu
    if n == 7_696_902:
        _, lab, _ = synth.frustum7m().generate()
    else:
        lab = np.random.default_rng(n).integers(0, 4, n).astype(np.uint8)
    dl = torch.from_numpy(lab).to("cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    out = aptstat.permute_labels(dl, seed, ws=ws, status=status).cpu().numpy()
    assert int(status.item()) == 0
    assert np.array_equal(out, orc.permute_labels(lab, seed))


# ---------------------------------------------------------------------------
# batched null-model replicates
# ---------------------------------------------------------------------------

PAIRS6 = [(AL, SC), (AL, SI), (SC, AL), (SC, SI), (SI, AL), (SI, SC)]


def _looped(gpu, cloud_args, pairs, seeds, d_srf, r_max, n_bins, k, kb_rmax, kb_nbins):
    """The definition: plain calls on apt_permute_labels' labels."""
    aptstat, torch, ws = gpu
    xyz_t, lab_t, d_t = cloud_args
    out_r, out_k = [], []
    for sd in seeds:
        lab_r = aptstat.permute_labels(lab_t, sd, ws=ws)
        cloud = aptstat.Cloud(xyz_t, lab_r, d_t)
        rr, kk = [], []
        for A, B in pairs:
            r = aptstat.knn_rdf(cloud, A, B, d_srf, k, r_max=r_max, n_bins=n_bins, capacity=0,
                                kb_rmax=kb_rmax, kb_nbins=kb_nbins, ws=ws)
            rr.append(r.rdf_hist.clone())
            kk.append(r.knn_hist.clone())
        out_r.append(torch.stack(rr))
        out_k.append(torch.stack(kk))
    return torch.stack(out_r), torch.stack(out_k)


def test_batched_matches_oracle_on_permuted_labels(gpu, orc, small_needle):
    _say("case batched small needle vs oracle")
    aptstat, torch, ws = gpu
    xyz, lab, d = small_needle
    seeds = [101, 202, 303]
    pairs = [(A, B, 1.0) for A, B in PAIRS6]
    cloud = aptstat.Cloud(*_to_dev(torch, xyz, lab, d))
    rh, kh, st = aptstat.rdf_batched(cloud, pairs, seeds, r_max=2.0, n_bins=200, k=10, kb_rmax=5.0,
                                     kb_nbins=500, ws=ws)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    rh, kh = rh.cpu().numpy().astype(np.uint64), kh.cpu().numpy().astype(np.uint64)
    for r, sd in enumerate(seeds):
        lab_r = orc.permute_labels(lab, sd)
        for p, (A, B, ds) in enumerate(pairs):
            assert np.array_equal(rh[r, p], orc.rdf(xyz, lab_r, d, A, B, ds, 2.0, 200)), (r, p)
            assert np.array_equal(kh[r, p], orc.knn(xyz, lab_r, d, A, B, ds, 10, kb_rmax=5.0, kb_nbins=500)[3]), (r, p)


def test_batched_equals_looped_frustum7m(gpu, needle7m):
    _say("case batched frustum7m vs looped plain calls")
    aptstat, torch, ws = gpu
    xyz, lab, d = needle7m
    args = _to_dev(torch, xyz, lab, d)
    seeds = [7, 8]
    pairs = [(A, B, 1.0) for A, B in PAIRS6]
    rh, kh, st = aptstat.rdf_batched(aptstat.Cloud(*args), pairs, seeds, ws=ws)
    lr, lk = _looped(gpu, args, PAIRS6, seeds, 1.0, 2.0, 200, 10, 5.0, 5000)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert torch.equal(rh, lr) and torch.equal(kh, lk)


def test_batched_frustum7m_replicate_against_oracle(gpu, orc, needle7m):
    # the full-size batched call's first replicate, all six pairs, against
    # the oracle on the permuted labels
    _say("case batched frustum7m replicate 0 vs oracle, 6 pairs")
    aptstat, torch, ws = gpu
    xyz, lab, d = needle7m
    args = _to_dev(torch, xyz, lab, d)
    seeds = [7, 8]
    pairs = [(A, B, 1.0) for A, B in PAIRS6]
    rh, kh, st = aptstat.rdf_batched(aptstat.Cloud(*args), pairs, seeds, ws=ws)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    lab_r = orc.permute_labels(lab, seeds[0])
    assert np.array_equal(aptstat.permute_labels(args[1], seeds[0], ws=ws).cpu().numpy(), lab_r)
    for p, (A, B) in enumerate(PAIRS6):
        ref = orc.rdf(xyz, lab_r, d, A, B, 1.0, 2.0, 200)
        assert np.array_equal(rh[0, p].cpu().numpy().astype(np.uint64), ref), (A, B)
        kref = orc.knn(xyz, lab_r, d, A, B, 1.0, 10, kb_rmax=5.0, kb_nbins=5000)[3]
        assert np.array_equal(kh[0, p].cpu().numpy().astype(np.uint64), kref), (A, B)


def test_batched_many_replicates_cross_blocks(gpu, synth):
    _say("case batched 70 replicates (two launches)")
    aptstat, torch, ws = gpu
    s = synth.Specimen(shape="box", L=(12.0, 12.0, 12.0), n=20_000, seed=31, p_m_sc=0.05, p_m_si=0.1)
    xyz, lab, d = s.generate()
    args = _to_dev(torch, xyz, lab, d)
    seeds = list(range(1000, 1070))
    pairs = [(SC, SI), (SI, SI), (AL, SC)]
    rh, kh, st = aptstat.rdf_batched(aptstat.Cloud(*args), [(A, B, 0.5) for A, B in pairs], seeds,
                                     r_max=1.5, n_bins=30, k=3, kb_rmax=3.0, kb_nbins=60, ws=ws)
    lr, lk = _looped(gpu, args, pairs, seeds, 0.5, 1.5, 30, 3, 3.0, 60)
    torch.cuda.synchronize()
    assert torch.equal(rh, lr) and torch.equal(kh, lk)


def test_batched_lattice_ties_equal_looped(gpu, orc):
    """A simple cubic lattice (every distance shared by many pairs) with
    three species: dense Al targets take the tiles, whose k-th key is settled
    by the smallest index at the k-th distance, or left to the exact
    one-by-one search when the k-th distance is shared inside the k nearest.
    Equal to looped plain calls and to the oracle."""
    _say("case batched lattice ties")
    aptstat, torch, ws = gpu
    gl = np.arange(26, dtype=np.float32) * 0.5
    X, Y, Z = np.meshgrid(gl, gl, gl, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    rng = np.random.default_rng(12)
    xyz = xyz[rng.permutation(len(xyz))]
    lab = rng.choice(np.array([AL, SC, SI], np.uint8), len(xyz), p=[0.9, 0.04, 0.06])
    hi = 12.5
    d = np.minimum(xyz, hi - xyz).min(1).astype(np.float32)
    args = _to_dev(torch, xyz, lab, d)
    seeds = [5, 6, 7]
    pairs = [(AL, SC), (AL, SI), (SC, AL)]
    for k in (1, 6, 10):
        rh, kh, st = aptstat.rdf_batched(aptstat.Cloud(*args), [(A, B, 1.0) for A, B in pairs], seeds,
                                         r_max=2.0, n_bins=40, k=k, kb_rmax=3.0, kb_nbins=300, ws=ws)
        lr, lk = _looped(gpu, args, pairs, seeds, 1.0, 2.0, 40, k, 3.0, 300)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert torch.equal(rh, lr) and torch.equal(kh, lk), k
        lab_r = orc.permute_labels(lab, seeds[0])
        for p, (A, B) in enumerate(pairs):
            ok = orc.knn(xyz, lab_r, d, A, B, 1.0, k, kb_rmax=3.0, kb_nbins=300)[3]
            assert np.array_equal(kh[0, p].cpu().numpy().astype(np.uint64), ok), (k, p)


# ---------------------------------------------------------------------------
# one target per wavefront, 64 per wavefront sharing candidates, one per lane,
# kNN per lane + RDF per wavefront: forced
# ---------------------------------------------------------------------------

@pytest.fixture()
def policy(gpu):
    aptstat = gpu[0]

    def set_mode(tile_policy):
        # 42: the dense-neighbour mode (4) with its RDF one target per wavefront
        if tile_policy == 42:
            aptstat.set_tuning(tile_policy=4, rdf_kernel=2)
        else:
            aptstat.set_tuning(tile_policy=tile_policy)

    yield set_mode
    aptstat.set_tuning()          # back to the defaults


@pytest.mark.parametrize("mode", [1, 2, 3, 4, 42])
@pytest.mark.parametrize("A,B,k,d_srf,r_knn_max,rdf", [
    (SC, SC, 10, 1.0, math.inf, True), (AL, SC, 10, 1.0, math.inf, True), (AL, SI, 4, 1.0, math.inf, True),
    (ANY, SC, 1, 0.5, math.inf, True), (SC, ANY, 16, 1.0, math.inf, True), (AL, SC, 10, 1.0, 1.2, True),
    (AL, AL, 3, 2.0, math.inf, True), (AL, SC, 7, 1.0, math.inf, False), (SI, SI, 12, 0.0, math.inf, True),
])
def test_needle_queries_forced_mode(gpu, orc, small_needle, policy, mode, A, B, k, d_srf, r_knn_max, rdf):
    _say(f"case needle mode={mode} A={A} B={B} k={k} d_srf={d_srf} rknn={r_knn_max} rdf={rdf}")
    policy(mode)
    xyz, lab, d = small_needle
    g = run_gpu(gpu, xyz, lab, d, A, B, d_srf, k=k, r_knn_max=r_knn_max, want_rdf=rdf)
    check_against_oracle(orc, g, xyz, lab, d, A, B, d_srf, k=k, r_knn_max=r_knn_max, want_rdf=rdf)


@pytest.mark.parametrize("mode", [1, 2, 3, 4, 42])
def test_rdf_only_forced_mode(gpu, orc, small_needle, policy, mode):
    _say(f"case needle rdf-only mode={mode}")
    policy(mode)
    xyz, lab, d = small_needle
    g = run_gpu(gpu, xyz, lab, d, AL, SC, 1.0, k_on=False)
    check_against_oracle(orc, g, xyz, lab, d, AL, SC, 1.0, k_on=False)


@pytest.mark.parametrize("mode", [1, 2, 3, 4, 42])
def test_edge_cases_forced_mode(gpu, orc, synth, policy, mode):
    _say(f"case edge cases mode={mode}")
    policy(mode)
    xyz = np.array([[1, 1, 1], [1, 1, 1], [1, 1, 1], [1.5, 1, 1], [3, 3, 3], [np.nan, 0, 0]], np.float32)
    lab = np.array([SC, SC, AL, AL, SC, SC], np.uint8)
    for A, B in ((SC, ANY), (SC, SC), (ANY, ANY), (AL, SC)):
        g = run_gpu(gpu, xyz, lab, None, A, B, 0.0, k=3, r_max=1.0, n_bins=10)
        check_against_oracle(orc, g, xyz, lab, None, A, B, 0.0, k=3, r_max=1.0, n_bins=10)
    s = synth.Specimen(shape="box", L=(8.0, 8.0, 8.0), n=3000, seed=23, p_m_sc=0.3)
    xyz, lab, d = s.generate()
    g = run_gpu(gpu, xyz, lab, None, AL, SC, 0.0, k=4, capacity=50)
    check_against_oracle(orc, g, xyz, lab, None, AL, SC, 0.0, k=4)


@pytest.mark.parametrize("A,B", [(AL, SC), (AL, SI)])
def test_frustum7m_dense_targets(gpu, orc, needle7m, A, B):
    _say(f"case frustum7m dense targets A={A} B={B} (automatic mode)")
    xyz, lab, d = needle7m
    g = run_gpu(gpu, xyz, lab, d, A, B, 1.0, k=10)
    assert g["status"] == 0
    check_against_oracle(orc, g, xyz, lab, d, A, B, 1.0, k=10)
