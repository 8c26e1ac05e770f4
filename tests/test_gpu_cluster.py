"""GPU parity of the maximum-separation clustering against the oracle,
through the C ABI: labels, counts and size histograms bit for bit.

Cases: a small clustered needle (Sc at several d_max and N_min, with the
edge filter for truncated clusters; every ion at small d_max, where links
percolate through the cloud); the same needle at coordinates around
3000 nm; an exact chain at the inclusive threshold and one ulp below; a
simple cubic lattice linked into one cluster; NaN positions, no ion of the
species, N_min above every cluster, n = 0; the full 7.7e6-ion needle over
the benchmark's d_max sweep (0.10 to 0.70 nm in 0.05 nm steps, N_min = 5)
and with every ion at d_max = 0.25 nm.
"""
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

    assert torch.cuda.is_available()
    aptstat.lib()
    return aptstat, torch, aptstat.Workspace()


def run_ms(gpu, xyz, lab, d, A, d_max, n_min, d_srf=0.0, n_size_bins=64):
    aptstat, torch, ws = gpu
    dev = torch.device("cuda:0")
    cloud = aptstat.Cloud(torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).to(dev),
                          torch.from_numpy(np.ascontiguousarray(lab, np.uint8)).to(dev),
                          None if d is None else torch.from_numpy(np.ascontiguousarray(d, np.float32)).to(dev))
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    label, counts, hist, st = aptstat.cluster_ms(cloud, A, d_max, n_min, d_srf, n_size_bins, ws=ws, status=st)
    torch.cuda.synchronize()
    return (label.cpu().numpy(), counts.cpu().numpy(), None if hist is None else hist.cpu().numpy().astype(np.uint64),
            int(st.item()))


def check(orc, gpu, xyz, lab, d, A, d_max, n_min, d_srf=0.0, n_size_bins=64, expect_status=0):
    gl, gc, gh, st = run_ms(gpu, xyz, lab, d, A, d_max, n_min, d_srf, n_size_bins)
    assert st == expect_status
    ol, oc, oh = orc.cluster_ms(xyz, lab, d, A, d_max, n_min, d_srf, n_size_bins)
    bad = np.flatnonzero(gl != ol)
    assert len(bad) == 0, f"{len(bad)} labels differ, first {bad[:5].tolist()}: gpu {gl[bad[:5]]} oracle {ol[bad[:5]]}"
    assert np.array_equal(gc, oc), (gc, oc)
    if n_size_bins:
        assert np.array_equal(gh, oh)
    return gl, gc


@pytest.fixture(scope="module")
def small_needle(synth):
    return synth.clustered_needle(40.0, 12.0, 8.0, noise=0.2, seed=5).generate()


@pytest.mark.parametrize("A,d_max,n_min,d_srf", [
    (SC, 0.3, 1, 0.0), (SC, 0.5, 5, 1.0), (SC, 0.7, 5, 2.0), (SC, 1.0, 10, 1.0), (SI, 0.6, 3, 0.5),
    (ANY, 0.2, 2, 1.0), (ANY, 0.32, 5, 1.0), (AL, 0.27, 20, 0.0),
])
def test_needle(gpu, orc, small_needle, A, d_max, n_min, d_srf):
    _say(f"case cluster needle A={A} d_max={d_max} n_min={n_min}")
    xyz, lab, d = small_needle
    _, c = check(orc, gpu, xyz, lab, d, A, d_max, n_min, d_srf)
    assert c[0] > 0


def test_far_coordinates(gpu, orc, small_needle):
    _say("case cluster far coordinates")
    xyz, lab, d = small_needle
    far = (xyz.astype(np.float64) + np.array([3000.0, -2500.0, 3100.0])).astype(np.float32)
    for d_max in (0.45, 0.8):
        check(orc, gpu, far, lab, d, SC, d_max, 3, 1.0)


def test_chain_threshold_and_lattice(gpu, orc):
    _say("case cluster chain and lattice")
    n = 33
    xyz = np.zeros((n, 3), np.float32)
    xyz[:, 0] = np.arange(n, dtype=np.float32) * np.float32(0.5) + np.float32(2.0)
    lab = np.full(n, SC, np.uint8)
    gl, gc = check(orc, gpu, xyz, lab, None, SC, 0.5, 2)
    assert (gl == 0).all() and gc[0] == 1
    below = float(np.nextafter(np.float32(0.5), np.float32(0)))
    gl, gc = check(orc, gpu, xyz, lab, None, SC, below, 1)
    assert np.array_equal(gl, np.arange(n))
    # a simple cubic lattice at the threshold spacing: one cluster of all
    g = np.arange(24, dtype=np.float32) * np.float32(0.5)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    lat = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    perm = np.random.default_rng(9).permutation(len(lat))
    lat = lat[perm]
    labl = np.full(len(lat), AL, np.uint8)
    gl, gc = check(orc, gpu, lat, labl, None, AL, 0.5, 10, n_size_bins=2)
    assert gc[0] == 1 and (gl == 0).all()


def test_edge_cases(gpu, orc, small_needle):
    _say("case cluster edge cases")
    xyz, lab, d = small_needle
    bad = xyz.copy()
    sc = np.flatnonzero(lab == SC)
    bad[sc[:7]] = np.nan
    check(orc, gpu, bad, lab, d, SC, 0.6, 1, 1.0, expect_status=1)
    # no ion of the species
    gl, gc = check(orc, gpu, xyz, lab, d, 7, 0.6, 1)
    assert (gl == -1).all() and (gc == 0).all()
    # N_min above every cluster
    gl, gc = check(orc, gpu, xyz, lab, d, SC, 0.4, 100000)
    assert (gl == -1).all() and gc[0] == 0
    # no ions at all
    gl, gc, gh, st = run_ms(gpu, np.zeros((0, 3), np.float32), np.zeros(0, np.uint8), None, SC, 0.5, 1)
    assert len(gl) == 0 and (gc == 0).all() and gh.sum() == 0 and st == 0


def test_repeat_determinism(gpu, small_needle):
    xyz, lab, d = small_needle
    a = run_ms(gpu, xyz, lab, d, ANY, 0.3, 2, 1.0)
    b = run_ms(gpu, xyz, lab, d, ANY, 0.3, 2, 1.0)
    assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3]))


def test_frustum7m_sweep(gpu, orc, synth):
    xyz, lab, d = synth.frustum7m().generate()
    for d_max in np.round(np.arange(0.10, 0.7001, 0.05), 2):
        _say(f"case cluster frustum7m Sc d_max={d_max}")
        check(orc, gpu, xyz, lab, d, SC, float(d_max), 5, 1.0, n_size_bins=200)
    _say("case cluster frustum7m every ion d_max=0.25")
    _, c = check(orc, gpu, xyz, lab, d, ANY, 0.25, 5, 1.0, n_size_bins=200)
    assert c[0] > 100
