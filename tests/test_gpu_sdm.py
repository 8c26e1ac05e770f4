"""GPU parity of the two-point statistic (3-D displacement-vector
histogram) against the oracle, bit for bit, through the C ABI.

Cases: a small clustered needle (several species pairs, surface filter,
voxel counts 160 / 45 / 1); the same needle moved to coordinates around
3000 nm, where FP32 coordinates sit on a 2.4e-4 nm grid so that many
displacement components are exactly 0 (a face) or within 1e-5 nm of one;
the fcc lattice; coincident ions, NaN positions, empty species, n = 0;
the full 7.7e6-ion needle (Sc -> Al, R = 2 nm, 0.025 nm voxels).
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

    assert torch.cuda.is_available()
    aptstat.lib()
    return aptstat, torch, aptstat.Workspace()


def run_sdm(gpu, xyz, lab, d, A, B, d_srf, R, n_vox):
    aptstat, torch, ws = gpu
    dev = torch.device("cuda:0")
    cloud = aptstat.Cloud(torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).to(dev),
                          torch.from_numpy(np.ascontiguousarray(lab, np.uint8)).to(dev),
                          None if d is None else torch.from_numpy(np.ascontiguousarray(d, np.float32)).to(dev))
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    h = aptstat.sdm(cloud, A, B, d_srf, R, n_vox, ws=ws, status=st)
    torch.cuda.synchronize()
    return h.cpu().numpy().astype(np.uint64), int(st.item())


def check(orc, gpu, xyz, lab, d, A, B, d_srf, R, n_vox, expect_status=0):
    g, st = run_sdm(gpu, xyz, lab, d, A, B, d_srf, R, n_vox)
    assert st == expect_status
    ref = orc.sdm(xyz, lab, d, A, B, d_srf, R, n_vox)
    bad = np.argwhere(g != ref)
    assert len(bad) == 0, f"{len(bad)} voxels differ, first {bad[:5].tolist()}"
    return g


@pytest.fixture(scope="module")
def small_needle(synth):
    return synth.clustered_needle(40.0, 12.0, 8.0, noise=0.2, seed=5).generate()


@pytest.mark.parametrize("A,B,d_srf,R,n_vox", [
    (SC, AL, 1.0, 2.0, 160), (SC, SC, 1.0, 2.0, 160), (ANY, SI, 0.5, 1.5, 45), (AL, ANY, 2.0, 1.0, 1),
    (SI, SC, 0.0, 2.5, 100), (SC, ANY, 1.0, 0.6, 512),
])
def test_needle(gpu, orc, small_needle, A, B, d_srf, R, n_vox):
    _say(f"case sdm needle A={A} B={B} d_srf={d_srf} R={R} n={n_vox}")
    xyz, lab, d = small_needle
    g = check(orc, gpu, xyz, lab, d, A, B, d_srf, R, n_vox)
    assert g.sum() > 0


@pytest.mark.parametrize("A,B", [(SC, AL), (ANY, ANY)])
def test_far_coordinates_faces(gpu, orc, small_needle, A, B):
    # coordinates near 3000 nm: a 2.4e-4 nm FP32 grid, so many components are
    # exactly 0 (the face between voxels n/2 - 1 and n/2) or near a face
    _say(f"case sdm far coordinates A={A} B={B}")
    xyz, lab, d = small_needle
    far = (xyz.astype(np.float64) + 3000.0).astype(np.float32)
    dx = far[:, None, 0][:2000] - far[None, :2000, 0]
    assert (dx == 0).sum() > 2000            # many exact zero components
    check(orc, gpu, far, lab, d, A, B, 1.0, 2.0, 160)


def test_fcc_lattice(gpu, orc):
    _say("case sdm fcc lattice")
    a, M = 0.404, 14
    g = np.arange(2 * M)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    keep = (I + J + K) % 2 == 0
    xyz = (np.stack([I[keep], J[keep], K[keep]], 1) * (a / 2)).astype(np.float32)
    hi = (2 * M - 1) * a / 2
    d = np.minimum(xyz, hi - xyz).min(1).astype(np.float32)
    lab = np.zeros(len(xyz), np.uint8)
    h = check(orc, gpu, xyz, lab, d, AL, AL, 2.01, 2.0, 160)
    T = int((d >= np.float32(2.01)).sum())
    assert set(np.unique(h).tolist()) == {0, T} and int((h > 0).sum()) == 2092


def test_edge_cases(gpu, orc):
    _say("case sdm edge cases")
    xyz = np.array([[1, 1, 1], [1, 1, 1], [1.3, 1, 0.9], [np.nan, 1, 1], [1.2, 1.1, 1.0], [5, 5, 5]], np.float32)
    lab = np.array([SC, AL, AL, AL, SC, SC], np.uint8)
    # the NaN ion (an Al) sets the status bit when it is a target or neighbour
    for A, B, stat in ((SC, AL, 1), (SC, SC, 0), (ANY, ANY, 1), (SI, AL, 1), (AL, SI, 1)):
        check(orc, gpu, xyz, lab, None, A, B, 0.0, 1.0, 20, expect_status=stat)
    # coincident ions: v = 0 in the voxel (n/2, n/2, n/2)
    g, _ = run_sdm(gpu, xyz[:2], lab[:2], None, SC, AL, 0.0, 1.0, 20)
    assert g[10, 10, 10] == 1 and g.sum() == 1
    # no ions at all
    g, st = run_sdm(gpu, np.zeros((0, 3), np.float32), np.zeros(0, np.uint8), None, SC, AL, 0.0, 1.0, 8)
    assert g.sum() == 0 and st == 0


def test_repeat_determinism(gpu, small_needle):
    xyz, lab, d = small_needle
    a, _ = run_sdm(gpu, xyz, lab, d, SC, AL, 1.0, 2.0, 160)
    b, _ = run_sdm(gpu, xyz, lab, d, SC, AL, 1.0, 2.0, 160)
    assert np.array_equal(a, b)


def test_frustum7m_sc_al(gpu, orc, synth):
    _say("case sdm frustum7m Sc->Al R=2 n=160")
    xyz, lab, d = synth.frustum7m().generate()
    g = check(orc, gpu, xyz, lab, d, SC, AL, 1.0, 2.0, 160)
    # the voxel sum is the RDF's pair count within R
    assert int(g.sum()) == int(orc.rdf(xyz, lab, d, SC, AL, 1.0, 2.0, 1).sum())
