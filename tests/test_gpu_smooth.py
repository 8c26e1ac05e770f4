"""GPU parity of the Gaussian-smoothed RDF and its adjoint against the FP64
CPU oracle, finite differences and invariants.

Bars: forward per bin within 1e-12 relative of the oracle (both FP64, the
same expressions; only erfc's last bits and the summation order differ);
gradients within 1e-4 relative of the oracle (and, tighter, within the FP32
rounding of the returned gradient) and of central finite differences
(h = 1e-4 nm, truncation ~(h/sigma)^2/6 = 4e-6 per pair): in norm for the
plain differences, per component for their Richardson extrapolation.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

AL, SC, ANY = 0, 1, 255


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


def _dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).to("cuda:0")


def _cloud(gpu, xyz, lab, d=None):
    aptstat, torch, _ = gpu
    return aptstat.Cloud(_dev(torch, xyz, np.float32), _dev(torch, lab, np.uint8),
                         None if d is None else _dev(torch, d, np.float32))


def _zs(torch, s):
    return torch.tensor([s], dtype=torch.float64, device="cuda:0")


def gpu_fwd(gpu, cloud, A, B, d_srf, r_max, n_bins, sigma, s=1.0):
    aptstat, torch, ws = gpu
    st = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    h = aptstat.rdf_smooth(cloud, A, B, d_srf, r_max, n_bins, sigma, z_scale=_zs(torch, s), ws=ws, status=st)
    torch.cuda.synchronize()
    return h.cpu().numpy(), int(st.item())


def gpu_bwd(gpu, cloud, A, B, d_srf, r_max, n_bins, sigma, grad_h, s=1.0):
    aptstat, torch, ws = gpu
    gh = _dev(torch, grad_h, np.float64)
    gx, gs = aptstat.rdf_smooth_grad(cloud, A, B, d_srf, r_max, n_bins, sigma, gh, z_scale=_zs(torch, s), ws=ws)
    torch.cuda.synchronize()
    return gx.cpu().numpy(), float(gs.item())


def assert_fwd_close(h, ref):
    bad = np.abs(h - ref) > 1e-12 * np.abs(ref)
    assert not bad.any(), f"{bad.sum()} bins differ, worst {np.abs(h - ref)[bad].max()}"


def assert_grad_close(g, ref, tight=True):
    """g: FP32 from the GPU; ref: FP64 oracle (or finite differences)."""
    ref = np.asarray(ref, np.float64)
    g = np.asarray(g, np.float64)
    gmax = np.abs(ref).max()
    assert np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref)
    assert np.all(np.abs(g - ref) <= 1e-4 * np.maximum(np.abs(ref), 1e-3 * gmax))
    if tight:   # FP32 rounding of an FP64 result that agrees to ~1e-12
        assert np.all(np.abs(g - ref) <= 1.2e-7 * np.abs(ref) + 1e-11 * gmax)


def _box(synth, n, L, seed, p_m_sc=0.02, n_clusters=20, r_c=1.2):
    sp = synth.Specimen(shape="box", L=(L, L, L), n=n, seed=seed, p_m_sc=p_m_sc, p_c_sc=0.25,
                        n_clusters=n_clusters, r_c=r_c)
    xyz, lab, _ = sp.generate()
    d = np.minimum(xyz.min(1), L - xyz.max(1)).astype(np.float32)   # distance to the box faces
    return xyz, lab, d


PROBLEMS = [
    # (name, n, L, seed, query (A, B, use d_bnd, d_srf), r_max, n_bins, sigma)
    ("sc_sc", 120_000, 16.0, 11, (SC, SC, False, 0.0), 2.0, 200, 0.02),
    ("sc_any_dbnd", 30_000, 10.0, 12, (SC, ANY, True, 1.0), 2.0, 200, 0.02),
    ("al_sc_coarse", 30_000, 10.0, 13, (AL, SC, True, 0.5), 1.5, 37, 0.045),
    # windows wider than a wavefront (120 bins), histogram in registers
    ("sc_sc_wide", 30_000, 10.0, 14, (SC, SC, False, 0.0), 2.0, 200, 0.1),
    # more than 256 bins: histogram in LDS, windows of 180 bins
    ("sc_sc_fine_lds", 30_000, 10.0, 15, (SC, SC, False, 0.0), 2.0, 1000, 0.03),
]


@pytest.mark.parametrize("s", [1.0, 1.05])
@pytest.mark.parametrize("prob", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_smooth_forward_and_adjoint_match_oracle(gpu, orc, synth, prob, s):
    name, n, L, seed, (A, B, use_d, d_srf), r_max, n_bins, sigma = prob
    _say(f"smooth parity {name} s={s}")
    xyz, lab, d = _box(synth, n, L, seed)
    d = d if use_d else None
    cloud = _cloud(gpu, xyz, lab, d)
    h, st = gpu_fwd(gpu, cloud, A, B, d_srf, r_max, n_bins, sigma, s)
    assert st == 0
    ref = orc.smooth_fwd(xyz, lab, d, A, B, d_srf, r_max, n_bins, sigma, s)
    assert ref.sum() > 100
    assert_fwd_close(h, ref)
    gh = np.random.default_rng(seed).normal(size=n_bins)
    g, gs = gpu_bwd(gpu, cloud, A, B, d_srf, r_max, n_bins, sigma, gh, s)
    rg, rgs = orc.smooth_bwd(xyz, lab, d, A, B, d_srf, r_max, n_bins, sigma, s, gh)
    assert_grad_close(g, rg)
    assert abs(gs - rgs) <= 1e-9 * abs(rgs)


def test_smooth_is_reproducible_bit_for_bit(gpu, synth):
    xyz, lab, d = _box(synth, 120_000, 16.0, 14)
    cloud = _cloud(gpu, xyz, lab, d)
    gh = np.random.default_rng(1).normal(size=200)
    h1, _ = gpu_fwd(gpu, cloud, SC, ANY, 1.0, 2.0, 200, 0.02, 1.02)
    h2, _ = gpu_fwd(gpu, cloud, SC, ANY, 1.0, 2.0, 200, 0.02, 1.02)
    assert np.array_equal(h1.view(np.uint64), h2.view(np.uint64))
    g1, s1 = gpu_bwd(gpu, cloud, SC, ANY, 1.0, 2.0, 200, 0.02, gh, 1.02)
    g2, s2 = gpu_bwd(gpu, cloud, SC, ANY, 1.0, 2.0, 200, 0.02, gh, 1.02)
    assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32)) and s1 == s2


def test_smooth_adjoint_invariants(gpu, synth):
    xyz, lab, _ = _box(synth, 120_000, 16.0, 15)
    cloud = _cloud(gpu, xyz, lab)
    gh = np.random.default_rng(2).normal(size=200)
    P = xyz.astype(np.float64)
    for s in (1.0, 1.05):
        g, gs = gpu_bwd(gpu, cloud, SC, SC, 0.0, 2.0, 200, 0.02, gh, s)
        g = g.astype(np.float64)
        scale = np.abs(g).sum()
        assert np.abs(g.sum(0)).max() <= 1e-6 * scale            # translation (FP32 outputs)
        torque = np.cross(P, g).sum(0)
        assert abs(torque[2]) <= 1e-5 * (np.abs(P).max() * scale)
        if s == 1.0:
            assert np.abs(torque).max() <= 1e-5 * (np.abs(P).max() * scale)
        assert abs(gs - (P[:, 2] * g[:, 2]).sum() / s) <= 1e-6 * (abs(gs) + np.abs(P[:, 2] * g[:, 2]).sum())


def test_smooth_autograd_function(gpu, synth):
    aptstat, torch, _ = gpu
    xyz, lab, d = _box(synth, 30_000, 10.0, 16)
    X = _dev(torch, xyz, np.float32).requires_grad_(True)
    Z = torch.tensor(1.03, dtype=torch.float64, device="cuda:0", requires_grad=True)
    Lb, Db = _dev(torch, lab, np.uint8), _dev(torch, d, np.float32)
    t = torch.linspace(0, 50, 200, dtype=torch.float64, device="cuda:0")
    h = aptstat.RdfSmooth.apply(X, Z, Lb, Db, SC, ANY, 1.0, 2.0, 200, 0.02)
    assert h.dtype == torch.float64 and h.shape == (200,)
    loss = ((h - t) ** 2).sum()
    loss.backward()
    assert X.grad.dtype == torch.float32 and X.grad.shape == X.shape
    assert Z.grad.shape == Z.shape
    gx, gs = aptstat.rdf_smooth_grad(aptstat.Cloud(X.detach(), Lb, Db), SC, ANY, 1.0, 2.0, 200, 0.02,
                                     (2 * (h.detach() - t)).contiguous(), z_scale=Z.detach().reshape(1))
    assert torch.equal(X.grad, gx) and torch.equal(Z.grad.reshape(1), gs)
    # without z_scale
    X.grad = None
    h0 = aptstat.RdfSmooth.apply(X, None, Lb, Db, SC, ANY, 1.0, 2.0, 200, 0.02)
    h1 = aptstat.rdf_smooth(aptstat.Cloud(X.detach(), Lb, Db), SC, ANY, 1.0, 2.0, 200, 0.02,
                            z_scale=torch.ones(1, dtype=torch.float64, device="cuda:0"))
    assert torch.equal(h0, h1)
    h0.sum().backward()
    assert X.grad is not None


def test_smooth_edge_cases(gpu, orc):
    aptstat, torch, ws = gpu
    # empty cloud
    c0 = _cloud(gpu, np.zeros((0, 3), np.float32), np.zeros(0, np.uint8))
    h, st = gpu_fwd(gpu, c0, SC, SC, 0.0, 2.0, 50, 0.05)
    assert np.all(h == 0) and st == 0
    g, gs = gpu_bwd(gpu, c0, SC, SC, 0.0, 2.0, 50, 0.05, np.ones(50))
    assert g.shape == (0, 3) and gs == 0.0
    # coincident ions (D = 0), a pair beyond r_max but within 6 sigma, an
    # ion at the cut, non-finite positions, an ineligible (NaN d_bnd) target
    xyz = np.array([[1, 1, 1], [1, 1, 1], [1.5, 1, 1], [3.1, 1, 1], [1, 3.28, 1], [np.nan, 1, 1],
                    [1, np.inf, 1], [1.2, 1.1, 0.9], [0.4, 0.7, 1.3]], np.float32)
    lab = np.array([SC, SC, SC, SC, SC, SC, SC, AL, SC], np.uint8)
    d = np.array([5, 5, 5, 5, 5, 5, 5, 5, np.nan], np.float32)
    for B in (SC, ANY):
        cl = _cloud(gpu, xyz, lab, d)
        for s in (1.0, 0.9):
            h, st = gpu_fwd(gpu, cl, SC, B, 1.0, 2.0, 50, 0.05, s)
            assert st == aptstat.STATUS_NONFINITE
            ref = orc.smooth_fwd(xyz, lab, d, SC, B, 1.0, 2.0, 50, 0.05, s)
            assert ref.sum() > 0
            assert_fwd_close(h, ref)
            gh = np.linspace(-1, 2, 50)
            g, gs = gpu_bwd(gpu, cl, SC, B, 1.0, 2.0, 50, 0.05, gh, s)
            rg, rgs = orc.smooth_bwd(xyz, lab, d, SC, B, 1.0, 2.0, 50, 0.05, s, gh)
            assert_grad_close(g, rg)
            assert abs(gs - rgs) <= 1e-9 * abs(rgs)
            assert np.all(g[5:7] == 0)
    # z_scale None is s = 1
    cl = _cloud(gpu, xyz[:5], lab[:5])
    h1 = aptstat.rdf_smooth(cl, SC, SC, 0.0, 2.0, 50, 0.05, ws=ws)
    h2 = aptstat.rdf_smooth(cl, SC, SC, 0.0, 2.0, 50, 0.05, z_scale=_zs(torch, 1.0), ws=ws)
    assert torch.equal(h1, h2)
    # host-side errors
    with pytest.raises(aptstat.AptError, match="4096"):
        aptstat.rdf_smooth(cl, SC, SC, 0.0, 2.0, 5000, 0.05, ws=ws)
    with pytest.raises(aptstat.AptError, match="sigma"):
        aptstat.rdf_smooth(cl, SC, SC, 0.0, 2.0, 200, 2.0, ws=ws)
    with pytest.raises(aptstat.AptError, match="sigma"):
        aptstat.rdf_smooth(cl, SC, SC, 0.0, 2.0, 200, 0.0, ws=ws)


@pytest.mark.slow
def test_smooth_differentiable_workload_box1m(gpu, orc, synth):
    """1e6 ions in a 32 nm cube with 500 Sc clusters, sigma 0.02, 200 bins to
    2 nm; target curve from the next seed; at s = 1 and 1.05: forward and
    adjoint against the oracle, the adjoint against central finite
    differences on 5000 random Sc ions (h = 1e-4 nm) and on s (h = 1e-6)."""
    aptstat, torch, ws = gpu
    sp, sp2 = synth.box1m(1), synth.box1m(2)
    xyz, lab, _ = sp.generate()
    xyz2, lab2, _ = sp2.generate()
    args = (SC, SC, 0.0, 2.0, 200, 0.02)
    _say("box1m: oracle target curve")
    t = orc.smooth_fwd(xyz2, lab2, None, *args, 1.0)
    cloud = _cloud(gpu, xyz, lab)
    rng = np.random.default_rng(7)
    ions = np.sort(rng.choice(np.flatnonzero(lab == SC), 5000, replace=False))
    for s in (1.0, 1.05):
        _say(f"box1m: s = {s}")
        h, st = gpu_fwd(gpu, cloud, *args, s)
        assert st == 0
        ref = orc.smooth_fwd(xyz, lab, None, *args, s)
        assert_fwd_close(h, ref)
        gh = 2.0 * (ref - t)
        g, gs = gpu_bwd(gpu, cloud, *args, gh, s)
        rg, rgs = orc.smooth_bwd(xyz, lab, None, *args, s, gh)
        assert_grad_close(g, rg)
        assert abs(gs - rgs) <= 1e-9 * abs(rgs)
        # central differences, h = 1e-4 nm: within 1e-4 in norm.  Per
        # component the O(h^2) truncation of each pair does not cancel where
        # the pairs' contributions do, so the component-wise bar is applied
        # to the Richardson extrapolation of h = 1e-4 and 5e-5 nm (the loss
        # also jumps by ~Q(6) per pair crossing the 6-sigma window edge,
        # which rules out much smaller steps).
        fd1 = orc.smooth_fd(xyz, lab, None, *args, s, ref - t, ions, 1e-4)
        gi = g[ions].astype(np.float64)
        assert np.linalg.norm(gi - fd1) <= 1e-4 * np.linalg.norm(fd1)
        fd2 = orc.smooth_fd(xyz, lab, None, *args, s, ref - t, ions, 5e-5)
        assert_grad_close(gi, (4.0 * fd2 - fd1) / 3.0, tight=False)
        # z scale: central differences of the loss on the GPU forward
        hs = 1e-6
        Lp = ((gpu_fwd(gpu, cloud, *args, s + hs)[0] - t) ** 2).sum()
        Lm = ((gpu_fwd(gpu, cloud, *args, s - hs)[0] - t) ** 2).sum()
        assert abs((Lp - Lm) / (2 * hs) - gs) <= 1e-4 * abs(gs)
