"""Pairs aimed at bin edges: the FP32 fast path and its FP64 band against the
oracle, bit for bit, on a large population.

The GPU decides a pair's RDF bin (and a target's k-th distance bin) in FP32
and re-decides it in FP64 only inside a band around every edge; the oracle
decides every pair in FP64.  These clouds place every pair within 1e-5 nm of
an edge (r_max included): 1e8 target-neighbour pairs for the RDF, 1e6
targets whose k-th neighbour sits at a 0.001 nm edge of the k-th distance
histogram, with coordinates in three magnitude ranges up to the full-scale
needle's (2048-4096 nm, where one FP32 ulp is 2.4e-4 nm).  Each neighbour is
placed with two coordinates rounded first and the third solved from the
remaining squared distance and rounded last, along an axis the direction
barely follows, so that rounding to FP32 moves the distance by at most a few
1e-6 nm.
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

A_SP, B_SP = 1, 0
N_PAIRS = int(os.environ.get("APT_NEAR_EDGE_PAIRS", "100000000"))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_2004_05188_amd as aptstat

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    aptstat.lib()
    return aptstat, torch


def _place_once(rng, t, R, wmax):
    """Neighbours at FP64 distance ~R (array) from targets t [m,3] (float32
    values): two coordinates rounded to FP32 first, the third solved from the
    remaining squared distance and rounded last, along an axis the direction
    follows by at most wmax.  Returns float32 positions and the rows placed."""
    m = len(R)
    phi = rng.uniform(0.0, 2.0 * np.pi, m)
    w = rng.uniform(-1.0, 1.0, m) * wmax
    s = np.sqrt(1.0 - w * w)
    u = np.stack([s * np.cos(phi), s * np.sin(phi), w], axis=1)
    ax = rng.integers(0, 3, m)                      # which axis takes the small component
    u = np.take_along_axis(u, (np.arange(3)[None, :] - ax[:, None] + 2) % 3, axis=1)   # u[:, ax] = w
    t64 = t.astype(np.float64)
    p = (t64 + R[:, None] * u).astype(np.float32).astype(np.float64)
    d = p - t64
    rows = np.arange(m)
    d[rows, ax] = 0.0
    rem = R * R - (d * d).sum(axis=1)
    ok = rem >= 0.0
    sgn = np.where(u[rows, ax] < 0.0, -1.0, 1.0)
    p[rows, ax] = (t64[rows, ax] + sgn * np.sqrt(np.where(ok, rem, 0.0))).astype(np.float32)
    return p.astype(np.float32), ok


def _place_near(rng, t, R, e, tol=1e-5, tries=60):
    """As _place_once, redrawn until the FP64 distance of the stored values
    lies within tol of e (rows that never do are reported as not placed).
    The solved axis's rounding moves the distance by up to wmax * ulp / 2;
    a short distance at large coordinates needs a steeper direction for the
    two rounded coordinates to leave a real remainder."""
    q = np.spacing(np.abs(t).max(axis=1).astype(np.float32)).astype(np.float64)
    wmax = np.clip(np.sqrt(8.0 * q / R), 0.04, 0.95)
    p = np.zeros_like(t)
    done = np.zeros(len(R), bool)
    for _ in range(tries):
        todo = np.nonzero(~done)[0]
        if len(todo) == 0:
            break
        pp, ok = _place_once(rng, t[todo], R[todo], wmax[todo])
        D = np.sqrt(_D2(t[todo], pp))
        good = ok & (np.abs(D - e[todo]) <= tol)
        p[todo[good]] = pp[good]
        done[todo[good]] = True
    return p, done


def _D2(a, b):
    # the FP64 squared distance of stored FP32 values, ((dx*dx + dy*dy) + dz*dz)
    d = b.astype(np.float64) - a.astype(np.float64)
    return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]


def _lattice(rng, lo, hi, spacing, count):
    """`count` target sites on a cubic lattice of `spacing` inside [lo, hi)^3
    (jittered by +-0.05 spacing), float32."""
    per = int(math.floor((hi - lo) / spacing))
    assert per ** 3 >= count, (per, count)
    idx = rng.choice(per ** 3, size=count, replace=False)
    g = np.stack([idx % per, (idx // per) % per, idx // (per * per)], axis=1).astype(np.float64)
    x = lo + (g + 0.5) * spacing + rng.uniform(-0.05, 0.05, (count, 3)) * spacing
    return x.astype(np.float32)


def rdf_edge_cloud(n_pairs, r_max=2.0, n_bins=200, seed=5):
    """Targets (species A) each with one neighbour (species B) per bin edge
    e_b, b = 1..n_bins (r_max included), at e_b + delta, |delta| <= 1e-5 nm
    (FP64 distance of the stored values); targets 2 r_max + 0.5 nm apart, so
    that no other pair is within r_max.  Coordinates in three ranges: around
    3000 nm (most targets), 65-127 nm and -20-20 nm."""
    rng = np.random.default_rng(seed)
    nt = max(-(-n_pairs // n_bins), 3)
    spacing = 2.0 * r_max + 0.5
    ranges = [(2100.0, 4000.0), (65.0, 127.0), (-20.0, 20.0)]
    caps = [int(math.floor((hi - lo) / spacing)) ** 3 for lo, hi in ranges]
    c2, c3 = min(nt // 10, caps[1]), min(nt // 10, caps[2])
    counts = [nt - c2 - c3, c2, c3]
    e_all = np.arange(1, n_bins + 1, dtype=np.float64) * r_max / n_bins
    xyz_parts, lab_parts, near = [], [], 0
    for (lo, hi), c in zip(ranges, counts):
        t = _lattice(rng, lo, hi, spacing, c)
        for c0 in range(0, c, 50_000):
            tt = np.repeat(t[c0:c0 + 50_000], n_bins, axis=0)
            e = np.tile(e_all, len(tt) // n_bins)
            R = e + rng.uniform(-1e-5, 1e-5, len(tt))
            p, keep = _place_near(rng, tt, R, e)
            near += int(keep.sum())
            xyz_parts.append(p[keep])
            lab_parts.append(np.full(int(keep.sum()), B_SP, np.uint8))
        xyz_parts.append(t)
        lab_parts.append(np.full(len(t), A_SP, np.uint8))
    return np.concatenate(xyz_parts), np.concatenate(lab_parts), near


def kth_edge_cloud(n_targets, k=10, kb_rmax=5.0, kb_nbins=5000, seed=9):
    """Targets (indices 0..n_targets-1) whose k-th nearest neighbour (species
    B) lies within 1e-5 nm of an edge of the k-th distance histogram (edges
    0.1-5 nm; the last is its r_max), the k-1 nearer ones strictly inside;
    one target in ten has a (k+1)-th neighbour within 2e-6 nm of the k-th (a
    near tie).  Targets 12 nm apart: no other ion is within 5 nm.  Returns
    xyz, lab, the index of each target's k-th placed neighbour and of its
    tie partner (-1: none)."""
    rng = np.random.default_rng(seed)
    spacing = 12.0
    t = _lattice(rng, 2100.0, 4000.0, spacing, n_targets)
    b = rng.integers(100, kb_nbins + 1, n_targets)
    e = b * kb_rmax / kb_nbins
    Rk = e + rng.uniform(-1e-5, 1e-5, n_targets)
    parts, labs = [t], [np.full(n_targets, A_SP, np.uint8)]
    n = n_targets
    for j in range(k - 1):
        # strictly nearer than the k-th (plain rounding moves them < 3e-4 nm)
        Rj = rng.uniform(0.02, 1.0, n_targets) * (e - 0.01)
        u = rng.normal(size=(n_targets, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        parts.append((t.astype(np.float64) + Rj[:, None] * u).astype(np.float32))
        labs.append(np.full(n_targets, B_SP, np.uint8))
        n += n_targets
    p, ok = _place_near(rng, t, Rk, e)
    kth = np.full(n_targets, -1, np.int64)
    kth[ok] = n + np.arange(int(ok.sum()))
    parts.append(p[ok])
    labs.append(np.full(int(ok.sum()), B_SP, np.uint8))
    n += int(ok.sum())
    tie = np.nonzero(ok & (rng.uniform(0, 1, n_targets) < 0.1))[0]
    p2, ok2 = _place_near(rng, t[tie], Rk[tie] + rng.uniform(-2e-6, 2e-6, len(tie)), e[tie])
    partner = np.full(n_targets, -1, np.int64)
    partner[tie[ok2]] = n + np.arange(int(ok2.sum()))
    parts.append(p2[ok2])
    labs.append(np.full(int(ok2.sum()), B_SP, np.uint8))
    return np.concatenate(parts), np.concatenate(labs), kth, partner


def test_rdf_pairs_near_every_edge(gpu, orc):
    aptstat, torch = gpu
    _say(f"[near-edge] RDF: building {N_PAIRS} pairs within 1e-5 nm of the edges of 200 bins to 2 nm")
    xyz, lab, near = rdf_edge_cloud(N_PAIRS)
    _say(f"[near-edge] RDF: {len(xyz)} ions, {near} near-edge pairs")
    assert near >= 0.9 * N_PAIRS
    dev = torch.device("cuda:0")
    cloud = aptstat.Cloud(torch.from_numpy(xyz).to(dev), torch.from_numpy(lab).to(dev))
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    h = aptstat.rdf(cloud, A_SP, B_SP, 0.0, 2.0, 200, status=st)
    torch.cuda.synchronize()
    got = h.cpu().numpy().astype(np.uint64)
    assert int(st.item()) == 0
    del cloud
    torch.cuda.empty_cache()
    _say("[near-edge] RDF: oracle")
    ref = orc.rdf(xyz, lab, None, A_SP, B_SP, 0.0, 2.0, 200)
    bad = np.nonzero(got != ref)[0]
    assert len(bad) == 0, f"RDF differs in bins {bad[:10]}: gpu {got[bad[:10]]} oracle {ref[bad[:10]]}"
    # every pair sits near an edge and no other pair is within r_max: all
    # but about half of those at r_max count
    n_in = int(ref.sum())
    assert abs(n_in - near * 199.5 / 200) < 0.002 * near


def test_kth_distance_near_every_edge(gpu, orc):
    aptstat, torch = gpu
    n_t = 1_000_000
    _say(f"[near-edge] k-th histogram: {n_t} targets at 0.001 nm edges")
    xyz, lab, kth, partner = kth_edge_cloud(n_t)
    dev = torch.device("cuda:0")
    cloud = aptstat.Cloud(torch.from_numpy(xyz).to(dev), torch.from_numpy(lab).to(dev))
    r = aptstat.knn(cloud, A_SP, B_SP, 0.0, 10, kb_rmax=5.0, kb_nbins=5000)
    torch.cuda.synchronize()
    tid, dist, nid = (t.cpu().numpy() for t in r.trimmed())
    kh = r.knn_hist.cpu().numpy().astype(np.uint64)
    assert int(r.status.item()) == 0
    del cloud, r
    torch.cuda.empty_cache()
    _say("[near-edge] k-th histogram: oracle")
    otid, odist, onid, okh = orc.knn(xyz, lab, None, A_SP, B_SP, 0.0, 10, kb_rmax=5.0, kb_nbins=5000)
    assert np.array_equal(otid, np.arange(n_t))
    assert np.array_equal(tid, otid)
    assert np.array_equal(nid, onid), "kNN identities differ"
    assert np.array_equal(kh, okh), f"k-th histogram differs in {np.count_nonzero(kh != okh)} bins"
    assert int(okh[:-1].sum()) >= 0.99 * n_t
    # near ties: targets whose FP64 distances order the placed k-th neighbour
    # and its partner otherwise than the defined FP32 order (squared distance,
    # then index) that the rows follow; counted and reported
    tie = np.nonzero(partner >= 0)[0]
    Dk = _D2(xyz[tie], xyz[kth[tie]])
    Dp = _D2(xyz[tie], xyz[partner[tie]])
    fp64_partner_first = (Dp < Dk) | ((Dp == Dk) & (partner[tie] < kth[tie]))
    fp32_partner_first = onid[tie, -1] == partner[tie]  # the partner holds the k-th slot
    near_ties = int(np.count_nonzero(fp64_partner_first != fp32_partner_first))
    _say(f"[near-edge] k-th histogram: {len(tie)} designed ties, FP32 and FP64 orders differ for {near_ties}")
