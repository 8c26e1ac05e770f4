"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes one part of the oracle to the mathematics or to a published
value: brute force on tiny inputs, exact lattice sums, Poisson closed forms,
invariants and a library routine where the method reduces to one.  The
paper prints no kNN or RDF values for its specimens (its result figures are
not part of the text), so parity with the paper's own outputs is unpinned.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
AL, SC, SI, ANY = 0, 1, 2, 255


def _read_table(name):
    rows, meta = [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                parts = line[1:].split()
                if len(parts) == 2:
                    try:
                        meta[parts[0]] = float(parts[1])
                    except ValueError:
                        pass
                continue
            rows.append(line.split())
    return rows, meta


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------

def test_splitmix64_published_outputs(orc):
    rows, _ = _read_table("splitmix64_seed0.txt")
    for i, hx in rows:
        assert orc.splitmix64(0, int(i)) == int(hx, 16)


def test_permutation_is_uniform_on_four_items(orc):
    # every one of the 24 orderings of 4 distinct labels is equally likely
    lab = np.array([0, 1, 2, 3], dtype=np.uint8)
    counts = {}
    R = 24 * 400
    for r in range(R):
        out = orc.permute_labels(lab, 1000 + r)
        counts[tuple(out)] = counts.get(tuple(out), 0) + 1
    assert len(counts) == 24
    obs = np.array(list(counts.values()), dtype=float)
    chi2 = ((obs - R / 24) ** 2 / (R / 24)).sum()
    assert stats.chi2.sf(chi2, 23) > 1e-4


def test_permutation_preserves_species_and_moves_labels(orc, synth):
    xyz, lab, d = synth.box240k().generate()
    out = orc.permute_labels(lab, 7)
    assert np.array_equal(np.bincount(out, minlength=3), np.bincount(lab, minlength=3))
    # a uniform permutation keeps a label in place with probability ~ its fraction
    same = (out == lab).mean()
    p = (np.bincount(lab) / len(lab)) ** 2
    assert abs(same - p.sum()) < 5 * math.sqrt(p.sum() / len(lab)) + 1e-3
    assert not np.array_equal(out, orc.permute_labels(lab, 8))


def test_permutation_mean_matches_exact_null_expectation(orc, synth):
    # E_perm[H_b(A->B)] = H_b(eligible -> any) * N_A (N_B - d_AB) / (N (N-1)),
    # eligibility on positions only (no d_bnd here)
    xyz, lab, d = synth.Specimen(shape="box", L=(8.0, 8.0, 8.0), n=6000, seed=3, p_m_sc=0.1,
                                 p_m_si=0.05).generate()
    n = len(lab)
    NA, NB = (lab == SC).sum(), (lab == AL).sum()
    base = orc.rdf(xyz, lab, None, ANY, ANY, 0.0, 1.0, 10).astype(float)
    expect = base * NA * NB / (n * (n - 1.0))
    reps = np.array([orc.rdf(xyz, orc.permute_labels(lab, 100 + r), None, SC, AL, 0.0, 1.0, 10)
                     for r in range(48)], dtype=float)
    m, sd = reps.mean(0), reps.std(0, ddof=1)
    z = (m - expect) / (sd / math.sqrt(len(reps)) + 1e-9)
    assert np.all(np.abs(z) < 5.0), z


# --------------------------------------------------------------------------
# distances and bins
# --------------------------------------------------------------------------

def test_distances_exact_cases(orc):
    a = np.array([1.0, 2.0, 3.0], np.float32)
    b = np.array([4.0, 6.0, 3.0], np.float32)  # 3-4-5
    assert orc.D2(a, b) == 25.0 and orc.d2f(a, b) == 25.0
    c = np.array([1.0, 2.0, 15.0], np.float32)  # 0,0,12
    assert orc.D2(a, c) == 144.0
    # FP64 distance of the stored FP32 values, not of their decimal spelling
    p = np.array([0.1, 0.0, 0.0], np.float32)
    q = np.array([0.0, 0.0, 0.0], np.float32)
    assert orc.D2(p, q) == float(np.float64(np.float32(0.1))) ** 2


def test_edges_and_half_open_bins(orc):
    E2 = orc.edges2(2.0, 200)
    assert E2[0] == 0.0 and E2[200] == 4.0 and E2[50] == 0.25 and E2[100] == 1.0
    assert orc.bin_of(0.0, E2) == 0
    assert orc.bin_of(0.25, E2) == 50          # lower edge belongs to the bin
    assert orc.bin_of(np.nextafter(0.25, 0), E2) == 49
    assert orc.bin_of(4.0, E2) == 200          # r = r_max is outside
    assert orc.bin_of(np.nextafter(4.0, 0), E2) == 199


def _pair_cloud(d):
    xyz = np.array([[10.0, 10.0, 10.0], [10.0 + d, 10.0, 10.0]], np.float32)
    return xyz, np.array([SC, SC], np.uint8)


@pytest.mark.parametrize("d,expect", [
    (0.5, 50), (1.0, 100), (1.5, 150),                 # representable edges
    (0.5 + 2e-6, 50), (0.5 - 2e-6, 49), (1.0 - 1e-6, 99), (1.0 + 1e-6, 100),
    (0.25, 25), (2.0, None), (2.0 - 2e-6, 199),
])
def test_pairs_at_bin_edges(orc, d, expect):
    xyz, lab = _pair_cloud(d)
    h = orc.rdf(xyz, lab, None, SC, SC, 0.0, 2.0, 200, method="brute")
    D = orc.D2(xyz[0], xyz[1])
    if expect is None:
        assert h.sum() == 0
    else:
        # the bin follows the FP64 distance of the stored FP32 coordinates
        b = int(np.searchsorted(orc.edges2(2.0, 200), D, side="right") - 1)
        assert b == expect or abs(math.sqrt(D) - d) < 1e-5
        assert h[b] == 2 and h.sum() == 2  # ordered pairs both ways


# --------------------------------------------------------------------------
# brute force == grid on small inputs, including edge cases
# --------------------------------------------------------------------------

def _small_cloud(synth, n, seed, L=6.0):
    s = synth.Specimen(shape="box", L=(L, L, L), n=n, seed=seed, p_m_sc=0.2, p_m_si=0.1)
    return s.generate()


@pytest.mark.parametrize("A,B", [(SC, SC), (SC, AL), (AL, SC), (SI, ANY), (ANY, SC)])
@pytest.mark.parametrize("use_d", [False, True])
def test_rdf_brute_equals_grid(orc, synth, A, B, use_d):
    xyz, lab, d = _small_cloud(synth, 3000, 11)
    d = d if use_d else None
    hb = orc.rdf(xyz, lab, d, A, B, 0.7, 1.3, 37, method="brute")
    hg = orc.rdf(xyz, lab, d, A, B, 0.7, 1.3, 37, method="grid")
    assert np.array_equal(hb, hg)


@pytest.mark.parametrize("A,B,k,rk", [(SC, SC, 10, math.inf), (SC, AL, 5, math.inf),
                                      (SI, SC, 12, 1.0), (ANY, SI, 3, math.inf),
                                      (SC, SI, 40, math.inf)])
def test_knn_brute_equals_grid(orc, synth, A, B, k, rk):
    xyz, lab, d = _small_cloud(synth, 2500, 12)
    a = orc.knn(xyz, lab, d, A, B, 0.5, k, rk, kb_rmax=2.0, kb_nbins=50, method="brute")
    g = orc.knn(xyz, lab, d, A, B, 0.5, k, rk, kb_rmax=2.0, kb_nbins=50, method="grid")
    for u, v in zip(a, g):
        assert np.array_equal(u, v)
    tid, dist, nid, hist = a
    with np.errstate(invalid="ignore"):
        assert np.all((np.diff(dist, axis=1) >= 0) | np.isinf(dist[:, 1:]))  # rows ascending
    assert hist.sum() == len(tid)


def test_knn_fewer_than_k_and_empty_species(orc, synth):
    xyz, lab, d = _small_cloud(synth, 400, 13)
    lab = lab.copy()
    lab[lab == SI] = AL
    lab[np.flatnonzero(lab == AL)[:3]] = SI                 # exactly three Si
    tid, dist, nid, hist = orc.knn(xyz, lab, None, SC, SI, 0.0, 5, kb_rmax=5.0, kb_nbins=10,
                                   method="grid")
    assert np.all(nid[:, 3:] == -1) and np.all(np.isinf(dist[:, 3:]))
    assert np.all(nid[:, :3] >= 0)
    assert hist[10] == len(tid)                             # no 5th neighbour anywhere
    tid, dist, nid, hist = orc.knn(xyz, lab, None, SC, 77, 0.0, 5, kb_rmax=5.0, kb_nbins=10)
    assert np.all(nid == -1) and len(tid) == (lab == SC).sum()
    assert orc.rdf(xyz, lab, None, 77, SC, 0.0, 2.0, 20).sum() == 0


def test_eligibility_inclusive_nan_and_unfiltered_neighbours(orc):
    xyz = np.array([[0, 0, 0], [0.25, 0, 0], [0.5, 0, 0], [0.75, 0, 0]], np.float32)
    lab = np.array([SC, SC, SC, SC], np.uint8)
    d = np.array([1.0, np.nan, 0.999999, -5.0], np.float32)
    assert list(orc.select_targets(lab, d, SC, 1.0)) == [0]
    h = orc.rdf(xyz, lab, d, SC, SC, 1.0, 1.0, 10, method="brute")
    # target 0 sees 1 (0.25), 2 (0.5), 3 (0.75) although they are not targets
    assert h.sum() == 3 and h[2] == 1 and h[5] == 1 and h[7] == 1


def test_nonfinite_positions_take_part_in_no_pair(orc, synth):
    xyz, lab, d = _small_cloud(synth, 800, 14)
    xyz = xyz.copy()
    sc = np.flatnonzero(lab == SC)
    xyz[sc[0], 0] = np.nan          # a target with no neighbours
    xyz[sc[1], 2] = np.inf          # a neighbour at infinity
    xyz[3, 1] = -np.inf
    for method in ("brute", "grid"):
        tid, dist, nid, hist = orc.knn(xyz, lab, None, SC, SC, 0.0, 400, method=method)
        assert sc[1] not in nid and 3 not in nid
        row0 = list(tid).index(sc[0])
        assert np.all(nid[row0] == -1)
    a = orc.knn(xyz, lab, None, SC, ANY, 0.0, 7, method="brute")
    b = orc.knn(xyz, lab, None, SC, ANY, 0.0, 7, method="grid")
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert np.array_equal(orc.rdf(xyz, lab, None, SC, ANY, 0.0, 2.0, 40, method="brute"),
                          orc.rdf(xyz, lab, None, SC, ANY, 0.0, 2.0, 40, method="grid"))


def test_self_exclusion_by_index_and_coincident_ions(orc):
    xyz = np.array([[1, 1, 1], [1, 1, 1], [1.5, 1, 1]], np.float32)
    lab = np.array([SC, SC, AL], np.uint8)
    h = orc.rdf(xyz, lab, None, SC, ANY, 0.0, 1.0, 10, method="brute")
    assert h[0] == 2 and h[5] == 2 and h.sum() == 4          # coincident pair counts at 0
    tid, dist, nid, _ = orc.knn(xyz, lab, None, SC, ANY, 0.0, 2, method="brute")
    assert nid.tolist() == [[1, 2], [0, 2]] and dist[0, 0] == 0.0


# --------------------------------------------------------------------------
# RDF invariants
# --------------------------------------------------------------------------

def test_rdf_invariants(orc, synth):
    xyz, lab, d = _small_cloud(synth, 5000, 21, L=7.0)
    H = {(a, b): orc.rdf(xyz, lab, None, a, b, 0.0, 1.5, 30) for a in (AL, SC, SI, ANY)
         for b in (AL, SC, SI, ANY)}
    for a in (AL, SC, SI):
        for b in (AL, SC, SI):
            assert np.array_equal(H[a, b], H[b, a])         # symmetric without a filter
        assert np.all(H[a, a] % 2 == 0)                    # A->A counts both orders
        assert np.array_equal(H[a, AL] + H[a, SC] + H[a, SI], H[a, ANY])
    # sum over bins = number of ordered pairs closer than r_max (own count)
    sc = np.flatnonzero(lab == SC)
    P = xyz[sc].astype(np.float64)
    D2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(D2, np.inf)
    assert H[SC, SC].sum() == (D2 < 1.5 ** 2).sum()


# --------------------------------------------------------------------------
# exact lattice sums: fcc Al, a = 0.404 nm
# --------------------------------------------------------------------------

def _r3(n):
    k = int(math.isqrt(n)) + 1
    r = np.arange(-k, k + 1)
    s = r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2
    return int((s == n).sum())


def test_fcc_textbook_multiplicities_match_r3():
    rows, meta = _read_table("fcc_shells.txt")
    for m, sites in rows:
        assert _r3(2 * int(m)) == int(sites)


def test_rdf_fcc_lattice_exact_shells(orc):
    rows, meta = _read_table("fcc_shells.txt")
    a = meta["lattice_constant_nm"]
    M = 14
    g = np.arange(2 * M)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    keep = (I + J + K) % 2 == 0
    xyz = (np.stack([I[keep], J[keep], K[keep]], 1) * (a / 2)).astype(np.float32)
    hi = (2 * M - 1) * a / 2
    d = np.minimum(xyz, hi - xyz).min(1).astype(np.float32)
    lab = np.zeros(len(xyz), np.uint8)
    r_max, n_bins = 2.0, 200
    h = orc.rdf(xyz, lab, d, AL, AL, r_max + 0.01, r_max, n_bins)
    T = len(orc.select_targets(lab, d, AL, r_max + 0.01))
    assert T > 100
    expect = np.zeros(n_bins, np.int64)
    for m in range(1, int((r_max / a) ** 2 * 2) + 1):
        r = a * math.sqrt(m / 2)
        if r >= r_max:
            break
        edge = round(r / 0.01) * 0.01
        # FP32 coordinates below 6 nm move a distance by < 5e-7 nm; shell 13
        # (1.0300019 nm) sits 1.9e-6 nm above an edge and stays in its bin
        assert abs(r - edge) > 1e-6, "shell radius too close to a bin edge for this check"
        expect[int(r / 0.01)] += _r3(2 * m)
    # sites within 2 nm of an fcc Al site, by direct enumeration of the lattice
    g2 = np.arange(-12, 13)
    I2, J2, K2 = np.meshgrid(g2, g2, g2, indexing="ij")
    S2 = I2 ** 2 + J2 ** 2 + K2 ** 2
    assert expect.sum() == (((I2 + J2 + K2) % 2 == 0) & (S2 > 0) & (a / 2 * np.sqrt(S2) < r_max)).sum() == 2092
    assert np.array_equal(h, expect * T)


def test_knn_index_tiebreak_on_exact_lattice(orc):
    # simple cubic lattice with exactly representable coordinates: the 6
    # nearest sites are exactly equidistant, so the index decides
    g = np.arange(7, dtype=np.float32) * 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float32)
    rng = np.random.default_rng(5)
    perm = rng.permutation(len(xyz))
    xyz = xyz[perm]
    lab = np.zeros(len(xyz), np.uint8)
    centre = int(np.flatnonzero((xyz == 1.5).all(1))[0])
    d = np.full(len(xyz), -1.0, np.float32)
    d[centre] = 1.0
    tid, dist, nid, _ = orc.knn(xyz, lab, d, AL, AL, 0.0, 4, method="grid")
    first = np.flatnonzero(np.abs(np.linalg.norm(xyz - xyz[centre], axis=1) - 0.5) < 1e-6)
    assert len(first) == 6
    assert nid[0].tolist() == sorted(first.tolist())[:4]
    assert np.all(dist[0] == 0.5)


# --------------------------------------------------------------------------
# Poisson closed forms
# --------------------------------------------------------------------------

def _box_G(r, L):
    L1, L2, L3 = L
    return (L1 * L2 * L3 * 4 * math.pi / 3 * r ** 3 - (L1 * L2 + L2 * L3 + L3 * L1) * math.pi / 2 * r ** 4
            + (L1 + L2 + L3) * 8 / 15 * r ** 5 - r ** 6 / 6)


@pytest.mark.parametrize("A,B", [(SC, SC), (SC, AL)])
def test_rdf_matches_exact_box_expectation(orc, synth, A, B):
    # i.i.d. uniform points in a box: P(|p - q| < r) = G(r) / V^2 with the box's
    # set covariance G integrated over the ball (valid for r <= min side)
    spec = synth.box240k(seed=4)
    xyz, lab, _ = spec.generate()
    L = spec.L
    V = L[0] * L[1] * L[2]
    NA, NB = int((lab == A).sum()), int((lab == B).sum())
    pairs = NA * (NB - (1 if A == B else 0))
    n_bins, r_max = 200, 2.0
    h = orc.rdf(xyz, lab, None, A, B, 0.0, r_max, n_bins).astype(float)
    e = np.arange(n_bins + 1) * r_max / n_bins
    Gv = np.array([_box_G(x, L) for x in e])
    E = pairs * np.diff(Gv) / V ** 2
    var = (2.0 if A == B else 1.0) * E + 1e-12
    z = (h - E) / np.sqrt(var)
    assert np.abs(z).max() < 5.0
    chi2 = (z ** 2).sum()
    assert stats.chi2.sf(chi2, n_bins) > 1e-4
    ztot = (h.sum() - E.sum()) / math.sqrt((6.0 if A == B else 3.0) * E.sum())
    assert abs(ztot) < 5.0


@pytest.mark.parametrize("k", [1, 10])
def test_knn_matches_binomial_ball_law(orc, synth, k):
    # a target >= 4 nm inside the box with N_B - 1 other uniform points:
    # P(R_k <= r) = P(Binomial(N_B - 1, V_ball(r) / V) >= k).  Targets of one
    # cloud share neighbours, so the spread is taken across independent seeds.
    V = 20.0 ** 3
    qs = np.array([0.1, 0.25, 0.5, 0.75, 0.9])
    diffs, Ntot, means = [], 0, []
    for seed in range(1, 9):
        xyz, lab, _ = synth.box240k(seed=seed).generate()
        d = np.minimum(xyz, 20.0 - xyz).min(1).astype(np.float32)
        tid, dist, nid, _ = orc.knn(xyz, lab, d, SC, SC, 4.0, k)
        Rk = dist[:, k - 1].astype(np.float64)
        assert np.all(Rk < 4.0)
        NB = int((lab == SC).sum())
        cdf = lambda r: stats.binom.sf(k - 1, NB - 1, np.minimum(4 / 3 * math.pi * r ** 3 / V, 1.0))
        grid = np.linspace(0.05, 4.0, 4000)
        rq = np.interp(qs, cdf(grid), grid)            # theoretical quantiles
        diffs.append(np.array([(Rk <= r).mean() for r in rq]) - qs)
        Ntot += len(Rk)
        lam = (NB - 1) / V
        means.append(Rk.mean() - math.gamma(k + 1 / 3) / math.gamma(k) * (3 / (4 * math.pi * lam)) ** (1 / 3))
    diffs = np.array(diffs)
    se = np.maximum(diffs.std(0, ddof=1) / math.sqrt(len(diffs)), np.sqrt(qs * (1 - qs) / Ntot))
    assert np.all(np.abs(diffs.mean(0) / se) < 5.0), diffs.mean(0) / se
    means = np.array(means)
    assert abs(means.mean()) < 5 * means.std(ddof=1) / math.sqrt(len(means)) + 1e-4


def test_knn_kth_histogram_is_the_kth_distance(orc, synth):
    xyz, lab, d = _small_cloud(synth, 3000, 31)
    tid, dist, nid, hist = orc.knn(xyz, lab, d, SC, ANY, 0.5, 4, kb_rmax=1.0, kb_nbins=100)
    own = np.zeros(101, np.int64)
    for t, j in zip(tid, nid[:, 3]):
        own[orc.bin_of(orc.D2(xyz[t], xyz[j]), orc.edges2(1.0, 100))] += 1
    assert np.array_equal(hist, own)


# --------------------------------------------------------------------------
# smoothed RDF and its adjoint
# --------------------------------------------------------------------------

def test_smooth_single_pair_is_gaussian_bin_mass(orc):
    xyz = np.array([[3, 3, 3], [3.73, 3.1, 2.95]], np.float32)
    lab = np.array([SC, SC], np.uint8)
    sig, r_max, n_bins = 0.05, 2.0, 200
    h = orc.smooth_fwd(xyz, lab, None, SC, SC, 0.0, r_max, n_bins, sig)
    D = math.sqrt(orc.D2(xyz[0], xyz[1]))
    e = np.arange(n_bins + 1) * r_max / n_bins
    sig = float(np.float32(sig))                    # the width is passed as FP32
    lo, hi = (e[:-1] - D) / sig, (e[1:] - D) / sig
    w = np.where(lo >= 0, stats.norm.sf(lo) - stats.norm.sf(hi), stats.norm.cdf(hi) - stats.norm.cdf(lo))
    w[(e[1:] <= D - 6 * sig) | (e[:-1] >= D + 6 * sig)] = 0
    np.testing.assert_allclose(h, 2 * w, rtol=1e-12, atol=1e-15)


def test_smooth_small_sigma_recovers_exact_histogram(orc, synth):
    xyz, lab, d = _small_cloud(synth, 3000, 41)
    H = orc.rdf(xyz, lab, d, SC, ANY, 0.5, 1.5, 30).astype(float)
    h = orc.smooth_fwd(xyz, lab, d, SC, ANY, 0.5, 1.5, 30, 1e-6)
    assert np.abs(h - H).max() <= 2.0     # only pairs within ~6e-6 nm of an edge may split
    assert abs(h.sum() - H.sum()) <= 2.0


def _smooth_problem(synth):
    s = synth.Specimen(shape="box", L=(5.0, 5.0, 5.0), n=1500, seed=51, p_m_sc=0.3,
                       n_clusters=3, r_c=0.8, p_c_sc=0.6)
    xyz, lab, d = s.generate()
    return xyz, lab


def _loss(orc, xyz, lab, s, target):
    h = orc.smooth_fwd(xyz, lab, None, SC, SC, 0.0, 1.0, 50, 0.05, s)
    return float(((h - target) ** 2).sum()), h


def test_smooth_adjoint_matches_finite_differences(orc, synth):
    xyz, lab = _smooth_problem(synth)
    rng = np.random.default_rng(0)
    target = rng.uniform(0, 20, 50)
    s = 1.05
    L0, h = _loss(orc, xyz, lab, s, target)
    g, gs = orc.smooth_bwd(xyz, lab, None, SC, SC, 0.0, 1.0, 50, 0.05, s, 2 * (h - target))
    xyz64 = xyz.astype(np.float64)
    sc = np.flatnonzero(lab == SC)
    for i in rng.choice(sc, 6, replace=False):
        for a in range(3):
            # FP32 positions: step chosen so the perturbed value is exact in FP32
            step = np.float32(2 ** -12)
            xp, xm = xyz.copy(), xyz.copy()
            xp[i, a] += step
            xm[i, a] -= step
            hstep = (float(xp[i, a]) - float(xm[i, a])) / 2
            fd = (_loss(orc, xp, lab, s, target)[0] - _loss(orc, xm, lab, s, target)[0]) / (2 * hstep)
            assert abs(fd - g[i, a]) <= 2e-3 * max(abs(g[i, a]), 1e-2 * np.abs(g).max()), (i, a, fd, g[i, a])
    hs = 1e-6
    fds = (_loss(orc, xyz, lab, s + hs, target)[0] - _loss(orc, xyz, lab, s - hs, target)[0]) / (2 * hs)
    assert abs(fds - gs) <= 1e-4 * abs(gs)


def test_smooth_adjoint_invariants(orc, synth):
    xyz, lab = _smooth_problem(synth)
    rng = np.random.default_rng(1)
    target = rng.uniform(0, 20, 50)
    for s in (1.0, 1.05):
        _, h = _loss(orc, xyz, lab, s, target)
        g, gs = orc.smooth_bwd(xyz, lab, None, SC, SC, 0.0, 1.0, 50, 0.05, s, 2 * (h - target))
        scale = np.abs(g).sum()
        # translation invariance
        assert np.abs(g.sum(0)).max() <= 1e-10 * scale
        # rotation about z (any s) and about every axis at s = 1
        P = xyz.astype(np.float64)
        torque = np.cross(P, g).sum(0)
        assert abs(torque[2]) <= 1e-9 * scale * 5
        if s == 1.0:
            assert np.abs(torque).max() <= 1e-9 * scale * 5
        # dL/ds = (1/s) sum_i z_i dL/dz_i
        assert abs(gs - (P[:, 2] * g[:, 2]).sum() / s) <= 1e-9 * (abs(gs) + scale)


def test_smooth_local_fd_equals_full_recompute(orc, synth):
    """The per-ion finite differences (only the moved ion's pairs are
    re-evaluated) equal differences of the full loss, in both roles."""
    s = synth.Specimen(shape="box", L=(5.0, 5.0, 5.0), n=1500, seed=52, p_m_sc=0.3,
                       n_clusters=3, r_c=0.8, p_c_sc=0.6)
    xyz, lab, _ = s.generate()
    d = (np.minimum(xyz.min(1), 5.0 - xyz.max(1))).astype(np.float32)   # distance to the box faces
    rng = np.random.default_rng(3)
    target = rng.uniform(0, 20, 50)
    args = (SC, ANY, 0.4, 1.0, 50, 0.05)
    for sc in (1.0, 1.05):
        h = orc.smooth_fwd(xyz, lab, d, *args, sc)
        ions = np.concatenate([rng.choice(np.flatnonzero(lab == SC), 3, replace=False),
                               rng.choice(np.flatnonzero(lab != SC), 3, replace=False)])
        step = 2.0 ** -12           # exact in FP32 at these coordinates
        fd = orc.smooth_fd(xyz, lab, d, *args, sc, h - target, ions, step)
        for q, i in enumerate(ions):
            for a in range(3):
                xp, xm = xyz.copy(), xyz.copy()
                xp[i, a] += np.float32(step)
                xm[i, a] -= np.float32(step)
                Lp = ((orc.smooth_fwd(xp, lab, d, *args, sc) - target) ** 2).sum()
                Lm = ((orc.smooth_fwd(xm, lab, d, *args, sc) - target) ** 2).sum()
                full = (Lp - Lm) / (2 * step)
                assert abs(fd[q, a] - full) <= 1e-7 * max(abs(full), 1.0), (sc, i, a, fd[q, a], full)
        # and they agree with the adjoint to the truncation error of the step
        g, _ = orc.smooth_bwd(xyz, lab, d, *args, sc, 2 * (h - target))
        gi = g[ions]
        assert np.abs(fd - gi).max() <= 2e-3 * np.abs(gi).max()


# --------------------------------------------------------------------------
# exact rounding: the fixed FP32 and FP64 distance expressions, bit for bit
# --------------------------------------------------------------------------

def _round_binary(x, mant_bits, emin):
    """x (a Fraction) rounded to nearest, ties to even, in a binary format with
    `mant_bits` significand bits and smallest normal exponent `emin`
    (subnormals included; no overflow occurs for the values used here)."""
    from fractions import Fraction

    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, emin)
    q = Fraction(2) ** (e - (mant_bits - 1))
    m = a / q
    n = m.numerator // m.denominator
    rem = m - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return sign * n * q


def _rn32(x):
    return _round_binary(x, 24, -126)


def _rn64(x):
    return _round_binary(x, 53, -1022)


def _fr(v):
    from fractions import Fraction

    return Fraction(float(v))


def _d2f_variants(a, b):
    """Exact values of three FP32 evaluation orders of the squared distance:
    the defined one fmaf(dz,dz,fmaf(dy,dy,dx*dx)), the unfused sum, and the
    other nesting fmaf(dx,dx,fmaf(dy,dy,dz*dz))."""
    dx, dy, dz = (_rn32(_fr(b[c]) - _fr(a[c])) for c in range(3))
    defined = _rn32(dz * dz + _rn32(dy * dy + _rn32(dx * dx)))
    unfused = _rn32(_rn32(_rn32(dx * dx) + _rn32(dy * dy)) + _rn32(dz * dz))
    other = _rn32(dx * dx + _rn32(dy * dy + _rn32(dz * dz)))
    return defined, unfused, other


def test_d2f_fused_order_bit_exact(orc):
    # Random FP32 pairs at the coordinate scales of the workloads; the
    # expected bits come from exact rational arithmetic with one rounding to
    # FP32 per step of the defined expression.  Cases where an unfused sum or
    # the other nesting rounds differently must exist among them, so that a
    # plausible slip in the oracle's expression fails here.
    rng = np.random.default_rng(20040518)
    discriminating = 0
    for scale, spread in ((1.0, 2.0), (150.0, 2.0), (3000.0, 2.0), (20.0, 0.3)):
        for _ in range(400):
            a = (rng.uniform(0.0, scale, 3)).astype(np.float32)
            b = (a.astype(np.float64) + rng.uniform(-spread, spread, 3)).astype(np.float32)
            defined, unfused, other = _d2f_variants(a, b)
            got = orc.d2f(a, b)
            assert got == float(defined), (a, b, got, float(defined))
            if defined != unfused and defined != other:
                discriminating += 1
    assert discriminating >= 20, discriminating


def test_D2_association_order_bit_exact(orc):
    # FP64 squared distance of the stored FP32 values, ((dx*dx + dy*dy) + dz*dz)
    # with every operation rounded on its own.  The differences are exact in
    # FP64 for FP32 inputs; a square or a sum rounds only when the
    # differences span more than ~26 significant bits (at the workloads' large
    # coordinates every step is exact).  Two families make the alternatives
    # visible: coordinates of unlike magnitudes (inexact squares: a fused
    # last step differs) and one long with two tiny differences (each tiny
    # square below half an ulp of the first: the other association differs).
    rng = np.random.default_rng(7)
    other_differs = fused_differs = 0
    for it in range(2000):
        if it % 2:
            a = rng.uniform(0.0, 0.1, 3).astype(np.float32)
            b = rng.uniform(-1.0, 1.0, 3).astype(np.float32)
        else:
            a = np.zeros(3, np.float32)
            tiny = rng.choice([-1.0, 1.0], 2) * rng.uniform(0.7, 1.0, 2) * 2.0 ** -26.5
            b = np.array([rng.uniform(0.5, 1.0), *tiny], np.float32)
        dx, dy, dz = (_fr(b[c]) - _fr(a[c]) for c in range(3))
        sx, sy, sz = _rn64(dx * dx), _rn64(dy * dy), _rn64(dz * dz)
        defined = _rn64(_rn64(sx + sy) + sz)
        other = _rn64(sx + _rn64(sy + sz))
        fused = _rn64(dz * dz + _rn64(sx + sy))
        assert orc.D2(a, b) == float(defined), (a, b)
        other_differs += defined != other
        fused_differs += defined != fused
    assert other_differs >= 100 and fused_differs >= 20, (other_differs, fused_differs)


def test_splitmix64_seed_shift(orc):
    # the state after m steps from seed 0 is m * golden gamma (mod 2^64): the
    # stream of that seed is the seed-0 stream shifted by m
    gamma = 0x9E3779B97F4A7C15
    for m in (1, 2, 5, 1000):
        s = (gamma * m) % (1 << 64)
        for i in range(8):
            assert orc.splitmix64(s, i) == orc.splitmix64(0, i + m)


@pytest.mark.parametrize("n", [5, 9, 17, 33, 50])
def test_permutation_direction_bit_exact(orc, n):
    # out[i] = lab[pi(i)], pi = the indices sorted by (key(i), i): distinct
    # labels make the direction visible (out[pi(i)] = lab[i] differs)
    lab = np.arange(n, dtype=np.uint8)[::-1].copy()
    inverse_differs = 0
    for seed in (0, 1, 12345, 2**63 + 11):
        keys = [orc.splitmix64(seed, i) for i in range(n)]
        pi = sorted(range(n), key=lambda i: (keys[i], i))
        expect = np.array([lab[j] for j in pi], dtype=np.uint8)
        got = orc.permute_labels(lab, seed)
        assert np.array_equal(got, expect), (seed, got, expect)
        inv = np.empty_like(lab)
        inv[np.array(pi)] = lab
        inverse_differs += not np.array_equal(inv, expect)
    assert inverse_differs >= 3


# --------------------------------------------------------------------------
# two-point statistics (displacement-vector histogram)
# --------------------------------------------------------------------------

def _fcc_block(a, M):
    g = np.arange(2 * M)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    keep = (I + J + K) % 2 == 0
    xyz = (np.stack([I[keep], J[keep], K[keep]], 1) * (a / 2)).astype(np.float32)
    hi = (2 * M - 1) * a / 2
    d = np.minimum(xyz, hi - xyz).min(1).astype(np.float32)
    return xyz, d


def _voxel_of(v, R, n):
    # exact voxel of a displacement component v (a Fraction): largest m with
    # ((2m - n) R) / n <= v
    from fractions import Fraction

    m = math.floor((Fraction(v) + Fraction(R)) * n / (2 * Fraction(R)))
    return min(max(m, 0), n - 1)


def test_sdm_fcc_lattice_exact_vectors(orc):
    # Interior targets of an fcc lattice see every lattice vector (a/2)(h,k,l),
    # h+k+l even, |v| < R, exactly once: T counts in its voxel, 0 elsewhere.
    # Components are >= 2e-3 nm from any face (multiples of 0.202 nm against
    # faces every 0.025 nm) except 0, where the FP32 difference is exactly 0
    # and the half-open rule puts it in voxel n/2.
    from fractions import Fraction

    rows, meta = _read_table("fcc_shells.txt")
    a = meta["lattice_constant_nm"]
    R, n = 2.0, 160
    xyz, d = _fcc_block(a, 14)
    lab = np.zeros(len(xyz), np.uint8)
    h = orc.sdm(xyz, lab, d, AL, AL, R + 0.01, R, n)
    T = len(orc.select_targets(lab, d, AL, R + 0.01))
    assert T > 100
    expect = np.zeros((n, n, n), np.int64)
    half = Fraction(a) / 2
    g = range(-10, 11)
    vectors = 0
    for i in g:
        for j in g:
            for k in g:
                if (i + j + k) % 2 or (i, j, k) == (0, 0, 0) or float(half) ** 2 * (i * i + j * j + k * k) >= R * R:
                    continue
                mx, my, mz = (_voxel_of(half * c, R, n) for c in (i, j, k))
                assert expect[mz, my, mx] == 0          # one lattice vector per voxel
                expect[mz, my, mx] = T
                vectors += 1
    assert vectors == 2092
    assert np.array_equal(h.astype(np.int64), expect)


def test_sdm_sign_and_axes_on_placed_pairs(orc):
    # v = p_neighbour - p_target, voxel index (mz, my, mx): single pairs with
    # known displacements land in the voxels computed exactly by hand
    R, n = 1.0, 40                      # voxels of 0.05 nm
    t = np.array([5.0, 5.0, 5.0], np.float32)
    cases = [(0.31, 0.12, -0.23), (-0.6, 0.04, 0.3), (0.0, -0.5, 0.0), (0.7, 0.0, -0.04)]
    for v in cases:
        xyz = np.stack([t, (t.astype(np.float64) + v).astype(np.float32)])
        lab = np.array([SC, AL], np.uint8)
        h = orc.sdm(xyz, lab, None, SC, AL, 0.0, R, n, method="brute")
        assert h.sum() == 1
        dv = [float(np.float64(xyz[1, c]) - np.float64(xyz[0, c])) for c in range(3)]
        mx, my, mz = (_voxel_of(c, R, n) for c in dv)
        assert h[mz, my, mx] == 1, (v, np.argwhere(h))
        # the reverse query sees -v
        hr = orc.sdm(xyz, lab, None, AL, SC, 0.0, R, n, method="brute")
        rx, ry, rz = (_voxel_of(-c, R, n) for c in dv)
        assert hr[rz, ry, rx] == 1


@pytest.mark.parametrize("A,B,use_d", [(SC, SC, False), (SC, AL, True), (ANY, SI, False), (AL, ANY, True)])
def test_sdm_brute_equals_grid_and_sums_to_rdf(orc, synth, A, B, use_d):
    xyz, lab, d = synth.Specimen(shape="box", L=(9.0, 9.0, 9.0), n=6000, seed=41, p_m_sc=0.1,
                                 p_m_si=0.05, n_clusters=6, r_c=1.0).generate()
    d = d if use_d else None
    R, n = 1.5, 30
    hb = orc.sdm(xyz, lab, d, A, B, 0.5, R, n, method="brute")
    hg = orc.sdm(xyz, lab, d, A, B, 0.5, R, n, method="grid")
    assert np.array_equal(hb, hg)
    # every pair the RDF counts within R is in exactly one voxel
    assert int(hb.sum()) == int(orc.rdf(xyz, lab, d, A, B, 0.5, R, 7, method="brute").sum())


def test_sdm_inversion_symmetry_and_axis_swap(orc, synth):
    xyz, lab, d = synth.Specimen(shape="box", L=(10.0, 10.0, 10.0), n=8000, seed=43, p_m_sc=0.2).generate()
    R, n = 2.0, 32
    h = orc.sdm(xyz, lab, None, SC, SC, 0.0, R, n)
    # A->A without a surface filter: every unordered pair gives v and -v
    # (no component lies exactly on a face for these continuous positions)
    assert np.array_equal(h, h[::-1, ::-1, ::-1])
    assert h.sum() > 1000
    # swapping the x and y coordinates swaps the x and y voxel axes
    sw = np.ascontiguousarray(xyz[:, [1, 0, 2]])
    hs = orc.sdm(sw, lab, None, SC, SC, 0.0, R, n)
    assert np.array_equal(hs, np.transpose(h, (0, 2, 1)))
    assert not np.array_equal(h, np.transpose(h, (0, 2, 1)))


# --------------------------------------------------------------------------
# maximum-separation clustering
# --------------------------------------------------------------------------

def _partition(label):
    """{root: sorted member indices} of the kept clusters."""
    out = {}
    for i in np.flatnonzero(label >= 0):
        out.setdefault(int(label[i]), []).append(int(i))
    return out


def test_cluster_ms_inclusive_threshold_on_a_chain(orc):
    # ions 0.5 nm apart on a line (0.5 and its multiples are exact in FP32
    # and FP64): at d_max = 0.5 every neighbour pair is linked (<=), one ulp
    # below it none is
    n = 9
    xyz = np.zeros((n, 3), np.float32)
    xyz[:, 0] = np.arange(n, dtype=np.float32) * np.float32(0.5) + np.float32(3.0)
    lab = np.full(n, SC, np.uint8)
    label, counts, hist = orc.cluster_ms(xyz, lab, None, SC, 0.5, 2, n_size_bins=n + 1, method="brute")
    assert np.array_equal(label, np.zeros(n, np.int64)) and list(counts) == [1, 0, n]
    assert hist[n - 1] == 1 and hist.sum() == 1
    below = float(np.nextafter(np.float32(0.5), np.float32(0)))
    label, counts, hist = orc.cluster_ms(xyz, lab, None, SC, below, 1, n_size_bins=4, method="brute")
    assert np.array_equal(label, np.arange(n)) and list(counts) == [n, 0, n] and hist[0] == n
    # an ion of another species in the middle breaks the chain
    lab2 = lab.copy()
    lab2[4] = AL
    label, counts, _ = orc.cluster_ms(xyz, lab2, None, SC, 0.5, 1, method="brute")
    assert list(label) == [0, 0, 0, 0, -1, 5, 5, 5, 5] and list(counts) == [2, 0, 8]


def test_cluster_ms_known_blobs_sizes_and_truncation(orc):
    # compact blobs of known sizes on a 0.3 nm lattice, 5 nm apart, plus
    # isolated ions: at d_max = 0.35 the clusters are exactly the blobs
    rng = np.random.default_rng(3)
    sizes = [1, 2, 4, 5, 7, 12, 20, 33]
    pts, blob = [], []
    for b, s in enumerate(sizes):
        g = np.array([(x, y, z) for z in range(4) for y in range(4) for x in range(4)], np.float32)
        # a connected subset: the first s sites in an order that keeps it connected
        g = g[np.lexsort((g[:, 0], g[:, 1], g[:, 2]))][:s]
        pts.append(g * np.float32(0.3) + np.float32(5.0 * b))
        blob += [b] * s
    xyz = np.concatenate(pts).astype(np.float32)
    blob = np.array(blob)
    order = rng.permutation(len(xyz))
    xyz, blob = xyz[order], blob[order]
    lab = np.full(len(xyz), SC, np.uint8)
    d = np.full(len(xyz), 10.0, np.float32)
    d[np.flatnonzero(blob == 6)[0]] = 0.5          # one ion of the 20-ion blob at the edge
    for n_min in (1, 5, 13):
        label, counts, hist = orc.cluster_ms(xyz, lab, d, SC, 0.35, n_min, d_srf=1.0, n_size_bins=40,
                                             method="brute")
        kept = [b for b, s in enumerate(sizes) if s >= n_min]
        part = _partition(label)
        expect = {int(np.flatnonzero(blob == b).min()): sorted(np.flatnonzero(blob == b).tolist()) for b in kept}
        assert part == expect, n_min
        assert list(counts) == [len(kept), int(n_min <= 20), sum(sizes[b] for b in kept)]
        assert [int(hist[s - 1]) for s in sizes] == [1] * len(sizes) and hist.sum() == len(sizes)


def test_cluster_ms_equals_single_linkage(orc, synth):
    # MS clusters at d_max are the flat clusters of single-linkage
    # agglomeration cut at distance d_max (scipy, FP64 distances)
    from scipy.cluster.hierarchy import fcluster, linkage

    xyz, lab, _ = synth.Specimen(shape="box", L=(14.0, 14.0, 14.0), n=40_000, seed=51, p_m_sc=0.01,
                                 n_clusters=12, r_c=1.2).generate()
    sc = np.flatnonzero(lab == SC)
    assert 500 < len(sc) < 4000
    Z = linkage(xyz[sc].astype(np.float64), method="single", metric="euclidean")
    for d_max in (0.3, 0.45, 0.7, 1.0):
        t = float(np.float32(d_max))
        f = fcluster(Z, t=t, criterion="distance")
        expect = {}
        for c in np.unique(f):
            m = sorted(sc[f == c].tolist())
            if len(m) >= 3:
                expect[m[0]] = m
        label, counts, _ = orc.cluster_ms(xyz, lab, None, SC, d_max, 3)
        assert _partition(label) == expect, d_max
        assert counts[0] == len(expect) and counts[2] == sum(len(v) for v in expect.values())


@pytest.mark.parametrize("A,use_d", [(SC, False), (SI, True), (ANY, True)])
def test_cluster_ms_brute_equals_grid(orc, synth, A, use_d):
    xyz, lab, d = synth.Specimen(shape="box", L=(8.0, 8.0, 8.0), n=6000, seed=57, p_m_sc=0.08, p_m_si=0.05,
                                 n_clusters=5, r_c=1.0).generate()
    xyz[17] = np.nan                                 # a vertex with no links
    d = d if use_d else None
    d_max = 0.25 if A == ANY else 0.6
    b = orc.cluster_ms(xyz, lab, d, A, d_max, 2, d_srf=0.7, n_size_bins=30, method="brute")
    g = orc.cluster_ms(xyz, lab, d, A, d_max, 2, d_srf=0.7, n_size_bins=30, method="grid")
    for x, y in zip(b, g):
        assert np.array_equal(x, y)
    assert b[1][0] > 5


def test_cluster_ms_refines_and_relabels(orc, synth):
    xyz, lab, _ = synth.Specimen(shape="box", L=(10.0, 10.0, 10.0), n=20_000, seed=61, p_m_sc=0.02,
                                 n_clusters=8, r_c=1.0).generate()
    # a larger d_max only merges clusters: every cluster at 0.5 lies inside one at 0.8
    small, _, _ = orc.cluster_ms(xyz, lab, None, SC, 0.5, 1)
    large, _, _ = orc.cluster_ms(xyz, lab, None, SC, 0.8, 1)
    sc = lab == SC
    for r in np.unique(small[sc]):
        assert len(np.unique(large[small == r])) == 1
    assert len(np.unique(large[sc])) < len(np.unique(small[sc]))
    # renumbering the ions renumbers the clusters and nothing else
    perm = np.random.default_rng(5).permutation(len(xyz))
    lp, cp, _ = orc.cluster_ms(xyz[perm], lab[perm], None, SC, 0.5, 1)
    assert sorted(sorted(perm[m].tolist()) for m in _partition(lp).values()) == \
        sorted(_partition(small).values())


# --------------------------------------------------------------------------
# ion-to-edge distancing
# --------------------------------------------------------------------------

def _ulps(a, b):
    """FP32 ulps between two finite float32 arrays of one sign."""
    ia = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(ia - ib)


def test_edge_single_triangle_regions(orc):
    # the right triangle (0,0,0), (4,0,0), (0,4,0): exact distances per region
    tri = np.array([[[0, 0, 0], [4, 0, 0], [0, 4, 0]]], np.float32)
    pts = np.array([
        [1, 1, 3],        # above the interior: the height
        [1, 1, -2],       # below it
        [2, -3, 0],       # beyond the edge on the x axis: to the edge
        [-2, 1, 4],       # beyond the edge on the y axis, off the plane
        [3, 3, 0],        # beyond the hypotenuse, in the plane
        [6, -1, 2],       # beyond the vertex (4, 0, 0)
        [-3, -4, 0],      # beyond the vertex (0, 0, 0)
        [0, 0, 0],        # on a vertex
    ], np.float32)
    expect = [3.0, 2.0, 3.0, np.sqrt(4 + 16), np.sqrt(2.0), np.sqrt(4 + 1 + 4), 5.0, 0.0]
    got = orc.edge_distance(pts, tri, np.inf, method="brute")
    assert np.array_equal(got, np.array(expect, np.float32))
    # zero-area triangles are their edges: a segment and a point
    seg = np.array([[[0, 0, 0], [2, 0, 0], [1, 0, 0]]], np.float32)
    assert np.array_equal(orc.edge_distance(np.array([[1, 3, 4], [5, 0, 4]], np.float32), seg, np.inf, "brute"),
                          np.array([5.0, 5.0], np.float32))
    dot = np.array([[[1, 1, 1]] * 3], np.float32)
    assert orc.edge_distance(np.array([[4, 5, 1]], np.float32), dot, np.inf, "brute")[0] == np.float32(5.0)


def _box_mesh(lo, hi):
    c = np.array([[lo[0] if i & 1 == 0 else hi[0], lo[1] if i & 2 == 0 else hi[1], lo[2] if i & 4 == 0 else hi[2]]
                  for i in range(8)], np.float64)
    quads = [(0, 1, 3, 2), (4, 5, 7, 6), (0, 1, 5, 4), (2, 3, 7, 6), (0, 2, 6, 4), (1, 3, 7, 5)]
    tris = []
    for a, b, cc, d in quads:
        tris += [[c[a], c[b], c[cc]], [c[a], c[cc], c[d]]]
    return np.array(tris, np.float32)


def test_edge_box_surface_closed_form(orc):
    # a box surface of 12 triangles: inside, the distance to the nearest
    # face; outside, the Euclidean distance to the box
    lo, hi = np.array([1.0, 2.0, 0.5]), np.array([7.0, 5.0, 4.5])
    mesh = _box_mesh(lo, hi)
    rng = np.random.default_rng(11)
    p = rng.uniform(lo - 3.0, hi + 3.0, (20000, 3)).astype(np.float32)
    P = p.astype(np.float64)
    inside = np.all((P >= lo) & (P <= hi), 1)
    d_in = np.minimum(P - lo, hi - P).min(1)
    d_out = np.sqrt((np.maximum(np.maximum(lo - P, 0.0), P - hi) ** 2).sum(1))
    expect = np.where(inside, d_in, d_out).astype(np.float32)
    got = orc.edge_distance(p, mesh, np.inf, method="brute")
    assert inside.sum() > 1000 and (~inside).sum() > 1000
    assert _ulps(got, expect).max() <= 1
    g2 = orc.edge_distance(p, mesh, 1.5, method="grid")
    near = expect.astype(np.float64) < 1.5 * (1 - 1e-6)
    far = expect.astype(np.float64) > 1.5 * (1 + 1e-6)
    assert np.array_equal(g2[near], got[near]) and np.isinf(g2[far]).all()


def test_edge_sampled_triangles_bracket(orc):
    # the distance lies between the closest of a dense sample of the
    # triangle's points and that value less the sample spacing
    rng = np.random.default_rng(13)
    m = 60
    u, v = np.meshgrid(np.arange(m + 1) / m, np.arange(m + 1) / m)
    keep = (u + v) <= 1.0 + 1e-12
    u, v = u[keep], v[keep]
    for _ in range(20):
        T = rng.normal(0, 2, (3, 3)).astype(np.float32)
        q = rng.normal(0, 3, (50, 3)).astype(np.float32)
        S = T[0].astype(np.float64) + u[:, None] * (T[1] - T[0]).astype(np.float64) + \
            v[:, None] * (T[2] - T[0]).astype(np.float64)
        ds = np.sqrt(((q.astype(np.float64)[:, None, :] - S[None]) ** 2).sum(-1)).min(1)
        got = orc.edge_distance(q, T[None], np.inf, method="brute").astype(np.float64)
        spacing = max(np.linalg.norm((T[1] - T[0]).astype(np.float64)),
                      np.linalg.norm((T[2] - T[0]).astype(np.float64))) / m
        assert np.all(got <= ds * (1 + 1e-6) + 1e-6)
        assert np.all(got >= ds - spacing - 1e-6)


def test_edge_frustum_mesh_against_analytic_surface(orc, synth):
    # the hull is inscribed in the frustum: its distance differs from the
    # analytic surface distance by at most the chords' sagitta
    spec = synth.clustered_needle(30.0, 10.0, 6.0, seed=7)
    xyz, _, d_an = spec.generate()
    n_phi = 96
    mesh = synth.frustum_mesh(spec, n_phi, 60)
    got = orc.edge_distance(xyz, mesh, 3.0, method="grid")
    sag = spec.R0 * (1 - np.cos(np.pi / n_phi))
    near = d_an < 3.0 - sag - 1e-4
    assert near.sum() > 1000
    assert np.all(np.abs(got[near].astype(np.float64) - d_an[near]) <= sag + 1e-5)
    assert np.all(np.isinf(got[d_an > 3.0 + sag + 1e-4]))


def test_edge_brute_equals_grid_and_rigid_shift(orc, synth):
    spec = synth.clustered_needle(20.0, 8.0, 5.0, seed=9)
    xyz, _, _ = spec.generate()
    xyz = xyz[:20000].copy()
    xyz[5] = np.nan
    mesh = synth.frustum_mesh(spec, 48, 30)
    mesh[3, 1, 2] = np.inf                      # a triangle left out
    b = orc.edge_distance(xyz, mesh, 2.0, method="brute")
    g = orc.edge_distance(xyz, mesh, 2.0, method="grid")
    assert np.array_equal(b, g, equal_nan=True)
    assert np.isnan(b[5]) and np.isfinite(b).sum() > 1000
    # on a dyadic grid a shift by whole nanometres is exact: equal distances
    q = np.round(xyz[:3000] * 1024) / 1024
    t = np.round(mesh * 1024) / 1024
    t[3, 1, 2] = 0.5
    s = np.array([64.0, -128.0, 256.0], np.float32)
    d0 = orc.edge_distance(q.astype(np.float32), t.astype(np.float32), 2.0)
    d1 = orc.edge_distance((q + s).astype(np.float32), (t + s).astype(np.float32), 2.0)
    assert np.array_equal(d0, d1, equal_nan=True)
