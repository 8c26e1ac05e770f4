"""Host-side checks of the C ABI: the library loads, exports everything the
header declares, sizes workspaces, and rejects bad arguments before any GPU
work (these calls return before the first HIP call, so they run without a
GPU)."""
import ctypes
import glob
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def aptstat():
    import paper_2004_05188_amd as aptstat

    if not os.path.exists(aptstat.library_path()):
        aptstat.build()
    return aptstat


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(apt_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol(aptstat):
    L = aptstat.lib()
    names = _declared()
    assert {"apt_rdf", "apt_knn", "apt_knn_rdf", "apt_workspace_size", "apt_last_error"} <= names
    for name in names:
        assert hasattr(L, name), f"{name} declared in include/ but not exported"


def test_no_oracle_in_the_product():
    # the GPU library neither includes nor links the oracle
    for src in glob.glob(os.path.join(ROOT, "paper_2004_05188_amd", "**", "*"), recursive=True):
        if src.endswith((".hip", ".hpp", ".h", ".py")):
            text = open(src).read()
            assert "apt_oracle" not in text and "import oracle" not in text, src


def test_workspace_sizes(aptstat):
    for op in (aptstat.OP_RDF, aptstat.OP_KNN, aptstat.OP_KNN_RDF):
        a = aptstat.lib().apt_workspace_size(op, 1000, 0, 0)
        b = aptstat.lib().apt_workspace_size(op, 10_000_000, 0, 0)
        assert 0 < a < b
        assert b >= 40 * 10_000_000            # SoA, sort buffers and index lists
    assert aptstat.lib().apt_workspace_size(99, 1000, 0, 0) == 0
    assert aptstat.lib().apt_workspace_size(1, -1, 0, 0) == 0
    assert aptstat.lib().apt_workspace_size(1, 1 << 32, 0, 0) == 0


def _cloud(aptstat, n=10):
    c = aptstat._Cloud(0x1000, 0x2000, None, n)   # never dereferenced on the host
    return ctypes.byref(c)


def _err(aptstat):
    return aptstat.lib().apt_last_error().decode()


def test_argument_validation_before_gpu_work(aptstat):
    L = aptstat.lib()
    q = aptstat._query(1, 1, 0.0)
    good = aptstat._bins(2.0, 200)
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    st = ctypes.c_void_p(0x3000)
    h = ctypes.c_void_p(0x4000)
    # NULL cloud
    assert L.apt_rdf(None, q, good, h, st, ws, big, None) == -1
    assert "cloud" in _err(aptstat)
    # bad bins
    for bad in (aptstat._bins(0.0, 200), aptstat._bins(-1.0, 200), aptstat._bins(math.inf, 200),
                aptstat._bins(2.0, 0), aptstat._bins(2.0, 65537)):
        assert L.apt_rdf(_cloud(aptstat), q, bad, h, st, ws, big, None) == -1
    # NULL output, NULL status
    assert L.apt_rdf(_cloud(aptstat), q, good, None, st, ws, big, None) == -1
    assert L.apt_rdf(_cloud(aptstat), q, good, h, None, ws, big, None) == -1
    # NaN d_srf
    assert L.apt_rdf(_cloud(aptstat), aptstat._query(1, 1, math.nan), good, h, st, ws, big, None) == -1
    # too many ions
    c = aptstat._Cloud(0x1000, 0x2000, None, 1 << 32)
    assert L.apt_rdf(ctypes.byref(c), q, good, h, st, ws, big, None) == -3
    # workspace: NULL, misaligned, too small
    assert L.apt_rdf(_cloud(aptstat), q, good, h, st, None, big, None) == -2
    assert L.apt_rdf(_cloud(aptstat), q, good, h, st, ctypes.c_void_p(0x100001), big, None) == -2
    assert L.apt_rdf(_cloud(aptstat), q, good, h, st, ws, 1024, None) == -2
    assert "workspace" in _err(aptstat)


def test_knn_argument_validation(aptstat):
    L = aptstat.lib()
    q = aptstat._query(1, 1, 0.0)
    kb = aptstat._bins(5.0, 5000)
    p = ctypes.c_void_p(0x5000)
    ws, big = ctypes.c_void_p(0x100000), 1 << 40
    args = lambda k, rk, cap, tid: (_cloud(aptstat), q, k, rk, cap, tid, p, p, kb, None, p, p, ws, big, None)
    assert L.apt_knn(*args(0, math.inf, 10, p)) == -1          # k < 1
    assert L.apt_knn(*args(257, math.inf, 10, p)) == -3        # k too large
    assert L.apt_knn(*args(10, 0.0, 10, p)) == -1              # r_knn_max <= 0
    assert L.apt_knn(*args(10, math.nan, 10, p)) == -1
    assert L.apt_knn(*args(10, math.inf, -1, p)) == -1         # capacity < 0
    assert L.apt_knn(*args(10, math.inf, 10, None)) == -1      # NULL rows


def test_count_candidates_validation(aptstat):
    L = aptstat.lib()
    q = aptstat._query(1, 1, 0.0)
    p = ctypes.c_void_p(0x5000)
    ws, big = ctypes.c_void_p(0x100000), 1 << 40
    good = aptstat._bins(2.0, 200)
    assert L.apt_count_candidates(_cloud(aptstat), q, good, -1, p, p, ws, big, None) == -1
    assert L.apt_count_candidates(_cloud(aptstat), q, good, 0, None, p, ws, big, None) == -1
    assert "candidates" in _err(aptstat)
    assert L.apt_count_candidates(_cloud(aptstat), q, aptstat._bins(0.0, 200), 0, p, p, ws, big, None) == -1
    assert L.apt_count_candidates(_cloud(aptstat), q, good, 257, p, p, ws, big, None) == -3


def test_tuning_round_trip_and_validation(aptstat):
    """The tuning is host state: set, read back, rejected when out of range
    (unchanged then), and NULL restores the defaults."""
    try:
        aptstat.set_tuning(2, 3.0, 0.7, 0.5)
        assert aptstat.get_tuning() == {"tile_policy": 2, "cell_occ": 3.0, "h_min_frac": 0.699999988079071,
                                        "tile_occ": 0.5, "rdf_kernel": 0}
        for bad in ((5, 4.0, 0.5, 1.0), (-1, 4.0, 0.5, 1.0), (0, 0.0, 0.5, 1.0), (0, 4.0, math.nan, 1.0), (0, 4.0, 0.5, -1.0),
                    (0, 4.0, 0.5, math.inf), (0, 4.0, 0.5, 1.0, 3), (0, 4.0, 0.5, 1.0, -1)):
            with pytest.raises(aptstat.AptError):
                aptstat.set_tuning(*bad)
            assert aptstat.get_tuning()["tile_occ"] == 0.5
        aptstat.set_tuning(0, 4.0, 0.5, 0.0)           # 0 selects the default tile occupancy
        assert aptstat.get_tuning()["tile_occ"] == 1.0
        assert aptstat.lib().apt_set_tuning(None) == 0
        assert aptstat.get_tuning() == {"tile_policy": 0, "cell_occ": 4.0, "h_min_frac": 0.5, "tile_occ": 1.0,
                                        "rdf_kernel": 0}
    finally:
        aptstat.set_tuning()


def test_trace_enable_modes(aptstat):
    """0 off, 1 every stage, 2 the pair kernel only; anything else is refused."""
    L = aptstat.lib()
    try:
        for on in (0, 1, 2):
            assert L.apt_trace_enable(on) == 0
        for bad in (-1, 3, 7):
            assert L.apt_trace_enable(bad) == -1
            assert "apt_trace_enable" in _err(aptstat)
    finally:
        assert L.apt_trace_enable(0) == 0


def test_smooth_window_limit(aptstat):
    """sigma is limited by the edges one window buffers: 12 sigma may span
    up to 1020 bin widths; beyond, APT_E_UNSUPPORTED before any GPU work."""
    L = aptstat.lib()
    q = aptstat._query(1, 1, 0.0)
    bins = aptstat._bins(2.0, 200)                 # bin width 0.01 nm
    p = ctypes.c_void_p(0x5000)
    ws, big = ctypes.c_void_p(0x100000), 1 << 40
    # 12 sigma = 1030 widths: refused
    assert L.apt_rdf_smooth_fwd(_cloud(aptstat), q, bins, ctypes.c_float(0.01 * 1030 / 12), None, p, p, ws, big,
                                None) == -3
    assert "1020 bins" in _err(aptstat)
    # sigma <= 0 and NaN: invalid
    for bad in (0.0, -1.0, math.nan):
        assert L.apt_rdf_smooth_fwd(_cloud(aptstat), q, bins, ctypes.c_float(bad), None, p, p, ws, big, None) == -1


def test_batched_histogram_size_limit(aptstat):
    # the batched histograms are zeroed and indexed with 32-bit counts: calls
    # whose n_rep * n_pairs * bins reach 2^31 are rejected before GPU work
    L = aptstat.lib()
    p = ctypes.c_void_p(0x5000)
    ws, big = ctypes.c_void_p(0x100000), 1 << 40
    qs = (aptstat._Query * 16)(*[aptstat._query(a % 3, (a + 1) % 3, 1.0) for a in range(16)])
    n_rep = 2048
    seeds = (ctypes.c_uint64 * n_rep)(*range(1, n_rep + 1))
    rb, kb = aptstat._bins(2.0, 200), aptstat._bins(5.0, 65536)
    assert L.apt_rdf_batched(_cloud(aptstat), qs, 16, seeds, n_rep, rb, 10, kb, p, p, None, p, ws, big,
                             None) == -3
    assert "2^31" in _err(aptstat)
    # the same call without the k-th histogram passes the size check (and
    # stops at the workspace check instead)
    assert L.apt_rdf_batched(_cloud(aptstat), qs, 16, seeds, n_rep, rb, 10, kb, p, None, None, p, None, big,
                             None) == -2


def test_cluster_argument_validation(aptstat):
    L = aptstat.lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    lab, cnt, st, hist = (ctypes.c_void_p(a) for a in (0x3000, 0x4000, 0x5000, 0x6000))
    assert aptstat.lib().apt_workspace_size(aptstat.OP_CLUSTER, 1000, 0, 0) == \
        aptstat.lib().apt_workspace_size(aptstat.OP_RDF, 1000, 0, 0)

    def call(cloud=None, d_max=0.5, n_min=5, d_srf=0.0, label=lab, counts=cnt, h=None, nb=0, status=st, w=ws,
             wb=big):
        return L.apt_cluster_ms(cloud if cloud is not None else _cloud(aptstat), 1, d_max, n_min, d_srf, label,
                                counts, h, nb, status, w, wb, None)

    for bad in (0.0, -1.0, math.inf, math.nan):
        assert call(d_max=bad) == -1 and "d_max" in _err(aptstat)
    assert call(n_min=0) == -1 and "n_min" in _err(aptstat)
    assert call(d_srf=math.nan) == -1
    assert call(h=hist, nb=0) == -1 and call(h=hist, nb=65537) == -1
    assert call(counts=None) == -1 and call(status=None) == -1 and call(label=None) == -1
    c = aptstat._Cloud(0x1000, 0x2000, None, 1 << 31)
    assert call(cloud=ctypes.byref(c)) == -3 and "2^31" in _err(aptstat)
    assert call(w=None) == -2 and call(wb=1024) == -2


def test_edge_argument_validation(aptstat):
    L = aptstat.lib()
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 40
    tri, d, st = (ctypes.c_void_p(a) for a in (0x3000, 0x4000, 0x5000))
    a = L.apt_edge_workspace_size(1000, 100)
    assert a > L.apt_workspace_size(aptstat.OP_RDF, 1000, 0, 0)
    assert L.apt_edge_workspace_size(1000, 10_000_000) > a
    assert L.apt_edge_workspace_size(-1, 1) == 0 and L.apt_edge_workspace_size(1, -1) == 0

    def call(n_tri=100, t=tri, d_prb=2.5, out=d, status=st, w=ws, wb=big):
        return L.apt_edge_distance(_cloud(aptstat), t, n_tri, d_prb, out, status, w, wb, None)

    assert call(n_tri=-1) == -1
    assert call(n_tri=1 << 32) == -3
    assert call(t=None) == -1 and "tri" in _err(aptstat)
    for bad in (0.0, -1.0, math.nan):
        assert call(d_prb=bad) == -1 and "d_prb" in _err(aptstat)
    assert call(out=None) == -1 and call(status=None) == -1
    assert call(w=None) == -2 and call(wb=1024) == -2
