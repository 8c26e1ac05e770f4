"""Spatial statistics of atom-probe point clouds on the MI355X (gfx950).

Thin Python binding of ``libaptstat.so`` (C ABI in ``include/apt_stat.h``).
Arguments are torch tensors on the GPU; the binding only checks dtypes and
shapes, passes raw device pointers and the current HIP stream, and raises
on a non-zero return code.  Every step of the computation runs in the
library's HIP kernels; there is no CPU fallback: without the built library
every call raises.

Species are small integers (0..254); ``ANY`` (255) selects every species.
uint64 histograms are returned in int64 tensors (counts < 2^63).
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

from . import _build

ANY = 255
_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libaptstat.so")

STATUS_NONFINITE = 1
STATUS_CAPACITY = 2
OP_RDF, OP_KNN, OP_KNN_RDF, OP_PERMUTE, OP_BATCHED, OP_SMOOTH, OP_SDM, OP_CLUSTER = 1, 2, 3, 4, 5, 6, 7, 8


class AptError(RuntimeError):
    pass


class _Cloud(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("lab", ctypes.c_void_p), ("d_bnd", ctypes.c_void_p),
                ("n", ctypes.c_int64)]


class _Query(ctypes.Structure):
    _fields_ = [("target", ctypes.c_uint8), ("neighbor", ctypes.c_uint8), ("pad", ctypes.c_uint8 * 2),
                ("d_srf", ctypes.c_float)]


class _Tuning(ctypes.Structure):
    _fields_ = [("tile_policy", ctypes.c_int32), ("cell_occ", ctypes.c_float), ("h_min_frac", ctypes.c_float),
                ("tile_occ", ctypes.c_float), ("rdf_kernel", ctypes.c_int32)]


class _BatchedTuning(ctypes.Structure):
    _fields_ = [("cell_frac", ctypes.c_float), ("rep_block", ctypes.c_int32), ("tile_reach", ctypes.c_float),
                ("tiles", ctypes.c_int32)]


BATCHED_TUNING_KEYS = ("cell_frac", "rep_block", "tile_reach", "tiles")


class _Bins(ctypes.Structure):
    _fields_ = [("r_max", ctypes.c_float), ("n_bins", ctypes.c_int32)]


_P = ctypes.c_void_p
_lib = None

_SIGS = {
    "apt_workspace_size": ([ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32], ctypes.c_size_t),
    "apt_last_error": ([], ctypes.c_char_p),
    "apt_trace_enable": ([ctypes.c_int32], ctypes.c_int),
    "apt_set_tuning": ([ctypes.POINTER(_Tuning)], ctypes.c_int),
    "apt_get_tuning": ([ctypes.POINTER(_Tuning)], ctypes.c_int),
    "apt_trace_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
                       ctypes.c_int),
    "apt_count_targets": ([ctypes.POINTER(_Cloud), _Query, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "apt_count_candidates": ([ctypes.POINTER(_Cloud), _Query, _Bins, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t,
                              _P], ctypes.c_int),
    "apt_permute_labels": ([_P, ctypes.c_int64, ctypes.c_uint64, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "apt_rdf_batched": ([ctypes.POINTER(_Cloud), _P, ctypes.c_int32, _P, ctypes.c_int32, _Bins, ctypes.c_int32,
                         _Bins, _P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "apt_batched_plan": ([ctypes.POINTER(_Cloud), _P, ctypes.c_int32, _Bins, ctypes.c_int32, _Bins, ctypes.c_int32,
                          _P, _P], ctypes.c_int),
    "apt_batched_plan_clear": ([], ctypes.c_int),
    "apt_rdf": ([ctypes.POINTER(_Cloud), _Query, _Bins, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "apt_rdf_noalloc": ([ctypes.POINTER(_Cloud), _Query, _Bins, _P, _P, _P], ctypes.c_int),
    "apt_edge_workspace_size": ([ctypes.c_int64, ctypes.c_int64], ctypes.c_size_t),
    "apt_edge_distance": ([ctypes.POINTER(_Cloud), _P, ctypes.c_int64, ctypes.c_float, _P, _P, _P, ctypes.c_size_t,
                           _P], ctypes.c_int),
    "apt_cluster_ms": ([ctypes.POINTER(_Cloud), ctypes.c_uint8, ctypes.c_float, ctypes.c_int32, ctypes.c_float, _P, _P,
                        _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "apt_sdm": ([ctypes.POINTER(_Cloud), _Query, ctypes.c_float, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P],
                ctypes.c_int),
    "apt_knn": ([ctypes.POINTER(_Cloud), _Query, ctypes.c_int32, ctypes.c_float, ctypes.c_int64, _P, _P, _P,
                 _Bins, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "apt_knn_rdf": ([ctypes.POINTER(_Cloud), _Query, _Bins, _P, ctypes.c_int32, ctypes.c_float, ctypes.c_int64,
                     _P, _P, _P, _Bins, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "apt_rdf_smooth_fwd": ([ctypes.POINTER(_Cloud), _Query, _Bins, ctypes.c_float, _P, _P, _P, _P, ctypes.c_size_t,
                            _P], ctypes.c_int),
    "apt_rdf_smooth_bwd": ([ctypes.POINTER(_Cloud), _Query, _Bins, ctypes.c_float, _P, _P, _P, _P, _P, _P,
                            ctypes.c_size_t, _P], ctypes.c_int),
}


def library_path() -> str:
    return _SO


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise AptError(f"{_SO} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = ctypes.CDLL(_SO)
        for name, (args, res) in _SIGS.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
        _lib = L
    return _lib


def build() -> str:
    global _lib
    _lib = None
    return _build.build()


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().apt_last_error()
        raise AptError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise AptError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise AptError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise AptError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Cloud:
    """Positions xyz (float32 [n,3]), labels lab (uint8 [n]) and optional
    distance-to-surface d_bnd (float32 [n]), all on one GPU."""

    def __init__(self, xyz: torch.Tensor, lab: torch.Tensor, d_bnd: torch.Tensor | None = None):
        n = xyz.shape[0]
        _need(xyz, torch.float32, (n, 3), "xyz")
        _need(lab, torch.uint8, (n,), "lab")
        if d_bnd is not None:
            _need(d_bnd, torch.float32, (n,), "d_bnd")
            if d_bnd.device != xyz.device:
                raise AptError("d_bnd is on another device")
        if lab.device != xyz.device:
            raise AptError("lab is on another device")
        self.xyz, self.lab, self.d_bnd, self.n = xyz, lab, d_bnd, n
        self.device = xyz.device
        self._c = _Cloud(xyz.data_ptr(), lab.data_ptr(), d_bnd.data_ptr() if d_bnd is not None else None, n)

    def c(self):
        return ctypes.byref(self._c)


class Workspace:
    """Device scratch for the library calls; grows on demand and is reused."""

    def __init__(self, device=None):
        self.device = torch.device(device) if device is not None else None
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


def set_tuning(tile_policy: int = 0, cell_occ: float = 4.0, h_min_frac: float = 0.5, tile_occ: float = 1.0,
               rdf_kernel: int = 0):
    """Process-wide speed knobs (results do not depend on them).

    tile_policy: 0 automatic, 1 one target per wavefront, 2 64 targets per
    wavefront sharing staged candidates, 3 one target per lane, 4 the kNN one
    target per lane and the RDF one target per wavefront; rdf_kernel: the
    RDF kernel of the dense-neighbour mode (0 automatic, 1 neighbour-major,
    2 one target per wavefront)."""
    t = _Tuning(int(tile_policy), float(cell_occ), float(h_min_frac), float(tile_occ), int(rdf_kernel))
    _check(lib().apt_set_tuning(ctypes.byref(t)), "apt_set_tuning")


def get_tuning() -> dict:
    t = _Tuning()
    _check(lib().apt_get_tuning(ctypes.byref(t)), "apt_get_tuning")
    return {"tile_policy": t.tile_policy, "cell_occ": t.cell_occ, "h_min_frac": t.h_min_frac,
            "tile_occ": t.tile_occ, "rdf_kernel": t.rdf_kernel}


def trace_enable(on: bool = True, pair_only: bool = False):
    """Record HIP events around the stages of every following call (only
    around the pair kernel with pair_only)."""
    _check(lib().apt_trace_enable((2 if pair_only else 1) if on else 0), "apt_trace_enable")


def trace_read(stage: str):
    """(total ms, launches) of one stage ("binning", "pair", "tile", "permute" or
    "partition") since the last read."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(lib().apt_trace_read(stage.encode(), ctypes.byref(ms), ctypes.byref(n)), "apt_trace_read")
    return ms.value, n.value


def workspace_size(op: int, n: int, n_pairs: int = 0, n_rep: int = 0) -> int:
    s = lib().apt_workspace_size(op, n, n_pairs, n_rep)
    if s == 0:
        raise AptError(f"no workspace size for op {op}, n = {n}")
    return int(s)


def _query(target: int, neighbor: int, d_srf: float) -> _Query:
    q = _Query()
    q.target, q.neighbor, q.d_srf = int(target), int(neighbor), float(d_srf)
    return q


def _bins(r_max: float, n_bins: int) -> _Bins:
    b = _Bins()
    b.r_max, b.n_bins = float(r_max), int(n_bins)
    return b


def _ws(ws, op, cloud, n_pairs=0, n_rep=0):
    ws = ws if ws is not None else Workspace()
    nb = workspace_size(op, cloud.n, n_pairs, n_rep)
    return ws.get(nb, cloud.device), nb


def count_targets(cloud: Cloud, target: int, d_srf: float = 0.0, ws: Workspace | None = None,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """Eligible-target count as a device int64 tensor [1] (no host sync)."""
    buf, nb = _ws(ws, OP_KNN, cloud)
    out = out if out is not None else torch.empty(1, dtype=torch.int64, device=cloud.device)
    _check(lib().apt_count_targets(cloud.c(), _query(target, ANY, d_srf), _ptr(out), _ptr(buf), nb,
                                   _stream(cloud.xyz)), "apt_count_targets")
    return out


def count_candidates(cloud: Cloud, target: int, neighbor: int, d_srf: float, r_max: float = 2.0, n_bins: int = 200,
                     k: int = 0, ws: Workspace | None = None) -> torch.Tensor:
    """Diagnostic: neighbour records the pair kernel's first enumeration visits
    over all eligible targets (int64 tensor [1]); see apt_count_candidates."""
    buf, nb = _ws(ws, OP_KNN_RDF, cloud)
    out = torch.empty(1, dtype=torch.int64, device=cloud.device)
    status = torch.empty(1, dtype=torch.int32, device=cloud.device)
    _check(lib().apt_count_candidates(cloud.c(), _query(target, neighbor, d_srf), _bins(r_max, n_bins), int(k),
                                      _ptr(out), _ptr(status), _ptr(buf), nb, _stream(cloud.xyz)),
           "apt_count_candidates")
    return out


def permute_labels(lab: torch.Tensor, seed: int, out: torch.Tensor | None = None,
                   ws: Workspace | None = None, status: torch.Tensor | None = None) -> torch.Tensor:
    """Labels reordered by the SplitMix64-key permutation of `seed` (uint8 [n])."""
    n = lab.shape[0]
    _need(lab, torch.uint8, (n,), "lab")
    out = out if out is not None else torch.empty_like(lab)
    _need(out, torch.uint8, (n,), "out")
    ws = ws if ws is not None else Workspace()
    nb = workspace_size(OP_PERMUTE, n)
    buf = ws.get(nb, lab.device)
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=lab.device)
    _check(lib().apt_permute_labels(_ptr(lab), n, ctypes.c_uint64(seed & (2**64 - 1)), _ptr(out), _ptr(status),
                                    _ptr(buf), nb, _stream(lab)), "apt_permute_labels")
    return out


def rdf_batched(cloud: Cloud, pairs, seeds, r_max: float = 2.0, n_bins: int = 200, k: int = 10,
                kb_rmax: float = 5.0, kb_nbins: int = 5000, want_knn: bool = True,
                ws: Workspace | None = None, out=None, tuning: dict | None = None):
    """Null-model replicates: pairs = [(A, B, d_srf), ...], seeds = [seed_r, ...].

    Returns (rdf int64 [n_rep, n_pairs, n_bins], knn int64 [n_rep, n_pairs, kb_nbins + 1] or None,
    status int32 [1]); (r, p) equals knn_rdf of pair p on permute_labels(lab, seeds[r]).
    tuning: {cell_frac, rep_block, tile_reach, tiles} (missing keys: 0, the
    library's default), or None for the library's cached autotuned plan."""
    n_pairs, n_rep = len(pairs), len(seeds)
    qs = (_Query * n_pairs)(*[_query(a, b, d) for a, b, d in pairs])
    sd = (ctypes.c_uint64 * n_rep)(*[int(x) & (2**64 - 1) for x in seeds])
    dev = cloud.device
    if out is None:
        rh = torch.empty((n_rep, n_pairs, n_bins), dtype=torch.int64, device=dev)
        kh = torch.empty((n_rep, n_pairs, kb_nbins + 1), dtype=torch.int64, device=dev) if want_knn else None
        st = torch.empty(1, dtype=torch.int32, device=dev)
    else:
        rh, kh, st = out
    ws = ws if ws is not None else Workspace()
    nb = workspace_size(OP_BATCHED, cloud.n, n_pairs, n_rep)
    buf = ws.get(nb, dev)
    tu = None
    if tuning is not None:
        unknown = set(tuning) - set(BATCHED_TUNING_KEYS)
        if unknown:
            raise ValueError(f"unknown batched tuning keys {sorted(unknown)}")
        tu = ctypes.byref(_BatchedTuning(float(tuning.get("cell_frac", 0.0)), int(tuning.get("rep_block", 0)),
                                         float(tuning.get("tile_reach", 0.0)), int(tuning.get("tiles", 0))))
    _check(lib().apt_rdf_batched(cloud.c(), qs, n_pairs, sd, n_rep, _bins(r_max, n_bins), int(k),
                                 _bins(kb_rmax, kb_nbins), _ptr(rh), _ptr(kh), tu, _ptr(st), _ptr(buf), nb,
                                 _stream(cloud.xyz)), "apt_rdf_batched")
    return rh, kh, st


def batched_plan(cloud: Cloud, pairs, r_max: float = 2.0, n_bins: int = 200, k: int = 10, kb_rmax: float = 5.0,
                 kb_nbins: int = 5000, want_knn: bool = True):
    """The cached plan rdf_batched(tuning=None) uses for these arguments, or None."""
    n_pairs = len(pairs)
    qs = (_Query * n_pairs)(*[_query(a, b, d) for a, b, d in pairs])
    out = _BatchedTuning()
    cached = ctypes.c_int32(0)
    _check(lib().apt_batched_plan(cloud.c(), qs, n_pairs, _bins(r_max, n_bins), int(k), _bins(kb_rmax, kb_nbins),
                                  int(bool(want_knn)), ctypes.byref(out), ctypes.byref(cached)), "apt_batched_plan")
    if not cached.value:
        return None
    return {kk: getattr(out, kk) for kk in BATCHED_TUNING_KEYS}


def batched_plan_clear():
    """Empty the library's batched plan and graph caches."""
    _check(lib().apt_batched_plan_clear(), "apt_batched_plan_clear")


def rdf(cloud: Cloud, target: int, neighbor: int, d_srf: float, r_max: float, n_bins: int,
        ws: Workspace | None = None, out: torch.Tensor | None = None, status: torch.Tensor | None = None):
    """Ordered-pair counts per bin [0, r_max) / n_bins: int64 tensor [n_bins]."""
    buf, nb = _ws(ws, OP_RDF, cloud)
    dev = cloud.device
    out = out if out is not None else torch.empty(n_bins, dtype=torch.int64, device=dev)
    _need(out, torch.int64, (n_bins,), "out")
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().apt_rdf(cloud.c(), _query(target, neighbor, d_srf), _bins(r_max, n_bins), _ptr(out),
                         _ptr(status), _ptr(buf), nb, _stream(cloud.xyz)), "apt_rdf")
    return out


def sdm(cloud: Cloud, target: int, neighbor: int, d_srf: float, R: float = 2.0, n_vox: int = 160,
        ws: Workspace | None = None, out: torch.Tensor | None = None, status: torch.Tensor | None = None):
    """Two-point statistic: counts of pair displacement vectors p_j - p_i within R
    per cubic voxel of [-R, R)^3: int64 tensor [n_vox, n_vox, n_vox] indexed [mz, my, mx]."""
    buf, nb = _ws(ws, OP_SDM, cloud)
    dev = cloud.device
    out = out if out is not None else torch.empty((n_vox, n_vox, n_vox), dtype=torch.int64, device=dev)
    _need(out, torch.int64, (n_vox, n_vox, n_vox), "out")
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().apt_sdm(cloud.c(), _query(target, neighbor, d_srf), float(R), int(n_vox), _ptr(out),
                         _ptr(status), _ptr(buf), nb, _stream(cloud.xyz)), "apt_sdm")
    return out


def edge_distance(cloud: Cloud, tri: torch.Tensor, d_prb: float = float("inf"), ws: Workspace | None = None,
                  out: torch.Tensor | None = None, status: torch.Tensor | None = None):
    """Distance of every ion to the closest point of the triangle hull `tri`
    (float32 [n_tri, 3, 3] on the cloud's device): float32 [n], +inf at or
    beyond d_prb, NaN for a non-finite position.  Returns (d, status)."""
    dev = cloud.device
    _need(tri, torch.float32, None, "tri")
    if tri.dim() != 3 or tri.shape[1:] != (3, 3) or not tri.is_contiguous():
        raise AptError("tri must be a contiguous float32 tensor [n_tri, 3, 3]")
    n_tri = tri.shape[0]
    nb = lib().apt_edge_workspace_size(cloud.n, n_tri)
    if nb == 0:
        raise AptError("cloud or hull too large for apt_edge_distance")
    ws = ws if ws is not None else Workspace()
    buf = ws.get(nb, dev)
    d = out if out is not None else torch.empty(max(cloud.n, 1), dtype=torch.float32, device=dev)
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().apt_edge_distance(cloud.c(), _ptr(tri) if n_tri else None, n_tri, float(d_prb), _ptr(d),
                                   _ptr(status), _ptr(buf), nb, _stream(cloud.xyz)), "apt_edge_distance")
    return d[:cloud.n], status


def cluster_ms(cloud: Cloud, species: int, d_max: float, n_min: int, d_srf: float = 0.0, n_size_bins: int = 0,
               ws: Workspace | None = None, status: torch.Tensor | None = None):
    """Maximum-separation clustering of the ions of `species`: (label int64 [n]:
    the smallest ion index of the ion's kept cluster or -1, counts int64 [3]:
    kept clusters, kept clusters with an ion at the edge, ions in kept
    clusters, size_hist int64 [n_size_bins] or None, status int32 [1])."""
    buf, nb = _ws(ws, OP_CLUSTER, cloud)
    dev = cloud.device
    label = torch.empty(max(cloud.n, 1), dtype=torch.int64, device=dev)
    counts = torch.empty(3, dtype=torch.int64, device=dev)
    hist = torch.empty(n_size_bins, dtype=torch.int64, device=dev) if n_size_bins > 0 else None
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().apt_cluster_ms(cloud.c(), int(species), float(d_max), int(n_min), float(d_srf), _ptr(label),
                                _ptr(counts), _ptr(hist), int(n_size_bins), _ptr(status), _ptr(buf), nb,
                                _stream(cloud.xyz)), "apt_cluster_ms")
    return label[:cloud.n], counts, hist, status


class KnnResult:
    def __init__(self, target_id, dist, nbr_id, knn_hist, n_targets, status, rdf_hist=None):
        self.target_id, self.dist, self.nbr_id = target_id, dist, nbr_id
        self.knn_hist, self.n_targets, self.status, self.rdf_hist = knn_hist, n_targets, status, rdf_hist

    def trimmed(self):
        """(target_id, dist, nbr_id) cut to the number of targets (host sync)."""
        t = min(int(self.n_targets.item()), self.target_id.shape[0])
        return self.target_id[:t], self.dist[:t], self.nbr_id[:t]


def _knn_outputs(dev, capacity, k, kb_nbins, want_hist):
    return (torch.empty(max(capacity, 1), dtype=torch.int64, device=dev),
            torch.empty((max(capacity, 1), k), dtype=torch.float32, device=dev),
            torch.empty((max(capacity, 1), k), dtype=torch.int64, device=dev),
            torch.empty(kb_nbins + 1, dtype=torch.int64, device=dev) if want_hist else None,
            torch.empty(1, dtype=torch.int64, device=dev),
            torch.empty(1, dtype=torch.int32, device=dev))


def knn_rdf(cloud: Cloud, target: int, neighbor: int, d_srf: float, k: int, r_max: float = 2.0,
            n_bins: int = 200, r_knn_max: float = math.inf, capacity: int | None = None,
            kb_rmax: float = 5.0, kb_nbins: int = 5000, want_rdf: bool = True, want_hist: bool = True,
            ws: Workspace | None = None, outputs=None) -> KnnResult:
    """kNN rows (and optionally the RDF) of one query from one enumeration.

    capacity: rows to allocate; None counts the eligible targets first (one
    extra small library call and a host sync)."""
    dev = cloud.device
    if capacity is None:
        capacity = int(count_targets(cloud, target, d_srf, ws=ws).item())
    if outputs is None:
        tid, dist, nid, kh, nt, st = _knn_outputs(dev, capacity, k, kb_nbins, want_hist)
        rh = torch.empty(n_bins, dtype=torch.int64, device=dev) if want_rdf else None
    else:
        tid, dist, nid, kh, nt, st, rh = outputs
    op = OP_KNN_RDF if want_rdf else OP_KNN
    buf, nb = _ws(ws, op, cloud)
    s = _stream(cloud.xyz)
    if want_rdf:
        _check(lib().apt_knn_rdf(cloud.c(), _query(target, neighbor, d_srf), _bins(r_max, n_bins), _ptr(rh),
                                 int(k), float(r_knn_max), int(capacity), _ptr(tid), _ptr(dist), _ptr(nid),
                                 _bins(kb_rmax, kb_nbins), _ptr(kh), _ptr(nt), _ptr(st), _ptr(buf), nb, s),
               "apt_knn_rdf")
    else:
        _check(lib().apt_knn(cloud.c(), _query(target, neighbor, d_srf), int(k), float(r_knn_max),
                             int(capacity), _ptr(tid), _ptr(dist), _ptr(nid), _bins(kb_rmax, kb_nbins),
                             _ptr(kh), _ptr(nt), _ptr(st), _ptr(buf), nb, s), "apt_knn")
    return KnnResult(tid, dist, nid, kh, nt, st, rh)


def knn(cloud: Cloud, target: int, neighbor: int, d_srf: float, k: int, **kw) -> KnnResult:
    return knn_rdf(cloud, target, neighbor, d_srf, k, want_rdf=False, **kw)


# ---------------------------------------------------------------- smoothed RDF --
def _zscale(z_scale, dev):
    if z_scale is None:
        return None
    _need(z_scale, torch.float64, None, "z_scale")
    if z_scale.numel() != 1:
        raise AptError("z_scale must hold one value")
    if z_scale.device != dev:
        raise AptError("z_scale is on another device")
    return z_scale


def rdf_smooth(cloud: Cloud, target: int, neighbor: int, d_srf: float, r_max: float, n_bins: int, sigma: float,
               z_scale: torch.Tensor | None = None, ws: Workspace | None = None, out: torch.Tensor | None = None,
               status: torch.Tensor | None = None) -> torch.Tensor:
    """Gaussian-smoothed RDF (float64 [n_bins]) with positions (x, y, s z),
    s = z_scale (float64 device tensor with one value, or None for 1)."""
    dev = cloud.device
    zs = _zscale(z_scale, dev)
    buf, nb = _ws(ws, OP_SMOOTH, cloud)
    out = out if out is not None else torch.empty(n_bins, dtype=torch.float64, device=dev)
    _need(out, torch.float64, (n_bins,), "out")
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().apt_rdf_smooth_fwd(cloud.c(), _query(target, neighbor, d_srf), _bins(r_max, n_bins),
                                    float(sigma), _ptr(zs), _ptr(out), _ptr(status), _ptr(buf), nb,
                                    _stream(cloud.xyz)), "apt_rdf_smooth_fwd")
    return out


def rdf_smooth_grad(cloud: Cloud, target: int, neighbor: int, d_srf: float, r_max: float, n_bins: int,
                    sigma: float, grad_h: torch.Tensor, z_scale: torch.Tensor | None = None,
                    want_grad_s: bool = True, ws: Workspace | None = None, status: torch.Tensor | None = None):
    """Adjoint of rdf_smooth: (dL/dxyz float32 [n, 3], dL/ds float64 [1] or None)."""
    dev = cloud.device
    zs = _zscale(z_scale, dev)
    _need(grad_h, torch.float64, (n_bins,), "grad_h")
    buf, nb = _ws(ws, OP_SMOOTH, cloud)
    gx = torch.empty((cloud.n, 3), dtype=torch.float32, device=dev)
    gs = torch.empty(1, dtype=torch.float64, device=dev) if want_grad_s else None
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().apt_rdf_smooth_bwd(cloud.c(), _query(target, neighbor, d_srf), _bins(r_max, n_bins),
                                    float(sigma), _ptr(zs), _ptr(grad_h), _ptr(gx), _ptr(gs), _ptr(status),
                                    _ptr(buf), nb, _stream(cloud.xyz)), "apt_rdf_smooth_bwd")
    return gx, gs


class RdfSmooth(torch.autograd.Function):
    """h = RdfSmooth.apply(xyz, z_scale, lab, d_bnd, target, neighbor, d_srf, r_max, n_bins, sigma)

    Differentiable in xyz (float32 [n, 3]) and z_scale (float64 tensor with
    one value); the backward recomputes the pairs in the library's adjoint
    kernel.  lab and d_bnd are constants (d_bnd may be None)."""

    @staticmethod
    def forward(ctx, xyz, z_scale, lab, d_bnd, target, neighbor, d_srf, r_max, n_bins, sigma):
        xyz_d = xyz.detach()
        zs = z_scale.detach().reshape(1) if z_scale is not None else None
        cloud = Cloud(xyz_d, lab, d_bnd)
        h = rdf_smooth(cloud, target, neighbor, d_srf, r_max, n_bins, sigma, z_scale=zs)
        ctx.save_for_backward(xyz_d, zs, lab, d_bnd)
        ctx.args = (target, neighbor, d_srf, r_max, n_bins, sigma)
        ctx.zshape = None if z_scale is None else z_scale.shape
        return h

    @staticmethod
    def backward(ctx, grad_h):
        xyz, zs, lab, d_bnd = ctx.saved_tensors
        target, neighbor, d_srf, r_max, n_bins, sigma = ctx.args
        want_s = zs is not None and ctx.needs_input_grad[1]
        gx, gs = rdf_smooth_grad(Cloud(xyz, lab, d_bnd), target, neighbor, d_srf, r_max, n_bins, sigma,
                                 grad_h.contiguous().to(torch.float64), z_scale=zs, want_grad_s=want_s)
        return (gx if ctx.needs_input_grad[0] else None, gs.reshape(ctx.zshape) if want_s else None,
                None, None, None, None, None, None, None, None)

