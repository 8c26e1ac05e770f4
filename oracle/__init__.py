"""TEST INFRASTRUCTURE ONLY: ctypes front end of the CPU oracle (``apt_oracle.c``).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports it, and it imports
nothing from the GPU library.  Arrays are numpy, host memory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libaptoracle.so")
ANY = 255


def build(force: bool = True) -> str:
    """Compile the oracle: plain C, -O2, no contraction, no fast-math, OpenMP."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
                               os.path.join(_HERE, "apt_oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None
_p = ctypes.c_void_p
_i32, _i64, _u64, _f32, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float, ctypes.c_double


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        sig = {
            "orc_threads": ([], _i32),
            "orc_set_threads": ([_i32], None),
            "orc_sdm_faces": ([_f32, _i32, _p], None),
            "orc_sdm_brute": ([_p, _p, _p, _i64, _i32, _i32, _f32, _f32, _i32, _p], None),
            "orc_sdm_grid": ([_p, _p, _p, _i64, _i32, _i32, _f32, _f32, _i32, _p], None),
            "orc_cluster_ms_brute": ([_p, _p, _p, _i64, _i32, _f32, _i32, _f32, _p, _p, _p, _i32], None),
            "orc_cluster_ms_grid": ([_p, _p, _p, _i64, _i32, _f32, _i32, _f32, _p, _p, _p, _i32], None),
            "orc_edge_brute": ([_p, _i64, _p, _i64, _f32, _p], None),
            "orc_edge_grid": ([_p, _i64, _p, _i64, _f32, _p], None),
            "orc_d2f": ([_p, _p], _f32),
            "orc_D2": ([_p, _p], _f64),
            "orc_edges2": ([_f32, _i32, _p], None),
            "orc_bin_of": ([_f64, _p, _i32], _i32),
            "orc_select_targets": ([_i64, _p, _p, _i32, _f32, _p], _i64),
            "orc_rdf_brute": ([_p, _p, _p, _i64, _i32, _i32, _f32, _f32, _i32, _p], None),
            "orc_rdf_grid": ([_p, _p, _p, _i64, _i32, _i32, _f32, _f32, _i32, _p], None),
            "orc_knn_brute": ([_p, _p, _p, _i64, _i32, _i32, _f32, _i32, _f32, _p, _p, _p, _f32, _i32, _p], _i64),
            "orc_knn_grid": ([_p, _p, _p, _i64, _i32, _i32, _f32, _i32, _f32, _p, _p, _p, _f32, _i32, _p], _i64),
            "orc_splitmix64": ([_u64, _u64], _u64),
            "orc_permute_labels": ([_p, _i64, _u64, _p], None),
            "orc_smooth_fwd": ([_p, _p, _p, _i64, _i32, _i32, _f32, _f32, _i32, _f32, _f64, _p], None),
            "orc_smooth_bwd": ([_p, _p, _p, _i64, _i32, _i32, _f32, _f32, _i32, _f32, _f64, _p, _p, _p], None),
            "orc_smooth_fd": ([_p, _p, _p, _i64, _i32, _i32, _f32, _f32, _i32, _f32, _f64, _p, _p, _i64, _f64, _p],
                              None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _cloud(xyz, lab, d_bnd):
    xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    lab = np.ascontiguousarray(lab, dtype=np.uint8).reshape(-1)
    assert lab.shape[0] == xyz.shape[0]
    if d_bnd is not None:
        d_bnd = np.ascontiguousarray(d_bnd, dtype=np.float32).reshape(-1)
        assert d_bnd.shape[0] == xyz.shape[0]
    return xyz, lab, d_bnd


def threads() -> int:
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Threads the oracle's OpenMP loops use from now on."""
    _load().orc_set_threads(int(n))


def d2f(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    return _load().orc_d2f(a.ctypes.data, b.ctypes.data)


def D2(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    return _load().orc_D2(a.ctypes.data, b.ctypes.data)


def edges2(r_max: float, n_bins: int) -> np.ndarray:
    E2 = np.empty(n_bins + 1, dtype=np.float64)
    _load().orc_edges2(r_max, n_bins, E2.ctypes.data)
    return E2


def bin_of(D2v: float, E2: np.ndarray) -> int:
    E2 = np.ascontiguousarray(E2, dtype=np.float64)
    return _load().orc_bin_of(D2v, E2.ctypes.data, len(E2) - 1)


def select_targets(lab, d_bnd, A: int, d_srf: float) -> np.ndarray:
    lab = np.ascontiguousarray(lab, dtype=np.uint8)
    if d_bnd is not None:
        d_bnd = np.ascontiguousarray(d_bnd, dtype=np.float32)
    out = np.empty(len(lab), dtype=np.int64)
    t = _load().orc_select_targets(len(lab), lab.ctypes.data, _ptr(d_bnd), A, d_srf, out.ctypes.data)
    return out[:t].copy()


def rdf(xyz, lab, d_bnd, A: int, B: int, d_srf: float, r_max: float, n_bins: int,
        method: str = "grid") -> np.ndarray:
    """Ordered-pair counts per bin (uint64 [n_bins])."""
    xyz, lab, d_bnd = _cloud(xyz, lab, d_bnd)
    hist = np.zeros(n_bins, dtype=np.uint64)
    f = _load().orc_rdf_grid if method == "grid" else _load().orc_rdf_brute
    f(xyz.ctypes.data, lab.ctypes.data, _ptr(d_bnd), xyz.shape[0], A, B, d_srf, r_max, n_bins,
      hist.ctypes.data)
    return hist


def knn(xyz, lab, d_bnd, A: int, B: int, d_srf: float, k: int, r_knn_max: float = float("inf"),
        kb_rmax: float = 5.0, kb_nbins: int = 5000, method: str = "grid", want_hist: bool = True):
    """(target_id int64 [T], dist float32 [T,k], nbr_id int64 [T,k], knn_hist uint64 [kb_nbins+1] or None)."""
    xyz, lab, d_bnd = _cloud(xyz, lab, d_bnd)
    n = xyz.shape[0]
    T = int((select_targets(lab, d_bnd, A, d_srf)).shape[0])
    tid = np.empty(max(T, 1), dtype=np.int64)
    dist = np.empty((max(T, 1), k), dtype=np.float32)
    nid = np.empty((max(T, 1), k), dtype=np.int64)
    hist = np.zeros(kb_nbins + 1, dtype=np.uint64) if want_hist else None
    f = _load().orc_knn_grid if method == "grid" else _load().orc_knn_brute
    t = f(xyz.ctypes.data, lab.ctypes.data, _ptr(d_bnd), n, A, B, d_srf, k, r_knn_max,
          tid.ctypes.data, dist.ctypes.data, nid.ctypes.data, kb_rmax, kb_nbins, _ptr(hist))
    assert t == T
    return tid[:T], dist[:T], nid[:T], hist


def sdm_faces(R: float, n_vox: int) -> np.ndarray:
    """Voxel faces f_m = ((2m - n) R) / n, m = 0..n (FP64)."""
    F = np.empty(n_vox + 1, dtype=np.float64)
    _load().orc_sdm_faces(R, n_vox, F.ctypes.data)
    return F


def sdm(xyz, lab, d_bnd, A: int, B: int, d_srf: float, R: float, n_vox: int, method: str = "grid") -> np.ndarray:
    """Two-point statistic: counts of pair displacement vectors per cubic voxel,
    uint64 [n_vox, n_vox, n_vox] indexed [mz, my, mx]."""
    xyz, lab, d_bnd = _cloud(xyz, lab, d_bnd)
    hist = np.zeros(n_vox ** 3, dtype=np.uint64)
    f = _load().orc_sdm_grid if method == "grid" else _load().orc_sdm_brute
    f(xyz.ctypes.data, lab.ctypes.data, _ptr(d_bnd), xyz.shape[0], A, B, d_srf, R, n_vox, hist.ctypes.data)
    return hist.reshape(n_vox, n_vox, n_vox)


def cluster_ms(xyz, lab, d_bnd, A: int, d_max: float, n_min: int, d_srf: float = 0.0, n_size_bins: int = 0,
               method: str = "grid"):
    """Maximum-separation clustering of the ions of species A: (label int64
    [n], counts int64 [3] = kept clusters, truncated kept clusters, ions in
    kept clusters, size_hist uint64 [n_size_bins] or None)."""
    xyz, lab, d_bnd = _cloud(xyz, lab, d_bnd)
    n = xyz.shape[0]
    label = np.empty(n, dtype=np.int64)
    counts = np.zeros(3, dtype=np.int64)
    hist = np.zeros(n_size_bins, dtype=np.uint64) if n_size_bins > 0 else None
    f = _load().orc_cluster_ms_grid if method == "grid" else _load().orc_cluster_ms_brute
    f(xyz.ctypes.data, lab.ctypes.data, _ptr(d_bnd), n, A, d_max, n_min, d_srf, label.ctypes.data,
      counts.ctypes.data, _ptr(hist), n_size_bins)
    return label, counts, hist


def edge_distance(xyz, tri, d_prb: float = float("inf"), method: str = "grid") -> np.ndarray:
    """Distance of every ion to the closest point of the triangles (float32
    [n]): +inf at or beyond d_prb, NaN for a non-finite position.  The grid
    form needs a finite d_prb (the brute-force form is taken otherwise)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    tri = np.ascontiguousarray(tri, dtype=np.float32).reshape(-1, 9)
    d = np.empty(xyz.shape[0], dtype=np.float32)
    f = _load().orc_edge_grid if (method == "grid" and np.isfinite(d_prb)) else _load().orc_edge_brute
    f(xyz.ctypes.data, xyz.shape[0], tri.ctypes.data, tri.shape[0], d_prb, d.ctypes.data)
    return d


def splitmix64(seed: int, i: int) -> int:
    return int(_load().orc_splitmix64(seed, i))


def permute_labels(lab, seed: int) -> np.ndarray:
    lab = np.ascontiguousarray(lab, dtype=np.uint8)
    out = np.empty_like(lab)
    _load().orc_permute_labels(lab.ctypes.data, len(lab), seed, out.ctypes.data)
    return out


def smooth_fwd(xyz, lab, d_bnd, A: int, B: int, d_srf: float, r_max: float, n_bins: int,
               sigma: float, s: float = 1.0) -> np.ndarray:
    xyz, lab, d_bnd = _cloud(xyz, lab, d_bnd)
    h = np.zeros(n_bins, dtype=np.float64)
    _load().orc_smooth_fwd(xyz.ctypes.data, lab.ctypes.data, _ptr(d_bnd), xyz.shape[0], A, B, d_srf,
                           r_max, n_bins, sigma, s, h.ctypes.data)
    return h


def smooth_bwd(xyz, lab, d_bnd, A: int, B: int, d_srf: float, r_max: float, n_bins: int,
               sigma: float, s: float, grad_h):
    """(grad_xyz float64 [n,3], grad_s float)."""
    xyz, lab, d_bnd = _cloud(xyz, lab, d_bnd)
    gh = np.ascontiguousarray(grad_h, dtype=np.float64)
    assert gh.shape == (n_bins,)
    g = np.zeros((xyz.shape[0], 3), dtype=np.float64)
    gs = np.zeros(1, dtype=np.float64)
    _load().orc_smooth_bwd(xyz.ctypes.data, lab.ctypes.data, _ptr(d_bnd), xyz.shape[0], A, B, d_srf,
                           r_max, n_bins, sigma, s, gh.ctypes.data, g.ctypes.data, gs.ctypes.data)
    return g, float(gs[0])


def smooth_fd(xyz, lab, d_bnd, A: int, B: int, d_srf: float, r_max: float, n_bins: int, sigma: float,
              s: float, resid, ions, step: float = 1e-4) -> np.ndarray:
    """Central finite differences of sum_b (h_b - t_b)^2 (resid = h - t) with
    respect to the coordinates of `ions`: float64 [len(ions), 3]."""
    xyz, lab, d_bnd = _cloud(xyz, lab, d_bnd)
    r = np.ascontiguousarray(resid, dtype=np.float64)
    assert r.shape == (n_bins,)
    ids = np.ascontiguousarray(ions, dtype=np.int64)
    fd = np.zeros((len(ids), 3), dtype=np.float64)
    _load().orc_smooth_fd(xyz.ctypes.data, lab.ctypes.data, _ptr(d_bnd), xyz.shape[0], A, B, d_srf, r_max, n_bins,
                          sigma, s, r.ctypes.data, ids.ctypes.data, len(ids), step, fd.ctypes.data)
    return fd
