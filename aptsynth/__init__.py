"""Seeded synthetic atom-probe point clouds (input generator).

Serves the oracle, the tests and the benchmark alike; holds none of the
spatial-statistics arithmetic.  The C core (``synth.c``) draws every number
from a counter-based hash of (seed, stream, ion index), so any ion range can
be regenerated on its own, in parallel, with identical results.

Workloads follow the paper's synthetic specimens (Methods, Case studies,
"Benchmarking all functionality with synthetic datasets": a conical frustum
needle, Al matrix, Al3Sc-like spherical precipitates) with the sizes of the
five workloads this library is measured on:

* ``box240k``   240 000 ions in a 20 nm cube, Al 98 % / Sc 2 %, no clusters.
* ``frustum7m`` needle frustum H = 200 nm, R 25 -> 15 nm at 30 ions/nm^3
  (7 696 902 ions), Al 97.5 / Sc 1 / Si 1.5 %, half the Sc in 363 clusters of
  r = 1.5 nm at 25 at.% Sc, 0.2 nm Gaussian noise.
* ``box1m``     1e6 ions in a 32 nm cube, Al 98 / Sc 2 % matrix plus 500
  clusters of r = 1.2 nm at 25 at.% Sc.
* ``frustum2g`` 2e9 ions, the H = 2000 nm, R 60 -> 30 nm needle scaled by
  1.7159 in every length so that it holds 2e9 ions at 30 ions/nm^3; chemistry
  and cluster density as ``frustum7m``; no noise.

``frustum_mesh`` triangulates a frustum specimen's surface: the triangle
hull that the ion-to-edge distancing takes as its input.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libaptsynth.so")

AL, SC, SI = 0, 1, 2
SPECIES = {"Al": AL, "Sc": SC, "Si": SI}


def build(force: bool = True) -> str:
    """Compile the generator with the host C compiler (OpenMP)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "synth.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Params(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("L", ctypes.c_double * 3),
        ("H", ctypes.c_double), ("R0", ctypes.c_double), ("R1", ctypes.c_double),
        ("n", ctypes.c_int64), ("seed", ctypes.c_uint64),
        ("p_m_sc", ctypes.c_double), ("p_m_si", ctypes.c_double), ("p_c_sc", ctypes.c_double),
        ("n_clusters", ctypes.c_int64), ("r_c", ctypes.c_double), ("noise", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER(_Params)
        lib.synth_centres.argtypes = [P, ctypes.c_void_p]
        lib.synth_centres.restype = ctypes.c_int
        lib.synth_generate.argtypes = [P, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_generate.restype = ctypes.c_int
        lib.synth_volume.argtypes = [P]
        lib.synth_volume.restype = ctypes.c_double
        lib.synth_surface_distance.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.synth_surface_distance.restype = ctypes.c_double
        _lib = lib
    return _lib


@dataclass(frozen=True)
class Specimen:
    """Shape, size and chemistry of one synthetic specimen."""
    shape: str = "box"                 # "box" or "frustum"
    L: tuple = (20.0, 20.0, 20.0)      # box sides (nm)
    H: float = 0.0                     # frustum height (nm)
    R0: float = 0.0                    # frustum base radius (nm)
    R1: float = 0.0                    # frustum top radius (nm)
    n: int = 0
    seed: int = 1
    p_m_sc: float = 0.0
    p_m_si: float = 0.0
    p_c_sc: float = 0.25
    n_clusters: int = 0
    r_c: float = 0.0
    noise: float = 0.0
    meta: dict = field(default_factory=dict, compare=False, hash=False)

    def _c(self) -> _Params:
        p = _Params()
        p.shape = 1 if self.shape == "frustum" else 0
        p.L = (ctypes.c_double * 3)(*self.L)
        p.H, p.R0, p.R1 = self.H, self.R0, self.R1
        p.n, p.seed = int(self.n), int(self.seed)
        p.p_m_sc, p.p_m_si, p.p_c_sc = self.p_m_sc, self.p_m_si, self.p_c_sc
        p.n_clusters, p.r_c, p.noise = int(self.n_clusters), self.r_c, self.noise
        return p

    @property
    def volume(self) -> float:
        return _load().synth_volume(ctypes.byref(self._c()))

    def surface_distance(self, x: float, y: float, z: float) -> float:
        return _load().synth_surface_distance(ctypes.byref(self._c()), x, y, z)

    def with_seed(self, seed: int) -> "Specimen":
        return replace(self, seed=seed)

    def centres(self) -> np.ndarray:
        c = np.zeros((max(self.n_clusters, 1), 3), dtype=np.float64)
        if self.n_clusters > 0:
            rc = _load().synth_centres(ctypes.byref(self._c()), c.ctypes.data)
            if rc != 0:
                raise RuntimeError("cluster centre placement failed")
        return c[: self.n_clusters]

    def generate(self, i0: int = 0, i1: int | None = None, xyz=None, lab=None, d_bnd=None,
                 centres: np.ndarray | None = None):
        """Ions [i0, i1) as (xyz float32 [m,3], lab uint8 [m], d_bnd float32 [m]).

        Pre-allocated C-contiguous numpy outputs (e.g. views of pinned host
        tensors) may be passed in; they are filled in place."""
        i1 = self.n if i1 is None else i1
        m = i1 - i0
        if xyz is None:
            xyz = np.empty((m, 3), dtype=np.float32)
        if lab is None:
            lab = np.empty(m, dtype=np.uint8)
        if d_bnd is None:
            d_bnd = np.empty(m, dtype=np.float32)
        assert xyz.dtype == np.float32 and xyz.shape == (m, 3) and xyz.flags.c_contiguous
        assert lab.dtype == np.uint8 and lab.shape == (m,)
        assert d_bnd.dtype == np.float32 and d_bnd.shape == (m,)
        if centres is None:
            centres = self.centres()
        centres = np.ascontiguousarray(centres, dtype=np.float64)
        rc = _load().synth_generate(ctypes.byref(self._c()),
                                    centres.ctypes.data if len(centres) else None,
                                    i0, i1, xyz.ctypes.data, lab.ctypes.data, d_bnd.ctypes.data)
        if rc != 0:
            raise RuntimeError("generation failed")
        return xyz, lab, d_bnd


def _frustum_volume(H, R0, R1):
    return math.pi * H * (R0 * R0 + R0 * R1 + R1 * R1) / 3.0


def clustered_needle(H, R0, R1, density=30.0, f_sc=0.01, f_si=0.015, r_c=1.5, c_sc=0.25,
                     noise=0.0, seed=1, n=None, **meta) -> Specimen:
    """Needle frustum with half the Sc in Al3Sc-like clusters.

    The number of clusters puts half the Sc inside them at c_sc; the matrix
    probabilities then keep the global fractions f_sc and f_si (Si is matrix
    only).  Cluster overlap is ignored in this bookkeeping."""
    V = _frustum_volume(H, R0, R1)
    if n is None:
        n = int(round(density * V))
    v1 = 4.0 / 3.0 * math.pi * r_c ** 3
    n_cl = int(round(f_sc * 0.5 / c_sc * V / v1))
    phi = n_cl * v1 / V
    p_m_sc = (f_sc - phi * c_sc) / (1.0 - phi)
    p_m_si = f_si / (1.0 - phi)
    return Specimen(shape="frustum", H=H, R0=R0, R1=R1, n=n, seed=seed, p_m_sc=p_m_sc,
                    p_m_si=p_m_si, p_c_sc=c_sc, n_clusters=n_cl, r_c=r_c, noise=noise,
                    meta=dict(meta))


def scaled_needle(n, H, R0, R1, density=30.0, **kw) -> Specimen:
    """The needle (H, R0, R1) scaled uniformly so that it holds n ions at density."""
    s = (n / (density * _frustum_volume(H, R0, R1))) ** (1.0 / 3.0)
    return clustered_needle(H * s, R0 * s, R1 * s, density=density, n=n, scale=s, **kw)


def box240k(seed: int = 1) -> Specimen:
    return Specimen(shape="box", L=(20.0, 20.0, 20.0), n=240_000, seed=seed, p_m_sc=0.02)


def frustum7m(seed: int = 1) -> Specimen:
    return clustered_needle(200.0, 25.0, 15.0, noise=0.2, seed=seed)


def box1m(seed: int = 1) -> Specimen:
    return Specimen(shape="box", L=(32.0, 32.0, 32.0), n=1_000_000, seed=seed, p_m_sc=0.02,
                    p_c_sc=0.25, n_clusters=500, r_c=1.2)


def frustum2g(seed: int = 1, n: int = 2_000_000_000) -> Specimen:
    return scaled_needle(n, 2000.0, 60.0, 30.0, seed=seed)


def frustum200m(seed: int = 1) -> Specimen:
    """The full-scale needle's shape and chemistry at a tenth of its ions (same
    density: the same per-target work, for profiling runs)."""
    return frustum2g(seed=seed, n=200_000_000)


def frustum_mesh(spec: Specimen, n_phi: int, n_z: int) -> np.ndarray:
    """A closed triangle hull of a frustum specimen (side, bottom and top
    caps), float32 [n_tri, 3, 3]: the given edge of the ion-to-edge
    distancing.  The side is n_z rings of n_phi quads, each split into two
    triangles; each cap is a fan of n_phi triangles around the axis.  The
    vertices lie on the analytic surface, so the hull is inscribed in it
    (the side's chords sit at most R (1 - cos(pi / n_phi)) inside)."""
    H, R0, R1 = float(spec.H), float(spec.R0), float(spec.R1)
    phi = 2.0 * np.pi * np.arange(n_phi + 1) / n_phi
    phi[-1] = 0.0                                     # the seam closes exactly
    z = H * np.arange(n_z + 1) / n_z
    R = R0 + (R1 - R0) * z / H
    X = R[:, None] * np.cos(phi)[None, :]
    Y = R[:, None] * np.sin(phi)[None, :]
    Z = np.broadcast_to(z[:, None], X.shape)
    V = np.stack([X, Y, Z], -1)                       # [n_z + 1, n_phi + 1, 3]
    a, b = V[:-1, :-1], V[:-1, 1:]
    c, d = V[1:, :-1], V[1:, 1:]
    side = np.concatenate([np.stack([a, b, d], 2).reshape(-1, 3, 3), np.stack([a, d, c], 2).reshape(-1, 3, 3)])
    ctr0 = np.zeros((n_phi, 3))
    ctr1 = np.zeros((n_phi, 3))
    ctr1[:, 2] = H
    cap0 = np.stack([ctr0, V[0, 1:], V[0, :-1]], 1)
    cap1 = np.stack([ctr1, V[-1, :-1], V[-1, 1:]], 1)
    return np.ascontiguousarray(np.concatenate([side, cap0, cap1]).astype(np.float32))


WORKLOADS = {"box240k": box240k, "frustum7m": frustum7m, "box1m": box1m, "frustum2g": frustum2g,
             "frustum200m": frustum200m}


def to_device(spec: Specimen, torch, device, with_d_bnd: bool = True, chunk: int = 1 << 25, on_chunk=None,
              log=None):
    """Generate the specimen chunk by chunk straight into device tensors.

    Each chunk is generated into pinned host buffers and copied to the GPU
    (two buffers, so generation overlaps the copy).  on_chunk(i0, xyz, lab,
    d_bnd) may inspect each host chunk before it is reused.  Returns
    (xyz float32 [n,3], lab uint8 [n], d_bnd float32 [n] or None) on device."""
    n = spec.n
    xyz_d = torch.empty((n, 3), dtype=torch.float32, device=device)
    lab_d = torch.empty(n, dtype=torch.uint8, device=device)
    d_d = torch.empty(n, dtype=torch.float32, device=device) if with_d_bnd else None
    m = min(chunk, max(n, 1))
    bufs = [(torch.empty((m, 3), dtype=torch.float32, pin_memory=True),
             torch.empty(m, dtype=torch.uint8, pin_memory=True),
             torch.empty(m, dtype=torch.float32, pin_memory=True)) for _ in range(2)]
    events = [None, None]
    stream = torch.cuda.Stream(device=device)
    centres = spec.centres()
    for q, i0 in enumerate(range(0, n, m)):
        i1 = min(n, i0 + m)
        b = q & 1
        if events[b] is not None:
            events[b].synchronize()          # the copy out of this buffer is done
        hx, hl, hd = (t[: i1 - i0] for t in bufs[b])
        spec.generate(i0, i1, hx.numpy(), hl.numpy(), hd.numpy(), centres=centres)
        if on_chunk is not None:
            on_chunk(i0, hx.numpy(), hl.numpy(), hd.numpy())
        with torch.cuda.stream(stream):
            xyz_d[i0:i1].copy_(hx, non_blocking=True)
            lab_d[i0:i1].copy_(hl, non_blocking=True)
            if d_d is not None:
                d_d[i0:i1].copy_(hd, non_blocking=True)
            events[b] = torch.cuda.Event()
            events[b].record(stream)
        if log is not None and (q % 8 == 7 or i1 == n):
            log(f"generated {i1} of {n} ions")
    stream.synchronize()
    return xyz_d, lab_d, d_d
