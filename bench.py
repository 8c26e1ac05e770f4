"""Benchmark: target ions/s of kNN (k = 10) + RDF (r < 2 nm) on one MI355X.

A step is one pass of the whole plain path over the workload: for each
query of the workload, one apt_knn_rdf call (bounding box, target and
neighbour selection, cell binning, pair enumeration with RDF histogram and
exact kNN rows plus the k-th distance histogram).  Inputs are generated on
the host (seeded, synthetic), copied to HBM once, and are resident when the
timed region starts.

The headline workload is the full-scale needle: 2e9 ions, Sc -> any
species, d_srf = 2 nm.  Beside it the line carries the 7.7e6-ion needle's
three queries, the batched null-model replicates against looped plain calls
on that needle, and the smoothed RDF on the 1e6-ion box.

Prints one JSON line (rank 0).  --gpus above 1 is refused: the benchmark
measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target ions/s for kNN(k=10)+RDF(r≤2nm); batched vs looped replicates/s"
AL, SC, SI, ANY = 0, 1, 2, 255
NAMES = {AL: "Al", SC: "Sc", SI: "Si", ANY: "any"}

# workload -> (generator, queries (A, B), d_srf, use the surface filter)
WORKLOADS = {
    "frustum7m": ("frustum7m", [(SC, SC), (SC, AL), (SI, SC)], 1.0, True),
    "box240k": ("box240k", [(SC, SC)], 0.0, False),
    "frustum2g": ("frustum2g", [(SC, ANY)], 2.0, True),
    "frustum200m": ("frustum200m", [(SC, ANY)], 2.0, True),
}
K, R_MAX, N_BINS, KB_RMAX, KB_NBINS = 10, 2.0, 200, 5.0, 5000
# HBM bytes per launch of the roofline kernel, (workload, kernel) -> (bytes,
# source hash), from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a
# plain-copy calibration; valid only for the kernel sources they were taken
# on (the summaries under profiles/)
PAIR_TRAFFIC = {
    # profiles/counters_frustum2g.md: FETCH_SIZE 16 314 537.1 KiB x 2.0 +
    # WRITE_SIZE 74 091.3 KiB per k_rdf_nbr<1> launch
    ("frustum2g", "k_rdf_nbr"): (33_487_197_757, "3dec29db6eee67cd"),
}
PAIR_SOURCES = ("apt_pair.hip", "apt_pair.hpp", "apt_pairdev.hpp", "apt_internal.hpp", "apt_bin.hpp")
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X: 256 CU x 2.4 GHz x 256 FLOP/clk (packed FMA)
HBM_PEAK_GBPS = 8000.0            # MI355X HBM3E
FLOP_PER_PAIR = 8                 # 3 sub, 3 mul, 2 add per pair distance (no contraction)
# candidate pair-evaluations per second the FP32 vector units allow: 256 CU x
# 64 lanes x 2 (packed) x 2.4 GHz over 6 instructions per candidate
R_PAIR = 256 * 64 * 2 * 2.4e9 / 6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(spec_name, queries, d_srf, use_d, repeats=3):
    """The oracle (grid kNN + grid RDF, OpenMP) on a bounded sample of the
    workload: median of `repeats` runs on all host threads and on one."""
    import numpy as np

    import aptsynth
    import oracle

    spec = aptsynth.WORKLOADS[spec_name]()
    n = spec.n
    if n <= 8_000_000:
        xyz, lab, d = spec.generate()
        what = f"the whole {n}-ion cloud"
    else:
        # the 2e9-ion needle's ions are i.i.d. in the whole shape, so a prefix
        # would be 250x too thin; the same needle scaled to 8e6 ions has the
        # same density, composition and cluster density, hence the same
        # per-target work
        sub = aptsynth.WORKLOADS[spec_name](n=8_000_000)
        xyz, lab, d = sub.generate()
        what = (f"the same needle scaled to {sub.n} ions (same density, composition and clusters; "
                f"the full cloud has {n})")
    d = d if use_d else None

    def run(dd):
        targets = 0
        t0 = time.perf_counter()
        for A, B in queries:
            oracle.rdf(xyz, lab, dd, A, B, d_srf, R_MAX, N_BINS)
            tid, _, _, _ = oracle.knn(xyz, lab, dd, A, B, d_srf, K, kb_rmax=KB_RMAX, kb_nbins=KB_NBINS)
            targets += len(tid)
        return targets, time.perf_counter() - t0

    all_threads = oracle.threads()
    rates, secs = [], []
    for _ in range(repeats):
        t, dt = run(d)
        rates.append(t / dt)
        secs.append(dt)
    # one core: the whole of a smaller cloud of the same kind (the same
    # needle scaled to 2e6 ions: same density and chemistry, a quarter of
    # the targets), so that three runs stay within ~15 s
    if n > 2_000_000:
        sub1 = aptsynth.WORKLOADS[spec_name](n=2_000_000) if n > 8_000_000 else None
        if sub1 is not None:
            xyz, lab, d1 = sub1.generate()
            d1 = d1 if use_d else None
            what1 = f"the same needle scaled to {sub1.n} ions, the whole cloud"
        else:
            d1, what1 = d, what
    else:
        d1, what1 = d, what
    # (a whole cloud of more than 2e6 ions is timed once on one core)
    reps1 = 1 if (d1 is d and n > 2_000_000) else repeats
    oracle.set_threads(1)
    rates1, secs1 = [], []
    try:
        for _ in range(reps1):
            t, dt = run(d1)
            rates1.append(t / dt)
            secs1.append(dt)
    finally:
        oracle.set_threads(all_threads)
    qs = ", ".join(NAMES[a] + "->" + NAMES[b] for a, b in queries)
    return {"value": float(np.median(rates)), "unit": "target ions/s", "cores": all_threads, "kind": "oracle",
            "sample": f"{what}, queries {qs}, grid oracle (RDF + kNN k={K} + k-th histogram), median of "
                      f"{repeats} runs of {np.median(secs):.1f} s on {all_threads} threads",
            "one_core": {"value": float(np.median(rates1)), "unit": "target ions/s", "cores": 1,
                         "sample": f"{what1}, median of {reps1} runs of {np.median(secs1):.1f} s on 1 thread"}}


def smooth_timing(aptstat, torch, reps=10):
    """Gaussian-smoothed RDF (forward and adjoint) on the differentiable
    workload: 1e6 ions in a 32 nm cube with 500 Sc clusters, Sc -> Sc,
    sigma 0.02 nm, 200 bins to 2 nm, z scale 1.05; loss sum (h - t)^2 with
    the target curve of the next seed."""
    import aptsynth

    dev = torch.device("cuda:0")
    ws = aptstat.Workspace()
    curves = []
    for seed in (1, 2):
        xyz, lab, d = aptsynth.to_device(aptsynth.box1m(seed), torch, dev, with_d_bnd=False)
        curves.append((xyz, lab))
    zs = torch.tensor([1.05], dtype=torch.float64, device=dev)
    args = (SC, SC, 0.0, R_MAX, N_BINS, 0.02)
    t = aptstat.rdf_smooth(aptstat.Cloud(*curves[1]), *args, z_scale=zs, ws=ws)
    cloud = aptstat.Cloud(*curves[0])
    h = aptstat.rdf_smooth(cloud, *args, z_scale=zs, ws=ws)
    gh = (2.0 * (h - t)).contiguous()
    aptstat.rdf_smooth_grad(cloud, *args, gh, z_scale=zs, ws=ws)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        aptstat.rdf_smooth(cloud, *args, z_scale=zs, ws=ws, out=h)
    ev[1].record()
    for _ in range(reps):
        aptstat.rdf_smooth_grad(cloud, *args, gh, z_scale=zs, ws=ws)
    ev[2].record()
    torch.cuda.synchronize()
    return {"workload": "box1m", "query": "Sc->Sc", "sigma_nm": 0.02, "z_scale": 1.05,
            "forward_ms": ev[0].elapsed_time(ev[1]) / reps, "adjoint_ms": ev[1].elapsed_time(ev[2]) / reps,
            "smoothed_mass": float(h.sum().item())}


def sdm_timing(aptstat, torch, cloud, ws, reps=5):
    """Two-point statistic (3-D displacement histogram, R = 2 nm, 0.025 nm
    voxels: 160^3) of Sc -> Al on the 7.7e6-ion needle: ms per call and
    in-range pairs per second of its kernel."""
    R, n_vox = 2.0, 160
    h = aptstat.sdm(cloud, SC, AL, 1.0, R, n_vox, ws=ws)
    torch.cuda.synchronize()
    pairs = int(h.sum().item())
    for stage in ("sdm", "binning"):
        aptstat.trace_read(stage)
    aptstat.trace_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        aptstat.sdm(cloud, SC, AL, 1.0, R, n_vox, ws=ws, out=h)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    aptstat.trace_enable(False)
    k_ms = aptstat.trace_read("sdm")[0] / reps
    b_ms = aptstat.trace_read("binning")[0] / reps
    return {"workload": "frustum7m", "query": "Sc->Al", "d_srf_nm": 1.0, "R_nm": R, "n_vox": n_vox,
            "ms_per_call": 1e3 * dt, "kernel_ms": k_ms, "binning_ms": b_ms, "pairs": pairs,
            "pairs_per_s_kernel": pairs / (k_ms / 1e3) if k_ms > 0 else None}


def knn100_timing(aptstat, torch, cloud, ws, reps=5):
    """kNN with k = 100 (and the RDF to 2 nm, the k-th distance histogram at
    0.001 nm) of the 7.7e6-ion needle's queries Sc -> Sc and Sc -> Al
    (d_srf = 1 nm): ms per call and target ions per second."""
    out = {"workload": "frustum7m", "k": 100, "d_srf_nm": 1.0, "r_max_nm": R_MAX, "queries": {}}
    for name, (A, B) in (("Sc->Sc", (SC, SC)), ("Sc->Al", (SC, AL))):
        r = aptstat.knn_rdf(cloud, A, B, 1.0, 100, r_max=R_MAX, n_bins=N_BINS, kb_rmax=KB_RMAX,
                            kb_nbins=KB_NBINS, ws=ws)
        torch.cuda.synchronize()
        assert int(r.status.item()) == 0
        nt = int(r.n_targets.item())
        outs = (r.target_id, r.dist, r.nbr_id, r.knn_hist, r.n_targets, r.status, r.rdf_hist)
        t0 = time.perf_counter()
        for _ in range(reps):
            aptstat.knn_rdf(cloud, A, B, 1.0, 100, r_max=R_MAX, n_bins=N_BINS, capacity=r.target_id.shape[0],
                            kb_rmax=KB_RMAX, kb_nbins=KB_NBINS, ws=ws, outputs=outs)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out["queries"][name] = {"targets": nt, "ms_per_call": 1e3 * dt, "target_ions_per_s": nt / dt}
    return out


def cluster_timing(aptstat, torch, cloud, ws, reps=3):
    """Maximum-separation clustering of the Sc ions of the 7.7e6-ion needle
    over the d_max sweep of the paper's benchmark task (0.10 to 0.70 nm in
    steps of 0.05 nm, N_min = 5; clusters with an ion within 1 nm of the
    surface count as truncated): ms per run, and the kept clusters per d_max."""
    d_maxes = [round(0.10 + 0.05 * i, 2) for i in range(13)]
    kept, trunc = [], []
    for dm in d_maxes:
        _, c, _, st = aptstat.cluster_ms(cloud, SC, dm, 5, 1.0, ws=ws)
        c = c.cpu()
        kept.append(int(c[0]))
        trunc.append(int(c[1]))
    for stage in ("cluster", "binning"):
        aptstat.trace_read(stage)
    aptstat.trace_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for dm in d_maxes:
            aptstat.cluster_ms(cloud, SC, dm, 5, 1.0, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / (reps * len(d_maxes))
    aptstat.trace_enable(False)
    k_ms = aptstat.trace_read("cluster")[0] / (reps * len(d_maxes))
    b_ms = aptstat.trace_read("binning")[0] / (reps * len(d_maxes))
    return {"workload": "frustum7m", "species": "Sc", "d_max_nm": [0.10, 0.05, 0.70], "n_min": 5,
            "runs": len(d_maxes), "ms_per_run": 1e3 * dt, "cluster_kernels_ms": k_ms, "binning_ms": b_ms,
            "sweep_ms": 1e3 * dt * len(d_maxes), "kept_clusters": kept, "truncated_clusters": trunc}


def edge_timing(aptstat, torch, cloud, ws, reps=5):
    """Ion-to-edge distancing of the 7.7e6-ion needle against its inscribed
    hull (256 x 200 side quads and two caps: 102 912 triangles, about the
    paper's triangle density per surface area at 2e9 ions) at the benchmark's
    probe distance d_prb = 2.5 nm: ms per call and the ions within d_prb."""
    import aptsynth

    mesh = aptsynth.frustum_mesh(aptsynth.frustum7m(), 256, 200)
    tri = torch.from_numpy(mesh).to(cloud.device)
    d, st = aptstat.edge_distance(cloud, tri, 2.5, ws=ws)
    torch.cuda.synchronize()
    within = int(torch.isfinite(d).sum().item())
    for stage in ("edge", "binning"):
        aptstat.trace_read(stage)
    aptstat.trace_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        aptstat.edge_distance(cloud, tri, 2.5, ws=ws, out=d)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    aptstat.trace_enable(False)
    k_ms = aptstat.trace_read("edge")[0] / reps
    b_ms = aptstat.trace_read("binning")[0] / reps
    return {"workload": "frustum7m", "triangles": int(mesh.shape[0]), "d_prb_nm": 2.5, "ms_per_call": 1e3 * dt,
            "edge_kernels_ms": k_ms, "binning_ms": b_ms, "ions_within_d_prb": within,
            "ions_per_s": cloud.n / dt, "status": int(st.item())}


PAIRS6 = [(AL, SC), (AL, SI), (SC, AL), (SC, SI), (SI, AL), (SI, SC)]


def batched_vs_looped(aptstat, torch, cloud, ws, n_rep, n_loop):
    """Replicates/s of 6 ordered species pairs x n_rep label-randomised
    replicates in one batched call, against looped plain calls (one label
    permutation + one kNN+RDF call per pair and replicate) on the same GPU."""
    pairs = [(a, b, 1.0) for a, b in PAIRS6]
    base = 1000
    dev = cloud.device
    seeds = [base + r + 1 for r in range(n_rep)]
    rh = torch.empty((n_rep, len(pairs), N_BINS), dtype=torch.int64, device=dev)
    kh = torch.empty((n_rep, len(pairs), KB_NBINS + 1), dtype=torch.int64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    # warm-up: with tuning NULL the library tunes the plan for this call
    # (trial launches), caches it, captures the launch sequence in a graph
    # and launches it
    log(f"[bench] batched: warm-up ({n_rep} replicates; plan tuned and cached)")
    aptstat.batched_plan_clear()
    t0 = time.perf_counter()
    aptstat.rdf_batched(cloud, pairs, seeds, r_max=R_MAX, n_bins=N_BINS, k=K, kb_rmax=KB_RMAX,
                        kb_nbins=KB_NBINS, ws=ws, out=(rh, kh, st))
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    plan = aptstat.batched_plan(cloud, pairs, r_max=R_MAX, n_bins=N_BINS, k=K, kb_rmax=KB_RMAX, kb_nbins=KB_NBINS)
    log(f"[bench] batched: {n_rep} replicates x {len(pairs)} pairs")
    for stage in ("pair", "tile", "binning", "permute", "partition"):
        aptstat.trace_read(stage)
    aptstat.trace_enable(True)
    t0 = time.perf_counter()
    aptstat.rdf_batched(cloud, pairs, seeds, r_max=R_MAX, n_bins=N_BINS, k=K, kb_rmax=KB_RMAX,
                        kb_nbins=KB_NBINS, ws=ws, out=(rh, kh, st))
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    aptstat.trace_enable(False)
    stages = {s_: aptstat.trace_read(s_)[0] for s_ in ("pair", "tile", "binning", "permute", "partition")}
    # the library's own graph of the call (tracing off: replayed)
    log(f"[bench] batched: library graph replay")
    t0 = time.perf_counter()
    aptstat.rdf_batched(cloud, pairs, seeds, r_max=R_MAX, n_bins=N_BINS, k=K, kb_rmax=KB_RMAX,
                        kb_nbins=KB_NBINS, ws=ws, out=(rh, kh, st))
    torch.cuda.synchronize()
    t_lib = time.perf_counter() - t0
    # the same call captured once in a HIP graph and replayed (its outputs
    # must equal the eager call's)
    want = (rh.clone(), kh.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            aptstat.rdf_batched(cloud, pairs, seeds, r_max=R_MAX, n_bins=N_BINS, k=K, kb_rmax=KB_RMAX,
                                kb_nbins=KB_NBINS, ws=ws, out=(rh, kh, st))
    torch.cuda.synchronize()
    log(f"[bench] batched: graph replay")
    t0 = time.perf_counter()
    graph.replay()
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    graph_equal = bool(torch.equal(want[0], rh) and torch.equal(want[1], kh))
    del graph
    # looped: the definition of the batched result, call by call
    lab_r = torch.empty_like(cloud.lab)
    outs = (torch.empty(1, dtype=torch.int64, device=dev), torch.empty((1, K), dtype=torch.float32, device=dev),
            torch.empty((1, K), dtype=torch.int64, device=dev),
            torch.empty(KB_NBINS + 1, dtype=torch.int64, device=dev), torch.empty(1, dtype=torch.int64, device=dev),
            torch.empty(1, dtype=torch.int32, device=dev), torch.empty(N_BINS, dtype=torch.int64, device=dev))

    def loop(reps):
        for sd in reps:
            aptstat.permute_labels(cloud.lab, sd, out=lab_r, ws=ws)
            c = aptstat.Cloud(cloud.xyz, lab_r, cloud.d_bnd)
            for a, b, d in pairs:
                aptstat.knn_rdf(c, a, b, d, K, r_max=R_MAX, n_bins=N_BINS, capacity=0, kb_rmax=KB_RMAX,
                                kb_nbins=KB_NBINS, ws=ws, outputs=outs)

    log(f"[bench] looped: {n_loop} replicates x {len(pairs)} pairs")
    loop(seeds[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop(seeds[:n_loop])
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    return {"replicates": n_rep, "pairs": [f"{NAMES[a]}->{NAMES[b]}" for a, b, _ in pairs],
            "batched_replicates_per_s": n_rep / t_lib, "batched_s": t_lib, "traced_eager_s": tb,
            "batched_stage_ms": stages, "plan": plan, "first_call_s": t_first,
            "library_graph_replicates_per_s": n_rep / t_lib,
            "graph_replicates_per_s": n_rep / tg, "graph_equals_eager": graph_equal,
            "looped_replicates_per_s": n_loop / tl, "looped_replicates_timed": n_loop,
            "looped_calls_timed": n_loop * (1 + len(pairs)),
            "speedup": (n_rep / t_lib) / (n_loop / tl), "status": int(st.item())}


def traffic_for(workload, kernel):
    """HBM bytes per launch of the roofline kernel from committed counter
    runs, if the kernel sources still hash to the ones measured (else None)."""
    if (workload, kernel) not in PAIR_TRAFFIC:
        return None
    import hashlib

    csrc = os.path.join(ROOT, "paper_2004_05188_amd", "csrc")
    blob = b"".join(open(os.path.join(csrc, f), "rb").read() for f in PAIR_SOURCES)
    sha = hashlib.sha256(blob).hexdigest()[:16]
    return PAIR_TRAFFIC[(workload, kernel)][0] if sha == PAIR_TRAFFIC[(workload, kernel)][1] else None


def binning_bytes(n_ions, n_target_species, n_targets, n_neighbours):
    """Algorithmic HBM bytes of one call's binning: labels read (1 B/ion),
    d_bnd of the target species (4 B), positions of targets and neighbours
    (12 B), the neighbour records written (16 B) and the target order
    written (rank, index, position: 20 B).  The cell offsets, whose size is
    a choice of the index, are not counted."""
    return n_ions + 4 * n_target_species + 12 * (n_targets + n_neighbours) + 16 * n_neighbours + 20 * n_targets


def measure_plain(aptstat, torch, workload, steps, warmup, ws, with_candidates=True):
    """Target ions/s of the plain path on one workload, stage times, the pair
    kernel's roofline figures and the culling ratio."""
    import aptsynth

    gen_name, queries, d_srf, use_d = WORKLOADS[workload]
    spec = aptsynth.WORKLOADS[gen_name]()
    dev = torch.device("cuda:0")
    log(f"[bench] generating {workload}: {spec.n} ions into HBM")
    t = time.perf_counter()
    xyz_d, lab_d, d_d = aptsynth.to_device(spec, torch, dev, with_d_bnd=use_d, log=lambda m: log(f"[bench] {m}"))
    log(f"[bench] generated in {time.perf_counter() - t:.1f} s")
    cloud = aptstat.Cloud(xyz_d, lab_d, d_d)
    # outputs sized once from the exact target counts (outside the timed region)
    outs = []
    total_targets = 0
    for A, B in queries:
        cap = int(aptstat.count_targets(cloud, A, d_srf, ws=ws).item())
        total_targets += cap
        outs.append((torch.empty(max(cap, 1), dtype=torch.int64, device=dev),
                     torch.empty((max(cap, 1), K), dtype=torch.float32, device=dev),
                     torch.empty((max(cap, 1), K), dtype=torch.int64, device=dev),
                     torch.empty(KB_NBINS + 1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int64, device=dev),
                     torch.empty(1, dtype=torch.int32, device=dev),
                     torch.empty(N_BINS, dtype=torch.int64, device=dev), cap))

    def step():
        for (A, B), o in zip(queries, outs):
            aptstat.knn_rdf(cloud, A, B, d_srf, K, r_max=R_MAX, n_bins=N_BINS, capacity=o[7],
                            kb_rmax=KB_RMAX, kb_nbins=KB_NBINS, ws=ws, outputs=o[:7])

    log(f"[bench] {workload}: warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # in-range pairs per step (the algorithmic unit of the pair kernel)
    pairs = sum(int(o[6].sum().item()) for o in outs)
    status = [int(o[5].item()) for o in outs]
    for stage in ("pair", "tile", "nbr", "binning"):
        aptstat.trace_read(stage)
    # the timed steps record events around the pair kernel only (each event
    # is a GPU command of its own); the stage breakdown comes from a second,
    # separately traced run of the same steps
    aptstat.trace_enable(True, pair_only=True)
    log(f"[bench] {workload}: timing {steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    aptstat.trace_enable(False)
    pair_ms, pair_n = aptstat.trace_read("pair")
    nbr_ms, nbr_n = aptstat.trace_read("nbr")
    stage_steps = min(steps, 10)
    aptstat.trace_enable(True)
    for _ in range(stage_steps):
        step()
    torch.cuda.synchronize()
    aptstat.trace_enable(False)
    pair2_ms, _ = aptstat.trace_read("pair")
    tile_ms, _ = aptstat.trace_read("tile")
    nbr2_ms, _ = aptstat.trace_read("nbr")
    bin_ms, bin_n = aptstat.trace_read("binning")

    # binning's algorithmic bytes: species counts and cells from the inputs
    # (host reductions outside the timed region)
    n_ions = spec.n
    bbytes = 0
    for (A, B), o in zip(queries, outs):
        n_a = n_ions if A == ANY else int((lab_d == A).sum().item())
        n_b = n_ions if B == ANY else int((lab_d == B).sum().item())
        bbytes += binning_bytes(n_ions, n_a, o[7], n_b)

    cand = None
    if with_candidates:
        # culling: the neighbour records the pair kernel's first enumeration
        # visits (outside the timed region), against the in-range pairs
        cand = sum(int(aptstat.count_candidates(cloud, A, B, d_srf, R_MAX, N_BINS, k=K, ws=ws).item())
                   for A, B in queries)
    del cloud, xyz_d, lab_d, d_d, outs
    torch.cuda.empty_cache()

    # the RDF's pairs are counted by the neighbour-major kernel (dense
    # neighbours) or by the one-target-per-wavefront pair kernel: the
    # dominant of the two is the roofline kernel (on a mix of queries the
    # per-launch pair count is the mean over all queries)
    if nbr_ms > pair_ms:
        kname, k_ms, k_n = "k_rdf_nbr", nbr_ms, nbr_n
    else:
        kname, k_ms, k_n = "k_pair", pair_ms, pair_n
    flop_per_launch = FLOP_PER_PAIR * pairs / len(queries)
    k_avg_s = (k_ms / max(k_n, 1)) / 1e3
    achieved = flop_per_launch / k_avg_s / 1e12
    bin_s = bin_ms / stage_steps / 1e3
    res = {
        "workload": workload, "ions": spec.n, "queries": [f"{NAMES[a]}->{NAMES[b]}" for a, b in queries],
        "d_srf_nm": d_srf if use_d else None, "targets_per_step": total_targets,
        "ms_per_step": 1e3 * dt / steps, "target_ions_per_s": total_targets * steps / dt,
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic_for(workload, kname), "pairs_per_launch": pairs / len(queries),
                     "avg_launch_ms": k_ms / max(k_n, 1)},
        "stages_ms_per_step": {"binning": bin_ms / stage_steps, "pair": pair2_ms / stage_steps,
                               "tile": tile_ms / stage_steps, "nbr": nbr2_ms / stage_steps},
        "binning_hbm": {"algorithmic_bytes_per_step": bbytes, "achieved_GBps": bbytes / bin_s / 1e9 if bin_s else None,
                        "peak_GBps": HBM_PEAK_GBPS,
                        "frac": (bbytes / bin_s / 1e9) / HBM_PEAK_GBPS if bin_s else None},
        "in_range_pairs_per_step": pairs,
        "in_range_pairs_per_s": pairs * stage_steps / ((pair2_ms + tile_ms + nbr2_ms) / 1e3),
        "status": status,
    }
    if cand is not None:
        eval_ms = pair2_ms + nbr2_ms
        res["culling"] = {"candidates_per_step": cand, "ratio": cand / max(pairs, 1),
                          "candidate_evals_per_s": cand * stage_steps / (eval_ms / 1e3) if eval_ms > 0 else None,
                          "frac_of_r_pair": (cand * stage_steps / (eval_ms / 1e3)) / R_PAIR if eval_ms > 0 else None}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="frustum2g", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 7.7e6-ion needle, batched and smoothed-RDF measurements")
    ap.add_argument("--no-smooth", action="store_true", help="skip the smoothed-RDF timing")
    ap.add_argument("--batched-reps", type=int, default=256,
                    help="replicates of the batched null-model measurement (0 = skip)")
    ap.add_argument("--looped-reps", type=int, default=256,
                    help="replicates timed for the looped baseline (its rate is replicates/s)")
    ap.add_argument("--tile-policy", type=int, default=0,
                    help="pair mode (apt_set_tuning tile_policy; 0 = automatic) for profiling runs")
    ap.add_argument("--rdf-kernel", type=int, default=0,
                    help="RDF kernel of the dense-neighbour mode (apt_set_tuning rdf_kernel) for profiling runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (scale of the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs on "
              f"one GPU; how the path would shard over several is a design note, not code)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2004_05188_amd as aptstat

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "copy_calibration_bytes_written":
                          b.numel() * 4, "launches": 5}), flush=True)
        return

    if args.tile_policy or args.rdf_kernel:
        aptstat.set_tuning(tile_policy=args.tile_policy, rdf_kernel=args.rdf_kernel)
    ws = aptstat.Workspace()
    head = measure_plain(aptstat, torch, args.workload, args.steps, args.warmup, ws)
    gen_name, queries, d_srf, use_d = WORKLOADS[args.workload]
    line = {
        "metric": METRIC, "value": head["target_ions_per_s"], "unit": "target ions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "ions": head["ions"], "queries": head["queries"], "k": K,
                   "r_max_nm": R_MAX, "n_bins": N_BINS, "d_srf_nm": head["d_srf_nm"],
                   "knn_hist": [0.0, KB_RMAX / KB_NBINS, KB_RMAX], "targets_per_step": head["targets_per_step"]},
        "roofline": head["roofline"],
        "stages_ms_per_step": head["stages_ms_per_step"], "binning_hbm": head["binning_hbm"],
        "in_range_pairs_per_step": head["in_range_pairs_per_step"],
        "in_range_pairs_per_s": head["in_range_pairs_per_s"], "culling": head.get("culling"),
        "status": head["status"],
    }
    if not args.no_extra:
        if args.workload != "frustum7m":
            line["needle7m"] = measure_plain(aptstat, torch, "frustum7m", args.steps, args.warmup, ws)
        if args.batched_reps > 0:
            import aptsynth

            spec = aptsynth.frustum7m()
            xyz_d, lab_d, d_d = aptsynth.to_device(spec, torch, torch.device("cuda:0"), with_d_bnd=True)
            cloud = aptstat.Cloud(xyz_d, lab_d, d_d)
            line["batched"] = batched_vs_looped(aptstat, torch, cloud, ws, args.batched_reps,
                                                min(args.looped_reps, args.batched_reps))
            log("[bench] two-point statistic on frustum7m")
            line["sdm"] = sdm_timing(aptstat, torch, cloud, ws)
            log("[bench] kNN k = 100 on frustum7m")
            line["knn100"] = knn100_timing(aptstat, torch, cloud, ws)
            log("[bench] maximum-separation clustering sweep on frustum7m")
            line["cluster"] = cluster_timing(aptstat, torch, cloud, ws)
            log("[bench] ion-to-edge distancing on frustum7m")
            line["edge"] = edge_timing(aptstat, torch, cloud, ws)
            del cloud, xyz_d, lab_d, d_d
        if not args.no_smooth:
            log("[bench] smoothed RDF on box1m")
            line["smooth"] = smooth_timing(aptstat, torch)
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        line["cpu_baseline"] = cpu_baseline(gen_name, queries, d_srf, use_d)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
