"""apt_rdf_noalloc (static device scratch, no allocation) against apt_rdf.

Two calls in a row through the C ABI, the second on a smaller cloud and
another query: each histogram must equal apt_rdf's on the same input bit for
bit (the static scratch keeps the previous call's contents, which the call
must not depend on).  A cloud too large for the scratch is rejected before
any GPU work.
"""
import ctypes
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

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    aptstat.lib()
    return aptstat, torch


def _noalloc(aptstat, torch, cloud, A, B, d_srf, r_max, n_bins):
    dev = cloud.device
    h = torch.full((n_bins,), -7, dtype=torch.int64, device=dev)      # poisoned: must be overwritten
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    rc = aptstat.lib().apt_rdf_noalloc(cloud.c(), aptstat._query(A, B, d_srf), aptstat._bins(r_max, n_bins),
                                       ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(st.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    assert rc == 0, aptstat.lib().apt_last_error().decode()
    return h, st


def test_noalloc_equals_rdf_on_two_calls_in_a_row(gpu, synth):
    aptstat, torch = gpu
    dev = torch.device("cuda:0")
    cases = [
        ("box240k Sc->Sc", synth.box240k(), SC, SC, 0.0, False, 2.0, 200),
        ("box 60k clustered Sc->Al, d_bnd", synth.Specimen(shape="box", L=(13.0, 13.0, 13.0), n=60_000, seed=11,
                                                         p_m_sc=0.02, n_clusters=20, r_c=1.2),
         SC, AL, 1.0, True, 1.5, 300),
    ]
    ws = aptstat.Workspace()
    for name, spec, A, B, d_srf, use_d, r_max, n_bins in cases:
        _say(f"[no-alloc] {name}: {spec.n} ions")
        xyz, lab, d = spec.generate()
        cloud = aptstat.Cloud(torch.from_numpy(xyz).to(dev), torch.from_numpy(lab).to(dev),
                              torch.from_numpy(d).to(dev) if use_d else None)
        h, st = _noalloc(aptstat, torch, cloud, A, B, d_srf, r_max, n_bins)
        st_ref = torch.zeros(1, dtype=torch.int32, device=dev)
        ref = aptstat.rdf(cloud, A, B, d_srf, r_max, n_bins, ws=ws, status=st_ref)
        torch.cuda.synchronize()
        assert int(st.item()) == int(st_ref.item()) == 0
        assert int(ref.sum().item()) > 0
        assert torch.equal(h, ref), f"{name}: apt_rdf_noalloc differs from apt_rdf"


def test_noalloc_rejects_clouds_beyond_the_scratch(gpu):
    aptstat, torch = gpu
    L = aptstat.lib()
    # sizes only: the check precedes any GPU work and any pointer use
    c = aptstat._Cloud(0x1000, 0x2000, None, 4_000_000)
    rc = L.apt_rdf_noalloc(ctypes.byref(c), aptstat._query(SC, SC, 0.0), aptstat._bins(2.0, 200),
                           ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000), None)
    assert rc == -3
    assert "scratch" in L.apt_last_error().decode()
