"""The allocation-free entry point (lofp_amplitudes_device_noalloc) against
the ordinary device entry point and the oracle, on two calls in a row on one
circuit, the second smaller (the scratch array keeps the first call's
contents)."""
import numpy as np
import pytest

import oracle
from paper_2510_26408_amd import lofp, workloads

pytestmark = pytest.mark.gpu
ATOL = 1e-12


@pytest.fixture(autouse=True)
def gpu_only():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _flat(layers):
    return [bs for l in layers for bs in l]


@pytest.mark.parametrize("name,sizes", [("c2", (48, 20)), ("c5", (40, 9)), ("c3", (60, 33))])
def test_noalloc_matches_device_entry_point(name, sizes):
    import torch
    wl = workloads.make(name, seed=17, batch=max(sizes))
    c = lofp.Circuit(wl.m, wl.layers)
    T = torch.from_numpy(np.ascontiguousarray(wl.Ts)).cuda()
    opts = lofp.make_opts(method=lofp.METHOD_CONTRACT)
    # the ordinary call with one contraction per pattern, the form the
    # allocation-free call runs
    ref_opts = lofp.make_opts(method=lofp.METHOD_CONTRACT, split=lofp.SPLIT_NEVER)
    want = oracle.amplitudes(wl.m, wl.S, wl.Ts, _flat(wl.layers), nthreads=8)[0]
    # the ordinary call sets the circuit up on the device (it may allocate)
    ref = torch.zeros(wl.batch, dtype=torch.complex128, device="cuda")
    c.amplitudes_device(wl.S, T, ref, ref_opts)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    for b in sizes:
        out = torch.full((b,), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
        c.amplitudes_device_noalloc(wl.S, T[:b], out, opts)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # the same per-pattern kernel (the ordinary call's state size may
        # come from the device instead of the S-side bound, which can change
        # the block size and so the order of the final sum)
        assert np.abs(got - ref[:b]).max() <= 1e-14, name
        assert np.abs(got - want[:b]).max() <= ATOL


def test_noalloc_rejects_unprepared_circuit_and_oversized_batch():
    import torch
    wl = workloads.make("c2", seed=18, batch=8)
    c = lofp.Circuit(wl.m, wl.layers)
    T = torch.from_numpy(np.ascontiguousarray(wl.Ts)).cuda()
    out = torch.zeros(wl.batch, dtype=torch.complex128, device="cuda")
    with pytest.raises(lofp.LofpError) as e:
        c.amplitudes_device_noalloc(wl.S, T, out)
    assert e.value.status == lofp.EINVAL
    c.amplitudes_device(wl.S, T, out, lofp.make_opts(method=lofp.METHOD_CONTRACT))
    big = torch.zeros((200000, wl.m), dtype=torch.int32, device="cuda")
    big_out = torch.zeros(200000, dtype=torch.complex128, device="cuda")
    with pytest.raises(lofp.LofpError) as e:
        c.amplitudes_device_noalloc(wl.S, big, big_out)
    assert e.value.status == lofp.EINVAL and "scratch" in str(e.value)
