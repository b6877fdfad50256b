"""The allocation-free gradient entry point (skr_pairing_grads_noalloc) against the
allocating one (skr_pairing_grads), both called through the C ABI on the same device data.

Both evaluate the same products in the same order (the allocation-free one takes its
temporaries from a fixed device workspace and works through dsig in row chunks), so they
must agree to rounding; the bar is the FP64 parity bar, 1e-6 relative, and the observed
agreement is far tighter.  Two calls in a row, the second smaller, check that the shared
workspace's leftover contents do not leak into a later result.
"""
import ctypes

import numpy as np
import pytest

from paper_2311_16019_amd import _lib

OUTS = ("dC1", "dC2", "dsig", "dP1", "dP2")


def _inputs(seed, n1, n2, r, q, lx, ll):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = dict(X1=(n1, lx), X2=(n2, lx), L1=(n1, ll), L2=(n2, ll), C1=(n1, r), C2=(n2, r), P1=(n1, q),
                  P2=(n2, q))
    return {k: torch.from_numpy(rng.standard_normal(s)).cuda() for k, s in shapes.items()}


def _call(fn_name, t, n1, n2, r, q, lx, ll):
    import torch
    lib = _lib.load()
    outs = dict(dC1=torch.full((n1, r), np.nan, dtype=torch.float64, device="cuda"),
                dC2=torch.full((n2, r), np.nan, dtype=torch.float64, device="cuda"),
                dsig=torch.full((n1,), np.nan, dtype=torch.float64, device="cuda"),
                dP1=torch.full((n1, q), np.nan, dtype=torch.float64, device="cuda"),
                dP2=torch.full((n2, q), np.nan, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    loss = ctypes.c_double(np.nan)
    vp = lambda x: ctypes.c_void_p(x.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = getattr(lib, fn_name)(n1, n2, r, q, vp(t["X1"]), vp(t["X2"]), lx, vp(t["L1"]), vp(t["L2"]), ll,
                                 vp(t["C1"]), vp(t["C2"]), vp(t["P1"]), vp(t["P2"]), ctypes.byref(loss),
                                 *(vp(outs[k]) for k in OUTS), stream)
    _lib.check(code)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in outs.items()}
    res["loss"] = loss.value
    return res


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# (n1, n2, r, q, ellx, elll): first a large call (split reductions, dsig in several row
# chunks of the workspace), then a smaller one on the same workspace
SIZES = [(400_000, 300_000, 4, 4, 70, 60), (5_000, 7_000, 2, 3, 9, 11)]


@pytest.mark.gpu
def test_noalloc_matches_allocating_entry_point_twice():
    for seed, (n1, n2, r, q, lx, ll) in enumerate(SIZES):
        print(f"no-alloc pairing grads: seed {seed}, n1={n1} n2={n2} r={r} q={q} ellx={lx} elll={ll}", flush=True)
        t = _inputs(100 + seed, n1, n2, r, q, lx, ll)
        ref = _call("skr_pairing_grads", t, n1, n2, r, q, lx, ll)
        got = _call("skr_pairing_grads_noalloc", t, n1, n2, r, q, lx, ll)
        for k in OUTS:
            assert np.all(np.isfinite(got[k])), k
            assert _rel(got[k], ref[k]) <= 1e-6, (k, _rel(got[k], ref[k]))
        assert abs(got["loss"] - ref["loss"]) <= 1e-6 * abs(ref["loss"])
        # the dsig row chunks must reproduce the one-piece product
        assert _rel(got["dsig"], ref["dsig"]) <= 1e-12


@pytest.mark.gpu
def test_noalloc_rejects_sizes_beyond_the_workspace():
    import torch
    lib = _lib.load()
    t = _inputs(7, 64, 64, 2, 2, 4, 4)
    vp = lambda x: ctypes.c_void_p(x.data_ptr())
    out = torch.empty(64, dtype=torch.float64, device="cuda")
    loss = ctypes.c_double()
    # elll x ellx = 3000 x 2000 doubles (48 MB) is more than the 32 MiB workspace; the size
    # check runs on the host before any device work (the pointers are never read)
    code = lib.skr_pairing_grads_noalloc(64, 64, 2, 2, vp(t["X1"]), vp(t["X2"]), 2000, vp(t["L1"]), vp(t["L2"]),
                                         3000, vp(t["C1"]), vp(t["C2"]), vp(t["P1"]), vp(t["P2"]),
                                         ctypes.byref(loss), None, None, vp(out), None, None, None)
    assert code == _lib.SKR_EINVAL
    assert b"workspace" in lib.skr_last_error()
