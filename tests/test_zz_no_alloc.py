"""corutv_decompose_noalloc (scratch in the library's fixed per-device array)
against corutv_decompose (scratch from the context workspace) through the C
ABI: the same kernels, so U, T, V, the pivots and the residual are compared
bit for bit, on two calls in a row, the second with a smaller input (the
array keeps the first call's contents).  The F64 case is also checked against
the float64 oracle at the 1e-10 bar.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle.corutv import corutv, rel_err
from workloads import decaying, noisy_low_rank

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _both(ctx, A, k, p, q, seed, prec, tri):
    ref = ctx.decompose(A, k, p, q, seed, prec=prec, tri=tri, want_err=True)
    got = ctx.decompose_noalloc(A, k, p, q, seed, prec=prec, tri=tri, want_err=True)
    torch.cuda.synchronize()
    for a, b in zip(ref[:4], got[:4]):
        assert torch.equal(a, b)
    assert got[4]["rel_err"] == ref[4]["rel_err"]
    assert got[4]["passes"] == ref[4]["passes"] and got[4]["tri"] == ref[4]["tri"]
    return got


def test_noalloc_matches_decompose_two_calls():
    import paper_1906_04572_amd as cu

    ctx = cu.Context(workspace_bytes=cu.workspace_bytes(2000, 1500, 20, 10, 1, "f64"))
    _say("noalloc 1: 2000x1500 rank 20 + 1e-6 noise, l=30, q=1, lower, f64")
    A1 = noisy_low_rank(2000, 1500, 20, 1e-6, seed=1)
    U, T, V, piv, info = _both(ctx, torch.from_numpy(A1).cuda(), 20, 10, 1, 2024, "f64", "lower")
    ref = corutv(A1, 20, 10, 1, seed=2024, tri="lower")
    e_ref = rel_err(A1, ref["U"], ref["T"], ref["V"])
    assert abs(info["rel_err"] - e_ref) <= 1e-10
    Ah = U.cpu().numpy() @ T.cpu().numpy() @ V.cpu().numpy().T
    assert np.linalg.norm(Ah - ref["U"] @ ref["T"] @ ref["V"].T) / np.linalg.norm(A1) <= 1e-10

    _say("noalloc 2 (smaller): 700x450 exp decay, l=18, q=2, f32, column-major")
    A2 = decaying(700, 450, 60, 1e-4, seed=5, dtype=np.float32)
    A2d = torch.from_numpy(np.ascontiguousarray(A2.T)).cuda().t()
    _both(ctx, A2d, 12, 6, 2, 77, "f32", "auto")

    _say("noalloc 3 (wide, smaller still): 300x520, l=20, q=1, bf16x3")
    A3 = decaying(300, 520, 40, 1e-4, seed=6, dtype=np.float32)
    _both(ctx, torch.from_numpy(A3).cuda(), 15, 5, 1, 5, "bf16x3", "auto")
    ctx.close()


def test_noalloc_without_workspace_and_limits():
    import paper_1906_04572_amd as cu

    _say("noalloc: context without a workspace; over-limit shape")
    ctx = cu.Context(workspace_bytes=0)
    A = torch.from_numpy(decaying(900, 640, 50, 1e-4, seed=8)).cuda()
    U, T, V, piv, info = ctx.decompose_noalloc(A, 20, 10, 1, 9, prec="f64")
    # every workspace user reports that the (empty) workspace is too small
    assert ctx.decompose_rc(A, 20, 10, 1, 9, prec="f64") == cu.E_NOMEM
    ref = cu.Context(workspace_bytes=cu.workspace_bytes(900, 640, 20, 10, 1, "f64"))
    R = ref.decompose(A, 20, 10, 1, 9, prec="f64")
    for a, b in zip(R[:4], (U, T, V, piv)):
        assert torch.equal(a, b)
    ref.close()
    # more than the 64 MiB array holds
    big = torch.zeros((20000, 1500), dtype=torch.float64, device="cuda")
    assert cu.workspace_bytes(20000, 1500, 100, 10, 1, "f64") > 64 << 20
    out = ctx.alloc_outputs(big, 100, 10)
    info = cu.Info()
    opts = cu.Opts(cu.PREC["f64"], 0, 0, 0, 0)
    mu, mv = cu.mat(out[0]), cu.mat(out[2])
    rc = cu.lib.corutv_decompose_noalloc(ctx.h, ctypes.byref(cu.mat(big)), 100, 10, 1, 1, ctypes.byref(opts),
                                         ctypes.byref(mu), out[1].data_ptr(), 110, ctypes.byref(mv),
                                         out[3].data_ptr(), ctypes.byref(info))
    assert rc == cu.E_NOMEM
    # host-resident A is not accepted here
    opts_h = cu.Opts(cu.PREC["f64"], 0, 0, cu.FLAG_A_HOST, 0)
    Ah = torch.zeros((900, 640), dtype=torch.float64)
    o2 = ctx.alloc_outputs(A, 20, 10)
    mu2, mv2 = cu.mat(o2[0]), cu.mat(o2[2])
    rc = cu.lib.corutv_decompose_noalloc(ctx.h, ctypes.byref(cu.mat(Ah, host=True)), 20, 10, 1, 1,
                                         ctypes.byref(opts_h), ctypes.byref(mu2), o2[1].data_ptr(), 30,
                                         ctypes.byref(mv2), o2[3].data_ptr(), ctypes.byref(info))
    assert rc == cu.E_INVAL
    ctx.close()
