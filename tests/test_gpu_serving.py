"""GPU serving path (corutv_submit / corutv_poll / corutv_wait / corutv_cancel).

* A mixed stream of requests (shapes, precisions, q, orientations) runs with
  several requests in flight on different streams; every result is
  bit-identical to the same request run alone through corutv_decompose
  (kernel configurations depend only on the request shape).
* Admission by workspace: with room for one request at a time the others
  queue and still complete; a request larger than the whole workspace is
  rejected with E_NOMEM; a queued request can be cancelled; unknown tickets
  give E_NOTFOUND.
"""
import numpy as np
import pytest
import torch

from workloads import decaying

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


REQS = [  # m, n, k, p, q, prec
    (3000, 2000, 40, 10, 1, "f64"), (2500, 4000, 20, 10, 2, "f32"), (5000, 1200, 100, 10, 1, "f32"),
    (1800, 1800, 60, 5, 0, "f64"), (4000, 3000, 30, 10, 1, "f32"), (1000, 6000, 10, 10, 1, "f64"),
]


def _inputs():
    out = []
    for i, (m, n, k, p, q, prec) in enumerate(REQS):
        A = decaying(m, n, min(m, n) // 3, 1e-4, seed=100 + i, tau=max(k / 2, 3))
        dt = torch.float64 if prec == "f64" else torch.float32
        out.append(torch.from_numpy(A).to("cuda", dt))
    return out


def test_mix_is_bitwise_equal_to_alone():
    import paper_1906_04572_amd as cu

    _say("serving mix vs alone")
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(3)]
    ws = 3 * max(cu.workspace_bytes(m, n, k, p, q, pr) for m, n, k, p, q, pr in REQS)
    ctx = cu.Context(workspace_bytes=ws, streams=streams)
    As = _inputs()
    alone = []
    for (m, n, k, p, q, prec), A in zip(REQS, As):
        alone.append(ctx.decompose(A, k, p, q, seed=31, prec=prec))
    tickets = []
    for rep in range(2):
        for (m, n, k, p, q, prec), A in zip(REQS, As):
            tickets.append(ctx.submit(A, k, p, q, seed=31, prec=prec))
    results = [ctx.wait(t) for t in tickets]
    for i, res in enumerate(results):
        ref = alone[i % len(REQS)]
        for a, b in zip(res[:4], ref[:4]):
            assert torch.equal(a, b), (i, REQS[i % len(REQS)])
        assert res[4]["passes"] == ref[4]["passes"]
    ctx.close()


def test_admission_queueing_nomem_cancel():
    import paper_1906_04572_amd as cu

    _say("serving admission")
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(2)]
    m, n, k, p, q = 2000, 1500, 20, 10, 1
    need = cu.workspace_bytes(m, n, k, p, q, "f64")
    ctx = cu.Context(workspace_bytes=need + need // 2, streams=streams)  # room for one
    A = torch.from_numpy(decaying(m, n, 200, 1e-4, seed=5)).cuda()
    ref = ctx.decompose(A, k, p, q, seed=3)
    ts = [ctx.submit(A, k, p, q, seed=3) for _ in range(5)]
    # the last one is still queued behind the others: it can be cancelled
    assert cu.lib.corutv_cancel(ctx.h, ts[-1]) in (cu.OK, cu.E_BUSY)
    done = 0
    for t in ts[:-1]:
        U, T, V, piv, info = ctx.wait(t)
        assert torch.equal(U, ref[0]) and torch.equal(T, ref[1]) and torch.equal(V, ref[2])
        done += 1
    assert done == 4
    big = torch.zeros((20000, 15000), dtype=torch.float32, device="cuda")
    with pytest.raises(cu.CorutvError) as e:
        ctx.submit(big, 100, 10, 1, seed=1, prec="f32")
    assert e.value.code == cu.E_NOMEM
    assert cu.lib.corutv_poll(ctx.h, 987654321, None) == cu.E_NOTFOUND
    ctx.close()
