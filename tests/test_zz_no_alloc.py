"""GPU check of pdlp_unroll_forward_noalloc, the unrolled forward pass whose buffers live in the
library's per-GPU scratch array instead of device memory it allocates.

It runs the same kernels as pdlp_unroll_forward on the same data, so its outputs, and the
gradients of pdlp_unroll_backward after it, must equal the allocating entry point's bit for
bit.  Two calls in a row, the second on a smaller LP, cover the array keeping the last call's
contents; the size limit, the ownership check of the backward pass and a return to the
allocating entry point are covered too."""
import sys

import numpy as np
import pytest

import paper_2106_04756_amd as P
from workloads import lpgen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def _inputs(lp, seed):
    rng = np.random.default_rng(seed)
    c = lp.c * rng.uniform(0.9, 1.1, lp.n)
    q = lp.q * rng.uniform(0.9, 1.1, lp.m)
    gx = rng.standard_normal(lp.n)
    gy = rng.standard_normal(lp.m)
    return c, q, gx, gy


def _allocating(lp, c, q, gx, gy, T, segment):
    with P.Solver.from_lp(lp) as s:
        x, y = s.unroll_forward(c, q, T, segment)
        gc, gq = s.unroll_backward(gx, gy)
    return x, y, gc, gq


def _same(a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else a
    assert a.shape == b.shape and np.array_equal(a, b), float(np.abs(a - b).max())


def test_noalloc_matches_allocating_entry_point_twice():
    import torch
    big, _ = lpgen.unroll_lp()
    tiny = lpgen.tiny_lp()
    # first call: the unroll LP (2e4 x 5e4), device tensors in and out
    c, q, gx, gy = _inputs(big, 1)
    T, seg = 100, 25
    say("no-alloc call 1", big.name, "T", T, "segment", seg)
    ref = _allocating(big, c, q, gx, gy, T, seg)
    dev = lambda a: torch.from_numpy(a).cuda()
    with P.Solver.from_lp(big) as s:
        xo = torch.empty(big.n, dtype=torch.float64, device="cuda")
        yo = torch.empty(big.m, dtype=torch.float64, device="cuda")
        s.unroll_forward_noalloc(dev(c), dev(q), T, seg, 0.0, 0.0, xo, yo)
        torch.cuda.synchronize()
        info = s.unroll_info()
        assert info["device_bytes"] == 0 and info["checkpoints"] == 4 and info["ready"] == 1
        gc = torch.empty(big.n, dtype=torch.float64, device="cuda")
        gq = torch.empty(big.m, dtype=torch.float64, device="cuda")
        s.unroll_backward(dev(gx), dev(gy), gc, gq)
        torch.cuda.synchronize()
        assert s.unroll_info()["device_bytes"] == 0
        for a, b in zip((xo, yo, gc, gq), ref):
            _same(a, b)
    # second call, smaller input: the tiny LP (200 x 500), host arrays, on the array the first
    # call left behind
    c, q, gx, gy = _inputs(tiny, 2)
    T, seg = 33, 7
    say("no-alloc call 2", tiny.name, "T", T, "segment", seg)
    ref = _allocating(tiny, c, q, gx, gy, T, seg)
    with P.Solver.from_lp(tiny) as s:
        x, y = s.unroll_forward_noalloc(c, q, T, seg)
        gc, gq = s.unroll_backward(gx, gy)
        for a, b in zip((x, y, gc, gq), ref):
            _same(a, b)
        # back to the allocating entry point on the same solver
        x2, y2 = s.unroll_forward(c, q, T, seg)
        gc2, gq2 = s.unroll_backward(gx, gy)
        for a, b in zip((x2, y2, gc2, gq2), ref):
            _same(a, b)
        assert s.unroll_info()["device_bytes"] > 0


def test_noalloc_limits_and_ownership():
    tiny = lpgen.tiny_lp()
    big, _ = lpgen.unroll_lp()
    c, q, gx, gy = _inputs(tiny, 3)
    say("no-alloc limits and ownership")
    with P.Solver.from_lp(big) as sb:
        # every step's masks of a 1000-step unroll: 7e4 * 1000 bytes > 64 MiB
        with pytest.raises(P.PdlpError, match="scratch") as ei:
            sb.unroll_forward_noalloc(None, None, 1000, 0)
        assert ei.value.code == P.ERR_INVALID_ARGUMENT
        with P.Solver.from_lp(tiny) as sa:
            x, y = sa.unroll_forward_noalloc(c, q, 20, 5)
            sb.unroll_forward_noalloc(None, None, 10, 5)        # claims the array
            with pytest.raises(P.PdlpError) as ei:
                sa.unroll_backward(gx, gy)
            assert ei.value.code == P.ERR_INVALID_STATE
            # the claimer's own backward still works, and a new forward restores sa
            sb.unroll_backward(np.ones(big.n), None)
            x2, y2 = sa.unroll_forward_noalloc(c, q, 20, 5)
            gc, gq = sa.unroll_backward(gx, gy)
            _same(x2, x)
            _same(y2, y)
    ref = _allocating(tiny, c, q, gx, gy, 20, 5)
    _same(gc, ref[2])
    _same(gq, ref[3])
