"""Internal device buffers from torch's caching allocator (amg_set_allocator).

The same two-level mixed-precision solve is run with the library's own
hipMalloc buffers and with buffers taken from torch: the solutions agree, torch
accounts for the library's memory while the handles live and gets it back when
they are destroyed, and the default allocator is restored at the end.
"""
import gc

import numpy as np
import pytest

import synth
from gpu_util import dev, host, max_rel_err, u1_config, vectors

pytestmark = pytest.mark.gpu


def test_torch_allocator_matches_hipmalloc():
    import torch
    import paper_0707_4018_amd as amg
    print("torch caching allocator for the library's buffers", flush=True)
    L = 64
    U = u1_config(L, L, seed=3)
    m = 0.05
    vecs = [dev(vectors(8, L * L, 2, 31))]
    b = dev(synth.gaussian_field((2, L * L, 2, 1), synth.rng_for(17)))
    p = amg.MGParams(blocks=[(4, 4)], nvec=[8], inner_prec=amg.F32, p_bf16=True)
    g0 = amg.Gauge(dev(U), m)
    S0 = amg.Solver(g0, p, nullvecs=vecs)
    x0, info0 = S0.solve(b, tol=1e-10)
    del S0, g0
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    amg.use_torch_allocator(True)
    try:
        g1 = amg.Gauge(dev(U), m)
        S1 = amg.Solver(g1, p, nullvecs=vecs)
        x1, info1 = S1.solve(b, tol=1e-10)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - base
        # at least the fine FP64 links, the 8 near-null vectors and the outer work vectors
        assert held > 8 * L * L * 2 * 16, held
        assert all(i.converged for i in info0) and all(i.converged for i in info1)
        assert [i.iters for i in info0] == [i.iters for i in info1]
        assert max_rel_err(host(x1), host(x0)) < 1e-12
        del S1, g1
        gc.collect()
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated() - base
        assert after <= x1.numel() * 16 + (1 << 20), (held, after)
    finally:
        amg.use_torch_allocator(False)
    # hipMalloc again
    g2 = amg.Gauge(dev(U), m)
    x2, _ = amg.Solver(g2, p, nullvecs=vecs).solve(b, tol=1e-10)
    assert max_rel_err(host(x2), host(x0)) < 1e-12
