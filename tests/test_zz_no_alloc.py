"""amg_apply_noalloc (the application of D that allocates no device memory,
staging in the library's fixed scratch array) against amg_apply, through the
C ABI: two calls in a row, the second with a smaller input, FP64 and FP32,
2d and 4d; identical kernels, so the outputs must be bit-identical; both are
also checked against the oracle's D.  Sizes beyond the scratch array are
rejected before any launch."""
import numpy as np
import pytest

import synth
from oracle import dirac
from gpu_util import dev, host, max_rel_err, su3_config, u1_config

pytestmark = pytest.mark.gpu


def _noalloc(g, psi, prec, dagger=False):
    import torch
    import paper_0707_4018_amd as amg
    dt = torch.complex128 if prec == amg.F64 else torch.complex64
    x = dev(psi, dt)
    out = torch.empty_like(x)
    g.apply_noalloc(x, out, dagger=dagger, prec=prec)
    return host(out), host(g.apply(x, dagger=dagger, prec=prec))


@pytest.mark.parametrize("prec_name", ["f64", "f32"])
def test_noalloc_apply_2d_matches_apply(prec_name):
    import paper_0707_4018_amd as amg
    prec = amg.F64 if prec_name == "f64" else amg.F32
    print(f"noalloc apply 2d {prec_name}", flush=True)
    L1, L2 = 64, 48
    U = u1_config(L1, L2, seed=21)
    m = -0.04
    g = amg.Gauge(dev(U), m)
    tol = 1e-12 if prec == amg.F64 else 1e-5
    for nrhs, dagger in ((5, False), (2, True)):        # second call smaller
        psi = synth.gaussian_field((nrhs, L1 * L2, 2, 1), synth.rng_for(22, nrhs))
        out, ref = _noalloc(g, psi, prec, dagger)
        assert np.array_equal(out, ref), nrhs
        for k in range(nrhs):
            o = dirac.apply_D(U, psi[k].reshape(L2, L1, 2, 1), m, dagger=dagger).reshape(-1, 2, 1)
            assert max_rel_err(out[k], o) < tol, (nrhs, k)


def test_noalloc_apply_4d_then_smaller_lattice():
    import paper_0707_4018_amd as amg
    print("noalloc apply 4d, then a smaller 2d lattice", flush=True)
    dims = (8, 8, 4, 8)
    U = su3_config(dims, seed=23)
    V = int(np.prod(dims))
    g = amg.Gauge(dev(U), 0.07)
    psi = synth.gaussian_field((3, V, 4, 3), synth.rng_for(24))
    for prec in (amg.F64, amg.F32):
        out, ref = _noalloc(g, psi, prec)
        assert np.array_equal(out, ref)
    o = dirac.apply_D(U, psi[0].reshape(tuple(reversed(dims)) + (4, 3)), 0.07).reshape(V, 4, 3)
    assert max_rel_err(out[0], o) < 1e-5
    # a smaller input on another handle reuses the same array
    U2 = u1_config(8, 6, seed=25)
    g2 = amg.Gauge(dev(U2), 0.2)
    psi2 = synth.gaussian_field((1, 48, 2, 1), synth.rng_for(26))
    out2, ref2 = _noalloc(g2, psi2, amg.F64)
    assert np.array_equal(out2, ref2)
    assert max_rel_err(out2[0], dirac.apply_D(U2, psi2[0].reshape(6, 8, 2, 1), 0.2).reshape(-1, 2, 1)) < 1e-12


def test_noalloc_apply_rejects_oversize():
    """16^4 x 12 dof x 3 rhs in FP64 needs 2 x 37.7 MB of staging: AMG_ERR_ARG."""
    import torch
    import paper_0707_4018_amd as amg
    from paper_0707_4018_amd import binding as b
    print("noalloc apply oversize", flush=True)
    dims = (16, 16, 16, 16)
    U = np.zeros((4,) + dims + (3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    g = amg.Gauge(dev(U), 0.1)
    V = 16 ** 4
    x = torch.zeros((3, V, 4, 3), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    lib = b.load_library()
    assert lib.amg_apply_noalloc(g.handle, 0, amg.F64, b._ptr(x), b._ptr(y), 3, b._stream()) == 1
    assert b"scratch" in lib.amg_last_error()
    # one rhs fits (2 x 12.6 MB)
    g.apply_noalloc(x[:1].contiguous(), y[:1].contiguous())
