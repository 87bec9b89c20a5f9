"""Parity of the fine Wilson-Dirac stencil (HIP, through the C ABI) with the oracle.

Tolerances, element by element (max |out - ref| / max |ref|): 1e-12 in FP64,
1e-5 in FP32 (the inputs are rounded to FP32 first, so the FP32 bound covers
both input and arithmetic rounding of a 9-term complex sum).
"""
import numpy as np
import pytest

import synth
from oracle import dirac
from gpu_util import dev, host, max_rel_err, rel_err, su3_config, u1_config

pytestmark = pytest.mark.gpu

SHAPES_2D = [(32, 32), (8, 6), (34, 18), (256, 256), (4, 4), (130, 2)]


@pytest.mark.parametrize("L1,L2", SHAPES_2D)
@pytest.mark.parametrize("dagger", [0, 1])
def test_wilson2d_fp64(L1, L2, dagger):
    import paper_0707_4018_amd as amg
    print(f"wilson2d fp64 {L1}x{L2} dagger={dagger}", flush=True)
    U = u1_config(L1, L2)
    m = -0.07
    g = amg.Gauge(dev(U), m)
    nrhs = 3
    psi = synth.gaussian_field((nrhs, L2 * L1, 2, 1), synth.rng_for(1, L1, L2))
    out = host(g.apply(dev(psi), dagger=bool(dagger)))
    for k in range(nrhs):
        ref = dirac.apply_D(U, psi[k].reshape(L2, L1, 2, 1), m, dagger=bool(dagger)).reshape(-1, 2, 1)
        assert max_rel_err(out[k], ref) < 1e-12


@pytest.mark.parametrize("L1,L2", SHAPES_2D)
def test_wilson2d_fp32(L1, L2):
    import paper_0707_4018_amd as amg
    import torch
    print(f"wilson2d fp32 {L1}x{L2}", flush=True)
    U = u1_config(L1, L2, seed=1)
    g = amg.Gauge(dev(U), 0.1)
    psi = synth.gaussian_field((1, L2 * L1, 2, 1), synth.rng_for(2, L1, L2))
    for dagger in (False, True):
        out = host(g.apply(dev(psi, torch.complex64), dagger=dagger, prec=amg.F32))
        ref = dirac.apply_D(U, psi[0].reshape(L2, L1, 2, 1), 0.1, dagger=dagger).reshape(1, -1, 2, 1)
        assert max_rel_err(out, ref) < 1e-5


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (6, 4, 2, 4), (8, 8, 8, 8), (4, 4, 2, 12), (2, 2, 4, 2), (4, 2, 2, 20)])
def test_wilson4d(dims):
    import paper_0707_4018_amd as amg
    import torch
    print(f"wilson4d {dims}", flush=True)
    U = su3_config(dims)
    V = int(np.prod(dims))
    m = 0.05
    g = amg.Gauge(dev(U), m)
    psi = synth.gaussian_field((2, V, 4, 3), synth.rng_for(3, *dims))
    lat = tuple(reversed(dims))
    for dagger in (False, True):
        out = host(g.apply(dev(psi), dagger=dagger))
        out32 = host(g.apply(dev(psi, torch.complex64), dagger=dagger, prec=amg.F32))
        for k in range(2):
            ref = dirac.apply_D(U, psi[k].reshape(lat + (4, 3)), m, dagger=dagger).reshape(V, 4, 3)
            assert max_rel_err(out[k], ref) < 1e-12
            assert max_rel_err(out32[k], ref) < 1e-5


def test_apply_rejects_bad_arguments():
    import paper_0707_4018_amd as amg
    import torch
    from paper_0707_4018_amd import binding as b
    U = u1_config(8, 8)
    g = amg.Gauge(dev(U), 0.0)
    x = torch.zeros((1, 64, 2, 1), dtype=torch.complex128, device="cuda")
    lib = b.load_library()
    # in-place application and a bad precision are rejected before any launch
    assert lib.amg_apply(g.handle, 0, 0, b._ptr(x), b._ptr(x), 1, b._stream()) == 1
    y = torch.empty_like(x)
    assert lib.amg_apply(g.handle, 0, 7, b._ptr(x), b._ptr(y), 1, b._stream()) == 1
    assert lib.amg_apply(g.handle, 0, 0, b._ptr(x), b._ptr(y), 0, b._stream()) == 1
    with pytest.raises(ValueError):
        g.apply(torch.zeros((1, 64, 2, 1), dtype=torch.complex64, device="cuda"))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("L1,L2", [(1024, 1024), (64, 16384), (4096, 256), (262144, 4), (1040, 1024), (1024, 1032)])
def test_wilson2d_streaming_store_size(prec, L1, L2):
    """Lattices from 2^20 sites: streaming stores; with L1 a multiple of 64 and
    L2 of 16 the x_2-marching kernel (a single 64-site tile across x_1 at
    L1 = 64, so the periodic x_1 neighbours of lanes 0 and 63 lie in the same
    wave; at L2 = 4 one strip spans x_2 in FP64, so the rows below and above
    it are its own last and first rows), otherwise the one-site-per-thread
    kernel.  Two right-hand sides."""
    import paper_0707_4018_amd as amg
    import torch
    print(f"wilson2d {prec} {L1}x{L2} (streaming stores)", flush=True)
    b2 = min(8, L2)
    th = synth.u1_heatbath(8, b2, 6.0, 20, synth.rng_for(90, 600, 8, b2, 7))
    U = np.exp(1j * synth.tile_u1(th, L1 // 8, L2 // b2))[..., None, None]
    g = amg.Gauge(dev(U), 0.03)
    psi = synth.gaussian_field((2, L2 * L1, 2, 1), synth.rng_for(4, L1, L2))
    dt = torch.complex128 if prec == "f64" else torch.complex64
    for dagger in (False, True):
        out = host(g.apply(dev(psi, dt), dagger=dagger, prec=amg.F64 if prec == "f64" else amg.F32))
        for k in range(2):
            ref = dirac.apply_D(U, psi[k].reshape(L2, L1, 2, 1), 0.03, dagger=dagger).reshape(-1, 2, 1)
            if prec == "f64":
                assert max_rel_err(out[k], ref) < 1e-12, (dagger, k)
            else:
                assert max_rel_err(out[k], ref) < 1e-5, (dagger, k)


def test_wilson4d_streaming_store_size():
    """A 4d lattice of 2^20 sites takes the kernels' streaming-store path (FP64 and FP32)."""
    import paper_0707_4018_amd as amg
    import torch
    base = (8, 8, 8, 8)
    tile = (2, 2, 2, 32)
    dims = tuple(b * t for b, t in zip(base, tile))
    print(f"wilson4d {dims} (streaming stores)", flush=True)
    U = np.tile(su3_config(base, seed=3), (1,) + tuple(reversed(tile)) + (1, 1))
    V = int(np.prod(dims))
    m = 0.05
    g = amg.Gauge(dev(U), m)
    psi = synth.gaussian_field((1, V, 4, 3), synth.rng_for(5, *dims))
    lat = tuple(reversed(dims))
    ref = dirac.apply_D(U, psi[0].reshape(lat + (4, 3)), m).reshape(1, V, 4, 3)
    assert max_rel_err(host(g.apply(dev(psi))), ref) < 1e-12
    assert max_rel_err(host(g.apply(dev(psi, torch.complex64), prec=amg.F32)), ref) < 1e-5


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (8, 8, 8, 16)])
def test_wilson4d_non_su3_links_use_full_links(dims):
    """Links in U(3) but not SU(3) (a phase on every link): the library keeps
    the full 3 x 3 links (the two-row form needs det U = 1), with the same
    parity; SU(3) links take the two-row form."""
    import paper_0707_4018_amd as amg
    import torch
    print(f"wilson4d non-SU(3) links {dims}", flush=True)
    U = su3_config(dims, seed=7)
    V = int(np.prod(dims))
    assert amg.Gauge(dev(U), 0.05).links_compressed
    phase = np.exp(1j * synth.rng_for(8, *dims).uniform(-np.pi, np.pi, size=U.shape[:-2]))
    Up = U * phase[..., None, None]
    g = amg.Gauge(dev(Up), 0.05)
    assert not g.links_compressed
    psi = synth.gaussian_field((1, V, 4, 3), synth.rng_for(9, *dims))
    ref = dirac.apply_D(Up, psi[0].reshape(tuple(reversed(dims)) + (4, 3)), 0.05).reshape(V, 4, 3)
    assert max_rel_err(host(g.apply(dev(psi)))[0], ref) < 1e-12
    assert max_rel_err(host(g.apply(dev(psi, torch.complex64), prec=amg.F32))[0], ref) < 1e-5
