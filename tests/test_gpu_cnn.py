"""Parity of the proposal network's HIP kernels (forward, loss, backward,
proposals) with the FP64 oracle, and the learned setup's behaviour.

Same seeded configurations, parameters and targets on both sides.  FP32 mode
checks the kernels' arithmetic (FP32 rounding only); bf16 mode stores
activations and the compute weights in bfloat16 (8 mantissa bits), so its
bounds are those of a few bf16 roundings per layer.
"""
import numpy as np
import pytest

import synth
from oracle import cnn, mg
from gpu_util import dev, host, rel_err, u1_config, vectors

pytestmark = pytest.mark.gpu


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def _params(seed):
    rng = np.random.default_rng([77, seed])
    ps = cnn.init_params(rng)
    ps = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in ps]
    # the GPU holds FP32 parameters: give the oracle the same rounded values
    return [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in ps]


def _configs(B, L1, L2, seed=0):
    Us = [u1_config(L1, L2, beta=3.0 + 3 * i, sweeps=20, seed=seed + i).reshape(2, L1 * L2) for i in range(B)]
    return np.stack(Us)


def _oracle_fixed(U, L1, L2):
    theta = np.angle(U).reshape(2, L2, L1)
    phi = cnn.tree_gauge_phase(theta)
    return cnn.gauge_transform_u1(theta, phi), phi


def _oracle_forward(params, U, L1, L2):
    tf, _ = _oracle_fixed(U, L1, L2)
    out, _ = cnn.forward(params, cnn.network_input(tf)[None])
    return out[0]


@pytest.mark.parametrize("bf16,tol", [(False, 2e-6), (True, 3e-2)])
def test_forward_matches_oracle(bf16, tol):
    import paper_0707_4018_amd as amg
    print(f"cnn forward bf16={bf16}", flush=True)
    L1, L2, B = 32, 48, 2
    params = _params(1)
    U = _configs(B, L1, L2)
    net = amg.Cnn(_flat(params), bf16=bf16)
    out = host(net.forward(dev(U), L1, L2))
    for b in range(B):
        ref = _oracle_forward(params, U[b], L1, L2)
        assert rel_err(out[b], ref) < tol


@pytest.mark.parametrize("bf16,tol_l,tol_g", [(False, 1e-6, 1e-4), (True, 2e-2, 6e-2)])
def test_loss_and_gradients_match_oracle(bf16, tol_l, tol_g):
    import paper_0707_4018_amd as amg
    print(f"cnn loss/grad bf16={bf16}", flush=True)
    L1, L2, B = 32, 32, 2
    params = _params(2)
    U = _configs(B, L1, L2, seed=5)
    T = np.stack([vectors(8, L1 * L2, 2, 300 + b) for b in range(B)])
    net = amg.Cnn(_flat(params), bf16=bf16)
    loss, g = net.loss_grad(dev(U), dev(T), L1, L2)
    ref_loss = 0.0
    ref_g = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    for b in range(B):
        tf, phi = _oracle_fixed(U[b], L1, L2)
        tgt = T[b] * np.exp(1j * phi.ravel())[None, :, None]
        l, gr = cnn.loss_and_param_grads(params, tf, tgt)
        ref_loss += l / B
        ref_g = [(a[0] + c[0] / B, a[1] + c[1] / B) for a, c in zip(ref_g, gr)]
    assert abs(loss - ref_loss) <= tol_l * abs(ref_loss)
    gref = _flat(ref_g).astype(np.float64)
    assert rel_err(g, gref) < tol_g
    # layer by layer, so that a wrong layer cannot hide behind a large one
    off = 0
    for W, bb in ref_g:
        for part in (W, bb):
            n = part.size
            assert rel_err(g[off:off + n], part.ravel()) < 3 * tol_g
            off += n
    # parameters are unchanged by loss_grad
    np.testing.assert_array_equal(net.params(), _flat(params))


def test_proposals_match_oracle():
    import paper_0707_4018_amd as amg
    print("cnn proposals", flush=True)
    L1, L2 = 48, 32
    params = _params(3)
    U = _configs(1, L1, L2, seed=9)[0]
    net = amg.Cnn(_flat(params), bf16=False)
    v = host(net.propose(dev(U), L1, L2))
    _, phi = _oracle_fixed(U, L1, L2)
    ref = cnn.output_to_vectors(_oracle_forward(params, U, L1, L2)) * np.exp(-1j * phi.ravel())[None, :, None]
    assert rel_err(v, ref) < 2e-6


def test_training_reduces_loss():
    import paper_0707_4018_amd as amg
    print("cnn training", flush=True)
    L1 = L2 = 32
    B = 4
    U = _configs(B, L1, L2, seed=11)
    # targets with structure the network can learn: smooth fields in the tree gauge
    T = np.stack([vectors(8, L1 * L2, 2, 400 + b) for b in range(B)])
    net = amg.Cnn(_flat(_params(4)), bf16=True)
    dU, dT = dev(U), dev(T)
    l0 = net.loss_grad(dU, dT, L1, L2, grads=False)[0]
    for _ in range(40):
        net.train_step(dU, dT, L1, L2, lr=2e-3)
    l1 = net.loss_grad(dU, dT, L1, L2, grads=False)[0]
    assert np.isfinite(l1) and l1 < l0 - 0.02, (l0, l1)


def test_rejects_bad_shapes_and_values():
    import paper_0707_4018_amd as amg
    print("cnn argument checks", flush=True)
    p = _flat(_params(5))
    net = amg.Cnn(p, bf16=True)
    U = _configs(1, 32, 32)
    with pytest.raises(amg.AMGError):          # extents must be multiples of 16
        net.forward(dev(U), 8, 128)
    bad = p.copy()
    bad[3] = np.nan
    with pytest.raises(amg.AMGError):
        amg.Cnn(bad)
    with pytest.raises(amg.AMGError):
        net.set_params(bad)


def test_learned_setup_falls_back_on_useless_proposals():
    import paper_0707_4018_amd as amg
    print("learned setup fallback", flush=True)
    L1 = L2 = 32
    U = u1_config(L1, L2, beta=6.0, seed=3)
    m = 0.1
    g = amg.Gauge(dev(U), m)
    params = amg.MGParams(blocks=[(4, 4)], nvec=[8], coarse_tol=0.05, coarse_maxiter=200)
    init = [dev(vectors(8, L1 * L2, 2, 700))]
    chi = dev(synth.gaussian_field((1, L1 * L2, 2, 1), synth.rng_for(0)))
    plain = amg.Solver(g, params, init=init)
    rho_plain = plain.convergence(init[0][0], 8)
    # zero proposals: dependent vectors, the fallback is the plain adaptive setup
    zero = amg.Cnn(np.zeros(amg.Cnn.num_params(), np.float32))
    S, fell_back, rho = amg.Solver.learned(g, params, zero, init, rho_iters=8, rho_max=0.99)
    assert fell_back
    assert abs(rho - rho_plain) < 1e-12
    np.testing.assert_array_equal(host(S.nullvecs(0)), host(plain.nullvecs(0)))
    _, info = S.solve(chi, tol=1e-10)
    assert info[0].converged and info[0].true_rel_res <= 1e-10
    # a convergence factor above the threshold also falls back
    net = amg.Cnn(_flat(_params(6)))
    S, fell_back, rho = amg.Solver.learned(g, params, net, init, rho_iters=8, rho_max=1e-3)
    assert fell_back and abs(rho - rho_plain) < 1e-12
    # below it the proposals are kept, and the solve still reaches the FP64 residual
    S, fell_back, rho = amg.Solver.learned(g, params, net, init, rho_iters=8, rho_max=10.0)
    assert not fell_back and 0.0 < rho < 10.0
    _, info = S.solve(chi, tol=1e-10)
    assert info[0].converged and info[0].true_rel_res <= 1e-10
    # the kept proposals are the network's (no refinement requested)
    P = host(net.propose(dev(U.reshape(2, -1)), L1, L2))
    np.testing.assert_allclose(host(S.nullvecs(0)), P, rtol=0, atol=1e-12)


def test_refined_setup_adaptive_iterations_match_oracle():
    import paper_0707_4018_amd as amg
    print("refined setup vs oracle", flush=True)
    L1 = L2 = 16
    U = u1_config(L1, L2, beta=6.0, seed=8)
    m = 0.1
    A = mg.wilson_stencil(U, m)
    start = vectors(5, L1 * L2, 2, 900)
    rand = vectors(3, L1 * L2, 2, 901)
    po = mg.MGParams(blocks=[(4, 4)], nvec=[5], coarse_tol=1e-3, coarse_maxiter=200)
    pg = amg.MGParams(blocks=[(4, 4)], nvec=[5], coarse_tol=1e-3, coarse_maxiter=200)
    # oracle: 3 given vectors relaxed by 4 MR steps, then 2 adaptive iterations
    vecs = [mg.relax_homogeneous(A, start[k], 4, po.omega) for k in range(3)]
    for k in range(2):
        P = mg.build_prolongator(np.stack(vecs), A.dims, po.blocks[0])
        H2 = mg.Hierarchy([A, mg.galerkin(A, P)], [P], po)
        e = rand[k].copy()
        for _ in range(2):
            e = e - mg.vcycle(H2, 0, A.apply(e))
        vecs.append(e / mg.norm(e))
    S = amg.Solver.refined(amg.Gauge(dev(U), m), pg, dev(start), n_start=3, nu_ref=4, ncyc_ref=2, init=[dev(rand)])
    got = host(S.nullvecs(0))
    for k in range(5):
        assert rel_err(got[k], vecs[k]) < 1e-9, k


def test_convergence_factor_matches_oracle():
    import paper_0707_4018_amd as amg
    print("mg convergence factor", flush=True)
    L1 = L2 = 16
    U = u1_config(L1, L2, beta=6.0, seed=4)
    m = 0.1
    A = mg.wilson_stencil(U, m)
    vecs = [vectors(4, L1 * L2, 2, 800)]
    po = mg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_tol=1e-14, coarse_maxiter=500)
    pg = amg.MGParams(blocks=[(4, 4)], nvec=[4], coarse_tol=1e-14, coarse_maxiter=500)
    H = mg.build_hierarchy(A, vecs, po)
    S = amg.Solver(amg.Gauge(dev(U), m), pg, nullvecs=[dev(v) for v in vecs])
    e0 = synth.gaussian_field((L1 * L2, 2), synth.rng_for(801))
    e = e0.copy()
    for _ in range(3):
        e = e - mg.vcycle(H, 0, A.apply(e))
    ref = (np.linalg.norm(e) / np.linalg.norm(e0)) ** (1 / 3)
    got = S.convergence(dev(e0.reshape(L1 * L2, 2, 1)), 3)
    assert abs(got - ref) < 1e-8 * ref
