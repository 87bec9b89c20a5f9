"""GPU parity of the multigrid for the normal equations A = D^dag D (the
paper's own variant) against the oracle, through the C ABI.

Small lattices: every piece element by element (P, the Galerkin operators,
the frozen step lengths, the power estimate and damping of the smoothed P),
the V-cycle's output and its Hermiticity (Eq. (3)), CG and MG-CG iteration
counts and solutions, the adaptive vectors, the mass change.  The paper's
128^2 size: properties that hold at any size (Hermitian positive V, the true
residual with the oracle's D, MG-CG far below CG).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import dirac, mg, normal

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SA = 4.0 / 3.0


def _field(L, beta=6.0, sweeps=40, seed=0):
    return dirac.u1_field(synth.u1_heatbath(L, L, beta, sweeps, synth.rng_for(150, seed, L)))


def _inputs(L, blocks, nvec, seed=0):
    dims = [(L, L)]
    vecs, sb = [], []
    for l, (b, nv) in enumerate(zip(blocks, nvec)):
        V = dims[-1][0] * dims[-1][1]
        dof = 2 if l == 0 else nvec[l - 1]
        vecs.append(np.stack([synth.gaussian_field((V, dof), synth.rng_for(151, seed, l, k)) for k in range(nv)]))
        sb.append(synth.gaussian_field((V, dof), synth.rng_for(152, seed, l)))
        dims.append((dims[-1][0] // b[0], dims[-1][1] // b[1]))
    return vecs, sb


def _cuda(xs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]


def _gauge(U, m):
    import torch
    import paper_0707_4018_amd as amg
    return amg.Gauge(torch.from_numpy(U).cuda(), m)


def _params(blocks, nvec, sa):
    import paper_0707_4018_amd as amg
    return amg.NormalParams(blocks=blocks, nvec=nvec, sa_factor=sa)


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


CASES = [  # (L, blocks, nvec, smoothing factor, fine D^dag D as one box stencil)
    (16, [(4, 4)], [4], 0.0, True),
    (16, [(4, 4)], [4], SA, True),
    (24, [(4, 4), (2, 2)], [4, 3], 0.0, True),       # M changes between levels, coarse extent 3
    (48, [(4, 4), (4, 4)], [4, 4], SA, True),        # three levels, 12^2 then 3^2
    (48, [(4, 4), (4, 4)], [4, 4], SA, False),       # the same with D then D^dag (the large-lattice path)
]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"L{c[0]}-{len(c[1]) + 1}lv-sa{c[3] > 0}-box{int(c[4])}")
def given(request):
    import paper_0707_4018_amd as amg
    L, blocks, nvec, sa, fine_box = request.param
    print(f"normal MG given vectors L={L} blocks={blocks} nvec={nvec} sa={sa}", flush=True)
    m = 0.05
    U = _field(L)
    D = mg.wilson_stencil(U, m).to_sparse()
    vecs, sb = _inputs(L, blocks, nvec)
    H = normal.build(D, (L, L), vecs, blocks, [s.ravel() for s in sb], sa=sa)
    g = _gauge(U, m)
    prm = _params(blocks, nvec, sa)
    prm.fine_box = fine_box
    S = amg.NormalMG(g, prm, _cuda(sb), vecs=_cuda(vecs))
    return dict(L=L, U=U, D=D, H=H, g=g, S=S, blocks=blocks, nvec=nvec, sa=sa, vecs=vecs, sb=sb, m=m)


def test_hierarchy_matches_oracle(given):
    H, S = given["H"], given["S"]
    for l in range(H.nlevels - 1):
        P = S.export(l, 0).cpu().numpy()
        Po = H.Ps[l].toarray()
        assert _rel(P, Po) < 1e-13, l
        info = S.level_info(l)
        assert abs(info["taus"][0] - H.taus[l][0]) <= 1e-12 * abs(H.taus[l][0])
        assert abs(info["taus"][1] - H.taus[l][1]) <= 1e-12 * abs(H.taus[l][1])
        assert abs(info["sa_omega"] - H.sa_omegas[l]) <= 1e-12 * max(H.sa_omegas[l], 1e-300)
    for l in range(1, H.nlevels):
        A = S.export(l, 1).cpu().numpy()
        Ao = H.ops[l].M.toarray()
        assert np.abs(A - Ao).max() < 1e-12 * np.abs(Ao).max(), l


def test_level_operators_match_oracle(given):
    H, S = given["H"], given["S"]
    for l in range(H.nlevels):
        n = H.ops[l].n
        x = synth.gaussian_field((n,), synth.rng_for(153, l))
        shape = (n // 2, 2) if l == 0 else (n,)
        y = S.level_apply(l, _cuda([x.reshape(shape)])[0]).cpu().numpy().ravel()
        assert _rel(y, H.ops[l].M @ x) < 1e-13, l


def test_vcycle_matches_oracle_and_is_hermitian(given):
    H, S = given["H"], given["S"]
    n = H.ops[0].n
    xs = [synth.gaussian_field((n,), synth.rng_for(154, s)) for s in range(2)]
    Vx = [S.vcycle(_cuda([x.reshape(n // 2, 2)])[0]).cpu().numpy().ravel() for x in xs]
    for x, v in zip(xs, Vx):
        assert _rel(v, normal.vcycle(H, 0, x)) < 1e-11
    lhs, rhs = np.vdot(xs[0], Vx[1]), np.vdot(Vx[0], xs[1])
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    q = np.vdot(xs[0], Vx[0])
    assert q.real > 0 and abs(q.imag) < 1e-11 * abs(q)


def test_cg_and_mgcg_match_oracle(given):
    H, S, D, L = given["H"], given["S"], given["D"], given["L"]
    chi = synth.gaussian_field((L * L, 2), synth.rng_for(155))
    b = D.conj().T @ chi.ravel()
    x_o, i_o = normal.mgcg(H, b, 1e-12)
    psi, info = S.solve(_cuda([chi])[0], tol=1e-12, precond=True)
    psi = psi.cpu().numpy().ravel()
    print(f"MG-CG GPU {info.iters} it, oracle {i_o.iters}; D applications {info.n_fine_D}", flush=True)
    assert info.converged and i_o.converged
    assert abs(info.iters - i_o.iters) <= 1
    assert _rel(psi, x_o) < 1e-9
    assert np.linalg.norm(b - H.ops[0].M @ psi) <= 1e-12 * np.linalg.norm(b) * 1.01
    assert np.linalg.norm(chi.ravel() - D @ psi) / np.linalg.norm(chi) == pytest.approx(info.rel_res_D, rel=1e-6)
    # per iteration: 5 D and 5 D^dag (outer CG + 2 pre + residual + post), plus b = D^dag chi, the
    # residual checks and |chi - D psi|
    assert info.n_fine_D >= 5 * info.iters and info.n_fine_D <= 5 * info.iters + 4 + 2 * info.restarts
    x_c, i_c = normal.pcg(H.ops[0], b, None, 1e-12, 100000)
    psi_c, info_c = S.solve(_cuda([chi])[0], tol=1e-12, precond=False)
    print(f"CG GPU {info_c.iters} it, oracle {i_c.iters}", flush=True)
    assert info_c.converged and abs(info_c.iters - i_c.iters) <= max(2, i_c.iters // 50)
    assert _rel(psi_c.cpu().numpy().ravel(), x_c) < 1e-9
    assert info.iters < info_c.iters


def test_set_mass_rebuilds_the_hierarchy(given):
    H, S, L = given["H"], given["S"], given["L"]
    m2 = 0.2
    D2 = mg.wilson_stencil(given["U"], m2).to_sparse()
    H2 = normal.with_mass(D2, H, given["vecs"], given["blocks"], [s.ravel() for s in given["sb"]], (L, L),
                          sa=given["sa"])
    given["g"].set_mass(m2)
    S.set_mass(m2)
    try:
        for l in range(1, H2.nlevels):
            A = S.export(l, 1).cpu().numpy()
            Ao = H2.ops[l].M.toarray()
            assert np.abs(A - Ao).max() < 1e-12 * np.abs(Ao).max(), l
        for l in range(H2.nlevels - 1):
            assert abs(S.level_info(l)["taus"][0] - H2.taus[l][0]) <= 1e-12 * abs(H2.taus[l][0])
        n = H2.ops[0].n
        x = synth.gaussian_field((n,), synth.rng_for(156))
        v = S.vcycle(_cuda([x.reshape(n // 2, 2)])[0]).cpu().numpy().ravel()
        assert _rel(v, normal.vcycle(H2, 0, x)) < 1e-11
    finally:
        given["g"].set_mass(given["m"])
        S.set_mass(given["m"])


@pytest.mark.parametrize("L,blocks,nvec,nu0,ncyc,sa", [
    (32, [(4, 4)], [4], [10], [3], SA),
    (48, [(4, 4), (4, 4)], [4, 4], [10, 20], [3, 5], SA),
    (24, [(4, 4), (2, 2)], [4, 3], [10, 10], [3, 3], 0.0),
])
def test_adaptive_setup_matches_oracle(L, blocks, nvec, nu0, ncyc, sa):
    import paper_0707_4018_amd as amg
    print(f"normal MG adaptive L={L} blocks={blocks} nvec={nvec} sa={sa}", flush=True)
    U = _field(L, seed=1)
    m = -0.05
    D = mg.wilson_stencil(U, m).to_sparse()
    init, sb = _inputs(L, blocks, nvec, seed=1)
    H, vecs = normal.adaptive_setup(D, (L, L), blocks, nvec, init, [s.ravel() for s in sb], nu0=nu0, ncyc=ncyc,
                                    sa=sa, setup_dense_max=1024)
    S = amg.NormalMG(_gauge(U, m), _params(blocks, nvec, sa), _cuda(sb), init=_cuda(init), nu0=nu0, ncyc=ncyc)
    for l in range(len(blocks)):
        v = S.export(l, 2).cpu().numpy()
        assert _rel(v, vecs[l]) < 1e-8, l
    chi = synth.gaussian_field((L * L, 2), synth.rng_for(157))
    b = D.conj().T @ chi.ravel()
    _, i_o = normal.mgcg(H, b, 1e-10)
    _, info = S.solve(_cuda([chi])[0], tol=1e-10)
    assert info.converged and abs(info.iters - i_o.iters) <= 1


def test_errors_are_reported():
    import torch
    import paper_0707_4018_amd as amg
    L = 16
    U = _field(L)
    vecs, sb = _inputs(L, [(4, 4)], [4])
    g = _gauge(U, 0.05)
    bad = vecs[0].copy()
    bad[1] = bad[0]
    with pytest.raises(amg.AMGError) as e:
        amg.NormalMG(g, _params([(4, 4)], [4], 0.0), _cuda(sb), vecs=_cuda([bad]))
    assert e.value.status == 6                      # AMG_ERR_RANK
    with pytest.raises(amg.AMGError) as e:          # coarse extent 2: no colouring of period >= 3
        amg.NormalMG(g, _params([(8, 8)], [4], 0.0), _cuda(sb), vecs=_cuda([vecs[0]]))
    assert e.value.status == 2                      # AMG_ERR_SHAPE
    with pytest.raises(amg.AMGError) as e:          # smoothed P needs blocks >= 3
        v2, s2 = _inputs(L, [(2, 2)], [4])
        amg.NormalMG(g, _params([(2, 2)], [4], SA), _cuda(s2), vecs=_cuda(v2))
    assert e.value.status == 2
    U4 = synth.su3_haar((4, 4, 4, 4, 4), synth.rng_for(158))
    g4 = amg.Gauge(torch.from_numpy(np.ascontiguousarray(U4.reshape(4, 4, 4, 4, 4, 3, 3))).cuda(), 0.1)
    with pytest.raises(amg.AMGError) as e:
        amg.NormalMG(g4, _params([(2, 2)], [4], 0.0), _cuda(sb), vecs=_cuda([vecs[0]]))
    assert e.value.status == 2


@pytest.fixture(scope="module")
def paper128():
    """The 128^2, beta = 6, Q = 0 ensemble of the workload table, adaptive
    set-up at m_hat = 0.001 with the paper's blocks and M = 8 and smoothing."""
    import paper_0707_4018_amd as amg
    wl = json.load(open(os.path.join(ROOT, "synth", "workloads.json")))["paper128_b6_q0"]
    L = 128
    th = synth.u1_field_of(wl)
    assert synth.u1_mean_plaquette(th) == wl["plaquette"]
    U = dirac.u1_field(th)
    mc = wl["m_crit"]
    print(f"paper-size normal MG beta=6 Q=0 m_crit={mc}", flush=True)
    init, sb = _inputs(L, [(4, 4), (4, 4)], [8, 8], seed=2)
    g = _gauge(U, mc + 0.001)
    S = amg.NormalMG(g, _params([(4, 4), (4, 4)], [8, 8], SA), _cuda(sb), init=_cuda(init), nu0=[100, 500],
                     ncyc=[20, 200])
    return dict(U=U, mc=mc, g=g, S=S, L=L)


def test_paper_size_vcycle_is_hermitian_positive(paper128):
    S, L = paper128["S"], paper128["L"]
    n = L * L * 2
    xs = [synth.gaussian_field((n,), synth.rng_for(159, s)) for s in range(2)]
    Vx = [S.vcycle(_cuda([x.reshape(n // 2, 2)])[0]).cpu().numpy().ravel() for x in xs]
    lhs, rhs = np.vdot(xs[0], Vx[1]), np.vdot(Vx[0], xs[1])
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    for x, v in zip(xs, Vx):
        assert np.vdot(x, v).real > 0


def test_paper_size_mgcg_removes_critical_slowing_down(paper128):
    """m_hat = 0.1 and 0.01 with the set-up of m_hat = 0.001: MG-CG needs a
    few tens of iterations at both, CG many times more; the answer solves
    D psi = chi to the tolerance (residual with the oracle's D)."""
    S, g, U, mc, L = paper128["S"], paper128["g"], paper128["U"], paper128["mc"], paper128["L"]
    chi = np.zeros((L * L, 2), dtype=np.complex128)
    chi[0, 0] = 1.0
    its = {}
    try:
        for gap in (0.1, 0.01):
            g.set_mass(mc + gap)
            S.set_mass(mc + gap)
            psi, info = S.solve(_cuda([chi])[0], tol=1e-12)
            _, info_c = S.solve(_cuda([chi])[0], tol=1e-12, precond=False)
            Dm = mg.wilson_stencil(U, mc + gap).to_sparse()
            b = Dm.conj().T @ chi.ravel()
            x = psi.cpu().numpy().ravel()
            assert np.linalg.norm(b - Dm.conj().T @ (Dm @ x)) <= 1.01e-12 * np.linalg.norm(b)
            its[gap] = (info.iters, info_c.iters)
            print(f"m_hat {gap}: MG-CG {info.iters}, CG {info_c.iters}", flush=True)
    finally:
        g.set_mass(mc + 0.001)
        S.set_mass(mc + 0.001)
    assert its[0.01][0] <= 40 and its[0.1][0] <= 40
    assert its[0.01][1] > 20 * its[0.01][0]
