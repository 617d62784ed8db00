"""GPU tests of layers with different permeabilities (mu != 1): the HIP path
through the C ABI against the oracle evaluated live on small point sets.

mu enters the two 1-D interface problems and scales the TM part of the
reaction field by mu_target / mu_source; the adjoint and the source-position
gradients use the reciprocity G(x, y) mu(y) = G(y, x)^T mu(x), so their
references here come from the definition (the oracle's matrix, and central
differences of the oracle in the source positions), not from reciprocity.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu

MU3 = [1.0, 1.8, 0.7]
# recorded relative L2 errors against the oracle at p = 12 (free part p = 20),
# margin 3; on this small geometry the same-points case carries the larger
# truncation error at mu = 1 too (3.0e-5)
TOL_FWD = {"same points": 1e-4, "distinct targets": 2e-6}
TOL_REACT16 = 3.4e-6
TOL_ADJ = {"same points": 7e-5, "distinct targets": 2.1e-6}
TOL_GRAD = 3.4e-6
TOL_100K = 2.9e-6


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def cuda(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.fixture(scope="module")
def case():
    d, k, src, J = inputs.three_layer(160, seed=7, half_width=1.0)
    _, _, tgt, _ = inputs.three_layer(90, seed=8, half_width=1.0)
    gA = inputs.cotangent(tgt.shape[0], seed=7)
    return d, k, src, J, tgt, gA


def test_forward_with_mu(case):
    from oracle import oracle
    d, k, src, J, tgt, gA = case
    for pts_t, name in [(src, "same points"), (tgt, "distinct targets")]:
        print("case mu forward, %s" % name, flush=True)
        tg = None if pts_t is src else pts_t
        f = lmfmm.LayeredDyadicFMM(d, k, mu=MU3, p=12, p_free=20).build(src, tg)
        A = f.evaluate(cuda(J)).cpu().numpy()
        f.close()
        ref = oracle.direct(d, k, src, J, pts_t, mu=MU3)
        e = rel(A, ref)
        # the permeabilities change the answer: mu = 1 is far from it; the
        # same geometry at mu = 1 shows the FMM's truncation error there
        ref1 = oracle.direct(d, k, src, J, pts_t)
        f1 = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(src, tg)
        e1 = rel(f1.evaluate(cuda(J)).cpu().numpy(), ref1)
        f1.close()
        print("  rel err %.2e (at mu = 1: %.2e; mu = 1 differs by %.2e)" % (e, e1, rel(ref1, ref)), flush=True)
        assert e < TOL_FWD[name] and rel(ref1, ref) > 1e-2
        assert e <= 3 * e1 + 1e-7  # mu adds no error beyond the truncation at mu = 1


def test_two_layer_mu_reaction_part(case):
    """Two layers of different mu, reaction components only, p = 16."""
    from oracle import oracle
    d, k, x, J = inputs.tiny(seed=3)
    sel = np.arange(0, 600, 4)
    x, J = x[sel], J[sel]
    mu = [1.3, 0.6]
    print("case mu two-layer reaction p=16", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, mu=mu, p=16, components=2).build(x)
    A = f.evaluate(cuda(J)).cpu().numpy()
    f.close()
    ref = oracle.direct(d, k, x, J, x, mu=mu) - oracle.direct_free(d, k, x, J, x)
    e = rel(A, ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < TOL_REACT16


def _dense(oracle, d, k, src, tgt, mu):
    """M [3 n_tgt, 3 n_src] of the layered sum, by unit currents."""
    n = src.shape[0]
    M = np.zeros((3 * tgt.shape[0], 3 * n), dtype=complex)
    for c0 in range(0, 3 * n, 64):
        cols = np.arange(c0, min(3 * n, c0 + 64))
        E = np.zeros((cols.size, n, 3), dtype=complex)
        E[np.arange(cols.size), cols // 3, cols % 3] = 1.0
        M[:, cols] = oracle.direct(d, k, src, E, tgt, mu=mu).reshape(cols.size, -1).T
    return M


def test_adjoint_with_mu(case):
    from oracle import oracle
    d, k, src, J, tgt, gA = case
    for pts_t, name in [(src, "same points"), (tgt, "distinct targets")]:
        print("case mu adjoint, %s" % name, flush=True)
        g = gA if pts_t is tgt else inputs.cotangent(src.shape[0], seed=9)
        M = _dense(oracle, d, k, src, pts_t, MU3)
        ref = (M.conj().T @ g.ravel()).reshape(-1, 3)
        f = lmfmm.LayeredDyadicFMM(d, k, mu=MU3, p=12, p_free=20).build(src, None if pts_t is src else pts_t)
        gJ = f.evaluate_adjoint(cuda(g)).cpu().numpy()
        f.close()
        e = rel(gJ, ref)
        print("  rel err %.2e" % e, flush=True)
        assert e < TOL_ADJ[name]


def test_grad_src_with_mu(case):
    """dL/dx_j = Re sum_i gA_i^H d/dx_j G(x_i, x_j) J_j against central
    differences of the oracle (only source j moves; distinct targets)."""
    from oracle import oracle
    d, k, src, J, tgt, gA = case
    print("case mu source gradient", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, mu=MU3, p=12, p_free=20).build(src, tgt)
    gX = f.grad_src_xyz(cuda(J), cuda(gA)).cpu().numpy()
    f.close()
    js = inputs.sample_sources(src.shape[0], 6, seed=7)
    h = 1e-5
    ref = np.zeros((js.size, 3))
    for a, j in enumerate(js):
        for c in range(3):
            xp, xm = src[j:j + 1].copy(), src[j:j + 1].copy()
            xp[0, c] += h
            xm[0, c] -= h
            Ap = oracle.direct(d, k, xp, J[j:j + 1], tgt, mu=MU3)
            Am = oracle.direct(d, k, xm, J[j:j + 1], tgt, mu=MU3)
            ref[a, c] = np.real(np.vdot(gA, (Ap - Am) / (2 * h)))
    e = rel(gX[js], ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < TOL_GRAD


def test_mu_validation():
    for mu in ([1.0, 0.0], [1.0, -2.0], [1.0, float("inf")], [1.0, float("nan")]):
        with pytest.raises(lmfmm.LMError):
            lmfmm.LayeredDyadicFMM([0.0], [1.0, 1.5], mu=mu)
    with pytest.raises(lmfmm.LMError):
        lmfmm.LayeredDyadicFMM([0.0], [1.0, 1.5], mu=[1.0])


def test_three_layer_100k_mu_sampled():
    """1e5 points (the scale configuration) with permeabilities: 400-source
    sparse currents at full size, 64 sampled targets against the oracle."""
    from oracle import oracle
    d, k, x, J = inputs.three_layer(100000, seed=0)
    Js, keep = inputs.sparse_currents(J, 400, seed=0)
    idx = inputs.sample_targets(x.shape[0], count=64, seed=0)
    print("case mu three-layer n=100000 p=12 p_free=20 (sampled)", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, mu=MU3, p=12, p_free=20).build(x)
    A = f.evaluate(cuda(Js)).cpu().numpy()
    f.close()
    ref = oracle.direct(d, k, x[keep], Js[keep], x[idx], mu=MU3)
    e = rel(A[idx], ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < TOL_100K
