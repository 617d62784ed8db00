"""GPU parity at rounding level: the HIP path (through the C ABI) against the
CPU run of the same FMM (cpufmm/: the same plan, every table and pass
computed on the host by routes of its own -- densities by a dense 1-D solve,
reaction M2L tables by direct quadrature of the Legendre products instead of
the Chebyshev expansion, translations through Gaunt coefficients, special
functions in long double).

Agreement to 1e-12 (relative L2 over every target) pins each kernel below the
truncation error at which the comparisons with the oracle work: a kernel
mistake that stays under the method's error (a dropped table entry, a wrong
phase of a high-order term) shows here."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu
NTH = min(16, os.cpu_count() or 1)
TOL = 1e-12


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def cuda(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.fixture(scope="module")
def cf():
    from cpufmm import cpufmm
    cpufmm._load()
    return cpufmm


def gpu_eval(d, k, src, J, tgt=None, mu=None, h=False, **prm):
    f = lmfmm.LayeredDyadicFMM(d, k, mu=mu, **prm).build(src, tgt)
    st = f.stats()
    print("  plan: m2l free %d react %d, cases %d, near pairs %d, direct reaction pairs %d"
          % (st["m2l_pairs_free"], st["m2l_pairs_react"], st["n_cases"], st["p2p_pairs"], st["s2t_pairs"]),
          flush=True)
    out = (f.evaluate_h if h else f.evaluate)(cuda(J)).cpu().numpy()
    f.close()
    return out, st


CASES = {
    "tiny_p8": dict(p=8),
    "tiny_p12_pf16": dict(p=12, p_free=16),
    "tiny_free_m2l_p12": dict(p=12, free_depth=3),
    "tiny_direct_reaction_p8": dict(p=8, react_s2t=2),
    "tiny_no_adapt_p6": dict(p=6, m2l_adapt=0, free_depth=3),
}


@pytest.mark.parametrize("name", list(CASES))
def test_tiny_equals_cpu_run(cf, name):
    d, k, x, J = inputs.tiny(seed=0)
    prm = CASES[name]
    print("case %s %s" % (name, prm), flush=True)
    A, st = gpu_eval(d, k, x, J, **prm)
    ref = cf.run(d, k, x, J, n_threads=NTH, **prm)
    e = rel(A, ref)
    print("  GPU vs CPU run: rel L2 %.2e, max abs %.2e" % (e, np.abs(A - ref).max()), flush=True)
    assert e < TOL
    if name == "tiny_free_m2l_p12":
        assert st["m2l_pairs_free"] > 0
    if name == "tiny_direct_reaction_p8":
        assert st["s2t_pairs"] > 0


def test_three_layer_10k_equals_cpu_run(cf):
    """Three layers, 1e4 points in [-2, 2]^2 (deep reaction trees next to
    the 0.1 gaps, free M2L, direct reaction pairs chosen by the cost model),
    p = 8: every target."""
    d, k, x, J = inputs.three_layer(10000, seed=0, half_width=2.0)
    print("case three-layer 1e4 p=8", flush=True)
    A, st = gpu_eval(d, k, x, J, p=8)
    assert st["m2l_pairs_free"] > 0 and st["s2t_pairs"] > 0
    ref = cf.run(d, k, x, J, p=8, n_threads=NTH)
    e = rel(A, ref)
    print("  GPU vs CPU run: rel L2 %.2e" % e, flush=True)
    assert e < TOL


def test_three_layer_mu_distinct_targets_multi_rhs(cf):
    """Permeabilities, targets distinct from the sources, three right-hand
    sides in one call, p = 10."""
    d, k, src, J = inputs.three_layer(1500, seed=3, half_width=1.0, n_rhs=3)
    _, _, tgt, _ = inputs.three_layer(700, seed=4, half_width=1.0)
    mu = [1.0, 1.8, 0.7]
    print("case three-layer mu, 1500 -> 700, 3 rhs, p=10", flush=True)
    A, _ = gpu_eval(d, k, src, J, tgt, mu=mu, p=10)
    ref = cf.run(d, k, src, J, tgt, mu=mu, p=10, n_threads=NTH)
    for r in range(3):
        e = rel(A[r], ref[r])
        print("  rhs %d: rel L2 %.2e" % (r, e), flush=True)
        assert e < TOL


@pytest.mark.parametrize("direct", [0, 2])
def test_magnetic_equals_cpu_run(cf, direct):
    d, k, x, J = inputs.tiny(seed=0)
    print("case magnetic tiny p=12 p_free=16 react_s2t=%d" % direct, flush=True)
    H, _ = gpu_eval(d, k, x, J, h=True, p=12, p_free=16, react_s2t=direct)
    ref = cf.run(d, k, x, J, mode=1, p=12, p_free=16, react_s2t=direct, n_threads=NTH)
    e = rel(H, ref)
    print("  GPU vs CPU run: rel L2 %.2e" % e, flush=True)
    assert e < TOL


def test_adjoint_equals_cpu_run(cf):
    """gJ = G^H gA on distinct point sets: the GPU's swapped-role build
    against the CPU run of the forward sum with the roles exchanged (the
    reciprocity of the layered Green's function, mu-weighted)."""
    d, k, src, _ = inputs.three_layer(1200, seed=5, half_width=1.0)
    _, _, tgt, gA = inputs.three_layer(900, seed=6, half_width=1.0)
    mu = np.array([1.0, 1.8, 0.7])
    print("case adjoint 1200 sources, 900 targets, mu, p=8", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, mu=mu, p=8).build(src, tgt)
    gJ = f.evaluate_adjoint(cuda(gA)).cpu().numpy()
    f.close()

    def mu_of(z):
        return mu[np.where(z > d[0], 0, np.where(z > d[1], 1, 2))][:, None]

    B = cf.run(d, k, tgt, np.conj(gA * mu_of(tgt[:, 2])), src, mu=mu, p=8, n_threads=NTH)
    ref = np.conj(B) / mu_of(src[:, 2])
    e = rel(gJ, ref)
    print("  GPU vs CPU run: rel L2 %.2e" % e, flush=True)
    assert e < TOL


def test_uneven_geometries_equal_cpu_run(cf):
    """Five clustered geometries of uneven size in one plan (one launch per
    pass for all of them) against the CPU run of the same batch plan."""
    d, k, xs, Js = inputs.uneven_geometries(5, seed=2, n_min=150, n_max=2500)
    print("case batch of %s" % [x.shape[0] for x in xs], flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=8).build_batch(xs)
    A = f.evaluate(cuda(np.concatenate(Js))).cpu().numpy()
    so, to = f.src_off, f.tgt_off
    f.close()
    ref = cf.run(d, k, np.concatenate(xs), np.concatenate(Js), geoms=(so, to), p=8, n_threads=NTH)
    for g in range(len(xs)):
        e = rel(A[so[g]:so[g + 1]], ref[so[g]:so[g + 1]])
        print("  geometry %d (%d points): rel L2 %.2e" % (g, xs[g].shape[0], e), flush=True)
        assert e < TOL


def test_six_layers_equals_cpu_run(cf):
    d, k, x, J = inputs.six_layer(240, seed=0)
    print("case six layers, 240 points, p=8", flush=True)
    A, _ = gpu_eval(d, k, x, J, p=8)
    ref = cf.run(d, k, x, J, p=8, n_threads=NTH)
    e = rel(A, ref)
    print("  GPU vs CPU run: rel L2 %.2e" % e, flush=True)
    assert e < TOL


@pytest.mark.parametrize("direct", [0, 2])
def test_gradient_equals_cpu_run(cf, direct):
    """Source-position gradients (the far field's derivative expansions, the
    free dyadic's derivative, the direct pairs' Bessel-ladder derivatives) on
    distinct point sets with permeabilities and two right-hand sides."""
    d, k, src, J = inputs.three_layer(300, seed=11, half_width=1.0, n_rhs=2)
    _, _, tgt, _ = inputs.three_layer(200, seed=12, half_width=1.0)
    gA = inputs.cotangent(200, n_rhs=2, seed=13)
    mu = [1.0, 1.8, 0.7]
    print("case gradient 300 sources, 200 targets, 2 rhs, mu, p=8, react_s2t=%d" % direct, flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, mu=mu, p=8, react_s2t=direct).build(src, tgt)
    gX = f.grad_src_xyz(cuda(J), cuda(gA)).cpu().numpy()
    st = f.stats()
    f.close()
    ref = cf.grad_src_xyz(d, k, src, J, gA, tgt=tgt, mu=mu, p=8, react_s2t=direct, n_threads=NTH)
    e = rel(gX, ref)
    print("  GPU vs CPU run: rel L2 %.2e (direct reaction pairs of the forward plan: %d)"
          % (e, st["s2t_pairs"]), flush=True)
    assert e < TOL


def test_gradient_same_points_equals_cpu_run(cf):
    d, k, x, J = inputs.tiny(seed=0)
    gA = inputs.cotangent(600, seed=14)
    print("case gradient tiny, targets = sources, p=12, direct reaction pairs", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, react_s2t=2).build(x)
    gX = f.grad_src_xyz(cuda(J), cuda(gA)).cpu().numpy()
    f.close()
    ref = cf.grad_src_xyz(d, k, x, J, gA, p=12, react_s2t=2, n_threads=NTH)
    e = rel(gX, ref)
    print("  GPU vs CPU run: rel L2 %.2e" % e, flush=True)
    assert e < TOL
