"""GPU tests of the magnetic field H = G_H J (lm_evaluate_h) through the C ABI
against the oracle's magnetic dyadic (the J6..J9 spectral form, evaluated
live): the GPU path takes the curl of the electric field's local expansions
and the closed-form free-space curl, an independent route."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu

MU3 = [1.0, 1.8, 0.7]
# recorded relative L2 errors against the oracle (p = 12 unless noted, free part
# p = 20), margin 3
TOL = {"tiny12": 9.1e-7, "tiny16": 1.3e-7, "mu_same": 9e-6, "mu_distinct": 1.9e-6, "100k": 1.1e-5,
       "tiny_direct": 4.7e-7, "mu_direct": 8e-7}


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def cuda(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("p", [12, 16])
def test_magnetic_tiny(p):
    from oracle import oracle
    d, k, x, J = inputs.tiny(seed=0)
    sel = np.arange(0, 600, 3)
    x, J = x[sel], J[sel]
    print("case magnetic tiny n=%d p=%d p_free=20" % (x.shape[0], p), flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=p, p_free=20).build(x)
    H = f.evaluate_h(cuda(J)).cpu().numpy()
    H2 = f.evaluate_h(cuda(np.stack([J, 2j * J]))).cpu().numpy()
    f.close()
    ref = oracle.direct_h(d, k, x, J, x)
    e = rel(H, ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < TOL["tiny%d" % p]
    assert np.array_equal(H2[0], H) and rel(H2[1], 2j * H) < 1e-14


def test_magnetic_with_mu():
    from oracle import oracle
    d, k, src, J = inputs.three_layer(160, seed=7, half_width=1.0)
    _, _, tgt, _ = inputs.three_layer(90, seed=8, half_width=1.0)
    for name, tg in [("mu_same", None), ("mu_distinct", tgt)]:
        print("case magnetic three-layer with mu, %s" % name, flush=True)
        f = lmfmm.LayeredDyadicFMM(d, k, mu=MU3, p=12, p_free=20).build(src, tg)
        H = f.evaluate_h(cuda(J)).cpu().numpy()
        f.close()
        ref = oracle.direct_h(d, k, src, J, src if tg is None else tg, mu=MU3)
        e = rel(H, ref)
        print("  rel err %.2e" % e, flush=True)
        assert e < TOL[name]


def test_magnetic_tiny_direct_near_field():
    """Every adjacent reaction pair evaluated directly (the J6..J9 Sommerfeld
    integrals of the near-field kernel), two layers, p = 12."""
    from oracle import oracle
    d, k, x, J = inputs.tiny(seed=0)
    sel = np.arange(0, 600, 3)
    x, J = x[sel], J[sel]
    print("case magnetic tiny n=%d p=12 p_free=20, direct reaction near field" % x.shape[0], flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20, react_s2t=2).build(x)
    assert f.stats()["s2t_pairs"] > 0
    H = f.evaluate_h(cuda(J)).cpu().numpy()
    f.close()
    ref = oracle.direct_h(d, k, x, J, x)
    e = rel(H, ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < TOL["tiny_direct"]


def test_magnetic_mu_direct_near_field():
    from oracle import oracle
    d, k, src, J = inputs.three_layer(160, seed=7, half_width=1.0)
    print("case magnetic three-layer with mu, direct reaction near field", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, mu=MU3, p=12, p_free=20, react_s2t=2).build(src)
    assert f.stats()["s2t_pairs"] > 0
    H = f.evaluate_h(cuda(J)).cpu().numpy()
    f.close()
    ref = oracle.direct_h(d, k, src, J, src, mu=MU3)
    e = rel(H, ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < TOL["mu_direct"]


def test_magnetic_100k_sampled():
    """The scale configuration (its plan evaluates the reaction pairs next to
    the interfaces directly)."""
    from oracle import oracle
    d, k, x, J = inputs.three_layer(100000, seed=0)
    Js, keep = inputs.sparse_currents(J, 400, seed=0)
    idx = inputs.sample_targets(x.shape[0], count=64, seed=0)
    print("case magnetic three-layer n=100000 p=12 p_free=20 (sampled)", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(x)
    Jt = cuda(Js)
    t0 = time.time()
    H = f.evaluate_h(Jt)
    torch.cuda.synchronize()
    t1 = time.time()
    H = f.evaluate_h(Jt)
    torch.cuda.synchronize()
    t2 = time.time()
    H = H.cpu().numpy()
    f.close()
    ref = oracle.direct_h(d, k, x[keep], Js[keep], x[idx])
    e = rel(H[idx], ref)
    print("  rel err %.2e, first call %.2f s, then %.1f ms" % (e, t1 - t0, 1e3 * (t2 - t1)), flush=True)
    assert e < TOL["100k"]


def test_magnetic_batch_equals_separate_builds():
    """Several geometries in one plan (with direct reaction pairs): each
    geometry's H equals that of its own build."""
    d, k, xs, Js = inputs.uneven_geometries(4, seed=1, n_min=500, n_max=6000)
    print("case magnetic, 4 geometries, sizes %s" % [x.shape[0] for x in xs], flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=8).build_batch(xs)
    H = f.evaluate_h(cuda(np.concatenate(Js))).cpu().numpy()
    f.close()
    so = np.cumsum([0] + [x.shape[0] for x in xs])
    for g in range(len(xs)):
        fg = lmfmm.LayeredDyadicFMM(d, k, p=8).build(xs[g])
        Hg = fg.evaluate_h(cuda(Js[g])).cpu().numpy()
        fg.close()
        e = rel(H[so[g]:so[g + 1]], Hg)
        print("  geometry %d: rel diff %.3e" % (g, e), flush=True)
        assert e < 1e-12
