"""GPU parity tests: the HIP fast multipole path (through the C ABI) against
the CPU oracle (stored outputs in tests/golden/, written by
tests/golden/make_golden.py from oracle/ only, or computed live for small
cases).

Tolerances are the truncation errors recorded at each expansion order p
(the FMM is an approximation of the direct sum; the method converges
spectrally in p), with a margin of 3; exact (bitwise) equality is required
where the arithmetic is identical (repeat runs, batched vs single right-hand
sides).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def tiny():
    d, k, x, J = inputs.tiny(seed=0)
    g = np.load(os.path.join(GOLD, "tiny_oracle.npz"))
    return d, k, x, J, g


def run(d, k, x, J, **kw):
    f = lmfmm.LayeredDyadicFMM(d, k, **kw).build(x)
    print("  build ok: %s" % {a: int(b) for a, b in f.stats().items()
                              if a in ("m2l_pairs_free", "m2l_pairs_react", "n_cases")}, flush=True)
    A = f.evaluate(torch.tensor(J, device="cuda")).cpu().numpy()
    f.close()
    return A


# recorded truncation errors (relative L2 over all 600 targets) x 3
TINY_TOL = {4: 1e-4, 8: 3e-6, 12: 4e-7}
TINY_TOL_REACT = {4: 3e-2, 8: 5e-4, 12: 1.2e-5, 16: 5e-7}
COARSE_TOL = {8: 2.2e-4, 12: 1.4e-5}  # recorded 7.1e-5 and 4.4e-6, margin 3


@pytest.mark.parametrize("p", [4, 8, 12])
def test_tiny_full_field(tiny, p):
    d, k, x, J, g = tiny
    print("case tiny full p=%d" % p, flush=True)
    A = run(d, k, x, J, p=p)
    e = rel(A, g["A"])
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < TINY_TOL[p]


@pytest.mark.parametrize("p", [4, 8, 12, 16])
def test_tiny_reaction_part(tiny, p):
    d, k, x, J, g = tiny
    print("case tiny reaction p=%d" % p, flush=True)
    A = run(d, k, x, J, p=p, components=2)
    e = rel(A, g["A"] - g["A_free"])
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < TINY_TOL_REACT[p]


def test_tiny_free_part_and_subset(tiny):
    """The free part alone, over all targets and over a subset that excludes
    no near pairs of its own (the all-target norm is dominated by the closest
    pairs, which the near field computes directly)."""
    d, k, x, J, g = tiny
    print("case tiny free p=12", flush=True)
    A = run(d, k, x, J, p=12, components=1)
    assert rel(A, g["A_free"]) < 4e-7
    idx = np.arange(0, 600, 7)
    assert rel(A[idx], g["A_free"][idx]) < 1.2e-5


def test_spectral_convergence(tiny):
    d, k, x, J, g = tiny
    errs = [rel(run(d, k, x, J, p=p, components=2), g["A"] - g["A_free"]) for p in (4, 8, 12)]
    print("  reaction errors", errs, flush=True)
    assert errs[0] > 10 * errs[1] > 100 * errs[2]


def test_deterministic_and_batched(tiny):
    d, k, x, J, g = tiny
    print("case determinism / batching", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=8).build(x)
    Jt = torch.tensor(J, device="cuda")
    a1 = f.evaluate(Jt).cpu().numpy()
    a2 = f.evaluate(Jt).cpu().numpy()
    assert np.array_equal(a1, a2)
    rng = np.random.default_rng(3)
    J5 = rng.uniform(-1, 1, (5, 600, 3)) + 1j * rng.uniform(-1, 1, (5, 600, 3))
    J5[2] = J
    A5 = f.evaluate(torch.tensor(J5, device="cuda")).cpu().numpy()
    assert np.array_equal(A5[2], a1)
    for r in (0, 4):
        assert np.array_equal(A5[r], f.evaluate(torch.tensor(J5[r], device="cuda")).cpu().numpy())
    f.close()


def test_linearity_and_zero(tiny):
    d, k, x, J, g = tiny
    f = lmfmm.LayeredDyadicFMM(d, k, p=6).build(x)
    Jt = torch.tensor(J, device="cuda")
    z = f.evaluate(torch.zeros_like(Jt)).cpu().numpy()
    assert np.all(z == 0)
    a = f.evaluate(Jt).cpu().numpy()
    b = f.evaluate((2.0 - 1.0j) * Jt).cpu().numpy()
    assert rel(b, (2.0 - 1.0j) * a) < 1e-13
    f.close()


def test_distinct_targets_and_ragged_sizes():
    """Targets different from the sources, a ragged source count, a single
    source and a single target: against the oracle computed live."""
    from oracle import oracle
    d, k, x, J = inputs.tiny(seed=5)
    src, Js = x[:437], J[:437]
    tgt = x[437:] + np.array([0.013, -0.02, 0.0])
    tgt[:, 2] = np.where(np.abs(tgt[:, 2]) < 0.1, np.sign(tgt[:, 2]) * 0.15, tgt[:, 2])
    print("case distinct targets 437 x 163", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=10).build(src, tgt)
    A = f.evaluate(torch.tensor(Js, device="cuda")).cpu().numpy()
    f.close()
    ref = oracle.direct(d, k, src, Js, tgt)
    print("  rel L2 = %.3e" % rel(A, ref), flush=True)
    assert rel(A, ref) < 1e-5
    print("case single source / single target", flush=True)
    # well separated relative to the (single-point) root boxes: near exact
    s1 = np.array([[0.30, 0.20, 1.50]])
    t1 = np.array([[0.35, 0.10, -0.50]])
    f = lmfmm.LayeredDyadicFMM(d, k, p=12).build(s1, t1)
    A1 = f.evaluate(torch.tensor(Js[:1], device="cuda")).cpu().numpy()
    f.close()
    ref1 = oracle.direct(d, k, s1, Js[:1], t1)
    print("  single pair rel %.3e" % rel(A1, ref1), flush=True)
    assert rel(A1, ref1) < 1e-10
    # a pair at the worst admissible box geometry: error bounded by the
    # truncation of a single M2L with separation ratio ~0.6
    f = lmfmm.LayeredDyadicFMM(d, k, p=16).build(src[:1], tgt[:1])
    A1 = f.evaluate(torch.tensor(Js[:1], device="cuda")).cpu().numpy()
    f.close()
    ref1 = oracle.direct(d, k, src[:1], Js[:1], tgt[:1])
    print("  worst-geometry pair rel %.3e" % rel(A1, ref1), flush=True)
    assert rel(A1, ref1) < 1e-3


def test_empty_inputs():
    f = lmfmm.LayeredDyadicFMM([0.0], [1.0, 1.5], p=4).build(np.zeros((0, 3)), np.array([[0.0, 0.0, 0.5]]))
    A = f.evaluate(torch.zeros((0, 3), dtype=torch.complex128, device="cuda"))
    assert A.shape == (1, 3) and torch.all(A == 0)
    f.close()


def test_error_paths():
    f = lmfmm.LayeredDyadicFMM([0.0], [1.0, 1.5], p=4)
    with pytest.raises(lmfmm.LMError):
        f.evaluate(torch.zeros((2, 3), dtype=torch.complex128, device="cuda"))
    with pytest.raises(lmfmm.LMError):
        f.build(np.array([[0.0, 0.0, 0.0]]))      # point on the interface
    f.close()


# The accuracy the metric asks for (relative L2 <= 1e-6) at the benchmark
# configuration (p = 12, free part p = 20, automatic depths) on 256 sampled
# targets: recorded 3.27e-7 at 1e5 (depth 3) and 3.55e-7 at 1e6 (depth 4);
# free part p = 12 at depth 3: 4.2e-7.
@pytest.mark.parametrize("n,p,pf,fd,tol", [(100000, 12, 20, 0, 1e-6), (1000000, 12, 20, 0, 1e-6),
                                           (100000, 12, 12, 3, 1e-6)])
def test_three_layer_full_size_sampled(n, p, pf, fd, tol):
    """Three-layer workload at full size (the benchmark's tree and launch
    configuration), currents nonzero on 400 sources, oracle on 256 sampled
    targets."""
    fn = os.path.join(GOLD, "three_%d_sparse400_oracle.npz" % n)
    if not os.path.exists(fn):
        pytest.skip("stored oracle output missing: %s" % fn)
    g = np.load(fn)
    d, k, x, J = inputs.three_layer(n, seed=0)
    Js, keep = inputs.sparse_currents(J, 400, seed=0)
    assert np.array_equal(keep, g["keep"])
    print("case three-layer n=%d p=%d p_free=%d free_depth=%d" % (n, p, pf, fd), flush=True)
    A = run(d, k, x, Js, p=p, p_free=pf, free_depth=fd)
    e = rel(A[g["idx"]], g["A"])
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < tol


@pytest.mark.parametrize("p,pf", [(8, 12), (12, 8)])
def test_mixed_orders(tiny, p, pf):
    """Free-space and reaction parts with different expansion orders in one
    build (their M2L work shares one scratch buffer with per-block bases)."""
    d, k, x, J, g = tiny
    print("case mixed orders p=%d p_free=%d" % (p, pf), flush=True)
    A = run(d, k, x, J, p=p, p_free=pf)
    e = rel(A, g["A"])
    ref_err = max(TINY_TOL[8], 1e-12)
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < ref_err


def test_many_rhs_chunked(tiny):
    """More right-hand sides than one pass handles (processed in chunks of
    16): every column equals its single-rhs evaluation bitwise."""
    d, k, x, J, g = tiny
    print("case 21 right-hand sides", flush=True)
    rng = np.random.default_rng(9)
    Jm = rng.uniform(-1, 1, (21, 600, 3)) + 1j * rng.uniform(-1, 1, (21, 600, 3))
    f = lmfmm.LayeredDyadicFMM(d, k, p=6).build(x)
    Am = f.evaluate(torch.tensor(Jm, device="cuda")).cpu().numpy()
    for r in (0, 15, 16, 20):
        assert np.array_equal(Am[r], f.evaluate(torch.tensor(Jm[r], device="cuda")).cpu().numpy())
    f.close()


# direct reaction near field (S2T): reaction trees stop one level early next
# to the gap and adjacent leaves interact through the component's Sommerfeld
# integral; recorded errors x 3 (tiny: 783 direct pairs; reaction part
# p = 8 / 12: 1.24e-4 / 3.39e-6, full field p = 12 9.4e-8; 1e5 sampled with
# the cost model choosing the direct pairs: recorded below)
@pytest.mark.parametrize("p,tol", [(8, 5e-4), (12, 1.2e-5)])
def test_tiny_reaction_part_direct_near_field(tiny, p, tol):
    d, k, x, J, g = tiny
    print("case tiny reaction, direct near field, p=%d" % p, flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=p, components=2, react_s2t=2).build(x)
    assert f.stats()["s2t_pairs"] > 0
    A = f.evaluate(torch.tensor(J, device="cuda")).cpu().numpy()
    f.close()
    e = rel(A, g["A"] - g["A_free"])
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < tol


def test_tiny_full_field_direct_near_field(tiny):
    d, k, x, J, g = tiny
    A = run(d, k, x, J, p=12, react_s2t=2)
    e = rel(A, g["A"])
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < TINY_TOL[12]


def test_three_layer_100k_direct_near_field():
    n = 100000
    g = np.load(os.path.join(GOLD, "three_%d_sparse400_oracle.npz" % n))
    d, k, x, J = inputs.three_layer(n, seed=0)
    Js, keep = inputs.sparse_currents(J, 400, seed=0)
    print("case three-layer n=%d, direct near field chosen by the cost model" % n, flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20, react_s2t=1).build(x)
    npairs = f.stats()["s2t_pairs"]
    A = f.evaluate(torch.tensor(Js, device="cuda")).cpu().numpy()
    f.close()
    e = rel(A[g["idx"]], g["A"])
    print("  s2t pairs %d, rel L2 = %.3e" % (npairs, e), flush=True)
    assert npairs > 0 and e < 6e-6


def cuda(a):
    return torch.tensor(a, device="cuda")


@pytest.fixture(scope="module")
def largest():
    """Four-layer medium (interfaces 0, -1, -2.5; k = 1.0, 1.8, 2.4, 1.3),
    N = 2e6 points (half uniform, half in 20 Gaussian clusters), p = 16 (free
    part p = 20), built once for the forward and the adjoint test.  The M2L
    tile shape is fixed (variant 0, the one the autotuner keeps at the
    benchmark size; every variant gives bitwise the same result), so the
    first evaluation does not time each variant on 16 vectors at 2e6 points."""
    n, nr = 2000000, 16
    g = np.load(os.path.join(GOLD, "four_%d_rhs%d_sparse400_oracle.npz" % (n, nr)))
    d, k, x, J = inputs.four_layer(n, seed=0, n_rhs=nr)
    Js, keep = inputs.sparse_currents(J, 400, seed=0)
    del J
    assert np.array_equal(keep, g["keep"])
    print("case four-layer N=%d p=16 free p=20, %d right-hand sides" % (n, nr), flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=16, p_free=20, m2l_variant=0).build(x)
    print("  built: %s" % {a: f.stats()[a] for a in ("m2l_pairs_react", "m2l_pairs_free", "s2t_pairs")},
          flush=True)
    yield n, nr, g, f, Js
    f.close()


def test_four_layer_largest_sampled(largest):
    """16 current vectors in one evaluation at full size: sampled targets
    against the oracle (stored; 400 nonzero sources shared by the 16
    vectors).  The bound is the accuracy asked at p = 16 (relative L2 <=
    1e-6).  One column evaluated alone equals its column of the batch
    bitwise."""
    n, nr, g, f, Js = largest
    A = f.evaluate(cuda(Js))
    e = rel(A[:, g["idx"]].cpu().numpy(), g["A"])
    A3 = f.evaluate(cuda(Js[3])).cpu().numpy()
    same = np.array_equal(A3, A[3].cpu().numpy())
    del A
    print("  forward rel L2 = %.3e, column 3 alone bitwise equal: %s" % (e, same), flush=True)
    assert e < 1e-6 and same


def test_four_layer_largest_adjoint_sampled(largest):
    """The adjoint of the same 16-vector evaluation (400 nonzero output
    gradients shared by the vectors): sampled sources against the oracle
    (stored), relative L2 <= 1e-6."""
    n, nr, g, f, Js = largest
    gA = inputs.cotangent(n, n_rhs=nr, seed=0)
    gAs, keep_a = inputs.sparse_currents(gA, 400, seed=1)
    del gA
    assert np.array_equal(keep_a, g["keep_a"])
    gJ = f.evaluate_adjoint(cuda(gAs))
    ea = rel(gJ[:, g["idx_s"]].cpu().numpy(), g["gJ"])
    del gJ
    f.close()  # frees the device memory before the rest of the module
    print("  adjoint rel L2 = %.3e" % ea, flush=True)
    assert ea < 1e-6


def test_batched_rhs_200k_sampled():
    """Three-layer medium, N = 2e5, 64 current vectors on one tree in one call
    (M2L as a 64-column-per-pair contraction): 256 sampled targets against the
    oracle (stored; 400 nonzero sources shared by the 64 vectors) within the
    metric's 1e-6.  At this size the reaction order 12 leaves 1.48e-6 (the
    middle layer's reaction truncation, 4.9e-6 there); order 13 (free part
    20) gives 6.8e-7.  Single columns equal their batch column bitwise."""
    n, nr = 200000, 64
    g = np.load(os.path.join(GOLD, "three_%d_rhs%d_sparse400_oracle.npz" % (n, nr)))
    d, k, x, J = inputs.three_layer(n, seed=0, n_rhs=nr)
    Js, keep = inputs.sparse_currents(J, 400, seed=0)
    assert np.array_equal(keep, g["keep"])
    print("case three-layer N=%d p=13, %d right-hand sides" % (n, nr), flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=13, p_free=20).build(x)
    A = f.evaluate(cuda(Js)).cpu().numpy()
    e = rel(A[:, g["idx"]], g["A"])
    same = all(np.array_equal(A[r], f.evaluate(cuda(Js[r])).cpu().numpy()) for r in (0, 17, 63))
    f.close()
    print("  rel L2 = %.3e, single columns bitwise equal: %s" % (e, same), flush=True)
    assert e < 1e-6 and same


def test_direct_near_field_many_rhs(tiny):
    """The direct reaction near field evaluates its integrals once per pair
    for up to 4 right-hand sides: with 6 current vectors (groups of 4 and 2)
    every column equals its single-vector evaluation bitwise."""
    d, k, x, J, g = tiny
    rng = np.random.default_rng(12)
    Jm = rng.uniform(-1, 1, (6, 600, 3)) + 1j * rng.uniform(-1, 1, (6, 600, 3))
    f = lmfmm.LayeredDyadicFMM(d, k, p=8, react_s2t=2).build(x)
    assert f.stats()["s2t_pairs"] > 0
    Am = f.evaluate(cuda(Jm)).cpu().numpy()
    for r in range(6):
        assert np.array_equal(Am[r], f.evaluate(cuda(Jm[r])).cpu().numpy()), r
    f.close()


@pytest.mark.parametrize("p", [8, 12])
def test_coarse_trees_subset(tiny, p):
    """Every fifth point of the tiny workload (120 points): shallow trees, so
    the M2L tables of the coarse levels (large horizontal offsets on the
    contour piece Gamma_1) carry the reaction field."""
    from oracle import oracle
    d, k, x, J, g = tiny
    sel = np.arange(0, 600, 5)
    xs, Js = x[sel], J[sel]
    print("case tiny subset n=120 p=%d" % p, flush=True)
    A = run(d, k, xs, Js, p=p)
    ref = oracle.direct(d, k, xs, Js, xs)
    e = rel(A, ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < COARSE_TOL[p]


def test_all_reaction_pairs_direct_equals_oracle(tiny):
    """Every reaction pair through its component's Sommerfeld integral
    (react_s2t = 3: single-box reaction trees, no expansions): the paper's
    decomposition of the reaction field into components at images and
    effective locations (sigma_1..sigma_5 with the sigma_3 reading, the Z
    functions and signs) equals the oracle's undecomposed reaction field to
    the quadrature's accuracy, with no truncation of the method in between
    (recorded 8.2e-11 over all 600 targets)."""
    d, k, x, J, g = tiny
    print("case tiny, reaction part, every pair direct", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=8, components=2, react_s2t=3).build(x)
    st = f.stats()
    assert st["m2l_pairs_react"] == 0 and st["s2t_pairs"] == 600 * 600
    A = f.evaluate(torch.tensor(J, device="cuda")).cpu().numpy()
    f.close()
    e = rel(A, g["A"] - g["A_free"])
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < 2e-10


def test_all_reaction_pairs_direct_with_mu_equals_oracle():
    """The same on three layers with permeabilities, targets distinct from
    the sources (oracle computed live)."""
    from oracle import oracle
    d, k, src, J = inputs.three_layer(90, seed=21, half_width=1.0)
    _, _, tgt, _ = inputs.three_layer(60, seed=22, half_width=1.0)
    mu = [1.0, 1.8, 0.7]
    print("case three layers with mu, every reaction pair direct, 90 x 60", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, mu=mu, p=8, components=2, react_s2t=3).build(src, tgt)
    A = f.evaluate(torch.tensor(J, device="cuda")).cpu().numpy()
    f.close()
    full = oracle.direct(d, k, src, J, tgt, mu=mu)
    free = oracle.direct_free(d, k, src, J, tgt)
    e = rel(A, full - free)
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < 2e-10


def test_three_layer_dense_currents_sampled():
    """The scale workload (three layers, N = 1e5, p = 12, free part p = 20)
    with every current nonzero, as the benchmark evaluates it: 8 sampled
    targets against the oracle summing all 1e5 sources (stored; about 2
    minutes per target on 8 cores)."""
    n = 100000
    fn = os.path.join(GOLD, "three_%d_dense_oracle.npz" % n)
    g = np.load(fn)
    d, k, x, J = inputs.three_layer(n, seed=0)
    assert np.array_equal(g["idx"], inputs.sample_targets(n, g["idx"].size, seed=0))
    print("case three-layer n=%d dense currents p=12 p_free=20" % n, flush=True)
    A = run(d, k, x, J, p=12, p_free=20)
    e = rel(A[g["idx"]], g["A"])
    print("  rel L2 = %.3e" % e, flush=True)
    assert e < 1e-6
