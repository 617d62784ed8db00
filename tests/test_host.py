"""CPU tests of the library's host logic and of its C ABI (no GPU calls).

Covers: the shared library loads and exports every function declared in
include/lmfmm.h; the reaction-component enumeration (paper Sec. 3.1); the
Chebyshev identities of Appendices A and B; the planner (trees, lists,
refinement next to interfaces) and its error paths; the iterative solve's
host logic on dense host systems; loud failure without the built library or
without a device.
"""
import math
import os
import re

import numpy as np
import pytest
import scipy.special as sp

from paper_2507_18491_amd import inputs, lmfmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "lmfmm.h")).read()
    names = set(re.findall(r"^(?:int|const char\*)\s+(lm_\w+)\s*\(", header, flags=re.M))
    assert len(names) >= 12
    lib = lmfmm.load_library()
    for nm in sorted(names):
        assert hasattr(lib, nm), nm


@pytest.mark.parametrize("n_layers,count", [(1, 0), (2, 4), (3, 16), (4, 36), (5, 64)])
def test_component_counts(n_layers, count):
    d = -np.arange(n_layers - 1, dtype=float)
    k = np.linspace(1.0, 2.0, n_layers)
    c = lmfmm.host_components(d, k)
    assert c.shape[0] == count
    if n_layers >= 2:
        # every valid (target layer, source layer) pair is present, and only
        # directions with an interface on the corresponding side
        L = n_layers - 1
        for lt, ls, ut, us, sgn, at, as_, _ in c:
            assert (ut and lt <= L - 1) or (not ut and lt >= 1)
            assert (us and ls >= 1) or (not us and ls <= L - 1)
            assert sgn in (1, -1) and at in (1, -1) and as_ in (1, -1)


def test_three_layer_components_per_target_layer():
    """Components per target layer (4, 8, 4): the middle layer carries twice
    the reaction components of the outer ones, the 2:1 ratio of the
    paper's three-layer timings (Sec. 4 table)."""
    c = lmfmm.host_components([0.0, -1.5], [2.19, 1.79, 2.28])
    per = [int((c[:, 0] == l).sum()) for l in range(3)]
    assert per == [4, 8, 4]


def test_component_signs_and_images_follow_the_paper():
    """Same-layer reflection at the lower interface (target up, source down):
    s = +1, image reflected, effective location identity (Sec. 3.1)."""
    c = lmfmm.host_components([0.0], [1.0, 1.5])
    row = [r for r in c if r[0] == 0 and r[1] == 0][0]
    assert row[2] == 1 and row[3] == 0 and row[4] == 1 and row[5] == 1 and row[6] == -1
    # transmission from layer 1 up to layer 0 (target above source): no
    # reflection on either side and s = +1 (target layer index < source's)
    row = [r for r in c if r[0] == 0 and r[1] == 1][0]
    assert row[2] == 1 and row[3] == 1 and row[4] == 1 and row[5] == 1 and row[6] == 1
    # the reverse transmission (target below source, both waves going down): s = -1
    row = [r for r in c if r[0] == 1 and r[1] == 0][0]
    assert row[2] == 0 and row[3] == 0 and row[4] == -1 and row[5] == 1 and row[6] == 1


@pytest.mark.parametrize("a,b", [(0.49, 0.51), (0.36, 0.64), (1.0, 0.0), (0.8, 0.2)])
def test_appendix_a_affine_chebyshev(a, b):
    """T_j(a x + b) = sum_s C_js T_s(x) (Appendix A) against the closed form
    T_j(y) = cos(j arccos y) on [-1, 1]."""
    jmax = 18
    C = lmfmm.host_cheb_affine(jmax, a, b)
    x = np.linspace(-1, 1, 41)
    Ts = np.array([np.cos(s * np.arccos(x)) for s in range(jmax + 1)])
    y = np.clip(a * x + b, -1, 1)
    for j in range(jmax + 1):
        assert np.abs(C[j] @ Ts - np.cos(j * np.arccos(y))).max() < 5e-13
    # the paper's low-order values: C_10 = b, C_21 = 4ab
    assert abs(C[1, 0] - b) < 1e-15 and abs(C[2, 1] - 4 * a * b) < 1e-15


def test_appendix_b_legendre_chebyshev():
    """P^m_n(cos t) = tau_nm(t) sum_k B^k T_k(cos 2t) (Appendix B) against
    scipy's orthonormal spherical harmonics, for all n, m <= 16."""
    p = 16
    B = lmfmm.host_legendre_cheb(p)
    t = np.linspace(0.05, 1.5, 23)
    for n in range(p + 1):
        for m in range(n + 1):
            ref = np.real(sp.sph_harm_y(n, m, t, 0.0))
            if n % 2 == 0 and m % 2 == 0:
                tau = np.ones_like(t)
            elif n % 2 == 1 and m % 2 == 0:
                tau = 1 / np.cos(t)
            elif n % 2 == 1:
                tau = np.sin(t)
            else:
                tau = np.tan(t)
            K = n // 2 if n % 2 == 0 else ((n + 1) // 2 if m % 2 == 0 else (n - 1) // 2)
            row = B[n * (n + 1) // 2 + m]
            assert np.all(np.abs(row[K + 1:]) < 1e-14)
            val = tau * sum(row[kk] * np.cos(2 * kk * t) for kk in range(K + 1))
            assert np.abs(val - ref).max() < 5e-13 * max(1, np.abs(ref).max())


def test_appendix_b_top_coefficient():
    """Even n >= 2, even m: the leading coefficient B^{n/2}_{nm} equals the
    closed form of Appendix B, (-1)^{m/2} Gamma(n+1/2)/pi sqrt((2n+1)/((n-m)!(n+m)!))
    (the appendix's n = 0 value is twice the orthonormal one, so n = 0 is
    excluded here)."""
    p = 16
    B = lmfmm.host_legendre_cheb(p)
    for n in range(2, p + 1, 2):
        for m in range(0, n + 1, 2):
            ref = (-1) ** (m // 2) * math.gamma(n + 0.5) / math.pi * math.sqrt(
                (2 * n + 1) / (math.factorial(n - m) * math.factorial(n + m)))
            got = B[n * (n + 1) // 2 + m][n // 2]
            assert abs(got - ref) < 1e-13 * max(1, abs(ref)), (n, m, got, ref)


def test_plan_tiny_config():
    d, k, x, _ = inputs.tiny()
    s = lmfmm.host_plan_stats(d, k, x, p=8)
    assert s["n_free_inst"] == 2 and s["n_react_inst"] == 4
    assert s["free_depth"] == 2           # the tiny workload's octree depth
    assert s["m2l_pairs_react"] > 0 and s["n_cases"] > 0 and s["p2p_pairs"] > 0
    # near field covers at least every same-box pair
    assert s["p2p_pairs"] >= 600


def test_plan_three_layer_small():
    d, k, x, _ = inputs.three_layer(20000)
    s = lmfmm.host_plan_stats(d, k, x, p=12)
    assert s["n_free_inst"] == 3 and s["n_react_inst"] == 16
    # every reaction interaction is an M2L (boxes next to the interfaces are
    # refined until no adjacent source/target boxes remain): planning succeeds
    assert s["m2l_pairs_react"] > 0


def test_plan_external_tree_sort_route_gives_the_same_plan():
    """The route lm_build takes (octree records keyed and sorted outside the
    planner, all trees in one call; on the device there) gives the plan of
    the planner's own sort: a plain host implementation of that route's
    contract (bit-by-bit Morton keys, a stable sort per tree) against the
    planner's radix sort, by 64-bit plan digests, on one and on several
    geometries, with targets distinct from the sources, and with every
    reaction pair direct (single-box reaction trees)."""
    d, k, x, _ = inputs.tiny()
    a, b = lmfmm.host_plan_digests(d, k, [x], p=8)
    assert a == b
    d, k, x, _ = inputs.three_layer(20000, seed=1)
    a, b = lmfmm.host_plan_digests(d, k, [x], p=12)
    assert a == b
    d, k, xs, _ = inputs.uneven_geometries(5, seed=2, n_min=100, n_max=3000)
    ys = [xx[::2] + np.array([0.011, -0.017, 0.0]) for xx in xs]
    for y in ys:
        y[:, 2] = np.where(np.abs(y[:, 2]) < 0.06, np.sign(y[:, 2]) * 0.08, y[:, 2])
        y[:, 2] = np.where(np.abs(y[:, 2] + 1.2) < 0.06, -1.2 + np.sign(y[:, 2] + 1.2) * 0.08, y[:, 2])
    a, b = lmfmm.host_plan_digests(d, k, xs, ys, p=8)
    assert a == b
    a2, b2 = lmfmm.host_plan_digests(d, k, xs, ys, p=8, react_s2t=3)
    assert a2 == b2 and a2 != a
    # the digest sees a change of one tree: a point moved by one lattice cell
    xs2 = [xx.copy() for xx in xs]
    xs2[0][0, 0] += 0.37
    a3, b3 = lmfmm.host_plan_digests(d, k, xs2, ys, p=8)
    assert a3 == b3 and a3 != a


def test_plan_does_not_depend_on_the_host_thread_count(monkeypatch):
    """The planner's threaded steps (instance trees and lists, box records,
    the M2L pair list and its class keys, class tables, work blocks) write
    ranges sized beforehand and keep every first-use numbering serial, so
    one thread and several give the same plan: equal digests with
    LMFMM_HOST_THREADS = 1, 3 and 8 on clustered points, uneven geometries
    with distinct targets, and six layers."""
    cases = []
    d, k, x, _ = inputs.clustered_three_layer(30000, seed=7)
    cases.append((d, k, [x], None, dict(p=12, p_free=16)))
    d, k, xs, _ = inputs.uneven_geometries(12, seed=8, n_min=200, n_max=4000)
    ys = [xx[::3] + np.array([0.013, -0.019, 0.0]) for xx in xs]
    for y in ys:
        y[:, 2] = np.where(np.abs(y[:, 2]) < 0.06, np.sign(y[:, 2]) * 0.08, y[:, 2])
        y[:, 2] = np.where(np.abs(y[:, 2] + 1.2) < 0.06, -1.2 + np.sign(y[:, 2] + 1.2) * 0.08, y[:, 2])
    cases.append((d, k, xs, ys, dict(p=8)))
    d, k, x, _ = inputs.six_layer(8000, seed=9)
    cases.append((d, k, [x], None, dict(p=10)))
    for d, k, srcs, tgts, prm in cases:
        got = []
        for nth in ("1", "3", "8"):
            monkeypatch.setenv("LMFMM_HOST_THREADS", nth)
            got.append(lmfmm.host_plan_digests(d, k, srcs, tgts, **prm))
        assert got[0][0] == got[0][1]
        assert got[0] == got[1] == got[2], got


def test_plan_rejects_point_on_interface():
    d, k, x, _ = inputs.tiny()
    x = x.copy()
    x[3, 2] = 0.0
    with pytest.raises(lmfmm.LMError):
        lmfmm.host_plan_stats(d, k, x, p=8)


def test_plan_rejects_points_too_close_to_interface():
    d, k, x, _ = inputs.tiny()
    x = x.copy()
    x[3, 2] = 1e-7
    x[400, 2] = -1e-7
    with pytest.raises(lmfmm.LMError, match="too close"):
        lmfmm.host_plan_stats(d, k, x, p=8, max_depth=10)


@pytest.mark.parametrize("d,k", [([0.0, 0.5], [1, 2, 3]), ([0.0], [1.0, -1.0]), ([0.0], [1.0, float("nan")])])
def test_plan_rejects_bad_medium(d, k):
    x = np.array([[0.0, 0.0, 0.5], [0.1, 0.0, -0.5]])
    with pytest.raises(lmfmm.LMError):
        lmfmm.host_plan_stats(d, k, x, p=4)


def test_plan_rejects_bad_order():
    x = np.array([[0.0, 0.0, 0.5], [0.1, 0.0, -0.5]])
    with pytest.raises(lmfmm.LMError):
        lmfmm.host_plan_stats([0.0], [1.0, 1.5], x, p=21)


def test_plan_adaptive_orders_reduce_work():
    """Per-offset orders never exceed p: the adaptive plan does no more M2L
    work than the uniform one, and a larger margin never does less."""
    d, k, x, _ = inputs.three_layer(20000)
    s0 = lmfmm.host_plan_stats(d, k, x, p=12, m2l_adapt=0)
    s2 = lmfmm.host_plan_stats(d, k, x, p=12, m2l_adapt=1, m2l_margin=2.0)
    s3 = lmfmm.host_plan_stats(d, k, x, p=12, m2l_adapt=1, m2l_margin=3.0)
    s30 = lmfmm.host_plan_stats(d, k, x, p=12, m2l_adapt=1, m2l_margin=30.0)
    assert s2["m2l_cmac_useful"] <= s3["m2l_cmac_useful"] <= s0["m2l_cmac_useful"]
    assert s3["m2l_cmac_useful"] < s0["m2l_cmac_useful"]
    assert s30["m2l_cmac_useful"] == s0["m2l_cmac_useful"]
    assert s3["m2l_pairs_free"] == s0["m2l_pairs_free"] and s3["m2l_pairs_react"] == s0["m2l_pairs_react"]


@pytest.mark.parametrize("kw", [{"m2l_adapt": 2}, {"m2l_margin": -1.0}, {"m2l_margin": float("nan")}])
def test_plan_rejects_bad_adaptive_params(kw):
    d, k, x, _ = inputs.tiny()
    with pytest.raises(lmfmm.LMError):
        lmfmm.host_plan_stats(d, k, x, p=8, **kw)


def test_real_bessel_coefficient_table():
    """The committed J0/J1 coefficient header (polynomial forms used on the
    real tail of the direct reaction near field), evaluated on the host with
    the kernel's steps, against scipy's J0 and J1."""
    import re
    import sys
    from scipy import special
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2507_18491_amd", "csrc")
    sys.path.insert(0, csrc)
    try:
        import gen_bessel_pq as g
    finally:
        sys.path.pop(0)
    h = open(os.path.join(csrc, "bessel_pq.h")).read()
    assert int(re.search(r"#define LM_BPQ_NSER (\d+)", h).group(1)) == g.NSER
    assert int(re.search(r"#define LM_BPQ_DEG (\d+)", h).group(1)) == g.DEG
    assert int(re.search(r"#define LM_BPQ_NSERC (\d+)", h).group(1)) == g.NSERC
    c = [float(v) for v in re.findall(r"^\s+([-0-9.e+]+),", h, re.M)]
    assert len(c) == g.NSERC + 2 * (g.DEG + 1)
    cs, cp, cq = c[:g.NSER], c[g.NSERC:g.NSERC + g.DEG + 1], c[g.NSERC + g.DEG + 1:]
    x = np.concatenate([np.linspace(0.0, 12.0, 2401), np.linspace(12.0, 400.0, 2001), [1e-12, 6.0 - 1e-12, 6.0]])
    j = np.array([g.j01(cs, cp, cq, float(v)) for v in x])
    assert np.abs(j[:, 0] - special.j0(x)).max() < 1e-14
    assert np.abs(j[:, 1] - special.j1(x)).max() < 1e-14

    # the complex series of the Gamma_1 nodes: J0 = S(w), J1 = -(z/2) S'(w),
    # J2 = w S''(w), w = z^2/4, with the term count the library picks for
    # the largest |z| of a component
    rng = np.random.default_rng(3)
    for zmax in (0.3, 1.5, 4.0, 7.5):
        n, term, zh = 1, 1.0, 0.5 * zmax
        while n < g.NSERC:
            term *= zh * zh / (n * n)
            if term < 1e-19:
                break
            n += 1
        z = zmax * np.sqrt(rng.uniform(0, 1, 200)) * np.exp(1j * rng.uniform(0, 2 * np.pi, 200))
        z = np.concatenate([z, [0.0, zmax, 1j * zmax]])
        w = 0.25 * z * z
        v = np.full_like(z, c[n - 1]); d1 = np.zeros_like(z); d2 = np.zeros_like(z)
        for kk in range(n - 2, -1, -1):
            d2 = d2 * w + d1
            d1 = d1 * w + v
            v = v * w + c[kk]
        scale = np.exp(np.abs(z.imag))
        for val, order in ((v, 0), (-0.5 * z * d1, 1), (2.0 * w * d2, 2)):
            assert (np.abs(val - sp.jv(order, z)) / scale).max() < 2e-14, (zmax, order)


# ---------------------------------------------------------------- GMRES host logic
def _rand_system(n, seed, shift=4.0):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    A += shift * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_gmres_host_logic_solves_with_restarts():
    A, b = _rand_system(60, 1)
    x, it, rr = lmfmm.host_gmres_dense(A, b, tol=1e-12, restart=8, max_iter=500)
    ref = np.linalg.solve(A, b)
    assert rr <= 1e-12
    assert it > 8  # several restart cycles
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.linalg.norm(b - A @ x) <= 1.01e-12 * np.linalg.norm(b)


def test_gmres_minimal_residual_over_the_krylov_space():
    """One cycle of m steps from x0 = 0 returns the minimiser of |b - A x|
    over the Krylov space span{b, Ab, ..., A^{m-1} b} (the defining property
    of GMRES), here computed by a least-squares solve on an explicit basis."""
    A, b = _rand_system(40, 2, shift=1.5)
    for m in (1, 3, 7, 12):
        x, it, rr = lmfmm.host_gmres_dense(A, b, tol=1e-15, restart=m, max_iter=m)
        assert it == m
        K = np.empty((40, m), dtype=complex)
        v = b.copy()
        for j in range(m):
            K[:, j] = v
            v = A @ v
        Q, _ = np.linalg.qr(K)
        y = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
        rmin = np.linalg.norm(b - A @ (Q @ y)) / np.linalg.norm(b)
        assert abs(rr - rmin) <= 1e-9 * max(rmin, 1e-12) + 1e-13, (m, rr, rmin)
        assert np.abs(x - Q @ y).max() <= 1e-9 * np.abs(Q @ y).max()


def test_gmres_finite_termination_and_breakdown():
    # a full cycle solves an order-n system in at most n steps (up to rounding)
    A, b = _rand_system(12, 3, shift=0.3)
    x, it, rr = lmfmm.host_gmres_dense(A, b, tol=1e-11, restart=12, max_iter=40)
    assert rr <= 1e-11 and it <= 14
    # invariant Krylov space at the first step: A = c I
    c = 2.0 - 0.5j
    x, it, rr = lmfmm.host_gmres_dense(c * np.eye(9), b[:9], tol=1e-13, restart=5)
    assert it == 1 and rr <= 1e-13
    assert np.abs(x - b[:9] / c).max() <= 1e-14 * np.abs(b).max()


def test_gmres_zero_rhs_and_iteration_cap():
    A, b = _rand_system(20, 4, shift=0.2)
    x, it, rr = lmfmm.host_gmres_dense(A, np.zeros(20), x0=np.ones(20), tol=1e-8)
    assert it == 0 and rr == 0.0 and not np.any(x)
    x, it, rr = lmfmm.host_gmres_dense(A, b, tol=1e-14, restart=3, max_iter=5)
    assert it == 5 and rr > 1e-14
    assert rr == pytest.approx(np.linalg.norm(b - A @ x) / np.linalg.norm(b), rel=1e-9)


def test_gmres_rejects_bad_arguments():
    A, b = _rand_system(5, 5)
    for kw in (dict(restart=0), dict(restart=65), dict(max_iter=0), dict(tol=0.0), dict(tol=float("inf")),
               dict(tol=float("nan"))):
        with pytest.raises(lmfmm.LMError):
            lmfmm.host_gmres_dense(A, b, **kw)


def test_gmres_lockstep_columns_match_single_solves():
    """Several right-hand sides in lockstep: each column converges on its own
    step count (a zero column at once, an eigenvector column in one step, a
    generic column later), stops updating once converged, and agrees with its
    single-column solve."""
    n = 30
    A, b = _rand_system(n, 6, shift=2.5)
    lam, V = np.linalg.eig(A)
    cols = [b, np.zeros(n, dtype=complex), V[:, 0] * (1.5 - 0.5j), _rand_system(n, 7)[1]]
    B = np.stack(cols)
    tol = 1e-11
    X, it, rr = lmfmm.host_gmres_dense(A, B, tol=tol, restart=7, max_iter=400)
    assert rr.shape == (4,) and np.all(rr <= tol)
    assert rr[1] == 0.0 and not np.any(X[1])
    Ainv = np.linalg.norm(np.linalg.inv(A), 2)
    for r in (0, 2, 3):
        xs, its, rrs = lmfmm.host_gmres_dense(A, cols[r], tol=tol, restart=7, max_iter=400)
        assert its <= it
        assert np.linalg.norm(B[r] - A @ X[r]) <= 1.01 * tol * np.linalg.norm(B[r])
        lim = 2.2 * Ainv * tol * np.linalg.norm(B[r])
        assert np.linalg.norm(X[r] - xs) <= lim
    # the eigenvector column: one Arnoldi step solves it exactly
    xe, ite, _ = lmfmm.host_gmres_dense(A, cols[2], tol=tol, restart=7)
    assert ite == 1
    assert np.abs(X[2] - cols[2] / lam[0]).max() <= 1e-10 * np.abs(cols[2] / lam[0]).max()


def test_gmres_lockstep_iteration_cap_per_column():
    A, b = _rand_system(25, 8, shift=0.1)
    B = np.stack([b, 2.0 * b])
    X, it, rr = lmfmm.host_gmres_dense(A, B, tol=1e-14, restart=4, max_iter=6)
    assert it == 6 and np.all(rr > 1e-14)
    # the problem is linear: the second column is twice the first throughout
    assert np.abs(X[1] - 2.0 * X[0]).max() <= 1e-12 * np.abs(X[1]).max()
    assert rr[1] == pytest.approx(rr[0], rel=1e-10)
    for r in range(2):
        assert rr[r] == pytest.approx(np.linalg.norm(B[r] - A @ X[r]) / np.linalg.norm(B[r]), rel=1e-9)


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library every entry point raises: there is no
    fallback path."""
    monkeypatch.setattr(lmfmm, "_lib", None)
    monkeypatch.setattr(lmfmm, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "liblmfmm.so"))
    with pytest.raises(RuntimeError, match="not built"):
        lmfmm.load_library()
    with pytest.raises(RuntimeError, match="not built"):
        lmfmm.LayeredDyadicFMM([0.0], [1.0, 1.5])


def test_no_device_fails_loudly():
    """On a machine without a GPU, creating a context raises (the library
    computes nothing on the host)."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(lmfmm.LMError, match="lm_create"):
        lmfmm.LayeredDyadicFMM([0.0], [1.0, 1.5])


def test_requested_accuracy_out_of_reach_is_lm_eaccuracy():
    """lm_params.tol checks the plan's quadrature rules: a tolerance the
    direct reaction pairs' integrals cannot reach (their tail cut at 28
    e-folds) or a table tail cut coarser than tol fails with LM_EACCURACY;
    tolerances within reach, or no tolerance, plan normally."""
    d, k, x, J = inputs.tiny()
    # every reaction pair direct: their integrals reach about 2.5e-9
    lmfmm.host_plan_stats(d, k, x, p=8, react_s2t=3, tol=1e-6)
    with pytest.raises(lmfmm.LMError) as e:
        lmfmm.host_plan_stats(d, k, x, p=8, react_s2t=3, tol=1e-10)
    assert e.value.code == lmfmm.LM_EACCURACY and "direct reaction pairs" in str(e.value)
    # no direct pairs: the same tolerance is within reach of the tables
    lmfmm.host_plan_stats(d, k, x, p=8, react_s2t=0, tol=1e-10)
    with pytest.raises(lmfmm.LMError) as e:
        lmfmm.host_plan_stats(d, k, x, p=8, react_s2t=0, tail_digits=10.0, tol=1e-6)
    assert e.value.code == lmfmm.LM_EACCURACY and "tail" in str(e.value)
    with pytest.raises(lmfmm.LMError) as e:
        lmfmm.host_plan_stats(d, k, x, p=8, react_s2t=0, gamma1_panels=2, tol=1e-10)
    assert e.value.code == lmfmm.LM_EACCURACY
    with pytest.raises(lmfmm.LMError):
        lmfmm.host_plan_stats(d, k, x, p=8, tol=-1.0)
