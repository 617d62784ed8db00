"""GPU tests of many right-hand sides and many geometries (through the C
ABI): several independent geometries built into one plan give, for each
geometry, the result of its own separate build (one launch per pass for all
of them); an evaluation captured in a HIP graph replays to the eager result.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cuda(a):
    return torch.tensor(a, device="cuda")


def separate(d, k, xs, Js, p, tgts=None):
    outs = []
    for g, (x, J) in enumerate(zip(xs, Js)):
        y = None if tgts is None else tgts[g]
        if x.shape[0] == 0 or (y is not None and y.shape[0] == 0):
            outs.append(np.zeros(((x if y is None else y).shape[0], 3), dtype=complex))
            continue
        f = lmfmm.LayeredDyadicFMM(d, k, p=p).build(x, y)
        outs.append(f.evaluate(cuda(J)).cpu().numpy())
        f.close()
    return outs


def test_batch_geometries_equal_separate_builds():
    d, k, xs, Js = inputs.uneven_geometries(6, seed=0, n_min=200, n_max=4000)
    print("case 6 geometries, sizes %s" % [x.shape[0] for x in xs], flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=8).build_batch(xs)
    A = f.evaluate(cuda(np.concatenate(Js))).cpu().numpy()
    f.close()
    ref = separate(d, k, xs, Js, 8)
    so = np.cumsum([0] + [x.shape[0] for x in xs])
    for g in range(len(xs)):
        e = rel(A[so[g]:so[g + 1]], ref[g])
        print("  geometry %d: rel diff %.3e" % (g, e), flush=True)
        assert e < 1e-12


def test_batch_distinct_targets_empty_geometry_and_adjoint():
    d, k, xs, Js = inputs.uneven_geometries(3, seed=1, n_min=300, n_max=1500)
    ys = [x[::3] + np.array([0.01, -0.02, 0.0]) for x in xs]
    for y in ys:
        y[:, 2] = np.where(np.abs(y[:, 2]) < 0.06, np.sign(y[:, 2]) * 0.08, y[:, 2])
        y[:, 2] = np.where(np.abs(y[:, 2] + 1.2) < 0.06, -1.2 + np.sign(y[:, 2] + 1.2) * 0.08, y[:, 2])
    xs.insert(1, np.zeros((0, 3)))
    Js.insert(1, np.zeros((0, 3), dtype=complex))
    ys.insert(1, np.zeros((0, 3)))
    print("case 4 geometries (one empty), distinct targets", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=8).build_batch(xs, ys)
    A = f.evaluate(cuda(np.concatenate(Js))).cpu().numpy()
    G = inputs.cotangent(sum(y.shape[0] for y in ys), seed=4)
    gJ = f.evaluate_adjoint(cuda(G)).cpu().numpy()
    f.close()
    ref = separate(d, k, xs, Js, 8, ys)
    to = np.cumsum([0] + [y.shape[0] for y in ys])
    so = np.cumsum([0] + [x.shape[0] for x in xs])
    for g in range(len(xs)):
        if ys[g].shape[0] == 0:
            continue
        assert rel(A[to[g]:to[g + 1]], ref[g]) < 1e-12
        fg = lmfmm.LayeredDyadicFMM(d, k, p=8).build(xs[g], ys[g])
        one = fg.evaluate_adjoint(cuda(G[to[g]:to[g + 1]])).cpu().numpy()
        fg.close()
        e = rel(gJ[so[g]:so[g + 1]], one)
        print("  geometry %d adjoint rel diff %.3e" % (g, e), flush=True)
        assert e < 1e-12


def test_graph_capture_replays_eager_result():
    """An evaluation captured in a HIP graph (after one eager call sized the
    work buffers) replays, several times with eager work in between, to the
    eager result bitwise."""
    d, k, x, J = inputs.tiny(seed=0)
    f = lmfmm.LayeredDyadicFMM(d, k, p=8).build(x)
    Jt = cuda(J).reshape(1, -1, 3)
    out = torch.empty((1, x.shape[0], 3), dtype=torch.complex128, device="cuda")
    ref = f.evaluate(Jt, out=out).clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        f.evaluate(Jt, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    out.zero_()
    with torch.cuda.graph(g):
        f.evaluate(Jt, out=out)
    for it in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), "replay %d differs" % it
        other = f.evaluate(cuda(J[::-1].copy()).reshape(1, -1, 3))   # eager work between replays
        torch.cuda.synchronize()
        del other
    # a new current vector copied into the captured input buffer
    J2 = inputs.cotangent(x.shape[0], seed=8)
    Jt.copy_(cuda(J2).reshape(1, -1, 3))
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, f.evaluate(cuda(J2)).reshape(1, -1, 3))
    f.close()


@pytest.mark.slow
def test_uneven_geometries_full_size():
    """32 clustered geometries of 5e3 .. 2e5 points in one plan: every
    geometry equals its separate build (p = 12, free part p = 20)."""
    d, k, xs, Js = inputs.uneven_geometries(32, seed=0)
    print("case 32 uneven geometries, %d points" % sum(x.shape[0] for x in xs), flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build_batch(xs)
    A = f.evaluate(cuda(np.concatenate(Js))).cpu().numpy()
    f.close()
    so = np.cumsum([0] + [x.shape[0] for x in xs])
    worst = 0.0
    for g in range(len(xs)):
        fg = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(xs[g])
        one = fg.evaluate(cuda(Js[g])).cpu().numpy()
        fg.close()
        worst = max(worst, rel(A[so[g]:so[g + 1]], one))
    print("  worst per-geometry rel diff %.3e" % worst, flush=True)
    assert worst < 1e-12


def test_uneven_geometries_against_oracle():
    """The 32 uneven clustered geometries (5e3 .. 2e5 points each, 1.34e6
    in all) in one plan, as the benchmark replays them: per geometry 200
    nonzero currents and 8 sampled targets against the oracle (stored), at
    p = 12 (free part 20); every geometry within the metric's 1e-6."""
    import os
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                             "uneven_32_sparse200_oracle.npz"))
    d, k, xs, Js = inputs.uneven_geometries(32, seed=0)
    Jsp = []
    for gi, J in enumerate(Js):
        Jg, keep = inputs.sparse_currents(J, 200, seed=gi)
        assert np.array_equal(keep, g["keep%d" % gi])
        Jsp.append(Jg)
    print("case 32 uneven geometries against the oracle, p=12 p_free=20", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build_batch(xs)
    A = f.evaluate(cuda(np.concatenate(Jsp))).cpu().numpy()
    so = f.src_off
    f.close()
    num = den = 0.0
    worst = 0.0
    for gi in range(32):
        Ag = A[so[gi]:so[gi + 1]][g["idx%d" % gi]]
        ref = g["A%d" % gi]
        eg = rel(Ag, ref)
        worst = max(worst, eg)
        num += np.linalg.norm(Ag - ref) ** 2
        den += np.linalg.norm(ref) ** 2
    e = np.sqrt(num / den)
    print("  rel L2 over the 256 targets %.3e, worst geometry %.3e" % (e, worst), flush=True)
    assert e < 1e-6 and worst < 1e-6
