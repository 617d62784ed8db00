"""GPU tests of media with more layers (six layers, 100 reaction components)
and of higher frequencies: the HIP path through the C ABI against the
oracle evaluated live."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu

# recorded relative L2 errors at p = 12 (free part p = 20), margin 3
TOL_SMALL = 1.3e-7
TOL_50K = 2.5e-6


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_six_layers_small():
    from oracle import oracle
    d, k, x, J = inputs.six_layer(240, seed=0)
    assert lmfmm.host_components(d, k).shape[0] == 100
    idx = inputs.sample_targets(x.shape[0], count=80, seed=0)
    print("case six layers n=240 p=12 p_free=20", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(x)
    A = f.evaluate(torch.tensor(J, device="cuda")).cpu().numpy()
    f.close()
    ref = oracle.direct(d, k, x, J, x[idx])
    e = rel(A[idx], ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < TOL_SMALL


def test_six_layers_50k_sampled():
    from oracle import oracle
    d, k, x, J = inputs.six_layer(50000, seed=1, half_width=3.0)
    Js, keep = inputs.sparse_currents(J, 300, seed=1)
    idx = inputs.sample_targets(x.shape[0], count=48, seed=1)
    print("case six layers n=50000 p=12 p_free=20 (sampled)", flush=True)
    t0 = time.time()
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(x)
    tb = time.time() - t0
    Jt = torch.tensor(Js, device="cuda")
    A = f.evaluate(Jt)
    torch.cuda.synchronize()
    t0 = time.time()
    A = f.evaluate(Jt)
    torch.cuda.synchronize()
    te = time.time() - t0
    st = f.stats()
    A = A.cpu().numpy()
    f.close()
    ref = oracle.direct(d, k, x[keep], Js[keep], x[idx])
    e = rel(A[idx], ref)
    print("  rel err %.2e, build %.2f s, evaluation %.1f ms, %d components, %d table cases" % (
        e, tb, 1e3 * te, st["n_react_inst"], st["n_cases"]), flush=True)
    assert e < TOL_50K


@pytest.mark.parametrize("scale,half_width,p,tol", [(3.0, 2.0, 12, 1.5e-6), (4.0, 1.5, 16, 1.9e-7)])
def test_higher_frequency_sampled(scale, half_width, p, tol):
    """The three-layer medium at 3x and 4x the wavenumbers (k_max 6 over a
    4-wide domain, k_max 8 over a 3-wide one: up to about four wavelengths
    across), 2e4 points, 200-source sparse currents, 48 sampled targets.
    Tolerances: recorded 4.8e-7 and 6.4e-8, margin 3."""
    from oracle import oracle
    d, k, x, J = inputs.three_layer(20000, seed=5, half_width=half_width)
    k = k * scale
    Js, keep = inputs.sparse_currents(J, 200, seed=5)
    idx = inputs.sample_targets(x.shape[0], count=48, seed=5)
    print("case higher frequency k x%.0f, n=20000, p=%d, p_free=20" % (scale, p), flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=p, p_free=20).build(x)
    A = f.evaluate(torch.tensor(Js, device="cuda")).cpu().numpy()
    f.close()
    ref = oracle.direct(d, k, x[keep], Js[keep], x[idx])
    e = rel(A[idx], ref)
    print("  rel err %.2e" % e, flush=True)
    assert e < tol
