"""GPU tests of the M2L GEMM tile-shape variants and their autotuner
(through the C ABI): every variant, fixed or chosen per launch by the
autotuner, gives bitwise the same result, for one and for several
right-hand sides; the autotuner reports a choice and a time for every
launch; out-of-range variants are rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu


def run(d, k, x, J, **kw):
    f = lmfmm.LayeredDyadicFMM(d, k, **kw).build(x)
    A = f.evaluate(torch.tensor(J, device="cuda")).cpu().numpy()
    return f, A


@pytest.mark.parametrize("case", ["tiny", "three_20k_3rhs"])
def test_variants_bitwise_equal(case):
    if case == "tiny":
        d, k, x, J = inputs.tiny()
        kw = dict(p=12)
    else:
        d, k, x, J = inputs.three_layer(20000, seed=4, n_rhs=3)
        kw = dict(p=12, p_free=16)
    print("case %s n %d rhs %d" % (case, x.shape[0], J.shape[0] if J.ndim == 3 else 1), flush=True)
    out = {}
    for v in range(lmfmm.M2L_VARIANTS):
        f, out[v] = run(d, k, x, J, m2l_variant=v, **kw)
        f.close()
    f, A = run(d, k, x, J, **kw)           # autotuned
    A2 = f.evaluate(torch.tensor(J, device="cuda")).cpu().numpy()
    n_rhs = J.shape[0] if J.ndim == 3 else 1
    var, ms = f.m2l_variants(n_rhs)
    f.close()
    print("  chosen variants %s" % var, flush=True)
    print("  ms per variant (sum over launches) %s" % np.round(ms.sum(axis=0), 3).tolist(), flush=True)
    for v in range(1, lmfmm.M2L_VARIANTS):
        assert np.array_equal(out[v], out[0]), v
    assert np.array_equal(A, out[0]) and np.array_equal(A2, out[0])
    assert len(var) > 0 and all(0 <= v < lmfmm.M2L_VARIANTS for v in var)
    assert (ms >= 0).all()
    for i, v in enumerate(var):
        assert ms[i, v] == ms[i].min()


def test_variant_out_of_range():
    d, k, x, J = inputs.tiny()
    for bad in (-2, lmfmm.M2L_VARIANTS):
        with pytest.raises(lmfmm.LMError, match="m2l_variant"):
            lmfmm.LayeredDyadicFMM(d, k, p=8, m2l_variant=bad)
