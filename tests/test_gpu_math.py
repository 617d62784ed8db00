"""GPU unit test of the near-field arithmetic (through the C ABI): the
reduced-range sin/cos (Cody-Waite reduction by pi/2, Taylor polynomials) and
the refined reciprocal square root, against numpy's fp64 routines."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu


def test_near_field_sincos_and_rsqrt():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        np.linspace(-60.0, 60.0, 200001),
        rng.uniform(0, 8.0e5, 100000),
        np.arange(-64, 65) * (np.pi / 2),                    # near the reduction boundaries
        np.arange(-64, 65) * (np.pi / 2) + 1e-9,
        [0.0, 1e-300, 1e-10, -1e-10, 0.7853981633974483, 8.23548e5, 8.3e5, 1e7],
    ])
    out = lmfmm.selftest_math(torch.tensor(x, device="cuda")).cpu().numpy()
    es = np.abs(out[:, 0] - np.sin(x))
    ec = np.abs(out[:, 1] - np.cos(x))
    print("max |sin err| %.3e, max |cos err| %.3e" % (es.max(), ec.max()), flush=True)
    assert es.max() < 4e-16 and ec.max() < 4e-16
    a = x * x + 1e-300
    ref = 1.0 / np.sqrt(a)
    er = np.abs(out[:, 2] - ref) / ref
    print("max rsqrt rel err %.3e" % er.max(), flush=True)
    assert er.max() < 5e-16
