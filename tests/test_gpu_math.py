"""GPU unit test of the near-field arithmetic (through the C ABI): the
reduced-range sin/cos (Cody-Waite reduction by pi/2, Taylor polynomials), the
refined reciprocal square root, against numpy's fp64 routines, and the
polynomial J0, J1 of the direct reaction near field against scipy's."""
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


def test_real_bessel_j0_j1():
    from scipy import special
    x = np.concatenate([
        np.linspace(0.0, 12.0, 120001),          # both sides of the switch at x = 6
        np.linspace(12.0, 400.0, 100001),
        np.geomspace(400.0, 2000.0, 2000),   # (beyond, rounding of x - pi/4 grows with x)
        [1e-300, 1e-12, 1e-3, 6.0 - 1e-12, 6.0, 6.0 + 1e-12],
    ])
    out = lmfmm.selftest_math(torch.tensor(x, device="cuda")).cpu().numpy()
    e0 = np.abs(out[:, 4] - special.j0(x))
    e1 = np.abs(out[:, 5] - special.j1(x))
    print("max |J0 err| %.3e, max |J1 err| %.3e" % (e0.max(), e1.max()), flush=True)
    # absolute bound from the generator's fit and the series' cancellation
    # near the switch (about 3e-15), plus scipy's own rounding
    assert e0.max() < 1e-14 and e1.max() < 1e-14
