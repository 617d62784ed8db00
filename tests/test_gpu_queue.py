"""GPU tests of the persistent work-queue launches (near field, direct
reaction pairs): which block takes which work item varies from launch to
launch, but every item writes outputs of its own, so repeated evaluations
must agree bitwise; the queue counters are cleared by the last block of
each launch, so launches of different sizes may follow each other on one
stream (two contexts interleaved, one with targets distinct from the
sources, which takes the one-sided near-field kernel)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu


def test_repeated_evaluations_bitwise_equal_across_queue_orders():
    d, k, x, J = inputs.three_layer(100000, seed=11)
    print("case three-layer n=1e5 p=12 p_free=20, repeated evaluations", flush=True)
    f = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(x)
    st = f.stats()
    assert st["p2p_kernel_evals"] > 0 and st["s2t_pairs"] > 0
    Jt = torch.tensor(J, device="cuda")
    ref = f.evaluate(Jt).cpu().numpy()
    for it in range(3):
        assert np.array_equal(f.evaluate(Jt).cpu().numpy(), ref), it
    f.close()


def test_interleaved_contexts_share_a_stream():
    d, k, x, J = inputs.three_layer(30000, seed=12)
    y = x[::3] + np.array([0.017, -0.011, 0.0])
    y[:, 2] = np.where(np.abs(y[:, 2]) < 0.06, np.sign(y[:, 2]) * 0.08, y[:, 2])
    y[:, 2] = np.where(np.abs(y[:, 2] + 1.2) < 0.06, -1.2 + np.sign(y[:, 2] + 1.2) * 0.08, y[:, 2])
    print("case two contexts (targets = sources, distinct targets), interleaved", flush=True)
    fa = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(x)
    fb = lmfmm.LayeredDyadicFMM(d, k, p=12, p_free=20).build(x, y)
    Jt = torch.tensor(J, device="cuda")
    ra = fa.evaluate(Jt).cpu().numpy()
    rb = fb.evaluate(Jt).cpu().numpy()
    J2 = torch.stack([Jt, 2.0 * Jt])  # a launch twice the size on the same counters
    for it in range(2):
        Aa = fa.evaluate(Jt)
        Ab = fb.evaluate(Jt)
        A2 = fa.evaluate(J2).cpu().numpy()
        assert np.array_equal(Aa.cpu().numpy(), ra) and np.array_equal(Ab.cpu().numpy(), rb), it
        # a batch column equals its single-vector run; the doubled currents
        # give exactly twice the field (every operation is linear)
        assert np.array_equal(A2[0], ra) and np.array_equal(A2[1], 2.0 * ra), it
    fa.close()
    fb.close()
