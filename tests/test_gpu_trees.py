"""GPU tests of the octrees keyed and sorted on the device (through the C
ABI): lm_build with the device sort (the default) and with the host sort
(lm_params.host_trees = 1) must give the same plan -- equal 64-bit plan
digests over the trees, interaction lists, M2L schedule, table cases and
nodes -- and bitwise equal evaluations, on uniform, clustered, six-layer,
many-geometry and distinct-target builds (paper Sec. 3.3: one octree per
free-space layer part and per reaction component; Morton order, with equal
keys in input order)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2507_18491_amd import inputs, lmfmm  # noqa: E402

pytestmark = pytest.mark.gpu


def cuda(a):
    return torch.tensor(a, device="cuda")


def digest(st):
    return (int(st["plan_digest_hi"]), int(st["plan_digest_lo"]))


def both(d, k, build, J, p=8, **kw):
    out = []
    for host in (0, 1):
        f = lmfmm.LayeredDyadicFMM(d, k, p=p, host_trees=host, **kw)
        build(f)
        st = f.stats()
        A = f.evaluate(cuda(J)).cpu().numpy()
        f.close()
        out.append((st, A))
    (sd, Ad), (sh, Ah) = out
    print("  records %d, device sort %.3f ms; digests %s %s" % (
        sd["tree_records"], sd["tree_sort_ms"], digest(sd), digest(sh)), flush=True)
    assert sd["tree_records"] > 0 and sd["tree_sort_ms"] > 0
    assert sh["tree_records"] == 0 and sh["tree_sort_ms"] == 0
    assert digest(sd) == digest(sh)
    assert np.array_equal(Ad, Ah)
    return sd


@pytest.mark.parametrize("n", [600, 20000])
def test_device_trees_three_layer(n):
    d, k, x, J = inputs.tiny() if n == 600 else inputs.three_layer(n, seed=3)
    print("case three-layer-style n=%d" % n, flush=True)
    both(d, k, lambda f: f.build(x), J)


def test_device_trees_clustered_and_six_layer():
    d, k, x, J = inputs.clustered_three_layer(30000, seed=5)
    print("case clustered 3e4", flush=True)
    both(d, k, lambda f: f.build(x), J)
    d, k, x, J = inputs.six_layer(12000, seed=2)
    print("case six layers 1.2e4", flush=True)
    both(d, k, lambda f: f.build(x), J)


def test_device_trees_many_geometries_and_distinct_targets():
    d, k, xs, Js = inputs.uneven_geometries(300, seed=4, n_min=50, n_max=600)
    print("case 300 geometries (more than 256 trees: two tree-id passes)", flush=True)
    st = both(d, k, lambda f: f.build_batch(xs), np.concatenate(Js), p=6)
    assert st["n_free_inst"] + 2 * st["n_react_inst"] > 256
    d, k, x, J = inputs.three_layer(8000, seed=6)
    y = x[::2] + np.array([0.013, -0.021, 0.0])
    y[:, 2] = np.where(np.abs(y[:, 2]) < 0.06, np.sign(y[:, 2]) * 0.08, y[:, 2])
    y[:, 2] = np.where(np.abs(y[:, 2] + 1.2) < 0.06, -1.2 + np.sign(y[:, 2] + 1.2) * 0.08, y[:, 2])
    print("case distinct targets", flush=True)
    both(d, k, lambda f: f.build(x, y), J)
