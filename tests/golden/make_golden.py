"""Writes the stored oracle outputs used by the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded synthetic workloads of
paper_2507_18491_amd.inputs (which draws points and currents and contains no
arithmetic of the method).  Usage: python tests/golden/make_golden.py [name...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2507_18491_amd import inputs  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def tiny():
    """Two-layer 600-point workload: every target, full field, plus the
    free-space part alone."""
    d, k, x, J = inputs.tiny(seed=0)
    A = oracle.direct(d, k, x, J, x)
    Af = oracle.direct_free(d, k, x, J, x)
    np.savez_compressed(os.path.join(OUT, "tiny_oracle.npz"), A=A, A_free=Af, seed=0)


def scale_sparse(n=100000, n_active=400, n_tgt=128):
    """Three-layer workload at n points with only n_active nonzero currents;
    oracle on n_tgt sampled targets (sampled outputs at full size)."""
    d, k, x, J = inputs.three_layer(n, seed=0)
    Js, keep = inputs.sparse_currents(J, n_active, seed=0)
    idx = inputs.sample_targets(n, n_tgt, seed=0)
    A = oracle.direct(d, k, x[keep], J[keep], x[idx])
    np.savez_compressed(os.path.join(OUT, "three_%d_sparse%d_oracle.npz" % (n, n_active)), A=A, idx=idx,
                        keep=keep, seed=0)


if __name__ == "__main__":
    names = sys.argv[1:] or ["tiny"]
    for nm in names:
        t = time.time()
        if nm == "tiny":
            tiny()
        elif nm.startswith("scale"):
            parts = nm.split(":")
            n = int(parts[1]) if len(parts) > 1 else 100000
            scale_sparse(n=n)
        print(nm, "done in %.1f s" % (time.time() - t), flush=True)
