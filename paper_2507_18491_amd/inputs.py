"""Seeded synthetic workloads (positions, currents) for tests and benchmarks.

This module holds no arithmetic of the method: it only draws points and
current vectors (and, for the coupled-dipole solve, the diagonal of the
system, a material input).  Both the GPU path's tests and the oracle's tests take their
inputs from here.

Workloads follow the paper's numerical-test setup (Sec. 4: uniformly
distributed particles in each layer, real wavenumbers) at the sizes of the
benchmark configurations:

* ``tiny``     2 layers, interface z=0, k=(1.0, 1.5); 300 points uniform in
               [-1,1]^2 x [0.1,2.1] and 300 in [-1,1]^2 x [-2.1,-0.1].
* ``three``    3 layers, interfaces z=0, -1.2, k=(1.2, 2.0, 1.5); N points
               uniform in [-4,4]^2 per layer slab, split 40/30/30 %, at least
               0.05 from every interface.  The half-space slabs are 1.2 thick
               beyond the 0.05 margin: [0.05,1.25] and [-2.45,-1.25]; the
               middle slab is [-1.15,-0.05].
* ``four``     4 layers, interfaces z=0, -1, -2.5, k=(1.0, 1.8, 2.4, 1.3);
               half the points uniform (25 % per layer), half in 20 Gaussian
               blobs (sigma 0.3, 5 per layer).
* ``clustered`` the three-layer medium with Gaussian blobs (sigma 0.3).
* ``six_layer`` 6 layers, interfaces z=0, -0.8, -1.5, -2.4, -3.0,
               k=(1.0, 1.6, 2.2, 1.3, 1.9, 1.1); N points uniform in
               [-w,w]^2 x each layer's slab, equal shares.
* ``near_interface`` the three-layer medium with a third of the points in
               thin sheets between m and 2m from each interface, both
               sides (m = 0.02 and 0.005 in the tests: the slow-decay regime
               of the Sommerfeld tail).
* ``dipole_lattice`` the three-layer medium filled with a jittered cubic
               lattice of small dielectric spheres: the coupled-dipole system
               (diag - G) X = B of the iterative solve.

Currents are complex128 3-vectors with real and imaginary parts U[-1,1].
"""
import numpy as np

MEDIA = {
    "two": dict(d=[0.0], k=[1.0, 1.5]),
    "three": dict(d=[0.0, -1.2], k=[1.2, 2.0, 1.5]),
    "four": dict(d=[0.0, -1.0, -2.5], k=[1.0, 1.8, 2.4, 1.3]),
    "six": dict(d=[0.0, -0.8, -1.5, -2.4, -3.0], k=[1.0, 1.6, 2.2, 1.3, 1.9, 1.1]),
}

MARGIN = 0.05
HALFSPACE_THICKNESS = 1.2


def layer_slabs(d, margin=MARGIN, thick=HALFSPACE_THICKNESS):
    """z-extent of the point slab in each layer (top to bottom)."""
    d = list(d)
    slabs = []
    for l in range(len(d) + 1):
        if l == 0:
            slabs.append((d[0] + margin, d[0] + margin + thick))
        elif l == len(d):
            slabs.append((d[-1] - margin - thick, d[-1] - margin))
        else:
            slabs.append((d[l] + margin, d[l - 1] - margin))
    return slabs


def _uniform_layers(rng, counts, slabs, half_width):
    pts = []
    for n, (lo, hi) in zip(counts, slabs):
        xy = rng.uniform(-half_width, half_width, (n, 2))
        z = rng.uniform(lo, hi, (n, 1))
        pts.append(np.hstack([xy, z]))
    return np.vstack(pts)


def currents(rng, n, n_rhs=1):
    J = rng.uniform(-1, 1, (n_rhs, n, 3)) + 1j * rng.uniform(-1, 1, (n_rhs, n, 3))
    return J[0] if n_rhs == 1 else J


def tiny(seed=0):
    """Two-layer 600-point workload; returns (d, k, xyz[600,3], J[600,3])."""
    rng = np.random.default_rng(seed)
    m = MEDIA["two"]
    xyz = _uniform_layers(rng, [300, 300], [(0.1, 2.1), (-2.1, -0.1)], 1.0)
    J = currents(rng, xyz.shape[0])
    return np.array(m["d"]), np.array(m["k"]), xyz, J


def three_layer(n, seed=0, n_rhs=1, split=(0.4, 0.3, 0.3), half_width=4.0):
    """Three-layer uniform workload; returns (d, k, xyz[n,3], J)."""
    rng = np.random.default_rng(seed)
    m = MEDIA["three"]
    counts = [int(round(n * s)) for s in split[:-1]]
    counts.append(n - sum(counts))
    xyz = _uniform_layers(rng, counts, layer_slabs(m["d"]), half_width)
    J = currents(rng, n, n_rhs)
    return np.array(m["d"]), np.array(m["k"]), xyz, J


def _blobs(rng, n, slabs, n_blobs_per_layer, sigma, half_width, layer_probs):
    """n points in Gaussian blobs; points outside their slab or the box are
    redrawn from the same blob."""
    L = len(slabs)
    centers = []
    for l, (lo, hi) in enumerate(slabs):
        for _ in range(n_blobs_per_layer):
            c = np.array([rng.uniform(-half_width, half_width), rng.uniform(-half_width, half_width),
                          rng.uniform(lo, hi)])
            centers.append((l, c))
    probs = np.repeat(np.asarray(layer_probs, dtype=float) / n_blobs_per_layer, n_blobs_per_layer)
    probs = probs / probs.sum()
    which = rng.choice(len(centers), size=n, p=probs)
    out = np.empty((n, 3))
    for i, b in enumerate(which):
        l, c = centers[b]
        lo, hi = slabs[l]
        while True:
            p = c + sigma * rng.standard_normal(3)
            if lo <= p[2] <= hi and abs(p[0]) <= half_width and abs(p[1]) <= half_width:
                out[i] = p
                break
    return out


def clustered_three_layer(n, seed=0, n_blobs=8, sigma=0.3, n_rhs=1):
    """Three-layer medium, n points in n_blobs Gaussian blobs (40/30/30 %)."""
    rng = np.random.default_rng(seed)
    m = MEDIA["three"]
    slabs = layer_slabs(m["d"])
    per = max(1, n_blobs // 3)
    xyz = _blobs(rng, n, slabs, per, sigma, 4.0, [0.4, 0.3, 0.3])
    J = currents(rng, n, n_rhs)
    return np.array(m["d"]), np.array(m["k"]), xyz, J


def near_interface(n, margin, seed=0, n_rhs=1, half_width=1.0):
    """Three-layer points crowding the interfaces: two thirds uniform in the
    layer slabs kept `margin` from the interfaces, one third in thin sheets
    between `margin` and 2 `margin` on both sides of each interface (so the
    images and effective locations of the reaction components come within
    2 `margin` of each other).  Returns (d, k, xyz[n,3], J)."""
    rng = np.random.default_rng(seed + 9000)
    m = MEDIA["three"]
    d = m["d"]
    n_sheet = n // 3
    per = [n_sheet // (2 * len(d))] * (2 * len(d))
    per[-1] += n_sheet - sum(per)
    n_uni = n - n_sheet
    counts = [int(round(n_uni * s)) for s in (0.4, 0.3)]
    counts.append(n_uni - sum(counts))
    pts = [_uniform_layers(rng, counts, layer_slabs(d, margin=margin), half_width)]
    q = 0
    for di in d:
        for sgn in (1.0, -1.0):
            xy = rng.uniform(-half_width, half_width, (per[q], 2))
            z = di + sgn * rng.uniform(margin, 2.0 * margin, (per[q], 1))
            pts.append(np.hstack([xy, z]))
            q += 1
    xyz = np.vstack(pts)
    J = currents(rng, n, n_rhs)
    return np.array(d), np.array(m["k"]), xyz, J


def four_layer(n, seed=0, n_rhs=1):
    """Four-layer workload: n/2 uniform (25 % per layer) + n/2 in 20 blobs."""
    rng = np.random.default_rng(seed)
    m = MEDIA["four"]
    slabs = layer_slabs(m["d"])
    nu = n // 2
    counts = [nu // 4] * 3 + [nu - 3 * (nu // 4)]
    a = _uniform_layers(rng, counts, slabs, 4.0)
    b = _blobs(rng, n - nu, slabs, 5, 0.3, 4.0, [1, 1, 1, 1])
    xyz = np.vstack([a, b])
    J = currents(rng, n, n_rhs)
    return np.array(m["d"]), np.array(m["k"]), xyz, J


def sample_targets(n, count=256, seed=0):
    """Indices of sampled targets for the oracle comparison."""
    rng = np.random.default_rng(seed + 1000)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))


def sparse_currents(J, count, seed=0):
    """Copy of J with all but `count` randomly chosen sources zeroed (for
    oracle checks at full problem size); returns (J_sparse, kept indices)."""
    n = J.shape[-2]
    rng = np.random.default_rng(seed + 2000)
    keep = np.sort(rng.choice(n, size=min(count, n), replace=False))
    Js = np.zeros_like(J)
    Js[..., keep, :] = J[..., keep, :]
    return Js, keep


def tiny_targets(count=200, seed=0):
    """Target points distinct from the tiny workload's sources, drawn in the
    same two slabs (half above, half below the interface)."""
    rng = np.random.default_rng(seed + 4000)
    a = count // 2
    return _uniform_layers(rng, [a, count - a], [(0.1, 2.1), (-2.1, -0.1)], 1.0)


def cotangent(n, n_rhs=1, seed=0):
    """Seeded complex128 vectors [n, 3] (or [n_rhs, n, 3]) used as output
    gradients gA in the adjoint and gradient checks."""
    rng = np.random.default_rng(seed + 3000)
    return currents(rng, n, n_rhs)


def sample_sources(n, count, seed=0):
    """Sorted distinct source indices for sampled gradient checks."""
    rng = np.random.default_rng(seed + 5000)
    return np.sort(rng.choice(n, count, replace=False))


def uneven_geometries(n_geom=32, seed=0, n_min=5000, n_max=200000):
    """Many independent three-layer geometries of uneven size: N_g =
    round(exp(U(ln n_min, ln n_max))), each clustered (8 Gaussian blobs,
    sigma 0.3, 40/30/30 layer choice) with seed g.  Returns (d, k, [xyz_g],
    [J_g])."""
    rng = np.random.default_rng(seed + 6000)
    sizes = np.round(np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_geom))).astype(int)
    xs, Js = [], []
    d = k = None
    for g, n in enumerate(sizes):
        d, k, x, J = clustered_three_layer(int(n), seed=seed * 1000 + g)
        xs.append(x)
        Js.append(J)
    return d, k, xs, Js


def dipole_lattice(n, seed=0, n_rhs=1, eps_r=2.25, jitter=0.1, split=(0.4, 0.3, 0.3), half_width=4.0):
    """Coupled-dipole workload for the iterative solve: about n points on a
    jittered cubic lattice filling the three-layer slabs (40/30/30 %), the
    diagonal of the system and seeded excitations.

    Each layer's slab [-w, w]^2 x [lo, hi] gets a lattice of spacing h_l
    chosen so that the slab holds its share of points; every point is moved
    by U(-jitter, jitter) h_l per coordinate (nearest neighbours stay at least
    (1 - 2 jitter) h_l apart).  A point of layer l is a small sphere of
    relative permittivity eps_r in its layer: Clausius-Mossotti polarisability
    alpha = 3 h_l^3 chi / (4 pi), chi = (eps_r - 1) / (eps_r + 2), with the
    radiation-reaction term, so the diagonal is
        diag = 1 / (alpha k_l^2) - i k_l / (6 pi)
    in the units where the field of the dipoles is G applied to them.
    Returns (d, k, xyz [n', 3], diag [n'] complex128, B) with B complex128
    [n', 3] (n_rhs = 1) or [n_rhs, n', 3]; n' is close to n."""
    rng = np.random.default_rng(seed + 7000)
    m = MEDIA["three"]
    d, k = np.array(m["d"]), np.array(m["k"])
    slabs = layer_slabs(m["d"])
    chi = (eps_r - 1.0) / (eps_r + 2.0)
    pts, diag = [], []
    for l, ((lo, hi), s) in enumerate(zip(slabs, split)):
        vol = (2 * half_width) ** 2 * (hi - lo)
        h = (vol / (n * s)) ** (1.0 / 3.0)
        nx = max(1, int(round(2 * half_width / h)))
        nz = max(1, int(round((hi - lo) / h)))
        hx, hz = 2 * half_width / nx, (hi - lo) / nz
        gx = -half_width + (np.arange(nx) + 0.5) * hx
        gz = lo + (np.arange(nz) + 0.5) * hz
        X, Y, Z = np.meshgrid(gx, gx, gz, indexing="ij")
        p = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        p[:, :2] += rng.uniform(-jitter, jitter, (p.shape[0], 2)) * hx
        p[:, 2] += rng.uniform(-jitter, jitter, p.shape[0]) * hz
        hv = (hx * hx * hz) ** (1.0 / 3.0)
        alpha = 3.0 * hv ** 3 * chi / (4.0 * np.pi)
        pts.append(p)
        diag.append(np.full(p.shape[0], 1.0 / (alpha * k[l] ** 2) - 1j * k[l] / (6.0 * np.pi)))
    xyz = np.vstack(pts)
    B = currents(rng, xyz.shape[0], n_rhs)
    return d, k, xyz, np.concatenate(diag), B


def six_layer(n, seed=0, n_rhs=1, half_width=1.0):
    """Six-layer uniform workload (equal shares per layer); returns (d, k, xyz, J)."""
    rng = np.random.default_rng(seed + 8000)
    m = MEDIA["six"]
    counts = [n // 6] * 5
    counts.append(n - sum(counts))
    xyz = _uniform_layers(rng, counts, layer_slabs(m["d"]), half_width)
    J = currents(rng, n, n_rhs)
    return np.array(m["d"]), np.array(m["k"]), xyz, J
