"""Python access to the CPU oracle (test infrastructure only).

The oracle is the plain fp64 definition of the layered-media electric dyadic
Green's function sum that the GPU fast multipole path is checked against, of
the magnetic dyadic sum (the J6..J9 form of Sec. 3.1), and of the solution of
the coupled-dipole system (diag - G) X = B (dense LU of the assembled sum).
Layers may have relative permeabilities mu (default 1).  It is loaded only by
the tests, by the package smoke check and by the CPU-baseline leg of the
benchmark; the product path never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lm_oracle.c")
_LIB = os.path.join(_HERE, "liblmoracle.so")
_lib = None


def build(force=True):
    """Compile the oracle shared library with gcc (OpenMP, fp64, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        lib.lm_oracle_pair.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, P]
        lib.lm_oracle_reaction_pair.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, P]
        lib.lm_oracle_free_check.argtypes = [ctypes.c_double, P, P, P, P]
        lib.lm_oracle_pair_h.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, P]
        lib.lm_oracle_free_check_h.argtypes = [ctypes.c_double, P, P, P, P]
        lib.lm_oracle_direct_h.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int64, P, ctypes.c_int, P,
                                           ctypes.c_int64, P, P, ctypes.c_int]
        lib.lm_oracle_spectral.argtypes = [ctypes.c_int, P, P, P, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, P]
        lib.lm_oracle_bessel012.argtypes = [ctypes.c_double, ctypes.c_double, P]
        lib.lm_oracle_bessel012.restype = None
        lib.lm_oracle_direct.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int64, P, ctypes.c_int, P,
                                         ctypes.c_int64, P, P, ctypes.c_int]
        lib.lm_oracle_direct_free.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int64, P, P,
                                              ctypes.c_int64, P, P, ctypes.c_int]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _medium(d, k, mu=None):
    """(d, k, mu): mu = None means every relative permeability is 1."""
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1))
    k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1))
    if d.size == 0:
        d = np.zeros(1)
    if mu is None:
        return d, k, None
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    if mu.size != k.size:
        raise ValueError("mu needs one value per layer")
    return d, k, mu


def _pm(mu):
    return None if mu is None else _p(mu)


def pair(d, k, x, xp, quad_scale=1.0, mu=None):
    """Full 3x3 G(x, x') (free part for same-layer distinct points + reaction)."""
    d, k, mu = _medium(d, k, mu)
    x = np.ascontiguousarray(x, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    out = np.zeros(18)
    rc = _load().lm_oracle_pair(k.size, _p(d), _p(k), _pm(mu), _p(x), _p(xp), quad_scale, _p(out))
    if rc:
        raise ValueError("oracle rejected the medium (rc=%d)" % rc)
    return out.view(np.complex128).reshape(3, 3)


def pair_h(d, k, x, xp, quad_scale=1.0, mu=None):
    """Magnetic dyadic G_H(x, x') = (1/mu_t) curl_x G(x, x'), 3x3: the J6..J9
    form of the spectral dyadic (Sec. 3.1) plus, for the same layer and
    distinct points, the free-space curl grad g x (.) / mu."""
    d, k, mu = _medium(d, k, mu)
    x = np.ascontiguousarray(x, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    out = np.zeros(18)
    rc = _load().lm_oracle_pair_h(k.size, _p(d), _p(k), _pm(mu), _p(x), _p(xp), quad_scale, _p(out))
    if rc:
        raise ValueError("oracle rejected the medium (rc=%d)" % rc)
    return out.view(np.complex128).reshape(3, 3)


def free_check_h(k, x, xp):
    """(Sommerfeld-route free curl dyadic, closed form grad g x (.))."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    a = np.zeros(18)
    b = np.zeros(18)
    _load().lm_oracle_free_check_h(float(k), _p(x), _p(xp), _p(a), _p(b))
    return a.view(np.complex128).reshape(3, 3), b.view(np.complex128).reshape(3, 3)


def reaction_pair(d, k, x, xp, quad_scale=1.0, mu=None):
    """Reaction part G^r(x, x') only."""
    d, k, mu = _medium(d, k, mu)
    x = np.ascontiguousarray(x, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    out = np.zeros(18)
    rc = _load().lm_oracle_reaction_pair(k.size, _p(d), _p(k), _pm(mu), _p(x), _p(xp), quad_scale,
                                         _p(out))
    if rc:
        raise ValueError("oracle rejected the medium (rc=%d)" % rc)
    return out.view(np.complex128).reshape(3, 3)


def free_check(k, x, xp):
    """(Sommerfeld-route free dyadic, closed-form free dyadic)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    a = np.zeros(18)
    b = np.zeros(18)
    _load().lm_oracle_free_check(float(k), _p(x), _p(xp), _p(a), _p(b))
    return a.view(np.complex128).reshape(3, 3), b.view(np.complex128).reshape(3, 3)


def spectral(d, k, kr, z, zp, mu=None):
    """Reaction scalars [pol][R, dzR, dz'R, dzdz'R], pol 0 = TE, 1 = TM, of the
    normalised 1-D problems (no mu_t / mu_s factor)."""
    d, k, mu = _medium(d, k, mu)
    out = np.zeros(16)
    kr = complex(kr)
    rc = _load().lm_oracle_spectral(k.size, _p(d), _p(k), _pm(mu), kr.real, kr.imag, float(z), float(zp),
                                    _p(out))
    if rc:
        raise ValueError("oracle rejected the medium (rc=%d)" % rc)
    return out.view(np.complex128).reshape(2, 4)


def bessel012(z):
    out = np.zeros(6)
    z = complex(z)
    _load().lm_oracle_bessel012(z.real, z.imag, _p(out))
    return out.view(np.complex128)


def direct(d, k, src, J, tgt, n_threads=None, mu=None):
    """A[r, i] = sum_j G(tgt_i, src_j) J[r, j]  (complex128 [n_rhs, n_tgt, 3]).

    J may be [n_src, 3] (one right-hand side) or [n_rhs, n_src, 3]."""
    d, k, mu = _medium(d, k, mu)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    tgt = np.ascontiguousarray(tgt, dtype=np.float64).reshape(-1, 3)
    J = np.asarray(J, dtype=np.complex128)
    single = J.ndim == 2
    J = np.ascontiguousarray(J.reshape(-1, src.shape[0], 3))
    A = np.zeros((J.shape[0], tgt.shape[0], 3), dtype=np.complex128)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    Jr = J.view(np.float64)
    Ar = A.view(np.float64)
    rc = _load().lm_oracle_direct(k.size, _p(d), _p(k), _pm(mu), src.shape[0], _p(src), J.shape[0],
                                  _p(Jr), tgt.shape[0], _p(tgt), _p(Ar), int(n_threads))
    if rc:
        raise ValueError("oracle failed (rc=%d)" % rc)
    return A[0] if single else A


def direct_h(d, k, src, J, tgt, n_threads=None, mu=None):
    """H[r, i] = sum_j G_H(tgt_i, src_j) J[r, j] (complex128 [n_rhs, n_tgt, 3])."""
    d, k, mu = _medium(d, k, mu)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    tgt = np.ascontiguousarray(tgt, dtype=np.float64).reshape(-1, 3)
    J = np.asarray(J, dtype=np.complex128)
    single = J.ndim == 2
    J = np.ascontiguousarray(J.reshape(-1, src.shape[0], 3))
    H = np.zeros((J.shape[0], tgt.shape[0], 3), dtype=np.complex128)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = _load().lm_oracle_direct_h(k.size, _p(d), _p(k), _pm(mu), src.shape[0], _p(src), J.shape[0],
                                    _p(J.view(np.float64)), tgt.shape[0], _p(tgt), _p(H.view(np.float64)),
                                    int(n_threads))
    if rc:
        raise ValueError("oracle failed (rc=%d)" % rc)
    return H[0] if single else H


def direct_free(d, k, src, J, tgt, n_threads=None):
    """Free-space part only (closed form), one right-hand side."""
    d, k, mu = _medium(d, k)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    tgt = np.ascontiguousarray(tgt, dtype=np.float64).reshape(-1, 3)
    J = np.ascontiguousarray(np.asarray(J, dtype=np.complex128).reshape(-1, 3))
    A = np.zeros((tgt.shape[0], 3), dtype=np.complex128)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = _load().lm_oracle_direct_free(k.size, _p(d), _p(k), _pm(mu), src.shape[0], _p(src),
                                       _p(J.view(np.float64)), tgt.shape[0], _p(tgt),
                                       _p(A.view(np.float64)), int(n_threads))
    if rc:
        raise ValueError("oracle failed (rc=%d)" % rc)
    return A


def dense_operator(d, k, pts, n_threads=None, mu=None):
    """The matrix M [3n, 3n] of the layered sum on one point set (sources =
    targets): (M J)[3i + a] = sum_j sum_b G_ab(x_i, x_j) J[3j + b], built
    column by column from the direct sum applied to unit currents."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    M = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    for c0 in range(0, 3 * n, 64):
        cols = np.arange(c0, min(3 * n, c0 + 64))
        E = np.zeros((cols.size, n, 3), dtype=np.complex128)
        E[np.arange(cols.size), cols // 3, cols % 3] = 1.0
        A = direct(d, k, pts, E, pts, n_threads, mu=mu)
        M[:, cols] = A.reshape(cols.size, 3 * n).T
    return M


def solve(d, k, pts, diag, B, n_threads=None, mu=None):
    """Solution X of the coupled-dipole system (diag - G) X = B on one point
    set: diag [n] complex (one value per point, on its three components),
    B [n, 3] or [n_rhs, n, 3] complex.  Dense LU of the assembled matrix
    (the system whose matrix-vector product is the layered sum of the paper's
    Sec. 3.3, the integral-equation use the paper's introduction names)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    B = np.asarray(B, dtype=np.complex128)
    single = B.ndim == 2
    Bm = B.reshape(-1, 3 * n).T
    K = np.diag(np.repeat(np.asarray(diag, dtype=np.complex128).reshape(n), 3)) - dense_operator(
        d, k, pts, n_threads, mu=mu)
    X = np.linalg.solve(K, Bm).T.reshape(-1, n, 3)
    return X[0] if single else X
