"""A CPU run of the layered-media dyadic FMM (test infrastructure only).

`libcpufmm.so` executes the same fast multipole algorithm as the HIP library
-- the same plan (trees, lists, M2L orders, quadrature nodes, taken from the
library's planner), every table and pass computed on the host in plain loops
by routes of its own (see cpufmm.cpp) -- so that each HIP kernel can be
compared with it at rounding level.  Only the tests use it; the product path
never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_LIB = os.path.join(_HERE, "libcpufmm.so")
_SRC = [os.path.join(_HERE, "cpufmm.cpp"),
        os.path.join(_ROOT, "paper_2507_18491_amd", "csrc", "plan.cpp")]
_lib = None


def build(force=True):
    """Compiles libcpufmm.so (host code only: the planner and this file)."""
    if force or not os.path.exists(_LIB):
        hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
        tmp = _LIB + ".tmp"
        subprocess.check_call([hipcc, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-fPIC",
                               "-shared", "-Wno-unused-result", "-o", tmp] + _SRC + ["-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        I64 = ctypes.POINTER(ctypes.c_int64)
        lib.lmc_run.argtypes = [ctypes.c_int, P, P, P, ctypes.c_void_p, ctypes.c_int, I64, P, I64, P,
                                ctypes.c_int, P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
        lib.lmc_ladder.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        lib.lmc_eval_regular.argtypes = [ctypes.c_int, ctypes.c_double, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _medium(d, k, mu):
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1))
    if d.size == 0:
        d = np.zeros(1)
    k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1))
    mu_a = None if mu is None else np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    return d, k, mu_a


def _run(d, k, mu, src, tgt, J, W, mode, n_threads, geoms, params):
    from paper_2507_18491_amd import lmfmm
    lib = _load()
    prm = lmfmm.make_params(**params)
    d, k, mu_a = _medium(d, k, mu)
    n_rhs = J.shape[0]
    if geoms is None:
        so = np.array([0, src.shape[0]], dtype=np.int64)
        to = np.array([0, tgt.shape[0]], dtype=np.int64)
    else:
        so = np.ascontiguousarray(geoms[0], dtype=np.int64)
        to = np.ascontiguousarray(geoms[1], dtype=np.int64)
    if mode == 2:
        out = np.zeros((tgt.shape[0], 3))
        outp = _p(out)
    else:
        out = np.zeros((n_rhs, tgt.shape[0], 3), dtype=np.complex128)
        outp = _p(out.view(np.float64))
    err = ctypes.create_string_buffer(1024)
    i64 = ctypes.POINTER(ctypes.c_int64)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rc = lib.lmc_run(k.size, _p(d), _p(k), None if mu_a is None else _p(mu_a), ctypes.addressof(prm),
                     so.size - 1, so.ctypes.data_as(i64), _p(src), to.ctypes.data_as(i64), _p(tgt), n_rhs,
                     _p(J.view(np.float64)), None if W is None else _p(W.view(np.float64)), int(mode), outp,
                     int(n_threads), err, 1024)
    if rc:
        raise RuntimeError("cpu FMM failed (%d): %s" % (rc, err.value.decode()))
    return out


def _pts(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3))


def _vecs(a, n):
    a = np.asarray(a, dtype=np.complex128)
    return a.ndim == 2, np.ascontiguousarray(a.reshape(-1, n, 3))


def run(d, k, src, J, tgt=None, mu=None, mode=0, n_threads=None, geoms=None, **params):
    """A = G J (mode 0) or H = G_H J (mode 1) by the CPU run of the FMM.

    d, k, mu: the medium; src [n, 3]; J [n, 3] or [n_rhs, n, 3] complex;
    tgt: targets (None: the sources).  params: lm_params fields (the
    library's defaults otherwise).  geoms: None, or (src_off, tgt_off) of a
    batch of geometries (as lm_build_batch)."""
    src = _pts(src)
    tgt = src if tgt is None else _pts(tgt)
    single, Jr = _vecs(J, src.shape[0])
    out = _run(d, k, mu, src, tgt, Jr, None, mode, n_threads, geoms, params)
    return out[0] if single else out


def _mu_of(d, mu, z):
    if mu is None:
        return np.ones_like(z)
    d = np.asarray(d, dtype=np.float64).reshape(-1)
    lay = np.zeros(z.shape, dtype=np.int64)
    for l in range(d.size):
        lay += (z < d[l]).astype(np.int64)
    return np.asarray(mu, dtype=np.float64)[lay]


def adjoint(d, k, src, gA, tgt=None, mu=None, n_threads=None, **params):
    """gJ = G^H gA through reciprocity, as the library computes it: the
    forward sum with the roles of the point sets exchanged, applied to
    conj(mu gA) and conjugated, divided by mu at the sources."""
    src = _pts(src)
    tgt = src if tgt is None else _pts(tgt)
    single, g = _vecs(gA, tgt.shape[0])
    mt = _mu_of(d, mu, tgt[:, 2])[None, :, None]
    ms = _mu_of(d, mu, src[:, 2])[None, :, None]
    B = _run(d, k, mu, tgt, src, np.ascontiguousarray(np.conj(g * mt)), None, 0, n_threads, None, params)
    out = np.conj(B) / ms
    return out[0] if single else out


def grad_src_xyz(d, k, src, J, gA, tgt=None, mu=None, n_threads=None, **params):
    """Source-position gradient [n_src, 3] of a real loss with dL/dA = gA
    (summed over right-hand sides), as the library computes it: the field of
    the currents conj(mu gA) at the targets, differentiated at the sources
    (roles exchanged) and contracted with J, divided by mu at the sources."""
    src = _pts(src)
    tgt = src if tgt is None else _pts(tgt)
    _, Jr = _vecs(J, src.shape[0])
    _, g = _vecs(gA, tgt.shape[0])
    mt = _mu_of(d, mu, tgt[:, 2])[None, :, None]
    ms = _mu_of(d, mu, src[:, 2])[:, None]
    gX = _run(d, k, mu, tgt, src, np.ascontiguousarray(np.conj(g * mt)), Jr, 2, n_threads, None, params)
    return gX / ms


def ladder(c, order, direction):
    """(d/dx + i d/dy)/k (0), (d/dx - i d/dy)/k (1) or (d/dz)/k (2) of the
    regular expansion with coefficients c [(order+1)^2]: coefficients
    [(order+2)^2]."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
    out = np.zeros((order + 2) ** 2, dtype=np.complex128)
    rc = _load().lmc_ladder(order, direction, _p(c.view(np.float64)), _p(out.view(np.float64)))
    if rc:
        raise RuntimeError("lmc_ladder failed")
    return out


def eval_regular(c, order, k, dvec):
    """sum_nm c_nm j_n(k|d|) Y^m_n(d)."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
    dv = np.ascontiguousarray(np.asarray(dvec, dtype=np.float64))
    out = np.zeros(1, dtype=np.complex128)
    rc = _load().lmc_eval_regular(order, float(k), _p(c.view(np.float64)), _p(dv), _p(out.view(np.float64)))
    if rc:
        raise RuntimeError("lmc_eval_regular failed")
    return out[0]
