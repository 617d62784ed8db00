"""Python binding of the layered-media dyadic FMM library (liblmfmm.so).

Argument marshalling only: every step of the evaluation runs in the HIP
library.  PyTorch provides device memory and the current stream.  The
binding raises if the library is missing; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblmfmm.so")

LM_OK = 0
LM_EACCURACY = -6
STAT_NAMES = ["n_free_inst", "n_react_inst", "m2l_pairs_free", "m2l_pairs_react", "p2p_pairs",
              "n_cases", "n_nodes", "mat_bytes", "me_bytes_per_rhs", "le_bytes_per_rhs",
              "t_plan_ms", "t_upload_ms", "t_tables_ms", "n_src_boxes", "n_tgt_boxes",
              "n_m2l_classes", "n_m2l_tiles_1rhs", "m2l_cmac_useful", "m2l_cmac_exec",
              "n_leaves_p2m", "free_depth", "s2t_pairs", "m2l_flop_exec", "p2m_flops", "m2m_flops",
              "l2l_flops", "l2p_flops", "reduce_bytes", "s2t_node_evals", "m2l_cmac_dense",
              "p2p_kernel_evals", "tree_records", "tree_sort_ms", "plan_digest_hi", "plan_digest_lo"]


PHASE_NAMES = ["clear", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p"]


class lm_params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("p_free", ctypes.c_int), ("free_depth", ctypes.c_int),
                ("max_depth", ctypes.c_int), ("gamma1_panels", ctypes.c_int),
                ("contour_a", ctypes.c_double), ("tail_digits", ctypes.c_double),
                ("components", ctypes.c_int), ("m2l_adapt", ctypes.c_int),
                ("m2l_margin", ctypes.c_double), ("react_s2t", ctypes.c_int),
                ("m2l_variant", ctypes.c_int), ("tol", ctypes.c_double), ("host_trees", ctypes.c_int)]

M2L_VARIANTS = 3
NOALLOC_SCRATCH_BYTES = 256 << 20
SOLVE_MAX_RESTART = 64


class lm_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvecs", ctypes.c_int), ("cycles", ctypes.c_int),
                ("converged", ctypes.c_int), ("ms_total", ctypes.c_double), ("ms_matvec", ctypes.c_double),
                ("ms_krylov", ctypes.c_double), ("krylov_bytes", ctypes.c_double)]


_lib = None


def load_library():
    """Loads liblmfmm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblmfmm.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    D = P(ctypes.c_double)
    vp = ctypes.c_void_p
    lib.lm_default_params.argtypes = [P(lm_params)]
    lib.lm_create.argtypes = [P(vp), ctypes.c_int]
    lib.lm_destroy.argtypes = [vp]
    lib.lm_last_error.argtypes = [vp]
    lib.lm_last_error.restype = ctypes.c_char_p
    lib.lm_set_layers.argtypes = [vp, ctypes.c_int, D, D, D]
    lib.lm_set_params.argtypes = [vp, P(lm_params)]
    lib.lm_build.argtypes = [vp, ctypes.c_int64, D, ctypes.c_int64, D, vp]
    lib.lm_evaluate.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.lm_evaluate_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.lm_selftest_math.argtypes = [ctypes.c_int64, vp, vp, vp]
    lib.lm_build_batch.argtypes = [vp, ctypes.c_int, P(ctypes.c_int64), D, P(ctypes.c_int64), D, vp]
    lib.lm_evaluate_adjoint.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.lm_evaluate_h.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.lm_grad_src_xyz.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    lib.lm_stats.argtypes = [vp, D, ctypes.c_int]
    lib.lm_m2l_variants.argtypes = [vp, ctypes.c_int, P(ctypes.c_int), D, ctypes.c_int]
    lib.lm_set_timing.argtypes = [vp, ctypes.c_int]
    lib.lm_timings.argtypes = [vp, D, ctypes.c_int]
    lib.lm_host_components.argtypes = [ctypes.c_int, D, D, P(ctypes.c_int), ctypes.c_int]
    lib.lm_host_cheb_affine.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, D]
    lib.lm_host_legendre_cheb.argtypes = [ctypes.c_int, D, P(ctypes.c_int)]
    lib.lm_solve.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, D,
                             P(lm_solve_info), vp]
    lib.lm_host_gmres_dense.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, P(ctypes.c_int), D]
    lib.lm_host_plan_stats.argtypes = [ctypes.c_int, D, D, P(lm_params), ctypes.c_int64, D, ctypes.c_int64,
                                       D, D, ctypes.c_int, ctypes.c_char_p, ctypes.c_int]
    I64 = P(ctypes.c_int64)
    lib.lm_host_plan_digests.argtypes = [ctypes.c_int, D, D, P(lm_params), ctypes.c_int, I64, D, I64, D,
                                         P(ctypes.c_uint64), ctypes.c_char_p, ctypes.c_int]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _medium(d, k):
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1))
    k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1))
    return (d if d.size else np.zeros(1)), k


def make_params(**kw):
    prm = lm_params()
    load_library().lm_default_params(ctypes.byref(prm))
    for key, v in kw.items():
        if v is None:
            continue
        if not hasattr(prm, key):
            raise TypeError("unknown parameter %s" % key)
        setattr(prm, key, v)
    return prm


class LMError(RuntimeError):
    pass


class LayeredDyadicFMM:
    """A = G J for the layered electric dyadic Green's function on one GPU.

    d: interfaces (top to bottom), k: layer wavenumbers (top to bottom),
    mu: relative permeabilities (top to bottom; None = all 1).
    Keyword parameters are those of lm_params (p, p_free, free_depth, ...).
    """

    def __init__(self, d, k, device=0, mu=None, **params):
        self.lib = load_library()
        self.ctx = ctypes.c_void_p()
        rc = self.lib.lm_create(ctypes.byref(self.ctx), int(device))
        if rc != LM_OK:
            raise LMError("lm_create failed (%d)" % rc)
        self.device = int(device)
        self.d, self.k = _medium(d, k)
        self.mu = None
        if mu is not None:
            self.mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
            if self.mu.size != self.k.size:
                raise LMError("mu needs one value per layer")
        self._check(self.lib.lm_set_layers(self.ctx, self.k.size, _dp(self.d), _dp(self.k),
                                           None if self.mu is None else _dp(self.mu)))
        self.params = make_params(**params)
        self._check(self.lib.lm_set_params(self.ctx, ctypes.byref(self.params)))
        self.n_src = self.n_tgt = None

    def _check(self, rc):
        if rc != LM_OK:
            msg = self.lib.lm_last_error(self.ctx)
            e = LMError("lmfmm error %d: %s" % (rc, msg.decode() if msg else ""))
            e.code = rc
            raise e

    def build(self, src, tgt=None, stream=None):
        import torch
        src = np.ascontiguousarray(np.asarray(src, dtype=np.float64).reshape(-1, 3))
        tgt = src if tgt is None else np.ascontiguousarray(np.asarray(tgt, dtype=np.float64).reshape(-1, 3))
        if stream is None:
            with torch.cuda.device(self.device):
                stream = torch.cuda.current_stream().cuda_stream
        self._check(self.lib.lm_build(self.ctx, src.shape[0], _dp(src), tgt.shape[0], _dp(tgt),
                                      ctypes.c_void_p(stream)))
        self.n_src, self.n_tgt = src.shape[0], tgt.shape[0]
        self._src_host, self._src_dev = src, None
        return self

    def build_batch(self, srcs, tgts=None, stream=None):
        """Several independent geometries in one plan (each pass launched for
        all of them together, see lm_build_batch).  srcs: list of [n_g, 3] arrays; tgts: list or None (targets
        = sources).  Currents and outputs are the concatenations in order;
        self.src_off / self.tgt_off give the geometry boundaries."""
        import torch
        srcs = [np.asarray(a, dtype=np.float64).reshape(-1, 3) for a in srcs]
        tgts = srcs if tgts is None else [np.asarray(a, dtype=np.float64).reshape(-1, 3) for a in tgts]
        if len(tgts) != len(srcs):
            raise LMError("srcs and tgts must have the same number of geometries")
        so = np.zeros(len(srcs) + 1, dtype=np.int64)
        to = np.zeros(len(srcs) + 1, dtype=np.int64)
        so[1:] = np.cumsum([a.shape[0] for a in srcs])
        to[1:] = np.cumsum([a.shape[0] for a in tgts])
        src = np.ascontiguousarray(np.concatenate(srcs)) if srcs else np.zeros((0, 3))
        tgt = src if tgts is srcs else (np.ascontiguousarray(np.concatenate(tgts)) if tgts else np.zeros((0, 3)))
        if stream is None:
            with torch.cuda.device(self.device):
                stream = torch.cuda.current_stream().cuda_stream
        i64 = ctypes.POINTER(ctypes.c_int64)
        self._check(self.lib.lm_build_batch(self.ctx, len(srcs), so.ctypes.data_as(i64), _dp(src),
                                            to.ctypes.data_as(i64), _dp(tgt), ctypes.c_void_p(stream)))
        self.n_src, self.n_tgt = int(so[-1]), int(to[-1])
        self.src_off, self.tgt_off = so, to
        self._src_host, self._src_dev = src, None
        return self

    def evaluate(self, J, out=None, stream=None):
        """J: complex128 CUDA tensor [n_src, 3] or [n_rhs, n_src, 3]; returns A (same rank)."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        single, n_rhs, Jr = self._rhs_view(J, self.n_src, "J")
        out = self._out(out, (n_rhs, self.n_tgt, 3), torch.complex128, J)
        if stream is None:
            stream = torch.cuda.current_stream(J.device).cuda_stream
        self._check(self.lib.lm_evaluate(self.ctx, n_rhs, ctypes.c_void_p(Jr.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
        return out.view(self.n_tgt, 3) if single else out.view(n_rhs, self.n_tgt, 3)

    def evaluate_noalloc(self, J, out, stream=None):
        """A = G J by lm_evaluate_noalloc: the library allocates nothing (its
        work buffers live in a static device array of
        NOALLOC_SCRATCH_BYTES per GPU); `out` must be given.  Calls that
        overlap in time on one GPU race."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        single, n_rhs, Jr = self._rhs_view(J, self.n_src, "J")
        out = self._out(out, (n_rhs, self.n_tgt, 3), torch.complex128, J)
        if stream is None:
            stream = torch.cuda.current_stream(J.device).cuda_stream
        self._check(self.lib.lm_evaluate_noalloc(self.ctx, n_rhs, ctypes.c_void_p(Jr.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
        return out.view(self.n_tgt, 3) if single else out.view(n_rhs, self.n_tgt, 3)

    def evaluate_h(self, J, out=None, stream=None):
        """Magnetic field H = G_H J, G_H = (1/mu) curl G (Faraday's law).
        J: complex128 CUDA tensor [n_src, 3] or [n_rhs, n_src, 3]."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        single, n_rhs, Jr = self._rhs_view(J, self.n_src, "J")
        out = self._out(out, (n_rhs, self.n_tgt, 3), torch.complex128, J)
        if stream is None:
            stream = torch.cuda.current_stream(J.device).cuda_stream
        self._check(self.lib.lm_evaluate_h(self.ctx, n_rhs, ctypes.c_void_p(Jr.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
        return out.view(self.n_tgt, 3) if single else out.view(n_rhs, self.n_tgt, 3)

    def _rhs_view(self, X, n, name):
        import torch
        if not (X.is_cuda and X.dtype == torch.complex128):
            raise LMError("%s must be a complex128 CUDA tensor" % name)
        if X.device.index != self.device:
            raise LMError("%s must be on cuda:%d (the device of the build)" % (name, self.device))
        single = X.dim() == 2
        n_rhs = 1 if single else X.shape[0]
        if X.dim() not in (2, 3) or X.numel() != n_rhs * n * 3:
            raise LMError("%s must have shape [%d, 3] or [n_rhs, %d, 3], got %s" % (name, n, n, tuple(X.shape)))
        return single, n_rhs, X.reshape(n_rhs, n, 3).contiguous()

    def _out(self, out, shape, dtype, like, name="out"):
        """A new output tensor, or the caller's after checking everything the
        library relies on (the C ABI itself checks only pointer alignment):
        dtype, device, contiguity and size."""
        import torch
        if out is None:
            return torch.empty(shape, dtype=dtype, device=like.device)
        if not (out.is_cuda and out.dtype == dtype):
            raise LMError("%s must be a %s CUDA tensor" % (name, str(dtype).replace("torch.", "")))
        if out.device != like.device:
            raise LMError("%s must be on %s (the input's device)" % (name, like.device))
        if not out.is_contiguous():
            raise LMError("%s must be contiguous" % name)
        n = 1
        for v in shape:
            n *= v
        if out.numel() != n:
            raise LMError("%s must hold %d elements (shape %s), got %d" % (name, n, tuple(shape), out.numel()))
        return out

    def evaluate_adjoint(self, gA, out=None, stream=None):
        """gJ = G^H gA.  gA: complex128 CUDA tensor [n_tgt, 3] or [n_rhs, n_tgt, 3]."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        single, n_rhs, g = self._rhs_view(gA, self.n_tgt, "gA")
        out = self._out(out, (n_rhs, self.n_src, 3), torch.complex128, gA)
        if stream is None:
            stream = torch.cuda.current_stream(gA.device).cuda_stream
        self._check(self.lib.lm_evaluate_adjoint(self.ctx, n_rhs, ctypes.c_void_p(g.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
        return out.view(self.n_src, 3) if single else out.view(n_rhs, self.n_src, 3)

    def grad_src_xyz(self, J, gA, out=None, stream=None):
        """Gradient [n_src, 3] (fp64) of a real loss with dL/dA = gA with respect to
        the source positions (targets fixed), summed over right-hand sides."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        _, n_rhs, Jr = self._rhs_view(J, self.n_src, "J")
        _, n_rhs2, g = self._rhs_view(gA, self.n_tgt, "gA")
        if n_rhs2 != n_rhs:
            raise LMError("J and gA have different numbers of right-hand sides")
        if gA.device != J.device:
            raise LMError("J and gA must be on the same device")
        out = self._out(out, (self.n_src, 3), torch.float64, J)
        if stream is None:
            stream = torch.cuda.current_stream(J.device).cuda_stream
        self._check(self.lib.lm_grad_src_xyz(self.ctx, n_rhs, ctypes.c_void_p(Jr.data_ptr()),
                                             ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(stream)))
        return out

    def solve(self, diag, B, X=None, tol=1e-6, restart=30, max_iter=1000, stream=None):
        """Solves (diag - G) X = B by restarted GMRES on the built point set
        (sources = targets).  diag: complex128 CUDA tensor [n] or None (zero);
        B: complex128 CUDA tensor [n, 3] or [n_rhs, n, 3]; X: initial guess
        of the same shape (zeros if None), overwritten with the solution.
        Returns (X, info) with info a dict: iters, matvecs, cycles,
        converged, relres (per right-hand side), ms_total, ms_matvec,
        ms_krylov, krylov_bytes."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        single, n_rhs, Bv = self._rhs_view(B, self.n_src, "B")
        if X is None:
            X = torch.zeros_like(Bv)
        else:
            if not (X.is_cuda and X.dtype == torch.complex128 and X.is_contiguous()
                    and X.numel() == Bv.numel()):
                raise LMError("X must be a contiguous complex128 CUDA tensor shaped like B")
            if X.data_ptr() == Bv.data_ptr():
                raise LMError("X must not share memory with B")
        if diag is not None:
            if not (diag.is_cuda and diag.dtype == torch.complex128 and diag.numel() == self.n_src):
                raise LMError("diag must be a complex128 CUDA tensor [n]")
            diag = diag.contiguous()
        if stream is None:
            stream = torch.cuda.current_stream(Bv.device).cuda_stream
        rel = np.zeros(n_rhs)
        info = lm_solve_info()
        self._check(self.lib.lm_solve(self.ctx, n_rhs, ctypes.c_void_p(diag.data_ptr() if diag is not None else 0),
                                      ctypes.c_void_p(Bv.data_ptr()), ctypes.c_void_p(X.data_ptr()), float(tol),
                                      int(restart), int(max_iter), _dp(rel), ctypes.byref(info),
                                      ctypes.c_void_p(stream)))
        out = {f: getattr(info, f) for f, _ in lm_solve_info._fields_}
        out["converged"] = bool(out["converged"])
        out["relres"] = rel
        Xv = X.reshape(n_rhs, self.n_src, 3)
        return (Xv[0] if single else Xv), out

    def stats(self):
        buf = np.zeros(len(STAT_NAMES))
        self._check(self.lib.lm_stats(self.ctx, _dp(buf), buf.size))
        return dict(zip(STAT_NAMES, buf.tolist()))

    def source_positions(self, requires_grad=False):
        """The source positions of the build as a new float64 CUDA tensor
        [n_src, 3] (a leaf; with requires_grad=True, pass it to apply() to get
        the gradient of a loss with respect to the source positions)."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        X = torch.tensor(self._src_host, dtype=torch.float64, device="cuda:%d" % self.device)
        return X.requires_grad_(requires_grad)

    def apply(self, J, X=None):
        """A = G J as a differentiable torch operation (torch.autograd.Function):
        the backward pass gives dL/dJ = G^H dL/dA (lm_evaluate_adjoint, the
        transposed FMM by reciprocity, its upward pass recomputed) and, when X
        is given, dL/dX for the source positions (lm_grad_src_xyz).  The
        positions are fixed by the build: X must hold exactly the built source
        positions (e.g. source_positions(requires_grad=True)) and only carries
        their gradient.  J: complex128 CUDA tensor [n_src, 3] or
        [n_rhs, n_src, 3]."""
        import torch
        if self.n_src is None:
            raise LMError("build() must be called first")
        if X is not None:
            if X.dtype != torch.float64 or tuple(X.shape) != (self.n_src, 3):
                raise LMError("X must be a float64 tensor [n_src, 3]")
            if X.is_cuda:
                if self._src_dev is None or self._src_dev.device != X.device:
                    self._src_dev = torch.tensor(self._src_host, dtype=torch.float64, device=X.device)
                same = torch.equal(X.detach(), self._src_dev)
            else:
                same = np.array_equal(X.detach().numpy(), self._src_host)
            if not same:
                raise LMError("X differs from the source positions of the build (rebuild for new positions)")
        return _fmm_function().apply(self, J, X)

    def m2l_variants(self, n_rhs=1):
        """(variant, ms) for each M2L GEMM launch of the n_rhs schedule: the
        variant the autotuner chose (-1: not tuned yet) and its timings of the
        M2L_VARIANTS variants in ms (negative: not measured)."""
        cap = 4096
        var = (ctypes.c_int * cap)()
        ms = np.zeros(cap * M2L_VARIANTS)
        n = self.lib.lm_m2l_variants(self.ctx, n_rhs, var, _dp(ms), cap)
        if n < 0:
            self._check(n)
        n = min(n, cap)
        return [int(var[i]) for i in range(n)], ms[:n * M2L_VARIANTS].reshape(n, M2L_VARIANTS)

    def set_timing(self, enable=True):
        self._check(self.lib.lm_set_timing(self.ctx, 1 if enable else 0))

    def timings(self):
        """Milliseconds per phase summed over the timed evaluations, and their count."""
        buf = np.zeros(len(PHASE_NAMES) + 3)
        self._check(self.lib.lm_timings(self.ctx, _dp(buf), buf.size))
        n = len(PHASE_NAMES)
        return dict(zip(PHASE_NAMES, buf[:n].tolist())), int(buf[n])

    KERNEL_TIMING_NAMES = ["m2l_gemm", "m2l_reduce", "p2p", "s2t"]

    def kernel_timings(self):
        """{kernel: (milliseconds, launches)} summed over the timed
        evaluations, from HIP events around each launch of the M2L GEMM, the
        M2L reduction, the free-space near field and the direct reaction
        pairs on the evaluation stream."""
        n = len(PHASE_NAMES)
        buf = np.zeros(n + 1 + 2 * len(self.KERNEL_TIMING_NAMES))
        self._check(self.lib.lm_timings(self.ctx, _dp(buf), buf.size))
        return {nm: (float(buf[n + 1 + 2 * i]), int(buf[n + 2 + 2 * i]))
                for i, nm in enumerate(self.KERNEL_TIMING_NAMES)}

    def m2l_gemm_timing(self):
        """Milliseconds spent in the M2L GEMM kernel alone (HIP events around
        each launch on the evaluation stream) over the timed evaluations, and
        the number of its launches."""
        buf = np.zeros(len(PHASE_NAMES) + 3)
        self._check(self.lib.lm_timings(self.ctx, _dp(buf), buf.size))
        n = len(PHASE_NAMES)
        return float(buf[n + 1]), int(buf[n + 2])

    def close(self):
        if self.ctx:
            self.lib.lm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_FMM_FUNCTION = None


def _fmm_function():
    """The torch.autograd.Function behind LayeredDyadicFMM.apply (created on
    first use, so that importing this module does not import torch)."""
    global _FMM_FUNCTION
    if _FMM_FUNCTION is None:
        import torch

        class FMMApply(torch.autograd.Function):
            @staticmethod
            def forward(ctx, fmm, J, X):
                ctx.fmm = fmm
                ctx.x_on_cpu = X is not None and not X.is_cuda
                ctx.save_for_backward(J)
                return fmm.evaluate(J)

            @staticmethod
            def backward(ctx, gA):
                (J,) = ctx.saved_tensors
                gA = gA.contiguous()
                gJ = ctx.fmm.evaluate_adjoint(gA) if ctx.needs_input_grad[1] else None
                gX = None
                if ctx.needs_input_grad[2]:
                    gX = ctx.fmm.grad_src_xyz(J.detach(), gA)
                    if ctx.x_on_cpu:
                        gX = gX.cpu()
                return None, gJ, gX

        _FMM_FUNCTION = FMMApply
    return _FMM_FUNCTION


# ---------------------------------------------------------------- host-only helpers
def host_components(d, k):
    lib = load_library()
    d, k = _medium(d, k)
    buf = (ctypes.c_int * (8 * 4096))()
    n = lib.lm_host_components(k.size, _dp(d), _dp(k), buf, 4096)
    if n < 0:
        raise LMError("lm_host_components failed (%d)" % n)
    return np.array(buf[:8 * n], dtype=np.int64).reshape(n, 8)


def host_cheb_affine(jmax, a, b):
    out = np.zeros((jmax + 1) * (jmax + 1))
    rc = load_library().lm_host_cheb_affine(jmax, a, b, _dp(out))
    if rc:
        raise LMError("lm_host_cheb_affine failed")
    return out.reshape(jmax + 1, jmax + 1)


def host_legendre_cheb(p):
    stride = ctypes.c_int()
    out = np.zeros((p + 1) * (p + 2) // 2 * ((p + 1) // 2 + 2))
    rc = load_library().lm_host_legendre_cheb(p, _dp(out), ctypes.byref(stride))
    if rc:
        raise LMError("lm_host_legendre_cheb failed")
    return out.reshape(-1, stride.value)


def host_plan_digests(d, k, srcs, tgts=None, **params):
    """Digests of the host-planned geometries (lists of [n_g, 3] arrays) with
    the octree records sorted by the external route's contract in plain host
    code, and by the planner's own sort (lm_host_plan_digests)."""
    lib = load_library()
    d, k = _medium(d, k)
    srcs = [np.asarray(a, dtype=np.float64).reshape(-1, 3) for a in srcs]
    tgts = srcs if tgts is None else [np.asarray(a, dtype=np.float64).reshape(-1, 3) for a in tgts]
    soff = np.ascontiguousarray(np.cumsum([0] + [a.shape[0] for a in srcs]), dtype=np.int64)
    toff = np.ascontiguousarray(np.cumsum([0] + [a.shape[0] for a in tgts]), dtype=np.int64)
    src = np.ascontiguousarray(np.concatenate(srcs) if srcs else np.zeros((0, 3)))
    tgt = np.ascontiguousarray(np.concatenate(tgts) if tgts else np.zeros((0, 3)))
    prm = make_params(**params)
    out = (ctypes.c_uint64 * 2)()
    err = ctypes.create_string_buffer(1024)
    I64 = ctypes.POINTER(ctypes.c_int64)
    rc = lib.lm_host_plan_digests(k.size, _dp(d), _dp(k), ctypes.byref(prm), len(srcs),
                                  soff.ctypes.data_as(I64), _dp(src), toff.ctypes.data_as(I64), _dp(tgt),
                                  out, err, 1024)
    if rc:
        e = LMError("planning failed (%d): %s" % (rc, err.value.decode()))
        e.code = rc
        raise e
    return int(out[0]), int(out[1])


def host_plan_stats(d, k, src, tgt=None, **params):
    lib = load_library()
    d, k = _medium(d, k)
    src = np.ascontiguousarray(np.asarray(src, dtype=np.float64).reshape(-1, 3))
    tgt = src if tgt is None else np.ascontiguousarray(np.asarray(tgt, dtype=np.float64).reshape(-1, 3))
    prm = make_params(**params)
    out = np.zeros(len(STAT_NAMES))
    err = ctypes.create_string_buffer(1024)
    rc = lib.lm_host_plan_stats(k.size, _dp(d), _dp(k), ctypes.byref(prm), src.shape[0], _dp(src),
                                tgt.shape[0], _dp(tgt), _dp(out), out.size, err, 1024)
    if rc:
        e = LMError("planning failed (%d): %s" % (rc, err.value.decode()))
        e.code = rc
        raise e
    return dict(zip(STAT_NAMES, out.tolist()))


def host_gmres_dense(A, b, x0=None, tol=1e-10, restart=30, max_iter=1000):
    """The solve's host logic on a dense complex system A x = b (host
    arrays; b of shape [n] or [n_rhs, n]); returns (x, iters, relres) with
    relres a float for one right-hand side, else an array [n_rhs]."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    n = A.shape[0]
    b = np.asarray(b, dtype=np.complex128)
    single = b.ndim == 1
    b = np.ascontiguousarray(b.reshape(-1, n))
    nr = b.shape[0]
    x = np.zeros((nr, n), dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128).reshape(nr, n)
    x = np.ascontiguousarray(x)
    it = ctypes.c_int()
    rr = np.zeros(nr)
    rc = load_library().lm_host_gmres_dense(n, nr, _dp(A.view(np.float64)), _dp(b.view(np.float64)),
                                            _dp(x.view(np.float64)), float(tol), int(restart), int(max_iter),
                                            ctypes.byref(it), _dp(rr))
    if rc:
        raise LMError("lm_host_gmres_dense failed (%d)" % rc)
    return (x[0], it.value, float(rr[0])) if single else (x, it.value, rr)


def selftest_math(x):
    """(sin, cos, refined 1/sqrt(x^2), library 1/sqrt(x^2), J0(|x|), J1(|x|))
    of a float64 CUDA tensor x by the near-field device routines; returns a
    [n, 6] tensor."""
    import torch
    lib = load_library()
    x = x.contiguous()
    out = torch.empty((x.numel(), 6), dtype=torch.float64, device=x.device)
    rc = lib.lm_selftest_math(x.numel(), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
    if rc:
        raise LMError("lm_selftest_math failed (%d)" % rc)
    return out
