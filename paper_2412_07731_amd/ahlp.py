"""ctypes binding of libahlp.so (declared in include/ahlp.h).

Only argument marshalling lives here: every step of the Newton solve and of the
interior-point loop runs in the library's HIP kernels.  PyTorch supplies device
memory and the stream.  There is no fallback: if the library is missing or no
GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libahlp.so")

FP64, FP32_REFINE = 0, 1
STATUS = {0: "ok", -1: "einval", -2: "enomem", -3: "ehip", -4: "estate", -5: "enumeric",
          1: "wmaxiter", 2: "wstall"}
STAGES = ["prep", "syrk", "factor", "schur", "tfactor", "solve", "resid", "arows"]

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class Desc(C.Structure):
    _fields_ = [("N", C.c_int32), ("n0", C.c_int32), ("m", _i32p), ("n", _i32p), ("l", _i32p),
                ("A", _f64p), ("C", _f64p), ("FR", _f64p), ("FL", _f64p), ("F0", _f64p),
                ("b", _f64p), ("c", _f64p), ("ng", C.c_int32), ("Wg", _f64p), ("Wg0", _f64p),
                ("ub", _f64p)]


class FactorOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("rho", C.c_double), ("delta", C.c_double)]


class IpmOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("eta", C.c_double),
                ("rho", C.c_double), ("delta", C.c_double), ("max_refine", C.c_int32),
                ("refine_tol", C.c_double), ("precision", C.c_int), ("mu_switch", C.c_double),
                ("start", C.c_int32), ("verbose", C.c_int32), ("timing", C.c_int32),
                ("fp32_accept", C.c_double), ("graph", C.c_int32), ("gondzio", C.c_int32)]


class IpmResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("refine_steps", C.c_int32),
                ("pivots_modified", C.c_int32), ("fp32_iterations", C.c_int32),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double), ("rel_gap", C.c_double),
                ("rel_pinf", C.c_double), ("rel_dinf", C.c_double), ("mu", C.c_double),
                ("max_bkerr", C.c_double), ("t_total_ms", C.c_double),
                ("t_stage_ms", C.c_double * 8), ("n_stage", C.c_int32 * 8),
                ("rows_bytes", C.c_double), ("correctors", C.c_int32),
                ("start_bkerr", C.c_double * 2), ("t_stage32_ms", C.c_double * 8),
                ("n_stage32", C.c_int32 * 8)]


class IpmIter(C.Structure):
    _fields_ = [("mu", C.c_double), ("sigma", C.c_double), ("alpha_p", C.c_double),
                ("alpha_d", C.c_double), ("bkerr_pred", C.c_double), ("bkerr_corr", C.c_double),
                ("refine_pred", C.c_int32), ("refine_corr", C.c_int32), ("fp32", C.c_int32),
                ("correctors", C.c_int32)]


# Every exported symbol with its signature (argtypes, restype).
SIGNATURES = {
    "ahlp_ipm_default_opts": ([C.POINTER(IpmOpts)], None),
    "ahlp_problem_create": ([C.POINTER(Desc), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "ahlp_problem_destroy": ([C.c_void_p], C.c_int),
    "ahlp_kkt_factor": ([C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(FactorOpts), C.c_void_p],
                        C.c_int),
    "ahlp_kkt_solve": ([C.c_void_p] + [C.c_void_p] * 6 + [C.c_int32, C.c_double,
                                                          C.POINTER(C.c_double), C.c_void_p],
                       C.c_int),
    "ahlp_kkt_solve_noalloc": ([C.c_void_p] + [C.c_void_p] * 6 + [C.c_int32, C.c_double,
                                                                  C.POINTER(C.c_double), C.c_void_p],
                               C.c_int),
    "ahlp_kkt_adjoint": ([C.c_void_p] + [C.c_void_p] * 6 + [C.c_int32, C.c_double,
                                                            C.POINTER(C.c_double), C.c_void_p],
                         C.c_int),
    "ahlp_lp_gradient": ([C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_int32,
                          C.c_double, C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "ahlp_problem_set_bc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "ahlp_problem_set_launch": ([C.c_void_p, C.c_int32], C.c_int),
    "ahlp_autotune": ([C.c_void_p, C.c_char_p, C.POINTER(C.c_int32), C.c_void_p], C.c_int),
    "ahlp_ipm_solve": ([C.c_void_p, C.POINTER(IpmOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                        C.POINTER(IpmResult), C.c_void_p], C.c_int),
    "ahlp_ipm_history": ([C.c_void_p, C.POINTER(IpmIter), C.c_int32, C.POINTER(C.c_int32)],
                         C.c_int),
    "ahlp_kkt_factor_bounded": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.POINTER(FactorOpts), C.c_void_p], C.c_int),
    "ahlp_ipm_bound_duals": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "ahlp_last_error": ([], C.c_char_p),
    "ahlp_problem_sizes": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                            C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int),
    "ahlp_debug_block": ([C.c_void_p, C.c_int32, _f64p, _f64p], C.c_int),
    "ahlp_debug_schur": ([C.c_void_p, _f64p], C.c_int),
    "ahlp_debug_pivots": ([C.c_void_p, C.POINTER(C.c_int32)], C.c_int),
    "ahlp_ceiling_mfma": ([C.c_int32, C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "ahlp_ceiling_hbm_read": ([C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "ahlp_ceiling_tile_chol": ([C.c_int32, C.POINTER(C.c_double), C.c_void_p], C.c_int),
}

_lib = None


class AHLPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


def lib():
    """Load libahlp.so (built by paper_2412_07731_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run python -m paper_2412_07731_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code, allow_warn=False):
    if code == 0 or (allow_warn and code > 0):
        return code
    raise AHLPError(code, lib().ahlp_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(_f64p) if a is not None else None


def _cat(blocks):
    if not blocks:
        return np.zeros(1)
    return np.ascontiguousarray(np.concatenate([np.ascontiguousarray(b, dtype=np.float64).ravel()
                                                for b in blocks]))


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "need contiguous cuda float64"
    return C.c_void_p(t.data_ptr())


def ceiling_mfma(precision=FP64, stream=None):
    """ahlp_ceiling_mfma: the device's measured MFMA throughput (TFLOP/s) for
    the instruction the factorization uses in this precision."""
    v = C.c_double()
    _check(lib().ahlp_ceiling_mfma(int(precision), C.byref(v), _stream(stream)))
    return v.value


def ceiling_hbm_read(buf, stream=None):
    """ahlp_ceiling_hbm_read: streaming read bandwidth (GB/s) over the
    contiguous cuda float64 tensor buf (make it a GiB or more)."""
    v = C.c_double()
    _check(lib().ahlp_ceiling_hbm_read(_dptr(buf), int(buf.numel()), C.byref(v), _stream(stream)))
    return v.value


def ceiling_tile_chol(beside_mfma=False, stream=None):
    """ahlp_ceiling_tile_chol: microseconds per one-wave FP64 tile Cholesky,
    alone on its SIMD or beside a wave that streams FP64 MFMAs."""
    v = C.c_double()
    _check(lib().ahlp_ceiling_tile_chol(int(bool(beside_mfma)), C.byref(v), _stream(stream)))
    return v.value


class Problem:
    """A packed arrowhead LP on the current HIP device (see include/ahlp.h)."""

    def __init__(self, inst, stream=None):
        L = lib()
        self.N, self.n0 = int(inst.N), int(inst.n0)
        Wg_list = getattr(inst, "Wg", None)
        self.ng = 0 if Wg_list is None else int(Wg_list[0].shape[0])
        m = np.ascontiguousarray(inst.m, dtype=np.int32)
        n = np.ascontiguousarray(inst.n, dtype=np.int32)
        l = np.ascontiguousarray(inst.l if len(inst.l) else np.zeros(1), dtype=np.int32)
        A = _cat(inst.A)
        Cm = _cat(inst.C) if self.n0 > 0 else None
        FR, FL = _cat(inst.FR), _cat(inst.FL)
        F0 = np.ascontiguousarray(inst.F0, dtype=np.float64) if inst.F0 is not None else None
        b = np.ascontiguousarray(inst.b, dtype=np.float64)
        c = np.ascontiguousarray(inst.c, dtype=np.float64)
        Wg = _cat(Wg_list) if self.ng > 0 else None
        Wg0 = (np.ascontiguousarray(inst.Wg0, dtype=np.float64)
               if self.ng > 0 and self.n0 > 0 and inst.Wg0 is not None else None)
        ubv = getattr(inst, "ub", None)
        ub = np.ascontiguousarray(ubv, dtype=np.float64) if ubv is not None else None
        self.bounded = ub is not None and bool(np.isfinite(ub).any())
        self._keep = (m, n, l, A, Cm, FR, FL, F0, b, c, Wg, Wg0, ub)
        d = Desc(self.N, self.n0, m.ctypes.data_as(_i32p), n.ctypes.data_as(_i32p),
                 l.ctypes.data_as(_i32p), _ptr(A), _ptr(Cm), _ptr(FR), _ptr(FL), _ptr(F0),
                 _ptr(b), _ptr(c), self.ng, _ptr(Wg), _ptr(Wg0), _ptr(ub))
        h = C.c_void_p()
        _check(L.ahlp_problem_create(C.byref(d), _stream(stream), C.byref(h)))
        self._keep = None
        self.h = h
        nt, mt, nl, n0 = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(L.ahlp_problem_sizes(h, C.byref(nt), C.byref(mt), C.byref(nl), C.byref(n0)))
        self.n_tot, self.m_tot, self.n_link = nt.value, mt.value, nl.value
        self.m = m.copy()
        self.kdims = [int((inst.l[i - 1] if i >= 1 else 0) + (inst.l[i] if i < self.N - 1 else 0)
                          + self.ng + self.n0) for i in range(self.N)]

    def close(self):
        if getattr(self, "h", None):
            lib().ahlp_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- calls
    def factor(self, x, z, rho=0.0, delta=0.0, precision=FP64, stream=None):
        o = FactorOpts(precision, rho, delta)
        _check(lib().ahlp_kkt_factor(self.h, _dptr(x), _dptr(z), C.byref(o), _stream(stream)))

    def factor_bounded(self, x, z, q, rho=0.0, delta=0.0, precision=FP64, stream=None):
        """ahlp_kkt_factor_bounded: the factorization with Q = diag(q) in the
        (x, x) block (upper bounds inside the iteration, q = w / s)."""
        o = FactorOpts(precision, rho, delta)
        _check(lib().ahlp_kkt_factor_bounded(self.h, _dptr(x), _dptr(z), _dptr(q), C.byref(o),
                                             _stream(stream)))

    def bound_duals(self, stream=None):
        """(s, w) of the last ipm() on a problem with upper bounds (device tensors)."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        s = torch.empty(self.n_tot, dtype=torch.float64, device=dev)
        w = torch.empty_like(s)
        _check(lib().ahlp_ipm_bound_duals(self.h, _dptr(s), _dptr(w), _stream(stream)))
        return s, w

    def solve(self, rx, ry, rz, max_refine=0, refine_tol=1e-10, stream=None, out=None):
        import torch
        if out is None:
            out = (torch.empty_like(rx), torch.empty_like(ry), torch.empty_like(rz))
        dx, dy, dz = out
        be = C.c_double(-1.0)
        _check(lib().ahlp_kkt_solve(self.h, _dptr(rx), _dptr(ry), _dptr(rz), _dptr(dx), _dptr(dy),
                                    _dptr(dz), int(max_refine), float(refine_tol), C.byref(be),
                                    _stream(stream)))
        return dx, dy, dz, be.value

    def solve_noalloc(self, rx, ry, rz, max_refine=0, refine_tol=1e-10, stream=None, out=None):
        """ahlp_kkt_solve_noalloc: the solve with its workspace in the library's
        static device array (no allocation in the call; the outputs are the
        caller's)."""
        import torch
        if out is None:
            out = (torch.empty_like(rx), torch.empty_like(ry), torch.empty_like(rz))
        dx, dy, dz = out
        be = C.c_double(-1.0)
        _check(lib().ahlp_kkt_solve_noalloc(self.h, _dptr(rx), _dptr(ry), _dptr(rz), _dptr(dx),
                                            _dptr(dy), _dptr(dz), int(max_refine),
                                            float(refine_tol), C.byref(be), _stream(stream)))
        return dx, dy, dz, be.value

    def adjoint(self, gx, gy, gz, max_refine=0, refine_tol=1e-10, stream=None, out=None):
        """(wx, wy, wz, bkerr) with K' w = g at the last factorization (ahlp_kkt_adjoint)."""
        import torch
        if out is None:
            out = (torch.empty_like(gx), torch.empty_like(gy), torch.empty_like(gz))
        wx, wy, wz = out
        be = C.c_double(-1.0)
        _check(lib().ahlp_kkt_adjoint(self.h, _dptr(gx), _dptr(gy), _dptr(gz), _dptr(wx),
                                      _dptr(wy), _dptr(wz), int(max_refine), float(refine_tol),
                                      C.byref(be), _stream(stream)))
        return wx, wy, wz, be.value

    def lp_gradient(self, gx, gf, max_refine=10, refine_tol=1e-12, stream=None, out=None):
        """(dL/db, dL/dc, bkerr) for L(x*, f*) with dL/dx* = gx (device tensor or
        None) and dL/df* = gf (a number) at the last factorization (ahlp_lp_gradient)."""
        import torch
        if out is None:
            dev = torch.device("cuda", torch.cuda.current_device())
            out = (torch.empty(self.m_tot, dtype=torch.float64, device=dev),
                   torch.empty(self.n_tot, dtype=torch.float64, device=dev))
        gb, gc = out
        be = C.c_double(-1.0)
        _check(lib().ahlp_lp_gradient(self.h, _dptr(gx) if gx is not None else None, float(gf),
                                      _dptr(gb), _dptr(gc), int(max_refine), float(refine_tol),
                                      C.byref(be), _stream(stream)))
        return gb, gc, be.value

    def autotune(self, cache_path=None, stream=None):
        """Pick the block-factor kernel per bordered tile-row count (ahlp_autotune);
        returns how many counts were measured (0: all from the cache)."""
        n = C.c_int32(0)
        path = cache_path.encode() if cache_path else None
        _check(lib().ahlp_autotune(self.h, path, C.byref(n), _stream(stream)))
        return n.value

    LAUNCH_MODES = {"batched": 0, "per_block": 1, "fused": 2}

    def set_launch(self, per_block=False, mode=None):
        """How the per-block factorization stages are launched
        (ahlp_problem_set_launch): mode "batched" (the default: one launch per
        stage over all blocks), "per_block" or "fused" (the panel bucket in one
        persistent launch); per_block=True means "per_block"."""
        m = self.LAUNCH_MODES[mode] if mode is not None else (1 if per_block else 0)
        _check(lib().ahlp_problem_set_launch(self.h, m))

    def set_bc(self, b, c, stream=None):
        """Replace the LP's b and c with device vectors (ahlp_problem_set_bc)."""
        _check(lib().ahlp_problem_set_bc(self.h, _dptr(b), _dptr(c), _stream(stream)))

    def ipm(self, x=None, y=None, z=None, stream=None, **opts):
        import torch
        o = IpmOpts()
        lib().ahlp_ipm_default_opts(C.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        dev = torch.device("cuda", torch.cuda.current_device())
        x = x if x is not None else torch.zeros(self.n_tot, dtype=torch.float64, device=dev)
        y = y if y is not None else torch.zeros(self.m_tot, dtype=torch.float64, device=dev)
        z = z if z is not None else torch.zeros(self.n_tot, dtype=torch.float64, device=dev)
        r = IpmResult()
        code = lib().ahlp_ipm_solve(self.h, C.byref(o), _dptr(x), _dptr(y), _dptr(z), C.byref(r),
                                    _stream(stream))
        _check(code, allow_warn=True)
        res = {f: getattr(r, f) for f, _ in IpmResult._fields_
               if f not in ("t_stage_ms", "n_stage", "start_bkerr", "t_stage32_ms", "n_stage32")}
        res["start_bkerr"] = [r.start_bkerr[0], r.start_bkerr[1]]
        res["t_stage32_ms"] = {STAGES[i]: r.t_stage32_ms[i] for i in range(8)}
        res["n_stage32"] = {STAGES[i]: r.n_stage32[i] for i in range(8)}
        res["status_name"] = STATUS.get(code, str(code))
        res["t_stage_ms"] = {STAGES[i]: r.t_stage_ms[i] for i in range(8)}
        res["n_stage"] = {STAGES[i]: r.n_stage[i] for i in range(8)}
        return x, y, z, res

    def history(self):
        """Per-iteration records of the last ipm() (ahlp_ipm_history), as dicts."""
        cnt = C.c_int32(0)
        _check(lib().ahlp_ipm_history(self.h, None, 0, C.byref(cnt)))
        buf = (IpmIter * max(cnt.value, 1))()
        _check(lib().ahlp_ipm_history(self.h, buf, cnt.value, C.byref(cnt)))
        return [{f: getattr(buf[i], f) for f, _ in IpmIter._fields_} for i in range(cnt.value)]

    # --- inspection
    def debug_block(self, i):
        mi, k = int(self.m[i]), self.kdims[i]
        Lm = np.zeros((mi, mi))
        W = np.zeros((mi, max(k, 1)))
        _check(lib().ahlp_debug_block(self.h, int(i), Lm.ctypes.data_as(_f64p), W.ctypes.data_as(_f64p)))
        return Lm, W[:, :k]

    def debug_schur(self):
        dim = self.n_link + self.ng + self.n0
        S = np.zeros((max(dim, 1), max(dim, 1)))
        _check(lib().ahlp_debug_schur(self.h, S.ctypes.data_as(_f64p)))
        return S[:dim, :dim]

    def pivots(self):
        c = C.c_int32()
        _check(lib().ahlp_debug_pivots(self.h, C.byref(c)))
        return c.value
