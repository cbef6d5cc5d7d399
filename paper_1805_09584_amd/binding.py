"""ctypes binding of include/ndtm.h.  Same names as the C entry points."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

NDTM_OK = 0
NDTM_PREC_F64, NDTM_PREC_F32, NDTM_PREC_F16, NDTM_PREC_F32_H16 = 0, 1, 2, 3
(NDTM_OP_QHAT, NDTM_OP_QHAT2, NDTM_OP_SHAT_SHIFT, NDTM_OP_DFULL, NDTM_OP_HOP_EO,
 NDTM_OP_HOP_OE) = range(6)
NDTM_NMMS_AUTO = -1
NDTM_SMOOTH_MR, NDTM_SMOOTH_SAP = 0, 1
NDTM_GUESS_ZERO, NDTM_GUESS_LAGRANGE, NDTM_GUESS_MLP, NDTM_GUESS_PROJECTION, NDTM_GUESS_MMS = 0, 1, 2, 3, 4
PROF_CLASSES = ("hop_f64", "hop_f32", "hop_f16", "mms_update", "mms_resid", "restrict", "prolong",
                "coarse")
MAX_SHIFTS = 16
MLP_NFEAT, MLP_KMAX, MLP_NPARAM = 59, 11, 8715

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOCONV", -4: "EBREAKDOWN", -5: "ESTATE",
           -6: "EHIP"}


class NdtmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ndtm {_STATUS.get(code, code)}: {msg}")
        self.code = code


class MGParams(C.Structure):
    _fields_ = [("block", C.c_int * 4), ("n_vec", C.c_int), ("setup_iters", C.c_int),
                ("setup_smooth", C.c_int), ("setup_refine", C.c_int), ("setup_nd", C.c_int),
                ("smooth_iters", C.c_int), ("coarse_iters", C.c_int),
                ("coarse_mu_factor", C.c_double), ("seed", C.c_ulonglong), ("precision", C.c_int),
                ("coarse_tol", C.c_double), ("coarse_cycles", C.c_int), ("coarse_eo", C.c_int),
                ("keep_f64", C.c_int), ("pair_signs", C.c_int), ("smoother", C.c_int), ("sap_mr_iters", C.c_int),
                ("setup_prec", C.c_int)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("n_mmscg", C.c_int), ("guess", C.c_int),
                ("precision", C.c_int), ("poll_every", C.c_int), ("mg_tol", C.c_double),
                ("fgmres_restart", C.c_int), ("fgmres_maxiter", C.c_int), ("max_rounds", C.c_int),
                ("use_graphs", C.c_int), ("mms_defer", C.c_int),
                ("mms_predict", C.c_int)]


_D16 = C.c_double * MAX_SHIFTS
_I16 = C.c_int * MAX_SHIFTS


class SolveReport(C.Structure):
    _fields_ = [("status", C.c_int), ("n_shifts", C.c_int), ("mms_iterations", C.c_int),
                ("sigma", _D16), ("input_index", _I16), ("method", _I16), ("iterations", _I16),
                ("rounds", _I16), ("true_res", _D16), ("guess_res", _D16), ("lagrange_res", _D16),
                ("mlp_res", _D16), ("guess_kind", _I16), ("t_mms_ms", C.c_double),
                ("t_guess_ms", C.c_double), ("t_mg_ms", C.c_double), ("t_total_ms", C.c_double),
                ("hop_ms", C.c_double), ("hop_launches", C.c_longlong), ("n_mmscg", C.c_int),
                ("mms_it32", C.c_int), ("mms_it16", C.c_int)]

    def to_dict(self):
        n = self.n_shifts
        d = {k: getattr(self, k) for k in ("status", "n_shifts", "mms_iterations", "t_mms_ms", "t_guess_ms",
                                          "t_mg_ms", "t_total_ms", "hop_ms", "hop_launches", "n_mmscg",
                                          "mms_it32", "mms_it16")}
        for k in ("sigma", "input_index", "method", "iterations", "rounds", "true_res", "guess_res",
                  "lagrange_res", "mlp_res", "guess_kind"):
            d[k] = list(getattr(self, k)[:n])
        return d


def lib_path():
    return os.path.join(_HERE, "libndtm.so")


def load_library():
    """Loads libndtm.so; raises if it is missing (there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or "
                           "python paper_1805_09584_amd/build.py")
    lib = C.CDLL(path)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    fp = C.POINTER(C.c_float)
    sig = {
        "ndtm_create": (i, [C.POINTER(C.c_int), i, i, C.POINTER(vp)]),
        "ndtm_destroy": (None, [vp]),
        "ndtm_last_error": (C.c_char_p, [vp]),
        "ndtm_half_volume": (C.c_longlong, [vp]),
        "ndtm_set_gauge": (i, [vp, vp, vp]),
        "ndtm_set_params": (i, [vp, d, d, d]),
        "ndtm_set_shifts": (i, [vp, i, C.POINTER(C.c_double)]),
        "ndtm_set_clover": (i, [vp, d]),
        "ndtm_apply": (i, [vp, i, i, vp, vp, d, vp]),
        "ndtm_mg_default_params": (None, [C.POINTER(MGParams)]),
        "ndtm_mg_setup": (i, [vp, C.POINTER(MGParams), vp, vp]),
        "ndtm_mg_coarse_volume": (C.c_longlong, [vp]),
        "ndtm_mg_restrict": (i, [vp, vp, vp, vp]),
        "ndtm_mg_prolong": (i, [vp, vp, vp, vp]),
        "ndtm_mg_transfer_cycle": (i, [vp, i, vp, vp, vp]),
        "ndtm_mg_smooth": (i, [vp, vp, vp, d, vp]),
        "ndtm_mg_cycle": (i, [vp, vp, vp, d, vp]),
        "ndtm_mg_coarse_apply": (i, [vp, vp, vp, d, vp]),
        "ndtm_mg_coarse_solve": (i, [vp, vp, vp, d, vp]),
        "ndtm_mg_coarse_apply_multi": (i, [vp, vp, vp, i, C.POINTER(C.c_double), vp]),
        "ndtm_mg_coarse_solve_multi": (i, [vp, vp, vp, i, C.POINTER(C.c_double), vp]),
        "ndtm_solve_default_params": (None, [C.POINTER(SolveParams)]),
        "ndtm_solve": (i, [vp, C.POINTER(vp), vp, C.POINTER(SolveParams), C.POINTER(SolveReport), vp]),
        "ndtm_zolotarev": (i, [i, d, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "ndtm_hybrid_split": (i, [i, C.POINTER(C.c_double), d, d, d, d, d, C.POINTER(C.c_int)]),
        "ndtm_spectrum_estimate": (i, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "ndtm_solve_rational": (i, [vp, vp, vp, i, d, d, C.POINTER(SolveParams), C.POINTER(SolveReport), vp]),
        "ndtm_mlp_set_weights": (i, [vp, fp, C.c_size_t]),
        "ndtm_mlp_get_weights": (i, [vp, fp, C.c_size_t]),
        "ndtm_mlp_forward": (i, [vp, i, fp, fp, fp, fp, i, fp, fp]),
        "ndtm_mlp_grad": (i, [vp, i, fp, fp, fp, fp, fp, fp]),
        "ndtm_mlp_train": (i, [vp, i, fp, fp, fp, fp, i, C.c_float, fp]),
        "ndtm_mlp_sample": (i, [vp, i, C.POINTER(vp), C.POINTER(C.c_double), d, vp, fp, fp, fp, fp,
                                C.POINTER(C.c_double), vp]),
        "ndtm_stream_bandwidth": (i, [vp, C.c_size_t, i, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
        "ndtm_workspace_bytes": (i, [vp, i, C.POINTER(MGParams), C.POINTER(SolveParams),
                                     C.POINTER(C.c_size_t)]),
        "ndtm_set_workspace": (i, [vp, vp, C.c_size_t]),
        "ndtm_trim": (i, [vp]),
        "ndtm_set_stencil_tile": (i, [vp, i, i]),
        "ndtm_apply_noalloc": (i, [vp, i, vp, vp, d, vp]),
        "ndtm_apply_noalloc_max_bytes": (C.c_size_t, []),
        "ndtm_workspace_stats": (i, [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                     C.POINTER(C.c_longlong)]),
        "ndtm_profile_moved": (i, [vp, i, C.POINTER(C.c_double)]),
        "ndtm_profile_enable": (i, [vp, i]),
        "ndtm_profile_read": (i, [vp, i, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                                  C.POINTER(C.c_double), i]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def zolotarev(n, eps):
    """(c_1..c_2n, a, delta) of Zolotarev's approximation of 1/sqrt(y) on [eps, 1] (host)."""
    c = (C.c_double * max(2 * n, 1))()
    a, d = C.c_double(), C.c_double()
    rc = load_library().ndtm_zolotarev(int(n), float(eps), c, C.byref(a), C.byref(d))
    if rc != 0:
        raise NdtmError(rc, "ndtm_zolotarev: bad order or interval")
    return np.array(c[:2 * n]), a.value, d.value


def hybrid_split(sigma_desc, lambda_min, lambda_max, tol, ms_per_iteration, ms_per_mg_shift):
    """n of the section 4.4 cost model (host computation)."""
    sig = (C.c_double * len(sigma_desc))(*[float(v) for v in sigma_desc])
    n = C.c_int()
    rc = load_library().ndtm_hybrid_split(len(sigma_desc), sig, float(lambda_min), float(lambda_max), float(tol),
                                          float(ms_per_iteration), float(ms_per_mg_shift), C.byref(n))
    if rc != 0:
        raise NdtmError(rc, "ndtm_hybrid_split: inconsistent arguments")
    return n.value


def _fp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    assert t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous(), "need a contiguous complex128 CUDA tensor"
    return C.c_void_p(t.data_ptr())


class Context:
    """One lattice on one GPU (ndtm_create .. ndtm_destroy)."""

    def __init__(self, dims, bc_flags=0, device=0):
        self.lib = load_library()
        self.dims = tuple(int(x) for x in dims)
        self.device = device
        h = C.c_void_p()
        arr = (C.c_int * 4)(*self.dims)
        rc = self.lib.ndtm_create(arr, bc_flags, device, C.byref(h))
        if rc != NDTM_OK:
            raise NdtmError(rc, "ndtm_create failed")
        self.h = h
        self.V = 1
        for x in self.dims:
            self.V *= x
        self.vh = self.V // 2

    def close(self):
        if getattr(self, "h", None):
            self.lib.ndtm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != NDTM_OK:
            msg = self.lib.ndtm_last_error(self.h)
            raise NdtmError(rc, msg.decode() if msg else "")
        return rc

    # -- setup ----------------------------------------------------------------
    def ndtm_set_gauge(self, U):
        """U: complex128 CUDA tensor (V, 4, 3, 3)."""
        assert U.numel() == self.V * 36
        self._check(self.lib.ndtm_set_gauge(self.h, _ptr(U), _stream()))

    def ndtm_set_params(self, kappa, mubar, epsbar):
        self._check(self.lib.ndtm_set_params(self.h, kappa, mubar, epsbar))

    def ndtm_set_clover(self, csw):
        self._check(self.lib.ndtm_set_clover(self.h, float(csw)))

    def ndtm_set_shifts(self, sigma):
        arr = (C.c_double * len(sigma))(*[float(s) for s in sigma])
        self._check(self.lib.ndtm_set_shifts(self.h, len(sigma), arr))
        self.n_shifts = len(sigma)

    # -- device storage -------------------------------------------------------
    def ndtm_workspace_bytes(self, n_shifts, mg_params=None, solve_params=None):
        nb = C.c_size_t()
        self._check(self.lib.ndtm_workspace_bytes(
            self.h, int(n_shifts), C.byref(mg_params) if mg_params is not None else None,
            C.byref(solve_params) if solve_params is not None else None, C.byref(nb)))
        return nb.value

    def ndtm_set_workspace(self, region):
        """region: a CUDA tensor the caller keeps alive (None: back to hipMalloc storage)."""
        if region is None:
            self._check(self.lib.ndtm_set_workspace(self.h, None, 0))
            self._region = None
            return
        assert region.is_cuda and region.is_contiguous()
        self._check(self.lib.ndtm_set_workspace(self.h, C.c_void_p(region.data_ptr()),
                                                region.numel() * region.element_size()))
        self._region = region

    def ndtm_set_stencil_tile(self, bz, by=0):
        self._check(self.lib.ndtm_set_stencil_tile(self.h, int(bz), int(by)))

    def ndtm_trim(self):
        self._check(self.lib.ndtm_trim(self.h))

    def ndtm_workspace_stats(self):
        live, peak, n = C.c_size_t(), C.c_size_t(), C.c_longlong()
        self._check(self.lib.ndtm_workspace_stats(self.h, C.byref(live), C.byref(peak), C.byref(n)))
        return {"live": live.value, "peak": peak.value, "device_allocs": n.value}

    # -- operators ------------------------------------------------------------
    def ndtm_apply(self, op, x, param=0.0, prec=NDTM_PREC_F64, out=None):
        if out is None:
            out = torch.empty_like(x)
        self._check(self.lib.ndtm_apply(self.h, op, prec, _ptr(out), _ptr(x), float(param), _stream()))
        return out

    def ndtm_apply_noalloc(self, op, x, param=0.0, out=None):
        """ndtm_apply in FP64 with the library's fixed scratch array (no device allocation)."""
        if out is None:
            out = torch.empty_like(x)
        self._check(self.lib.ndtm_apply_noalloc(self.h, op, _ptr(out), _ptr(x), float(param), _stream()))
        return out

    # -- multigrid ------------------------------------------------------------
    @staticmethod
    def mg_params(**kw):
        p = MGParams()
        load_library().ndtm_mg_default_params(C.byref(p))
        for k, v in kw.items():
            if k == "block":
                p.block = (C.c_int * 4)(*v)
            else:
                setattr(p, k, v)
        return p

    def ndtm_mg_setup(self, params=None, test_vectors=None):
        p = params if params is not None else self.mg_params()
        tv = _ptr(test_vectors) if test_vectors is not None else None
        self._check(self.lib.ndtm_mg_setup(self.h, C.byref(p), tv, _stream()))
        self.Vc = int(self.lib.ndtm_mg_coarse_volume(self.h))
        self.n_vec = p.n_vec

    def ndtm_mg_restrict(self, v):
        out = torch.empty((self.Vc, 2, 2 * self.n_vec), dtype=torch.complex128, device=v.device)
        self._check(self.lib.ndtm_mg_restrict(self.h, _ptr(out), _ptr(v), _stream()))
        return out

    def ndtm_mg_prolong(self, vc):
        out = torch.empty((self.V, 2, 4, 3), dtype=torch.complex128, device=vc.device)
        self._check(self.lib.ndtm_mg_prolong(self.h, _ptr(out), _ptr(vc), _stream()))
        return out

    def ndtm_mg_transfer_cycle(self, direction, x):
        """direction 0: restriction of a full-lattice field; 1: prolongation of a coarse one,
        both as the cycle runs them (its precision and storage of P)."""
        if direction == 0:
            out = torch.empty((self.Vc, 2, 2 * self.n_vec), dtype=torch.complex128, device=x.device)
        else:
            out = torch.empty((self.V, 2, 4, 3), dtype=torch.complex128, device=x.device)
        self._check(self.lib.ndtm_mg_transfer_cycle(self.h, int(direction), _ptr(out), _ptr(x), _stream()))
        return out

    def ndtm_mg_cycle(self, r, m=0.0):
        """One two-level cycle for D'(m) z = r (full-lattice doublet); returns z."""
        out = torch.empty_like(r)
        self._check(self.lib.ndtm_mg_cycle(self.h, _ptr(out), _ptr(r), float(m), _stream()))
        return out

    def ndtm_mg_smooth(self, z, r, m=0.0):
        """The cycle's post-smoother on D'(m) z = r from z (full-lattice doublets); returns the
        smoothed z (a new tensor; the argument is not changed)."""
        out = z.clone()
        self._check(self.lib.ndtm_mg_smooth(self.h, _ptr(out), _ptr(r), float(m), _stream()))
        return out

    def ndtm_mg_coarse_apply(self, xc, m=0.0):
        out = torch.empty_like(xc)
        self._check(self.lib.ndtm_mg_coarse_apply(self.h, _ptr(out), _ptr(xc), float(m), _stream()))
        return out

    def ndtm_mg_coarse_apply_multi(self, xc, ms, out=None):
        """D'_c(m_r) x_r for the k systems stacked in xc (complex128 CUDA (k, Vc, 2, 2Nv))."""
        k = xc.shape[0]
        mm = (C.c_double * k)(*[float(v) for v in ms])
        y = torch.empty_like(xc) if out is None else out
        self._check(self.lib.ndtm_mg_coarse_apply_multi(self.h, _ptr(y), _ptr(xc), int(k), mm, _stream()))
        return y

    def ndtm_mg_coarse_solve(self, bc, m=0.0):
        out = torch.empty_like(bc)
        self._check(self.lib.ndtm_mg_coarse_solve(self.h, _ptr(out), _ptr(bc), float(m), _stream()))
        return out

    def ndtm_mg_coarse_solve_multi(self, bc, ms, out=None):
        """D'_c(m_r)^-1 b_r for the k systems stacked in bc (complex128 CUDA (k, Vc, 2, 2Nv)), FP64."""
        k = bc.shape[0]
        mm = (C.c_double * k)(*[float(v) for v in ms])
        x = torch.empty_like(bc) if out is None else out
        self._check(self.lib.ndtm_mg_coarse_solve_multi(self.h, _ptr(x), _ptr(bc), int(k), mm, _stream()))
        return x

    # -- solve ----------------------------------------------------------------
    @staticmethod
    def solve_params(**kw):
        p = SolveParams()
        load_library().ndtm_solve_default_params(C.byref(p))
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    def ndtm_solve(self, b, params=None, xs=None, check=True):
        """Solves all shifts for b (complex128 CUDA (V/2,2,4,3)); returns (xs, report dict)."""
        p = params if params is not None else self.solve_params()
        if xs is None:
            xs = [torch.empty_like(b) for _ in range(self.n_shifts)]
        arr = (C.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        rep = SolveReport()
        rc = self.lib.ndtm_solve(self.h, arr, _ptr(b), C.byref(p), C.byref(rep), _stream())
        if check:
            self._check(rc)
        d = rep.to_dict()
        d["rc"] = rc
        return xs, d

    def ndtm_spectrum_estimate(self):
        """(lambda_min, lambda_max) of Q^2 from the last FP64 multi-shift solve's Lanczos matrix."""
        lo, hi = C.c_double(), C.c_double()
        self._check(self.lib.ndtm_spectrum_estimate(self.h, C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    # -- rational approximation -----------------------------------------------
    def ndtm_solve_rational(self, b, n, eps, lam, params=None, check=True):
        """y ~ (Q^2)^{-1/2} b by the order-n Zolotarev approximation on [eps lam, lam];
        the context's shifts become the approximation's.  Returns (y, report dict)."""
        p = params if params is not None else self.solve_params()
        y = torch.empty_like(b)
        rep = SolveReport()
        rc = self.lib.ndtm_solve_rational(self.h, _ptr(y), _ptr(b), int(n), float(eps), float(lam), C.byref(p),
                                          C.byref(rep), _stream())
        if check:
            self._check(rc)
        self.n_shifts = int(n)
        d = rep.to_dict()
        d["rc"] = rc
        return y, d

    # -- learned guess proposer -----------------------------------------------
    def ndtm_mlp_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(self.lib.ndtm_mlp_set_weights(self.h, _fp(w), w.size))

    def ndtm_mlp_get_weights(self):
        w = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(self.lib.ndtm_mlp_get_weights(self.h, _fp(w), w.size))
        return w

    def ndtm_mlp_forward(self, feat, mask=None, G=None, h=None, bf16=False):
        feat = np.ascontiguousarray(feat, dtype=np.float32)
        B = feat.shape[0]
        y = np.zeros((B, MLP_KMAX), dtype=np.float32)
        loss = np.zeros(B, dtype=np.float32)
        arr = [None if a is None else np.ascontiguousarray(a, dtype=np.float32) for a in (mask, G, h)]
        self._check(self.lib.ndtm_mlp_forward(self.h, B, _fp(feat), *[_fp(a) for a in arr], 1 if bf16 else 0,
                                              _fp(y), _fp(loss)))
        return y, loss

    def ndtm_mlp_grad(self, feat, mask, G, h):
        arr = [np.ascontiguousarray(a, dtype=np.float32) for a in (feat, mask, G, h)]
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        m = np.zeros(1, dtype=np.float32)
        self._check(self.lib.ndtm_mlp_grad(self.h, arr[0].shape[0], *[_fp(a) for a in arr], _fp(g), _fp(m)))
        return g, float(m[0])

    def ndtm_mlp_train(self, feat, mask, G, h, steps, lr):
        arr = [np.ascontiguousarray(a, dtype=np.float32) for a in (feat, mask, G, h)]
        hist = np.zeros(steps, dtype=np.float32)
        self._check(self.lib.ndtm_mlp_train(self.h, arr[0].shape[0], *[_fp(a) for a in arr], steps, float(lr),
                                            _fp(hist)))
        return hist

    def ndtm_mlp_sample(self, xs, nodes, sig_t, b):
        K = len(xs)
        ptrs = (C.c_void_p * K)(*[x.data_ptr() for x in xs])
        nd_ = (C.c_double * K)(*[float(s) for s in nodes])
        feat = np.zeros(MLP_NFEAT, dtype=np.float32)
        mask = np.zeros(MLP_KMAX, dtype=np.float32)
        G = np.zeros((MLP_KMAX, MLP_KMAX), dtype=np.float32)
        h = np.zeros(MLP_KMAX, dtype=np.float32)
        info = (C.c_double * 4)()
        self._check(self.lib.ndtm_mlp_sample(self.h, K, ptrs, nd_, float(sig_t), _ptr(b), _fp(feat), _fp(mask),
                                             _fp(G), _fp(h), info, _stream()))
        return feat, mask, G, h, list(info)

    # -- profiling --------------------------------------------------------------
    def ndtm_stream_bandwidth(self, nbytes=1 << 30, reps=10):
        """(copy, read, write) GB/s of the streaming reference kernels on this device."""
        out = [C.c_double(), C.c_double(), C.c_double()]
        self._check(self.lib.ndtm_stream_bandwidth(self.h, nbytes, reps, *[C.byref(o) for o in out]))
        return tuple(o.value for o in out)

    def ndtm_profile_enable(self, mask=0xFF):
        """Bit k of mask enables event timing of kernel class k (PROF_CLASSES); 0 disables."""
        self._check(self.lib.ndtm_profile_enable(self.h, int(mask)))

    def ndtm_profile_read(self, kernel_class=0, reset=False):
        """(milliseconds, launches, algorithmic bytes) of one kernel class since the last reset."""
        ms = C.c_double()
        n = C.c_longlong()
        by = C.c_double()
        self._check(self.lib.ndtm_profile_read(self.h, kernel_class, C.byref(ms), C.byref(n), C.byref(by),
                                               1 if reset else 0))
        return ms.value, n.value, by.value

    def ndtm_profile_moved(self, kernel_class=0):
        """Bytes moved by the class's timed launches (algorithmic + fused epilogue vectors)."""
        mv = C.c_double()
        self._check(self.lib.ndtm_profile_moved(self.h, kernel_class, C.byref(mv)))
        return mv.value
