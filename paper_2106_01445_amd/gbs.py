"""ctypes binding of libgbs.so (include/gbs.h).  Argument marshalling only: every
step of the computation runs in the HIP kernels behind the C ABI.

Host-array calls take numpy arrays; the *_dev calls take torch CUDA tensors (or
raw device pointers) and are ordered on the context's stream.  There is no CPU
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbs.so")

GBS_OK, GBS_E_INVAL, GBS_E_NOTPD, GBS_E_NOMEM, GBS_E_HIP, GBS_E_STATE, GBS_W_PATTERN = 0, -1, -2, -3, -4, -5, 1
GBS_PREC_FP64, GBS_PREC_MIXED = 0, 1
GBS_PS_FIT_NOCONV, GBS_PS_CONTOUR, GBS_PS_PIVOT, GBS_PS_ESCALATED, GBS_PS_CANCEL, GBS_PS_BADROW = 1, 2, 4, 8, 16, 32
GBS_PS_FAILED = GBS_PS_FIT_NOCONV | GBS_PS_PIVOT | GBS_PS_CANCEL | GBS_PS_BADROW

EXPORTS = ["gbs_create", "gbs_destroy", "gbs_last_error", "gbs_set_model", "gbs_set_model_dev",
           "gbs_set_covariance", "gbs_get_model", "gbs_prob_exact", "gbs_prob_approx",
           "gbs_prob_approx_plain", "gbs_plan_get_params", "gbs_plan_set_params", "gbs_plan_tune",
           "gbs_plan_create", "gbs_plan_destroy", "gbs_plan_freeze", "gbs_prob_approx_dev",
           "gbs_grad", "gbs_grad_dev", "gbs_plan_info", "gbs_set_timing", "gbs_timing",
           "gbs_stream", "gbs_click_distribution", "gbs_prob_exact_dev", "gbs_prob_exact_dev_noalloc",
           "gbs_mcmc_step_dev", "gbs_mcmc_da_step_dev", "gbs_set_deterministic"]
TIMING_GROUPS = ["model", "row_setup", "work_queue", "contour_clusters", "dft_fit", "exact",
                 "adjoint_fit_dft", "adjoint_contour_clusters", "adjoint_rows_scatter",
                 "adjoint_model", "second_pass"]

_lib = None


class GBSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gbs error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libgbs.so and declare the C signatures.  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not built; run paper_2106_01445_amd/build.py "
                          "(or __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname; importing it first
    # makes libgbs.so bind to that one copy instead of mapping a second runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, ip, dp, i32p = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "gbs_create": ([pp, ip, vp], ip),
        "gbs_destroy": ([vp], ip),
        "gbs_last_error": ([vp], ctypes.c_char_p),
        "gbs_set_model": ([vp, ip, dp, dp, dp, dp], ip),
        "gbs_set_model_dev": ([vp, ip, dp, dp, dp, dp], ip),
        "gbs_set_timing": ([vp, ip], ip),
        "gbs_timing": ([vp, dp, i32p], ip),
        "gbs_set_covariance": ([vp, ip, dp], ip),
        "gbs_get_model": ([vp, dp, dp], ip),
        "gbs_prob_exact": ([vp, ip, i32p, i32p, ip, dp, dp, dp, i32p], ip),
        "gbs_prob_approx": ([vp, ip, i32p, i32p, ip, ip, dp, i32p], ip),
        "gbs_prob_approx_plain": ([vp, ip, i32p, i32p, ip, ip, dp, i32p], ip),
        "gbs_plan_get_params": ([vp, i32p], ip),
        "gbs_plan_set_params": ([vp, i32p], ip),
        "gbs_plan_tune": ([vp, vp, ip, i32p], ip),
        "gbs_plan_create": ([vp, ip, i32p, i32p, ip, ip, pp], ip),
        "gbs_plan_destroy": ([vp], ip),
        "gbs_plan_freeze": ([vp, ip], ip),
        "gbs_prob_approx_dev": ([vp, vp, dp, i32p], ip),
        "gbs_grad": ([vp, ip, i32p, i32p, ip, ip, dp, dp, dp, dp, i32p], ip),
        "gbs_grad_dev": ([vp, vp, dp, dp, dp, dp, i32p], ip),
        "gbs_plan_info": ([vp, dp, dp, i32p, i32p, dp], ip),
        "gbs_stream": ([vp], vp),
        "gbs_click_distribution": ([vp, ip, ip, i32p, dp, dp, i32p], ip),
        "gbs_prob_exact_dev": ([vp, ip, i32p, i32p, ip, dp, dp, dp, i32p], ip),
        "gbs_prob_exact_dev_noalloc": ([vp, ip, i32p, i32p, ip, dp, dp, dp, i32p], ip),
        "gbs_mcmc_step_dev": ([vp, vp, dp, i32p, dp, i32p], ip),
        "gbs_mcmc_da_step_dev": ([vp, vp, dp, i32p, dp, dp, i32p], ip),
        "gbs_set_deterministic": ([vp, ip], ip),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _dptr(t, dtype: str = None, numel: Optional[int] = None, name: str = "tensor"):
    """Device pointer of a torch tensor (or an int address, passed through
    unchecked).  A tensor must live on a GPU, be contiguous, and, where given,
    have the C type `dtype` ("float64" or "int32") and `numel` elements."""
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor, got one on {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    def __init__(self, ctx: "Context", handle: ctypes.c_void_p, P: int, nnz: int = 0):
        self.ctx, self.handle, self.P, self.nnz = ctx, handle, P, nnz

    def freeze(self, on: bool = True):
        self.ctx._check(load().gbs_plan_freeze(self.handle, int(on)))

    def info(self):
        rho, rc, err = np.zeros(self.P), np.zeros(self.P), np.zeros(self.P)
        K, ns = np.zeros(self.P, np.int32), np.zeros(self.P, np.int32)
        self.ctx._check(load().gbs_plan_info(self.handle, _ptr(rho), _ptr(rc), _ptr(K), _ptr(ns), _ptr(err)))
        return dict(rho=rho, rconv=rc, K=K, nsectors=ns, err=err)

    def get_params(self):
        prm = np.zeros(4, np.int32)
        self.ctx._check(load().gbs_plan_get_params(self.handle, _ptr(prm)))
        return prm

    def set_params(self, params):
        self.ctx._check(load().gbs_plan_set_params(self.handle, _ptr(_i32(params))))

    def tune(self, what: int = 3):
        """gbs_plan_tune: bit 0 forward choices, bit 1 adjoint choices."""
        prm = np.zeros(4, np.int32)
        self.ctx._check(load().gbs_plan_tune(self.ctx.handle, self.handle, what, _ptr(prm)))
        return prm

    def close(self):
        if self.handle:
            load().gbs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One gbs_ctx on a HIP device.  stream: a hipStream_t address (int) or None."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        lib = load()
        h = ctypes.c_void_p()
        rc = lib.gbs_create(ctypes.byref(h), device, ctypes.c_void_p(stream) if stream else None)
        if rc != GBS_OK:
            raise GBSError(rc, "gbs_create failed (is a GPU visible?)")
        self.handle = h
        self.M = None

    def _check(self, rc: int, allow_pattern: bool = True) -> int:
        if rc < 0:
            raise GBSError(rc, load().gbs_last_error(self.handle).decode())
        return rc

    def close(self):
        if getattr(self, "handle", None):
            load().gbs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self) -> int:
        return load().gbs_stream(self.handle) or 0

    # model -----------------------------------------------------------------
    def gbs_set_model(self, U: np.ndarray, r: np.ndarray, eta: np.ndarray):
        M = U.shape[0]
        ure, uim = _f64(U.real), _f64(U.imag)
        self._check(load().gbs_set_model(self.handle, M, _ptr(ure), _ptr(uim), _ptr(_f64(r)),
                                         _ptr(_f64(eta))))
        self.M = M

    def gbs_set_model_dev(self, U_re_dev, U_im_dev, r_dev, eta_dev):
        """Stream-ordered model build from device tensors (float64, contiguous;
        U planes M x M, r and eta of length M)."""
        M = int(r_dev.shape[0])
        f = "float64"
        self._check(load().gbs_set_model_dev(self.handle, M, _dptr(U_re_dev, f, M * M, "U_re"),
                                             _dptr(U_im_dev, f, M * M, "U_im"), _dptr(r_dev, f, M, "r"),
                                             _dptr(eta_dev, f, M, "eta")))
        self.M = M

    def gbs_set_timing(self, on: bool = True):
        self._check(load().gbs_set_timing(self.handle, int(on)))

    def gbs_timing(self):
        """{group: (total ms, launches)} since the last call (synchronises)."""
        ms = np.zeros(len(TIMING_GROUPS))
        cnt = np.zeros(len(TIMING_GROUPS), np.int32)
        self._check(load().gbs_timing(self.handle, _ptr(ms), _ptr(cnt)))
        return {g: (float(ms[i]), int(cnt[i])) for i, g in enumerate(TIMING_GROUPS)}

    def gbs_set_covariance(self, sigma: np.ndarray):
        M = sigma.shape[0] // 2
        self._check(load().gbs_set_covariance(self.handle, M, _ptr(_f64(sigma))))
        self.M = M

    def gbs_get_model(self) -> Tuple[np.ndarray, float]:
        D = 2 * self.M
        qi = np.zeros((D, D))
        ld = np.zeros(1)
        self._check(load().gbs_get_model(self.handle, _ptr(qi), _ptr(ld)))
        return qi, float(ld[0])

    # probabilities ----------------------------------------------------------
    def gbs_prob_exact(self, offsets, modes, prec: int = GBS_PREC_FP64):
        off, mod = _i32(offsets), _i32(modes)
        P = len(off) - 1
        p, lp, kap = np.zeros(P), np.zeros(P), np.zeros(P)
        st = np.zeros(P, np.int32)
        self._check(load().gbs_prob_exact(self.handle, P, _ptr(off), _ptr(mod), prec, _ptr(p),
                                          _ptr(lp), _ptr(kap), _ptr(st)))
        return dict(p=p, logp=lp, kappa=kap, status=st)

    def gbs_prob_exact_dev(self, offsets_dev, modes_dev, max_clicks: int, p_dev, logp_dev=None,
                           kappa_dev=None, status_dev=None, noalloc: bool = False):
        """Stream-ordered exact probabilities from device CSR (int32) into
        device outputs (float64; status int32).  noalloc: the entry point that
        allocates nothing (gbs_prob_exact_dev_noalloc)."""
        P = int(offsets_dev.shape[0]) - 1 if not isinstance(offsets_dev, int) else int(p_dev.shape[0])
        fn = load().gbs_prob_exact_dev_noalloc if noalloc else load().gbs_prob_exact_dev
        return self._check(fn(
            self.handle, P, _dptr(offsets_dev, "int32", P + 1, "offsets"), _dptr(modes_dev, "int32", None, "modes"),
            int(max_clicks), _dptr(p_dev, "float64", P, "p"), _dptr(logp_dev, "float64", P, "logp"),
            _dptr(kappa_dev, "float64", P, "kappa"), _dptr(status_dev, "int32", P, "status")))

    def gbs_prob_approx(self, offsets, modes, order: int, prec: int = GBS_PREC_FP64):
        off, mod = _i32(offsets), _i32(modes)
        P = len(off) - 1
        lp = np.zeros(P)
        st = np.zeros(P, np.int32)
        self._check(load().gbs_prob_approx(self.handle, P, _ptr(off), _ptr(mod), order, prec,
                                           _ptr(lp), _ptr(st)))
        return dict(logp=lp, status=st)

    def gbs_prob_approx_plain(self, offsets, modes, order: int, prec: int = GBS_PREC_FP64):
        off, mod = _i32(offsets), _i32(modes)
        P = len(off) - 1
        lp = np.zeros(P)
        st = np.zeros(P, np.int32)
        self._check(load().gbs_prob_approx_plain(self.handle, P, _ptr(off), _ptr(mod), order, prec,
                                                 _ptr(lp), _ptr(st)))
        return dict(logp=lp, status=st)

    def gbs_click_distribution(self, order: int, ks=()):
        """p(n), n = 0..M, of the whole device and the sector curves p_k(n) for
        k in ks (order-j estimate); returns dict(p_n, p_k[len(ks), M+1], status)."""
        kk = _i32(list(ks))
        pn = np.zeros(self.M + 1)
        pk = np.zeros((len(kk), self.M + 1))
        st = np.zeros(1, np.int32)
        self._check(load().gbs_click_distribution(self.handle, order, len(kk), _ptr(kk) if len(kk) else None,
                                                  _ptr(pn), _ptr(pk) if len(kk) else None, _ptr(st)))
        return dict(p_n=pn, p_k=pk, status=int(st[0]))

    def gbs_plan_create(self, offsets, modes, order: int, prec: int = GBS_PREC_FP64) -> Plan:
        off, mod = _i32(offsets), _i32(modes)
        h = ctypes.c_void_p()
        self._check(load().gbs_plan_create(self.handle, len(off) - 1, _ptr(off), _ptr(mod), order,
                                           prec, ctypes.byref(h)))
        return Plan(self, h, len(off) - 1, int(off[-1]) if len(off) else 0)

    def gbs_prob_approx_dev(self, plan: Plan, logp_dev, status_dev=None):
        return self._check(load().gbs_prob_approx_dev(self.handle, plan.handle,
                                                      _dptr(logp_dev, "float64", plan.P, "logp"),
                                                      _dptr(status_dev, "int32", plan.P, "status")))

    def gbs_grad(self, offsets, modes, order: int, dL_dlogp, prec: int = GBS_PREC_FP64):
        off, mod = _i32(offsets), _i32(modes)
        P = len(off) - 1
        lp = np.zeros(P)
        st = np.zeros(P, np.int32)
        gr, ge = np.zeros(self.M), np.zeros(self.M)
        self._check(load().gbs_grad(self.handle, P, _ptr(off), _ptr(mod), order, prec,
                                    _ptr(_f64(dL_dlogp)), _ptr(lp), _ptr(gr), _ptr(ge), _ptr(st)))
        return dict(logp=lp, grad_r=gr, grad_eta=ge, status=st)

    def gbs_mcmc_step_dev(self, plan: Plan, u_dev, modes_dev, logp_dev, accepted_dev=None):
        """One Metropolis-Hastings step of the plan's chains (device arrays:
        uniforms float64[3P], the chains' CSR modes int32 (in/out), their
        log p_hat float64[P] (in/out), accepted int32[P] or None)."""
        P = plan.P
        return self._check(load().gbs_mcmc_step_dev(self.handle, plan.handle, _dptr(u_dev, "float64", 3 * P, "u"),
                                                    _dptr(modes_dev, "int32", plan.nnz, "modes"),
                                                    _dptr(logp_dev, "float64", P, "logp"),
                                                    _dptr(accepted_dev, "int32", P, "accepted")))

    def gbs_set_deterministic(self, on: bool):
        """Gradients summed in a fixed order (bitwise reproducible) or not."""
        return self._check(load().gbs_set_deterministic(self.handle, 1 if on else 0))

    def gbs_mcmc_da_step_dev(self, plan: Plan, u_dev, modes_dev, logp_hat_dev, logp_exact_dev, accepted_dev=None):
        """One two-stage step of the plan's chains, target the exact p (device
        arrays: uniforms float64[4P], the chains' CSR modes int32 (in/out), their
        log p_hat and exact log p float64[P] (in/out), codes int32[P] or None)."""
        P = plan.P
        return self._check(load().gbs_mcmc_da_step_dev(
            self.handle, plan.handle, _dptr(u_dev, "float64", 4 * P, "u"),
            _dptr(modes_dev, "int32", plan.nnz, "modes"), _dptr(logp_hat_dev, "float64", P, "logp_hat"),
            _dptr(logp_exact_dev, "float64", P, "logp_exact"), _dptr(accepted_dev, "int32", P, "accepted")))

    def gbs_grad_dev(self, plan: Plan, dl_dev, logp_dev, grad_r_dev, grad_eta_dev, status_dev=None):
        P, M, f = plan.P, self.M, "float64"
        return self._check(load().gbs_grad_dev(self.handle, plan.handle, _dptr(dl_dev, f, P, "dL_dlogp"),
                                               _dptr(logp_dev, f, P, "logp"), _dptr(grad_r_dev, f, M, "grad_r"),
                                               _dptr(grad_eta_dev, f, M, "grad_eta"),
                                               _dptr(status_dev, "int32", P, "status")))
