"""ctypes binding of libifsvgp.so (argument marshalling only).

Every computation happens in the HIP library; this module checks tensor
shapes, dtypes and devices, passes raw device pointers and the current torch
stream, and turns status codes into exceptions.  PyTorch is used only for
device memory and streams.  There is no fallback: if the library or a GPU is
missing, calls raise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libifsvgp.so")

PREC = {"fp32": 0, "bf16": 1, "fp16": 2}
LIK = {"gaussian": 0, "probit": 1}
N_TERMS = 8
TERM_NAMES = ["data", "KL", "sum_var", "resid", "trW", "trPK", "quad", "logdet"]

OK, EINVAL, EDOMAIN, EHIP, ENONFINITE, ENOMEM, ESTATE, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double

_SIGS = {
    "ifsvgp_version": (_I, []),
    "ifsvgp_strerror": (ctypes.c_char_p, [_I]),
    "ifsvgp_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, _I, _I, _I]),
    "ifsvgp_create_group": (_I, [ctypes.POINTER(_P), _I, _I, _I, _I, _I, _I, _I]),
    "ifsvgp_step_group": (_I, [_P, _P, _I, _I, _D, _P, _I]),
    "ifsvgp_destroy": (None, [_P]),
    "ifsvgp_set_stream": (_I, [_P, _P]),
    "ifsvgp_set_graphs": (_I, [_P, _I]),
    "ifsvgp_set_kuf_mode": (_I, [_P, _I]),
    "ifsvgp_adam": (_I, [_P, _P, _P, _P, _P, ctypes.c_long, ctypes.c_float, ctypes.c_float,
                         ctypes.c_float, ctypes.c_float, _I, _I]),
    "ifsvgp_status": (_I, [_P]),
    "ifsvgp_gh_rule": (_I, [_I, _P, _P]),
    "ifsvgp_natgrad": (_I, [_P, _P, _P, _P, _P, _P, _P, _I, _P]),
    "ifsvgp_natgrad_tol": (_I, [_P, _P, _P, _P, _P, _P, _P, _I, ctypes.c_float, _P, _P]),
    "ifsvgp_natgrad_gap": (_I, [_P, _P, _I, _P, _P, _P, _P, _P, _P, _P, _I, ctypes.c_float,
                                ctypes.c_float, _P, _P]),
    "ifsvgp_bound_hutch": (_I, [_P, _P, _P, _I, _D, _P, _P, _P, _P, _P, _P, _P, _P, _I,
                                _P, _P]),
    "ifsvgp_bound_hutch_bwd": (_I, [_P, _P, _P, _I, _D, _P, _P, _P, _P, _P, _P, _P, _P,
                                    _I, _P, _P, _P, _P, _P, _P, _P]),
    "ifsvgp_bound_multi": (_I, [_P, _P, _P, _I, _I, _D, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ifsvgp_bound_multi_bwd": (_I, [_P, _P, _P, _I, _I, _D, _P, _P, _P, _P, _P, _P, _P, _P,
                                    _P, _P, _P, _P, _P, _P]),
    "ifsvgp_bound": (_I, [_P, _P, _P, _I, _D, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ifsvgp_bound_bwd": (_I, [_P, _P, _P, _I, _D, _P, _P, _P, _P, _P, _P, _P, _P,
                              _P, _P, _P, _P, _P, _P]),
    "ifsvgp_step": (_I, [_P, _P, _P, _I, _D, _P, _P, _P, _P, _P, _P, _P, _P, _I,
                         _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ifsvgp_step_noalloc": (_I, [_P, _I, _I, _I, _I, _I, _P, _P, _I, _D, _P, _P, _P, _P, _P,
                                 _P, _P, _P, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ifsvgp_predict": (_I, [_P, _P, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ifsvgp_timing_enable": (_I, [_P, ctypes.c_longlong]),
    "ifsvgp_timing_read": (_I, [_P, _I, _P, _P, _P]),
    "ifsvgp_kernel_flops": (_I, [_P, _I, _I, _P, _P]),
}

EXPORTED = sorted(_SIGS)


class IFSVGPError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else strerror(code))


def load(path=LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} not found: build it with `python -m paper_2604_00697_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code):
    return load().ifsvgp_strerror(code).decode()


def gh_rule(n):
    """The library's Gauss-Hermite rule (host code, no GPU needed)."""
    t = np.zeros(max(n, 1))
    w = np.zeros(max(n, 1))
    rc = load().ifsvgp_gh_rule(n, t.ctypes.data, w.ctypes.data)
    if rc != OK:
        raise IFSVGPError(rc, "ifsvgp_gh_rule")
    return t, w


def _check(rc, what):
    if rc != OK:
        raise IFSVGPError(rc, what)


def _ptr(t, shape, name, dtype=None, optional=False):
    import torch
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    dtype = dtype or torch.float32
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


class Problem(ctypes.Structure):
    """One problem of a grouped call (the arguments of ifsvgp_step)."""
    _fields_ = [(n, _P) for n in ("X", "y", "ell", "sf2", "noise_var", "Z", "m_tilde", "s_tilde",
                                   "L", "out_bound", "out_terms", "out_resid", "g_ell", "g_sf2",
                                   "g_noise", "g_Z", "g_m", "g_s")]


def step_noalloc(X, y, N, ell, sf2, noise, Z, m, s, L, gammas, prec="fp32", lik="gaussian",
                 n_gh=20, out=None, terms=None, resid=None, grads=None, flag=None,
                 want=("ell", "sf2", "noise_var", "Z", "m")):
    """One training iteration through the allocation-free entry point (no
    context; the library's static device workspace on the current device).
    The caller provides every output buffer through the keyword arguments
    (or this wrapper allocates them with torch before the call).  Returns
    (F, terms, resid, grads, flag); flag is the call's device error bits."""
    import torch
    B, D = X.shape
    M = Z.shape[0]
    dev = X.device
    gm = np.ascontiguousarray(np.asarray(gammas, np.float32).reshape(-1))
    n = gm.shape[0]
    f64 = dict(dtype=torch.float64, device=dev)
    out = torch.empty(1, **f64) if out is None else out
    terms = torch.empty(N_TERMS, **f64) if terms is None else terms
    if resid is None and n > 0:
        resid = torch.empty(n, **f64)
    flag = torch.empty(1, dtype=torch.int32, device=dev) if flag is None else flag
    if grads is None:
        shapes = {"ell": (D,), "sf2": (1,), "noise_var": (1,), "Z": (M, D), "m": (M,), "s": (M,)}
        grads = {k: torch.empty(shapes[k], dtype=torch.float32, device=dev)
                 for k in want if not (k == "noise_var" and lik != "gaussian")}
    stream = torch.cuda.current_stream(dev).cuda_stream
    _check(load().ifsvgp_step_noalloc(
        stream, M, D, PREC[prec], LIK[lik], int(n_gh),
        _ptr(X, (B, D), "X"), _ptr(y, (B,), "y"), B, float(N), _ptr(ell, (D,), "ell"),
        _ptr(sf2, (1,), "sf2"), _ptr(noise, (1,), "noise_var", optional=lik != "gaussian"),
        _ptr(Z, (M, D), "Z"), _ptr(m, (M,), "m_tilde"), _ptr(s, (M,), "s_tilde"),
        _ptr(L, (M, M), "L"), gm.ctypes.data if n else None, n,
        _ptr(out, (1,), "out", torch.float64), _ptr(terms, (N_TERMS,), "terms", torch.float64),
        _ptr(resid, (n,), "resid", torch.float64) if n else None,
        *Context._grad_ptrs(grads), _ptr(flag, (1,), "flag", torch.int32)),
        "ifsvgp_step_noalloc")
    return out, terms, resid, grads, flag


class Context:
    """One library context: fixed M, B_max, D, precision and likelihood."""

    def __init__(self, M, B_max, D, prec="fp32", lik="gaussian", n_gh=20, device=None):
        import torch
        lib = load()
        self.M, self.B_max, self.D = int(M), int(B_max), int(D)
        self.prec, self.lik, self.n_gh = prec, lik, int(n_gh)
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        h = _P()
        with torch.cuda.device(self.device):
            _check(lib.ifsvgp_create(ctypes.byref(h), self.M, self.B_max, self.D,
                                     PREC[prec], LIK[lik], self.n_gh), "ifsvgp_create")
        self._h = h
        self._lib = lib
        self.generation = 0   # incremented by every forward (bound / step)

    def close(self):
        if getattr(self, "_h", None):
            import torch
            torch.cuda.synchronize(self.device)
            self._lib.ifsvgp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- plumbing
    def _stream(self):
        import torch
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(self._lib.ifsvgp_set_stream(self._h, s), "ifsvgp_set_stream")

    def adam(self, param, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
             ascend=False):
        """One in-place Adam step on fp32 CUDA tensors of one shape (m, v start
        at zero; step >= 1)."""
        n = param.numel()
        ptrs = [_ptr(t, tuple(param.shape), nm) for t, nm in
                ((param, "param"), (grad, "grad"), (m, "m"), (v, "v"))]
        self._stream()
        _check(self._lib.ifsvgp_adam(self._h, *ptrs, n, lr, beta1, beta2, eps, int(step),
                                     1 if ascend else 0), "ifsvgp_adam")

    def set_graphs(self, enable):
        """Record and replay repeated calls as HIP graphs (enable=True), or run
        every call directly (the default)."""
        _check(self._lib.ifsvgp_set_graphs(self._h, 1 if enable else 0), "ifsvgp_set_graphs")

    def set_kuf_mode(self, mode):
        """Where the bf16 / fp16 forms form K_uf's tiles: "in_product" (the
        default: inside V's launch, never stored), "stored" (once, beside the
        NG step) or "auto" (stored from M * B = 2^23 on); results are
        bit-identical."""
        modes = {"in_product": 0, "stored": 1, "auto": 2}
        if mode not in modes:
            raise ValueError(f"mode must be one of {sorted(modes)}")
        _check(self._lib.ifsvgp_set_kuf_mode(self._h, modes[mode]), "ifsvgp_set_kuf_mode")

    def status(self):
        """Synchronise and return (and clear) the device error flag code."""
        return self._lib.ifsvgp_status(self._h)

    def raise_status(self):
        _check(self.status(), "device check")

    def _inputs(self, X, y, ell, sf2, noise, Z, m, s, L):
        B = X.shape[0]
        M, D = self.M, self.D
        return dict(
            X=_ptr(X, (B, D), "X"), y=_ptr(y, (B,), "y"), B=B,
            ell=_ptr(ell, (D,), "ell"), sf2=_ptr(sf2, (1,), "sf2"),
            noise=_ptr(noise, (1,), "noise_var", optional=self.lik != "gaussian"),
            Z=_ptr(Z, (M, D), "Z"), m=_ptr(m, (M,), "m_tilde"),
            s=_ptr(s, (M,), "s_tilde"), L=_ptr(L, (M, M), "L"))

    # ---------------------------------------------------------------- calls
    def natgrad(self, Z, ell, sf2, s, L, gammas, resid=None):
        """n NG steps on L in place; returns the fp64 residual tensor (n,)."""
        import torch
        g = np.ascontiguousarray(np.asarray(gammas, np.float32).reshape(-1))
        n = g.shape[0]
        if resid is None:
            resid = torch.empty(n, dtype=torch.float64, device=self.device)
        self._stream()
        _check(self._lib.ifsvgp_natgrad(
            self._h, _ptr(Z, (self.M, self.D), "Z"), _ptr(ell, (self.D,), "ell"),
            _ptr(sf2, (1,), "sf2"), _ptr(s, (self.M,), "s_tilde"),
            _ptr(L, (self.M, self.M), "L"), g.ctypes.data, n,
            _ptr(resid, (n,), "resid", torch.float64)), "ifsvgp_natgrad")
        return resid

    def natgrad_tol(self, Z, ell, sf2, s, L, gammas, tol):
        """Up to len(gammas) NG steps on L in place, stopping once the residual
        falls below tol; returns (residuals fp64 tensor, steps applied int32
        tensor of one element)."""
        import torch
        g = np.ascontiguousarray(np.asarray(gammas, np.float32).reshape(-1))
        n = g.shape[0]
        resid = torch.empty(n, dtype=torch.float64, device=self.device)
        steps = torch.empty(1, dtype=torch.int32, device=self.device)
        self._stream()
        _check(self._lib.ifsvgp_natgrad_tol(
            self._h, _ptr(Z, (self.M, self.D), "Z"), _ptr(ell, (self.D,), "ell"),
            _ptr(sf2, (1,), "sf2"), _ptr(s, (self.M,), "s_tilde"),
            _ptr(L, (self.M, self.M), "L"), g.ctypes.data, n, float(tol),
            _ptr(resid, (n,), "resid", torch.float64), _ptr(steps, (1,), "steps", torch.int32)),
            "ifsvgp_natgrad_tol")
        return resid, steps

    def natgrad_gap(self, X, Z, ell, sf2, noise, s, L, gammas, sigma2, eps):
        """Up to len(gammas) NG steps on L in place, stopping once the variance
        gap on the batch X falls to 2 noise eps or below (Gaussian only);
        returns (gaps fp64 tensor, steps applied int32 tensor of one element)."""
        import torch
        g = np.ascontiguousarray(np.asarray(gammas, np.float32).reshape(-1))
        n = g.shape[0]
        B = X.shape[0]
        gaps = torch.empty(n, dtype=torch.float64, device=self.device)
        steps = torch.empty(1, dtype=torch.int32, device=self.device)
        self._stream()
        _check(self._lib.ifsvgp_natgrad_gap(
            self._h, _ptr(X, (B, self.D), "X"), B, _ptr(Z, (self.M, self.D), "Z"),
            _ptr(ell, (self.D,), "ell"), _ptr(sf2, (1,), "sf2"), _ptr(noise, (1,), "noise_var"),
            _ptr(s, (self.M,), "s_tilde"), _ptr(L, (self.M, self.M), "L"), g.ctypes.data, n,
            float(sigma2), float(eps), _ptr(gaps, (n,), "gaps", torch.float64),
            _ptr(steps, (1,), "steps", torch.int32)), "ifsvgp_natgrad_gap")
        return gaps, steps

    def bound(self, X, y, N, ell, sf2, noise, Z, m, s, L, out=None, terms=None):
        """F (fp64 tensor (1,)) and terms (fp64 tensor (8,)) at the given L."""
        import torch
        a = self._inputs(X, y, ell, sf2, noise, Z, m, s, L)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        terms = torch.empty(N_TERMS, dtype=torch.float64, device=self.device) if terms is None else terms
        self._stream()
        _check(self._lib.ifsvgp_bound(
            self._h, a["X"], a["y"], a["B"], float(N), a["ell"], a["sf2"], a["noise"], a["Z"],
            a["m"], a["s"], a["L"], _ptr(out, (1,), "out", torch.float64),
            _ptr(terms, (N_TERMS,), "terms", torch.float64)), "ifsvgp_bound")
        self.generation += 1
        return out, terms

    def bound_hutch(self, X, y, N, ell, sf2, noise, Z, m, s, L, Omega_t, out=None, terms=None):
        """Bound with Hutchinson trace estimates from the probes in the rows of
        Omega_t (fp32 [K, M]); F (fp64 (1,)) and terms (fp64 (8,))."""
        import torch
        a = self._inputs(X, y, ell, sf2, noise, Z, m, s, L)
        K = Omega_t.shape[0]
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        terms = torch.empty(N_TERMS, dtype=torch.float64, device=self.device) if terms is None else terms
        self._stream()
        _check(self._lib.ifsvgp_bound_hutch(
            self._h, a["X"], a["y"], a["B"], float(N), a["ell"], a["sf2"], a["noise"], a["Z"],
            a["m"], a["s"], a["L"], _ptr(Omega_t, (K, self.M), "Omega_t"), K,
            _ptr(out, (1,), "out", torch.float64),
            _ptr(terms, (N_TERMS,), "terms", torch.float64)), "ifsvgp_bound_hutch")
        return out, terms

    def bound_hutch_bwd(self, X, y, N, ell, sf2, noise, Z, m, s, L, Omega_t, grad_scale=None,
                        want=("ell", "sf2", "noise_var", "Z", "m")):
        """Gradients of the preceding bound_hutch's estimate at its probes
        Omega_t (fp32 [K, M]); dict of fp32 tensors (no "s")."""
        import torch
        if "s" in want:
            raise ValueError("bound_hutch_bwd offers no gradient with respect to s~")
        a = self._inputs(X, y, ell, sf2, noise, Z, m, s, L)
        K = Omega_t.shape[0]
        g = self._grad_buffers(want)
        self._stream()
        gs = None if grad_scale is None else _ptr(grad_scale, (1,), "grad_scale", torch.float64)
        _check(self._lib.ifsvgp_bound_hutch_bwd(
            self._h, a["X"], a["y"], a["B"], float(N), a["ell"], a["sf2"], a["noise"], a["Z"],
            a["m"], a["s"], a["L"], _ptr(Omega_t, (K, self.M), "Omega_t"), K, gs,
            *self._grad_ptrs(g)), "ifsvgp_bound_hutch_bwd")
        return g

    def _multi_inputs(self, X, Y, ell, sf2, noise, Z, Mt, s, L):
        B, Q = X.shape[0], Mt.shape[0]
        M, D = self.M, self.D
        return (_ptr(X, (B, D), "X"), _ptr(Y, (B, Q), "Y"), B, Q), (
            _ptr(ell, (D,), "ell"), _ptr(sf2, (1,), "sf2"),
            _ptr(noise, (1,), "noise_var", optional=self.lik != "gaussian"),
            _ptr(Z, (M, D), "Z"), _ptr(Mt, (Q, M), "Mt"), _ptr(s, (M,), "s_tilde"),
            _ptr(L, (M, M), "L"))

    def bound_multi(self, X, Y, N, ell, sf2, noise, Z, Mt, s, L, out=None, terms=None):
        """Multi-output bound: targets Y (B, Q), inducing means Mt (Q, M);
        F (fp64 (1,)) and terms (fp64 (8,))."""
        import torch
        (x, y, B, Q), rest = self._multi_inputs(X, Y, ell, sf2, noise, Z, Mt, s, L)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        terms = torch.empty(N_TERMS, dtype=torch.float64, device=self.device) if terms is None else terms
        self._stream()
        _check(self._lib.ifsvgp_bound_multi(
            self._h, x, y, B, Q, float(N), *rest, _ptr(out, (1,), "out", torch.float64),
            _ptr(terms, (N_TERMS,), "terms", torch.float64)), "ifsvgp_bound_multi")
        self.generation += 1
        return out, terms

    def bound_multi_bwd(self, X, Y, N, ell, sf2, noise, Z, Mt, s, L, grad_scale=None,
                        want=("ell", "sf2", "noise_var", "Z", "m")):
        """Gradients of the preceding bound_multi's F; dict of fp32 tensors,
        "m" of shape (Q, M) (no "s")."""
        import torch
        if "s" in want:
            raise ValueError("bound_multi_bwd offers no gradient with respect to s~")
        (x, y, B, Q), rest = self._multi_inputs(X, Y, ell, sf2, noise, Z, Mt, s, L)
        g = self._grad_buffers([k for k in want if k != "m"])
        if "m" in want:
            g["m"] = torch.empty((Q, self.M), dtype=torch.float32, device=self.device)
        self._stream()
        gs = None if grad_scale is None else _ptr(grad_scale, (1,), "grad_scale", torch.float64)
        _check(self._lib.ifsvgp_bound_multi_bwd(
            self._h, x, y, B, Q, float(N), *rest, gs, *self._grad_ptrs(g)),
            "ifsvgp_bound_multi_bwd")
        return g

    def bound_bwd(self, X, y, N, ell, sf2, noise, Z, m, s, L, grad_scale=None,
                  want=("ell", "sf2", "noise_var", "Z", "m")):
        """Gradients of the preceding forward's F; dict of fp32 tensors."""
        import torch
        a = self._inputs(X, y, ell, sf2, noise, Z, m, s, L)
        g = self._grad_buffers(want)
        self._stream()
        gs = None if grad_scale is None else _ptr(grad_scale, (1,), "grad_scale", torch.float64)
        _check(self._lib.ifsvgp_bound_bwd(
            self._h, a["X"], a["y"], a["B"], float(N), a["ell"], a["sf2"], a["noise"], a["Z"],
            a["m"], a["s"], a["L"], gs, *self._grad_ptrs(g)), "ifsvgp_bound_bwd")
        return g

    def step(self, X, y, N, ell, sf2, noise, Z, m, s, L, gammas, out=None, terms=None,
             resid=None, want=("ell", "sf2", "noise_var", "Z", "m"), grads=None):
        """One training iteration: NG steps on L (in place), bound and gradient."""
        import torch
        a = self._inputs(X, y, ell, sf2, noise, Z, m, s, L)
        gm = np.ascontiguousarray(np.asarray(gammas, np.float32).reshape(-1))
        n = gm.shape[0]
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        terms = torch.empty(N_TERMS, dtype=torch.float64, device=self.device) if terms is None else terms
        if resid is None and n > 0:
            resid = torch.empty(n, dtype=torch.float64, device=self.device)
        g = grads if grads is not None else self._grad_buffers(want)
        self._stream()
        _check(self._lib.ifsvgp_step(
            self._h, a["X"], a["y"], a["B"], float(N), a["ell"], a["sf2"], a["noise"], a["Z"],
            a["m"], a["s"], a["L"], gm.ctypes.data if n else None, n,
            _ptr(out, (1,), "out", torch.float64), _ptr(terms, (N_TERMS,), "terms", torch.float64),
            _ptr(resid, (n,), "resid", torch.float64) if n else None,
            *self._grad_ptrs(g)), "ifsvgp_step")
        self.generation += 1
        return out, terms, resid, g

    def predict(self, X, ell, sf2, Z, m, s, L, y=None, noise=None):
        """Predictive mean and variance of f at the rows of X (any count), and
        with targets y the per-point log predictive density and the NLPD.
        Returns (mu, var, lpd, nlpd); lpd and nlpd are None without y."""
        import torch
        n = X.shape[0]
        M, D = self.M, self.D
        mu = torch.empty(n, dtype=torch.float32, device=self.device)
        var = torch.empty(n, dtype=torch.float32, device=self.device)
        lpd = nlpd = None
        if y is not None:
            lpd = torch.empty(n, dtype=torch.float32, device=self.device)
            nlpd = torch.empty(1, dtype=torch.float64, device=self.device)
        self._stream()
        _check(self._lib.ifsvgp_predict(
            self._h, _ptr(X, (n, D), "X"), n, _ptr(y, (n,), "y", optional=True),
            _ptr(ell, (D,), "ell"), _ptr(sf2, (1,), "sf2"),
            _ptr(noise, (1,), "noise_var", optional=True), _ptr(Z, (M, D), "Z"),
            _ptr(m, (M,), "m_tilde"), _ptr(s, (M,), "s_tilde"), _ptr(L, (M, M), "L"),
            mu.data_ptr(), var.data_ptr(), None if lpd is None else lpd.data_ptr(),
            None if nlpd is None else nlpd.data_ptr()), "ifsvgp_predict")
        return mu, var, lpd, nlpd

    def _grad_buffers(self, want):
        import torch
        shapes = {"ell": (self.D,), "sf2": (1,), "noise_var": (1,),
                  "Z": (self.M, self.D), "m": (self.M,), "s": (self.M,)}
        return {k: torch.empty(shapes[k], dtype=torch.float32, device=self.device)
                for k in want if not (k == "noise_var" and self.lik != "gaussian")}

    @staticmethod
    def _grad_ptrs(g):
        return [g[k].data_ptr() if k in g else None
                for k in ("ell", "sf2", "noise_var", "Z", "m", "s")]

    # ---------------------------------------------------------------- profiling
    def timing(self, kinds):
        """Time launches of the named kernel kinds (a list of names, True for
        all, False/None to stop)."""
        if kinds is True:
            mask = -1
        elif not kinds:
            mask = 0
        else:
            names = list(self.kernel_flops(1))
            mask = 0
            for k in kinds:
                mask |= 1 << names.index(k)
        _check(self._lib.ifsvgp_timing_enable(self._h, mask), "timing_enable")

    def timing_read(self):
        cap = 64
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int * cap)()
        names = (ctypes.c_char_p * cap)()
        n = self._lib.ifsvgp_timing_read(self._h, cap, ms, cnt, names)
        if n < 0:
            raise IFSVGPError(n, "timing_read")
        return {names[k].decode(): (ms[k], cnt[k]) for k in range(n)}

    def kernel_flops(self, B):
        """Algorithmic flops of one launch of each kernel kind at batch size B."""
        cap = 64
        f = (ctypes.c_double * cap)()
        names = (ctypes.c_char_p * cap)()
        n = self._lib.ifsvgp_kernel_flops(self._h, int(B), cap, f, names)
        if n < 0:
            raise IFSVGPError(n, "kernel_flops")
        return {names[k].decode(): f[k] for k in range(n)}


class GroupContext(Context):
    """G independent problems of the same sizes, advanced by one grouped
    launch per kernel (ifsvgp_step_group)."""

    def __init__(self, G, M, B_max, D, prec="fp32", lik="gaussian", n_gh=20, device=None):
        import torch
        lib = load()
        self.G = int(G)
        self.M, self.B_max, self.D = int(M), int(B_max), int(D)
        self.prec, self.lik, self.n_gh = prec, lik, int(n_gh)
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        h = _P()
        with torch.cuda.device(self.device):
            _check(lib.ifsvgp_create_group(ctypes.byref(h), self.G, self.M, self.B_max, self.D,
                                           PREC[prec], LIK[lik], self.n_gh),
                   "ifsvgp_create_group")
        self._h = h
        self._lib = lib
        self.generation = 0

    def step_group(self, problems, N, gammas, want=("ell", "sf2", "noise_var", "Z", "m")):
        """problems: G dicts with X, y, ell, sf2, noise, Z, m, s, L (L updated in
        place).  Returns a list of (F, terms, resid, grads) per problem."""
        import torch
        if len(problems) != self.G:
            raise ValueError(f"expected {self.G} problems, got {len(problems)}")
        gm = np.ascontiguousarray(np.asarray(gammas, np.float32).reshape(-1))
        n = gm.shape[0]
        B = problems[0]["X"].shape[0]
        arr = (Problem * self.G)()
        outs = []
        for g, p in enumerate(problems):
            a = self._inputs(p["X"], p["y"], p["ell"], p["sf2"], p.get("noise"), p["Z"], p["m"],
                             p["s"], p["L"])
            if a["B"] != B:
                raise ValueError("every problem of a group takes the same batch size")
            F = torch.empty(1, dtype=torch.float64, device=self.device)
            terms = torch.empty(N_TERMS, dtype=torch.float64, device=self.device)
            resid = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)
            gr = self._grad_buffers(want)
            gp = self._grad_ptrs(gr)
            arr[g] = Problem(a["X"], a["y"], a["ell"], a["sf2"], a["noise"], a["Z"], a["m"],
                             a["s"], a["L"], F.data_ptr(), terms.data_ptr(),
                             resid.data_ptr() if n else None, *gp)
            outs.append((F, terms, resid[:n], gr))
        self._stream()
        _check(self._lib.ifsvgp_step_group(self._h, ctypes.cast(arr, _P), self.G, B, float(N),
                                           gm.ctypes.data if n else None, n),
               "ifsvgp_step_group")
        self.generation += 1
        return outs
