"""ctypes binding of libscc (same names as the C ABI in include/scc.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SCC_OK = 0
ERRORS = {0: "SCC_OK", -1: "SCC_EINVAL", -2: "SCC_ESTATE", -3: "SCC_ENOCONV", -4: "SCC_ECOMPLEX",
          -5: "SCC_ESINGULAR", -6: "SCC_EDEVICE", -7: "SCC_ENOMEM"}
FIELD_T, FIELD_R, FIELD_L, FIELD_E0, FIELD_OMEGA = 0, 1, 2, 3, 4
# GEMM kernels whose launches scc_profile totals
GEMM_F64, GEMM_F64_TWO, GEMM_F32, GEMM_F32_TWO, GEMM_F64_MULTI, GEMM_F32_MULTI = 0, 1, 2, 3, 4, 5
GEMM_KERNEL_NAMES = ["gemm_f64_kernel", "gemm_f64_two_kernel", "gemm_f32acc_kernel", "gemm_f32acc_two_kernel",
                     "gemm_f64_multi_kernel", "gemm_f32acc_multi_kernel"]

EXPORTED_SYMBOLS = ["scc_workspace_bytes", "scc_create", "scc_destroy", "scc_last_error",
                    "scc_set_hamiltonian", "scc_set_hamiltonian_fixed_basis", "scc_ground", "scc_excited", "scc_multipliers",
                    "scc_densities", "scc_gradient", "scc_nac", "scc_gradients_and_couplings", "scc_multiplier_length",
                    "scc_get", "scc_eval_residual",
                    "scc_eval_sigma", "scc_eval_left", "scc_profile", "scc_profile_kernels",
                    "scc_mlp_param_count", "scc_mlp_workspace_bytes", "scc_mlp_forward", "scc_mlp_forward_noalloc",
                    "scc_mlp_loss_grad",
                    "scc_mlp_train", "scc_pca_workspace_bytes", "scc_pca_fit", "scc_pca_expand"]


class Dims(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int), ("nvirt", ctypes.c_int), ("nchol", ctypes.c_int),
                ("nstates", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("tol_residual", ctypes.c_double), ("tol_overlap", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("scc", ctypes.c_int), ("verbose", ctypes.c_int),
                ("precision", ctypes.c_int), ("eager", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("residual", ctypes.c_double), ("seconds", ctypes.c_double), ("flops_mfma", ctypes.c_double),
                ("precision", ctypes.c_int)]


class MlpDims(ctypes.Structure):
    _fields_ = [("nin", ctypes.c_int), ("nhidden", ctypes.c_int), ("nout", ctypes.c_int)]


class SccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def library_path():
    return os.path.join(HERE, "libscc.so")


def load_library():
    """Load the in-tree libscc.so; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"libscc.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.scc_workspace_bytes.argtypes = [ctypes.POINTER(Dims), ctypes.POINTER(Options), ctypes.POINTER(S)]
    lib.scc_create.argtypes = [ctypes.POINTER(Dims), ctypes.POINTER(Options), P, S, P, ctypes.POINTER(P)]
    lib.scc_destroy.argtypes = [P]
    lib.scc_destroy.restype = None
    lib.scc_last_error.argtypes = [P]
    lib.scc_last_error.restype = ctypes.c_char_p
    lib.scc_set_hamiltonian.argtypes = [P, P, P, D]
    lib.scc_set_hamiltonian_fixed_basis.argtypes = [P, P, P, D, P, P, ctypes.POINTER(Info)]
    lib.scc_ground.argtypes = [P, P, P, ctypes.POINTER(Info)]
    lib.scc_excited.argtypes = [P, I, P, P, P, ctypes.POINTER(Info)]
    lib.scc_multipliers.argtypes = [P, I, I, I, P, P, ctypes.POINTER(Info)]
    lib.scc_densities.argtypes = [P, I, I, I, P, P, P]
    lib.scc_gradient.argtypes = [P, I, I, P, P, P, ctypes.POINTER(Info)]
    lib.scc_nac.argtypes = [P, I, I, I, P, P, P, ctypes.POINTER(Info)]
    lib.scc_get.argtypes = [P, I, I, P]
    lib.scc_gradients_and_couplings.argtypes = [P, I, P, I, P, I, P, P, P, P, P, P, ctypes.POINTER(Info)]
    lib.scc_multiplier_length.argtypes = [ctypes.POINTER(Dims), ctypes.POINTER(ctypes.c_longlong)]
    lib.scc_eval_residual.argtypes = [P, P, P, P, P]
    lib.scc_eval_sigma.argtypes = [P, P, P]
    lib.scc_eval_left.argtypes = [P, P, P]
    lib.scc_profile.argtypes = [P, I, I, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong),
                                ctypes.POINTER(D)]
    lib.scc_profile_kernels.argtypes = [P, ctypes.c_uint]
    MD = ctypes.POINTER(MlpDims)
    lib.scc_mlp_param_count.argtypes = [MD, ctypes.POINTER(ctypes.c_longlong)]
    lib.scc_mlp_workspace_bytes.argtypes = [MD, I, ctypes.POINTER(S)]
    lib.scc_mlp_forward.argtypes = [MD, P, I, P, P, P, S, P]
    lib.scc_mlp_forward_noalloc.argtypes = [MD, P, I, P, P, P]
    lib.scc_mlp_loss_grad.argtypes = [MD, P, I, P, P, P, P, P, S, P]
    lib.scc_mlp_train.argtypes = [MD, P, P, P, I, P, P, I, I, P, ctypes.c_float, I, P, P, S, P]
    lib.scc_pca_workspace_bytes.argtypes = [I, ctypes.c_longlong, I, ctypes.POINTER(S)]
    lib.scc_pca_fit.argtypes = [I, ctypes.c_longlong, I, P, P, P, P, P, P, S, P]
    lib.scc_pca_expand.argtypes = [I, ctypes.c_longlong, I, P, P, P, P, P]
    for name in EXPORTED_SYMBOLS:
        fn = getattr(lib, name)
        if name not in ("scc_destroy", "scc_last_error"):
            fn.restype = ctypes.c_int
    _LIB = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def workspace_bytes(o, v, nj, nstates, opts=None):
    lib = load_library()
    d = Dims(o, v, nj, nstates)
    n = ctypes.c_size_t(0)
    rc = lib.scc_workspace_bytes(ctypes.byref(d), ctypes.byref(opts) if opts else None, ctypes.byref(n))
    if rc != SCC_OK:
        raise SccError(rc, "workspace size")
    return n.value


class Context:
    """Owns a libscc context plus its workspace (a torch uint8 CUDA tensor)."""

    def __init__(self, o, v, nj, nstates, tol=1e-10, tol_overlap=1e-11, max_iter=200, scc=True,
                 verbose=False, device="cuda:0", stream=None, precision="fp64", eager=False):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.o, self.v, self.nj, self.ns = o, v, nj, nstates
        self.n = o + v
        self.nov = o * v
        self.device = torch.device(device)
        if precision not in ("fp64", "fp32"):
            raise ValueError("precision must be 'fp64' or 'fp32'")
        self.opts = Options(tol, tol_overlap, max_iter, 1 if scc else 0, 1 if verbose else 0,
                            1 if precision == "fp32" else 0, 1 if eager else 0)
        self.dims = Dims(o, v, nj, nstates)
        nbytes = ctypes.c_size_t(0)
        self._check(self.lib.scc_workspace_bytes(ctypes.byref(self.dims), ctypes.byref(self.opts),
                                                 ctypes.byref(nbytes)), None)
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self.lib.scc_create(ctypes.byref(self.dims), ctypes.byref(self.opts),
                                 ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value + 256,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != SCC_OK:
            raise SccError(rc, "scc_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.scc_destroy(self.h)
            self.h = None
        # the workspace goes back to torch's allocator with the context
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != SCC_OK:
            msg = self.lib.scc_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise SccError(rc, f"{what}: {msg}")

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.float64).contiguous()
        return t.as_tensor(a, dtype=t.float64).to(self.device).contiguous()

    def zeros(self, *shape):
        return self.torch.zeros(*shape, dtype=self.torch.float64, device=self.device)

    # --- calls ---------------------------------------------------------------
    def set_hamiltonian(self, h, chol, e_nuc=0.0):
        self._h = self._dev(h)
        self._L = self._dev(chol)
        self._check(self.lib.scc_set_hamiltonian(self.h, _ptr(self._h), _ptr(self._L), float(e_nuc)),
                    "scc_set_hamiltonian")

    def set_hamiltonian_fixed_basis(self, h, chol, e_nuc=0.0, orbitals_guess=None):
        """RHF on the device, then as set_hamiltonian; returns the orbitals."""
        self._h = self._dev(h)
        self._L = self._dev(chol)
        g = None if orbitals_guess is None else self._dev(orbitals_guess)
        C = self.zeros(self.n, self.n)
        info = Info()
        self._check(self.lib.scc_set_hamiltonian_fixed_basis(self.h, _ptr(self._h), _ptr(self._L), float(e_nuc),
                                                             _ptr(g), _ptr(C), ctypes.byref(info)),
                    "scc_set_hamiltonian_fixed_basis")
        return C, info

    def ground(self, guess=None):
        e0 = self.zeros(1)
        info = Info()
        g = None if guess is None else self._dev(guess)
        self._check(self.lib.scc_ground(self.h, _ptr(g), _ptr(e0), ctypes.byref(info)), "scc_ground")
        return float(e0.cpu()[0]), info

    def excited(self, guess=None):
        """guess: None or [ns * (1 + nov + nov^2) + npairs] (right vectors, then zeta)."""
        e = self.zeros(self.ns)
        z = self.zeros(max(1, self.ns * (self.ns - 1) // 2))
        info = Info()
        g = None if guess is None else self._dev(guess)
        self._check(self.lib.scc_excited(self.h, self.ns, _ptr(g), _ptr(e), _ptr(z), ctypes.byref(info)),
                    "scc_excited")
        return e.cpu().numpy(), z.cpu().numpy()[:self.ns * (self.ns - 1) // 2], info

    def multipliers(self, kind, m, n, guess=None, out=False):
        """Multipliers of one target; returns info, plus the converged multipliers (device
        [multiplier_length]) when out=True.  guess: starting multipliers of that length."""
        info = Info()
        g = None if guess is None else self._dev(guess)
        x = self.zeros(self.multiplier_length()) if out else None
        self._check(self.lib.scc_multipliers(self.h, kind, m, n, _ptr(g), _ptr(x), ctypes.byref(info)),
                    "scc_multipliers")
        return (info, x) if out else info

    def densities(self, kind, m, n):
        """Effective densities of the gradient of state n (kind 0) or of the
        coupling d_mn (kind 1): (d1 [N][N], z3 [N_J][N][N], kappa_bar [v][o])."""
        d1 = self.zeros(self.n, self.n)
        z3 = self.zeros(self.nj, self.n, self.n)
        kb = self.zeros(self.v, self.o)
        self._check(self.lib.scc_densities(self.h, kind, m, n, _ptr(d1), _ptr(z3), _ptr(kb)), "scc_densities")
        return d1, z3, kb

    def gradient(self, n, dh, dchol):
        dh, dl = self._dev(dh), self._dev(dchol)
        out = self.zeros(dh.shape[0])
        info = Info()
        self._check(self.lib.scc_gradient(self.h, n, dh.shape[0], _ptr(dh), _ptr(dl), _ptr(out),
                                          ctypes.byref(info)), "scc_gradient")
        return out.cpu().numpy(), info

    def nac(self, m, n, dh, dchol):
        dh, dl = self._dev(dh), self._dev(dchol)
        out = self.zeros(dh.shape[0])
        info = Info()
        self._check(self.lib.scc_nac(self.h, m, n, dh.shape[0], _ptr(dh), _ptr(dl), _ptr(out),
                                     ctypes.byref(info)), "scc_nac")
        return out.cpu().numpy(), info

    def multiplier_length(self):
        n = ctypes.c_longlong(0)
        self._check(self.lib.scc_multiplier_length(ctypes.byref(self.dims), ctypes.byref(n)), "scc_multiplier_length")
        return n.value

    def gradients_and_couplings(self, states, pairs, dh, dchol, guess=None, multipliers=False):
        """All requested gradients and couplings in one call; returns (grads, nacs, info) host arrays, plus
        the converged multipliers (device [ntarget][multiplier_length]) when multipliers=True.  guess:
        starting multipliers of the same shape (each judged by its residual)."""
        dh, dl = self._dev(dh), self._dev(dchol)
        nc = dh.shape[0]
        st = (ctypes.c_int * max(1, len(states)))(*states)
        flat = [x for p in pairs for x in p]
        pr = (ctypes.c_int * max(1, len(flat)))(*flat)
        g = self.zeros(max(1, len(states)), nc)
        d = self.zeros(max(1, len(pairs)), nc)
        nt = len(states) + len(pairs)
        gs = None if guess is None else self._dev(guess)
        mo = self.zeros(nt, self.multiplier_length()) if multipliers else None
        info = Info()
        self._check(self.lib.scc_gradients_and_couplings(self.h, len(states), ctypes.cast(st, ctypes.c_void_p),
                                                         len(pairs), ctypes.cast(pr, ctypes.c_void_p), nc, _ptr(dh),
                                                         _ptr(dl), _ptr(gs), _ptr(mo), _ptr(g), _ptr(d),
                                                         ctypes.byref(info)),
                    "scc_gradients_and_couplings")
        out = (g.cpu().numpy()[:len(states)], d.cpu().numpy()[:len(pairs)], info)
        return out + (mo,) if multipliers else out

    def get(self, field, k=0):
        nvt = self.nov + self.nov * self.nov
        size = {FIELD_T: nvt, FIELD_R: 1 + nvt, FIELD_L: 1 + nvt, FIELD_E0: 1, FIELD_OMEGA: nvt}[field]
        out = self.zeros(size)
        self._check(self.lib.scc_get(self.h, field, k, _ptr(out)), "scc_get")
        return out

    def eval_residual(self, t, zeta=None, xs=None):
        out = self.zeros(1 + self.nov + self.nov * self.nov)
        t = self._dev(t)
        z = None if zeta is None else self._dev(zeta)
        x = None if xs is None else self._dev(xs)
        self._check(self.lib.scc_eval_residual(self.h, _ptr(t), _ptr(z), _ptr(x), _ptr(out)),
                    "scc_eval_residual")
        return out

    def eval_sigma(self, vec):
        out = self.zeros(1 + self.nov + self.nov * self.nov)
        v = self._dev(vec)
        self._check(self.lib.scc_eval_sigma(self.h, _ptr(v), _ptr(out)), "scc_eval_sigma")
        return out

    def profile_kernels(self, kernels):
        """time only these GEMM kernels (ids) while profiling"""
        mask = 0
        for k in kernels:
            mask |= 1 << k
        self._check(self.lib.scc_profile_kernels(self.h, mask), "scc_profile_kernels")

    def profile(self, enable, kernel=GEMM_F64):
        """(milliseconds, flops, launches, bytes) of one GEMM kernel so far"""
        ms, fl, n, by = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_longlong(0), ctypes.c_double(0)
        self._check(self.lib.scc_profile(self.h, 1 if enable else 0, kernel, ctypes.byref(ms), ctypes.byref(fl),
                                         ctypes.byref(n), ctypes.byref(by)), "scc_profile")
        return ms.value, fl.value, n.value, by.value

    def eval_left(self, vec):
        out = self.zeros(1 + self.nov + self.nov * self.nov)
        v = self._dev(vec)
        self._check(self.lib.scc_eval_left(self.h, _ptr(v), _ptr(out)), "scc_eval_left")
        return out


# --- learned initial-guess model (include/scc_learn.h) -------------------------
def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _chk(rc, what):
    if rc != SCC_OK:
        raise SccError(rc, what)


class Mlp:
    """Tanh perceptron (nin, nhidden, nhidden, nout) in FP32 on the device;
    params is a flat float32 CUDA tensor [W1|b1|W2|b2|W3|b3]."""

    def __init__(self, nin, nhidden, nout, params, device="cuda:0"):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.d = MlpDims(nin, nhidden, nout)
        n = ctypes.c_longlong(0)
        _chk(self.lib.scc_mlp_param_count(ctypes.byref(self.d), ctypes.byref(n)), "scc_mlp_param_count")
        self.count = n.value
        self.params = torch.as_tensor(params, dtype=torch.float32).to(device).contiguous().clone()
        assert self.params.numel() == self.count
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.steps = 0
        self.device = device

    def _ws(self, batch):
        b = ctypes.c_size_t(0)
        _chk(self.lib.scc_mlp_workspace_bytes(ctypes.byref(self.d), batch, ctypes.byref(b)), "workspace")
        return self.torch.empty(b.value + 8 * (batch * (self.d.nin + self.d.nout) + self.count + 64),
                                dtype=self.torch.uint8, device=self.device)

    def _f32(self, a):
        return self.torch.as_tensor(a, dtype=self.torch.float32).to(self.device).contiguous()

    def forward(self, X):
        X = self._f32(X)
        Y = self.torch.empty((X.shape[0], self.d.nout), dtype=self.torch.float32, device=self.device)
        ws = self._ws(X.shape[0])
        _chk(self.lib.scc_mlp_forward(ctypes.byref(self.d), _ptr(self.params), X.shape[0], _ptr(X), _ptr(Y), _ptr(ws),
                                      ws.numel(), _stream()), "scc_mlp_forward")
        return Y

    def forward_noalloc(self, X):
        """As forward, without a workspace (library-owned device scratch)."""
        X = self._f32(X)
        Y = self.torch.empty((X.shape[0], self.d.nout), dtype=self.torch.float32, device=self.device)
        _chk(self.lib.scc_mlp_forward_noalloc(ctypes.byref(self.d), _ptr(self.params), X.shape[0], _ptr(X), _ptr(Y),
                                              _stream()), "scc_mlp_forward_noalloc")
        return Y

    def loss_grad(self, X, T):
        X, T = self._f32(X), self._f32(T)
        loss = self.torch.zeros(1, dtype=self.torch.float32, device=self.device)
        g = self.torch.empty_like(self.params)
        ws = self._ws(X.shape[0])
        _chk(self.lib.scc_mlp_loss_grad(ctypes.byref(self.d), _ptr(self.params), X.shape[0], _ptr(X), _ptr(T),
                                        _ptr(loss), _ptr(g), _ptr(ws), ws.numel(), _stream()), "scc_mlp_loss_grad")
        return float(loss.cpu()[0]), g

    def train(self, X, T, order, lr=1e-3):
        """order: int array [nsteps][batch] of sample indices."""
        import numpy as np
        X, T = self._f32(X), self._f32(T)
        order = np.asarray(order, dtype=np.int32)
        nsteps, batch = order.shape
        od = self.torch.as_tensor(order).to(self.device).contiguous()
        losses = self.torch.zeros(nsteps, dtype=self.torch.float32, device=self.device)
        ws = self._ws(batch)
        _chk(self.lib.scc_mlp_train(ctypes.byref(self.d), _ptr(self.params), _ptr(self.m), _ptr(self.v), X.shape[0],
                                    _ptr(X), _ptr(T), nsteps, batch, _ptr(od), float(lr), self.steps, _ptr(losses),
                                    _ptr(ws), ws.numel(), _stream()), "scc_mlp_train")
        self.steps += nsteps
        return losses.cpu().numpy()


def pca_fit(X, k):
    """X: float64 CUDA tensor [n][d] -> (mean [d], basis [k][d], coef [n][k], eigenvalues [k] host)."""
    import torch
    lib = load_library()
    X = X.to(torch.float64).contiguous()
    n, d = X.shape
    b = ctypes.c_size_t(0)
    _chk(lib.scc_pca_workspace_bytes(n, d, k, ctypes.byref(b)), "scc_pca_workspace_bytes")
    ws = torch.empty(b.value, dtype=torch.uint8, device=X.device)
    mean = torch.empty(d, dtype=torch.float64, device=X.device)
    basis = torch.empty((k, d), dtype=torch.float64, device=X.device)
    coef = torch.empty((n, k), dtype=torch.float64, device=X.device)
    w = (ctypes.c_double * k)()
    _chk(lib.scc_pca_fit(n, d, k, _ptr(X), _ptr(mean), _ptr(basis), _ptr(coef), ctypes.cast(w, ctypes.c_void_p),
                         _ptr(ws), ws.numel(), _stream()), "scc_pca_fit")
    return mean, basis, coef, list(w)


def pca_expand(mean, basis, coef):
    import torch
    lib = load_library()
    coef = coef.to(torch.float64).contiguous()
    m, k = coef.shape
    d = mean.numel()
    out = torch.empty((m, d), dtype=torch.float64, device=mean.device)
    _chk(lib.scc_pca_expand(m, d, k, _ptr(mean), _ptr(basis), _ptr(coef), _ptr(out), _stream()), "scc_pca_expand")
    return out
