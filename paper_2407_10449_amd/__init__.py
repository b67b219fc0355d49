"""Linear elliptical slice sampling on MI355X (gfx950).

Python binding of libess (include/ess.h).  The functions below carry the C
names and only marshal arguments: every step of a transition runs in the HIP
kernels of libess.so.  PyTorch supplies device memory and the stream.

The library must have been built (``python -m paper_2407_10449_amd.build`` or
``__graft_entry__.build()``); importing the binding does not build it, and
every call fails loudly if it is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libess.so")

ESS_OK = 0
ESS_ERR_INVALID_ARG = 1
ESS_ERR_INFEASIBLE_START = 2
ESS_ERR_HIP = 3
ESS_ERR_OOM = 4
ESS_ERR_UNSUPPORTED = 5
ESS_X0_BROADCAST = 1
ESS_SORT_FULL = 2
ESS_LIKELIHOOD_MIDPOINT = 16
ESS_BRUTE_FORCE = 32
ESS_PER_CHAIN_B = 4
ESS_EAGER = 8

STATUS_NAMES = {0: "ESS_OK", 1: "ESS_ERR_INVALID_ARG", 2: "ESS_ERR_INFEASIBLE_START",
                3: "ESS_ERR_HIP", 4: "ESS_ERR_OOM", 5: "ESS_ERR_UNSUPPORTED"}


class EssError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class EssProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("m", ctypes.c_int32), ("n_chains", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("A", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("trim_eps", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


_LIB = None

_P = ctypes.c_void_p
_SIGS = {
    "ess_init": ([ctypes.POINTER(EssProblem), _P, ctypes.POINTER(_P)], ctypes.c_int),
    "ess_init_batched": ([ctypes.POINTER(EssProblem), ctypes.c_int32, _P, ctypes.POINTER(_P)],
                         ctypes.c_int),
    "ess_step": ([_P, _P], ctypes.c_int),
    "ess_run": ([_P, ctypes.c_int64, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ess_get_state": ([_P, _P, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "ess_set_state": ([_P, _P, ctypes.c_uint64], ctypes.c_int),
    "ess_rejections": ([_P, _P], ctypes.c_int),
    "ess_transition_explicit": ([_P] * 10, ctypes.c_int),
    "ess_transition_explicit_static": ([ctypes.c_int32] * 4 + [_P, _P, ctypes.c_double] + [_P] * 9,
                                       ctypes.c_int),
    "ess_draw": ([_P, ctypes.c_uint64, _P, _P], ctypes.c_int),
    "ess_profile": ([_P, ctypes.c_int], ctypes.c_int),
    "ess_profile_read": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "ess_set_state_gated": ([_P, _P, _P, ctypes.c_uint64, _P], ctypes.c_int),
    "ess_mlp_create": ([ctypes.c_int32, _P, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "ess_mlp_num_params": ([_P], ctypes.c_int64),
    "ess_mlp_set_params": ([_P, _P], ctypes.c_int),
    "ess_mlp_get_params": ([_P, _P], ctypes.c_int),
    "ess_mlp_forward": ([_P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "ess_mlp_gradients": ([_P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)],
                          ctypes.c_int),
    "ess_mlp_adam": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
                     ctypes.c_int),
    "ess_mlp_destroy": ([_P], None),
    "ess_autotune": ([_P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32], ctypes.c_int),
    "ess_destroy": ([_P], None),
    "ess_cholesky": ([_P, ctypes.c_int32, _P], ctypes.c_int),
    "ess_whiten": ([_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P],
                   ctypes.c_int),
    "ess_unwhiten": ([_P, ctypes.c_int64, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P],
                     ctypes.c_int),
    "ess_last_error": ([], ctypes.c_char_p),
}


def lib():
    """The loaded libess.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        # torch first: libess.so must bind to the HIP runtime torch has loaded
        # (loading libess.so first brings in a second runtime, which then sees
        # no device)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libess.so is not built at {LIB_PATH}; run "
                              "`python -m paper_2407_10449_amd.build` first")
        h = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = h
    return _LIB


def _check(status):
    if status != ESS_OK:
        raise EssError(status, lib().ess_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ----------------------------------------------------------- C-named calls
def ess_init(problem, stream=None):
    ctx = ctypes.c_void_p()
    _check(lib().ess_init(ctypes.byref(problem), _stream_handle(stream), ctypes.byref(ctx)))
    return ctx


def ess_init_batched(problems, stream=None):
    """problems: a sequence of EssProblem."""
    arr = (EssProblem * len(problems))(*problems)
    ctx = ctypes.c_void_p()
    _check(lib().ess_init_batched(arr, len(problems), _stream_handle(stream), ctypes.byref(ctx)))
    return ctx


def ess_step(ctx, x_out=None):
    _check(lib().ess_step(ctx, _ptr(x_out)))


def ess_run(ctx, n_steps, thin=1, trace=None, want_rejections=False):
    nrej = ctypes.c_int64(0)
    _check(lib().ess_run(ctx, int(n_steps), int(thin), _ptr(trace),
                         ctypes.byref(nrej) if want_rejections else None))
    return nrej.value if want_rejections else None


def ess_get_state(ctx, x_out=None):
    step = ctypes.c_uint64(0)
    _check(lib().ess_get_state(ctx, _ptr(x_out), ctypes.byref(step)))
    return step.value


def ess_set_state(ctx, x_in, step):
    _check(lib().ess_set_state(ctx, _ptr(x_in), int(step)))


def ess_set_state_gated(ctx, x_candidate, x_fallback, step, n_chains):
    acc = np.zeros(n_chains, dtype=np.int32)
    _check(lib().ess_set_state_gated(ctx, _ptr(x_candidate), _ptr(x_fallback), int(step),
                                     acc.ctypes.data_as(ctypes.c_void_p)))
    return acc


def ess_mlp_create(widths, stream=None):
    w = (ctypes.c_int32 * len(widths))(*widths)
    net = ctypes.c_void_p()
    _check(lib().ess_mlp_create(len(widths) - 1, w, _stream_handle(stream), ctypes.byref(net)))
    return net


def ess_mlp_num_params(net):
    return int(lib().ess_mlp_num_params(net))


def ess_mlp_set_params(net, params):
    _check(lib().ess_mlp_set_params(net, _ptr(params)))


def ess_mlp_get_params(net, params):
    _check(lib().ess_mlp_get_params(net, _ptr(params)))


def ess_mlp_forward(net, inp, out):
    _check(lib().ess_mlp_forward(net, _ptr(inp), int(inp.shape[0]), _ptr(out)))


def ess_mlp_gradients(net, inp, target, grads=None, want_loss=True):
    loss = ctypes.c_double(0.0)
    _check(lib().ess_mlp_gradients(net, _ptr(inp), _ptr(target), int(inp.shape[0]), _ptr(grads),
                                   ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def ess_mlp_adam(net, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().ess_mlp_adam(net, float(lr), float(beta1), float(beta2), float(eps)))


def ess_mlp_destroy(net):
    if net:
        lib().ess_mlp_destroy(net)


def ess_rejections(ctx, n_chains):
    out = np.zeros(n_chains, dtype=np.int64)
    _check(lib().ess_rejections(ctx, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def ess_transition_explicit(ctx, x, nu, u, x_new, intervals=None, n_intervals=None,
                            theta=None, rejected=None, pq=None):
    _check(lib().ess_transition_explicit(ctx, _ptr(x), _ptr(nu), _ptr(u), _ptr(x_new),
                                         _ptr(intervals), _ptr(n_intervals), _ptr(theta),
                                         _ptr(rejected), _ptr(pq)))


def ess_transition_explicit_static(d, m, n_chains, precision, A, b, trim_eps, x, nu, u, x_new,
                                   intervals=None, n_intervals=None, theta=None, rejected=None,
                                   stream=None):
    """The context-free transition that allocates no device memory (its
    buffers live in the library's static array)."""
    _check(lib().ess_transition_explicit_static(
        int(d), int(m), int(n_chains), int(precision), _ptr(A), _ptr(b), float(trim_eps), _ptr(x),
        _ptr(nu), _ptr(u), _ptr(x_new), _ptr(intervals), _ptr(n_intervals), _ptr(theta),
        _ptr(rejected), _stream_handle(stream)))


def ess_draw(ctx, step, nu=None, u=None):
    _check(lib().ess_draw(ctx, int(step), _ptr(nu), _ptr(u)))


ESS_KERNEL_PROJECT = 0
ESS_KERNEL_SAMPLE = 1
ESS_KERNEL_OTHER = 2
ESS_KERNEL_BATCHED = 3


def ess_profile(ctx, enable):
    _check(lib().ess_profile(ctx, int(bool(enable))))


def ess_profile_read(ctx, kind):
    """(total milliseconds, launch count) of one kernel kind since the last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().ess_profile_read(ctx, int(kind), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def ess_autotune(ctx, steps_per_trial=8):
    """Tunes the context in place; returns the per-trial report."""
    buf = ctypes.create_string_buffer(8192)
    _check(lib().ess_autotune(ctx, int(steps_per_trial), buf, len(buf)))
    return buf.value.decode()


def ess_destroy(ctx):
    if ctx:
        lib().ess_destroy(ctx)


def ess_last_error():
    return lib().ess_last_error().decode()


# ----------------------------------------------------------- convenience
def ess_cholesky(sigma):
    """Host Cholesky factor (float64, lower) of a host matrix."""
    sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64))
    d = sig.shape[0]
    L = np.empty_like(sig)
    _check(lib().ess_cholesky(sig.ctypes.data_as(_P), d, L.ctypes.data_as(_P)))
    return L


def ess_whiten(A, b, L, mu, A_out, b_out, precision, stream=None):
    m, d = A.shape
    _check(lib().ess_whiten(_ptr(A), _ptr(b), _ptr(L), _ptr(mu), m, d, precision, _ptr(A_out),
                            _ptr(b_out), _stream_handle(stream)))


def ess_unwhiten(U, L, mu, X_out, precision, stream=None):
    d = U.shape[-1]
    n = U.numel() // d
    _check(lib().ess_unwhiten(_ptr(U), n, d, _ptr(L), _ptr(mu), precision, _ptr(X_out),
                              _stream_handle(stream)))


class Gaussian:
    """Appendix A: x ~ N(mu, Sigma) truncated to {A x <= b} as x = L u + mu,
    u ~ N(0, I) truncated to {(A L) u <= b - A mu}.  Give Sigma (factored by
    the library's host Cholesky) or its lower factor L.  `A`, `b` hold the
    whitened problem on the device (for Sampler, whose start is given in u:
    u = 0 is x = mu); map() takes states or traces of u back to x."""

    def __init__(self, A, b, mu, Sigma=None, L=None, precision=32, device="cuda", stream=None):
        import torch
        if (Sigma is None) == (L is None):
            raise ValueError("give exactly one of Sigma and L")
        self.torch = torch
        self.precision = precision
        self.dtype = torch.float32 if precision == 32 else torch.float64
        self.device = torch.device(device)
        self.stream = stream
        if L is None:
            L = ess_cholesky(np.asarray(Sigma, dtype=np.float64))
        self.L = torch.as_tensor(np.asarray(L, dtype=np.float64)).to(self.device).contiguous()
        self.mu = torch.as_tensor(np.asarray(mu, dtype=np.float64)).to(self.device).contiguous()
        A_in = torch.as_tensor(np.asarray(A)).to(self.device, self.dtype).contiguous()
        b_in = torch.as_tensor(np.asarray(b, dtype=np.float64)).to(self.device).contiguous()
        self.A = torch.empty_like(A_in)
        self.b = torch.empty_like(b_in)
        ess_whiten(A_in, b_in, self.L, self.mu, self.A, self.b, precision, stream)

    def map(self, U, out=None):
        """x = L u + mu for every row u of U (states (C, d) or traces (T, C, d))."""
        U = U.contiguous()
        if out is None:
            out = self.torch.empty_like(U)
        ess_unwhiten(U, self.L, self.mu, out, self.precision, self.stream)
        return out


def _same_device(a, b):
    import torch
    a, b = torch.device(a), torch.device(b)
    if a.type != b.type:
        return False
    if a.type != "cuda":
        return True
    cur = torch.cuda.current_device()
    return (cur if a.index is None else a.index) == (cur if b.index is None else b.index)


def _check_out(out, shape, dtype, device):
    if (tuple(out.shape) != tuple(shape) or out.dtype != dtype
            or not _same_device(out.device, device) or not out.is_contiguous()):
        raise ValueError(f"trace buffer must be a contiguous {dtype} tensor of shape {shape} "
                         f"on {device}, got {tuple(out.shape)} {out.dtype} on {out.device}")


class Sampler:
    """Owns one ess_ctx.  A, b, x0 may be numpy arrays or torch tensors; they
    are copied to the device in the working precision before ess_init.

    b of shape (n_chains, m) gives every chain its own right-hand side.
    full_sort=True builds every chain's intervals with the full sort (the same
    intervals); method="midpoint" uses Section 2.2's likelihood testing at
    midpoints and method="alg2" Algorithm 2's sequential intersection instead
    of Algorithm 3 (the quadratic comparators, m <= 4096);
    eager=True launches kernel by kernel instead of replaying a HIP graph."""

    def __init__(self, A, b, x0, n_chains, seed=0, precision=32, trim_eps=None,
                 device="cuda", stream=None, full_sort=False, eager=False, method="alg3"):
        import torch
        self.torch = torch
        self.dtype = torch.float32 if precision == 32 else torch.float64
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream
        A = torch.as_tensor(np.asarray(A) if not torch.is_tensor(A) else A)
        self.m, self.d = A.shape
        self.n_chains = int(n_chains)
        self.A = A.to(self.device, self.dtype).contiguous()
        self.b = torch.as_tensor(np.asarray(b) if not torch.is_tensor(b) else b).to(
            self.device, torch.float64).contiguous()
        x0 = torch.as_tensor(np.asarray(x0) if not torch.is_tensor(x0) else x0).to(
            self.device, self.dtype).contiguous()
        flags = (ESS_X0_BROADCAST if x0.dim() == 1 else 0) | (ESS_SORT_FULL if full_sort else 0)
        if self.b.dim() == 2:       # one right-hand side per chain
            flags |= ESS_PER_CHAIN_B
        if eager:
            flags |= ESS_EAGER
        if method == "midpoint":    # Section 2.2's likelihood testing (comparator)
            flags |= ESS_LIKELIHOOD_MIDPOINT
        elif method == "alg2":      # Algorithm 2's sequential intersection (comparator)
            flags |= ESS_BRUTE_FORCE
        elif method != "alg3":
            raise ValueError("method must be 'alg3', 'alg2' or 'midpoint'")
        if trim_eps is None:
            trim_eps = 1e-6 if precision == 32 else 0.0
        self.trim_eps = float(trim_eps)
        self.problem = EssProblem(self.d, self.m, self.n_chains, precision, self.A.data_ptr(),
                                  self.b.data_ptr(), x0.data_ptr(), int(seed), self.trim_eps, flags)
        self.ctx = ess_init(self.problem, stream)

    def _empty(self, *shape, dtype=None):
        return self.torch.empty(*shape, device=self.device, dtype=dtype or self.dtype)

    def step(self):
        x = self._empty(self.n_chains, self.d)
        ess_step(self.ctx, x)
        return x

    def run(self, n_steps, thin=1, keep_trace=True, count_rejections=True, out=None):
        """n_steps transitions; the trace (every thin-th state) goes to `out`
        when given (a reused buffer lets later runs replay the same captured
        graph), else to a new tensor."""
        shape = (n_steps // thin, self.n_chains, self.d)
        if out is not None:
            _check_out(out, shape, self.dtype, self.device)
            tr = out
        else:
            tr = self._empty(*shape) if keep_trace and n_steps // thin else None
        nrej = ess_run(self.ctx, n_steps, thin, tr, count_rejections)
        return tr, nrej

    def state(self):
        x = self._empty(self.n_chains, self.d)
        step = ess_get_state(self.ctx, x)
        return x, step

    def set_state(self, x, step):
        x = self.torch.as_tensor(x).to(self.device, self.dtype).contiguous()
        ess_set_state(self.ctx, x, step)

    def rejections(self):
        return ess_rejections(self.ctx, self.n_chains)

    def set_state_gated(self, x_candidate, x_fallback, step=0):
        t = self.torch
        xc = t.as_tensor(x_candidate).to(self.device, self.dtype).contiguous()
        xf = t.as_tensor(x_fallback).to(self.device, self.dtype).contiguous()
        return ess_set_state_gated(self.ctx, xc, xf, step, self.n_chains)

    def draw(self, step):
        nu = self._empty(self.n_chains, self.d)
        u = self._empty(self.n_chains, dtype=self.torch.float64)
        ess_draw(self.ctx, step, nu, u)
        return nu, u

    def transition_explicit(self, x, nu, u):
        t = self.torch
        x = t.as_tensor(x).to(self.device, self.dtype).contiguous()
        nu = t.as_tensor(nu).to(self.device, self.dtype).contiguous()
        u = t.as_tensor(u).to(self.device, t.float64).contiguous()
        C, m = self.n_chains, self.m
        out = dict(x_new=self._empty(C, self.d),
                   intervals=t.zeros(C, m + 1, 2, device=self.device, dtype=t.float64),
                   n_intervals=t.zeros(C, device=self.device, dtype=t.int32),
                   theta=t.zeros(C, device=self.device, dtype=t.float64),
                   rejected=t.zeros(C, device=self.device, dtype=t.int32),
                   pq=t.zeros(2, C, m, device=self.device, dtype=self.dtype))
        ess_transition_explicit(self.ctx, x, nu, u, out["x_new"], out["intervals"],
                                out["n_intervals"], out["theta"], out["rejected"], out["pq"])
        return out

    def close(self):
        if getattr(self, "ctx", None):
            ess_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedSampler:
    """Owns one batched ess_ctx over several problems (float32).

    problems: sequence of dicts with keys A, b, x0, n_chains and optionally
    seed and trim_eps.  State and trace tensors hold the problems one after
    another, each as n_chains x d; `split` cuts them per problem."""

    def __init__(self, problems, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.keep = []
        probs = []
        self.shapes = []
        for pr in problems:
            A = torch.as_tensor(np.asarray(pr["A"])).to(self.device, torch.float32).contiguous()
            b = torch.as_tensor(np.asarray(pr["b"])).to(self.device, torch.float64).contiguous()
            x0 = torch.as_tensor(np.asarray(pr["x0"])).to(self.device, torch.float32).contiguous()
            m, d = A.shape
            C = int(pr["n_chains"])
            flags = ESS_X0_BROADCAST if x0.dim() == 1 else 0
            probs.append(EssProblem(d, m, C, 32, A.data_ptr(), b.data_ptr(), x0.data_ptr(),
                                    int(pr.get("seed", 0)), float(pr.get("trim_eps", 1e-6)), flags))
            self.keep += [A, b, x0]
            self.shapes.append((C, d))
        self.n_state = sum(C * d for C, d in self.shapes)
        self.n_chains = sum(C for C, _ in self.shapes)
        self.ctx = ess_init_batched(probs, stream)

    def split(self, flat):
        """(..., sum C d) -> list of (..., C, d) views, one per problem."""
        out, off = [], 0
        for C, d in self.shapes:
            out.append(flat[..., off:off + C * d].reshape(*flat.shape[:-1], C, d))
            off += C * d
        return out

    def run(self, n_steps, thin=1, keep_trace=True, count_rejections=True, out=None):
        t = self.torch
        shape = (n_steps // thin, self.n_state)
        if out is not None:
            _check_out(out, shape, t.float32, self.device)
            tr = out
        else:
            tr = (t.empty(*shape, device=self.device, dtype=t.float32)
                  if keep_trace and n_steps // thin else None)
        nrej = ess_run(self.ctx, n_steps, thin, tr, count_rejections)
        return tr, nrej

    def state(self):
        x = self.torch.empty(self.n_state, device=self.device, dtype=self.torch.float32)
        step = ess_get_state(self.ctx, x)
        return x, step

    def set_state(self, x, step):
        x = self.torch.as_tensor(x).to(self.device, self.torch.float32).contiguous()
        ess_set_state(self.ctx, x, step)

    def rejections(self):
        return ess_rejections(self.ctx, self.n_chains)

    def close(self):
        if getattr(self, "ctx", None):
            ess_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The warm-start network (bfloat16 matrix-core kernels, float32 masters)."""

    def __init__(self, widths, params=None, seed=0, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.widths = list(widths)
        self.device = torch.device(device)
        self.net = ess_mlp_create(self.widths, stream)
        self.n_params = ess_mlp_num_params(self.net)
        if params is None:
            params = self.init_params(seed)
        self.set_params(params)

    def init_params(self, seed):
        """Glorot-uniform weights, zero biases (host numpy, seeded)."""
        rng = np.random.default_rng(seed)
        parts = []
        for i, o in zip(self.widths[:-1], self.widths[1:]):
            lim = np.sqrt(6.0 / (i + o))
            parts += [rng.uniform(-lim, lim, size=o * i), np.zeros(o)]
        return np.concatenate(parts).astype(np.float32)

    def unflatten(self, flat):
        """flat -> [(W (out, in), c (out,))] (numpy)."""
        flat = np.asarray(flat)
        out, off = [], 0
        for i, o in zip(self.widths[:-1], self.widths[1:]):
            W = flat[off:off + o * i].reshape(o, i)
            off += o * i
            c = flat[off:off + o]
            off += o
            out.append((W, c))
        return out

    def set_params(self, flat):
        t = self.torch
        p = t.as_tensor(np.asarray(flat, dtype=np.float32)).to(self.device).contiguous()
        ess_mlp_set_params(self.net, p)

    def params(self):
        p = self.torch.empty(self.n_params, device=self.device, dtype=self.torch.float32)
        ess_mlp_get_params(self.net, p)
        return p

    def forward(self, inp):
        t = self.torch
        inp = t.as_tensor(inp).to(self.device, t.float32).contiguous()
        out = t.empty(inp.shape[0], self.widths[-1], device=self.device, dtype=t.float32)
        ess_mlp_forward(self.net, inp, out)
        return out

    def gradients(self, inp, target):
        t = self.torch
        inp = t.as_tensor(inp).to(self.device, t.float32).contiguous()
        target = t.as_tensor(target).to(self.device, t.float32).contiguous()
        g = t.empty(self.n_params, device=self.device, dtype=t.float32)
        loss = ess_mlp_gradients(self.net, inp, target, g)
        return g, loss

    def train_step(self, inp, target, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        loss = ess_mlp_gradients(self.net, inp, target, None, want_loss=False)
        ess_mlp_adam(self.net, lr, beta1, beta2, eps)
        return loss

    def close(self):
        if getattr(self, "net", None):
            ess_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
