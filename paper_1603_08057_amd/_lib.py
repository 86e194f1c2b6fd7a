"""ctypes binding of include/rsfgp.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
MATERN12, MATERN32, MATERN52, RQ, MATERN32_ANISO, RQ_ANISO = 0, 1, 2, 3, 4, 5

_ERRORS = {-1: "RSF_E_INVALID", -2: "RSF_E_NOT_SPD", -3: "RSF_E_OOM", -4: "RSF_E_HIP",
           -5: "RSF_E_DUPLICATE", -6: "RSF_E_NONFINITE"}


class RsfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_ERRORS.get(code, str(code)), msg))
        self.code = code
        self.name = _ERRORS.get(code, str(code))


PRECISIONS = {"fp64": 0, "mixed": 1}
PEELINGS = {"weak": 0, "strong": 1}


class Options(C.Structure):
    _fields_ = [("n_prox", C.c_int), ("prox_rings", C.c_int), ("r_near", C.c_double),
                ("prox_r_in", C.c_double), ("prox_r_out", C.c_double), ("rq_alpha", C.c_double),
                ("mem_cap_bytes", C.c_size_t), ("precision", C.c_int), ("with_score", C.c_int),
                ("peeling", C.c_int)]


class GradInfo(C.Structure):
    _fields_ = [("q", C.c_double * 3), ("t", C.c_double * 3), ("trace_inv", C.c_double),
                ("peel_levels", C.c_int), ("peel_cols", C.c_int * 32), ("peel_rank", C.c_int * 32),
                ("leaf_cols", C.c_int), ("seconds", C.c_double * 4)]


class TreeInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("depth", C.c_int), ("nbox", C.c_int), ("root_size", C.c_int),
                ("factor_bytes", C.c_int64)]


_lib = None


def library_path():
    return os.environ.get("RSFGP_LIB", os.path.join(HERE, "librsfgp.so"))


def load():
    """Loads librsfgp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError("librsfgp.so not built at %s (run paper_1603_08057_amd/build.py)" % path)
    lib = C.CDLL(path)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    sigs = {
        "rsf_opts_default": ([C.POINTER(Options)], C.c_int),
        "rsf_factor_create": ([vp, i64, dp, C.c_int, C.c_int, C.c_double, C.c_int, C.POINTER(Options), vp,
                               C.POINTER(vp)], C.c_int),
        "rsf_factor_destroy": ([vp], None),
        "rsf_logdet": ([vp, dp], C.c_int),
        "rsf_solve": ([vp, vp, vp, i64, i64, vp], C.c_int),
        "rsf_solve_noalloc": ([vp, vp, vp, i64, i64, vp], C.c_int),
        "rsf_apply": ([vp, vp, vp, i64, i64, vp], C.c_int),
        "rsf_apply_sqrt": ([vp, vp, vp, i64, i64, vp], C.c_int),
        "rsf_loglik": ([vp, vp, dp, vp, vp], C.c_int),
        "rsf_grad": ([vp, vp, C.c_double, C.c_uint64, dp, C.POINTER(GradInfo), vp], C.c_int),
        "rsf_tree_export": ([vp, C.POINTER(C.c_int32), C.POINTER(TreeInfo)], C.c_int),
        "rsf_skeleton_export": ([vp, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)], C.c_int),
        "rsf_last_error": ([], C.c_char_p),
        "rsf_factor_create_batched": ([C.POINTER(vp), C.POINTER(i64), C.c_int, dp, C.c_int, C.c_int, C.c_double,
                                       C.c_int, C.POINTER(Options), vp, C.POINTER(vp)], C.c_int),
        "rsf_batch_size": ([vp, C.POINTER(C.c_int)], C.c_int),
        "rsf_logdet_batched": ([vp, dp], C.c_int),
        "rsf_loglik_batched": ([vp, C.POINTER(vp), dp, vp], C.c_int),
        "rsf_grad_batched": ([vp, C.POINTER(vp), C.c_double, C.c_uint64, dp, C.POINTER(GradInfo), vp], C.c_int),
        "rsf_grad_hutch": ([vp, vp, C.c_int, C.c_uint64, dp, C.POINTER(GradInfo), vp], C.c_int),
        "rsf_cond_mean": ([vp, vp, vp, vp, C.c_int64, vp], C.c_int),
        "rsf_profile_loglik": ([vp, vp, C.c_double, C.c_uint64, dp, dp, C.POINTER(GradInfo), vp], C.c_int),
        "rsf_cond_sample": ([vp, vp, vp, vp, C.c_int64, vp], C.c_int),
        "rsf_grad_hutch_batched": ([vp, C.POINTER(vp), C.c_int, C.c_uint64, dp, C.POINTER(GradInfo), vp], C.c_int),
        "rsf_graph_state": ([vp, C.POINTER(C.c_int)], C.c_int),
        "rsf_trace_enable": ([C.c_int], C.c_int),
        "rsf_trace_read": ([dp, dp, dp, C.POINTER(C.c_int64), C.c_int], C.c_int),
        "rsf_trace_phases": ([C.c_char_p, C.c_size_t], C.c_int),
        "rsf_trace_busy": ([dp], C.c_int),
        "rsf_trace_kernels": ([C.c_char_p, C.c_size_t], C.c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise RsfError(rc, load().rsf_last_error().decode(errors="replace"))


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(x, shape=None):
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(x, dtype=torch.float64)
    x = x.to(device="cuda", dtype=torch.float64)
    if shape is not None:
        x = x.reshape(shape)
    return x.contiguous()


def _colmajor(b, n):
    """(n,) or (n, nrhs) tensor -> (device column-major buffer as (nrhs, n) tensor, nrhs, squeeze)."""
    b = _dev_f64(b)
    if b.dim() == 1:
        return b.reshape(1, n).contiguous(), 1, True
    return b.t().contiguous(), b.shape[1], False


def cond_mean(F, F22, z):
    """E[z' | z] = Sigma_12 Sigma_22^-1 z: F factors the joint sites [x'; x]
    (prediction sites first), F22 the observed sites x; z is (n2,) or
    (n2, k); returns (n1,) or (n1, k) on the device."""
    torch = _torch()
    n2, n1 = F22.n, F.n - F22.n
    cm, k, sq = _colmajor(z, n2)
    out = torch.empty((k, max(n1, 1)), dtype=torch.float64, device=cm.device)  # the library checks n1 >= 1
    _check(load().rsf_cond_mean(F._h, F22._h, C.c_void_p(cm.data_ptr()), C.c_void_p(out.data_ptr()), k, _stream()))
    return out.reshape(-1) if sq else out.t()


def cond_sample(F, F22, xi):
    """The conditional deviation S xi (S S^T = Sigma_11 - Sigma_12 Sigma_22^-1
    Sigma_21) for standard normal draws xi of size (n,) or (n, k), n = n1 + n2;
    a conditional sample is cond_mean(...) + this."""
    torch = _torch()
    n1 = F.n - F22.n
    cm, k, sq = _colmajor(xi, F.n)
    out = torch.empty((k, max(n1, 1)), dtype=torch.float64, device=cm.device)
    _check(load().rsf_cond_sample(F._h, F22._h, C.c_void_p(cm.data_ptr()), C.c_void_p(out.data_ptr()), k,
                                  _stream()))
    return out.reshape(-1) if sq else out.t()


def trace_enable(on=True):
    """Starts / stops event tracing of the batched matrix-core GEMM launches."""
    _check(load().rsf_trace_enable(1 if on else 0))


def trace_busy_ms():
    """Union of the traced launches' intervals (ms) as of the last trace_read."""
    out = C.c_double()
    _check(load().rsf_trace_busy(C.byref(out)))
    return out.value


def trace_kernels():
    """Algorithmic work per kernel while tracing was on: dict kernel ->
    (flops, bytes, dispatches); read before trace_read(reset=True)."""
    buf = C.create_string_buffer(1 << 16)
    _check(load().rsf_trace_kernels(buf, 1 << 16))
    out = {}
    for item in buf.value.decode().split(";"):
        if item:
            name, f, b, n = item.rsplit(":", 3)
            out[name] = (float(f), float(b), float(n))
    return out


def trace_read(reset=False, phases=False):
    """(kernel ms, flops, bytes, launches) accumulated while tracing was on;
    with phases=True also a dict phase -> (ms, flops)."""
    ms, fl, by, n = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
    _check(load().rsf_trace_read(C.byref(ms), C.byref(fl), C.byref(by), C.byref(n), 0))
    ph = {}
    if phases:
        buf = C.create_string_buffer(1 << 16)
        _check(load().rsf_trace_phases(buf, 1 << 16))
        for item in buf.value.decode().split(";"):
            if item:
                name, t, f = item.split(":")
                ph[name] = (float(t), float(f))
    if reset:
        _check(load().rsf_trace_read(None, None, None, None, 1))
    out = (ms.value, fl.value, by.value, n.value)
    return out + (ph,) if phases else out


class Factor:
    """F ~= Sigma(theta) for observation sites `points` (n x 2)."""

    def __init__(self, points, theta, kernel=MATERN32, eps=1e-6, leaf=64, n_prox=256, prox_rings=4,
                 r_near=1.8, prox_r_in=1.75, prox_r_out=2.45, rq_alpha=1.0, mem_cap_bytes=0,
                 precision="fp64", with_score=False, peeling="weak"):
        lib = load()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("rsfgp needs a HIP device")
        pts = _dev_f64(points)
        if pts.dim() != 2 or pts.shape[1] != 2:
            raise ValueError("points must be n x 2")
        self.n = pts.shape[0]
        self.points = pts
        opts = Options()
        lib.rsf_opts_default(C.byref(opts))
        opts.n_prox, opts.prox_rings, opts.r_near = n_prox, prox_rings, r_near
        opts.prox_r_in, opts.prox_r_out, opts.rq_alpha = prox_r_in, prox_r_out, rq_alpha
        opts.mem_cap_bytes = mem_cap_bytes
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
        opts.precision = PRECISIONS[precision]
        opts.with_score = 1 if with_score else 0
        if peeling not in PEELINGS:
            raise ValueError("peeling must be one of %s" % sorted(PEELINGS))
        opts.peeling = PEELINGS[peeling]
        self.precision = precision
        th = (C.c_double * 3)(*[float(v) for v in theta])
        h = C.c_void_p()
        _check(lib.rsf_factor_create(C.c_void_p(pts.data_ptr()), self.n, th, 3, int(kernel), float(eps),
                                     int(leaf), C.byref(opts), _stream(), C.byref(h)))
        self._h = h
        self.theta = tuple(float(v) for v in theta)

    def close(self):
        if getattr(self, "_h", None):
            load().rsf_factor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def logdet(self):
        out = C.c_double()
        _check(load().rsf_logdet(self._h, C.byref(out)))
        return out.value

    def _block(self, fn, b):
        torch = _torch()
        cm, nrhs, sq = _colmajor(b, self.n)
        out = torch.empty_like(cm)
        _check(fn(self._h, C.c_void_p(cm.data_ptr()), C.c_void_p(out.data_ptr()), nrhs, self.n, _stream()))
        return out.reshape(-1) if sq else out.t()

    def solve(self, b):
        return self._block(load().rsf_solve, b)

    def solve_noalloc(self, b):
        """F^-1 b with the library's fixed work space (no device allocation
        inside the library; the result tensor is allocated here)."""
        return self._block(load().rsf_solve_noalloc, b)

    def apply(self, x):
        return self._block(load().rsf_apply, x)

    def apply_sqrt(self, w):
        return self._block(load().rsf_apply_sqrt, w)

    def loglik(self, z, want_alpha=False):
        torch = _torch()
        z = _dev_f64(z, (self.n,))
        out = C.c_double()
        alpha = torch.empty_like(z) if want_alpha else None
        _check(load().rsf_loglik(self._h, C.c_void_p(z.data_ptr()), C.byref(out),
                                 C.c_void_p(alpha.data_ptr()) if want_alpha else None, _stream()))
        return (out.value, alpha) if want_alpha else out.value

    def grad(self, z, eps_peel=None, seed=0):
        z = _dev_f64(z, (self.n,))
        g = (C.c_double * 3)()
        info = GradInfo()
        eps_peel = float(eps_peel) if eps_peel is not None else -1.0
        _check(load().rsf_grad(self._h, C.c_void_p(z.data_ptr()), eps_peel, int(seed), g, C.byref(info),
                               _stream()))
        return [g[0], g[1], g[2]], info

    def profile_loglik(self, z, eps_peel=None, seed=0, grad=True):
        """Log profile likelihood (eq. prof) and, with grad, its gradient and info."""
        z = _dev_f64(z, (self.n,))
        ell = C.c_double()
        g = (C.c_double * 3)()
        info = GradInfo()
        eps_peel = float(eps_peel) if eps_peel is not None else -1.0
        _check(load().rsf_profile_loglik(self._h, C.c_void_p(z.data_ptr()), eps_peel, int(seed), C.byref(ell),
                                         g if grad else None, C.byref(info), _stream()))
        return (ell.value, [g[0], g[1], g[2]], info) if grad else ell.value

    def grad_hutch(self, z, nprobe, seed=0):
        """The score with Hutchinson trace estimates from nprobe Rademacher probes."""
        z = _dev_f64(z, (self.n,))
        g = (C.c_double * 3)()
        info = GradInfo()
        _check(load().rsf_grad_hutch(self._h, C.c_void_p(z.data_ptr()), int(nprobe), int(seed), g,
                                     C.byref(info), _stream()))
        return [g[0], g[1], g[2]], info

    @property
    def graph_state(self):
        """0: the log-likelihood graph is not recorded yet, 1: recorded (later
        loglik calls replay it), -1: eager only."""
        st = C.c_int()
        _check(load().rsf_graph_state(self._h, C.byref(st)))
        return st.value

    def tree_info(self, want_perm=False):
        info = TreeInfo()
        perm = (C.c_int32 * self.n)() if want_perm else None
        _check(load().rsf_tree_export(self._h, perm, C.byref(info)))
        d = {"n": info.n, "depth": info.depth, "nbox": info.nbox, "root_size": info.root_size,
             "factor_bytes": info.factor_bytes}
        if want_perm:
            d["perm"] = list(perm)
        return d

    def skeletons(self, level):
        """(offsets, caller indices) of the skeletons of the boxes at `level`."""
        nb = C.c_int32()
        _check(load().rsf_skeleton_export(self._h, level, None, None, C.byref(nb)))
        offs = (C.c_int32 * (nb.value + 1))()
        _check(load().rsf_skeleton_export(self._h, level, offs, None, C.byref(nb)))
        idx = (C.c_int32 * max(1, offs[nb.value]))()
        _check(load().rsf_skeleton_export(self._h, level, offs, idx, C.byref(nb)))
        return list(offs), list(idx)[:offs[nb.value]]


class BatchedFactor:
    """F_i ~= Sigma_i(theta_i) for independent instances, factored together:
    every quadtree level of all instances is one set of launches."""

    def __init__(self, points_list, thetas, kernel=MATERN32, eps=1e-6, leaf=64, n_prox=256, prox_rings=4,
                 r_near=1.8, prox_r_in=1.75, prox_r_out=2.45, rq_alpha=1.0, mem_cap_bytes=0,
                 precision="fp64", with_score=False, peeling="weak"):
        lib = load()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("rsfgp needs a HIP device")
        pts = [_dev_f64(p) for p in points_list]
        for p in pts:
            if p.dim() != 2 or p.shape[1] != 2:
                raise ValueError("points must be n x 2")
        self.nb = len(pts)
        self.ns = [int(p.shape[0]) for p in pts]
        self.points = pts
        th = [float(v) for t in thetas for v in t]
        if len(th) != 3 * self.nb:
            raise ValueError("need 3 parameters per instance")
        opts = Options()
        lib.rsf_opts_default(C.byref(opts))
        opts.n_prox, opts.prox_rings, opts.r_near = n_prox, prox_rings, r_near
        opts.prox_r_in, opts.prox_r_out, opts.rq_alpha = prox_r_in, prox_r_out, rq_alpha
        opts.mem_cap_bytes = mem_cap_bytes
        opts.precision = PRECISIONS[precision]
        opts.with_score = 1 if with_score else 0
        if peeling not in PEELINGS:
            raise ValueError("peeling must be one of %s" % sorted(PEELINGS))
        opts.peeling = PEELINGS[peeling]
        ptrs = (C.c_void_p * self.nb)(*[p.data_ptr() for p in pts])
        ns = (C.c_int64 * self.nb)(*self.ns)
        tharr = (C.c_double * len(th))(*th)
        h = C.c_void_p()
        _check(lib.rsf_factor_create_batched(ptrs, ns, self.nb, tharr, 3, int(kernel), float(eps), int(leaf),
                                             C.byref(opts), _stream(), C.byref(h)))
        self._h = h
        self.thetas = [tuple(t) for t in thetas]

    def close(self):
        if getattr(self, "_h", None):
            load().rsf_factor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, zs):
        zs = [_dev_f64(z).reshape(-1) for z in zs]
        if len(zs) != self.nb or any(z.numel() != m for z, m in zip(zs, self.ns)):
            raise ValueError("need one vector of n_i values per instance")
        return zs, (C.c_void_p * self.nb)(*[z.data_ptr() for z in zs])

    def apply_sqrt(self, ws):
        """[F_i^(1/2) w_i] for one vector per instance (draws from N(0, F_i))."""
        ws, _ = self._ptrs(ws)
        w = _torch().cat(ws)
        z = _torch().empty_like(w)
        _check(load().rsf_apply_sqrt(self._h, C.c_void_p(w.data_ptr()), C.c_void_p(z.data_ptr()), 1, w.numel(),
                                     _stream()))
        return list(_torch().split(z, self.ns))

    @property
    def logdets(self):
        out = (C.c_double * self.nb)()
        _check(load().rsf_logdet_batched(self._h, out))
        return list(out)

    def loglik(self, zs):
        zs, ptrs = self._ptrs(zs)
        out = (C.c_double * self.nb)()
        _check(load().rsf_loglik_batched(self._h, ptrs, out, _stream()))
        return list(out)

    def grad(self, zs, eps_peel=0.0, seed=0):
        """(nb x 3 scores, GradInfo of instance 0 and the shared peeling)."""
        zs, ptrs = self._ptrs(zs)
        g = (C.c_double * (3 * self.nb))()
        info = GradInfo()
        _check(load().rsf_grad_batched(self._h, ptrs, float(eps_peel), int(seed), g, C.byref(info), _stream()))
        return [tuple(g[3 * i:3 * i + 3]) for i in range(self.nb)], info

    def grad_hutch(self, zs, nprobe, seed=0):
        """Scores of every instance with Hutchinson trace estimates."""
        zs, ptrs = self._ptrs(zs)
        g = (C.c_double * (3 * self.nb))()
        info = GradInfo()
        _check(load().rsf_grad_hutch_batched(self._h, ptrs, int(nprobe), int(seed), g, C.byref(info), _stream()))
        return [tuple(g[3 * i:3 * i + 3]) for i in range(self.nb)], info

    def tree_info(self):
        info = TreeInfo()
        _check(load().rsf_tree_export(self._h, None, C.byref(info)))
        return {"n": info.n, "depth": info.depth, "nbox": info.nbox, "root_size": info.root_size,
                "factor_bytes": info.factor_bytes}
