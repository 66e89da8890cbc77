"""Python front end of the DMPT library: torch tensors in, torch tensors out.

PyTorch is used only for device memory and streams; every operation of the
method runs in libdmpt.so (the C ABI of include/dmpt.h).  A Context works in
order with torch's current stream at the time it is created: a side stream
is handed to the library as its stream; torch's default (null) stream is
handed over as NULL, and the library then orders its private stream after
the null stream's queued work at every call (see dmpt_init).
All matrices are N x N float64 CUDA (HIP) tensors; inputs are used through
their symmetric part.
"""
import ctypes
import math

from . import _lib as L


class DMPTError(RuntimeError):
    """A non-OK status from the library; ``status`` holds the code."""

    def __init__(self, status, msg, stats=None):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.stats = stats


class Response(tuple):
    """(P0, [P1], [P2], mu_jet, stats) of a canonical solve; .P3 holds [P3] (order 3)."""

    def __new__(cls, P0, P1, P2, mu, stats, P3=()):
        r = super().__new__(cls, (P0, P1, P2, mu, stats))
        r.P3 = list(P3)
        return r


class Pass(tuple):
    """(P0, [P1], [P2], stats) of one pass at a fixed mu jet; .P3 holds [P3] (order 3)."""

    def __new__(cls, P0, P1, P2, stats, P3=()):
        r = super().__new__(cls, (P0, P1, P2, stats))
        r.P3 = list(P3)
        return r


def _torch():
    import torch
    return torch


def options(prec="fp64", solver="cg", guess="prev", tol_occ=0.0, tol_cg=0.0, max_newton=50,
            max_cg=60, refine=0, ckpt_every=5, check=0, staged=1, warm_traj=1, schedule=1,
            acc64=1, autotune=0, grouped=1):
    """Build an options struct; 0 tolerances select the precision's defaults."""
    lib = L.load()
    o = L.Options()
    lib.dmpt_default_options(ctypes.byref(o))
    o.prec = L.PREC[prec] if isinstance(prec, str) else int(prec)
    o.solver = L.SOLVER[solver] if isinstance(solver, str) else int(solver)
    o.guess = L.GUESS[guess] if isinstance(guess, str) else int(guess)
    o.tol_occ, o.tol_cg = float(tol_occ), float(tol_cg)
    o.max_newton, o.max_cg, o.refine = int(max_newton), int(max_cg), int(refine)
    o.ckpt_every, o.check, o.staged = int(ckpt_every), int(check), int(staged)
    o.warm_traj = int(warm_traj)
    o.schedule = int(schedule)
    o.acc64 = int(acc64)
    o.autotune = int(autotune)
    o.grouped = int(grouped)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _ptr_array(ts):
    if ts is None:
        return None
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr() if t is not None else None
    return arr


def _check_mat(t, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (n, n):
        raise ValueError(f"{name} must be a contiguous ({n}, {n}) float64 GPU tensor")


class Context:
    """A library context (device workspace for N <= n_max, dirs_max directions).

    ``stream`` (default: torch's current stream on ``device``) is the stream the
    context's calls are ordered with for its whole life."""

    def __init__(self, n_max, dirs_max=1, device=0, stream=None, **opts):
        torch = _torch()
        self.lib = L.load()
        self.device = device
        self.opts = options(**opts)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.dmpt_init(ctypes.byref(h), device, int(n_max), int(dirs_max),
                                ctypes.byref(self.opts), ctypes.c_void_p(stream.cuda_stream))
        if st != L.DMPT_OK:
            raise DMPTError(st, self.lib.dmpt_last_error(None).decode())
        self.h = h
        self.n_max, self.dirs_max = n_max, dirs_max

    def close(self):
        if getattr(self, "h", None):
            self.lib.dmpt_finalize(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_options(self, **opts):
        o = options(**opts)
        st = self.lib.dmpt_set_options(self.h, ctypes.byref(o))
        self._raise(st)
        self.opts = o

    def _raise(self, st, stats=None):
        if st != L.DMPT_OK:
            raise DMPTError(st, self.lib.dmpt_last_error(self.h).decode(), stats)

    def _empty(self, n):
        torch = _torch()
        return torch.empty((n, n), dtype=torch.float64, device=f"cuda:{self.device}")

    def profile(self, enable=True):
        """Start (resetting the totals) or stop device timing of every product launch."""
        self._raise(self.lib.dmpt_profile(self.h, 1 if enable else 0))

    def profile_get(self):
        """Totals since the last reset: launches, ms, mfma_flops, useful_flops, and per engine."""
        d = L.ProfileData()
        self._raise(self.lib.dmpt_profile_get(self.h, ctypes.byref(d)))
        names = ["fp64", "fp32", "bf16x3", "bf16x6", "int8x13", "int8x6"]
        return dict(launches=d.launches, ms=d.ms, mfma_flops=d.mfma_flops,
                    useful_flops=d.useful_flops,
                    engines={names[i]: dict(launches=d.eng_launches[i], ms=d.eng_ms[i],
                                            mfma_flops=d.eng_mfma_flops[i], bytes=d.eng_bytes[i],
                                            useful_flops=d.eng_useful_flops[i])
                         for i in range(len(names))})

    def bench_product(self, N, prec=None, variant=0, reps=10):
        """Mean device ms and TFLOP/s of the product kernel (a variant) alone at size N."""
        p = self.opts.prec if prec is None else L.PREC[prec]
        ms, tf = ctypes.c_double(), ctypes.c_double()
        self._raise(self.lib.dmpt_bench_product(self.h, int(N), int(p), int(variant), int(reps),
                                                ctypes.byref(ms), ctypes.byref(tf)))
        return ms.value, tf.value

    def autotune(self, N):
        """Pick the fastest product-kernel variant for size N (kept for later calls)."""
        t = ctypes.c_int()
        self._raise(self.lib.dmpt_autotune(self.h, int(N), ctypes.byref(t)))
        return t.value

    def set_variant(self, N, variant, prec=None):
        """Pin a product-kernel variant for the padded size of N."""
        p = self.opts.prec if prec is None else L.PREC[prec]
        self._raise(self.lib.dmpt_set_variant(self.h, int(N), int(p), int(variant)))

    def get_variant(self, N, prec=None):
        """(variant, tuned, name) the products at the padded size of N use."""
        p = self.opts.prec if prec is None else L.PREC[prec]
        v, t = ctypes.c_int(), ctypes.c_int()
        buf = ctypes.create_string_buffer(96)
        self._raise(self.lib.dmpt_get_variant(self.h, int(N), int(p), ctypes.byref(v), ctypes.byref(t),
                                              buf, 96))
        return v.value, bool(t.value), buf.value.decode()

    # ------------------------------------------------------------------ calls
    def fermi_recursion(self, H0, beta, mu, n, out=None):
        """Grand-canonical P0 at fixed mu (Eq. Rec_F_2).  Returns (P0, stats)."""
        N = H0.shape[0]
        _check_mat(H0, N, "H0")
        P0 = out if out is not None else self._empty(N)
        s = L.Stats()
        st = self.lib.dmpt_fermi_recursion(self.h, N, _ptr(H0), float(beta), float(mu), int(n),
                                           _ptr(P0), ctypes.byref(s))
        self._raise(st, s)
        return P0, s.as_dict()

    def response(self, H0, H1=(), H2=None, beta=1.0, n=20, order=0, mu=(0.0,), raise_on_error=True,
                 H3=None):
        """One pass at a fixed mu jet (orders 0..3).  Returns Pass(P0, [P1], [P2], stats), .P3."""
        N = H0.shape[0]
        _check_mat(H0, N, "H0")
        d = len(H1) if order >= 1 else 0
        for i, h in enumerate(H1[:d]):
            _check_mat(h, N, f"H1[{i}]")
        h2 = None
        if order >= 2 and H2 is not None:
            for i, h in enumerate(H2):
                if h is not None:
                    _check_mat(h, N, f"H2[{i}]")
            h2 = _ptr_array(list(H2))
        h3 = self._opt_mats(H3, N, "H3") if order >= 3 else None
        mu = [float(m) for m in mu]
        if len(mu) < 1 + order * d:
            raise ValueError(f"mu must hold 1 + order*d = {1 + order * d} values")
        P0 = self._empty(N)
        P1 = [self._empty(N) for _ in range(d)] if order >= 1 else []
        P2 = [self._empty(N) for _ in range(d)] if order >= 2 else []
        P3 = [self._empty(N) for _ in range(d)] if order >= 3 else []
        s = L.Stats()
        mu_arr = (ctypes.c_double * len(mu))(*mu)
        st = self.lib.dmpt_response(self.h, N, _ptr(H0), d, _ptr_array(list(H1[:d])), h2, h3,
                                    float(beta), int(n), int(order), mu_arr, _ptr(P0),
                                    _ptr_array(P1) if P1 else None, _ptr_array(P2) if P2 else None,
                                    _ptr_array(P3) if P3 else None, ctypes.byref(s))
        stats = s.as_dict(d, order)
        if raise_on_error:
            self._raise(st, stats)
        stats["status"] = st
        return Pass(P0, P1, P2, stats, P3)

    def mu_newton(self, H0, H1=(), H2=None, beta=1.0, Ne=1.0, n=20, order=0, mu=None,
                  raise_on_error=True, H3=None):
        """Canonical response (Algorithm 1, orders 0..3).

        Returns Response(P0, [P1], [P2], mu_jet, stats) with .P3 ([P3] for order 3).
        """
        N = H0.shape[0]
        _check_mat(H0, N, "H0")
        d = len(H1) if order >= 1 else 0
        for i, h in enumerate(H1[:d]):
            _check_mat(h, N, f"H1[{i}]")
        h2 = None
        if order >= 2 and H2 is not None:
            for i, h in enumerate(H2):
                if h is not None:
                    _check_mat(h, N, f"H2[{i}]")
            h2 = _ptr_array(list(H2))
        h3 = self._opt_mats(H3, N, "H3") if order >= 3 else None
        nmu = 1 + order * d
        m = [math.nan] * nmu
        if mu is not None:
            for i, v in enumerate(mu[:nmu]):
                m[i] = float(v)
        mu_arr = (ctypes.c_double * nmu)(*m)
        P0 = self._empty(N)
        P1 = [self._empty(N) for _ in range(d)] if order >= 1 else []
        P2 = [self._empty(N) for _ in range(d)] if order >= 2 else []
        P3 = [self._empty(N) for _ in range(d)] if order >= 3 else []
        s = L.Stats()
        st = self.lib.dmpt_mu_newton(self.h, N, _ptr(H0), d, _ptr_array(list(H1[:d])), h2, h3,
                                     float(beta), float(Ne), int(n), int(order), mu_arr, _ptr(P0),
                                     _ptr_array(P1) if P1 else None,
                                     _ptr_array(P2) if P2 else None,
                                     _ptr_array(P3) if P3 else None, ctypes.byref(s))
        stats = s.as_dict(d, order)
        stats["status"] = st
        if raise_on_error:
            self._raise(st, stats)
        return Response(P0, P1, P2, list(mu_arr), stats, P3)

    @staticmethod
    def _opt_mats(Hs, N, name):
        """Pointer array for an optional per-direction list (None entries: zero)."""
        if Hs is None:
            return None
        for i, h in enumerate(Hs):
            if h is not None:
                _check_mat(h, N, f"{name}[{i}]")
        return _ptr_array(list(Hs))

    def congruence(self, Z, A, mode, out=None):
        """mode 0: Z^T A Z (into the orthogonalised basis); mode 1: Z A Z^T (back)."""
        N = A.shape[0]
        _check_mat(Z, N, "Z")
        _check_mat(A, N, "A")
        B = out if out is not None else self._empty(N)
        s = L.Stats()
        self._raise(self.lib.dmpt_congruence(self.h, N, _ptr(Z), _ptr(A), _ptr(B), int(mode),
                                             ctypes.byref(s)))
        return B

    def mu_newton_nonorthogonal(self, F0, Z, F1=(), F2=None, beta=1.0, Ne=1.0, n=20, order=0,
                                mu=None, F3=None):
        """Canonical response in a non-orthogonal basis (Sec. II, self-consistent response).

        The perturbed operators F^(k) are taken to the orthogonalised basis,
        F_perp = Z^T F Z (Z^T S Z = I), solved there with Tr P_perp = Ne, and the
        density matrix and its responses brought back, D^(k) = Z P^(k) Z^T.
        Returns Response(D0, [D1], [D2], mu_jet, stats) with .P3 = [D3].
        """
        to = lambda X: None if X is None else self.congruence(Z, X, 0)
        back = lambda X: self.congruence(Z, X, 1)
        r = self.mu_newton(to(F0), [to(f) for f in F1], None if F2 is None else [to(f) for f in F2],
                           beta=beta, Ne=Ne, n=n, order=order, mu=mu,
                           H3=None if F3 is None else [to(f) for f in F3])
        P0, P1, P2, m, st = r
        return Response(back(P0), [back(p) for p in P1], [back(p) for p in P2], m, st,
                        [back(p) for p in r.P3])

    def mu_newton_batched(self, H0s, H1s=None, betas=(), Nes=(), n=20, order=0, mus=None,
                          raise_on_error=True):
        """Canonical responses of many systems of uneven size in one batched solve.

        H0s: list of (N_s, N_s) tensors; H1s: list (per system) of d tensors;
        betas, Nes: per system.  Returns (P0s, P1s, P2s, mus, stats) with P1s and
        P2s lists of per-system lists and mus a list of jets (1 + 2d values).
        """
        nsys = len(H0s)
        d = len(H1s[0]) if (order >= 1 and H1s) else 0
        J = 1 + 2 * d
        Ns = (ctypes.c_int64 * nsys)(*[h.shape[0] for h in H0s])
        for s_, h in enumerate(H0s):
            _check_mat(h, h.shape[0], f"H0s[{s_}]")
        flat_h1 = []
        for s_ in range(nsys):
            for z in range(d):
                _check_mat(H1s[s_][z], H0s[s_].shape[0], f"H1s[{s_}][{z}]")
                flat_h1.append(H1s[s_][z])
        P0 = [self._empty(h.shape[0]) for h in H0s]
        P1 = [[self._empty(h.shape[0]) for _ in range(d)] for h in H0s] if order >= 1 else []
        P2 = [[self._empty(h.shape[0]) for _ in range(d)] for h in H0s] if order >= 2 else []
        m = [math.nan] * (nsys * J)
        if mus is not None:
            for s_, jet in enumerate(mus):
                for j, v in enumerate(jet[:J]):
                    m[s_ * J + j] = float(v)
        mu_arr = (ctypes.c_double * (nsys * J))(*m)
        b_arr = (ctypes.c_double * nsys)(*[float(b) for b in betas])
        ne_arr = (ctypes.c_double * nsys)(*[float(x) for x in Nes])
        st_ = L.Stats()
        flat_p1 = [p for row in P1 for p in row]
        flat_p2 = [p for row in P2 for p in row]
        st = self.lib.dmpt_mu_newton_batched(
            self.h, nsys, Ns, _ptr_array(list(H0s)), d, _ptr_array(flat_h1) if d else None, b_arr,
            ne_arr, int(n), int(order), mu_arr, _ptr_array(P0), _ptr_array(flat_p1) if d else None,
            _ptr_array(flat_p2) if flat_p2 else None, ctypes.byref(st_))
        stats = st_.as_dict()
        stats["status"] = st
        if raise_on_error:
            self._raise(st, stats)
        jets = [list(mu_arr[s_ * J:(s_ + 1) * J]) for s_ in range(nsys)]
        return P0, P1, P2, jets, stats

    def sparse_response(self, H0, H1=(), beta=1.0, Ne=1.0, n=20, order=0, tau=1e-8, count_thr=1e-5,
                        blocks_per_row=0, mu=None, outputs=True, raise_on_error=True):
        """Thresholded block-sparse canonical response (Sec. V.B; dmpt_sparse_response).

        tau: relative truncation of every intermediate; count_thr: the element magnitude counted
        into the statistics (nnz_p0, nnz_p1, nnz_p2).  With outputs=False only statistics are
        produced.  Returns (P0, [P1], [P2], mu_jet, stats) (P's None without outputs).
        """
        N = H0.shape[0]
        _check_mat(H0, N, "H0")
        d = len(H1) if order >= 1 else 0
        for i, h in enumerate(H1[:d]):
            _check_mat(h, N, f"H1[{i}]")
        nmu = 1 + order * d
        m = [math.nan] * nmu
        if mu is not None:
            for i, v in enumerate(mu[:nmu]):
                m[i] = float(v)
        mu_arr = (ctypes.c_double * nmu)(*m)
        P0 = self._empty(N) if outputs else None
        P1 = [self._empty(N) for _ in range(d)] if (outputs and order >= 1) else []
        P2 = [self._empty(N) for _ in range(d)] if (outputs and order >= 2) else []
        s = L.SparseStats()
        st = self.lib.dmpt_sparse_response(self.h, N, _ptr(H0), d, _ptr_array(list(H1[:d])) if d else None,
                                           float(beta), float(Ne), int(n), int(order), float(tau),
                                           float(count_thr), int(blocks_per_row), mu_arr, _ptr(P0),
                                           _ptr_array(P1) if P1 else None, _ptr_array(P2) if P2 else None,
                                           ctypes.byref(s))
        stats = s.as_dict(d, order)
        stats["status"] = st
        if raise_on_error:
            self._raise(st, stats)
        return P0, P1, P2, list(mu_arr), stats

    def backward(self, H0, beta, Ne, n, Abar, mu0=None):
        """Adjoint G = d Tr(Abar P0)/d H0 of the canonical map.  Returns (G, stats)."""
        N = H0.shape[0]
        _check_mat(H0, N, "H0")
        _check_mat(Abar, N, "Abar")
        G = self._empty(N)
        s = L.Stats()
        m = (ctypes.c_double * 1)(float(mu0)) if mu0 is not None else None
        st = self.lib.dmpt_backward(self.h, N, _ptr(H0), float(beta), float(Ne), int(n), m,
                                    _ptr(Abar), _ptr(G), ctypes.byref(s))
        self._raise(st, s.as_dict())
        return G, s.as_dict()
