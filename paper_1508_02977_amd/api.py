"""Python binding of the sfdd C ABI (``include/sfdd.h``).

Argument marshalling only: every step of the method runs in the HIP library
``libsfdd.so``.  Functions carry the C names; arrays are torch tensors on the
GPU (float64, contiguous, the layouts of ``sfdd.h``).  Negative statuses and
SF_NOT_SPD / SF_NONFINITE raise :class:`SfError`; SF_NOT_CONVERGED is returned
by :func:`sf_schwarz_solve` because the iterate is still written.

There is no fallback: if the library is missing the import of a function
raises.  Build it with ``python -m paper_1508_02977_amd.build``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfdd.so")

SF_OK = 0
SF_ERR_INVALID = -1
SF_ERR_HIP = -2
SF_ERR_OOM = -3
SF_ERR_STATE = -4
SF_ERR_DEVICE = -5
SF_NOT_SPD = 1
SF_NOT_CONVERGED = 2
SF_NONFINITE = 3
SF_FP64 = 0
SF_FP32 = 1
SF_FP32_FACTOR = 2
SF_SIGMA_MAX = 16.0
SF_NOALLOC_SCRATCH_BYTES = 1 << 20

c_int32 = ctypes.c_int32
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p


class sf_config(ctypes.Structure):
    _fields_ = [
        ("width", c_int32), ("height", c_int32), ("batch", c_int32),
        ("parts_x", c_int32), ("parts_y", c_int32), ("overlap", c_int32),
        ("lambda_", c_double), ("sigma", c_double),
        ("factor_precision", c_int32), ("band_tile", c_int32),
        ("rho", c_double), ("pivot_tol", c_double),
        ("deferred_status", c_int32),
    ]


class SfError(RuntimeError):
    def __init__(self, code: int, where: str, detail=None):
        self.code = code
        self.detail = detail
        msg = f"{where}: {status_string(code)} ({code})"
        if detail is not None:
            msg += f" detail={detail}"
        super().__init__(msg)


# name -> (restype, argtypes)
_SIGS = {
    "sf_create": (c_int32, [ctypes.POINTER(sf_config), c_void_p, ctypes.POINTER(c_void_p)]),
    "sf_destroy": (None, [c_void_p]),
    "sf_assemble": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sf_factor_subdomains": (c_int32, [c_void_p]),
    "sf_sync": (c_int32, [c_void_p]),
    "sf_set_wait_limit": (c_int32, [c_void_p, ctypes.c_int64]),
    "sf_schwarz_solve": (c_int32, [c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p]),
    "sf_schwarz_solve_graph": (c_int32, [c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p]),
    "sf_autotune": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    "sf_adjoint": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                             c_int32, c_void_p, c_void_p]),
    "sf_update_alpha": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_double, c_double, c_void_p]),
    "sf_error_detail": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sf_status_string": (ctypes.c_char_p, [c_int32]),
    "sf_rhs": (c_int32, [c_void_p, c_void_p]),
    "sf_residual": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sf_residual_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sf_indicator": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "sf_plan": (c_int32, [ctypes.POINTER(sf_config), c_void_p]),
    "sf_memory_bytes": (c_int32, [ctypes.POINTER(sf_config), ctypes.POINTER(ctypes.c_int64)]),
    "sf_num_subdomains": (c_int32, [c_void_p]),
    "sf_factor_fallbacks": (c_int32, [c_void_p]),
    "sf_subdomain_geometry": (c_int32, [c_void_p, c_int32, c_void_p]),
    "sf_subdomain_solve": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "sf_profile": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "sf_choose_split": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "sf_build_digest": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libsfdd.so`` (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (its libamdhip64 becomes the process HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1508_02977_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        from . import build
        built, now = L.sf_build_digest().decode(), build.source_digest()
        if built != now:
            raise ImportError(f"{LIB_PATH} was built from other sources than the tree holds (library {built[:12]}, "
                              f"sources {now[:12]}); rebuild with `python -m paper_1508_02977_amd.build`")
        _lib = L
        import atexit
        atexit.register(_close_all)
    return _lib


def exported_symbols() -> list[str]:
    return list(_SIGS)


def status_string(code: int) -> str:
    try:
        return lib().sf_status_string(code).decode()
    except ImportError:
        return f"status {code}"


# ---- argument helpers ----------------------------------------------------

def _dev(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return c_void_p(t.data_ptr())


def _check(code: int, where: str, ctx=None, allow=()):
    if code == SF_OK or code in allow:
        return code
    detail = None
    if ctx is not None and code in (SF_NOT_SPD, SF_ERR_DEVICE):
        detail = sf_error_detail(ctx)
    raise SfError(code, where, detail)


_LIVE = []   # weak references to open contexts, closed at interpreter exit


def _close_all():
    """Destroy every context still open, while the HIP runtime is alive."""
    for ref in list(_LIVE):
        c = ref()
        if c is not None:
            try:
                c.close()
            except Exception:
                pass
    _LIVE.clear()


@dataclasses.dataclass
class Context:
    """Owning handle of an ``sf_context``; shapes of its arrays."""

    handle: c_void_p
    cfg: sf_config
    version: int = 0          # bumped by every assemble / factor through this module

    @property
    def W(self):
        return self.cfg.width

    @property
    def H(self):
        return self.cfg.height

    @property
    def B(self):
        return self.cfg.batch

    def frame_shape(self):
        return (self.B, self.H, self.W)

    def alpha_shape(self):
        return (self.B, self.H - 1, self.W - 1, 2)

    def field_shape(self):
        return (self.B, 3, self.H, self.W)

    def close(self):
        if self.handle:
            lib().sf_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_config(width, height, batch=1, parts_x=1, parts_y=1, overlap=0, lam=1.0, sigma=0.0,
                factor_precision=SF_FP64, band_tile=0, rho=0.0, pivot_tol=0.0, deferred_status=0) -> sf_config:
    return sf_config(width, height, batch, parts_x, parts_y, overlap, lam, sigma, factor_precision, band_tile,
                     rho, pivot_tol, deferred_status)


# ---- the C entry points --------------------------------------------------

def sf_create(width, height, batch=1, parts_x=1, parts_y=1, overlap=0, lam=1.0, sigma=0.0,
              factor_precision=SF_FP64, band_tile=0, stream=None, rho=0.0, pivot_tol=0.0,
              deferred_status=0) -> Context:
    import torch
    cfg = make_config(width, height, batch, parts_x, parts_y, overlap, lam, sigma, factor_precision, band_tile,
                      rho, pivot_tol, deferred_status)
    if stream is None:
        stream = torch.cuda.current_stream()
    h = c_void_p()
    _check(lib().sf_create(ctypes.byref(cfg), c_void_p(stream.cuda_stream), ctypes.byref(h)), "sf_create")
    ctx = Context(h, cfg)
    import weakref
    _LIVE.append(weakref.ref(ctx))
    return ctx


def sf_destroy(ctx: Context) -> None:
    ctx.close()


def sf_assemble(ctx: Context, I0, I1, alpha) -> None:
    ctx.version += 1
    _check(lib().sf_assemble(ctx.handle, _dev(I0, ctx.frame_shape(), "I0"), _dev(I1, ctx.frame_shape(), "I1"),
                             _dev(alpha, ctx.alpha_shape(), "alpha")), "sf_assemble")


def sf_factor_subdomains(ctx: Context) -> None:
    ctx.version += 1
    _check(lib().sf_factor_subdomains(ctx.handle), "sf_factor_subdomains", ctx)


def sf_sync(ctx: Context) -> None:
    """Wait for the context's stream; raises the status that a deferred
    sf_assemble / sf_factor_subdomains left pending."""
    _check(lib().sf_sync(ctx.handle), "sf_sync", ctx)


def sf_set_wait_limit(ctx: Context, polls: int) -> None:
    """Bound every device-side wait of the context's later launches to
    `polls` unsuccessful polls (default 2**20); a call whose wait exceeds it
    raises SF_ERR_DEVICE."""
    _check(lib().sf_set_wait_limit(ctx.handle, int(polls)), "sf_set_wait_limit", ctx)


def sf_schwarz_solve(ctx: Context, U, rtol: float, max_sweeps: int):
    """Returns (status, sweeps[B], relres[B]); status is SF_OK or SF_NOT_CONVERGED."""
    sw = (c_int32 * ctx.B)()
    rr = (c_double * ctx.B)()
    code = lib().sf_schwarz_solve(ctx.handle, _dev(U, ctx.field_shape(), "U"), float(rtol), int(max_sweeps),
                                  ctypes.cast(sw, c_void_p), ctypes.cast(rr, c_void_p))
    _check(code, "sf_schwarz_solve", ctx, allow=(SF_NOT_CONVERGED,))
    return code, list(sw), list(rr)


def sf_schwarz_solve_graph(ctx: Context, U, rtol: float, max_sweeps: int):
    """As :func:`sf_schwarz_solve`, with every 4 iterations replayed from one
    captured HIP graph (identical results)."""
    sw = (c_int32 * ctx.B)()
    rr = (c_double * ctx.B)()
    code = lib().sf_schwarz_solve_graph(ctx.handle, _dev(U, ctx.field_shape(), "U"), float(rtol),
                                        int(max_sweeps), ctypes.cast(sw, c_void_p), ctypes.cast(rr, c_void_p))
    _check(code, "sf_schwarz_solve_graph", ctx, allow=(SF_NOT_CONVERGED,))
    return code, list(sw), list(rr)


def sf_autotune(ctx: Context, U, trials: int = 3) -> int:
    """Time the sweep's launch shapes on the current factors and keep the
    fastest; returns the chosen workgroups per chain.  ``U`` is overwritten."""
    bt = c_int32()
    _check(lib().sf_autotune(ctx.handle, _dev(U, ctx.field_shape(), "U"), int(trials), ctypes.byref(bt)),
           "sf_autotune", ctx)
    return bt.value


def sf_adjoint(ctx: Context, U, G, P, dI0=None, dI1=None, dalpha=None, rtol: float = 1e-10,
               max_sweeps: int = 1000):
    """Adjoint state P (A P = G, P is the initial iterate) and the gradients
    dI0, dI1 [B,H,W], dalpha [B,H-1,W-1,2] (each optional, written in place).
    Returns (status, sweeps[B], relres[B])."""
    sw = (c_int32 * ctx.B)()
    rr = (c_double * ctx.B)()

    def opt(t, shape, name):
        return c_void_p() if t is None else _dev(t, shape, name)

    code = lib().sf_adjoint(ctx.handle, _dev(U, ctx.field_shape(), "U"), _dev(G, ctx.field_shape(), "G"),
                            _dev(P, ctx.field_shape(), "P"), opt(dI0, ctx.frame_shape(), "dI0"),
                            opt(dI1, ctx.frame_shape(), "dI1"), opt(dalpha, ctx.alpha_shape(), "dalpha"),
                            float(rtol), int(max_sweeps), ctypes.cast(sw, c_void_p), ctypes.cast(rr, c_void_p))
    _check(code, "sf_adjoint", ctx, allow=(SF_NOT_CONVERGED,))
    return code, list(sw), list(rr)


def sf_update_alpha(ctx: Context, U, alpha, kappa=1.0, eta_thr=0.1, alpha_th=1e-3):
    """Updates ``alpha`` in place; returns ||eta||_inf per pair."""
    em = (c_double * ctx.B)()
    ctx.version += 1
    _check(lib().sf_update_alpha(ctx.handle, _dev(U, ctx.field_shape(), "U"),
                                 _dev(alpha, ctx.alpha_shape(), "alpha"), float(kappa), float(eta_thr),
                                 float(alpha_th), ctypes.cast(em, c_void_p)), "sf_update_alpha", ctx)
    return list(em)


def sf_error_detail(ctx: Context):
    p, s, r = c_int32(), c_int32(), ctypes.c_int64()
    code = lib().sf_error_detail(ctx.handle, ctypes.byref(p), ctypes.byref(s), ctypes.byref(r))
    return dict(code=code, pair=p.value, subdomain=s.value, row=r.value)


def sf_status_string(code: int) -> str:
    return status_string(code)


def sf_rhs(ctx: Context, F) -> None:
    _check(lib().sf_rhs(ctx.handle, _dev(F, ctx.field_shape(), "F")), "sf_rhs", ctx)


def sf_residual(ctx: Context, U, r):
    n2 = (c_double * ctx.B)()
    _check(lib().sf_residual(ctx.handle, _dev(U, ctx.field_shape(), "U"), _dev(r, ctx.field_shape(), "r"),
                             ctypes.cast(n2, c_void_p)), "sf_residual", ctx)
    return list(n2)


def sf_residual_noalloc(ctx: Context, U, r, norms=True):
    """As :func:`sf_residual`, with the reduction scratch in the library's
    static device array (the call allocates nothing); ``norms=False`` passes
    NULL (no synchronisation) and returns None."""
    n2 = (c_double * ctx.B)()
    _check(lib().sf_residual_noalloc(ctx.handle, _dev(U, ctx.field_shape(), "U"), _dev(r, ctx.field_shape(), "r"),
                                     ctypes.cast(n2, c_void_p) if norms else c_void_p()), "sf_residual_noalloc", ctx)
    return list(n2) if norms else None


def sf_indicator(ctx: Context, U, eta) -> None:
    _check(lib().sf_indicator(ctx.handle, _dev(U, ctx.field_shape(), "U"), _dev(eta, ctx.alpha_shape(), "eta")),
           "sf_indicator", ctx)


def sf_plan(width, height, batch=1, parts_x=1, parts_y=1, overlap=0, lam=1.0):
    """Host-only geometry: list of dicts per subdomain (no GPU needed)."""
    cfg = make_config(width, height, batch, parts_x, parts_y, overlap, lam)
    n = lib().sf_plan(ctypes.byref(cfg), None)
    _check(min(n, 0), "sf_plan")
    g = (c_int32 * (10 * n))()
    lib().sf_plan(ctypes.byref(cfg), ctypes.cast(g, c_void_p))
    return [_geom(list(g[10 * i:10 * i + 10])) for i in range(n)]


def sf_memory_bytes(width, height, batch=1, parts_x=1, parts_y=1, overlap=0, lam=1.0, sigma=0.0,
                    factor_precision=SF_FP64, rho=0.0) -> int:
    """Host-only: device bytes a context of this configuration allocates."""
    cfg = make_config(width, height, batch, parts_x, parts_y, overlap, lam, sigma, factor_precision, 0, rho)
    out = ctypes.c_int64()
    _check(lib().sf_memory_bytes(ctypes.byref(cfg), ctypes.byref(out)), "sf_memory_bytes")
    return out.value


def _geom(g):
    out = dict(pair=g[0], box=(g[1], g[2], g[3], g[4]), own=(g[5], g[6], g[7], g[8]), cols=bool(g[9]))
    if len(g) > 10:
        out.update(P=g[10], chains=g[11], kmid=g[12])
    return out


def sf_choose_split(width: int, height: int, nparts: int):
    """(parts_x, parts_y, ratio) with the largest area / perimeter of a part (host-only)."""
    px, py, r = c_int32(), c_int32(), c_double()
    _check(lib().sf_choose_split(int(width), int(height), int(nparts), ctypes.byref(px), ctypes.byref(py),
                                 ctypes.byref(r)), "sf_choose_split")
    return px.value, py.value, r.value


PROFILE_CLASSES = ("sweep", "factor", "residual", "other")


def sf_profile(ctx: Context, enable: int = -1):
    """Per-kernel-class event timings: {class: (total_ms, launches)}."""
    ms = (c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _check(lib().sf_profile(ctx.handle, int(enable), ctypes.cast(ms, c_void_p), ctypes.cast(n, c_void_p)),
           "sf_profile")
    return {k: (ms[i], n[i]) for i, k in enumerate(PROFILE_CLASSES)}


def sf_num_subdomains(ctx: Context) -> int:
    return lib().sf_num_subdomains(ctx.handle)


def sf_factor_fallbacks(ctx: Context) -> int:
    """SF_FP32_FACTOR: subdomains the last factorisation redid in FP64."""
    return lib().sf_factor_fallbacks(ctx.handle)


def sf_subdomain_geometry(ctx: Context, sub: int):
    g = (c_int32 * 13)()
    _check(lib().sf_subdomain_geometry(ctx.handle, int(sub), ctypes.cast(g, c_void_p)), "sf_subdomain_geometry")
    return _geom(list(g))


def sf_subdomain_solve(ctx: Context, sub: int, b, x) -> None:
    geo = sf_subdomain_geometry(ctx, sub)
    x0, x1, y0, y1 = geo["box"]
    n = 3 * (x1 - x0) * (y1 - y0)
    _check(lib().sf_subdomain_solve(ctx.handle, int(sub), _dev(b, (n,), "b"), _dev(x, (n,), "x")),
           "sf_subdomain_solve", ctx)


# ---- the adaptive pipeline (Section 2.3 loop on the fixed pixel mesh) ------

@dataclasses.dataclass
class PipelineResult:
    sweeps: list          # per solve: list over pairs
    relres: list
    eta_max: list         # per alpha update: list over pairs
    status: int


def run_pipeline(ctx: Context, I0, I1, alpha, U, rtol=1e-8, max_sweeps=1000, passes=0, kappa=1.0,
                 eta_thr=0.1, alpha_th=1e-3, sweeps_per_solve=None, graph=False) -> PipelineResult:
    """assemble -> factor -> solve -> (update_alpha -> factor -> solve) x passes.

    ``alpha`` is updated in place and ``U`` holds the final iterate (each solve
    warm-starts from the previous one).  ``sweeps_per_solve`` forces exact
    sweep counts (rtol 0), for comparisons at equal sweep counts.  ``graph``
    solves with :func:`sf_schwarz_solve_graph` (identical results).
    """
    solve = sf_schwarz_solve_graph if graph else sf_schwarz_solve
    sf_assemble(ctx, I0, I1, alpha)
    sweeps, rels, etas = [], [], []
    status = SF_OK
    for it in range(passes + 1):
        sf_factor_subdomains(ctx)
        if sweeps_per_solve is not None:
            code, sw, rr = solve(ctx, U, 0.0, sweeps_per_solve[it])
        else:
            code, sw, rr = solve(ctx, U, rtol, max_sweeps)
            status = max(status, code)
        sweeps.append(sw)
        rels.append(rr)
        if it < passes:
            etas.append(sf_update_alpha(ctx, U, alpha, kappa, eta_thr, alpha_th))
    return PipelineResult(sweeps, rels, etas, status)


def run_pipeline_waves(I0, I1, alpha, U, parts_x, parts_y, overlap, lam=1.0, budget_bytes=None, band_tile=0,
                       factor_precision=SF_FP64, **pipeline_kw):
    """:func:`run_pipeline` over N pairs (I0, I1 [N,H,W], alpha [N,H-1,W-1,2]
    updated in place, U [N,3,H,W] written) in waves of as many pairs as a
    context can hold within ``budget_bytes`` of device memory (default: 90%
    of the free memory).  One context serves all full waves and one more the
    last, smaller wave.  Returns (wave size, [PipelineResult per wave])."""
    import torch
    N, H, W = I0.shape
    if budget_bytes is None:
        budget_bytes = int(0.9 * torch.cuda.mem_get_info(I0.device)[0])

    def need(b):
        return sf_memory_bytes(W, H, b, parts_x, parts_y, overlap, lam, 0.0, factor_precision)

    # the largest batch that fits (need grows with the batch: bisection)
    if need(1) > budget_bytes:
        raise SfError(SF_ERR_OOM, f"run_pipeline_waves: one pair needs {need(1)} bytes, budget {budget_bytes}")
    lo, hi = 1, N
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if need(mid) <= budget_bytes:
            lo = mid
        else:
            hi = mid - 1
    wave = lo
    results, ctxs = [], {}
    try:
        for s0 in range(0, N, wave):
            s1 = min(N, s0 + wave)
            b = s1 - s0
            if b not in ctxs:
                ctxs[b] = sf_create(W, H, b, parts_x, parts_y, overlap, lam=lam, band_tile=band_tile,
                                    factor_precision=factor_precision)
            U[s0:s1].zero_()
            results.append(run_pipeline(ctxs[b], I0[s0:s1], I1[s0:s1], alpha[s0:s1], U[s0:s1], **pipeline_kw))
    finally:
        for c in ctxs.values():
            c.close()
    return wave, results


# ---- autograd ----------------------------------------------------------------

def _schwarz_solve_function():
    import torch

    class SchwarzSolve(torch.autograd.Function):
        """U = A(I0, alpha)^{-1} F(I0, I1) by the RAS solver; the backward pass
        is the adjoint solve of ``sf_adjoint`` with the same factors.  The
        context must not be re-assembled or re-factored between the two."""

        @staticmethod
        def forward(fctx, ctx, I0, I1, alpha, rtol, max_sweeps):
            I0c, I1c, alc = (t.detach().contiguous() for t in (I0, I1, alpha))
            sf_assemble(ctx, I0c, I1c, alc)
            sf_factor_subdomains(ctx)
            U = torch.zeros(ctx.field_shape(), dtype=torch.float64, device=I0.device)
            sf_schwarz_solve(ctx, U, rtol, max_sweeps)
            fctx.sf = (ctx, ctx.version, rtol, max_sweeps)
            fctx.save_for_backward(U)
            return U

        @staticmethod
        def backward(fctx, gU):
            ctx, version, rtol, max_sweeps = fctx.sf
            if ctx.version != version:
                raise RuntimeError("SchwarzSolve backward: the context was re-assembled or re-factored "
                                   "after the forward pass")
            (U,) = fctx.saved_tensors
            need = fctx.needs_input_grad
            P = torch.zeros_like(U)
            dI0 = torch.empty(ctx.frame_shape(), dtype=torch.float64, device=U.device) if need[1] else None
            dI1 = torch.empty(ctx.frame_shape(), dtype=torch.float64, device=U.device) if need[2] else None
            dal = torch.empty(ctx.alpha_shape(), dtype=torch.float64, device=U.device) if need[3] else None
            sf_adjoint(ctx, U, gU.contiguous(), P, dI0, dI1, dal, rtol, max_sweeps)
            return None, dI0, dI1, dal, None, None

    return SchwarzSolve


_SCHWARZ_SOLVE = None


def schwarz_solve(ctx: Context, I0, I1, alpha, rtol: float = 1e-10, max_sweeps: int = 1000):
    """Differentiable solve: U [B,3,H,W] from I0, I1 [B,H,W] and alpha
    [B,H-1,W-1,2] (float64 CUDA tensors); gradients by the adjoint method."""
    global _SCHWARZ_SOLVE
    if _SCHWARZ_SOLVE is None:
        _SCHWARZ_SOLVE = _schwarz_solve_function()
    return _SCHWARZ_SOLVE.apply(ctx, I0, I1, alpha, float(rtol), int(max_sweeps))
