"""Python front end of libmuffin: a ``Solver`` per cube.

PyTorch provides the device memory (inputs, workspace, outputs) and the
stream; the reconstruction itself runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_char_p, c_double, c_void_p

import torch

from . import lib as L

PARAM_NAMES = ("mu_eps", "mu_s", "mu_nu", "rho_P", "rho_T", "rho_V", "rho_S",
               "check_every", "eps_abs", "eps_rel", "spatial", "spectral")

# Section 4's spatial dictionary: the Dirac basis and Db1..Db8
PAPER_DICTIONARY = (0, 1, 2, 3, 4, 5, 6, 7, 8)


def _load_cache(path):
    import json
    import os
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def _store_cache(path, table):
    import json
    import os
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def best_ckpt_every(K: int, budget: float, nbytes) -> int:
    """Checkpoint spacing C of a reverse sweep of K passes: among the C in
    1..K whose scratch nbytes(C) fits in ``budget``, the one that recomputes
    the fewest passes ((ceil(K / C) - 1) C: every segment but the last runs
    twice; C = K recomputes none), the smaller scratch on a tie; 1 when
    none fits."""
    K = max(1, int(K))
    best = None
    for C in range(1, K + 1):
        need = nbytes(C)
        if need > budget:
            continue
        key = ((-(-K // C)) - 1) * C, need
        if best is None or key < best[0]:
            best = (key, C)
    return 1 if best is None else best[1]


def _as_cube(a, dtype, device):
    t = a if isinstance(a, torch.Tensor) else torch.as_tensor(a)
    t = t.to(device=device, dtype=dtype).contiguous()
    if t.dim() != 3:
        raise ValueError(f"expected a [L][ny][nx] cube, got shape {tuple(t.shape)}")
    return t


class Solver:
    """ADMM reconstruction of one wide-band cube (Algorithm 1 of the paper).

    ``psf`` and ``dirty`` are [L][ny][nx] arrays (PSF peak at (ny/2, nx/2)).
    Keyword parameters: mu_eps, mu_s, mu_nu, rho_P, rho_T, rho_V, rho_S
    (defaults: the paper's Section 4 values), ``rho`` to set the four rho's
    at once, check_every, eps_abs, eps_rel, ``spatial`` (the spatial
    dictionary: 0 for the Dirac basis first, then Daubechies orders 1..8;
    ``PAPER_DICTIONARY`` is Section 4's; default the Dirac basis alone),
    ``spectral`` (the spectral bases W_nu along the bands: a code or a tuple of
    distinct codes, 0 the DCT-II, 1 the orthonormalised Chebyshev
    polynomials, 2 the identity; default the DCT alone), and ``dtype``
    (torch.float32 or torch.float64) for the iteration's precision.
    """

    def __init__(self, psf, dirty, *, dtype=torch.float32, device="cuda", stream=None, graph=False,
                 **params):
        self._lib = L.load()
        self._ctx = c_void_p()
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        psf_t = _as_cube(psf, dtype, self.device)
        dirty_t = _as_cube(dirty, dtype, self.device)
        if psf_t.shape != dirty_t.shape:
            raise ValueError("psf and dirty must have the same shape")
        Lb, ny, nx = psf_t.shape
        self.shape = (Lb, ny, nx)
        self._shape = L.MuffinShape(nx, ny, Lb, L.MUFFIN_F64 if dtype == torch.float64 else L.MUFFIN_F32)
        self._params = self._make_params(params)
        ws_bytes = self._lib.muffin_workspace_bytes(byref(self._shape), byref(self._params))
        if ws_bytes == 0:
            rc = self._lib.muffin_validate(byref(self._shape), byref(self._params))
            L.check(rc, "muffin_validate", self._lib)
        self._ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        self._ws_ptr = self._ws.data_ptr() + off
        self._ws_bytes = ws_bytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        rc = self._lib.muffin_setup(byref(self._ctx), byref(self._shape), byref(self._params),
                                    c_void_p(psf_t.data_ptr()), c_void_p(dirty_t.data_ptr()),
                                    c_void_p(self._ws_ptr), ws_bytes,
                                    c_void_p(self.stream.cuda_stream))
        L.check(rc, "muffin_setup", self._lib)
        self._owner = True
        if graph:
            self.set_graph(True)

    @classmethod
    def _view(cls, lib, ctx, shape, dtype, device, stream, params):
        """A Solver over a context owned by a Batch (closing it frees nothing)."""
        self = cls.__new__(cls)
        self._lib, self._ctx, self._owner = lib, c_void_p(ctx), False
        self.dtype, self.device, self.stream = dtype, device, stream
        self.shape = shape
        self._params = params
        return self

    def set_graph(self, enable: bool = True):
        """Replay each pass from a HIP graph (bitwise identical results)."""
        L.check(self._lib.muffin_set_graph(self._ctx, 1 if enable else 0), "muffin_set_graph", self._lib)

    # -------------------------------------------------------------- schedules
    @property
    def schedule_key(self) -> str:
        Lb, ny, nx = self.shape
        return f"{'f64' if self.dtype == torch.float64 else 'f32'}:{nx}x{ny}x{Lb}"

    @property
    def schedule(self) -> tuple:
        """(row variant, column variant, fused flag)."""
        sch = (ctypes.c_int * 3)()
        L.check(self._lib.muffin_get_schedule(self._ctx, sch), "muffin_get_schedule", self._lib)
        return (sch[0], sch[1], sch[2])

    def set_schedule(self, schedule):
        sch = (ctypes.c_int * 3)(*schedule)
        L.check(self._lib.muffin_set_schedule(self._ctx, sch), "muffin_set_schedule", self._lib)

    @property
    def fused_available(self) -> bool:
        return bool(self._lib.muffin_fused_available(self._ctx))

    def autotune(self, reps: int = 10, cache: str | None = None) -> tuple:
        """Pick the fastest FFT tile schedule for this shape.  With ``cache`` (a
        JSON file), a schedule stored there for the same shape and dtype is
        reused, and a newly timed one is added."""
        key = self.schedule_key
        table = _load_cache(cache)
        if key in table:
            self.set_schedule(table[key])
            return tuple(table[key])
        sch = (ctypes.c_int * 3)()
        L.check(self._lib.muffin_autotune(self._ctx, int(reps), sch), "muffin_autotune", self._lib)
        if cache:
            table[key] = [sch[0], sch[1], sch[2]]
            _store_cache(cache, table)
        return (sch[0], sch[1], sch[2])

    # -------------------------------------------------------------- params
    def _make_params(self, params):
        kw = dict(params)
        if "rho" in kw:
            r = kw.pop("rho")
            for k in ("rho_P", "rho_T", "rho_V", "rho_S"):
                kw.setdefault(k, r)
        unknown = set(kw) - set(PARAM_NAMES)
        if unknown:
            raise TypeError(f"unknown parameters {sorted(unknown)}")
        if "spatial" in kw:
            kw["spatial"] = tuple(int(b) for b in kw["spatial"])
            kw["n_s"] = len(kw["spatial"])
        if "spectral" in kw:
            sp = kw["spectral"]
            kw["spectral"] = tuple(int(b) for b in sp) if isinstance(sp, (tuple, list)) else (int(sp),)
        return L.make_params(self._lib, **kw)

    @property
    def params(self):
        d = {k: getattr(self._params, k) for k in PARAM_NAMES if k not in ("spatial", "spectral")}
        d["spatial"] = tuple(self._params.spatial[i] for i in range(self._params.n_s))
        d["spectral"] = tuple(self._params.spectral[i] for i in range(self._params.n_nu))
        return d

    def set_params(self, **params):
        cur = self.params
        cur.update(params)
        if "rho" in params:
            r = cur.pop("rho")
            for k in ("rho_P", "rho_T", "rho_V", "rho_S"):
                cur[k] = r
        p = self._make_params(cur)
        L.check(self._lib.muffin_set_params(self._ctx, byref(p)), "muffin_set_params", self._lib)
        self._params = p

    # -------------------------------------------------------------- iteration
    def iterate(self, n: int = 1):
        L.check(self._lib.muffin_iterate(self._ctx, int(n)), "muffin_iterate", self._lib)
        return self

    def step_report(self) -> dict:
        rep = L.MuffinReport()
        L.check(self._lib.muffin_step_report(self._ctx, byref(rep)), "muffin_step_report", self._lib)
        return rep.asdict()

    def solve(self, max_iter: int = 350, adaptive=None) -> dict:
        """Iterate until the Boyd stopping rule holds or max_iter passes.
        ``adaptive=(mu, tau)`` balances the residuals by scaling the four
        rho's (muffin_solve_adaptive); ``params`` then shows the final rho's."""
        rep = L.MuffinReport()
        if adaptive is None:
            rc = L.check(self._lib.muffin_solve(self._ctx, int(max_iter), byref(rep)), "muffin_solve", self._lib)
        else:
            mu, tau = adaptive
            rc = L.check(self._lib.muffin_solve_adaptive(self._ctx, int(max_iter), float(mu), float(tau),
                                                         byref(rep)), "muffin_solve_adaptive", self._lib)
            p = L.MuffinParams()
            L.check(self._lib.muffin_get_params(self._ctx, byref(p)), "muffin_get_params", self._lib)
            self._params = p
        d = rep.asdict()
        d["status"] = rc
        return d

    @property
    def iterations(self) -> int:
        return self._lib.muffin_iterations(self._ctx)

    def _empty_cube(self):
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    @property
    def x(self) -> torch.Tensor:
        """Current X iterate (step I output)."""
        out = self._empty_cube()
        L.check(self._lib.muffin_get_x(self._ctx, c_void_p(out.data_ptr())), "muffin_get_x", self._lib)
        return out

    @property
    def p(self) -> torch.Tensor:
        """Current P = max(0, X - Gamma_P / rho_P)."""
        out = self._empty_cube()
        L.check(self._lib.muffin_get_p(self._ctx, c_void_p(out.data_ptr())), "muffin_get_p", self._lib)
        return out

    # -------------------------------------------------------------- state
    def state_bytes(self) -> int:
        return self._lib.muffin_state_bytes(self._ctx)

    def get_state(self) -> torch.Tensor:
        n = self.state_bytes()
        buf = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + n]
        L.check(self._lib.muffin_get_state(self._ctx, c_void_p(view.data_ptr())), "muffin_get_state", self._lib)
        return view

    def set_state(self, state: torch.Tensor):
        if state.data_ptr() % 256:
            aligned = torch.empty(state.numel() + 256, dtype=torch.uint8, device=self.device)
            off = (-aligned.data_ptr()) % 256
            aligned[off:off + state.numel()].copy_(state)
            state = aligned[off:off + state.numel()]
        L.check(self._lib.muffin_set_state(self._ctx, c_void_p(state.data_ptr())), "muffin_set_state", self._lib)

    def reset(self):
        L.check(self._lib.muffin_reset(self._ctx), "muffin_reset", self._lib)

    # -------------------------------------------------------------- gradients
    def grad_workspace_bytes(self, K: int, ckpt_every: int, dirty: bool = False) -> int:
        """Device bytes of the reverse sweep's scratch (muffin_grad_workspace_bytes)."""
        return int(self._lib.muffin_grad_workspace_bytes(self._ctx, int(K), int(ckpt_every), 1 if dirty else 0))

    def sweep_ckpt_every(self, K: int, dirty: bool = False, fraction: float = 0.5,
                         budget: int | None = None) -> int:
        """Checkpoint spacing for a reverse sweep of K passes
        (``best_ckpt_every``) within ``budget`` bytes, by default ``fraction``
        of the device memory available: free, plus what torch's allocator
        holds unused (the sweep's workspace comes from it)."""
        if budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
            budget = fraction * (free + max(0, cached))
        return best_ckpt_every(K, budget, lambda C: self.grad_workspace_bytes(K, C, dirty))

    def _sweep(self, name, K, ckpt_every, dirty, call):
        """Run one reverse sweep in a workspace allocated for it (released
        to torch's allocator afterwards)."""
        nbytes = self.grad_workspace_bytes(K, ckpt_every, dirty)
        if nbytes == 0:
            raise L.MuffinError(L.MUFFIN_EINVAL, "muffin_grad_workspace_bytes", L.last_error(self._lib))
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
        L.check(self._lib.muffin_set_grad_workspace(self._ctx, c_void_p(ptr), nbytes),
                "muffin_set_grad_workspace", self._lib)
        try:
            with torch.cuda.stream(self.stream):
                rc = call()
            L.check(rc, name, self._lib)
        finally:
            self._lib.muffin_set_grad_workspace(self._ctx, None, 0)
            del ws

    def grad(self, K: int, *, sky=None, gx=None, ckpt_every: int | None = None):
        """Gradient with respect to (mu_s, mu_nu, rho) of a loss of X^K, the X
        iterate after K passes from the zero state (rho: the common value of
        the four rho's, derivative along (1, 1, 1, 1)).  Give ``sky`` for
        loss = ||X^K - sky||^2, or ``gx`` = dloss/dX^K.  Returns (loss, grad)
        with grad a length-3 numpy array (loss is 0.0 with gx).  Afterwards
        the solver holds the state after K passes.  ckpt_every: the
        checkpoint spacing, by default ``sweep_ckpt_every(K)``."""
        import numpy as np
        if ckpt_every is None:
            ckpt_every = self.sweep_ckpt_every(K)
        if (sky is None) == (gx is None):
            raise ValueError("give exactly one of sky and gx")
        ref = _as_cube(sky if sky is not None else gx, self.dtype, self.device)
        if tuple(ref.shape) != tuple(self.shape):
            raise ValueError(f"expected a cube of shape {self.shape}, got {tuple(ref.shape)}")
        mode = L.MUFFIN_MODE_MSE if sky is not None else L.MUFFIN_MODE_VJP
        loss = c_double()
        g = (c_double * 3)()
        self._sweep("muffin_grad", K, ckpt_every, False,
                    lambda: self._lib.muffin_grad(self._ctx, int(K), int(ckpt_every), c_void_p(ref.data_ptr()),
                                                  mode, byref(loss), g))
        return loss.value, np.array([g[0], g[1], g[2]])

    GRAD_PARAMS = ("mu_eps", "mu_s", "mu_nu", "rho_P", "rho_T", "rho_V", "rho_S")

    def grad_params(self, K: int, *, sky=None, gx=None, ckpt_every: int | None = None):
        """As ``grad``, with the derivative along each parameter on its own:
        returns (loss, {name: d loss / d name}) for GRAD_PARAMS."""
        if ckpt_every is None:
            ckpt_every = self.sweep_ckpt_every(K)
        if (sky is None) == (gx is None):
            raise ValueError("give exactly one of sky and gx")
        ref = _as_cube(sky if sky is not None else gx, self.dtype, self.device)
        if tuple(ref.shape) != tuple(self.shape):
            raise ValueError(f"expected a cube of shape {self.shape}, got {tuple(ref.shape)}")
        mode = L.MUFFIN_MODE_MSE if sky is not None else L.MUFFIN_MODE_VJP
        loss = c_double()
        g = (c_double * 7)()
        self._sweep("muffin_grad_params", K, ckpt_every, False,
                    lambda: self._lib.muffin_grad_params(self._ctx, int(K), int(ckpt_every),
                                                         c_void_p(ref.data_ptr()), mode, byref(loss), g))
        return loss.value, {n: g[i] for i, n in enumerate(self.GRAD_PARAMS)}

    def grad_dirty(self, K: int, *, sky=None, gx=None, ckpt_every: int | None = None):
        """Cotangent of the dirty images: returns (loss, dL/dY) with dL/dY a
        cube on the device (muffin_grad_dirty)."""
        if ckpt_every is None:
            ckpt_every = self.sweep_ckpt_every(K, dirty=True)
        if (sky is None) == (gx is None):
            raise ValueError("give exactly one of sky and gx")
        ref = _as_cube(sky if sky is not None else gx, self.dtype, self.device)
        if tuple(ref.shape) != tuple(self.shape):
            raise ValueError(f"expected a cube of shape {self.shape}, got {tuple(ref.shape)}")
        mode = L.MUFFIN_MODE_MSE if sky is not None else L.MUFFIN_MODE_VJP
        loss = c_double()
        gy = self._empty_cube()
        self._sweep("muffin_grad_dirty", K, ckpt_every, True,
                    lambda: self._lib.muffin_grad_dirty(self._ctx, int(K), int(ckpt_every),
                                                        c_void_p(ref.data_ptr()), mode, byref(loss),
                                                        c_void_p(gy.data_ptr())))
        return loss.value, gy

    def grad_record(self, K: int, *, ckpt_every: int | None = None, dirty: bool = False):
        """The forward half of a reverse sweep (muffin_grad_record): K passes
        from the zero state, checkpointed into a workspace held until
        ``grad_replay``; afterwards ``x`` is X^K.  ``dirty``: the replay
        will also return the cotangent of the dirty images."""
        if ckpt_every is None:
            ckpt_every = self.sweep_ckpt_every(K, dirty=dirty)
        self._drop_record()
        nbytes = self.grad_workspace_bytes(K, ckpt_every, dirty)
        if nbytes == 0:
            raise L.MuffinError(L.MUFFIN_EINVAL, "muffin_grad_workspace_bytes", L.last_error(self._lib))
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
        L.check(self._lib.muffin_set_grad_workspace(self._ctx, c_void_p(ptr), nbytes),
                "muffin_set_grad_workspace", self._lib)
        self._rec = (ws, bool(dirty))
        try:
            with torch.cuda.stream(self.stream):
                rc = self._lib.muffin_grad_record(self._ctx, int(K), int(ckpt_every), 1 if dirty else 0)
            L.check(rc, "muffin_grad_record", self._lib)
        except Exception:
            self._drop_record()
            raise

    def grad_replay(self, *, sky=None, gx=None):
        """The reverse half of the sweep ``grad_record`` ran: returns (loss,
        {name: d loss / d name} for GRAD_PARAMS, dL/dY or None)."""
        rec = getattr(self, "_rec", None)
        if rec is None:
            raise L.MuffinError(L.MUFFIN_EINVAL, "muffin_grad_replay", "no recorded forward sweep")
        if (sky is None) == (gx is None):
            raise ValueError("give exactly one of sky and gx")
        ref = _as_cube(sky if sky is not None else gx, self.dtype, self.device)
        if tuple(ref.shape) != tuple(self.shape):
            raise ValueError(f"expected a cube of shape {self.shape}, got {tuple(ref.shape)}")
        mode = L.MUFFIN_MODE_MSE if sky is not None else L.MUFFIN_MODE_VJP
        loss = c_double()
        g = (c_double * 7)()
        gy = self._empty_cube() if rec[1] else None
        try:
            with torch.cuda.stream(self.stream):
                rc = self._lib.muffin_grad_replay(self._ctx, c_void_p(ref.data_ptr()), mode, byref(loss), g,
                                                  c_void_p(gy.data_ptr()) if gy is not None else None)
            L.check(rc, "muffin_grad_replay", self._lib)
        finally:
            self._drop_record()
        return loss.value, {n: g[i] for i, n in enumerate(self.GRAD_PARAMS)}, gy

    def _drop_record(self):
        if getattr(self, "_rec", None) is not None:
            self._lib.muffin_set_grad_workspace(self._ctx, None, 0)
            self._rec = None

    # -------------------------------------------------------------- timing
    def profile(self, n_iter: int = 10) -> dict:
        cap = 16
        ms = (c_double * cap)()
        names = (c_char_p * cap)()
        k = L.check(self._lib.muffin_profile(self._ctx, int(n_iter), ms, names, cap), "muffin_profile", self._lib)
        return {names[i].decode(): ms[i] for i in range(k)}

    # -------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            if getattr(self, "_owner", False):
                self._lib.muffin_destroy(self._ctx)
            self._ctx = c_void_p()
        self._rec = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
