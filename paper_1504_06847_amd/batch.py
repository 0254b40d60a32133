"""Python front end of the batched form: many independent cubes of uneven
size and band count iterating together through grouped launches (a batch
context of the C ABI, muffin_setup_batch).  Each cube is also reachable as a
``Solver`` view."""
from __future__ import annotations

import ctypes
from ctypes import byref, c_void_p

import torch

from . import lib as L
from .solver import Solver, _as_cube, _load_cache, _store_cache


class Batch:
    """``cubes``: a list of (psf, dirty) pairs of [L][ny][nx] arrays (shapes may
    differ).  ``params``: one dict of solver parameters for every cube, or a
    list with one dict per cube."""

    def __init__(self, cubes, *, dtype=torch.float32, device="cuda", stream=None, graph=False,
                 params=None):
        self._lib = L.load()
        self._b = c_void_p()
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        n = len(cubes)
        if n < 1:
            raise ValueError("a batch needs at least one cube")
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        plist = params if isinstance(params, (list, tuple)) else [params or {}] * n
        if len(plist) != n:
            raise ValueError("params: one dict per cube")
        dt = L.MUFFIN_F64 if dtype == torch.float64 else L.MUFFIN_F32
        shapes = (L.MuffinShape * n)()
        prm = (L.MuffinParams * n)()
        self._inputs = []
        self.shapes = []
        for i, ((psf, dirty), p) in enumerate(zip(cubes, plist)):
            a, b = _as_cube(psf, dtype, self.device), _as_cube(dirty, dtype, self.device)
            if a.shape != b.shape:
                raise ValueError(f"cube {i}: psf and dirty differ in shape")
            Lb, ny, nx = a.shape
            shapes[i] = L.MuffinShape(nx, ny, Lb, dt)
            prm[i] = Solver._make_params(self, dict(p))
            self._inputs += [a, b]
            self.shapes.append((Lb, ny, nx))
        self._prm = prm
        ws = self._lib.muffin_batch_workspace_bytes(n, shapes, prm)
        if ws == 0:
            for i in range(n):
                L.check(self._lib.muffin_validate(byref(shapes[i]), byref(prm[i])), "muffin_validate", self._lib)
            raise L.MuffinError(L.MUFFIN_EINVAL, "muffin_batch_workspace_bytes", L.last_error(self._lib))
        self._ws = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        psfs = (c_void_p * n)(*[self._inputs[2 * i].data_ptr() for i in range(n)])
        dirts = (c_void_p * n)(*[self._inputs[2 * i + 1].data_ptr() for i in range(n)])
        rc = self._lib.muffin_setup_batch(byref(self._b), n, shapes, prm, psfs, dirts,
                                          c_void_p(self._ws.data_ptr() + off), ws,
                                          c_void_p(self.stream.cuda_stream))
        L.check(rc, "muffin_setup_batch", self._lib)
        self._inputs = None          # setup keeps no pointer to them
        self.n = n
        if graph:
            self.set_graph(True)

    def __len__(self):
        return self.n

    def cube(self, i: int) -> Solver:
        """Solver view of cube i (x, step_report, solve, set_params, state ...)."""
        if not 0 <= i < self.n:
            raise IndexError(i)
        ctx = self._lib.muffin_batch_cube(self._b, int(i))
        if not ctx:
            raise L.MuffinError(L.MUFFIN_EINVAL, "muffin_batch_cube", L.last_error(self._lib))
        return Solver._view(self._lib, ctx, self.shapes[i], self.dtype, self.device, self.stream,
                            self._prm[i])

    def iterate(self, n: int = 1):
        L.check(self._lib.muffin_iterate(self._b, int(n)), "muffin_iterate", self._lib)
        return self

    def set_graph(self, enable: bool = True):
        L.check(self._lib.muffin_set_graph(self._b, 1 if enable else 0), "muffin_set_graph", self._lib)

    @property
    def launches(self) -> int:
        """Grouped launches per pass."""
        return self._lib.muffin_batch_launches(self._b)

    @property
    def iterations(self) -> int:
        """Batch passes run since setup."""
        return self._lib.muffin_iterations(self._b)

    def autotune(self, reps: int = 10):
        L.check(self._lib.muffin_batch_autotune(self._b, int(reps)), "muffin_batch_autotune", self._lib)

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._lib.muffin_destroy(self._b)
            self._b = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
