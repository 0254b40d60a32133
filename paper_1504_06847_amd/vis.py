"""The visibility-domain model (Section 2 of the paper: the data are the
sampled visibilities; step I of Algorithm 1 by conjugate gradients) through
muffin_setup_vis.  Argument marshalling only: the setup sums, the CG and the
ADMM steps run in the library's kernels."""
from __future__ import annotations

from ctypes import POINTER, byref, c_double, c_int, c_void_p

import numpy as np
import torch

from . import lib as L
from .solver import Solver


class VisSolver(Solver):
    """One cube reconstructed from visibilities: ``uv[l]`` ([M_l][2], the
    (u, v) of band l's visibilities in cells of the nx x ny Fourier grid),
    ``vis[l]`` (M_l complex), the image ``shape`` (L, ny, nx) and ``n_cg``
    CG iterations per band and pass.  Parameters as for ``Solver`` (Dirac
    spatial basis only).  iterate, x, p, get_state / set_state, set_params,
    reset, set_graph and close work as for ``Solver``."""

    def __init__(self, uv, vis, shape, *, n_cg: int = 10, dtype=torch.float32, device="cuda", stream=None,
                 graph=False, **params):
        self._lib = L.load()
        self._ctx = c_void_p()
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        Lb, ny, nx = (int(v) for v in shape)
        if len(uv) != Lb or len(vis) != Lb:
            raise ValueError(f"expected {Lb} bands of uv and vis")
        self.shape = (Lb, ny, nx)
        self._shape = L.MuffinShape(nx, ny, Lb, L.MUFFIN_F64 if dtype == torch.float64 else L.MUFFIN_F32)
        self._params = self._make_params(params)
        counts = [int(np.asarray(v).size) for v in vis]
        for l in range(Lb):
            if np.asarray(uv[l]).shape != (counts[l], 2):
                raise ValueError(f"band {l}: uv must be [{counts[l]}][2]")
        uv_all = np.ascontiguousarray(np.concatenate([np.asarray(a, np.float64).reshape(-1, 2) for a in uv])
                                      if sum(counts) else np.zeros((0, 2)), dtype=np.float64)
        vis_all = np.concatenate([np.asarray(a, np.complex128).ravel() for a in vis]) if sum(counts) \
            else np.zeros(0, np.complex128)
        vis_ri = np.ascontiguousarray(np.stack([vis_all.real, vis_all.imag], axis=1), dtype=np.float64)
        n_vis = (c_int * Lb)(*counts)
        ws_bytes = self._lib.muffin_vis_workspace_bytes(byref(self._shape), byref(self._params))
        if ws_bytes == 0:
            raise L.MuffinError(L.MUFFIN_EINVAL, "muffin_vis_workspace_bytes", L.last_error(self._lib))
        self._ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = self._ws.data_ptr() + (-self._ws.data_ptr()) % 256
        self._ws_bytes = ws_bytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        rc = self._lib.muffin_setup_vis(byref(self._ctx), byref(self._shape), byref(self._params), n_vis,
                                        uv_all.ctypes.data_as(POINTER(c_double)),
                                        vis_ri.ctypes.data_as(POINTER(c_double)), int(n_cg),
                                        c_void_p(self._ws_ptr), ws_bytes, c_void_p(self.stream.cuda_stream))
        L.check(rc, "muffin_setup_vis", self._lib)
        self._owner = True
        if graph:
            self.set_graph(True)

    @property
    def n_cg(self) -> int:
        return int(L.check(self._lib.muffin_vis_cg_iters(self._ctx), "muffin_vis_cg_iters", self._lib))
