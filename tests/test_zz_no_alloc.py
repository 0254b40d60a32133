"""muffin_grad_noalloc (the reverse sweep with its scratch in the library's
static device array) against muffin_grad with a caller workspace, through
the C ABI: two calls in a row, the second on a smaller cube, each equal bit
for bit (same kernels, same order, other scratch addresses); a sweep larger
than the static array is refused before touching the device."""
import ctypes
import sys

import numpy as np
import pytest

from synth import get_config, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(ny, nx, L, seed):
    c = get_config("grad64")
    inst = make_instance(ny, nx, L, n_points=c.n_points, n_gauss=c.n_gauss, n_ant=c.n_ant,
                         noise_sigma=c.noise_sigma, seed=seed)
    p = c.params
    return inst, dict(mu_eps=p.mu_eps, mu_s=p.mu_s, mu_nu=p.mu_nu, rho=p.rho_P)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noalloc_gradient_equals_workspace_gradient(gpu_lib, dtype):
    from paper_1504_06847_amd import Solver
    from paper_1504_06847_amd import lib as L
    lib = gpu_lib
    # (ny, nx, L, K, ckpt_every): the second call on a smaller cube
    for ny, nx, Lb, K, C in ((64, 64, 8, 10, 4), (32, 32, 4, 6, 3)):
        _say("noalloc", dtype, (Lb, ny, nx), "K", K, "C", C)
        inst, kw = _case(ny, nx, Lb, seed=11 + Lb)
        s = Solver(inst.psf, inst.dirty, dtype=dtype, **kw)
        sky = torch.as_tensor(inst.sky, dtype=dtype, device=s.device).contiguous()
        loss_ws, g_ws = s.grad(K, sky=sky, ckpt_every=C)
        x_ws = s.x.cpu()
        s.reset()
        loss = ctypes.c_double()
        g = (ctypes.c_double * 3)()
        with torch.cuda.stream(s.stream):
            rc = lib.muffin_grad_noalloc(s._ctx, K, C, ctypes.c_void_p(sky.data_ptr()), L.MUFFIN_MODE_MSE,
                                         ctypes.byref(loss), g)
        assert rc == 0, L.last_error(lib)
        g_na = np.array([g[0], g[1], g[2]])
        _say("  workspace", loss_ws, g_ws, " static", loss.value, g_na)
        assert loss.value == loss_ws and np.array_equal(g_na, g_ws)
        assert torch.equal(s.x.cpu(), x_ws)             # the state after K passes, as muffin_grad leaves it
        assert s.iterations == K
        s.close()


def test_noalloc_refuses_a_sweep_larger_than_its_scratch(gpu_lib):
    from paper_1504_06847_amd import Solver
    from paper_1504_06847_amd import lib as L
    lib = gpu_lib
    inst, kw = _case(64, 64, 8, seed=3)
    s = Solver(inst.psf, inst.dirty, **kw)
    K = 400                                     # every pass stored: 4 + 5 K + 11 cubes of 128 KiB
    assert s.grad_workspace_bytes(K, K) > (L.MUFFIN_NOALLOC_SCRATCH_MIB << 20)
    sky = torch.as_tensor(inst.sky, device=s.device).contiguous()
    loss = ctypes.c_double()
    g = (ctypes.c_double * 3)()
    rc = lib.muffin_grad_noalloc(s._ctx, K, K, ctypes.c_void_p(sky.data_ptr()), L.MUFFIN_MODE_MSE,
                                 ctypes.byref(loss), g)
    assert rc == L.MUFFIN_EWORKSPACE and "static scratch" in L.last_error(lib)
    assert s.iterations == 0
    s.close()
