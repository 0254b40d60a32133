"""The C ABI without a GPU: the library loads, exports every entry point that
include/muffin.h declares, and its host-only validation returns the documented
codes.  No call here reaches the device."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "muffin.h")

pytestmark = pytest.mark.cpu


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(muffin_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1504_06847_amd import lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libmuffin.so is not built: run python -m paper_1504_06847_amd.build")
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1504_06847_amd import lib as L
    bound = {n for n, _, _ in L.SIGNATURES}
    assert set(_declared_functions()) == bound


def test_struct_layouts_match_header():
    from paper_1504_06847_amd import lib as L
    # muffin_params: 7 doubles, n_s, spatial[9], n_nu, spectral[4], check_every, 2 doubles
    assert ctypes.sizeof(L.MuffinParams) == 7 * 8 + 4 + 36 + 4 + 16 + 4 + 2 * 8
    assert ctypes.sizeof(L.MuffinShape) == 16
    assert ctypes.sizeof(L.MuffinReport) == 8 + 6 * 8


def _shape(L, nx=64, ny=64, Lb=8, dtype=0):
    return L.MuffinShape(nx, ny, Lb, dtype)


def test_default_params_are_the_papers(lib):
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib)
    assert (p.mu_eps, p.mu_s, p.mu_nu) == (1e-3, 0.5, 1.0)
    assert (p.rho_P, p.rho_T, p.rho_V, p.rho_S) == (1.0, 5.0, 2.0, 1.0)
    assert p.n_s == 1 and p.spatial[0] == L.MUFFIN_DIRAC and p.check_every == 10


@pytest.mark.parametrize("field,value,code", [
    ("mu_s", -1.0, -1), ("mu_nu", float("nan"), -1), ("mu_eps", float("inf"), -1),
    ("rho_P", 0.0, -1), ("rho_T", -2.0, -1), ("rho_V", float("nan"), -1),
    ("check_every", 0, -1), ("eps_abs", -1e-3, -1), ("n_s", 10, -2), ("n_s", 0, -2), ("n_nu", 0, -2), ("n_nu", 5, -2),
])
def test_parameter_validation(lib, field, value, code):
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib, **{field: value})
    s = _shape(L)
    assert lib.muffin_validate(ctypes.byref(s), ctypes.byref(p)) == code
    assert lib.muffin_workspace_bytes(ctypes.byref(s), ctypes.byref(p)) == 0
    assert field.split("_")[0] in L.last_error(lib) or field in L.last_error(lib)


@pytest.mark.parametrize("nx,ny,Lb,dtype,code", [
    (64, 64, 8, 0, 0), (8, 8, 1, 1, 0), (4096, 8, 64, 0, 0), (64, 64, 15, 0, 0),
    (64, 64, 0, 0, -1), (0, 64, 8, 0, -1), (60, 64, 8, 0, -2), (64, 8192, 8, 0, -2),
    (4, 64, 8, 0, -2), (64, 64, 129, 0, -2), (64, 64, 48, 0, -2), (64, 64, 96, 0, -2),
    (64, 64, 128, 0, 0), (64, 64, 256, 0, 0), (64, 64, 257, 0, -2), (64, 64, 512, 0, -2), (64, 64, 8, 7, -2),
])
def test_shape_validation(lib, nx, ny, Lb, dtype, code):
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib)
    s = L.MuffinShape(nx, ny, Lb, dtype)
    assert lib.muffin_validate(ctypes.byref(s), ctypes.byref(p)) == code
    ws = lib.muffin_workspace_bytes(ctypes.byref(s), ctypes.byref(p))
    assert (ws > 0) == (code == 0)


def test_workspace_grows_with_the_cube(lib):
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib)
    a = lib.muffin_workspace_bytes(ctypes.byref(L.MuffinShape(64, 64, 8, 0)), ctypes.byref(p))
    b = lib.muffin_workspace_bytes(ctypes.byref(L.MuffinShape(64, 64, 16, 0)), ctypes.byref(p))
    c = lib.muffin_workspace_bytes(ctypes.byref(L.MuffinShape(64, 64, 8, 1)), ctypes.byref(p))
    V = 64 * 64 * 8
    # 7 cubes + 3 half-spectrum cube equivalents (packed Z, Yf) + |h|^2 at least
    assert a >= 9 * 4 * V and b > a and c > a


def test_setup_rejects_bad_arguments_before_touching_the_device(lib):
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib)
    s = L.MuffinShape(64, 64, 8, 0)
    ctx = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)
    assert lib.muffin_setup(None, ctypes.byref(s), ctypes.byref(p), dummy, dummy, dummy, 1 << 30, None) == -1
    assert lib.muffin_setup(ctypes.byref(ctx), ctypes.byref(s), ctypes.byref(p), None, dummy, dummy, 1 << 30, None) == -1
    assert lib.muffin_setup(ctypes.byref(ctx), ctypes.byref(s), ctypes.byref(p), dummy, dummy, dummy, 16, None) == -3
    bad = ctypes.c_void_p(0x1001)
    assert lib.muffin_setup(ctypes.byref(ctx), ctypes.byref(s), ctypes.byref(p), dummy, dummy, bad, 1 << 40, None) == -3
    p2 = L.make_params(lib, rho_S=0.0)
    assert lib.muffin_setup(ctypes.byref(ctx), ctypes.byref(s), ctypes.byref(p2), dummy, dummy, dummy, 1 << 40, None) == -1
    assert ctx.value is None


def test_null_context_calls_fail_cleanly(lib):
    from paper_1504_06847_amd import lib as L
    assert lib.muffin_iterate(None, 1) == -1
    assert lib.muffin_get_x(None, None) == -1
    assert lib.muffin_reset(None) == -1
    assert lib.muffin_destroy(None) == 0
    assert lib.muffin_state_bytes(None) == 0
    rep = L.MuffinReport()
    assert lib.muffin_solve(None, 10, ctypes.byref(rep)) == -1


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_validation_unit_under_host_sanitizers(tmp_path):
    """Build the host-only validation unit with ASan + UBSan and drive it."""
    csrc = os.path.join(ROOT, "paper_1504_06847_amd", "csrc")
    exe = tmp_path / "validate_san"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{ROOT}/include", f"-I{csrc}",
           os.path.join(csrc, "muffin_validate.cpp"),
           os.path.join(ROOT, "tests", "host", "validate_driver.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout


def test_batch_validation_without_device(lib):
    from paper_1504_06847_amd import lib as L
    n = 3
    shapes = (L.MuffinShape * n)(L.MuffinShape(64, 64, 8, 0), L.MuffinShape(32, 128, 16, 0),
                                 L.MuffinShape(16, 16, 15, 0))
    prm = (L.MuffinParams * n)(*[L.make_params(lib) for _ in range(n)])
    total = lib.muffin_batch_workspace_bytes(n, shapes, prm)
    per = sum(-(-lib.muffin_workspace_bytes(ctypes.byref(shapes[i]), ctypes.byref(prm[i])) // 256) * 256
              for i in range(n))
    assert total > per                       # plus the launch descriptors
    assert lib.muffin_batch_workspace_bytes(0, shapes, prm) == 0
    assert lib.muffin_batch_workspace_bytes(L.MUFFIN_MAX_BATCH + 1, shapes, prm) == 0
    mixed = (L.MuffinShape * 2)(L.MuffinShape(64, 64, 8, 0), L.MuffinShape(64, 64, 8, 1))
    assert lib.muffin_batch_workspace_bytes(2, mixed, prm) == 0
    assert "dtype" in L.last_error(lib)
    bad = (L.MuffinShape * 2)(L.MuffinShape(64, 64, 8, 0), L.MuffinShape(60, 64, 8, 0))
    assert lib.muffin_batch_workspace_bytes(2, bad, prm) == 0
    wide = (L.MuffinShape * 2)(L.MuffinShape(64, 64, 8, 0), L.MuffinShape(64, 64, 256, 0))
    assert lib.muffin_batch_workspace_bytes(2, wide, prm) == 0      # batches take L <= 128
    assert "128" in L.last_error(lib)
    b = ctypes.c_void_p()
    dummy = (ctypes.c_void_p * n)(0x1000, 0x1000, 0x1000)
    assert lib.muffin_setup_batch(ctypes.byref(b), 0, shapes, prm, dummy, dummy,
                                  ctypes.c_void_p(0x1000), 1 << 40, None) == -1
    assert lib.muffin_setup_batch(ctypes.byref(b), n, shapes, prm, dummy, dummy,
                                  ctypes.c_void_p(0x1000), 16, None) == -3
    assert lib.muffin_setup_batch(ctypes.byref(b), n, shapes, prm, None, dummy,
                                  ctypes.c_void_p(0x1000), 1 << 40, None) == -1
    assert lib.muffin_setup_batch(None, n, shapes, prm, dummy, dummy,
                                  ctypes.c_void_p(0x1000), 1 << 40, None) == -1
    assert b.value is None
    assert lib.muffin_iterate(None, 1) == -1
    assert lib.muffin_batch_cube(None, 0) is None
    assert "batch context" in L.last_error(lib)
    assert lib.muffin_batch_autotune(None, 1) == -1
    assert lib.muffin_batch_launches(None) == -1
    assert lib.muffin_destroy(None) == 0


def test_gradient_workspace_calls_without_device(lib):
    """The reverse sweep's scratch size and the workspace calls on a NULL
    context (no device needed)."""
    assert lib.muffin_grad_workspace_bytes(None, 20, 5, 0) == 0
    assert lib.muffin_set_grad_workspace(None, None, 0) == -1
    g = (ctypes.c_double * 3)()
    loss = ctypes.c_double()
    assert lib.muffin_grad(None, 20, 5, ctypes.c_void_p(0x1000), 0, ctypes.byref(loss), g) == -1


def test_schedule_calls_reject_bad_arguments(lib):
    sch = (ctypes.c_int * 2)(0, 0)
    assert lib.muffin_autotune(None, 3, sch) == -1
    assert lib.muffin_set_schedule(None, sch) == -1
    assert lib.muffin_get_schedule(None, sch) == -1


def test_wavelet_filter_matches_the_oracle(lib):
    """The library's Daubechies filters (host FP64, its own root finder)
    against the oracle's spectral factorisation."""
    import oracle as O
    for p in range(1, 9):
        h = (ctypes.c_double * 16)()
        assert lib.muffin_wavelet_filter(p, h) == 0
        np.testing.assert_allclose(np.array(h[:2 * p]), O.daubechies_filter(p), atol=2e-14, rtol=0)
    h = (ctypes.c_double * 16)()
    assert lib.muffin_wavelet_filter(0, h) == -1 and lib.muffin_wavelet_filter(9, h) == -1
    assert lib.muffin_wavelet_filter(2, None) == -1


@pytest.mark.parametrize("spatial,code", [
    ((0,), 0), ((0, 1, 2, 3, 4, 5, 6, 7, 8), 0), ((0, 8, 8), 0), ((1, 2), -2), ((0, 9), -2), ((0, 0), -2),
])
def test_spatial_dictionary_validation(lib, spatial, code):
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib, n_s=len(spatial), spatial=spatial)
    s = _shape(L)
    assert lib.muffin_validate(ctypes.byref(s), ctypes.byref(p)) == code
    if code:
        assert "spatial" in L.last_error(lib)


def test_workspace_grows_by_one_cube_per_wavelet_basis(lib):
    from paper_1504_06847_amd import lib as L
    s = L.MuffinShape(64, 32, 4, 0)
    one = lib.muffin_workspace_bytes(ctypes.byref(s), ctypes.byref(L.make_params(lib)))
    nine = lib.muffin_workspace_bytes(ctypes.byref(s), ctypes.byref(
        L.make_params(lib, n_s=9, spatial=(0, 1, 2, 3, 4, 5, 6, 7, 8))))
    V = 64 * 32 * 4 * 4
    # 8 coefficient cubes plus each basis's DWT scratch of levels 1..3
    # (V/4 + V/16 + V/64), the filter table, the reporting pass's three
    # cubes and up to eight FP64 sums per analysis work-group: at 32 x 64
    # each of the 4 levels is one 16 x 32 tile per band and basis
    extra = 8 * (V + V // 4 + V // 16 + V // 64) + 3 * V + 4 * 4 * 8 * 8 * 8
    assert extra <= nine - one <= extra + 40 * 256



def test_checkpoint_spacing_minimises_recomputed_passes():
    """Solver's spacing rule on the scratch sizes the header documents for
    the Dirac basis (4 ceil(K/C) + 10 C + 6 cubes, 4 + 5 K + 6 at C = K): the
    spacing with the fewest recomputed passes among those that fit, not the
    largest."""
    from paper_1504_06847_amd.solver import best_ckpt_every

    def cubes(K, C):
        n = -(-K // C)
        return 4 + 5 * K + 6 if n == 1 else 4 * n + 10 * C + 6

    # K = 20, room for 105 cubes: C = 8 (98 cubes) recomputes 16 passes,
    # C = 7 (88 cubes) 14
    assert best_ckpt_every(20, 105, lambda C: cubes(20, C)) == 7
    # K = 120, room for 600 cubes: C = 54 would recompute 108, C = 40 only 80
    assert best_ckpt_every(120, 600, lambda C: cubes(120, C)) == 40
    # everything fits: no recompute
    assert best_ckpt_every(20, 1e9, lambda C: cubes(20, C)) == 20
    assert best_ckpt_every(20, 10, lambda C: cubes(20, C)) == 1


@pytest.mark.parametrize("spectral,code", [((0,), 0), ((1,), 0), ((2,), 0), ((0, 1), 0), ((0, 1, 2), 0),
                                           ((3,), -2), ((0, 0), -1), ((1, 2, 1), -1)])
def test_spectral_dictionary_validation(lib, spectral, code):
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib, spectral=spectral)
    assert p.n_nu == len(spectral)
    s = L.MuffinShape(32, 32, 16, 0)
    assert lib.muffin_validate(ctypes.byref(s), ctypes.byref(p)) == code


@pytest.mark.parametrize("Lb,spectral,code", [(64, (1,), 0), (128, (1,), -2), (48, (0,), -2), (24, (0, 2), 0),
                                              (256, (0,), 0), (256, (0, 1), -2), (128, (0,), 0)])
def test_spectral_dictionary_band_limits(lib, Lb, spectral, code):
    """Bases other than the DCT alone take a dense transform: L <= 32 or 64."""
    from paper_1504_06847_amd import lib as L
    p = L.make_params(lib, spectral=spectral)
    s = L.MuffinShape(32, 32, Lb, 0)
    assert lib.muffin_validate(ctypes.byref(s), ctypes.byref(p)) == code


def test_union_workspace_adds_two_cubes_per_basis(lib):
    """A union of m bases carries one coefficient cube per basis in each of
    the two state sets."""
    from paper_1504_06847_amd import lib as L
    s = L.MuffinShape(32, 32, 16, 0)
    one = lib.muffin_workspace_bytes(ctypes.byref(s), ctypes.byref(L.make_params(lib, spectral=(1,))))
    two = lib.muffin_workspace_bytes(ctypes.byref(s), ctypes.byref(L.make_params(lib, spectral=(0, 1))))
    cube = 32 * 32 * 16 * 4
    assert two - one >= 4 * cube and two - one < 4 * cube + 16 * 16 * 4 + 16 * 256


@pytest.mark.parametrize("L_", [1, 2, 3, 8, 15, 32, 64])
def test_spectral_bases_match_the_oracle(lib, L_):
    """The library's bases (the Chebyshev one by a long-double Lanczos
    recurrence) against the oracle's (exact rational Gram-Schmidt, the DCT by
    scipy, the identity)."""
    import oracle as O
    for code in (0, 1, 2):
        W = (ctypes.c_double * (L_ * L_))()
        assert lib.muffin_spectral_basis(code, L_, W) == 0
        Wl = np.array(W[:]).reshape(L_, L_)
        np.testing.assert_allclose(Wl, O.basis_matrix(code, L_), atol=2e-15, rtol=0)
    W = (ctypes.c_double * 4)()
    assert lib.muffin_spectral_basis(5, 2, W) == -1
    assert lib.muffin_spectral_basis(1, 0, W) == -1


def test_visibility_workspace_and_validation(lib):
    """muffin_vis_workspace_bytes: the image context, the 2ny x 2nx
    convolution context and three cubes of CG vectors; 0 (with a reason) for
    the wavelet dictionary and for images over 2048 on a side."""
    from paper_1504_06847_amd import lib as L
    s = L.MuffinShape(32, 16, 4, 0)
    p = L.make_params(lib)
    vb = lib.muffin_vis_workspace_bytes(ctypes.byref(s), ctypes.byref(p))
    one = lib.muffin_workspace_bytes(ctypes.byref(s), ctypes.byref(p))
    big = lib.muffin_workspace_bytes(ctypes.byref(L.MuffinShape(64, 32, 4, 0)), ctypes.byref(p))
    assert vb >= one + big + 3 * 32 * 16 * 4 * 4
    p9 = L.make_params(lib, spatial=(0, 1, 2), n_s=3)
    assert lib.muffin_vis_workspace_bytes(ctypes.byref(s), ctypes.byref(p9)) == 0
    assert "Dirac" in L.last_error(lib)
    assert lib.muffin_vis_workspace_bytes(ctypes.byref(L.MuffinShape(4096, 16, 4, 0)), ctypes.byref(p)) == 0
    assert "2048" in L.last_error(lib)


def test_setup_vis_rejects_bad_arguments_before_touching_the_gpu(lib):
    from ctypes import POINTER, byref, c_double, c_int, c_void_p
    from paper_1504_06847_amd import lib as L
    s = L.MuffinShape(16, 16, 2, 0)
    p = L.make_params(lib)
    ctx = c_void_p()
    n_vis = (c_int * 2)(3, 2)
    uv = (c_double * 10)(*([0.5] * 10))
    vis = (c_double * 10)(*([1.0] * 10))
    ws_ok = lib.muffin_vis_workspace_bytes(byref(s), byref(p))
    fake = c_void_p(1 << 20)                # never dereferenced on these paths

    def setup(nv=n_vis, u=uv, v=vis, n_cg=4, ws=fake, nb=ws_ok, out=True):
        return lib.muffin_setup_vis(byref(ctx) if out else None, byref(s), byref(p), nv, u, v, n_cg, ws, nb, None)

    assert setup(out=False) == L.MUFFIN_EINVAL
    assert setup(nv=None) == L.MUFFIN_EINVAL
    assert setup(n_cg=0) == L.MUFFIN_EINVAL and "n_cg" in L.last_error(lib)
    assert setup(n_cg=100001) == L.MUFFIN_EINVAL
    assert setup(nv=(c_int * 2)(3, -1)) == L.MUFFIN_EINVAL
    assert setup(u=None) == L.MUFFIN_EINVAL
    bad = (c_double * 10)(*([0.5] * 9 + [float("nan")]))
    assert setup(u=bad) == L.MUFFIN_ENONFINITE
    assert setup(nb=ws_ok - 1) == L.MUFFIN_EWORKSPACE
    assert setup(ws=c_void_p((1 << 20) + 8)) == L.MUFFIN_EWORKSPACE and "aligned" in L.last_error(lib)
    assert not ctx.value
