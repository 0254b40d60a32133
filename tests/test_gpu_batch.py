"""The batched form (grouped launches over cubes of uneven size and band
count) and the FFT tile schedules.  A grouped launch runs the per-tile code
of the single-cube launch of the same schedule: results are compared bit for
bit.  Other schedules evaluate the same formulas in other instruction
sequences (the compiler contracts a product and a sum into one FMA in some
and not in others): results are compared at a few ulps of the cube's
largest value, with the differences printed.  One batched cube is checked
against the FP64 oracle."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (L, ny, nx): uneven sizes and band counts, a dense-DCT band count (15), and
# pixel counts below one 256-thread block (8 x 16)
BATCH = [(8, 32, 32), (16, 64, 32), (4, 32, 64), (8, 64, 64), (15, 32, 32), (16, 16, 16),
         (2, 8, 16), (8, 32, 32), (32, 16, 64)]
PARAMS = dict(mu_eps=1e-3, mu_s=0.05, mu_nu=0.05, rho_P=1.0, rho_T=1.0, rho_V=1.0, rho_S=1.0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _relmax(a, b):
    a, b = a.double(), b.double()
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


# FP32 / FP64 bars for results that take other instruction sequences to the
# same values (other tile shapes, grouped launches): a few ulps of the cube's
# largest value after several passes
TOL = {torch.float32: 1e-6, torch.float64: 1e-14}


def _cubes(shapes, seed0=300):
    out = []
    for i, (L, ny, nx) in enumerate(shapes):
        inst = make_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.005,
                             seed=seed0 + i)
        out.append((inst.psf, inst.dirty))
    return out


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("graph", [False, True], ids=["launch", "graph"])
def test_batch_is_bitwise_the_single_cube_runs(gpu_lib, dtype, graph):
    from paper_1504_06847_amd import Batch, Solver
    cubes = _cubes(BATCH)
    _say("batch", dtype, "graph" if graph else "launch", len(cubes), "cubes")
    b = Batch(cubes, dtype=dtype, graph=graph, params=PARAMS)
    singles = [Solver(p, d, dtype=dtype, **PARAMS) for p, d in cubes]
    # cubes with the fused pass built (FP32, 64 <= nx <= 1024, L in 4..64)
    # run it in the batch too; the others the three-launch pass
    if dtype == torch.float32:
        assert [s.fused_available for s in singles] == [False, False, True, True, False, False, False,
                                                       False, True]
    # 4 shape classes of row passes (nx 16, 32, 64), ... at most 4 x 9 launches
    assert b.launches <= 4 * len(cubes)
    for k in range(6):
        b.iterate(1)
        for s in singles:
            s.iterate(1)
        torch.cuda.synchronize()
        for i, s in enumerate(singles):
            assert torch.equal(b.cube(i).x, s.x), f"pass {k + 1}, cube {i} {BATCH[i]}"
    # a reporting pass on one cube (switches its state set) and a parameter
    # change on another, then more batched passes
    ra, rb = b.cube(2).step_report(), singles[2].step_report()
    assert ra == rb
    b.cube(5).set_params(rho=1.7)
    singles[5].set_params(rho=1.7)
    b.iterate(20)
    for s in singles:
        s.iterate(20)
    torch.cuda.synchronize()
    for i, s in enumerate(singles):
        assert torch.equal(b.cube(i).x, s.x), f"cube {i} {BATCH[i]} after report/set_params"
        assert b.cube(i).iterations == s.iterations
    b.close()


def test_batched_cube_matches_the_oracle(gpu_lib):
    from paper_1504_06847_amd import Batch
    cubes = _cubes(BATCH[:4], seed0=310)
    b = Batch(cubes, params=PARAMS)
    b.iterate(30)
    torch.cuda.synchronize()
    p = O.Params(**PARAMS)
    for i in (1, 3):
        prob = O.Problem(cubes[i][0], cubes[i][1], p)
        st = O.State.zeros(prob.shape)
        for _ in range(30):
            st = O.admm_iteration(prob, st)
        x = b.cube(i).x.cpu().double().numpy()
        err = np.linalg.norm(x - st.X) / np.linalg.norm(st.X)
        _say("batched cube", i, "rel err", err)
        assert err < 1e-5


# shapes whose column tiles take all three widths (ny = 1024 reaches the
# widest tile, 147 KiB of LDS) and whose row tiles take 1..4 rows (nx = 2048)
SCHED_SHAPES = [(2, 1024, 32), (1, 64, 2048), (3, 256, 128)]


@pytest.mark.parametrize("shape", SCHED_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_every_schedule_agrees_to_rounding(gpu_lib, shape, dtype):
    from paper_1504_06847_amd import Solver
    L, ny, nx = shape
    inst = make_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.005, seed=21)
    _say("schedules", shape, dtype)
    ref = Solver(inst.psf, inst.dirty, dtype=dtype, **PARAMS)
    assert ref.schedule == (1, 1, 1)
    ref.set_schedule((1, 1, 0))
    ref.iterate(3)
    xr = ref.x
    for rv in range(3):
        for cv in range(3):
            for fu in range(2):
                s = Solver(inst.psf, inst.dirty, dtype=dtype, **PARAMS)
                s.set_schedule((rv, cv, fu))
                s.iterate(3)
                d = _relmax(s.x, xr)
                _say("schedule", (rv, cv, fu), "max rel diff", d)
                assert d <= TOL[dtype], f"schedule {(rv, cv, fu)}"
                s.close()


def test_autotune_keeps_results_and_state(gpu_lib, tmp_path):
    from paper_1504_06847_amd import Solver
    L, ny, nx = 8, 256, 256
    inst = make_instance(ny, nx, L, n_points=3, n_gauss=1, n_ant=10, noise_sigma=0.005, seed=22)
    a = Solver(inst.psf, inst.dirty, **PARAMS)
    b = Solver(inst.psf, inst.dirty, **PARAMS)
    a.iterate(4)
    b.iterate(4)
    x0 = b.x
    st0 = b.get_state().clone()
    cache = str(tmp_path / "sched.json")
    sch = b.autotune(reps=3, cache=cache)
    _say("autotuned schedule", sch)
    assert 0 <= sch[0] < 3 and 0 <= sch[1] < 3 and sch[2] in (0, 1, 2) and b.schedule == tuple(sch)
    torch.cuda.synchronize()
    assert torch.equal(b.x, x0)                     # the timing leaves X and the state alone
    assert torch.equal(b.get_state(), st0)
    a.iterate(5)
    b.iterate(5)
    torch.cuda.synchronize()
    assert _relmax(b.x, a.x) <= TOL[torch.float32]
    c = Solver(inst.psf, inst.dirty, **PARAMS)
    assert c.autotune(cache=cache) == tuple(sch)    # read back from the cache file


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_128_band_cubes_batch_bitwise(gpu_lib, dtype):
    """128-band cubes take the two-wave spectral pass (64 pixels per block)
    in grouped launches as on their own: the batch repeats the single-cube
    runs bit for bit, next to a cube of another band count."""
    from paper_1504_06847_amd import Batch, Solver
    cubes = _cubes([(128, 16, 16), (128, 8, 32), (64, 8, 8)], seed0=360)
    b = Batch(cubes, dtype=dtype, params=PARAMS)
    singles = [Solver(p, d, dtype=dtype, **PARAMS) for p, d in cubes]
    b.iterate(5)
    for s in singles:
        s.iterate(5)
    torch.cuda.synchronize()
    for i, s in enumerate(singles):
        assert torch.equal(b.cube(i).x, s.x), f"cube {i}"
        assert torch.equal(b.cube(i).get_state(), s.get_state()), f"cube {i}"
    b.close()


def test_batch_runs_fused_form_2_as_form_1(gpu_lib):
    """A cube set to the two-pixel fused form joins the batch's grouped
    fused launch, which has one pixel per thread: the batch repeats the
    single-cube runs of form 1 bit for bit."""
    from paper_1504_06847_amd import Batch, Solver
    cubes = _cubes([(64, 16, 256), (64, 8, 512), (8, 32, 32)], seed0=340)
    b = Batch(cubes, params=PARAMS)
    singles = [Solver(p, d, **PARAMS) for p, d in cubes]
    for i in (0, 1):
        b.cube(i).set_schedule((1, 1, 2))
    b.iterate(4)
    for s in singles:
        s.iterate(4)
    torch.cuda.synchronize()
    for i, s in enumerate(singles):
        assert torch.equal(b.cube(i).x, s.x), f"cube {i}"
    b.close()


def test_batch_autotune_keeps_results(gpu_lib):
    from paper_1504_06847_amd import Batch
    cubes = _cubes(BATCH[:5], seed0=320)
    a = Batch(cubes, params=PARAMS)
    b = Batch(cubes, params=PARAMS)
    a.iterate(3)
    b.iterate(3)
    b.autotune(reps=2)
    a.iterate(4)
    b.iterate(4)
    torch.cuda.synchronize()
    for i in range(len(cubes)):
        d = _relmax(b.cube(i).x, a.cube(i).x)
        _say("batch autotune: cube", i, "max rel diff", d)
        assert d <= TOL[torch.float32]


@pytest.mark.parametrize("graph", [False, True], ids=["launch", "graph"])
def test_batch_with_wavelet_dictionaries_bitwise(gpu_lib, graph):
    """Cubes with wavelet bases in W_s (the paper's dictionary, a subset, the
    Dirac basis alone) batched with others: each cube's wavelet launches
    follow its grouped ones on its lane, so every cube repeats its single
    run bit for bit."""
    from paper_1504_06847_amd import Batch, Solver
    shapes = [(8, 32, 32), (8, 64, 64), (4, 32, 64), (8, 32, 32), (16, 16, 16)]
    bases = [(0, 1, 2, 3, 4, 5, 6, 7, 8), (0,), (0, 2, 5), (0, 8), (0, 1, 2, 3, 4, 5, 6, 7, 8)]
    cubes = _cubes(shapes, seed0=400)
    prm = [dict(PARAMS, spatial=sp) for sp in bases]
    _say("wavelet batch", "graph" if graph else "launch")
    b = Batch(cubes, dtype=torch.float32, graph=graph, params=prm)
    singles = [Solver(p, d, dtype=torch.float32, spatial=sp, **PARAMS) for (p, d), sp in zip(cubes, bases)]
    for k in range(5):
        b.iterate(1)
        for s in singles:
            s.iterate(1)
        torch.cuda.synchronize()
        for i, s in enumerate(singles):
            assert torch.equal(b.cube(i).x, s.x), f"pass {k + 1}, cube {i} {shapes[i]} {bases[i]}"
    # a reporting pass on a batched cube with the paper's dictionary (its
    # wavelet report launches), then more batched passes
    ra, rb = b.cube(0).step_report(), singles[0].step_report()
    assert ra == rb
    b.iterate(6)
    for s in singles:
        s.iterate(6)
    torch.cuda.synchronize()
    for i, s in enumerate(singles):
        assert torch.equal(b.cube(i).get_state(), s.get_state()), f"cube {i}"
    b.close()
