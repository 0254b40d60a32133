"""Parity with the FP64 oracle at the shapes and schedules the benchmark
runs: the FP64 instantiation at 512^2 and 1024^2 with the tile schedules
the autotuner picks there, image heights of 512 in both precisions, a
2048 x 2048 cube, the 16-cube batch of uneven shapes in both grouped pass
forms, and every iterate of the 300-pass 256^2 x 32 run.

Error metric: relative L2 over the whole cube per iterate.  Bars: FP32
1e-5 per iterate (1e-4 on the final cube) against the float64 oracle, FP64
1e-12 against the oracle in extended precision."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from synth import get_config, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TIED = dict(mu_eps=1e-3, mu_s=0.02, mu_nu=0.02, rho_P=1.0, rho_T=1.0, rho_V=1.0, rho_S=1.0)
BAR = {torch.float32: 1e-5, torch.float64: 1e-12}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))
    yield


def _instance(L, ny, nx, seed):
    c = get_config("fp32_256")
    return make_instance(ny, nx, L, n_points=c.n_points, n_gauss=c.n_gauss, n_ant=c.n_ant,
                         noise_sigma=c.noise_sigma, seed=seed)


def _per_iterate(inst, dtype, K, schedule=None, params=TIED):
    from paper_1504_06847_amd import Solver
    s = Solver(inst.psf, inst.dirty, dtype=dtype, **params)
    if schedule is not None:
        s.set_schedule(schedule)
    # FP64 against the oracle in extended precision, FP32 against float64
    prob = O.Problem(inst.psf, inst.dirty, O.Params(**params),
                     dtype=np.longdouble if dtype == torch.float64 else np.float64)
    st = O.State.zeros(prob.shape)
    errs = []
    for _ in range(K):
        s.iterate(1)
        st = O.admm_iteration(prob, st)
        errs.append(rel(s.x.cpu().double().numpy(), st.X.astype(np.float64)))
    s.close()
    return errs


# (L, ny, nx, dtype, schedule): the FP64 schedule the autotuner picks at
# 1024 x 1024 x 64 ([0, 2, 0]) and the default, at 512^2 and 1024^2; image
# heights of 512 (column transforms of 512 points) in both precisions
CASES = [
    (8, 512, 512, torch.float64, (0, 2, 0)),
    (8, 512, 512, torch.float64, (1, 1, 1)),
    (8, 1024, 1024, torch.float64, (0, 2, 0)),
    (4, 1024, 1024, torch.float64, (1, 1, 1)),
    (16, 512, 64, torch.float64, (1, 1, 1)),
    (16, 512, 64, torch.float32, (1, 1, 1)),
    (64, 512, 128, torch.float32, (1, 1, 1)),
    (64, 512, 128, torch.float32, (1, 1, 0)),
    (32, 16, 512, torch.float32, (1, 1, 1)),
    (32, 32, 512, torch.float32, (1, 1, 0)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-{str(c[3])[-7:]}-{''.join(map(str, c[4]))}")
def test_shapes_and_schedules_match_oracle(gpu_lib, case):
    L, ny, nx, dtype, sch = case
    _say("case", case)
    errs = _per_iterate(_instance(L, ny, nx, seed=500 + L + ny), dtype, 4, schedule=sch)
    _say("per-iterate rel err", errs)
    assert max(errs) < BAR[dtype], errs


@pytest.mark.timeout(300)
def test_2048_cube_fp32(gpu_lib):
    """2048 x 2048 x 2: row transforms of 2048 points and columns of 2048."""
    _say("2048 x 2048 x 2 fp32")
    errs = _per_iterate(_instance(2, 2048, 2048, seed=77), torch.float32, 3)
    _say("per-iterate rel err", errs)
    assert max(errs) < 1e-5, errs


@pytest.mark.timeout(300)
def test_4096_wide_fp32(gpu_lib):
    """8 x 4096 x 2: row transforms of 4096 points."""
    _say("8 x 4096 x 2 fp32")
    errs = _per_iterate(_instance(2, 8, 4096, seed=78), torch.float32, 3)
    _say("per-iterate rel err", errs)
    assert max(errs) < 1e-5, errs


@pytest.fixture(scope="module")
def batch_reference():
    """The 16-cube batch and the oracle's X^1, X^2 of every cube."""
    from synth.configs import batch_instances
    O.set_workers(min(16, os.cpu_count() or 1))
    cubes, p = batch_instances()
    ref = []
    for psf, dirty in cubes:
        prob = O.Problem(psf, dirty, O.Params(**p.asdict()))
        st = O.State.zeros(prob.shape)
        xs = []
        for _ in range(2):
            st = O.admm_iteration(prob, st)
            xs.append(st.X)
        ref.append(xs)
    return cubes, p, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("fused", [False, True], ids=["three-launch", "fused"])
def test_config3_batch_matches_oracle(gpu_lib, batch_reference, fused):
    """The benchmark's 16-cube batch (N in {128, 256, 512}, L in {16 .. 128})
    through grouped launches, each cube per iterate against the oracle."""
    from paper_1504_06847_amd import Batch
    cubes, p, ref = batch_reference
    b = Batch(cubes, params=p.asdict())
    forms = []
    for i in range(len(cubes)):
        c = b.cube(i)
        if not fused:
            c.set_schedule((1, 1, 0))
        forms.append(c.schedule[2] if c.fused_available else 0)
    _say("batch", "fused" if fused else "three-launch", "launches per pass", b.launches, "fused cubes", sum(forms))
    if fused:
        assert sum(forms) > 0
    worst = 0.0
    for k in range(2):
        b.iterate(1)
        torch.cuda.synchronize()
        for i in range(len(cubes)):
            e = rel(b.cube(i).x.cpu().double().numpy(), ref[i][k])
            worst = max(worst, e)
            assert e < 1e-5, (i, cubes[i][0].shape, k + 1, e)
    _say("worst per-iterate rel err over the batch", worst)
    b.close()


@pytest.mark.timeout(900)
def test_fp32_256x256x32_every_iterate(gpu_lib):
    """256 x 256 x 32, rho = 1, mu_s = mu_nu = 0.02: all 300 iterates."""
    cfg = get_config("fp32_256")
    _say("fp32_256, all 300 iterates")
    p = cfg.params
    errs = _per_iterate(cfg.make(), torch.float32, cfg.iters, params=p.asdict())
    _say("max", max(errs), "at", int(np.argmax(errs)) + 1, "final", errs[-1])
    assert max(errs) < 1e-5 and errs[-1] < 1e-4
