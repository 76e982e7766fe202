"""The allocation-free V-cycle (xdg_vcycle_noalloc) against xdg_vcycle on the
same handle: same kernels, so the results agree bit for bit.  Two calls in a
row on different handles, the second with a smaller problem (the fixed work
array then still holds the first call's larger contents), in FP64 and in the
FP32 cycle; handles it cannot serve are refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a device"
    return t


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_vcycle_equals_vcycle(prec, torch):
    from paper_2003_02431_amd import binding as B
    from xdg_inputs import problems
    P = B.XDG_FP64 if prec == "fp64" else B.XDG_MIXED
    big = problems.c2(seed=1, n=16)
    small = problems.c2(seed=3, n=8, hier=[("p", 1), ("h", 1)])
    for name, pr in (("16^3", big), ("8^3", small)):
        S = B.Solver(pr, B.options(precision=P, krylov=B.XDG_FGMRES if P else B.XDG_CG))
        n = S.level_len(0)
        for k in range(2):
            r = S.vec(0, np.random.default_rng(40 + k).uniform(-1, 1, n))
            z_ref, z_na = S.vec(0), S.vec(0)
            z_na.fill_(np.nan)
            B.xdg_vcycle(S.h, r, z_ref)
            B.xdg_vcycle_noalloc(S.h, r, z_na)
            torch.cuda.synchronize()
            same = bool(torch.equal(z_ref, z_na))
            _log(f"  {prec} {name} call {k}: no-alloc V-cycle bit-identical: {same}")
            assert same
        S.close()


def test_noalloc_refuses_16_columns(torch):
    from paper_2003_02431_amd import binding as B
    from xdg_inputs import problems
    pr = problems.c2(seed=3, n=8, hier=[("p", 1), ("h", 1)])
    pr.b = np.zeros((pr.n_rows * pr.np, 16))
    S = B.Solver(pr, B.options(krylov=B.XDG_FGMRES, precision=B.XDG_MIXED, nrhs=16))
    with pytest.raises(B.XdgError) as e:
        B.xdg_vcycle_noalloc(S.h, S.vec(0), S.vec(0))
    assert e.value.code == B.XDG_EINVAL
    S.close()
