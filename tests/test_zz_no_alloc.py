"""asdg_apply_operator_static (the entry point that allocates nothing and
uses the library's static device workspace) against asdg_apply's operator
step on the same handle: bitwise equal, on two calls in a row with the
second problem smaller than the first (the static array keeps the first
call's contents)."""
import numpy as np
import pytest

from paper_1903_11357_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_static_operator_apply_equals_bound_apply_big_then_small():
    import torch

    from paper_1903_11357_amd import asdg

    problems = [I.voronoi_problem(1500, 41, p=3, bx=3, by=3, q=1),  # 15000 DoFs
                I.voronoi_problem(200, 42, p=2, bx=2, by=2, q=1)]   # 1200 DoFs
    sizes = []
    for k, P in enumerate(problems):
        print(f"[static apply] call {k}: n={P.n_dofs}", flush=True)
        pr = asdg.setup_problem(P, asdg.FP64, device="cuda:0", factor=False)
        v = torch.from_numpy(np.random.default_rng(10 + k).standard_normal(pr.n)).cuda()
        ref = pr.apply(asdg.APPLY_OPERATOR, v)
        got = pr.apply_operator_static(v)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        sizes.append(pr.n)
    assert sizes[1] < sizes[0]
