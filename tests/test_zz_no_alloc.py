"""hpdg_apply_B_noalloc: z = B r with B's work vectors in the library's static
scratch array, against hpdg_apply_B (the same kernels on the operator's own
work vectors). Two calls in a row share the array, the second on a smaller
system, so stale contents of the first call would show. The bar is the one
for FP64 preconditioner applications (1e-12 relative); the kernels and their
summation orders are the same, so the results are expected bitwise equal.
"""
import numpy as np
import pytest

import hpinputs as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_2009_01287_amd")


def _pair(op, n, nrhs, seed):
    r = torch.from_numpy(np.random.default_rng(seed).standard_normal(n * nrhs)).cuda()
    z_ref = torch.empty_like(r)
    z_new = torch.full_like(r, float("nan"))
    op.apply_B(r, z_ref, nrhs=nrhs)
    op.apply_B_noalloc(r, z_new, nrhs=nrhs)
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_new.cpu().numpy()


def _check(a, b):
    assert np.all(np.isfinite(b))
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec_fp32", [False, True])
@pytest.mark.parametrize("nrhs", [1, 4])
def test_noalloc_matches_apply_B_two_calls(prec_fp32, nrhs):
    big = H.random_mesh(2, 6, 0.3, 2, 1, 6, seed=21)
    small = H.hanging_mesh(3, 2, seed=2, pmin=1, pmax=4)
    ops = []
    for md, form in ((big, "sipg"), (small, "br2")):
        m = G.Mesh(md)
        ops.append((G.Operator(m, form=form, eta=1.0 if form == "sipg" else 0.0, prec_fp32=prec_fp32,
                               max_nrhs=4, max_block=64), m.ndof))
    assert ops[1][1] < ops[0][1]
    for i, (op, n) in enumerate(ops):
        a, b = _pair(op, n, nrhs, seed=100 + i)
        _check(a, b)
    # the first system again, after the smaller one
    a, b = _pair(ops[0][0], ops[0][1], nrhs, seed=200)
    _check(a, b)


def test_noalloc_rejects_work_beyond_scratch():
    md = H.random_mesh(2, 16, 0.3, 2, 4, 8, seed=22)   # 40,232 DOFs
    m = G.Mesh(md)
    op = G.Operator(m, max_nrhs=256)
    need = m.ndof * 256 * 8
    assert need > 64 << 20
    r = torch.zeros(m.ndof * 256, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    with pytest.raises(G.HpdgError) as ei:
        op.apply_B_noalloc(r, z, nrhs=256)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    # a smaller nrhs on the same operator fits and agrees with apply_B
    a, b = _pair(op, m.ndof, 1, seed=7)
    _check(a, b)
