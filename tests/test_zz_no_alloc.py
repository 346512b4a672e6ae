"""pmg_solve_noalloc (Krylov scratch in the library's fixed device array)
against pmg_solve: the same kernels on the same inputs, so the solutions and
per-problem records must be bit-identical; two calls in a row, the second on
a smaller batch of a smaller shape; a batch beyond the fixed size is refused
before anything is launched."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2504_10710_amd import pmg  # noqa: E402
from tests.gpu_helpers import gpu_batch, problems  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(kind, seeds, p, **kw):
    probs = problems(kind, seeds)
    s, f, g = gpu_batch(probs, p, **kw)
    b = torch.empty_like(f)
    pmg.pmg_rhs(s.h, f, g, b)
    x_ref = torch.empty_like(b)
    pmg.pmg_solve(s.h, b, x_ref, s.info)
    torch.cuda.synchronize()
    info_ref = s.info_host().copy()
    x_na = torch.full_like(b, float("nan"))
    s.info.fill_(0)
    pmg.pmg_solve_noalloc(s.h, b, x_na, s.info)
    torch.cuda.synchronize()
    info_na = s.info_host().copy()
    return x_ref.cpu().numpy(), info_ref, x_na.cpu().numpy(), info_na


@pytest.mark.parametrize("first,second", [
    (("cfg2", [0, 1, 2], 32, dict(gamma=2, alpha=0.16, smoother=pmg.PMG_SMOOTHER_FEM)),
     ("cfg2", [3, 4], 16, dict(gamma=3, alpha=0.16, smoother=pmg.PMG_SMOOTHER_FEM))),
    (("cfg3", [0, 1], 16, dict(gamma=2, alpha=0.16, smoother=pmg.PMG_SMOOTHER_FEM,
                               inner_prec=pmg.PMG_F32, restart=20)),
     ("cfg1", [5], 8, dict(gamma=1, alpha=2.0 / 3.0, smoother=pmg.PMG_SMOOTHER_GLL,
                           krylov=pmg.PMG_PCG))),
])
def test_noalloc_equals_solve_twice(first, second):
    for kind, seeds, p, kw in (first, second):
        print(f"[noalloc] {kind} p={p} batch={len(seeds)} {kw}", flush=True)
        x_ref, i_ref, x_na, i_na = _both(kind, seeds, p, **kw)
        assert np.all(i_ref["status"] == 0), i_ref
        assert np.array_equal(x_na, x_ref)
        assert np.array_equal(i_na["iterations"], i_ref["iterations"])
        assert np.array_equal(i_na["relres"], i_ref["relres"])
        assert np.array_equal(i_na["status"], i_ref["status"])


def test_noalloc_refuses_batches_beyond_the_fixed_array():
    probs = problems("cfg2", list(range(10)))
    s, f, g = gpu_batch(probs, 128, gamma=1, alpha=0.16, smoother=pmg.PMG_SMOOTHER_FEM)
    b = torch.zeros_like(f)
    x = torch.zeros_like(f)
    with pytest.raises(pmg.PmgError) as e:
        pmg.pmg_solve_noalloc(s.h, b, x, s.info)
    assert e.value.code == pmg.PMG_ENOMEM and "scratch" in str(e.value)
