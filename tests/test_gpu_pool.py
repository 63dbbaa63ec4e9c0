"""GPU: factorizations that reuse the scratch kept from earlier ones.

The workspace and staging of a finished factorization are kept and handed to
the next one of a similar size, so the second factorization of the same
samples runs on buffers that still hold the first one's values.  No kernel
may depend on fresh memory: the second factor, and a third one after the
kept buffers were released, must equal the first bit for bit, in both
precisions.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2311_01451_amd import inputs, rsrs  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _factor(op, tc, s, k, precision):
    dt = rsrs.RSRS_BF16 if precision == rsrs.RSRS_PREC_F32_MIXED else rsrs.RSRS_F64
    smp = rsrs.rsrs_sample(tc, op, s, inputs.BASE_SEED, dtype=dt, symmetric=True)
    return rsrs.rsrs_factor(tc, smp, k, precision=precision, symmetric=True)


def _blocks(F):
    out = []
    for i in range(F.info()["nboxes"]):
        b = F.box(i)
        out.append([np.asarray(b[key]).copy() for key in ("S", "R", "T", "XRR", "KU", "KL")])
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reused_scratch_gives_identical_factors(precision):
    need_gpu()
    prec = rsrs.RSRS_PREC_F32_MIXED if precision == "mixed" else rsrs.RSRS_PREC_F64
    n, m, k = 64, 32, 16
    pts = inputs.grid2d(n)
    N = n * n
    print(f"[pool] N={N} m={m} k={k} precision={precision}", flush=True)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D, pts, 1.0 / n)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    f = torch.tensor(inputs.rhs(N, 4), dtype=torch.float64, device="cuda")
    F1 = _factor(op, tc, s, k, prec)
    ref, u1 = _blocks(F1), F1.solve(f).cpu().numpy()
    del F1
    F2 = _factor(op, tc, s, k, prec)   # runs on the kept buffers
    got2, u2 = _blocks(F2), F2.solve(f).cpu().numpy()
    del F2
    rsrs.rsrs_release_cached()
    F3 = _factor(op, tc, s, k, prec)   # fresh allocations again
    got3, u3 = _blocks(F3), F3.solve(f).cpu().numpy()
    for got in (got2, got3):
        assert len(got) == len(ref)
        for a, b in zip(ref, got):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
    assert np.array_equal(u1, u2) and np.array_equal(u1, u3)
