"""GPU: solves replayed from HIP graphs equal direct launches.

Each graph replay is checked against the direct result, several times in a
row with other work and synchronisations in between, for FP64 and mixed
factors, solve and apply, both orientations, and widths inside and between
the padding buckets (and one beyond the largest, which runs direct).  The
padded columns of a bucket are computed independently of the others by the
same kernels, so the results agree bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2311_01451_amd import inputs, rsrs  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replays_equal_direct(mixed):
    need_gpu()
    n, m, k = 48, 32, 16
    pts = inputs.jittered_grid2d(n, seed_offset=21)
    tc = rsrs.rsrs_build_tree(pts, m)
    s = tc.samples_required(k, k)
    op = rsrs.rsrs_op_create_kernel(rsrs.RSRS_OP_LOG2D_SKEW, pts, 1.0 / n, 2e-3)
    dt = rsrs.RSRS_F32 if mixed else rsrs.RSRS_F64
    prec = rsrs.RSRS_PREC_F32_MIXED if mixed else rsrs.RSRS_PREC_F64
    F = rsrs.rsrs_factor(tc, rsrs.rsrs_sample(tc, op, s, 5, dtype=dt), k, precision=prec)
    rng = np.random.default_rng(2)
    try:
        for w in (1, 5, 16, 17, 100, 300, 1024, 1100):
            X = torch.tensor(rng.standard_normal((n * n, w)), dtype=torch.float64, device="cuda")
            for fn in (F.solve, F.apply):
                for tr in (False, True):
                    rsrs.rsrs_solve_graphs(False)
                    ref = fn(X, transpose=tr)
                    torch.cuda.synchronize()
                    rsrs.rsrs_solve_graphs(True)
                    for rep in range(3):
                        out = fn(X, transpose=tr)
                        op.matvec(X)                 # other work between replays
                        torch.cuda.synchronize()
                        assert torch.equal(out, ref), (w, fn.__name__, tr, rep)
            print(f"[graphs] mixed={mixed} w={w}: replays equal direct", flush=True)
    finally:
        rsrs.rsrs_solve_graphs(True)
