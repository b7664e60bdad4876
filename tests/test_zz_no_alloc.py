"""The allocation-free feasibility entry point (counts in a static device
array) against ct_feasibility, through the C ABI: two calls in a row, the
second with a smaller batch, each H identical to the allocating entry
point's (same kernels, same order of additions)."""
import numpy as np
import pytest

from paper_2411_11833_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _reference(B, gp, T, n, penalty, stream):
    counts = torch.full((gp.n_constraint,), -1, dtype=torch.int32, device="cuda")
    H = torch.full((1,), np.nan, dtype=torch.float32, device="cuda")
    B.ct_feasibility(gp.handle, T.data_ptr(), n, T.shape[1], penalty, counts.data_ptr(), H.data_ptr(), stream)
    return counts, H


def test_noalloc_feasibility_matches_allocating_entry_point():
    from paper_2411_11833_amd import binding as B
    from paper_2411_11833_amd.planner import GpuProblem
    stream = torch.cuda.current_stream().cuda_stream
    prob = I.packing(0, 0)
    gp = GpuProblem(prob)
    n_big = 3000
    X = gp.from_rows(I.uniform_particles(prob, n_big, seed=77))
    _, T, _ = gp.cost(X, n_big, terms=True)
    results = []
    for n in (n_big, 700):              # the second call is smaller
        penalty = float(-n)
        counts, H_ref = _reference(B, gp, T, n, penalty, stream)
        H = torch.full((1,), np.nan, dtype=torch.float32, device="cuda")
        B.ct_feasibility_noalloc(gp.handle, T.data_ptr(), n, T.shape[1], penalty, H.data_ptr(), stream)
        torch.cuda.synchronize()
        c = counts.cpu().numpy()
        assert np.all(c >= 0) and np.all(c <= n)
        assert (c == 0).any() and (c > 0).any()      # both branches of h_c
        assert float(H.item()) == float(H_ref.item()), (n, float(H.item()), float(H_ref.item()))
        results.append(float(H.item()))
    assert results[0] != results[1]


def test_noalloc_feasibility_two_problems_in_a_row():
    """The static counts are shared by every call on the GPU: a call for a
    problem with fewer constraints after one with more must not see the
    earlier call's counts."""
    from paper_2411_11833_amd import binding as B
    from paper_2411_11833_amd.planner import GpuProblem
    stream = torch.cuda.current_stream().cuda_stream
    out = []
    for prob, n in ((I.packing(2, 3, n_objects=6, n_obstacles=4), 500), (I.single_pick_place(0, 0), 200)):
        gp = GpuProblem(prob)
        X = gp.from_rows(I.uniform_particles(prob, n, seed=5))
        _, T, _ = gp.cost(X, n, terms=True)
        _, H_ref = _reference(B, gp, T, n, -1000.0, stream)
        H = torch.empty(1, dtype=torch.float32, device="cuda")
        B.ct_feasibility_noalloc(gp.handle, T.data_ptr(), n, T.shape[1], -1000.0, H.data_ptr(), stream)
        torch.cuda.synchronize()
        assert float(H.item()) == float(H_ref.item())
        out.append(float(H.item()))
    assert len(out) == 2


def test_noalloc_feasibility_rejects_bad_arguments():
    from paper_2411_11833_amd import binding as B
    from paper_2411_11833_amd.planner import GpuProblem
    prob = I.single_pick_place(0, 0)
    gp = GpuProblem(prob)
    H = torch.empty(1, dtype=torch.float32, device="cuda")
    for args in ((gp.handle, None, 10, 64, -1.0, H.data_ptr()),     # no terms for n > 0
                 (gp.handle, None, 0, 64, -1.0, None),             # no H
                 (gp.handle, None, 0, 64, float("nan"), H.data_ptr())):
        with pytest.raises(B.CtError):
            B.ct_feasibility_noalloc(*args, stream=torch.cuda.current_stream().cuda_stream)
